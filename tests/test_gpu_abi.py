"""GPU-side contract of the C ABI: aliasing, mismatches, unsupported
combinations, wrap checks, padding never written, yardstick kernels."""
import numpy as np
import pytest
import torch

import oracle as O
import testgen
import paper_1710_09409_amd as su3
from gpu_util import assert_parity, run_expr, upload

pytestmark = pytest.mark.gpu

DIMS = (3, 5, 7, 11)
V = testgen.volume(DIMS)


def _status(fn, *a):
    try:
        fn(*a)
    except su3.Su3Error as e:
        return e.status
    return su3.SU3_OK


def test_in_place_and_self_product():
    x = testgen.su3_field(V, field_id=50)
    y = testgen.su3_field(V, field_id=51)
    s = torch.cuda.current_stream()
    for prec in (su3.SU3_F64, su3.SU3_F32, su3.SU3_F16_F32ACC, su3.SU3_C12_F32):
        for lay, lanes in ((su3.SU3_LAYOUT_SOA, 0), (su3.SU3_LAYOUT_AOSOA, 16),
                           (su3.SU3_LAYOUT_AOS, 0)):
            want = O.get().reference(su3.SU3_EXPR_MUL, prec, [x, y])
            fx = upload(DIMS, prec, lay, lanes, x, s)
            fy = upload(DIMS, prec, lay, lanes, y, s)
            su3.su3_mult(fx, fx, fy, s)          # x <- x * y
            assert_parity(prec, 0, su3.su3_field_download(fx, s), want, "in-place")
            fy2 = upload(DIMS, prec, lay, lanes, y, s)
            su3.su3_mult(fy2, fy2, fy2, s)       # y <- y * y
            want2 = O.get().reference(su3.SU3_EXPR_MUL, prec, [y, y])
            assert_parity(prec, 0, su3.su3_field_download(fy2, s), want2, "square")


def test_partial_overlap_rejected():
    n = su3.su3_field_bytes(DIMS, su3.SU3_F64, su3.SU3_LAYOUT_SOA)
    t = torch.zeros(2 * n, dtype=torch.uint8, device="cuda")
    a = su3.su3_field_wrap(t, DIMS, su3.SU3_F64, su3.SU3_LAYOUT_SOA)
    b = su3.su3_field_wrap(t[1024:], DIMS, su3.SU3_F64, su3.SU3_LAYOUT_SOA)
    c = su3.field_tensor(DIMS, su3.SU3_F64, su3.SU3_LAYOUT_SOA)
    assert _status(su3.su3_mult, b, a, c) == su3.SU3_ERR_ALIAS
    assert _status(su3.su3_mult, a, c, b) == su3.SU3_ERR_ALIAS
    assert _status(su3.su3_mult, c, a, b) == su3.SU3_OK  # operands may overlap


def test_mismatch_and_unsupported():
    f64 = su3.field_tensor(DIMS, su3.SU3_F64, su3.SU3_LAYOUT_SOA)
    f32 = su3.field_tensor(DIMS, su3.SU3_F32, su3.SU3_LAYOUT_SOA)
    other = su3.field_tensor((3, 5, 7, 12), su3.SU3_F64, su3.SU3_LAYOUT_SOA)
    aosoa8 = su3.field_tensor(DIMS, su3.SU3_F64, su3.SU3_LAYOUT_AOSOA, 8)
    aosoa16 = su3.field_tensor(DIMS, su3.SU3_F64, su3.SU3_LAYOUT_AOSOA, 16)
    aos = su3.field_tensor(DIMS, su3.SU3_F64, su3.SU3_LAYOUT_AOS)
    assert _status(su3.su3_mult, f64, f64, f32) == su3.SU3_ERR_MISMATCH
    assert _status(su3.su3_mult, f64, other, f64) == su3.SU3_ERR_MISMATCH
    assert _status(su3.su3_mult, aosoa8, aosoa8, aosoa16) == su3.SU3_ERR_MISMATCH
    assert _status(su3.su3_mult, aos, aos, f64) == su3.SU3_ERR_MISMATCH
    c12 = [su3.field_tensor(DIMS, su3.SU3_C12_F32, su3.SU3_LAYOUT_SOA) for _ in range(5)]
    for expr in (su3.SU3_EXPR_ADD, su3.SU3_EXPR_APB_AB):
        assert _status(su3.su3_fused_eval, c12[0], expr, c12[1:3]) == su3.SU3_ERR_UNSUPPORTED
    assert _status(su3.su3_fused_eval, c12[0], su3.SU3_EXPR_MULADD,
                   c12[1:5]) == su3.SU3_ERR_UNSUPPORTED
    assert _status(su3.su3_fused_eval, f64, su3.SU3_EXPR_MUL3,
                   [f64, f64]) == su3.SU3_ERR_INVALID_ARG
    assert _status(su3.su3_fused_eval, f64, 7, [f64, f64]) == su3.SU3_ERR_INVALID_ARG


def test_lds_stage_limit():
    """A staged launch whose LDS tiles exceed 64 KB is refused up front."""
    d = (4, 4, 4, 4)
    f = [su3.field_tensor(d, su3.SU3_F64, su3.SU3_LAYOUT_AOS) for _ in range(5)]
    cfg = dict(block=128, persistent=0, nontemporal=3, xcd_remap=0,
               lds_stage=1, tile_sites=4096)
    su3.su3_launch_set(su3.SU3_EXPR_MULADD, su3.SU3_F64, su3.SU3_LAYOUT_AOS, 0, d, cfg)
    try:
        assert _status(su3.su3_fused_eval, f[0], su3.SU3_EXPR_MULADD,
                       f[1:5]) == su3.SU3_ERR_UNSUPPORTED
    finally:
        su3.su3_launch_reset()


def test_wrap_checks():
    n = su3.su3_field_bytes(DIMS, su3.SU3_F32, su3.SU3_LAYOUT_SOA)
    t = torch.zeros(n + 64, dtype=torch.uint8, device="cuda")
    assert _status(su3.su3_field_wrap, t[:n - 1], DIMS, su3.SU3_F32,
                   su3.SU3_LAYOUT_SOA) == su3.SU3_ERR_INVALID_ARG
    assert _status(su3.su3_field_wrap, t[8:], DIMS, su3.SU3_F32,
                   su3.SU3_LAYOUT_SOA) == su3.SU3_ERR_INVALID_ARG
    host = torch.zeros(n, dtype=torch.uint8)
    assert _status(su3.su3_field_wrap, host.data_ptr(), DIMS, su3.SU3_F32,
                   su3.SU3_LAYOUT_SOA, 0, n) == su3.SU3_ERR_INVALID_ARG
    assert _status(su3.su3_field_wrap, t, DIMS, su3.SU3_F32,
                   su3.SU3_LAYOUT_SOA) == su3.SU3_OK


def test_alloc_owns_zeroed_memory():
    f = su3.su3_field_alloc(DIMS, su3.SU3_F64, su3.SU3_LAYOUT_AOSOA, 32)
    raw = su3.su3_field_download_raw(f)
    assert raw.size == su3.su3_field_bytes(DIMS, su3.SU3_F64, su3.SU3_LAYOUT_AOSOA, 32)
    assert not raw.any()
    su3.su3_field_free(f)


def _padding_bytes(prec, lay, lanes):
    """Boolean mask over the stored image: True on bytes of padding sites
    (built from the layout's definition with numpy reshapes)."""
    E = 6 if prec == su3.SU3_C12_F32 else 9
    rb = {0: 8, 1: 4, 2: 2, 3: 4}[prec]
    if lay == su3.SU3_LAYOUT_SOA:
        Vpad = -(-V // 64) * 64
        L = Vpad
    else:
        L, Vpad = lanes, -(-V // lanes) * lanes
    valid = np.zeros((Vpad, E, 2), dtype=bool)
    valid[:V] = True
    img = valid.reshape(Vpad // L, L, E, 2).transpose(0, 2, 1, 3).reshape(-1)
    return np.repeat(~img, rb)


@pytest.mark.parametrize("lay,lanes", [(su3.SU3_LAYOUT_SOA, 0),
                                       (su3.SU3_LAYOUT_AOSOA, 64)])
def test_padding_never_written(lay, lanes):
    """Padding sites keep whatever bytes they held across compute calls."""
    s = torch.cuda.current_stream()
    x = testgen.su3_field(V, field_id=52)
    for prec in (su3.SU3_F64, su3.SU3_F32, su3.SU3_F16_F32ACC, su3.SU3_C12_F32):
        n = su3.su3_field_bytes(DIMS, prec, lay, lanes)
        t = torch.full((n,), 0xAB, dtype=torch.uint8, device="cuda")
        z = su3.su3_field_wrap(t, DIMS, prec, lay, lanes)
        fx = upload(DIMS, prec, lay, lanes, x, s)
        su3.su3_mult(z, fx, fx, s)
        su3.su3_sync(s)
        raw = su3.su3_field_download_raw(z)
        pad = _padding_bytes(prec, lay, lanes)
        assert pad.size == raw.size and pad.any()
        assert np.all(raw[pad] == 0xAB), prec
        assert not np.all(raw[~pad] == 0xAB), prec


def test_triad_and_copy():
    n = 1_000_003
    b = torch.randn(n, dtype=torch.float64, device="cuda")
    c = torch.randn(n, dtype=torch.float64, device="cuda")
    a = torch.empty_like(b)
    su3.su3_triad(a.data_ptr(), b.data_ptr(), c.data_ptr(), 3.0, n)
    su3.su3_sync()
    assert torch.allclose(a, b + 3.0 * c, rtol=1e-15, atol=1e-15)
    src = torch.randint(0, 255, (1 << 20,), dtype=torch.uint8, device="cuda")
    dst = torch.zeros_like(src)
    su3.su3_copy(dst.data_ptr(), src.data_ptr(), src.numel())
    su3.su3_sync()
    assert torch.equal(dst, src)
