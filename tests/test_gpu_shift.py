"""Shifted operands on the GPU: Cshift (a copy, so bit-exact against the
oracle's shift of the stored values) and z(x) = x(x) * y(x + k mu_hat)
(within the product's tolerance), every precision x layout x direction,
both signs, shifts beyond the extent, ragged lattices; aliasing rules; full
48^4 double precision."""
import numpy as np
import pytest
import torch

import oracle as O
import testgen
import paper_1710_09409_amd as su3
from gpu_util import LAYOUTS, LAYOUT_NAMES, PREC_NAMES, PRECS, assert_parity, upload

pytestmark = pytest.mark.gpu

DIMS = ((3, 5, 7, 11), (8, 8, 8, 8), (1, 2, 1, 3))
SHIFTS = (1, -1, 2, 13)


@pytest.mark.parametrize("dims", DIMS, ids=["x".join(map(str, d)) for d in DIMS])
@pytest.mark.parametrize("prec", PRECS, ids=[PREC_NAMES[p] for p in PRECS])
def test_shift_parity(dims, prec):
    s = torch.cuda.current_stream()
    V = testgen.volume(dims)
    x = testgen.su3_field(V, field_id=60)
    y = testgen.su3_field(V, field_id=61)
    qx, qy = O.get().roundtrip(prec, x), O.get().roundtrip(prec, y)
    for lay, lanes in LAYOUTS:
        fx = upload(dims, prec, lay, lanes, x, s)
        fy = upload(dims, prec, lay, lanes, y, s)
        fz = su3.field_tensor(dims, prec, lay, lanes)
        for mu in range(4):
            for k in SHIFTS:
                want = O.get().cshift(qy, dims, mu, k)
                for nt in (3, 7):
                    cfg = dict(block=64, persistent=0, nontemporal=nt, xcd_remap=0,
                               lds_stage=0, tile_sites=4096, occupancy=0, schedule=0)
                    su3.su3_launch_set(su3.SU3_EXPR_CSHIFT, prec, lay, lanes, dims, cfg)
                    try:
                        su3.su3_cshift(fz, fy, mu, k, s)
                    finally:
                        su3.su3_launch_reset()
                    got = su3.su3_field_download(fz, s)
                    assert np.array_equal(got, want), (LAYOUT_NAMES[lay], lanes, mu, k, nt)
                ref = O.get().mult(qx, want)
                prev = None
                for sched, nt in ((0, 3), (1, 3), (1, 7)):
                    cfg = dict(block=64, persistent=0, nontemporal=nt, xcd_remap=0,
                               lds_stage=0, tile_sites=4096, occupancy=4,
                               schedule=sched)
                    su3.su3_launch_set(su3.SU3_EXPR_MUL_SHIFTED, prec, lay, lanes,
                                       dims, cfg)
                    try:
                        su3.su3_mult_shifted(fz, fx, fy, mu, k, s)
                    finally:
                        su3.su3_launch_reset()
                    got = su3.su3_field_download(fz, s)
                    assert_parity(prec, su3.SU3_EXPR_MUL, got, ref,
                                  f"shifted {LAYOUT_NAMES[lay]}{lanes} mu {mu} k {k}")
                    assert prev is None or np.array_equal(got, prev)
                    prev = got


def test_shift_rules():
    s = torch.cuda.current_stream()
    d = (4, 4, 4, 6)
    V = testgen.volume(d)
    x = testgen.su3_field(V, field_id=62)
    y = testgen.su3_field(V, field_id=63)
    fx = upload(d, 0, 1, 0, x, s)
    fy = upload(d, 0, 1, 0, y, s)
    f32 = su3.field_tensor(d, 1, 1, 0)

    def status(fn, *a):
        try:
            fn(*a)
        except su3.Su3Error as e:
            return e.status
        return 0
    assert status(su3.su3_cshift, fx, fx, 0, 1, s) == su3.SU3_ERR_ALIAS
    assert status(su3.su3_cshift, f32, fx, 0, 1, s) == su3.SU3_ERR_MISMATCH
    assert status(su3.su3_cshift, fy, fx, 4, 1, s) == su3.SU3_ERR_INVALID_ARG
    assert status(su3.su3_mult_shifted, fy, fx, fy, 1, 1, s) == su3.SU3_ERR_ALIAS
    # in place on the unshifted operand: x <- x * y(x + t_hat)
    su3.su3_mult_shifted(fx, fx, fy, 3, 1, s)
    want = O.get().mult_shifted(x, y, d, 3, 1)
    assert_parity(0, su3.SU3_EXPR_MUL, su3.su3_field_download(fx, s), want, "in place")


@pytest.mark.parametrize("mu", [0, 3])
def test_shift_48_f64(mu):
    s = torch.cuda.current_stream()
    d = (48, 48, 48, 48)
    V = testgen.volume(d)
    x = testgen.su3_field(V, field_id=testgen.FID_X)
    y = testgen.su3_field(V, field_id=testgen.FID_Y)
    fx, fy = upload(d, 0, 1, 0, x, s), upload(d, 0, 1, 0, y, s)
    fz = su3.field_tensor(d, 0, 1, 0)
    su3.su3_cshift(fz, fy, mu, -1, s)
    sy = O.get().cshift(y, d, mu, -1)
    assert np.array_equal(su3.su3_field_download(fz, s), sy)
    su3.su3_mult_shifted(fz, fx, fy, mu, -1, s)
    assert_parity(0, su3.SU3_EXPR_MUL, su3.su3_field_download(fz, s),
                  O.get().mult(x, sy), f"48^4 shifted mu {mu}")
