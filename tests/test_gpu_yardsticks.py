"""Bandwidth yardsticks and the layout recommendation on the GPU.

Every stream kind gives its defined result in every launch form the tuner
can choose: blocks of 64 to 1024 lanes, occupancy caps, nontemporal loads
and stores, and write-through streaming stores. The stream tuner returns
one of those forms. The layout recommendation returns a layout whose
tuned product matches the oracle. Inputs are integer-valued, so the triad
is exact in any evaluation order and is compared bit for bit."""
import numpy as np
import pytest
import torch

import oracle as O
import testgen
import paper_1710_09409_amd as su3
from gpu_util import assert_parity, run_expr

pytestmark = pytest.mark.gpu

# (block, occupancy cap, nontemporal bits): plain, nontemporal loads and
# stores, write-through stores alone and with nontemporal loads
CFGS = ((64, 0, 0), (64, 8, 3), (128, 0, 6), (256, 4, 7), (512, 0, 2), (1024, 1, 7),
        (192, 0, 1))
# element counts (16-byte elements) with a ragged last workgroup, and one
# smaller than a workgroup
N16 = (100_003, 37)


def _arrays(n16, seed):
    g = torch.Generator(device="cpu").manual_seed(seed)
    b = torch.randint(-1000, 1000, (2 * n16,), generator=g).to(torch.float64).cuda()
    c = torch.randint(-1000, 1000, (2 * n16,), generator=g).to(torch.float64).cuda()
    # a guard element after a's n16 elements must stay as it was
    a = torch.full((2 * n16 + 2,), 7.5, dtype=torch.float64, device="cuda")
    return a, b, c


@pytest.mark.parametrize("n16", N16)
@pytest.mark.parametrize("block,occ,nt", CFGS)
def test_stream_kinds_every_launch_form(block, occ, nt, n16):
    s = torch.cuda.current_stream()
    cfg = dict(block=block, occupancy=occ, nontemporal=nt)
    nbytes = 16 * n16
    a, b, c = _arrays(n16, seed=block + nt)
    # triad: a = b + 3 c, exact on integers
    su3.su3_stream(su3.SU3_STREAM_TRIAD, a.data_ptr(), b.data_ptr(), c.data_ptr(), 3.0,
                   nbytes, cfg, s)
    su3.su3_sync(s)
    assert torch.equal(a[:2 * n16], b + 3.0 * c)
    assert torch.all(a[2 * n16:] == 7.5)
    # write: a = s in every double
    su3.su3_stream(su3.SU3_STREAM_WRITE, a.data_ptr(), None, None, -2.25, nbytes, cfg, s)
    su3.su3_sync(s)
    assert torch.all(a[:2 * n16] == -2.25) and torch.all(a[2 * n16:] == 7.5)
    # copy: a = b
    su3.su3_stream(su3.SU3_STREAM_COPY, a.data_ptr(), b.data_ptr(), None, 0.0, nbytes, cfg, s)
    su3.su3_sync(s)
    assert torch.equal(a[:2 * n16], b) and torch.all(a[2 * n16:] == 7.5)
    # read: writes nothing unless an element of b + c is (s, -s)
    a.fill_(7.5)
    su3.su3_stream(su3.SU3_STREAM_READ, a.data_ptr(), b.data_ptr(), c.data_ptr(), 1e9,
                   nbytes, cfg, s)
    su3.su3_sync(s)
    assert torch.all(a == 7.5)
    # ... and writes a's first element when one is
    k = n16 // 2
    b2 = b.clone()
    b2[2 * k] = 5.0 - c[2 * k]
    b2[2 * k + 1] = -5.0 - c[2 * k + 1]
    su3.su3_stream(su3.SU3_STREAM_READ, a.data_ptr(), b2.data_ptr(), c.data_ptr(), 5.0,
                   nbytes, cfg, s)
    su3.su3_sync(s)
    assert a[0].item() == 5.0 and a[1].item() == -5.0 and torch.all(a[2:] == 7.5)


def test_stream_rejects_bad_arguments():
    a = torch.zeros(64, dtype=torch.float64, device="cuda")
    for nbytes, cfg in ((24, None), (0, None), (512, dict(block=96)),
                        (512, dict(block=2048)), (512, dict(block=64, nontemporal=4))):
        with pytest.raises(su3.Su3Error) as e:
            su3.su3_stream(su3.SU3_STREAM_WRITE, a.data_ptr(), None, None, 1.0, nbytes, cfg)
        assert e.value.status == su3.SU3_ERR_INVALID_ARG, (nbytes, cfg)


def test_stream_autotune_returns_a_valid_form():
    s = torch.cuda.current_stream()
    n16 = 1 << 16
    a, b, c = _arrays(n16, seed=3)
    best, us = su3.su3_stream_autotune(su3.SU3_STREAM_TRIAD, a.data_ptr(), b.data_ptr(),
                                       c.data_ptr(), 16 * n16, s)
    assert us > 0 and 64 <= best.block <= 1024 and best.block % 64 == 0
    assert best.nontemporal in (0, 1, 2, 3, 6, 7)
    # the tuned form computes the triad
    su3.su3_stream(su3.SU3_STREAM_TRIAD, a.data_ptr(), b.data_ptr(), c.data_ptr(), 3.0,
                   16 * n16, best, s)
    su3.su3_sync(s)
    assert torch.equal(a[:2 * n16], b + 3.0 * c)


@pytest.mark.parametrize("prec", [su3.SU3_F64, su3.SU3_C12_F32], ids=["f64", "c12"])
def test_layout_recommendation_runs_and_matches_oracle(prec):
    dims = (8, 8, 6, 10)
    s = torch.cuda.current_stream()
    try:
        lay, lanes, best, us = su3.su3_layout_recommend(su3.SU3_EXPR_MUL, prec, dims, s)
        assert us > 0
        assert (lay, lanes) == (su3.SU3_LAYOUT_SOA, 0) or (
            lay == su3.SU3_LAYOUT_AOSOA and lanes in (8, 16, 32, 64))
        # the recommended layout keeps its tuned launch, as su3_autotune does
        assert su3.su3_launch_get(su3.SU3_EXPR_MUL, prec, lay, lanes,
                                  dims).as_dict() == best.as_dict()
        V = testgen.volume(dims)
        host = [testgen.su3_field(V, field_id=testgen.FID_X),
                testgen.su3_field(V, field_id=testgen.FID_Y)]
        got, _ = run_expr(dims, prec, lay, lanes, su3.SU3_EXPR_MUL, host)
        assert_parity(prec, su3.SU3_EXPR_MUL, got,
                      O.get().reference(su3.SU3_EXPR_MUL, prec, host), "recommended")
    finally:
        su3.su3_launch_reset()
