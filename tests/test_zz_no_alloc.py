"""The allocation-free batch entry point (su3_batch_run, through the C ABI)
against the allocating one (su3_batch_create + su3_batch_launch) and the
oracle: two calls in a row, the second with fewer and smaller items, in a
one-shot and in a persistent launch (whose ticket counter lives in the
shared scratch array too)."""
import numpy as np
import pytest
import torch

import testgen
import paper_1710_09409_amd as su3
from gpu_util import assert_parity, reference, upload

pytestmark = pytest.mark.gpu

ITEMS = [  # (dims, prec, layout, lanes, expr): precisions, layouts, ragged volumes
    ((2, 3, 5, 7), su3.SU3_F64, su3.SU3_LAYOUT_SOA, 0, su3.SU3_EXPR_MUL),
    ((8, 8, 8, 8), su3.SU3_C12_F32, su3.SU3_LAYOUT_SOA, 0, su3.SU3_EXPR_MUL),
    ((4, 4, 4, 9), su3.SU3_F64, su3.SU3_LAYOUT_AOSOA, 16, su3.SU3_EXPR_MUL3),
    ((3, 5, 7, 11), su3.SU3_F32, su3.SU3_LAYOUT_SOA, 0, su3.SU3_EXPR_MULADD),
    ((5, 5, 5, 5), su3.SU3_F16_F32ACC, su3.SU3_LAYOUT_AOSOA, 32, su3.SU3_EXPR_MUL),
    ((5, 5, 5, 7), su3.SU3_F16_F32ACC, su3.SU3_LAYOUT_SOA, 0, su3.SU3_EXPR_APB_AB),
    ((4, 5, 6, 7), su3.SU3_C12_F32, su3.SU3_LAYOUT_SOA, 0, su3.SU3_EXPR_MUL3),
    ((6, 6, 6, 6), su3.SU3_F64, su3.SU3_LAYOUT_AOSOA, 64, su3.SU3_EXPR_ADD),
    ((16, 16, 16, 16), su3.SU3_F64, su3.SU3_LAYOUT_SOA, 0, su3.SU3_EXPR_MUL),
]
SMALL = [  # the second call: fewer items, smaller lattices
    ((1, 1, 1, 1), su3.SU3_F64, su3.SU3_LAYOUT_SOA, 0, su3.SU3_EXPR_MUL),
    ((3, 3, 3, 5), su3.SU3_F32, su3.SU3_LAYOUT_AOSOA, 8, su3.SU3_EXPR_MUL),
    ((2, 2, 2, 9), su3.SU3_C12_F32, su3.SU3_LAYOUT_SOA, 0, su3.SU3_EXPR_MUL),
]


def _build(items, stream, base):
    zs, ops, hosts, exprs = [], [], [], []
    for i, (dims, prec, lay, lanes, expr) in enumerate(items):
        V = testgen.volume(dims)
        h = [testgen.su3_field(V, field_id=testgen.FID_BATCH_BASE + 4 * (base + i) + k)
             for k in range(su3.N_OPERANDS[expr])]
        ops.append([upload(dims, prec, lay, lanes, x, stream) for x in h])
        zs.append(su3.field_tensor(dims, prec, lay, lanes))
        hosts.append(h)
        exprs.append(expr)
    return zs, ops, hosts, exprs


@pytest.mark.parametrize("pers,tile,block", [(0, 256, 128), (2, 512, 256)],
                         ids=["one-shot", "persistent"])
def test_batch_run_matches_batch_launch(pers, tile, block):
    s = torch.cuda.current_stream()
    try:
        for items, base in ((ITEMS, 0), (SMALL, 40)):
            zs, ops, hosts, exprs = _build(items, s, base)
            dims0, prec0, lay0, lanes0, expr0 = items[0]
            total = sum(testgen.volume(d) for d, *_ in items)
            key = su3.SU3_EXPR_BATCH + expr0
            cfg = su3.su3_launch_get(key, prec0, lay0, lanes0, (total, 1, 1, 1))
            cfg.persistent, cfg.tile_sites, cfg.block, cfg.nontemporal = pers, tile, block, 7
            su3.su3_launch_set(key, prec0, lay0, lanes0, (total, 1, 1, 1), cfg)
            # the allocating form
            b = su3.su3_batch_create(exprs, zs, ops, s)
            su3.su3_batch_launch(b, s)
            su3.su3_sync(s)
            su3.su3_batch_destroy(b)
            want = [su3.su3_field_download(z, s) for z in zs]
            # the allocation-free form, into overwritten outputs
            for z in zs:
                z.owner.fill_(0x7f)
            su3.su3_batch_run(exprs, zs, ops, s)
            su3.su3_sync(s)
            for i, ((dims, prec, lay, lanes, expr), h, z) in enumerate(zip(items, hosts, zs)):
                got = su3.su3_field_download(z, s)
                assert np.array_equal(got, want[i]), (base, i)
                assert_parity(prec, expr, got, reference(prec, expr, h), f"run item {i}")
    finally:
        su3.su3_launch_reset()


def test_batch_run_limit():
    """More items than the scratch array holds: a clear error, nothing run."""
    s = torch.cuda.current_stream()
    f = su3.field_tensor((2, 2, 2, 2), su3.SU3_F64, su3.SU3_LAYOUT_SOA)
    with pytest.raises(su3.Su3Error) as e:
        su3.su3_batch_run([su3.SU3_EXPR_MUL] * 1025, [f] * 1025, [[f, f]] * 1025, s)
    assert e.value.status == su3.SU3_ERR_INVALID_ARG
    assert "1024" in str(e.value)
