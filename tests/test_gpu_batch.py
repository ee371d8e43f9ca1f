"""Batched persistent launch: tile table bit-exact against the oracle's
recompute, every graph replay bit-identical to unbatched launches."""
import numpy as np
import pytest
import torch

import oracle as O
import testgen
import paper_1710_09409_amd as su3
from gpu_util import assert_parity, run_expr, upload

pytestmark = pytest.mark.gpu

ITEMS_MIXED = [  # (dims, prec, layout, lanes, expr) -- the streaming mix
    ((2, 3, 5, 7), su3.SU3_F64, su3.SU3_LAYOUT_SOA, 0, su3.SU3_EXPR_MUL),
    ((8, 8, 8, 8), su3.SU3_C12_F32, su3.SU3_LAYOUT_SOA, 0, su3.SU3_EXPR_MUL),
    ((4, 4, 4, 9), su3.SU3_F64, su3.SU3_LAYOUT_AOSOA, 16, su3.SU3_EXPR_MUL),
    ((1, 1, 1, 1), su3.SU3_C12_F32, su3.SU3_LAYOUT_AOSOA, 8, su3.SU3_EXPR_MUL),
    ((6, 6, 6, 6), su3.SU3_F64, su3.SU3_LAYOUT_SOA, 0, su3.SU3_EXPR_MUL),
]
ITEMS_ANY = ITEMS_MIXED + [
    ((3, 5, 7, 11), su3.SU3_F32, su3.SU3_LAYOUT_SOA, 0, su3.SU3_EXPR_MULADD),
    ((5, 5, 5, 5), su3.SU3_F16_F32ACC, su3.SU3_LAYOUT_AOSOA, 32, su3.SU3_EXPR_MUL),
    ((5, 5, 5, 7), su3.SU3_F16_F32ACC, su3.SU3_LAYOUT_SOA, 0, su3.SU3_EXPR_APB_AB),
    ((4, 5, 6, 7), su3.SU3_C12_F32, su3.SU3_LAYOUT_SOA, 0, su3.SU3_EXPR_MUL3),
    ((4, 4, 4, 4), su3.SU3_F64, su3.SU3_LAYOUT_AOSOA, 64, su3.SU3_EXPR_ADD),
]


def _build(items, stream, tile_sites):
    zs, ops, hosts, exprs = [], [], [], []
    for i, (dims, prec, lay, lanes, expr) in enumerate(items):
        V = testgen.volume(dims)
        h = [testgen.su3_field(V, field_id=testgen.FID_BATCH_BASE + 4 * i + k)
             for k in range(su3.N_OPERANDS[expr])]
        ops.append([upload(dims, prec, lay, lanes, x, stream) for x in h])
        zs.append(su3.field_tensor(dims, prec, lay, lanes))
        hosts.append(h)
        exprs.append(expr)
    return zs, ops, hosts, exprs


@pytest.mark.parametrize("items", [ITEMS_MIXED, ITEMS_ANY], ids=["mixed", "any"])
@pytest.mark.parametrize("tile,pers,sched,nt", [(64, 0, 1, 3), (256, 2, 0, 3), (4096, 0, 0, 3),
                                                (4096, 4, 1, 3), (2048, 0, 1, 7),
                                                (512, 2, 0, 7)])
def test_batch_matches_unbatched(items, tile, pers, sched, nt):
    s = torch.cuda.current_stream()
    dims0, prec0, lay0, lanes0, expr0 = items[0]
    total = sum(testgen.volume(d) for d, *_ in items)
    key = su3.SU3_EXPR_BATCH + expr0
    cfg = su3.su3_launch_get(key, prec0, lay0, lanes0, (total, 1, 1, 1))
    cfg.tile_sites, cfg.persistent, cfg.schedule, cfg.nontemporal = tile, pers, sched, nt
    su3.su3_launch_set(key, prec0, lay0, lanes0, (total, 1, 1, 1), cfg)
    try:
        zs, ops, hosts, exprs = _build(items, s, tile)
        b = su3.su3_batch_create(exprs, zs, ops, s)
    finally:
        su3.su3_launch_reset()
    # tile table, bit-exact against the oracle's recompute
    rows = su3.su3_batch_tiles(b)
    vols = [testgen.volume(d) for d, *_ in items]
    precs = [p for _, p, *_ in items]
    starts, want_rows = O.tile_table(vols, tile, precs)
    assert np.array_equal(rows, np.array(want_rows, dtype=np.int32).reshape(-1, 4))
    # unbatched results
    singles = []
    for (dims, prec, lay, lanes, expr), h in zip(items, hosts):
        got, _ = run_expr(dims, prec, lay, lanes, expr, h)
        assert_parity(prec, expr, got, O.get().reference(expr, prec, h), "single")
        singles.append(got)
    # several replays with eager work and synchronisation in between
    for rep in range(3):
        for z in zs:
            z.owner.fill_(rep + 1)
        su3.su3_batch_launch(b, s)
        su3.su3_sync(s)
        for i, z in enumerate(zs):
            got = su3.su3_field_download(z, s)
            assert np.array_equal(got, singles[i]), (rep, i)
    su3.su3_batch_destroy(b)


def test_batch_rejects_bad_items():
    s = torch.cuda.current_stream()
    a = su3.field_tensor((4, 4, 4, 4), su3.SU3_F64, su3.SU3_LAYOUT_AOS)
    with pytest.raises(su3.Su3Error) as e:
        su3.su3_batch_create([su3.SU3_EXPR_MUL], [a], [[a, a]], s)
    assert e.value.status == su3.SU3_ERR_UNSUPPORTED
    b = su3.field_tensor((4, 4, 4, 4), su3.SU3_F64, su3.SU3_LAYOUT_SOA)
    c = su3.field_tensor((4, 4, 4, 4), su3.SU3_F32, su3.SU3_LAYOUT_SOA)
    with pytest.raises(su3.Su3Error) as e:
        su3.su3_batch_create([su3.SU3_EXPR_MUL], [b], [[b, c]], s)
    assert e.value.status == su3.SU3_ERR_MISMATCH


def test_batch_autotune_then_create():
    """The batch autotuner's candidates all run; the batch created after it
    (with the tuned launch) matches unbatched launches bit for bit."""
    s = torch.cuda.current_stream()
    try:
        zs, ops, hosts, exprs = _build(ITEMS_MIXED, s, 0)
        best = su3.su3_batch_autotune(exprs, zs, ops, s)
        assert best.tile_sites % 64 == 0
        b = su3.su3_batch_create(exprs, zs, ops, s)
        for z in zs:
            z.owner.fill_(7)
        su3.su3_batch_launch(b, s)
        su3.su3_sync(s)
        for (dims, prec, lay, lanes, expr), h, z in zip(ITEMS_MIXED, hosts, zs):
            single, _ = run_expr(dims, prec, lay, lanes, expr, h)
            assert np.array_equal(su3.su3_field_download(z, s), single)
        su3.su3_batch_destroy(b)
    finally:
        su3.su3_launch_reset()
