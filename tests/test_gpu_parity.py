"""GPU parity: every precision x layout x expression against the FP64
oracle, through the C ABI, at sizes the oracle finishes in seconds (several
workgroups and a ragged tail), plus the exact pins that carry over to the
kernels."""
import itertools

import numpy as np
import pytest
import torch

import oracle as O
import testgen
import paper_1710_09409_amd as su3
from gpu_util import (EXPR_NAMES, LAYOUTS, LAYOUT_NAMES, PREC_NAMES, PRECS,
                      assert_parity, exprs_for, operands, reference, run_expr,
                      upload)

pytestmark = pytest.mark.gpu

# 1 site; 5^4 = 625 and 3x5x7x11 = 1155 (ragged against every lane count and
# sites-per-lane); 8^4 = 4096 (the small workload)
SIZES = ((1, 1, 1, 1), (5, 5, 5, 5), (3, 5, 7, 11), (8, 8, 8, 8))

CASES = [(p, e, lay, lanes, d)
         for p in PRECS for e in exprs_for(p) for (lay, lanes) in LAYOUTS
         for d in SIZES]


def _id(c):
    p, e, lay, lanes, d = c
    return f"{PREC_NAMES[p]}-{EXPR_NAMES[e]}-{LAYOUT_NAMES[lay]}{lanes or ''}-{'x'.join(map(str, d))}"


_ref_cache = {}


def _inputs_and_ref(prec, expr, dims):
    key = (prec, expr, dims)
    if key not in _ref_cache:
        ops = operands(dims, expr)
        _ref_cache[key] = (ops, reference(prec, expr, ops))
    return _ref_cache[key]


@pytest.mark.parametrize("case", CASES, ids=[_id(c) for c in CASES])
def test_parity(case):
    prec, expr, layout, lanes, dims = case
    ops, want = _inputs_and_ref(prec, expr, dims)
    got, _ = run_expr(dims, prec, layout, lanes, expr, ops)
    assert_parity(prec, expr, got, want, _id(case))


@pytest.mark.parametrize("prec", PRECS, ids=[PREC_NAMES[p] for p in PRECS])
def test_aos_lds_staged(prec):
    """The LDS-staged AoS kernel gives the same bits as the direct one."""
    dims = (3, 5, 7, 11)
    for expr in exprs_for(prec):
        ops, want = _inputs_and_ref(prec, expr, dims)
        direct, _ = run_expr(dims, prec, su3.SU3_LAYOUT_AOS, 0, expr, ops)
        cfg = su3.su3_launch_get(expr, prec, su3.SU3_LAYOUT_AOS, 0, dims)
        E, rb = (6, 4) if prec == su3.SU3_C12_F32 else (9, {0: 8, 1: 4, 2: 2}[prec])
        for block in (64, 128):
            if su3.N_OPERANDS[expr] * block * E * 2 * rb > 65536:
                continue  # beyond the staging limit (tested in test_gpu_abi)
            cfg.lds_stage, cfg.block = 1, block
            su3.su3_launch_set(expr, prec, su3.SU3_LAYOUT_AOS, 0, dims, cfg)
            try:
                staged, _ = run_expr(dims, prec, su3.SU3_LAYOUT_AOS, 0, expr, ops)
            finally:
                su3.su3_launch_reset()
            assert np.array_equal(staged, direct), (prec, expr, block)
        assert_parity(prec, expr, direct, want, f"aos-direct {prec} {expr}")


@pytest.mark.parametrize("prec", PRECS, ids=[PREC_NAMES[p] for p in PRECS])
def test_layouts_bit_identical(prec):
    """Per-site arithmetic does not depend on the stored layout."""
    dims = (3, 5, 7, 11)
    for expr in exprs_for(prec):
        ops, _ = _inputs_and_ref(prec, expr, dims)
        outs = [run_expr(dims, prec, lay, lanes, expr, ops)[0]
                for lay, lanes in LAYOUTS]
        for o in outs[1:]:
            assert np.array_equal(o, outs[0]), (prec, expr)


LAUNCHES = [dict(block=b, persistent=p, nontemporal=nt, xcd_remap=x,
                 lds_stage=0, tile_sites=4096, occupancy=occ, schedule=sc,
                 sites_per_lane=0)
            for b, p, nt, x, occ, sc in itertools.product(
                (64, 256), (0, 1), (0, 3, 7), (0, 1), (0, 3), (0, 1))]
# write-through streaming stores, 512- and 1024-lane workgroups (streaming
# or nontemporal stores), one site per lane, and (the product outside half
# storage) twice the natural sites per lane, one-shot and persistent
LAUNCHES += [dict(block=b, persistent=p, nontemporal=nt, xcd_remap=x,
                  lds_stage=0, tile_sites=4096, occupancy=occ, schedule=sc,
                  sites_per_lane=spl)
             for b, p, nt, x, occ, sc, spl in (
                 (64, 0, 6, 0, 5, 1, 0), (512, 0, 7, 0, 2, 1, 0), (512, 1, 3, 1, 0, 0, 0),
                 (1024, 0, 3, 0, 1, 0, 0), (1024, 1, 7, 0, 0, 1, 0),
                 (128, 0, 7, 0, 4, 1, 1), (64, 1, 0, 0, 0, 0, 1),
                 (64, 0, 7, 0, 4, 1, -2), (256, 1, 7, 1, 0, 0, -2), (1024, 0, 7, 0, 1, 1, -2))]


def _launch_for(cfg, prec, expr):
    """The setting with sites_per_lane -2 read as twice the natural count
    (offered for the product outside half storage); None where not offered."""
    if cfg["sites_per_lane"] != -2:
        return cfg
    if expr != su3.SU3_EXPR_MUL or prec == su3.SU3_F16_F32ACC:
        return None
    return dict(cfg, sites_per_lane=2 if prec == su3.SU3_F64 else 4)


@pytest.mark.parametrize("prec", PRECS, ids=[PREC_NAMES[p] for p in PRECS])
def test_launch_settings_bit_identical(prec):
    """Every launch setting (block, persistent grid-stride, nontemporal and
    streaming-store bits, XCD remap, occupancy cap, load/store schedule,
    sites per lane) yields the same bits for every expression; the
    persistent grid of one workgroup per CU exercises the grid-stride loop
    at 16^4, and 3 x 5 x 7 x 11 leaves ragged tails for every sites-per-lane
    count."""
    layout = su3.SU3_LAYOUT_SOA
    try:
        for dims in ((16, 16, 16, 16), (3, 5, 7, 11)):
            for expr in exprs_for(prec):
                ops, want = _inputs_and_ref(prec, expr, dims)
                base = None
                for cfg0 in LAUNCHES:
                    cfg = _launch_for(cfg0, prec, expr)
                    if cfg is None:
                        continue
                    su3.su3_launch_set(expr, prec, layout, 0, dims, cfg)
                    got, _ = run_expr(dims, prec, layout, 0, expr, ops)
                    if base is None:
                        base = got
                        assert_parity(prec, expr, got, want, f"launch {cfg}")
                    assert np.array_equal(got, base), (dims, expr, cfg)
    finally:
        su3.su3_launch_reset()


def test_identity_exact():
    """I*y = y and x*I = x bit-exactly (up to the sign of zero) in every
    precision: multiplying by exact 0 and 1 rounds nothing."""
    dims = (3, 5, 7, 11)
    V = testgen.volume(dims)
    x = testgen.su3_field(V, field_id=40)
    eye = testgen.identity(V)
    for prec in PRECS:
        xs = O.get().roundtrip(prec, x)
        for lay, lanes in LAYOUTS:
            for ops in ((eye, x), (x, eye)):
                got, _ = run_expr(dims, prec, lay, lanes, su3.SU3_EXPR_MUL, list(ops))
                rows = 2 if prec == su3.SU3_C12_F32 else 3
                assert np.array_equal(got[:, :rows], xs[:, :rows]), (prec, lay, lanes)


def test_signed_permutations_exact():
    """Products of the 24 signed permutation matrices are exact on the GPU."""
    mats = testgen.signed_permutations()
    pairs = list(itertools.product(range(24), repeat=2))
    x = testgen.from_int_matrices([mats[i] for i, _ in pairs])
    y = testgen.from_int_matrices([mats[j] for _, j in pairs])
    want = testgen.from_int_matrices([mats[i] @ mats[j] for i, j in pairs])
    dims = (len(pairs), 1, 1, 1)
    for prec in PRECS:
        for lay, lanes in LAYOUTS:
            got, _ = run_expr(dims, prec, lay, lanes, su3.SU3_EXPR_MUL, [x, y])
            assert np.array_equal(got, want), (prec, lay, lanes)


def test_constant_fields_composite():
    """The sum and the sum-plus-product of the constant SU(3)-typed fields
    1*I and 2*I (Section 3's composite-expression example, Listing 2) are
    exactly 3*I and 5*I in every precision that takes sums and every layout."""
    from pins import read_golden
    g = read_golden("composite_constants.txt")
    dims = (4, 4, 4, 4)
    V = testgen.volume(dims)
    a, b = testgen.identity(V, g["a"]), testgen.identity(V, g["b"])
    for prec in (su3.SU3_F64, su3.SU3_F32, su3.SU3_F16_F32ACC):
        for lay, lanes in LAYOUTS:
            got, _ = run_expr(dims, prec, lay, lanes, su3.SU3_EXPR_ADD, [a, b])
            assert np.array_equal(got, testgen.identity(V, g["ADD"]))
            got, _ = run_expr(dims, prec, lay, lanes, su3.SU3_EXPR_APB_AB, [a, b])
            assert np.array_equal(got, testgen.identity(V, g["APB_AB"]))


def test_fused_reductions_exact():
    """MUL3(a, I, c) = MUL(a, c) and MULADD(a, c, 0, 0) = MUL(a, c)
    bit-exactly on the GPU (F64, F32; MUL3 also for the compressed form)."""
    dims = (3, 5, 7, 11)
    V = testgen.volume(dims)
    a, c = (testgen.su3_field(V, field_id=f) for f in (41, 42))
    eye, zero = testgen.identity(V), np.zeros((V, 3, 3, 2))
    for prec in (su3.SU3_F64, su3.SU3_F32, su3.SU3_C12_F32):
        ac, _ = run_expr(dims, prec, su3.SU3_LAYOUT_SOA, 0, su3.SU3_EXPR_MUL, [a, c])
        m3, _ = run_expr(dims, prec, su3.SU3_LAYOUT_SOA, 0, su3.SU3_EXPR_MUL3,
                         [a, eye, c])
        assert np.array_equal(m3, ac), prec
        if prec != su3.SU3_C12_F32:
            ma, _ = run_expr(dims, prec, su3.SU3_LAYOUT_SOA, 0,
                             su3.SU3_EXPR_MULADD, [a, c, zero, zero])
            assert np.array_equal(ma, ac), prec


def test_pack_bit_exact():
    """The library's upload (quantise + pack) writes exactly the oracle's
    stored image, padding included."""
    for dims in ((1, 1, 1, 1), (3, 5, 7, 11), (8, 8, 8, 8)):
        V = testgen.volume(dims)
        x = testgen.su3_field(V, field_id=43)
        for prec in PRECS:
            for lay, lanes in LAYOUTS:
                f = upload(dims, prec, lay, lanes, x, torch.cuda.current_stream())
                raw = su3.su3_field_download_raw(f)
                want = O.get().pack(x, prec, lay, lanes)
                assert np.array_equal(raw, want), (dims, prec, lay, lanes)
                back = su3.su3_field_download(f)
                assert np.array_equal(back, O.get().roundtrip(prec, x))
