"""Parity at the benchmark's full sizes, in the launch configuration the
benchmark times (the autotuner's choice): every site of 48^4 for each
storage precision, the fused expressions on four link fields at 32^4, and
every site of every lattice of the 64-lattice batch.  Also reports the
end-to-end error of the reduced-precision forms against the FP64 truth
(max elementwise error, normwise relative error, unitarity and determinant
deviation), printed and, when SU3_REPORT_DIR names a folder, written there
as precision_errors.json."""
import json
import os

import numpy as np
import pytest
import torch

import oracle as O
import testgen
import paper_1710_09409_amd as su3
from gpu_util import PREC_NAMES, assert_parity

pytestmark = pytest.mark.gpu

D48 = (48, 48, 48, 48)
D32 = (32, 32, 32, 32)
_host = {}


def host(V, fid):
    if (V, fid) not in _host:
        _host[(V, fid)] = testgen.su3_field(V, field_id=fid)
    return _host[(V, fid)]


def run_tuned(dims, prec, expr, fids, layout=su3.SU3_LAYOUT_SOA, lanes=0):
    """Autotune like bench.py, upload, evaluate, download."""
    s = torch.cuda.current_stream()
    V = testgen.volume(dims)
    cfg = su3.su3_autotune(expr, prec, layout, lanes, dims, s)
    fs = []
    for fid in fids:
        f = su3.field_tensor(dims, prec, layout, lanes)
        su3.su3_field_upload(f, host(V, fid), s)
        fs.append(f)
    z = su3.field_tensor(dims, prec, layout, lanes)
    su3.su3_fused_eval(z, expr, fs, s)
    su3.su3_sync(s)
    out = su3.su3_field_download(z, s)
    del fs, z
    torch.cuda.empty_cache()
    return out, cfg


LAYS = [(su3.SU3_LAYOUT_SOA, 0), (su3.SU3_LAYOUT_AOSOA, 64)]


@pytest.mark.parametrize("lay,lanes", LAYS, ids=["soa", "aosoa64"])
@pytest.mark.parametrize("prec", [0, 1, 2, 3], ids=[PREC_NAMES[p] for p in range(4)])
def test_mult_48(prec, lay, lanes):
    V = testgen.volume(D48)
    fids = (testgen.FID_X, testgen.FID_Y)
    got, cfg = run_tuned(D48, prec, su3.SU3_EXPR_MUL, fids, lay, lanes)
    ops = [host(V, f) for f in fids]
    want = O.get().reference(su3.SU3_EXPR_MUL, prec, ops)
    worst = assert_parity(prec, su3.SU3_EXPR_MUL, got, want, f"48^4 {PREC_NAMES[prec]} {cfg.as_dict()}")
    print(f"48^4 {PREC_NAMES[prec]}: worst {worst:.3e} with launch {cfg.as_dict()}")


def test_mult_shard():
    """One t-slab of a 48^4 lattice cut into 8 (48^3 x 6), FP64 SoA, in the
    tuned launch; every site compared with the oracle."""
    dims = (48, 48, 48, 6)
    V = testgen.volume(dims)
    fids = (60, 61)
    got, cfg = run_tuned(dims, 0, su3.SU3_EXPR_MUL, fids)
    want = O.get().reference(su3.SU3_EXPR_MUL, 0, [host(V, f) for f in fids])
    assert_parity(0, su3.SU3_EXPR_MUL, got, want, f"48^3x6 f64 {cfg.as_dict()}")


@pytest.mark.parametrize("lay,lanes", LAYS, ids=["soa", "aosoa64"])
@pytest.mark.parametrize("prec", [0, 1], ids=["f64", "f32"])
@pytest.mark.parametrize("expr", [su3.SU3_EXPR_MUL3, su3.SU3_EXPR_MULADD], ids=["mul3", "muladd"])
def test_fused_32(prec, expr, lay, lanes):
    V = testgen.volume(D32)
    n = su3.N_OPERANDS[expr]
    fids = tuple(testgen.FID_U0 + mu for mu in range(n))
    got, cfg = run_tuned(D32, prec, expr, fids, lay, lanes)
    want = O.get().reference(expr, prec, [host(V, f) for f in fids])
    assert_parity(prec, expr, got, want, f"32^4 fused {expr} {PREC_NAMES[prec]}")


def test_batch_64_every_site():
    """The benchmark's 64-lattice batch (seed 1710, each item stored in the
    layout the library recommends for its lattice and precision, the batch
    autotuner's launch) against the oracle at every site of every lattice;
    then the other kind of grid (a persistent grid looping over the tiles if
    the tuned launch is one-shot, else one workgroup per tile) replayed into
    fresh outputs gives the same bits."""
    s = torch.cuda.current_stream()
    lat = testgen.batch_lattices(64)
    exprs = [su3.SU3_EXPR_MUL] * 64
    rec = {}
    for d, comp in lat:
        prec = su3.SU3_C12_F32 if comp else su3.SU3_F64
        if (d, prec) not in rec:
            rec[(d, prec)] = su3.su3_layout_recommend(su3.SU3_EXPR_MUL, prec, d, s)[:2]
    zs, ops = [], []
    for i, (d, comp) in enumerate(lat):
        prec = su3.SU3_C12_F32 if comp else su3.SU3_F64
        lay, lanes = rec[(d, prec)]
        V = testgen.volume(d)
        row = []
        for k in range(2):
            f = su3.field_tensor(d, prec, lay, lanes)
            su3.su3_field_upload(f, testgen.su3_field(V, field_id=testgen.FID_BATCH_BASE + 4 * i + k), s)
            row.append(f)
        ops.append(row)
        zs.append(su3.field_tensor(d, prec, lay, lanes))
    cfg = su3.su3_batch_autotune(exprs, zs, ops, s)
    b = su3.su3_batch_create(exprs, zs, ops, s)
    su3.su3_batch_launch(b, s)
    su3.su3_sync(s)
    su3.su3_batch_destroy(b)
    for i, (d, comp) in enumerate(lat):
        prec = su3.SU3_C12_F32 if comp else su3.SU3_F64
        V = testgen.volume(d)
        x = testgen.su3_field(V, field_id=testgen.FID_BATCH_BASE + 4 * i)
        y = testgen.su3_field(V, field_id=testgen.FID_BATCH_BASE + 4 * i + 1)
        want = O.get().reference(su3.SU3_EXPR_MUL, prec, [x, y])
        got = su3.su3_field_download(zs[i], s)
        assert_parity(prec, su3.SU3_EXPR_MUL, got, want, f"batch lattice {i} {d} {cfg.as_dict()}")
    # the other grid kind, same tile table rules, bit for bit
    other = su3.su3_launch(**cfg.as_dict())
    if cfg.persistent:
        other.persistent = 0
    else:
        other.persistent, other.block, other.tile_sites = 2, 256, 2048
    total = sum(testgen.volume(d) for d, _ in lat)
    kprec = su3.SU3_C12_F32 if lat[0][1] else su3.SU3_F64
    klay, klanes = rec[(lat[0][0], kprec)]
    key = su3.SU3_EXPR_BATCH + su3.SU3_EXPR_MUL
    z2 = [su3.field_tensor(d, p, *rec[(d, p)])
          for d, p in ((d, su3.SU3_C12_F32 if c else su3.SU3_F64) for d, c in lat)]
    su3.su3_launch_set(key, kprec, klay, klanes, (total, 1, 1, 1), other)
    try:
        b = su3.su3_batch_create(exprs, z2, ops, s)
    finally:
        su3.su3_launch_reset()
    su3.su3_batch_launch(b, s)
    su3.su3_sync(s)
    su3.su3_batch_destroy(b)
    for i in range(64):
        assert torch.equal(zs[i].owner, z2[i].owner), (i, other.as_dict())


def test_precision_error_report():
    """End-to-end error of each storage form against z = x*y in FP64 on the
    original inputs, at 32^4 and 48^4."""
    report = {}
    for dims in (D32, D48):
        V = testgen.volume(dims)
        x, y = host(V, testgen.FID_X), host(V, testgen.FID_Y)
        truth = O.get().mult(x, y)
        key = "x".join(map(str, dims))
        report[key] = {}
        for prec in (0, 1, 2, 3):
            got, cfg = run_tuned(dims, prec, su3.SU3_EXPR_MUL, (testgen.FID_X, testgen.FID_Y))
            m = O.get().metrics(got, truth)
            report[key][PREC_NAMES[prec]] = {k: float(v) for k, v in m.items()}
            print(key, PREC_NAMES[prec], {k: f"{v:.3e}" for k, v in m.items()})
        r = report[key]
        assert r["f64"]["r_max"] <= 1e-14
        assert 1e-8 < r["f32"]["e_max"] < 1e-6 and r["f32"]["d_u"] < 1e-6
        assert 1e-5 < r["f16"]["e_max"] < 4e-3 and r["f16"]["d_u"] < 1e-2
        assert 1e-8 < r["c12"]["e_max"] < 2e-6 and r["c12"]["d_u"] < 2e-6
    out = os.environ.get("SU3_REPORT_DIR")
    if out:
        os.makedirs(out, exist_ok=True)
        with open(os.path.join(out, "precision_errors.json"), "w") as f:
            json.dump(report, f, indent=1)
