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


# Fields at the size limit: 2^31 - 1 reals per field (offsets are 32-bit in
# units of reals).  128^3 x 56 FP64 sites hold 18 x 117,440,512 =
# 2,113,929,216 reals and 128^3 x 85 two-row FP32 sites 12 x 178,257,920 =
# 2,139,095,040 (one more t-slice of either passes the limit): about 51
# and 26 GB for three fields.  The inputs are made
# on the device from a seeded 16^4 block of SU(3) matrices: site s holds
# block matrix s mod 65536 times the cube root of unity w^k(s), k a hash of
# s, so every site stays in SU(3) (w^k is central) and a site offset by a
# multiple of the block reads a different matrix.  Sampled sites -- the
# first and last 64 and 4096 drawn at random -- are read back from the
# stored operands and checked against the oracle's product.
LIMIT_CASES = [(su3.SU3_F64, (128, 128, 128, 56)), (su3.SU3_C12_F32, (128, 128, 128, 85))]
LIMIT_LAUNCHES = (  # the headline's launch (write-through stores), a plain one, wide blocks
    dict(block=64, persistent=0, nontemporal=7, xcd_remap=0, lds_stage=0, tile_sites=4096,
         occupancy=5, schedule=1, sites_per_lane=0),
    dict(block=256, persistent=0, nontemporal=0, xcd_remap=1, lds_stage=0, tile_sites=4096,
         occupancy=0, schedule=0, sites_per_lane=0),
    dict(block=1024, persistent=0, nontemporal=3, xcd_remap=0, lds_stage=0, tile_sites=4096,
         occupancy=0, schedule=1, sites_per_lane=0),
)


def _stored(f, prec, V):
    """The SoA image of a field as a (E, V, 2) tensor (V a multiple of 64)."""
    E = 9 if prec == su3.SU3_F64 else 6
    dt = torch.float64 if prec == su3.SU3_F64 else torch.float32
    return f.owner.view(dt).view(E, V, 2)


def _limit_field(dims, prec, fid, salt, s):
    n0 = 65536
    small = su3.field_tensor((16, 16, 16, 16), prec, su3.SU3_LAYOUT_SOA)
    su3.su3_field_upload(small, testgen.su3_field(n0, field_id=fid), s)
    sv = _stored(small, prec, n0).to(torch.float64)
    V = testgen.volume(dims)
    big = su3.field_tensor(dims, prec, su3.SU3_LAYOUT_SOA)
    bv = _stored(big, prec, V)
    cw = torch.tensor([1.0, -0.5, -0.5], dtype=torch.float64, device="cuda")
    sw = torch.tensor([0.0, 0.75 ** 0.5, -(0.75 ** 0.5)], dtype=torch.float64, device="cuda")
    chunk = 1 << 23
    for a in range(0, V, chunk):
        idx = torch.arange(a, min(V, a + chunk), dtype=torch.int64, device="cuda")
        k = ((idx * 2654435761 + salt) >> 11) % 3
        blk = sv[:, idx % n0, :]
        re, im = blk[..., 0], blk[..., 1]
        bv[:, a:a + idx.numel(), 0] = (re * cw[k] - im * sw[k]).to(bv.dtype)
        bv[:, a:a + idx.numel(), 1] = (re * sw[k] + im * cw[k]).to(bv.dtype)
    del small, sv
    return big


def _canonical(stored, prec):
    """(E, n, 2) stored values at sampled sites -> (n, 3, 3, 2) doubles
    (two-row form: row 2 left zero; the oracle's reference rebuilds it)."""
    a = stored.to(torch.float64).cpu().numpy().transpose(1, 0, 2)
    n = a.shape[0]
    out = np.zeros((n, 3, 3, 2))
    rows = 3 if prec == su3.SU3_F64 else 2
    out[:, :rows] = a.reshape(n, rows, 3, 2)
    return out


@pytest.mark.parametrize("prec,dims", LIMIT_CASES, ids=["f64", "c12"])
def test_mult_at_field_size_limit(prec, dims):
    s = torch.cuda.current_stream()
    V = testgen.volume(dims)
    E = 9 if prec == su3.SU3_F64 else 6
    assert V % 64 == 0 and E * 2 * V <= 2 ** 31 - 1 < E * 2 * (V + 128 ** 3)
    x = _limit_field(dims, prec, testgen.FID_X, 11, s)
    y = _limit_field(dims, prec, testgen.FID_Y, 29, s)
    z = su3.field_tensor(dims, prec, su3.SU3_LAYOUT_SOA)
    g = np.random.default_rng(1710)
    sites = np.unique(np.concatenate([np.arange(64), np.arange(V - 64, V),
                                      g.integers(0, V, 4096)]))
    si = torch.from_numpy(sites).cuda()
    xs = _canonical(_stored(x, prec, V)[:, si, :], prec)
    ys = _canonical(_stored(y, prec, V)[:, si, :], prec)
    want = O.get().reference(su3.SU3_EXPR_MUL, prec, [xs, ys])
    try:
        for cfg in LIMIT_LAUNCHES:
            su3.su3_launch_set(su3.SU3_EXPR_MUL, prec, su3.SU3_LAYOUT_SOA, 0, dims, cfg)
            z.owner.zero_()
            su3.su3_mult(z, x, y, s)
            su3.su3_sync(s)
            got = _canonical(_stored(z, prec, V)[:, si, :], prec)
            assert_parity(prec, su3.SU3_EXPR_MUL, got, want, f"size limit {dims} {cfg}")
    finally:
        su3.su3_launch_reset()
        del x, y, z
        torch.cuda.empty_cache()
