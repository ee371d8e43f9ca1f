"""Wilson hopping term on the GPU against the oracle: every precision pair
(F64/F64, F32/F32, F32 spinors with compressed links) in every layout on
ragged lattices (extents 1 and 2 included, where forward and backward
neighbours coincide), bitwise agreement across launch settings (one site
per lane and t-walks of several lengths, ragged last walk included),
argument rules, and the full 48^4 lattice in the tuned launch.

Tolerance (absolute, per real entry).  Each output entry is a sum over 8
hops of +-1 or +-i times an entry of U h (or U^dagger h), h a sum of two
input entries.  With mag(x, a) = sum over hops and colours b of |U_ab| *
(1-norm over spins and re/im of the input's colour b at the neighbour), a
chain of k roundings errs by at most about k u mag; k = 1 (projection) + 6
(complex 3-term dot product in FMAs) + 8 (accumulation) = 15, +4 when the
links' third row is rebuilt in single precision.  Enforced with a factor 2,
plus the rounding of the stored result (u |out|)."""
import numpy as np
import pytest
import torch

import oracle as O
import testgen
import paper_1710_09409_amd as su3
from gpu_util import LAYOUTS, LAYOUT_NAMES

pytestmark = pytest.mark.gpu

PAIRS = ((su3.SU3_F64, su3.SU3_F64), (su3.SU3_F32, su3.SU3_F32),
         (su3.SU3_F32, su3.SU3_C12_F32))
PAIR_IDS = ["f64", "f32", "f32c12"]
DIMS = ((3, 5, 7, 11), (1, 2, 1, 3), (8, 8, 8, 8), (4, 6, 2, 10))
FID_SPINOR = 200


def magnitude(links, psi, dims):
    """mag[s, a] of the module docstring (numpy, canonical arrays)."""
    V = testgen.volume(dims)
    shape = tuple(reversed(dims))  # (t, z, y, x)
    absu = [np.hypot(u[..., 0], u[..., 1]) for u in links]        # (V, 3, 3)
    colour = np.abs(psi).sum(axis=(1, 3))                          # (V, 3)
    mag = np.zeros((V, 3))
    for mu in range(4):
        axis = 3 - mu
        c4 = colour.reshape(shape + (3,))
        fwd = np.roll(c4, -1, axis=axis).reshape(V, 3)   # colour(x + mu)
        bwd = np.roll(c4, 1, axis=axis).reshape(V, 3)    # colour(x - mu)
        u4 = absu[mu].reshape(shape + (3, 3))
        ub = np.roll(u4, 1, axis=axis).reshape(V, 3, 3)  # |U_mu(x - mu)|
        mag += np.einsum("sab,sb->sa", absu[mu], fwd)
        mag += np.einsum("sba,sb->sa", ub, bwd)
    return mag


def quantised_spinor(prec, psi):
    return psi if prec == su3.SU3_F64 else psi.astype(np.float32).astype(np.float64)


def assert_dslash(sp, lp, got, want, mag, where=""):
    u = 2.0 ** -53 if sp == su3.SU3_F64 else 2.0 ** -24
    k = 15 + (4 if lp == su3.SU3_C12_F32 else 0)
    tol = 2.0 * k * u * mag[:, None, :, None] + u * np.abs(want)
    excess = np.abs(got - want) - tol
    bad = np.argwhere(excess > 0)
    assert bad.size == 0, (
        f"{where}: {len(bad)} entries beyond tolerance, first at {tuple(bad[0])}: "
        f"got {got[tuple(bad[0])]!r} want {want[tuple(bad[0])]!r}")
    return float(np.max(np.abs(got - want))) if got.size else 0.0


def host_inputs(dims, seed=testgen.DEFAULT_SEED):
    V = testgen.volume(dims)
    links = [testgen.su3_field(V, seed=seed, field_id=testgen.FID_U0 + mu)
             for mu in range(4)]
    psi = testgen.spinor_field(V, seed=seed, field_id=FID_SPINOR)
    return links, psi


def device_inputs(dims, sp, lp, lay, lanes, links, psi, s):
    fu = []
    for u in links:
        f = su3.field_tensor(dims, lp, lay, lanes)
        su3.su3_field_upload(f, u, s)
        fu.append(f)
    fin = su3.spinor_tensor(dims, sp, lay, lanes)
    su3.su3_field_upload(fin, psi, s)
    return fu, fin


def reference(sp, lp, links, psi, dims):
    q = [O.get().roundtrip(lp, u) for u in links]
    qpsi = quantised_spinor(sp, psi)
    return O.get().dslash(q, qpsi, dims), magnitude(q, qpsi, dims)


@pytest.mark.parametrize("dims", DIMS, ids=["x".join(map(str, d)) for d in DIMS])
@pytest.mark.parametrize("pair", PAIRS, ids=PAIR_IDS)
def test_dslash_parity(pair, dims):
    sp, lp = pair
    s = torch.cuda.current_stream()
    links, psi = host_inputs(dims)
    want, mag = reference(sp, lp, links, psi, dims)
    for lay, lanes in LAYOUTS:
        fu, fin = device_inputs(dims, sp, lp, lay, lanes, links, psi, s)
        fout = su3.spinor_tensor(dims, sp, lay, lanes)
        prev = None
        # one site per lane; walks of 3 t-slices; one walk over all of t;
        # walks of 4 and 2; site tiles 8x4x2x2, 4x4x4x1, 8x2x2x8 (ragged
        # against these lattices); LDS-tiled walks of 3 and of all of t;
        # the one-buffer tiles 8x8, 8x4, 16x8 and 16x4 (blocks up to 512, walks of
        # 2, 3, 5 and all of t, nontemporal link loads or not); whole x rows
        # with one and with two buffers; persistent walks over (tile, slice)
        # spans; tiles in XCD slabs; rows of 3 x 3 (one and two buffers);
        # the same rows with a halo of projected face sites (lexicographic
        # layouts; the virtual-node layout falls back to rows without one)
        for cfg in (dict(block=64, nontemporal=0, occupancy=0, xcd_remap=0, tile_sites=1,
                         schedule=0),
                    dict(block=256, nontemporal=3, occupancy=4, xcd_remap=1, tile_sites=3,
                         schedule=0),
                    dict(block=128, nontemporal=2, occupancy=2, xcd_remap=0,
                         tile_sites=4096, schedule=0),
                    dict(block=128, nontemporal=2, occupancy=0, xcd_remap=1, tile_sites=4,
                         schedule=0),
                    dict(block=64, nontemporal=2, occupancy=0, xcd_remap=0, tile_sites=2,
                         schedule=0),
                    dict(block=128, nontemporal=2, occupancy=0, xcd_remap=1, tile_sites=1,
                         schedule=1),
                    dict(block=64, nontemporal=2, occupancy=0, xcd_remap=0, tile_sites=1,
                         schedule=2),
                    dict(block=256, nontemporal=2, occupancy=2, xcd_remap=1, tile_sites=1,
                         schedule=3),
                    dict(block=128, nontemporal=2, occupancy=0, xcd_remap=0, tile_sites=3,
                         schedule=4),
                    dict(block=256, nontemporal=2, occupancy=0, xcd_remap=1, tile_sites=4096,
                         schedule=4),
                    dict(block=128, nontemporal=3, occupancy=0, xcd_remap=0, tile_sites=3,
                         schedule=5),
                    dict(block=256, nontemporal=2, occupancy=0, xcd_remap=1, tile_sites=4096,
                         schedule=5),
                    dict(block=512, nontemporal=2, occupancy=0, xcd_remap=0, tile_sites=2,
                         schedule=5),
                    dict(block=128, nontemporal=2, occupancy=0, xcd_remap=1, tile_sites=5,
                         schedule=6),
                    dict(block=256, nontemporal=3, occupancy=0, xcd_remap=0, tile_sites=4096,
                         schedule=6),
                    dict(block=256, nontemporal=2, occupancy=0, xcd_remap=0, tile_sites=3,
                         schedule=7),
                    dict(block=512, nontemporal=3, occupancy=0, xcd_remap=1, tile_sites=4096,
                         schedule=7),
                    dict(block=256, nontemporal=2, occupancy=0, xcd_remap=1, tile_sites=3,
                         schedule=8),
                    dict(block=512, nontemporal=2, occupancy=0, xcd_remap=0, tile_sites=4096,
                         schedule=8),
                    dict(block=64, nontemporal=2, occupancy=0, xcd_remap=0, tile_sites=3,
                         schedule=9),
                    dict(block=256, nontemporal=3, occupancy=0, xcd_remap=1, tile_sites=4096,
                         schedule=10),
                    dict(block=128, nontemporal=2, occupancy=0, xcd_remap=0, tile_sites=2,
                         schedule=11),
                    dict(block=256, nontemporal=2, occupancy=0, xcd_remap=1, tile_sites=5,
                         schedule=12),
                    dict(block=64, nontemporal=2, occupancy=0, xcd_remap=1, tile_sites=3,
                         schedule=13),
                    dict(block=256, nontemporal=2, occupancy=0, xcd_remap=0, tile_sites=4096,
                         schedule=16),
                    dict(block=256, persistent=1, nontemporal=2, occupancy=0, xcd_remap=0,
                         tile_sites=1, schedule=8),
                    dict(block=256, persistent=2, nontemporal=2, occupancy=0, xcd_remap=1,
                         tile_sites=1, schedule=11),
                    dict(block=256, persistent=3, nontemporal=2, occupancy=0, xcd_remap=0,
                         tile_sites=1, schedule=16),
                    dict(block=256, nontemporal=2, occupancy=0, xcd_remap=2, tile_sites=3,
                         schedule=11),
                    dict(block=128, nontemporal=2, occupancy=0, xcd_remap=2, tile_sites=4096,
                         schedule=4),
                    dict(block=256, nontemporal=2, occupancy=0, xcd_remap=0, tile_sites=3,
                         schedule=17),
                    dict(block=256, nontemporal=2, occupancy=0, xcd_remap=1, tile_sites=5,
                         schedule=18),
                    dict(block=256, persistent=2, nontemporal=2, occupancy=0, xcd_remap=0,
                         tile_sites=1, schedule=18),
                    dict(block=64, nontemporal=2, occupancy=0, xcd_remap=0, tile_sites=3,
                         schedule=19),
                    dict(block=256, nontemporal=2, occupancy=0, xcd_remap=1, tile_sites=4096,
                         schedule=22),
                    dict(block=256, persistent=2, nontemporal=2, occupancy=0, xcd_remap=0,
                         tile_sites=1, schedule=26),
                    dict(block=256, nontemporal=2, occupancy=0, xcd_remap=2, tile_sites=5,
                         schedule=27),
                    dict(block=256, nontemporal=2, occupancy=0, xcd_remap=0, tile_sites=3,
                         schedule=28),
                    dict(block=256, persistent=1, nontemporal=2, occupancy=0, xcd_remap=0,
                         tile_sites=1, schedule=20)):
            full = dict(dict(persistent=0, lds_stage=0), **cfg)
            su3.su3_launch_set(su3.SU3_EXPR_DSLASH, lp, lay, lanes, dims, full)
            try:
                su3.su3_dslash(fout, fu, fin, s)
            finally:
                su3.su3_launch_reset()
            su3.su3_sync(s)
            got = su3.su3_field_download(fout, s)
            assert_dslash(sp, lp, got, want, mag,
                          f"{PAIR_IDS[PAIRS.index(pair)]} {LAYOUT_NAMES[lay]}{lanes} {cfg}")
            assert prev is None or np.array_equal(got, prev), "launch settings differ"
            prev = got


def test_dslash_leaves_padding_and_inputs_alone():
    """SoA pads the volume to a multiple of 64 sites: the padding of the
    output stays as it was, and inputs are unchanged bytes."""
    s = torch.cuda.current_stream()
    dims = (3, 5, 7, 11)
    links, psi = host_inputs(dims)
    fu, fin = device_inputs(dims, su3.SU3_F64, su3.SU3_F64, su3.SU3_LAYOUT_SOA, 0,
                            links, psi, s)
    fout = su3.spinor_tensor(dims, su3.SU3_F64, su3.SU3_LAYOUT_SOA, 0)
    fout.owner.fill_(0x5a)
    before_in = su3.su3_field_download_raw(fin, s)
    before_u = [su3.su3_field_download_raw(f, s) for f in fu]
    su3.su3_dslash(fout, fu, fin, s)
    su3.su3_sync(s)
    raw = su3.su3_field_download_raw(fout, s).view(np.float64)
    V, Vpad = 3 * 5 * 7 * 11, (3 * 5 * 7 * 11 + 63) // 64 * 64
    planes = raw.reshape(12, Vpad, 2)
    assert np.all(planes[:, V:, :].view(np.uint8) == 0x5a)
    assert np.array_equal(before_in, su3.su3_field_download_raw(fin, s))
    for f, b in zip(fu, before_u):
        assert np.array_equal(b, su3.su3_field_download_raw(f, s))


def test_dslash_rules():
    s = torch.cuda.current_stream()
    d = (2, 3, 2, 3)
    u64 = [su3.field_tensor(d, su3.SU3_F64, su3.SU3_LAYOUT_SOA) for _ in range(4)]
    u16 = [su3.field_tensor(d, su3.SU3_F16_F32ACC, su3.SU3_LAYOUT_SOA) for _ in range(4)]
    c12 = [su3.field_tensor(d, su3.SU3_C12_F32, su3.SU3_LAYOUT_SOA) for _ in range(4)]
    a = su3.spinor_tensor(d, su3.SU3_F64, su3.SU3_LAYOUT_SOA)
    b = su3.spinor_tensor(d, su3.SU3_F64, su3.SU3_LAYOUT_SOA)
    f32 = su3.spinor_tensor(d, su3.SU3_F32, su3.SU3_LAYOUT_SOA)
    aos = su3.spinor_tensor(d, su3.SU3_F64, su3.SU3_LAYOUT_AOS)
    other = su3.spinor_tensor((2, 3, 2, 4), su3.SU3_F64, su3.SU3_LAYOUT_SOA)
    m = su3.field_tensor(d, su3.SU3_F64, su3.SU3_LAYOUT_SOA)
    cases = [
        ((a, u64, a), su3.SU3_ERR_ALIAS),
        ((a, u64, f32), su3.SU3_ERR_MISMATCH),
        ((a, u64, aos), su3.SU3_ERR_MISMATCH),
        ((a, u64, other), su3.SU3_ERR_MISMATCH),
        ((a, u64, m), su3.SU3_ERR_MISMATCH),
        ((a, u16, b), su3.SU3_ERR_UNSUPPORTED),
        ((a, c12, b), su3.SU3_ERR_UNSUPPORTED),
        ((f32, u64, f32), su3.SU3_ERR_UNSUPPORTED),
        ((a, [u64[0], u64[1], c12[2], u64[3]], b), su3.SU3_ERR_MISMATCH),
    ]
    for (out, links, inp), want in cases:
        with pytest.raises(su3.Su3Error) as e:
            su3.su3_dslash(out, links, inp, s)
        assert e.value.status == want, e.value
    # a spinor field is not a matrix operand
    with pytest.raises(su3.Su3Error) as e:
        su3.su3_mult(m, a, b, s)
    assert e.value.status == su3.SU3_ERR_MISMATCH
    # an output sharing memory with a link field
    t = torch.zeros(su3.su3_spinor_bytes(d, su3.SU3_F64, su3.SU3_LAYOUT_SOA),
                    dtype=torch.uint8, device="cuda")
    link0 = su3.su3_field_wrap(t, d, su3.SU3_F64, su3.SU3_LAYOUT_SOA)
    out = su3.su3_spinor_wrap(t, d, su3.SU3_F64, su3.SU3_LAYOUT_SOA)
    with pytest.raises(su3.Su3Error) as e:
        su3.su3_dslash(out, [link0] + u64[1:], b, s)
    assert e.value.status == su3.SU3_ERR_ALIAS
    su3.su3_dslash(a, u64, b, s)
    su3.su3_sync(s)


def test_dslash_gamma5_hermiticity_on_device():
    """gamma5 D gamma5 = D^dagger, through two device applications:
    <chi, D psi> == conj(<psi, g5 D g5 chi>), in double precision, with
    g5 = diag(1, 1, -1, -1) in spin (its sign cancels)."""
    s = torch.cuda.current_stream()
    dims = (4, 6, 2, 10)
    V = testgen.volume(dims)
    links, psi = host_inputs(dims)
    chi = testgen.spinor_field(V, field_id=FID_SPINOR + 1)
    g5 = np.array([1.0, 1.0, -1.0, -1.0])[None, :, None, None]  # chiral basis
    fu, fin = device_inputs(dims, su3.SU3_F64, su3.SU3_F64, su3.SU3_LAYOUT_AOSOA, 16,
                            links, psi, s)
    fchi = su3.spinor_tensor(dims, su3.SU3_F64, su3.SU3_LAYOUT_AOSOA, 16)
    su3.su3_field_upload(fchi, g5 * chi, s)
    out = su3.spinor_tensor(dims, su3.SU3_F64, su3.SU3_LAYOUT_AOSOA, 16)
    su3.su3_dslash(out, fu, fin, s)
    dpsi = su3.su3_field_download(out, s)
    su3.su3_dslash(out, fu, fchi, s)
    dchi = g5 * su3.su3_field_download(out, s)

    def cplx(a):
        return a[..., 0] + 1j * a[..., 1]
    lhs = np.vdot(cplx(chi).ravel(), cplx(dpsi).ravel())
    rhs = np.conj(np.vdot(cplx(psi).ravel(), cplx(dchi).ravel()))
    assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs)), (lhs, rhs)


FULL = (48, 48, 48, 48)


def test_dslash_full_48_tuned():
    """48^4 in the tuned launch for each precision pair, on SoA and
    AoSoA(64) fields; every site compared with the oracle."""
    s = torch.cuda.current_stream()
    links, psi = host_inputs(FULL)
    for sp, lp in PAIRS:
        want, mag = reference(sp, lp, links, psi, FULL)
        for lay, lanes in ((su3.SU3_LAYOUT_SOA, 0), (su3.SU3_LAYOUT_AOSOA, 64)):
            cfg = su3.su3_autotune(su3.SU3_EXPR_DSLASH, lp, lay, lanes, FULL, s)
            fu, fin = device_inputs(FULL, sp, lp, lay, lanes, links, psi, s)
            fout = su3.spinor_tensor(FULL, sp, lay, lanes)
            su3.su3_dslash(fout, fu, fin, s)
            su3.su3_sync(s)
            got = su3.su3_field_download(fout, s)
            del fu, fin, fout
            torch.cuda.empty_cache()
            worst = assert_dslash(sp, lp, got, want, mag,
                                  f"48^4 {sp}/{lp} layout {lay} {cfg.as_dict()}")
            print(f"48^4 dslash spinor {sp} links {lp} layout {lay}: worst {worst:.3e} "
                  f"launch {cfg.as_dict()}")


@pytest.mark.parametrize("pair", PAIRS, ids=PAIR_IDS)
def test_dslash_persistent_spans(pair):
    """LDS-tiled walks with k workgroups per CU, each walking an equal share
    of the (tile, t-slice) pairs: at 16x16x16x40 there are more pairs than
    workgroups and the shares (not divisors of 40) continue from one tile
    into the next.  Parity with the oracle, bit-identical to the default
    launch."""
    sp, lp = pair
    s = torch.cuda.current_stream()
    dims = (16, 16, 16, 40)
    links, psi = host_inputs(dims)
    want, mag = reference(sp, lp, links, psi, dims)
    lay, lanes = su3.SU3_LAYOUT_SOA, 0
    fu, fin = device_inputs(dims, sp, lp, lay, lanes, links, psi, s)
    fout = su3.spinor_tensor(dims, sp, lay, lanes)
    su3.su3_launch_reset()
    su3.su3_dslash(fout, fu, fin, s)
    su3.su3_sync(s)
    base = su3.su3_field_download(fout, s)
    assert_dslash(sp, lp, base, want, mag, "default launch")
    for sched in (8, 11, 12, 16, 17):
        for k in (1, 2, 3):
            cfg = dict(block=256, persistent=k, nontemporal=2, xcd_remap=k & 1,
                       lds_stage=0, tile_sites=1, occupancy=0, schedule=sched)
            su3.su3_launch_set(su3.SU3_EXPR_DSLASH, lp, lay, lanes, dims, cfg)
            try:
                fout.owner.zero_()
                su3.su3_dslash(fout, fu, fin, s)
            finally:
                su3.su3_launch_reset()
            su3.su3_sync(s)
            got = su3.su3_field_download(fout, s)
            assert np.array_equal(got, base), f"schedule {sched} persistent {k}"


@pytest.mark.parametrize("dims,pair", [((160, 2, 2, 4), (su3.SU3_F64, su3.SU3_F64)),
                                       ((100, 2, 3, 4), (su3.SU3_F64, su3.SU3_F64)),
                                       ((300, 2, 2, 2), (su3.SU3_F32, su3.SU3_F32)),
                                       ((64, 4, 4, 4), (su3.SU3_F32, su3.SU3_C12_F32))],
                         ids=["f64_rows_too_long", "f64_rows_of_2x2", "f32_rows_too_long",
                              "f32c12_one_buffer"])
def test_dslash_default_fallbacks(dims, pair):
    """The default launch takes whole x rows; rows too long for a workgroup
    (or two buffers too large for the LDS) fall back to the rows with one
    buffer, to Lx x 2 x 2 or to 16 x 4 x 4 tiles: still the hopping term."""
    sp, lp = pair
    s = torch.cuda.current_stream()
    links, psi = host_inputs(dims)
    want, mag = reference(sp, lp, links, psi, dims)
    fu, fin = device_inputs(dims, sp, lp, su3.SU3_LAYOUT_SOA, 0, links, psi, s)
    fout = su3.spinor_tensor(dims, sp, su3.SU3_LAYOUT_SOA)
    su3.su3_launch_reset()
    su3.su3_dslash(fout, fu, fin, s)
    su3.su3_sync(s)
    assert_dslash(sp, lp, su3.su3_field_download(fout, s), want, mag, f"{dims}")


SHARD = (48, 48, 48, 6)


def test_dslash_shard_tuned():
    """One t-slab of a 48^4 lattice cut into 8 (48^3 x 6, periodic in t)
    in the tuned FP64 launch; every site compared with the oracle."""
    s = torch.cuda.current_stream()
    links, psi = host_inputs(SHARD)
    sp = lp = su3.SU3_F64
    cfg = su3.su3_autotune(su3.SU3_EXPR_DSLASH, lp, su3.SU3_LAYOUT_SOA, 0, SHARD, s)
    fu, fin = device_inputs(SHARD, sp, lp, su3.SU3_LAYOUT_SOA, 0, links, psi, s)
    fout = su3.spinor_tensor(SHARD, sp, su3.SU3_LAYOUT_SOA)
    su3.su3_dslash(fout, fu, fin, s)
    su3.su3_sync(s)
    got = su3.su3_field_download(fout, s)
    del fu, fin, fout
    torch.cuda.empty_cache()
    want, mag = reference(sp, lp, links, psi, SHARD)
    assert_dslash(sp, lp, got, want, mag, f"48^3x6 {cfg.as_dict()}")
