"""Grid's virtual-node layout on the GPU: the stored image equals the
oracle's virtual-node walk byte for byte (matrices in every precision,
spinors), Grid-layout data written by the host is used in place with no
repacking, and products, fused expressions, shifts, Dslash and batches on
virtual-node fields agree with the oracle (shifts bit-exact)."""
import numpy as np
import pytest
import torch

import oracle as O
import testgen
import paper_1710_09409_amd as su3
from gpu_util import PREC_NAMES, PRECS, assert_parity, exprs_for

pytestmark = pytest.mark.gpu

CASES = [((4, 2, 6, 4), (2, 1, 2, 2)), ((3, 5, 7, 2), (1, 1, 1, 2)),
         ((8, 8, 8, 8), (2, 2, 2, 2)), ((8, 4, 8, 16), (1, 1, 4, 4)),
         ((16, 8, 8, 8), (4, 2, 2, 4)), ((2, 2, 2, 2), (1, 1, 1, 1))]
IDS = ["%s_%s" % ("x".join(map(str, d)), "".join(map(str, s))) for d, s in CASES]
M, SP = su3.SU3_KIND_MATRIX, su3.SU3_KIND_SPINOR


def vfield(dims, prec, simd, host, s, kind=M):
    f = su3.vnode_tensor(dims, prec, simd, kind)
    su3.su3_field_upload(f, host, s)
    return f


@pytest.mark.parametrize("dims,simd", CASES, ids=IDS)
@pytest.mark.parametrize("prec", PRECS, ids=[PREC_NAMES[p] for p in PRECS])
def test_vnode_image_and_expressions(dims, simd, prec):
    s = torch.cuda.current_stream()
    V = testgen.volume(dims)
    ops = [testgen.su3_field(V, field_id=70 + k) for k in range(4)]
    fs = [vfield(dims, prec, simd, h, s) for h in ops]
    for f, h in zip(fs, ops):
        assert np.array_equal(su3.su3_field_download_raw(f, s),
                              O.get().vnode_pack(h, dims, simd, prec))
    z = su3.vnode_tensor(dims, prec, simd)
    for expr in exprs_for(prec):
        n = su3.N_OPERANDS[expr]
        su3.su3_fused_eval(z, expr, fs[:n], s)
        su3.su3_sync(s)
        got = su3.su3_field_download(z, s)
        want = O.get().reference(expr, prec, ops[:n])
        assert_parity(prec, expr, got, want, f"vnode {dims} {simd} expr {expr}")


@pytest.mark.parametrize("dims,simd", CASES, ids=IDS)
def test_vnode_no_repack(dims, simd):
    """Grid-layout bytes built on the host (the oracle's walk) are wrapped
    in place; the product's stored result is the oracle's walk of the
    expected product."""
    s = torch.cuda.current_stream()
    V = testgen.volume(dims)
    x, y = testgen.su3_field(V, field_id=80), testgen.su3_field(V, field_id=81)
    tx = torch.from_numpy(O.get().vnode_pack(x, dims, simd, su3.SU3_F64)).cuda()
    ty = torch.from_numpy(O.get().vnode_pack(y, dims, simd, su3.SU3_F64)).cuda()
    tz = torch.zeros_like(tx)
    fx = su3.su3_vnode_wrap(tx, dims, su3.SU3_F64, M, simd)
    fy = su3.su3_vnode_wrap(ty, dims, su3.SU3_F64, M, simd)
    fz = su3.su3_vnode_wrap(tz, dims, su3.SU3_F64, M, simd)
    su3.su3_mult(fz, fx, fy, s)
    su3.su3_sync(s)
    got = O.get().vnode_unpack(tz.cpu().numpy(), dims, simd, su3.SU3_F64)
    assert_parity(su3.SU3_F64, su3.SU3_EXPR_MUL, got, O.get().mult(x, y), "no repack")


@pytest.mark.parametrize("dims,simd", CASES, ids=IDS)
@pytest.mark.parametrize("prec", PRECS, ids=[PREC_NAMES[p] for p in PRECS])
def test_vnode_shifts(dims, simd, prec):
    s = torch.cuda.current_stream()
    V = testgen.volume(dims)
    x, y = testgen.su3_field(V, field_id=82), testgen.su3_field(V, field_id=83)
    qx, qy = O.get().roundtrip(prec, x), O.get().roundtrip(prec, y)
    fx, fy = vfield(dims, prec, simd, x, s), vfield(dims, prec, simd, y, s)
    fz = su3.vnode_tensor(dims, prec, simd)
    for mu in range(4):
        for k in (1, -1, 2, -3, dims[mu] + 1):
            want = O.get().cshift(qy, dims, mu, k)
            su3.su3_cshift(fz, fy, mu, k, s)
            assert np.array_equal(su3.su3_field_download(fz, s), want), (mu, k)
            su3.su3_mult_shifted(fz, fx, fy, mu, k, s)
            assert_parity(prec, su3.SU3_EXPR_MUL, su3.su3_field_download(fz, s),
                          O.get().mult(qx, want), f"vnode shifted mu {mu} k {k}")


@pytest.mark.parametrize("dims,simd", CASES, ids=IDS)
def test_vnode_dslash(dims, simd):
    from test_gpu_dslash import PAIRS, assert_dslash, reference
    s = torch.cuda.current_stream()
    V = testgen.volume(dims)
    links = [testgen.su3_field(V, field_id=testgen.FID_U0 + mu) for mu in range(4)]
    psi = testgen.spinor_field(V, field_id=201)
    for sp, lp in PAIRS:
        fu = [vfield(dims, lp, simd, u, s) for u in links]
        fin = vfield(dims, sp, simd, psi, s, SP)
        assert np.array_equal(su3.su3_field_download_raw(fin, s),
                              O.get().vnode_pack(psi, dims, simd, sp))
        fout = su3.vnode_tensor(dims, sp, simd, SP)
        want, mag = reference(sp, lp, links, psi, dims)
        # one site per lane, then row tiles of outer sites with all their
        # virtual nodes (one and two buffers, walks, persistent shares, XCD
        # slabs, rows of 3 x 3), then the default launch: all bit-identical
        nsub = int(np.prod(simd))
        first = None
        for cfg in (dict(block=64, schedule=0, tile_sites=1),
                    dict(block=256, schedule=9, tile_sites=2),
                    dict(block=256, schedule=12, tile_sites=4096, xcd_remap=1),
                    dict(block=256, schedule=13, tile_sites=3),
                    dict(block=256, schedule=16, tile_sites=1, persistent=2),
                    dict(block=256, schedule=11, tile_sites=1, xcd_remap=2),
                    dict(block=256, schedule=17, tile_sites=3),
                    dict(block=256, schedule=18, tile_sites=1, persistent=1, xcd_remap=1),
                    None):
            if cfg is not None:
                full = dict(dict(persistent=0, nontemporal=2, xcd_remap=0, lds_stage=0,
                                 occupancy=0), **cfg)
                su3.su3_launch_set(su3.SU3_EXPR_DSLASH, lp, su3.SU3_LAYOUT_VNODE, nsub,
                                   dims, full)
            try:
                su3.su3_dslash(fout, fu, fin, s)
            finally:
                su3.su3_launch_reset()
            su3.su3_sync(s)
            got = su3.su3_field_download(fout, s)
            if first is None:
                first = got
                assert_dslash(sp, lp, got, want, mag, f"vnode {dims} {simd} {sp}/{lp}")
            assert np.array_equal(got, first), f"vnode {dims} {simd} {sp}/{lp} {cfg}"


def test_vnode_batch():
    """Virtual-node items (N_sub >= 4) mixed with AoSoA and SoA items in
    one batch, each equal to its own unbatched evaluation."""
    s = torch.cuda.current_stream()
    items = [((8, 8, 8, 8), su3.SU3_F64, (2, 2, 2, 2)),
             ((8, 4, 8, 16), su3.SU3_C12_F32, (1, 1, 4, 4)),
             ((16, 8, 8, 8), su3.SU3_F64, (4, 2, 2, 4)),
             ((4, 4, 4, 4), su3.SU3_F32, None)]
    zs, refs, ops = [], [], []
    for i, (d, prec, simd) in enumerate(items):
        V = testgen.volume(d)
        hs = [testgen.su3_field(V, field_id=90 + 2 * i + k) for k in range(2)]
        if simd:
            fo = [vfield(d, prec, simd, h, s) for h in hs]
            zs.append(su3.vnode_tensor(d, prec, simd))
            refs.append(su3.vnode_tensor(d, prec, simd))
        else:
            fo = []
            for h in hs:
                f = su3.field_tensor(d, prec, su3.SU3_LAYOUT_AOSOA, 16)
                su3.su3_field_upload(f, h, s)
                fo.append(f)
            zs.append(su3.field_tensor(d, prec, su3.SU3_LAYOUT_AOSOA, 16))
            refs.append(su3.field_tensor(d, prec, su3.SU3_LAYOUT_AOSOA, 16))
        ops.append(fo)
        su3.su3_mult(refs[-1], fo[0], fo[1], s)
    b = su3.su3_batch_create([su3.SU3_EXPR_MUL] * len(items), zs, ops, s)
    for _ in range(2):
        su3.su3_batch_launch(b, s)
        su3.su3_sync(s)
        for z, r in zip(zs, refs):
            assert np.array_equal(su3.su3_field_download_raw(z, s),
                                  su3.su3_field_download_raw(r, s))
    su3.su3_batch_destroy(b)


def test_vnode_rules():
    s = torch.cuda.current_stream()
    d = (4, 4, 4, 4)
    a = su3.vnode_tensor(d, su3.SU3_F64, (2, 2, 1, 1))
    b = su3.vnode_tensor(d, su3.SU3_F64, (1, 1, 2, 2))
    c = su3.field_tensor(d, su3.SU3_F64, su3.SU3_LAYOUT_AOSOA, 8)
    for x, y in ((a, b), (a, c)):
        with pytest.raises(su3.Su3Error) as e:
            su3.su3_mult(a, x, y, s)
        assert e.value.status == su3.SU3_ERR_MISMATCH
    for simd in ((3, 1, 1, 1), (1, 1, 1, 0)):
        with pytest.raises(su3.Su3Error) as e:
            su3.su3_vnode_bytes(d, su3.SU3_F64, M, simd)
        assert e.value.status == su3.SU3_ERR_INVALID_ARG
    two = [su3.vnode_tensor(d, su3.SU3_F64, (2, 1, 1, 1)) for _ in range(3)]
    with pytest.raises(su3.Su3Error) as e:
        su3.su3_batch_create([su3.SU3_EXPR_MUL], [two[0]], [two[1:]], s)
    assert e.value.status == su3.SU3_ERR_UNSUPPORTED
    # tuning keys of the layout are N_sub
    cfg = su3.su3_autotune(su3.SU3_EXPR_MUL, su3.SU3_F64, su3.SU3_LAYOUT_VNODE, 16,
                           (8, 8, 8, 8), s)
    assert su3.su3_launch_get(su3.SU3_EXPR_MUL, su3.SU3_F64, su3.SU3_LAYOUT_VNODE, 16,
                              (8, 8, 8, 8)).as_dict() == cfg.as_dict()
    su3.su3_launch_reset()


def test_vnode_full_size_matches_soa():
    """48^4 in Grid's usual split of the two slowest directions (N_sub = 4):
    the product and the Wilson hopping term on virtual-node fields equal,
    bit for bit, the same operations on SoA fields (same arithmetic, other
    storage order)."""
    s = torch.cuda.current_stream()
    dims, simd = (48, 48, 48, 48), (1, 1, 2, 2)
    V = testgen.volume(dims)
    x = testgen.su3_field(V, field_id=testgen.FID_X)
    y = testgen.su3_field(V, field_id=testgen.FID_Y)
    fx = vfield(dims, su3.SU3_F64, simd, x, s)
    fy = vfield(dims, su3.SU3_F64, simd, y, s)
    fz = su3.vnode_tensor(dims, su3.SU3_F64, simd)
    su3.su3_mult(fz, fx, fy, s)
    got = su3.su3_field_download(fz, s)
    del fx, fy, fz
    gx = su3.field_tensor(dims, su3.SU3_F64, su3.SU3_LAYOUT_SOA)
    gy = su3.field_tensor(dims, su3.SU3_F64, su3.SU3_LAYOUT_SOA)
    gz = su3.field_tensor(dims, su3.SU3_F64, su3.SU3_LAYOUT_SOA)
    su3.su3_field_upload(gx, x, s)
    su3.su3_field_upload(gy, y, s)
    su3.su3_mult(gz, gx, gy, s)
    assert np.array_equal(got, su3.su3_field_download(gz, s))
    del gx, gy, gz, x, y
    torch.cuda.empty_cache()
    # Dslash at 32^4 (the SoA launch may be any kernel variant)
    dims = (32, 32, 32, 32)
    V = testgen.volume(dims)
    links = [testgen.su3_field(V, field_id=testgen.FID_U0 + mu) for mu in range(4)]
    psi = testgen.spinor_field(V, field_id=200)
    fu = [vfield(dims, su3.SU3_F64, simd, u, s) for u in links]
    fin = vfield(dims, su3.SU3_F64, simd, psi, s, SP)
    fout = su3.vnode_tensor(dims, su3.SU3_F64, simd, SP)
    su3.su3_dslash(fout, fu, fin, s)
    got = su3.su3_field_download(fout, s)
    del fu, fin, fout
    gu = []
    for u in links:
        f = su3.field_tensor(dims, su3.SU3_F64, su3.SU3_LAYOUT_SOA)
        su3.su3_field_upload(f, u, s)
        gu.append(f)
    gin = su3.spinor_tensor(dims, su3.SU3_F64, su3.SU3_LAYOUT_SOA)
    su3.su3_field_upload(gin, psi, s)
    gout = su3.spinor_tensor(dims, su3.SU3_F64, su3.SU3_LAYOUT_SOA)
    su3.su3_autotune(su3.SU3_EXPR_DSLASH, su3.SU3_F64, su3.SU3_LAYOUT_SOA, 0, dims, s)
    su3.su3_dslash(gout, gu, gin, s)
    assert np.array_equal(got, su3.su3_field_download(gout, s))
    su3.su3_launch_reset()


@pytest.mark.parametrize("simd", [(1, 1, 2, 2), (2, 2, 2, 2)], ids=["nsub4", "nsub16"])
def test_vnode_dslash_tuned(simd):
    """The autotuner's choice for the hopping term on virtual-node fields
    (row tiles of outer sites among the candidates) at 16^3 x 32 gives the
    one-site result bit for bit."""
    from test_gpu_dslash import assert_dslash, reference
    s = torch.cuda.current_stream()
    dims = (16, 16, 16, 32)
    V = testgen.volume(dims)
    nsub = int(np.prod(simd))
    links = [testgen.su3_field(V, field_id=testgen.FID_U0 + mu) for mu in range(4)]
    psi = testgen.spinor_field(V, field_id=202)
    fu = [vfield(dims, su3.SU3_F64, simd, u, s) for u in links]
    fin = vfield(dims, su3.SU3_F64, simd, psi, s, SP)
    fout = su3.vnode_tensor(dims, su3.SU3_F64, simd, SP)
    one = dict(block=64, persistent=0, nontemporal=2, xcd_remap=0, lds_stage=0,
               tile_sites=1, occupancy=0, schedule=0)
    su3.su3_launch_set(su3.SU3_EXPR_DSLASH, su3.SU3_F64, su3.SU3_LAYOUT_VNODE, nsub, dims, one)
    su3.su3_dslash(fout, fu, fin, s)
    su3.su3_sync(s)
    base = su3.su3_field_download(fout, s)
    want, mag = reference(su3.SU3_F64, su3.SU3_F64, links, psi, dims)
    assert_dslash(su3.SU3_F64, su3.SU3_F64, base, want, mag, f"vnode {simd} one site")
    try:
        cfg = su3.su3_autotune(su3.SU3_EXPR_DSLASH, su3.SU3_F64, su3.SU3_LAYOUT_VNODE, nsub,
                               dims, s)
        fout.owner.zero_()
        su3.su3_dslash(fout, fu, fin, s)
        su3.su3_sync(s)
        got = su3.su3_field_download(fout, s)
    finally:
        su3.su3_launch_reset()
    print(f"vnode {simd} tuned: {cfg.as_dict()}")
    assert np.array_equal(got, base), cfg.as_dict()


def test_vnode_dslash_full_48_tuned():
    """48^4 in the tuned launches the benchmark times: the hopping term on
    virtual-node fields (N_sub = 4 and 16) equals, bit for bit, the tuned
    hopping term on SoA fields (every kernel accumulates in one order)."""
    s = torch.cuda.current_stream()
    dims = (48, 48, 48, 48)
    V = testgen.volume(dims)
    links = [testgen.su3_field(V, field_id=testgen.FID_U0 + mu) for mu in range(4)]
    psi = testgen.spinor_field(V, field_id=203)
    gu = []
    for u in links:
        f = su3.field_tensor(dims, su3.SU3_F64, su3.SU3_LAYOUT_SOA)
        su3.su3_field_upload(f, u, s)
        gu.append(f)
    gin = su3.spinor_tensor(dims, su3.SU3_F64, su3.SU3_LAYOUT_SOA)
    su3.su3_field_upload(gin, psi, s)
    gout = su3.spinor_tensor(dims, su3.SU3_F64, su3.SU3_LAYOUT_SOA)
    try:
        su3.su3_autotune(su3.SU3_EXPR_DSLASH, su3.SU3_F64, su3.SU3_LAYOUT_SOA, 0, dims, s)
        su3.su3_dslash(gout, gu, gin, s)
        su3.su3_sync(s)
        want = su3.su3_field_download(gout, s)
        del gu, gin, gout
        torch.cuda.empty_cache()
        for simd in ((1, 1, 2, 2), (2, 2, 2, 2)):
            nsub = int(np.prod(simd))
            fu = [vfield(dims, su3.SU3_F64, simd, u, s) for u in links]
            fin = vfield(dims, su3.SU3_F64, simd, psi, s, SP)
            fout = su3.vnode_tensor(dims, su3.SU3_F64, simd, SP)
            cfg = su3.su3_autotune(su3.SU3_EXPR_DSLASH, su3.SU3_F64, su3.SU3_LAYOUT_VNODE,
                                   nsub, dims, s)
            su3.su3_dslash(fout, fu, fin, s)
            su3.su3_sync(s)
            got = su3.su3_field_download(fout, s)
            del fu, fin, fout
            torch.cuda.empty_cache()
            assert np.array_equal(got, want), f"{simd} {cfg.as_dict()}"
    finally:
        su3.su3_launch_reset()
