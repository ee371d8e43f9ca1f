"""Pins of the FP64 oracle against facts fixed by mathematics, by library
routines or by the worked example of the paper -- never by the oracle
itself.

Each pin takes an ``oracle.Oracle`` and raises AssertionError when the
oracle is wrong.  ``test_oracle_pins`` runs them on the real oracle;
``test_oracle_mutants`` runs them on copies with planted mistakes and
requires every mistake to be caught.
"""
from __future__ import annotations

import itertools
import os

import numpy as np

import oracle as O
import testgen

U64 = 2.0 ** -53
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def to_complex(a):
    a = np.asarray(a)
    return a[..., 0] + 1j * a[..., 1]


def from_complex(c):
    c = np.asarray(c)
    return np.stack([c.real, c.imag], axis=-1).astype(np.float64)


def read_golden_rows(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append([int(x) if i < 2 else float(x)
                             for i, x in enumerate(line.split())])
    return rows


def read_golden(name):
    vals = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, v = line.split()
            vals[k] = float(v)
    return vals


# ------------------------------------------------------------ O1 product

def pin_identity(orc):
    """I*y = y and x*I = x bit-exactly (1*a and 0*b are exact; adding a
    signed zero to a nonzero value is exact)."""
    V = 97
    x = testgen.su3_field(V, field_id=11)
    eye = testgen.identity(V)
    assert np.array_equal(orc.mult(eye, x), x)
    assert np.array_equal(orc.mult(x, eye), x)


def pin_phase_diag(orc):
    """Closed form: diag(e^{ia}, e^{ib}, e^{-i(a+b)}) products are diagonal
    with summed phases."""
    rng = np.random.default_rng(5)
    V = 64
    a1, b1, a2, b2 = (rng.uniform(-np.pi, np.pi, V) for _ in range(4))
    z = orc.mult(testgen.phase_diag(a1, b1), testgen.phase_diag(a2, b2))
    want = testgen.phase_diag(a1 + a2, b1 + b2)
    assert np.max(np.abs(z - want)) <= 8 * U64


def pin_signed_permutations(orc):
    """The 24 signed permutation matrices with det 1 form a group; every
    product is exact and equals the integer matrix product."""
    mats = testgen.signed_permutations()
    assert len(mats) == 24
    pairs = list(itertools.product(range(24), repeat=2))
    x = testgen.from_int_matrices([mats[i] for i, _ in pairs])
    y = testgen.from_int_matrices([mats[j] for _, j in pairs])
    want = testgen.from_int_matrices([mats[i] @ mats[j] for i, j in pairs])
    assert np.array_equal(orc.mult(x, y), want)


def pin_unitary_inverse(orc):
    """x * x^dagger = I within a few ulps for x in SU(3)."""
    V = 256
    x = testgen.su3_field(V, field_id=12)
    xd = from_complex(np.conj(np.transpose(to_complex(x), (0, 2, 1))))
    z = orc.mult(x, xd)
    assert np.max(np.abs(z - testgen.identity(V))) <= 8 * U64


def pin_numpy_matmul(orc):
    """Brute force on 1^4 and 2^4 lattices (and a 3^4 one) against a
    pure-Python triple loop on complex numbers and numpy.matmul on
    complex128."""
    for V, fx, fy in ((1, 13, 14), (16, 15, 16), (81, 17, 18)):
        x = testgen.su3_field(V, field_id=fx)
        y = testgen.su3_field(V, field_id=fy)
        z = to_complex(orc.mult(x, y))
        xc, yc = to_complex(x), to_complex(y)
        assert np.max(np.abs(z - np.matmul(xc, yc))) <= 4 * U64
        if V <= 16:
            for s in range(V):
                for i in range(3):
                    for j in range(3):
                        acc = 0j
                        for k in range(3):
                            acc += complex(xc[s, i, k]) * complex(yc[s, k, j])
                        assert abs(z[s, i, j] - acc) <= 4 * U64


def pin_nonsymmetric(orc):
    """Integer-valued, non-symmetric, non-unitary matrices: every product
    is exact, so a transposed operand or a lost term shows as a mismatch."""
    rng = np.random.default_rng(7)
    V = 200
    xr, xi, yr, yi = (rng.integers(-9, 10, (V, 3, 3)) for _ in range(4))
    x = np.stack([xr, xi], -1).astype(np.float64)
    y = np.stack([yr, yi], -1).astype(np.float64)
    want = np.matmul(xr + 1j * xi, yr + 1j * yi)
    assert np.array_equal(to_complex(orc.mult(x, y)), want)


def pin_product_invariants(orc):
    """SU(3) x SU(3) stays in SU(3): unitarity and det = 1 (checked with
    numpy, independent of the oracle's metrics)."""
    V = 512
    z = to_complex(orc.mult(testgen.su3_field(V, field_id=19),
                            testgen.su3_field(V, field_id=20)))
    zzd = np.matmul(z, np.conj(np.transpose(z, (0, 2, 1))))
    assert np.max(np.abs(zzd - np.eye(3))) <= 8e-15
    assert np.max(np.abs(np.linalg.det(z) - 1.0)) <= 8e-15


def pin_associative(orc):
    V = 256
    x, y, w = (testgen.su3_field(V, field_id=f) for f in (21, 22, 23))
    lhs = orc.mult(orc.mult(x, y), w)
    rhs = orc.mult(x, orc.mult(y, w))
    assert np.max(np.abs(lhs - rhs)) <= 3e-15


# --------------------------------------------------------- O2 fused

def pin_constant_fields_fused(orc):
    """The sum and the sum-plus-product of the constant SU(3)-typed fields
    1*I and 2*I (the inputs of Section 3's composite-expression example,
    Listing 2) are exactly 3*I and 5*I."""
    g = read_golden("composite_constants.txt")
    V = 8
    a = testgen.identity(V, g["a"])
    b = testgen.identity(V, g["b"])
    assert np.array_equal(orc.fused(O.ADD, [a, b]), testgen.identity(V, g["ADD"]))
    assert np.array_equal(orc.fused(O.APB_AB, [a, b]),
                          testgen.identity(V, g["APB_AB"]))


def pin_fused_reductions(orc):
    """MUL3(a, I, c) = MUL(a, c) and MULADD(a, b, 0, 0) = MUL(a, b)
    bit-exactly; MUL equals the product."""
    V = 128
    a, b, c = (testgen.su3_field(V, field_id=f) for f in (24, 25, 26))
    eye, zero = testgen.identity(V), np.zeros_like(a)
    ac = orc.mult(a, c)
    assert np.array_equal(orc.fused(O.MUL3, [a, eye, c]), ac)
    assert np.array_equal(orc.fused(O.MULADD, [a, c, zero, zero]), ac)
    assert np.array_equal(orc.fused(O.MUL, [a, c]), ac)


def pin_fused_numpy(orc):
    """Each expression against numpy on complex128 (integer-valued inputs,
    so every result is exact)."""
    rng = np.random.default_rng(8)
    V = 100
    ops = [rng.integers(-5, 6, (V, 3, 3, 2)).astype(np.float64)
           for _ in range(4)]
    a, b, c, d = (to_complex(o) for o in ops)
    want = {O.MUL: a @ b, O.MUL3: (a @ b) @ c, O.MULADD: a @ b + c @ d,
            O.ADD: a + b, O.APB_AB: (a + b) + a @ b}
    for expr, w in want.items():
        got = orc.fused(expr, ops[:O.N_OPERANDS[expr]])
        assert np.array_equal(to_complex(got), w), expr


def pin_fused_unitary(orc):
    V = 256
    a, b, c = (testgen.su3_field(V, field_id=f) for f in (27, 28, 29))
    z = to_complex(orc.fused(O.MUL3, [a, b, c]))
    zzd = np.matmul(z, np.conj(np.transpose(z, (0, 2, 1))))
    assert np.max(np.abs(zzd - np.eye(3))) <= 1.2e-14
    assert np.max(np.abs(np.linalg.det(z) - 1.0)) <= 1.2e-14


# ---------------------------------------------- O3 quantisers and layouts

def special_reals():
    f16max = 65504.0
    vals = [0.0, -0.0, 1.0, -1.0, 0.5, 1.0 / 3.0, 2.0 ** -14, 2.0 ** -24,
            2.0 ** -25, 1.5 * 2.0 ** -25, 2.0 ** -26, 3 * 2.0 ** -25,
            2.0 ** -24 * 1.5, 2.0 ** -24 * 2.5, f16max, 65519.0, 65520.0,
            65536.0, 1e6, 1e-10, 2.0 ** -149, 2.0 ** -126, 1e39, -1e39,
            np.inf, -np.inf, 1 + 2.0 ** -11, 1 + 3 * 2.0 ** -11,
            1 + 2.0 ** -11 + 2.0 ** -30, 2049.0, 2051.0, 4097.0]
    # ties and near-ties in float -> half at several binades
    for e in range(-24, 16):
        for m in (1025, 1027, 2047):
            v = m * 2.0 ** (e - 11)
            vals += [v, -v, np.nextafter(v, 0), np.nextafter(v, np.inf)]
    return np.array(vals, dtype=np.float64)


def pin_quantisers(orc):
    """double->float and double->float->half are bit-exact against numpy's
    round-to-nearest-even conversions; half->double is exact."""
    rng = np.random.default_rng(9)
    v = np.concatenate([special_reals(),
                        rng.standard_normal(20000),
                        rng.standard_normal(20000) * 10.0 ** rng.integers(-9, 6, 20000)])
    f = orc.quant_f32(v)
    assert np.array_equal(f.view(np.uint32), v.astype(np.float32).view(np.uint32))
    h = orc.quant_f16(v)
    want = v.astype(np.float32).astype(np.float16)
    assert np.array_equal(h, want.view(np.uint16))
    back = orc.dequant_f16(h)
    assert np.array_equal(back, want.astype(np.float64))
    # every half bit pattern except NaNs widens exactly
    allh = np.arange(65536, dtype=np.uint16)
    ref = allh.view(np.float16).astype(np.float64)
    got = orc.dequant_f16(allh)
    ok = ~np.isnan(ref)
    assert np.array_equal(got[ok], ref[ok])
    assert np.all(np.isnan(got[~ok]))


def pin_c12_rebuild(orc):
    """Row 2 rebuilt as conj(row0 x row1) against numpy.cross; on SU(3)
    input the rebuilt matrix equals the original."""
    V = 300
    rng = np.random.default_rng(10)
    m = rng.standard_normal((V, 3, 3, 2))
    got = to_complex(orc.c12_rebuild(m))
    mc = to_complex(m)
    want_row2 = np.conj(np.cross(mc[:, 0, :], mc[:, 1, :]))
    assert np.max(np.abs(got[:, 2, :] - want_row2)) <= 1e-13 * np.max(np.abs(want_row2))
    assert np.array_equal(got[:, :2, :], mc[:, :2, :])
    u = testgen.su3_field(V, field_id=30)
    assert np.max(np.abs(orc.c12_rebuild(u) - u)) <= 4 * U64


def _stored_numpy(a, prec, layout, lanes):
    """Stored image built with numpy reshapes: the entry axis is moved
    outside the site-in-block axis, padding sites are zero."""
    V = a.shape[0]
    E = 6 if prec == O.C12 else 9
    ent = a.reshape(V, 9, 2)[:, :E, :]
    if layout == O.AOS:
        L, Vpad = 1, V
    elif layout == O.SOA:
        Vpad = -(-V // 64) * 64
        L = Vpad
    else:
        L, Vpad = lanes, -(-V // lanes) * lanes
    padded = np.zeros((Vpad, E, 2))
    padded[:V] = ent
    img = padded.reshape(Vpad // L, L, E, 2).transpose(0, 2, 1, 3).reshape(-1)
    if prec == O.F64:
        return img.view(np.uint8)
    if prec == O.F16:
        return img.astype(np.float32).astype(np.float16).view(np.uint8)
    return img.astype(np.float32).view(np.uint8)


LAYOUT_CASES = [(O.AOS, 0), (O.SOA, 0), (O.AOSOA, 8), (O.AOSOA, 16),
                (O.AOSOA, 32), (O.AOSOA, 64)]


def pin_layouts(orc):
    """Stored images equal numpy's reshape/transpose construction for every
    precision and layout, including ragged volumes; unpack inverts pack
    (exactly for double)."""
    for V in (1, 5, 64, 77, 130):
        x = testgen.su3_field(V, field_id=31)
        for prec in (O.F64, O.F32, O.F16, O.C12):
            for layout, lanes in LAYOUT_CASES:
                img = orc.pack(x, prec, layout, lanes)
                want = _stored_numpy(x, prec, layout, lanes)
                assert img.size == want.size == orc.field_bytes(prec, layout, lanes, V)
                assert np.array_equal(img, want), (V, prec, layout, lanes)
                back = orc.unpack(img, V, prec, layout, lanes)
                assert np.array_equal(back, orc.roundtrip(prec, x)), (V, prec, layout)
        assert np.array_equal(orc.unpack(orc.pack(x, O.F64, O.SOA), V, O.F64, O.SOA), x)


def pin_roundtrip(orc):
    V = 50
    x = testgen.su3_field(V, field_id=32)
    assert np.array_equal(orc.roundtrip(O.F64, x), x)
    assert np.array_equal(orc.roundtrip(O.F32, x),
                          x.astype(np.float32).astype(np.float64))
    assert np.array_equal(orc.roundtrip(O.F16, x),
                          x.astype(np.float32).astype(np.float16).astype(np.float64))
    r = orc.roundtrip(O.C12, x)
    xc = to_complex(x.astype(np.float32).astype(np.float64))
    assert np.array_equal(to_complex(r)[:, :2], xc[:, :2])
    assert np.max(np.abs(to_complex(r)[:, 2] -
                         np.conj(np.cross(xc[:, 0], xc[:, 1])))) <= 1e-15


# ------------------------------------------------------------ O5 metrics

def pin_metrics(orc):
    """Closed-form values: 2I has |2I (2I)^dagger - I| = 3 and det 8; a
    single perturbed entry gives the expected absolute and relative
    error."""
    V = 4
    m = orc.metrics(testgen.identity(V, 2.0))
    assert m["d_u"] == 3.0 and m["d_det"] == 7.0
    u = testgen.su3_field(V, field_id=33)
    m0 = orc.metrics(u, u)
    assert m0["e_max"] == 0.0 and m0["r_max"] == 0.0
    assert m0["d_u"] < 1e-15 and m0["d_det"] < 1e-15
    p = u.copy()
    p[2, 1, 2, 1] += 1e-3
    m1 = orc.metrics(p, u)
    assert abs(m1["e_max"] - 1e-3) < 1e-15
    den = np.max(np.abs(to_complex(u[2])))
    assert abs(m1["r_max"] - 1e-3 / den) < 1e-12
    # diag(i, i, -1): unitary with det = i*i*(-1) = 1
    dph = testgen.phase_diag(np.full(V, np.pi / 2), np.full(V, np.pi / 2))
    m2 = orc.metrics(dph)
    assert m2["d_u"] < 1e-15 and m2["d_det"] < 1e-15
    # diag(i, 1, 1): unitary, det = i -> |i - 1| = sqrt 2
    q = testgen.identity(V)
    q[:, 0, 0] = (0.0, 1.0)
    m3 = orc.metrics(q)
    assert m3["d_u"] < 1e-15 and abs(m3["d_det"] - np.sqrt(2.0)) < 1e-15


# ------------------------------------------------------- shifted fields

def _coord_field(dims):
    """A field whose site (x,y,z,t) holds the diagonal matrix
    diag(x, y, z) + i t: each coordinate readable from the value."""
    V = int(np.prod(dims))
    f = np.zeros((V, 3, 3, 2))
    idx = np.arange(V)
    x = idx % dims[0]
    y = (idx // dims[0]) % dims[1]
    z = (idx // (dims[0] * dims[1])) % dims[2]
    t = idx // (dims[0] * dims[1] * dims[2])
    f[:, 0, 0, 0], f[:, 1, 1, 0], f[:, 2, 2, 0] = x, y, z
    f[:, 0, 0, 1] = t
    return f, (x, y, z, t)


def pin_cshift(orc):
    """Shifting a coordinate-valued field by k along mu reads the value of
    the site whose mu coordinate is (c_mu + k) mod L_mu (closed form);
    shifting by L_mu is the identity; +k then -k is the identity; shifts in
    different directions commute (numpy.roll along the lattice axes as a
    library check)."""
    dims = (3, 4, 5, 2)
    f, coords = _coord_field(dims)
    for mu in range(4):
        for k in (1, -1, 2, dims[mu], -3):
            g = orc.cshift(f, dims, mu, k)
            want = [c.copy() for c in coords]
            want[mu] = (coords[mu] + k) % dims[mu]
            assert np.array_equal(g[:, 0, 0, 0], want[0]), (mu, k)
            assert np.array_equal(g[:, 1, 1, 0], want[1]), (mu, k)
            assert np.array_equal(g[:, 2, 2, 0], want[2]), (mu, k)
            assert np.array_equal(g[:, 0, 0, 1], want[3]), (mu, k)
    u = testgen.su3_field(int(np.prod(dims)), field_id=34)
    assert np.array_equal(orc.cshift(u, dims, 2, dims[2]), u)
    assert np.array_equal(orc.cshift(orc.cshift(u, dims, 1, 1), dims, 1, -1), u)
    a = orc.cshift(orc.cshift(u, dims, 0, 1), dims, 3, -1)
    b = orc.cshift(orc.cshift(u, dims, 3, -1), dims, 0, 1)
    assert np.array_equal(a, b)
    # numpy.roll on the (t, z, y, x) array: shift by +k reads c + k
    arr = u.reshape(dims[3], dims[2], dims[1], dims[0], 3, 3, 2)
    for mu in range(4):
        want = np.roll(arr, -1, axis=3 - mu).reshape(u.shape)
        assert np.array_equal(orc.cshift(u, dims, mu, 1), want), mu


# ---------------------------------------------------------- Wilson hopping

def _plane_wave(dims, p, spin, colour=0):
    """psi(x) = exp(i p.x) e_spin (x) e_colour, shape (V, 4, 3, 2)."""
    V = int(np.prod(dims))
    idx = np.arange(V)
    c = [idx % dims[0], (idx // dims[0]) % dims[1],
         (idx // (dims[0] * dims[1])) % dims[2], idx // (dims[0] * dims[1] * dims[2])]
    ph = sum(p[m] * c[m] for m in range(4))
    psi = np.zeros((V, 4, 3, 2))
    psi[:, spin, colour, 0] = np.cos(ph)
    psi[:, spin, colour, 1] = np.sin(ph)
    return psi, ph


def free_spin_matrix(orc, dims, p):
    """M(p) with (D psi)(x) = exp(i p.x) M(p) chi for psi = exp(i p.x) chi
    on the unit gauge field; also checks that D maps each plane wave to a
    plane wave of the same momentum (translation invariance)."""
    V = int(np.prod(dims))
    unit = [testgen.identity(V) for _ in range(4)]
    M = np.zeros((4, 4), dtype=complex)
    for sp in range(4):
        psi, ph = _plane_wave(dims, p, sp)
        out = orc.dslash(unit, psi, dims)
        outc = out[..., 0] + 1j * out[..., 1]           # (V, 4, 3)
        col = outc * np.exp(-1j * ph)[:, None, None]    # remove the phase
        assert np.max(np.abs(col - col[0])) < 1e-12     # same at every site
        assert np.max(np.abs(col[0][:, 1:])) < 1e-14    # colour untouched
        M[:, sp] = col[0][:, 0]
    return M


def oracle_gammas(orc, dims=(4, 4, 4, 4)):
    """gamma_mu read off the oracle: with momentum pi/2 along mu only,
    M = 2 cos(pi/2) + 6 - 2i sin(pi/2) gamma_mu = 6 - 2i gamma_mu."""
    g = []
    for mu in range(4):
        p = [0.0] * 4
        p[mu] = 2 * np.pi / dims[mu]  # = pi/2 on an extent of 4
        M = free_spin_matrix(orc, dims, p)
        g.append((6 * np.eye(4) - M) / 2j)
    return g


def pin_dslash_free_field(orc):
    """Clifford algebra {g_mu, g_nu} = 2 delta, hermiticity, and the free
    spin matrix M(p) = sum_mu (2 cos p_mu - 2i sin p_mu g_mu) at generic
    momenta on a 4x6x3x5 lattice; the basis is the declared one."""
    g = oracle_gammas(orc)
    for a in range(4):
        assert np.allclose(g[a], g[a].conj().T, atol=1e-12)
        for b in range(4):
            anti = g[a] @ g[b] + g[b] @ g[a]
            assert np.allclose(anti, 2 * np.eye(4) * (a == b), atol=1e-12), (a, b)
    vals = read_golden_rows("chiral_gamma.txt")
    for mu in range(4):
        want = np.array([[complex(r[2 + 2 * c], r[3 + 2 * c]) for c in range(4)]
                         for r in vals if r[0] == mu])
        assert np.allclose(g[mu], want, atol=1e-12), mu
    dims = (4, 6, 3, 5)
    n = (1, 2, 1, 3)
    p = [2 * np.pi * n[m] / dims[m] for m in range(4)]
    M = free_spin_matrix(orc, dims, p)
    c = sum(2 * np.cos(q) for q in p)
    S = M - c * np.eye(4)
    # -2i sum sin(p) gamma: anti-Hermitian, and S S^dagger = 4 sum sin^2 p
    assert np.allclose(S, -S.conj().T, atol=1e-12)
    assert np.allclose(S @ S.conj().T, 4 * sum(np.sin(q) ** 2 for q in p) * np.eye(4), atol=1e-11)


def _random_spinor(V, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((V, 4, 3, 2))


def _spin_apply(mat, psi):
    pc = psi[..., 0] + 1j * psi[..., 1]
    out = np.einsum('ab,vbc->vac', mat, pc)
    return np.stack([out.real, out.imag], -1)


def pin_dslash_gamma5_hermitian(orc):
    """<phi, D psi> = <g5 D g5 phi, psi> on random SU(3) links (g5 =
    g1 g2 g3 g4 from the oracle's own matrices)."""
    g = oracle_gammas(orc)
    g5 = g[0] @ g[1] @ g[2] @ g[3]
    dims = (3, 4, 2, 5)
    V = int(np.prod(dims))
    links = [testgen.su3_field(V, field_id=70 + m) for m in range(4)]
    phi, psi = _random_spinor(V, 1), _random_spinor(V, 2)
    cdot = lambda a, b: np.sum((a[..., 0] - 1j * a[..., 1]) * (b[..., 0] + 1j * b[..., 1]))
    lhs = cdot(phi, orc.dslash(links, psi, dims))
    rhs = cdot(_spin_apply(g5, orc.dslash(links, _spin_apply(g5, phi), dims)), psi)
    assert abs(lhs - rhs) < 1e-11 * abs(lhs)


def pin_dslash_gauge_covariant(orc):
    """U'_mu(x) = g(x) U_mu(x) g(x + mu)^dagger, psi'(x) = g(x) psi(x)
    give (D' psi')(x) = g(x) (D psi)(x) for random SU(3) g."""
    dims = (3, 4, 2, 5)
    V = int(np.prod(dims))
    links = [testgen.su3_field(V, field_id=74 + m) for m in range(4)]
    g = to_complex(testgen.su3_field(V, field_id=78))
    psi = _random_spinor(V, 3)
    arr = lambda f: f.reshape(dims[3], dims[2], dims[1], dims[0], *f.shape[1:])
    def shift(f, mu):  # f(x + mu)
        return np.roll(arr(f), -1, axis=3 - mu).reshape(f.shape)
    newl = []
    for mu in range(4):
        u = to_complex(links[mu])
        gn = shift(g, mu)
        newl.append(from_complex(g @ u @ np.conj(np.transpose(gn, (0, 2, 1)))))
    pc = psi[..., 0] + 1j * psi[..., 1]
    psi2 = np.einsum('vab,vsb->vsa', g, pc)
    psi2 = np.stack([psi2.real, psi2.imag], -1)
    lhs = orc.dslash(newl, psi2, dims)
    d = orc.dslash(links, psi, dims)
    dc = d[..., 0] + 1j * d[..., 1]
    rhs = np.einsum('vab,vsb->vsa', g, dc)
    assert np.max(np.abs((lhs[..., 0] + 1j * lhs[..., 1]) - rhs)) < 1e-12


def _vnode_numpy(a, dims, simd, prec):
    """Virtual-node image built with numpy: each lattice axis split into
    (node, outer) coordinates, then the outer axes moved outside the entry
    axis and the node axes inside it."""
    V = a.shape[0]
    canon = a.shape[1] * a.shape[2]  # 9 or 12 complex entries
    E = 6 if (canon == 9 and prec == O.C12) else canon
    Lx, Ly, Lz, Lt = dims
    sx, sy, sz, st = simd
    ent = a.reshape(V, canon, 2)[:, :E, :]
    g = ent.reshape(st, Lt // st, sz, Lz // sz, sy, Ly // sy, sx, Lx // sx, E, 2)
    # axes: 0 nt 1 ot 2 nz 3 oz 4 ny 5 oy 6 nx 7 ox 8 e 9 c
    img = g.transpose(1, 3, 5, 7, 8, 0, 2, 4, 6, 9).reshape(-1)
    if prec == O.F64:
        return img.view(np.uint8)
    if prec == O.F16:
        return img.astype(np.float32).astype(np.float16).view(np.uint8)
    return img.astype(np.float32).view(np.uint8)


VNODE_CASES = [((4, 2, 6, 4), (2, 1, 2, 2)), ((2, 4, 4, 8), (1, 1, 2, 4)),
               ((8, 3, 2, 2), (8, 1, 1, 1)), ((3, 5, 7, 2), (1, 1, 1, 2)),
               ((4, 4, 4, 4), (2, 2, 2, 2)), ((2, 2, 2, 2), (1, 1, 1, 1))]


def pin_vnode_layout(orc):
    """Grid's virtual-node images equal numpy's split/transpose
    construction (matrices in every precision, spinors in F64/F32); with
    one virtual node the image is the AoS one, with the x extent split
    into single-site nodes it is AoSoA(Lx); unpack inverts pack."""
    for dims, simd in VNODE_CASES:
        V = int(np.prod(dims))
        x = testgen.su3_field(V, field_id=32)
        for prec in (O.F64, O.F32, O.F16, O.C12):
            img = orc.vnode_pack(x, dims, simd, prec)
            assert np.array_equal(img, _vnode_numpy(x, dims, simd, prec)), (dims, simd, prec)
        psi = testgen.spinor_field(V, field_id=33)
        for prec in (O.F64, O.F32):
            img = orc.vnode_pack(psi, dims, simd, prec)
            assert np.array_equal(img, _vnode_numpy(psi, dims, simd, prec)), (dims, simd)
        back = orc.vnode_unpack(orc.vnode_pack(psi, dims, simd, O.F64), dims, simd, O.F64,
                                spinor=True)
        assert np.array_equal(back, psi)
        if simd == (1, 1, 1, 1):
            assert np.array_equal(orc.vnode_pack(x, dims, simd, O.F64),
                                  orc.pack(x, O.F64, O.AOS))
    dims = (8, 3, 2, 2)
    x = testgen.su3_field(96, field_id=34)
    for prec in (O.F64, O.F16, O.C12):
        assert np.array_equal(orc.vnode_pack(x, dims, (8, 1, 1, 1), prec),
                              orc.pack(x, prec, O.AOSOA, 8))


def pin_expr_constant_fields(orc):
    """Through the expression evaluator: constant real fields 1 and 2 (the
    inputs of Section 3's composite-expression example, Listing 2) assigned
    from constant expressions; their sum is exactly 3 and the sum plus their
    product exactly 5; on SU(3)-typed fields 1*I and 2*I the second gives
    5*I."""
    g = read_golden("composite_constants.txt")
    V = 12
    a = orc.eval_expr(repr(g["a"]), [], [], V=V)
    b = orc.eval_expr(repr(g["b"]), [], [], V=V)
    assert np.array_equal(a, np.full(V, g["a"])) and np.array_equal(b, np.full(V, g["b"]))
    assert np.array_equal(orc.eval_expr("a+b", [a, b], [2, 2]), np.full(V, g["real_ADD"]))
    assert np.array_equal(orc.eval_expr("a+b+a*b", [a, b], [2, 2]),
                          np.full(V, g["real_APB_AB"]))
    x = testgen.identity(V, g["a"])
    y = testgen.identity(V, g["b"])
    assert np.array_equal(orc.eval_expr("a+b+a*b", [x, y], [0, 0]),
                          testgen.identity(V, g["APB_AB"]))


def pin_expr_matches_fixed(orc):
    """Matrix expressions equal the (separately pinned) fixed expressions
    bit for bit: same association, same textbook sums."""
    V = 40
    ops = [testgen.su3_field(V, field_id=40 + k) for k in range(4)]
    for text, expr in (("a*b", O.MUL), ("a*b*c", O.MUL3), ("a*b+c*d", O.MULADD),
                       ("a+b", O.ADD), ("a+b+a*b", O.APB_AB)):
        n = {O.MUL: 2, O.MUL3: 3, O.MULADD: 4, O.ADD: 2, O.APB_AB: 2}[expr]
        got = orc.eval_expr(text, ops[:n], [0] * n)
        assert np.array_equal(got, orc.fused(expr, ops[:n])), text


def _cx_mat(a):
    return a[..., 0] + 1j * a[..., 1]


def pin_expr_numpy(orc):
    """Functions, scalar-matrix mixing and complex constants against numpy
    on random complex inputs (not unitary, so no identity hides an error)."""
    rng = np.random.default_rng(5)
    V = 30
    a = rng.standard_normal((V, 3, 3, 2))
    b = rng.standard_normal((V, 3, 3, 2))
    c = rng.standard_normal((V, 2))
    r = rng.standard_normal(V)
    A, B, C = _cx_mat(a), _cx_mat(b), c[:, 0] + 1j * c[:, 1]
    eye = np.eye(3)[None]
    fields, kinds = [a, b, c, r], [0, 0, 3, 2]
    cases = [
        ("adj(a)", np.conj(np.transpose(A, (0, 2, 1)))),
        ("transpose(a)", np.transpose(A, (0, 2, 1))),
        ("conj(a)", np.conj(A)),
        ("trace(a*b)", np.einsum("sij,sji->s", A, B)),
        ("2*i*a - b", 2j * A - B),
        ("c*a + b", C[:, None, None] * A + B),
        ("a - c", A - C[:, None, None] * eye),
        ("c - a", C[:, None, None] * eye - A),
        ("d*a*c", (r * C)[:, None, None] * A),
        ("-a*b", -(A @ B)),
        ("real(trace(a)) + imag(c)", np.trace(A, axis1=1, axis2=2).real + C.imag),
        ("a*transpose(b)", A @ np.transpose(B, (0, 2, 1))),
        ("conj(c)*d", np.conj(C) * r),
    ]
    for text, want in cases:
        got = orc.eval_expr(text, fields, kinds)
        if got.ndim == 4:
            got = _cx_mat(got)
        elif got.ndim == 2:
            got = got[:, 0] + 1j * got[:, 1]
        assert got.shape == want.shape, text
        assert np.max(np.abs(got - want)) <= 1e-13 * (1 + np.max(np.abs(want))), text


def pin_expr_rejects(orc):
    """Malformed and ill-typed expressions are refused."""
    V = 4
    x = testgen.su3_field(V)
    for bad in ("a+", "a*(b", "x", "real(a)", "b", "adj a", "1..2"):
        try:
            orc.eval_expr(bad, [x], [0])
        except ValueError:
            continue
        raise AssertionError(f"{bad!r} accepted")


ALL_PINS = [pin_identity, pin_phase_diag, pin_signed_permutations,
            pin_unitary_inverse, pin_numpy_matmul, pin_nonsymmetric,
            pin_product_invariants, pin_associative, pin_constant_fields_fused,
            pin_fused_reductions, pin_fused_numpy, pin_fused_unitary,
            pin_quantisers, pin_c12_rebuild, pin_layouts, pin_roundtrip,
            pin_metrics, pin_cshift, pin_dslash_free_field,
            pin_dslash_gamma5_hermitian, pin_dslash_gauge_covariant,
            pin_vnode_layout, pin_expr_constant_fields, pin_expr_matches_fixed,
            pin_expr_numpy, pin_expr_rejects]
