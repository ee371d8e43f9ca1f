"""Expression programs on the GPU against the oracle's own expression
evaluator: the composite-expression example of Section 3 (Listing 2) on
real (double) fields, mixed matrix / real /
complex expressions in every layout (virtual nodes included), double and
single arithmetic (single with compressed matrix operands too), in-place
outputs, compressed outputs of SU(3)-valued expressions, argument rules,
and the streaming product written as a program at 48^4, bit-identical to
su3_mult.

Tolerance (absolute, per real entry): |got - want| <= 64 u (1 + max|want|)
with u = 2^-53 (double) or 2^-24 (single): each expression here is at most
eight operations deep, each a chain of at most six roundings over terms
bounded by the largest value (inputs are SU(3) matrices and scalars of
size O(1)), plus the rounding of the stored result."""
import numpy as np
import pytest
import torch

import oracle as O
import testgen
import paper_1710_09409_amd as su3

pytestmark = pytest.mark.gpu

M, R, C = su3.SU3_KIND_MATRIX, su3.SU3_KIND_REAL, su3.SU3_KIND_COMPLEX
EXPRS = [
    ("a+b+a*b", (R, R)),
    ("a*b", (M, M)),
    ("a*b*c", (M, M, M)),
    ("trace(a*adj(b)) * c + d", (M, M, C, C)),
    ("2*i*a - b*c", (M, M, C)),
    ("(a*b)*(c*d) + a - d", (M, M, M, M)),
    # seven matrix registers: the 8-register kernel (in double it spills)
    ("(a*b+c*d)*(a*c+b*d) + (a-b)*(c-d)", (M, M, M, M)),
    ("real(trace(a)) * b + c", (M, M, R)),
    # every mixed scalar/matrix opcode, a self product and a negated matrix
    ("a*a - 2*a + 1.5", (M,)),
    ("c - a*b*c + trace(a)*c - 0.5*i - (-b)", (M, M, C)),
    ("trace(a) + b*adj(b)", (M, M)),
    # a multiply-add in programs of two registers (run by the 4-register
    # variant) and of one
    ("a*b + a", (M, M)),
    ("a*a + a*a", (M,)),
    # a matrix operand as the result (no instruction), and unary opcodes
    # applied twice in place
    ("a", (M,)),
    ("adj(adj(a)) - transpose(transpose(b)) + conj(conj(a))", (M, M)),
    ("adj(a)*transpose(b) - conj(a)", (M, M)),
    ("c*d - imag(c) + 0.5", (M, M, C, R)),
    ("1.0", ()),
    ("a", (C,)),
    ("-(a - b) * imag(a) + conj(b) - 0.25 * c", (R, R, R)),
    ("((a*b)*(c*a))*((b*c)*(a-b)) + ((a+c)*(b+c))*((a*a)*(c-b))", (R, R, R)),
]
LAYS = [(su3.SU3_LAYOUT_SOA, 0, None), (su3.SU3_LAYOUT_AOSOA, 64, None),
        (su3.SU3_LAYOUT_AOS, 0, None), (su3.SU3_LAYOUT_VNODE, 0, (2, 1, 2, 2))]
LAY_IDS = ["soa", "aosoa64", "aos", "vnode"]
DIMS = (4, 6, 8, 10)


def make(dims, prec, kind, lay, host, s):
    layout, lanes, simd = lay
    if layout == su3.SU3_LAYOUT_VNODE:
        f = su3.vnode_tensor(dims, prec, simd, kind)
    elif kind == M:
        f = su3.field_tensor(dims, prec, layout, lanes)
    else:
        f = su3.scalar_tensor(dims, prec, layout, kind, lanes)
    if host is not None:
        su3.su3_field_upload(f, host, s)
    return f


def host_operand(V, kind, k):
    if kind == M:
        return testgen.su3_field(V, field_id=300 + k)
    x = 3.0 * testgen.su3_field(V, field_id=310 + k).reshape(V, 18)
    return x[:, 0].copy() if kind == R else x[:, :2].copy()


def quantise(x, kind, prec):
    if kind == M:
        return O.get().roundtrip(prec, x)
    return x if prec == su3.SU3_F64 else x.astype(np.float32).astype(np.float64)


def tol(got, want, single):
    u = 2.0 ** -24 if single else 2.0 ** -53
    bound = 64 * u * (1 + (np.max(np.abs(want)) if want.size else 0))
    return float(np.max(np.abs(got - want))) if got.size else 0.0, bound


@pytest.mark.parametrize("lay", LAYS, ids=LAY_IDS)
@pytest.mark.parametrize("arith", [0, 1, 3], ids=["f64", "f32", "f32c12"])
def test_program_parity(arith, lay):
    s = torch.cuda.current_stream()
    V = testgen.volume(DIMS)
    for text, kinds in EXPRS:
        precs = [arith if k == M else (0 if arith == 0 else 1) for k in kinds]
        hosts = [host_operand(V, k, i) for i, k in enumerate(kinds)]
        fs = [make(DIMS, p, k, lay, h, s) for p, k, h in zip(precs, kinds, hosts)]
        prog = su3.Program(text, kinds)
        info = prog.info()
        rk = info["result_kind"]
        zprec = (1 if arith == 3 else arith) if rk == M else (0 if arith == 0 else 1)
        z = make(DIMS, zprec, rk, lay, None, s)
        q = [quantise(h, k, p) for h, k, p in zip(hosts, kinds, precs)]
        want = O.get().eval_expr(text, q, [int(k) for k in kinds], V=V)
        su3.su3_program_eval(prog, z, fs, s)
        su3.su3_sync(s)
        got = su3.su3_field_download(z, s)
        err, bound = tol(got, want.reshape(got.shape), arith != 0)
        assert err <= bound, f"{text} {LAY_IDS[LAYS.index(lay)]}: {err:.3e} > {bound:.3e}"


def test_constant_fields_real():
    """Constant real fields a = 1 and b = 2 (assigned from constant
    expressions) give a+b = 3 and a+b+a*b = 5 exactly at a ragged volume in
    SoA, and the padding of the output is left alone."""
    s = torch.cuda.current_stream()
    dims = (3, 5, 7, 11)
    V = testgen.volume(dims)
    lay = (su3.SU3_LAYOUT_SOA, 0, None)
    a, b, z = (make(dims, su3.SU3_F64, R, lay, None, s) for _ in range(3))
    z.owner.fill_(0x77)
    su3.su3_program_eval(su3.Program("1.0", []), a, [], s)
    su3.su3_program_eval(su3.Program("2.0", []), b, [], s)
    su3.su3_program_eval(su3.Program("a+b", [R, R]), z, [a, b], s)
    assert np.array_equal(su3.su3_field_download(z, s), np.full(V, 3.0))
    su3.su3_program_eval(su3.Program("a+b+a*b", [R, R]), z, [a, b], s)
    su3.su3_sync(s)
    assert np.array_equal(su3.su3_field_download(z, s), np.full(V, 5.0))
    raw = su3.su3_field_download_raw(z, s)
    assert np.all(raw[8 * V:] == 0x77)  # padding of the 64-site round-up


def test_program_in_place_and_compressed():
    s = torch.cuda.current_stream()
    dims = (4, 4, 4, 8)
    V = testgen.volume(dims)
    lay = (su3.SU3_LAYOUT_AOSOA, 16, None)
    x, y = testgen.su3_field(V, field_id=320), testgen.su3_field(V, field_id=321)
    fx = make(dims, su3.SU3_F64, M, lay, x, s)
    fy = make(dims, su3.SU3_F64, M, lay, y, s)
    su3.su3_program_eval(su3.Program("a*b - adj(b)", [M, M]), fx, [fx, fy], s)
    want = O.get().eval_expr("a*b - adj(b)", [x, y], [0, 0])
    err, bound = tol(su3.su3_field_download(fx, s), want, False)
    assert err <= bound
    # compressed output of an SU(3)-valued expression
    cx = make(dims, su3.SU3_C12_F32, M, lay, x, s)
    cy = make(dims, su3.SU3_C12_F32, M, lay, y, s)
    cz = make(dims, su3.SU3_C12_F32, M, lay, None, s)
    su3.su3_program_eval(su3.Program("adj(a)*b*transpose(a)", [M, M]), cz, [cx, cy], s)
    q = [O.get().roundtrip(su3.SU3_C12_F32, h) for h in (x, y)]
    want = O.get().eval_expr("adj(a)*b*transpose(a)", q, [0, 0])
    got = su3.su3_field_download(cz, s)
    err, bound = tol(got[:, :2], want[:, :2], True)
    assert err <= bound


def test_program_rules():
    s = torch.cuda.current_stream()
    d = (2, 2, 2, 2)
    lay = (su3.SU3_LAYOUT_SOA, 0, None)
    m64 = make(d, su3.SU3_F64, M, lay, None, s)
    m32 = make(d, su3.SU3_F32, M, lay, None, s)
    r64 = make(d, su3.SU3_F64, R, lay, None, s)
    c12 = make(d, su3.SU3_C12_F32, M, lay, None, s)
    other = make((2, 2, 2, 4), su3.SU3_F64, M, lay, None, s)
    p = su3.Program("a*b", [M, M])
    for z, ops, st in ((m64, [m64, m32], su3.SU3_ERR_MISMATCH),
                       (m64, [m64, r64], su3.SU3_ERR_MISMATCH),
                       (r64, [m64, m64], su3.SU3_ERR_MISMATCH),
                       (m64, [m64, other], su3.SU3_ERR_MISMATCH),
                       (m64, [m64], su3.SU3_ERR_INVALID_ARG)):
        with pytest.raises(su3.Su3Error) as e:
            su3.su3_program_eval(p, z, ops, s)
        assert e.value.status == st
    with pytest.raises(su3.Su3Error) as e:
        su3.su3_program_eval(su3.Program("a+a", [M]), c12, [c12], s)
    assert e.value.status == su3.SU3_ERR_UNSUPPORTED
    for bad, kinds in (("a+", [M]), ("q", [M]), ("real(a)", [M]), ("b", [M])):
        with pytest.raises(su3.Su3Error) as e:
            su3.Program(bad, kinds)
        assert e.value.status == su3.SU3_ERR_INVALID_ARG
    with pytest.raises(su3.Su3Error) as e:
        su3.Program("a", [su3.SU3_KIND_SPINOR])
    assert e.value.status == su3.SU3_ERR_UNSUPPORTED


def test_program_product_full_size():
    """a*b as a program at 48^4 (FP64 SoA, tuned launch) is bit-identical
    to su3_mult's result."""
    s = torch.cuda.current_stream()
    dims = (48, 48, 48, 48)
    V = testgen.volume(dims)
    lay = (su3.SU3_LAYOUT_SOA, 0, None)
    fx = make(dims, su3.SU3_F64, M, lay, testgen.su3_field(V, field_id=testgen.FID_X), s)
    fy = make(dims, su3.SU3_F64, M, lay, testgen.su3_field(V, field_id=testgen.FID_Y), s)
    z1 = make(dims, su3.SU3_F64, M, lay, None, s)
    z2 = make(dims, su3.SU3_F64, M, lay, None, s)
    su3.su3_autotune(su3.SU3_EXPR_PROGRAM, su3.SU3_F64, su3.SU3_LAYOUT_SOA, 0, dims, s)
    su3.su3_program_eval(su3.Program("a*b", [M, M]), z1, [fx, fy], s)
    su3.su3_mult(z2, fx, fy, s)
    su3.su3_sync(s)
    assert torch.equal(z1.owner, z2.owner)


@pytest.mark.parametrize("prec", [su3.SU3_F64, su3.SU3_F32], ids=["f64", "f32"])
def test_constant_fields_real_full_size(prec):
    """a+b+a*b on real fields at 48^4 in the launch the benchmark times (the
    real-valued kernel): constant fields 1 and 2 give 5 at every site
    exactly, and seeded random fields agree with the oracle."""
    s = torch.cuda.current_stream()
    dims = (48, 48, 48, 48)
    V = testgen.volume(dims)
    lay = (su3.SU3_LAYOUT_SOA, 0, None)
    su3.su3_autotune(su3.SU3_EXPR_PROGRAM, prec, su3.SU3_LAYOUT_SOA, 0, dims, s)
    try:
        a, b, z = (make(dims, prec, R, lay, None, s) for _ in range(3))
        su3.su3_program_eval(su3.Program("1.0", []), a, [], s)
        su3.su3_program_eval(su3.Program("2.0", []), b, [], s)
        prog = su3.Program("a+b+a*b", [R, R])
        su3.su3_program_eval(prog, z, [a, b], s)
        su3.su3_sync(s)
        assert np.array_equal(su3.su3_field_download(z, s), np.full(V, 5.0))
        hosts = [host_operand(V, R, k) for k in range(2)]
        q = [quantise(h, R, prec) for h in hosts]
        for f, h in zip((a, b), hosts):
            su3.su3_field_upload(f, h, s)
        su3.su3_program_eval(prog, z, [a, b], s)
        su3.su3_sync(s)
        got = su3.su3_field_download(z, s)
        want = O.get().eval_expr("a+b+a*b", q, [int(R), int(R)], V=V)
        err, bound = tol(got, want.reshape(got.shape), prec != su3.SU3_F64)
        assert err <= bound, f"{err:.3e} > {bound:.3e}"
    finally:
        su3.su3_launch_reset()


@pytest.mark.parametrize("prec", [su3.SU3_F64, su3.SU3_F32], ids=["f64", "f32"])
def test_trace_full_size_scalar_result_key(prec):
    """A matrix-valued program with a complex result (the trace of a
    product) at 48^4, in the launch tuned for its own key
    (SU3_EXPR_PROGRAM_SCALAR, as the benchmark tunes it), against the
    oracle on every site; the matrix-result key keeps its own setting."""
    s = torch.cuda.current_stream()
    dims = (48, 48, 48, 48)
    V = testgen.volume(dims)
    lay = (su3.SU3_LAYOUT_SOA, 0, None)
    try:
        other = su3.su3_launch_get(su3.SU3_EXPR_PROGRAM, prec, su3.SU3_LAYOUT_SOA, 0, dims)
        best = su3.su3_autotune(su3.SU3_EXPR_PROGRAM_SCALAR, prec, su3.SU3_LAYOUT_SOA, 0,
                                dims, s)
        assert su3.su3_launch_get(su3.SU3_EXPR_PROGRAM_SCALAR, prec, su3.SU3_LAYOUT_SOA, 0,
                                  dims).as_dict() == best.as_dict()
        assert su3.su3_launch_get(su3.SU3_EXPR_PROGRAM, prec, su3.SU3_LAYOUT_SOA, 0,
                                  dims).as_dict() == other.as_dict()
        hosts = [testgen.su3_field(V, field_id=testgen.FID_U0 + k) for k in range(2)]
        a, b = (make(dims, prec, M, lay, h, s) for h in hosts)
        z = make(dims, prec, C, lay, None, s)
        su3.su3_program_eval(su3.Program("trace(a*adj(b))", [M, M]), z, [a, b], s)
        su3.su3_sync(s)
        got = su3.su3_field_download(z, s)
        q = [quantise(h, M, prec) for h in hosts]
        want = O.get().eval_expr("trace(a*adj(b))", q, [int(M), int(M)], V=V)
        err, bound = tol(got, want.reshape(got.shape), prec != su3.SU3_F64)
        assert err <= bound, f"{err:.3e} > {bound:.3e}"
    finally:
        su3.su3_launch_reset()
