"""Plain FP64 CPU oracle (Python side).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The GPU library never imports it and
it never imports the GPU library.

Wraps ``oracle.c`` (built with gcc -O2 -ffp-contract=off) and adds the
pure-Python pieces: the batched workload's tile table and the reduced
precision reference.  Every field is a float64 array of shape (V, 3, 3, 2)
in the canonical host layout (site, row, column, re/im).

Codes: precision F64=0, F32=1, F16 (single-precision arithmetic)=2,
two-row compressed single precision C12=3; layout AOS=0, SOA=1, AOSOA=2;
expressions MUL=0, MUL3=1, MULADD=2, ADD=3, APB_AB=4.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

F64, F32, F16, C12 = 0, 1, 2, 3
AOS, SOA, AOSOA = 0, 1, 2
MUL, MUL3, MULADD, ADD, APB_AB = 0, 1, 2, 3, 4
N_OPERANDS = {MUL: 2, MUL3: 3, MULADD: 4, ADD: 2, APB_AB: 2}


def build(src: str = _SRC, out: str = _LIB) -> str:
    """Compile the oracle (always recompiles).  `src`/`out` let a test build
    a modified copy elsewhere."""
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", "-std=c11", src, "-o", out + ".tmp", "-lm"]
    subprocess.check_call(cmd)
    os.replace(out + ".tmp", out)
    return out


def _bind(lib):
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
    lib.oracle_mult.argtypes = [vp, vp, vp, i64]
    lib.oracle_mult.restype = None
    lib.oracle_fused.argtypes = [i32, vp, vp, vp, vp, vp, i64]
    lib.oracle_fused.restype = i32
    lib.oracle_quant_f32.argtypes = [vp, vp, i64]
    lib.oracle_quant_f32.restype = None
    lib.oracle_quant_f16.argtypes = [vp, vp, i64]
    lib.oracle_quant_f16.restype = None
    lib.oracle_dequant_f16.argtypes = [vp, vp, i64]
    lib.oracle_dequant_f16.restype = None
    lib.oracle_c12_rebuild.argtypes = [vp, i64]
    lib.oracle_c12_rebuild.restype = None
    lib.oracle_roundtrip.argtypes = [i32, vp, vp, i64]
    lib.oracle_roundtrip.restype = i32
    lib.oracle_field_bytes.argtypes = [i32, i32, i32, i64]
    lib.oracle_field_bytes.restype = i64
    lib.oracle_pack.argtypes = [vp, i64, i32, i32, i32, vp]
    lib.oracle_pack.restype = i32
    lib.oracle_unpack.argtypes = [vp, i64, i32, i32, i32, vp]
    lib.oracle_unpack.restype = i32
    lib.oracle_metrics.argtypes = [vp, vp, i64, vp]
    lib.oracle_metrics.restype = None
    lib.oracle_threads.argtypes = []
    lib.oracle_threads.restype = i32
    lib.oracle_cshift.argtypes = [vp, vp, vp, i32, i64]
    lib.oracle_cshift.restype = i32
    lib.oracle_dslash.argtypes = [vp, vp, vp, vp]
    lib.oracle_dslash.restype = i32
    lib.oracle_set_threads.argtypes = [i32]
    lib.oracle_set_threads.restype = None
    lib.oracle_vnode_pack.argtypes = [vp, vp, vp, i32, i32, i32, vp]
    lib.oracle_vnode_pack.restype = i32
    lib.oracle_vnode_unpack.argtypes = [vp, vp, vp, i32, i32, i32, vp]
    lib.oracle_vnode_unpack.restype = i32
    lib.oracle_eval_expr.argtypes = [ctypes.c_char_p, i32, vp, vp, vp, i64]
    lib.oracle_eval_expr.restype = i32
    return lib


class Oracle:
    """One loaded copy of the oracle library (the default one, or a copy
    built from modified source by a test)."""

    def __init__(self, path: str = _LIB):
        if path == _LIB and not os.path.exists(path):
            build()
        self.lib = _bind(ctypes.CDLL(path))

    @staticmethod
    def _p(a):
        return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None

    @staticmethod
    def _field(a):
        a = np.ascontiguousarray(a, dtype=np.float64)
        assert a.ndim == 4 and a.shape[1:] == (3, 3, 2), a.shape
        return a

    def threads(self):
        """OpenMP threads of the oracle's site loops."""
        return int(self.lib.oracle_threads())

    def set_threads(self, n):
        self.lib.oracle_set_threads(int(n))

    def mult(self, x, y):
        """z(s) = x(s) y(s): the product written out, k ascending."""
        x, y = self._field(x), self._field(y)
        assert x.shape == y.shape
        z = np.empty_like(x)
        self.lib.oracle_mult(self._p(x), self._p(y), self._p(z), x.shape[0])
        return z

    def fused(self, expr, ops):
        """MUL a*b, MUL3 (a*b)*c, MULADD (a*b)+(c*d), ADD a+b,
        APB_AB (a+b)+(a*b)."""
        ops = [self._field(o) for o in ops]
        need = N_OPERANDS[expr]
        assert len(ops) == need, (expr, len(ops))
        V = ops[0].shape[0]
        full = ops + [None] * (4 - need)
        z = np.empty_like(ops[0])
        rc = self.lib.oracle_fused(expr, *[self._p(o) for o in full],
                                   self._p(z), V)
        assert rc == 0
        return z

    def cshift(self, a, dims, mu, shift):
        """b(c) = a(c + shift * mu_hat), periodic."""
        a = self._field(a)
        d = np.ascontiguousarray(np.asarray(dims, dtype=np.int32))
        assert a.shape[0] == int(np.prod(d))
        out = np.empty_like(a)
        rc = self.lib.oracle_cshift(self._p(a), self._p(out), self._p(d), mu, shift)
        assert rc == 0
        return out

    def mult_shifted(self, x, y, dims, mu, shift):
        """z(c) = x(c) * y(c + shift * mu_hat)."""
        return self.mult(x, self.cshift(y, dims, mu, shift))

    def dslash(self, links, psi, dims):
        """Wilson hopping term: sum over mu of (1 - gamma_mu) U_mu(x)
        psi(x + mu) + (1 + gamma_mu) U_mu(x - mu)^dagger psi(x - mu).
        links: 4 link fields; psi: spinor field, shape (V, 4, 3, 2)."""
        u = [self._field(l) for l in links]
        psi = np.ascontiguousarray(psi, dtype=np.float64)
        assert psi.shape[1:] == (4, 3, 2)
        d = np.ascontiguousarray(np.asarray(dims, dtype=np.int32))
        arr = (ctypes.c_void_p * 4)(*[l.ctypes.data for l in u])
        out = np.empty_like(psi)
        rc = self.lib.oracle_dslash(ctypes.cast(arr, ctypes.c_void_p), self._p(psi),
                                    self._p(out), self._p(d))
        assert rc == 0
        return out

    def quant_f32(self, a):
        a = np.ascontiguousarray(a, dtype=np.float64)
        out = np.empty(a.shape, dtype=np.float32)
        self.lib.oracle_quant_f32(self._p(a), self._p(out), a.size)
        return out

    def quant_f16(self, a):
        """Bits of the half-precision value, double -> float -> half."""
        a = np.ascontiguousarray(a, dtype=np.float64)
        out = np.empty(a.shape, dtype=np.uint16)
        self.lib.oracle_quant_f16(self._p(a), self._p(out), a.size)
        return out

    def dequant_f16(self, h):
        h = np.ascontiguousarray(h, dtype=np.uint16)
        out = np.empty(h.shape, dtype=np.float64)
        self.lib.oracle_dequant_f16(self._p(h), self._p(out), h.size)
        return out

    def c12_rebuild(self, a):
        """Copy of `a` with row 2 replaced by conj(row0 x row1)."""
        a = self._field(a).copy()
        self.lib.oracle_c12_rebuild(self._p(a), a.shape[0])
        return a

    def roundtrip(self, prec, a):
        """What a field stored in `prec` holds, widened to double."""
        a = self._field(a)
        out = np.empty_like(a)
        rc = self.lib.oracle_roundtrip(prec, self._p(a), self._p(out),
                                       a.shape[0])
        assert rc == 0
        return out

    def field_bytes(self, prec, layout, lanes, V):
        return int(self.lib.oracle_field_bytes(prec, layout, lanes, V))

    def pack(self, a, prec, layout, lanes=0):
        """Stored image (raw bytes, uint8) of a canonical field."""
        a = self._field(a)
        n = self.field_bytes(prec, layout, lanes, a.shape[0])
        assert n >= 0
        out = np.zeros(n, dtype=np.uint8)
        rc = self.lib.oracle_pack(self._p(a), a.shape[0], prec, layout,
                                  lanes, self._p(out))
        assert rc == 0
        return out

    def unpack(self, raw, V, prec, layout, lanes=0):
        raw = np.ascontiguousarray(raw).view(np.uint8)
        assert raw.size >= self.field_bytes(prec, layout, lanes, V)
        out = np.zeros((V, 3, 3, 2), dtype=np.float64)
        rc = self.lib.oracle_unpack(self._p(raw), V, prec, layout, lanes,
                                    self._p(out))
        assert rc == 0
        return out

    def vnode_pack(self, a, dims, simd, prec):
        """Stored image (uint8) of a canonical matrix field (V, 3, 3, 2) or
        spinor field (V, 4, 3, 2) in Grid's virtual-node layout."""
        a = np.ascontiguousarray(a, dtype=np.float64)
        canon = 12 if a.shape[1:] == (4, 3, 2) else 9
        entries = 6 if (canon == 9 and prec == 3) else canon
        rb = {0: 8, 1: 4, 2: 2, 3: 4}[prec]
        out = np.zeros(a.shape[0] * entries * 2 * rb, dtype=np.uint8)
        d = np.ascontiguousarray(np.asarray(dims, dtype=np.int32))
        sm = np.ascontiguousarray(np.asarray(simd, dtype=np.int32))
        rc = self.lib.oracle_vnode_pack(self._p(a), self._p(d), self._p(sm), prec,
                                        entries, canon, self._p(out))
        assert rc == 0
        return out

    def vnode_unpack(self, raw, dims, simd, prec, spinor=False):
        """Canonical field from a virtual-node image (compressed rows 0-1
        only: row 2 is left zero)."""
        raw = np.ascontiguousarray(raw).view(np.uint8)
        V = int(np.prod(dims))
        canon = 12 if spinor else 9
        entries = 6 if (not spinor and prec == 3) else canon
        out = np.zeros((V, 4 if spinor else 3, 3, 2), dtype=np.float64)
        d = np.ascontiguousarray(np.asarray(dims, dtype=np.int32))
        sm = np.ascontiguousarray(np.asarray(simd, dtype=np.int32))
        rc = self.lib.oracle_vnode_unpack(self._p(raw), self._p(d), self._p(sm), prec,
                                          entries, canon, self._p(out))
        assert rc == 0
        return out

    def eval_expr(self, text, fields, kinds, V=None):
        """Evaluate a site-local expression over operand fields a, b, ...
        (canonical arrays: matrices (V, 3, 3, 2), real (V,), complex (V, 2));
        kinds 0 matrix, 2 real, 3 complex.  Returns the result in the same
        forms; raises ValueError for a malformed or ill-typed expression."""
        fs = [np.ascontiguousarray(f, dtype=np.float64) for f in fields]
        if V is None:
            V = fs[0].shape[0]
        out = np.zeros(V * 18, dtype=np.float64)
        kk = np.ascontiguousarray(np.asarray(kinds, dtype=np.int32))
        arr = (ctypes.c_void_p * max(1, len(fs)))(*[f.ctypes.data for f in fs])
        rk = self.lib.oracle_eval_expr(text.encode(), len(fs), self._p(kk),
                                       ctypes.cast(arr, ctypes.c_void_p), self._p(out), V)
        if rk < 0:
            raise ValueError(f"expression {text!r} rejected")
        if rk == 0:
            return out.reshape(V, 3, 3, 2)
        if rk == 3:
            return out[:2 * V].reshape(V, 2).copy()
        return out[:V].copy()

    def metrics(self, zh, z=None):
        """dict(e_max, r_max, d_u, d_det) of zh (against z where given)."""
        zh = self._field(zh)
        if z is not None:
            z = self._field(z)
            assert z.shape == zh.shape
        out = np.zeros(4, dtype=np.float64)
        self.lib.oracle_metrics(self._p(zh), self._p(z), zh.shape[0],
                                self._p(out))
        return dict(e_max=out[0], r_max=out[1], d_u=out[2], d_det=out[3])

    # -------------------------------------------------- reduced precision

    def reference(self, expr, prec, ops):
        """The kernel-arithmetic reference: evaluate `expr` in double on the
        operands as stored in `prec` (quantised then widened; compressed
        operands get row 2 rebuilt in double)."""
        return self.fused(expr, [self.roundtrip(prec, o) for o in ops])


_default = None


def get() -> Oracle:
    global _default
    if _default is None:
        _default = Oracle()
    return _default


# ------------------------------------------------------------ tile table

def tile_table(volumes, tile_sites, precisions):
    """Work list of the batched launch, recomputed from its definition.

    Lattice i of V_i sites is cut into tiles_i = ceil(V_i / T) tiles of T
    sites; its tiles start at start_i = tiles_0 + ... + tiles_{i-1}; tile
    start_i + k covers sites [k T, min((k+1) T, V_i)).  Returns
    (starts, rows) where rows[t] = (lattice, first_site, count, precision).
    """
    starts, rows = [], []
    nxt = 0
    for i, V in enumerate(volumes):
        starts.append(nxt)
        k = 0
        while k * tile_sites < V:
            first = k * tile_sites
            rows.append((i, first, min(tile_sites, V - first), precisions[i]))
            k += 1
        nxt += k
    return starts, rows
