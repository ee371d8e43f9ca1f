"""Python binding of libsu3 (the MI355X SU(3) x SU(3) streaming library).

Argument marshalling only: every function below calls the C entry point of
the same name in ``libsu3.so`` (declared in ``include/su3.h``) and raises
``Su3Error`` on a non-OK status.  All arithmetic runs in the library's HIP
kernels; PyTorch only provides device memory and streams.

The HIP runtime is the one PyTorch loads: torch is imported before the
library so that libsu3's ``libamdhip64`` dependency binds to the same copy
(streams and pointers are then shared).  ``load()`` raises if the library
is missing or if two different HIP runtimes are mapped -- there is no
fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

import torch  # noqa: F401  (must precede loading libsu3; see module doc)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsu3.so")

# enums of su3.h
SU3_OK = 0
SU3_ERR_INVALID_ARG = -1
SU3_ERR_MISMATCH = -2
SU3_ERR_UNSUPPORTED = -3
SU3_ERR_OUT_OF_MEMORY = -4
SU3_ERR_ALIAS = -5
SU3_ERR_HIP = -6

SU3_F64, SU3_F32, SU3_F16_F32ACC, SU3_C12_F32 = 0, 1, 2, 3
SU3_LAYOUT_AOS, SU3_LAYOUT_SOA, SU3_LAYOUT_AOSOA, SU3_LAYOUT_VNODE = 0, 1, 2, 3
SU3_KIND_MATRIX, SU3_KIND_SPINOR, SU3_KIND_REAL, SU3_KIND_COMPLEX = 0, 1, 2, 3
SU3_EXPR_MUL, SU3_EXPR_MUL3, SU3_EXPR_MULADD, SU3_EXPR_ADD, SU3_EXPR_APB_AB = range(5)
SU3_EXPR_CSHIFT, SU3_EXPR_MUL_SHIFTED = 5, 6  # launch-tuning keys only
SU3_EXPR_DSLASH = 7  # launch-tuning key of su3_dslash (precision = links')
SU3_EXPR_PROGRAM = 8  # launch-tuning key of su3_program_eval (arithmetic precision)
SU3_EXPR_PROGRAM_SCALAR = 9  # the same for matrix-valued programs with a scalar result
SU3_EXPR_BATCH = 32  # + leading item's expression: launch-tuning key of a batch
N_OPERANDS = {0: 2, 1: 3, 2: 4, 3: 2, 4: 2}

# exported symbols of su3.h, in declaration order
SYMBOLS = (
    "su3_field_bytes", "su3_field_alloc", "su3_field_wrap", "su3_field_free",
    "su3_field_data", "su3_field_upload", "su3_field_download",
    "su3_field_download_raw", "su3_mult", "su3_fused_eval", "su3_cshift",
    "su3_mult_shifted", "su3_spinor_bytes", "su3_spinor_alloc",
    "su3_spinor_wrap", "su3_dslash", "su3_vnode_bytes", "su3_vnode_alloc",
    "su3_scalar_bytes", "su3_scalar_alloc", "su3_scalar_wrap",
    "su3_program_create", "su3_program_info", "su3_program_eval",
    "su3_program_destroy", "su3_vnode_wrap",
    "su3_batch_create", "su3_batch_run", "su3_batch_launch", "su3_batch_destroy",
    "su3_batch_tiles", "su3_autotune", "su3_layout_recommend", "su3_batch_autotune",
    "su3_launch_get",
    "su3_launch_set",
    "su3_launch_reset", "su3_stream", "su3_stream_autotune", "su3_triad",
    "su3_copy", "su3_sync",
    "su3_status_string", "su3_last_error",
)


class Su3Error(RuntimeError):
    def __init__(self, status: int, func: str, detail: str):
        self.status = status
        super().__init__(f"{func}: {_status_name(status)}: {detail}")


class su3_launch(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32), ("persistent", ctypes.c_int32),
                ("nontemporal", ctypes.c_int32), ("xcd_remap", ctypes.c_int32),
                ("lds_stage", ctypes.c_int32), ("tile_sites", ctypes.c_int32),
                ("occupancy", ctypes.c_int32), ("schedule", ctypes.c_int32),
                ("sites_per_lane", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def _hip_runtimes_mapped():
    paths = set()
    try:
        with open("/proc/self/maps") as f:
            for line in f:
                if "libamdhip64" in line:
                    paths.add(os.path.realpath(line.split()[-1]))
    except OSError:
        pass
    return paths


def load():
    """Load libsu3.so (built in-tree by build.py / __graft_entry__.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with "
            "`python -c 'import __graft_entry__ as g; g.build()'`")
    lib = ctypes.CDLL(LIB_PATH)
    runtimes = _hip_runtimes_mapped()
    if len(runtimes) > 1:
        raise ImportError("two HIP runtimes are mapped (%s); libsu3 must share "
                          "torch's" % ", ".join(sorted(runtimes)))
    vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    pp = ctypes.POINTER(ctypes.c_void_p)
    dims_t = ctypes.POINTER(ctypes.c_int32)
    L = ctypes.POINTER(su3_launch)
    sig = {
        "su3_field_bytes": [dims_t, i32, i32, i32, ctypes.POINTER(sz)],
        "su3_field_alloc": [pp, dims_t, i32, i32, i32],
        "su3_field_wrap": [pp, vp, sz, dims_t, i32, i32, i32],
        "su3_field_free": [vp],
        "su3_field_data": [vp, pp, ctypes.POINTER(sz)],
        "su3_field_upload": [vp, vp, vp],
        "su3_field_download": [vp, vp, vp],
        "su3_field_download_raw": [vp, vp, sz, vp],
        "su3_mult": [vp, vp, vp, vp],
        "su3_fused_eval": [vp, i32, vp, i32, vp],
        "su3_cshift": [vp, vp, i32, i32, vp],
        "su3_mult_shifted": [vp, vp, vp, i32, i32, vp],
        "su3_spinor_bytes": [dims_t, i32, i32, i32, ctypes.POINTER(sz)],
        "su3_spinor_alloc": [pp, dims_t, i32, i32, i32],
        "su3_spinor_wrap": [pp, vp, sz, dims_t, i32, i32, i32],
        "su3_dslash": [vp, vp, vp, vp],
        "su3_scalar_bytes": [dims_t, i32, i32, i32, i32, ctypes.POINTER(sz)],
        "su3_scalar_alloc": [pp, dims_t, i32, i32, i32, i32],
        "su3_scalar_wrap": [pp, vp, sz, dims_t, i32, i32, i32, i32],
        "su3_program_create": [pp, ctypes.c_char_p, i32, vp],
        "su3_program_info": [vp, ctypes.POINTER(i32), ctypes.POINTER(i32),
                             ctypes.POINTER(i32)],
        "su3_program_eval": [vp, vp, vp, i32, vp],
        "su3_program_destroy": [vp],
        "su3_vnode_bytes": [dims_t, i32, i32, dims_t, ctypes.POINTER(sz)],
        "su3_vnode_alloc": [pp, dims_t, i32, i32, dims_t],
        "su3_vnode_wrap": [pp, vp, sz, dims_t, i32, i32, dims_t],
        "su3_batch_create": [pp, vp, vp, vp, i32, vp],
        "su3_batch_run": [vp, vp, vp, i32, vp],
        "su3_batch_launch": [vp, vp],
        "su3_batch_destroy": [vp],
        "su3_batch_tiles": [vp, vp, i64, ctypes.POINTER(i64)],
        "su3_autotune": [i32, i32, i32, i32, dims_t, vp, L],
        "su3_layout_recommend": [i32, i32, dims_t, vp, ctypes.POINTER(i32),
                                 ctypes.POINTER(i32), L, ctypes.POINTER(ctypes.c_double)],
        "su3_batch_autotune": [vp, vp, vp, i32, vp, L],
        "su3_launch_get": [i32, i32, i32, i32, dims_t, L],
        "su3_launch_set": [i32, i32, i32, i32, dims_t, L],
        "su3_launch_reset": [],
        "su3_stream": [i32, vp, vp, vp, ctypes.c_double, sz, L, vp],
        "su3_stream_autotune": [i32, vp, vp, vp, sz, vp, L,
                                ctypes.POINTER(ctypes.c_double)],
        "su3_triad": [vp, vp, vp, ctypes.c_double, i64, vp],
        "su3_copy": [vp, vp, sz, vp],
        "su3_sync": [vp],
    }
    for name, argtypes in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = argtypes
        fn.restype = ctypes.c_int
    lib.su3_status_string.argtypes = [ctypes.c_int]
    lib.su3_status_string.restype = ctypes.c_char_p
    lib.su3_last_error.argtypes = []
    lib.su3_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _status_name(status):
    return load().su3_status_string(status).decode()


def _check(func, status):
    if status != SU3_OK:
        raise Su3Error(status, func, load().su3_last_error().decode())


def _dims(dims):
    d = [int(x) for x in dims]
    if len(d) != 4:
        raise ValueError("dims must have 4 entries")
    return (ctypes.c_int32 * 4)(*d)


def _stream(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream  # torch.cuda.Stream


def volume(dims):
    v = 1
    for d in dims:
        v *= int(d)
    return v


# ---------------------------------------------------------------- fields

def su3_field_bytes(dims, prec, layout, lanes=0):
    n = ctypes.c_size_t()
    _check("su3_field_bytes",
           load().su3_field_bytes(_dims(dims), prec, layout, lanes, ctypes.byref(n)))
    return n.value


@dataclass
class Field:
    """A library field handle plus what keeps its memory alive."""
    handle: int
    dims: tuple
    prec: int
    layout: int
    lanes: int
    owner: object = None  # torch tensor for wrapped fields
    spinor: bool = False
    simd: tuple = None    # virtual nodes per direction (VNODE layout)
    kind: int = None      # su3_kind (matrix unless set)

    def __post_init__(self):
        if self.kind is None:
            self.kind = SU3_KIND_SPINOR if self.spinor else SU3_KIND_MATRIX
        self.spinor = self.kind == SU3_KIND_SPINOR

    @property
    def V(self):
        return volume(self.dims)

    @property
    def site_shape(self):
        """Canonical host shape of one site."""
        return {SU3_KIND_MATRIX: (3, 3, 2), SU3_KIND_SPINOR: (4, 3, 2),
                SU3_KIND_REAL: (), SU3_KIND_COMPLEX: (2,)}[self.kind]

    def __del__(self):
        if self.handle and _lib is not None:
            _lib.su3_field_free(self.handle)
            self.handle = None


def su3_field_alloc(dims, prec, layout, lanes=0):
    h = ctypes.c_void_p()
    _check("su3_field_alloc",
           load().su3_field_alloc(ctypes.byref(h), _dims(dims), prec, layout, lanes))
    return Field(h.value, tuple(dims), prec, layout, lanes)


def su3_field_wrap(tensor_or_ptr, dims, prec, layout, lanes=0, nbytes=None):
    """Describe device memory as a field.  A torch tensor is kept alive by
    the returned Field; a raw pointer needs `nbytes`."""
    if isinstance(tensor_or_ptr, torch.Tensor):
        t = tensor_or_ptr
        ptr = t.data_ptr()
        nbytes = t.numel() * t.element_size() if nbytes is None else nbytes
        owner = t
    else:
        ptr, owner = int(tensor_or_ptr), None
        if nbytes is None:
            raise ValueError("nbytes is required with a raw pointer")
    h = ctypes.c_void_p()
    _check("su3_field_wrap",
           load().su3_field_wrap(ctypes.byref(h), ptr, nbytes, _dims(dims),
                                 prec, layout, lanes))
    return Field(h.value, tuple(dims), prec, layout, lanes, owner)


def field_tensor(dims, prec, layout, lanes=0, device="cuda"):
    """A torch byte tensor sized for a field, wrapped as a Field."""
    n = su3_field_bytes(dims, prec, layout, lanes)
    t = torch.zeros(n, dtype=torch.uint8, device=device)
    return su3_field_wrap(t, dims, prec, layout, lanes)


def su3_field_free(f: Field):
    if f.handle:
        _check("su3_field_free", load().su3_field_free(f.handle))
        f.handle = None


def su3_field_data(f: Field):
    p, n = ctypes.c_void_p(), ctypes.c_size_t()
    _check("su3_field_data", load().su3_field_data(f.handle, ctypes.byref(p),
                                                   ctypes.byref(n)))
    return p.value, n.value


def su3_field_upload(f: Field, host, stream=None):
    a = np.ascontiguousarray(host, dtype=np.float64)
    n = f.V * int(np.prod(f.site_shape))
    if a.size != n:
        raise ValueError(f"expected {n} doubles, got {a.size}")
    _check("su3_field_upload",
           load().su3_field_upload(f.handle, a.ctypes.data, _stream(stream)))


def su3_field_download(f: Field, stream=None):
    out = np.empty((f.V,) + f.site_shape, dtype=np.float64)
    _check("su3_field_download",
           load().su3_field_download(f.handle, out.ctypes.data, _stream(stream)))
    return out


def su3_field_download_raw(f: Field, stream=None):
    _, n = su3_field_data(f)
    out = np.empty(n, dtype=np.uint8)
    _check("su3_field_download_raw",
           load().su3_field_download_raw(f.handle, out.ctypes.data, n,
                                         _stream(stream)))
    return out


# --------------------------------------------------------------- compute

def su3_mult(z: Field, x: Field, y: Field, stream=None):
    _check("su3_mult", load().su3_mult(z.handle, x.handle, y.handle,
                                       _stream(stream)))


def su3_fused_eval(z: Field, expr, ops, stream=None):
    arr = (ctypes.c_void_p * max(1, len(ops)))(*[o.handle if o is not None else None
                                                 for o in ops])
    _check("su3_fused_eval",
           load().su3_fused_eval(z.handle if z is not None else None, expr, arr,
                                 len(ops), _stream(stream)))


def su3_cshift(dst: Field, src: Field, mu, shift, stream=None):
    _check("su3_cshift", load().su3_cshift(dst.handle, src.handle, int(mu),
                                           int(shift), _stream(stream)))


def su3_mult_shifted(z: Field, x: Field, y: Field, mu, shift, stream=None):
    _check("su3_mult_shifted",
           load().su3_mult_shifted(z.handle, x.handle, y.handle, int(mu),
                                   int(shift), _stream(stream)))


# ---------------------------------------------------------- spinor fields

def su3_spinor_bytes(dims, prec, layout, lanes=0):
    n = ctypes.c_size_t()
    _check("su3_spinor_bytes",
           load().su3_spinor_bytes(_dims(dims), prec, layout, lanes, ctypes.byref(n)))
    return n.value


def su3_spinor_alloc(dims, prec, layout, lanes=0):
    h = ctypes.c_void_p()
    _check("su3_spinor_alloc",
           load().su3_spinor_alloc(ctypes.byref(h), _dims(dims), prec, layout, lanes))
    return Field(h.value, tuple(dims), prec, layout, lanes, spinor=True)


def su3_spinor_wrap(tensor_or_ptr, dims, prec, layout, lanes=0, nbytes=None):
    """Describe device memory as a spinor field (as su3_field_wrap)."""
    if isinstance(tensor_or_ptr, torch.Tensor):
        t = tensor_or_ptr
        ptr = t.data_ptr()
        nbytes = t.numel() * t.element_size() if nbytes is None else nbytes
        owner = t
    else:
        ptr, owner = int(tensor_or_ptr), None
        if nbytes is None:
            raise ValueError("nbytes is required with a raw pointer")
    h = ctypes.c_void_p()
    _check("su3_spinor_wrap",
           load().su3_spinor_wrap(ctypes.byref(h), ptr, nbytes, _dims(dims),
                                  prec, layout, lanes))
    return Field(h.value, tuple(dims), prec, layout, lanes, owner, spinor=True)


def spinor_tensor(dims, prec, layout, lanes=0, device="cuda"):
    """A torch byte tensor sized for a spinor field, wrapped as a Field."""
    n = su3_spinor_bytes(dims, prec, layout, lanes)
    t = torch.zeros(n, dtype=torch.uint8, device=device)
    return su3_spinor_wrap(t, dims, prec, layout, lanes)


def su3_dslash(out: Field, links, inp: Field, stream=None):
    """Wilson hopping term out = D in with links[mu], mu = 0..3."""
    if len(links) != 4:
        raise ValueError("links must hold 4 fields")
    arr = (ctypes.c_void_p * 4)(*[u.handle if u is not None else None
                                  for u in links])
    _check("su3_dslash",
           load().su3_dslash(out.handle if out is not None else None, arr,
                             inp.handle if inp is not None else None,
                             _stream(stream)))


# ------------------------------------------------------- scalar fields

def su3_scalar_bytes(dims, prec, layout, lanes, kind):
    n = ctypes.c_size_t()
    _check("su3_scalar_bytes",
           load().su3_scalar_bytes(_dims(dims), prec, layout, lanes, kind, ctypes.byref(n)))
    return n.value


def su3_scalar_alloc(dims, prec, layout, lanes, kind):
    h = ctypes.c_void_p()
    _check("su3_scalar_alloc",
           load().su3_scalar_alloc(ctypes.byref(h), _dims(dims), prec, layout, lanes, kind))
    return Field(h.value, tuple(dims), prec, layout, lanes, kind=kind)


def su3_scalar_wrap(tensor_or_ptr, dims, prec, layout, lanes, kind, nbytes=None):
    """Describe device memory as a real or complex scalar field."""
    if isinstance(tensor_or_ptr, torch.Tensor):
        t = tensor_or_ptr
        ptr = t.data_ptr()
        nbytes = t.numel() * t.element_size() if nbytes is None else nbytes
        owner = t
    else:
        ptr, owner = int(tensor_or_ptr), None
        if nbytes is None:
            raise ValueError("nbytes is required with a raw pointer")
    h = ctypes.c_void_p()
    _check("su3_scalar_wrap",
           load().su3_scalar_wrap(ctypes.byref(h), ptr, nbytes, _dims(dims), prec, layout,
                                  lanes, kind))
    return Field(h.value, tuple(dims), prec, layout, lanes, owner, kind=kind)


def scalar_tensor(dims, prec, layout, kind, lanes=0, device="cuda"):
    """A torch byte tensor sized for a scalar field, wrapped."""
    n = su3_scalar_bytes(dims, prec, layout, lanes, kind)
    t = torch.zeros(n, dtype=torch.uint8, device=device)
    return su3_scalar_wrap(t, dims, prec, layout, lanes, kind)


# ---------------------------------------------------- expression programs

class Program:
    """A compiled site-local expression (su3_program_create)."""

    def __init__(self, expr, kinds):
        arr = (ctypes.c_int32 * max(1, len(kinds)))(*[int(k) for k in kinds])
        h = ctypes.c_void_p()
        _check("su3_program_create",
               load().su3_program_create(ctypes.byref(h), expr.encode(), len(kinds),
                                         ctypes.cast(arr, ctypes.c_void_p)))
        self.handle = h.value
        self.expr = expr
        self.kinds = tuple(kinds)

    def info(self):
        k, n, r = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check("su3_program_info", load().su3_program_info(self.handle, ctypes.byref(k),
                                                             ctypes.byref(n), ctypes.byref(r)))
        return {"result_kind": k.value, "n_instr": n.value, "n_regs": r.value}

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.su3_program_destroy(self.handle)
            self.handle = None


def su3_program_create(expr, kinds):
    return Program(expr, kinds)


def su3_program_info(p: Program):
    return p.info()


def su3_program_eval(p: Program, z: Field, ops, stream=None):
    arr = (ctypes.c_void_p * max(1, len(ops)))(*[o.handle if o is not None else None
                                                 for o in ops])
    _check("su3_program_eval",
           load().su3_program_eval(p.handle, z.handle if z is not None else None, arr,
                                   len(ops), _stream(stream)))


def su3_program_destroy(p: Program):
    if p.handle:
        _check("su3_program_destroy", load().su3_program_destroy(p.handle))
        p.handle = None


# ------------------------------------------------- virtual-node layout

def su3_vnode_bytes(dims, prec, kind, simd):
    n = ctypes.c_size_t()
    _check("su3_vnode_bytes",
           load().su3_vnode_bytes(_dims(dims), prec, kind, _dims(simd), ctypes.byref(n)))
    return n.value


def su3_vnode_alloc(dims, prec, kind, simd):
    h = ctypes.c_void_p()
    _check("su3_vnode_alloc",
           load().su3_vnode_alloc(ctypes.byref(h), _dims(dims), prec, kind, _dims(simd)))
    return Field(h.value, tuple(dims), prec, SU3_LAYOUT_VNODE, volume(simd),
                 simd=tuple(simd), kind=kind)


def su3_vnode_wrap(tensor_or_ptr, dims, prec, kind, simd, nbytes=None):
    """Describe Grid-layout device memory as a field (as su3_field_wrap)."""
    if isinstance(tensor_or_ptr, torch.Tensor):
        t = tensor_or_ptr
        ptr = t.data_ptr()
        nbytes = t.numel() * t.element_size() if nbytes is None else nbytes
        owner = t
    else:
        ptr, owner = int(tensor_or_ptr), None
        if nbytes is None:
            raise ValueError("nbytes is required with a raw pointer")
    h = ctypes.c_void_p()
    _check("su3_vnode_wrap",
           load().su3_vnode_wrap(ctypes.byref(h), ptr, nbytes, _dims(dims), prec, kind,
                                 _dims(simd)))
    return Field(h.value, tuple(dims), prec, SU3_LAYOUT_VNODE, volume(simd), owner,
                 simd=tuple(simd), kind=kind)


def vnode_tensor(dims, prec, simd, kind=SU3_KIND_MATRIX, device="cuda"):
    """A torch byte tensor sized for a virtual-node field, wrapped."""
    n = su3_vnode_bytes(dims, prec, kind, simd)
    t = torch.zeros(n, dtype=torch.uint8, device=device)
    return su3_vnode_wrap(t, dims, prec, kind, simd)


# --------------------------------------------------------------- batches

class Batch:
    def __init__(self, handle, fields):
        self.handle = handle
        self._fields = fields  # keep every field alive with the batch

    def __del__(self):
        if self.handle and _lib is not None:
            _lib.su3_batch_destroy(self.handle)
            self.handle = None


def su3_batch_create(exprs, zs, ops, stream=None):
    """exprs[i], zs[i] and ops[i] (a list of operand Fields) per item."""
    n, ex, zz, oo = _batch_args(exprs, zs, ops)
    h = ctypes.c_void_p()
    _check("su3_batch_create",
           load().su3_batch_create(ctypes.byref(h), ex, zz, oo, n, _stream(stream)))
    return Batch(h.value, (list(zs), [list(o) for o in ops]))


def _batch_args(exprs, zs, ops):
    n = len(exprs)
    ex = (ctypes.c_int32 * n)(*exprs)
    zz = (ctypes.c_void_p * n)(*[z.handle for z in zs])
    flat = []
    for o in ops:
        flat.extend([f.handle for f in o] + [None] * (4 - len(o)))
    oo = (ctypes.c_void_p * (4 * n))(*flat)
    return n, ex, zz, oo


def su3_batch_autotune(exprs, zs, ops, stream=None):
    n, ex, zz, oo = _batch_args(exprs, zs, ops)
    best = su3_launch()
    _check("su3_batch_autotune",
           load().su3_batch_autotune(ex, zz, oo, n, _stream(stream), ctypes.byref(best)))
    return best


def su3_batch_run(exprs, zs, ops, stream=None):
    """The batch's items evaluated once, with no device allocation."""
    n, ex, zz, oo = _batch_args(exprs, zs, ops)
    _check("su3_batch_run", load().su3_batch_run(ex, zz, oo, n, _stream(stream)))


def su3_batch_launch(b: Batch, stream=None):
    _check("su3_batch_launch", load().su3_batch_launch(b.handle, _stream(stream)))


def su3_batch_destroy(b: Batch):
    if b.handle:
        _check("su3_batch_destroy", load().su3_batch_destroy(b.handle))
        b.handle = None


def su3_batch_tiles(b: Batch):
    n = ctypes.c_int64()
    _check("su3_batch_tiles", load().su3_batch_tiles(b.handle, None, 0, ctypes.byref(n)))
    rows = np.zeros((n.value, 4), dtype=np.int32)
    _check("su3_batch_tiles",
           load().su3_batch_tiles(b.handle, rows.ctypes.data, n.value, ctypes.byref(n)))
    return rows


# ----------------------------------------------------------- launch tuning

def su3_autotune(expr, prec, layout, lanes, dims, stream=None):
    best = su3_launch()
    _check("su3_autotune", load().su3_autotune(expr, prec, layout, lanes, _dims(dims),
                                               _stream(stream), ctypes.byref(best)))
    return best


def su3_layout_recommend(expr, prec, dims, stream=None):
    """Returns (layout, lanes, tuned launch, median microseconds)."""
    lay, lanes = ctypes.c_int32(), ctypes.c_int32()
    best, us = su3_launch(), ctypes.c_double()
    _check("su3_layout_recommend",
           load().su3_layout_recommend(expr, prec, _dims(dims), _stream(stream),
                                       ctypes.byref(lay), ctypes.byref(lanes),
                                       ctypes.byref(best), ctypes.byref(us)))
    return lay.value, lanes.value, best, us.value


def su3_launch_get(expr, prec, layout, lanes, dims):
    out = su3_launch()
    _check("su3_launch_get", load().su3_launch_get(expr, prec, layout, lanes,
                                                   _dims(dims), ctypes.byref(out)))
    return out


def su3_launch_set(expr, prec, layout, lanes, dims, cfg):
    if isinstance(cfg, dict):
        cfg = su3_launch(**cfg)
    _check("su3_launch_set", load().su3_launch_set(expr, prec, layout, lanes,
                                                   _dims(dims), ctypes.byref(cfg)))


def su3_launch_reset():
    _check("su3_launch_reset", load().su3_launch_reset())


# ------------------------------------------------------------ yardsticks

SU3_STREAM_TRIAD, SU3_STREAM_READ, SU3_STREAM_WRITE, SU3_STREAM_COPY = range(4)


def su3_stream(kind, a, b, c, s, nbytes, cfg=None, stream=None):
    if isinstance(cfg, dict):
        cfg = su3_launch(**cfg)
    _check("su3_stream", load().su3_stream(kind, a, b, c, float(s), int(nbytes),
                                           ctypes.byref(cfg) if cfg is not None else None,
                                           _stream(stream)))


def su3_stream_autotune(kind, a, b, c, nbytes, stream=None):
    """Returns (best launch, its median microseconds)."""
    best = su3_launch()
    us = ctypes.c_double()
    _check("su3_stream_autotune",
           load().su3_stream_autotune(kind, a, b, c, int(nbytes), _stream(stream),
                                      ctypes.byref(best), ctypes.byref(us)))
    return best, us.value


def su3_triad(a, b, c, s, n, stream=None):
    _check("su3_triad", load().su3_triad(a, b, c, float(s), int(n), _stream(stream)))


def su3_copy(dst, src, nbytes, stream=None):
    _check("su3_copy", load().su3_copy(dst, src, int(nbytes), _stream(stream)))


def su3_sync(stream=None):
    _check("su3_sync", load().su3_sync(_stream(stream)))


def su3_status_string(status):
    return _status_name(status)


def su3_last_error():
    return load().su3_last_error().decode()
