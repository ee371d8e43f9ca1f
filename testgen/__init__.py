"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the
benchmark.

Holds no product arithmetic: it only draws Haar-random SU(3) matrices
(``gen.c``), builds small structured fixtures (identity, diagonal phases,
signed permutations, scalar multiples of the identity) and the seeded list
of uneven lattices of the batched workload.  Everything is returned in the
canonical host layout: float64 array of shape (V, 3, 3, 2), site-major,
row i, column j, (re, im).
"""
from __future__ import annotations

import ctypes
import hashlib
import itertools
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.c")
_LIB = os.path.join(_HERE, "libsu3gen.so")

DEFAULT_SEED = 1710
# field ids of the named workloads
FID_X, FID_Y = 0, 1
FID_U0 = 2            # U_mu = 2 + mu
FID_BATCH_LIST = 100  # stream that draws the batch's lattice list
FID_BATCH_BASE = 1000 # lattice i uses 1000 + 4*i + k for operand k


def build() -> str:
    """Compile gen.c into libsu3gen.so (always recompiles)."""
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
           "-D_DEFAULT_SOURCE", _SRC, "-o", _LIB + ".tmp", "-lm"]
    subprocess.check_call(cmd)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        lib.su3gen_u64.restype = ctypes.c_uint64
        lib.su3gen_u64.argtypes = [ctypes.c_uint64] * 3
        lib.su3gen_field.restype = None
        lib.su3gen_field.argtypes = [ctypes.c_uint64, ctypes.c_uint64,
                                     ctypes.c_int64, ctypes.c_int64,
                                     ctypes.c_void_p]
        lib.su3gen_sites.restype = None
        lib.su3gen_spinor.argtypes = [ctypes.c_uint64, ctypes.c_uint64,
                                      ctypes.c_int64, ctypes.c_int64,
                                      ctypes.c_void_p]
        lib.su3gen_spinor.restype = None
        lib.su3gen_sites.argtypes = [ctypes.c_uint64, ctypes.c_uint64,
                                     ctypes.c_void_p, ctypes.c_int64,
                                     ctypes.c_void_p]
        _lib = lib
    return _lib


def volume(dims) -> int:
    v = 1
    for d in dims:
        v *= int(d)
    return v


def u64(seed: int, field_id: int, n: int) -> int:
    """The n-th raw 64-bit draw of stream (seed, field_id)."""
    return int(_load().su3gen_u64(seed, field_id, n))


def su3_field(V: int, seed: int = DEFAULT_SEED, field_id: int = FID_X,
              s_begin: int = 0) -> np.ndarray:
    """Random SU(3) matrices of sites s_begin .. s_begin+V-1, shape (V,3,3,2)."""
    out = np.empty((V, 3, 3, 2), dtype=np.float64)
    if V:
        _load().su3gen_field(seed, field_id, s_begin, V,
                             out.ctypes.data_as(ctypes.c_void_p))
    return out


def su3_sites(sites, seed: int = DEFAULT_SEED,
              field_id: int = FID_X) -> np.ndarray:
    """Random SU(3) matrices of an arbitrary list of sites (same values as
    su3_field at those sites)."""
    s = np.ascontiguousarray(np.asarray(sites, dtype=np.int64))
    out = np.empty((s.size, 3, 3, 2), dtype=np.float64)
    if s.size:
        _load().su3gen_sites(seed, field_id,
                             s.ctypes.data_as(ctypes.c_void_p), s.size,
                             out.ctypes.data_as(ctypes.c_void_p))
    return out


def spinor_field(V: int, seed: int = DEFAULT_SEED, field_id: int = 200,
                 s_begin: int = 0) -> np.ndarray:
    """Gaussian spinor field, shape (V, 4, 3, 2): spin, colour, re/im."""
    out = np.empty((V, 4, 3, 2), dtype=np.float64)
    if V:
        _load().su3gen_spinor(seed, field_id, s_begin, V,
                              out.ctypes.data_as(ctypes.c_void_p))
    return out


def buffer_sha256(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).view(np.uint8)).hexdigest()


# ---------------------------------------------------------------- fixtures

def identity(V: int, scale: float = 1.0) -> np.ndarray:
    out = np.zeros((V, 3, 3, 2), dtype=np.float64)
    for i in range(3):
        out[:, i, i, 0] = scale
    return out


def phase_diag(alpha: np.ndarray, beta: np.ndarray) -> np.ndarray:
    """diag(e^{i a}, e^{i b}, e^{-i(a+b)}) per site (an SU(3) element)."""
    alpha = np.asarray(alpha, dtype=np.float64)
    beta = np.asarray(beta, dtype=np.float64)
    V = alpha.size
    out = np.zeros((V, 3, 3, 2), dtype=np.float64)
    for i, ph in enumerate((alpha, beta, -(alpha + beta))):
        out[:, i, i, 0] = np.cos(ph)
        out[:, i, i, 1] = np.sin(ph)
    return out


def signed_permutations() -> list:
    """All 3x3 real signed permutation matrices with determinant +1
    (a group of order 24), as integer arrays."""
    mats = []
    for perm in itertools.permutations(range(3)):
        for signs in itertools.product((1, -1), repeat=3):
            m = np.zeros((3, 3), dtype=np.int64)
            for i in range(3):
                m[i, perm[i]] = signs[i]
            if round(np.linalg.det(m)) == 1:
                mats.append(m)
    return mats


def from_int_matrices(mats) -> np.ndarray:
    """Canonical field from a list of integer 3x3 matrices (real entries)."""
    V = len(mats)
    out = np.zeros((V, 3, 3, 2), dtype=np.float64)
    for s, m in enumerate(mats):
        out[s, :, :, 0] = m
    return out


# ------------------------------------------------------- batched workload

BATCH_VOLUMES = ((8, 8, 8, 8), (12, 12, 12, 12), (16, 16, 16, 32),
                 (24, 24, 24, 48), (32, 32, 32, 32))


def batch_lattices(n: int = 64, seed: int = DEFAULT_SEED):
    """The seeded list of uneven lattices of the batched workload.

    Lattice i draws r = u64(seed, FID_BATCH_LIST, i); its dims are
    BATCH_VOLUMES[r % 5] and its storage is double precision when bit 32 of
    r is clear, compressed two-row single precision when it is set.
    Returns a list of (dims, compressed: bool).
    """
    out = []
    for i in range(n):
        r = u64(seed, FID_BATCH_LIST, i)
        out.append((BATCH_VOLUMES[r % 5], bool((r >> 32) & 1)))
    return out
