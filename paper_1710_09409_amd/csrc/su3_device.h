// Device-side building blocks of the site-local kernels (gfx950, wave64).
//
// One lane evaluates the expression for S consecutive sites.  In the
// blocked layouts (SoA, AoSoA with L >= S) the S sites' copies of one
// complex entry are adjacent, so each entry of each operand is a single
// 16-byte load per lane and a wave moves 1 KB per instruction: the
// coalesced access that the paper's AoS-vs-coalesced measurements
// (Section 4) and its vector layout (Section 5) are about.  S = 16 bytes /
// (2 * sizeof(stored real)): double 1, float 2, half 4.
//
// Arithmetic: double for F64 storage, single otherwise; products use fused
// multiply-add.  The compressed form keeps rows 0-1 and rebuilds row 2 of
// every right-hand operand as conj(row0 x row1) in registers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "su3_internal.h"

namespace su3k {

using su3i::Geom;

template <int P> struct PrecT;
template <> struct PrecT<su3i::F64> {
    using R = double;   // stored real
    using T = double;   // arithmetic
    static constexpr int E = 9;
    static constexpr int SN = 1;
};
template <> struct PrecT<su3i::F32> {
    using R = float;
    using T = float;
    static constexpr int E = 9;
    static constexpr int SN = 2;
};
template <> struct PrecT<su3i::F16> {
    using R = _Float16;
    using T = float;
    static constexpr int E = 9;
    static constexpr int SN = 4;
};
template <> struct PrecT<su3i::C12> {
    using R = float;
    using T = float;
    static constexpr int E = 6;
    static constexpr int SN = 2;
};

template <int P, int X> struct Supported {
    static constexpr bool value =
        P != su3i::C12 || X == su3i::MUL || X == su3i::MUL3;
};

template <int X> struct NOps {
    static constexpr int value =
        X == su3i::MUL3 ? 3 : (X == su3i::MULADD ? 4 : 2);
};

template <class T> struct Cx {
    T re, im;
};

template <class R, int N> struct VecOf {
    typedef R type __attribute__((ext_vector_type(N)));
};

// Nontemporal bit 0 = loads, bit 1 = stores, bit 2 (with bit 1) =
// write-through streaming stores (below).
template <int NT, class V>
__device__ __forceinline__ V vload(const V *p)
{
    if constexpr (NT & 1)
        return __builtin_nontemporal_load(p);
    else
        return *p;
}

// Buffer descriptor word 3 of the gfx9 family (raw byte buffer) and the
// cache-policy bits of a streaming store: nt (bit 1) with sc1 (bit 4),
// i.e. nontemporal and written through at system scope.  On gfx950 these
// stores stream results to HBM 1.5-2 % faster than plain nontemporal
// stores (2:1 read:write mixes at 48^4) and no kernel here reads back
// what it writes.
constexpr int kBufWord3 = 0x00020000;
constexpr int kStreamStoreAux = 2 | 16;

// A wave-uniform buffer base for streaming stores: the first active lane's
// address less 2 GiB, and this lane's 32-bit offset from it.  Every lane of
// the wave within 2 GiB of that address (all stores of these kernels: a
// wave writes consecutive sites) gets a valid offset, whatever the field's
// size; a uniform displacement (another entry plane) moves the base only.
struct StreamBase {
    uint64_t base;  // wave-uniform
    uint32_t off;   // per lane
};

__device__ __forceinline__ StreamBase stream_base(const void *p)
{
    const uint64_t a = reinterpret_cast<uint64_t>(p);
    const uint32_t lo = __builtin_amdgcn_readfirstlane(uint32_t(a));
    const uint32_t hi = __builtin_amdgcn_readfirstlane(uint32_t(a >> 32));
    const uint64_t base = ((uint64_t(hi) << 32) | lo) - (uint64_t(1) << 31);
    return {base, uint32_t(a - base)};
}

// Streaming store of one 2-, 4-, 8-, 16- or 32-byte value at b.base +
// delta + b.off (delta wave-uniform).
template <class V>
__device__ __forceinline__ void stream_store_at(const StreamBase &b, uint64_t delta, V v)
{
    typedef unsigned U2 __attribute__((ext_vector_type(2)));
    typedef unsigned U4 __attribute__((ext_vector_type(4)));
    typedef unsigned U8 __attribute__((ext_vector_type(8)));
    const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(
        reinterpret_cast<void *>(b.base + delta), (short)0, -1, kBufWord3);
    const uint32_t off = b.off;
    if constexpr (sizeof(V) == 32) {
        const U8 w = __builtin_bit_cast(U8, v);
        __builtin_amdgcn_raw_buffer_store_b128(w.lo, r, off, 0, kStreamStoreAux);
        __builtin_amdgcn_raw_buffer_store_b128(w.hi, r, off + 16, 0, kStreamStoreAux);
    } else if constexpr (sizeof(V) == 16)
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(U4, v), r, off, 0,
                                               kStreamStoreAux);
    else if constexpr (sizeof(V) == 8)
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(U2, v), r, off, 0,
                                              kStreamStoreAux);
    else if constexpr (sizeof(V) == 4)
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, off,
                                              0, kStreamStoreAux);
    else {
        static_assert(sizeof(V) == 2, "stream_store: 2, 4, 8, 16 or 32 bytes");
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, v), r,
                                              off, 0, kStreamStoreAux);
    }
}

// Streaming store of one value at p (its own wave-uniform base).
template <class V>
__device__ __forceinline__ void stream_store(V *p, V v)
{
    stream_store_at(stream_base(p), 0, v);
}

template <int NT, class V>
__device__ __forceinline__ void vstore(V *p, V v)
{
    if constexpr ((NT & 6) == 6)
        stream_store(p, v);
    else if constexpr (NT & 2)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

// Offset (stored reals) of entry 0 of site s; s is a multiple of S.
__device__ __forceinline__ uint32_t site_offset(const Geom &g, uint32_t s)
{
    return (s >> g.lg) * g.bstride + ((s & g.mask) << 1);
}

// ------------------------------------------------------- matrix algebra

// Fused multiply-add in the arithmetic type (float stays float).
__device__ __forceinline__ float fma_t(float a, float b, float c)
{
    return __builtin_fmaf(a, b, c);
}
__device__ __forceinline__ double fma_t(double a, double b, double c)
{
    return __builtin_fma(a, b, c);
}

// c = a * b for rows 0 .. ROWS-1 of c:  c_ij = sum_k a_ik b_kj.
template <int ROWS, class T>
__device__ __forceinline__ void mat_mul(const Cx<T> (&a)[9],
                                        const Cx<T> (&b)[9], Cx<T> (&c)[9])
{
#pragma unroll
    for (int i = 0; i < ROWS; ++i) {
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            T re = a[3 * i].re * b[j].re;
            T im = a[3 * i].re * b[j].im;
            re = fma_t(-a[3 * i].im, b[j].im, re);
            im = fma_t(a[3 * i].im, b[j].re, im);
#pragma unroll
            for (int k = 1; k < 3; ++k) {
                re = fma_t(a[3 * i + k].re, b[3 * k + j].re, re);
                re = fma_t(-a[3 * i + k].im, b[3 * k + j].im, re);
                im = fma_t(a[3 * i + k].re, b[3 * k + j].im, im);
                im = fma_t(a[3 * i + k].im, b[3 * k + j].re, im);
            }
            c[3 * i + j].re = re;
            c[3 * i + j].im = im;
        }
    }
}

template <class T>
__device__ __forceinline__ void mat_add(const Cx<T> (&a)[9],
                                        const Cx<T> (&b)[9], Cx<T> (&c)[9])
{
#pragma unroll
    for (int t = 0; t < 9; ++t) {
        c[t].re = a[t].re + b[t].re;
        c[t].im = a[t].im + b[t].im;
    }
}

// Row 2 of an SU(3) matrix from rows 0 and 1: r2_k = conj(r0_p r1_q -
// r0_q r1_p) with (k, p, q) cyclic.
template <class T>
__device__ __forceinline__ void rebuild_row2(Cx<T> (&m)[9])
{
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int p = (k + 1) % 3, q = (k + 2) % 3;
        const Cx<T> a = m[p], b = m[3 + q], c = m[q], d = m[3 + p];
        T re = a.re * b.re;
        re = fma_t(-a.im, b.im, re);
        re = fma_t(-c.re, d.re, re);
        re = fma_t(c.im, d.im, re);
        T im = a.re * b.im;
        im = fma_t(a.im, b.re, im);
        im = fma_t(-c.re, d.im, im);
        im = fma_t(-c.im, d.re, im);
        m[6 + k].re = re;
        m[6 + k].im = -im;
    }
}

// z = X(ops) for one site.  For the compressed form only rows 0-1 of z are
// produced and right-hand operands get row 2 rebuilt first.
template <int P, int X, class T>
__device__ __forceinline__ void eval_site(Cx<T> (&o)[NOps<X>::value][9],
                                          Cx<T> (&z)[9])
{
    constexpr bool c12 = P == su3i::C12;
    constexpr int ROWS = c12 ? 2 : 3;
    if constexpr (X == su3i::MUL) {
        if constexpr (c12)
            rebuild_row2(o[1]);
        mat_mul<ROWS>(o[0], o[1], z);
    } else if constexpr (X == su3i::MUL3) {
        Cx<T> t[9];
        if constexpr (c12) {
            rebuild_row2(o[1]);
            rebuild_row2(o[2]);
        }
        mat_mul<ROWS>(o[0], o[1], t);
        mat_mul<ROWS>(t, o[2], z);
    } else if constexpr (X == su3i::MULADD) {
        Cx<T> t[9], u[9];
        mat_mul<3>(o[0], o[1], t);
        mat_mul<3>(o[2], o[3], u);
        mat_add(t, u, z);
    } else if constexpr (X == su3i::ADD) {
        mat_add(o[0], o[1], z);
    } else {  // APB_AB = (a + b) + (a * b)
        Cx<T> t[9], u[9];
        mat_add(o[0], o[1], t);
        mat_mul<3>(o[0], o[1], u);
        mat_add(t, u, z);
    }
}

// ----------------------------------------------- one group of S sites

// Sites per lane: one 16-byte access per entry (double 1, float 2, half 4),
// except half storage with 3-4 operands, which takes 2 sites (8-byte
// accesses, still whole 128-byte lines per wave) to stay within the
// register file.
template <int P, int X> struct SitesPerLane {
    static constexpr int value =
        (P == su3i::F16 && NOps<X>::value > 2) ? 2 : PrecT<P>::SN;
};

template <int P, int S>
using RawVec = typename VecOf<typename PrecT<P>::R, 2 * S>::type;

// Load stored entries e0 .. e0+NE-1 of S adjacent sites of one operand as
// raw vectors (FULL), or of the first `cnt` of them (tail group; the other
// slots are zero and never stored).
template <int P, int S, int NT, bool FULL, int E0, int NE>
__device__ __forceinline__ void load_entries(const typename PrecT<P>::R *base,
                                             uint32_t off, uint32_t plane,
                                             int cnt, RawVec<P, S> *raw)
{
    using R = typename PrecT<P>::R;
    using V = RawVec<P, S>;
    using V2 = typename VecOf<R, 2>::type;
#pragma unroll
    for (int t = 0; t < NE; ++t) {
        const R *p = base + off + (E0 + t) * plane;
        if constexpr (FULL) {
            raw[t] = vload<NT>(reinterpret_cast<const V *>(p));
        } else {
            V v;
#pragma unroll
            for (int j = 0; j < S; ++j) {
                V2 w;
                if (j < cnt) {
                    w = vload<NT>(reinterpret_cast<const V2 *>(p + 2 * j));
                } else {
                    w[0] = R(0);
                    w[1] = R(0);
                }
                v[2 * j] = w[0];
                v[2 * j + 1] = w[1];
            }
            raw[t] = v;
        }
    }
}

template <int P, int S, int NT, bool FULL, int E0, int NE>
__device__ __forceinline__ void store_entries(typename PrecT<P>::R *base,
                                              uint32_t off, uint32_t plane,
                                              int cnt,
                                              const RawVec<P, S> *raw)
{
    using R = typename PrecT<P>::R;
    using V = RawVec<P, S>;
    using V2 = typename VecOf<R, 2>::type;
    if constexpr (FULL && (NT & 6) == 6) {
        // streaming stores: one wave-uniform base for every entry, each
        // entry plane a uniform displacement of it
        const StreamBase b = stream_base(base + off + E0 * plane);
#pragma unroll
        for (int t = 0; t < NE; ++t)
            stream_store_at(b, uint64_t(t) * plane * sizeof(R), raw[t]);
        return;
    }
#pragma unroll
    for (int t = 0; t < NE; ++t) {
        R *p = base + off + (E0 + t) * plane;
        if constexpr (FULL) {
            vstore<NT>(reinterpret_cast<V *>(p), raw[t]);
        } else {
#pragma unroll
            for (int j = 0; j < S; ++j) {
                if (j < cnt) {
                    V2 w;
                    w[0] = raw[t][2 * j];
                    w[1] = raw[t][2 * j + 1];
                    vstore<NT>(reinterpret_cast<V2 *>(p + 2 * j), w);
                }
            }
        }
    }
}

// Widen entry slot `t` of site `j` from a raw vector.
template <int P, int S>
__device__ __forceinline__ Cx<typename PrecT<P>::T> widen(const RawVec<P, S> &v,
                                                          int j)
{
    using T = typename PrecT<P>::T;
    Cx<T> c;
    c.re = (T)v[2 * j];
    c.im = (T)v[2 * j + 1];
    return c;
}

template <int P, int S>
__device__ __forceinline__ void narrow(RawVec<P, S> &v, int j,
                                       const Cx<typename PrecT<P>::T> &c)
{
    using R = typename PrecT<P>::R;
    using T = typename PrecT<P>::T;
    T re = c.re, im = c.im;
    if constexpr (P == su3i::F16) {
        // Keep the single-precision result: without the barrier the
        // compiler fuses the last FMA with the conversion (v_fma_mixlo_f16,
        // one rounding) in some code shapes and not in others, so results
        // would depend on the launch settings.  The declared convention is
        // FP32 arithmetic, then one round-to-nearest-even to half.
        __asm__("" : "+v"(re));
        __asm__("" : "+v"(im));
    }
    v[2 * j] = (R)re;
    v[2 * j + 1] = (R)im;
}

// Which operands an expression reads row by row (left) and in full (right).
template <int X> struct Split;
template <> struct Split<su3i::MUL> {
    static constexpr int NL = 1, NR = 1;
    static constexpr int L[1] = {0}, Rt[1] = {1};
};
template <> struct Split<su3i::MUL3> {
    static constexpr int NL = 1, NR = 2;
    static constexpr int L[1] = {0}, Rt[2] = {1, 2};
};
template <> struct Split<su3i::MULADD> {
    static constexpr int NL = 2, NR = 2;
    static constexpr int L[2] = {0, 2}, Rt[2] = {1, 3};
};
template <> struct Split<su3i::ADD> {
    static constexpr int NL = 2, NR = 0;
    static constexpr int L[2] = {0, 1}, Rt[1] = {0};
};
template <> struct Split<su3i::APB_AB> {
    static constexpr int NL = 1, NR = 1;
    static constexpr int L[1] = {0}, Rt[1] = {1};
};

template <int X>
__device__ __forceinline__ constexpr bool is_right(int k)
{
    for (int i = 0; i < Split<X>::NR; ++i)
        if (Split<X>::Rt[i] == k)
            return true;
    return false;
}

// Schedule 0: every operand entry of the group is loaded (as raw stored
// vectors), then evaluated, then every result entry is stored.
template <int P, int X, int S, int NT, bool FULL>
__device__ __forceinline__ void group_all(void *zp, const void *const (&opp)[4],
                                          uint32_t off, uint32_t off_r,
                                          uint32_t plane, int cnt)
{
    using R = typename PrecT<P>::R;
    using T = typename PrecT<P>::T;
    constexpr int N = NOps<X>::value;
    constexpr int E = PrecT<P>::E;
    RawVec<P, S> raw[N][E];
#pragma unroll
    for (int k = 0; k < N; ++k)
        load_entries<P, S, NT, FULL, 0, E>(static_cast<const R *>(opp[k]),
                                           is_right<X>(k) ? off_r : off, plane,
                                           cnt, raw[k]);
    RawVec<P, S> zr[E];
#pragma unroll
    for (int j = 0; j < S; ++j) {
        Cx<T> o[N][9];
#pragma unroll
        for (int k = 0; k < N; ++k)
#pragma unroll
            for (int e = 0; e < E; ++e)
                o[k][e] = widen<P, S>(raw[k][e], j);
        Cx<T> z[9];
        eval_site<P, X>(o, z);
#pragma unroll
        for (int e = 0; e < E; ++e)
            narrow<P, S>(zr[e], j, z[e]);
    }
    store_entries<P, S, NT, FULL, 0, E>(static_cast<R *>(zp), off, plane, cnt,
                                        zr);
}

// Row i of a product: c_i = a_i * b, the same FMA sequence as mat_mul.
template <class T>
__device__ __forceinline__ void row_mul(const Cx<T> *a, const Cx<T> (&b)[9],
                                        Cx<T> *c)
{
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        T re = a[0].re * b[j].re;
        T im = a[0].re * b[j].im;
        re = fma_t(-a[0].im, b[j].im, re);
        im = fma_t(a[0].im, b[j].re, im);
#pragma unroll
        for (int k = 1; k < 3; ++k) {
            re = fma_t(a[k].re, b[3 * k + j].re, re);
            re = fma_t(-a[k].im, b[3 * k + j].im, re);
            im = fma_t(a[k].re, b[3 * k + j].im, im);
            im = fma_t(a[k].im, b[3 * k + j].re, im);
        }
        c[j].re = re;
        c[j].im = im;
    }
}

template <class T>
__device__ __forceinline__ void row_add(const Cx<T> *a, const Cx<T> *b, Cx<T> *c)
{
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        c[j].re = a[j].re + b[j].re;
        c[j].im = a[j].im + b[j].im;
    }
}

// Row i of z from the rows i of the left operands and the full right ones.
template <int X, class T>
__device__ __forceinline__ void eval_row(const Cx<T> (&l)[2][3],
                                         const Cx<T> (&r)[2][9], int i,
                                         Cx<T> *z)
{
    if constexpr (X == su3i::MUL) {
        row_mul(l[0], r[0], z);
    } else if constexpr (X == su3i::MUL3) {
        Cx<T> t[3];
        row_mul(l[0], r[0], t);
        row_mul(t, r[1], z);
    } else if constexpr (X == su3i::MULADD) {
        Cx<T> t[3], u[3];
        row_mul(l[0], r[0], t);
        row_mul(l[1], r[1], u);
        row_add(t, u, z);
    } else if constexpr (X == su3i::ADD) {
        row_add(l[0], l[1], z);
    } else {  // APB_AB = (a + b) + (a * b)
        Cx<T> t[3], u[3];
        row_add(l[0], &r[0][3 * i], t);
        row_mul(l[0], r[0], u);
        row_add(t, u, z);
    }
}

// Schedule 1, row-phased: the right-hand operands are loaded in full, then
// for each result row the left operands' row is loaded, the row evaluated
// and stored before the next row's loads, so every wave alternates loads
// and stores instead of issuing all loads and then all stores.  Same
// arithmetic, same bits as schedule 0.
template <int P, int X, int S, int NT, bool FULL>
__device__ __forceinline__ void group_rows(void *zp, const void *const (&opp)[4],
                                           uint32_t off, uint32_t off_r,
                                           uint32_t plane, int cnt)
{
    using R = typename PrecT<P>::R;
    using T = typename PrecT<P>::T;
    using SP = Split<X>;
    constexpr int E = PrecT<P>::E;
    constexpr int ROWS = E / 3;
    RawVec<P, S> rr[SP::NR > 0 ? SP::NR : 1][E];
#pragma unroll
    for (int k = 0; k < SP::NR; ++k)
        load_entries<P, S, NT, FULL, 0, E>(static_cast<const R *>(opp[SP::Rt[k]]),
                                           off_r, plane, cnt, rr[k]);
#pragma unroll
    for (int i = 0; i < ROWS; ++i) {
        RawVec<P, S> lr[SP::NL][3];
#pragma unroll
        for (int k = 0; k < SP::NL; ++k) {
            const R *base = static_cast<const R *>(opp[SP::L[k]]);
            if (i == 0)
                load_entries<P, S, NT, FULL, 0, 3>(base, off, plane, cnt, lr[k]);
            else if (i == 1)
                load_entries<P, S, NT, FULL, 3, 3>(base, off, plane, cnt, lr[k]);
            else
                load_entries<P, S, NT, FULL, 6, 3>(base, off, plane, cnt, lr[k]);
        }
        __builtin_amdgcn_sched_barrier(0);
        RawVec<P, S> zr[3];
#pragma unroll
        for (int j = 0; j < S; ++j) {
            Cx<T> l[2][3], r[2][9];
#pragma unroll
            for (int k = 0; k < SP::NL; ++k)
#pragma unroll
                for (int e = 0; e < 3; ++e)
                    l[k][e] = widen<P, S>(lr[k][e], j);
#pragma unroll
            for (int k = 0; k < SP::NR; ++k) {
#pragma unroll
                for (int e = 0; e < E; ++e)
                    r[k][e] = widen<P, S>(rr[k][e], j);
                if constexpr (P == su3i::C12)
                    rebuild_row2(r[k]);
            }
            Cx<T> z[3];
            eval_row<X>(l, r, i, z);
#pragma unroll
            for (int e = 0; e < 3; ++e)
                narrow<P, S>(zr[e], j, z[e]);
        }
        R *zb = static_cast<R *>(zp);
        if (i == 0)
            store_entries<P, S, NT, FULL, 0, 3>(zb, off, plane, cnt, zr);
        else if (i == 1)
            store_entries<P, S, NT, FULL, 3, 3>(zb, off, plane, cnt, zr);
        else
            store_entries<P, S, NT, FULL, 6, 3>(zb, off, plane, cnt, zr);
        __builtin_amdgcn_sched_barrier(0);
    }
}

// Evaluate X for the group of S sites at stored offset `off` (the result
// and the left operands); the right-hand operands are read at `off_r`
// (equal to `off` except for a shifted operand).  Every operand entry a
// result entry depends on is loaded before that result entry is stored, so
// z may be one of the operands read at `off` (in-place).
template <int P, int X, int S, int NT, bool FULL, int SCHED>
__device__ __forceinline__ void do_group(void *zp, const void *const (&opp)[4],
                                         uint32_t off, uint32_t off_r,
                                         uint32_t plane, int cnt)
{
    if constexpr (SCHED == 0)
        group_all<P, X, S, NT, FULL>(zp, opp, off, off_r, plane, cnt);
    else
        group_rows<P, X, S, NT, FULL>(zp, opp, off, off_r, plane, cnt);
}

// Workgroup id remapped so that each XCD (workgroups are dealt to the 8
// XCDs round-robin) owns one contiguous range of ids.  A bijection on
// [0, n).
__device__ __forceinline__ int xcd_remap(int b, int n)
{
    const int xcd = b & 7, idx = b >> 3;
    const int q = n >> 3, r = n & 7;
    return xcd * q + (xcd < r ? xcd : r) + idx;
}

}  // namespace su3k
