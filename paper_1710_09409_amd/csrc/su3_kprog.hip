// Program kernel: evaluates a compiled site-local expression (see
// su3_program.cpp) at every site.  One site per lane.  The operand fields
// the program reads are loaded into registers 0 .. nops-1 up front, so all
// of a lane's loads are in flight together; the instructions then run on
// registers, each a uniform branch on the opcode (matrix programs through
// an accumulator, below), and the result register is stored.
//
// A register holds a 3x3 complex matrix (NE = 9; a scalar uses entry 0).
// Programs without matrix values run in their own kernel, whose registers
// hold one complex value for each of the lane's S sites; programs whose
// every value is real (operands, intermediates and result, as in the
// real-valued composite example of Section 3, Listing 2) in a third, whose registers hold one real per site.  Register
// indices are uniform across the wave and are resolved by a chain of
// compare-and-copy branches, so the register file stays in VGPRs.
#include <type_traits>

#include "su3_device.h"
#include "su3_program.h"

namespace su3k {
namespace prog {

using su3i::ProgArgs;
using su3i::ProgInstr;

template <class T, int NE>
struct Reg {
    Cx<T> m[NE];
};

// End of a branch that wrote registers: an empty asm statement with an
// immediate unique to the branch, so that no two branches are merged into
// one copy through a selected address (which would move the register file
// to scratch memory).
template <int N>
__device__ __forceinline__ void branch_end()
{
    __asm__ volatile("" ::"n"(N));
}

struct NoReg {};

template <class T, int NE, int NR, int K>
using RegIf = typename std::conditional<(K < NR), Reg<T, NE>, NoReg>::type;

// The register file as separate members (never an indexable array).
template <class T, int NE, int NR>
struct RegFile {
    RegIf<T, NE, NR, 0> r0;
    RegIf<T, NE, NR, 1> r1;
    RegIf<T, NE, NR, 2> r2;
    RegIf<T, NE, NR, 3> r3;
    RegIf<T, NE, NR, 4> r4;
    RegIf<T, NE, NR, 5> r5;
    RegIf<T, NE, NR, 6> r6;
    RegIf<T, NE, NR, 7> r7;

    template <int K>
    __device__ __forceinline__ RegIf<T, NE, NR, K> &at()
    {
        if constexpr (K == 0) return r0;
        else if constexpr (K == 1) return r1;
        else if constexpr (K == 2) return r2;
        else if constexpr (K == 3) return r3;
        else if constexpr (K == 4) return r4;
        else if constexpr (K == 5) return r5;
        else if constexpr (K == 6) return r6;
        else return r7;
    }
};

template <class T, int NE, int NR, int K = 0>
__device__ __forceinline__ void get(RegFile<T, NE, NR> &R, int i, Reg<T, NE> &out)
{
    if constexpr (K < NR) {
        if (i == K) {
            out = R.template at<K>();
            branch_end<K>();
        } else {
            get<T, NE, NR, K + 1>(R, i, out);
        }
    }
}

template <class T, int NE, int NR, int K = 0>
__device__ __forceinline__ void put(RegFile<T, NE, NR> &R, int i, const Reg<T, NE> &v)
{
    if constexpr (K < NR) {
        if (i == K) {
            R.template at<K>() = v;
            branch_end<K + 16>();
        } else {
            put<T, NE, NR, K + 1>(R, i, v);
        }
    }
}

template <class T>
__device__ __forceinline__ Cx<T> cmul(Cx<T> a, Cx<T> b)
{
    return {fma_t(a.re, b.re, -(a.im * b.im)), fma_t(a.re, b.im, a.im * b.re)};
}

// Load a matrix operand of storage precision P into r (F32 arithmetic for
// F32 and the compressed form, whose third row is rebuilt).
template <int P, int NT>
__device__ __forceinline__ void load_matrix(const void *base, const su3i::Geom &g,
                                            uint32_t s, Reg<typename PrecT<P>::T, 9> &r)
{
    constexpr int E = PrecT<P>::E;
    RawVec<P, 1> raw[E];
    load_entries<P, 1, NT, true, 0, E>(static_cast<const typename PrecT<P>::R *>(base),
                                       site_offset(g, s), g.plane, 1, raw);
#pragma unroll
    for (int e = 0; e < E; ++e)
        r.m[e] = widen<P, 1>(raw[e], 0);
    if constexpr (P == su3i::C12)
        rebuild_row2(r.m);
}

template <class T, int NE, int NT>
__device__ __forceinline__ void load_operand(const ProgArgs &a, int k, uint32_t s,
                                             Reg<T, NE> &r)
{
    const void *base = a.op[k];
    switch (a.kind[k]) {
    case su3i::FK_MATRIX:
        if constexpr (NE == 9) {
            if constexpr (sizeof(T) == 8) {
                load_matrix<su3i::F64, NT>(base, a.g[k], s, r);
                branch_end<32>();
            } else {
                if (a.prec[k] == su3i::C12) {
                    load_matrix<su3i::C12, NT>(base, a.g[k], s, r);
                    branch_end<33>();
                } else {
                    load_matrix<su3i::F32, NT>(base, a.g[k], s, r);
                    branch_end<34>();
                }
            }
        }
        break;
    case su3i::FK_REAL:
        r.m[0] = {vload<NT & 1>(static_cast<const T *>(base) + s), T(0)};
        branch_end<35>();
        break;
    default: {  // complex scalar
        using V2 = typename VecOf<T, 2>::type;
        const V2 v = vload<NT & 1>(static_cast<const V2 *>(base) + s);
        r.m[0] = {v[0], v[1]};
        branch_end<36>();
        break;
    }
    }
}

// Matrix-form instructions work on an accumulator X: X holds r[a] when an
// instruction starts (it is copied in only when it holds another register)
// and r[d] when it ends (it is copied out every time, so the register file
// stays current).  A binary instruction reads r[b] in place through a
// branch per register, so the kernel keeps the file, X and a row of
// temporaries live instead of three matrix copies.

// X = X * B, one row at a time (row i of the product needs row i of X
// only); each entry is summed as in mat_mul.
template <class T>
__device__ __forceinline__ void mul_into(Reg<T, 9> &X, const Reg<T, 9> &B)
{
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        Cx<T> r[3];
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            T re = X.m[3 * i].re * B.m[j].re;
            T im = X.m[3 * i].re * B.m[j].im;
            re = fma_t(-X.m[3 * i].im, B.m[j].im, re);
            im = fma_t(X.m[3 * i].im, B.m[j].re, im);
#pragma unroll
            for (int k = 1; k < 3; ++k) {
                re = fma_t(X.m[3 * i + k].re, B.m[3 * k + j].re, re);
                re = fma_t(-X.m[3 * i + k].im, B.m[3 * k + j].im, re);
                im = fma_t(X.m[3 * i + k].re, B.m[3 * k + j].im, im);
                im = fma_t(X.m[3 * i + k].im, B.m[3 * k + j].re, im);
            }
            r[j] = {re, im};
        }
#pragma unroll
        for (int j = 0; j < 3; ++j)
            X.m[3 * i + j] = r[j];
    }
}

// X = X (op) B for the binary opcodes OP_ADD_MM .. OP_SUB_MS.  Where a
// scalar X meets a matrix B, entry 0 of X is read by every entry of the
// result and is overwritten last.
template <class T>
__device__ __forceinline__ void binary(int op, Reg<T, 9> &X, const Reg<T, 9> &B)
{
    switch (op) {
    case su3i::OP_ADD_SS:
        X.m[0] = {X.m[0].re + B.m[0].re, X.m[0].im + B.m[0].im};
        break;
    case su3i::OP_SUB_SS:
        X.m[0] = {X.m[0].re - B.m[0].re, X.m[0].im - B.m[0].im};
        break;
    case su3i::OP_MUL_SS:
        X.m[0] = cmul(X.m[0], B.m[0]);
        break;
    case su3i::OP_ADD_MM:
#pragma unroll
        for (int e = 0; e < 9; ++e)
            X.m[e] = {X.m[e].re + B.m[e].re, X.m[e].im + B.m[e].im};
        break;
    case su3i::OP_SUB_MM:
#pragma unroll
        for (int e = 0; e < 9; ++e)
            X.m[e] = {X.m[e].re - B.m[e].re, X.m[e].im - B.m[e].im};
        break;
    case su3i::OP_MUL_MM:
        mul_into(X, B);
        break;
    case su3i::OP_MUL_SM:
#pragma unroll
        for (int e = 8; e >= 0; --e)
            X.m[e] = cmul(X.m[0], B.m[e]);
        break;
    case su3i::OP_MUL_MS:
#pragma unroll
        for (int e = 0; e < 9; ++e)
            X.m[e] = cmul(X.m[e], B.m[0]);
        break;
    case su3i::OP_ADD_SM:
#pragma unroll
        for (int e = 8; e >= 0; --e)
            X.m[e] = e % 4 == 0 ? Cx<T>{X.m[0].re + B.m[e].re, X.m[0].im + B.m[e].im} : B.m[e];
        break;
    case su3i::OP_ADD_MS:
#pragma unroll
        for (int e = 0; e < 9; e += 4)
            X.m[e] = {X.m[e].re + B.m[0].re, X.m[e].im + B.m[0].im};
        break;
    case su3i::OP_SUB_SM:
#pragma unroll
        for (int e = 8; e >= 0; --e)
            X.m[e] = e % 4 == 0 ? Cx<T>{X.m[0].re - B.m[e].re, X.m[0].im - B.m[e].im}
                                : Cx<T>{-B.m[e].re, -B.m[e].im};
        break;
    default:  // OP_SUB_MS
#pragma unroll
        for (int e = 0; e < 9; e += 4)
            X.m[e] = {X.m[e].re - B.m[0].re, X.m[e].im - B.m[0].im};
        break;
    }
}

// The binary instruction with r[i] as B, read where it lives.
template <class T, int NR, int K = 0>
__device__ __forceinline__ void binary_with(RegFile<T, 9, NR> &R, int i, int op, Reg<T, 9> &X)
{
    if constexpr (K < NR) {
        if (i == K) {
            binary<T>(op, X, R.template at<K>());
            branch_end<K + 48>();
        } else {
            binary_with<T, NR, K + 1>(R, i, op, X);
        }
    }
}

// X = op(X) for the other opcodes (OP_CONST ignores X and sets imm[a]).
template <class T>
__device__ __forceinline__ void unary(const ProgInstr in, const ProgArgs &a, Reg<T, 9> &X)
{
    switch (in.op) {
    case su3i::OP_CONST:
        X.m[0] = {T(a.imm[in.a][0]), T(a.imm[in.a][1])};
        break;
    case su3i::OP_NEG_S:
        X.m[0] = {-X.m[0].re, -X.m[0].im};
        break;
    case su3i::OP_CONJ_S:
        X.m[0] = {X.m[0].re, -X.m[0].im};
        break;
    case su3i::OP_REAL:
        X.m[0] = {X.m[0].re, T(0)};
        break;
    case su3i::OP_IMAG:
        X.m[0] = {X.m[0].im, T(0)};
        break;
    case su3i::OP_NEG_M:
#pragma unroll
        for (int e = 0; e < 9; ++e)
            X.m[e] = {-X.m[e].re, -X.m[e].im};
        break;
    case su3i::OP_CONJ_M:
#pragma unroll
        for (int e = 0; e < 9; ++e)
            X.m[e] = {X.m[e].re, -X.m[e].im};
        break;
    case su3i::OP_ADJ_M:
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            X.m[4 * i].im = -X.m[4 * i].im;
#pragma unroll
            for (int j = i + 1; j < 3; ++j) {
                const Cx<T> u = X.m[3 * i + j], v = X.m[3 * j + i];
                X.m[3 * i + j] = {v.re, -v.im};
                X.m[3 * j + i] = {u.re, -u.im};
            }
        }
        break;
    case su3i::OP_TRANS_M:
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = i + 1; j < 3; ++j) {
                const Cx<T> u = X.m[3 * i + j];
                X.m[3 * i + j] = X.m[3 * j + i];
                X.m[3 * j + i] = u;
            }
        break;
    case su3i::OP_TRACE:
        X.m[0] = {(X.m[0].re + X.m[4].re) + X.m[8].re, (X.m[0].im + X.m[4].im) + X.m[8].im};
        break;
    default:
        break;
    }
}

template <class T, int NE>
__device__ __forceinline__ void exec(const ProgInstr in, const ProgArgs &a,
                                     const Reg<T, NE> &A, const Reg<T, NE> &B,
                                     Reg<T, NE> &C)
{
    switch (in.op) {
    case su3i::OP_CONST:
        C.m[0] = {T(a.imm[in.a][0]), T(a.imm[in.a][1])};
        branch_end<96>();
        break;
    case su3i::OP_ADD_SS:
        C.m[0] = {A.m[0].re + B.m[0].re, A.m[0].im + B.m[0].im};
        branch_end<97>();
        break;
    case su3i::OP_SUB_SS:
        C.m[0] = {A.m[0].re - B.m[0].re, A.m[0].im - B.m[0].im};
        branch_end<98>();
        break;
    case su3i::OP_MUL_SS:
        C.m[0] = cmul(A.m[0], B.m[0]);
        branch_end<99>();
        break;
    case su3i::OP_NEG_S:
        C.m[0] = {-A.m[0].re, -A.m[0].im};
        branch_end<100>();
        break;
    case su3i::OP_CONJ_S:
        C.m[0] = {A.m[0].re, -A.m[0].im};
        branch_end<101>();
        break;
    case su3i::OP_REAL:
        C.m[0] = {A.m[0].re, T(0)};
        branch_end<102>();
        break;
    case su3i::OP_IMAG:
        C.m[0] = {A.m[0].im, T(0)};
        branch_end<103>();
        break;
    default:
        branch_end<104>();
        break;
    }
}

template <class T, int NE, int NR, int NT, int K = 0>
__device__ __forceinline__ void load_all(const ProgArgs &a, uint32_t s,
                                         RegFile<T, NE, NR> &R)
{
    if constexpr (K < NR) {
        if (K < a.nops) {
            if ((a.used >> K) & 1)
                load_operand<T, NE, NT>(a, K, s, R.template at<K>());
            load_all<T, NE, NR, NT, K + 1>(a, s, R);
        }
    }
}

template <class T, int NE, int NR, int NT>
__global__ __launch_bounds__(256) void k_program(ProgArgs a)
{
    extern __shared__ char occupancy_reserve[];
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < (uint32_t)a.nsites) {
        RegFile<T, NE, NR> R;
        load_all<T, NE, NR, NT>(a, s, R);
        Reg<T, NE> Z;   // the accumulator
        int held = -1;  // the register Z is a copy of (the same in every lane)
        for (int pc = 0; pc < a.ninstr; ++pc) {
            const ProgInstr in = a.ins[pc];
            if (in.op != su3i::OP_CONST && in.a != held)
                get(R, in.a, Z);
            if (in.op >= su3i::OP_ADD_MM && in.op <= su3i::OP_SUB_MS)
                binary_with<T, NR>(R, in.b, in.op, Z);
            else
                unary<T>(in, a, Z);
            put(R, in.d, Z);
            held = in.d;
        }
        if (a.result != held)
            get(R, a.result, Z);
        switch (a.zkind) {
        case su3i::FK_MATRIX:
            if constexpr (NE == 9) {
                if constexpr (sizeof(T) == 8) {
                    RawVec<su3i::F64, 1> raw[9];
#pragma unroll
                    for (int e = 0; e < 9; ++e)
                        narrow<su3i::F64, 1>(raw[e], 0, Z.m[e]);
                    store_entries<su3i::F64, 1, NT, true, 0, 9>(
                        static_cast<double *>(a.z), site_offset(a.gz, s), a.gz.plane, 1, raw);
                } else if (a.zprec == su3i::C12) {
                    RawVec<su3i::C12, 1> raw[6];
#pragma unroll
                    for (int e = 0; e < 6; ++e)
                        narrow<su3i::C12, 1>(raw[e], 0, Z.m[e]);
                    store_entries<su3i::C12, 1, NT, true, 0, 6>(
                        static_cast<float *>(a.z), site_offset(a.gz, s), a.gz.plane, 1, raw);
                } else {
                    RawVec<su3i::F32, 1> raw[9];
#pragma unroll
                    for (int e = 0; e < 9; ++e)
                        narrow<su3i::F32, 1>(raw[e], 0, Z.m[e]);
                    store_entries<su3i::F32, 1, NT, true, 0, 9>(
                        static_cast<float *>(a.z), site_offset(a.gz, s), a.gz.plane, 1, raw);
                }
            }
            break;
        case su3i::FK_REAL:
            vstore<NT & 2>(static_cast<T *>(a.z) + s, Z.m[0].re);
            break;
        default: {
            using V2 = typename VecOf<T, 2>::type;
            V2 v;
            v[0] = Z.m[0].re;
            v[1] = Z.m[0].im;
            vstore<NT & 2>(static_cast<V2 *>(a.z) + s, v);
            break;
        }
        }
    }
    if (a.nsites < 0)
        occupancy_reserve[threadIdx.x] = 0;
}

// Scalar-only programs: each lane evaluates S consecutive sites (one
// complex value per site in each register), so a site costs 1/S of the
// instruction dispatch and operands move in S-wide vector accesses.
template <class T, int S>
struct SReg {
    Cx<T> v[S];
};

template <class T, int S, int NT>
__device__ __forceinline__ void load_scalars(const ProgArgs &a, int k, uint32_t s0,
                                             int cnt, SReg<T, S> &r)
{
    if (a.kind[k] == su3i::FK_REAL) {
        const T *p = static_cast<const T *>(a.op[k]) + s0;
        if (cnt == S) {
            // 16-byte pieces
            constexpr int W = 16 / sizeof(T);
            using V = typename VecOf<T, W>::type;
#pragma unroll
            for (int q = 0; q < S / W; ++q) {
                const V w = vload<NT & 1>(reinterpret_cast<const V *>(p) + q);
#pragma unroll
                for (int j = 0; j < W; ++j)
                    r.v[q * W + j] = {w[j], T(0)};
            }
        } else {
#pragma unroll
            for (int j = 0; j < S; ++j)
                r.v[j] = {j < cnt ? p[j] : T(0), T(0)};
        }
        branch_end<40>();
    } else {
        using V2 = typename VecOf<T, 2>::type;
        const V2 *p = static_cast<const V2 *>(a.op[k]) + s0;
#pragma unroll
        for (int j = 0; j < S; ++j) {
            V2 w;
            if (cnt == S || j < cnt) {
                w = vload<NT & 1>(p + j);
            } else {
                w[0] = T(0);
                w[1] = T(0);
            }
            r.v[j] = {w[0], w[1]};
        }
        branch_end<41>();
    }
}

template <class T, int S>
__device__ __forceinline__ void exec_scalars(const ProgInstr in, const ProgArgs &a,
                                             const SReg<T, S> &A, const SReg<T, S> &B,
                                             SReg<T, S> &C)
{
#pragma unroll
    for (int j = 0; j < S; ++j) {
        Reg<T, 1> x, y, z;
        x.m[0] = A.v[j];
        y.m[0] = B.v[j];
        exec<T, 1>(in, a, x, y, z);
        C.v[j] = z.m[0];
    }
}

template <class T, int S, int NR, int K = 0>
__device__ __forceinline__ void sget(RegFile<T, S, NR> &R, int i, SReg<T, S> &out)
{
    if constexpr (K < NR) {
        if (i == K) {
            const Reg<T, S> &r = R.template at<K>();
#pragma unroll
            for (int j = 0; j < S; ++j)
                out.v[j] = r.m[j];
            branch_end<K + 48>();
        } else {
            sget<T, S, NR, K + 1>(R, i, out);
        }
    }
}

template <class T, int S, int NR, int K = 0>
__device__ __forceinline__ void sput(RegFile<T, S, NR> &R, int i, const SReg<T, S> &v)
{
    if constexpr (K < NR) {
        if (i == K) {
            Reg<T, S> &r = R.template at<K>();
#pragma unroll
            for (int j = 0; j < S; ++j)
                r.m[j] = v.v[j];
            branch_end<K + 56>();
        } else {
            sput<T, S, NR, K + 1>(R, i, v);
        }
    }
}

template <class T, int S, int NR, int NT, int K = 0>
__device__ __forceinline__ void sload_all(const ProgArgs &a, uint32_t s0, int cnt,
                                          RegFile<T, S, NR> &R)
{
    if constexpr (K < NR) {
        if (K < a.nops) {
            if ((a.used >> K) & 1) {
                SReg<T, S> t;
                load_scalars<T, S, NT>(a, K, s0, cnt, t);
                sput<T, S, NR>(R, K, t);
            }
            sload_all<T, S, NR, NT, K + 1>(a, s0, cnt, R);
        }
    }
}

// Registers here hold S sites' values (RegFile entries reused as S-wide).
template <class T, int S, int NR, int NT>
__global__ __launch_bounds__(256) void k_program_scalar(ProgArgs a)
{
    extern __shared__ char occupancy_reserve[];
    const uint32_t s0 = (blockIdx.x * blockDim.x + threadIdx.x) * S;
    if (s0 < (uint32_t)a.nsites) {
        const int cnt = (uint32_t)a.nsites - s0 < (uint32_t)S ? int(a.nsites - s0) : S;
        RegFile<T, S, NR> R;
        sload_all<T, S, NR, NT>(a, s0, cnt, R);
        for (int pc = 0; pc < a.ninstr; ++pc) {
            const ProgInstr in = a.ins[pc];
            SReg<T, S> A, B, C;
            sget(R, in.a, A);
            sget(R, in.b, B);
            exec_scalars<T, S>(in, a, A, B, C);
            sput(R, in.d, C);
        }
        SReg<T, S> Z;
        sget(R, a.result, Z);
        if (a.zkind == su3i::FK_REAL) {
            T *p = static_cast<T *>(a.z) + s0;
            if (cnt == S) {
                constexpr int W = 16 / sizeof(T);
                using V = typename VecOf<T, W>::type;
#pragma unroll
                for (int q = 0; q < S / W; ++q) {
                    V w;
#pragma unroll
                    for (int j = 0; j < W; ++j)
                        w[j] = Z.v[q * W + j].re;
                    vstore<NT & 2>(reinterpret_cast<V *>(p) + q, w);
                }
            } else {
#pragma unroll
                for (int j = 0; j < S; ++j)
                    if (j < cnt)
                        p[j] = Z.v[j].re;
            }
        } else {
            using V2 = typename VecOf<T, 2>::type;
            V2 *p = static_cast<V2 *>(a.z) + s0;
#pragma unroll
            for (int j = 0; j < S; ++j)
                if (cnt == S || j < cnt) {
                    V2 w;
                    w[0] = Z.v[j].re;
                    w[1] = Z.v[j].im;
                    vstore<NT & 2>(p + j, w);
                }
        }
    }
    if (a.nsites < 0)
        occupancy_reserve[threadIdx.x] = 0;
}

// ------------------------------------------------ real-valued programs
//
// Every operand, intermediate and the result are real fields (one value
// per site).  A lane holds S = 2 W sites in each register, W = values per
// 16-byte vector: vector q (0, 1) of lane l in the lane group g = gid / 64
// is vector (2 g + q) * 64 + l of the field, so each load and store
// instruction of a wave moves 1 KiB of consecutive bytes.  Block sizes
// are multiples of 64, so the lane groups are the hardware waves.

template <class T, int S>
struct RVal {
    T v[S];
};

template <class T, int S, int NR, int K>
using RValIf = typename std::conditional<(K < NR), RVal<T, S>, NoReg>::type;

template <class T, int S, int NR>
struct RealFile {
    RValIf<T, S, NR, 0> r0;
    RValIf<T, S, NR, 1> r1;
    RValIf<T, S, NR, 2> r2;
    RValIf<T, S, NR, 3> r3;
    RValIf<T, S, NR, 4> r4;
    RValIf<T, S, NR, 5> r5;
    RValIf<T, S, NR, 6> r6;
    RValIf<T, S, NR, 7> r7;

    template <int K>
    __device__ __forceinline__ RValIf<T, S, NR, K> &at()
    {
        if constexpr (K == 0) return r0;
        else if constexpr (K == 1) return r1;
        else if constexpr (K == 2) return r2;
        else if constexpr (K == 3) return r3;
        else if constexpr (K == 4) return r4;
        else if constexpr (K == 5) return r5;
        else if constexpr (K == 6) return r6;
        else return r7;
    }
};

template <class T, int S, int NR, int K = 0>
__device__ __forceinline__ void rget(RealFile<T, S, NR> &R, int i, RVal<T, S> &out)
{
    if constexpr (K < NR) {
        if (i == K) {
            out = R.template at<K>();
            branch_end<K + 112>();
        } else {
            rget<T, S, NR, K + 1>(R, i, out);
        }
    }
}

template <class T, int S, int NR, int K = 0>
__device__ __forceinline__ void rput(RealFile<T, S, NR> &R, int i, const RVal<T, S> &v)
{
    if constexpr (K < NR) {
        if (i == K) {
            R.template at<K>() = v;
            branch_end<K + 120>();
        } else {
            rput<T, S, NR, K + 1>(R, i, v);
        }
    }
}

// The lane's values of a real field p of n sites; v0 = the lane's first
// vector.  Sites past n read as zero.
template <class T, int S, int NT>
__device__ __forceinline__ void rload(const T *p, uint32_t v0, uint32_t n, RVal<T, S> &r)
{
    constexpr int W = 16 / sizeof(T);
    using V = typename VecOf<T, W>::type;
#pragma unroll
    for (int q = 0; q < S / W; ++q) {
        const uint32_t vi = v0 + 64u * q, s = vi * W;
        if (s + W <= n) {
            const V w = vload<NT & 1>(reinterpret_cast<const V *>(p) + vi);
#pragma unroll
            for (int j = 0; j < W; ++j)
                r.v[q * W + j] = w[j];
        } else {
#pragma unroll
            for (int j = 0; j < W; ++j)
                r.v[q * W + j] = s + j < n ? p[s + j] : T(0);
        }
    }
}

template <class T, int S, int NT>
__device__ __forceinline__ void rstore(T *p, uint32_t v0, uint32_t n, const RVal<T, S> &r)
{
    constexpr int W = 16 / sizeof(T);
    using V = typename VecOf<T, W>::type;
#pragma unroll
    for (int q = 0; q < S / W; ++q) {
        const uint32_t vi = v0 + 64u * q, s = vi * W;
        if (s + W <= n) {
            V w;
#pragma unroll
            for (int j = 0; j < W; ++j)
                w[j] = r.v[q * W + j];
            vstore<NT & 2>(reinterpret_cast<V *>(p) + vi, w);
        } else {
#pragma unroll
            for (int j = 0; j < W; ++j)
                if (s + j < n)
                    p[s + j] = r.v[q * W + j];
        }
    }
}

// One instruction on S sites: one branch on the opcode for all of them.
// Real values take only the real-closed opcodes (constants are real, the
// conjugate and the real part are the identity, the imaginary part is
// zero).
template <class T, int S>
__device__ __forceinline__ void exec_real(const ProgInstr in, const ProgArgs &a,
                                          const RVal<T, S> &A, const RVal<T, S> &B,
                                          RVal<T, S> &C)
{
    switch (in.op) {
    case su3i::OP_CONST: {
        const T c = T(a.imm[in.a][0]);
#pragma unroll
        for (int j = 0; j < S; ++j)
            C.v[j] = c;
        branch_end<128>();
        break;
    }
    case su3i::OP_ADD_SS:
#pragma unroll
        for (int j = 0; j < S; ++j)
            C.v[j] = A.v[j] + B.v[j];
        branch_end<129>();
        break;
    case su3i::OP_SUB_SS:
#pragma unroll
        for (int j = 0; j < S; ++j)
            C.v[j] = A.v[j] - B.v[j];
        branch_end<130>();
        break;
    case su3i::OP_MUL_SS:
#pragma unroll
        for (int j = 0; j < S; ++j)
            C.v[j] = A.v[j] * B.v[j];
        branch_end<131>();
        break;
    case su3i::OP_NEG_S:
#pragma unroll
        for (int j = 0; j < S; ++j)
            C.v[j] = -A.v[j];
        branch_end<132>();
        break;
    case su3i::OP_IMAG:
#pragma unroll
        for (int j = 0; j < S; ++j)
            C.v[j] = T(0);
        branch_end<133>();
        break;
    default:  // OP_CONJ_S, OP_REAL
        C = A;
        branch_end<134>();
        break;
    }
}

template <class T, int S, int NR, int NT, int K = 0>
__device__ __forceinline__ void rload_all(const ProgArgs &a, uint32_t v0, uint32_t n,
                                          RealFile<T, S, NR> &R)
{
    if constexpr (K < NR) {
        if (K < a.nops) {
            if ((a.used >> K) & 1) {
                RVal<T, S> t;
                rload<T, S, NT>(static_cast<const T *>(a.op[K]), v0, n, t);
                rput<T, S, NR>(R, K, t);
            }
            rload_all<T, S, NR, NT, K + 1>(a, v0, n, R);
        }
    }
}

template <class T, int S, int NR, int NT>
__global__ __launch_bounds__(256) void k_program_real(ProgArgs a)
{
    extern __shared__ char occupancy_reserve[];
    constexpr int W = 16 / sizeof(T);
    const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t v0 = (gid >> 6) * (64u * (S / W)) + (gid & 63u);
    const uint32_t n = (uint32_t)a.nsites;
    if (a.nsites > 0 && v0 * W < n) {
        RealFile<T, S, NR> R;
        rload_all<T, S, NR, NT>(a, v0, n, R);
        for (int pc = 0; pc < a.ninstr; ++pc) {
            const ProgInstr in = a.ins[pc];
            RVal<T, S> A, B, C;
            rget(R, in.a, A);
            rget(R, in.b, B);
            exec_real<T, S>(in, a, A, B, C);
            rput(R, in.d, C);
        }
        RVal<T, S> Z;
        rget(R, a.result, Z);
        rstore<T, S, NT>(static_cast<T *>(a.z), v0, n, Z);
    }
    if (a.nsites < 0)
        occupancy_reserve[threadIdx.x] = 0;
}

template <class T, int NE, int NR>
static hipError_t go(int nt, int block, int grid, size_t shm, const ProgArgs &a,
                     hipStream_t st)
{
    if ((nt & 3) == 3)
        hipLaunchKernelGGL((k_program<T, NE, NR, 3>), dim3(grid), dim3(block), shm, st, a);
    else if ((nt & 3) == 2)
        hipLaunchKernelGGL((k_program<T, NE, NR, 2>), dim3(grid), dim3(block), shm, st, a);
    else
        hipLaunchKernelGGL((k_program<T, NE, NR, 0>), dim3(grid), dim3(block), shm, st, a);
    return hipGetLastError();
}

// Sites per lane of scalar-only programs: 32 bytes of each real operand
// (two 16-byte accesses).
template <class T>
constexpr int kScalarSites = 32 / sizeof(T);

template <class T, int NR>
static hipError_t go_scalar(int nt, int block, int grid, size_t shm,
                            const ProgArgs &a, hipStream_t st)
{
    constexpr int S = kScalarSites<T>;
    if ((nt & 3) == 3)
        hipLaunchKernelGGL((k_program_scalar<T, S, NR, 3>), dim3(grid), dim3(block), shm, st, a);
    else if ((nt & 3) == 2)
        hipLaunchKernelGGL((k_program_scalar<T, S, NR, 2>), dim3(grid), dim3(block), shm, st, a);
    else
        hipLaunchKernelGGL((k_program_scalar<T, S, NR, 0>), dim3(grid), dim3(block), shm, st, a);
    return hipGetLastError();
}

template <class T, int NR>
static hipError_t go_real(int nt, int block, int grid, size_t shm,
                          const ProgArgs &a, hipStream_t st)
{
    constexpr int S = kScalarSites<T>;
    if ((nt & 3) == 3)
        hipLaunchKernelGGL((k_program_real<T, S, NR, 3>), dim3(grid), dim3(block), shm, st, a);
    else if ((nt & 3) == 2)
        hipLaunchKernelGGL((k_program_real<T, S, NR, 2>), dim3(grid), dim3(block), shm, st, a);
    else
        hipLaunchKernelGGL((k_program_real<T, S, NR, 0>), dim3(grid), dim3(block), shm, st, a);
    return hipGetLastError();
}

template <class T>
static hipError_t go_t(int form, int nregs, int nt, int block, int grid,
                       size_t shm, const ProgArgs &a, hipStream_t st)
{
    if (form == su3i::PF_REAL)
        return nregs <= 4 ? go_real<T, 4>(nt, block, grid, shm, a, st)
                          : go_real<T, 8>(nt, block, grid, shm, a, st);
    if (form == su3i::PF_SCALAR)
        return nregs <= 4 ? go_scalar<T, 4>(nt, block, grid, shm, a, st)
                          : go_scalar<T, 8>(nt, block, grid, shm, a, st);
    // waves per SIMD the register file allows (double / single): 2 / 5
    // for two registers, 1 / 3 for four, 1 / 2 for eight (in double the
    // eight matrices fill the VGPRs and AGPRs of one wave)
    if (nregs <= 2)
        return go<T, 9, 2>(nt, block, grid, shm, a, st);
    if (nregs <= 4)
        return go<T, 9, 4>(nt, block, grid, shm, a, st);
    return go<T, 9, 8>(nt, block, grid, shm, a, st);
}

}  // namespace prog
}  // namespace su3k

namespace su3i {

int program_sites_per_lane(int arith, int form)
{
    if (form == PF_MATRIX)
        return 1;
    return arith == F64 ? su3k::prog::kScalarSites<double>
                        : su3k::prog::kScalarSites<float>;
}

hipError_t launch_program(int arith, int form, int nregs, int nt,
                          int block, int grid, size_t shm, const ProgArgs &a,
                          hipStream_t st)
{
    using namespace su3k::prog;
    if (block > 256 || block % 64 || nregs < 1 || nregs > kProgMaxRegs ||
        form < PF_MATRIX || form > PF_REAL)
        return hipErrorInvalidValue;
    if (arith == F64)
        return go_t<double>(form, nregs, nt, block, grid, shm, a, st);
    if (arith == F32)
        return go_t<float>(form, nregs, nt, block, grid, shm, a, st);
    return hipErrorInvalidValue;
}

}  // namespace su3i
