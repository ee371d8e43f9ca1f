// Site kernels of one storage precision.  This unit is compiled once per
// precision with -DSU3_PREC=<0..3> so the four precisions build in
// parallel; su3_kmisc.hip dispatches to the per-precision entry points.
//
// k_site:     one lane per group of S sites, blocked layouts (S natural) or
//             AoS (S = 1).  One-shot grid, or grid-stride when the grid is
//             smaller than the work (persistent launch).
// k_site_lds: AoS with each workgroup's tile of sites staged through LDS by
//             coalesced 16-byte copies, then evaluated one site per lane.
#include "su3_device.h"

#ifndef SU3_PREC
#error "compile with -DSU3_PREC=<precision code>"
#endif

#define SU3_CAT2(a, b) a##b
#define SU3_CAT(a, b) SU3_CAT2(a, b)

// Each precision's kernels live in their own namespace (su3k::p0 .. p3):
// the four units instantiate templates of the same shape, and without a
// distinct name the linker would fold one precision's kernel into another's.
namespace su3k {
namespace SU3_CAT(p, SU3_PREC) {

constexpr int P = SU3_PREC;
constexpr int kMaxSiteBlock = 256;
// k_site variants for workgroups of 512 and 1024 lanes
constexpr int kWideBlock = 1024;
using R = typename PrecT<P>::R;
using T = typename PrecT<P>::T;

template <int X, int S, int NT, int SCHED, int MAXB>
__global__ __launch_bounds__(MAXB) void k_site(su3i::SiteArgs a)
{
    // Dynamic LDS is reserved only to cap how many workgroups share a CU
    // (the launch's occupancy setting); it is never read.
    extern __shared__ char occupancy_reserve[];
    const int nb = gridDim.x;
    const int b = a.xcd_remap ? xcd_remap(blockIdx.x, nb) : (int)blockIdx.x;
    const int B = blockDim.x;
    const void *const ops[4] = {a.op[0], a.op[1], a.op[2], a.op[3]};
    for (int g = b * B + threadIdx.x; g < a.ngroups; g += nb * B) {
        const uint32_t s0 = uint32_t(g) * S;
        const uint32_t off = site_offset(a.g, s0);
        const int cnt = a.nsites - int(s0);
        if (cnt >= S)
            do_group<P, X, S, NT, true, SCHED>(a.z, ops, off, off, a.g.plane, S);
        else
            do_group<P, X, S, NT, false, SCHED>(a.z, ops, off, off, a.g.plane, cnt);
    }
    if (a.nsites < 0)
        occupancy_reserve[threadIdx.x] = 0;
}

// Shifted operand (Cshift and products with a shifted right operand), one
// site per lane: the lane of site s reads y at the neighbour s' of s along
// one direction, periodic.  Consecutive lanes read consecutive sites of
// the neighbouring row/plane, so the gather stays coalesced except at the
// wrap of the shifted coordinate.
template <int MODE, int NT, int SCHED>
__global__ __launch_bounds__(kMaxSiteBlock) void k_shift(su3i::ShiftArgs a)
{
    extern __shared__ char occupancy_reserve[];
    constexpr int E = PrecT<P>::E;
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < (uint32_t)a.nsites) {
        // coordinate along the direction: outer part o, lane part l
        const uint32_t o = (s / a.stride) % a.extent;
        uint32_t l = 0, x = o;
        if (a.nlanes > 1) {
            l = ((s & a.lmask) / a.lstride) % a.nlanes;
            x = l * a.extent + o;
        }
        const uint32_t ext = a.extent * a.nlanes;
        uint32_t xn = x + a.shift;
        if (xn >= ext)
            xn -= ext;
        uint32_t on = xn, ln = 0;
        if (a.nlanes > 1) {
            ln = xn / a.extent;
            on = xn - ln * a.extent;
        }
        // modulo 2^32, in range
        const uint32_t sn = s + (on - o) * a.stride + (ln - l) * a.lstride;
        const uint32_t off = site_offset(a.g, s);
        const uint32_t offn = site_offset(a.g, sn);
        if constexpr (MODE == 0) {
            RawVec<P, 1> yr[E];
            load_entries<P, 1, NT, true, 0, E>(static_cast<const R *>(a.y), offn,
                                               a.g.plane, 1, yr);
            store_entries<P, 1, NT, true, 0, E>(static_cast<R *>(a.z), off,
                                                a.g.plane, 1, yr);
        } else {
            const void *const ops[4] = {a.x, a.y, nullptr, nullptr};
            do_group<P, su3i::MUL, 1, NT, true, SCHED>(a.z, ops, off, offn,
                                                       a.g.plane, 1);
        }
    }
    if (a.nsites < 0)
        occupancy_reserve[threadIdx.x] = 0;
}

// Copy `nbytes` bytes between global memory and LDS with the whole
// workgroup: 16-byte pieces when the count allows, else 4-byte pieces
// (every stored site is a multiple of 4 bytes).
template <int NT>
__device__ __forceinline__ void copy_in(unsigned char *lds,
                                        const unsigned char *g, int nbytes)
{
    using V4 = VecOf<unsigned, 4>::type;
    if ((nbytes & 15) == 0) {
        for (int i = threadIdx.x; i < (nbytes >> 4); i += blockDim.x)
            reinterpret_cast<V4 *>(lds)[i] =
                vload<NT>(reinterpret_cast<const V4 *>(g) + i);
    } else {
        for (int i = threadIdx.x; i < (nbytes >> 2); i += blockDim.x)
            reinterpret_cast<unsigned *>(lds)[i] =
                reinterpret_cast<const unsigned *>(g)[i];
    }
}

template <int NT>
__device__ __forceinline__ void copy_out(unsigned char *g,
                                         const unsigned char *lds, int nbytes)
{
    using V4 = VecOf<unsigned, 4>::type;
    if ((nbytes & 15) == 0) {
        for (int i = threadIdx.x; i < (nbytes >> 4); i += blockDim.x)
            vstore<NT>(reinterpret_cast<V4 *>(g) + i,
                       reinterpret_cast<const V4 *>(lds)[i]);
    } else {
        for (int i = threadIdx.x; i < (nbytes >> 2); i += blockDim.x)
            reinterpret_cast<unsigned *>(g)[i] =
                reinterpret_cast<const unsigned *>(lds)[i];
    }
}

constexpr int kLdsMaxBlock = 128;

template <int X, int NT>
__global__ __launch_bounds__(kLdsMaxBlock) void k_site_lds(su3i::SiteArgs a)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
    constexpr int N = NOps<X>::value;
    constexpr int E = PrecT<P>::E;
    constexpr int REC = E * 2 * (int)sizeof(R);  // bytes per AoS site
    using V2 = typename VecOf<R, 2>::type;
    const int B = blockDim.x;
    const int t = threadIdx.x;
    const int ntiles = (a.nsites + B - 1) / B;
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int s0 = tile * B;
        const int cnt = min(B, a.nsites - s0);
        const size_t gbase = (size_t)s0 * REC;
        const int nbytes = cnt * REC;
#pragma unroll
        for (int k = 0; k < N; ++k)
            copy_in<NT>(lds + k * B * REC,
                        static_cast<const unsigned char *>(a.op[k]) + gbase,
                        nbytes);
        __syncthreads();
        Cx<T> z[9];
        if (t < cnt) {
            Cx<T> o[N][9];
#pragma unroll
            for (int k = 0; k < N; ++k) {
                const R *site = reinterpret_cast<const R *>(lds + k * B * REC + t * REC);
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    const V2 v = reinterpret_cast<const V2 *>(site)[e];
                    o[k][e].re = (T)v[0];
                    o[k][e].im = (T)v[1];
                }
            }
            eval_site<P, X>(o, z);
        }
        __syncthreads();
        if (t < cnt) {
            R *site = reinterpret_cast<R *>(lds + t * REC);
#pragma unroll
            for (int e = 0; e < E; ++e) {
                RawVec<P, 1> v;
                narrow<P, 1>(v, 0, z[e]);
                reinterpret_cast<V2 *>(site)[e] = v;
            }
        }
        __syncthreads();
        copy_out<NT>(static_cast<unsigned char *>(a.z) + gbase, lds, nbytes);
        __syncthreads();
    }
}

// ------------------------------------------------------------ dispatch

template <int X, int S, int NT>
static hipError_t run_site(int sched, int block, int grid, size_t shm,
                           const su3i::SiteArgs &a, hipStream_t st)
{
    if (block <= kMaxSiteBlock) {
        if (sched)
            hipLaunchKernelGGL((k_site<X, S, NT, 1, kMaxSiteBlock>), dim3(grid),
                               dim3(block), shm, st, a);
        else
            hipLaunchKernelGGL((k_site<X, S, NT, 0, kMaxSiteBlock>), dim3(grid),
                               dim3(block), shm, st, a);
        return hipGetLastError();
    }
    // 512 and 1024 lanes: compiled for the streaming store settings only
    if constexpr ((NT & 3) == 3) {
        if (block > kWideBlock)
            return hipErrorInvalidValue;
        if (sched)
            hipLaunchKernelGGL((k_site<X, S, NT, 1, kWideBlock>), dim3(grid),
                               dim3(block), shm, st, a);
        else
            hipLaunchKernelGGL((k_site<X, S, NT, 0, kWideBlock>), dim3(grid),
                               dim3(block), shm, st, a);
        return hipGetLastError();
    } else {
        return hipErrorInvalidValue;
    }
}

template <int X, int S>
static hipError_t pick_nt(int nt, int sched, int block, int grid, size_t shm,
                          const su3i::SiteArgs &a, hipStream_t st)
{
    switch (nt) {
    case 0: return run_site<X, S, 0>(sched, block, grid, shm, a, st);
    case 1: return run_site<X, S, 1>(sched, block, grid, shm, a, st);
    case 2: return run_site<X, S, 2>(sched, block, grid, shm, a, st);
    case 3: return run_site<X, S, 3>(sched, block, grid, shm, a, st);
    case 6: return run_site<X, S, 6>(sched, block, grid, shm, a, st);
    case 7: return run_site<X, S, 7>(sched, block, grid, shm, a, st);
    }
    return hipErrorInvalidValue;
}

template <int X>
static hipError_t pick_s(int S, int nt, int sched, int block, int grid,
                         size_t shm, const su3i::SiteArgs &a, hipStream_t st)
{
    if constexpr (!Supported<P, X>::value) {
        return hipErrorInvalidValue;
    } else {
        constexpr int SN = SitesPerLane<P, X>::value;
        if (S == 1)
            return pick_nt<X, 1>(nt, sched, block, grid, shm, a, st);
        if (S == SN)
            return pick_nt<X, SN>(nt, sched, block, grid, shm, a, st);
        // twice the natural count (32 bytes per lane and entry): the
        // streaming product in double, single and compressed storage
        if constexpr (X == su3i::MUL && P != su3i::F16) {
            if (S == 2 * SN)
                return pick_nt<X, 2 * SN>(nt, sched, block, grid, shm, a, st);
        }
        return hipErrorInvalidValue;
    }
}

template <int X>
static hipError_t run_lds(int nt, int block, int grid,
                          const su3i::SiteArgs &a, hipStream_t st)
{
    if constexpr (!Supported<P, X>::value) {
        return hipErrorInvalidValue;
    } else {
        if (block > kLdsMaxBlock)
            return hipErrorInvalidValue;
        const size_t shm = (size_t)NOps<X>::value * block * PrecT<P>::E * 2 *
                           sizeof(R);
        if ((nt & 3) == 3)
            hipLaunchKernelGGL((k_site_lds<X, 3>), dim3(grid), dim3(block), shm,
                               st, a);
        else
            hipLaunchKernelGGL((k_site_lds<X, 0>), dim3(grid), dim3(block), shm,
                               st, a);
        return hipGetLastError();
    }
}

}  // namespace p<SU3_PREC>
}  // namespace su3k

namespace su3i {

hipError_t SU3_CAT(launch_site_p, SU3_PREC)(int expr, int S, int nt,
                                             int sched, int block, int grid,
                                             size_t shm, const SiteArgs &a,
                                             hipStream_t st)
{
    using namespace su3k::SU3_CAT(p, SU3_PREC);
    switch (expr) {
    case MUL: return pick_s<MUL>(S, nt, sched, block, grid, shm, a, st);
    case MUL3: return pick_s<MUL3>(S, nt, sched, block, grid, shm, a, st);
    case MULADD: return pick_s<MULADD>(S, nt, sched, block, grid, shm, a, st);
    case ADD: return pick_s<ADD>(S, nt, sched, block, grid, shm, a, st);
    case APB_AB: return pick_s<APB_AB>(S, nt, sched, block, grid, shm, a, st);
    }
    return hipErrorInvalidValue;
}

hipError_t SU3_CAT(launch_shift_p, SU3_PREC)(int mode, int nt, int sched,
                                              int block, int grid, size_t shm,
                                              const ShiftArgs &a,
                                              hipStream_t st)
{
    using namespace su3k::SU3_CAT(p, SU3_PREC);
    if (block > kMaxSiteBlock)
        return hipErrorInvalidValue;
    // nontemporal settings compiled: 0, 3 and 7 (others run as 0 or 3)
    const int ntv = nt == 7 ? 7 : ((nt & 3) == 3 ? 3 : 0);
    if (mode == 0) {
        if (ntv == 7)
            hipLaunchKernelGGL((k_shift<0, 7, 0>), dim3(grid), dim3(block), shm, st, a);
        else if (ntv == 3)
            hipLaunchKernelGGL((k_shift<0, 3, 0>), dim3(grid), dim3(block), shm, st, a);
        else
            hipLaunchKernelGGL((k_shift<0, 0, 0>), dim3(grid), dim3(block), shm, st, a);
    } else {
        const int v = (ntv == 7 ? 4 : (ntv == 3 ? 2 : 0)) + (sched ? 1 : 0);
        switch (v) {
        case 0: hipLaunchKernelGGL((k_shift<1, 0, 0>), dim3(grid), dim3(block), shm, st, a); break;
        case 1: hipLaunchKernelGGL((k_shift<1, 0, 1>), dim3(grid), dim3(block), shm, st, a); break;
        case 2: hipLaunchKernelGGL((k_shift<1, 3, 0>), dim3(grid), dim3(block), shm, st, a); break;
        case 3: hipLaunchKernelGGL((k_shift<1, 3, 1>), dim3(grid), dim3(block), shm, st, a); break;
        case 4: hipLaunchKernelGGL((k_shift<1, 7, 0>), dim3(grid), dim3(block), shm, st, a); break;
        default: hipLaunchKernelGGL((k_shift<1, 7, 1>), dim3(grid), dim3(block), shm, st, a); break;
        }
    }
    return hipGetLastError();
}

hipError_t SU3_CAT(launch_site_lds_p, SU3_PREC)(int expr, int nt, int block,
                                                 int grid, const SiteArgs &a,
                                                 hipStream_t st)
{
    using namespace su3k::SU3_CAT(p, SU3_PREC);
    switch (expr) {
    case MUL: return run_lds<MUL>(nt, block, grid, a, st);
    case MUL3: return run_lds<MUL3>(nt, block, grid, a, st);
    case MULADD: return run_lds<MULADD>(nt, block, grid, a, st);
    case ADD: return run_lds<ADD>(nt, block, grid, a, st);
    case APB_AB: return run_lds<APB_AB>(nt, block, grid, a, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace su3i
