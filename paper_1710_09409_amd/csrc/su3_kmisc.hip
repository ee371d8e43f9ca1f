// Batched persistent kernel, bandwidth yardsticks (triad, copy) and the
// per-precision dispatch of the site kernels.
#include "su3_device.h"

namespace su3i {
hipError_t launch_site_p0(int, int, int, int, int, int, size_t, const SiteArgs &, hipStream_t);
hipError_t launch_site_p1(int, int, int, int, int, int, size_t, const SiteArgs &, hipStream_t);
hipError_t launch_site_p2(int, int, int, int, int, int, size_t, const SiteArgs &, hipStream_t);
hipError_t launch_site_p3(int, int, int, int, int, int, size_t, const SiteArgs &, hipStream_t);
hipError_t launch_shift_p0(int, int, int, int, int, size_t, const ShiftArgs &, hipStream_t);
hipError_t launch_shift_p1(int, int, int, int, int, size_t, const ShiftArgs &, hipStream_t);
hipError_t launch_shift_p2(int, int, int, int, int, size_t, const ShiftArgs &, hipStream_t);
hipError_t launch_shift_p3(int, int, int, int, int, size_t, const ShiftArgs &, hipStream_t);
hipError_t launch_site_lds_p0(int, int, int, int, const SiteArgs &, hipStream_t);
hipError_t launch_site_lds_p1(int, int, int, int, const SiteArgs &, hipStream_t);
hipError_t launch_site_lds_p2(int, int, int, int, const SiteArgs &, hipStream_t);
hipError_t launch_site_lds_p3(int, int, int, int, const SiteArgs &, hipStream_t);
}  // namespace su3i

namespace su3k {

using su3i::BatchItem;

// Evaluate one tile: `count` sites of item `it` from site `first` (a
// multiple of the tile size, hence of S), lanes striding over its groups.
template <int P, int X, int NT, int SCHED>
__device__ __forceinline__ void tile_run(const BatchItem &it, int first,
                                         int count)
{
    constexpr int S = SitesPerLane<P, X>::value;
    const void *const ops[4] = {it.op[0], it.op[1], it.op[2], it.op[3]};
    const int ng = (count + S - 1) / S;
    for (int g = threadIdx.x; g < ng; g += blockDim.x) {
        const uint32_t s0 = uint32_t(first + g * S);
        const uint32_t off = site_offset(it.g, s0);
        const int cnt = first + count - int(s0);
        if (cnt >= S)
            do_group<P, X, S, NT, true, SCHED>(it.z, ops, off, off, it.g.plane, S);
        else
            do_group<P, X, S, NT, false, SCHED>(it.z, ops, off, off, it.g.plane, cnt);
    }
}

template <int P, int NT, int SCHED>
__device__ __forceinline__ void tile_any_expr(const BatchItem &it, int first,
                                              int count)
{
    switch (it.expr) {
    case su3i::MUL: tile_run<P, su3i::MUL, NT, SCHED>(it, first, count); break;
    case su3i::MUL3: tile_run<P, su3i::MUL3, NT, SCHED>(it, first, count); break;
    default:
        if constexpr (P != su3i::C12) {
            switch (it.expr) {
            case su3i::MULADD: tile_run<P, su3i::MULADD, NT, SCHED>(it, first, count); break;
            case su3i::ADD: tile_run<P, su3i::ADD, NT, SCHED>(it, first, count); break;
            case su3i::APB_AB: tile_run<P, su3i::APB_AB, NT, SCHED>(it, first, count); break;
            }
        }
        break;
    }
}

// Batched kernel over the tile table.  Item i owns tiles tile_start_i ..
// tile_start_{i+1} - 1, each of T sites (the item's last tile may be
// shorter).  Workgroup b takes tiles b, b + G, b + 2G, ...; it finds a
// tile's item by binary search over the items' tile starts -- a small
// array every workgroup reads, so it stays in the scalar cache and no
// per-tile record has to come from memory before the data loads start.
// The branch on precision and expression is uniform across the workgroup.
// Every workgroup leaves after its last tile.
template <int MODE, int NT, int SCHED>
__global__ __launch_bounds__(256) void k_batch(const BatchItem *items,
                                               int nitems, int ntiles, int T)
{
    // dynamic LDS only caps the workgroups per CU; never read
    extern __shared__ char occupancy_reserve[];
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        int lo = 0, hi = nitems - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (items[mid].tile_start <= t)
                lo = mid;
            else
                hi = mid - 1;
        }
        const BatchItem &it = items[lo];
        const int first = (t - it.tile_start) * T;
        const int count = min(T, it.nsites - first);
        if constexpr (MODE == 0) {
            if (it.prec == su3i::F64)
                tile_run<su3i::F64, su3i::MUL, NT, SCHED>(it, first, count);
            else
                tile_run<su3i::C12, su3i::MUL, NT, SCHED>(it, first, count);
        } else {
            switch (it.prec) {
            case su3i::F64: tile_any_expr<su3i::F64, NT, SCHED>(it, first, count); break;
            case su3i::F32: tile_any_expr<su3i::F32, NT, SCHED>(it, first, count); break;
            case su3i::F16: tile_any_expr<su3i::F16, NT, SCHED>(it, first, count); break;
            case su3i::C12: tile_any_expr<su3i::C12, NT, SCHED>(it, first, count); break;
            }
        }
    }
    if (ntiles < 0)
        occupancy_reserve[threadIdx.x] = 0;
}

template <int NT>
__global__ __launch_bounds__(256) void k_triad(double *a, const double *b,
                                               const double *c, double s,
                                               int64_t n)
{
    using D2 = VecOf<double, 2>::type;
    const int64_t n2 = n >> 1;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n2;
         i += stride) {
        const D2 bv = vload<NT>(reinterpret_cast<const D2 *>(b) + i);
        const D2 cv = vload<NT>(reinterpret_cast<const D2 *>(c) + i);
        vstore<NT>(reinterpret_cast<D2 *>(a) + i, bv + s * cv);
    }
    if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0)
        a[n - 1] = b[n - 1] + s * c[n - 1];
}

template <int NT>
__global__ __launch_bounds__(256) void k_copy(void *dst, const void *src,
                                              int64_t n16)
{
    using V4 = VecOf<unsigned, 4>::type;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16;
         i += stride)
        vstore<NT>(reinterpret_cast<V4 *>(dst) + i,
                   vload<NT>(reinterpret_cast<const V4 *>(src) + i));
}

}  // namespace su3k

namespace su3i {

hipError_t launch_site(int prec, int expr, int S, int nt, int sched, int block,
                       int grid, size_t shm, const SiteArgs &a, hipStream_t st)
{
    switch (prec) {
    case F64: return launch_site_p0(expr, S, nt, sched, block, grid, shm, a, st);
    case F32: return launch_site_p1(expr, S, nt, sched, block, grid, shm, a, st);
    case F16: return launch_site_p2(expr, S, nt, sched, block, grid, shm, a, st);
    case C12: return launch_site_p3(expr, S, nt, sched, block, grid, shm, a, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_shift(int prec, int mode, int nt, int sched, int block,
                        int grid, size_t shm, const ShiftArgs &a, hipStream_t st)
{
    switch (prec) {
    case F64: return launch_shift_p0(mode, nt, sched, block, grid, shm, a, st);
    case F32: return launch_shift_p1(mode, nt, sched, block, grid, shm, a, st);
    case F16: return launch_shift_p2(mode, nt, sched, block, grid, shm, a, st);
    case C12: return launch_shift_p3(mode, nt, sched, block, grid, shm, a, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_site_lds(int prec, int expr, int nt, int block, int grid,
                           const SiteArgs &a, hipStream_t st)
{
    switch (prec) {
    case F64: return launch_site_lds_p0(expr, nt, block, grid, a, st);
    case F32: return launch_site_lds_p1(expr, nt, block, grid, a, st);
    case F16: return launch_site_lds_p2(expr, nt, block, grid, a, st);
    case C12: return launch_site_lds_p3(expr, nt, block, grid, a, st);
    }
    return hipErrorInvalidValue;
}

template <int MODE, int NT, int SCHED>
static void batch_go(const BatchItem *items, int32_t nitems, int32_t ntiles,
                     int32_t T, int block, int grid, size_t shm, hipStream_t st)
{
    hipLaunchKernelGGL((su3k::k_batch<MODE, NT, SCHED>), dim3(grid), dim3(block),
                       shm, st, items, nitems, ntiles, T);
}

hipError_t launch_batch(int mode, const BatchItem *items, int32_t nitems,
                        int32_t ntiles, int32_t tile_sites, int nt, int sched,
                        int block, int grid, size_t shm, hipStream_t st)
{
    if (block > 256)
        return hipErrorInvalidValue;
    const bool ntb = (nt & 3) == 3;
    const int v = (mode ? 4 : 0) + (ntb ? 2 : 0) + (sched ? 1 : 0);
#define SU3_BATCH(M, N, S) \
    batch_go<M, N, S>(items, nitems, ntiles, tile_sites, block, grid, shm, st)
    switch (v) {
    case 0: SU3_BATCH(0, 0, 0); break;
    case 1: SU3_BATCH(0, 0, 1); break;
    case 2: SU3_BATCH(0, 3, 0); break;
    case 3: SU3_BATCH(0, 3, 1); break;
    case 4: SU3_BATCH(1, 0, 0); break;
    case 5: SU3_BATCH(1, 0, 1); break;
    case 6: SU3_BATCH(1, 3, 0); break;
    default: SU3_BATCH(1, 3, 1); break;
    }
#undef SU3_BATCH
    return hipGetLastError();
}

static int one_shot_grid(int64_t items, int block)
{
    int64_t g = (items + block - 1) / block;
    if (g > (int64_t)1 << 30)
        g = (int64_t)1 << 30;
    return (int)(g < 1 ? 1 : g);
}

// Yardsticks: one-shot grids of 64-lane workgroups stream best here.
hipError_t launch_triad(double *a, const double *b, const double *c, double s,
                        int64_t n, hipStream_t st)
{
    const int block = 64;
    hipLaunchKernelGGL(su3k::k_triad<3>, dim3(one_shot_grid(n / 2, block)),
                       dim3(block), 0, st, a, b, c, s, n);
    return hipGetLastError();
}

hipError_t launch_copy(void *dst, const void *src, size_t bytes,
                       hipStream_t st)
{
    const int block = 64;
    const int64_t n16 = (int64_t)(bytes / 16);
    hipLaunchKernelGGL(su3k::k_copy<3>, dim3(one_shot_grid(n16, block)),
                       dim3(block), 0, st, dst, src, n16);
    return hipGetLastError();
}

}  // namespace su3i
