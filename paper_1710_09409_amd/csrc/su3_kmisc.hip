// Batched persistent kernel, bandwidth yardsticks (triad, read-only,
// write-only, copy) and the
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

// One tile of the batch: find its item by binary search over the items'
// tile starts -- a small array every workgroup reads, so it stays in the
// scalar cache and no per-tile record has to come from memory before the
// data loads start -- and evaluate it.  The branch on precision and
// expression is uniform across the workgroup.
template <int MODE, int NT, int SCHED>
__device__ __forceinline__ void batch_tile(const BatchItem *items, int nitems, int t,
                                           int T)
{
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

// Batched kernel over the tile table.  Item i owns tiles tile_start_i ..
// tile_start_{i+1} - 1, each of T sites (the item's last tile may be
// shorter).
//   queue == nullptr: one workgroup per tile (a one-shot grid; workgroup b
//     takes tiles b, b + G, ... when the grid is smaller).
//   queue != nullptr: a persistent grid whose workgroups take tiles from a
//     ticket counter in queue[0], in order, until the tiles run out: lane 0
//     draws ticket v and the workgroup takes tile v mod (ntiles + G); a
//     value >= ntiles means no tile is left and the workgroup leaves.  Every
//     workgroup draws once more after its last tile, so a launch draws
//     exactly ntiles + G tickets and leaves the counter at the next
//     multiple of it: the queue never needs resetting between launches of
//     the same batch (it starts at 0).  The next ticket is drawn while the
//     current tile is evaluated, so its latency is hidden.  The ticket goes
//     from lane 0 to the workgroup through the first bytes of the dynamic
//     LDS (the host reserves at least 16).
template <int MODE, int NT, int SCHED>
__global__ __launch_bounds__(256) void k_batch(const BatchItem *items, int nitems,
                                               int ntiles, int T,
                                               unsigned long long *queue)
{
    // dynamic LDS: the ticket of the queued form, and the reserve that
    // caps the workgroups per CU (otherwise never read)
    extern __shared__ char occupancy_reserve[];
    if (!queue) {
        for (int t = blockIdx.x; t < ntiles; t += gridDim.x)
            batch_tile<MODE, NT, SCHED>(items, nitems, t, T);
        if (ntiles < 0)
            occupancy_reserve[threadIdx.x] = 0;
        return;
    }
    volatile int *ticket = reinterpret_cast<volatile int *>(occupancy_reserve);
    const unsigned long long m = (unsigned long long)ntiles + gridDim.x;
    unsigned long long next = 0;
    if (threadIdx.x == 0)
        next = atomicAdd(queue, 1ull);
    for (;;) {
        if (threadIdx.x == 0)
            *ticket = (int)(next % m);
        __syncthreads();
        const int t = *ticket;
        __syncthreads();
        if (t >= ntiles)
            break;
        if (threadIdx.x == 0)
            next = atomicAdd(queue, 1ull);
        batch_tile<MODE, NT, SCHED>(items, nitems, t, T);
    }
}

// Item records of a batch written from kernel arguments (the allocation-
// free batch: no copy from host memory, so the write can sit in a captured
// graph); with `queue`, also zero the persistent grid's ticket counter.
__global__ __launch_bounds__(64) void k_put_items(BatchItem *dst, su3i::ItemChunk c,
                                                  int count, unsigned long long *queue)
{
    const int i = threadIdx.x;
    if (i < count)
        dst[i] = c.it[i];
    if (queue && i == 0)
        *queue = 0ull;
}

// Bandwidth yardsticks, one 16-byte element per lane, one-shot grid:
// triad a = b + s*c (doubles), read-only (b and c), write-only (a = s),
// copy (a = b).  The read-only kind writes a[0] only if an element of
// b + c equals (s, -s), which keeps its loads without a store stream.
// With `tail` the triad also covers the double after the last element.
template <int KIND, int NT>
__global__ __launch_bounds__(1024) void k_stream(void *a, const void *b,
                                                 const void *c, double s,
                                                 int64_t n16, int tail)
{
    extern __shared__ char occupancy_reserve[];
    using D2 = VecOf<double, 2>::type;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    D2 *A = static_cast<D2 *>(a);
    const D2 *Bv = static_cast<const D2 *>(b);
    const D2 *C = static_cast<const D2 *>(c);
    if (i < n16) {
        if constexpr (KIND == su3i::STREAM_TRIAD) {
            const D2 bv = vload<NT>(Bv + i);
            const D2 cv = vload<NT>(C + i);
            vstore<NT>(A + i, bv + s * cv);
        } else if constexpr (KIND == su3i::STREAM_READ) {
            const D2 v = vload<NT>(Bv + i) + vload<NT>(C + i);
            if (v[0] == s && v[1] == -s)
                A[0] = v;
        } else if constexpr (KIND == su3i::STREAM_WRITE) {
            D2 v;
            v[0] = s;
            v[1] = s;
            vstore<NT>(A + i, v);
        } else {
            vstore<NT>(A + i, vload<NT>(Bv + i));
        }
    }
    if constexpr (KIND == su3i::STREAM_TRIAD) {
        if (tail && i == 0) {
            const int64_t k = 2 * n16;
            static_cast<double *>(a)[k] = static_cast<const double *>(b)[k] +
                                          s * static_cast<const double *>(c)[k];
        }
    }
    if (n16 < 0)
        occupancy_reserve[threadIdx.x] = 0;
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
static void batch_go(const BatchItem *items, int32_t nitems, int32_t ntiles, int32_t T,
                     unsigned long long *queue, int block, int grid, size_t shm,
                     hipStream_t st)
{
    hipLaunchKernelGGL((su3k::k_batch<MODE, NT, SCHED>), dim3(grid), dim3(block), shm, st,
                       items, nitems, ntiles, T, queue);
}

hipError_t launch_batch(int mode, const BatchItem *items, int32_t nitems,
                        int32_t ntiles, int32_t tile_sites, int nt, int sched,
                        int block, int grid, size_t shm, unsigned long long *queue,
                        hipStream_t st)
{
    if (block > 256)
        return hipErrorInvalidValue;
    if (queue && shm < 16)
        shm = 16;  // the ticket
    // nontemporal settings compiled: 0, 3 and 7 (others run as 0 or 3)
    const int ntv = nt == 7 ? 2 : ((nt & 3) == 3 ? 1 : 0);
    const int v = (mode ? 6 : 0) + 2 * ntv + (sched ? 1 : 0);
#define SU3_BATCH(M, N, S) \
    batch_go<M, N, S>(items, nitems, ntiles, tile_sites, queue, block, grid, shm, st)
    switch (v) {
    case 0: SU3_BATCH(0, 0, 0); break;
    case 1: SU3_BATCH(0, 0, 1); break;
    case 2: SU3_BATCH(0, 3, 0); break;
    case 3: SU3_BATCH(0, 3, 1); break;
    case 4: SU3_BATCH(0, 7, 0); break;
    case 5: SU3_BATCH(0, 7, 1); break;
    case 6: SU3_BATCH(1, 0, 0); break;
    case 7: SU3_BATCH(1, 0, 1); break;
    case 8: SU3_BATCH(1, 3, 0); break;
    case 9: SU3_BATCH(1, 3, 1); break;
    case 10: SU3_BATCH(1, 7, 0); break;
    default: SU3_BATCH(1, 7, 1); break;
    }
#undef SU3_BATCH
    return hipGetLastError();
}

hipError_t launch_put_items(BatchItem *dst, const BatchItem *items, int n,
                            unsigned long long *queue, hipStream_t st)
{
    for (int first = 0; first < n; first += kItemChunk) {
        ItemChunk c;
        const int count = n - first < kItemChunk ? n - first : kItemChunk;
        for (int i = 0; i < count; ++i)
            c.it[i] = items[first + i];
        hipLaunchKernelGGL(su3k::k_put_items, dim3(1), dim3(64), 0, st, dst + first, c,
                           count, first == 0 ? queue : nullptr);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

template <int KIND, int NT>
static void stream_go(void *a, const void *b, const void *c, double s,
                      int64_t n16, int tail, int block, int grid, size_t shm,
                      hipStream_t st)
{
    hipLaunchKernelGGL((su3k::k_stream<KIND, NT>), dim3(grid), dim3(block), shm,
                       st, a, b, c, s, n16, tail);
}

template <int KIND>
static hipError_t stream_nt(int nt, void *a, const void *b, const void *c,
                            double s, int64_t n16, int tail, int block,
                            int grid, size_t shm, hipStream_t st)
{
    switch (nt) {
    case 0: stream_go<KIND, 0>(a, b, c, s, n16, tail, block, grid, shm, st); break;
    case 1: stream_go<KIND, 1>(a, b, c, s, n16, tail, block, grid, shm, st); break;
    case 2: stream_go<KIND, 2>(a, b, c, s, n16, tail, block, grid, shm, st); break;
    case 3: stream_go<KIND, 3>(a, b, c, s, n16, tail, block, grid, shm, st); break;
    case 6: stream_go<KIND, 6>(a, b, c, s, n16, tail, block, grid, shm, st); break;
    case 7: stream_go<KIND, 7>(a, b, c, s, n16, tail, block, grid, shm, st); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_stream(int kind, void *a, const void *b, const void *c,
                         double s, int64_t n16, int tail, int nt, int block,
                         size_t shm, hipStream_t st)
{
    if (block < 64 || block > 1024 || block % 64)
        return hipErrorInvalidValue;
    const int64_t g = (n16 + block - 1) / block;
    if (g > ((int64_t)1 << 31) - 1)
        return hipErrorInvalidValue;
    const int grid = g < 1 ? 1 : (int)g;
    switch (kind) {
    case STREAM_TRIAD: return stream_nt<STREAM_TRIAD>(nt, a, b, c, s, n16, tail, block, grid, shm, st);
    case STREAM_READ: return stream_nt<STREAM_READ>(nt, a, b, c, s, n16, tail, block, grid, shm, st);
    case STREAM_WRITE: return stream_nt<STREAM_WRITE>(nt, a, b, c, s, n16, tail, block, grid, shm, st);
    case STREAM_COPY: return stream_nt<STREAM_COPY>(nt, a, b, c, s, n16, tail, block, grid, shm, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace su3i
