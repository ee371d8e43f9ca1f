// Internal interface between the host C-ABI unit (su3_api.cpp) and the
// site, shift, batch and yardstick kernel units (su3_kprec.hip,
// su3_kmisc.hip); shared definitions (precisions, expressions, layouts,
// index geometry) of every kernel unit.  Not installed, not part of the
// ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace su3i {

enum Prec { F64 = 0, F32 = 1, F16 = 2, C12 = 3, NPREC = 4 };
enum Expr { MUL = 0, MUL3 = 1, MULADD = 2, ADD = 3, APB_AB = 4, NEXPR = 5 };
enum Layout { AOS = 0, SOA = 1, AOSOA = 2 };

// Stored complex entries per site and bytes per stored real.
inline int entries_of(int prec) { return prec == C12 ? 6 : 9; }
inline int real_bytes(int prec) { return prec == F64 ? 8 : (prec == F16 ? 2 : 4); }
inline int operands_of(int expr)
{
    return expr == MUL3 ? 3 : (expr == MULADD ? 4 : 2);
}
// Sites one lane handles in the blocked layouts: 16-byte accesses (double
// 1, float 2, half 4), except half storage with 3-4 operands (2 sites).
inline int natural_sites(int prec, int expr)
{
    if (prec == F64)
        return 1;
    if (prec == F16)
        return operands_of(expr) > 2 ? 2 : 4;
    return 2;
}

// Index geometry of a stored field, in units of stored reals: site s (a
// multiple of the sites-per-lane count), entry e, re/im c live at
//     (s >> lg) * bstride + e * plane + ((s & mask) << 1) + c.
// AoS: lg 0, mask 0, plane 2, bstride 2E.  AoSoA(L): lg log2 L,
// mask L-1, plane 2L, bstride 2EL.  SoA: lg 31, mask 2^31-1 (one block),
// plane 2 V_pad.
struct Geom {
    uint32_t lg;
    uint32_t mask;
    uint32_t plane;
    uint32_t bstride;
};

// Arguments of the one-launch site kernels.
struct SiteArgs {
    void *z;
    const void *op[4];
    Geom g;
    int32_t nsites;   // V
    int32_t ngroups;  // ceil(V / S)
    int32_t xcd_remap;
};

// Arguments of the shifted-operand kernels: the operand y is read at the
// neighbour s' of storage site s along one direction.  The coordinate
// along the direction is x = l * extent + o with the outer coordinate
// o = (s / stride) % extent and (virtual-node layout only, else l = 0)
// the lane coordinate l = ((s & lmask) / lstride) % nlanes;
// x' = (x + shift) mod (extent * nlanes) and
// s' = s + (o' - o) * stride + (l' - l) * lstride.
struct ShiftArgs {
    void *z;
    const void *x;   // unshifted left operand (product only)
    const void *y;   // shifted operand
    Geom g;
    int32_t nsites;
    uint32_t stride;  // storage sites between outer neighbours
    uint32_t extent;  // outer extent along the direction
    uint32_t shift;   // in [0, extent * nlanes)
    uint32_t nlanes;  // virtual nodes along the direction (1: none)
    uint32_t lstride; // lanes between virtual-node neighbours
    uint32_t lmask;   // N_sub - 1 (0 outside the virtual-node layout)
};

// One item of a batched launch (device-resident table).  The item owns
// tiles tile_start .. (next item's tile_start) - 1 of the batch's tile
// table, each of the batch's tile size T in sites (the last may be short).
struct BatchItem {
    void *z;
    const void *op[4];
    Geom g;
    int32_t nsites;
    int32_t prec;
    int32_t expr;
    int32_t tile_start;
};

// Sites per lane the site kernels are compiled for: 1, the natural count,
// and for the streaming product (MUL) outside half storage twice the
// natural count (32 bytes per lane and entry).
inline bool sites_compiled(int prec, int expr, int S)
{
    const int n = natural_sites(prec, expr);
    return S == 1 || S == n || (expr == MUL && prec != F16 && S == 2 * n);
}

// Kernel-unit entry points.  Each returns the launch's hipError_t.
// `sites_per_lane` as sites_compiled (the natural count or 1 in the AoS
// layout); `sched` 0 = all loads then all stores, 1 = row-phased; `nt` in
// {0, 1, 2, 3, 6, 7} (bit 2: write-through streaming stores); `shm` is LDS
// reserved per workgroup to cap occupancy (never read); block <= 256, or
// 512 / 1024 with nt 3 or 7.
hipError_t launch_site(int prec, int expr, int sites_per_lane, int nt,
                       int sched, int block, int grid, size_t shm,
                       const SiteArgs &a, hipStream_t stream);
// AoS with LDS staging: one lane per site, `block` sites per workgroup.
hipError_t launch_site_lds(int prec, int expr, int nt, int block, int grid,
                           const SiteArgs &a, hipStream_t stream);
// Batched launch over `ntiles` tiles of `tile_sites` sites.  queue ==
// nullptr: `grid` workgroups each taking tiles blockIdx.x, blockIdx.x +
// grid, ... (one per tile when grid == ntiles); else a persistent grid
// drawing tiles from the ticket counter *queue, which must start at 0 and
// is left at a multiple of ntiles + grid by every launch.  mode 0: every
// item is MUL in F64 or C12 (the mixed-precision streaming workload,
// smallest register footprint); mode 1: any supported item.
hipError_t launch_batch(int mode, const BatchItem *items, int32_t nitems,
                        int32_t ntiles, int32_t tile_sites, int nt, int sched,
                        int block, int grid, size_t shm, unsigned long long *queue,
                        hipStream_t stream);
// mode 0: z(s) = y(s'); mode 1: z(s) = x(s) * y(s').  One site per lane.
hipError_t launch_shift(int prec, int mode, int nt, int sched, int block,
                        int grid, size_t shm, const ShiftArgs &a,
                        hipStream_t stream);
// Item records passed by value to the kernel that writes a batch's table
// (kItemChunk per launch, well inside the kernel-argument space).
constexpr int kItemChunk = 24;
struct ItemChunk {
    BatchItem it[kItemChunk];
};
// Write items[0 .. n-1] to dst on `stream` with kernels (ceil(n /
// kItemChunk) launches, no host-to-device copy); queue != nullptr: also
// zero the ticket counter *queue.
hipError_t launch_put_items(BatchItem *dst, const BatchItem *items, int n,
                            unsigned long long *queue, hipStream_t stream);
// Bandwidth yardsticks over n16 16-byte elements per array (kinds below);
// `tail` adds the triad's trailing double; nt in {0, 1, 2, 3, 6, 7};
// block a multiple of 64 up to 1024; `shm` as for launch_site.
enum StreamKind { STREAM_TRIAD = 0, STREAM_READ = 1, STREAM_WRITE = 2, STREAM_COPY = 3 };
hipError_t launch_stream(int kind, void *a, const void *b, const void *c,
                         double s, int64_t n16, int tail, int nt, int block,
                         size_t shm, hipStream_t stream);

// Largest block of the site kernels (512 and 1024 take nt 3 or 7 only).
constexpr int kMaxBlock = 1024;

}  // namespace su3i
