// Internal interface of the Wilson hopping kernel unit (su3_kdslash.hip)
// for the host C-ABI unit.  Not installed, not part of the ABI.
#pragma once

#include "su3_internal.h"

namespace su3i {

// Arguments of the Wilson hopping kernel.  Spinor fields store 12 complex
// entries per site (spin-major: entry 3 * spin + colour), link fields 9 (or
// 6 for the two-row form); both share dims, layout and lanes, so one site
// index addresses either through its own Geom.  Direction mu has extent
// dims[mu] and neighbour stride stride[mu] (x fastest).
// In the virtual-node layout dims/stride describe the outer sub-lattice
// (storage site s = osite * N_sub + lane, stride in storage sites) and
// nlanes/lstride the lanes; elsewhere nlanes = 1, lg = lmask = 0.
struct DslashArgs {
    void *out;
    const void *in;
    const void *u[4];
    Geom gs;          // spinor geometry
    Geom gl;          // link geometry
    int32_t nsites;
    int32_t xcd_remap;  // 1: contiguous workgroup ranges per XCD
    uint32_t walk;      // t-slices per lane (1: one site per lane)
    uint32_t span;      // LDS-tiled walk: > 0, (tile, slice) pairs per workgroup
    uint32_t dims[4];   // outer extents
    uint32_t stride[4]; // outer strides (storage sites)
    uint32_t nlanes[4]; // virtual nodes per direction
    uint32_t lstride[4];
    uint32_t lg;        // log2 N_sub
    uint32_t lmask;     // N_sub - 1
    // one site per lane (walk == 1), lexicographic fields: tile[0] > 0
    // gives each workgroup a tile[0] x tile[1] x tile[2] x tile[3] block of
    // sites (product = block), tiles x-fastest over ntile[0..2] per
    // direction; tile[0] == 0 takes sites in index order
    uint32_t tile[4];
    uint32_t ntile[4];
    // LDS-tiled walk: the schedule (4..28) whose tile each workgroup holds
    // (lds_shape), walking `walk` t-slices; ntile[0..2] tiles per
    // direction.  0: no LDS tile
    uint32_t lds_tile;
    uint32_t lds_tx;    // row tiles (schedules 9..28): the tile's x extent
};

// Tile of the LDS-tiled walk: tx x ty x tz (x, y, z) sites -- outer sites
// with all their nsub virtual nodes in the virtual-node layout -- one lane
// per site, and nb slice buffers in LDS (2: one barrier per slice, 1: two).
// halo: each buffer also holds the slice's y and z face sites, spin
// projected for the hop that reads them (6 complex numbers each).
struct LdsShape {
    int tx, ty, tz, nb, nsub;
    int halo;
};

// Face sites of a row tile's halo: the rows just below and just above the
// tile in y (tx * tz sites each) and in z (tx * ty each).
inline long halo_faces(const LdsShape &s)
{
    return s.halo ? 2L * s.tx * (s.ty + s.tz) : 0L;
}

inline size_t lds_shape_bytes(const LdsShape &s, int cbytes)
{
    return (size_t)s.nb *
           ((size_t)12 * s.nsub * s.tx * s.ty * s.tz + (size_t)6 * halo_faces(s)) * cbytes;
}

// Tile by schedule and block B:
//   4: 8 x 8 x B/64, two buffers     5: 8 x 8 x B/64, one buffer
//   6: 8 x 4 x B/32, one buffer      7: 16 x 8 x B/128, one buffer
//   8: 16 x 4 x B/64, one buffer
// A shape exists for block 128, 256 or 512 (schedule 6: 128 or 256,
// schedules 7 and 8: 256 or 512) when its buffers, nb * 12 * B complex
// numbers of cbytes bytes each, fit in 48 KiB of LDS; lexicographic
// fields only (nsub 1).
// Schedules 9..12 take rows, tx x 2 x 2, tx x 2 x 4, tx x 4 x 2,
// tx x 4 x 4 (outer) sites, with one buffer, 13..16 the same with two, 17
// and 18 tx x 3 x 3 with one and two; B is
// ignored: tx is the lattice's (outer) x extent lx when nsub * lx * ty * tz
// lanes fit a workgroup (rows_max_lanes), else (virtual-node fields only)
// the largest divisor of lx that does, and the buffers must fit the 160 KiB
// of LDS of a compute unit.  19..28: the shapes of 9..18 on lexicographic
// fields with a halo (the tile's y and z face sites of each slice, loaded
// and spin projected in the step before the slice, next to the interior
// loads of the tiles that own them).
// Most lanes of a row-tile workgroup: 512 for double spinors, 768 for
// single ones on virtual-node fields (whose kernels need more registers:
// three waves per SIMD), else 1024.
inline int rows_max_lanes(int cbytes, int nsub)
{
    return cbytes == 16 ? 512 : nsub > 1 ? 768 : 1024;
}

inline bool lds_shape(int schedule, int block, int cbytes, int lx, int nsub, LdsShape &s)
{
    if (nsub < 1)
        return false;
    const int halo = schedule >= 19 && schedule <= 28;
    if (halo) {
        if (nsub != 1)
            return false;
        schedule -= 10;
    }
    if (schedule >= 9 && schedule <= 18) {
        static const int rows[4][2] = {{2, 2}, {2, 4}, {4, 2}, {4, 4}};
        const int r = (schedule - 9) % 4;
        const long maxl = rows_max_lanes(cbytes, nsub);
        if (schedule >= 17) {
            s = {lx, 3, 3, schedule == 18 ? 2 : 1, nsub, halo};
        } else {
            s = {lx, rows[r][0], rows[r][1], schedule >= 13 ? 2 : 1, nsub, halo};
        }
        const long per_x = (long)nsub * s.ty * s.tz;  // lanes per unit of tx
        if (lx < 1 || per_x > maxl || (nsub == 1 && per_x * lx > maxl))
            return false;
        while (per_x * s.tx > maxl || lx % s.tx != 0)
            --s.tx;
        return lds_shape_bytes(s, cbytes) <= 160 * 1024;
    }
    if (nsub != 1 || (block != 128 && block != 256 && block != 512))
        return false;
    switch (schedule) {
    case 4: s = {8, 8, block / 64, 2, 1}; break;
    case 5: s = {8, 8, block / 64, 1, 1}; break;
    case 6:
        if (block > 256)
            return false;
        s = {8, 4, block / 32, 1, 1};
        break;
    case 7:
        if (block < 256)
            return false;
        s = {16, 8, block / 128, 1, 1};
        break;
    case 8:
        if (block < 256)
            return false;
        s = {16, 4, block / 64, 1, 1};
        break;
    default: return false;
    }
    return (long)s.nb * 12 * block * cbytes <= 48 * 1024;
}

// Wilson hopping term: spinor precision F64 with F64 links, F32 with F32
// or C12 links.  walk == 1: one site per lane, grid * block >= nsites;
// walk > 1 (lexicographic site order only): one lane per (x, y, z) site
// and chunk of `walk` t-slices,
// grid * block >= stride[3] * ceil(dims[3] / walk).  With a tile:
// grid = ntile[0] * ntile[1] * ntile[2] * ntile[3].  LDS-tiled walk
// (lds_tile = schedule with a shape for this block and spinor precision):
// grid = ntile[0] * ntile[1] * ntile[2] * ceil(dims[3] / walk), or with
// span > 0 ceil(ntile[0] * ntile[1] * ntile[2] * dims[3] / span); shm =
// lds_shape_bytes; its stores are always nontemporal.
// Nontemporal bit 0 applies to link loads only: each spinor is read by
// nine sites and stays cached.
hipError_t launch_dslash(int spinor_prec, int link_prec, int nt, int block,
                         int grid, size_t shm, const DslashArgs &a,
                         hipStream_t stream);

}  // namespace su3i
