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
    // 1: LDS-tiled walk (8 x 8 x block/64 tiles of (x, y, z) sites, each
    // workgroup walking `walk` t-slices; ntile[0..2] tiles per direction)
    uint32_t lds_tile;
};

// Wilson hopping term: spinor precision F64 with F64 links, F32 with F32
// or C12 links.  walk == 1: one site per lane, grid * block >= nsites;
// walk > 1 (lexicographic site order only): one lane per (x, y, z) site
// and chunk of `walk` t-slices,
// grid * block >= stride[3] * ceil(dims[3] / walk).  With a tile:
// grid = ntile[0] * ntile[1] * ntile[2] * ntile[3].  LDS-tiled walk
// (lds_tile = 1; block 128, or 256 for single-precision spinors): grid =
// ntile[0] * ntile[1] * ntile[2] * ceil(dims[3] / walk).
hipError_t launch_dslash(int spinor_prec, int link_prec, int nt, int block,
                         int grid, size_t shm, const DslashArgs &a,
                         hipStream_t stream);

}  // namespace su3i
