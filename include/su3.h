/*
 * su3.h -- C ABI of the MI355X (gfx950) SU(3) x SU(3) streaming library.
 *
 * The library evaluates site-local expressions of 3x3 complex matrix
 * fields over a 4D lattice, z(x) = x(x) * y(x) first of all: the
 * lattice-wide SU(3) x SU(3) streaming test of Boyle et al., "Performance
 * Portability Strategies for Grid C++ Expression Templates" (Lattice 2017),
 * Section 4 (Listing 3), evaluated site by site as in Section 3
 * (Listing 1: _odata[ss] = eval(ss, expr)), in the coalesced layouts that
 * Sections 4 and 5 motivate.
 *
 * Conventions shared by every entry point:
 *   - Plain C types only.  Handles are opaque.  No C++ exception crosses
 *     the boundary; every call returns an su3_status, and su3_last_error()
 *     gives a thread-local text for the last failing call.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream of
 *     the current device), e.g. torch.cuda.current_stream().cuda_stream.
 *     Compute calls are asynchronous on that stream.  Uploads and downloads
 *     complete before they return.
 *   - Arguments are validated before any HIP call; a failed validation
 *     launches nothing and changes nothing.
 *   - Asynchronous kernel faults surface at the next call that
 *     synchronises (su3_sync, upload, download) as SU3_ERR_HIP.
 *   - Values are not inspected: NaN and Inf pass through.
 *
 * Canonical host layout (upload/download): double at
 * ((s*3 + i)*3 + j)*2 + c for site s = x + Lx*(y + Ly*(z + Lz*t)), row i,
 * column j, c = 0 real / 1 imaginary (18 doubles per site).
 *
 * Stored layouts on the device.  A field of V sites stores E complex
 * entries per site (E = 9; E = 6 for SU3_C12_F32, rows 0 and 1).  Sites are
 * grouped in lane-blocks of L sites, padded to V_pad = a multiple of L:
 *     AOS    L = 1,        V_pad = V          (Section 4's scalar layout)
 *     AOSOA  L = lanes,    V_pad = roundup(V, lanes), lanes in {8,16,32,64}
 *            (Section 5's vector layout: each scalar leaf holds L lanes)
 *     SOA    L = V_pad,    V_pad = roundup(V, 64)  (one block: entry planes)
 * Real number (s, e, c) sits at element
 *     ((s / L) * E + e) * 2L + (s % L) * 2 + c
 * of an array of the stored real type (double, float, or IEEE half).  The
 * field occupies V_pad * E * 2 * sizeof(real) bytes.  Padding sites are
 * zero after su3_field_alloc/su3_field_upload and are never written by a
 * compute call.
 *     VNODE  Grid's virtual-node layout (Section 5), made by su3_vnode_*:
 *            the lattice is split into N_sub = simd[0]*simd[1]*simd[2]*
 *            simd[3] virtual nodes, one per SIMD lane, each a sub-lattice
 *            of extents r[mu] = dims[mu] / simd[mu].  Site x has lane
 *            coordinates l[mu] = x[mu] / r[mu] and outer coordinates
 *            o[mu] = x[mu] % r[mu]; lane = l0 + simd0*(l1 + simd1*(l2 +
 *            simd2*l3)), osite = o0 + r0*(o1 + r1*(o2 + r2*o3)).  It is
 *            stored as AOSOA with L = N_sub at s = osite * N_sub + lane
 *            (each scalar leaf is a vector of N_sub lanes, (re, im)
 *            interleaved per lane), V_pad = V.
 */
#ifndef SU3_H
#define SU3_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum su3_status {
    SU3_OK = 0,
    SU3_ERR_INVALID_ARG = -1,   /* null pointer, bad size/enum, bad buffer */
    SU3_ERR_MISMATCH = -2,      /* operands differ in dims/precision/layout */
    SU3_ERR_UNSUPPORTED = -3,   /* valid arguments, combination not offered */
    SU3_ERR_OUT_OF_MEMORY = -4, /* device allocation failed */
    SU3_ERR_ALIAS = -5,         /* output partially overlaps an operand */
    SU3_ERR_HIP = -6            /* HIP runtime error (text in su3_last_error) */
} su3_status;

/* Storage precision.  Arithmetic is double for SU3_F64 and single for the
 * others (fused multiply-add allowed).  Quantisation from double uses
 * round-to-nearest-even: F32 once; F16 double->float->half (two roundings,
 * subnormals kept); C12 stores rows 0-1 as float and rebuilds row 2 as
 * conj(row0 x row1) in registers. */
typedef enum su3_precision {
    SU3_F64 = 0,
    SU3_F32 = 1,
    SU3_F16_F32ACC = 2,
    SU3_C12_F32 = 3
} su3_precision;

typedef enum su3_layout {
    SU3_LAYOUT_AOS = 0,
    SU3_LAYOUT_SOA = 1,
    SU3_LAYOUT_AOSOA = 2,
    /* made by su3_vnode_alloc / su3_vnode_wrap only; as a launch-tuning
     * key its `lanes` is N_sub */
    SU3_LAYOUT_VNODE = 3
} su3_layout;

/* What a field holds per site: a 3x3 complex matrix or a spinor (4 spins x
 * 3 colours). */
typedef enum su3_kind {
    SU3_KIND_MATRIX = 0,
    SU3_KIND_SPINOR = 1,
    SU3_KIND_REAL = 2,    /* one real per site */
    SU3_KIND_COMPLEX = 3  /* one complex number per site */
} su3_kind;

/* Fixed site-local expressions (Section 3, Listings 1-2; sums and
 * products associate left to right, as C++ expressions do):
 *   MUL    z = a*b            (2 operands)  -- the streaming test, Listing 3
 *   MUL3   z = (a*b)*c        (3 operands)
 *   MULADD z = (a*b) + (c*d)  (4 operands)
 *   ADD    z = a + b          (2 operands)
 *   APB_AB z = (a+b) + (a*b)  (2 operands)
 * Intermediates stay in registers in the arithmetic precision.
 * SU3_C12_F32 supports MUL and MUL3 only (sums leave SU(3)). */
typedef enum su3_expr {
    SU3_EXPR_MUL = 0,
    SU3_EXPR_MUL3 = 1,
    SU3_EXPR_MULADD = 2,
    SU3_EXPR_ADD = 3,
    SU3_EXPR_APB_AB = 4,
    /* launch-tuning keys of su3_cshift and su3_mult_shifted (accepted by
     * su3_autotune / su3_launch_get / su3_launch_set only) */
    SU3_EXPR_CSHIFT = 5,
    SU3_EXPR_MUL_SHIFTED = 6,
    /* launch-tuning key of su3_dslash; its precision is the links' one
     * (SU3_F64, SU3_F32 or SU3_C12_F32) */
    SU3_EXPR_DSLASH = 7,
    /* launch-tuning key of su3_program_eval; its precision is the
     * arithmetic one (SU3_F64 or SU3_F32) */
    SU3_EXPR_PROGRAM = 8,
    /* the same for programs with matrix values and a real or complex
     * result (a trace: nearly read-only streams, whose best launch differs
     * from a matrix result's); su3_autotune times it on trace(a*adj(b)) */
    SU3_EXPR_PROGRAM_SCALAR = 9,
    /* launch-tuning keys of batches: SU3_EXPR_BATCH + the leading item's
     * expression (MUL .. APB_AB), with its precision, layout and lanes, at
     * the batch's total volume (su3_launch_get / su3_launch_set; what
     * su3_batch_autotune tunes and su3_batch_create reads) */
    SU3_EXPR_BATCH = 32
} su3_expr;

typedef struct su3_field su3_field;
typedef struct su3_batch su3_batch;
typedef struct su3_program su3_program;

/* How a compute call is launched.  Any valid setting gives bit-identical
 * results; only speed differs.
 *   block       lanes per workgroup: 64, 128 or 256; 512 and 1024 for the
 *               site-local calls with nontemporal 3 or 7 and for
 *               su3_dslash's LDS-tiled walks (512)
 *   persistent  0: one lane per site group (one-shot grid); batches: one
 *               workgroup per tile.  k > 0: k workgroups per compute unit
 *               loop over the work (grid-stride over site groups or tiles;
 *               su3_dslash's LDS-tiled walks: each workgroup walks an equal
 *               share of the (tile, t-slice) pairs, tile after tile)
 *   nontemporal bit 0: nontemporal loads, bit 1: nontemporal stores,
 *               bit 2 (with bit 1; site-local calls, shifts, batches and
 *               the yardsticks only): write-through streaming stores,
 *               nontemporal at system scope, which move results to HBM
 *               faster than nontemporal stores on gfx950; values 0-3, 6, 7
 *               (su3_dslash and programs 0-3; su3_dslash: bit 0 applies to
 *               link loads only; the LDS-tiled walks always load cached,
 *               store nontemporal)
 *   xcd_remap   1: hand each of the 8 XCDs a contiguous range of
 *               workgroups instead of the hardware's round-robin;
 *               2 (su3_dslash's LDS-tiled walks): each XCD walks one
 *               contiguous range of tiles, chunk after chunk
 *   lds_stage   AOS only: 1 stages each workgroup's sites through LDS with
 *               coalesced 16-byte copies (block <= 128)
 *   tile_sites  batched launch: sites per tile (multiple of 64).
 *               su3_dslash: t-slices each lane walks (1..4096, clipped to
 *               the t extent; 1 = one site per lane)
 *   occupancy   0: no cap; k > 0: at most k workgroups per compute unit
 *               (enforced by reserving LDS): fewer waves with their loads
 *               in flight keep HBM streaming efficiently
 *   schedule    0: each lane loads every operand entry, then stores every
 *               result entry; 1: row-phased -- right-hand operands in
 *               full, then per result row the left operands' row, the
 *               row's evaluation and its stores.
 *               su3_dslash (lexicographic layouts): with one site per
 *               lane, 0 takes sites in index order and 1..3 give each
 *               workgroup a 4D tile of sites, 8x4x2x(B/64), 4x4x4x(B/64),
 *               8x2x2x(B/32) for block B; 4..16 are LDS-tiled walks:
 *               each workgroup holds a tile of (x, y, z) sites and walks
 *               tile_sites t-slices, sharing each slice's spinors through
 *               LDS: 4: 8x8x(B/64) with two slice buffers, 5: 8x8x(B/64),
 *               6: 8x4x(B/32), 7: 16x8x(B/128), 8: 16x4x(B/64) with one
 *               buffer; B = 128, 256 or 512 (6: 128 or 256, 7 and 8: 256
 *               or 512), limited to 48 KiB of buffers (a larger tile falls
 *               back to the schedule's smallest); 9..12 take whole x
 *               rows, tx x 2 x 2, tx x 2 x 4, tx x 4 x 2, tx x 4 x 4,
 *               where tx is the lattice's x extent (every x hop then
 *               comes from LDS); 13..16 the same with two slice buffers;
 *               17 and 18 take tx x 3 x 3 with one and two buffers;
 *               19..28 are the shapes of 9..18 with a halo: the tile's y
 *               and z face sites of each slice are loaded, spin
 *               projected, into LDS in the step before the slice
 *               (lexicographic fields; too large: one buffer, else no
 *               halo).  B is ignored: one lane per
 *               tile site, at most 512 for double spinors and 1024 for
 *               single, buffers in 160 KiB (else the rows with one
 *               buffer, rows of 2 x 2, or 16x4x4).  On virtual-node fields
 *               only schedules 9..18 apply, over outer sites with all
 *               their virtual nodes, tx the largest divisor of the outer
 *               x extent that fits 512 lanes (else one site per lane)
 *   sites_per_lane  site-local calls in the blocked layouts: consecutive
 *               sites each lane evaluates, 0 = the natural count (16-byte
 *               accesses: 1 double, 2 single or compressed, 4 half sites;
 *               2 half sites for 3-4 operands), else 1, the natural count,
 *               or for MUL outside half storage twice the natural count
 *               (32-byte accesses); the lane-block L must be a multiple
 *               (SU3_ERR_INVALID_ARG otherwise).  Ignored elsewhere       */
typedef struct su3_launch {
    int32_t block;
    int32_t persistent;
    int32_t nontemporal;
    int32_t xcd_remap;
    int32_t lds_stage;
    int32_t tile_sites;
    int32_t occupancy;
    int32_t schedule;
    int32_t sites_per_lane;
} su3_launch;

/* ------------------------------------------------------------- fields */

/* A field is the lattice-wide object of Section 4, Listing 3 (a
 * Lattice<Su3f> built on a grid: one 3x3 complex matrix per site of the 4D
 * lattice `dims`), stored in one of the layouts above.
 *
 * Bytes a field of lattice `dims` (4 extents, each > 0) occupies in the
 * given precision and layout.  `lanes` is read for SU3_LAYOUT_AOSOA only
 * (power of two in [8, 64]).  Fails with SU3_ERR_INVALID_ARG when the
 * stored field would hold 2^31 reals or more.  Pure host computation. */
su3_status su3_field_bytes(const int32_t dims[4], su3_precision prec,
                           su3_layout layout, int32_t lanes, size_t *bytes);

/* Allocate a zeroed field on the current device (the Lattice<Su3f>
 * construction of Section 4, Listing 3).  The handle owns its memory;
 * su3_field_free releases it.  SU3_ERR_OUT_OF_MEMORY when the
 * device allocation fails. */
su3_status su3_field_alloc(su3_field **out, const int32_t dims[4],
                           su3_precision prec, su3_layout layout,
                           int32_t lanes);

/* Describe caller-owned device memory (e.g. a torch tensor's storage) as a
 * field (Section 4, Listing 3's lattice object over memory the caller
 * owns, in place of the paper's managed memory, Section 3).  Non-owning: the caller keeps the memory alive until
 * su3_field_free(handle).  `dev_ptr` must be 16-byte aligned device memory
 * of the current device with at least su3_field_bytes() bytes
 * (SU3_ERR_INVALID_ARG otherwise).  Contents are used as they are. */
su3_status su3_field_wrap(su3_field **out, void *dev_ptr, size_t bytes,
                          const int32_t dims[4], su3_precision prec,
                          su3_layout layout, int32_t lanes);

/* Release a handle (and its memory if owning): the end of the lattice
 * object of Section 4, Listing 3.  NULL is accepted. */
su3_status su3_field_free(su3_field *f);

/* Device address and size of a field's storage (the stored layouts of
 * Sections 4-5). */
su3_status su3_field_data(const su3_field *f, void **dev_ptr, size_t *bytes);

/* Fill a field with its site values (the initial values of Listing 3's
 * operands, Section 4; in the stored layout of Sections 4-5).  Quantise
 * and pack V*18 canonical doubles (V*24 for a spinor field) into the field
 * (padding sites written as zero).  Completes before returning. */
su3_status su3_field_upload(su3_field *f, const double *host_aos,
                            void *stream);

/* Read a field's site values back (the inverse of su3_field_upload; the
 * result of Section 4, Listing 3's assignment, read back to check it).
 * Unpack the field into V*18 canonical doubles (V*24 for a spinor field;
 * exact widening).  For
 * SU3_C12_F32, rows 0-1 are the stored values and row 2 is rebuilt in
 * double as conj(row0 x row1).  Completes before returning. */
su3_status su3_field_download(const su3_field *f, double *host_aos,
                              void *stream);

/* Copy the stored image byte for byte into host memory (`bytes` must be at
 * least the field's size): the layouts of Sections 4-5 as stored.
 * Completes before returning. */
su3_status su3_field_download_raw(const su3_field *f, void *host,
                                  size_t bytes, void *stream);

/* ------------------------------------------------------------ compute */

/* z = x * y at every site (Section 4, Listing 3).  Same as
 * su3_fused_eval(z, SU3_EXPR_MUL, {x, y}, 2, stream). */
su3_status su3_mult(su3_field *z, const su3_field *x, const su3_field *y,
                    void *stream);

/* z = expr(ops[0..n_ops-1]) at every site, in one kernel: the expression
 * template engine's assignment of Section 3, Listing 1 (z[ss] =
 * eval(ss, expr) for every site ss), for the composite expressions of the
 * kind Listing 2 builds (sums and products of fields, left to right).
 * All fields share dims, precision, layout and lanes (SU3_ERR_MISMATCH otherwise);
 * n_ops must match the expression (SU3_ERR_INVALID_ARG).  z may be one of
 * the operands exactly (in-place); a partial overlap with any operand is
 * SU3_ERR_ALIAS. */
su3_status su3_fused_eval(su3_field *z, su3_expr expr,
                          const su3_field *const *ops, int32_t n_ops,
                          void *stream);

/* --------------------------------------------------- shifted operands */

/* dst(x) = src(x + shift * mu_hat) at every site, periodic in direction mu
 * (0..3 = x, y, z, t; site index x + Lx(y + Ly(z + Lz t))): the lattice
 * shift (Cshift) that the paper's outlook (Section 6) names as the routine
 * outside the expression engine that a stencil port needs.  Any integer
 * shift; dst and src share dims, precision, layout and lanes
 * (SU3_ERR_MISMATCH) and must not overlap at all (SU3_ERR_ALIAS: a shift
 * is a gather and cannot run in place). */
su3_status su3_cshift(su3_field *dst, const su3_field *src, int32_t mu,
                      int32_t shift, void *stream);

/* z(x) = x(x) * y(x + shift * mu_hat), periodic, in one kernel without an
 * intermediate shifted field: a product with a Cshift-ed operand, the
 * stencil pattern of the outlook (Section 6).  z may be x exactly; z must not overlap y
 * (SU3_ERR_ALIAS).  The compressed form rebuilds the shifted operand's
 * third row in registers. */
su3_status su3_mult_shifted(su3_field *z, const su3_field *x,
                            const su3_field *y, int32_t mu, int32_t shift,
                            void *stream);

/* ------------------------------------------------------ spinor fields */

/* A spinor field holds 4 spins x 3 colours of complex numbers per site
 * (12 complex entries, entry 3 * spin + colour, stored like a matrix
 * field's entries in the same layouts): the fermion fields the Dslash of
 * Section 6 acts on.  Precisions SU3_F64 and SU3_F32
 * (SU3_ERR_UNSUPPORTED otherwise).  The handles are su3_field handles:
 * su3_field_free, su3_field_data, su3_field_upload / su3_field_download
 * (V*24 canonical doubles: site, spin, colour, re/im) and
 * su3_field_download_raw apply to them; every matrix routine rejects them
 * (SU3_ERR_MISMATCH).  Arguments and errors as for the su3_field_* calls. */
su3_status su3_spinor_bytes(const int32_t dims[4], su3_precision prec,
                            su3_layout layout, int32_t lanes, size_t *bytes);
su3_status su3_spinor_alloc(su3_field **out, const int32_t dims[4],
                            su3_precision prec, su3_layout layout,
                            int32_t lanes);
su3_status su3_spinor_wrap(su3_field **out, void *dev_ptr, size_t bytes,
                           const int32_t dims[4], su3_precision prec,
                           su3_layout layout, int32_t lanes);

/* Wilson hopping term, the stencil of the Dslash operator that the
 * conclusions (Section 6) name as the next port, periodic in all four
 * directions (0..3 = x, y, z, t, x fastest):
 *   out(x) = sum_mu [ (1 - g_mu) U_mu(x) in(x + mu_hat)
 *                   + (1 + g_mu) U_mu(x - mu_hat)^dagger in(x - mu_hat) ]
 * with Euclidean chiral-basis gamma matrices g_k = [[0, -i s_k],
 * [i s_k, 0]] (s_k the Pauli matrices), g_4 = [[0, 1], [1, 0]].
 * `links[mu]` are four matrix fields (one per direction) and `in` / `out`
 * spinor fields, all of one lattice, layout and lanes on one device
 * (SU3_ERR_MISMATCH otherwise).  Precisions: SU3_F64 spinors with SU3_F64
 * links (double arithmetic), SU3_F32 spinors with SU3_F32 or SU3_C12_F32
 * links (single arithmetic; the compressed third row is rebuilt in
 * registers); other pairs SU3_ERR_UNSUPPORTED.  `out` must not overlap
 * `in` or a link field (SU3_ERR_ALIAS).  Asynchronous on `stream`. */
su3_status su3_dslash(su3_field *out, su3_field *const links[4],
                      const su3_field *in, void *stream);

/* ------------------------------------------------------ scalar fields */

/* Real or complex scalar fields (kind SU3_KIND_REAL / SU3_KIND_COMPLEX),
 * like the Lattice<double> fields of Section 3, Listing 2: one entry per
 * site, stored with E = 1 (real: V_pad reals; complex: V_pad (re, im)
 * pairs), so the layout changes only the padding.  Precisions SU3_F64 and
 * SU3_F32.  Host canonical data for upload/download: V doubles (real) or
 * V (re, im) pairs (complex).  Only expression programs (below) compute on
 * them.  Arguments and errors as su3_field_bytes / alloc / wrap;
 * SU3_ERR_INVALID_ARG for another kind. */
su3_status su3_scalar_bytes(const int32_t dims[4], su3_precision prec,
                            su3_layout layout, int32_t lanes, su3_kind kind,
                            size_t *bytes);
su3_status su3_scalar_alloc(su3_field **out, const int32_t dims[4],
                            su3_precision prec, su3_layout layout,
                            int32_t lanes, su3_kind kind);
su3_status su3_scalar_wrap(su3_field **out, void *dev_ptr, size_t bytes,
                           const int32_t dims[4], su3_precision prec,
                           su3_layout layout, int32_t lanes, su3_kind kind);

/* ------------------------------------------------ expression programs */

/* General site-local expressions (Section 3: the expression template
 * engine evaluates arbitrary expressions of lattice fields, real-valued
 * ones included (Listing 2), site by site (Listing 1)), compiled on the host into a register program
 * that one precompiled kernel evaluates at every site.  Grammar:
 *   expr    := term (('+' | '-') term)*
 *   term    := unary ('*' unary)*
 *   unary   := '-' unary | primary
 *   primary := number | 'i' | operand | func '(' expr ')' | '(' expr ')'
 *   operand := 'a' .. 'h'   (operand fields 0 .. 7, kinds[k] their kinds)
 *   func    := adj | conj | transpose | trace | real | imag
 * Values are real scalars, complex scalars or 3x3 complex matrices
 * (SU3_KIND_MATRIX operands); a scalar meets a matrix as a multiple of
 * the identity (s + M adds s to the diagonal, s * M scales), trace maps a
 * matrix to a complex scalar, real/imag map scalars to real scalars.
 * Products associate left to right: a*b*c = (a*b)*c.  A constant alone
 * ("1.0") assigns it to every site.  Spinor operands are unsupported.
 * SU3_ERR_INVALID_ARG for a syntax or type error, or an expression needing
 * more than 8 registers or 48 instructions (text in su3_last_error). */
su3_status su3_program_create(su3_program **out, const char *expr,
                              int32_t n_ops, const su3_kind *kinds);

/* Result kind (matrix, real or complex), instruction and register count
 * of a compiled expression (Section 3's expression, as compiled here). */
su3_status su3_program_info(const su3_program *p, su3_kind *result_kind,
                            int32_t *n_instr, int32_t *n_regs);

/* z = expr(ops[0..n_ops-1]) at every site, in one kernel.  Every field
 * shares dims, layout, lanes (and virtual-node split) with z; ops[k] has
 * kind kinds[k] and z the result kind (SU3_ERR_MISMATCH otherwise).
 * Arithmetic is double when every field is SU3_F64 and single when every
 * field is SU3_F32 or SU3_C12_F32 (mixed: SU3_ERR_MISMATCH; half:
 * SU3_ERR_UNSUPPORTED).  A compressed output needs an SU(3)-valued
 * expression (products, adj, transpose, conj of matrices)
 * (SU3_ERR_UNSUPPORTED otherwise).  Programs with matrix values run in
 * kernel variants of 2, 4 or 8 registers; the 8-register one runs one
 * wave per SIMD in double and two in single, and is slower per byte than
 * the others.  z may be an operand exactly; a partial overlap is
 * SU3_ERR_ALIAS.  The launch setting of SU3_EXPR_PROGRAM (tuned or set)
 * applies in full to programs with matrix values and a matrix result,
 * that of SU3_EXPR_PROGRAM_SCALAR to programs with matrix values and a
 * real or complex result; programs without a matrix value
 * take only its nontemporal bits and run 256-lane workgroups with no
 * occupancy cap. */
su3_status su3_program_eval(const su3_program *p, su3_field *z,
                            const su3_field *const *ops, int32_t n_ops,
                            void *stream);

/* Release a program (Section 3's expression, as compiled here).  NULL is
 * accepted. */
su3_status su3_program_destroy(su3_program *p);

/* --------------------------------------------- Grid virtual-node layout */

/* Fields in Grid's virtual-node layout (SU3_LAYOUT_VNODE above; Section 5):
 * Grid-layout data on the device is used as it is, with no repacking.
 * `simd[mu]` (each >= 1, N_sub = their product a power of two <= 256)
 * must divide dims[mu] (SU3_ERR_INVALID_ARG otherwise).  Every call that
 * takes fields accepts these handles: site-local expressions and batches
 * run on the storage as AoSoA(N_sub) (batches need N_sub >= 4), shifts
 * and Dslash follow the virtual-node neighbours, and upload/download
 * convert from/to the canonical host order.  Fields are compatible only
 * with fields of the same dims, precision, kind and simd.  Arguments and
 * errors otherwise as su3_field_bytes / su3_field_alloc / su3_field_wrap
 * (matrix kind) and su3_spinor_* (spinor kind). */
su3_status su3_vnode_bytes(const int32_t dims[4], su3_precision prec,
                           su3_kind kind, const int32_t simd[4],
                           size_t *bytes);
su3_status su3_vnode_alloc(su3_field **out, const int32_t dims[4],
                           su3_precision prec, su3_kind kind,
                           const int32_t simd[4]);
su3_status su3_vnode_wrap(su3_field **out, void *dev_ptr, size_t bytes,
                          const int32_t dims[4], su3_precision prec,
                          su3_kind kind, const int32_t simd[4]);

/* ------------------------------------------------------------ batches */

/* A batch evaluates n independent (expr, z, operands) items -- fields of
 * different lattices, precisions and layouts -- in one persistent launch:
 * Section 3, Listing 1's site loop run over several lattices at once, with
 * each workgroup holding several vectors of lanes as Section 5 proposes
 * (the paper itself times one lattice per launch)
 * over a table of tiles, captured once in a HIP graph and replayed by
 * su3_batch_launch.  ops holds 4 pointers per item (unused = NULL).  Each
 * item obeys the rules of su3_fused_eval.  The tile table (see
 * su3_batch_tiles) is built on the host from the items' volumes and the
 * tuned tile size; the batch owns its device copy and its graph.  Fields
 * must outlive the batch.  Creation runs on `stream` and completes before
 * returning. */
su3_status su3_batch_create(su3_batch **out, const su3_expr *exprs,
                            su3_field *const *z, const su3_field *const *ops,
                            int32_t n, void *stream);

/* Evaluate the items of a batch once, in one launch, allocating no device
 * memory -- for callers that cannot allocate: code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc.  The items, their
 * rules and the results are those of su3_batch_create + su3_batch_launch;
 * the launch is the tuned (or set) setting of the batch key
 * (SU3_EXPR_BATCH + exprs[0], leading item's precision, layout and lanes,
 * total volume).  The item table (and a persistent grid's ticket counter)
 * go into a fixed scratch array that each device holds for the life of
 * the process, about 72 KiB for at most 1024 items (SU3_ERR_INVALID_ARG
 * beyond); small kernels on `stream` write it from their arguments, with
 * no copy from host memory, so the call can be captured into a graph.
 * Every call on a device shares that device's array and leaves its last
 * contents there: calls that overlap on one device (different streams, or
 * threads issuing to one stream unordered) race and give wrong results --
 * the caller orders them.  The fields must be on the current device
 * (SU3_ERR_MISMATCH).  Asynchronous on `stream`. */
su3_status su3_batch_run(const su3_expr *exprs, su3_field *const *z,
                         const su3_field *const *ops, int32_t n, void *stream);

/* Replay the batch's graph on `stream` (asynchronous): one pass of
 * Section 3, Listing 1's site loop over every item. */
su3_status su3_batch_launch(su3_batch *b, void *stream);

/* Release a batch (the batch of Section 3's site loop over several
 * lattices): its tile table and graph; the fields are untouched. */
su3_status su3_batch_destroy(su3_batch *b);

/* Copy the batch's tile table from the device: 4 int32 per tile, (item,
 * first site, site count, precision); item i's tiles are consecutive, in
 * site order, each covering tile_sites sites except the item's last.
 * `*n_tiles` receives the tile count; rows are written when cap >= it. */
su3_status su3_batch_tiles(const su3_batch *b, int32_t *rows, int64_t cap,
                           int64_t *n_tiles);
/* (The kernel itself holds only each item's first tile index and the tile
 * size, and finds a tile's item by binary search; su3_batch_tiles expands
 * the rows from exactly those device-resident values.) */

/* ------------------------------------------------------ launch tuning */

/* Run the autotuner for one (expr, precision, layout, lanes) at lattice
 * dims -- the block-size / vector-length study of Section 5 (Fig. 4) and
 * Section 4's observation that launch choices alone separate two ports of
 * the same loop, done per configuration at run time: time each candidate
 * launch (median of 10 after 3 warm-ups) on
 * scratch fields and keep the fastest for every later call whose volume
 * falls in the same power-of-two bucket.  The result persists in the JSON
 * file named by the SU3_TUNE_CACHE environment variable, if set.  Fields
 * are allocated and freed internally; when one set of operands takes 64
 * to 512 MiB, enough sets for 1 GiB are allocated and launched in
 * rotation, so the launch is tuned for operands that are not in the
 * Infinity Cache.  `best` may be NULL. */
su3_status su3_autotune(su3_expr expr, su3_precision prec, su3_layout layout,
                        int32_t lanes, const int32_t dims[4], void *stream,
                        su3_launch *best);

/* Recommend a storage layout for `expr` (a site-local expression, MUL ..
 * APB_AB) in precision `prec` at lattice `dims`: run su3_autotune for SoA
 * and for AoSoA with 64, 32, 16 and 8 lanes (each tuned launch is kept as
 * su3_autotune keeps it) and return the layout and lanes whose tuned
 * launch is fastest, with that launch in *best and its median time in *us
 * (best and us may be NULL) -- Section 5's vector-length study (Fig. 4),
 * done per configuration at run time.  The AoS layout (the negative
 * control of Section 4) and Grid's virtual-node layout (the caller's
 * choice of split) are not candidates.  Completes before returning. */
su3_status su3_layout_recommend(su3_expr expr, su3_precision prec,
                                const int32_t dims[4], void *stream,
                                su3_layout *layout, int32_t *lanes,
                                su3_launch *best, double *us);

/* Autotune a batch (Section 5's launch-shape study, applied to the batch
 * of Section 3's loop over several lattices): build the batch with each
 * candidate launch (tile size,
 * one workgroup per tile or k per CU, occupancy cap, schedule, nontemporal
 * bits), time graph replays (median of 5 after 2), and keep the fastest for
 * later su3_batch_create calls on items of the same leading (expr,
 * precision, layout, lanes) and total-volume bucket.  Arguments as for
 * su3_batch_create.  The candidates write the items' outputs (with the
 * correct values).  Persists in SU3_TUNE_CACHE like su3_autotune.  `best`
 * may be NULL. */
su3_status su3_batch_autotune(const su3_expr *exprs, su3_field *const *z,
                              const su3_field *const *ops, int32_t n,
                              void *stream, su3_launch *best);

/* Launch settings used for a key (tuned, set, or the built-in default):
 * the launch choices of Sections 4-5 that the autotuner makes. */
su3_status su3_launch_get(su3_expr expr, su3_precision prec,
                          su3_layout layout, int32_t lanes,
                          const int32_t dims[4], su3_launch *out);

/* Force the launch settings for a key (validated; SU3_ERR_INVALID_ARG for
 * an unsupported setting), as su3_launch_get (Sections 4-5). */
su3_status su3_launch_set(su3_expr expr, su3_precision prec,
                          su3_layout layout, int32_t lanes,
                          const int32_t dims[4], const su3_launch *cfg);

/* Forget every tuned or set launch (the JSON cache file is left alone),
 * as su3_launch_get (Sections 4-5). */
su3_status su3_launch_reset(void);

/* ------------------------------------------- bandwidth yardsticks */

/* The STREAM-style yardsticks that the paper measures the product against
 * (Section 5, the triad beside the vector-layout kernel), as launchable
 * kernels with the same launch knobs as the product, so that the ceiling
 * of each read:write mix can be tuned like the product itself.  Arrays
 * a, b, c of `bytes` bytes each (a positive multiple of 16; 16-byte aligned
 * device pointers of the current device), one 16-byte element per lane:
 *   SU3_STREAM_TRIAD  a = b + s*c over doubles: reads 2 x bytes, writes
 *                     bytes (the 2:1 mix of z = x*y)
 *   SU3_STREAM_READ   reads b and c (2 x bytes), writes nothing: a's first
 *                     16 bytes are written only if an element of b + c
 *                     equals (s, -s)
 *   SU3_STREAM_WRITE  a = s: writes bytes (b, c unused, may be NULL)
 *   SU3_STREAM_COPY   a = b: reads bytes, writes bytes (c unused)
 * `cfg` (NULL = the kind's default) is read for block (64..1024, a multiple
 * of 64), occupancy and nontemporal (0-3, 6, 7); its other fields are
 * ignored.  Asynchronous on `stream`. */
typedef enum su3_stream_kind {
    SU3_STREAM_TRIAD = 0,
    SU3_STREAM_READ = 1,
    SU3_STREAM_WRITE = 2,
    SU3_STREAM_COPY = 3
} su3_stream_kind;

su3_status su3_stream(su3_stream_kind kind, void *a, const void *b,
                      const void *c, double s, size_t bytes,
                      const su3_launch *cfg, void *stream);

/* Section 5's yardstick, tuned: time every candidate launch of a
 * yardstick on the caller's arrays
 * (median of 10 launches after 3) and return the fastest in *best and its
 * time in *us (either may be NULL).  Overwrites `a`.  Completes before
 * returning. */
su3_status su3_stream_autotune(su3_stream_kind kind, void *a, const void *b,
                               const void *c, size_t bytes, void *stream,
                               su3_launch *best, double *us);

/* STREAM-style triad (Section 5's yardstick) a[i] = b[i] + s*c[i] over n
 * doubles with the default
 * launch of SU3_STREAM_TRIAD.  Device pointers, 16-byte aligned,
 * asynchronous on `stream`. */
su3_status su3_triad(double *a, const double *b, const double *c, double s,
                     int64_t n, void *stream);

/* Plain copy dst[i] = src[i] over `bytes` bytes (multiple of 16, 16-byte
 * aligned device pointers) with the default launch of SU3_STREAM_COPY
 * (Section 5's yardsticks; the copy that calibrates the HBM counters),
 * asynchronous on `stream`. */
su3_status su3_copy(void *dst, const void *src, size_t bytes, void *stream);

/* --------------------------------------------------------- utilities */

/* Wait for `stream` and report any pending HIP error (asynchronous kernel
 * faults surface here): where a timed pass of Section 4, Listing 3's loop
 * ends. */
su3_status su3_sync(void *stream);

/* Static text of a status code (the boundary's own error reporting; no
 * passage of the paper defines it). */
const char *su3_status_string(su3_status s);

/* Detail of the last failing call on this thread ("" if none; the
 * boundary's own error reporting, as su3_status_string). */
const char *su3_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SU3_H */
