/*
 * Plain FP64 CPU oracle for the SU(3) x SU(3) streaming product and the
 * fixed set of fused site-local expressions.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code
 * with the GPU library: its own complex arithmetic, its own walk over the
 * stored layouts, its own float -> half rounding.
 *
 * Built with gcc -O2 -ffp-contract=off (no fused multiply-add, no
 * intrinsics), so every result is the textbook sequence of IEEE double
 * operations written below.
 *
 * Canonical host layout: double at ((s*3 + i)*3 + j)*2 + c for site s,
 * row i, column j, c = 0 real / 1 imaginary.
 *
 * Paper anchors (Boyle et al., "Performance Portability Strategies for Grid
 * C++ Expression Templates", Lattice 2017):
 *   - the streaming test assigns z = x*y site by site over a lattice of
 *     3x3 single-precision complex matrices (Section 4, Listing 3); the
 *     matrix class is a templated N x N complex matrix (Section 4);
 *   - expressions are evaluated site by site, _odata[ss] = eval(ss, expr)
 *     (Section 3, Listing 1), and composite expressions -- sums of fields
 *     and sums with products, as in the example of Section 3, Listing 2 --
 *     associate left to right;
 *   - the scalar (AoS) layout and the vector (AoSoV) layout whose scalar
 *     leaves hold several lanes (Sections 4 and 5), including Grid's split
 *     of the lattice into virtual nodes, one per SIMD lane (Section 5).
 * The reduced-precision storage forms (single, half with single-precision
 * arithmetic, two-row compressed) are not in the paper; their steps follow
 * the stated convention: quantise with round-to-nearest-even, widen
 * exactly, rebuild the third row as conj(row0 x row1).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { P_F64 = 0, P_F32 = 1, P_F16 = 2, P_C12 = 3 };
enum { L_AOS = 0, L_SOA = 1, L_AOSOA = 2 };
enum { X_MUL = 0, X_MUL3 = 1, X_MULADD = 2, X_ADD = 3, X_APB_AB = 4 };

/* Threads the site loops use (1 without OpenMP). */
int oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Set the thread count of later site loops (n <= 0: leave unchanged). */
void oracle_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0)
        omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------ one site */

/* 3x3 complex matrix as 18 doubles, entry (i,j) at 2*(3i+j) (+1 for im). */
static double re_(const double *m, int i, int j) { return m[2 * (3 * i + j)]; }
static double im_(const double *m, int i, int j) { return m[2 * (3 * i + j) + 1]; }

/* c = a * b, plain definition z_ij = sum_k a_ik b_kj, k ascending. */
static void mat_mul(const double *a, const double *b, double *c)
{
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j) {
            double re = 0.0, im = 0.0;
            for (int k = 0; k < 3; ++k) {
                double ar = re_(a, i, k), ai = im_(a, i, k);
                double br = re_(b, k, j), bi = im_(b, k, j);
                re += (ar * br) - (ai * bi);
                im += (ar * bi) + (ai * br);
            }
            c[2 * (3 * i + j)] = re;
            c[2 * (3 * i + j) + 1] = im;
        }
    }
}

static void mat_add(const double *a, const double *b, double *c)
{
    for (int t = 0; t < 18; ++t)
        c[t] = a[t] + b[t];
}

/* ------------------------------------------------------- whole lattice */

/* z(s) = x(s) * y(s) for every site. */
void oracle_mult(const double *x, const double *y, double *z, int64_t V)
{
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < V; ++s)
        mat_mul(x + 18 * s, y + 18 * s, z + 18 * s);
}

/* Fixed fused expressions, evaluated with C++ left-to-right association:
 *   MUL    = a*b
 *   MUL3   = (a*b)*c
 *   MULADD = (a*b) + (c*d)
 *   ADD    = a + b
 *   APB_AB = (a + b) + (a*b)
 * Intermediates stay in double.  Returns 0, or -1 for an unknown expr. */
int oracle_fused(int expr, const double *a, const double *b, const double *c,
                 const double *d, double *z, int64_t V)
{
    if (expr < X_MUL || expr > X_APB_AB)
        return -1;
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < V; ++s) {
        const double *as = a + 18 * s, *bs = b + 18 * s;
        double t1[18], t2[18];
        double *zs = z + 18 * s;
        switch (expr) {
        case X_MUL:
            mat_mul(as, bs, zs);
            break;
        case X_MUL3:
            mat_mul(as, bs, t1);
            mat_mul(t1, c + 18 * s, zs);
            break;
        case X_MULADD:
            mat_mul(as, bs, t1);
            mat_mul(c + 18 * s, d + 18 * s, t2);
            mat_add(t1, t2, zs);
            break;
        case X_ADD:
            mat_add(as, bs, zs);
            break;
        case X_APB_AB:
            mat_add(as, bs, t1);
            mat_mul(as, bs, t2);
            mat_add(t1, t2, zs);
            break;
        }
    }
    return 0;
}

/* ------------------------------------------------------- shifted fields */

/* dst(c) = src(c + shift * mu_hat) with periodic wrap in direction mu, for
 * every site coordinate c = (x, y, z, t); site index x + Lx(y + Ly(z + Lz t)).
 * The lattice-wide shift of the paper's outlook (Section 6, Cshift).
 * Returns -1 for a bad direction or extent. */
int oracle_cshift(const double *src, double *dst, const int32_t dims[4],
                  int mu, int64_t shift)
{
    if (mu < 0 || mu > 3)
        return -1;
    for (int d = 0; d < 4; ++d)
        if (dims[d] <= 0)
            return -1;
    int64_t c[4];
    for (c[3] = 0; c[3] < dims[3]; ++c[3])
        for (c[2] = 0; c[2] < dims[2]; ++c[2])
            for (c[1] = 0; c[1] < dims[1]; ++c[1])
                for (c[0] = 0; c[0] < dims[0]; ++c[0]) {
                    int64_t n[4] = {c[0], c[1], c[2], c[3]};
                    n[mu] = ((c[mu] + shift) % dims[mu] + dims[mu]) % dims[mu];
                    int64_t s = c[0] + dims[0] * (c[1] + dims[1] * (c[2] + dims[2] * c[3]));
                    int64_t t = n[0] + dims[0] * (n[1] + dims[1] * (n[2] + dims[2] * n[3]));
                    memcpy(dst + 18 * s, src + 18 * t, 18 * sizeof(double));
                }
    return 0;
}

/* --------------------------------------------------------- Wilson hopping */

/* Euclidean Dirac matrices in the chiral basis, gamma_mu for directions
 * mu = 0..3 = x, y, z, t:
 *   gamma_k = [[0, -i sigma_k], [i sigma_k, 0]] (k = 1, 2, 3),
 *   gamma_4 = [[0, 1], [1, 0]],
 * stored as [mu][row][col][re/im]. */
static const double GAMMA[4][4][4][2] = {
    /* gamma_1 */
    {{{0, 0}, {0, 0}, {0, 0}, {0, -1}},
     {{0, 0}, {0, 0}, {0, -1}, {0, 0}},
     {{0, 0}, {0, 1}, {0, 0}, {0, 0}},
     {{0, 1}, {0, 0}, {0, 0}, {0, 0}}},
    /* gamma_2 */
    {{{0, 0}, {0, 0}, {0, 0}, {-1, 0}},
     {{0, 0}, {0, 0}, {1, 0}, {0, 0}},
     {{0, 0}, {1, 0}, {0, 0}, {0, 0}},
     {{-1, 0}, {0, 0}, {0, 0}, {0, 0}}},
    /* gamma_3 */
    {{{0, 0}, {0, 0}, {0, -1}, {0, 0}},
     {{0, 0}, {0, 0}, {0, 0}, {0, 1}},
     {{0, 1}, {0, 0}, {0, 0}, {0, 0}},
     {{0, 0}, {0, -1}, {0, 0}, {0, 0}}},
    /* gamma_4 */
    {{{0, 0}, {0, 0}, {1, 0}, {0, 0}},
     {{0, 0}, {0, 0}, {0, 0}, {1, 0}},
     {{1, 0}, {0, 0}, {0, 0}, {0, 0}},
     {{0, 0}, {1, 0}, {0, 0}, {0, 0}}},
};

/* Spinor fields: 4 spins x 3 colours complex per site, double at
 * ((s*4 + spin)*3 + colour)*2 + c. */

/* out = (1 + sign*gamma_mu) * (M v) for one site, where M is the link or
 * its conjugate transpose (dagger = 1), v a 4x3 spinor; accumulated into
 * acc.  Written as the full 4x4 spin matrix times the colour-rotated
 * spinor, without spin projection. */
static void hop_term(const double *m, int dagger, const double *v, int mu,
                     double sign, double *acc)
{
    double w[4][3][2];
    for (int sp = 0; sp < 4; ++sp)
        for (int a = 0; a < 3; ++a) {
            double re = 0.0, im = 0.0;
            for (int b = 0; b < 3; ++b) {
                /* M_ab = m_ab, or conj(m_ba) for the dagger */
                double mr = dagger ? re_(m, b, a) : re_(m, a, b);
                double mi = dagger ? -im_(m, b, a) : im_(m, a, b);
                double vr = v[(sp * 3 + b) * 2], vi = v[(sp * 3 + b) * 2 + 1];
                re += mr * vr - mi * vi;
                im += mr * vi + mi * vr;
            }
            w[sp][a][0] = re;
            w[sp][a][1] = im;
        }
    for (int sp = 0; sp < 4; ++sp)
        for (int a = 0; a < 3; ++a) {
            double re = w[sp][a][0], im = w[sp][a][1]; /* identity part */
            for (int q = 0; q < 4; ++q) {
                double gr = sign * GAMMA[mu][sp][q][0];
                double gi = sign * GAMMA[mu][sp][q][1];
                re += gr * w[q][a][0] - gi * w[q][a][1];
                im += gr * w[q][a][1] + gi * w[q][a][0];
            }
            acc[(sp * 3 + a) * 2] += re;
            acc[(sp * 3 + a) * 2 + 1] += im;
        }
}

/* Wilson hopping term (the "Dslash" whose port the paper's outlook names):
 *   out(x) = sum_mu [ (1 - gamma_mu) U_mu(x) in(x + mu_hat)
 *                   + (1 + gamma_mu) U_mu(x - mu_hat)^dagger in(x - mu_hat) ]
 * periodic in every direction.  u[mu] are link fields (canonical 18
 * doubles per site), in/out spinor fields (24 doubles per site). */
int oracle_dslash(const double *const *u, const double *in, double *out,
                  const int32_t dims[4])
{
    for (int d = 0; d < 4; ++d)
        if (dims[d] <= 0)
            return -1;
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < dims[3]; ++t) {
        int64_t c[4];
        c[3] = t;
        for (c[2] = 0; c[2] < dims[2]; ++c[2])
            for (c[1] = 0; c[1] < dims[1]; ++c[1])
                for (c[0] = 0; c[0] < dims[0]; ++c[0]) {
                    int64_t s = c[0] + dims[0] * (c[1] + dims[1] * (c[2] + dims[2] * c[3]));
                    double acc[24];
                    for (int t = 0; t < 24; ++t)
                        acc[t] = 0.0;
                    for (int mu = 0; mu < 4; ++mu) {
                        int64_t f[4] = {c[0], c[1], c[2], c[3]};
                        int64_t b[4] = {c[0], c[1], c[2], c[3]};
                        f[mu] = (c[mu] + 1) % dims[mu];
                        b[mu] = (c[mu] + dims[mu] - 1) % dims[mu];
                        int64_t sf = f[0] + dims[0] * (f[1] + dims[1] * (f[2] + dims[2] * f[3]));
                        int64_t sb = b[0] + dims[0] * (b[1] + dims[1] * (b[2] + dims[2] * b[3]));
                        hop_term(u[mu] + 18 * s, 0, in + 24 * sf, mu, -1.0, acc);
                        hop_term(u[mu] + 18 * sb, 1, in + 24 * sb, mu, +1.0, acc);
                    }
                    memcpy(out + 24 * s, acc, sizeof acc);
                }
    }
    return 0;
}

/* ------------------------------------------------------ half precision */

/* IEEE binary32 -> binary16, round to nearest, ties to even, subnormals
 * kept, overflow to infinity.  NaN stays NaN (quiet). */
static uint16_t half_from_float(float f)
{
    uint32_t x;
    memcpy(&x, &f, 4);
    uint16_t sign = (uint16_t)((x >> 16) & 0x8000u);
    uint32_t bexp = (x >> 23) & 0xffu;
    uint32_t frac = x & 0x7fffffu;
    if (bexp == 0xffu)
        return (uint16_t)(sign | 0x7c00u | (frac ? 0x0200u : 0u));
    if (bexp == 0u) /* float zero or subnormal: below 2^-126, rounds to 0 */
        return sign;
    int e = (int)bexp - 127;        /* value = m * 2^(e-23) */
    uint32_t m = frac | 0x800000u;  /* 24-bit significand */
    int shift;                      /* bits to drop from m */
    int he;                         /* biased half exponent, 0 = subnormal */
    if (e >= -14) {
        shift = 13;
        he = e + 15;
    } else {
        shift = -e - 1;             /* unit of the result is 2^-24 */
        he = 0;
    }
    if (shift >= 25)
        return sign;
    uint32_t q = m >> shift;
    uint32_t rem = m & ((1u << shift) - 1u);
    uint32_t halfway = 1u << (shift - 1);
    if (rem > halfway || (rem == halfway && (q & 1u)))
        q += 1u;
    if (he == 0)                    /* q <= 0x400; 0x400 is the least normal */
        return (uint16_t)(sign | q);
    if (q == 0x800u) {              /* carried into the next binade */
        q = 0x400u;
        he += 1;
    }
    if (he >= 31)
        return (uint16_t)(sign | 0x7c00u);
    return (uint16_t)(sign | ((uint32_t)he << 10) | (q & 0x3ffu));
}

static double double_from_half(uint16_t h)
{
    int sgn = (h >> 15) & 1;
    int e = (h >> 10) & 31;
    int frac = h & 0x3ff;
    double v;
    if (e == 0)
        v = ldexp((double)frac, -24);
    else if (e == 31)
        v = frac ? NAN : INFINITY;
    else
        v = ldexp((double)(frac + 1024), e - 25);
    return sgn ? -v : v;
}

/* Quantisers on flat arrays of reals. */
void oracle_quant_f32(const double *in, float *out, int64_t n)
{
    for (int64_t t = 0; t < n; ++t)
        out[t] = (float)in[t];
}

/* double -> float (RNE) -> half (RNE): two roundings, the declared
 * convention for half storage. */
void oracle_quant_f16(const double *in, uint16_t *out, int64_t n)
{
    for (int64_t t = 0; t < n; ++t)
        out[t] = half_from_float((float)in[t]);
}

void oracle_dequant_f16(const uint16_t *in, double *out, int64_t n)
{
    for (int64_t t = 0; t < n; ++t)
        out[t] = double_from_half(in[t]);
}

/* ------------------------------------------- two-row compressed storage */

/* Overwrite row 2 of every matrix with conj(row0 x row1):
 *   r2_0 = conj(r0_1 r1_2 - r0_2 r1_1)
 *   r2_1 = conj(r0_2 r1_0 - r0_0 r1_2)
 *   r2_2 = conj(r0_0 r1_1 - r0_1 r1_0)                                   */
void oracle_c12_rebuild(double *m, int64_t V)
{
    for (int64_t s = 0; s < V; ++s) {
        double *ms = m + 18 * s;
        for (int k = 0; k < 3; ++k) {
            int p = (k + 1) % 3, q = (k + 2) % 3;
            double ar = re_(ms, 0, p), ai = im_(ms, 0, p);
            double br = re_(ms, 1, q), bi = im_(ms, 1, q);
            double cr = re_(ms, 0, q), ci = im_(ms, 0, q);
            double dr = re_(ms, 1, p), di = im_(ms, 1, p);
            double xr = (ar * br - ai * bi) - (cr * dr - ci * di);
            double xi = (ar * bi + ai * br) - (cr * di + ci * dr);
            ms[2 * (6 + k)] = xr;
            ms[2 * (6 + k) + 1] = -xi;
        }
    }
}

/* What a stored field holds, widened back to canonical double:
 * quantise every real, widen exactly; for the compressed form keep rows
 * 0-1 (single precision) and rebuild row 2 in double. */
int oracle_roundtrip(int prec, const double *in, double *out, int64_t V)
{
    int64_t n = 18 * V;
    switch (prec) {
    case P_F64:
        memcpy(out, in, (size_t)n * sizeof(double));
        return 0;
    case P_F32:
    case P_C12:
        for (int64_t t = 0; t < n; ++t)
            out[t] = (double)(float)in[t];
        if (prec == P_C12)
            oracle_c12_rebuild(out, V);
        return 0;
    case P_F16:
        for (int64_t t = 0; t < n; ++t)
            out[t] = double_from_half(half_from_float((float)in[t]));
        return 0;
    }
    return -1;
}

/* ------------------------------------------------------- stored layouts */

/* Entries stored per site: 9, or 6 (rows 0-1) for the compressed form. */
static int entries_of(int prec) { return prec == P_C12 ? 6 : 9; }
static int real_bytes(int prec)
{
    return prec == P_F64 ? 8 : (prec == P_F16 ? 2 : 4);
}

/* Sites per lane-block L and padded site count for a layout:
 *   AoS: L = 1, no padding;  AoSoA(lanes): L = lanes, pad to L;
 *   SoA: one block holding every site, padded to a multiple of 64.       */
static int layout_shape(int layout, int lanes, int64_t V, int64_t *L,
                        int64_t *Vpad)
{
    if (layout == L_AOS) {
        *L = 1;
        *Vpad = V;
    } else if (layout == L_SOA) {
        *Vpad = (V + 63) / 64 * 64;
        *L = *Vpad;
    } else if (layout == L_AOSOA) {
        if (lanes < 1)
            return -1;
        *L = lanes;
        *Vpad = (V + lanes - 1) / lanes * lanes;
    } else {
        return -1;
    }
    return 0;
}

int64_t oracle_field_bytes(int prec, int layout, int lanes, int64_t V)
{
    int64_t L, Vpad;
    if (layout_shape(layout, lanes, V, &L, &Vpad))
        return -1;
    return Vpad * entries_of(prec) * 2 * real_bytes(prec);
}

/* Write the stored image of a canonical field.  The stored order is the
 * nested walk: lane-block b, then entry e (row-major over the stored rows),
 * then site-in-block l, then re/im; padding sites are zero.  `out` must
 * hold oracle_field_bytes() bytes. */
int oracle_pack(const double *canon, int64_t V, int prec, int layout,
                int lanes, void *out)
{
    int64_t L, Vpad;
    if (layout_shape(layout, lanes, V, &L, &Vpad))
        return -1;
    int E = entries_of(prec);
    int64_t w = 0;
    for (int64_t b = 0; b < Vpad / L; ++b) {
        for (int e = 0; e < E; ++e) {
            for (int64_t l = 0; l < L; ++l) {
                int64_t s = b * L + l;
                for (int c = 0; c < 2; ++c, ++w) {
                    double v = s < V ? canon[18 * s + 2 * e + c] : 0.0;
                    if (prec == P_F64)
                        ((double *)out)[w] = v;
                    else if (prec == P_F16)
                        ((uint16_t *)out)[w] = half_from_float((float)v);
                    else
                        ((float *)out)[w] = (float)v;
                }
            }
        }
    }
    return 0;
}

/* Grid's virtual-node layout (Section 5): the lattice is split into
 * N_sub virtual nodes, simd[mu] of them along direction mu; each holds a
 * sub-lattice of extents r[mu] = dims[mu] / simd[mu] and occupies one SIMD
 * lane, so every scalar leaf of a site object is a vector of N_sub lanes.
 * The walk: outer site o (sub-lattice coordinates, x fastest), then entry
 * e, then virtual node n (node coordinates, x fastest), then re/im; the
 * lattice site is x[mu] = n[mu] * r[mu] + o[mu].  `entries` is the number
 * of stored complex entries per site and `canon_entries` the number per
 * canonical site (9 for matrices, 12 for spinors); the stored entries are
 * canonical entries 0 .. entries-1.  Returns -1 for an invalid split. */
static int vnode_walk_setup(const int32_t dims[4], const int32_t simd[4],
                            int64_t r[4], int64_t *nsub, int64_t *nouter)
{
    *nsub = 1;
    *nouter = 1;
    for (int mu = 0; mu < 4; ++mu) {
        if (dims[mu] <= 0 || simd[mu] <= 0 || dims[mu] % simd[mu] != 0)
            return -1;
        r[mu] = dims[mu] / simd[mu];
        *nsub *= simd[mu];
        *nouter *= r[mu];
    }
    return 0;
}

static int64_t vnode_site(const int32_t dims[4], const int64_t r[4],
                          const int32_t simd[4], int64_t o, int64_t n)
{
    int64_t site = 0, stride = 1;
    for (int mu = 0; mu < 4; ++mu) {
        const int64_t om = o % r[mu], nm = n % simd[mu];
        o /= r[mu];
        n /= simd[mu];
        site += (nm * r[mu] + om) * stride;
        stride *= dims[mu];
    }
    return site;
}

int oracle_vnode_pack(const double *canon, const int32_t dims[4],
                      const int32_t simd[4], int prec, int entries,
                      int canon_entries, void *out)
{
    int64_t r[4], nsub, nouter;
    if (vnode_walk_setup(dims, simd, r, &nsub, &nouter))
        return -1;
    int64_t w = 0;
    for (int64_t o = 0; o < nouter; ++o)
        for (int e = 0; e < entries; ++e)
            for (int64_t n = 0; n < nsub; ++n) {
                const int64_t site = vnode_site(dims, r, simd, o, n);
                for (int c = 0; c < 2; ++c, ++w) {
                    const double v = canon[2 * canon_entries * site + 2 * e + c];
                    if (prec == P_F64)
                        ((double *)out)[w] = v;
                    else if (prec == P_F16)
                        ((uint16_t *)out)[w] = half_from_float((float)v);
                    else
                        ((float *)out)[w] = (float)v;
                }
            }
    return 0;
}

/* Inverse of oracle_vnode_pack (exact widening; entries beyond `entries`
 * are left untouched). */
int oracle_vnode_unpack(const void *in, const int32_t dims[4],
                        const int32_t simd[4], int prec, int entries,
                        int canon_entries, double *canon)
{
    int64_t r[4], nsub, nouter;
    if (vnode_walk_setup(dims, simd, r, &nsub, &nouter))
        return -1;
    int64_t w = 0;
    for (int64_t o = 0; o < nouter; ++o)
        for (int e = 0; e < entries; ++e)
            for (int64_t n = 0; n < nsub; ++n) {
                const int64_t site = vnode_site(dims, r, simd, o, n);
                for (int c = 0; c < 2; ++c, ++w) {
                    double v;
                    if (prec == P_F64)
                        v = ((const double *)in)[w];
                    else if (prec == P_F16)
                        v = double_from_half(((const uint16_t *)in)[w]);
                    else
                        v = (double)((const float *)in)[w];
                    canon[2 * canon_entries * site + 2 * e + c] = v;
                }
            }
    return 0;
}

/* Inverse walk: stored image -> canonical double (exact widening); the
 * compressed form gets row 2 rebuilt in double. */
int oracle_unpack(const void *in, int64_t V, int prec, int layout, int lanes,
                  double *canon)
{
    int64_t L, Vpad;
    if (layout_shape(layout, lanes, V, &L, &Vpad))
        return -1;
    int E = entries_of(prec);
    int64_t w = 0;
    for (int64_t b = 0; b < Vpad / L; ++b) {
        for (int e = 0; e < E; ++e) {
            for (int64_t l = 0; l < L; ++l) {
                int64_t s = b * L + l;
                for (int c = 0; c < 2; ++c, ++w) {
                    if (s >= V)
                        continue;
                    double v;
                    if (prec == P_F64)
                        v = ((const double *)in)[w];
                    else if (prec == P_F16)
                        v = double_from_half(((const uint16_t *)in)[w]);
                    else
                        v = (double)((const float *)in)[w];
                    canon[18 * s + 2 * e + c] = v;
                }
            }
        }
    }
    if (prec == P_C12)
        oracle_c12_rebuild(canon, V);
    return 0;
}

/* ------------------------------------------------------------- metrics */

/* det of a 3x3 complex matrix by cofactor expansion along row 0. */
static void mat_det(const double *m, double *dr, double *di)
{
    double r = 0.0, i = 0.0;
    for (int j = 0; j < 3; ++j) {
        int p = (j + 1) % 3, q = (j + 2) % 3;
        /* cofactor C_0j = m1p m2q - m1q m2p (cyclic order keeps the sign) */
        double cr = (re_(m, 1, p) * re_(m, 2, q) - im_(m, 1, p) * im_(m, 2, q))
                  - (re_(m, 1, q) * re_(m, 2, p) - im_(m, 1, q) * im_(m, 2, p));
        double ci = (re_(m, 1, p) * im_(m, 2, q) + im_(m, 1, p) * re_(m, 2, q))
                  - (re_(m, 1, q) * im_(m, 2, p) + im_(m, 1, q) * re_(m, 2, p));
        r += re_(m, 0, j) * cr - im_(m, 0, j) * ci;
        i += re_(m, 0, j) * ci + im_(m, 0, j) * cr;
    }
    *dr = r;
    *di = i;
}

/* out[0] = E_max   = max |zh - z| over all reals
 * out[1] = r_max   = max over sites of max_ij |zh_ij - z_ij| / max_ij |z_ij|
 *                    (complex moduli; a site with z = 0 counts its
 *                    absolute error)
 * out[2] = D_U     = max over sites of max_ij |(zh zh^dagger)_ij - delta_ij|
 * out[3] = D_det   = max over sites of |det zh - 1|
 * `z` may be NULL: then only D_U and D_det of zh are computed.           */
void oracle_metrics(const double *zh, const double *z, int64_t V, double *out)
{
    double emax = 0.0, rmax = 0.0, du = 0.0, dd = 0.0;
    for (int64_t s = 0; s < V; ++s) {
        const double *a = zh + 18 * s;
        if (z) {
            const double *b = z + 18 * s;
            double num = 0.0, den = 0.0;
            for (int t = 0; t < 9; ++t) {
                double er = a[2 * t] - b[2 * t], ei = a[2 * t + 1] - b[2 * t + 1];
                double ae = fabs(er) > fabs(ei) ? fabs(er) : fabs(ei);
                if (ae > emax)
                    emax = ae;
                double d = sqrt(er * er + ei * ei);
                double m = sqrt(b[2 * t] * b[2 * t] + b[2 * t + 1] * b[2 * t + 1]);
                if (d > num)
                    num = d;
                if (m > den)
                    den = m;
            }
            double r = den > 0.0 ? num / den : num;
            if (r > rmax)
                rmax = r;
        }
        for (int i = 0; i < 3; ++i) {
            for (int j = 0; j < 3; ++j) {
                double re = 0.0, im = 0.0;
                for (int k = 0; k < 3; ++k) {
                    /* a_ik * conj(a_jk) */
                    re += re_(a, i, k) * re_(a, j, k) + im_(a, i, k) * im_(a, j, k);
                    im += im_(a, i, k) * re_(a, j, k) - re_(a, i, k) * im_(a, j, k);
                }
                if (i == j)
                    re -= 1.0;
                double dev = sqrt(re * re + im * im);
                if (dev > du)
                    du = dev;
            }
        }
        double dr, di;
        mat_det(a, &dr, &di);
        double dv = sqrt((dr - 1.0) * (dr - 1.0) + di * di);
        if (dv > dd)
            dd = dv;
    }
    out[0] = emax;
    out[1] = rmax;
    out[2] = du;
    out[3] = dd;
}

/* ------------------------------------------------------------------------
 * General site-local expressions (Section 3: the expression template
 * engine evaluates arbitrary expressions site by site, on real-valued
 * lattice fields too, as in its composite-expression example, Listing 2).  The text is parsed into a tree once
 * and the tree is evaluated at every site with plain double arithmetic.
 * Grammar: sums and differences of products of unary terms; a unary term
 * is an optional minus sign and a number, the imaginary unit i, an operand
 * a..h, a parenthesised expression, or adj / conj / transpose / trace /
 * real / imag of one.  Values are real scalars, complex scalars or 3x3
 * complex matrices; a scalar meets a matrix as that multiple of the
 * identity (added to the diagonal, or scaling every entry).
 * Operand kinds: 0 matrix (18 doubles per site), 2 real (1 double),
 * 3 complex (2 doubles).  Result written in the same forms.  Returns the
 * result kind, or -1 for a malformed or ill-typed expression.
 * ---------------------------------------------------------------------- */

enum { EN_OPND, EN_NUM, EN_NEG, EN_ADD, EN_SUB, EN_MUL, EN_FN };
enum { EF_ADJ, EF_CONJ, EF_TRANS, EF_TRACE, EF_REAL, EF_IMAG };
enum { ET_REAL = 0, ET_CPLX = 1, ET_MAT = 2 };

typedef struct {
    int kind, operand, fn, l, r, type;
    double re, im;
} enode;

typedef struct {
    const char *p;
    enode n[256];
    int count;
    int bad;
} eparse;

static int e_new(eparse *ps, int kind)
{
    if (ps->count >= 256) {
        ps->bad = 1;
        return 0;
    }
    enode *x = &ps->n[ps->count];
    memset(x, 0, sizeof *x);
    x->kind = kind;
    x->l = x->r = -1;
    return ps->count++;
}

static void e_space(eparse *ps)
{
    while (*ps->p == ' ' || *ps->p == '\t' || *ps->p == '\n')
        ps->p++;
}

static int e_sum(eparse *ps);

static int e_unary(eparse *ps)
{
    e_space(ps);
    if (ps->bad)
        return 0;
    const char c = *ps->p;
    if (c == '-') {
        ps->p++;
        int k = e_new(ps, EN_NEG);
        int child = e_unary(ps);
        ps->n[k].l = child;
        return k;
    }
    if ((c >= '0' && c <= '9') || c == '.') {
        char *end;
        double v = strtod(ps->p, &end);
        if (end == ps->p) {
            ps->bad = 1;
            return 0;
        }
        ps->p = end;
        int k = e_new(ps, EN_NUM);
        ps->n[k].re = v;
        return k;
    }
    if (c == '(') {
        ps->p++;
        int k = e_sum(ps);
        e_space(ps);
        if (*ps->p != ')')
            ps->bad = 1;
        else
            ps->p++;
        return k;
    }
    /* a name */
    char name[16];
    int len = 0;
    while (((*ps->p >= 'a' && *ps->p <= 'z') || (*ps->p >= 'A' && *ps->p <= 'Z')) &&
           len < 15)
        name[len++] = *ps->p++;
    name[len] = 0;
    if (len == 0) {
        ps->bad = 1;
        return 0;
    }
    if (len == 1 && name[0] == 'i') {
        int k = e_new(ps, EN_NUM);
        ps->n[k].im = 1.0;
        return k;
    }
    if (len == 1 && name[0] >= 'a' && name[0] <= 'h') {
        int k = e_new(ps, EN_OPND);
        ps->n[k].operand = name[0] - 'a';
        return k;
    }
    static const char *fns[] = {"adj", "conj", "transpose", "trace", "real", "imag"};
    for (int f = 0; f < 6; ++f)
        if (strcmp(name, fns[f]) == 0) {
            e_space(ps);
            if (*ps->p != '(') {
                ps->bad = 1;
                return 0;
            }
            ps->p++;
            int k = e_new(ps, EN_FN);
            ps->n[k].fn = f;
            int child = e_sum(ps);
            ps->n[k].l = child;
            e_space(ps);
            if (*ps->p != ')')
                ps->bad = 1;
            else
                ps->p++;
            return k;
        }
    ps->bad = 1;
    return 0;
}

static int e_product(eparse *ps)
{
    int k = e_unary(ps);
    for (;;) {
        e_space(ps);
        if (ps->bad || *ps->p != '*')
            return k;
        ps->p++;
        int m = e_new(ps, EN_MUL);
        int r = e_unary(ps);
        ps->n[m].l = k;
        ps->n[m].r = r;
        k = m;
    }
}

static int e_sum(eparse *ps)
{
    int k = e_product(ps);
    for (;;) {
        e_space(ps);
        if (ps->bad || (*ps->p != '+' && *ps->p != '-'))
            return k;
        int m = e_new(ps, *ps->p == '+' ? EN_ADD : EN_SUB);
        ps->p++;
        int r = e_product(ps);
        ps->n[m].l = k;
        ps->n[m].r = r;
        k = m;
    }
}

/* static types; -1 on a type error */
static int e_type(eparse *ps, int k, int nops, const int *kinds)
{
    enode *x = &ps->n[k];
    int a, b;
    switch (x->kind) {
    case EN_OPND:
        if (x->operand >= nops)
            return -1;
        x->type = kinds[x->operand] == 0 ? ET_MAT
                  : kinds[x->operand] == 2 ? ET_REAL
                  : kinds[x->operand] == 3 ? ET_CPLX
                                           : -1;
        return x->type;
    case EN_NUM:
        return x->type = x->im != 0.0 ? ET_CPLX : ET_REAL;
    case EN_NEG:
        return x->type = e_type(ps, x->l, nops, kinds);
    case EN_FN:
        a = e_type(ps, x->l, nops, kinds);
        if (a < 0)
            return -1;
        if (x->fn == EF_TRACE)
            return x->type = a == ET_MAT ? ET_CPLX : a;
        if (x->fn == EF_REAL || x->fn == EF_IMAG)
            return x->type = a == ET_MAT ? -1 : ET_REAL;
        return x->type = a;
    default:
        a = e_type(ps, x->l, nops, kinds);
        b = e_type(ps, x->r, nops, kinds);
        if (a < 0 || b < 0)
            return -1;
        if (a == ET_MAT || b == ET_MAT)
            return x->type = ET_MAT;
        return x->type = (a == ET_CPLX || b == ET_CPLX) ? ET_CPLX : ET_REAL;
    }
}

/* A value: 3x3 complex matrix m (row-major, re/im), or a scalar in m[0..1]. */
typedef struct {
    int mat;
    double m[18];
} evalue;

static void e_scalar_times(double sr, double si, const double *in, double *out)
{
    for (int e = 0; e < 9; ++e) {
        const double r = in[2 * e], i = in[2 * e + 1];
        out[2 * e] = sr * r - si * i;
        out[2 * e + 1] = sr * i + si * r;
    }
}

static evalue e_eval(const eparse *ps, int k, const double *const *fields,
                     const int *kinds, int64_t s)
{
    const enode *x = &ps->n[k];
    evalue v, a, b;
    memset(&v, 0, sizeof v);
    switch (x->kind) {
    case EN_OPND: {
        const double *f = fields[x->operand];
        if (kinds[x->operand] == 0) {
            v.mat = 1;
            memcpy(v.m, f + 18 * s, sizeof v.m);
        } else if (kinds[x->operand] == 2) {
            v.m[0] = f[s];
        } else {
            v.m[0] = f[2 * s];
            v.m[1] = f[2 * s + 1];
        }
        return v;
    }
    case EN_NUM:
        v.m[0] = x->re;
        v.m[1] = x->im;
        return v;
    case EN_NEG:
        a = e_eval(ps, x->l, fields, kinds, s);
        v.mat = a.mat;
        for (int t = 0; t < 18; ++t)
            v.m[t] = -a.m[t];
        return v;
    case EN_FN:
        a = e_eval(ps, x->l, fields, kinds, s);
        v.mat = a.mat;
        switch (x->fn) {
        case EF_ADJ:
        case EF_TRANS:
            if (!a.mat) {
                v = a;
                if (x->fn == EF_ADJ)
                    v.m[1] = -a.m[1];
                return v;
            }
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) {
                    v.m[2 * (3 * i + j)] = a.m[2 * (3 * j + i)];
                    v.m[2 * (3 * i + j) + 1] =
                        x->fn == EF_ADJ ? -a.m[2 * (3 * j + i) + 1] : a.m[2 * (3 * j + i) + 1];
                }
            return v;
        case EF_CONJ:
            v = a;
            for (int e = 0; e < 9; ++e)
                v.m[2 * e + 1] = -a.m[2 * e + 1];
            return v;
        case EF_TRACE:
            if (!a.mat)
                return a;
            v.mat = 0;
            v.m[0] = (a.m[0] + a.m[8]) + a.m[16];
            v.m[1] = (a.m[1] + a.m[9]) + a.m[17];
            return v;
        case EF_REAL:
            v.m[0] = a.m[0];
            return v;
        default:  /* imag */
            v.m[0] = a.m[1];
            return v;
        }
    default:
        break;
    }
    a = e_eval(ps, x->l, fields, kinds, s);
    b = e_eval(ps, x->r, fields, kinds, s);
    if (x->kind == EN_MUL) {
        if (a.mat && b.mat) {
            v.mat = 1;
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) {
                    double re = 0.0, im = 0.0;
                    for (int q = 0; q < 3; ++q) {
                        const double ar = a.m[2 * (3 * i + q)], ai = a.m[2 * (3 * i + q) + 1];
                        const double br = b.m[2 * (3 * q + j)], bi = b.m[2 * (3 * q + j) + 1];
                        re += ar * br - ai * bi;
                        im += ar * bi + ai * br;
                    }
                    v.m[2 * (3 * i + j)] = re;
                    v.m[2 * (3 * i + j) + 1] = im;
                }
        } else if (a.mat) {
            v.mat = 1;
            e_scalar_times(b.m[0], b.m[1], a.m, v.m);
        } else if (b.mat) {
            v.mat = 1;
            e_scalar_times(a.m[0], a.m[1], b.m, v.m);
        } else {
            v.m[0] = a.m[0] * b.m[0] - a.m[1] * b.m[1];
            v.m[1] = a.m[0] * b.m[1] + a.m[1] * b.m[0];
        }
        return v;
    }
    /* sum or difference; a scalar is added to (subtracted from) the diagonal */
    const double sg = x->kind == EN_ADD ? 1.0 : -1.0;
    if (!a.mat && !b.mat) {
        v.m[0] = a.m[0] + sg * b.m[0];
        v.m[1] = a.m[1] + sg * b.m[1];
        return v;
    }
    v.mat = 1;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            for (int c = 0; c < 2; ++c) {
                const int t = 2 * (3 * i + j) + c;
                const double av = a.mat ? a.m[t] : (i == j ? a.m[c] : 0.0);
                const double bv = b.mat ? b.m[t] : (i == j ? b.m[c] : 0.0);
                v.m[t] = av + sg * bv;
            }
    return v;
}

int oracle_eval_expr(const char *text, int nops, const int *kinds,
                     const double *const *fields, double *out, int64_t V)
{
    eparse ps;
    memset(&ps, 0, sizeof ps);
    ps.p = text;
    int root = e_sum(&ps);
    e_space(&ps);
    if (ps.bad || *ps.p)
        return -1;
    int ty = e_type(&ps, root, nops, kinds);
    if (ty < 0)
        return -1;
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < V; ++s) {
        evalue v = e_eval(&ps, root, fields, kinds, s);
        if (ty == ET_MAT)
            memcpy(out + 18 * s, v.m, sizeof v.m);
        else if (ty == ET_CPLX) {
            out[2 * s] = v.m[0];
            out[2 * s + 1] = v.m[1];
        } else {
            out[s] = v.m[0];
        }
    }
    return ty == ET_MAT ? 0 : (ty == ET_CPLX ? 3 : 2);
}
