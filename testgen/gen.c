/*
 * Seeded synthetic SU(3) link-field generator.
 *
 * Shared test input for both the oracle and the GPU library.  It draws
 * random matrices and nothing else: no product, fused expression,
 * quantiser or compressed-format code lives here.
 *
 * Recipe (one SU(3) matrix per lattice site, Haar distributed):
 *   - counter-based SplitMix64 (Steele, Lea & Flood, OOPSLA 2014):
 *       key   = mix64(seed ^ mix64(field_id + 1))
 *       r(n)  = mix64(key + (n + 1) * GOLDEN)
 *     with n = 12*s + m (m = 0..11) for site s; a redraw (attempt a > 0)
 *     adds a * REDRAW_STRIDE to n, so a site's matrix never depends on the
 *     lattice volume or on the thread count;
 *   - uniforms u = ((r >> 11) + 1) * 2^-53 in (0, 1];
 *   - Box-Muller on consecutive pairs: rho = sqrt(-2 ln u_a),
 *     g_a = rho cos(2 pi u_b), g_b = rho sin(2 pi u_b);
 *   - six complex Gaussian entries (g_2p + i g_2p+1), p = 0..5: entries 0-2
 *     form row 0, entries 3-5 form row 1;
 *   - Gram-Schmidt: row0 /= |row0|; row1 -= <row0,row1> row0 (inner product
 *     conjugate-linear in the first argument, projection applied twice);
 *     row1 /= |row1|;
 *   - row 2 completes the matrix as the conjugate of the cross product of
 *     rows 0 and 1, written with the Levi-Civita symbol.  Then
 *     det = row2 . (row0 x row1) = |row0 x row1|^2 = 1 and the rows are
 *     orthonormal, so the matrix is in SU(3).
 *
 * Output is the canonical host layout: double at ((s*3 + i)*3 + j)*2 + c,
 * c = 0 real, 1 imaginary, row i, column j.
 *
 * libm's log/cos/sin make the bits reproducible on one host; callers log a
 * hash of the buffer.
 */
#include <math.h>
#include <stdint.h>

#define GOLDEN 0x9E3779B97F4A7C15ULL
#define REDRAW_STRIDE (1ULL << 44)

static uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

uint64_t su3gen_key(uint64_t seed, uint64_t field_id)
{
    return mix64(seed ^ mix64(field_id + 1));
}

/* The n-th 64-bit draw of stream (seed, field_id). */
uint64_t su3gen_u64(uint64_t seed, uint64_t field_id, uint64_t n)
{
    return mix64(su3gen_key(seed, field_id) + (n + 1) * GOLDEN);
}

static double unit_open0(uint64_t r)
{
    return (double)((r >> 11) + 1) * 0x1.0p-53;
}

/* Draw one matrix into m[18]; returns 0 on success, 1 if a row was too
 * short to normalise (the caller redraws). */
static int draw_one(uint64_t key, uint64_t n0, double *m)
{
    double g[12];
    for (int p = 0; p < 6; ++p) {
        double ua = unit_open0(mix64(key + (n0 + 2 * p + 1) * GOLDEN));
        double ub = unit_open0(mix64(key + (n0 + 2 * p + 2) * GOLDEN));
        double rho = sqrt(-2.0 * log(ua));
        double th = 2.0 * M_PI * ub;
        g[2 * p] = rho * cos(th);
        g[2 * p + 1] = rho * sin(th);
    }
    /* a[k] = row 0, b[k] = row 1 as (re, im) pairs */
    double ar[3], ai[3], br[3], bi[3];
    for (int k = 0; k < 3; ++k) {
        ar[k] = g[2 * k];
        ai[k] = g[2 * k + 1];
        br[k] = g[6 + 2 * k];
        bi[k] = g[6 + 2 * k + 1];
    }
    double na = 0.0;
    for (int k = 0; k < 3; ++k)
        na += ar[k] * ar[k] + ai[k] * ai[k];
    na = sqrt(na);
    if (!(na > 1e-12))
        return 1;
    for (int k = 0; k < 3; ++k) {
        ar[k] /= na;
        ai[k] /= na;
    }
    /* p = sum_k conj(a_k) b_k; the projection is applied twice
     * ("twice is enough" re-orthogonalisation) to keep rounding low */
    for (int pass = 0; pass < 2; ++pass) {
        double pr = 0.0, pi = 0.0;
        for (int k = 0; k < 3; ++k) {
            pr += ar[k] * br[k] + ai[k] * bi[k];
            pi += ar[k] * bi[k] - ai[k] * br[k];
        }
        for (int k = 0; k < 3; ++k) {
            br[k] -= pr * ar[k] - pi * ai[k];
            bi[k] -= pr * ai[k] + pi * ar[k];
        }
    }
    double nb = 0.0;
    for (int k = 0; k < 3; ++k)
        nb += br[k] * br[k] + bi[k] * bi[k];
    nb = sqrt(nb);
    if (!(nb > 1e-12))
        return 1;
    for (int k = 0; k < 3; ++k) {
        br[k] /= nb;
        bi[k] /= nb;
    }
    /* c_k = conj( sum_{i,j} eps_{kij} a_i b_j ) */
    double cr[3] = {0, 0, 0}, ci[3] = {0, 0, 0};
    for (int k = 0; k < 3; ++k) {
        for (int i = 0; i < 3; ++i) {
            for (int j = 0; j < 3; ++j) {
                int eps = 0;
                if (i == (k + 1) % 3 && j == (k + 2) % 3)
                    eps = 1;
                else if (i == (k + 2) % 3 && j == (k + 1) % 3)
                    eps = -1;
                if (eps == 0)
                    continue;
                double tr = ar[i] * br[j] - ai[i] * bi[j];
                double ti = ar[i] * bi[j] + ai[i] * br[j];
                cr[k] += eps * tr;
                ci[k] += eps * ti;
            }
        }
        ci[k] = -ci[k];
    }
    for (int k = 0; k < 3; ++k) {
        m[0 * 6 + 2 * k] = ar[k];
        m[0 * 6 + 2 * k + 1] = ai[k];
        m[1 * 6 + 2 * k] = br[k];
        m[1 * 6 + 2 * k + 1] = bi[k];
        m[2 * 6 + 2 * k] = cr[k];
        m[2 * 6 + 2 * k + 1] = ci[k];
    }
    return 0;
}

/* Fill out[count*18] with the matrices of sites s_begin .. s_begin+count-1
 * of stream (seed, field_id). */
void su3gen_field(uint64_t seed, uint64_t field_id, int64_t s_begin,
                  int64_t count, double *out)
{
    const uint64_t key = su3gen_key(seed, field_id);
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < count; ++t) {
        uint64_t s = (uint64_t)(s_begin + t);
        for (uint64_t a = 0;; ++a) {
            if (draw_one(key, 12 * s + a * REDRAW_STRIDE, out + 18 * t) == 0)
                break;
        }
    }
}

/* Draw a matrix of the given sites list (for sampled checks at large V). */
void su3gen_sites(uint64_t seed, uint64_t field_id, const int64_t *sites,
                  int64_t count, double *out)
{
    const uint64_t key = su3gen_key(seed, field_id);
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < count; ++t) {
        uint64_t s = (uint64_t)sites[t];
        for (uint64_t a = 0;; ++a) {
            if (draw_one(key, 12 * s + a * REDRAW_STRIDE, out + 18 * t) == 0)
                break;
        }
    }
}

/* Gaussian spinor field: 4 spins x 3 colours, each component a complex
 * Gaussian (re, im independent standard normals), site s drawing
 * n = 24*s + m from the same counter stream; out[count*24] in the layout
 * ((s*4 + spin)*3 + colour)*2 + c. */
void su3gen_spinor(uint64_t seed, uint64_t field_id, int64_t s_begin,
                   int64_t count, double *out)
{
    const uint64_t key = su3gen_key(seed, field_id);
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < count; ++t) {
        const uint64_t n0 = 24 * (uint64_t)(s_begin + t);
        for (int p = 0; p < 12; ++p) {
            double ua = unit_open0(mix64(key + (n0 + 2 * p + 1) * GOLDEN));
            double ub = unit_open0(mix64(key + (n0 + 2 * p + 2) * GOLDEN));
            double rho = sqrt(-2.0 * log(ua));
            out[24 * t + 2 * p] = rho * cos(2.0 * M_PI * ub);
            out[24 * t + 2 * p + 1] = rho * sin(2.0 * M_PI * ub);
        }
    }
}
