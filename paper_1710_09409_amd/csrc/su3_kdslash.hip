// Wilson hopping term on one GPU:
//   out(x) = sum_mu [ (1 - gamma_mu) U_mu(x) psi(x + mu_hat)
//                   + (1 + gamma_mu) U_mu(x - mu_hat)^dagger psi(x - mu_hat) ]
// periodic, in the chiral basis gamma_mu = [[0, A_mu], [A_mu^dagger, 0]]
// with A_1 = -i sigma_1, A_2 = -i sigma_2, A_3 = -i sigma_3, A_4 = 1.
//
// Each hop uses the spin projection: with h = psi_up + s A psi_dn,
// (1 + s gamma) psi = (h, s A^dagger h), so only the two spin components of
// h are colour-rotated (two 3x3 matrix-vector products instead of four).
// Three kernels, one lane per site each: k_dslash (sites in index order or
// in 4D tiles), k_dslash_walk (a lane walks t) and k_dslash_lds (a
// workgroup's tile of (x, y, z) sites walks t, sharing each slice through
// LDS).  Neighbours from the site index (x fastest), periodic.
#include <mutex>

#include "su3_device.h"
#include "su3_dslash.h"

namespace su3k {
namespace dslash {

template <class T>
__device__ __forceinline__ Cx<T> cadd(Cx<T> a, Cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <class T>
__device__ __forceinline__ Cx<T> csub(Cx<T> a, Cx<T> b) { return {a.re - b.re, a.im - b.im}; }
// i a and -i a
template <class T>
__device__ __forceinline__ Cx<T> ci(Cx<T> a) { return {-a.im, a.re}; }
template <class T>
__device__ __forceinline__ Cx<T> cmi(Cx<T> a) { return {a.im, -a.re}; }
template <class T>
__device__ __forceinline__ Cx<T> cscale(T s, Cx<T> a) { return {s * a.re, s * a.im}; }

// h = psi_up + s A_mu psi_dn  (psi[spin][colour])
template <int MU, int SGN, class T>
__device__ __forceinline__ void project(const Cx<T> (&p)[4][3], Cx<T> (&h)[2][3])
{
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        if constexpr (MU == 0) {        // A = [[0, -i], [-i, 0]]
            h[0][c] = SGN > 0 ? cadd(p[0][c], cmi(p[3][c])) : csub(p[0][c], cmi(p[3][c]));
            h[1][c] = SGN > 0 ? cadd(p[1][c], cmi(p[2][c])) : csub(p[1][c], cmi(p[2][c]));
        } else if constexpr (MU == 1) { // A = [[0, -1], [1, 0]]
            h[0][c] = SGN > 0 ? csub(p[0][c], p[3][c]) : cadd(p[0][c], p[3][c]);
            h[1][c] = SGN > 0 ? cadd(p[1][c], p[2][c]) : csub(p[1][c], p[2][c]);
        } else if constexpr (MU == 2) { // A = diag(-i, i)
            h[0][c] = SGN > 0 ? cadd(p[0][c], cmi(p[2][c])) : csub(p[0][c], cmi(p[2][c]));
            h[1][c] = SGN > 0 ? cadd(p[1][c], ci(p[3][c])) : csub(p[1][c], ci(p[3][c]));
        } else {                        // A = 1
            h[0][c] = SGN > 0 ? cadd(p[0][c], p[2][c]) : csub(p[0][c], p[2][c]);
            h[1][c] = SGN > 0 ? cadd(p[1][c], p[3][c]) : csub(p[1][c], p[3][c]);
        }
    }
}

// acc_up += w, acc_dn += s A_mu^dagger w
template <int MU, int SGN, class T>
__device__ __forceinline__ void reconstruct(const Cx<T> (&w)[2][3], Cx<T> (&acc)[4][3])
{
    const T s = SGN > 0 ? T(1) : T(-1);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        acc[0][c] = cadd(acc[0][c], w[0][c]);
        acc[1][c] = cadd(acc[1][c], w[1][c]);
        if constexpr (MU == 0) {        // A^dagger = [[0, i], [i, 0]]
            acc[2][c] = cadd(acc[2][c], cscale(s, ci(w[1][c])));
            acc[3][c] = cadd(acc[3][c], cscale(s, ci(w[0][c])));
        } else if constexpr (MU == 1) { // A^dagger = [[0, 1], [-1, 0]]
            acc[2][c] = cadd(acc[2][c], cscale(s, w[1][c]));
            acc[3][c] = csub(acc[3][c], cscale(s, w[0][c]));
        } else if constexpr (MU == 2) { // A^dagger = diag(i, -i)
            acc[2][c] = cadd(acc[2][c], cscale(s, ci(w[0][c])));
            acc[3][c] = cadd(acc[3][c], cscale(s, cmi(w[1][c])));
        } else {                        // A^dagger = 1
            acc[2][c] = cadd(acc[2][c], cscale(s, w[0][c]));
            acc[3][c] = cadd(acc[3][c], cscale(s, w[1][c]));
        }
    }
}

// w_k = M h_k (DAG = 0) or M^dagger h_k (DAG = 1) for both spin components
template <int DAG, class T>
__device__ __forceinline__ void color_mul(const Cx<T> (&m)[9], const Cx<T> (&h)[2][3],
                                          Cx<T> (&w)[2][3])
{
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            T re = T(0), im = T(0);
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const Cx<T> u = DAG ? m[3 * b + a] : m[3 * a + b];
                const T ui = DAG ? -u.im : u.im;
                re = fma_t(u.re, h[k][b].re, re);
                re = fma_t(-ui, h[k][b].im, re);
                im = fma_t(u.re, h[k][b].im, im);
                im = fma_t(ui, h[k][b].re, im);
            }
            w[k][a].re = re;
            w[k][a].im = im;
        }
}

template <int SP, int NT>
__device__ __forceinline__ void load_spinor(const void *base, uint32_t off, uint32_t plane,
                                            Cx<typename PrecT<SP>::T> (&p)[4][3])
{
    RawVec<SP, 1> raw[12];
    load_entries<SP, 1, NT, true, 0, 12>(static_cast<const typename PrecT<SP>::R *>(base),
                                         off, plane, 1, raw);
#pragma unroll
    for (int e = 0; e < 12; ++e)
        p[e / 3][e % 3] = widen<SP, 1>(raw[e], 0);
}

template <int LP, int NT>
__device__ __forceinline__ void load_link(const void *base, uint32_t off, uint32_t plane,
                                          Cx<typename PrecT<LP>::T> (&m)[9])
{
    constexpr int E = PrecT<LP>::E;
    RawVec<LP, 1> raw[E];
    load_entries<LP, 1, NT, true, 0, E>(static_cast<const typename PrecT<LP>::R *>(base),
                                        off, plane, 1, raw);
#pragma unroll
    for (int e = 0; e < E; ++e)
        m[e] = widen<LP, 1>(raw[e], 0);
    if constexpr (LP == su3i::C12)
        rebuild_row2(m);
}

// Pin the accumulators at this point of the instruction stream: every
// operation of the hop before must finish first, and (the asm being
// volatile) no load after it moves above it, so only one hop's operands
// are live at a time.
template <class T, int N>
__device__ __forceinline__ void fence_acc(Cx<T> (&acc)[N][3])
{
#pragma unroll
    for (int sp = 0; sp < N; ++sp)
#pragma unroll
        for (int c = 0; c < 3; ++c)
            __asm__ volatile("" : "+v"(acc[sp][c].re), "+v"(acc[sp][c].im));
}

// Pass an index through an empty volatile asm: loads addressed by it stay
// after the fences before it (the compiler cannot hoist them into an
// earlier hop, where their registers would add to that hop's).
__device__ __forceinline__ uint32_t pin(uint32_t x)
{
    __asm__ volatile("" : "+v"(x));
    return x;
}

// Forward hop (1 - gamma_mu) U_mu(x) psi(x + mu) from site sf.
template <int MU, int SP, int LP, int NT>
__device__ __forceinline__ void hop_fwd(const su3i::DslashArgs &a, uint32_t s,
                                        uint32_t sf,
                                        Cx<typename PrecT<SP>::T> (&acc)[4][3])
{
    using T = typename PrecT<SP>::T;
    Cx<T> p[4][3], m[9], h[2][3], w[2][3];
    load_spinor<SP, NT & 2>(a.in, site_offset(a.gs, pin(sf)), a.gs.plane, p);
    load_link<LP, NT>(a.u[MU], site_offset(a.gl, pin(s)), a.gl.plane, m);
    project<MU, -1>(p, h);
    color_mul<0>(m, h, w);
    reconstruct<MU, -1>(w, acc);
}

// Backward hop (1 + gamma_mu) U_mu(x - mu)^dagger psi(x - mu) from site sb.
template <int MU, int SP, int LP, int NT>
__device__ __forceinline__ void hop_bwd(const su3i::DslashArgs &a, uint32_t sb,
                                        Cx<typename PrecT<SP>::T> (&acc)[4][3])
{
    using T = typename PrecT<SP>::T;
    Cx<T> p[4][3], m[9], h[2][3], w[2][3];
    const uint32_t sbp = pin(sb);
    load_spinor<SP, NT & 2>(a.in, site_offset(a.gs, sbp), a.gs.plane, p);
    load_link<LP, NT>(a.u[MU], site_offset(a.gl, sbp), a.gl.plane, m);
    project<MU, +1>(p, h);
    color_mul<1>(m, h, w);
    reconstruct<MU, +1>(w, acc);
}

// Periodic neighbours of storage site s along MU (modulo 2^32, in range).
// c: outer coordinate, l: lane coordinate (0 outside the virtual-node
// layout).  Within the outer sub-lattice a step is +-stride; across its
// edge the outer coordinate wraps and the lane coordinate steps (wrapping
// over the lattice when there is one lane).
template <int MU>
__device__ __forceinline__ uint32_t fwd_site(const su3i::DslashArgs &a, uint32_t s,
                                             uint32_t c, uint32_t l)
{
    const uint32_t stride = a.stride[MU], L = a.dims[MU];
    const uint32_t n = a.nlanes[MU], ls = a.lstride[MU];
    const uint32_t wrap = s - (L - 1) * stride + (l + 1 == n ? 0u - (n - 1) * ls : ls);
    return c + 1 == L ? wrap : s + stride;
}

template <int MU>
__device__ __forceinline__ uint32_t bwd_site(const su3i::DslashArgs &a, uint32_t s,
                                             uint32_t c, uint32_t l)
{
    const uint32_t stride = a.stride[MU], L = a.dims[MU];
    const uint32_t n = a.nlanes[MU], ls = a.lstride[MU];
    const uint32_t wrap = s + (L - 1) * stride + (l == 0 ? (n - 1) * ls : 0u - ls);
    return c == 0 ? wrap : s - stride;
}

// Both hops of direction MU (forward first).
template <int MU, int SP, int LP, int NT>
__device__ __forceinline__ void hop(const su3i::DslashArgs &a, uint32_t s,
                                    uint32_t c, uint32_t l,
                                    Cx<typename PrecT<SP>::T> (&acc)[4][3])
{
    hop_fwd<MU, SP, LP, NT>(a, s, fwd_site<MU>(a, s, c, l), acc);
    fence_acc(acc);
    hop_bwd<MU, SP, LP, NT>(a, bwd_site<MU>(a, s, c, l), acc);
    fence_acc(acc);
}

// Outer and lane coordinates of storage site s.
__device__ __forceinline__ void coords(const su3i::DslashArgs &a, uint32_t s,
                                       uint32_t (&c)[4], uint32_t (&l)[4])
{
    uint32_t r = s >> a.lg;
#pragma unroll
    for (int mu = 0; mu < 3; ++mu) {
        c[mu] = r % a.dims[mu];
        r /= a.dims[mu];
    }
    c[3] = r;
    if (a.lmask) {
        uint32_t q = s & a.lmask;
#pragma unroll
        for (int mu = 0; mu < 3; ++mu) {
            l[mu] = q % a.nlanes[mu];
            q /= a.nlanes[mu];
        }
        l[3] = q;
    } else {
#pragma unroll
        for (int mu = 0; mu < 4; ++mu)
            l[mu] = 0;
    }
}

template <int SP, int LP, int NT, int WPE = SP == su3i::F64 ? 3 : 4>
// WPE: at least this many waves per SIMD (caps the register budget)
__global__ __launch_bounds__(256, WPE) void k_dslash(su3i::DslashArgs a)
{
    extern __shared__ char occupancy_reserve[];
    using T = typename PrecT<SP>::T;
    const uint32_t blk = a.xcd_remap ? (uint32_t)xcd_remap(blockIdx.x, gridDim.x)
                                     : blockIdx.x;
    uint32_t s, c[4], l[4];
    bool inside;
    if (a.tile[0] == 0) {
        s = blk * blockDim.x + threadIdx.x;
        inside = s < (uint32_t)a.nsites;
        if (inside)
            coords(a, s, c, l);
    } else {
        // a workgroup covers a tile[0] x .. x tile[3] block of sites
        // (lexicographic fields only); tiles in x-fastest order
        uint32_t q = blk, r = threadIdx.x;
        inside = true;
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) {
            const uint32_t tq = mu < 3 ? q % a.ntile[mu] : q;
            q = mu < 3 ? q / a.ntile[mu] : 0;
            const uint32_t tr = mu < 3 ? r % a.tile[mu] : r;
            r = mu < 3 ? r / a.tile[mu] : 0;
            c[mu] = tq * a.tile[mu] + tr;
            l[mu] = 0;
            inside = inside && c[mu] < a.dims[mu];
        }
        s = c[0] + a.dims[0] * (c[1] + a.dims[1] * (c[2] + a.dims[2] * c[3]));
    }
    if (inside) {
        Cx<T> acc[4][3];
#pragma unroll
        for (int sp = 0; sp < 4; ++sp)
#pragma unroll
            for (int cc = 0; cc < 3; ++cc)
                acc[sp][cc] = {T(0), T(0)};
        // accumulation order shared with the walk kernels (results are
        // bitwise independent of the launch): t backward, then x, y, z
        // (forward, backward), then t forward
        hop_bwd<3, SP, LP, NT>(a, bwd_site<3>(a, s, c[3], l[3]), acc);
        fence_acc(acc);
        hop<0, SP, LP, NT>(a, s, c[0], l[0], acc);
        hop<1, SP, LP, NT>(a, s, c[1], l[1], acc);
        hop<2, SP, LP, NT>(a, s, c[2], l[2], acc);
        hop_fwd<3, SP, LP, NT>(a, s, fwd_site<3>(a, s, c[3], l[3]), acc);
        RawVec<SP, 1> raw[12];
#pragma unroll
        for (int e = 0; e < 12; ++e)
            narrow<SP, 1>(raw[e], 0, acc[e / 3][e % 3]);
        store_entries<SP, 1, NT, true, 0, 12>(static_cast<typename PrecT<SP>::R *>(a.out),
                                              site_offset(a.gs, s), a.gs.plane, 1, raw);
    }
    if (a.nsites < 0)
        occupancy_reserve[threadIdx.x] = 0;
}

// t-walk (lexicographic site order): a lane owns one (x, y, z) site and
// walks t-slices t0 .. t1-1.
// Along t each spinor and each t-link is loaded once per walk: at slice t
// the lane loads psi(t+1) and U_t(t) for the forward t-hop, and from the
// same registers prepares the next slice's backward t-hop,
//   wb(t+1) = U_t(t)^dagger (P+ psi(t)),  hc = P+ psi(t+1),
// carrying two half spinors (wb, hc) between slices.  The x, y, z hops
// are the one-site hops; their neighbours are loaded by adjacent lanes at
// about the same time and come from cache.  The result of slice t is
// stored after its forward t-hop (x, y, z hops first: the accumulation
// order of the one-site kernel).
template <int SP, int LP, int NT, int WPE = SP == su3i::F64 ? 2 : LP == su3i::C12 ? 3 : 4>
__global__ __launch_bounds__(256, WPE) void k_dslash_walk(su3i::DslashArgs a)
{
    extern __shared__ char occupancy_reserve[];
    using T = typename PrecT<SP>::T;
    const uint32_t blk = a.xcd_remap ? (uint32_t)xcd_remap(blockIdx.x, gridDim.x)
                                     : blockIdx.x;
    // lanes in site order over the (x, y, z) volume, then t-chunks
    const uint32_t tid = blk * blockDim.x + threadIdx.x;
    const uint32_t V3 = a.stride[3], Lt = a.dims[3];
    const uint32_t chunk = tid / V3, r = tid - chunk * V3;
    const uint32_t t0 = chunk * a.walk;
    if (t0 < Lt) {
        uint32_t c[3], q = r;
#pragma unroll
        for (int mu = 0; mu < 2; ++mu) {
            c[mu] = q % a.dims[mu];
            q /= a.dims[mu];
        }
        c[2] = q;
        const uint32_t t1 = t0 + a.walk < Lt ? t0 + a.walk : Lt;
        Cx<T> wb[2][3], hc[2][3];
        {   // backward t-hop of slice t0 and P+ psi(t0)
            const uint32_t sm = r + V3 * (t0 == 0 ? Lt - 1 : t0 - 1);
            Cx<T> p[4][3], m[9], h[2][3];
            load_spinor<SP, NT & 2>(a.in, site_offset(a.gs, sm), a.gs.plane, p);
            load_link<LP, NT>(a.u[3], site_offset(a.gl, sm), a.gl.plane, m);
            project<3, +1>(p, h);
            color_mul<1>(m, h, wb);
        }
        fence_acc(wb);
        {
            Cx<T> p[4][3];
            load_spinor<SP, NT & 2>(a.in, site_offset(a.gs, r + V3 * t0), a.gs.plane, p);
            project<3, +1>(p, hc);
        }
        fence_acc(hc);
        for (uint32_t t = t0; t < t1; ++t) {
            const uint32_t s = r + V3 * t;
            Cx<T> acc[4][3];
#pragma unroll
            for (int sp = 0; sp < 4; ++sp)
#pragma unroll
                for (int cc = 0; cc < 3; ++cc)
                    acc[sp][cc] = {T(0), T(0)};
            reconstruct<3, +1>(wb, acc);
            fence_acc(acc);
            hop<0, SP, LP, NT>(a, s, c[0], 0u, acc);
            hop<1, SP, LP, NT>(a, s, c[1], 0u, acc);
            hop<2, SP, LP, NT>(a, s, c[2], 0u, acc);
            {   // forward t-hop and the result; then from the same
                // registers the next slice's backward t-hop and P+ psi
                const uint32_t sp1 = r + V3 * (t + 1 == Lt ? 0 : t + 1);
                Cx<T> p[4][3], m[9], h[2][3], w[2][3];
                load_spinor<SP, NT & 2>(a.in, site_offset(a.gs, sp1), a.gs.plane, p);
                load_link<LP, NT>(a.u[3], site_offset(a.gl, s), a.gl.plane, m);
                project<3, -1>(p, h);
                color_mul<0>(m, h, w);
                reconstruct<3, -1>(w, acc);
                fence_acc(acc);
                RawVec<SP, 1> raw[12];
#pragma unroll
                for (int e = 0; e < 12; ++e)
                    narrow<SP, 1>(raw[e], 0, acc[e / 3][e % 3]);
                store_entries<SP, 1, NT, true, 0, 12>(
                    static_cast<typename PrecT<SP>::R *>(a.out), site_offset(a.gs, s),
                    a.gs.plane, 1, raw);
                color_mul<1>(m, hc, wb);
                project<3, +1>(p, hc);
            }
            fence_acc(wb);
            fence_acc(hc);
        }
    }
    if (a.nsites < 0)
        occupancy_reserve[threadIdx.x] = 0;
}

// ---------------------------------------------------------------------
// LDS-tiled walk: a workgroup owns a TX x TY x TZ tile of (x, y, z) sites
// (one lane each) and walks a chunk of t-slices.  Each step a lane loads
// psi(x, t+1) for its forward t-hop and also writes it to LDS, where it
// serves the tile's x, y and z hops of the next slice; only neighbours
// across the tile's faces (and across the lattice's periodic wrap) are
// read from global memory.  TX = 0: the tile spans whole x rows (TX is
// the lattice's x extent) and the x hops, periodic wrap included, all
// come from LDS.  NB = 2: two slice buffers and one barrier per step
// (slice t is read from one while slice t+1 is written to the other);
// NB = 1: one buffer, a barrier after the x, y, z hops and one after the
// write.  Accumulation order and arithmetic as in the other Dslash kernels.
// LDS layout: [buffer][entry][site of the tile], ns sites per entry.

template <int MU, int SP, int LP, int NT>
__device__ __forceinline__ void hop_fwd_tile(const su3i::DslashArgs &a, uint32_t s,
                                             uint32_t sf, bool in_tile, int lf,
                                             const Cx<typename PrecT<SP>::T> *tile, int ns,
                                             Cx<typename PrecT<SP>::T> (&acc)[4][3])
{
    using T = typename PrecT<SP>::T;
    Cx<T> p[4][3], m[9], h[2][3], w[2][3];
    if (in_tile) {
        // the LDS address is formed here, not hoisted out of the walk
        const Cx<T> *q = tile + pin((uint32_t)lf);
#pragma unroll
        for (int e = 0; e < 12; ++e)
            p[e / 3][e % 3] = q[e * ns];
    } else {
        load_spinor<SP, NT & 2>(a.in, site_offset(a.gs, sf), a.gs.plane, p);
    }
    load_link<LP, NT>(a.u[MU], site_offset(a.gl, s), a.gl.plane, m);
    project<MU, -1>(p, h);
    color_mul<0>(m, h, w);
    reconstruct<MU, -1>(w, acc);
}

template <int MU, int SP, int LP, int NT>
__device__ __forceinline__ void hop_bwd_tile(const su3i::DslashArgs &a, uint32_t sb,
                                             bool in_tile, int lb,
                                             const Cx<typename PrecT<SP>::T> *tile, int ns,
                                             Cx<typename PrecT<SP>::T> (&acc)[4][3])
{
    using T = typename PrecT<SP>::T;
    Cx<T> p[4][3], m[9], h[2][3], w[2][3];
    if (in_tile) {
        const Cx<T> *q = tile + pin((uint32_t)lb);
#pragma unroll
        for (int e = 0; e < 12; ++e)
            p[e / 3][e % 3] = q[e * ns];
    } else {
        load_spinor<SP, NT & 2>(a.in, site_offset(a.gs, sb), a.gs.plane, p);
    }
    load_link<LP, NT>(a.u[MU], site_offset(a.gl, sb), a.gl.plane, m);
    project<MU, +1>(p, h);
    color_mul<1>(m, h, w);
    reconstruct<MU, +1>(w, acc);
}

// Halo walks (row tiles on lexicographic fields): the y and z neighbours
// across the tile's faces are taken from the halo, where each face site
// waits already projected for the hop that reads it.  Face f of a halo
// buffer of nf sites holds its 6 complex numbers at f, f + nf, ...
template <int MU, int SP, int LP, int NT>
__device__ __forceinline__ void hop_fwd_halo(const su3i::DslashArgs &a, uint32_t s,
                                             bool in_tile, int lf,
                                             const Cx<typename PrecT<SP>::T> *tile, int ns,
                                             const Cx<typename PrecT<SP>::T> *halo, int nf,
                                             int face, Cx<typename PrecT<SP>::T> (&acc)[4][3])
{
    using T = typename PrecT<SP>::T;
    Cx<T> m[9], h[2][3], w[2][3];
    if (in_tile) {
        Cx<T> p[4][3];
        const Cx<T> *q = tile + pin((uint32_t)lf);
#pragma unroll
        for (int e = 0; e < 12; ++e)
            p[e / 3][e % 3] = q[e * ns];
        project<MU, -1>(p, h);
    } else {
        const Cx<T> *q = halo + pin((uint32_t)face);
#pragma unroll
        for (int e = 0; e < 6; ++e)
            h[e / 3][e % 3] = q[e * nf];
    }
    load_link<LP, NT>(a.u[MU], site_offset(a.gl, s), a.gl.plane, m);
    color_mul<0>(m, h, w);
    reconstruct<MU, -1>(w, acc);
}

template <int MU, int SP, int LP, int NT>
__device__ __forceinline__ void hop_bwd_halo(const su3i::DslashArgs &a, uint32_t sb,
                                             bool in_tile, int lb,
                                             const Cx<typename PrecT<SP>::T> *tile, int ns,
                                             const Cx<typename PrecT<SP>::T> *halo, int nf,
                                             int face, Cx<typename PrecT<SP>::T> (&acc)[4][3])
{
    using T = typename PrecT<SP>::T;
    Cx<T> m[9], h[2][3], w[2][3];
    if (in_tile) {
        Cx<T> p[4][3];
        const Cx<T> *q = tile + pin((uint32_t)lb);
#pragma unroll
        for (int e = 0; e < 12; ++e)
            p[e / 3][e % 3] = q[e * ns];
        project<MU, +1>(p, h);
    } else {
        const Cx<T> *q = halo + pin((uint32_t)face);
#pragma unroll
        for (int e = 0; e < 6; ++e)
            h[e / 3][e % 3] = q[e * nf];
    }
    load_link<LP, NT>(a.u[MU], site_offset(a.gl, sb), a.gl.plane, m);
    color_mul<1>(m, h, w);
    reconstruct<MU, +1>(w, acc);
}

// Face f of the halo of slice tt of tile (y0, z0): faces 0 .. tx*TZ-1 are
// the row below the tile in y (y0 - 1, periodic), then the row above its
// last row (y0 + TY, or 0 past the lattice's end), then the same two in z
// (tx*TY each); x fastest within a face.  Returns the face's kind (0, 1:
// below and above in y, 2, 3 in z) and its site, or -1 for a face site
// past the lattice in the other direction (a partial tile: no lane of the
// tile reads it).
template <int TY, int TZ>
__device__ __forceinline__ int halo_face(const su3i::DslashArgs &a, uint32_t y0, uint32_t z0,
                                         uint32_t tt, int tx, int f, uint32_t &site)
{
    const int fy = tx * TZ, fz = tx * TY;
    const uint32_t Ly = a.dims[1], Lz = a.dims[2];
    int kind, g;
    if (f < 2 * fy) {
        kind = f < fy ? 0 : 1;
        g = f - kind * fy;
    } else {
        kind = f < 2 * fy + fz ? 2 : 3;
        g = f - 2 * fy - (kind - 2) * fz;
    }
    const uint32_t x = (uint32_t)(g % tx), w = (uint32_t)(g / tx);
    uint32_t y, z;
    if (kind < 2) {
        z = z0 + w;
        y = kind == 0 ? (y0 == 0 ? Ly - 1 : y0 - 1) : (y0 + TY < Ly ? y0 + TY : 0u);
        if (z >= Lz)
            return -1;
    } else {
        y = y0 + w;
        z = kind == 2 ? (z0 == 0 ? Lz - 1 : z0 - 1) : (z0 + TZ < Lz ? z0 + TZ : 0u);
        if (y >= Ly)
            return -1;
    }
    site = x + a.stride[1] * y + a.stride[2] * z + a.stride[3] * tt;
    return kind;
}

// Project a face site's spinor for the hop that reads it (the sites below
// for backward hops, those above for forward ones) into halo slot f.
template <class T>
__device__ __forceinline__ void put_face(int kind, const Cx<T> (&p)[4][3], Cx<T> *halo,
                                         int nf, int f)
{
    Cx<T> h[2][3];
    if (kind == 0)
        project<1, +1>(p, h);
    else if (kind == 1)
        project<1, -1>(p, h);
    else if (kind == 2)
        project<2, +1>(p, h);
    else
        project<2, -1>(p, h);
#pragma unroll
    for (int e = 0; e < 6; ++e)
        halo[e * nf + f] = h[e / 3][e % 3];
}

// Fill halo faces first, first + nlanes, ... of slice tt (the workgroup's
// lanes share them).
template <int SP, int NT, int TY, int TZ>
__device__ __forceinline__ void load_halo(const su3i::DslashArgs &a, uint32_t y0, uint32_t z0,
                                          uint32_t tt, int tx, int first, int nlanes,
                                          Cx<typename PrecT<SP>::T> *halo)
{
    using T = typename PrecT<SP>::T;
    const int nf = 2 * tx * (TY + TZ);
    for (int f = first; f < nf; f += nlanes) {
        uint32_t site;
        const int kind = halo_face<TY, TZ>(a, y0, z0, tt, tx, f, site);
        if (kind < 0)
            continue;
        Cx<T> p[4][3];
        load_spinor<SP, NT & 2>(a.in, site_offset(a.gs, site), a.gs.plane, p);
        put_face(kind, p, halo, nf, f);
    }
}

// Most lanes a workgroup of the LDS-tiled walk has (row tiles: as many as
// rows_max_lanes allows) and the fewest waves per SIMD it must fit.
template <int SP, int TX, int TY, int TZ, bool VN>
constexpr int lds_max_lanes()
{
    return TX ? TX * TY * TZ : (SP == su3i::F64 ? 512 : VN ? 768 : 1024);
}
template <int SP, bool VN>
constexpr int lds_min_waves()
{
    return SP == su3i::F64 ? 2 : (VN ? 3 : 4);
}

template <int SP, int LP, int NT, int TX, int TY, int TZ, int NB, bool VN, bool HALO>
__global__ __launch_bounds__((lds_max_lanes<SP, TX, TY, TZ, VN>()), (lds_min_waves<SP, VN>()))
void k_dslash_lds(su3i::DslashArgs a)
{
    using T = typename PrecT<SP>::T;
    // VN: virtual-node fields, nl sites per outer site (one per virtual
    // node) stored side by side; the tile is tx x TY x TZ outer sites with
    // all their virtual nodes, lane l = node + nl * (outer site in tile)
    const int nl = VN ? (int)a.lmask + 1 : 1;
    const int tx = TX ? TX : (int)a.lds_tx;
    const int ns = nl * tx * TY * TZ;
    static_assert(!HALO || (!VN && TX == 0), "halos are built for whole rows of lexicographic fields");
    // the slice buffers in the dynamic LDS the host sizes to NB * 12 * ns
    // complex numbers, then (halo walks) NB halo buffers of 6 * nf
    extern __shared__ char occupancy_reserve[];
    Cx<T> *tile = reinterpret_cast<Cx<T> *>(occupancy_reserve);
    const int nf = HALO ? 2 * tx * (TY + TZ) : 0;
    Cx<T> *halo = tile + NB * 12 * ns;
    const uint32_t blk = a.xcd_remap == 1 ? (uint32_t)xcd_remap(blockIdx.x, gridDim.x)
                                          : blockIdx.x;
    const uint32_t ntiles = a.ntile[0] * a.ntile[1] * a.ntile[2];
    const uint32_t V3 = a.stride[3], Lt = a.dims[3];
    const int l = threadIdx.x;
    const int node = VN ? (l & (int)a.lmask) : 0, lo = VN ? (l >> a.lg) : l;
    const int lx = lo % tx, ly = (lo / tx) % TY, lz = lo / (tx * TY);
    // this site's virtual-node coordinate along each direction
    uint32_t ln[4] = {0u, 0u, 0u, 0u};
    if constexpr (VN) {
#pragma unroll
        for (int mu = 0; mu < 4; ++mu)
            ln[mu] = ((uint32_t)node / a.lstride[mu]) % a.nlanes[mu];
    }
    // the (tile, t-slice) pairs, tile-major, this workgroup walks: one
    // chunk of `walk` slices of one tile (workgroups chunk-major), or with
    // span > 0 the span pairs from blk * span on, continuing into the next
    // tile after its last slice (the same for every lane)
    uint32_t q, qend;
    if (a.span) {
        q = blk * a.span;
        qend = q + a.span < ntiles * Lt ? q + a.span : ntiles * Lt;
    } else {
        uint32_t chunk, tile_id;
        if (a.xcd_remap == 2) {
            // XCD slabs: workgroups are dealt to the 8 XCDs round-robin;
            // XCD k walks the tiles k * T8 .. (k + 1) * T8 - 1, chunk after
            // chunk, so the workgroups it runs together are neighbouring
            // tiles at the same t (their shared faces can hit its L2)
            const uint32_t t8 = (ntiles + 7) / 8, m = blk >> 3;
            chunk = m / t8;
            tile_id = (blk & 7) * t8 + (m - chunk * t8);
        } else {
            chunk = blk / ntiles;
            tile_id = blk - chunk * ntiles;
        }
        q = tile_id * Lt + chunk * a.walk;
        qend = tile_id * Lt + (chunk * a.walk + a.walk < Lt ? chunk * a.walk + a.walk : Lt);
        if (tile_id >= ntiles)
            qend = q;  // a slab's padding (the same for every lane)
    }
    while (q < qend) {
        const uint32_t tid = q / Lt, t0 = q - tid * Lt;
        const uint32_t t1 = t0 + (qend - q) < Lt ? t0 + (qend - q) : Lt;
        q += t1 - t0;
        uint32_t c[3];
        c[0] = (tid % a.ntile[0]) * tx + lx;
        c[1] = (tid / a.ntile[0] % a.ntile[1]) * TY + ly;
        c[2] = (tid / (a.ntile[0] * a.ntile[1])) * TZ + lz;
        const bool valid = c[0] < a.dims[0] && c[1] < a.dims[1] && c[2] < a.dims[2];
        const uint32_t r =
            VN ? (uint32_t)node + c[0] * a.stride[0] + c[1] * a.stride[1] + c[2] * a.stride[2]
               : c[0] + a.dims[0] * (c[1] + a.dims[1] * c[2]);
        // neighbours held by the tile (no periodic wrap, inside the lattice;
        // whole rows hold both x neighbours, across the wrap too, where the
        // x neighbour of a row end is the next virtual node's row start)
        // (lexicographic row tiles always span whole rows)
        const bool wrow = TX == 0 && (!VN || tx == (int)a.dims[0]);
        const bool xf = wrow || (lx + 1 < tx && c[0] + 1 < a.dims[0]);
        const bool xb = wrow || lx > 0;
        int nxf = node, nxb = node;
        if constexpr (VN) {
            const int ls = (int)a.lstride[0], nx = (int)a.nlanes[0];
            nxf = (int)ln[0] + 1 == nx ? node - (nx - 1) * ls : node + ls;
            nxb = ln[0] == 0 ? node + (nx - 1) * ls : node - ls;
        }
        const int lxf = lx + 1 < tx ? l + nl : nxf + nl * (lo - (tx - 1));
        const int lxb = lx > 0 ? l - nl : nxb + nl * (lo + (tx - 1));
        // (lexicographic fields: nl = 1, node = 0, l = lo)
        const bool yf = ly + 1 < TY && c[1] + 1 < a.dims[1], yb = ly > 0;
        const bool zf = lz + 1 < TZ && c[2] + 1 < a.dims[2], zb = lz > 0;

        Cx<T> wb[2][3];
        if (valid) {
            {   // backward t-hop of slice t0
                const uint32_t sm = VN ? bwd_site<3>(a, r + V3 * t0, t0, ln[3])
                                       : r + V3 * (t0 == 0 ? Lt - 1 : t0 - 1);
                Cx<T> p[4][3], m[9], h[2][3];
                load_spinor<SP, NT & 2>(a.in, site_offset(a.gs, sm), a.gs.plane, p);
                load_link<LP, NT>(a.u[3], site_offset(a.gl, sm), a.gl.plane, m);
                project<3, +1>(p, h);
                color_mul<1>(m, h, wb);
            }
            fence_acc(wb);
            {   // the tile's slice t0
                Cx<T> p[4][3];
                load_spinor<SP, NT & 2>(a.in, site_offset(a.gs, r + V3 * t0), a.gs.plane, p);
#pragma unroll
                for (int e = 0; e < 12; ++e)
                    tile[e * ns + l] = p[e / 3][e % 3];
            }
        }
        const uint32_t y0 = c[1] - ly, z0 = c[2] - lz;  // the tile's corner
        if constexpr (HALO)
            load_halo<SP, NT, TY, TZ>(a, y0, z0, t0, tx, l, (int)blockDim.x, halo);
        __syncthreads();
        int cur = 0;
        for (uint32_t t = t0; t < t1; ++t) {
            const uint32_t s = r + V3 * t;
            Cx<T> acc[4][3];
            if (valid) {
#pragma unroll
                for (int sp = 0; sp < 4; ++sp)
#pragma unroll
                    for (int cc = 0; cc < 3; ++cc)
                        acc[sp][cc] = {T(0), T(0)};
                reconstruct<3, +1>(wb, acc);
                fence_acc(acc);
                const Cx<T> *cur_tile = tile + cur * 12 * ns;
                const int ry = nl * tx, rz = nl * tx * TY;  // LDS strides of y, z
                hop_fwd_tile<0, SP, LP, NT>(a, s, fwd_site<0>(a, s, c[0], ln[0]), xf, lxf,
                                            cur_tile, ns, acc);
                fence_acc(acc);
                hop_bwd_tile<0, SP, LP, NT>(a, bwd_site<0>(a, s, c[0], ln[0]), xb, lxb,
                                            cur_tile, ns, acc);
                fence_acc(acc);
                if constexpr (HALO) {
                    const Cx<T> *cur_halo = halo + cur * 6 * nf;
                    const int fy = tx * TZ, fz = 2 * fy + lx;
                    hop_fwd_halo<1, SP, LP, NT>(a, s, yf, l + ry, cur_tile, ns, cur_halo, nf,
                                                fy + lx + tx * lz, acc);
                    fence_acc(acc);
                    hop_bwd_halo<1, SP, LP, NT>(a, bwd_site<1>(a, s, c[1], ln[1]), yb, l - ry,
                                                cur_tile, ns, cur_halo, nf, lx + tx * lz, acc);
                    fence_acc(acc);
                    hop_fwd_halo<2, SP, LP, NT>(a, s, zf, l + rz, cur_tile, ns, cur_halo, nf,
                                                fz + tx * TY + tx * ly, acc);
                    fence_acc(acc);
                    hop_bwd_halo<2, SP, LP, NT>(a, bwd_site<2>(a, s, c[2], ln[2]), zb, l - rz,
                                                cur_tile, ns, cur_halo, nf, fz + tx * ly, acc);
                    fence_acc(acc);
                } else {
                    hop_fwd_tile<1, SP, LP, NT>(a, s, fwd_site<1>(a, s, c[1], ln[1]), yf,
                                                l + ry, cur_tile, ns, acc);
                    fence_acc(acc);
                    hop_bwd_tile<1, SP, LP, NT>(a, bwd_site<1>(a, s, c[1], ln[1]), yb,
                                                l - ry, cur_tile, ns, acc);
                    fence_acc(acc);
                    hop_fwd_tile<2, SP, LP, NT>(a, s, fwd_site<2>(a, s, c[2], ln[2]), zf,
                                                l + rz, cur_tile, ns, acc);
                    fence_acc(acc);
                    hop_bwd_tile<2, SP, LP, NT>(a, bwd_site<2>(a, s, c[2], ln[2]), zb,
                                                l - rz, cur_tile, ns, acc);
                    fence_acc(acc);
                }
            }
            if constexpr (NB == 1)
                __syncthreads();  // slice t read by the whole tile
            if (valid) {
                {   // forward t-hop; the next slice's backward t-hop from this
                    // site's own psi(t) (still in LDS: each lane reads its
                    // own slot before writing it); next slice into LDS
                    const uint32_t sp1 = VN ? fwd_site<3>(a, s, t, ln[3])
                                            : r + V3 * (t + 1 == Lt ? 0 : t + 1);
                    Cx<T> p[4][3], m[9], h[2][3], w[2][3];
                    load_spinor<SP, NT & 2>(a.in, site_offset(a.gs, sp1), a.gs.plane, p);
                    load_link<LP, NT>(a.u[3], site_offset(a.gl, s), a.gl.plane, m);
                    project<3, -1>(p, h);
                    color_mul<0>(m, h, w);
                    reconstruct<3, -1>(w, acc);
                    {
                        const Cx<T> *own = tile + cur * 12 * ns + pin((uint32_t)l);
                        Cx<T> q[4][3], hc[2][3];
#pragma unroll
                        for (int e = 0; e < 12; ++e)
                            q[e / 3][e % 3] = own[e * ns];
                        project<3, +1>(q, hc);
                        color_mul<1>(m, hc, wb);
                    }
                    Cx<T> *next = tile + (NB == 1 ? 0 : (cur ^ 1) * 12 * ns);
#pragma unroll
                    for (int e = 0; e < 12; ++e)
                        next[e * ns + l] = p[e / 3][e % 3];
                }
                fence_acc(acc);
                fence_acc(wb);
                RawVec<SP, 1> raw[12];
#pragma unroll
                for (int e = 0; e < 12; ++e)
                    narrow<SP, 1>(raw[e], 0, acc[e / 3][e % 3]);
                store_entries<SP, 1, 2, true, 0, 12>(static_cast<typename PrecT<SP>::R *>(a.out),
                                                     site_offset(a.gs, s), a.gs.plane, 1, raw);
            }
            if constexpr (HALO) {
                // the next slice's faces, in the step in which the tiles
                // that own them load that slice (the same for every lane)
                if (t + 1 < t1)
                    load_halo<SP, NT, TY, TZ>(a, y0, z0, t + 1, tx, l, (int)blockDim.x,
                                              halo + (NB == 1 ? 0 : (cur ^ 1) * 6 * nf));
            }
            __syncthreads();
            if constexpr (NB == 2)
                cur ^= 1;
        }
    }
}

template <int SP, int LP, int NT, int TX, int TY, int TZ, int NB, bool VN = false,
          bool HALO = false>
static hipError_t launch_lds(int block, int grid, size_t shm, const su3i::DslashArgs &a,
                             hipStream_t st)
{
    auto *k = k_dslash_lds<SP, LP, NT, TX, TY, TZ, NB, VN, HALO>;
    if (block > lds_max_lanes<SP, TX, TY, TZ, VN>())
        return hipErrorInvalidValue;
    if (shm > 64 * 1024) {
        // beyond the default dynamic LDS of a workgroup: raise this kernel's
        // limit once per device (and whenever a larger tile needs more)
        static std::mutex mu;
        static int granted[64];
        int dev = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e != hipSuccess)
            return e;
        std::lock_guard<std::mutex> lock(mu);
        if (dev < 0 || dev >= 64 || granted[dev] < (int)shm) {
            e = hipFuncSetAttribute(reinterpret_cast<const void *>(k),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
            if (e != hipSuccess)
                return e;
            if (dev >= 0 && dev < 64)
                granted[dev] = (int)shm;
        }
    }
    hipLaunchKernelGGL(k, dim3(grid), dim3(block), shm, st, a);
    return hipGetLastError();
}

// Row tiles (schedules 9..16: tx x {2, 4} x {2, 4}, one or two buffers;
// 17, 18: tx x 3 x 3), lexicographic or virtual-node fields; 19..28 the
// same shapes with a halo (lexicographic fields).
template <int SP, int LP, int NT, bool VN, bool HALO>
static hipError_t go_rows_as(int shape, int block, int grid, size_t shm,
                             const su3i::DslashArgs &a, hipStream_t st)
{
    switch (shape) {
    case 9: return launch_lds<SP, LP, NT, 0, 2, 2, 1, VN, HALO>(block, grid, shm, a, st);
    case 10: return launch_lds<SP, LP, NT, 0, 2, 4, 1, VN, HALO>(block, grid, shm, a, st);
    case 11: return launch_lds<SP, LP, NT, 0, 4, 2, 1, VN, HALO>(block, grid, shm, a, st);
    case 12: return launch_lds<SP, LP, NT, 0, 4, 4, 1, VN, HALO>(block, grid, shm, a, st);
    case 13: return launch_lds<SP, LP, NT, 0, 2, 2, 2, VN, HALO>(block, grid, shm, a, st);
    case 14: return launch_lds<SP, LP, NT, 0, 2, 4, 2, VN, HALO>(block, grid, shm, a, st);
    case 15: return launch_lds<SP, LP, NT, 0, 4, 2, 2, VN, HALO>(block, grid, shm, a, st);
    case 16: return launch_lds<SP, LP, NT, 0, 4, 4, 2, VN, HALO>(block, grid, shm, a, st);
    case 17: return launch_lds<SP, LP, NT, 0, 3, 3, 1, VN, HALO>(block, grid, shm, a, st);
    case 18: return launch_lds<SP, LP, NT, 0, 3, 3, 2, VN, HALO>(block, grid, shm, a, st);
    default: return hipErrorInvalidValue;
    }
}

template <int SP, int LP, int NT, bool VN>
static hipError_t go_rows(int block, int grid, size_t shm, const su3i::DslashArgs &a,
                          hipStream_t st)
{
    if (a.lds_tile <= 18)
        return go_rows_as<SP, LP, NT, VN, false>((int)a.lds_tile, block, grid, shm, a, st);
    if constexpr (VN)
        return hipErrorInvalidValue;
    else
        return go_rows_as<SP, LP, NT, false, true>((int)a.lds_tile - 10, block, grid, shm, a,
                                                  st);
}

// The LDS-tiled walk by schedule and block (the shapes lds_shape accepts;
// those over 48 KiB of double-precision buffers are not instantiated).
template <int SP, int LP, int NT>
static hipError_t go_lds(int block, int grid, size_t shm, const su3i::DslashArgs &a,
                         hipStream_t st)
{
    constexpr bool single = SP != su3i::F64;
    if (a.lds_tile >= 9)  // row tiles: any lane count
        return a.lmask ? go_rows<SP, LP, NT, true>(block, grid, shm, a, st)
                       : go_rows<SP, LP, NT, false>(block, grid, shm, a, st);
    if (a.lmask)
        return hipErrorInvalidValue;  // fixed tiles: lexicographic fields only
    switch (a.lds_tile * 2048 + block) {
    case 4 * 2048 + 128: return launch_lds<SP, LP, NT, 8, 8, 2, 2>(block, grid, shm, a, st);
    case 5 * 2048 + 128: return launch_lds<SP, LP, NT, 8, 8, 2, 1>(block, grid, shm, a, st);
    case 5 * 2048 + 256: return launch_lds<SP, LP, NT, 8, 8, 4, 1>(block, grid, shm, a, st);
    case 6 * 2048 + 128: return launch_lds<SP, LP, NT, 8, 4, 4, 1>(block, grid, shm, a, st);
    case 6 * 2048 + 256: return launch_lds<SP, LP, NT, 8, 4, 8, 1>(block, grid, shm, a, st);
    case 7 * 2048 + 256: return launch_lds<SP, LP, NT, 16, 8, 2, 1>(block, grid, shm, a, st);
    case 8 * 2048 + 256: return launch_lds<SP, LP, NT, 16, 4, 4, 1>(block, grid, shm, a, st);
    default: break;
    }
    if constexpr (single) {
        switch (a.lds_tile * 2048 + block) {
        case 4 * 2048 + 256: return launch_lds<SP, LP, NT, 8, 8, 4, 2>(block, grid, shm, a, st);
        case 5 * 2048 + 512: return launch_lds<SP, LP, NT, 8, 8, 8, 1>(block, grid, shm, a, st);
        case 7 * 2048 + 512: return launch_lds<SP, LP, NT, 16, 8, 4, 1>(block, grid, shm, a, st);
        case 8 * 2048 + 512: return launch_lds<SP, LP, NT, 16, 4, 8, 1>(block, grid, shm, a, st);
        default: break;
        }
    }
    return hipErrorInvalidValue;
}

template <int SP, int LP, int NT>
static void go_nt(int block, int grid, size_t shm, const su3i::DslashArgs &a,
                  hipStream_t st)
{
    if (a.walk > 1)
        hipLaunchKernelGGL((k_dslash_walk<SP, LP, NT>), dim3(grid), dim3(block), shm, st, a);
    else
        hipLaunchKernelGGL((k_dslash<SP, LP, NT>), dim3(grid), dim3(block), shm, st, a);
}

template <int SP, int LP>
static hipError_t go(int nt, int block, int grid, size_t shm, const su3i::DslashArgs &a,
                     hipStream_t st)
{
    if (a.lds_tile)  // cached loads and nontemporal stores, whatever nt asks
        return go_lds<SP, LP, 2>(block, grid, shm, a, st);
    switch (nt & 3) {
    case 0:
        go_nt<SP, LP, 0>(block, grid, shm, a, st);
        break;
    case 1:
        go_nt<SP, LP, 1>(block, grid, shm, a, st);
        break;
    case 2:
        go_nt<SP, LP, 2>(block, grid, shm, a, st);
        break;
    default:
        go_nt<SP, LP, 3>(block, grid, shm, a, st);
        break;
    }
    return hipGetLastError();
}

}  // namespace dslash
}  // namespace su3k

namespace su3i {

hipError_t launch_dslash(int spinor_prec, int link_prec, int nt, int block,
                         int grid, size_t shm, const DslashArgs &a,
                         hipStream_t st)
{
    using namespace su3k::dslash;
    if (a.lds_tile) {
        LdsShape sh;
        const int cbytes = spinor_prec == F64 ? 16 : 8;
        if (!lds_shape((int)a.lds_tile, block, cbytes, (int)a.dims[0], (int)a.lmask + 1, sh) ||
            block != sh.nsub * sh.tx * sh.ty * sh.tz || (uint32_t)sh.tx != a.lds_tx ||
            shm < lds_shape_bytes(sh, cbytes))
            return hipErrorInvalidValue;
    } else if (block > 256) {
        return hipErrorInvalidValue;
    }
    if (spinor_prec == F64 && link_prec == F64)
        return go<F64, F64>(nt, block, grid, shm, a, st);
    if (spinor_prec == F32 && link_prec == F32)
        return go<F32, F32>(nt, block, grid, shm, a, st);
    if (spinor_prec == F32 && link_prec == C12)
        return go<F32, C12>(nt, block, grid, shm, a, st);
    return hipErrorInvalidValue;
}

}  // namespace su3i
