// libsu3's C ABI and kernels run on the CPU (emulated launches, see
// hip/hip_runtime.h) against the FP64 oracle, under AddressSanitizer and
// UBSan: every precision x layout x expression on ragged lattices with two
// launch settings (which must agree), persistent grids, LDS staging, the
// batch (tile rows, replays, autotuner), the shifted operands and the
// Wilson hopping term (every precision pair and layout, two launch
// settings, argument validation), Grid's virtual-node layout (stored
// image, products, shifts, Dslash) and expression programs.  Any
// out-of-bounds access in a kernel's indexing aborts the run.  Prints
// "fails 0" on success.
#include "su3.h"
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>
#include <hip/hip_runtime.h>
extern "C" {
void su3gen_field(uint64_t seed, uint64_t field_id, int64_t s_begin, int64_t count, double *out);
int oracle_fused(int expr, const double *a, const double *b, const double *c, const double *d, double *z, int64_t V);
int oracle_roundtrip(int prec, const double *in, double *out, int64_t V);
int oracle_cshift(const double *src, double *dst, const int32_t dims[4], int mu, int64_t shift);
void oracle_mult(const double *x, const double *y, double *z, int64_t V);
int oracle_dslash(const double *const *u, const double *in, double *out, const int32_t dims[4]);
void su3gen_spinor(uint64_t seed, uint64_t field_id, int64_t s_begin, int64_t count, double *out);
int oracle_vnode_pack(const double *canon, const int32_t dims[4], const int32_t simd[4], int prec, int entries, int canon_entries, void *out);
int oracle_eval_expr(const char *text, int nops, const int *kinds, const double *const *fields, double *out, int64_t V);
}
static int nops_of(int e) { return e == 1 ? 3 : (e == 2 ? 4 : 2); }
static int fails = 0;

static double run_case(const int dims[4], int prec, int layout, int lanes, int expr, su3_launch *cfg)
{
    int64_t V = (int64_t)dims[0] * dims[1] * dims[2] * dims[3];
    int n = nops_of(expr);
    std::vector<std::vector<double>> h(n, std::vector<double>(18 * V)), hq(n, std::vector<double>(18 * V));
    for (int k = 0; k < n; ++k) {
        su3gen_field(1710, 100 + k, 0, V, h[k].data());
        oracle_roundtrip(prec, h[k].data(), hq[k].data(), V);
    }
    std::vector<double> want(18 * V), got(18 * V);
    oracle_fused(expr, hq[0].data(), hq[1].data(), n > 2 ? hq[2].data() : nullptr, n > 3 ? hq[3].data() : nullptr, want.data(), V);
    su3_field *f[5];
    for (int k = 0; k <= n; ++k) {
        if (su3_field_alloc(&f[k], dims, (su3_precision)prec, (su3_layout)layout, lanes) != SU3_OK) { printf("alloc: %s\n", su3_last_error()); fails++; return 1e30; }
        if (k) su3_field_upload(f[k], h[k - 1].data(), nullptr);
    }
    if (cfg) su3_launch_set((su3_expr)expr, (su3_precision)prec, (su3_layout)layout, lanes, dims, cfg);
    const su3_field *ops[4] = {f[1], f[2], f[3], f[4]};
    su3_status st = su3_fused_eval(f[0], (su3_expr)expr, ops, n, nullptr);
    if (cfg) su3_launch_reset();
    if (st != SU3_OK) { printf("eval: %s\n", su3_last_error()); fails++; return 1e30; }
    su3_field_download(f[0], got.data(), nullptr);
    double err = 0;
    int rows = prec == 3 ? 2 : 3;
    int nbad16 = 0;
    for (int64_t s = 0; s < V; ++s)
        for (int t = 0; t < rows * 6; ++t) {
            double d = std::fabs(got[18 * s + t] - want[18 * s + t]);
            err = std::max(err, d);
            if (prec == 2 && d > std::ldexp(std::fabs(want[18 * s + t]), -11) + 12 * std::ldexp(1.0, -24) * 3 + std::ldexp(1.0, -25)) nbad16++;
        }
    if (nbad16) printf("F16 elementwise bound violated at %d entries (expr %d)\n", nbad16, expr);
    for (int k = 0; k <= n; ++k) su3_field_free(f[k]);
    double tol = prec == 0 ? 1e-13 : (prec == 2 ? 5e-3 : 1e-5);
    if (!(err <= tol)) { fails++; printf("FAIL "); }
    return err;
}

int main(int argc, char **argv)
{
    int sizes[][4] = {{1, 1, 1, 1}, {3, 5, 7, 11}, {8, 8, 8, 8}};
    int lays[][2] = {{0, 0}, {1, 0}, {2, 8}, {2, 16}, {2, 32}, {2, 64}};
    for (auto &d : sizes)
        for (int prec = 0; prec < 4; ++prec)
            for (auto &l : lays)
                for (int expr = 0; expr < 5; ++expr) {
                    if (prec == 3 && expr > 1) continue;
                    su3_launch c0 = {64, 0, 3, 0, 0, 4096, 0, 0};
                    su3_launch c1 = {128, 0, 3, 1, 0, 4096, 4, 1};
                    if (l[0] == 0) c1.schedule = 0;
                    // streaming stores, 1024-lane persistent workgroups, and
                    // twice the natural sites per lane for the product
                    const int spl = (expr == 0 && prec != 2 && l[0] != 0) ? (prec == 0 ? 2 : 4) : 0;
                    su3_launch c2 = {1024, 1, 7, 0, 0, 4096, 0, l[0] == 0 ? 0 : 1, spl};
                    su3_launch c3 = {64, 0, 6, 0, 0, 4096, 2, 0, l[0] == 0 ? 0 : 1};
                    double e = run_case(d, prec, l[0], l[1], expr, &c0);
                    double e1 = run_case(d, prec, l[0], l[1], expr, &c1);
                    double e2 = run_case(d, prec, l[0], l[1], expr, &c2);
                    double e3 = run_case(d, prec, l[0], l[1], expr, &c3);
                    if (e != e1 || e != e2 || e != e3) { printf("launch settings differ: "); fails++; }
                    if (e > (prec == 0 ? 1e-13 : 1e-5) || argc > 1)
                        printf("dims %dx%dx%dx%d prec %d layout %d/%d expr %d err %.3e\n", d[0], d[1], d[2], d[3], prec, l[0], l[1], expr, e);
                }
    // persistent + remap settings
    su3_launch c = {64, 1, 3, 1, 0, 4096, 3, 1};
    int d16[4] = {16, 16, 16, 16};
    for (int prec = 0; prec < 4; ++prec) {
        double e = run_case(d16, prec, 1, 0, 0, &c);
        printf("persistent prec %d err %.3e\n", prec, e);
    }
    // LDS staged (threaded emulation for barriers)
    emu_threaded = true;
    su3_launch lds = {64, 0, 3, 0, 1, 4096, 0, 0};
    int dl[4] = {3, 5, 7, 11};
    for (int prec = 0; prec < 4; ++prec)
        for (int expr = 0; expr < 5; ++expr) {
            if (prec == 3 && expr > 1) continue;
            double e = run_case(dl, prec, 0, 0, expr, &lds);
            printf("lds prec %d expr %d err %.3e\n", prec, expr, e);
        }
    emu_threaded = false;
    // batch: mixed items, compare each replay with unbatched results
    {
        struct It { int d[4]; int prec, lay, lanes, expr; };
        It items[] = {{{2, 3, 5, 7}, 0, 1, 0, 0}, {{8, 8, 8, 8}, 3, 1, 0, 0}, {{4, 4, 4, 9}, 0, 2, 16, 0},
                      {{1, 1, 1, 1}, 3, 2, 8, 0}, {{3, 5, 7, 11}, 1, 1, 0, 2}, {{5, 5, 5, 5}, 2, 2, 32, 0},
                      {{5, 5, 5, 7}, 2, 1, 0, 4}, {{4, 5, 6, 7}, 3, 1, 0, 1}, {{4, 4, 4, 4}, 0, 2, 64, 3}};
        for (int mode = 0; mode < 2; ++mode)
        for (int T : {64, 256, 4096}) {
            int n = mode == 0 ? 4 : 9;
            std::vector<su3_field *> zs(n), ref(n);
            std::vector<const su3_field *> ops(4 * n, nullptr);
            std::vector<su3_expr> ex(n);
            int64_t total = 0;
            for (int i = 0; i < n; ++i) {
                It &it = items[i];
                int64_t V = (int64_t)it.d[0] * it.d[1] * it.d[2] * it.d[3];
                total += V;
                int no = nops_of(it.expr);
                su3_field_alloc(&zs[i], it.d, (su3_precision)it.prec, (su3_layout)it.lay, it.lanes);
                su3_field_alloc(&ref[i], it.d, (su3_precision)it.prec, (su3_layout)it.lay, it.lanes);
                for (int k = 0; k < no; ++k) {
                    su3_field *f;
                    su3_field_alloc(&f, it.d, (su3_precision)it.prec, (su3_layout)it.lay, it.lanes);
                    std::vector<double> h(18 * V);
                    su3gen_field(7, 1000 + 4 * i + k, 0, V, h.data());
                    su3_field_upload(f, h.data(), nullptr);
                    ops[4 * i + k] = f;
                }
                ex[i] = (su3_expr)it.expr;
                if (su3_fused_eval(ref[i], ex[i], &ops[4 * i], no, nullptr) != SU3_OK) { printf("ref eval %s\n", su3_last_error()); fails++; }
            }
            int td[4] = {(int)total, 1, 1, 1};
            su3_launch c = {256, (T == 256 ? 2 : 0), 3, 0, 0, T, 3, (T == 64 ? 1 : 0)};
            su3_launch_set((su3_expr)(SU3_EXPR_BATCH + ex[0]), (su3_precision)items[0].prec, (su3_layout)items[0].lay, items[0].lanes, td, &c);
            su3_batch *b;
            if (T == 4096) {
                su3_launch best;
                if (su3_batch_autotune(ex.data(), zs.data(), ops.data(), n, nullptr, &best) != SU3_OK) { printf("batch autotune %s\n", su3_last_error()); fails++; }
                else printf("batch autotune picked tile %d pers %d\n", best.tile_sites, best.persistent);
                su3_launch_set((su3_expr)(SU3_EXPR_BATCH + ex[0]), (su3_precision)items[0].prec, (su3_layout)items[0].lay, items[0].lanes, td, &c);
            }
            if (su3_batch_create(&b, ex.data(), zs.data(), ops.data(), n, nullptr) != SU3_OK) { printf("batch %s\n", su3_last_error()); fails++; continue; }
            su3_launch_reset();
            int64_t nt;
            su3_batch_tiles(b, nullptr, 0, &nt);
            {
                std::vector<int32_t> rows(4 * nt);
                su3_batch_tiles(b, rows.data(), nt, &nt);
                int64_t t = 0; int bad = 0;
                for (int i = 0; i < n; ++i) {
                    int64_t V = (int64_t)items[i].d[0] * items[i].d[1] * items[i].d[2] * items[i].d[3];
                    for (int64_t f = 0; f < V; f += T, ++t)
                        if (rows[4 * t] != i || rows[4 * t + 1] != f || rows[4 * t + 2] != std::min<int64_t>(T, V - f) || rows[4 * t + 3] != items[i].prec) bad++;
                }
                if (bad || t != nt) { printf("tile rows bad %d\n", bad); fails++; }
            }
            // persistent grids share each drawn tile through LDS behind
            // barriers: run the replays with one thread per lane
            emu_threaded = true;
            for (int rep = 0; rep < 2; ++rep) {
                su3_batch_launch(b, nullptr);
                int bad = 0;
                for (int i = 0; i < n; ++i) {
                    void *p1, *p2; size_t n1, n2;
                    su3_field_data(zs[i], &p1, &n1);
                    su3_field_data(ref[i], &p2, &n2);
                    if (memcmp(p1, p2, n1) != 0) bad++;
                }
                printf("batch mode %d T %d tiles %lld rep %d mismatching items %d\n", mode, T, (long long)nt, rep, bad);
                fails += bad;
            }
            emu_threaded = false;
            // the allocation-free form on the same items (the whole batch,
            // then its first items only), into zeroed outputs
            for (int m : {n, (n + 1) / 2}) {
                su3_launch_set((su3_expr)(SU3_EXPR_BATCH + ex[0]), (su3_precision)items[0].prec, (su3_layout)items[0].lay, items[0].lanes, td, &c);
                for (int i = 0; i < m; ++i) { void *p; size_t nb; su3_field_data(zs[i], &p, &nb); memset(p, 0, nb); }
                emu_threaded = true;
                if (su3_batch_run(ex.data(), zs.data(), ops.data(), m, nullptr) != SU3_OK) { printf("batch run %s\n", su3_last_error()); fails++; }
                emu_threaded = false;
                su3_launch_reset();
                int bad = 0;
                for (int i = 0; i < m; ++i) {
                    void *p1, *p2; size_t n1, n2;
                    su3_field_data(zs[i], &p1, &n1);
                    su3_field_data(ref[i], &p2, &n2);
                    if (memcmp(p1, p2, n1) != 0) bad++;
                }
                printf("batch run mode %d T %d items %d mismatching %d\n", mode, T, m, bad);
                fails += bad;
            }
            su3_batch_destroy(b);
            for (auto *f : zs) su3_field_free(f);
            for (auto *f : ref) su3_field_free(f);
            for (auto *f : ops) su3_field_free((su3_field *)f);
        }
    }
    // shifted operands
    {
        int sd[][4] = {{3, 5, 7, 11}, {4, 4, 4, 4}, {1, 2, 1, 3}};
        for (auto &d : sd)
            for (int prec = 0; prec < 4; ++prec)
                for (auto &l : lays)
                    for (int mu = 0; mu < 4; ++mu)
                        for (int sh : {1, -1, 2, 13}) {
                            int64_t V = (int64_t)d[0] * d[1] * d[2] * d[3];
                            std::vector<double> hx(18 * V), hy(18 * V), qx(18 * V), qy(18 * V), sy(18 * V), want(18 * V), got(18 * V);
                            su3gen_field(5, 1, 0, V, hx.data()); su3gen_field(5, 2, 0, V, hy.data());
                            oracle_roundtrip(prec, hx.data(), qx.data(), V); oracle_roundtrip(prec, hy.data(), qy.data(), V);
                            oracle_cshift(qy.data(), sy.data(), d, mu, sh);
                            su3_field *fx, *fy, *fz;
                            su3_field_alloc(&fx, d, (su3_precision)prec, (su3_layout)l[0], l[1]);
                            su3_field_alloc(&fy, d, (su3_precision)prec, (su3_layout)l[0], l[1]);
                            su3_field_alloc(&fz, d, (su3_precision)prec, (su3_layout)l[0], l[1]);
                            su3_field_upload(fx, hx.data(), nullptr); su3_field_upload(fy, hy.data(), nullptr);
                            if (su3_cshift(fz, fy, mu, sh, nullptr) != SU3_OK) { printf("cshift %s\n", su3_last_error()); fails++; }
                            su3_field_download(fz, got.data(), nullptr);
                            if (memcmp(got.data(), sy.data(), 8 * 18 * V) != 0) { printf("cshift mismatch prec %d lay %d mu %d sh %d\n", prec, l[0], mu, sh); fails++; }
                            su3_launch cs = {64, 0, 3, 0, 0, 4096, 4, (mu + sh) & 1};
                            su3_launch_set(SU3_EXPR_MUL_SHIFTED, (su3_precision)prec, (su3_layout)l[0], l[1], d, &cs);
                            if (su3_mult_shifted(fz, fx, fy, mu, sh, nullptr) != SU3_OK) { printf("mult_shifted %s\n", su3_last_error()); fails++; }
                            su3_launch_reset();
                            su3_field_download(fz, got.data(), nullptr);
                            oracle_mult(qx.data(), sy.data(), want.data(), V);
                            double err = 0; int rows = prec == 3 ? 2 : 3;
                            for (int64_t s = 0; s < V; ++s) for (int t = 0; t < rows * 6; ++t) err = std::max(err, std::fabs(got[18 * s + t] - want[18 * s + t]));
                            if (err > (prec == 0 ? 1e-14 : (prec == 2 ? 2e-3 : 2e-6))) { printf("mult_shifted err %.3e prec %d lay %d mu %d sh %d\n", err, prec, l[0], mu, sh); fails++; }
                            su3_field_free(fx); su3_field_free(fy); su3_field_free(fz);
                        }
        printf("shift cases done\n");
    }
    // Wilson hopping term
    {
        int dd[][4] = {{3, 5, 7, 11}, {1, 2, 1, 3}, {4, 4, 4, 4}, {2, 6, 3, 4}};
        int pairs[][2] = {{0, 0}, {1, 1}, {1, 3}};  // (spinor, links)
        for (auto &d : dd)
            for (auto &pr : pairs)
                for (auto &l : lays) {
                    const int sp = pr[0], lp = pr[1];
                    // the LDS-tiled walks (threads per lane, slow) on every
                    // layout of the first two lattices, SoA on the others
                    const bool lds_too = &d - dd < 2 || (l[0] == 1);
                    int64_t V = (int64_t)d[0] * d[1] * d[2] * d[3];
                    std::vector<double> hu[4], qu[4], hin(24 * V), qin(24 * V), want(24 * V), got(24 * V), got1(24 * V);
                    const double *up[4];
                    su3_field *fu[4], *fin, *fout;
                    for (int mu = 0; mu < 4; ++mu) {
                        hu[mu].resize(18 * V);
                        qu[mu].resize(18 * V);
                        su3gen_field(9, 2 + mu, 0, V, hu[mu].data());
                        oracle_roundtrip(lp, hu[mu].data(), qu[mu].data(), V);
                        up[mu] = qu[mu].data();
                        su3_field_alloc(&fu[mu], d, (su3_precision)lp, (su3_layout)l[0], l[1]);
                        su3_field_upload(fu[mu], hu[mu].data(), nullptr);
                    }
                    su3gen_spinor(9, 200, 0, V, hin.data());
                    for (int64_t i = 0; i < 24 * V; ++i)
                        qin[i] = sp == 0 ? hin[i] : (double)(float)hin[i];
                    oracle_dslash(up, qin.data(), want.data(), d);
                    su3_spinor_alloc(&fin, d, (su3_precision)sp, (su3_layout)l[0], l[1]);
                    su3_spinor_alloc(&fout, d, (su3_precision)sp, (su3_layout)l[0], l[1]);
                    su3_field_upload(fin, hin.data(), nullptr);
                    // one site per lane; walks of 3 t-slices; one walk over all of t;
                    // walks of 4 and 2 (ragged last walks)
                    // site tiles 8x4x2x2, 4x4x4x1, 8x2x2x8 (ragged against these lattices)
                    // LDS-tiled walks of 3 and of all of t, blocks 128 and 256
                    // (run with one thread per lane: they synchronise); the
                    // other tiles (one buffer: 8x8, 8x4, 16x8, 16x4, blocks up to
                    // 512, walks of 2, 3, 5 and all of t); whole x rows
                    // (x hops and their wrap from LDS), one or two buffers;
                    // persistent walks over (tile, slice) spans; XCD slabs;
                    // rows of 3 x 3 (ragged here), one and two buffers; the same
                    // rows with a halo of projected face sites
                    su3_launch cs[41] = {{64, 0, 0, 0, 0, 1, 0, 0}, {256, 0, 3, 1, 0, 3, 4, 0},
                                         {128, 0, 2, 0, 0, 4096, 0, 0}, {128, 0, 2, 1, 0, 4, 0, 0},
                                         {64, 0, 2, 0, 0, 2, 0, 0}, {128, 0, 2, 1, 0, 1, 0, 1},
                                         {64, 0, 2, 0, 0, 1, 0, 2}, {256, 0, 2, 1, 0, 1, 0, 3},
                                         {128, 0, 2, 0, 0, 3, 0, 4}, {256, 0, 2, 1, 0, 4096, 0, 4},
                                         {128, 0, 3, 1, 0, 1, 0, 4},
                                         {128, 0, 3, 0, 0, 3, 0, 5}, {256, 0, 2, 1, 0, 4096, 0, 5},
                                         {512, 0, 2, 0, 0, 2, 0, 5}, {128, 0, 2, 1, 0, 5, 0, 6},
                                         {256, 0, 3, 0, 0, 4096, 0, 6}, {256, 0, 2, 0, 0, 3, 0, 7},
                                         {512, 0, 3, 1, 0, 4096, 0, 7}, {256, 0, 2, 1, 0, 3, 0, 8},
                                         {512, 0, 2, 0, 0, 4096, 0, 8}, {64, 0, 2, 0, 0, 3, 0, 9},
                                         {256, 0, 3, 1, 0, 4096, 0, 10}, {128, 0, 2, 0, 0, 2, 0, 11},
                                         {256, 0, 2, 1, 0, 5, 0, 12}, {64, 0, 2, 1, 0, 3, 0, 13},
                                         {256, 0, 2, 0, 0, 4096, 0, 16}, {256, 1, 2, 0, 0, 1, 0, 8},
                                         {256, 2, 2, 1, 0, 1, 0, 11}, {256, 3, 2, 0, 0, 1, 0, 16},
                                         {256, 0, 2, 2, 0, 3, 0, 11}, {128, 0, 2, 2, 0, 4096, 0, 4},
                                         {256, 0, 2, 0, 0, 3, 0, 17}, {256, 0, 2, 1, 0, 5, 0, 18},
                                         {256, 2, 2, 0, 0, 1, 0, 18},
                                         {64, 0, 2, 0, 0, 3, 0, 19}, {256, 0, 2, 1, 0, 4096, 0, 22},
                                         {256, 2, 2, 0, 0, 1, 0, 26}, {256, 0, 2, 0, 0, 5, 0, 27},
                                         {256, 0, 2, 2, 0, 3, 0, 28}, {128, 0, 2, 0, 0, 2, 0, 23},
                                         {256, 1, 2, 0, 0, 1, 0, 20}};
                    for (int k = 0; k < 41; ++k) {
                        if (cs[k].schedule >= 4 && !lds_too)
                            continue;
                        su3_launch_set(SU3_EXPR_DSLASH, (su3_precision)lp, (su3_layout)l[0], l[1], d, &cs[k]);
                        emu_threaded = cs[k].schedule >= 4;
                        if (su3_dslash(fout, fu, fin, nullptr) != SU3_OK) { printf("dslash %s\n", su3_last_error()); fails++; }
                        emu_threaded = false;
                        su3_field_download(fout, k ? got1.data() : got.data(), nullptr);
                        if (k && memcmp(got.data(), got1.data(), 8 * 24 * V) != 0) { printf("dslash launch settings differ (%d)\n", k); fails++; }
                    }
                    su3_launch_reset();
                    double err = 0;
                    for (int64_t i = 0; i < 24 * V; ++i) err = std::max(err, std::fabs(got[i] - want[i]));
                    if (err > (sp == 0 ? 1e-13 : 2e-5)) { printf("dslash err %.3e sp %d lp %d lay %d/%d dims %dx%dx%dx%d\n", err, sp, lp, l[0], l[1], d[0], d[1], d[2], d[3]); fails++; }
                    su3_field_free(fin); su3_field_free(fout);
                    for (int mu = 0; mu < 4; ++mu) su3_field_free(fu[mu]);
                }
        // validation
        int d[4] = {2, 3, 2, 3};
        su3_field *u64[4], *u16, *s64a, *s64b, *s32, *m64;
        for (int mu = 0; mu < 4; ++mu) su3_field_alloc(&u64[mu], d, SU3_F64, SU3_LAYOUT_SOA, 0);
        su3_field_alloc(&u16, d, SU3_F16_F32ACC, SU3_LAYOUT_SOA, 0);
        su3_field_alloc(&m64, d, SU3_F64, SU3_LAYOUT_SOA, 0);
        su3_spinor_alloc(&s64a, d, SU3_F64, SU3_LAYOUT_SOA, 0);
        su3_spinor_alloc(&s64b, d, SU3_F64, SU3_LAYOUT_SOA, 0);
        su3_spinor_alloc(&s32, d, SU3_F32, SU3_LAYOUT_SOA, 0);
        su3_field *bad16[4] = {u16, u16, u16, u16};
        su3_field *mixed[4] = {u64[0], u64[1], u16, u64[3]};
        const su3_field *mops[2] = {s64a, s64b};
        struct { su3_status got, want; const char *what; } v[] = {
            {su3_dslash(s64a, u64, s64a, nullptr), SU3_ERR_ALIAS, "in place"},
            {su3_dslash(s64a, u64, s32, nullptr), SU3_ERR_MISMATCH, "spinor precisions"},
            {su3_dslash(s32, u64, s32, nullptr), SU3_ERR_UNSUPPORTED, "f32 spinors with f64 links"},
            {su3_dslash(s64a, mixed, s64b, nullptr), SU3_ERR_MISMATCH, "mixed links"},
            {su3_dslash(s64a, u64, m64, nullptr), SU3_ERR_MISMATCH, "matrix as spinor"},
            {su3_dslash(s64a, bad16, s64b, nullptr), SU3_ERR_UNSUPPORTED, "f16 links"},
            {su3_dslash(s64a, nullptr, s64b, nullptr), SU3_ERR_INVALID_ARG, "null links"},
            {su3_fused_eval(m64, SU3_EXPR_MUL, mops, 2, nullptr), SU3_ERR_MISMATCH, "spinors in mult"},
            {su3_cshift(s64a, s64b, 0, 1, nullptr), SU3_ERR_MISMATCH, "spinor cshift"},
            {su3_dslash(s64a, u64, s64b, nullptr), SU3_OK, "valid"},
        };
        for (auto &x : v)
            if (x.got != x.want) { printf("dslash validation %s: got %d want %d\n", x.what, x.got, x.want); fails++; }
        // default launches (whole x rows) on lattices too long in x for
        // them: the fallbacks (rows with one buffer, Lx x 2 x 2, 16 x 4 x 4)
        // agree with the oracle
        {
            int fd[][5] = {{130, 1, 2, 2, 0}, {100, 2, 3, 2, 0}, {300, 1, 1, 2, 1}, {64, 4, 4, 2, 1}};
            for (auto &q : fd) {
                int dl[4] = {q[0], q[1], q[2], q[3]};
                const int sp = q[4], lp = q[4];
                int64_t V = (int64_t)dl[0] * dl[1] * dl[2] * dl[3];
                std::vector<double> hu[4], qu[4], hin(24 * V), qin(24 * V), want(24 * V), got(24 * V);
                const double *up[4];
                su3_field *fu[4], *fin, *fout;
                for (int mu = 0; mu < 4; ++mu) {
                    hu[mu].resize(18 * V);
                    qu[mu].resize(18 * V);
                    su3gen_field(9, 2 + mu, 0, V, hu[mu].data());
                    oracle_roundtrip(lp, hu[mu].data(), qu[mu].data(), V);
                    up[mu] = qu[mu].data();
                    su3_field_alloc(&fu[mu], dl, (su3_precision)lp, SU3_LAYOUT_SOA, 0);
                    su3_field_upload(fu[mu], hu[mu].data(), nullptr);
                }
                su3gen_spinor(9, 200, 0, V, hin.data());
                for (int64_t i = 0; i < 24 * V; ++i)
                    qin[i] = sp == 0 ? hin[i] : (double)(float)hin[i];
                oracle_dslash(up, qin.data(), want.data(), dl);
                su3_spinor_alloc(&fin, dl, (su3_precision)sp, SU3_LAYOUT_SOA, 0);
                su3_spinor_alloc(&fout, dl, (su3_precision)sp, SU3_LAYOUT_SOA, 0);
                su3_field_upload(fin, hin.data(), nullptr);
                su3_launch_reset();
                emu_threaded = true;
                if (su3_dslash(fout, fu, fin, nullptr) != SU3_OK) { printf("fallback dslash %s\n", su3_last_error()); fails++; }
                emu_threaded = false;
                su3_field_download(fout, got.data(), nullptr);
                double err = 0;
                for (int64_t i = 0; i < 24 * V; ++i) err = std::max(err, std::fabs(got[i] - want[i]));
                if (err > (sp == 0 ? 1e-13 : 2e-5)) { printf("fallback dslash err %.3e dims %dx%dx%dx%d\n", err, dl[0], dl[1], dl[2], dl[3]); fails++; }
                su3_field_free(fin); su3_field_free(fout);
                for (int mu = 0; mu < 4; ++mu) su3_field_free(fu[mu]);
            }
        }
        // every LDS-tiled launch the table accepts runs, in both spinor
        // precisions (a tile too large for doubles falls back)
        {
            su3_field *u32[4], *s32b;
            for (int mu = 0; mu < 4; ++mu) su3_field_alloc(&u32[mu], d, SU3_F32, SU3_LAYOUT_SOA, 0);
            su3_spinor_alloc(&s32b, d, SU3_F32, SU3_LAYOUT_SOA, 0);
            for (int sched = 4; sched <= 29; ++sched)
                for (int b : {64, 128, 256, 512, 1024})
                    for (int lp : {0, 1}) {
                        su3_launch c = {b, 0, 2, 0, 0, 2, 0, sched};
                        if (su3_launch_set(SU3_EXPR_DSLASH, (su3_precision)lp, SU3_LAYOUT_SOA, 0, d, &c) != SU3_OK)
                            continue;
                        emu_threaded = true;
                        su3_status st = lp == 0 ? su3_dslash(s64a, u64, s64b, nullptr)
                                                : su3_dslash(s32, u32, s32b, nullptr);
                        emu_threaded = false;
                        if (st != SU3_OK) { printf("lds launch sched %d block %d prec %d: %s\n", sched, b, lp, su3_last_error()); fails++; }
                    }
            su3_launch_reset();
            for (int mu = 0; mu < 4; ++mu) su3_field_free(u32[mu]);
            su3_field_free(s32b);
        }
        su3_field *links_c12[4];
        for (int mu = 0; mu < 4; ++mu) su3_field_alloc(&links_c12[mu], d, SU3_C12_F32, SU3_LAYOUT_SOA, 0);
        if (su3_dslash(s64a, links_c12, s64b, nullptr) != SU3_ERR_UNSUPPORTED) { printf("f64 spinor with c12 links accepted\n"); fails++; }
        for (int mu = 0; mu < 4; ++mu) { su3_field_free(u64[mu]); su3_field_free(links_c12[mu]); }
        su3_field_free(u16); su3_field_free(m64); su3_field_free(s64a); su3_field_free(s64b); su3_field_free(s32);
        printf("dslash cases done\n");
    }
    // virtual-node layout
    {
        struct Vn { int d[4]; int simd[4]; };
        Vn cases[] = {{{4, 2, 6, 4}, {2, 1, 2, 2}}, {{3, 5, 7, 2}, {1, 1, 1, 2}}, {{2, 4, 4, 8}, {1, 1, 2, 4}},
                      {{4, 4, 4, 4}, {2, 2, 2, 2}}, {{8, 3, 2, 2}, {8, 1, 1, 1}}, {{2, 2, 2, 2}, {1, 1, 1, 1}},
                      {{4, 4, 8, 8}, {2, 2, 4, 2}}};
        for (auto &c : cases) {
            const int *d = c.d;
            int64_t V = (int64_t)d[0] * d[1] * d[2] * d[3];
            for (int prec = 0; prec < 4; ++prec) {
                std::vector<double> hx(18 * V), hy(18 * V), qx(18 * V), qy(18 * V), want(18 * V), got(18 * V), sy(18 * V);
                su3gen_field(11, 1, 0, V, hx.data()); su3gen_field(11, 2, 0, V, hy.data());
                oracle_roundtrip(prec, hx.data(), qx.data(), V); oracle_roundtrip(prec, hy.data(), qy.data(), V);
                su3_field *fx, *fy, *fz;
                if (su3_vnode_alloc(&fx, d, (su3_precision)prec, SU3_KIND_MATRIX, c.simd) != SU3_OK) { printf("vnode alloc %s\n", su3_last_error()); fails++; continue; }
                su3_vnode_alloc(&fy, d, (su3_precision)prec, SU3_KIND_MATRIX, c.simd);
                su3_vnode_alloc(&fz, d, (su3_precision)prec, SU3_KIND_MATRIX, c.simd);
                su3_field_upload(fx, hx.data(), nullptr); su3_field_upload(fy, hy.data(), nullptr);
                // stored image
                {
                    void *p; size_t n;
                    su3_field_data(fx, &p, &n);
                    std::vector<unsigned char> img(n);
                    oracle_vnode_pack(hx.data(), d, c.simd, prec, prec == 3 ? 6 : 9, 9, img.data());
                    if (memcmp(p, img.data(), n) != 0) { printf("vnode image differs prec %d\n", prec); fails++; }
                }
                for (int expr = 0; expr < (prec == 3 ? 2 : 5); ++expr) {
                    int n = nops_of(expr);
                    const su3_field *ops[4] = {fx, fy, fx, fy};
                    const double *qo[4] = {qx.data(), qy.data(), qx.data(), qy.data()};
                    oracle_fused(expr, qo[0], qo[1], n > 2 ? qo[2] : nullptr, n > 3 ? qo[3] : nullptr, want.data(), V);
                    if (su3_fused_eval(fz, (su3_expr)expr, ops, n, nullptr) != SU3_OK) { printf("vnode eval %s\n", su3_last_error()); fails++; }
                    su3_field_download(fz, got.data(), nullptr);
                    double err = 0; int rows = prec == 3 ? 2 : 3;
                    for (int64_t s = 0; s < V; ++s) for (int t = 0; t < rows * 6; ++t) err = std::max(err, std::fabs(got[18 * s + t] - want[18 * s + t]));
                    if (err > (prec == 0 ? 1e-13 : (prec == 2 ? 5e-3 : 1e-5))) { printf("vnode expr %d prec %d err %.3e\n", expr, prec, err); fails++; }
                }
                for (int mu = 0; mu < 4; ++mu)
                    for (int sh : {1, -1, 3, -5}) {
                        oracle_cshift(qy.data(), sy.data(), d, mu, sh);
                        if (su3_cshift(fz, fy, mu, sh, nullptr) != SU3_OK) { printf("vnode cshift %s\n", su3_last_error()); fails++; }
                        su3_field_download(fz, got.data(), nullptr);
                        if (memcmp(got.data(), sy.data(), 8 * 18 * V) != 0) { printf("vnode cshift mismatch prec %d mu %d sh %d simd %d%d%d%d\n", prec, mu, sh, c.simd[0], c.simd[1], c.simd[2], c.simd[3]); fails++; }
                        if (su3_mult_shifted(fz, fx, fy, mu, sh, nullptr) != SU3_OK) { printf("vnode mult_shifted %s\n", su3_last_error()); fails++; }
                        su3_field_download(fz, got.data(), nullptr);
                        oracle_mult(qx.data(), sy.data(), want.data(), V);
                        double err = 0; int rows = prec == 3 ? 2 : 3;
                        for (int64_t s = 0; s < V; ++s) for (int t = 0; t < rows * 6; ++t) err = std::max(err, std::fabs(got[18 * s + t] - want[18 * s + t]));
                        if (err > (prec == 0 ? 1e-14 : (prec == 2 ? 2e-3 : 2e-6))) { printf("vnode mult_shifted err %.3e\n", err); fails++; }
                    }
                su3_field_free(fx); su3_field_free(fy); su3_field_free(fz);
            }
            // Dslash
            int pairs[][2] = {{0, 0}, {1, 1}, {1, 3}};
            for (auto &pr : pairs) {
                const int sp = pr[0], lp = pr[1];
                std::vector<double> hu[4], qu[4], hin(24 * V), qin(24 * V), want(24 * V), got(24 * V);
                const double *up[4];
                su3_field *fu[4], *fin, *fout;
                for (int mu = 0; mu < 4; ++mu) {
                    hu[mu].resize(18 * V); qu[mu].resize(18 * V);
                    su3gen_field(12, 2 + mu, 0, V, hu[mu].data());
                    oracle_roundtrip(lp, hu[mu].data(), qu[mu].data(), V);
                    up[mu] = qu[mu].data();
                    su3_vnode_alloc(&fu[mu], d, (su3_precision)lp, SU3_KIND_MATRIX, c.simd);
                    su3_field_upload(fu[mu], hu[mu].data(), nullptr);
                }
                su3gen_spinor(12, 200, 0, V, hin.data());
                for (int64_t i = 0; i < 24 * V; ++i) qin[i] = sp == 0 ? hin[i] : (double)(float)hin[i];
                oracle_dslash(up, qin.data(), want.data(), d);
                su3_vnode_alloc(&fin, d, (su3_precision)sp, SU3_KIND_SPINOR, c.simd);
                su3_vnode_alloc(&fout, d, (su3_precision)sp, SU3_KIND_SPINOR, c.simd);
                su3_field_upload(fin, hin.data(), nullptr);
                {
                    void *p; size_t n;
                    su3_field_data(fin, &p, &n);
                    std::vector<unsigned char> img(n);
                    oracle_vnode_pack(hin.data(), d, c.simd, sp, 12, 12, img.data());
                    if (memcmp(p, img.data(), n) != 0) { printf("vnode spinor image differs\n"); fails++; }
                }
                // one site per lane, then row tiles of outer sites with all
                // their virtual nodes (one and two buffers, walks, persistent
                // shares, XCD slabs, rows of 3 x 3), then the default launch
                const int nsub = c.simd[0] * c.simd[1] * c.simd[2] * c.simd[3];
                su3_launch vcs[9] = {{64, 0, 2, 0, 0, 1, 0, 0}, {256, 0, 2, 0, 0, 2, 0, 9},
                                     {256, 0, 2, 1, 0, 4096, 0, 12}, {256, 0, 2, 0, 0, 3, 0, 13},
                                     {256, 2, 2, 0, 0, 1, 0, 16}, {256, 0, 2, 2, 0, 1, 0, 11},
                                     {256, 0, 2, 0, 0, 3, 0, 17}, {256, 1, 2, 1, 0, 1, 0, 18},
                                     {0, 0, 0, 0, 0, 0, 0, 0}};
                std::vector<double> got0(24 * V);
                for (int k = 0; k < 9; ++k) {
                    if (k < 8)
                        su3_launch_set(SU3_EXPR_DSLASH, (su3_precision)lp, SU3_LAYOUT_VNODE, nsub, d, &vcs[k]);
                    else
                        su3_launch_reset();
                    emu_threaded = k > 0;
                    if (su3_dslash(fout, fu, fin, nullptr) != SU3_OK) { printf("vnode dslash %s\n", su3_last_error()); fails++; }
                    emu_threaded = false;
                    su3_field_download(fout, k ? got.data() : got0.data(), nullptr);
                    if (k && memcmp(got.data(), got0.data(), 8 * 24 * V) != 0) { printf("vnode dslash launch %d differs simd %d%d%d%d\n", k, c.simd[0], c.simd[1], c.simd[2], c.simd[3]); fails++; }
                }
                su3_launch_reset();
                double err = 0;
                for (int64_t i = 0; i < 24 * V; ++i) err = std::max(err, std::fabs(got0[i] - want[i]));
                if (err > (sp == 0 ? 1e-13 : 2e-5)) { printf("vnode dslash err %.3e sp %d lp %d simd %d%d%d%d\n", err, sp, lp, c.simd[0], c.simd[1], c.simd[2], c.simd[3]); fails++; }
                su3_field_free(fin); su3_field_free(fout);
                for (int mu = 0; mu < 4; ++mu) su3_field_free(fu[mu]);
            }
        }
        // rules
        int d[4] = {4, 4, 4, 4}, s1[4] = {2, 2, 1, 1}, s2[4] = {1, 1, 2, 2}, bad[4] = {3, 1, 1, 1}, odd[4] = {1, 1, 1, 3};
        su3_field *a, *b, *z;
        su3_vnode_alloc(&a, d, SU3_F64, SU3_KIND_MATRIX, s1);
        su3_vnode_alloc(&b, d, SU3_F64, SU3_KIND_MATRIX, s2);
        su3_vnode_alloc(&z, d, SU3_F64, SU3_KIND_MATRIX, s1);
        if (su3_mult(z, a, b, nullptr) != SU3_ERR_MISMATCH) { printf("vnode simd mismatch accepted\n"); fails++; }
        if (su3_mult(z, a, a, nullptr) != SU3_OK) { printf("vnode mult %s\n", su3_last_error()); fails++; }
        su3_field *t;
        size_t nb;
        if (su3_vnode_alloc(&t, d, SU3_F64, SU3_KIND_MATRIX, bad) != SU3_ERR_INVALID_ARG) { printf("vnode non-dividing simd accepted\n"); fails++; }
        int d12[4] = {4, 4, 4, 12};
        if (su3_vnode_bytes(d12, SU3_F64, SU3_KIND_MATRIX, odd, &nb) != SU3_ERR_INVALID_ARG) { printf("vnode N_sub 3 accepted\n"); fails++; }
        if (su3_field_alloc(&t, d, SU3_F64, SU3_LAYOUT_VNODE, 4) != SU3_ERR_INVALID_ARG) { printf("vnode via field_alloc accepted\n"); fails++; }
        if (su3_vnode_bytes(d, SU3_F16_F32ACC, SU3_KIND_SPINOR, s1, &nb) != SU3_ERR_UNSUPPORTED) { printf("f16 vnode spinor accepted\n"); fails++; }
        su3_field_free(a); su3_field_free(b); su3_field_free(z);
        printf("vnode cases done\n");
    }
    // expression programs
    {
        struct Ex { const char *text; int n; int kinds[4]; };
        Ex exs[] = {{"a+b+a*b", 2, {2, 2}}, {"1.0", 0, {}}, {"a*b", 2, {0, 0}},
                    {"trace(a*adj(b)) * c + d", 4, {0, 0, 3, 3}}, {"2*i*a - b*c", 3, {0, 0, 3}},
                    {"(a*b)*(c*d) + a - d", 4, {0, 0, 0, 0}}, {"real(trace(a)) * b + c", 3, {0, 0, 2}},
                    {"adj(a)*transpose(b) - conj(a)", 2, {0, 0}}, {"a", 1, {3}},
                    {"a*a - 2*a + 1.5", 1, {0}}, {"c - a*b*c + trace(a)*c - 0.5*i - (-b)", 3, {0, 0, 3}},
                    {"trace(a) + b*adj(b)", 2, {0, 0}},
                    {"a*b + a", 2, {0, 0}}, {"a*a + a*a", 1, {0}}, {"a", 1, {0}},
                    {"adj(adj(a)) - transpose(transpose(b)) + conj(conj(a))", 2, {0, 0}},
                    {"(a*b+c*d)*(a*c+b*d) + (a-b)*(c-d)", 4, {0, 0, 0, 0}},
                    {"((a*b)*(c*d))*((a*c)*(b*d))", 4, {0, 0, 0, 0}},
                    {"-(a - b) * imag(a) + conj(b) - 0.25 * c", 3, {2, 2, 2}},
                    {"((a*b)*(c*a))*((b*c)*(a-b)) + ((a+c)*(b+c))*((a*a)*(c-b))", 3, {2, 2, 2}}};
        int dims_list[][4] = {{3, 5, 7, 11}, {4, 4, 4, 4}};
        int lays[][2] = {{0, 0}, {1, 0}, {2, 16}, {3, 0}};
        int simd[4] = {2, 1, 1, 2};
        for (auto &d : dims_list)
            for (auto &l : lays) {
                if (l[0] == 3 && d[0] % 2) continue;  // virtual nodes need even x, t
                int64_t V = (int64_t)d[0] * d[1] * d[2] * d[3];
                for (int arith : {0, 1, 3}) {  // F64; F32; F32 with compressed matrices
                    for (auto &ex : exs) {
                        std::vector<std::vector<double>> host(4), q(4);
                        std::vector<su3_field *> fs(4, nullptr);
                        const double *qp[4] = {nullptr, nullptr, nullptr, nullptr};
                        bool ok = true;
                        for (int k = 0; k < ex.n; ++k) {
                            const int kind = ex.kinds[k];
                            const int prec = kind == 0 ? arith : (arith == 0 ? 0 : 1);
                            const int64_t per = kind == 0 ? 18 : (kind == 3 ? 2 : 1);
                            host[k].resize(per * V);
                            q[k].resize(per * V);
                            if (kind == 0) {
                                su3gen_field(13, 50 + k, 0, V, host[k].data());
                                oracle_roundtrip(prec, host[k].data(), q[k].data(), V);
                            } else {
                                std::vector<double> tmp(18 * V);
                                su3gen_field(13, 60 + k, 0, V, tmp.data());
                                for (int64_t i = 0; i < per * V; ++i) {
                                    host[k][i] = tmp[i] * 3.0;
                                    q[k][i] = prec == 0 ? host[k][i] : (double)(float)host[k][i];
                                }
                            }
                            qp[k] = q[k].data();
                            su3_status st;
                            if (l[0] == 3)
                                st = su3_vnode_alloc(&fs[k], d, (su3_precision)prec, (su3_kind)kind, simd);
                            else if (kind == 0)
                                st = su3_field_alloc(&fs[k], d, (su3_precision)prec, (su3_layout)l[0], l[1]);
                            else
                                st = su3_scalar_alloc(&fs[k], d, (su3_precision)prec, (su3_layout)l[0], l[1], (su3_kind)kind);
                            if (st != SU3_OK) { printf("program operand alloc %s\n", su3_last_error()); fails++; ok = false; break; }
                            su3_field_upload(fs[k], host[k].data(), nullptr);
                        }
                        if (!ok) continue;
                        su3_program *p;
                        su3_kind kinds[4];
                        for (int k = 0; k < 4; ++k) kinds[k] = (su3_kind)ex.kinds[k];
                        if (su3_program_create(&p, ex.text, ex.n, kinds) != SU3_OK) { printf("program %s: %s\n", ex.text, su3_last_error()); fails++; continue; }
                        su3_kind rk; int32_t ni, nr;
                        su3_program_info(p, &rk, &ni, &nr);
                        const int zprec = rk == SU3_KIND_MATRIX ? (arith == 3 ? 1 : arith) : (arith == 0 ? 0 : 1);
                        su3_field *z;
                        if (l[0] == 3)
                            su3_vnode_alloc(&z, d, (su3_precision)zprec, rk, simd);
                        else if (rk == SU3_KIND_MATRIX)
                            su3_field_alloc(&z, d, (su3_precision)zprec, (su3_layout)l[0], l[1]);
                        else
                            su3_scalar_alloc(&z, d, (su3_precision)zprec, (su3_layout)l[0], l[1], rk);
                        const int64_t per = rk == SU3_KIND_MATRIX ? 18 : (rk == SU3_KIND_COMPLEX ? 2 : 1);
                        std::vector<double> want(18 * V), got(per * V);
                        int okinds[4];
                        for (int k = 0; k < 4; ++k) okinds[k] = ex.kinds[k];
                        const int ork = oracle_eval_expr(ex.text, ex.n, okinds, qp, want.data(), V);
                        if (ork != (int)rk) { printf("program %s: oracle kind %d vs %d\n", ex.text, ork, (int)rk); fails++; }
                        su3_status st = su3_program_eval(p, z, fs.data(), ex.n, nullptr);
                        // (double programs of 5-8 matrix registers run the
                        // 8-register variant, checked like the others)
                        if (st != SU3_OK) {
                            printf("program eval %s: %s\n", ex.text, su3_last_error()); fails++;
                        } else {
                            su3_field_download(z, got.data(), nullptr);
                            double err = 0, mag = 0;
                            for (int64_t i = 0; i < per * V; ++i) { err = std::max(err, std::fabs(got[i] - want[i])); mag = std::max(mag, std::fabs(want[i])); }
                            if (err > (arith == 0 ? 1e-13 : 2e-6) * (1 + mag)) { printf("program %s arith %d layout %d err %.3e\n", ex.text, arith, l[0], err); fails++; }
                        }
                        su3_field_free(z);
                        su3_program_destroy(p);
                        for (auto *f : fs) su3_field_free(f);
                    }
                }
            }
        // rules
        int d[4] = {2, 2, 2, 2};
        su3_field *m64, *m32, *r64, *c64;
        su3_field_alloc(&m64, d, SU3_F64, SU3_LAYOUT_SOA, 0);
        su3_field_alloc(&m32, d, SU3_F32, SU3_LAYOUT_SOA, 0);
        su3_scalar_alloc(&r64, d, SU3_F64, SU3_LAYOUT_SOA, 0, SU3_KIND_REAL);
        su3_scalar_alloc(&c64, d, SU3_F64, SU3_LAYOUT_SOA, 0, SU3_KIND_COMPLEX);
        su3_program *p;
        su3_kind mm[2] = {SU3_KIND_MATRIX, SU3_KIND_MATRIX};
        su3_program_create(&p, "a*b", 2, mm);
        const su3_field *mixed[2] = {m64, m32}, *wrongkind[2] = {m64, r64}, *good[2] = {m64, m64};
        if (su3_program_eval(p, m64, mixed, 2, nullptr) != SU3_ERR_MISMATCH) { printf("mixed precision accepted\n"); fails++; }
        if (su3_program_eval(p, m64, wrongkind, 2, nullptr) != SU3_ERR_MISMATCH) { printf("wrong kind accepted\n"); fails++; }
        if (su3_program_eval(p, c64, good, 2, nullptr) != SU3_ERR_MISMATCH) { printf("wrong result kind accepted\n"); fails++; }
        if (su3_program_eval(p, m64, good, 1, nullptr) != SU3_ERR_INVALID_ARG) { printf("operand count accepted\n"); fails++; }
        if (su3_program_eval(p, m64, good, 2, nullptr) != SU3_OK) { printf("in-place program: %s\n", su3_last_error()); fails++; }
        su3_program_destroy(p);
        su3_program *q;
        if (su3_program_create(&q, "a+*b", 2, mm) != SU3_ERR_INVALID_ARG) { printf("syntax error accepted\n"); fails++; }
        su3_kind sp[1] = {SU3_KIND_SPINOR};
        if (su3_program_create(&q, "a", 1, sp) != SU3_ERR_UNSUPPORTED) { printf("spinor operand accepted\n"); fails++; }
        su3_field *c12a, *c12z;
        su3_field_alloc(&c12a, d, SU3_C12_F32, SU3_LAYOUT_SOA, 0);
        su3_field_alloc(&c12z, d, SU3_C12_F32, SU3_LAYOUT_SOA, 0);
        su3_kind m1[1] = {SU3_KIND_MATRIX};
        su3_program_create(&q, "a + a", 1, m1);
        const su3_field *one[1] = {c12a};
        if (su3_program_eval(q, c12z, one, 1, nullptr) != SU3_ERR_UNSUPPORTED) { printf("non-SU(3) compressed output accepted\n"); fails++; }
        su3_program_destroy(q);
        su3_program_create(&q, "adj(a)*a", 1, m1);
        if (su3_program_eval(q, c12z, one, 1, nullptr) != SU3_OK) { printf("SU(3) compressed output refused: %s\n", su3_last_error()); fails++; }
        su3_program_destroy(q);
        su3_field_free(m64); su3_field_free(m32); su3_field_free(r64); su3_field_free(c64);
        su3_field_free(c12a); su3_field_free(c12z);
        printf("program cases done\n");
    }
    printf("fails %d\n", fails);
    return fails != 0;
}
