// C ABI of the SU(3) streaming library: validation, field handles, host
// pack/unpack, launch planning and tuning, batches.  Declarations and the
// contract of every entry point are in include/su3.h.
#include "su3.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <array>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "su3_dslash.h"
#include "su3_internal.h"
#include "su3_program.h"

using namespace su3i;

struct su3_field {
    void *ptr;
    size_t bytes;
    int32_t dims[4];
    int64_t V;
    int64_t Vpad;
    int64_t L;  // sites per lane-block (V_pad for SoA)
    int32_t prec;
    int32_t layout;
    int32_t lanes;
    int32_t E;
    int32_t rbytes;
    int32_t owns;
    int32_t device;
    int32_t kind;   // su3_kind
    int32_t canon;  // entries per site on the host (9, 12 or 1)
    int32_t ncomp;  // reals per entry (2 complex, 1 real)
    int32_t simd[4];  // virtual nodes per direction (all 1 unless VNODE)
};

enum { KIND_MATRIX = 0, KIND_SPINOR = 1, KIND_REAL = 2, KIND_COMPLEX = 3 };
static const int kSpinorEntries = 12;

struct su3_batch {
    void *d_mem;       // one allocation: the ticket counter, then the items
    unsigned long long *d_queue;  // persistent grids only, else nullptr
    BatchItem *d_items;
    int32_t nitems;
    int32_t ntiles;
    int32_t mode;
    su3_launch cfg;
    int32_t grid;
    int32_t device;
    hipGraph_t graph;
    hipGraphExec_t exec;
};

// ------------------------------------------------------------- errors

static thread_local std::string g_last_error;

static su3_status fail(su3_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

static su3_status hip_fail(hipError_t e, const char *what)
{
    return fail(SU3_ERR_HIP, "%s: %s (%d)", what, hipGetErrorString(e), (int)e);
}

#define HIP_TRY(call, what)                 \
    do {                                    \
        hipError_t e_ = (call);             \
        if (e_ != hipSuccess)               \
            return hip_fail(e_, what);      \
    } while (0)

// ------------------------------------------------------------- geometry

struct Shape {
    int64_t V, Vpad, L;
    int32_t E, ncomp, rbytes;
    size_t bytes;
};

static su3_status make_shape(const int32_t dims[4], int prec, int layout,
                             int32_t lanes, Shape *out,
                             int kind = KIND_MATRIX,
                             const int32_t *simd = nullptr)
{
    if (!dims)
        return fail(SU3_ERR_INVALID_ARG, "dims is NULL");
    if (prec < SU3_F64 || prec > SU3_C12_F32)
        return fail(SU3_ERR_INVALID_ARG, "unknown precision %d", prec);
    if (kind < KIND_MATRIX || kind > KIND_COMPLEX)
        return fail(SU3_ERR_INVALID_ARG, "unknown field kind %d", kind);
    if (kind != KIND_MATRIX && prec != SU3_F64 && prec != SU3_F32)
        return fail(SU3_ERR_UNSUPPORTED,
                    "spinor and scalar fields are stored in SU3_F64 or SU3_F32");
    if (layout < SU3_LAYOUT_AOS || layout > SU3_LAYOUT_VNODE)
        return fail(SU3_ERR_INVALID_ARG, "unknown layout %d", layout);
    if (layout == SU3_LAYOUT_VNODE && !simd)
        return fail(SU3_ERR_INVALID_ARG,
                    "virtual-node fields are made by su3_vnode_alloc / "
                    "su3_vnode_wrap");
    int64_t V = 1;
    for (int d = 0; d < 4; ++d) {
        if (dims[d] <= 0)
            return fail(SU3_ERR_INVALID_ARG, "dims[%d] = %d must be > 0", d,
                        dims[d]);
        V *= dims[d];
        if (V > ((int64_t)1 << 31))
            return fail(SU3_ERR_INVALID_ARG, "lattice too large");
    }
    Shape s;
    s.V = V;
    s.E = kind == KIND_SPINOR ? kSpinorEntries
          : kind == KIND_MATRIX ? entries_of(prec)
                                : 1;
    s.ncomp = kind == KIND_REAL ? 1 : 2;
    s.rbytes = real_bytes(prec);
    if (layout == SU3_LAYOUT_AOS) {
        s.L = 1;
        s.Vpad = V;
    } else if (layout == SU3_LAYOUT_VNODE) {
        int64_t n = 1;
        for (int d = 0; d < 4; ++d) {
            if (simd[d] < 1 || dims[d] % simd[d] != 0)
                return fail(SU3_ERR_INVALID_ARG,
                            "simd[%d] = %d must be >= 1 and divide dims[%d] = %d",
                            d, simd[d], d, dims[d]);
            n *= simd[d];
        }
        if (n > 256 || (n & (n - 1)) != 0)
            return fail(SU3_ERR_INVALID_ARG,
                        "N_sub = %lld virtual nodes must be a power of two <= 256",
                        (long long)n);
        s.L = n;
        s.Vpad = V;
    } else if (layout == SU3_LAYOUT_SOA) {
        s.Vpad = (V + 63) / 64 * 64;
        s.L = s.Vpad;
    } else {
        if (lanes != 8 && lanes != 16 && lanes != 32 && lanes != 64)
            return fail(SU3_ERR_INVALID_ARG,
                        "AoSoA lanes must be 8, 16, 32 or 64 (got %d)", lanes);
        s.L = lanes;
        s.Vpad = (V + lanes - 1) / lanes * lanes;
    }
    const int64_t reals = s.Vpad * s.E * s.ncomp;
    if (reals >= ((int64_t)1 << 31))
        return fail(SU3_ERR_INVALID_ARG,
                    "field holds %lld reals; the limit is 2^31 - 1",
                    (long long)reals);
    s.bytes = (size_t)reals * s.rbytes;
    *out = s;
    return SU3_OK;
}

// Storage site of lattice site s: s itself, or osite * N_sub + lane in the
// virtual-node layout.
static int64_t storage_site(const su3_field *f, int64_t s)
{
    if (f->layout != SU3_LAYOUT_VNODE)
        return s;
    int64_t osite = 0, lane = 0, ostride = 1, lstride = 1;
    for (int d = 0; d < 4; ++d) {
        const int64_t x = s % f->dims[d];
        s /= f->dims[d];
        const int64_t r = f->dims[d] / f->simd[d];
        osite += (x % r) * ostride;
        lane += (x / r) * lstride;
        ostride *= r;
        lstride *= f->simd[d];
    }
    return osite * f->L + lane;
}

static Geom geom_of(const su3_field *f)
{
    Geom g;
    if (f->layout == SU3_LAYOUT_AOS) {
        g.lg = 0;
        g.mask = 0;
        g.plane = 2;
        g.bstride = 2 * f->E;
    } else if (f->layout == SU3_LAYOUT_SOA) {
        g.lg = 31;
        g.mask = 0x7fffffffu;
        g.plane = (uint32_t)(2 * f->Vpad);
        g.bstride = 0;
    } else {
        uint32_t lg = 0;
        while ((1 << lg) < f->L)
            ++lg;
        g.lg = lg;
        g.mask = (uint32_t)(f->L - 1);
        g.plane = (uint32_t)(2 * f->L);
        g.bstride = (uint32_t)(2 * f->E * f->L);
    }
    return g;
}

// Stored-real index of (site s, entry e, c) -- the host twin of the
// kernels' addressing.
static inline int64_t stored_index(const su3_field *f, int64_t s, int e, int c)
{
    s = storage_site(f, s);
    return ((s / f->L) * f->E + e) * f->ncomp * f->L + (s % f->L) * f->ncomp + c;
}

// ------------------------------------------------------------ fields

static su3_status bytes_of_kind(const int32_t dims[4], int prec, int layout,
                                int32_t lanes, size_t *bytes, int kind)
{
    if (!bytes)
        return fail(SU3_ERR_INVALID_ARG, "bytes is NULL");
    Shape s;
    su3_status st = make_shape(dims, prec, layout, lanes, &s, kind);
    if (st != SU3_OK)
        return st;
    *bytes = s.bytes;
    return SU3_OK;
}

extern "C" su3_status su3_field_bytes(const int32_t dims[4],
                                      su3_precision prec, su3_layout layout,
                                      int32_t lanes, size_t *bytes)
{
    return bytes_of_kind(dims, prec, layout, lanes, bytes, KIND_MATRIX);
}

extern "C" su3_status su3_spinor_bytes(const int32_t dims[4],
                                       su3_precision prec, su3_layout layout,
                                       int32_t lanes, size_t *bytes)
{
    return bytes_of_kind(dims, prec, layout, lanes, bytes, KIND_SPINOR);
}

static su3_field *new_handle(const int32_t dims[4], int prec, int layout,
                             int32_t lanes, const Shape &s, int kind,
                             const int32_t *simd = nullptr)
{
    su3_field *f = new su3_field();
    f->ptr = nullptr;
    f->bytes = s.bytes;
    std::memcpy(f->dims, dims, sizeof f->dims);
    f->V = s.V;
    f->Vpad = s.Vpad;
    f->L = s.L;
    f->prec = prec;
    f->layout = layout;
    f->lanes = layout == SU3_LAYOUT_AOSOA ? lanes
               : layout == SU3_LAYOUT_VNODE ? (int32_t)s.L
                                            : 0;
    f->E = s.E;
    f->rbytes = s.rbytes;
    f->owns = 0;
    f->device = -1;
    f->kind = kind;
    f->canon = kind == KIND_SPINOR ? kSpinorEntries : kind == KIND_MATRIX ? 9 : 1;
    f->ncomp = s.ncomp;
    for (int d = 0; d < 4; ++d)
        f->simd[d] = simd ? simd[d] : 1;
    return f;
}

static su3_status alloc_of_kind(su3_field **out, const int32_t dims[4],
                                int prec, int layout, int32_t lanes, int kind,
                                const int32_t *simd = nullptr)
{
    if (!out)
        return fail(SU3_ERR_INVALID_ARG, "out is NULL");
    Shape s;
    su3_status st = make_shape(dims, prec, layout, lanes, &s, kind, simd);
    if (st != SU3_OK)
        return st;
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, s.bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(SU3_ERR_OUT_OF_MEMORY, "hipMalloc(%zu bytes): %s", s.bytes,
                    hipGetErrorString(e));
    }
    e = hipMemset(p, 0, s.bytes);
    if (e != hipSuccess) {
        (void)hipFree(p);
        return hip_fail(e, "hipMemset");
    }
    su3_field *f = new_handle(dims, prec, layout, lanes, s, kind, simd);
    f->ptr = p;
    f->owns = 1;
    f->device = dev;
    *out = f;
    return SU3_OK;
}

extern "C" su3_status su3_field_alloc(su3_field **out, const int32_t dims[4],
                                      su3_precision prec, su3_layout layout,
                                      int32_t lanes)
{
    return alloc_of_kind(out, dims, prec, layout, lanes, KIND_MATRIX);
}

extern "C" su3_status su3_spinor_alloc(su3_field **out, const int32_t dims[4],
                                       su3_precision prec, su3_layout layout,
                                       int32_t lanes)
{
    return alloc_of_kind(out, dims, prec, layout, lanes, KIND_SPINOR);
}

static su3_status wrap_of_kind(su3_field **out, void *dev_ptr, size_t bytes,
                               const int32_t dims[4], int prec, int layout,
                               int32_t lanes, int kind,
                               const int32_t *simd = nullptr)
{
    if (!out)
        return fail(SU3_ERR_INVALID_ARG, "out is NULL");
    if (!dev_ptr)
        return fail(SU3_ERR_INVALID_ARG, "dev_ptr is NULL");
    if (((uintptr_t)dev_ptr & 15) != 0)
        return fail(SU3_ERR_INVALID_ARG, "dev_ptr is not 16-byte aligned");
    Shape s;
    su3_status st = make_shape(dims, prec, layout, lanes, &s, kind, simd);
    if (st != SU3_OK)
        return st;
    if (bytes < s.bytes)
        return fail(SU3_ERR_INVALID_ARG,
                    "buffer of %zu bytes is smaller than the field (%zu)",
                    bytes, s.bytes);
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
    hipPointerAttribute_t attr;
    std::memset(&attr, 0, sizeof attr);
    hipError_t e = hipPointerGetAttributes(&attr, dev_ptr);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(SU3_ERR_INVALID_ARG,
                    "dev_ptr is not device memory known to HIP (%s)",
                    hipGetErrorString(e));
    }
    if (attr.type != hipMemoryTypeDevice || attr.device != dev)
        return fail(SU3_ERR_INVALID_ARG,
                    "dev_ptr is not device memory of the current device %d",
                    dev);
    su3_field *f = new_handle(dims, prec, layout, lanes, s, kind, simd);
    f->ptr = dev_ptr;
    f->owns = 0;
    f->device = dev;
    *out = f;
    return SU3_OK;
}

extern "C" su3_status su3_field_wrap(su3_field **out, void *dev_ptr,
                                     size_t bytes, const int32_t dims[4],
                                     su3_precision prec, su3_layout layout,
                                     int32_t lanes)
{
    return wrap_of_kind(out, dev_ptr, bytes, dims, prec, layout, lanes,
                        KIND_MATRIX);
}

extern "C" su3_status su3_spinor_wrap(su3_field **out, void *dev_ptr,
                                      size_t bytes, const int32_t dims[4],
                                      su3_precision prec, su3_layout layout,
                                      int32_t lanes)
{
    return wrap_of_kind(out, dev_ptr, bytes, dims, prec, layout, lanes,
                        KIND_SPINOR);
}

// ---------------------------------------------------- scalar fields

static su3_status check_scalar_kind(int kind)
{
    if (kind != KIND_REAL && kind != KIND_COMPLEX)
        return fail(SU3_ERR_INVALID_ARG,
                    "scalar fields are SU3_KIND_REAL or SU3_KIND_COMPLEX");
    return SU3_OK;
}

extern "C" su3_status su3_scalar_bytes(const int32_t dims[4],
                                       su3_precision prec, su3_layout layout,
                                       int32_t lanes, su3_kind kind,
                                       size_t *bytes)
{
    su3_status st = check_scalar_kind(kind);
    return st != SU3_OK ? st
                        : bytes_of_kind(dims, prec, layout, lanes, bytes, kind);
}

extern "C" su3_status su3_scalar_alloc(su3_field **out, const int32_t dims[4],
                                       su3_precision prec, su3_layout layout,
                                       int32_t lanes, su3_kind kind)
{
    su3_status st = check_scalar_kind(kind);
    return st != SU3_OK ? st
                        : alloc_of_kind(out, dims, prec, layout, lanes, kind);
}

extern "C" su3_status su3_scalar_wrap(su3_field **out, void *dev_ptr,
                                      size_t bytes, const int32_t dims[4],
                                      su3_precision prec, su3_layout layout,
                                      int32_t lanes, su3_kind kind)
{
    su3_status st = check_scalar_kind(kind);
    return st != SU3_OK ? st
                        : wrap_of_kind(out, dev_ptr, bytes, dims, prec, layout,
                                       lanes, kind);
}

// --------------------------------------------- virtual-node fields

static su3_status check_simd(const int32_t *simd)
{
    if (!simd)
        return fail(SU3_ERR_INVALID_ARG, "simd is NULL");
    return SU3_OK;
}

extern "C" su3_status su3_vnode_bytes(const int32_t dims[4],
                                      su3_precision prec, su3_kind kind,
                                      const int32_t simd[4], size_t *bytes)
{
    su3_status st = check_simd(simd);
    if (st != SU3_OK)
        return st;
    if (!bytes)
        return fail(SU3_ERR_INVALID_ARG, "bytes is NULL");
    Shape s;
    st = make_shape(dims, prec, SU3_LAYOUT_VNODE, 0, &s, kind, simd);
    if (st != SU3_OK)
        return st;
    *bytes = s.bytes;
    return SU3_OK;
}

extern "C" su3_status su3_vnode_alloc(su3_field **out, const int32_t dims[4],
                                      su3_precision prec, su3_kind kind,
                                      const int32_t simd[4])
{
    su3_status st = check_simd(simd);
    if (st != SU3_OK)
        return st;
    return alloc_of_kind(out, dims, prec, SU3_LAYOUT_VNODE, 0, kind, simd);
}

extern "C" su3_status su3_vnode_wrap(su3_field **out, void *dev_ptr,
                                     size_t bytes, const int32_t dims[4],
                                     su3_precision prec, su3_kind kind,
                                     const int32_t simd[4])
{
    su3_status st = check_simd(simd);
    if (st != SU3_OK)
        return st;
    return wrap_of_kind(out, dev_ptr, bytes, dims, prec, SU3_LAYOUT_VNODE, 0,
                        kind, simd);
}

extern "C" su3_status su3_field_free(su3_field *f)
{
    if (!f)
        return SU3_OK;
    hipError_t e = hipSuccess;
    if (f->owns && f->ptr)
        e = hipFree(f->ptr);
    delete f;
    if (e != hipSuccess)
        return hip_fail(e, "hipFree");
    return SU3_OK;
}

extern "C" su3_status su3_field_data(const su3_field *f, void **dev_ptr,
                                     size_t *bytes)
{
    if (!f)
        return fail(SU3_ERR_INVALID_ARG, "field is NULL");
    if (dev_ptr)
        *dev_ptr = f->ptr;
    if (bytes)
        *bytes = f->bytes;
    return SU3_OK;
}

// double -> float -> half, each step rounding to nearest even.  The empty
// asm keeps the intermediate float: without it the optimiser folds the two
// conversions into one double -> half rounding, which differs whenever the
// float lands exactly halfway between two halves.
static inline _Float16 half_of(double v)
{
    float f = (float)v;
    __asm__ volatile("" : "+x"(f));
    return (_Float16)f;
}

// Host quantisers: round to nearest even (float: one rounding; half:
// double -> float -> half).
static inline void put_real(void *img, int prec, int64_t idx, double v)
{
    if (prec == SU3_F64)
        static_cast<double *>(img)[idx] = v;
    else if (prec == SU3_F16_F32ACC)
        static_cast<_Float16 *>(img)[idx] = half_of(v);
    else
        static_cast<float *>(img)[idx] = (float)v;
}

static inline double get_real(const void *img, int prec, int64_t idx)
{
    if (prec == SU3_F64)
        return static_cast<const double *>(img)[idx];
    if (prec == SU3_F16_F32ACC)
        return (double)(float)static_cast<const _Float16 *>(img)[idx];
    return (double)static_cast<const float *>(img)[idx];
}

extern "C" su3_status su3_field_upload(su3_field *f, const double *host,
                                       void *stream)
{
    if (!f || !host)
        return fail(SU3_ERR_INVALID_ARG, "field or host buffer is NULL");
    std::vector<unsigned char> img(f->bytes, 0);
    for (int64_t s = 0; s < f->V; ++s)
        for (int e = 0; e < f->E; ++e)
            for (int c = 0; c < f->ncomp; ++c)
                put_real(img.data(), f->prec, stored_index(f, s, e, c),
                         host[f->ncomp * (f->canon * s + e) + c]);
    hipStream_t st = static_cast<hipStream_t>(stream);
    HIP_TRY(hipMemcpyAsync(f->ptr, img.data(), f->bytes,
                           hipMemcpyHostToDevice, st),
            "upload copy");
    HIP_TRY(hipStreamSynchronize(st), "upload sync");
    return SU3_OK;
}

extern "C" su3_status su3_field_download_raw(const su3_field *f, void *host,
                                             size_t bytes, void *stream)
{
    if (!f || !host)
        return fail(SU3_ERR_INVALID_ARG, "field or host buffer is NULL");
    if (bytes < f->bytes)
        return fail(SU3_ERR_INVALID_ARG, "host buffer of %zu bytes < %zu",
                    bytes, f->bytes);
    hipStream_t st = static_cast<hipStream_t>(stream);
    HIP_TRY(hipMemcpyAsync(host, f->ptr, f->bytes, hipMemcpyDeviceToHost, st),
            "download copy");
    HIP_TRY(hipStreamSynchronize(st), "download sync");
    return SU3_OK;
}

extern "C" su3_status su3_field_download(const su3_field *f, double *host,
                                         void *stream)
{
    if (!f || !host)
        return fail(SU3_ERR_INVALID_ARG, "field or host buffer is NULL");
    std::vector<unsigned char> img(f->bytes);
    su3_status st = su3_field_download_raw(f, img.data(), img.size(), stream);
    if (st != SU3_OK)
        return st;
    for (int64_t s = 0; s < f->V; ++s) {
        double *m = host + f->ncomp * f->canon * s;
        for (int e = 0; e < f->E; ++e)
            for (int c = 0; c < f->ncomp; ++c)
                m[f->ncomp * e + c] = get_real(img.data(), f->prec,
                                               stored_index(f, s, e, c));
        if (f->kind == KIND_MATRIX && f->prec == SU3_C12_F32) {
            // row 2 = conj(row0 x row1), in double
            for (int k = 0; k < 3; ++k) {
                const int p = (k + 1) % 3, q = (k + 2) % 3;
                const double ar = m[2 * p], ai = m[2 * p + 1];
                const double br = m[2 * (3 + q)], bi = m[2 * (3 + q) + 1];
                const double cr = m[2 * q], ci = m[2 * q + 1];
                const double dr = m[2 * (3 + p)], di = m[2 * (3 + p) + 1];
                m[2 * (6 + k)] = (ar * br - ai * bi) - (cr * dr - ci * di);
                m[2 * (6 + k) + 1] = -((ar * bi + ai * br) - (cr * di + ci * dr));
            }
        }
    }
    return SU3_OK;
}

// -------------------------------------------------------- device facts

struct DeviceFacts {
    int cus;
    int lds_per_cu;
    int lds_per_block;
};

static DeviceFacts device_facts(int dev)
{
    static std::mutex mu;
    static std::map<int, DeviceFacts> cache;
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(dev);
    if (it != cache.end())
        return it->second;
    DeviceFacts f;
    if (hipDeviceGetAttribute(&f.cus, hipDeviceAttributeMultiprocessorCount,
                              dev) != hipSuccess || f.cus <= 0)
        f.cus = 256;
    if (hipDeviceGetAttribute(&f.lds_per_cu,
                              hipDeviceAttributeMaxSharedMemoryPerMultiprocessor,
                              dev) != hipSuccess || f.lds_per_cu <= 0)
        f.lds_per_cu = 64 * 1024;
    if (hipDeviceGetAttribute(&f.lds_per_block,
                              hipDeviceAttributeMaxSharedMemoryPerBlock,
                              dev) != hipSuccess || f.lds_per_block <= 0)
        f.lds_per_block = 64 * 1024;
    cache[dev] = f;
    return f;
}

static int device_cus(int dev) { return device_facts(dev).cus; }

// LDS to reserve per workgroup so that at most `occupancy` workgroups fit
// on a CU (0: none).  The reserve is never read by the kernels.
static size_t occupancy_reserve(int dev, int occupancy)
{
    if (occupancy <= 0)
        return 0;
    const DeviceFacts f = device_facts(dev);
    size_t r = (size_t)f.lds_per_cu / (size_t)occupancy;
    r = std::min(r, (size_t)f.lds_per_block);
    return r / 256 * 256;
}

// ------------------------------------------------------- launch table

using Key = std::tuple<int, int, int, int, int>;  // expr prec layout lanes vbucket

static int vbucket(int64_t V)
{
    int b = 0;
    while (((int64_t)1 << b) < V)
        ++b;
    return b;
}

static std::mutex g_tune_mu;
static std::map<Key, su3_launch> g_tuned;
static bool g_cache_loaded = false;

static su3_launch default_launch(int expr, int prec, int layout)
{
    su3_launch c;
    c.block = 64;
    c.persistent = 0;
    c.nontemporal = 3;
    c.xcd_remap = 0;
    c.lds_stage = 0;
    c.tile_sites = 4096;
    c.occupancy = layout == SU3_LAYOUT_AOS ? 0 : 5;
    c.schedule = layout == SU3_LAYOUT_AOS ? 0 : 1;
    c.sites_per_lane = 0;
    if (expr == SU3_EXPR_PROGRAM || expr == SU3_EXPR_PROGRAM_SCALAR) {
        c.block = 128;
        c.occupancy = 0;
        c.schedule = 0;
    }
    if (expr == SU3_EXPR_DSLASH) {
        // the LDS-tiled walk over whole x rows (smaller tiles where the rows
        // are too long): Lx x 3 x 3 with one buffer walking 8 t-slices for
        // double spinors, Lx x 4 x 4 with two buffers walking 7 for single
        // (the fastest chunked walks at 48^4); cached loads (neighbours
        // re-read each spinor), nontemporal stores
        const bool dbl = prec == SU3_F64;
        c.block = 256;
        c.nontemporal = 2;
        c.occupancy = 0;
        c.schedule = dbl ? 17 : 16;
        c.tile_sites = dbl ? 8 : 7;
        c.xcd_remap = 0;
    }
    return c;
}

// Launch-tuning keys of batches are SU3_EXPR_BATCH + the leading item's
// expression, so that a batch's tuned tile and grid never stand in for a
// single field's launch of the same volume bucket (and the reverse).
static bool is_batch_key(int expr)
{
    return expr >= SU3_EXPR_BATCH && expr <= SU3_EXPR_BATCH + SU3_EXPR_APB_AB;
}

static bool nt_valid(int nt, bool streaming)
{
    return (nt >= 0 && nt <= 3) || (streaming && (nt == 6 || nt == 7));
}

static su3_status check_launch(const su3_launch &c, int layout, int expr)
{
    const bool lds_walk = expr == SU3_EXPR_DSLASH && c.schedule >= 4;
    const bool site = expr >= SU3_EXPR_MUL && expr <= SU3_EXPR_APB_AB;
    const bool batch = is_batch_key(expr);
    const bool streaming = site || batch || expr == SU3_EXPR_CSHIFT ||
                           expr == SU3_EXPR_MUL_SHIFTED;
    const bool wide = site && (c.nontemporal & 3) == 3 && !c.lds_stage;
    if (c.block != 64 && c.block != 128 && c.block != 256 &&
        !(lds_walk && c.block == 512) &&
        !(wide && (c.block == 512 || c.block == 1024)))
        return fail(SU3_ERR_INVALID_ARG,
                    "block %d not in {64, 128, 256}%s", c.block,
                    lds_walk ? " or 512"
                    : site   ? " (512 or 1024 need nontemporal 3 or 7)"
                             : "");
    if (!nt_valid(c.nontemporal, streaming))
        return fail(SU3_ERR_INVALID_ARG, "nontemporal %d not in %s",
                    c.nontemporal, streaming ? "{0, 1, 2, 3, 6, 7}" : "[0, 3]");
    if (c.sites_per_lane != 0 && c.sites_per_lane != 1 &&
        c.sites_per_lane != 2 && c.sites_per_lane != 4 &&
        c.sites_per_lane != 8)
        return fail(SU3_ERR_INVALID_ARG,
                    "sites_per_lane %d not in {0, 1, 2, 4, 8}",
                    c.sites_per_lane);
    if (c.persistent < 0 || c.persistent > 64)
        return fail(SU3_ERR_INVALID_ARG, "persistent %d not in [0, 64]",
                    c.persistent);
    if (c.xcd_remap < 0 || c.xcd_remap > (lds_walk ? 2 : 1))
        return fail(SU3_ERR_INVALID_ARG, "xcd_remap must be 0 or 1%s",
                    lds_walk ? " or 2" : "");
    if (c.lds_stage < 0 || c.lds_stage > 1 ||
        (c.lds_stage && layout != SU3_LAYOUT_AOS))
        return fail(SU3_ERR_INVALID_ARG, "lds_stage is for the AoS layout only");
    if (c.lds_stage && c.block > 128)
        return fail(SU3_ERR_INVALID_ARG, "lds_stage needs block <= 128");
    if (expr == SU3_EXPR_DSLASH) {
        if (c.tile_sites < 1 || c.tile_sites > 4096)
            return fail(SU3_ERR_INVALID_ARG,
                        "Dslash tile_sites (t-slices per lane) must be in "
                        "[1, 4096]");
    } else if (c.tile_sites < 64 || c.tile_sites % 64 != 0 ||
               c.tile_sites > (1 << 24)) {
        return fail(SU3_ERR_INVALID_ARG,
                    "tile_sites must be a positive multiple of 64");
    }
    if (c.occupancy < 0 || c.occupancy > 64)
        return fail(SU3_ERR_INVALID_ARG, "occupancy %d not in [0, 64]",
                    c.occupancy);
    if (expr == SU3_EXPR_DSLASH) {
        LdsShape sh;
        if (c.schedule < 0 || c.schedule > 28)
            return fail(SU3_ERR_INVALID_ARG,
                        "Dslash schedule (site tile) must be in [0, 28]");
        if (lds_walk && c.schedule <= 8 && !lds_shape(c.schedule, c.block, 8, 0, 1, sh))
            return fail(SU3_ERR_INVALID_ARG,
                        "the LDS-tiled Dslash (schedule %d) has no tile for "
                        "block %d", c.schedule, c.block);
    } else if (c.schedule < 0 || c.schedule > 1) {
        return fail(SU3_ERR_INVALID_ARG, "schedule must be 0 or 1");
    }
    return SU3_OK;
}

static void load_cache_locked();

static su3_launch lookup_launch(int expr, int prec, int layout, int lanes,
                                int64_t V)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_cache_locked();
    auto it = g_tuned.find(Key(expr, prec, layout, lanes, vbucket(V)));
    if (it != g_tuned.end())
        return it->second;
    return default_launch(expr, prec, layout);
}

// JSON cache: one object per line with integer fields.
static std::string device_tag()
{
    int dev = 0;
    hipDeviceProp_t p;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipGetDeviceProperties(&p, dev) != hipSuccess)
        return "unknown";
    char buf[300];
    snprintf(buf, sizeof buf, "%s:%d", p.gcnArchName, p.multiProcessorCount);
    return buf;
}

static bool parse_int(const std::string &line, const char *key, int *v)
{
    std::string pat = std::string("\"") + key + "\":";
    size_t pos = line.find(pat);
    if (pos == std::string::npos)
        return false;
    *v = atoi(line.c_str() + pos + pat.size());
    return true;
}

static void load_cache_locked()
{
    if (g_cache_loaded)
        return;
    g_cache_loaded = true;
    const char *path = getenv("SU3_TUNE_CACHE");
    if (!path || !*path)
        return;
    FILE *fp = fopen(path, "r");
    if (!fp)
        return;
    const std::string tag = device_tag();
    char buf[1024];
    while (fgets(buf, sizeof buf, fp)) {
        std::string line(buf);
        if (line.find("\"device\":\"" + tag + "\"") == std::string::npos)
            continue;
        int ex, pr, la, ln, vb;
        su3_launch c;
        if (!parse_int(line, "expr", &ex) || !parse_int(line, "prec", &pr) ||
            !parse_int(line, "layout", &la) || !parse_int(line, "lanes", &ln) ||
            !parse_int(line, "vbucket", &vb) ||
            !parse_int(line, "block", &c.block) ||
            !parse_int(line, "persistent", &c.persistent) ||
            !parse_int(line, "nontemporal", &c.nontemporal) ||
            !parse_int(line, "xcd_remap", &c.xcd_remap) ||
            !parse_int(line, "lds_stage", &c.lds_stage) ||
            !parse_int(line, "tile_sites", &c.tile_sites) ||
            !parse_int(line, "occupancy", &c.occupancy) ||
            !parse_int(line, "schedule", &c.schedule))
            continue;
        if (!parse_int(line, "sites_per_lane", &c.sites_per_lane))
            c.sites_per_lane = 0;
        if (check_launch(c, la, ex) != SU3_OK)
            continue;
        g_tuned[Key(ex, pr, la, ln, vb)] = c;
    }
    fclose(fp);
}

static void append_cache(const Key &k, const su3_launch &c, double us)
{
    const char *path = getenv("SU3_TUNE_CACHE");
    if (!path || !*path)
        return;
    FILE *fp = fopen(path, "a");
    if (!fp)
        return;
    fprintf(fp,
            "{\"device\":\"%s\",\"expr\":%d,\"prec\":%d,\"layout\":%d,"
            "\"lanes\":%d,\"vbucket\":%d,\"block\":%d,\"persistent\":%d,"
            "\"nontemporal\":%d,\"xcd_remap\":%d,\"lds_stage\":%d,"
            "\"tile_sites\":%d,\"occupancy\":%d,\"schedule\":%d,"
            "\"sites_per_lane\":%d,\"us\":%.3f}\n",
            device_tag().c_str(), std::get<0>(k), std::get<1>(k),
            std::get<2>(k), std::get<3>(k), std::get<4>(k), c.block,
            c.persistent, c.nontemporal, c.xcd_remap, c.lds_stage,
            c.tile_sites, c.occupancy, c.schedule, c.sites_per_lane, us);
    fclose(fp);
}

// --------------------------------------------------------- validation

static bool same_geometry(const su3_field *a, const su3_field *b)
{
    return a->layout == b->layout && a->lanes == b->lanes &&
           std::memcmp(a->dims, b->dims, sizeof a->dims) == 0 &&
           std::memcmp(a->simd, b->simd, sizeof a->simd) == 0 &&
           a->device == b->device;
}

static bool same_shape(const su3_field *a, const su3_field *b)
{
    return a->kind == b->kind && a->prec == b->prec && same_geometry(a, b);
}

static bool overlaps(const su3_field *a, const su3_field *b)
{
    const uintptr_t a0 = (uintptr_t)a->ptr, a1 = a0 + a->bytes;
    const uintptr_t b0 = (uintptr_t)b->ptr, b1 = b0 + b->bytes;
    return a0 < b1 && b0 < a1;
}

static su3_status validate_item(const su3_field *z, int expr,
                                const su3_field *const *ops, int32_t n_ops)
{
    if (!z)
        return fail(SU3_ERR_INVALID_ARG, "output field is NULL");
    if (z->kind != KIND_MATRIX)
        return fail(SU3_ERR_MISMATCH,
                    "a spinor field where an SU(3) matrix field is expected");
    if (expr < SU3_EXPR_MUL || expr > SU3_EXPR_APB_AB)
        return fail(SU3_ERR_INVALID_ARG, "unknown expression %d", expr);
    if (!ops)
        return fail(SU3_ERR_INVALID_ARG, "operand list is NULL");
    if (n_ops != operands_of(expr))
        return fail(SU3_ERR_INVALID_ARG, "expression %d takes %d operands, got %d",
                    expr, operands_of(expr), n_ops);
    for (int k = 0; k < n_ops; ++k) {
        if (!ops[k])
            return fail(SU3_ERR_INVALID_ARG, "operand %d is NULL", k);
        if (!same_shape(z, ops[k]))
            return fail(SU3_ERR_MISMATCH,
                        "operand %d differs from the output in dims, "
                        "precision, layout, lanes or device", k);
    }
    if (z->prec == SU3_C12_F32 && expr != SU3_EXPR_MUL &&
        expr != SU3_EXPR_MUL3)
        return fail(SU3_ERR_UNSUPPORTED,
                    "the two-row compressed form supports MUL and MUL3 only "
                    "(sums leave SU(3))");
    for (int k = 0; k < n_ops; ++k)
        if (overlaps(z, ops[k]) &&
            !(z->ptr == ops[k]->ptr && z->bytes == ops[k]->bytes))
            return fail(SU3_ERR_ALIAS,
                        "output partially overlaps operand %d", k);
    return SU3_OK;
}

// ------------------------------------------------------------ compute

// LDS one staged workgroup may take (operand tiles, reused for the result).
static const size_t kLdsStageMaxBytes = 65536;

static su3_status launch_item(su3_field *z, int expr,
                              const su3_field *const *ops, int32_t n_ops,
                              const su3_launch &c, hipStream_t st)
{
    SiteArgs a;
    std::memset(&a, 0, sizeof a);
    a.z = z->ptr;
    for (int k = 0; k < n_ops; ++k)
        a.op[k] = ops[k]->ptr;
    a.g = geom_of(z);
    a.nsites = (int32_t)z->V;
    a.xcd_remap = c.xcd_remap;
    hipError_t e;
    if (z->layout == SU3_LAYOUT_AOS && c.lds_stage) {
        const size_t shm = (size_t)n_ops * c.block * z->E * 2 * z->rbytes;
        if (shm > kLdsStageMaxBytes)
            return fail(SU3_ERR_UNSUPPORTED,
                        "LDS staging of %d operands x %d sites needs %zu bytes "
                        "of LDS (limit %zu)", n_ops, c.block, shm,
                        kLdsStageMaxBytes);
        const int64_t tiles = (z->V + c.block - 1) / c.block;
        int64_t grid = tiles;
        if (c.persistent)
            grid = std::min<int64_t>(grid, (int64_t)c.persistent *
                                               device_cus(z->device));
        a.ngroups = (int32_t)z->V;
        e = launch_site_lds(z->prec, expr, c.nontemporal, c.block, (int)grid,
                            a, st);
    } else {
        // S sites per lane must sit in one lane-block: the natural count
        // (or 1 where the blocks are shorter), or the launch's own count
        int S = natural_sites(z->prec, expr);
        if (c.sites_per_lane > 0) {
            S = c.sites_per_lane;
            if (!sites_compiled(z->prec, expr, S) ||
                (S > 1 && (z->layout == SU3_LAYOUT_AOS || z->L % S != 0)))
                return fail(SU3_ERR_INVALID_ARG,
                            "sites_per_lane %d is not offered for this "
                            "expression, precision and lane-block", S);
        } else if (z->layout == SU3_LAYOUT_AOS || z->L % S != 0) {
            S = 1;
        }
        a.ngroups = (int32_t)((z->V + S - 1) / S);
        int64_t grid = (a.ngroups + c.block - 1) / c.block;
        if (c.persistent)
            grid = std::min<int64_t>(grid, (int64_t)c.persistent *
                                               device_cus(z->device));
        e = launch_site(z->prec, expr, S, c.nontemporal, c.schedule, c.block,
                        (int)grid, occupancy_reserve(z->device, c.occupancy), a,
                        st);
    }
    if (e != hipSuccess)
        return hip_fail(e, "kernel launch");
    return SU3_OK;
}

extern "C" su3_status su3_fused_eval(su3_field *z, su3_expr expr,
                                     const su3_field *const *ops,
                                     int32_t n_ops, void *stream)
{
    su3_status st = validate_item(z, expr, ops, n_ops);
    if (st != SU3_OK)
        return st;
    const su3_launch c =
        lookup_launch(expr, z->prec, z->layout, z->lanes, z->V);
    return launch_item(z, expr, ops, n_ops, c,
                       static_cast<hipStream_t>(stream));
}

extern "C" su3_status su3_mult(su3_field *z, const su3_field *x,
                               const su3_field *y, void *stream)
{
    const su3_field *ops[2] = {x, y};
    return su3_fused_eval(z, SU3_EXPR_MUL, ops, 2, stream);
}

// ----------------------------------------------------- shifted operands

// Launch of the shifted-operand kernels: the tuned (or default) setting of
// the key (SU3_EXPR_CSHIFT or SU3_EXPR_MUL_SHIFTED, precision, layout,
// lanes, volume); one site per lane, one-shot grid.
static su3_status launch_shift_op(int mode, su3_field *z, const su3_field *x,
                                  const su3_field *y, int32_t mu,
                                  int32_t shift, void *stream,
                                  const su3_launch *forced = nullptr)
{
    const su3_launch c =
        forced ? *forced
               : lookup_launch(mode ? SU3_EXPR_MUL_SHIFTED : SU3_EXPR_CSHIFT,
                               z->prec, z->layout, z->lanes, z->V);
    ShiftArgs a;
    std::memset(&a, 0, sizeof a);
    a.z = z->ptr;
    a.x = x ? x->ptr : nullptr;
    a.y = y->ptr;
    a.g = geom_of(z);
    a.nsites = (int32_t)z->V;
    // outer stride (storage sites) and extent along mu; lane stride and
    // count along mu (1 lane outside the virtual-node layout)
    int64_t ostride = z->layout == SU3_LAYOUT_VNODE ? z->L : 1;
    int64_t lstride = 1;
    for (int d = 0; d < mu; ++d) {
        ostride *= z->dims[d] / z->simd[d];
        lstride *= z->simd[d];
    }
    const int64_t L = z->dims[mu];
    a.stride = (uint32_t)ostride;
    a.extent = (uint32_t)(L / z->simd[mu]);
    a.nlanes = (uint32_t)z->simd[mu];
    a.lstride = (uint32_t)lstride;
    a.lmask = z->layout == SU3_LAYOUT_VNODE ? (uint32_t)(z->L - 1) : 0u;
    a.shift = (uint32_t)(((int64_t)shift % L + L) % L);
    const int64_t grid = (z->V + c.block - 1) / c.block;
    hipError_t e = launch_shift(z->prec, mode, c.nontemporal, c.schedule,
                                c.block, (int)grid,
                                occupancy_reserve(z->device, c.occupancy), a,
                                static_cast<hipStream_t>(stream));
    if (e != hipSuccess)
        return hip_fail(e, "shift kernel launch");
    return SU3_OK;
}

extern "C" su3_status su3_cshift(su3_field *dst, const su3_field *src,
                                 int32_t mu, int32_t shift, void *stream)
{
    if (!dst || !src)
        return fail(SU3_ERR_INVALID_ARG, "field is NULL");
    if (mu < 0 || mu > 3)
        return fail(SU3_ERR_INVALID_ARG, "direction %d not in [0, 3]", mu);
    if (dst->kind != KIND_MATRIX || src->kind != KIND_MATRIX)
        return fail(SU3_ERR_MISMATCH,
                    "a spinor field where an SU(3) matrix field is expected");
    if (!same_shape(dst, src))
        return fail(SU3_ERR_MISMATCH, "dst and src differ in dims, precision, "
                                      "layout, lanes or device");
    if (overlaps(dst, src))
        return fail(SU3_ERR_ALIAS, "dst overlaps src (a shift is a gather: "
                                   "it cannot run in place)");
    return launch_shift_op(0, dst, nullptr, src, mu, shift, stream);
}

extern "C" su3_status su3_mult_shifted(su3_field *z, const su3_field *x,
                                       const su3_field *y, int32_t mu,
                                       int32_t shift, void *stream)
{
    if (!z || !x || !y)
        return fail(SU3_ERR_INVALID_ARG, "field is NULL");
    if (mu < 0 || mu > 3)
        return fail(SU3_ERR_INVALID_ARG, "direction %d not in [0, 3]", mu);
    if (z->kind != KIND_MATRIX)
        return fail(SU3_ERR_MISMATCH,
                    "a spinor field where an SU(3) matrix field is expected");
    if (!same_shape(z, x) || !same_shape(z, y))
        return fail(SU3_ERR_MISMATCH, "operands differ in dims, precision, "
                                      "layout, lanes or device");
    if (overlaps(z, y))
        return fail(SU3_ERR_ALIAS, "z overlaps the shifted operand y");
    if (overlaps(z, x) && !(z->ptr == x->ptr && z->bytes == x->bytes))
        return fail(SU3_ERR_ALIAS, "z partially overlaps x");
    return launch_shift_op(1, z, x, y, mu, shift, stream);
}

// ------------------------------------------------------ Wilson hopping

// Site tiles of the one-site Dslash kernel by `schedule` (1..3) and block
// B: 8 x 4 x 2 x B/64, 4 x 4 x 4 x B/64, 8 x 2 x 2 x B/32.
static void dslash_tile(int schedule, int block, uint32_t t[4])
{
    static const uint32_t shape[3][3] = {{8, 4, 2}, {4, 4, 4}, {8, 2, 2}};
    const uint32_t *sh = shape[(schedule - 1) % 3];
    t[0] = sh[0];
    t[1] = sh[1];
    t[2] = sh[2];
    t[3] = (uint32_t)block / (sh[0] * sh[1] * sh[2]);
}

static int spinor_prec_of_links(int link_prec)
{
    return link_prec == SU3_F64 ? SU3_F64 : SU3_F32;
}

// One site per lane, one-shot grid, the tuned (or default) block and
// occupancy of the key (SU3_EXPR_DSLASH, link precision, layout, lanes,
// volume).
static su3_status launch_dslash_op(su3_field *out, su3_field *const links[4],
                                   const su3_field *in, void *stream,
                                   const su3_launch *forced = nullptr)
{
    const su3_field *u0 = links[0];
    su3_launch c =
        forced ? *forced
               : lookup_launch(SU3_EXPR_DSLASH, u0->prec, u0->layout,
                               u0->lanes, u0->V);
    const int cbytes = 2 * out->rbytes;  // one complex spinor entry
    const bool vn = out->layout == SU3_LAYOUT_VNODE;
    const int nsub = vn ? (int)out->L : 1;
    const int lx = (int)(out->dims[0] / out->simd[0]);  // (outer) x extent
    LdsShape sh = {0, 0, 0, 0, 1};
    // LDS-tiled walks: schedules 4.. on lexicographic fields, the row tiles
    // (9..18) on virtual-node fields
    bool lds = c.schedule >= (vn ? 9 : 4);
    if (lds && c.schedule >= 19 && !lds_shape(c.schedule, c.block, cbytes, lx, nsub, sh)) {
        // a halo walk that does not fit: its rows with one buffer and a
        // halo, else the same rows without a halo (and their fallbacks)
        const int rows = c.schedule - 10;
        const int one_buffer = rows == 18 ? 17 : rows >= 13 && rows <= 16 ? rows - 4 : 0;
        c.schedule = one_buffer && lds_shape(one_buffer + 10, 0, cbytes, lx, nsub, sh)
                         ? one_buffer + 10
                         : rows;
    }
    if (lds && !lds_shape(c.schedule, c.block, cbytes, lx, nsub, sh)) {
        // buffers too large: the same rows with one buffer, else rows of
        // 2 x 2; a fixed tile too large for double spinors: the schedule's
        // smallest; else 16 x 4 x 4 (virtual nodes: one site per lane)
        const int one_buffer = c.schedule == 18                         ? 17
                               : c.schedule >= 13 && c.schedule <= 16 ? c.schedule - 4
                                                                      : 0;
        if (one_buffer && lds_shape(one_buffer, 0, cbytes, lx, nsub, sh)) {
            c.schedule = one_buffer;
        } else if (c.schedule >= 9 && lds_shape(9, 0, cbytes, lx, nsub, sh)) {
            c.schedule = 9;
        } else if (vn) {
            lds = false;
        } else {
            if (c.schedule >= 9)
                c.schedule = 8;
            c.block = c.schedule >= 7 ? 256 : 128;
            lds_shape(c.schedule, c.block, cbytes, lx, 1, sh);
        }
    }
    if (lds)
        c.block = sh.nsub * sh.tx * sh.ty * sh.tz;
    else if (c.block > 256)
        c.block = 256;  // the one-site and walk kernels take at most 256
    DslashArgs a;
    std::memset(&a, 0, sizeof a);
    a.out = out->ptr;
    a.in = in->ptr;
    for (int mu = 0; mu < 4; ++mu)
        a.u[mu] = links[mu]->ptr;
    a.gs = geom_of(out);
    a.gl = geom_of(u0);
    a.nsites = (int32_t)out->V;
    a.xcd_remap = c.xcd_remap;
    // outer extents and strides (storage sites), lane counts and strides
    int64_t ostride = vn ? out->L : 1, lstride = 1;
    uint32_t lg = 0;
    while (vn && ((int64_t)1 << lg) < out->L)
        ++lg;
    a.lg = lg;
    a.lmask = vn ? (uint32_t)(out->L - 1) : 0u;
    for (int mu = 0; mu < 4; ++mu) {
        a.dims[mu] = (uint32_t)(out->dims[mu] / out->simd[mu]);
        a.stride[mu] = (uint32_t)ostride;
        a.nlanes[mu] = (uint32_t)out->simd[mu];
        a.lstride[mu] = (uint32_t)lstride;
        ostride *= a.dims[mu];
        lstride *= out->simd[mu];
    }
    // lanes: one per site, or (lexicographic site order only) one per
    // (x, y, z) site and chunk of `walk` t-slices
    const int64_t Lt = a.dims[3];  // (outer) t extent
    a.walk = vn ? 1u : (uint32_t)std::min<int64_t>(std::max(c.tile_sites, 1), Lt);
    const int64_t lanes = a.walk <= 1 ? out->V
                                      : a.stride[3] * ((Lt + a.walk - 1) / a.walk);
    int64_t grid = (lanes + c.block - 1) / c.block;
    if (lds) {
        // LDS-tiled walk: tiles of (x, y, z) sites walking t
        a.lds_tile = (uint32_t)c.schedule;
        a.lds_tx = (uint32_t)sh.tx;
        a.walk = (uint32_t)std::min<int64_t>(std::max(c.tile_sites, 1), Lt);
        const uint32_t tdim[3] = {(uint32_t)sh.tx, (uint32_t)sh.ty, (uint32_t)sh.tz};
        grid = (Lt + a.walk - 1) / a.walk;
        int64_t ntiles = 1;
        for (int mu = 0; mu < 3; ++mu) {
            a.ntile[mu] = (a.dims[mu] + tdim[mu] - 1) / tdim[mu];
            ntiles *= a.ntile[mu];
        }
        grid *= ntiles;
        if (c.xcd_remap == 2)  // XCD slabs: 8 ranges of ceil(ntiles / 8) tiles
            grid = (Lt + a.walk - 1) / a.walk * 8 * ((ntiles + 7) / 8);
        if (c.persistent > 0) {
            // k workgroups per CU, each an equal share of the (tile, slice)
            // pairs: no tail of partly filled rounds, few walk starts
            const int64_t pairs = ntiles * Lt;
            const int64_t g = std::min<int64_t>(
                pairs, (int64_t)device_cus(out->device) * c.persistent);
            a.span = (uint32_t)((pairs + g - 1) / g);
            grid = (pairs + a.span - 1) / a.span;
        }
    } else if (a.walk <= 1 && !vn && c.schedule > 0) {
        dslash_tile(c.schedule, c.block, a.tile);
        grid = 1;
        for (int mu = 0; mu < 4; ++mu) {
            a.ntile[mu] = (uint32_t)((out->dims[mu] + a.tile[mu] - 1) / a.tile[mu]);
            grid *= a.ntile[mu];
        }
    }
    size_t shm = occupancy_reserve(out->device, c.occupancy);
    if (a.lds_tile)  // the tile's slice buffers (no occupancy cap)
        shm = lds_shape_bytes(sh, cbytes);
    hipError_t e = launch_dslash(out->prec, u0->prec, c.nontemporal, c.block,
                                 (int)grid, shm, a,
                                 static_cast<hipStream_t>(stream));
    if (e != hipSuccess)
        return hip_fail(e, "Dslash kernel launch");
    return SU3_OK;
}

extern "C" su3_status su3_dslash(su3_field *out, su3_field *const links[4],
                                 const su3_field *in, void *stream)
{
    if (!out || !in || !links)
        return fail(SU3_ERR_INVALID_ARG, "field or link list is NULL");
    for (int mu = 0; mu < 4; ++mu)
        if (!links[mu])
            return fail(SU3_ERR_INVALID_ARG, "links[%d] is NULL", mu);
    if (out->kind != KIND_SPINOR || in->kind != KIND_SPINOR)
        return fail(SU3_ERR_MISMATCH, "in and out must be spinor fields");
    if (!same_shape(out, in))
        return fail(SU3_ERR_MISMATCH, "in and out differ in dims, precision, "
                                      "layout, lanes or device");
    for (int mu = 0; mu < 4; ++mu) {
        const su3_field *u = links[mu];
        if (u->kind != KIND_MATRIX)
            return fail(SU3_ERR_MISMATCH, "links[%d] is not a matrix field", mu);
        if (!same_shape(u, links[0]))
            return fail(SU3_ERR_MISMATCH,
                        "links[%d] differs from links[0] in dims, precision, "
                        "layout, lanes or device", mu);
        if (!same_geometry(u, out))
            return fail(SU3_ERR_MISMATCH,
                        "links[%d] differs from the spinors in dims, layout, "
                        "lanes, virtual nodes or device", mu);
    }
    const int lp = links[0]->prec;
    if (lp == SU3_F16_F32ACC || spinor_prec_of_links(lp) != out->prec)
        return fail(SU3_ERR_UNSUPPORTED,
                    "precision pair (spinor %d, links %d) not supported: "
                    "F64 spinors take F64 links, F32 spinors F32 or C12 links",
                    out->prec, lp);
    if (overlaps(out, in))
        return fail(SU3_ERR_ALIAS, "out overlaps in (a stencil gathers "
                                   "neighbours: it cannot run in place)");
    for (int mu = 0; mu < 4; ++mu)
        if (overlaps(out, links[mu]))
            return fail(SU3_ERR_ALIAS, "out overlaps links[%d]", mu);
    return launch_dslash_op(out, links, in, stream);
}

// ------------------------------------------------ expression programs

struct su3_program {
    ProgCode code;
    int32_t kinds[kProgMaxOps];
};

static const char *kind_name(int k)
{
    switch (k) {
    case KIND_MATRIX: return "matrix";
    case KIND_SPINOR: return "spinor";
    case KIND_REAL: return "real";
    case KIND_COMPLEX: return "complex";
    }
    return "unknown";
}

extern "C" su3_status su3_program_create(su3_program **out, const char *expr,
                                         int32_t n_ops, const su3_kind *kinds)
{
    if (!out || !expr)
        return fail(SU3_ERR_INVALID_ARG, "out or expression is NULL");
    if (n_ops < 0 || n_ops > kProgMaxOps)
        return fail(SU3_ERR_INVALID_ARG, "n_ops %d not in [0, %d]", n_ops,
                    kProgMaxOps);
    if (n_ops > 0 && !kinds)
        return fail(SU3_ERR_INVALID_ARG, "kinds is NULL");
    int k32[kProgMaxOps] = {0};
    for (int k = 0; k < n_ops; ++k) {
        if (kinds[k] < KIND_MATRIX || kinds[k] > KIND_COMPLEX)
            return fail(SU3_ERR_INVALID_ARG, "unknown kind %d of operand %d",
                        (int)kinds[k], k);
        if (kinds[k] == KIND_SPINOR)
            return fail(SU3_ERR_UNSUPPORTED,
                        "expressions take matrix, real and complex fields");
        k32[k] = kinds[k];
    }
    su3_program *p = new su3_program();
    char err[256];
    if (!compile_program(expr, n_ops, k32, &p->code, err, sizeof err)) {
        delete p;
        return fail(SU3_ERR_INVALID_ARG, "expression \"%s\": %s", expr, err);
    }
    for (int k = 0; k < kProgMaxOps; ++k)
        p->kinds[k] = k < n_ops ? k32[k] : -1;
    *out = p;
    return SU3_OK;
}

extern "C" su3_status su3_program_info(const su3_program *p,
                                       su3_kind *result_kind,
                                       int32_t *n_instr, int32_t *n_regs)
{
    if (!p)
        return fail(SU3_ERR_INVALID_ARG, "program is NULL");
    if (result_kind)
        *result_kind = (su3_kind)p->code.result_kind;
    if (n_instr)
        *n_instr = p->code.ninstr;
    if (n_regs)
        *n_regs = p->code.nregs;
    return SU3_OK;
}

extern "C" su3_status su3_program_destroy(su3_program *p)
{
    delete p;
    return SU3_OK;
}

static su3_status launch_program_op(const su3_program *p, su3_field *z,
                                    const su3_field *const *ops, int arith,
                                    hipStream_t st,
                                    const su3_launch *forced = nullptr)
{
    const int form = p->code.real_only ? PF_REAL
                     : p->code.scalar_only ? PF_SCALAR
                                           : PF_MATRIX;
    // matrix-valued programs with a real or complex result (a trace) read
    // far more than they write, and are tuned under their own key
    const su3_expr key = form == PF_MATRIX && p->code.result_kind != FK_MATRIX
                             ? SU3_EXPR_PROGRAM_SCALAR
                             : SU3_EXPR_PROGRAM;
    su3_launch c =
        forced ? *forced : lookup_launch(key, arith, z->layout, z->lanes, z->V);
    if (!forced && form != PF_MATRIX) {
        // the block and occupancy cap are the matrix kernel's (a wave of it
        // keeps up to 18 KB of loads in flight); a scalar-valued wave keeps
        // 2-4 KB per operand, so it runs in full workgroups, uncapped
        c.block = 256;
        c.occupancy = 0;
    }
    ProgArgs a;
    std::memset(&a, 0, sizeof a);
    a.z = z->ptr;
    a.gz = geom_of(z);
    a.zkind = (uint8_t)z->kind;
    a.zprec = (uint8_t)z->prec;
    for (int k = 0; k < p->code.nops; ++k) {
        a.op[k] = ops[k]->ptr;
        a.g[k] = geom_of(ops[k]);
        a.kind[k] = (uint8_t)ops[k]->kind;
        a.prec[k] = (uint8_t)ops[k]->prec;
    }
    a.nops = (uint8_t)p->code.nops;
    a.ninstr = (uint8_t)p->code.ninstr;
    a.result = (uint8_t)p->code.result;
    a.used = (uint8_t)p->code.used;
    a.nsites = (int32_t)z->V;
    for (int t = 0; t < p->code.ninstr; ++t)
        a.ins[t] = p->code.ins[t];
    for (int k = 0; k < p->code.nimm; ++k) {
        a.imm[k][0] = p->code.imm[k][0];
        a.imm[k][1] = p->code.imm[k][1];
    }
    const int64_t per = program_sites_per_lane(arith, form);
    const int64_t lanes = (z->V + per - 1) / per;
    const int64_t grid = (lanes + c.block - 1) / c.block;
    hipError_t e = launch_program(arith, form, p->code.nregs,
                                  c.nontemporal, c.block, (int)grid,
                                  occupancy_reserve(z->device, c.occupancy), a,
                                  st);
    if (e != hipSuccess)
        return hip_fail(e, "program kernel launch");
    return SU3_OK;
}

extern "C" su3_status su3_program_eval(const su3_program *p, su3_field *z,
                                       const su3_field *const *ops,
                                       int32_t n_ops, void *stream)
{
    if (!p || !z)
        return fail(SU3_ERR_INVALID_ARG, "program or output is NULL");
    if (n_ops != p->code.nops)
        return fail(SU3_ERR_INVALID_ARG, "the program takes %d operands, got %d",
                    p->code.nops, n_ops);
    if (n_ops > 0 && !ops)
        return fail(SU3_ERR_INVALID_ARG, "operand list is NULL");
    if (z->kind != p->code.result_kind)
        return fail(SU3_ERR_MISMATCH,
                    "the expression is %s-valued, the output a %s field",
                    kind_name(p->code.result_kind), kind_name(z->kind));
    if (z->prec == SU3_F16_F32ACC)
        return fail(SU3_ERR_UNSUPPORTED, "expressions take F64, F32 or C12 fields");
    const int arith = z->prec == SU3_F64 ? SU3_F64 : SU3_F32;
    for (int k = 0; k < n_ops; ++k) {
        const su3_field *o = ops[k];
        if (!o)
            return fail(SU3_ERR_INVALID_ARG, "operand %d is NULL", k);
        if (o->kind != p->kinds[k])
            return fail(SU3_ERR_MISMATCH,
                        "operand %d is a %s field, the program declared %s", k,
                        kind_name(o->kind), kind_name(p->kinds[k]));
        if (!same_geometry(o, z))
            return fail(SU3_ERR_MISMATCH,
                        "operand %d differs from the output in dims, layout, "
                        "lanes, virtual nodes or device", k);
        if (o->prec == SU3_F16_F32ACC)
            return fail(SU3_ERR_UNSUPPORTED,
                        "expressions take F64, F32 or C12 fields");
        if ((o->prec == SU3_F64) != (arith == SU3_F64))
            return fail(SU3_ERR_MISMATCH,
                        "operand %d: an expression is evaluated in one precision "
                        "(all fields F64, or all F32/C12)", k);
        if (overlaps(z, o) && !(z->ptr == o->ptr && z->bytes == o->bytes))
            return fail(SU3_ERR_ALIAS, "output partially overlaps operand %d", k);
    }
    if (z->prec == SU3_C12_F32 && !p->code.su3_closed)
        return fail(SU3_ERR_UNSUPPORTED,
                    "a compressed output needs an SU(3)-valued expression "
                    "(products, adjoints, transposes, conjugates of matrices)");
    return launch_program_op(p, z, ops, arith, static_cast<hipStream_t>(stream));
}

// ------------------------------------------------------- launch tuning

// The virtual-node split a tuning key of N_sub = lanes stands for: factors
// of two handed to t, z, y, x in turn where the extent allows.
static su3_status default_simd(const int32_t dims[4], int32_t lanes,
                               int32_t simd[4])
{
    if (!dims)
        return fail(SU3_ERR_INVALID_ARG, "dims is NULL");
    if (lanes < 1 || lanes > 256 || (lanes & (lanes - 1)) != 0)
        return fail(SU3_ERR_INVALID_ARG,
                    "virtual-node lanes %d must be a power of two <= 256",
                    lanes);
    for (int d = 0; d < 4; ++d)
        simd[d] = 1;
    int left = lanes;
    for (int round = 0; left > 1 && round < 64; ++round)
        for (int d = 3; d >= 0 && left > 1; --d)
            if (dims[d] > 0 && dims[d] % (2 * simd[d]) == 0) {
                simd[d] *= 2;
                left /= 2;
            }
    if (left > 1)
        return fail(SU3_ERR_INVALID_ARG,
                    "dims cannot be split into %d virtual nodes", lanes);
    return SU3_OK;
}

static su3_status key_of(su3_expr expr, su3_precision prec, su3_layout layout,
                         int32_t lanes, const int32_t dims[4], Key *k,
                         Shape *shape)
{
    if ((expr < SU3_EXPR_MUL || expr > SU3_EXPR_PROGRAM_SCALAR) && !is_batch_key(expr))
        return fail(SU3_ERR_INVALID_ARG, "unknown expression %d", expr);
    const int base = is_batch_key(expr) ? expr - SU3_EXPR_BATCH : (int)expr;
    if ((expr == SU3_EXPR_PROGRAM || expr == SU3_EXPR_PROGRAM_SCALAR) && prec != SU3_F64 &&
        prec != SU3_F32)
        return fail(SU3_ERR_UNSUPPORTED,
                    "expression programs evaluate in F64 or F32");
    if (expr == SU3_EXPR_DSLASH && prec == SU3_F16_F32ACC)
        return fail(SU3_ERR_UNSUPPORTED,
                    "Dslash links are stored in F64, F32 or C12");
    int32_t simd[4] = {1, 1, 1, 1};
    if (layout == SU3_LAYOUT_VNODE) {
        su3_status st = default_simd(dims, lanes, simd);
        if (st != SU3_OK)
            return st;
    }
    Shape s;
    su3_status st = make_shape(dims, prec, layout, lanes, &s, KIND_MATRIX,
                               layout == SU3_LAYOUT_VNODE ? simd : nullptr);
    if (st != SU3_OK)
        return st;
    if (prec == SU3_C12_F32 &&
        (base == SU3_EXPR_MULADD || base == SU3_EXPR_ADD ||
         base == SU3_EXPR_APB_AB))
        return fail(SU3_ERR_UNSUPPORTED,
                    "the two-row compressed form supports MUL and MUL3 only");
    *k = Key(expr, prec, layout,
             layout == SU3_LAYOUT_AOSOA || layout == SU3_LAYOUT_VNODE ? lanes : 0,
             vbucket(s.V));
    if (shape)
        *shape = s;
    return SU3_OK;
}

extern "C" su3_status su3_launch_get(su3_expr expr, su3_precision prec,
                                     su3_layout layout, int32_t lanes,
                                     const int32_t dims[4], su3_launch *out)
{
    if (!out)
        return fail(SU3_ERR_INVALID_ARG, "out is NULL");
    Key k;
    Shape s;
    su3_status st = key_of(expr, prec, layout, lanes, dims, &k, &s);
    if (st != SU3_OK)
        return st;
    *out = lookup_launch(expr, prec, layout, std::get<3>(k), s.V);
    return SU3_OK;
}

extern "C" su3_status su3_launch_set(su3_expr expr, su3_precision prec,
                                     su3_layout layout, int32_t lanes,
                                     const int32_t dims[4],
                                     const su3_launch *cfg)
{
    if (!cfg)
        return fail(SU3_ERR_INVALID_ARG, "cfg is NULL");
    Key k;
    su3_status st = key_of(expr, prec, layout, lanes, dims, &k, nullptr);
    if (st != SU3_OK)
        return st;
    st = check_launch(*cfg, layout, expr);
    if (st != SU3_OK)
        return st;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_cache_locked();
    g_tuned[k] = *cfg;
    return SU3_OK;
}

extern "C" su3_status su3_launch_reset(void)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned.clear();
    g_cache_loaded = true;  // do not reload the file
    return SU3_OK;
}

// Candidate launches of the autotuner's sweep for a site-local expression
// (or a shift: expr CSHIFT / MUL_SHIFTED, one site per lane, blocks up to
// 256).  Persistent grid-stride launches are kept as a few samples only: on
// this hardware one-shot grids stream writes far better.
static std::vector<su3_launch> candidates(int layout, int expr, int prec)
{
    std::vector<su3_launch> out;
    su3_launch c;
    c.persistent = 0;
    c.xcd_remap = 0;
    c.lds_stage = 0;
    c.tile_sites = 4096;
    c.sites_per_lane = 0;
    if (layout == SU3_LAYOUT_AOS) {
        for (int b : {64, 128, 256})
            for (int nt : {0, 3, 7})
                for (int lds = 0; lds < 2; ++lds) {
                    if (lds && (b > 128 || nt == 7))
                        continue;
                    c.block = b;
                    c.nontemporal = nt;
                    c.lds_stage = lds;
                    c.occupancy = 0;
                    c.schedule = 0;
                    out.push_back(c);
                }
        return out;
    }
    const bool site = expr >= SU3_EXPR_MUL && expr <= SU3_EXPR_APB_AB;
    // sites per lane: the natural count, and twice it for the product
    std::vector<int> spl = {0};
    if (expr == SU3_EXPR_MUL && prec != SU3_F16_F32ACC)
        spl.push_back(2 * natural_sites(prec, expr));
    for (int S : spl)
        for (int b : {64, 128, 256})
            for (int occ : {0, 2, 3, 4, 5, 6, 8})
                for (int sched : {0, 1})
                    for (int nt : {0, 2, 3, 7})
                        for (int x : {0, 1}) {
                            if (S && (nt != 7 || x))
                                continue;  // wide lanes: streaming stores only
                            c.block = b;
                            c.occupancy = occ;
                            c.schedule = sched;
                            c.nontemporal = nt;
                            c.xcd_remap = x;
                            c.sites_per_lane = S;
                            out.push_back(c);
                        }
    c.xcd_remap = 0;
    c.sites_per_lane = 0;
    // 512- and 1024-lane workgroups (streaming stores), at most 32 waves
    // per compute unit
    if (site)
        for (int b : {512, 1024})
            for (int occ : {0, 1, 2, 3, 4})
                for (int sched : {0, 1}) {
                    if (occ * (b / 64) > 32)
                        continue;
                    c.block = b;
                    c.occupancy = occ;
                    c.schedule = sched;
                    c.nontemporal = 7;
                    out.push_back(c);
                }
    for (int b : {64, 256})
        for (int p : {2, 4})
            for (int sched : {0, 1}) {
                c.block = b;
                c.persistent = p;
                c.occupancy = 0;
                c.schedule = sched;
                c.nontemporal = 7;
                out.push_back(c);
            }
    return out;
}

// Candidates for the Wilson hopping kernel: t-slices per lane (1: one
// site per lane, in index order or in site tiles), block, occupancy cap,
// XCD remapping (nontemporal stores, cached spinor loads); LDS-tiled
// walks of every tile that fits the precision (cbytes per complex entry)
// and the lattice's x extent lx (whole-row tiles).
static std::vector<su3_launch> dslash_candidates(int cbytes, int lx, int nsub)
{
    std::vector<su3_launch> out;
    su3_launch c = default_launch(SU3_EXPR_DSLASH, SU3_F64, SU3_LAYOUT_SOA);
    c.nontemporal = 2;
    // virtual nodes: one site per lane in index order, or row tiles
    for (int walk : {1, 4, 8})
        for (int sched = 0; sched <= (walk == 1 && nsub == 1 ? 3 : 0); ++sched)
            for (int b : {64, 128, 256})
                for (int occ : {0, 2, 3, 4, 6})
                    for (int x : {0, 1}) {
                        if (nsub > 1 && walk > 1)
                            continue;
                        c.tile_sites = walk;
                        c.schedule = sched;
                        c.block = b;
                        c.occupancy = occ;
                        c.xcd_remap = x;
                        out.push_back(c);
                    }
    // LDS-tiled walks: every tile shape that fits this spinor precision and
    // lattice (cached loads; nontemporal stores), with and without a halo
    for (int sched = 4; sched <= 28; ++sched)
        for (int b : {128, 256, 512}) {
            LdsShape sh;
            if (!lds_shape(sched, b, cbytes, lx, nsub, sh) || (sched >= 9 && b != 256))
                continue;
            for (int walk : {4, 5, 6, 7, 8, 12, 16, 48})
                for (int x : {0, 1, 2}) {
                    c.tile_sites = walk;
                    c.schedule = sched;
                    c.block = b;
                    c.occupancy = 0;
                    c.xcd_remap = x;
                    out.push_back(c);
                }
            // k workgroups per CU, equal shares of the (tile, slice) pairs
            for (int k : {1, 2, 3}) {
                c.tile_sites = 1;
                c.schedule = sched;
                c.block = b;
                c.occupancy = 0;
                c.xcd_remap = 0;
                c.nontemporal = 2;
                c.persistent = k;
                out.push_back(c);
                c.persistent = 0;
            }
        }
    return out;
}

// Candidates for the program kernel: one site per lane, one-shot grid;
// block, occupancy cap, nontemporal bits.
static std::vector<su3_launch> program_candidates()
{
    std::vector<su3_launch> out;
    su3_launch c = default_launch(SU3_EXPR_PROGRAM, SU3_F64, SU3_LAYOUT_SOA);
    for (int b : {64, 128, 256})
        for (int occ : {0, 2, 3, 4, 6, 8})
            for (int nt : {0, 2, 3}) {
                c.block = b;
                c.occupancy = occ;
                c.nontemporal = nt;
                out.push_back(c);
            }
    return out;
}

// Median time (microseconds) of `reps` launches after `warm` warm-ups, each
// launch bracketed by its own events.
template <class F>
static su3_status time_launch(F launch, hipStream_t st, int warm, int reps,
                              double *us)
{
    for (int i = 0; i < warm; ++i) {
        su3_status s = launch();
        if (s != SU3_OK)
            return s;
    }
    std::vector<hipEvent_t> ev(2 * reps);
    for (auto &e : ev)
        HIP_TRY(hipEventCreate(&e), "hipEventCreate");
    su3_status result = SU3_OK;
    for (int i = 0; i < reps && result == SU3_OK; ++i) {
        (void)hipEventRecord(ev[2 * i], st);
        result = launch();
        (void)hipEventRecord(ev[2 * i + 1], st);
    }
    hipError_t e = hipStreamSynchronize(st);
    std::vector<double> t;
    for (int i = 0; i < reps && result == SU3_OK && e == hipSuccess; ++i) {
        float ms = 0;
        if (hipEventElapsedTime(&ms, ev[2 * i], ev[2 * i + 1]) == hipSuccess)
            t.push_back(ms * 1000.0);
    }
    for (auto &x : ev)
        (void)hipEventDestroy(x);
    if (result != SU3_OK)
        return result;
    if (e != hipSuccess)
        return hip_fail(e, "autotune sync");
    if (t.empty())
        return fail(SU3_ERR_HIP, "no timing recorded");
    std::sort(t.begin(), t.end());
    *us = t[t.size() / 2];
    return SU3_OK;
}

static su3_status autotune_impl(su3_expr expr, su3_precision prec,
                                su3_layout layout, int32_t lanes,
                                const int32_t dims[4], void *stream,
                                su3_launch *best, double *best_us)
{
    if (is_batch_key(expr))
        return fail(SU3_ERR_INVALID_ARG,
                    "batch keys are tuned by su3_batch_autotune");
    Key k;
    Shape s;
    su3_status st = key_of(expr, prec, layout, lanes, dims, &k, &s);
    if (st != SU3_OK)
        return st;
    hipStream_t hs = static_cast<hipStream_t>(stream);
    const bool dslash = expr == SU3_EXPR_DSLASH;
    // Dslash: f[0] out, f[1] in (spinors), f[2..5] links
    const int nops = expr == SU3_EXPR_CSHIFT ? 1
                     : dslash              ? 5
                                           : operands_of(expr);
    int32_t simd[4] = {1, 1, 1, 1};
    if (layout == SU3_LAYOUT_VNODE)
        (void)default_simd(dims, lanes, simd);  // checked by key_of
    // Operand sets: one, or -- when a set of 64 to 512 MiB fits twice into
    // the 256 MiB Infinity Cache -- as many as make 1 GiB, launched in
    // rotation, so that each timed launch finds its operands in HBM (tuning
    // on one cache-resident set picked launches up to 23 % slower cold at
    // 32^4).  Below 64 MiB launches are short enough that per-launch timing
    // of rotating sets misleads (16^4: the hot choice is faster hot and
    // cold), so they keep one set.
    std::vector<std::array<su3_field *, 6>> sets(1);
    sets[0].fill(nullptr);
    for (size_t n = 0; n < sets.size() && st == SU3_OK; ++n) {
        su3_field **f = sets[n].data();
        size_t set_bytes = 0;
        for (int i = 0; i <= nops && st == SU3_OK; ++i) {
            const bool spinor = dslash && i < 2;
            const int fp = spinor ? spinor_prec_of_links(prec) : prec;
            const int kind = spinor                                          ? KIND_SPINOR
                             : i == 0 && expr == SU3_EXPR_PROGRAM_SCALAR ? KIND_COMPLEX
                                                                          : KIND_MATRIX;
            if (layout == SU3_LAYOUT_VNODE)
                st = alloc_of_kind(&f[i], dims, fp, layout, 0, kind, simd);
            else
                st = alloc_of_kind(&f[i], dims, fp, layout, lanes, kind);
            if (st == SU3_OK) {
                set_bytes += f[i]->bytes;
                // a non-zero bit pattern (finite in every precision)
                hipError_t e = hipMemsetD32Async((hipDeviceptr_t)f[i]->ptr,
                                                 0x3c003c00u, f[i]->bytes / 4, hs);
                if (e != hipSuccess)
                    st = hip_fail(e, "fill");
            }
        }
        if (n == 0 && st == SU3_OK && set_bytes < ((size_t)512 << 20) &&
            set_bytes >= ((size_t)64 << 20)) {
            const size_t want = (((size_t)1 << 30) + set_bytes - 1) / set_bytes;
            sets.resize(std::max<size_t>(2, want));
            for (size_t m = 1; m < sets.size(); ++m)
                sets[m].fill(nullptr);
        }
    }
    size_t turn = 0;
    su3_launch win = default_launch(expr, prec, layout);
    double win_us = 1e300;
    // expression programs are timed on the streaming product a*b, those
    // with a scalar result on the trace of a product
    const bool program = expr == SU3_EXPR_PROGRAM || expr == SU3_EXPR_PROGRAM_SCALAR;
    su3_program prog;
    if (st == SU3_OK && program) {
        const int kinds[2] = {KIND_MATRIX, KIND_MATRIX};
        char err[128];
        const char *text = expr == SU3_EXPR_PROGRAM ? "a*b" : "trace(a*adj(b))";
        if (!compile_program(text, 2, kinds, &prog.code, err, sizeof err))
            st = fail(SU3_ERR_HIP, "internal program: %s", err);
    }
    if (st == SU3_OK) {
        const su3_field *f0 = sets[0][0];
        for (const su3_launch &c : dslash ? dslash_candidates(2 * f0->rbytes,
                                                              f0->dims[0] / f0->simd[0],
                                                              layout == SU3_LAYOUT_VNODE
                                                                  ? (int)f0->L : 1)
                                   : program ? program_candidates()
                                                              : candidates(layout, expr, prec)) {
            if (expr == SU3_EXPR_CSHIFT && c.schedule)
                continue;  // a copy has no row phases
            double us = 0;
            su3_status r = time_launch(
                [&]() {
                    su3_field *const *f = sets[turn++ % sets.size()].data();
                    const su3_field *ops[4] = {f[1], f[2], f[3], f[4]};
                    su3_field *links[4] = {f[2], f[3], f[4], f[5]};
                    if (dslash)
                        return launch_dslash_op(f[0], links, f[1], stream, &c);
                    if (program)
                        return launch_program_op(&prog, f[0], ops, prec, hs, &c);
                    if (expr == SU3_EXPR_CSHIFT)
                        return launch_shift_op(0, f[0], nullptr, f[1], 1, 1,
                                               stream, &c);
                    if (expr == SU3_EXPR_MUL_SHIFTED)
                        return launch_shift_op(1, f[0], f[1], f[2], 1, 1,
                                               stream, &c);
                    return launch_item(f[0], expr, ops, nops, c, hs);
                },
                hs, 3, 10, &us);
            if (r != SU3_OK) {
                (void)hipGetLastError();
                continue;  // a launch shape the device refused
            }
            if (us < win_us) {
                win_us = us;
                win = c;
            }
        }
        if (win_us >= 1e300)
            st = fail(SU3_ERR_HIP, "no candidate launch ran");
    }
    for (auto &set : sets)
        for (su3_field *fi : set)
            su3_field_free(fi);
    if (st != SU3_OK)
        return st;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        load_cache_locked();
        g_tuned[k] = win;
    }
    append_cache(k, win, win_us);
    if (best)
        *best = win;
    if (best_us)
        *best_us = win_us;
    return SU3_OK;
}

extern "C" su3_status su3_autotune(su3_expr expr, su3_precision prec,
                                   su3_layout layout, int32_t lanes,
                                   const int32_t dims[4], void *stream,
                                   su3_launch *best)
{
    return autotune_impl(expr, prec, layout, lanes, dims, stream, best, nullptr);
}

extern "C" su3_status su3_layout_recommend(su3_expr expr, su3_precision prec,
                                           const int32_t dims[4], void *stream,
                                           su3_layout *layout, int32_t *lanes,
                                           su3_launch *best, double *us)
{
    if (expr < SU3_EXPR_MUL || expr > SU3_EXPR_APB_AB)
        return fail(SU3_ERR_INVALID_ARG,
                    "layouts are recommended for the site-local expressions");
    if (!layout || !lanes)
        return fail(SU3_ERR_INVALID_ARG, "layout or lanes is NULL");
    // the candidates: SoA and AoSoA with every lane count; each tuned (and
    // its launch kept, as su3_autotune does); the fastest tuned time wins,
    // ties to the earlier (larger contiguous runs first)
    const struct { su3_layout lay; int32_t L; } cand[] = {
        {SU3_LAYOUT_SOA, 0}, {SU3_LAYOUT_AOSOA, 64}, {SU3_LAYOUT_AOSOA, 32},
        {SU3_LAYOUT_AOSOA, 16}, {SU3_LAYOUT_AOSOA, 8}};
    double win_us = 1e300;
    for (const auto &c : cand) {
        su3_launch l;
        double t = 0;
        su3_status st = autotune_impl(expr, prec, c.lay, c.L, dims, stream, &l, &t);
        if (st != SU3_OK)
            return st;
        if (t < win_us) {
            win_us = t;
            *layout = c.lay;
            *lanes = c.L;
            if (best)
                *best = l;
        }
    }
    if (us)
        *us = win_us;
    return SU3_OK;
}

// ------------------------------------------------------------ batches

// The items of a batch as the kernel reads them, validated (each item by
// su3_fused_eval's rules; batch-level rules here), with the tile table
// of the launch `cfg`: forced (the autotuner), else the tuned (or default)
// setting of the batch key (SU3_EXPR_BATCH + leading expression, leading
// item's precision, layout, lanes) at the total volume.
struct BatchPlan {
    std::vector<BatchItem> items;
    int mode;
    int device;
    int64_t ntiles;
    su3_launch cfg;
};

static su3_status plan_batch(const su3_expr *exprs, su3_field *const *z,
                             const su3_field *const *ops, int32_t n,
                             const su3_launch *forced, BatchPlan *plan)
{
    if (!exprs || !z || !ops)
        return fail(SU3_ERR_INVALID_ARG, "NULL argument");
    if (n <= 0)
        return fail(SU3_ERR_INVALID_ARG, "batch needs at least one item");
    std::vector<BatchItem> &items = plan->items;
    items.assign(n, BatchItem());
    int mode = 0;
    int64_t total_sites = 0;
    int dev = -1;
    for (int i = 0; i < n; ++i) {
        const int nops = (exprs[i] >= SU3_EXPR_MUL && exprs[i] <= SU3_EXPR_APB_AB)
                             ? operands_of(exprs[i])
                             : 0;
        su3_status st = validate_item(z[i], exprs[i], ops + 4 * i, nops);
        if (st != SU3_OK)
            return fail(st, "batch item %d: %s", i, g_last_error.c_str());
        for (int k = nops; k < 4; ++k)
            if (ops[4 * i + k])
                return fail(SU3_ERR_INVALID_ARG,
                            "batch item %d: unused operand slot %d not NULL",
                            i, k);
        if (dev < 0)
            dev = z[i]->device;
        else if (z[i]->device != dev)
            return fail(SU3_ERR_MISMATCH, "batch items on different devices");
        if (z[i]->layout == SU3_LAYOUT_AOS ||
            (z[i]->layout == SU3_LAYOUT_VNODE && z[i]->L < 4))
            return fail(SU3_ERR_UNSUPPORTED,
                        "batch item %d: batches take SoA, AoSoA or "
                        "virtual-node fields with N_sub >= 4", i);
        BatchItem &it = items[i];
        std::memset(&it, 0, sizeof it);
        it.z = z[i]->ptr;
        for (int k = 0; k < nops; ++k)
            it.op[k] = ops[4 * i + k]->ptr;
        it.g = geom_of(z[i]);
        it.nsites = (int32_t)z[i]->V;
        it.prec = z[i]->prec;
        it.expr = exprs[i];
        if (!(exprs[i] == SU3_EXPR_MUL &&
              (z[i]->prec == SU3_F64 || z[i]->prec == SU3_C12_F32)))
            mode = 1;
        total_sites += z[i]->V;
    }
    const su3_launch cfg =
        forced ? *forced
               : lookup_launch(SU3_EXPR_BATCH + exprs[0], z[0]->prec,
                               z[0]->layout, z[0]->lanes, total_sites);
    const int T = cfg.tile_sites;
    // tile table: item i owns ceil(V_i / T) tiles starting at the exclusive
    // prefix sum of its predecessors' counts
    int64_t ntiles = 0;
    for (int i = 0; i < n; ++i) {
        items[i].tile_start = (int32_t)ntiles;
        ntiles += (z[i]->V + T - 1) / T;
        if (ntiles >= ((int64_t)1 << 31))
            return fail(SU3_ERR_INVALID_ARG, "too many tiles");
    }
    plan->mode = mode;
    plan->device = dev;
    plan->ntiles = ntiles;
    plan->cfg = cfg;
    return SU3_OK;
}

// Workgroups of a batch launch: k per CU for a persistent grid (at most one
// per tile), else one per tile.
static int32_t batch_grid(const BatchPlan &p)
{
    return p.cfg.persistent > 0
               ? (int32_t)std::min<int64_t>(p.ntiles, (int64_t)p.cfg.persistent *
                                                          device_cus(p.device))
               : (int32_t)p.ntiles;
}

static su3_status batch_create(su3_batch **out, const su3_expr *exprs,
                               su3_field *const *z, const su3_field *const *ops,
                               int32_t n, void *stream, const su3_launch *forced)
{
    if (!out)
        return fail(SU3_ERR_INVALID_ARG, "NULL argument");
    BatchPlan plan;
    su3_status pst = plan_batch(exprs, z, ops, n, forced, &plan);
    if (pst != SU3_OK)
        return pst;
    const std::vector<BatchItem> &items = plan.items;
    const int mode = plan.mode, dev = plan.device;
    const int64_t ntiles = plan.ntiles;
    const su3_launch cfg = plan.cfg;
    const int T = cfg.tile_sites;
    su3_batch *b = new su3_batch();
    std::memset(b, 0, sizeof *b);
    b->nitems = n;
    b->ntiles = (int32_t)ntiles;
    b->mode = mode;
    b->cfg = cfg;
    b->device = dev;
    // persistent k > 0: k workgroups per CU draw the tiles from a ticket
    // counter; 0: one workgroup per tile
    b->grid = batch_grid(plan);
    hipStream_t hs = static_cast<hipStream_t>(stream);
    // the counter (16 bytes, zero) and the item table in one allocation
    const size_t bytes = 16 + sizeof(BatchItem) * n;
    std::vector<unsigned char> image(bytes, 0);
    std::memcpy(image.data() + 16, items.data(), sizeof(BatchItem) * n);
    hipError_t e = hipMalloc(&b->d_mem, bytes);
    if (e == hipSuccess) {
        b->d_queue = cfg.persistent > 0 ? static_cast<unsigned long long *>(b->d_mem)
                                        : nullptr;
        b->d_items = reinterpret_cast<BatchItem *>(static_cast<unsigned char *>(b->d_mem) + 16);
        e = hipMemcpyAsync(b->d_mem, image.data(), bytes, hipMemcpyHostToDevice, hs);
    }
    if (e == hipSuccess)
        e = hipStreamSynchronize(hs);
    // Capture the one launch on a private stream and instantiate the graph.
    hipStream_t cap = nullptr;
    if (e == hipSuccess)
        e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
    if (e == hipSuccess)
        e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        hipError_t le = launch_batch(b->mode, b->d_items, b->nitems, b->ntiles,
                                     T, cfg.nontemporal, cfg.schedule, cfg.block,
                                     b->grid, occupancy_reserve(dev, cfg.occupancy),
                                     b->d_queue, cap);
        hipError_t ce = hipStreamEndCapture(cap, &b->graph);
        e = le != hipSuccess ? le : ce;
    }
    if (e == hipSuccess)
        e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    if (cap)
        (void)hipStreamDestroy(cap);
    if (e != hipSuccess) {
        su3_status r = hip_fail(e, "batch create");
        su3_batch_destroy(b);
        return r;
    }
    *out = b;
    return SU3_OK;
}

extern "C" su3_status su3_batch_create(su3_batch **out, const su3_expr *exprs,
                                       su3_field *const *z,
                                       const su3_field *const *ops, int32_t n,
                                       void *stream)
{
    return batch_create(out, exprs, z, ops, n, stream, nullptr);
}

// ------------------------------------------- allocation-free batches

// Scratch of su3_batch_run: the persistent grid's ticket counter (bytes
// 0..15) and up to kRunMaxItems item records (from byte 256).  A
// file-scope device array: every device the library runs on holds one
// copy for the life of the process, at its own address, which host code
// reaches only through run_scratch() (the array's name is a host-side
// stand-in, not a device address).
static const int kRunMaxItems = 1024;
static const size_t kRunScratchBytes = 256 + sizeof(BatchItem) * kRunMaxItems;
static __device__ __align__(256) unsigned char scratch[kRunScratchBytes];

// Device address of `scratch` on device `dev` (the current device),
// looked up once per device.
static su3_status run_scratch(int dev, unsigned char **out)
{
    static std::mutex mu;
    static unsigned char *ptrs[64];
    if (dev < 0 || dev >= 64)
        return fail(SU3_ERR_UNSUPPORTED, "device %d beyond the 64 the library serves", dev);
    std::lock_guard<std::mutex> lk(mu);
    if (!ptrs[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess)
            return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p)
            return fail(SU3_ERR_HIP, "no device address for the batch scratch");
        ptrs[dev] = static_cast<unsigned char *>(p);
    }
    *out = ptrs[dev];
    return SU3_OK;
}

extern "C" su3_status su3_batch_run(const su3_expr *exprs, su3_field *const *z,
                                    const su3_field *const *ops, int32_t n,
                                    void *stream)
{
    if (n > kRunMaxItems)
        return fail(SU3_ERR_INVALID_ARG,
                    "su3_batch_run takes at most %d items (got %d); "
                    "su3_batch_create takes any number", kRunMaxItems, n);
    BatchPlan plan;
    su3_status st = plan_batch(exprs, z, ops, n, nullptr, &plan);
    if (st != SU3_OK)
        return st;
    int cur = -1;
    HIP_TRY(hipGetDevice(&cur), "hipGetDevice");
    if (cur != plan.device)
        return fail(SU3_ERR_MISMATCH,
                    "the batch's fields are on device %d, the current device is %d",
                    plan.device, cur);
    unsigned char *sp = nullptr;
    st = run_scratch(plan.device, &sp);
    if (st != SU3_OK)
        return st;
    unsigned long long *queue =
        plan.cfg.persistent > 0 ? reinterpret_cast<unsigned long long *>(sp) : nullptr;
    BatchItem *items = reinterpret_cast<BatchItem *>(sp + 256);
    hipStream_t hs = static_cast<hipStream_t>(stream);
    hipError_t e = launch_put_items(items, plan.items.data(), n, queue, hs);
    if (e == hipSuccess)
        e = launch_batch(plan.mode, items, n, (int32_t)plan.ntiles,
                         plan.cfg.tile_sites, plan.cfg.nontemporal, plan.cfg.schedule,
                         plan.cfg.block, batch_grid(plan),
                         occupancy_reserve(plan.device, plan.cfg.occupancy), queue, hs);
    if (e != hipSuccess)
        return hip_fail(e, "batch run launch");
    return SU3_OK;
}

extern "C" su3_status su3_batch_launch(su3_batch *b, void *stream)
{
    if (!b)
        return fail(SU3_ERR_INVALID_ARG, "batch is NULL");
    HIP_TRY(hipGraphLaunch(b->exec, static_cast<hipStream_t>(stream)),
            "hipGraphLaunch");
    return SU3_OK;
}

extern "C" su3_status su3_batch_destroy(su3_batch *b)
{
    if (!b)
        return SU3_OK;
    if (b->exec)
        (void)hipGraphExecDestroy(b->exec);
    if (b->graph)
        (void)hipGraphDestroy(b->graph);
    if (b->d_mem)
        (void)hipFree(b->d_mem);
    delete b;
    return SU3_OK;
}

// Candidate launches of the batch autotuner: for each tile size, one-shot
// grids (one workgroup per tile: blocks of 64 or 128, occupancy caps,
// schedules, nontemporal or streaming stores) and persistent grids drawing
// the tiles from the ticket counter (blocks of 64 or 256, 2-8 workgroups
// per CU, streaming stores).
static std::vector<su3_launch> batch_candidates()
{
    std::vector<su3_launch> out;
    su3_launch c;
    c.xcd_remap = 0;
    c.lds_stage = 0;
    c.sites_per_lane = 0;
    for (int tile : {64, 128, 256, 512, 2048, 8192}) {
        c.tile_sites = tile;
        c.persistent = 0;
        for (int b : {64, 128})
            for (int occ : {0, 4, 6})
                for (int sched : {0, 1})
                    for (int nt : {3, 7}) {
                        c.block = b;
                        c.occupancy = occ;
                        c.schedule = sched;
                        c.nontemporal = nt;
                        out.push_back(c);
                    }
        c.occupancy = 0;
        c.nontemporal = 7;
        for (int b : {64, 256})
            for (int k : {2, 4, 8})
                for (int sched : {0, 1}) {
                    c.block = b;
                    c.persistent = k;
                    c.schedule = sched;
                    out.push_back(c);
                }
    }
    return out;
}

extern "C" su3_status su3_batch_autotune(const su3_expr *exprs,
                                         su3_field *const *z,
                                         const su3_field *const *ops,
                                         int32_t n, void *stream,
                                         su3_launch *best)
{
    if (!exprs || !z || !ops || n <= 0 || !z[0])
        return fail(SU3_ERR_INVALID_ARG, "NULL argument or empty batch");
    hipStream_t hs = static_cast<hipStream_t>(stream);
    int64_t total = 0;
    for (int i = 0; i < n; ++i)
        if (z[i])
            total += z[i]->V;
    su3_launch win = default_launch(exprs[0], z[0]->prec, z[0]->layout);
    double win_us = 1e300;
    for (const su3_launch &c : batch_candidates()) {
        su3_batch *b = nullptr;
        su3_status st = batch_create(&b, exprs, z, ops, n, stream, &c);
        if (st != SU3_OK)
            return st;  // invalid items: report, nothing tuned
        double us = 0;
        st = time_launch([&]() { return su3_batch_launch(b, stream); }, hs, 2,
                         5, &us);
        su3_batch_destroy(b);
        if (st != SU3_OK)
            return st;
        if (us < win_us) {
            win_us = us;
            win = c;
        }
    }
    const Key k(SU3_EXPR_BATCH + exprs[0], z[0]->prec, z[0]->layout,
                z[0]->lanes, vbucket(total));
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        load_cache_locked();
        g_tuned[k] = win;
    }
    append_cache(k, win, win_us);
    if (best)
        *best = win;
    return SU3_OK;
}

extern "C" su3_status su3_batch_tiles(const su3_batch *b, int32_t *rows,
                                      int64_t cap, int64_t *n_tiles)
{
    if (!b || !n_tiles)
        return fail(SU3_ERR_INVALID_ARG, "NULL argument");
    *n_tiles = b->ntiles;
    if (!rows || cap < b->ntiles)
        return SU3_OK;
    // expand the table from the items the kernel reads (tile starts, sizes)
    std::vector<BatchItem> items(b->nitems);
    HIP_TRY(hipMemcpy(items.data(), b->d_items, sizeof(BatchItem) * b->nitems,
                      hipMemcpyDeviceToHost),
            "batch items copy");
    const int64_t T = b->cfg.tile_sites;
    for (int i = 0; i < b->nitems; ++i) {
        const int64_t end = i + 1 < b->nitems ? items[i + 1].tile_start : b->ntiles;
        for (int64_t t = items[i].tile_start; t < end; ++t) {
            const int64_t first = (t - items[i].tile_start) * T;
            rows[4 * t + 0] = i;
            rows[4 * t + 1] = (int32_t)first;
            rows[4 * t + 2] = (int32_t)std::min<int64_t>(T, items[i].nsites - first);
            rows[4 * t + 3] = items[i].prec;
        }
    }
    return SU3_OK;
}

// ------------------------------------------------------ yardsticks

// Default launch of each yardstick kind (the fastest of its sweep at 2.29
// GB on MI355X): 64-lane workgroups, 20 per compute unit for the triad,
// 16 for read-only, no cap for copy; 128-lane workgroups, 12 per compute
// unit, for the write-only stream; write-through streaming stores and
// nontemporal loads.
static su3_launch stream_default(int kind)
{
    su3_launch c;
    std::memset(&c, 0, sizeof c);
    c.block = kind == SU3_STREAM_WRITE ? 128 : 64;
    c.occupancy = kind == SU3_STREAM_TRIAD  ? 20
                  : kind == SU3_STREAM_READ ? 16
                  : kind == SU3_STREAM_WRITE ? 12
                                             : 0;
    c.nontemporal = 7;
    c.tile_sites = 4096;
    return c;
}

static su3_status stream_launch(int kind, void *a, const void *b,
                                const void *c, double s, int64_t n16,
                                int tail, const su3_launch &cfg,
                                hipStream_t st)
{
    if (kind < SU3_STREAM_TRIAD || kind > SU3_STREAM_COPY)
        return fail(SU3_ERR_INVALID_ARG, "unknown yardstick kind %d", kind);
    const bool reads_b = kind != SU3_STREAM_WRITE;
    const bool reads_c = kind == SU3_STREAM_TRIAD || kind == SU3_STREAM_READ;
    if (!a || (reads_b && !b) || (reads_c && !c))
        return fail(SU3_ERR_INVALID_ARG, "NULL array");
    if (n16 < 0 || (n16 == 0 && !tail))
        return fail(SU3_ERR_INVALID_ARG, "empty arrays");
    if (((uintptr_t)a | (uintptr_t)(reads_b ? b : a) |
         (uintptr_t)(reads_c ? c : a)) & 15)
        return fail(SU3_ERR_INVALID_ARG, "arrays must be 16-byte aligned");
    if (cfg.block < 64 || cfg.block > 1024 || cfg.block % 64)
        return fail(SU3_ERR_INVALID_ARG,
                    "block %d not a multiple of 64 in [64, 1024]", cfg.block);
    if (!nt_valid(cfg.nontemporal, true))
        return fail(SU3_ERR_INVALID_ARG, "nontemporal %d not in {0, 1, 2, 3, 6, 7}",
                    cfg.nontemporal);
    if (cfg.occupancy < 0 || cfg.occupancy > 64)
        return fail(SU3_ERR_INVALID_ARG, "occupancy %d not in [0, 64]",
                    cfg.occupancy);
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
    hipError_t e = launch_stream(kind, a, b, c, s, n16, tail,
                                 cfg.nontemporal, cfg.block,
                                 occupancy_reserve(dev, cfg.occupancy), st);
    if (e != hipSuccess)
        return hip_fail(e, "yardstick launch");
    return SU3_OK;
}

extern "C" su3_status su3_stream(su3_stream_kind kind, void *a, const void *b,
                                 const void *c, double s, size_t bytes,
                                 const su3_launch *cfg, void *stream)
{
    if (bytes == 0 || bytes % 16)
        return fail(SU3_ERR_INVALID_ARG,
                    "bytes must be a positive multiple of 16");
    const su3_launch l = cfg ? *cfg : stream_default(kind);
    return stream_launch(kind, a, b, c, s, (int64_t)(bytes / 16), 0, l,
                         static_cast<hipStream_t>(stream));
}

extern "C" su3_status su3_stream_autotune(su3_stream_kind kind, void *a,
                                          const void *b, const void *c,
                                          size_t bytes, void *stream,
                                          su3_launch *best, double *us_out)
{
    if (bytes == 0 || bytes % 16)
        return fail(SU3_ERR_INVALID_ARG,
                    "bytes must be a positive multiple of 16");
    hipStream_t hs = static_cast<hipStream_t>(stream);
    su3_launch win = stream_default(kind);
    double win_us = 1e300;
    su3_launch l = win;
    for (int blk : {64, 128, 256, 512, 1024})
        for (int occ : {0, 1, 2, 3, 4, 6, 8, 12, 16, 20, 24, 32})
            for (int nt : {0, 2, 3, 6, 7}) {
                if (occ * (blk / 64) > 32 || (occ == 0 && blk > 256) ||
                    (occ == 1 && blk < 512))
                    continue;
                l.block = blk;
                l.occupancy = occ;
                l.nontemporal = nt;
                double us = 0;
                su3_status st = time_launch(
                    [&]() {
                        return stream_launch(kind, a, b, c, 3.0,
                                             (int64_t)(bytes / 16), 0, l, hs);
                    },
                    hs, 3, 10, &us);
                if (st != SU3_OK && win_us >= 1e300)
                    return st;  // invalid arguments: nothing tuned
                if (st != SU3_OK) {
                    (void)hipGetLastError();
                    continue;
                }
                if (us < win_us) {
                    win_us = us;
                    win = l;
                }
            }
    if (best)
        *best = win;
    if (us_out)
        *us_out = win_us;
    return SU3_OK;
}

extern "C" su3_status su3_triad(double *a, const double *b, const double *c,
                                double s, int64_t n, void *stream)
{
    if (n <= 0)
        return fail(SU3_ERR_INVALID_ARG, "n must be > 0");
    return stream_launch(SU3_STREAM_TRIAD, a, b, c, s, n / 2, (int)(n & 1),
                         stream_default(SU3_STREAM_TRIAD),
                         static_cast<hipStream_t>(stream));
}

extern "C" su3_status su3_copy(void *dst, const void *src, size_t bytes,
                               void *stream)
{
    if (bytes == 0 || bytes % 16)
        return fail(SU3_ERR_INVALID_ARG,
                    "bytes must be a positive multiple of 16");
    return stream_launch(SU3_STREAM_COPY, dst, src, nullptr, 0.0,
                         (int64_t)(bytes / 16), 0,
                         stream_default(SU3_STREAM_COPY),
                         static_cast<hipStream_t>(stream));
}

// ------------------------------------------------------------ misc

extern "C" su3_status su3_sync(void *stream)
{
    HIP_TRY(hipStreamSynchronize(static_cast<hipStream_t>(stream)),
            "hipStreamSynchronize");
    HIP_TRY(hipGetLastError(), "pending error");
    return SU3_OK;
}

extern "C" const char *su3_status_string(su3_status s)
{
    switch (s) {
    case SU3_OK: return "SU3_OK";
    case SU3_ERR_INVALID_ARG: return "SU3_ERR_INVALID_ARG";
    case SU3_ERR_MISMATCH: return "SU3_ERR_MISMATCH";
    case SU3_ERR_UNSUPPORTED: return "SU3_ERR_UNSUPPORTED";
    case SU3_ERR_OUT_OF_MEMORY: return "SU3_ERR_OUT_OF_MEMORY";
    case SU3_ERR_ALIAS: return "SU3_ERR_ALIAS";
    case SU3_ERR_HIP: return "SU3_ERR_HIP";
    }
    return "SU3_ERR_UNKNOWN";
}

extern "C" const char *su3_last_error(void)
{
    return g_last_error.c_str();
}
