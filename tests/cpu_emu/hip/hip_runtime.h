// Host-side stand-in for the slice of the HIP API that libsu3 uses, so that
// the library's kernels and C ABI can be compiled as ordinary C++ and run on
// the CPU under AddressSanitizer/UBSan (test infrastructure only; the
// product is never built against it).  A kernel launch runs every
// (workgroup, lane) of the grid in turn -- or, for kernels with barriers,
// each workgroup's lanes as threads meeting at a std::barrier; device memory
// is host memory, streams are no-ops, graph capture records the launches.
#pragma once
#include <cstddef>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <cstdio>
#include <functional>
#include <vector>
#include <thread>
#include <barrier>
#include <algorithm>

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __shared__
#define __align__(n) __attribute__((aligned(n)))

typedef int hipError_t;
enum { hipSuccess = 0, hipErrorInvalidValue = 1, hipErrorOutOfMemory = 2 };
typedef void *hipStream_t;
typedef void *hipDeviceptr_t;
typedef void *hipEvent_t;
typedef void *hipGraph_t;
typedef void *hipGraphExec_t;
enum { hipMemcpyHostToDevice = 1, hipMemcpyDeviceToHost = 2 };
enum { hipMemoryTypeDevice = 2 };
enum { hipStreamNonBlocking = 1 };
enum { hipStreamCaptureModeThreadLocal = 1 };
enum { hipFuncAttributeMaxDynamicSharedMemorySize = 8 };
inline hipError_t hipFuncSetAttribute(const void *, int, int) { return hipSuccess; }
enum { hipDeviceAttributeMultiprocessorCount = 1, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor = 2, hipDeviceAttributeMaxSharedMemoryPerBlock = 3 };
inline void __builtin_amdgcn_sched_barrier(int) {}
// Buffer stores and readfirstlane for one lane at a time: the wave-uniform
// base of a lane is its own address, and a store is bounds-checked against
// the descriptor's record count before it lands (AddressSanitizer checks
// the address itself).
struct emu_buffer_rsrc { char *base; uint32_t records; };
typedef emu_buffer_rsrc __amdgpu_buffer_rsrc_t;
inline uint32_t __builtin_amdgcn_readfirstlane(uint32_t v) { return v; }
inline unsigned long long atomicAdd(unsigned long long *p, unsigned long long v)
{
    return __atomic_fetch_add(p, v, __ATOMIC_SEQ_CST);
}
inline emu_buffer_rsrc __builtin_amdgcn_make_buffer_rsrc(void *p, short, int records, int)
{
    return {static_cast<char *>(p), static_cast<uint32_t>(records)};
}
template <class V>
inline void emu_buffer_store(V v, emu_buffer_rsrc r, uint32_t off, uint32_t soff)
{
    const uint64_t at = (uint64_t)off + soff;
    if (at + sizeof(V) > r.records) {
        std::fprintf(stderr, "buffer store out of the descriptor's range\n");
        std::abort();
    }
    std::memcpy(r.base + at, &v, sizeof(V));
}
#define __builtin_amdgcn_raw_buffer_store_b128(v, r, off, soff, aux) emu_buffer_store(v, r, off, soff)
#define __builtin_amdgcn_raw_buffer_store_b64(v, r, off, soff, aux) emu_buffer_store(v, r, off, soff)
#define __builtin_amdgcn_raw_buffer_store_b32(v, r, off, soff, aux) emu_buffer_store(v, r, off, soff)
#define __builtin_amdgcn_raw_buffer_store_b16(v, r, off, soff, aux) emu_buffer_store(v, r, off, soff)
struct hipPointerAttribute_t { int type; int device; };
struct hipDeviceProp_t { char gcnArchName[64]; int multiProcessorCount; };

struct dim3 { unsigned x, y, z; dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {} };
struct emu_idx { unsigned x, y, z; };
extern thread_local emu_idx blockIdx, threadIdx;
extern emu_idx blockDim, gridDim;
extern std::barrier<> *emu_bar;
inline void __syncthreads() { if (emu_bar) emu_bar->arrive_and_wait(); }
using std::min;
using std::max;

extern bool emu_capturing;
extern std::vector<std::function<void()>> emu_graph;
extern unsigned char emu_lds[1 << 18];
extern int emu_launches;
extern bool emu_threaded;  // run each block's threads as OS threads (barriers)

template <class K, class... A>
inline void emu_run(K k, dim3 g, dim3 b, A... a)
{
    emu_launches++;
    gridDim = {g.x, 1, 1};
    blockDim = {b.x, 1, 1};
    if (emu_threaded) {
        // one thread per lane for the whole launch; the workgroups run one
        // after another, all lanes meeting at a barrier between them
        std::barrier<> bar(b.x);
        emu_bar = &bar;
        std::vector<std::thread> th;
        for (unsigned t = 0; t < b.x; ++t)
            th.emplace_back([=, &bar]() {
                for (unsigned bi = 0; bi < g.x; ++bi) {
                    blockIdx = {bi, 0, 0};
                    threadIdx = {t, 0, 0};
                    k(a...);
                    bar.arrive_and_wait();
                }
            });
        for (auto &x : th) x.join();
        emu_bar = nullptr;
        return;
    }
    for (unsigned bi = 0; bi < g.x; ++bi)
        for (unsigned t = 0; t < b.x; ++t) {
            blockIdx = {bi, 0, 0};
            threadIdx = {t, 0, 0};
            k(a...);
        }
}

template <class K, class... A>
inline void emu_launch(K k, dim3 g, dim3 b, size_t shm, A... a)
{
    if (shm > (160u << 10)) {  // a compute unit's LDS
        std::fprintf(stderr, "launch with %zu bytes of dynamic LDS\n", shm);
        std::abort();
    }
    if (emu_capturing)
        emu_graph.push_back([=]() { emu_run(k, g, b, a...); });
    else
        emu_run(k, g, b, a...);
}
#define hipLaunchKernelGGL(K, G, B, SHM, ST, ...) emu_launch(K, G, B, SHM, __VA_ARGS__)

#define HIP_SYMBOL(x) (reinterpret_cast<const void *>(&(x)))
inline hipError_t hipGetSymbolAddress(void **p, const void *symbol) { *p = const_cast<void *>(symbol); return hipSuccess; }
inline hipError_t hipGetLastError() { return hipSuccess; }
inline const char *hipGetErrorString(hipError_t e) { return e ? "emu error" : "success"; }
inline hipError_t hipGetDevice(int *d) { *d = 0; return hipSuccess; }
template <class Q> inline hipError_t hipMalloc(Q **pp, size_t n) { void **p = (void **)pp; *p = std::aligned_alloc(256, (n + 255) / 256 * 256); return *p ? hipSuccess : hipErrorOutOfMemory; }
inline hipError_t hipFree(void *p) { std::free(p); return hipSuccess; }
inline hipError_t hipMemset(void *p, int v, size_t n) { std::memset(p, v, n); return hipSuccess; }
inline hipError_t hipMemsetD32Async(hipDeviceptr_t p, int v, size_t n, hipStream_t) { auto *q = (uint32_t *)p; for (size_t i = 0; i < n; ++i) q[i] = (uint32_t)v; return hipSuccess; }
inline hipError_t hipMemcpyAsync(void *d, const void *s, size_t n, int, hipStream_t) { std::memcpy(d, s, n); return hipSuccess; }
inline hipError_t hipMemcpy(void *d, const void *s, size_t n, int) { std::memcpy(d, s, n); return hipSuccess; }
inline hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
inline hipError_t hipPointerGetAttributes(hipPointerAttribute_t *a, const void *) { a->type = hipMemoryTypeDevice; a->device = 0; return hipSuccess; }
// three compute units: persistent grids loop several times and the
// Dslash walk's equal shares of (tile, slice) pairs cross tiles
inline hipError_t hipDeviceGetAttribute(int *v, int a, int) { *v = a == 1 ? 3 : (a == 2 ? 160 * 1024 : 64 * 1024); return hipSuccess; }
inline hipError_t hipGetDeviceProperties(hipDeviceProp_t *p, int) { std::strcpy(p->gcnArchName, "emu"); p->multiProcessorCount = 3; return hipSuccess; }
inline hipError_t hipEventCreate(hipEvent_t *e) { *e = nullptr; return hipSuccess; }
inline hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
inline hipError_t hipEventElapsedTime(float *ms, hipEvent_t, hipEvent_t) { *ms = 1.0f; return hipSuccess; }
inline hipError_t hipEventDestroy(hipEvent_t) { return hipSuccess; }
inline hipError_t hipStreamCreateWithFlags(hipStream_t *s, int) { *s = (void *)1; return hipSuccess; }
inline hipError_t hipStreamDestroy(hipStream_t) { return hipSuccess; }
inline hipError_t hipStreamBeginCapture(hipStream_t, int) { emu_capturing = true; emu_graph.clear(); return hipSuccess; }
inline hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t *g) { emu_capturing = false; *g = new std::vector<std::function<void()>>(emu_graph); return hipSuccess; }
inline hipError_t hipGraphInstantiate(hipGraphExec_t *e, hipGraph_t g, void *, void *, size_t) { *e = g; return hipSuccess; }
inline hipError_t hipGraphLaunch(hipGraphExec_t e, hipStream_t) { for (auto &f : *(std::vector<std::function<void()>> *)e) f(); return hipSuccess; }
inline hipError_t hipGraphExecDestroy(hipGraphExec_t) { return hipSuccess; }
inline hipError_t hipGraphDestroy(hipGraph_t g) { delete (std::vector<std::function<void()>> *)g; return hipSuccess; }
