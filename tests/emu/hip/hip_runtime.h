// Host emulation of the HIP subset libara uses, for the CPU tests of the
// kernels (tests/test_emu_kernels.py).  Test infrastructure only: the
// library's sources compile against this header with a host compiler, every
// GPU thread runs as a host thread, and a block's threads run concurrently.
//
// * Lanes of a wavefront run freely between synchronisation points.
//   wave_sync() (fence + wave barrier) and __syncthreads() are barriers that
//   order memory (acquire/release), so a missing one shows up as a data race
//   under ThreadSanitizer.  Cross-lane operations (ballot, shuffles,
//   readlane) exchange values through relaxed atomics: they order no memory,
//   as on the GPU, where they are not fences.
// * __shared__ arrays are function-static: blocks run one after another, and
//   each block starts with whatever the previous block left there.
// * Device memory is host memory (AddressSanitizer sees every access);
//   streams and events are synchronous.
#pragma once

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstddef>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <tuple>
#include <utility>

#define __global__
#define __device__
#define __constant__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __shared__ static
#define __align__(n) __attribute__((aligned(n)))
#define HIP_SYMBOL(x) ((const void*)&(x))
#define amdgpu_waves_per_eu(...)
#define amdgpu_flat_work_group_size(...)

inline int __float_as_int(float f) { int i; std::memcpy(&i, &f, 4); return i; }
inline unsigned __float_as_uint(float f) { unsigned i; std::memcpy(&i, &f, 4); return i; }
inline float __int_as_float(int i) { float f; std::memcpy(&f, &i, 4); return f; }
inline float __uint_as_float(unsigned i) { float f; std::memcpy(&f, &i, 4); return f; }
inline int min(int a, int b) { return a < b ? a : b; }
inline int max(int a, int b) { return a > b ? a : b; }
inline unsigned min(unsigned a, unsigned b) { return a < b ? a : b; }
inline unsigned max(unsigned a, unsigned b) { return a > b ? a : b; }
inline long min(long a, long b) { return a < b ? a : b; }
inline long max(long a, long b) { return a > b ? a : b; }
inline long long min(long long a, long long b) { return a < b ? a : b; }
inline long long max(long long a, long long b) { return a > b ? a : b; }

// ---------------------------------------------------------------- vector types
struct alignas(16) uint4 { uint32_t x, y, z, w; };
struct alignas(16) int4 { int32_t x, y, z, w; };
struct alignas(16) float4 { float x, y, z, w; };
struct alignas(8) float2 { float x, y; };
inline uint4 make_uint4(uint32_t x, uint32_t y, uint32_t z, uint32_t w) { return uint4{x, y, z, w}; }
inline int4 make_int4(int32_t x, int32_t y, int32_t z, int32_t w) { return int4{x, y, z, w}; }
inline float4 make_float4(float x, float y, float z, float w) { return float4{x, y, z, w}; }
inline float2 make_float2(float x, float y) { return float2{x, y}; }

struct dim3 {
    uint32_t x, y, z;
    dim3(uint32_t a = 1, uint32_t b = 1, uint32_t c = 1) : x(a), y(b), z(c) {}
};
extern thread_local dim3 blockIdx, blockDim, gridDim;
namespace emu {
dim3 thread_idx();                     // the running fiber's thread index
}
#define threadIdx (emu::thread_idx())

// ---------------------------------------------------------------- runtime API
typedef int hipError_t;
constexpr hipError_t hipSuccess = 0;
constexpr hipError_t hipErrorOutOfMemory = 2;
constexpr hipError_t hipErrorInvalidValue = 1;
typedef struct emu_stream* hipStream_t;
typedef struct emu_event* hipEvent_t;
enum hipMemcpyKind { hipMemcpyHostToHost = 0, hipMemcpyHostToDevice = 1, hipMemcpyDeviceToHost = 2,
                     hipMemcpyDeviceToDevice = 3, hipMemcpyDefault = 4 };
enum hipMemoryType { hipMemoryTypeHost = 0, hipMemoryTypeDevice = 1 };
struct hipPointerAttribute_t { hipMemoryType type; int device; void* devicePointer; void* hostPointer; };
constexpr unsigned hipHostMallocDefault = 0;
constexpr unsigned hipEventDisableTiming = 2;

hipError_t hipGetDeviceCount(int* n);
hipError_t hipSetDevice(int d);
hipError_t hipMalloc(void** p, size_t n);
hipError_t hipFree(void* p);
hipError_t hipHostMalloc(void** p, size_t n, unsigned flags = 0);
hipError_t hipHostFree(void* p);
hipError_t hipMemcpy(void* d, const void* s, size_t n, hipMemcpyKind k);
hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind k, hipStream_t st = nullptr);
hipError_t hipMemset(void* d, int v, size_t n);
hipError_t hipMemsetAsync(void* d, int v, size_t n, hipStream_t st = nullptr);
hipError_t hipStreamSynchronize(hipStream_t s);
hipError_t hipDeviceSynchronize();
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned flags);
hipError_t hipEventCreate(hipEvent_t* e);
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned flags);
hipError_t hipEventDestroy(hipEvent_t e);
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s = nullptr);
hipError_t hipEventSynchronize(hipEvent_t e);
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b);
hipError_t hipPointerGetAttributes(hipPointerAttribute_t* a, const void* p);
hipError_t hipGetSymbolAddress(void** p, const void* sym);
hipError_t hipGetLastError();
const char* hipGetErrorString(hipError_t e);

// ---------------------------------------------------------------- execution
namespace emu {
// Runs fn(arg) on grid.x blocks of block.x threads each (blocks one after
// another, the threads of a block concurrently).
void launch(dim3 grid, dim3 block, void (*thread_body)(void*), void* arg);
void wave_barrier();                  // orders memory within the wavefront
void block_barrier();                 // orders memory within the block
uint64_t exchange(uint64_t v, int src); // value of lane src (0..63) of this wavefront, no ordering
uint64_t ballot(bool p);
int lane();

template <typename T>
inline uint64_t bits_of(T v)
{
    static_assert(sizeof(T) <= 8, "exchange of at most 8 bytes");
    uint64_t u = 0;
    std::memcpy(&u, &v, sizeof(T));
    return u;
}
template <typename T>
inline T from_bits(uint64_t u)
{
    T v;
    std::memcpy(&v, &u, sizeof(T));
    return v;
}
template <typename F, typename Tuple, size_t... I>
inline void apply_kernel(F f, Tuple& t, std::index_sequence<I...>)
{
    f(std::get<I>(t)...);
}
}  // namespace emu

template <typename... KArgs, typename... Args>
inline void emu_launch_kernel(void (*k)(KArgs...), dim3 grid, dim3 block, Args&&... args)
{
    struct Pack {
        void (*k)(KArgs...);
        std::tuple<KArgs...> a;
    };
    Pack p{k, std::tuple<KArgs...>((KArgs)args...)};
    emu::launch(grid, block,
                [](void* v) {
                    Pack* q = (Pack*)v;
                    std::tuple<KArgs...> local = q->a;      // each thread takes its own copy of the arguments
                    emu::apply_kernel(q->k, local, std::index_sequence_for<KArgs...>{});
                },
                &p);
}
#define hipLaunchKernelGGL(k, grid, block, shmem, stream, ...) emu_launch_kernel(k, dim3(grid), dim3(block), ##__VA_ARGS__)

// ---------------------------------------------------------------- device builtins
inline void __syncthreads() { emu::block_barrier(); }
#define __builtin_amdgcn_wave_barrier() emu::wave_barrier()
#define __builtin_amdgcn_fence(order, scope) ((void)0)
#define __builtin_amdgcn_logf(x) log2f(x)
#define __builtin_amdgcn_rcpf(x) (1.0f / (x))
inline int emu_frexp_exp(float x)
{
    int e;
    frexpf(x, &e);
    return e;
}
#define __builtin_amdgcn_frexp_expf(x) emu_frexp_exp(x)
#define __builtin_amdgcn_readlane(v, i) ((int)emu::exchange((uint64_t)(uint32_t)(v), (i)))
#define __builtin_amdgcn_readfirstlane(v) ((int)emu::exchange((uint64_t)(uint32_t)(v), -1))

inline uint64_t __ballot(int p) { return emu::ballot(p != 0); }
template <typename T>
inline T __shfl(T v, int src, int width = 64)
{
    (void)width;
    return emu::from_bits<T>(emu::exchange(emu::bits_of(v), src & 63));
}
template <typename T>
inline T __shfl_up(T v, unsigned d, int width = 64)
{
    (void)width;
    const int l = emu::lane();
    const T o = emu::from_bits<T>(emu::exchange(emu::bits_of(v), l >= (int)d ? l - (int)d : l));
    return o;
}
template <typename T>
inline T __shfl_xor(T v, int m, int width = 64)
{
    (void)width;
    return emu::from_bits<T>(emu::exchange(emu::bits_of(v), (emu::lane() ^ m) & 63));
}
inline int __popcll(unsigned long long v) { return __builtin_popcountll(v); }
inline int __ffsll(long long v) { return __builtin_ffsll(v); }
inline int __ffsll(unsigned long long v) { return __builtin_ffsll((long long)v); }
inline float __expf(float x) { return expf(x); }
inline double normcdf(double x) { return 0.5 * erfc(-x * 0.70710678118654752440); }
// inverse of the normal CDF by bisection (slow, exact enough for tests)
inline double normcdfinv(double p)
{
    double lo = -40.0, hi = 40.0;
    for (int i = 0; i < 200; ++i) {
        const double m = 0.5 * (lo + hi);
        (normcdf(m) < p ? lo : hi) = m;
    }
    return 0.5 * (lo + hi);
}
inline float normcdfinvf(float p) { return (float)normcdfinv((double)p); }

template <typename T>
inline T atomicAdd(T* p, T v) { return __atomic_fetch_add(p, v, __ATOMIC_RELAXED); }
inline float atomicAdd(float* p, float v)
{
    uint32_t cur = __atomic_load_n((uint32_t*)p, __ATOMIC_RELAXED);
    for (;;) {
        float old;
        std::memcpy(&old, &cur, 4);
        const float nv = old + v;
        uint32_t nb;
        std::memcpy(&nb, &nv, 4);
        if (__atomic_compare_exchange_n((uint32_t*)p, &cur, nb, false, __ATOMIC_RELAXED, __ATOMIC_RELAXED)) return old;
    }
}
inline double atomicAdd(double* p, double v)
{
    uint64_t cur = __atomic_load_n((uint64_t*)p, __ATOMIC_RELAXED);
    for (;;) {
        double old;
        std::memcpy(&old, &cur, 8);
        const double nv = old + v;
        uint64_t nb;
        std::memcpy(&nb, &nv, 8);
        if (__atomic_compare_exchange_n((uint64_t*)p, &cur, nb, false, __ATOMIC_RELAXED, __ATOMIC_RELAXED)) return old;
    }
}
template <typename T>
inline T atomicMax(T* p, T v) { return __atomic_fetch_max(p, v, __ATOMIC_RELAXED); }
template <typename T>
inline T atomicCAS(T* p, T cmp, T v)
{
    __atomic_compare_exchange_n(p, &cmp, v, false, __ATOMIC_RELAXED, __ATOMIC_RELAXED);
    return cmp;
}

// v_mfma_f32_16x16x32_f16: D = A B + C for a 16 x 32 A, 32 x 16 B and 16 x 16
// C/D, with lane l (q = l / 16) holding A[l % 16][8q + t], B[8q + t][l % 16]
// and D[4q + r][l % 16] (t < 8, r < 4).
typedef _Float16 emu_h8 __attribute__((ext_vector_type(8)));
typedef float emu_f4 __attribute__((ext_vector_type(4)));
namespace emu {
emu_f4 mfma_16x16x32_f16(emu_h8 a, emu_h8 b, emu_f4 c);
}
inline emu_f4 emu_mfma_call(emu_h8 a, emu_h8 b, emu_f4 c, int, int, int) { return emu::mfma_16x16x32_f16(a, b, c); }
#define __builtin_amdgcn_mfma_f32_16x16x32_f16(...) emu_mfma_call(__VA_ARGS__)
