// Host emulation of the HIP runtime and of wavefront execution for the CPU
// tests of libara's kernels (see hip/hip_runtime.h in this directory).
#include <hip/hip_runtime.h>

#include <ucontext.h>

#include <cstdio>
#include <map>
#include <memory>
#include <mutex>
#include <vector>

#if defined(__has_feature)
#if __has_feature(thread_sanitizer)
#define EMU_TSAN 1
#endif
#if __has_feature(address_sanitizer)
#define EMU_ASAN 1
#endif
#endif
#ifdef EMU_TSAN
extern "C" {
void* __tsan_get_current_fiber(void);
void* __tsan_create_fiber(unsigned flags);
void __tsan_destroy_fiber(void* fiber);
void __tsan_switch_to_fiber(void* fiber, unsigned flags);
}
#endif
#ifdef EMU_ASAN
extern "C" {
void __sanitizer_start_switch_fiber(void** fake_stack_save, const void* bottom, size_t size);
void __sanitizer_finish_switch_fiber(void* fake_stack_save, const void** bottom_old, size_t* size_old);
}
#endif

thread_local dim3 blockIdx, blockDim, gridDim;

namespace emu {

// A block runs as one fiber per GPU thread, all on the calling OS thread.  A
// fiber runs until it reaches a barrier, then the scheduler resumes the next
// runnable fiber; a barrier opens once every live fiber of its scope (the
// wavefront, or the block) has reached it.  Under ThreadSanitizer each fiber
// is a thread of its own: switches at a memory-ordering barrier synchronise,
// switches at an exchange (ballot, shuffle, readlane) do not, so accesses
// that only an exchange separates are reported as races.
namespace {
constexpr size_t kStack = 1 << 20;

enum State { RUN, WAIT_WAVE_SYNC, WAIT_WAVE_XCHG, WAIT_BLOCK, DONE };

struct Fiber {
    ucontext_t ctx;
    char* stack = nullptr;
    int st = RUN;                      // State; accessed through ld/st below (scheduler and fiber both touch it)
    int tid = 0;
    void* tsan = nullptr;
};

struct BlockRun {
    std::vector<Fiber> f;
    ucontext_t sched;
    void* sched_tsan = nullptr;
    int nt = 0;
    int cur = -1;
    void (*body)(void*) = nullptr;
    void* arg = nullptr;
    dim3 grid, block, bidx;
    uint64_t slot[64 * 16];            // exchange values, per wavefront
    bool sync_switch = true;           // whether the current switch orders memory
};

thread_local BlockRun* t_run = nullptr;
thread_local std::vector<std::unique_ptr<char[]>> t_stacks;   // fiber stacks, reused by every block

// emulator bookkeeping shared between fibers and the scheduler: atomic, so it
// is never itself reported as a race
inline int ld(const int& v) { return __atomic_load_n(&v, __ATOMIC_RELAXED); }
inline void st_(int& v, int x) { __atomic_store_n(&v, x, __ATOMIC_RELAXED); }
inline uint64_t ld(const uint64_t& v) { return __atomic_load_n(&v, __ATOMIC_RELAXED); }
inline void st_(uint64_t& v, uint64_t x) { __atomic_store_n(&v, x, __ATOMIC_RELAXED); }
#ifdef EMU_ASAN
thread_local void* t_fake = nullptr;
thread_local const void* t_sched_bottom = nullptr;   // the scheduler's (OS thread's) stack
thread_local size_t t_sched_size = 0;
#endif

// to_stack null: the switch goes back to the scheduler
void switch_to(ucontext_t* from, ucontext_t* to, void* to_tsan, const void* to_stack, size_t to_size, bool sync)
{
#ifdef EMU_TSAN
    __tsan_switch_to_fiber(to_tsan, sync ? 0u : 1u);   // 1 = __tsan_switch_to_fiber_no_sync
#else
    (void)to_tsan;
    (void)sync;
#endif
#ifdef EMU_ASAN
    const bool to_sched = to_stack == nullptr;
    if (to_sched) __sanitizer_start_switch_fiber(&t_fake, t_sched_bottom, t_sched_size);
    else __sanitizer_start_switch_fiber(&t_fake, to_stack, to_size);
    swapcontext(from, to);
    // resumed: in a fiber (it had gone to the scheduler) or in the scheduler
    if (to_sched) __sanitizer_finish_switch_fiber(t_fake, &t_sched_bottom, &t_sched_size);
    else __sanitizer_finish_switch_fiber(t_fake, nullptr, nullptr);
#else
    (void)to_stack;
    (void)to_size;
    swapcontext(from, to);
#endif
}

// from a fiber back to the scheduler
void yield_to_scheduler(State st, bool sync)
{
    BlockRun& R = *t_run;
    Fiber& F = R.f[ld(R.cur)];
    st_(F.st, st);
    switch_to(&F.ctx, &R.sched, R.sched_tsan, nullptr, 0, sync);
}

void fiber_entry(unsigned lo, unsigned hi)
{
    (void)lo;
    (void)hi;
    BlockRun& R = *t_run;
#ifdef EMU_ASAN
    __sanitizer_finish_switch_fiber(t_fake, &t_sched_bottom, &t_sched_size);
#endif
    R.body(R.arg);
    yield_to_scheduler(DONE, true);
}

bool all_at(BlockRun& R, int lo, int hi, State st)
{
    bool any = false;
    for (int i = lo; i < hi; ++i) {
        if (ld(R.f[i].st) == DONE) continue;
        if (ld(R.f[i].st) != st) return false;
        any = true;
    }
    return any;
}
}  // namespace

int lane() { return ld(t_run->cur) & 63; }
dim3 thread_idx() { return dim3((uint32_t)ld(t_run->cur), 0, 0); }

void wave_barrier() { yield_to_scheduler(WAIT_WAVE_SYNC, true); }
void block_barrier() { yield_to_scheduler(WAIT_BLOCK, true); }

uint64_t exchange(uint64_t v, int src)
{
    BlockRun& R = *t_run;
    const int me = ld(R.cur), w0 = me & ~63;
    st_(R.slot[me], v);
    yield_to_scheduler(WAIT_WAVE_XCHG, false);
    const uint64_t r = ld(R.slot[w0 + (src < 0 ? 0 : src)]);
    yield_to_scheduler(WAIT_WAVE_XCHG, false);
    return r;
}

uint64_t ballot(bool p)
{
    BlockRun& R = *t_run;
    const int me = ld(R.cur), w0 = me & ~63;
    st_(R.slot[me], (uint64_t)(p ? 1u : 0u));
    yield_to_scheduler(WAIT_WAVE_XCHG, false);
    uint64_t m = 0;
    for (int i = w0; i < std::min(w0 + 64, R.nt); ++i)
        if (ld(R.f[i].st) != DONE && ld(R.slot[i])) m |= 1ull << (i - w0);
    yield_to_scheduler(WAIT_WAVE_XCHG, false);
    return m;
}

emu_f4 mfma_16x16x32_f16(emu_h8 a, emu_h8 b, emu_f4 c)
{
    // gather every lane's fragments, then form this lane's four outputs
    float A[16][32], B[32][16];
    for (int t = 0; t < 8; ++t) {
        const uint64_t ab = (uint64_t)bits_of((float)a[t]) | ((uint64_t)bits_of((float)b[t]) << 32);
        for (int src = 0; src < 64; ++src) {
            const uint64_t o = exchange(ab, src);
            const int q = src >> 4, i = src & 15;
            A[i][8 * q + t] = from_bits<float>((uint32_t)o);
            B[8 * q + t][i] = from_bits<float>((uint32_t)(o >> 32));
        }
    }
    const int q = lane() >> 4, col = lane() & 15;
    emu_f4 d;
    for (int r = 0; r < 4; ++r) {
        float s = c[r];
        for (int k = 0; k < 32; ++k) s += A[4 * q + r][k] * B[k][col];
        d[r] = s;
    }
    return d;
}

void launch(dim3 grid, dim3 block, void (*body)(void*), void* arg)
{
    const int nt = (int)block.x;
    if (nt > 64 * 16) {
        std::fprintf(stderr, "emu: blocks of more than 1024 threads\n");
        std::abort();
    }
    for (uint32_t bz = 0; bz < grid.z; ++bz)
        for (uint32_t by = 0; by < grid.y; ++by)
            for (uint32_t bx = 0; bx < grid.x; ++bx) {
                BlockRun R;
                R.nt = nt;
                R.body = body;
                R.arg = arg;
                R.f.resize(nt);
                BlockRun* prev = t_run;
                t_run = &R;
                blockIdx = dim3(bx, by, bz);
                blockDim = block;
                gridDim = grid;
#ifdef EMU_TSAN
                R.sched_tsan = __tsan_get_current_fiber();
#endif
                while ((int)t_stacks.size() < nt) t_stacks.emplace_back(new char[kStack]);
                for (int t = 0; t < nt; ++t) {
                    Fiber& F = R.f[t];
                    F.tid = t;
                    F.stack = t_stacks[t].get();
                    getcontext(&F.ctx);
                    F.ctx.uc_stack.ss_sp = F.stack;
                    F.ctx.uc_stack.ss_size = kStack;
                    F.ctx.uc_link = nullptr;
                    makecontext(&F.ctx, (void (*)())fiber_entry, 2, 0u, 0u);
#ifdef EMU_TSAN
                    F.tsan = __tsan_create_fiber(0);
#endif
                }
                // round-robin over runnable fibers; open barriers whose scope has fully arrived
                for (;;) {
                    bool progressed = false, live = false;
                    for (int t = 0; t < nt; ++t) {
                        Fiber& F = R.f[t];
                        if (ld(F.st) == DONE) continue;
                        live = true;
                        if (ld(F.st) != RUN) continue;
                        st_(R.cur, t);
                        switch_to(&R.sched, &F.ctx, F.tsan, F.stack, kStack, true);
                        progressed = true;
                    }
                    if (!live) break;
                    for (int w0 = 0; w0 < nt; w0 += 64) {
                        const int w1 = std::min(w0 + 64, nt);
                        for (State st : {WAIT_WAVE_SYNC, WAIT_WAVE_XCHG})
                            if (all_at(R, w0, w1, st)) {
                                for (int i = w0; i < w1; ++i)
                                    if (ld(R.f[i].st) == st) st_(R.f[i].st, RUN);
                                progressed = true;
                            }
                    }
                    if (all_at(R, 0, nt, WAIT_BLOCK)) {
                        for (int i = 0; i < nt; ++i)
                            if (ld(R.f[i].st) == WAIT_BLOCK) st_(R.f[i].st, RUN);
                        progressed = true;
                    }
                    if (!progressed) {
                        std::fprintf(stderr, "emu: block %u deadlocked: lanes wait at different barriers\n", bx);
                        for (int i = 0; i < nt; ++i) std::fprintf(stderr, " %d", ld(R.f[i].st));
                        std::fprintf(stderr, "\n");
                        std::abort();
                    }
                }
#ifdef EMU_TSAN
                for (auto& F : R.f) __tsan_destroy_fiber(F.tsan);
#endif
                t_run = prev;
            }
}

}  // namespace emu

// ---------------------------------------------------------------- runtime API
namespace {
std::mutex g_mu;
std::map<uintptr_t, size_t> g_dev;     // device allocations: start -> size
hipError_t g_last = hipSuccess;
struct emu_event_rec { int dummy; };
}  // namespace
struct emu_event : emu_event_rec {};

hipError_t hipGetDeviceCount(int* n) { *n = 1; return hipSuccess; }
hipError_t hipSetDevice(int d) { return d == 0 ? hipSuccess : hipErrorInvalidValue; }
hipError_t hipMalloc(void** p, size_t n)
{
    *p = std::malloc(n ? n : 1);
    if (!*p) return hipErrorOutOfMemory;
    std::lock_guard<std::mutex> g(g_mu);
    g_dev[(uintptr_t)*p] = n;
    return hipSuccess;
}
hipError_t hipFree(void* p)
{
    if (!p) return hipSuccess;
    {
        std::lock_guard<std::mutex> g(g_mu);
        g_dev.erase((uintptr_t)p);
    }
    std::free(p);
    return hipSuccess;
}
hipError_t hipHostMalloc(void** p, size_t n, unsigned) { *p = std::malloc(n ? n : 1); return *p ? hipSuccess : hipErrorOutOfMemory; }
hipError_t hipHostFree(void* p) { std::free(p); return hipSuccess; }
hipError_t hipMemcpy(void* d, const void* s, size_t n, hipMemcpyKind) { if (n) std::memmove(d, s, n); return hipSuccess; }
hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind k, hipStream_t) { return hipMemcpy(d, s, n, k); }
hipError_t hipMemset(void* d, int v, size_t n) { if (n) std::memset(d, v, n); return hipSuccess; }
hipError_t hipMemsetAsync(void* d, int v, size_t n, hipStream_t) { return hipMemset(d, v, n); }
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipDeviceSynchronize() { return hipSuccess; }
hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t, unsigned) { return hipSuccess; }
hipError_t hipEventCreate(hipEvent_t* e) { *e = new emu_event(); return hipSuccess; }
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { return hipEventCreate(e); }
hipError_t hipEventDestroy(hipEvent_t e) { delete e; return hipSuccess; }
hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
hipError_t hipEventElapsedTime(float* ms, hipEvent_t, hipEvent_t) { *ms = 0.0f; return hipSuccess; }
hipError_t hipPointerGetAttributes(hipPointerAttribute_t* a, const void* p)
{
    std::lock_guard<std::mutex> g(g_mu);
    auto it = g_dev.upper_bound((uintptr_t)p);
    a->type = hipMemoryTypeHost;
    if (it != g_dev.begin()) {
        --it;
        if ((uintptr_t)p < it->first + std::max<size_t>(it->second, 1)) a->type = hipMemoryTypeDevice;
    }
    a->device = 0;
    a->devicePointer = const_cast<void*>(p);
    a->hostPointer = nullptr;
    return hipSuccess;
}
hipError_t hipGetSymbolAddress(void** p, const void* sym) { *p = const_cast<void*>(sym); return hipSuccess; }
hipError_t hipGetLastError() { hipError_t e = g_last; g_last = hipSuccess; return e; }
const char* hipGetErrorString(hipError_t e) { return e == hipSuccess ? "no error" : "emulated HIP error"; }
