// CPU stand-in for the subset of the HIP runtime that libnopcs uses, so the
// library's kernels can be compiled with g++ and AddressSanitizer and run on
// the host: every block runs as blockDim fibers that meet at __syncthreads;
// __shared__ arrays become function statics (one block runs at a time);
// device memory is host memory.  Test infrastructure only.
#pragma once
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <vector>
#include <sys/mman.h>
#include <unistd.h>
#include <map>
#include <mutex>

// Guarded allocation: the buffer sits between two PROT_NONE regions so that
// any access before its start or after its end (up to the guard size) faults.
inline std::map<void *, std::pair<void *, size_t>> &emu_allocs() {
    static std::map<void *, std::pair<void *, size_t>> m;
    return m;
}
inline std::mutex &emu_alloc_mu() {
    static std::mutex m;
    return m;
}
inline void *emu_guarded_alloc(size_t n) {
    const size_t pg = (size_t)sysconf(_SC_PAGESIZE), guard = (size_t)4 << 20;
    const size_t body = ((n ? n : 1) + pg - 1) / pg * pg;
    const size_t total = guard + body + guard;
    char *base = (char *)mmap(nullptr, total, PROT_READ | PROT_WRITE, MAP_PRIVATE | MAP_ANONYMOUS, -1, 0);
    if (base == MAP_FAILED) return nullptr;
    mprotect(base, guard, PROT_NONE);
    mprotect(base + guard + body, guard, PROT_NONE);
    // end of the buffer flush with the trailing guard: a read one byte past the
    // end faults.  The start then has the alignment of n within the page (a
    // state of an even number of points is 16-byte aligned, a workspace sized
    // in 256-byte units 256-byte aligned; the library rejects anything less).
    char *p = base + guard + body - n;
    std::lock_guard<std::mutex> lk(emu_alloc_mu());
    emu_allocs()[p] = {base, total};
    return p;
}
inline void emu_guarded_free(void *p) {
    if (!p) return;
    std::lock_guard<std::mutex> lk(emu_alloc_mu());
    auto it = emu_allocs().find(p);
    if (it != emu_allocs().end()) {
        munmap(it->second.first, it->second.second);
        emu_allocs().erase(it);
    }
}

#define __global__
#define __device__
#define __host__
#define __shared__ static
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __restrict__
#define __align__(n) __attribute__((aligned(n)))
#define HIP_SYMBOL(X) X

using std::max;
using std::min;
using std::sqrt;

struct dim3 {
    unsigned x = 1, y = 1, z = 1;
    dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};
struct int2 {
    int x, y;
};
inline int2 make_int2(int a, int b) { return int2{a, b}; }
struct alignas(16) double2 {
    double x, y;
};
inline double2 make_double2(double a, double b) { return double2{a, b}; }
struct alignas(8) float2 {
    float x, y;
};

// Device threads are fibers on the launching host thread (see emu_launch):
// the scheduler sets these before it resumes a fiber.
inline dim3 threadIdx, blockIdx;
inline dim3 gridDim, blockDim;
inline void emu_barrier();
inline void __syncthreads() { emu_barrier(); }

// Lane exchange inside a 64-wide wavefront: every thread of the block must call
// it the same number of times (as every lane of a wavefront does on the GPU).
inline double emu_shfl_buf[1024];
inline double __shfl_xor(double v, int mask, int width = 64) {
    const unsigned t = threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
    emu_shfl_buf[t] = v;
    emu_barrier();
    const unsigned lane = t % (unsigned)width, src = t - lane + ((lane ^ (unsigned)mask) % (unsigned)width);
    const double r = emu_shfl_buf[src];
    emu_barrier();
    return r;
}

// sin(pi x), cos(pi x) (host libm; the device function is more accurate)
inline void sincospi(double x, double *s, double *c) { *s = std::sin(M_PI * x); *c = std::cos(M_PI * x); }

typedef int hipError_t;
enum { hipSuccess = 0, hipErrorInvalidValue = 1, hipErrorOutOfMemory = 2 };
typedef void *hipStream_t;
typedef struct emu_event *hipEvent_t;
struct emu_event { std::chrono::steady_clock::time_point t; };
enum hipMemcpyKind { hipMemcpyHostToDevice, hipMemcpyDeviceToHost, hipMemcpyDeviceToDevice, hipMemcpyHostToHost,
                     hipMemcpyDefault };

inline const char *hipGetErrorString(hipError_t) { return "emulated HIP error"; }
inline hipError_t hipGetLastError() { return hipSuccess; }
inline hipError_t hipGetDevice(int *d) { *d = 0; return hipSuccess; }
inline hipError_t hipSetDevice(int) { return hipSuccess; }
inline hipError_t hipMalloc(void **p, size_t n) { *p = emu_guarded_alloc(n); return *p ? hipSuccess : hipErrorOutOfMemory; }
inline hipError_t hipFree(void *p) { emu_guarded_free(p); return hipSuccess; }
// stream-ordered allocation: work on a stream runs at once here (outside a capture)
inline hipError_t hipMallocAsync(void **p, size_t n, hipStream_t) { return hipMalloc(p, n); }
inline hipError_t hipFreeAsync(void *p, hipStream_t) { return hipFree(p); }
inline hipError_t hipMemcpy(void *d, const void *s, size_t n, hipMemcpyKind) { std::memcpy(d, s, n); return hipSuccess; }
inline hipError_t hipMemcpyAsync(void *d, const void *s, size_t n, hipMemcpyKind, hipStream_t);
inline hipError_t hipMemsetAsync(void *d, int v, size_t n, hipStream_t);
inline hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
enum { hipStreamNonBlocking = 1, hipEventDisableTiming = 2, hipErrorNotReady = 600 };
inline hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned) { *s = (hipStream_t) new char; return hipSuccess; }
inline hipError_t hipStreamDestroy(hipStream_t s) { delete (char *)s; return hipSuccess; }
inline hipError_t hipGetDeviceCount(int *n) { *n = 1; return hipSuccess; }
// a __device__ variable is a host variable here
template <class T>
inline hipError_t hipGetSymbolAddress(void **p, const T &sym) { *p = (void *)&sym; return hipSuccess; }
// Graphs: a capture records, on the capturing thread, every launch, copy and
// fill in issue order (whatever the stream: the library captures forked branch
// streams from that thread); a replay runs them in that order, which is one of
// the orders the captured dependencies allow.
#include <functional>
struct emu_graph { std::vector<std::function<void()>> ops; };
struct emu_graph_exec { std::vector<std::function<void()>> ops; };
typedef emu_graph *hipGraph_t;
typedef emu_graph_exec *hipGraphExec_t;
enum { hipStreamCaptureModeThreadLocal = 1, hipErrorNotSupported = 801, hipErrorIllegalState = 401 };
inline thread_local emu_graph *emu_capture = nullptr;
inline hipError_t hipStreamBeginCapture(hipStream_t, int) {
    if (emu_capture) return hipErrorIllegalState;
    emu_capture = new emu_graph();
    return hipSuccess;
}
inline hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t *g) {
    if (!emu_capture) return hipErrorIllegalState;
    *g = emu_capture;
    emu_capture = nullptr;
    return hipSuccess;
}
inline hipError_t hipGraphInstantiate(hipGraphExec_t *x, hipGraph_t g, void *, void *, size_t) {
    *x = new emu_graph_exec{g->ops};
    return hipSuccess;
}
inline hipError_t hipGraphLaunch(hipGraphExec_t x, hipStream_t) {
    if (emu_capture) return hipErrorNotSupported;
    for (auto &op : x->ops) op();
    return hipSuccess;
}
inline hipError_t hipGraphExecDestroy(hipGraphExec_t x) { delete x; return hipSuccess; }
inline hipError_t hipMemcpyAsync(void *d, const void *s, size_t n, hipMemcpyKind, hipStream_t) {
    if (emu_capture) emu_capture->ops.push_back([=] { std::memcpy(d, s, n); });
    else std::memcpy(d, s, n);
    return hipSuccess;
}
inline hipError_t hipMemsetAsync(void *d, int v, size_t n, hipStream_t) {
    if (emu_capture) emu_capture->ops.push_back([=] { std::memset(d, v, n); });
    else std::memset(d, v, n);
    return hipSuccess;
}
inline hipError_t hipGraphDestroy(hipGraph_t g) { delete g; return hipSuccess; }
inline hipError_t hipDeviceSynchronize() { return hipSuccess; }
inline hipError_t hipEventCreate(hipEvent_t *e) { *e = new emu_event(); return hipSuccess; }
inline hipError_t hipEventDestroy(hipEvent_t e) { delete e; return hipSuccess; }
inline hipError_t hipEventRecord(hipEvent_t e, hipStream_t) { e->t = std::chrono::steady_clock::now(); return hipSuccess; }
inline hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
inline hipError_t hipEventQuery(hipEvent_t) { return hipSuccess; }
inline hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned) { *e = new emu_event(); return hipSuccess; }
// every launch completes before it returns, so a wait on an event has nothing to wait for
inline hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t, unsigned) { return hipSuccess; }
inline hipError_t hipEventElapsedTime(float *ms, hipEvent_t a, hipEvent_t b) {
    *ms = std::chrono::duration<float, std::milli>(b->t - a->t).count();
    return hipSuccess;
}

// Device threads as fibers.  A launch runs its blocks one after the other on
// the calling host thread; the threads of a block are fibers (own stacks,
// switched by emu_ctx_switch, defined in driver.cpp) that a scheduler resumes
// in turn.  __syncthreads() switches back to the scheduler, which resumes a
// fiber again only after every live fiber of the block has reached the
// barrier, so block-wide barriers keep their meaning.  Launches from several
// host threads are serialised (the fibers' globals belong to one launch).
extern "C" void emu_ctx_switch(void **save_sp, void *new_sp);
#if defined(__SANITIZE_ADDRESS__)
extern "C" void __sanitizer_start_switch_fiber(void **fake_stack_save, const void *bottom, size_t size);
extern "C" void __sanitizer_finish_switch_fiber(void *fake_stack_save, const void **bottom_old, size_t *size_old);
extern "C" void __asan_unpoison_memory_region(void const volatile *addr, size_t size);
#endif

#if defined(__SANITIZE_THREAD__) && !defined(EMU_TSAN)
#define EMU_TSAN 1
#endif
#if defined(__has_feature)
#if __has_feature(thread_sanitizer) && !defined(EMU_TSAN)
#define EMU_TSAN 1
#endif
#endif
#if defined(EMU_TSAN)
extern "C" void *__tsan_get_current_fiber(void);
extern "C" void *__tsan_create_fiber(unsigned flags);
extern "C" void __tsan_destroy_fiber(void *fiber);
extern "C" void __tsan_switch_to_fiber(void *fiber, unsigned flags);
#endif

struct EmuFiber {
    void *tsan = nullptr;     // ThreadSanitizer's fiber of this device thread
    void *sp = nullptr;
    char *stack = nullptr;
    bool done = false;
    unsigned long nbar = 0;   // barriers reached
};
struct EmuSched {
#if defined(EMU_TSAN)
    static constexpr size_t kStack = (size_t)4 << 20;     // instrumented frames are larger
#else
    static constexpr size_t kStack = (size_t)512 << 10;
#endif
    std::mutex launch_mu;
    std::vector<EmuFiber> fib;
    void *sched_sp = nullptr;
    unsigned cur = 0;
    dim3 block;
    std::function<void()> body;
    const void *sched_bottom = nullptr;   // the scheduler's own stack (for the sanitizer)
    size_t sched_size = 0;
    void *sched_tsan = nullptr;           // ThreadSanitizer's fiber of the launching thread
    // switch from the running fiber to the scheduler; dying: the fiber never returns
    void to_sched(bool dying) {
#if defined(__SANITIZE_ADDRESS__)
        void *fake = nullptr;
        __sanitizer_start_switch_fiber(dying ? nullptr : &fake, sched_bottom, sched_size);
        emu_ctx_switch(&fib[cur].sp, sched_sp);
        __sanitizer_finish_switch_fiber(fake, nullptr, nullptr);
#elif defined(EMU_TSAN)
        (void)dying;
        __tsan_switch_to_fiber(sched_tsan, 0);
        emu_ctx_switch(&fib[cur].sp, sched_sp);
#else
        (void)dying;
        emu_ctx_switch(&fib[cur].sp, sched_sp);
#endif
    }
    // switch from the scheduler to fiber t
    void to_fiber(unsigned t) {
        cur = t;
        threadIdx = dim3(t % block.x, (t / block.x) % block.y, t / (block.x * block.y));
#if defined(__SANITIZE_ADDRESS__)
        void *fake = nullptr;
        __sanitizer_start_switch_fiber(&fake, fib[t].stack, kStack);
        emu_ctx_switch(&sched_sp, fib[t].sp);
        __sanitizer_finish_switch_fiber(fake, nullptr, nullptr);
#elif defined(EMU_TSAN)
        sched_tsan = __tsan_get_current_fiber();
        __tsan_switch_to_fiber(fib[t].tsan, 0);
        emu_ctx_switch(&sched_sp, fib[t].sp);
#else
        emu_ctx_switch(&sched_sp, fib[t].sp);
#endif
    }
    static void entry();
    // a fresh frame at the top of fiber t's stack that emu_ctx_switch "returns" into entry()
    void reset(unsigned t) {
        EmuFiber &f = fib[t];
        if (!f.stack) {
            f.stack = (char *)mmap(nullptr, kStack, PROT_READ | PROT_WRITE, MAP_PRIVATE | MAP_ANONYMOUS, -1, 0);
            if (f.stack == (char *)MAP_FAILED) std::abort();
            mprotect(f.stack, (size_t)sysconf(_SC_PAGESIZE), PROT_NONE);   // overflow guard
        }
#if defined(EMU_TSAN)
        // entry() never returns, so a fiber's shadow call stack would keep its
        // frames from one block to the next: a fresh sanitizer fiber per block
        if (f.tsan) __tsan_destroy_fiber(f.tsan);
        f.tsan = __tsan_create_fiber(0);
#endif
#if defined(__SANITIZE_ADDRESS__)
        __asan_unpoison_memory_region(f.stack, kStack);
#endif
        uint64_t *top = (uint64_t *)(f.stack + kStack);   // 16-byte aligned
        top[-1] = 0;                                        // entry() never returns
        top[-2] = (uint64_t)(uintptr_t)&EmuSched::entry;    // popped by ret
        for (int r = 3; r <= 8; ++r) top[-r] = 0;           // rbp, rbx, r12-r15
        top[-9] = 0x037F00001F80ull;                        // MXCSR (low), x87 control word
        f.sp = top - 9;
        f.done = false;
        f.nbar = 0;
    }
    void run_block(unsigned nt) {
        for (unsigned t = 0; t < nt; ++t) reset(t);
        // rounds: every live fiber runs up to its next barrier (or its end);
        // the fibers still alive after a round must all wait at the same barrier
        for (unsigned long round = 1;; ++round) {
            bool any = false;
            for (unsigned t = 0; t < nt; ++t) {
                if (fib[t].done) continue;
                to_fiber(t);
                if (fib[t].done) continue;
                any = true;
                if (fib[t].nbar != round) {
                    std::fprintf(stderr, "emulated block: thread %u at barrier %lu in round %lu\n", t, fib[t].nbar,
                                 round);
                    std::abort();
                }
            }
            if (!any) break;
        }
    }
};
inline EmuSched &emu_sched() {
    static EmuSched *s = new EmuSched();
    return *s;
}
inline void EmuSched::entry() {
    EmuSched &s = emu_sched();
#if defined(__SANITIZE_ADDRESS__)
    __sanitizer_finish_switch_fiber(nullptr, &s.sched_bottom, &s.sched_size);
#endif
    s.body();
    s.fib[s.cur].done = true;
    s.to_sched(true);
    std::abort();   // a finished fiber is never resumed
}
inline void emu_barrier() {
    EmuSched &s = emu_sched();
    ++s.fib[s.cur].nbar;
    s.to_sched(false);
}

template <class K, class... A>
void emu_launch_now(K kernel, dim3 grid, dim3 block, A... args);
template <class K, class... A>
void emu_launch(K kernel, dim3 grid, dim3 block, A... args) {
    if (emu_capture) {   // recorded with its arguments, run at each replay
        emu_capture->ops.push_back([=] { emu_launch_now(kernel, grid, block, args...); });
        return;
    }
    emu_launch_now(kernel, grid, block, args...);
}
template <class K, class... A>
void emu_launch_now(K kernel, dim3 grid, dim3 block, A... args) {
    // NOPCS_EMUL_HOST_ONLY=1: launches do nothing (host-side checks of the
    // runtime's own logic, e.g. under ThreadSanitizer; results are not computed)
    static const bool host_only = [] {
        const char *e = std::getenv("NOPCS_EMUL_HOST_ONLY");
        return e && e[0] == '1';
    }();
    if (host_only) return;
    EmuSched &s = emu_sched();
    std::lock_guard<std::mutex> serial(s.launch_mu);
    const unsigned nt = block.x * block.y * block.z;
    const unsigned nb = grid.x * grid.y * grid.z;
    if (s.fib.size() < nt) s.fib.resize(nt);
    gridDim = grid;
    blockDim = block;
    s.block = block;
    s.body = [&] { kernel(args...); };
    for (unsigned b = 0; b < nb; ++b) {
        blockIdx = dim3(b % grid.x, (b / grid.x) % grid.y, b / (grid.x * grid.y));
        s.run_block(nt);
    }
}
#define hipLaunchKernelGGL(K, G, B, SHM, ST, ...) emu_launch(K, G, B, __VA_ARGS__)
