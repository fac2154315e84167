// CPU stand-in for the subset of the HIP runtime that libnopcs uses, so the
// library's kernels can be compiled with g++ and AddressSanitizer and run on
// the host: every block runs as blockDim threads that meet at a std::barrier
// for __syncthreads; __shared__ arrays become function statics (one block runs
// at a time); device memory is host memory.  Test infrastructure only.
#pragma once
#include <algorithm>
#include <barrier>
#include <chrono>
#include <condition_variable>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <thread>
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
    // end of the buffer flush with the trailing guard, start kept 256-byte aligned
    char *p = base + guard + body - ((n + 255) & ~(size_t)255);
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

inline thread_local dim3 threadIdx, blockIdx;
inline dim3 gridDim, blockDim;   // written by every pool thread of a launch with the same value
inline thread_local std::barrier<> *emu_bar = nullptr;
inline void __syncthreads() { emu_bar->arrive_and_wait(); }

// Lane exchange inside a 64-wide wavefront: every thread of the block must call
// it the same number of times (as every lane of a wavefront does on the GPU).
inline double emu_shfl_buf[1024];
inline double __shfl_xor(double v, int mask, int width = 64) {
    const unsigned t = threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
    emu_shfl_buf[t] = v;
    emu_bar->arrive_and_wait();
    const unsigned lane = t % (unsigned)width, src = t - lane + ((lane ^ (unsigned)mask) % (unsigned)width);
    const double r = emu_shfl_buf[src];
    emu_bar->arrive_and_wait();
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
inline hipError_t hipMemcpy(void *d, const void *s, size_t n, hipMemcpyKind) { std::memcpy(d, s, n); return hipSuccess; }
inline hipError_t hipMemcpyAsync(void *d, const void *s, size_t n, hipMemcpyKind, hipStream_t) { std::memcpy(d, s, n); return hipSuccess; }
inline hipError_t hipMemsetAsync(void *d, int v, size_t n, hipStream_t) { std::memset(d, v, n); return hipSuccess; }
inline hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
enum { hipStreamNonBlocking = 1, hipEventDisableTiming = 2, hipErrorNotReady = 600 };
inline hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned) { *s = (hipStream_t) new char; return hipSuccess; }
inline hipError_t hipStreamDestroy(hipStream_t s) { delete (char *)s; return hipSuccess; }
inline hipError_t hipGetDeviceCount(int *n) { *n = 1; return hipSuccess; }
// graphs: not available in the host build (capture reports an error; nothing is launched)
typedef struct emu_graph *hipGraph_t;
typedef struct emu_graph_exec *hipGraphExec_t;
enum { hipStreamCaptureModeThreadLocal = 1, hipErrorNotSupported = 801 };
inline hipError_t hipStreamBeginCapture(hipStream_t, int) { return hipErrorNotSupported; }
inline hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t *g) { *g = nullptr; return hipErrorNotSupported; }
inline hipError_t hipGraphInstantiate(hipGraphExec_t *, hipGraph_t, void *, void *, size_t) { return hipErrorNotSupported; }
inline hipError_t hipGraphLaunch(hipGraphExec_t, hipStream_t) { return hipErrorNotSupported; }
inline hipError_t hipGraphExecDestroy(hipGraphExec_t) { return hipSuccess; }
inline hipError_t hipGraphDestroy(hipGraph_t) { return hipSuccess; }
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

// A pool of host threads that play the device threads of one block at a time;
// created once and reused by every launch (launches from several host threads
// are serialised).
struct EmuPool {
    std::mutex mu, launch_mu;
    std::condition_variable cv, cv_done;
    std::vector<std::thread> th;
    std::function<void(unsigned)> job;
    unsigned job_nt = 0, active = 0;
    unsigned long long gen = 0;
    void loop(unsigned id) {
        unsigned long long seen = 0;
        for (;;) {
            std::function<void(unsigned)> f;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv.wait(lk, [&] { return gen != seen; });
                seen = gen;
                if (id >= job_nt) continue;
                f = job;
            }
            f(id);
            std::lock_guard<std::mutex> lk(mu);
            if (--active == 0) cv_done.notify_all();
        }
    }
    void run(unsigned nt, std::function<void(unsigned)> f) {
        std::lock_guard<std::mutex> serial(launch_mu);
        std::unique_lock<std::mutex> lk(mu);
        while (th.size() < nt) {
            const unsigned id = (unsigned)th.size();
            th.emplace_back([this, id] { loop(id); });
            th.back().detach();
        }
        job = std::move(f);
        job_nt = nt;
        active = nt;
        ++gen;
        cv.notify_all();
        cv_done.wait(lk, [&] { return active == 0; });
    }
};
inline EmuPool &emu_pool() {
    static EmuPool *p = new EmuPool();   // never destroyed: detached threads outlive main
    return *p;
}

template <class K, class... A>
void emu_launch(K kernel, dim3 grid, dim3 block, A... args) {
    const unsigned nt = block.x * block.y * block.z;
    const unsigned nb = grid.x * grid.y * grid.z;
    // blocks run one after the other, separated by a barrier so that
    // block-shared (static) arrays are reused safely
    std::barrier<> bar((std::ptrdiff_t)nt);
    emu_pool().run(nt, [&](unsigned t) {
        gridDim = grid;
        blockDim = block;
        threadIdx = dim3(t % block.x, (t / block.x) % block.y, t / (block.x * block.y));
        emu_bar = &bar;
        for (unsigned b = 0; b < nb; ++b) {
            blockIdx = dim3(b % grid.x, (b / grid.x) % grid.y, b / (grid.x * grid.y));
            kernel(args...);
            bar.arrive_and_wait();
        }
    });
}
#define hipLaunchKernelGGL(K, G, B, SHM, ST, ...) emu_launch(K, G, B, __VA_ARGS__)
