// batch.hpp -- one launch over many boxes.
//
// A stage kernel is written as a body, Body::run(args, b, nb), that does the
// work of block b of the nb blocks one box needs.  A single-box launch runs
// block b = xcd_swizzle(blockIdx.x, gridDim.x) of its own grid; a batched
// launch reads a device table with one entry per box (the box's arguments,
// its first item and its block count; each box's items padded to a multiple
// of 8 so that the XCD mapping inside a box is the single-box one), and each
// of its blocks takes one item (box, block of that box) of the table.  One
// launch per kernel thus covers every box of a batch.  (A persistent walk of
// the items by a fixed grid was compiled too: its loop around the body costs
// registers -- 175 instead of 166 VGPRs for the viscous kernel, 223 instead of
// 167 for the x sweep, one wave per SIMD fewer -- so every block takes one
// item.)  A box's blocks do exactly the arithmetic of its single-box launch,
// so its results do not depend on the other boxes of the batch.
#pragma once

#include <cstring>
#include <map>
#include <type_traits>
#include <vector>

#include "common.hpp"

namespace nopcs {

template <class A>
struct BatchItem {
    A a;          // the box's kernel arguments
    int start;    // the box's first item
    int count;    // blocks of the box (items start .. start + count - 1 do work)
};

// items of a box in a batch table: its block count rounded up to a multiple of 8
inline int batch_items(int count) { return (count + 7) & ~7; }

template <class Body>
__device__ inline void batch_walk(const BatchItem<typename Body::Args> *__restrict__ tab, int ntab) {
    const int item = blockIdx.x;
    int e = 0;   // the entry holding this item (scan of a few entries)
    while (e + 1 < ntab && tab[e + 1].start <= item) ++e;
    e = NOPCS_UNIFORM(e);
    const int local = item - tab[e].start, count = tab[e].count;
    if (local < count) {
        // a copy of the box's arguments: the table is read-only during the
        // launch, and loading every field before the body stores anything
        // keeps them uniform (scalar registers), as kernel arguments are
        const typename Body::Args a = tab[e].a;
        Body::run(a, xcd_swizzle(local, count), count);
    }
}

// Wavefronts per SIMD a body's kernels are compiled for (Body::kMinWaves, else
// 1): the register budget of each thread is the SIMD's file divided by it.
template <class B, class = void>
struct body_min_waves {
    static constexpr int value = 1;
};
template <class B>
struct body_min_waves<B, std::void_t<decltype(B::kMinWaves)>> {
    static constexpr int value = B::kMinWaves;
};

// Kernels running a body: one box (block b of its own grid), or a batch.
template <class Body, int NT>
__global__ __launch_bounds__(NT, body_min_waves<Body>::value) void k_one(typename Body::Args a) {
    Body::run(a, xcd_swizzle(blockIdx.x, gridDim.x), gridDim.x);
}
template <class Body, int NT>
__global__ __launch_bounds__(NT, body_min_waves<Body>::value) void k_many(
    const BatchItem<typename Body::Args> *__restrict__ tab, int ntab) {
    batch_walk<Body>(tab, ntab);
}

// ---------------------------------------------------------------------------
// Host side: collecting the launches of many boxes into batched launches.
// ---------------------------------------------------------------------------
// Launcher of one kernel instantiation over a device table (identifies the
// instantiation: launches of many boxes with the same launcher are merged).
using BatchLauncher = hipError_t (*)(const void *tab, int ntab, int total, dim3 blk, hipStream_t st);

struct BatchLaunch {
    BatchLauncher launch = nullptr;
    dim3 blk;
    size_t item_bytes = 0;
    std::vector<unsigned char> items;   // BatchItem<Args> of every box, packed
    int ntab = 0, total = 0;
    size_t dev_off = 0;                 // offset of the table in the batch's device buffer
};

// The launches of one batched RK4 step, grouped by phase: every launch of a
// phase may run in any order (each touches its own boxes), phases run in
// order.  A single-box launcher given a collector adds its box here instead
// of launching.
struct BatchCollector {
    std::map<int, std::vector<BatchLaunch>> phases;
    template <class Args>
    void add(int phase, BatchLauncher fn, dim3 blk, const Args &a, int count) {
        std::vector<BatchLaunch> &v = phases[phase];
        BatchLaunch *L = nullptr;
        for (BatchLaunch &x : v)
            if (x.launch == fn && x.blk.x == blk.x && x.blk.y == blk.y) { L = &x; break; }
        if (!L) {
            v.emplace_back();
            L = &v.back();
            L->launch = fn;
            L->blk = blk;
            L->item_bytes = sizeof(BatchItem<Args>);
        }
        BatchItem<Args> it;
        std::memset(static_cast<void *>(&it), 0, sizeof it);
        it.a = a;
        it.start = L->total;
        it.count = count;
        const size_t off = L->items.size();
        L->items.resize(off + sizeof it);
        std::memcpy(L->items.data() + off, &it, sizeof it);
        L->ntab += 1;
        L->total += batch_items(count);
    }
};

template <class Body, int NT>
hipError_t launch_many(const void *tab, int ntab, int total, dim3 blk, hipStream_t st) {
    hipLaunchKernelGGL((k_many<Body, NT>), dim3((unsigned)total), blk, 0, st,
                       static_cast<const BatchItem<typename Body::Args> *>(tab), ntab);
    return hipGetLastError();
}

// Launch `count` blocks of Body for one box, or add the box to a batch.
template <class Body, int NT>
hipError_t run_body(const typename Body::Args &a, int count, dim3 blk, hipStream_t st, BatchCollector *col,
                    int phase) {
    if (count <= 0) return hipSuccess;
    if (col) {
        col->add(phase, &launch_many<Body, NT>, blk, a, count);
        return hipSuccess;
    }
    hipLaunchKernelGGL((k_one<Body, NT>), dim3((unsigned)count), blk, 0, st, a);
    return hipGetLastError();
}

}  // namespace nopcs
