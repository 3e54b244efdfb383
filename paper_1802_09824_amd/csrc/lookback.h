// Single-pass prefix sums over the workgroups of one kernel (decoupled
// look-back), shared by the scan kernels (scan.hip) and the list builder's
// one-pass stages (tree.hip).
//
// A workgroup takes its tile number from a ticket counter, so every tile it
// may wait for has already started and publishes without waiting itself.
// Per summed quantity a tile publishes one 64-bit word: (aggregate << 2) | 1,
// later (inclusive prefix << 2) | 2; 0 means not yet published.  The ticket
// and every word sit on cache lines of their own (kLbWordStride words
// apart), so that a tile's publishes and its neighbours' polls do not
// contend for one line.  A word is
// read and written whole by agent-scope atomics, so a value and its flag are
// never seen apart.  The workspace holds two regions (a ticket, then the
// words), used by consecutive kernels in turn: a region is zero when a
// kernel starts in it, because every such kernel clears the other region
// (the one its predecessor used and its successor will use).  A wait that
// does not end within kLbSpins polls gives up and sets overflow bit 6 of the
// count slots (when given), so that the call fails instead of hanging.
#pragma once
#include "pp_internal.h"

namespace pp {

constexpr int kLbSpins = 1 << 22;
constexpr int kLbWordStride = 16;

// One kernel's share of the workspace: its region (ticket, then words) and
// the region it clears.
struct LbArgs {
    unsigned long long* cur;
    unsigned long long* other;
    int64_t nclear;
};

__device__ __forceinline__ void lb_publish(unsigned long long* w, int64_t v, unsigned st) {
    __hip_atomic_store(w, ((unsigned long long)v << 2) | st, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Grid-stride clear of the other region.
__device__ __forceinline__ void lb_clear_other(const LbArgs& lb) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = g; i < lb.nclear; i += stride) lb.other[i] = 0ull;
}

// Exclusive prefix of `tile` for quantity c of NV, walked back by a whole
// wave after the tile's aggregate was published: each lane reads one of the
// 64 nearest earlier tiles (lane 0 the nearest), waits until it is
// published, and the wave adds the words up to the nearest inclusive one;
// with none among them it adds all 64 and moves 64 tiles further back.
// Tiles before the first count as an inclusive zero.
template <int NV>
__device__ int64_t lb_walk_back(const unsigned long long* words, int64_t tile, int c, int64_t* sizes,
                                int lane) {
    int64_t excl = 0;
    for (int64_t j = tile - 1;; j -= 64) {
        const int64_t k = j - lane;
        unsigned long long w = 2ull;
        if (k >= 0) {
            for (int spin = 0;; ++spin) {
                w = __hip_atomic_load(words + (k * NV + c) * kLbWordStride, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (w & 3ull) break;
                if (spin > kLbSpins) {
                    if (sizes) atomicOr(reinterpret_cast<unsigned long long*>(sizes + kOverflow), 64ull);
                    w = 2ull;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        const unsigned long long incl = __ballot((w & 3ull) == 2ull);
        const int stop = incl ? __builtin_ctzll(incl) : 64;
        int64_t v = lane <= stop ? (int64_t)(w >> 2) : 0;
        for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d);
        excl += v;
        if (incl) return excl;
    }
}

// One wave of a tile: publishes the tile's aggregate agg (quantity c of NV),
// walks back, publishes the inclusive prefix and returns the exclusive one
// (the same in every lane).
template <int NV>
__device__ int64_t lb_tile_prefix(const LbArgs& lb, int64_t tile, int c, int64_t agg, int64_t* sizes,
                                  int lane) {
    unsigned long long* words = lb.cur + kLbWordStride;
    unsigned long long* w = words + (tile * NV + c) * kLbWordStride;
    if (tile == 0) {
        if (lane == 0) lb_publish(w, agg, 2u);
        return 0;
    }
    if (lane == 0) lb_publish(w, agg, 1u);
    const int64_t ex = lb_walk_back<NV>(words, tile, c, sizes, lane);
    if (lane == 0) lb_publish(w, ex + agg, 2u);
    return ex;
}

// Host side (scan.hip): makes the workspace hold two regions of at least
// `words` words plus the ticket each, a line apart (fresh memory is cleared
// on s).
int grow_lookback(DevBuf& ws, int64_t words, hipStream_t s);
// The regions of the next kernel that uses the workspace, which must hold
// `words` words per region (grown beforehand); flips the region for the
// kernel after it.
int lookback_args(DevBuf& ws, int64_t words, LbArgs* out);

}  // namespace pp
