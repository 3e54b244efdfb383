// Single-pass exclusive scans of int32 counts into int64 offsets (decoupled
// look-back), used by every stage that turns per-item counts into output
// positions.
//
// A workgroup sums a tile of kScanTile counts.  It takes its tile number
// from a ticket counter, so every tile it may wait for has already started
// and publishes without waiting itself.  Per scanned array it publishes one
// 64-bit word: (aggregate << 2) | 1, later (inclusive prefix << 2) | 2;
// 0 means not yet published.  Its exclusive prefix is the sum of the words
// of the tiles before it, walked back to the first inclusive one.  A word
// is read and written whole by agent-scope atomics, so a value and its flag
// are never seen apart.
//
// Workspace (uint64): two regions, each a ticket and the words, used by
// consecutive scans in turn.  A region is zero whenever a scan starts in it:
// both are cleared when allocated, and every scan clears the other region
// (the one its predecessor used, and its successor will use).  A wait that
// does not end within kSpins polls gives up and sets overflow bit 6 of the
// count slots (when given), so that the call fails instead of hanging.
#include "pp_internal.h"

namespace pp {
namespace {

constexpr int kScanWG = 256;
constexpr int kScanIPT = 8;
constexpr int64_t kScanTile = (int64_t)kScanWG * kScanIPT;
constexpr int kSpins = 1 << 22;

struct ScanIO {
    const int32_t* in[2];
    int64_t* out[2];
};

__device__ __forceinline__ void publish(unsigned long long* w, int64_t v, unsigned st) {
    __hip_atomic_store(w, ((unsigned long long)v << 2) | st, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Exclusive prefix of `tile` for array c of NV, walked back by a whole wave
// after the tile's aggregate was published: each lane reads one of the 64
// nearest earlier tiles (lane 0 the nearest), waits until it is published,
// and the wave adds the words up to the nearest inclusive one; with none
// among them it adds all 64 and moves 64 tiles further back.  Tiles before
// the first count as an inclusive zero.
template <int NV>
__device__ int64_t walk_back(const unsigned long long* words, int64_t tile, int c, int64_t* sizes,
                             int lane) {
    int64_t excl = 0;
    for (int64_t j = tile - 1;; j -= 64) {
        const int64_t k = j - lane;
        unsigned long long w = 2ull;
        if (k >= 0) {
            for (int spin = 0;; ++spin) {
                w = __hip_atomic_load(words + k * NV + c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (w & 3ull) break;
                if (spin > kSpins) {
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

// out[c][i] = sum of in[c][0 .. i) for i in [0, n]; ntile = tiles over n + 1.
// `cur` is this scan's region (ticket, then words), `other` the region to
// clear (nclear words).  The tile's counts come in and its offsets go out
// through LDS, so that the global loads and stores of a wave are contiguous
// while every thread scans kScanIPT consecutive counts.
template <int NV>
__global__ __launch_bounds__(kScanWG) void scan_counts_kernel(ScanIO io, int64_t n,
                                                              unsigned long long* cur,
                                                              unsigned long long* other, int64_t nclear,
                                                              int64_t* sizes) {
    __shared__ int32_t s_in[NV][kScanTile];
    __shared__ int64_t s_out[NV][kScanTile];
    __shared__ unsigned s_tile;
    __shared__ int64_t s_wave[NV][kScanWG / 64];
    __shared__ int64_t s_pre[NV];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    unsigned long long* words = cur + 1;
    for (int64_t i = (int64_t)blockIdx.x * kScanWG + t; i < nclear; i += (int64_t)gridDim.x * kScanWG)
        other[i] = 0ull;
    if (t == 0) s_tile = (unsigned)atomicAdd(cur, 1ull);
    __syncthreads();
    const int64_t tile = s_tile;
    const int64_t t0 = tile * kScanTile;
    if (t0 + kScanTile <= n) {           // a full tile: all loads issued before any is used
        int32_t r[NV][kScanIPT];
#pragma unroll
        for (int c = 0; c < NV; ++c)
#pragma unroll
            for (int k = 0; k < kScanIPT; ++k) r[c][k] = io.in[c][t0 + k * kScanWG + t];
#pragma unroll
        for (int c = 0; c < NV; ++c)
#pragma unroll
            for (int k = 0; k < kScanIPT; ++k) s_in[c][k * kScanWG + t] = r[c][k];
    } else {
#pragma unroll
        for (int c = 0; c < NV; ++c)
            for (int k = 0; k < kScanIPT; ++k) {
                const int64_t i = t0 + k * kScanWG + t;
                s_in[c][k * kScanWG + t] = i < n ? io.in[c][i] : 0;
            }
    }
    __syncthreads();
    int32_t v[NV][kScanIPT];
    int64_t tsum[NV], inc[NV];
#pragma unroll
    for (int c = 0; c < NV; ++c) {
        tsum[c] = 0;
#pragma unroll
        for (int k = 0; k < kScanIPT; ++k) {
            v[c][k] = s_in[c][t * kScanIPT + k];
            tsum[c] += v[c][k];
        }
        inc[c] = tsum[c];
    }
    for (int d = 1; d < 64; d <<= 1) {
#pragma unroll
        for (int c = 0; c < NV; ++c) {
            const int64_t u = __shfl_up(inc[c], d);
            if (lane >= d) inc[c] += u;
        }
    }
    if (lane == 63) {
#pragma unroll
        for (int c = 0; c < NV; ++c) s_wave[c][wave] = inc[c];
    }
    __syncthreads();
    if (wave < NV) {                     // wave c looks back for array c
        const int c = wave;
        int64_t agg = 0;
        for (int k = 0; k < kScanWG / 64; ++k) agg += s_wave[c][k];
        unsigned long long* w = words + tile * NV + c;
        int64_t ex = 0;
        if (tile == 0) {
            if (lane == 0) publish(w, agg, 2u);
        } else {
            if (lane == 0) publish(w, agg, 1u);
            ex = walk_back<NV>(words, tile, c, sizes, lane);
            if (lane == 0) publish(w, ex + agg, 2u);
        }
        if (lane == 0) s_pre[c] = ex;
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < NV; ++c) {
        int64_t run = s_pre[c] + inc[c] - tsum[c];
        for (int k = 0; k < wave; ++k) run += s_wave[c][k];
#pragma unroll
        for (int k = 0; k < kScanIPT; ++k) {
            s_out[c][t * kScanIPT + k] = run;
            run += v[c][k];
        }
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < NV; ++c)
#pragma unroll
        for (int k = 0; k < kScanIPT; ++k) {
            const int64_t i = t0 + k * kScanWG + t;
            if (i <= n) io.out[c][i] = s_out[c][k * kScanWG + t];
        }
}

__global__ void scan_clear_kernel(unsigned long long* p, int64_t n) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = g; i < n; i += stride) p[i] = 0ull;
}

__global__ void set_zero2_kernel(int64_t* a, int64_t* b) {
    if (a) *a = 0;
    if (b) *b = 0;
}

int64_t tiles_for(int64_t n) { return (n + 1 + kScanTile - 1) / kScanTile; }

template <int NV>
int launch(const ScanIO& io, int64_t n, DevBuf& ws, hipStream_t s, int64_t* sizes) {
    if (n == 0) {
        hipLaunchKernelGGL(set_zero2_kernel, dim3(1), dim3(1), 0, s, io.out[0], NV > 1 ? io.out[1] : nullptr);
        PP_HIP(hipGetLastError());
        return PP_OK;
    }
    PP_TRY(grow_scan(ws, NV * n, s));
    const int64_t nt = tiles_for(n);
    const int64_t region = (int64_t)(ws.bytes / sizeof(unsigned long long)) / 2;
    unsigned long long* base = ws.as<unsigned long long>();
    if (1 + nt * NV > region) return fail(PP_EDEVICE, "scan workspace smaller than its tiles");
    const uint32_t r = ws.tag & 1u;             // the region this scan uses
    hipLaunchKernelGGL(scan_counts_kernel<NV>, dim3((unsigned)nt), dim3(kScanWG), 0, s, io, n,
                       base + r * region, base + (1 - r) * region, region, sizes);
    PP_HIP(hipGetLastError());
    ws.tag ^= 1u;
    return PP_OK;
}

}  // namespace

int scan_workspace(int64_t n, size_t* bytes) {
    // two regions of a ticket and one word per tile (two arrays take n = 2 x count)
    *bytes = 2 * sizeof(unsigned long long) * (size_t)(1 + tiles_for(n) + 2);
    return PP_OK;
}

int grow_scan(DevBuf& buf, int64_t n, hipStream_t s) {
    size_t need = 0;
    PP_TRY(scan_workspace(n, &need));
    const uint64_t gen = alloc_generation();
    PP_TRY(buf.reserve(need));
    if (alloc_generation() != gen) {            // fresh memory: clear all of it
        const int64_t m = (int64_t)(buf.bytes / sizeof(unsigned long long));
        const int64_t g = (m + 255) / 256;
        hipLaunchKernelGGL(scan_clear_kernel, dim3((unsigned)(g < 1 ? 1 : (g > 4096 ? 4096 : g))), dim3(256), 0,
                           s, buf.as<unsigned long long>(), m);
        PP_HIP(hipGetLastError());
    }
    return PP_OK;
}

int launch_scan_i32_to_i64(const int32_t* in, int64_t* off, int64_t n, DevBuf& ws, hipStream_t s,
                           int64_t* sizes) {
    ScanIO io{{in, nullptr}, {off, nullptr}};
    return launch<1>(io, n, ws, s, sizes);
}

int launch_scan2_i32_to_i64(const int32_t* a, const int32_t* b, int64_t* oa, int64_t* ob, int64_t n,
                            DevBuf& ws, hipStream_t s, int64_t* sizes) {
    ScanIO io{{a, b}, {oa, ob}};
    return launch<2>(io, n, ws, s, sizes);
}

}  // namespace pp
