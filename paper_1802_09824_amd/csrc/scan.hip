// Single-pass exclusive scans of int32 counts into int64 offsets, used by
// every stage that turns per-item counts into output positions: tiles of
// kScanTile counts with decoupled look-back between them (lookback.h).
#include "lookback.h"

namespace pp {
namespace {

constexpr int kScanWG = 256;
template <int NV>
struct ScanTile {
    static constexpr int kIPT = 8;
    static constexpr int64_t kSize = (int64_t)kScanWG * kIPT;
};
constexpr int64_t kScanMinTile = ScanTile<2>::kSize;
struct ScanIO {
    const int32_t* in[2];
    int64_t* out[2];
};

// out[c][i] = sum of in[c][0 .. i) for i in [0, n]; ntile = tiles over n + 1.
// `cur` is this scan's region (ticket, then words), `other` the region to
// clear (nclear words).  The tile's counts come in and its offsets go out
// through LDS, so that the global loads and stores of a wave are contiguous
// while every thread scans kScanIPT consecutive counts.
// With note.slot >= 0 the last tile also records the total of array 0 in
// the count slots: sizes[need_slot] = total, sizes[slot] (and slot2) =
// min(total, cap), and the overflow bit when total > cap.
template <int NV>
__global__ __launch_bounds__(kScanWG) void scan_counts_kernel(ScanIO io, int64_t n, LbArgs lb,
                                                              int64_t* sizes, int64_t ntile, ScanNote note) {
    constexpr int kScanIPT = ScanTile<NV>::kIPT;
    constexpr int64_t kScanTile = ScanTile<NV>::kSize;
    __shared__ int32_t s_in[NV][kScanTile];
    __shared__ int64_t s_out[NV][kScanTile];
    __shared__ unsigned s_tile;
    __shared__ int64_t s_wave[NV][kScanWG / 64];
    __shared__ int64_t s_pre[NV];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    lb_clear_other(lb);
    if (t == 0) s_tile = (unsigned)atomicAdd(lb.cur, 1ull);
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
        const int64_t ex = lb_tile_prefix<NV>(lb, tile, c, agg, sizes, lane);
        if (lane == 0) {
            s_pre[c] = ex;
            if (c == 0 && note.slot >= 0 && tile == ntile - 1) {
                const int64_t total = ex + agg;
                const int64_t kept = total < note.cap ? total : note.cap;
                sizes[note.need_slot] = total;
                sizes[note.slot] = kept;
                if (note.slot2 >= 0) sizes[note.slot2] = kept;
                if (total > note.cap)
                    atomicOr(reinterpret_cast<unsigned long long*>(sizes + kOverflow), note.bit);
            }
        }
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

template <int NV>
int64_t tiles_for(int64_t n) { return (n + 1 + ScanTile<NV>::kSize - 1) / ScanTile<NV>::kSize; }

// look-back words for n counts of each of up to two arrays
int64_t words_for(int64_t n) { return 2 * ((n + 1 + kScanMinTile - 1) / kScanMinTile) + 2; }

__global__ void note_zero_kernel(int64_t* __restrict__ sizes, ScanNote note) {
    sizes[note.need_slot] = 0;
    sizes[note.slot] = 0;
    if (note.slot2 >= 0) sizes[note.slot2] = 0;
}

template <int NV>
int launch(const ScanIO& io, int64_t n, DevBuf& ws, hipStream_t s, int64_t* sizes, const ScanNote* note) {
    if (note && !sizes) return fail(PP_EINVAL, "a scan note needs the count slots");
    if (n == 0) {
        hipLaunchKernelGGL(set_zero2_kernel, dim3(1), dim3(1), 0, s, io.out[0], NV > 1 ? io.out[1] : nullptr);
        if (note) hipLaunchKernelGGL(note_zero_kernel, dim3(1), dim3(1), 0, s, sizes, *note);
        PP_HIP(hipGetLastError());
        return PP_OK;
    }
    const int64_t nt = tiles_for<NV>(n);
    PP_TRY(grow_lookback(ws, nt * NV, s));
    LbArgs lb;
    PP_TRY(lookback_args(ws, nt * NV, &lb));
    const ScanNote none{-1, -1, 0, 0ull, -1};
    hipLaunchKernelGGL(scan_counts_kernel<NV>, dim3((unsigned)nt), dim3(kScanWG), 0, s, io, n, lb, sizes, nt,
                       note ? *note : none);
    PP_HIP(hipGetLastError());
    return PP_OK;
}

}  // namespace

int scan_workspace(int64_t n, size_t* bytes) {
    // two regions of a ticket and the words, a line each
    *bytes = 2 * sizeof(unsigned long long) * (size_t)(1 + (words_for(n) + 1) * kLbWordStride + 2);
    return PP_OK;
}

int grow_scan(DevBuf& buf, int64_t n, hipStream_t s) { return grow_lookback(buf, words_for(n), s); }

int lookback_args(DevBuf& ws, int64_t words, LbArgs* out) {
    words = (words + 1) * kLbWordStride;      // the ticket's line, then a line per word
    const int64_t region = (int64_t)(ws.bytes / sizeof(unsigned long long)) / 2;
    if (1 + words > region) return fail(PP_EDEVICE, "look-back workspace smaller than its tiles");
    unsigned long long* base = ws.as<unsigned long long>();
    const uint32_t r = ws.tag & 1u;             // the region this kernel uses
    out->cur = base + r * region;
    out->other = base + (1 - r) * region;
    out->nclear = region;
    ws.tag ^= 1u;
    return PP_OK;
}

int grow_lookback(DevBuf& buf, int64_t words, hipStream_t s) {
    words = (words + 1) * kLbWordStride;
    const size_t need = 2 * sizeof(unsigned long long) * (size_t)(1 + words + 2);
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
                           int64_t* sizes, const ScanNote* note) {
    ScanIO io{{in, nullptr}, {off, nullptr}};
    return launch<1>(io, n, ws, s, sizes, note);
}

int launch_scan2_i32_to_i64(const int32_t* a, const int32_t* b, int64_t* oa, int64_t* ob, int64_t n,
                            DevBuf& ws, hipStream_t s, int64_t* sizes) {
    ScanIO io{{a, b}, {oa, ob}};
    return launch<2>(io, n, ws, s, sizes, nullptr);
}

}  // namespace pp
