// Peano-Hilbert keys, key sort and the gather into key order.
//
// Keys follow sec. 4.1 (a 2^(3b) grid labelled along a Peano-Hilbert
// curve).  The curve is J. Skilling's ("Programming the Hilbert curve",
// AIP Conf. Proc. 707, 2004): coordinates are turned into the "transposed"
// index by undoing reflections and axis exchanges from the coarsest level
// down, Gray-encoding across axes, and interleaving with x as the most
// significant bit of every 3-bit digit.  The sort makes every octree node a
// contiguous run of particles (sec. 3.2).
#include <cstring>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>
#include <rocprim/iterator/transform_iterator.hpp>

#include "pp_internal.h"

namespace pp {
namespace {

#pragma clang fp contract(off)
// Wrap into [0, L) exactly as written: x - L * floor(x / L), each operation
// rounded on its own (no fused multiply-add), so that every consumer of the
// wrapped positions and of the grid cells sees identical values.
__device__ __forceinline__ double wrap_pos(double x, double L) {
    return x - L * floor(x / L);
}

__device__ __forceinline__ uint32_t quantise(double w, double scale, uint32_t qmax) {
    double f = floor(w * scale);
    if (!(f > 0.0)) return 0u;             // also maps -0 and tiny negatives to 0
    if (f > (double)qmax) return qmax;
    return (uint32_t)f;
}
#pragma clang fp contract(on)

// Spread the low 21 bits of v so that bit l lands on bit 3l.
__device__ __forceinline__ uint64_t spread3(uint32_t v) {
    uint64_t x = v & 0x1fffffu;
    x = (x | (x << 32)) & 0x001f00000000ffffull;
    x = (x | (x << 16)) & 0x001f0000ff0000ffull;
    x = (x | (x << 8)) & 0x100f00f00f00f00full;
    x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}

__device__ __forceinline__ uint64_t hilbert_index(uint32_t x, uint32_t y, uint32_t z, int b) {
    uint32_t X0 = x, X1 = y, X2 = z;
    const uint32_t top = 1u << (b - 1);
    // Undo the excess work, coarsest level first: at level Q an axis whose
    // bit is set reflects the lower bits of axis 0, otherwise the lower bits
    // of that axis and axis 0 are exchanged.
    for (uint32_t Q = top; Q > 1; Q >>= 1) {
        const uint32_t P = Q - 1;
        // axis 0 (its exchange with itself is a no-op)
        if (X0 & Q) X0 ^= P;
        if (X1 & Q) {
            X0 ^= P;
        } else {
            uint32_t t = (X0 ^ X1) & P;
            X0 ^= t;
            X1 ^= t;
        }
        if (X2 & Q) {
            X0 ^= P;
        } else {
            uint32_t t = (X0 ^ X2) & P;
            X0 ^= t;
            X2 ^= t;
        }
    }
    // Gray encode across axes
    X1 ^= X0;
    X2 ^= X1;
    uint32_t t = 0;
    for (uint32_t Q = top; Q > 1; Q >>= 1)
        if (X2 & Q) t ^= Q - 1;
    X0 ^= t;
    X1 ^= t;
    X2 ^= t;
    return (spread3(X0) << 2) | (spread3(X1) << 1) | spread3(X2);
}

__global__ void __launch_bounds__(256) keys_kernel(const double* __restrict__ pos, int64_t n,
                                                   double L, double scale, int b, uint32_t qmax,
                                                   uint64_t* __restrict__ keys,
                                                   int32_t* __restrict__ iota, int* bad) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    double x = pos[k], y = pos[n + k], z = pos[2 * n + k];
    if (!isfinite(x) || !isfinite(y) || !isfinite(z)) {
        atomicOr(bad, 1);
        x = y = z = 0.0;
    }
    uint32_t qx = quantise(wrap_pos(x, L), scale, qmax);
    uint32_t qy = quantise(wrap_pos(y, L), scale, qmax);
    uint32_t qz = quantise(wrap_pos(z, L), scale, qmax);
    keys[k] = hilbert_index(qx, qy, qz, b);
    if (iota) iota[k] = (int32_t)k;
}

template <class M>
__global__ void __launch_bounds__(256) gather_kernel(const double* __restrict__ pos,
                                                     const M* __restrict__ mass,
                                                     const int32_t* __restrict__ perm, int64_t n,
                                                     double L, double* __restrict__ pos_s,
                                                     M* __restrict__ mass_s, int* bad) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    int64_t i = perm[k];
    for (int a = 0; a < 3; ++a) {
        double x = pos[a * n + i];
        pos_s[a * n + k] = isfinite(x) ? wrap_pos(x, L) : 0.0;
    }
    M m = mass[i];
    if (!isfinite((double)m)) {
        atomicOr(bad, 1);
        m = 0;
    }
    mass_s[k] = m;
}

__global__ void set_zero_i64(int64_t* p) { *p = 0; }

struct to_i64 {
    __device__ __host__ int64_t operator()(int32_t v) const { return (int64_t)v; }
};

inline unsigned blocks_for(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

int launch_keys(const double* pos, int64_t n, double L, int bits, uint64_t* keys, int32_t* iota,
                int* bad_flag, hipStream_t s) {
    if (n == 0) return PP_OK;
    const double scale = ldexp(1.0, bits) / L;
    const uint32_t qmax = (1u << bits) - 1u;
    hipLaunchKernelGGL(keys_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, pos, n, L, scale,
                       bits, qmax, keys, iota, bad_flag);
    PP_HIP(hipGetLastError());
    return PP_OK;
}

int sort_workspace(int64_t n, int bits, size_t* bytes) {
    size_t b = 0;
    PP_HIP(rocprim::radix_sort_pairs((void*)nullptr, b, (const uint64_t*)nullptr, (uint64_t*)nullptr,
                                     (const int32_t*)nullptr, (int32_t*)nullptr, (size_t)n, 0,
                                     3 * bits, (hipStream_t)0));
    *bytes = b;
    return PP_OK;
}

int launch_sort(const uint64_t* keys, const int32_t* idx_in, uint64_t* keys_out, int32_t* perm_out,
                int64_t n, int bits, void* ws, size_t ws_bytes, hipStream_t s) {
    if (n == 0) return PP_OK;
    size_t b = ws_bytes;
    PP_HIP(rocprim::radix_sort_pairs(ws, b, keys, keys_out, idx_in, perm_out, (size_t)n, 0, 3 * bits,
                                     s));
    return PP_OK;
}

int launch_gather(const double* pos, const float* mass_f, const double* mass_d,
                  const int32_t* perm, int64_t n, double L, double* pos_s, float* mass_s_f,
                  double* mass_s_d, int* bad_flag, hipStream_t s) {
    if (n == 0) return PP_OK;
    if (mass_f)
        hipLaunchKernelGGL(gather_kernel<float>, dim3(blocks_for(n, 256)), dim3(256), 0, s, pos,
                           mass_f, perm, n, L, pos_s, mass_s_f, bad_flag);
    else
        hipLaunchKernelGGL(gather_kernel<double>, dim3(blocks_for(n, 256)), dim3(256), 0, s, pos,
                           mass_d, perm, n, L, pos_s, mass_s_d, bad_flag);
    PP_HIP(hipGetLastError());
    return PP_OK;
}

int scan_workspace(int64_t n, size_t* bytes) {
    size_t b = 0;
    rocprim::transform_iterator<const int32_t*, to_i64, int64_t> it((const int32_t*)nullptr, to_i64());
    PP_HIP(rocprim::inclusive_scan((void*)nullptr, b, it, (int64_t*)nullptr, (size_t)n,
                                   rocprim::plus<int64_t>(), (hipStream_t)0));
    *bytes = b;
    return PP_OK;
}

int launch_scan_i32_to_i64(const int32_t* in, int64_t* off, int64_t n, void* ws, size_t ws_bytes,
                           hipStream_t s) {
    hipLaunchKernelGGL(set_zero_i64, dim3(1), dim3(1), 0, s, off);
    PP_HIP(hipGetLastError());
    if (n == 0) return PP_OK;
    size_t b = ws_bytes;
    rocprim::transform_iterator<const int32_t*, to_i64, int64_t> it(in, to_i64());
    PP_HIP(rocprim::inclusive_scan(ws, b, it, off + 1, (size_t)n, rocprim::plus<int64_t>(), s));
    return PP_OK;
}

}  // namespace pp
