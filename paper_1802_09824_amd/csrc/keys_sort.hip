// Peano-Hilbert keys, key sort and the gather into key order.
//
// Keys follow sec. 4.1 (a 2^(3b) grid labelled along a Peano-Hilbert
// curve).  The curve is J. Skilling's ("Programming the Hilbert curve",
// AIP Conf. Proc. 707, 2004): coordinates are turned into the "transposed"
// index by undoing reflections and axis exchanges from the coarsest level
// down, Gray-encoding across axes, and interleaving with x as the most
// significant bit of every 3-bit digit.  The sort makes every octree node a
// contiguous run of particles (sec. 3.2); in a batch each box is sorted as
// its own segment.
#include <cstring>

#include <rocprim/device/device_radix_sort.hpp>

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
        if (X0 & Q) X0 ^= P;               // axis 0 (its exchange with itself is a no-op)
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

__device__ __forceinline__ uint64_t key_of(double x, double y, double z, double L, double scale,
                                           int b) {
    const uint32_t qmax = (1u << b) - 1u;
    return hilbert_index(quantise(wrap_pos(x, L), scale, qmax), quantise(wrap_pos(y, L), scale, qmax),
                         quantise(wrap_pos(z, L), scale, qmax), b);
}

__global__ void __launch_bounds__(256) keys_kernel(BatchDev bd, const double* __restrict__ pos,
                                                   int64_t N, uint64_t* __restrict__ keys,
                                                   int32_t* __restrict__ iota, int* bad) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N) return;
    const BoxDev& B = bd.box[box_of(bd.poff, bd.nbox, k)];
    double x = pos[k], y = pos[N + k], z = pos[2 * N + k];
    if (!isfinite(x) || !isfinite(y) || !isfinite(z)) {
        atomicOr(bad, 1);
        x = y = z = 0.0;
    }
    keys[k] = key_of(x, y, z, B.L, B.qscale, bd.bits);
    iota[k] = (int32_t)k;
}

__global__ void __launch_bounds__(256) keys_raw_kernel(const double* __restrict__ pos, int64_t n,
                                                       double L, double scale, int b,
                                                       uint64_t* __restrict__ keys) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    keys[k] = key_of(pos[k], pos[n + k], pos[2 * n + k], L, scale, b);
}

// Input order -> one 32-byte record per particle (wrapped position, mass),
// read and written in order, so that the permuted gather below touches one
// record per particle instead of four arrays.
template <class M>
__global__ void __launch_bounds__(256) pack_kernel(BatchDev bd, const double* __restrict__ pos,
                                                   const M* __restrict__ mass, int64_t N,
                                                   double4* __restrict__ rec, int* bad) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const double L = bd.box[box_of(bd.poff, bd.nbox, i)].L;
    double4 r;
    const double x = pos[i], y = pos[N + i], z = pos[2 * N + i];
    r.x = isfinite(x) ? wrap_pos(x, L) : 0.0;
    r.y = isfinite(y) ? wrap_pos(y, L) : 0.0;
    r.z = isfinite(z) ? wrap_pos(z, L) : 0.0;
    M m = mass[i];
    if (!isfinite((double)m)) {
        atomicOr(bad, 1);
        m = 0;
    }
    r.w = (double)m;
    rec[i] = r;
}

template <class M>
__global__ void __launch_bounds__(256) gather_kernel(const double4* __restrict__ rec,
                                                     const int32_t* __restrict__ perm, int64_t N,
                                                     double* __restrict__ pos_s, M* __restrict__ mass_s) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N) return;
    const double4 r = rec[perm[k]];
    pos_s[k] = r.x;
    pos_s[N + k] = r.y;
    pos_s[2 * N + k] = r.z;
    mass_s[k] = (M)r.w;
}


__global__ void fill_i32_kernel(int32_t* __restrict__ p, int64_t n, int32_t v) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x < n) p[x] = v;
}

// flag[box] = 1 where some mass of the box differs from the box's first one
// (a plain store of the same value by every such lane; no atomics).
__global__ void __launch_bounds__(256) mass_flag_kernel(BatchDev bd, const float* __restrict__ mass_s,
                                                        int64_t N, int32_t* __restrict__ flag) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N) return;
    const int x = box_of(bd.poff, bd.nbox, k);
    if (mass_s[k] != mass_s[bd.poff[x]]) flag[x] = 1;
}

__global__ void __launch_bounds__(256) wrap_copy_kernel(BatchDev bd, const double* __restrict__ in,
                                                        int64_t N, double* __restrict__ out) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N) return;
    const double L = bd.box[box_of(bd.poff, bd.nbox, k)].L;
    for (int a = 0; a < 3; ++a) {
        const double x = in[a * N + k];
        out[a * N + k] = isfinite(x) ? wrap_pos(x, L) : 0.0;
    }
}

// Box id (the second sort key) of every particle after the key sort.
__global__ void __launch_bounds__(256) box_ids_kernel(BatchDev bd, const int32_t* __restrict__ idx,
                                                      int64_t N, uint16_t* __restrict__ box) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N) return;
    box[k] = (uint16_t)box_of(bd.poff, bd.nbox, idx[k]);
}

__global__ void __launch_bounds__(256) gather_keys_kernel(const uint64_t* __restrict__ keys,
                                                          const int32_t* __restrict__ perm,
                                                          int64_t N, uint64_t* __restrict__ out) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N) return;
    out[k] = keys[perm[k]];
}

// Reuse of the lists: particle k of the stored key order (input particle
// perm[k]) moves from its reference position by its minimum-image
// displacement, so it stays at the periodic image the lists were built for;
// its mass is gathered too.  A displacement of at least half_skin sets
// sizes[kMoved] (the lists may then miss pairs and are rebuilt), a
// non-finite position or mass the bad flag.
__global__ void __launch_bounds__(256) regather_kernel(BatchDev bd, const double* __restrict__ pos,
                                                       const float* __restrict__ mass,
                                                       const int32_t* __restrict__ perm,
                                                       const double* __restrict__ ref, int64_t N,
                                                       int64_t n_in, double half_skin2,
                                                       double* __restrict__ pos_s,
                                                       float* __restrict__ mass_s,
                                                       int64_t* __restrict__ sizes, int* __restrict__ bad) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N) return;
    const int x = box_of(bd.poff, bd.nbox, k);
    const double L = bd.box[x].L;
    const int64_t i = perm[k];
    double d2 = 0.0;
    bool finite = true;
    for (int a = 0; a < 3; ++a) {
        const double xn = pos[a * n_in + i], xr = ref[a * N + k];
        finite = finite && isfinite(xn);
        double d = xn - xr;
        d -= L * rint(d / L);
        pos_s[a * N + k] = xr + d;
        d2 += d * d;
    }
    const float m = mass[i];
    mass_s[k] = m;
    if (!finite || !isfinite(m)) *bad = 1;
    else if (d2 >= half_skin2) sizes[kMoved] = 1;
}

// The key sort: one-sweep radix with 10-bit digits (7 passes over 63 key
// bits instead of 8 with the library's 8-bit default for this target).
using key_sort_config = rocprim::radix_sort_config<
    rocprim::default_config, rocprim::default_config,
    rocprim::radix_sort_onesweep_config<rocprim::kernel_config<1024, 8>, rocprim::kernel_config<1024, 8>,
                                        10, rocprim::block_radix_rank_algorithm::match>>;

}  // namespace

int stage_mass_flags(const BatchDev& bd, int64_t N, Work& w, hipStream_t s) {
    PP_TRY(w.mass_flag.reserve(sizeof(int32_t) * (bd.nbox + 1)));
    hipLaunchKernelGGL(fill_i32_kernel, dim3(blocks_for(bd.nbox, 64)), dim3(64), 0, s,
                       w.mass_flag.as<int32_t>(), (int64_t)bd.nbox, 0);
    if (N > 0)
        hipLaunchKernelGGL(mass_flag_kernel, dim3(blocks_for(N, 256)), dim3(256), 0, s, bd,
                           w.mass_s.as<float>(), N, w.mass_flag.as<int32_t>());
    PP_HIP(hipGetLastError());
    return PP_OK;
}

int stage_wrap_copy(const BatchDev& bd, int64_t N, const double* in, double* out, hipStream_t s) {
    if (N == 0) return PP_OK;
    hipLaunchKernelGGL(wrap_copy_kernel, dim3(blocks_for(N, 256)), dim3(256), 0, s, bd, in, N, out);
    PP_HIP(hipGetLastError());
    return PP_OK;
}

int stage_keys(const BatchDev& bd, int64_t N, const double* pos, Work& w, hipStream_t s) {
    if (N == 0) return PP_OK;
    hipLaunchKernelGGL(keys_kernel, dim3(blocks_for(N, 256)), dim3(256), 0, s, bd, pos, N,
                       w.keys.as<uint64_t>(), w.iota.as<int32_t>(), w.bad.as<int>());
    PP_HIP(hipGetLastError());
    return PP_OK;
}

int launch_keys_raw(const double* pos, int64_t n, double L, int bits, uint64_t* keys,
                    hipStream_t s) {
    if (n == 0) return PP_OK;
    hipLaunchKernelGGL(keys_raw_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, pos, n, L,
                       ldexp(1.0, bits) / L, bits, keys);
    PP_HIP(hipGetLastError());
    return PP_OK;
}

int sort_workspace(int64_t n, int nbox, int bits, size_t* bytes) {
    size_t b = 0, b2 = 0;
    PP_HIP(rocprim::radix_sort_pairs<key_sort_config>((void*)nullptr, b, (const uint64_t*)nullptr, (uint64_t*)nullptr,
                                     (const int32_t*)nullptr, (int32_t*)nullptr, (size_t)n, 0,
                                     3 * bits, (hipStream_t)0));
    if (nbox > 1) {
        PP_HIP(rocprim::radix_sort_pairs((void*)nullptr, b2, (const uint16_t*)nullptr,
                                         (uint16_t*)nullptr, (const int32_t*)nullptr,
                                         (int32_t*)nullptr, (size_t)n, 0, 16, (hipStream_t)0));
    }
    *bytes = b > b2 ? b : b2;
    return PP_OK;
}

int launch_sort_raw(const uint64_t* keys, const int32_t* idx_in, uint64_t* keys_out,
                    int32_t* perm_out, int64_t n, int bits, void* ws, size_t ws_bytes,
                    hipStream_t s) {
    if (n == 0) return PP_OK;
    size_t b = ws_bytes;
    PP_HIP(rocprim::radix_sort_pairs<key_sort_config>(ws, b, keys, keys_out, idx_in, perm_out, (size_t)n, 0, 3 * bits,
                                     s));
    return PP_OK;
}

int stage_sort(const BatchDev& bd, int64_t N, Work& w, hipStream_t s) {
    if (N == 0) return PP_OK;
    size_t need = 0;
    PP_TRY(sort_workspace(N, bd.nbox, bd.bits, &need));
    PP_TRY(w.sort_ws.reserve(need + 1));
    size_t b = w.sort_ws.bytes;
    if (bd.nbox <= 1) {
        PP_HIP(rocprim::radix_sort_pairs<key_sort_config>(w.sort_ws.p, b, w.keys.as<uint64_t>(),
                                         w.keys_s.as<uint64_t>(), w.iota.as<int32_t>(),
                                         w.perm.as<int32_t>(), (size_t)N, 0, 3 * bd.bits, s));
        return PP_OK;
    }
    // Batches: a stable sort by key, then a stable sort by box id, gives the
    // (box, key, index) order; both are one-sweep radix sorts over the whole
    // batch (a per-segment sort is far slower for many small segments).
    PP_TRY(w.sort_tmp.reserve((sizeof(uint16_t) * 2 + sizeof(int32_t)) * (size_t)(N + 64)));
    uint16_t* box_a = w.sort_tmp.as<uint16_t>();
    uint16_t* box_b = box_a + N + 32;
    int32_t* idx1 = reinterpret_cast<int32_t*>(box_b + N + 32);
    PP_HIP(rocprim::radix_sort_pairs<key_sort_config>(w.sort_ws.p, b, w.keys.as<uint64_t>(), w.keys_s.as<uint64_t>(),
                                     w.iota.as<int32_t>(), idx1, (size_t)N, 0, 3 * bd.bits, s));
    hipLaunchKernelGGL(box_ids_kernel, dim3(blocks_for(N, 256)), dim3(256), 0, s, bd, idx1, N, box_a);
    PP_HIP(hipGetLastError());
    b = w.sort_ws.bytes;
    PP_HIP(rocprim::radix_sort_pairs(w.sort_ws.p, b, box_a, box_b, idx1, w.perm.as<int32_t>(),
                                     (size_t)N, 0, 16, s));
    hipLaunchKernelGGL(gather_keys_kernel, dim3(blocks_for(N, 256)), dim3(256), 0, s,
                       w.keys.as<uint64_t>(), w.perm.as<int32_t>(), N, w.keys_s.as<uint64_t>());
    PP_HIP(hipGetLastError());
    return PP_OK;
}

int stage_regather(const BatchDev& bd, int64_t N, const double* pos, const float* mass,
                   const double* ref, double half_skin, Work& w, hipStream_t s) {
    if (N == 0) return PP_OK;
    hipLaunchKernelGGL(regather_kernel, dim3(blocks_for(N, 256)), dim3(256), 0, s, bd, pos, mass,
                       w.perm.as<int32_t>(), ref, N, w.pos_n, half_skin * half_skin, w.pos_s.as<double>(),
                       w.mass_s.as<float>(), w.sizes.as<int64_t>(), w.bad.as<int>());
    PP_HIP(hipGetLastError());
    return PP_OK;
}

int stage_gather(const BatchDev& bd, int64_t N, const double* pos, const float* mass_f,
                 const double* mass_d, Work& w, hipStream_t s) {
    if (N == 0) return PP_OK;
    PP_TRY(w.rec.reserve(sizeof(double4) * N));
    double4* rec = w.rec.as<double4>();
    const int32_t* perm = w.perm.as<int32_t>();
    if (mass_f) {
        hipLaunchKernelGGL(pack_kernel<float>, dim3(blocks_for(N, 256)), dim3(256), 0, s, bd, pos, mass_f, N,
                           rec, w.bad.as<int>());
        hipLaunchKernelGGL(gather_kernel<float>, dim3(blocks_for(N, 256)), dim3(256), 0, s, rec, perm, N,
                           w.pos_s.as<double>(), w.mass_s.as<float>());
    } else {
        hipLaunchKernelGGL(pack_kernel<double>, dim3(blocks_for(N, 256)), dim3(256), 0, s, bd, pos, mass_d,
                           N, rec, w.bad.as<int>());
        hipLaunchKernelGGL(gather_kernel<double>, dim3(blocks_for(N, 256)), dim3(256), 0, s, rec, perm, N,
                           w.pos_s.as<double>(), w.mass_sd.as<double>());
    }
    PP_HIP(hipGetLastError());
    return PP_OK;
}

}  // namespace pp
