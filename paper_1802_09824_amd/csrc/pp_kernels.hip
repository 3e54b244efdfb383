// The PP (particle-particle) kernels: short-range pair sums over the block
// lists, FP32 (the hot path), FP64 (the yardstick) and an FP64 pair count.
//
// Per pair (sec. 3.1, Eq. equ:split, with Plummer softening):
//   a_i += G m_j d g(s_eps / 2 r_s) / s_eps^3,   kept iff s < r_cut.
// FP32 form.  Lengths are in units of r_cut, relative to the FP64 centre of
// the target block (the origin subtraction is done in FP64 when a source
// tile is staged, so the FP32 offsets are small and precise).  With
// r2 = s_eps^2, y = 1/s_eps (hardware reciprocal square root) and
// u = x^2 = r2 k^2, k = r_cut / (2 r_s):
//   g / s_eps^3 = y^3 - k^3 H(u),   g(x) = 1 - x^3 H(x^2),
// H a fitted polynomial (split_poly.h).  Softening enters r2 through the
// first fused multiply-add; the cut test compares r2 with 1 + eps^2.
// Sources are staged 64 at a time in LDS and broadcast to the 64 lanes
// (one target per lane).  Each tile of 64 pairs is summed in FP32 and the
// tile sums enter a Kahan-compensated per-target total.  Work items are
// (target block, chunk of its source list); their partial sums are reduced
// in FP64 in a fixed order, so results do not depend on scheduling.
#include <cmath>

#include "pp_internal.h"
#include "split_poly.h"

namespace pp {
namespace {

inline unsigned blocks_for(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

// Items are laid out so that the 8 XCDs (which take workgroups round-robin)
// each see one contiguous stretch of items: neighbouring target blocks share
// most of their sources, which then stay in that XCD's L2.
__device__ __forceinline__ int64_t xcd_item(int64_t bid, int64_t per_xcd) {
    return (bid & 7) * per_xcd + (bid >> 3);
}

__device__ __forceinline__ int64_t find_range(const int32_t* __restrict__ rpre, int64_t lo,
                                              int64_t hi, int32_t p) {
    // last r in [lo, hi] with rpre[r] <= p (rpre ascending, rpre[lo] = 0 <= p)
    while (lo < hi) {
        int64_t mid = (lo + hi + 1) >> 1;
        if (rpre[mid] <= p) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

struct ItemArgs {
    const int32_t* iblock;
    const int32_t* is0;
    int64_t nitem, per_xcd;
    const IBox* bbox;
    const int64_t* roff;
    const int32_t* rbeg;
    const int32_t* rpre;
    const uint8_t* rcode;
    const int32_t* slen;
    int chunk;
};

template <bool NEWTON>
__global__ void __launch_bounds__(64) pp_f32_kernel(ItemArgs ia, const double* __restrict__ pos_s,
                                                    const float* __restrict__ mass_s, int64_t n,
                                                    double L, double cell, double inv_rcut,
                                                    PolyF32 P, float* __restrict__ partial) {
    const int64_t item = xcd_item(blockIdx.x, ia.per_xcd);
    if (item >= ia.nitem) return;
    const int lane = threadIdx.x;
    const int32_t b = ia.iblock[item];
    const int32_t s0 = ia.is0[item];
    const int32_t S = ia.slen[b];
    const int32_t s1 = s0 + ia.chunk < S ? s0 + ia.chunk : S;
    const IBox B = ia.bbox[b];
    const double ox = 0.5 * (double)(B.lo[0] + B.hi[0]) * cell;
    const double oy = 0.5 * (double)(B.lo[1] + B.hi[1]) * cell;
    const double oz = 0.5 * (double)(B.lo[2] + B.hi[2]) * cell;
    const int64_t t = (int64_t)b * kBlock + lane;
    float xi = 0.f, yi = 0.f, zi = 0.f;
    if (t < n) {
        xi = (float)((pos_s[t] - ox) * inv_rcut);
        yi = (float)((pos_s[n + t] - oy) * inv_rcut);
        zi = (float)((pos_s[2 * n + t] - oz) * inv_rcut);
    }
    const int64_t r_lo = ia.roff[b], r_hi = ia.roff[b + 1] - 1;
    __shared__ float4 tile[kBlock];
    float ax = 0.f, ay = 0.f, az = 0.f, cx = 0.f, cy = 0.f, cz = 0.f;
    for (int32_t base = s0; base < s1; base += kBlock) {
        const int32_t p = base + lane;
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (p < s1) {
            const int64_t r = find_range(ia.rpre, r_lo, r_hi, p);
            const int64_t j = (int64_t)ia.rbeg[r] + (p - ia.rpre[r]);
            const int c = ia.rcode[r];
            const double sx = (double)(c / 9 - 1) * L;
            const double sy = (double)((c / 3) % 3 - 1) * L;
            const double sz = (double)(c % 3 - 1) * L;
            v.x = (float)((pos_s[j] + sx - ox) * inv_rcut);
            v.y = (float)((pos_s[n + j] + sy - oy) * inv_rcut);
            v.z = (float)((pos_s[2 * n + j] + sz - oz) * inv_rcut);
            v.w = mass_s[j];
        }
        __syncthreads();
        tile[lane] = v;
        __syncthreads();
        float tx = 0.f, ty = 0.f, tz = 0.f;
#pragma unroll 8
        for (int q = 0; q < kBlock; ++q) {
            const float4 sj = tile[q];
            const float dx = sj.x - xi, dy = sj.y - yi, dz = sj.z - zi;
            float r2 = fmaf(dx, dx, P.eps2n);
            r2 = fmaf(dy, dy, r2);
            r2 = fmaf(dz, dz, r2);
            float y = __builtin_amdgcn_rsqf(r2);
            if (NEWTON) y = y * fmaf(-0.5f * r2 * y, y, 1.5f);
            const float u = fmaf(r2, P.tscale, -1.f);
            float h = P.c[9];
            h = fmaf(h, u, P.c[8]);
            h = fmaf(h, u, P.c[7]);
            h = fmaf(h, u, P.c[6]);
            h = fmaf(h, u, P.c[5]);
            h = fmaf(h, u, P.c[4]);
            h = fmaf(h, u, P.c[3]);
            h = fmaf(h, u, P.c[2]);
            h = fmaf(h, u, P.c[1]);
            h = fmaf(h, u, P.c[0]);
            const float y3 = y * y * y;
            float F = (y3 - h) * sj.w;
            F = r2 < P.cut2 ? F : 0.f;
            tx = fmaf(F, dx, tx);
            ty = fmaf(F, dy, ty);
            tz = fmaf(F, dz, tz);
        }
        // Kahan: true sum ~ a - c
        float yk, tk;
        yk = tx - cx; tk = ax + yk; cx = (tk - ax) - yk; ax = tk;
        yk = ty - cy; tk = ay + yk; cy = (tk - ay) - yk; ay = tk;
        yk = tz - cz; tk = az + yk; cz = (tk - az) - yk; az = tk;
    }
    float* o = partial + item * 6 * kBlock;
    o[0 * kBlock + lane] = ax;
    o[1 * kBlock + lane] = ay;
    o[2 * kBlock + lane] = az;
    o[3 * kBlock + lane] = cx;
    o[4 * kBlock + lane] = cy;
    o[5 * kBlock + lane] = cz;
}

__global__ void __launch_bounds__(256) reduce_f32_kernel(const int64_t* __restrict__ ioff,
                                                         const float* __restrict__ partial,
                                                         const int32_t* __restrict__ perm,
                                                         int64_t n, double scale,
                                                         float* __restrict__ acc) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int64_t b = t / kBlock;
    const int l = (int)(t % kBlock);
    double sx = 0, sy = 0, sz = 0;
    for (int64_t it = ioff[b]; it < ioff[b + 1]; ++it) {
        const float* o = partial + it * 6 * kBlock;
        sx += (double)o[0 * kBlock + l] - (double)o[3 * kBlock + l];
        sy += (double)o[1 * kBlock + l] - (double)o[4 * kBlock + l];
        sz += (double)o[2 * kBlock + l] - (double)o[5 * kBlock + l];
    }
    const int64_t i = perm[t];
    acc[i] = (float)(sx * scale);
    acc[n + i] = (float)(sy * scale);
    acc[2 * n + i] = (float)(sz * scale);
}

// ------------------------------------------------------------------ FP64 --
#pragma clang fp contract(off)
// The split factor (Eq. equ:split) in FP64 with the device erfc/exp.
__device__ __forceinline__ double split_factor_f64(double x) {
    return erfc(x) + 2.0 * x / 1.7724538509055160272981674833411 * exp(-x * x);
}

template <bool COUNT>
__global__ void __launch_bounds__(64) pp_f64_kernel(ItemArgs ia, const double* __restrict__ pos_s,
                                                    const double* __restrict__ mass_s, int64_t n,
                                                    double L, double rs, double rcut, double eps,
                                                    double G, double* __restrict__ partial,
                                                    int32_t* __restrict__ pcount) {
    const int64_t item = xcd_item(blockIdx.x, ia.per_xcd);
    if (item >= ia.nitem) return;
    const int lane = threadIdx.x;
    const int32_t b = ia.iblock[item];
    const int32_t s0 = ia.is0[item];
    const int32_t S = ia.slen[b];
    const int32_t s1 = s0 + ia.chunk < S ? s0 + ia.chunk : S;
    const int64_t t = (int64_t)b * kBlock + lane;
    double xi = 0, yi = 0, zi = 0;
    if (t < n) {
        xi = pos_s[t];
        yi = pos_s[n + t];
        zi = pos_s[2 * n + t];
    }
    const int64_t r_lo = ia.roff[b], r_hi = ia.roff[b + 1] - 1;
    __shared__ double4 tile[kBlock];
    __shared__ int64_t tj[kBlock];
    __shared__ int tc[kBlock];
    const double rcut2 = rcut * rcut, eps2 = eps * eps;
    double ax = 0, ay = 0, az = 0;
    int32_t cnt = 0;
    for (int32_t base = s0; base < s1; base += kBlock) {
        const int32_t p = base + lane;
        double4 v = make_double4(0, 0, 0, 0);
        int64_t j = -1;
        int c = 13;
        if (p < s1) {
            const int64_t r = find_range(ia.rpre, r_lo, r_hi, p);
            j = (int64_t)ia.rbeg[r] + (p - ia.rpre[r]);
            c = ia.rcode[r];
            v.x = pos_s[j];
            v.y = pos_s[n + j];
            v.z = pos_s[2 * n + j];
            v.w = COUNT ? 0.0 : mass_s[j];
        }
        __syncthreads();
        tile[lane] = v;
        tj[lane] = j;
        tc[lane] = c;
        __syncthreads();
        for (int q = 0; q < kBlock; ++q) {
            const int64_t jj = tj[q];
            if (jj < 0 || jj == t) continue;
            const double4 sj = tile[q];
            const int cc = tc[q];
            // same operation order as the minimum-image difference:
            // (x_j - x_i), then the periodic shift
            const double dx = (sj.x - xi) + (double)(cc / 9 - 1) * L;
            const double dy = (sj.y - yi) + (double)((cc / 3) % 3 - 1) * L;
            const double dz = (sj.z - zi) + (double)(cc % 3 - 1) * L;
            const double s2 = dx * dx + dy * dy + dz * dz;
            if (!(s2 < rcut2)) continue;
            if (COUNT) {
                ++cnt;
                continue;
            }
            if (!(s2 > 0)) continue;
            const double se = sqrt(s2 + eps2);
            const double f = G * sj.w * split_factor_f64(se / (2.0 * rs)) / (se * se * se);
            ax += f * dx;
            ay += f * dy;
            az += f * dz;
        }
    }
    if (COUNT) {
        pcount[item * kBlock + lane] = cnt;
    } else {
        double* o = partial + item * 3 * kBlock;
        o[0 * kBlock + lane] = ax;
        o[1 * kBlock + lane] = ay;
        o[2 * kBlock + lane] = az;
    }
}
#pragma clang fp contract(on)

__global__ void __launch_bounds__(256) reduce_f64_kernel(const int64_t* __restrict__ ioff,
                                                         const double* __restrict__ partial,
                                                         const int32_t* __restrict__ perm,
                                                         int64_t n, double* __restrict__ acc) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int64_t b = t / kBlock;
    const int l = (int)(t % kBlock);
    double sx = 0, sy = 0, sz = 0;
    for (int64_t it = ioff[b]; it < ioff[b + 1]; ++it) {
        const double* o = partial + it * 3 * kBlock;
        sx += o[0 * kBlock + l];
        sy += o[1 * kBlock + l];
        sz += o[2 * kBlock + l];
    }
    const int64_t i = perm[t];
    acc[i] = sx;
    acc[n + i] = sy;
    acc[2 * n + i] = sz;
}

__global__ void __launch_bounds__(256) reduce_count_kernel(const int64_t* __restrict__ ioff,
                                                           const int32_t* __restrict__ pc,
                                                           const int32_t* __restrict__ perm,
                                                           int64_t n, int64_t* __restrict__ counts,
                                                           unsigned long long* __restrict__ total) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int64_t b = t / kBlock;
    const int l = (int)(t % kBlock);
    int64_t s = 0;
    for (int64_t it = ioff[b]; it < ioff[b + 1]; ++it) s += pc[it * kBlock + l];
    if (counts) counts[perm[t]] = s;
    atomicAdd(total, (unsigned long long)s);
}

ItemArgs item_args(const BlockLists& bl, int chunk) {
    ItemArgs ia;
    ia.iblock = bl.iblock.as<int32_t>();
    ia.is0 = bl.is0.as<int32_t>();
    ia.nitem = bl.nitem;
    ia.per_xcd = (bl.nitem + 7) / 8;
    ia.bbox = bl.box.as<IBox>();
    ia.roff = bl.roff.as<int64_t>();
    ia.rbeg = bl.rbeg.as<int32_t>();
    ia.rpre = bl.rpre.as<int32_t>();
    ia.rcode = bl.rcode.as<uint8_t>();
    ia.slen = bl.slen.as<int32_t>();
    ia.chunk = chunk;
    return ia;
}

}  // namespace

int make_poly(const pp_box_params& p, PolyF32* out) {
    const double k = p.rcut / (2.0 * p.rs);          // x = s_n k with s_n = s / rcut
    const double K = k * k * k;
    for (int j = 0; j <= SPLIT_POLY_DEGREE; ++j) out->c[j] = (float)(K * SPLIT_POLY_C[j]);
    out->tscale = (float)(2.0 * k * k / SPLIT_POLY_U_MAX);
    double e2 = (p.eps / p.rcut) * (p.eps / p.rcut);
    const double floor2 = ldexp(1.0, -60);          // keeps y^3 finite for s = eps = 0
    if (e2 < floor2) e2 = floor2;
    out->eps2n = (float)e2;
    out->cut2 = (float)(1.0 + e2);
    return PP_OK;
}

int launch_pp_f32(const BlockLists& bl, const double* pos_s, const float* mass_s, int64_t n,
                  const pp_box_params& p, const PolyF32& poly, int chunk, float* partial,
                  hipStream_t s) {
    if (bl.nitem == 0) return PP_OK;
    ItemArgs ia = item_args(bl, chunk);
    const double cell = p.L / (double)(1ll << p.key_bits);
    hipLaunchKernelGGL(pp_f32_kernel<false>, dim3((unsigned)(ia.per_xcd * 8)), dim3(kBlock), 0, s,
                       ia, pos_s, mass_s, n, p.L, cell, 1.0 / p.rcut, poly, partial);
    PP_HIP(hipGetLastError());
    return PP_OK;
}

int launch_reduce_f32(const BlockLists& bl, const float* partial, const int32_t* perm, int64_t n,
                      double scale, float* acc, hipStream_t s) {
    if (n == 0) return PP_OK;
    hipLaunchKernelGGL(reduce_f32_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s,
                       bl.ioff.as<int64_t>(), partial, perm, n, scale, acc);
    PP_HIP(hipGetLastError());
    return PP_OK;
}

int launch_pp_f64(const BlockLists& bl, const double* pos_s, const double* mass_s, int64_t n,
                  const pp_box_params& p, int chunk, double* partial, hipStream_t s) {
    if (bl.nitem == 0) return PP_OK;
    ItemArgs ia = item_args(bl, chunk);
    hipLaunchKernelGGL(pp_f64_kernel<false>, dim3((unsigned)(ia.per_xcd * 8)), dim3(kBlock), 0, s,
                       ia, pos_s, mass_s, n, p.L, p.rs, p.rcut, p.eps, p.G, partial,
                       (int32_t*)nullptr);
    PP_HIP(hipGetLastError());
    return PP_OK;
}

int launch_reduce_f64(const BlockLists& bl, const double* partial, const int32_t* perm, int64_t n,
                      double* acc, hipStream_t s) {
    if (n == 0) return PP_OK;
    hipLaunchKernelGGL(reduce_f64_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s,
                       bl.ioff.as<int64_t>(), partial, perm, n, acc);
    PP_HIP(hipGetLastError());
    return PP_OK;
}

int launch_count(const BlockLists& bl, const double* pos_s, int64_t n, const pp_box_params& p,
                 int chunk, int32_t* partial_counts, hipStream_t s) {
    if (bl.nitem == 0) return PP_OK;
    ItemArgs ia = item_args(bl, chunk);
    hipLaunchKernelGGL(pp_f64_kernel<true>, dim3((unsigned)(ia.per_xcd * 8)), dim3(kBlock), 0, s,
                       ia, pos_s, (const double*)nullptr, n, p.L, p.rs, p.rcut, p.eps, p.G,
                       (double*)nullptr, partial_counts);
    PP_HIP(hipGetLastError());
    return PP_OK;
}

int launch_reduce_count(const BlockLists& bl, const int32_t* partial, const int32_t* perm,
                        int64_t n, int64_t* counts, unsigned long long* total, hipStream_t s) {
    if (n == 0) return PP_OK;
    hipLaunchKernelGGL(reduce_count_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s,
                       bl.ioff.as<int64_t>(), partial, perm, n, counts, total);
    PP_HIP(hipGetLastError());
    return PP_OK;
}

}  // namespace pp
