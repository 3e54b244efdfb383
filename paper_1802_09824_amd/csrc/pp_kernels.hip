// The PP (particle-particle) kernels: short-range pair sums over the block
// lists, FP32 (the hot path), FP64 (the yardstick) and an FP64 pair count.
//
// Per pair (sec. 3.1, Eq. equ:split, with Plummer softening):
//   a_i += G m_j d g(s_eps / 2 r_s) / s_eps^3,   kept iff s < r_cut.
// FP32 form.  Lengths are in units of ell = 2 r_s sqrt(U_MAX / 2),
// relative to the FP64 centre of the target block (the origin subtraction
// is done in FP64 when a source is staged, so the FP32 offsets are small
// and precise).  With g(x) = 1 - x^3 H(x^2), H a polynomial fitted on
// u = x^2 in [0, U_MAX] in the variable t = 2u / U_MAX - 1 (split_poly.h),
// r2 = s_eps^2 / ell^2 and y = 1 / sqrt(r2) (hardware reciprocal square
// root), the unit makes t = r2 - 1 and
//   ell^3 g / s_eps^3 = y^3 - (U_MAX / 2)^(3/2) H(u),
// so the polynomial's coefficients are the same literals for every box and
// G / ell^2 scales the sum at the end.  Softening enters r2 through the
// first fused multiply-add; the cut test compares r2 with
// (r_cut^2 + eps^2) / ell^2.  Every operand of the pair arithmetic is a
// VGPR or a literal: on gfx950 two waves' VALU instructions issue together
// only then.
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

struct ItemArgs {
    const int32_t* iblock;
    const int32_t* is0;
    const int64_t* sizes;      // the counts of the lists (SizeSlot), on the device
    const int32_t* bstart;
    const int32_t* bcount;
    const IBox* bbox;
    const int32_t* bboxid;
    const int64_t* roff;
    const int32_t* rbeg;
    const int32_t* rpre;
    const uint8_t* rcode;
    const int32_t* slen;
    const int64_t* ioff;
    const BoxDev* box;
    const int32_t* perm;       // key order -> input order
    const int32_t* mass_flag;  // per box: 1 where the masses are not all equal
    const float4* split_tab;   // the interpolated split table (variant bit 8)
    float* acc;                // FP32 output (single-item blocks write it directly)
    const uint8_t* active;     // per input particle: outputs written only where set (null: all)
};

__device__ __forceinline__ bool target_on(const ItemArgs& ia, int64_t i) {
    return !ia.active || ia.active[i] != 0;
}

ItemArgs item_args(const BatchDev& bd, const Work& w) {
    ItemArgs ia;
    ia.iblock = w.iblock.as<int32_t>();
    ia.is0 = w.is0.as<int32_t>();
    ia.sizes = w.sizes.as<int64_t>();
    ia.bstart = w.bstart.as<int32_t>();
    ia.bcount = w.bcount.as<int32_t>();
    ia.bbox = w.bbox.as<IBox>();
    ia.bboxid = w.bboxid.as<int32_t>();
    ia.roff = w.roff.as<int64_t>();
    ia.rbeg = w.rbeg.as<int32_t>();
    ia.rpre = w.rpre.as<int32_t>();
    ia.rcode = w.rcode.as<uint8_t>();
    ia.slen = w.slen.as<int32_t>();
    ia.ioff = w.ioff.as<int64_t>();
    ia.box = bd.box;
    ia.perm = w.perm.as<int32_t>();
    ia.mass_flag = w.mass_flag.as<int32_t>();
    ia.split_tab = w.split_tab.as<float4>();
    ia.acc = nullptr;
    ia.active = w.active;
    return ia;
}

// Items are laid out so that the 8 XCDs (which take workgroups round-robin)
// each see one contiguous stretch of items: neighbouring target blocks share
// most of their sources, which then stay in that XCD's L2.  The grid is
// sized for the item capacity, which may exceed the count: a workgroup past
// its XCD's stretch gets -1 (mapping it into the next stretch would run
// that item twice).
__device__ __forceinline__ int64_t xcd_item(int64_t bid, int64_t nitem) {
    const int64_t per_xcd = (nitem + 7) / 8;
    const int64_t k = bid >> 3;
    const int64_t item = (bid & 7) * per_xcd + k;
    return k < per_xcd && item < nitem ? item : -1;
}

__device__ __forceinline__ int64_t find_range(const int32_t* __restrict__ rpre, int64_t lo,
                                              int64_t hi, int32_t p) {
    // last r in [lo, hi] with rpre[r] <= p (rpre ascending, rpre[lo] <= p)
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (rpre[mid] <= p) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// The same search by a whole wave, for a wave-uniform p: each round reads
// 64 evenly spaced entries and keeps the stretch between two of them, so
// the dependent loads number log_64 of the range count instead of log_2.
__device__ __forceinline__ int64_t find_range_wave(const int32_t* __restrict__ rpre, int64_t lo,
                                                   int64_t hi, int32_t p) {
    const int lane = threadIdx.x & 63;
    while (lo < hi) {
        const int64_t stride = (hi - lo + 64) / 64;   // ceil((hi - lo + 1) / 64)
        const int64_t q = lo + lane * stride;
        const bool le = q <= hi && rpre[q] <= p;
        const int c = __popcll(__ballot(le));        // >= 1: rpre[lo] <= p
        lo += (int64_t)(c - 1) * stride;
        const int64_t top = lo + stride - 1;
        hi = top < hi ? top : hi;
        if (stride == 1) break;
    }
    return lo;
}

constexpr double csqrt(double x) {
    double r = x > 1.0 ? x : 1.0;
    for (int i = 0; i < 64; ++i) r = 0.5 * (r + x / r);
    return r;
}
// (U_MAX / 2)^(3/2): H's factor in the length unit ell
constexpr double kHScale = 0.5 * SPLIT_POLY_U_MAX * csqrt(0.5 * SPLIT_POLY_U_MAX);
// H's coefficients times (U_MAX / 2)^(3/2), rounded once to FP32: the pair
// loop's literal operands
struct HCoef {
    float c[SPLIT_POLY_DEGREE + 1];
};
constexpr HCoef make_hcoef() {
    HCoef h{};
    for (int j = 0; j <= SPLIT_POLY_DEGREE; ++j) h.c[j] = (float)(kHScale * SPLIT_POLY_C[j]);
    return h;
}
constexpr HCoef kHC = make_hcoef();

// (U_max/2)^{3/2} H(u) at r2 = s_eps^2 / ell^2: the polynomial in t = r2 - 1
// (Horner, one FMA per degree), or (TABLE) the interpolated table of the
// paper's design: kTabN quadratic pieces over r2 in [0, 2), each stored as
// (a, b, c) with h = a + z (b + z c), z the position inside the piece.  Past r2 = 2 the
// last piece is extrapolated; such pairs lie beyond the cut and are masked.
constexpr int kTabN = 128;

template <bool TABLE>
__device__ __forceinline__ float split_h(float r2, const float4* __restrict__ tab) {
    if (TABLE) {
        const float sidx = r2 * (float)(kTabN / 2);
        int k = (int)sidx;
        k = k < kTabN - 1 ? k : kTabN - 1;
        const float z = sidx - (float)k;
        const float4 c = tab[k];
        return fmaf(fmaf(c.z, z, c.y), z, c.x);
    }
    const float t = r2 - 1.f;
    float h = kHC.c[SPLIT_POLY_DEGREE];
#pragma unroll
    for (int j = SPLIT_POLY_DEGREE - 1; j >= 0; --j) h = fmaf(h, t, kHC.c[j]);
    return h;
}

// One source against the lane's target; adds into (tx, ty, tz).
template <bool NEWTON, bool TABLE = false>
__device__ __forceinline__ void pair_f32(const float4 sj, float xi, float yi, float zi,
                                         const PolyF32& P, float& tx, float& ty, float& tz,
                                         const float4* __restrict__ tab = nullptr) {
    const float dx = sj.x - xi, dy = sj.y - yi, dz = sj.z - zi;
    float r2 = fmaf(dx, dx, P.eps2n);
    r2 = fmaf(dy, dy, r2);
    r2 = fmaf(dz, dz, r2);
    float y = __builtin_amdgcn_rsqf(r2);
    if (NEWTON) y = y * fmaf(-0.5f * r2 * y, y, 1.5f);
    const float h = split_h<TABLE>(r2, tab);
    float F = fmaf(y * y, y, -h) * sj.w;
    F = r2 < P.cut2 ? F : 0.f;
    tx = fmaf(F, dx, tx);
    ty = fmaf(F, dy, ty);
    tz = fmaf(F, dz, tz);
}

// The same for a box whose masses are all equal: the source's w slot holds
// the cut on r2 instead of the mass (which joins the final scale), so the
// tile keeps its 16-byte entries and the mass multiply drops out.
template <bool NEWTON, bool TABLE = false>
__device__ __forceinline__ void pair_f32_eq(const float4 sj, float xi, float yi, float zi,
                                            float& tx, float& ty, float& tz, float eps2,
                                            const float4* __restrict__ tab = nullptr) {
    const float dx = sj.x - xi, dy = sj.y - yi, dz = sj.z - zi;
    float r2 = fmaf(dx, dx, eps2);
    r2 = fmaf(dy, dy, r2);
    r2 = fmaf(dz, dz, r2);
    float y = __builtin_amdgcn_rsqf(r2);
    if (NEWTON) y = y * fmaf(-0.5f * r2 * y, y, 1.5f);
    const float h = split_h<TABLE>(r2, tab);
    float F = fmaf(y * y, y, -h);
    F = r2 < sj.w ? F : 0.f;
    tx = fmaf(F, dx, tx);
    ty = fmaf(F, dy, ty);
    tz = fmaf(F, dz, tz);
}

__device__ __forceinline__ void kahan_add(float& s, float& c, float v) {
    const float y = v - c;
    const float t = s + y;
    c = (t - s) - y;
    s = t;
}

// Orders this wave's LDS accesses around a point.  Every caller works on
// LDS that only its own wave touches (a workgroup of K waves gives each wave
// its own slices), and a wave's LDS operations complete in issue order, so
// no s_barrier is needed.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ float readlane_f(float v, int lane) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

__device__ __forceinline__ int64_t readlane64(int64_t v, int lane) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, lane);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), lane);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// One work item of the FP32 PP kernel on one wave (target block, chunk of
// its source list).  Sources are fetched 64 list positions at a time.  A
// window inside the range at the wave's range cursor needs no mapping;
// otherwise the wave reads the 64 ranges from the cursor on (one per lane),
// marks in LDS the window positions where one of them starts, and each lane
// takes its position's range from the count of marks up to it and the
// range's first particle from the lane that read it; only a window that
// runs past those 64 ranges falls back to a binary search per lane.  Then each lane loads
// the FP64 position and the mass; the loads of the next window are issued
// before the current tile is swept.  A fetched source is shifted by its periodic image, made
// relative to the FP64 block centre, scaled by 1/ell and rounded to FP32,
// and dropped if it lies at r_cut or more from each of the four boxes
// around the block's runs of 16 targets.  Survivors are compacted with a
// ballot into a 128-entry LDS ring; every 64 survivors are swept by all
// lanes with broadcast LDS reads.
//
// K waves may share one item (the workgroup is K waves): wave k takes the
// windows k, k + K, k + 2K, ... of the item's list, stages and sweeps them
// into its own LDS ring and its own compensated sums, and the K sums are
// added in wave order in FP64 (through LDS) before the item's result is
// written.  The split does not depend on scheduling, so results stay
// reproducible for a given K.
template <int VAR, int K>
__device__ __forceinline__ void pp_item(const ItemArgs& ia, int64_t item,
                                        const double* __restrict__ pos_s,
                                        const float* __restrict__ mass_s, int64_t N,
                                        float* __restrict__ partial,
                                        unsigned long long& n_eval, unsigned long long& n_lane,
                                        float4* tile_all,
                                        const float4* __restrict__ tab, float4* qb_all,
                                        double* red, int* mark_all) {
    constexpr bool NEWTON = (VAR & 1) != 0;
    constexpr bool KAHAN = (VAR & 2) == 0;
    constexpr bool LOCAL = (VAR & 4) == 0;     // FP64 block-centre subtraction
    constexpr bool TABLE = (VAR & 8) != 0;     // interpolated split table
    const int lane = threadIdx.x & (kBlock - 1);
    const int wv = K > 1 ? (int)(threadIdx.x / kBlock) : 0;
    float4* tile = tile_all + wv * 2 * kBlock;
    const int32_t b = ia.iblock[item];
    const int32_t s0 = ia.is0[item];
    const int32_t S = ia.slen[b];
    const int32_t chunk = (int32_t)ia.sizes[kChunk];
    const int32_t s1 = s0 + chunk < S ? s0 + chunk : S;
    const int32_t nt = ia.bcount[b];
    const int xbox = ia.bboxid[b];
    const BoxDev& X = ia.box[xbox];
    const double L = X.L, cell = X.cell, inv_len = X.inv_len;
    const PolyF32 P = X.poly;
    // equal masses (the compensated form only): the mass joins the final scale
    const bool equal = KAHAN && ia.mass_flag[xbox] == 0;
    const float mu = equal ? mass_s[X.poff] : 1.f;
    const IBox B = ia.bbox[b];
    const double ox = 0.5 * (double)(B.lo[0] + B.hi[0]) * cell;
    const double oy = 0.5 * (double)(B.lo[1] + B.hi[1]) * cell;
    const double oz = 0.5 * (double)(B.lo[2] + B.hi[2]) * cell;
    // half sides of the block box in units of ell, widened slightly so the
    // pruning test can only keep too much
    const float hx = (float)(0.5 * (double)(B.hi[0] - B.lo[0]) * cell * inv_len) * 1.0001f + 1e-6f;
    const float hy = (float)(0.5 * (double)(B.hi[1] - B.lo[1]) * cell * inv_len) * 1.0001f + 1e-6f;
    const float hz = (float)(0.5 * (double)(B.hi[2] - B.lo[2]) * cell * inv_len) * 1.0001f + 1e-6f;
    const float keep2 = P.keep2;
    const int64_t t = (int64_t)ia.bstart[b] + lane;
    float xi = 0.f, yi = 0.f, zi = 0.f;
    if (lane < nt) {
        xi = (float)((pos_s[t] - (LOCAL ? ox : 0.0)) * inv_len);
        yi = (float)((pos_s[N + t] - (LOCAL ? oy : 0.0)) * inv_len);
        zi = (float)((pos_s[2 * N + t] - (LOCAL ? oz : 0.0)) * inv_len);
    }
    // Four boxes around the FP32 offsets of the four runs of 16 consecutive
    // targets (key order), kept in LDS: a source is staged when it comes
    // within the cut of any of them, which drops about 5 % of the sources
    // that pass the whole block's box.  Widened like the block box.
    constexpr int GROUPS = 4;
    constexpr int GW = kBlock / GROUPS;
    float4* qb = qb_all + wv * 2 * GROUPS;
    if (LOCAL) {
        float ax_ = lane < nt ? xi : INFINITY, bx_ = lane < nt ? xi : -INFINITY;
        float ay_ = lane < nt ? yi : INFINITY, by_ = lane < nt ? yi : -INFINITY;
        float az_ = lane < nt ? zi : INFINITY, bz_ = lane < nt ? zi : -INFINITY;
#pragma unroll
        for (int m = 1; m < GW; m <<= 1) {
            ax_ = fminf(ax_, __shfl_xor(ax_, m));
            bx_ = fmaxf(bx_, __shfl_xor(bx_, m));
            ay_ = fminf(ay_, __shfl_xor(ay_, m));
            by_ = fmaxf(by_, __shfl_xor(by_, m));
            az_ = fminf(az_, __shfl_xor(az_, m));
            bz_ = fmaxf(bz_, __shfl_xor(bz_, m));
        }
        // an empty group repeats group 0
        {
            const bool empty = lane >= nt;
            const float r0 = readlane_f(ax_, 0), r1 = readlane_f(bx_, 0), r2 = readlane_f(ay_, 0);
            const float r3 = readlane_f(by_, 0), r4 = readlane_f(az_, 0), r5 = readlane_f(bz_, 0);
            ax_ = empty ? r0 : ax_;
            bx_ = empty ? r1 : bx_;
            ay_ = empty ? r2 : ay_;
            by_ = empty ? r3 : by_;
            az_ = empty ? r4 : az_;
            bz_ = empty ? r5 : bz_;
        }
        wave_sync();
        if (lane % GW == 0) {
            const int g = lane / GW;
            qb[2 * g] = make_float4(0.5f * (ax_ + bx_), 0.5f * (ay_ + by_), 0.5f * (az_ + bz_),
                                    0.5f * (bx_ - ax_) * 1.0001f + 1e-6f);
            qb[2 * g + 1] = make_float4(0.5f * (by_ - ay_) * 1.0001f + 1e-6f,
                                        0.5f * (bz_ - az_) * 1.0001f + 1e-6f, 0.f, 0.f);
        }
        wave_sync();
    }
    const int64_t r_lo = ia.roff[b], r_hi = ia.roff[b + 1] - 1;
    float ax = 0.f, ay = 0.f, az = 0.f, cx = 0.f, cy = 0.f, cz = 0.f;
    int count = 0;                                   // staged sources (wave-uniform)
    int64_t staged = 0;
    const int32_t first = s0 + wv * kBlock;          // this wave's first window
    int64_t rcur = s1 > first ? find_range_wave(ia.rpre, r_lo, r_hi, first) : r_lo;
    int* mark = mark_all + wv * kBlock;

    double px = 0, py = 0, pz = 0;
    float pm = 0.f;
    int pc = 13;
    bool pv = false;
    auto fetch = [&](int32_t base) {
        const int32_t p = base + lane;
        pv = p < s1;
        const int32_t last = s1 - 1 < base + kBlock - 1 ? s1 - 1 : base + kBlock - 1;
        int64_t r;
        int32_t rb, rp;
        int code;
        const int32_t end_cur = rcur < r_hi ? ia.rpre[rcur + 1] : S;
        if (last < end_cur) {
            // the cursor's range holds the whole window: nothing to map
            r = rcur;
            rb = ia.rbeg[rcur];
            rp = ia.rpre[rcur];
            code = ia.rcode[rcur];
        } else {
            // the ranges rcur .. rcur + 63, one per lane
            const int64_t rq = rcur + lane;
            const bool rv = rq <= r_hi;
            const int32_t qpre = rv ? ia.rpre[rq] : INT32_MAX;
            const int32_t qbeg = rv ? ia.rbeg[rq] : 0;
            const int qcode = rv ? (int)ia.rcode[rq] : 13;
            // ranges that start at or before the window's first (last) position
            const int c0 = __popcll(__ballot(qpre <= base));
            const int c1 = __popcll(__ballot(qpre <= last));
            if (c1 < kBlock || rcur + (kBlock - 1) >= r_hi) {
                // every range of the window was read: mark where they start
                mark[lane] = 0;
                wave_sync();
                if (qpre > base && qpre <= last) mark[qpre - base] = 1;
                wave_sync();
                const uint64_t starts = __ballot(mark[lane] != 0);
                wave_sync();
                const uint64_t upto = lane == 63 ? ~0ull : (2ull << lane) - 1ull;
                const int idx = c0 - 1 + __popcll(starts & upto);
                rb = __shfl(qbeg, idx);
                rp = __shfl(qpre, idx);
                code = __shfl(qcode, idx);
                r = rcur + idx;
            } else {
                // more than 64 ranges in reach: the window starts at most K * 64
                // positions (so ranges) past the cursor's
                const int64_t top = rcur + K * kBlock < r_hi ? rcur + K * kBlock : r_hi;
                r = pv ? find_range(ia.rpre, rcur, top, p) : rcur;
                rb = ia.rbeg[r];
                rp = ia.rpre[r];
                code = ia.rcode[r];
            }
        }
        if (pv) {
            const int64_t j = (int64_t)rb + (p - rp);
            pc = code;
            px = pos_s[j];
            py = pos_s[N + j];
            pz = pos_s[2 * N + j];
            pm = mass_s[j];
        }
        rcur = readlane64(r, kBlock - 1);
    };
    wave_sync();
    if (first < s1) fetch(first);
    for (int32_t base = first; base < s1; base += K * kBlock) {
        bool keep = false;
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (pv) {
            const double sx = (double)(pc / 9 - 1) * L;
            const double sy = (double)((pc / 3) % 3 - 1) * L;
            const double sz = (double)(pc % 3 - 1) * L;
            v.x = (float)((px + sx - ox) * inv_len);
            v.y = (float)((py + sy - oy) * inv_len);
            v.z = (float)((pz + sz - oz) * inv_len);
            v.w = equal ? P.cut2 : pm;
            if (LOCAL) {
#pragma unroll
                for (int g = 0; g < GROUPS; ++g) {
                    const float4 c = qb[2 * g], h = qb[2 * g + 1];
                    const float gx = fmaxf(fabsf(v.x - c.x) - c.w, 0.f);
                    const float gy = fmaxf(fabsf(v.y - c.y) - h.x, 0.f);
                    const float gz = fmaxf(fabsf(v.z - c.z) - h.y, 0.f);
                    keep = keep || fmaf(gx, gx, fmaf(gy, gy, gz * gz)) < keep2;
                }
            } else {
                const float gx = fmaxf(fabsf(v.x) - hx, 0.f);
                const float gy = fmaxf(fabsf(v.y) - hy, 0.f);
                const float gz = fmaxf(fabsf(v.z) - hz, 0.f);
                keep = fmaf(gx, gx, fmaf(gy, gy, gz * gz)) < keep2;
            }
            if (!LOCAL) {
                v.x = (float)((px + sx) * inv_len);
                v.y = (float)((py + sy) * inv_len);
                v.z = (float)((pz + sz) * inv_len);
            }
        }
        const uint64_t bal = __ballot(keep);
        const int rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32),
                                                   __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
        if (keep) tile[count + rank] = v;
        const int got = __popcll(bal);
        count += got;
        staged += got;
        // the next window's loads stay in flight while this tile is swept
        if (base + K * kBlock < s1) fetch(base + K * kBlock);
        if (count >= kBlock) {
            wave_sync();
            float tx = 0.f, ty = 0.f, tz = 0.f;
            if (KAHAN) {
                if (equal) {
#pragma unroll 8
                    for (int q = 0; q < kBlock; ++q)
                        pair_f32_eq<NEWTON, TABLE>(tile[q], xi, yi, zi, tx, ty, tz, P.eps2n, tab);
                } else {
#pragma unroll 8
                    for (int q = 0; q < kBlock; ++q) pair_f32<NEWTON, TABLE>(tile[q], xi, yi, zi, P, tx, ty, tz, tab);
                }
                kahan_add(ax, cx, tx);
                kahan_add(ay, cy, ty);
                kahan_add(az, cz, tz);
            } else {
#pragma unroll 8
                for (int q = 0; q < kBlock; ++q) pair_f32<NEWTON, TABLE>(tile[q], xi, yi, zi, P, ax, ay, az, tab);
            }
            wave_sync();
            count -= kBlock;
            if (lane < count) tile[lane] = tile[kBlock + lane];
            wave_sync();
        }
    }
    if (count > 0) {
        wave_sync();
        float tx = 0.f, ty = 0.f, tz = 0.f;
        if (KAHAN) {
            if (equal) {
                for (int q = 0; q < count; ++q) pair_f32_eq<NEWTON, TABLE>(tile[q], xi, yi, zi, tx, ty, tz, P.eps2n, tab);
            } else {
                for (int q = 0; q < count; ++q) pair_f32<NEWTON, TABLE>(tile[q], xi, yi, zi, P, tx, ty, tz, tab);
            }
            kahan_add(ax, cx, tx);
            kahan_add(ay, cy, ty);
            kahan_add(az, cz, tz);
        } else {
            for (int q = 0; q < count; ++q) pair_f32<NEWTON, TABLE>(tile[q], xi, yi, zi, P, ax, ay, az, tab);
        }
    }
    n_eval += (unsigned long long)staged * (unsigned long long)nt;
    n_lane += (unsigned long long)staged * (unsigned long long)kBlock;
    // the compensated sums, then (K > 1) the waves' sums in wave order
    double sx = (double)ax - (double)cx, sy = (double)ay - (double)cy, sz = (double)az - (double)cz;
    if (K > 1) {
        __syncthreads();                 // every wave is done with the previous item's sums
        red[(wv * 3 + 0) * kBlock + lane] = sx;
        red[(wv * 3 + 1) * kBlock + lane] = sy;
        red[(wv * 3 + 2) * kBlock + lane] = sz;
        __syncthreads();
        if (wv != 0) return;
        sx = red[0 * kBlock + lane];
        sy = red[1 * kBlock + lane];
        sz = red[2 * kBlock + lane];
#pragma unroll
        for (int k = 1; k < K; ++k) {
            sx += red[(k * 3 + 0) * kBlock + lane];
            sy += red[(k * 3 + 1) * kBlock + lane];
            sz += red[(k * 3 + 2) * kBlock + lane];
        }
    }
    if (ia.acc && ia.ioff[b + 1] - ia.ioff[b] == 1) {
        // the block's only item: finish here, with the reduction's arithmetic
        if (lane < nt && target_on(ia, ia.perm[t])) {
            const int64_t i = ia.perm[t];
            const double sc = X.scale * (double)mu;
            ia.acc[i] = (float)(sx * sc);
            ia.acc[N + i] = (float)(sy * sc);
            ia.acc[2 * N + i] = (float)(sz * sc);
        }
        return;
    }
    // the compensated sum (times the equal mass, if any), rounded once
    float* o = partial + item * 3 * kBlock;
    o[0 * kBlock + lane] = (float)(sx * (double)mu);
    o[1 * kBlock + lane] = (float)(sy * (double)mu);
    o[2 * kBlock + lane] = (float)(sz * (double)mu);
}

// Monopoles (sec. 3.3, 1 to N): one wave per target block walks the block's
// entries of the list expansion in order.  An entry contributes the node it
// stands for when the breadth-first expansion accepted it, and the leaves and
// groups of 8 leaves the depth-first walk accepted under it.  Each accepted
// node becomes a source of its mass at its centre of mass (FP64 sums,
// shifted by its periodic image, relative to the FP64 block centre, in units
// of ell), staged into an LDS ring like the particles of pp_item and swept
// with the same pair arithmetic and the same cut.  The result is added to
// the accelerations the PP path wrote.
__global__ void __launch_bounds__(64) monopole_kernel(ItemArgs ia, const FEntry* __restrict__ ent,
                                                      const int64_t* __restrict__ eoff,
                                                      const uint64_t* __restrict__ mono0,
                                                      const uint8_t* __restrict__ mono1,
                                                      const TreeView* __restrict__ tvs,
                                                      const double4* __restrict__ mc,
                                                      const double* __restrict__ pos_s, int64_t N,
                                                      int64_t nblock,
                                                      unsigned long long* __restrict__ counter) {
    __shared__ float4 tile[2 * kBlock];
    const int64_t b = blockIdx.x;
    if (ia.sizes[kSkip] || b >= ia.sizes[kNBlock]) return;
    (void)nblock;
    if (ia.ioff[b + 1] == ia.ioff[b]) return;        // a block without active targets
    const int lane = threadIdx.x;
    const int xbox = ia.bboxid[b];
    const BoxDev& X = ia.box[xbox];
    const TreeView& tv = tvs[xbox];
    const double L = X.L, cell = X.cell, inv_len = X.inv_len;
    const PolyF32 P = X.poly;
    const IBox B = ia.bbox[b];
    const double ox = 0.5 * (double)(B.lo[0] + B.hi[0]) * cell;
    const double oy = 0.5 * (double)(B.lo[1] + B.hi[1]) * cell;
    const double oz = 0.5 * (double)(B.lo[2] + B.hi[2]) * cell;
    const int32_t nt = ia.bcount[b];
    const int64_t t = (int64_t)ia.bstart[b] + lane;
    float xi = 0.f, yi = 0.f, zi = 0.f;
    if (lane < nt) {
        xi = (float)((pos_s[t] - ox) * inv_len);
        yi = (float)((pos_s[N + t] - oy) * inv_len);
        zi = (float)((pos_s[2 * N + t] - oz) * inv_len);
    }
    float ax = 0.f, ay = 0.f, az = 0.f, cx = 0.f, cy = 0.f, cz = 0.f;
    int count = 0;
    int64_t taken = 0;
    // stage this lane's node (level, index) under shift code sc if `on`
    auto stage = [&](bool on, int lev, int64_t node, int sc) {
        bool keep = false;
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (on) {
            const double4 m = mc[tv.off[lev] + node];
            if (m.w > 0.0) {
                keep = true;
                const double sx = (double)(sc / 9 - 1) * L;
                const double sy = (double)((sc / 3) % 3 - 1) * L;
                const double sz = (double)(sc % 3 - 1) * L;
                v.x = (float)((m.x / m.w + sx - ox) * inv_len);
                v.y = (float)((m.y / m.w + sy - oy) * inv_len);
                v.z = (float)((m.z / m.w + sz - oz) * inv_len);
                v.w = (float)m.w;
            }
        }
        const uint64_t bal = __ballot(keep);
        const int rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32),
                                                   __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
        if (keep) tile[count + rank] = v;
        const int got = __popcll(bal);
        count += got;
        taken += got;
        if (count >= kBlock) {
            wave_sync();
            float tx = 0.f, ty = 0.f, tz = 0.f;
            for (int q = 0; q < kBlock; ++q) pair_f32<false>(tile[q], xi, yi, zi, P, tx, ty, tz);
            kahan_add(ax, cx, tx);
            kahan_add(ay, cy, ty);
            kahan_add(az, cz, tz);
            wave_sync();
            count -= kBlock;
            if (lane < count) tile[lane] = tile[kBlock + lane];
            wave_sync();
        }
    };
    const int64_t e_end = eoff[b + 1];
    // nodes the breadth-first expansion accepted: one per entry, 64 entries
    // at a time
    for (int64_t e0 = eoff[b]; e0 < e_end; e0 += kBlock) {
        const int64_t e = e0 + lane;
        FEntry E{};
        const bool in = e < e_end;
        if (in) E = ent[e];
        stage(in && E.mono, E.lev, E.node, E.sc);
    }
    // leaves and groups of 8 leaves the depth-first walk accepted
    if (mono0) {
        for (int64_t e = eoff[b]; e < e_end; ++e) {
            const uint64_t m0 = mono0[e];
            const uint32_t m1 = mono1[e];
            if ((m0 | m1) == 0) continue;
            const FEntry E = ent[e];
            const int64_t first = (int64_t)E.node << (3 * E.lev);
            if (m0) stage((m0 >> lane) & 1ull, 0, first + lane, E.sc);
            if (m1) stage(lane < 8 && ((m1 >> lane) & 1u), 1, (first >> 3) + lane, E.sc);
        }
    }
    if (count > 0) {
        wave_sync();
        float tx = 0.f, ty = 0.f, tz = 0.f;
        for (int q = 0; q < count; ++q) pair_f32<false>(tile[q], xi, yi, zi, P, tx, ty, tz);
        kahan_add(ax, cx, tx);
        kahan_add(ay, cy, ty);
        kahan_add(az, cz, tz);
    }
    if (taken == 0) return;
    if (lane < nt && target_on(ia, ia.perm[t])) {
        const int64_t i = ia.perm[t];
        ia.acc[i] += (float)(((double)ax - (double)cx) * X.scale);
        ia.acc[N + i] += (float)(((double)ay - (double)cy) * X.scale);
        ia.acc[2 * N + i] += (float)(((double)az - (double)cz) * X.scale);
    }
    if (counter && lane == 0) atomicAdd(counter, (unsigned long long)taken * (unsigned long long)nt);
}

// One workgroup per item.
// Both forms are bounded to 6 waves per SIMD (80 VGPRs) with one wave per
// block and to 5 with more: two waves' VALU instructions can issue in the
// same cycle, so more resident waves keep the pair loop's issue slots
// fuller.
template <int VAR, int K>
__global__ void __launch_bounds__(64 * K, K > 1 ? 5 : 6) pp_f32_kernel(ItemArgs ia, const double* __restrict__ pos_s,
                                                        const float* __restrict__ mass_s, int64_t N,
                                                        float* __restrict__ partial,
                                                        unsigned long long* __restrict__ counters) {
    __shared__ float4 tile[K * 2 * kBlock];
    __shared__ float4 qb[K * 8];
    __shared__ double red[K > 1 ? K * 3 * kBlock : 1];
    __shared__ float4 tab[(VAR & 8) ? kTabN : 1];
    __shared__ int mark[K * kBlock];
    if (ia.sizes[kSkip]) return;
    const int64_t nitem = ia.sizes[kNItem];
    const int64_t item = xcd_item(blockIdx.x, nitem);
    if (item < 0) return;
    if (VAR & 8) {
        for (int k = threadIdx.x; k < kTabN; k += 64 * K) tab[k] = ia.split_tab[k];
        __syncthreads();
    }
    unsigned long long n_eval = 0, n_lane = 0;
    pp_item<VAR, K>(ia, item, pos_s, mass_s, N, partial, n_eval, n_lane, tile, tab, qb, red, mark);
    if (counters && (threadIdx.x & (kBlock - 1)) == 0) {
        atomicAdd(counters, n_eval);
        atomicAdd(counters + 1, n_lane);
    }
}

// The same for launches of at most two waves per SIMD (short item lists,
// small boxes): compiled for two resident waves, so the register budget
// lets the compiler keep more of the unrolled sweep's pairs in flight, which
// a SIMD with only two waves to issue from needs.  Same arithmetic in the
// same order, so the same results.
template <int VAR, int K>
__global__ void __launch_bounds__(64 * K, 2) pp_f32_kernel_few(ItemArgs ia, const double* __restrict__ pos_s,
                                                               const float* __restrict__ mass_s, int64_t N,
                                                               float* __restrict__ partial,
                                                               unsigned long long* __restrict__ counters) {
    __shared__ float4 tile[K * 2 * kBlock];
    __shared__ float4 qb[K * 8];
    __shared__ double red[K > 1 ? K * 3 * kBlock : 1];
    __shared__ float4 tab[(VAR & 8) ? kTabN : 1];
    __shared__ int mark[K * kBlock];
    if (ia.sizes[kSkip]) return;
    const int64_t nitem = ia.sizes[kNItem];
    const int64_t item = xcd_item(blockIdx.x, nitem);
    if (item < 0) return;
    if (VAR & 8) {
        for (int k = threadIdx.x; k < kTabN; k += 64 * K) tab[k] = ia.split_tab[k];
        __syncthreads();
    }
    unsigned long long n_eval = 0, n_lane = 0;
    pp_item<VAR, K>(ia, item, pos_s, mass_s, N, partial, n_eval, n_lane, tile, tab, qb, red, mark);
    if (counters && (threadIdx.x & (kBlock - 1)) == 0) {
        atomicAdd(counters, n_eval);
        atomicAdd(counters + 1, n_lane);
    }
}

// Persistent form: a fixed grid of waves pulls items from 8 queues (one
// contiguous stretch of items per XCD, as above); a wave first drains the
// queue of its own XCD, then steals from the others.  Every wave leaves
// once all queues are empty.  The item count is read from device memory,
// so the launch can be replayed from a graph while the lists change.
template <int VAR, int K>
__global__ void __launch_bounds__(64 * K, K > 1 ? 5 : 6) pp_f32_persistent(ItemArgs ia,
                                                            const double* __restrict__ pos_s,
                                                            const float* __restrict__ mass_s, int64_t N,
                                                            float* __restrict__ partial,
                                                            unsigned long long* __restrict__ counters,
                                                            unsigned* __restrict__ queues) {
    __shared__ float4 tile[K * 2 * kBlock];
    __shared__ float4 qb[K * 8];
    __shared__ double red[K > 1 ? K * 3 * kBlock : 1];
    __shared__ float4 tab[(VAR & 8) ? kTabN : 1];
    __shared__ int mark[K * kBlock];
    __shared__ unsigned next_item;
    if (ia.sizes[kSkip]) return;
    if (VAR & 8) {
        for (int k = threadIdx.x; k < kTabN; k += 64 * K) tab[k] = ia.split_tab[k];
        __syncthreads();
    }
    const int64_t nitem = ia.sizes[kNItem];
    const int64_t per = (nitem + 7) / 8;
    const int my = blockIdx.x & 7;
    // the kernel counters, summed over this wave's items and added once
    unsigned long long n_eval = 0, n_lane = 0;
    for (int v = 0; v < 8; ++v) {
        const int q = (my + v) & 7;
        const int64_t qbeg = q * per;
        const int64_t qend = qbeg + per < nitem ? qbeg + per : nitem;
        if (qbeg >= qend) continue;
        const unsigned qlen = (unsigned)(qend - qbeg);
        for (;;) {
            unsigned i = 0;
            if (K == 1) {
                if (threadIdx.x == 0) i = atomicAdd(&queues[q * kQueueStride], 1u);
                i = (unsigned)__builtin_amdgcn_readfirstlane((int)i);
            } else {
                // one pop per workgroup, shared through LDS
                __syncthreads();
                if (threadIdx.x == 0) next_item = atomicAdd(&queues[q * kQueueStride], 1u);
                __syncthreads();
                i = next_item;
            }
            if (i >= qlen) break;
            pp_item<VAR, K>(ia, qbeg + (int64_t)i, pos_s, mass_s, N, partial, n_eval, n_lane, tile, tab, qb,
                            red, mark);
        }
    }
    if (counters && (threadIdx.x & (kBlock - 1)) == 0 && n_lane) {
        atomicAdd(counters, n_eval);
        atomicAdd(counters + 1, n_lane);
    }
}

// Clears the work queues and (when given) the three kernel counters.
__global__ void reset_queues_kernel(unsigned* q, unsigned long long* ctr) {
    if (q && threadIdx.x < 8) q[threadIdx.x * kQueueStride] = 0u;
    if (ctr && threadIdx.x < 3) ctr[threadIdx.x] = 0ull;
}

// One thread per (block, lane), grid-stride: sum the item partials of the
// block in order (FP64), scale by G / ell^2, scatter to input order.
__global__ void __launch_bounds__(256) reduce_f32_kernel(ItemArgs ia,
                                                         const float* __restrict__ partial,
                                                         const int32_t* __restrict__ perm,
                                                         int64_t N, float* __restrict__ acc) {
    if (ia.sizes[kSkip]) return;
    const int64_t nblock = ia.sizes[kNBlock];
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < nblock * kBlock;
         g += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = g / kBlock;
        const int l = (int)(g % kBlock);
        if (l >= ia.bcount[b]) continue;
        if (ia.ioff[b + 1] - ia.ioff[b] <= 1) continue;     // written by the PP kernel, or skipped
        double sx = 0, sy = 0, sz = 0;
        const int64_t end = ia.ioff[b + 1];
        int64_t it = ia.ioff[b];
        // four items' loads in flight at once; the sums keep item order
        for (; it + 4 <= end; it += 4) {
            float v[4][3];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const float* o = partial + (it + u) * 3 * kBlock;
                v[u][0] = o[0 * kBlock + l];
                v[u][1] = o[1 * kBlock + l];
                v[u][2] = o[2 * kBlock + l];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                sx += (double)v[u][0];
                sy += (double)v[u][1];
                sz += (double)v[u][2];
            }
        }
        for (; it < end; ++it) {
            const float* o = partial + it * 3 * kBlock;
            sx += (double)o[0 * kBlock + l];
            sy += (double)o[1 * kBlock + l];
            sz += (double)o[2 * kBlock + l];
        }
        const double scale = ia.box[ia.bboxid[b]].scale;
        const int64_t i = perm[(int64_t)ia.bstart[b] + l];
        if (!target_on(ia, i)) continue;
        acc[i] = (float)(sx * scale);
        acc[N + i] = (float)(sy * scale);
        acc[2 * N + i] = (float)(sz * scale);
    }
}

// ------------------------------------------------------------------ FP64 --
#pragma clang fp contract(off)
// The split factor (Eq. equ:split) in FP64 with the device erfc/exp.
__device__ __forceinline__ double split_factor_f64(double x) {
    return erfc(x) + 2.0 * x / 1.7724538509055160272981674833411 * exp(-x * x);
}

template <bool COUNT>
__global__ void __launch_bounds__(64) pp_f64_kernel(ItemArgs ia, const double* __restrict__ pos_s,
                                                    const double* __restrict__ mass_s, int64_t N,
                                                    double* __restrict__ partial,
                                                    int32_t* __restrict__ pcount) {
    if (ia.sizes[kSkip]) return;
    const int64_t nitem = ia.sizes[kNItem];
    const int64_t item = xcd_item(blockIdx.x, nitem);
    if (item < 0) return;
    const int lane = threadIdx.x;
    const int32_t b = ia.iblock[item];
    const int32_t s0 = ia.is0[item];
    const int32_t S = ia.slen[b];
    const int32_t chunk = (int32_t)ia.sizes[kChunk];
    const int32_t s1 = s0 + chunk < S ? s0 + chunk : S;
    const BoxDev& X = ia.box[ia.bboxid[b]];
    const double L = X.L, rs = X.rs, rcut = X.rcut, eps = X.eps, G = X.G;
    const bool active = lane < ia.bcount[b];
    const int64_t t = active ? (int64_t)ia.bstart[b] + lane : -2;
    double xi = 0, yi = 0, zi = 0;
    if (active) {
        xi = pos_s[t];
        yi = pos_s[N + t];
        zi = pos_s[2 * N + t];
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
            v.y = pos_s[N + j];
            v.z = pos_s[2 * N + j];
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

__global__ void __launch_bounds__(256) reduce_f64_kernel(ItemArgs ia,
                                                         const double* __restrict__ partial,
                                                         const int32_t* __restrict__ perm,
                                                         int64_t N, double* __restrict__ acc) {
    if (ia.sizes[kSkip]) return;
    const int64_t nblock = ia.sizes[kNBlock];
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t b = g / kBlock;
    const int l = (int)(g % kBlock);
    if (b >= nblock || l >= ia.bcount[b]) return;
    double sx = 0, sy = 0, sz = 0;
    for (int64_t it = ia.ioff[b]; it < ia.ioff[b + 1]; ++it) {
        const double* o = partial + it * 3 * kBlock;
        sx += o[0 * kBlock + l];
        sy += o[1 * kBlock + l];
        sz += o[2 * kBlock + l];
    }
    const int64_t i = perm[(int64_t)ia.bstart[b] + l];
    acc[i] = sx;
    acc[N + i] = sy;
    acc[2 * N + i] = sz;
}

__global__ void __launch_bounds__(256) reduce_count_kernel(ItemArgs ia,
                                                           const int32_t* __restrict__ pc,
                                                           const int32_t* __restrict__ perm,
                                                           int64_t* __restrict__ counts,
                                                           unsigned long long* __restrict__ total) {
    if (ia.sizes[kSkip]) return;
    const int64_t nblock = ia.sizes[kNBlock];
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t b = g / kBlock;
    const int l = (int)(g % kBlock);
    if (b >= nblock || l >= ia.bcount[b]) return;
    int64_t s = 0;
    for (int64_t it = ia.ioff[b]; it < ia.ioff[b + 1]; ++it) s += pc[it * kBlock + l];
    if (counts) counts[perm[(int64_t)ia.bstart[b] + l]] = s;
    atomicAdd(total, (unsigned long long)s);
}

}  // namespace

double pair_length_unit(const pp_box_params& p) {
    return 2.0 * p.rs * std::sqrt(0.5 * SPLIT_POLY_U_MAX);
}

int make_poly(const pp_box_params& p, PolyF32* out) {
    const double ell = pair_length_unit(p);
    double e2 = (p.eps / ell) * (p.eps / ell);
    const double floor2 = ldexp(1.0, -60);          // keeps y^3 finite for s = eps = 0
    if (e2 < floor2) e2 = floor2;
    const double c2 = (p.rcut / ell) * (p.rcut / ell);
    out->eps2n = (float)e2;
    out->cut2 = (float)(c2 + e2);
    out->keep2 = (float)c2 * 1.0002f;
    out->pad = 0.f;
    return PP_OK;
}

// H(u) = (1 - g(x)) / x^3, u = x^2, from g'(x) = -(4/sqrt(pi)) x^2 e^{-x^2}:
// 1 - g(x) = (4/sqrt(pi)) sum_n (-1)^n x^{2n+3} / (n! (2n+3)), so
// H(u) = (4/sqrt(pi)) sum_n (-u)^n / (n! (2n+3)).  In FP64 the alternating
// terms stay below 40 for u <= 5.2, so the sum keeps about 14 digits.
__device__ double split_H_series(double u) {
    double term = 1.0, sum = 1.0 / 3.0;
    for (int n = 1; n < 80; ++n) {
        term *= -u / (double)n;
        sum += term / (double)(2 * n + 3);
        if (fabs(term) < 1e-18) break;
    }
    return 4.0 / 1.7724538509055160272981674833411 * sum;
}

// Piece k of the table covers r2 in [2k/N, 2(k+1)/N); the quadratic through
// the piece's two ends and midpoint, in z = position inside the piece.
__global__ void split_table_kernel(float4* __restrict__ tab) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= kTabN) return;
    const double hu = 0.5 * SPLIT_POLY_U_MAX;           // u per unit of r2
    const double w = 2.0 / kTabN;
    const double f0 = kHScale * split_H_series(hu * (k * w));
    const double fm = kHScale * split_H_series(hu * ((k + 0.5) * w));
    const double f1 = kHScale * split_H_series(hu * ((k + 1) * w));
    tab[k] = make_float4((float)f0, (float)(-3.0 * f0 + 4.0 * fm - f1), (float)(2.0 * f0 - 4.0 * fm + 2.0 * f1),
                         0.f);
}

int launch_split_table(Work& w, hipStream_t s) {
    PP_TRY(w.split_tab.reserve(sizeof(float4) * kTabN));
    hipLaunchKernelGGL(split_table_kernel, dim3(1), dim3(kTabN), 0, s, w.split_tab.as<float4>());
    PP_HIP(hipGetLastError());
    return PP_OK;
}

int launch_reset_queues(unsigned* queues, hipStream_t s, unsigned long long* counters) {
    hipLaunchKernelGGL(reset_queues_kernel, dim3(1), dim3(64), 0, s, queues, counters);
    PP_HIP(hipGetLastError());
    return PP_OK;
}

template <int VAR, int K>
static int launch_pp_f32_var(const ItemArgs& ia, const Work& w, Mode mode, int waves_per_cu,
                             float* partial, unsigned long long* counters, unsigned* queues,
                             hipStream_t s) {
    if (mode == Mode::kPersistent) {
        int dev = 0, cus = 256;
        PP_HIP(hipGetDevice(&dev));
        PP_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        // waves_per_cu waves per CU in workgroups of K waves
        const int wpc = waves_per_cu > 0 ? waves_per_cu : 16;
        const unsigned grid = (unsigned)(cus * ((wpc + K - 1) / K));
        hipLaunchKernelGGL((pp_f32_persistent<VAR, K>), dim3(grid), dim3(kBlock * K), 0, s, ia,
                           w.pos_s.as<double>(), w.mass_s.as<float>(), w.pos_n, partial, counters,
                           queues);
    } else {
        // one workgroup per item, up to the item capacity (the count is on
        // the device; the workgroups past it return at once)
        const int64_t per = (w.cap_item + 7) / 8;
        if (per == 0) return PP_OK;
        // At most two waves per SIMD by the last call's item count (a hint
        // only: both forms give the same results), the form built for that.
        bool few = false;
        if constexpr (VAR == 0 || VAR == 8) {
            int dev = 0, cus = 256;
            PP_HIP(hipGetDevice(&dev));
            PP_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
            few = w.nitem > 0 && w.nitem * K <= 2 * 4 * (int64_t)cus;
            if (few)
                hipLaunchKernelGGL((pp_f32_kernel_few<VAR, K>), dim3((unsigned)(per * 8)), dim3(kBlock * K), 0,
                                   s, ia, w.pos_s.as<double>(), w.mass_s.as<float>(), w.pos_n, partial, counters);
        }
        if (!few)
            hipLaunchKernelGGL((pp_f32_kernel<VAR, K>), dim3((unsigned)(per * 8)), dim3(kBlock * K), 0, s,
                               ia, w.pos_s.as<double>(), w.mass_s.as<float>(), w.pos_n, partial, counters);
    }
    PP_HIP(hipGetLastError());
    return PP_OK;
}

template <int K>
static int launch_pp_f32_k(const ItemArgs& ia, const Work& w, Mode mode, int waves_per_cu,
                           int variant, float* partial, unsigned long long* counters,
                           unsigned* queues, hipStream_t s) {
    switch (variant) {
        case 0: return launch_pp_f32_var<0, K>(ia, w, mode, waves_per_cu, partial, counters, queues, s);
        case 8: return launch_pp_f32_var<8, K>(ia, w, mode, waves_per_cu, partial, counters, queues, s);
        default: return fail(PP_EINVAL, "more than one wave per block needs variant 0 or 8");
    }
}

int launch_pp_f32(const BatchDev& bd, const Work& w, int waves_per_block, Mode mode, int waves_per_cu,
                  int variant, float* partial, float* acc, unsigned long long* counters,
                  unsigned* queues, hipStream_t s) {
    ItemArgs ia = item_args(bd, w);
    ia.acc = acc;
    if (waves_per_block == 2)
        return launch_pp_f32_k<2>(ia, w, mode, waves_per_cu, variant & 15, partial, counters, queues, s);
    if (waves_per_block == 4)
        return launch_pp_f32_k<4>(ia, w, mode, waves_per_cu, variant & 15, partial, counters, queues, s);
    if (waves_per_block == 8)
        return launch_pp_f32_k<8>(ia, w, mode, waves_per_cu, variant & 15, partial, counters, queues, s);
    switch (variant & 15) {
        case 0: return launch_pp_f32_var<0, 1>(ia, w, mode, waves_per_cu, partial, counters, queues, s);
        case 1: return launch_pp_f32_var<1, 1>(ia, w, mode, waves_per_cu, partial, counters, queues, s);
        case 2: return launch_pp_f32_var<2, 1>(ia, w, mode, waves_per_cu, partial, counters, queues, s);
        case 3: return launch_pp_f32_var<3, 1>(ia, w, mode, waves_per_cu, partial, counters, queues, s);
        case 4: return launch_pp_f32_var<4, 1>(ia, w, mode, waves_per_cu, partial, counters, queues, s);
        case 5: return launch_pp_f32_var<5, 1>(ia, w, mode, waves_per_cu, partial, counters, queues, s);
        case 6: return launch_pp_f32_var<6, 1>(ia, w, mode, waves_per_cu, partial, counters, queues, s);
        case 7: return launch_pp_f32_var<7, 1>(ia, w, mode, waves_per_cu, partial, counters, queues, s);
        case 8: return launch_pp_f32_var<8, 1>(ia, w, mode, waves_per_cu, partial, counters, queues, s);
        case 9: return launch_pp_f32_var<9, 1>(ia, w, mode, waves_per_cu, partial, counters, queues, s);
        case 10: return launch_pp_f32_var<10, 1>(ia, w, mode, waves_per_cu, partial, counters, queues, s);
        case 11: return launch_pp_f32_var<11, 1>(ia, w, mode, waves_per_cu, partial, counters, queues, s);
        case 12: return launch_pp_f32_var<12, 1>(ia, w, mode, waves_per_cu, partial, counters, queues, s);
        case 13: return launch_pp_f32_var<13, 1>(ia, w, mode, waves_per_cu, partial, counters, queues, s);
        case 14: return launch_pp_f32_var<14, 1>(ia, w, mode, waves_per_cu, partial, counters, queues, s);
        default: return launch_pp_f32_var<15, 1>(ia, w, mode, waves_per_cu, partial, counters, queues, s);
    }
}

int launch_monopole(const BatchDev& bd, const Work& w, float* acc, unsigned long long* counter,
                    hipStream_t s) {
    if (w.cap_block == 0 || !w.ent_final) return PP_OK;
    ItemArgs ia = item_args(bd, w);
    ia.acc = acc;
    hipLaunchKernelGGL(monopole_kernel, dim3((unsigned)w.cap_block), dim3(kBlock), 0, s, ia, w.ent_final,
                       w.eoff.as<int64_t>(), w.mono0, w.mono1, w.tviews.as<TreeView>(),
                       w.tree_mc.as<double4>(), w.pos_s.as<double>(), w.pos_n, w.cap_block, counter);
    PP_HIP(hipGetLastError());
    return PP_OK;
}

int launch_reduce_f32(const BatchDev& bd, const Work& w, const float* partial, float* acc,
                      hipStream_t s) {
    ItemArgs ia = item_args(bd, w);
    // a fixed grid (grid-stride) so a captured graph stays valid as nblock changes
    hipLaunchKernelGGL(reduce_f32_kernel, dim3(2048), dim3(256), 0, s, ia, partial,
                       w.perm.as<int32_t>(), w.pos_n, acc);
    PP_HIP(hipGetLastError());
    return PP_OK;
}

int launch_pp_f64(const BatchDev& bd, const Work& w, double* partial, hipStream_t s) {
    const int64_t per = (w.cap_item + 7) / 8;
    if (per == 0) return PP_OK;
    ItemArgs ia = item_args(bd, w);
    hipLaunchKernelGGL(pp_f64_kernel<false>, dim3((unsigned)(per * 8)), dim3(kBlock), 0, s, ia,
                       w.pos_s.as<double>(), w.mass_sd.as<double>(), w.pos_n, partial,
                       (int32_t*)nullptr);
    PP_HIP(hipGetLastError());
    return PP_OK;
}

int launch_reduce_f64(const BatchDev& bd, const Work& w, const double* partial, double* acc,
                      hipStream_t s) {
    if (w.cap_block == 0) return PP_OK;
    ItemArgs ia = item_args(bd, w);
    hipLaunchKernelGGL(reduce_f64_kernel, dim3(blocks_for(w.cap_block * kBlock, 256)), dim3(256), 0, s,
                       ia, partial, w.perm.as<int32_t>(), w.pos_n, acc);
    PP_HIP(hipGetLastError());
    return PP_OK;
}

int launch_count(const BatchDev& bd, const Work& w, int32_t* partial, hipStream_t s) {
    const int64_t per = (w.cap_item + 7) / 8;
    if (per == 0) return PP_OK;
    ItemArgs ia = item_args(bd, w);
    hipLaunchKernelGGL(pp_f64_kernel<true>, dim3((unsigned)(per * 8)), dim3(kBlock), 0, s, ia,
                       w.pos_s.as<double>(), (const double*)nullptr, w.pos_n,
                       (double*)nullptr, partial);
    PP_HIP(hipGetLastError());
    return PP_OK;
}

int launch_reduce_count(const BatchDev& bd, const Work& w, const int32_t* partial, int64_t* counts,
                        unsigned long long* total, hipStream_t s) {
    if (w.cap_block == 0) return PP_OK;
    ItemArgs ia = item_args(bd, w);
    hipLaunchKernelGGL(reduce_count_kernel, dim3(blocks_for(w.cap_block * kBlock, 256)), dim3(256), 0,
                       s, ia, partial, w.perm.as<int32_t>(), counts, total);
    PP_HIP(hipGetLastError());
    return PP_OK;
}

}  // namespace pp
