// Octree leaves, the implicit trees over them, and the near-leaf lists, for
// a batch of boxes.
//
// Leaves (sec. 3.2-3.3): with particles in Peano-Hilbert key order every
// octree node (the particles sharing the top 3l key bits) is a contiguous
// run.  A leaf is a maximal node holding at most M = leaf_max particles
// ("a leaf is a package of a given number of particles", sec. 3.3).  The
// level of the leaf of particle k is found without building the tree: the
// level-l node of k holds more than M particles iff some run of M + 1
// consecutive particles (of the same box) containing k shares its top 3l
// key bits, so
//   level(k) = 1 + max over s in [k - M, k] of lcp(key[s], key[s + M])
// (lcp in 3-bit digits, capped at b; 0 when no such run exists).  The
// sliding maximum uses the van Herk / Gil-Werman block prefix/suffix maxima.
//
// Near lists (sec. 3.3, the N-to-M leaf pairs of the dual tree traversal,
// restricted to the short range): an implicit 8-ary tree over each box's
// leaf array (leaves are in key order, so consecutive leaves are close in
// space) is walked, pruning subtrees whose integer bounding box is at least
// r_cut away.  The leaf test is exact integer arithmetic, identical for the
// canonical list and for the block lists.
#include "pp_internal.h"

namespace pp {
namespace {

#pragma clang fp contract(off)
// Grid cell of one coordinate of an already wrapped position w (the gather
// stores x - L floor(x / L)): floor(w 2^b / L) clamped, exactly the
// quantisation the key kernel applies to the same wrapped value.
__device__ __forceinline__ uint32_t quantise_w(double w, double L, double scale, uint32_t qmax) {
    (void)L;
    double f = floor(w * scale);
    if (!(f > 0.0)) return 0u;
    if (f > (double)qmax) return qmax;
    return (uint32_t)f;
}
#pragma clang fp contract(on)

__device__ __forceinline__ int common_digits(uint64_t a, uint64_t b, int bits) {
    uint64_t x = a ^ b;
    if (x == 0) return bits;
    int lz = __clzll((long long)x);
    return (lz - (64 - 3 * bits)) / 3;
}

__device__ __forceinline__ uint64_t key_prefix(uint64_t key, int level, int bits) {
    return level == 0 ? 0ull : key >> (3 * (bits - level));
}

// lamp[s + M] = lcp(key[s], key[s + M]) for s, s + M in one box, else -1.
__global__ void lam_kernel(BatchDev bd, const uint64_t* __restrict__ keys, int64_t N,
                           int8_t* __restrict__ lamp) {
    const int M = bd.leaf_max;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N + M) return;
    const int64_t s = t - M;
    int8_t v = -1;
    if (s >= 0 && s + M < N &&
        (bd.nbox == 1 || box_of(bd.poff, bd.nbox, s) == box_of(bd.poff, bd.nbox, s + M)))
        v = (int8_t)common_digits(keys[s], keys[s + M], bd.bits);
    lamp[t] = v;
}

// Block prefix and suffix maxima over blocks of W = M + 1 entries.
__global__ void vhgw_kernel(const int8_t* __restrict__ a, int64_t len, int W,
                            int8_t* __restrict__ pmax, int8_t* __restrict__ smax) {
    const int64_t blk = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t b0 = blk * W;
    if (b0 >= len) return;
    const int64_t b1 = b0 + W < len ? b0 + W : len;
    int8_t m = -1;
    for (int64_t i = b0; i < b1; ++i) {
        m = a[i] > m ? a[i] : m;
        pmax[i] = m;
    }
    m = -1;
    for (int64_t i = b1 - 1; i >= b0; --i) {
        m = a[i] > m ? a[i] : m;
        smax[i] = m;
    }
}

__global__ void level_kernel(const int8_t* __restrict__ pmax, const int8_t* __restrict__ smax,
                             int64_t N, int M, int bits, int8_t* __restrict__ lev) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N) return;
    // window of lamp indices [k, k + M]
    const int8_t a = smax[k], b = pmax[k + M];
    const int m = a > b ? a : b;
    lev[k] = (int8_t)(m < 0 ? 0 : (m + 1 < bits ? m + 1 : bits));
}

__global__ void flag_kernel(BatchDev bd, const uint64_t* __restrict__ keys,
                            const int8_t* __restrict__ lev, int64_t N, int32_t* __restrict__ flag) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N) return;
    int f = 1;
    if (k > 0 && (bd.nbox == 1 || box_of(bd.poff, bd.nbox, k) == box_of(bd.poff, bd.nbox, k - 1))) {
        const int l = lev[k - 1];
        f = key_prefix(keys[k], l, bd.bits) != key_prefix(keys[k - 1], l, bd.bits);
    }
    flag[k] = f;
}

__global__ void leaf_fill_kernel(const uint64_t* __restrict__ keys, const int8_t* __restrict__ lev,
                                 const int32_t* __restrict__ flag, const int64_t* __restrict__ off,
                                 int64_t N, int bits, int64_t* __restrict__ begin,
                                 int32_t* __restrict__ level, uint64_t* __restrict__ prefix) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N || !flag[k]) return;
    const int64_t a = off[k];
    begin[a] = k;
    level[a] = lev[k];
    prefix[a] = key_prefix(keys[k], lev[k], bits);
}

__global__ void leaf_box_kernel(BatchDev bd, const double* __restrict__ pos_s, int64_t N,
                                const int64_t* __restrict__ begin, const int64_t* __restrict__ sizes,
                                int32_t* __restrict__ count, IBox* __restrict__ box) {
    const int64_t m = sizes[kNLeaf];
    for (int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; a < m;
         a += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b0 = begin[a], b1 = a + 1 < m ? begin[a + 1] : N;
    count[a] = (int32_t)(b1 - b0);
    const BoxDev& X = bd.box[box_of(bd.poff, bd.nbox, b0)];
    const uint32_t qmax = (uint32_t)(X.W - 1);
    IBox B;
    for (int ax = 0; ax < 3; ++ax) {
        uint32_t lo = 0xffffffffu, hi = 0;
        for (int64_t k = b0; k < b1; ++k) {
            const uint32_t q = quantise_w(pos_s[ax * N + k], X.L, X.qscale, qmax);
            lo = q < lo ? q : lo;
            hi = q > hi ? q : hi;
        }
        B.lo[ax] = (int32_t)lo;
        B.hi[ax] = (int32_t)hi + 1;
    }
    box[a] = B;
    }
}

// First leaf of every box: the first leaf starting at or after poff[x].
// First leaf of every box (and the leaf total at x = nbox): every box start
// starts a leaf, so the leaves before box x are the leaf starts before its
// first particle, the exclusive flag scan at that index.
__global__ void leaf_offsets_kernel(BatchDev bd, const int64_t* __restrict__ flag_off,
                                    int64_t* __restrict__ loff, int64_t* __restrict__ sizes) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x > bd.nbox) return;
    loff[x] = flag_off[bd.poff[x]];
    if (x == bd.nbox) sizes[kNLeaf] = loff[x];
}

// Tree shape of every box from its leaf count (one workgroup): level h of
// box x has cnt_h = ceil(cnt_{h-1} / 8) nodes while cnt_{h-1} > 1.  Level h
// of all boxes is contiguous, boxes in order: lp[h (nbox + 1) + x] is the
// number of level-h nodes of the boxes before x, and the levels follow one
// another; total[0] receives the node count.
__device__ __forceinline__ int64_t level_count(int64_t c0, int h) {
    int64_t c = c0;
    for (int k = 0; k < h; ++k) {
        if (c <= 1) return 0;
        c = (c + 7) / 8;
    }
    return c;
}

__global__ void __launch_bounds__(256) tree_views_kernel(const int64_t* __restrict__ loff, int nbox,
                                                         TreeView* __restrict__ tv,
                                                         int64_t* __restrict__ lp,
                                                         int64_t* __restrict__ total) {
    __shared__ int64_t wsum[4];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int per = (nbox + 255) / 256;
    const int x0 = t * per < nbox ? t * per : nbox;
    const int x1 = x0 + per < nbox ? x0 + per : nbox;
    int64_t base = 0;                     // first node of level h (same in every thread)
    int h = 0;
    for (; h < kTreeMaxLevels; ++h) {
        int64_t sum = 0;
        for (int x = x0; x < x1; ++x) sum += level_count(loff[x + 1] - loff[x], h);
        // inclusive scan of the 256 thread sums: inside each wave, then the
        // four wave totals
        int64_t inc = sum;
        for (int d = 1; d < 64; d <<= 1) {
            const int64_t u = __shfl_up(inc, d);
            if (lane >= d) inc += u;
        }
        if (lane == 63) wsum[wave] = inc;
        __syncthreads();
        int64_t before = 0, level_total = 0;
        for (int k = 0; k < 4; ++k) {
            if (k < wave) before += wsum[k];
            level_total += wsum[k];
        }
        __syncthreads();                  // wsum is rewritten at the next level
        int64_t acc = before + inc - sum;  // nodes of this level before box x0
        for (int x = x0; x < x1; ++x) {
            const int64_t c0 = loff[x + 1] - loff[x];
            const int64_t c = level_count(c0, h);
            lp[(int64_t)h * (nbox + 1) + x] = acc;
            TreeView& T = tv[x];
            if (h == 0) {
                int nl = 0;
                while (nl < kTreeMaxLevels && level_count(c0, nl) > 0) ++nl;
                T.nlev = c0 > 0 ? nl : 0;
                T.loff = loff[x];
                T.pad = 0;
            }
            T.cnt[h] = c;
            T.off[h] = c > 0 ? base + acc : 0;
            acc += c;
        }
        if (t == 0) lp[(int64_t)h * (nbox + 1) + nbox] = level_total;
        base += level_total;
        if (level_total == 0) break;      // no box has nodes here or above
    }
    // the levels above the last populated one: empty
    for (++h; h < kTreeMaxLevels; ++h) {
        for (int x = x0; x < x1; ++x) {
            lp[(int64_t)h * (nbox + 1) + x] = 0;
            tv[x].cnt[h] = 0;
            tv[x].off[h] = 0;
        }
        if (t == 0) lp[(int64_t)h * (nbox + 1) + nbox] = 0;
    }
    if (t == 0) total[0] = base;
}

// Level h >= 1 of every box's tree: node i of box x is the union of its
// (up to 8) children.  lp = per-box prefix of the level's node counts.
__global__ void tree_level_kernel(const TreeView* __restrict__ tv, const int64_t* __restrict__ lp,
                                  int nbox, int h, IBox* __restrict__ nodes) {
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < lp[nbox];
         g += (int64_t)gridDim.x * blockDim.x) {
    const int x = box_of(lp, nbox, g);
    const TreeView& T = tv[x];
    const int64_t i = g - lp[x];
    const int64_t nchild = T.cnt[h - 1];
    const IBox* child = nodes + T.off[h - 1];
    IBox P = child[8 * i];
    const int64_t e = 8 * i + 8 < nchild ? 8 * i + 8 : nchild;
    for (int64_t c = 8 * i + 1; c < e; ++c) {
        const IBox C = child[c];
        for (int ax = 0; ax < 3; ++ax) {
            P.lo[ax] = C.lo[ax] < P.lo[ax] ? C.lo[ax] : P.lo[ax];
            P.hi[ax] = C.hi[ax] > P.hi[ax] ? C.hi[ax] : P.hi[ax];
        }
    }
    nodes[T.off[h] + i] = P;
    }
}

// Mass and mass-weighted position sums of every tree node (x, y, z: sum of
// m x; w: sum of m), FP64, for monopole acceptance.  Level 0 from the
// particles of each leaf, in order; level h from its (up to 8) children.
__global__ void leaf_moment_kernel(const double* __restrict__ pos_s, const float* __restrict__ mass_s,
                                   int64_t N, const int64_t* __restrict__ begin,
                                   const int64_t* __restrict__ sizes, double4* __restrict__ mc) {
    const int64_t m = sizes[kNLeaf];
    for (int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; a < m;
         a += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b0 = begin[a], b1 = a + 1 < m ? begin[a + 1] : N;
    double sx = 0, sy = 0, sz = 0, sm = 0;
    for (int64_t k = b0; k < b1; ++k) {
        const double mk = (double)mass_s[k];
        sx += mk * pos_s[k];
        sy += mk * pos_s[N + k];
        sz += mk * pos_s[2 * N + k];
        sm += mk;
    }
    mc[a] = make_double4(sx, sy, sz, sm);
    }
}

__global__ void tree_moment_kernel(const TreeView* __restrict__ tv, const int64_t* __restrict__ lp,
                                   int nbox, int h, double4* __restrict__ mc) {
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < lp[nbox];
         g += (int64_t)gridDim.x * blockDim.x) {
    const int x = box_of(lp, nbox, g);
    const TreeView& T = tv[x];
    const int64_t i = g - lp[x];
    const int64_t nchild = T.cnt[h - 1];
    const double4* child = mc + T.off[h - 1];
    double4 P = child[8 * i];
    const int64_t e = 8 * i + 8 < nchild ? 8 * i + 8 : nchild;
    for (int64_t c = 8 * i + 1; c < e; ++c) {
        const double4 C = child[c];
        P.x += C.x;
        P.y += C.y;
        P.z += C.z;
        P.w += C.w;
    }
    mc[T.off[h] + i] = P;
    }
}

// ------------------------------------------------------------ box tests --
// Gap along one axis between target [loA, hiA) and source [loB, hiB)
// shifted by s * W (grid units).
__device__ __forceinline__ int64_t axis_gap(int64_t loA, int64_t hiA, int64_t loB, int64_t hiB,
                                            int s, int64_t W) {
    const int64_t sh = (int64_t)s * W;
    const int64_t g1 = loB + sh - hiA, g2 = loA - hiB - sh;
    const int64_t g = g1 > g2 ? g1 : g2;
    return g > 0 ? g : 0;
}

__device__ __forceinline__ int64_t gap2_shift(const IBox& A, const IBox& B, const int s[3],
                                              int64_t W) {
    int64_t r = 0;
    for (int ax = 0; ax < 3; ++ax) {
        const int64_t g = axis_gap(A.lo[ax], A.hi[ax], B.lo[ax], B.hi[ax], s[ax], W);
        r += g * g;
    }
    return r;
}

// Largest squared separation of the two boxes (every pair of points is
// closer): when it is below T every leaf under B passes the gap test.
__device__ __forceinline__ int64_t maxd2_shift(const IBox& A, const IBox& B, const int s[3],
                                               int64_t W) {
    int64_t r = 0;
    for (int ax = 0; ax < 3; ++ax) {
        const int64_t sh = (int64_t)s[ax] * W;
        const int64_t d1 = (int64_t)B.hi[ax] + sh - A.lo[ax];
        const int64_t d2 = (int64_t)A.hi[ax] - B.lo[ax] - sh;
        const int64_t d = d1 > d2 ? d1 : d2;
        r += d * d;
    }
    return r;
}

// Allowed shifts per axis: bit 0 -> -1, bit 1 -> 0, bit 2 -> +1.
__device__ __forceinline__ void allowed_shifts(const IBox& A, int64_t W, int64_t T, int mask[3]) {
    for (int ax = 0; ax < 3; ++ax) {
        const int64_t lo = A.lo[ax], up = W - A.hi[ax];
        mask[ax] = 2 | (lo * lo < T ? 1 : 0) | (up * up < T ? 4 : 0);
    }
}

__device__ __forceinline__ bool shift_allowed(const int mask[3], const int s[3]) {
    return (mask[0] >> (s[0] + 1) & 1) && (mask[1] >> (s[1] + 1) & 1) && (mask[2] >> (s[2] + 1) & 1);
}

__device__ __forceinline__ void decode_shift(int sc, int s[3]) {
    s[0] = sc / 9 - 1;
    s[1] = (sc / 3) % 3 - 1;
    s[2] = sc % 3 - 1;
}

// Minimum over the allowed shifts of the squared gap (a lower bound for
// every shift), used to prune subtrees when all shifts are walked at once.
__device__ __forceinline__ int64_t gap2_min(const IBox& A, const IBox& B, const int mask[3],
                                            int64_t W) {
    int64_t r = 0;
    for (int ax = 0; ax < 3; ++ax) {
        int64_t best = INT64_MAX;
        for (int s = -1; s <= 1; ++s) {
            if (!(mask[ax] >> (s + 1) & 1)) continue;
            const int64_t g = axis_gap(A.lo[ax], A.hi[ax], B.lo[ax], B.hi[ax], s, W);
            best = g < best ? g : best;
        }
        r += best * best;
    }
    return r;
}

// Monopole acceptance of the node of box B (global index g) for target box
// A (block b) under shift s (sec. 3.3), every enabled test required:
//  * geometric: (A + B) / R <= theta with A, B the longest box sides and R
//    the distance of the box centres, tested as (2 (A + B))^2 <= theta^2
//    (2R)^2 from integer half-cell coordinates (for theta < 1 this gives
//    B / (R - A) <= theta too);
//  * relative (Gadget-2, sec. 3.1): G M B^2 / r^4 <= alpha |a| with M the
//    node mass, r the gap between the boxes and |a| the smallest reference
//    acceleration of the block's targets, squared on both sides so that no
//    root is taken.
// Each side is a fixed sequence of FP64 operations on exact integers, the
// node mass and the block's |a|^2, so the oracle can repeat the decision.
struct MonoDev {
    double theta2, alpha;
    const double4* mc;
    const double* amin2;
};

__device__ __forceinline__ bool accept_monopole(const IBox& A, const IBox& B, const int s[3], int64_t W,
                                                const MonoDev& M, int64_t g, int64_t b, double G,
                                                double cell) {
#pragma clang fp contract(off)
    int64_t a = 0, bm = 0, r2 = 0;
    for (int ax = 0; ax < 3; ++ax) {
        const int64_t sa = (int64_t)A.hi[ax] - A.lo[ax], sb = (int64_t)B.hi[ax] - B.lo[ax];
        a = sa > a ? sa : a;
        bm = sb > bm ? sb : bm;
        const int64_t d = ((int64_t)B.lo[ax] + B.hi[ax] + 2 * (int64_t)s[ax] * W) - ((int64_t)A.lo[ax] + A.hi[ax]);
        r2 += d * d;
    }
    if (M.theta2 > 0.0) {
        const double lhs = (double)(2 * (a + bm));
        if (!(lhs * lhs <= M.theta2 * (double)r2)) return false;
    }
    if (M.alpha > 0.0) {
        const int64_t gap2 = gap2_shift(A, B, s, W);
        const double bc = (double)bm * cell;
        const double lhs = ((G * M.mc[g].w) * bc) * bc;
        const double g2 = ((double)gap2 * cell) * cell;
        const double rhs2 = ((M.alpha * M.alpha) * M.amin2[b]) * ((g2 * g2) * (g2 * g2));
        if (!(lhs * lhs <= rhs2)) return false;
    }
    return true;
}

// Smallest |a_ref|^2 over each block's targets (a_ref in input order).
__global__ void block_amin_kernel(const int32_t* __restrict__ bstart, const int32_t* __restrict__ bcount,
                                  const int32_t* __restrict__ perm, const float* __restrict__ acc_ref,
                                  int64_t N, const int64_t* __restrict__ sizes, double* __restrict__ amin2) {
#pragma clang fp contract(off)
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= sizes[kNBlock]) return;
    double m = 0.0;
    for (int32_t k = 0; k < bcount[b]; ++k) {
        const int64_t i = perm[(int64_t)bstart[b] + k];
        const double x = (double)acc_ref[i], y = (double)acc_ref[N + i], z = (double)acc_ref[2 * N + i];
        const double v = ((x * x) + (y * y)) + (z * z);
        m = k == 0 || v < m ? v : m;
    }
    amin2[b] = m;
}

// ------------------------------------------------------- canonical list --
// Depth-first walk of one tree in ascending leaf order.  test(B) decides
// whether to descend into / visit node box B; visit(leaf) is called for
// every leaf that passes.
template <class Test, class Visit>
__device__ void walk(const TreeView& tv, const IBox* nodes, Test&& test, Visit&& visit) {
    int h = tv.nlev - 1;
    int64_t i = 0;
    for (;;) {
        const bool pass = test(nodes[tv.off[h] + i]);
        if (pass && h == 0) visit(i);
        if (pass && h > 0) {
            h -= 1;
            i *= 8;
            continue;
        }
        for (;;) {
            if (h == tv.nlev - 1) return;
            const int64_t nx = i + 1;
            if ((nx & 7) != 0 && nx < tv.cnt[h]) {
                i = nx;
                break;
            }
            i >>= 3;
            h += 1;
        }
    }
}

// One thread per target leaf, all shifts in one walk, entries emitted in
// ascending (source, code) order.
template <bool FILL>
__global__ void canon_kernel(TreeView tv, const IBox* __restrict__ nodes, int64_t nleaf, int64_t W,
                             int64_t T, int32_t* __restrict__ cnt, const int64_t* __restrict__ off,
                             int32_t* __restrict__ src, uint8_t* __restrict__ code) {
    const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= nleaf) return;
    const IBox A = nodes[tv.off[0] + a];
    int mask[3];
    allowed_shifts(A, W, T, mask);
    int64_t k = FILL ? off[a] : 0;
    int32_t c = 0;
    walk(
        tv, nodes, [&](const IBox& B) { return gap2_min(A, B, mask, W) < T; },
        [&](int64_t b) {
            const IBox B = nodes[tv.off[0] + b];
            for (int sc = 0; sc < 27; ++sc) {
                int s[3];
                decode_shift(sc, s);
                if (!shift_allowed(mask, s)) continue;
                if (gap2_shift(A, B, s, W) < T) {
                    if (FILL) {
                        src[k] = (int32_t)b;
                        code[k] = (uint8_t)sc;
                        ++k;
                    } else {
                        ++c;
                    }
                }
            }
        });
    if (!FILL) cnt[a] = c;
}

// -------------------------------------------------------- target blocks --
// One wave per chunk of kBlock consecutive particles of one box.  Every
// lane quantises its particle; if the chunk's bounding box is at most emax
// grid units wide along every axis (the common case) the chunk is one
// block.  Otherwise lane 0 walks the chunk and starts a new block whenever
// adding the next particle would make the box wider than emax.
__device__ __forceinline__ int32_t wave_min_i(int32_t v) {
    for (int off = 32; off > 0; off >>= 1) {
        const int32_t o = __shfl_xor(v, off);
        v = o < v ? o : v;
    }
    return v;
}
__device__ __forceinline__ int32_t wave_max_i(int32_t v) {
    for (int off = 32; off > 0; off >>= 1) {
        const int32_t o = __shfl_xor(v, off);
        v = o > v ? o : v;
    }
    return v;
}

template <bool FILL>
__global__ void __launch_bounds__(64) block_split_kernel(
    BatchDev bd, const double* __restrict__ pos_s, int64_t N, const int64_t* __restrict__ choff,
    int64_t nchunk, int32_t* __restrict__ ccount, const int64_t* __restrict__ coff,
    int32_t* __restrict__ bstart, int32_t* __restrict__ bcount, IBox* __restrict__ box,
    int32_t* __restrict__ bboxid, int64_t cap) {
    const int64_t c = blockIdx.x;
    if (c >= nchunk) return;
    const int lane = threadIdx.x;
    const int x = box_of(choff, bd.nbox, c);
    const BoxDev& X = bd.box[x];
    const uint32_t qmax = (uint32_t)(X.W - 1);
    const int64_t k0 = X.poff + (c - choff[x]) * kBlock;
    const int64_t kend = X.poff + X.n;
    const int64_t k1 = k0 + kBlock < kend ? k0 + kBlock : kend;
    const int64_t k = k0 + lane;
    const bool valid = k < k1;
    __shared__ int32_t qs[3][kBlock];
    int32_t lo[3], hi[3];
    for (int ax = 0; ax < 3; ++ax) {
        const int32_t q = valid ? (int32_t)quantise_w(pos_s[ax * N + k], X.L, X.qscale, qmax) : 0;
        qs[ax][lane] = q;
        lo[ax] = wave_min_i(valid ? q : INT32_MAX);
        hi[ax] = wave_max_i(valid ? q + 1 : INT32_MIN);
    }
    const bool fits = (int64_t)(hi[0] - lo[0]) <= X.emax && (int64_t)(hi[1] - lo[1]) <= X.emax &&
                      (int64_t)(hi[2] - lo[2]) <= X.emax;
    if (fits) {
        if (lane == 0) {
            if (FILL) {
                const int64_t o = coff[c];
                if (o >= cap) return;          // too many blocks: reported by the count
                bstart[o] = (int32_t)k0;
                bcount[o] = (int32_t)(k1 - k0);
                IBox B;
                for (int ax = 0; ax < 3; ++ax) {
                    B.lo[ax] = lo[ax];
                    B.hi[ax] = hi[ax];
                }
                box[o] = B;
                bboxid[o] = x;
            } else {
                ccount[c] = 1;
            }
        }
        return;
    }
    __syncthreads();
    if (lane != 0) return;
    int64_t o = FILL ? coff[c] : 0;
    int32_t nb = 0;
    int64_t start = k0;
    IBox B;
    auto emit = [&](int64_t e) {
        if (FILL && o + nb < cap) {
            bstart[o + nb] = (int32_t)start;
            bcount[o + nb] = (int32_t)(e - start);
            box[o + nb] = B;
            bboxid[o + nb] = x;
        }
        ++nb;
    };
    for (int64_t kk = k0; kk < k1; ++kk) {
        const int l = (int)(kk - k0);
        const int32_t q[3] = {qs[0][l], qs[1][l], qs[2][l]};
        if (kk == start) {
            for (int ax = 0; ax < 3; ++ax) {
                B.lo[ax] = q[ax];
                B.hi[ax] = q[ax] + 1;
            }
            continue;
        }
        IBox U = B;
        bool wide = false;
        for (int ax = 0; ax < 3; ++ax) {
            U.lo[ax] = q[ax] < U.lo[ax] ? q[ax] : U.lo[ax];
            U.hi[ax] = q[ax] + 1 > U.hi[ax] ? q[ax] + 1 : U.hi[ax];
            wide |= (int64_t)(U.hi[ax] - U.lo[ax]) > X.emax;
        }
        if (wide) {
            emit(kk);
            start = kk;
            for (int ax = 0; ax < 3; ++ax) {
                B.lo[ax] = q[ax];
                B.hi[ax] = q[ax] + 1;
            }
        } else {
            B = U;
        }
    }
    emit(k1);
    if (!FILL) ccount[c] = nb;
}

// ----------------------------------------------------------- block lists --
// A node passes for target box A under shift s when its box is closer than
// r_cut (gap^2 < T); it is *inside* when even its farthest point is
// (maxdist^2 < T), and then every leaf under it passes, so the node's whole
// leaf interval is listed without descending.  The walk is level-synchronous
// from each box's root down to level 2 over all (block, shift, node) entries
// at once (one thread per entry, children written in order so entries stay
// sorted by block, shift, node); then one thread per entry walks its
// subtree (at most 64 leaves) depth-first, testing the 8 children of a node
// at once.  While the entries stay within a memory budget the breadth-first
// part goes one level further (down to level 1), which leaves a single
// 8-child test per entry.  Leaves (or inside intervals) come in ascending order and
// consecutive ones merge into one range of source particles.
constexpr int kDfsLevel = 2;
// Monopoles may be taken at every level: by the breadth-first expansion for
// nodes of level 2 and up, by the depth-first walk for groups of 8 leaves
// (level 1) and single leaves (level 0).
constexpr int kMonoMinLevel = 0;


// Test the children of (h, i): pass bits and inside bits (inside implies pass).
__device__ __forceinline__ void expand2(const TreeView& tv, const IBox* nodes, int h, int64_t i,
                                        const IBox& A, const int s[3], int64_t W, int64_t T,
                                        uint32_t& pass, uint32_t& inside) {
    const int64_t c0 = 8 * i, nc = tv.cnt[h - 1];
    const IBox* base = nodes + tv.off[h - 1];
    pass = 0;
    inside = 0;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        if (c0 + c < nc) {
            const IBox C = base[c0 + c];
            if (gap2_shift(A, C, s, W) < T) {
                pass |= 1u << c;
                if (maxd2_shift(A, C, s, W) < T) inside |= 1u << c;
            }
        }
    }
}

template <bool FILL>
__global__ void bfs_root_kernel(BatchDev bd, const TreeView* __restrict__ tvs,
                                const IBox* __restrict__ nodes, const IBox* __restrict__ bbox,
                                const int32_t* __restrict__ bboxid, const int64_t* __restrict__ sizes,
                                int64_t cap_in, int32_t* __restrict__ cnt,
                                const int64_t* __restrict__ off, FEntry* __restrict__ out,
                                int64_t cap_out, MonoDev mono) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= cap_in) return;
    if (b >= sizes[kNBlock]) {
        if (!FILL) cnt[b] = 0;
        return;
    }
    const int x = bboxid[b];
    const TreeView& tv = tvs[x];
    const int64_t W = bd.box[x].W, T = bd.box[x].T;
    const IBox A = bbox[b];
    int mask[3];
    allowed_shifts(A, W, T, mask);
    const int top = tv.nlev - 1;
    const IBox R = nodes[tv.off[top]];
    int64_t o = FILL ? off[b] : 0;
    int32_t c = 0;
    for (int sc = 0; sc < 27; ++sc) {
        int s[3];
        decode_shift(sc, s);
        if (!shift_allowed(mask, s)) continue;
        if (!(gap2_shift(A, R, s, W) < T)) continue;
        if (FILL) {
            FEntry e;
            e.blk = (int32_t)b;
            e.node = 0;
            e.sc = (uint8_t)sc;
            e.lev = (uint8_t)top;
            e.inside = maxd2_shift(A, R, s, W) < T;
            e.mono = (mono.theta2 > 0.0 || mono.alpha > 0.0) && top >= kMonoMinLevel &&
                     accept_monopole(A, R, s, W, mono, tv.off[top], b, bd.box[x].G, bd.box[x].cell);
            if (o < cap_out) out[o] = e;
            ++o;
        } else {
            ++c;
        }
    }
    if (!FILL) cnt[b] = c;
}

// One level down: entries above the DFS level that are not inside are
// replaced by their passing children; the others are carried unchanged.
// The count pass keeps each opened entry's child tests (passing children in
// the low byte, inside children in the next) in cmask, and the fill pass
// reads them back instead of testing the child boxes again.
template <bool FILL>
__global__ void bfs_level_kernel(BatchDev bd, const TreeView* __restrict__ tvs,
                                 const IBox* __restrict__ nodes, const IBox* __restrict__ bbox,
                                 const int32_t* __restrict__ bboxid, const FEntry* __restrict__ in,
                                 const int64_t* __restrict__ F_in, int64_t cap_in, int stop,
                                 int32_t* __restrict__ cnt, const int64_t* __restrict__ off,
                                 FEntry* __restrict__ out, int64_t cap_out, MonoDev mono,
                                 uint16_t* __restrict__ cmask) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= cap_in) return;
    if (e >= *F_in) {
        if (!FILL) cnt[e] = 0;
        return;
    }
    const FEntry E = in[e];
    // with monopole acceptance, inside entries are opened too (a child may
    // be accepted); accepted entries are final
    const bool mono_on = mono.theta2 > 0.0 || mono.alpha > 0.0;
    if (E.mono || E.lev <= stop || (E.inside && !mono_on)) {
        if (FILL) {
            if (off[e] < cap_out) out[off[e]] = E;
        } else {
            cnt[e] = 1;
        }
        return;
    }
    const int x = bboxid[E.blk];
    int s[3];
    decode_shift(E.sc, s);
    uint32_t pass, inside;
    if (!FILL) {
        expand2(tvs[x], nodes, E.lev, E.node, bbox[E.blk], s, bd.box[x].W, bd.box[x].T, pass, inside);
        cnt[e] = __popc(pass);
        cmask[e] = (uint16_t)(pass | (inside << 8));
        return;
    }
    const uint32_t m = cmask[e];
    pass = m & 0xffu;
    inside = m >> 8;
    int64_t o = off[e];
    while (pass) {
        const int c = __builtin_ctz(pass);
        pass &= pass - 1;
        FEntry C;
        C.blk = E.blk;
        C.node = 8 * E.node + c;
        C.sc = E.sc;
        C.lev = (uint8_t)(E.lev - 1);
        C.inside = (inside >> c) & 1u;
        C.mono = mono_on && C.lev >= kMonoMinLevel &&
                 accept_monopole(bbox[E.blk], nodes[tvs[x].off[C.lev] + C.node], s, bd.box[x].W, mono,
                                 tvs[x].off[C.lev] + C.node, E.blk, bd.box[x].G, bd.box[x].cell);
        if (o < cap_out) out[o] = C;
        ++o;
    }
}

// Depth-first walk of one entry's subtree (at most 8^2 = 64 leaves).  The
// count pass records which leaves of the subtree pass as a 64-bit mask
// (bit = leaf - first leaf of the subtree); the fill pass turns the mask
// back into runs without testing boxes again, writing them from range slot
// o and list position pos.  Inside entries and leaf entries are a single
// run and need no mask.  Returns the entry's runs (nr) and sources (tot);
// with monopole acceptance on (count pass), children met by the walk are
// tested too: accepted leaves go to m0 (bit = leaf - first leaf of the
// entry), accepted groups of 8 leaves to m1 (bit = group - first group),
// and are not listed.
template <bool FILL>
__device__ void entry_ranges(const BatchDev& bd, const TreeView* __restrict__ tvs,
                             const IBox* __restrict__ nodes, const FEntry E, int64_t e,
                             const IBox* __restrict__ bbox, const int32_t* __restrict__ bboxid,
                             const int64_t* __restrict__ leaf_begin,
                             const int32_t* __restrict__ leaf_count, uint64_t* __restrict__ lmask,
                             int32_t* __restrict__ rbeg, int32_t* __restrict__ rpre,
                             uint8_t* __restrict__ rcode, const MonoDev& mono, int64_t o,
                             int64_t pos, int64_t cap_range, int32_t& nr, int64_t& tot,
                             uint64_t& m0, uint32_t& m1) {
    const int x = bboxid[E.blk];
    const TreeView& tv = tvs[x];
    const int64_t nleaf = tv.cnt[0];
    const bool mono_on = !FILL && (mono.theta2 > 0.0 || mono.alpha > 0.0);
    m0 = 0;
    m1 = 0;
    nr = 0;
    tot = 0;
    // one run of local leaves [l0, l1]
    auto emit = [&](int64_t l0, int64_t l1) {
        const int64_t p0 = leaf_begin[tv.loff + l0];
        const int64_t p1 = leaf_begin[tv.loff + l1] + leaf_count[tv.loff + l1];
        if (FILL) {
            if (o < cap_range) {
                rbeg[o] = (int32_t)p0;
                rpre[o] = (int32_t)pos;
                rcode[o] = E.sc;
            }
            ++o;
        }
        ++nr;
        pos += p1 - p0;
        tot += p1 - p0;
    };
    const int64_t first = (int64_t)E.node << (3 * E.lev);
    int64_t last = (((int64_t)E.node + 1) << (3 * E.lev)) - 1;
    if (last > nleaf - 1) last = nleaf - 1;
    const bool walk_inside = mono.theta2 > 0.0 || mono.alpha > 0.0;   // inside nodes are opened too
    if (E.mono) {
        // a monopole: no source ranges
    } else if (E.lev == 0 || (E.inside && !walk_inside)) {
        emit(first, last);
    } else {
        uint64_t mask = 0;
        if (FILL) {
            mask = lmask[e];
        } else {
            const IBox A = bbox[E.blk];
            const int64_t W = bd.box[x].W, T = bd.box[x].T;
            int s[3];
            decode_shift(E.sc, s);
            // 16 bits per level: low byte pending children, high byte inside children
            uint64_t st = 0;
            int lev = E.lev;
            int64_t node = E.node;
            uint32_t pa, in;
            expand2(tv, nodes, lev, node, A, s, W, T, pa, in);
            st |= (uint64_t)(pa | (in << 8)) << (16 * (lev & 3));
            for (;;) {
                const uint32_t wv = (uint32_t)(st >> (16 * (lev & 3))) & 0xffffu;
                const uint32_t m = wv & 0xffu;
                if (m == 0) {
                    if (lev == E.lev) break;
                    ++lev;
                    node >>= 3;
                    continue;
                }
                const int c = __builtin_ctz(m);
                const uint32_t w2 = wv & ~(1u << c);
                st = (st & ~(0xffffull << (16 * (lev & 3)))) | ((uint64_t)w2 << (16 * (lev & 3)));
                const int64_t child = 8 * node + c;
                if (mono_on) {
                    const int64_t g = tv.off[lev - 1] + child;
                    if (accept_monopole(A, nodes[g], s, W, mono, g, E.blk, bd.box[x].G, bd.box[x].cell)) {
                        if (lev == 1) m0 |= 1ull << (child - first);
                        else m1 |= 1u << (child - (first >> 3));
                        continue;
                    }
                }
                if (lev == 1 || (!walk_inside && ((wv >> 8) >> c & 1u))) {
                    const int64_t l0 = child << (3 * (lev - 1));
                    int64_t l1 = ((child + 1) << (3 * (lev - 1))) - 1;
                    if (l1 > nleaf - 1) l1 = nleaf - 1;
                    for (int64_t l = l0; l <= l1; ++l) mask |= 1ull << (l - first);
                } else {
                    --lev;
                    node = child;
                    expand2(tv, nodes, lev, node, A, s, W, T, pa, in);
                    st = (st & ~(0xffffull << (16 * (lev & 3)))) |
                         ((uint64_t)(pa | (in << 8)) << (16 * (lev & 3)));
                }
            }
            lmask[e] = mask;
        }
        // runs of set bits, ascending
        while (mask) {
            const int a = __builtin_ctzll(mask);
            const uint64_t above = ~mask & (~0ull << a);      // first clear bit at or above a
            const int z = above ? __builtin_ctzll(above) : 64;
            emit(first + a, first + z - 1);
            mask = z >= 64 ? 0ull : mask & (~0ull << z);
        }
    }
}

// Count pass: every entry walks its subtree and records its runs (rcnt)
// and listed sources (scnt); entries past the entry count get zero.
__global__ void ranges_count_kernel(BatchDev bd, const TreeView* __restrict__ tvs,
                                    const IBox* __restrict__ nodes, const FEntry* __restrict__ ent,
                                    int64_t F, const IBox* __restrict__ bbox,
                                    const int32_t* __restrict__ bboxid,
                                    const int64_t* __restrict__ leaf_begin,
                                    const int32_t* __restrict__ leaf_count,
                                    uint64_t* __restrict__ lmask, int32_t* __restrict__ rcnt,
                                    int32_t* __restrict__ scnt, MonoDev mono,
                                    uint64_t* __restrict__ mono0, uint8_t* __restrict__ mono1,
                                    const int64_t* __restrict__ sizes) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= F) return;                       // F: the capacity of the entry buffer
    int32_t nr = 0;
    int64_t tot = 0;
    uint64_t m0 = 0;
    uint32_t m1 = 0;
    if (e < sizes[kNEntry])
        entry_ranges<false>(bd, tvs, nodes, ent[e], e, bbox, bboxid, leaf_begin, leaf_count, lmask,
                            nullptr, nullptr, nullptr, mono, 0, 0, 0, nr, tot, m0, m1);
    rcnt[e] = nr;
    scnt[e] = (int32_t)(tot < INT32_MAX ? tot : INT32_MAX);
    if (mono0) {
        mono0[e] = m0;
        mono1[e] = (uint8_t)m1;
    }
}

// Per-block range offsets and list lengths; flags a list longer than int32.
__global__ void block_sum_kernel(const int64_t* __restrict__ eoff, const int64_t* __restrict__ roff_e,
                                 const int64_t* __restrict__ soff_e, int64_t* __restrict__ sizes,
                                 int64_t cap_block, int64_t* __restrict__ roff,
                                 int32_t* __restrict__ slen) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nblock = sizes[kNBlock];
    if (b > nblock || b > cap_block) return;
    roff[b] = roff_e[eoff[b]];
    if (b == nblock) return;
    const int64_t len = soff_e[eoff[b + 1]] - soff_e[eoff[b]];
    if (len > INT32_MAX) atomicOr(reinterpret_cast<unsigned long long*>(sizes + kOverflow), 16ull);
    slen[b] = (int32_t)(len < INT32_MAX ? len : INT32_MAX);
}

// Fill pass: every entry writes its runs from its first range slot, with
// list positions relative to its block.
__global__ void ranges_fill_kernel(BatchDev bd, const TreeView* __restrict__ tvs,
                                   const IBox* __restrict__ nodes, const FEntry* __restrict__ ent,
                                   int64_t F, const IBox* __restrict__ bbox,
                                   const int32_t* __restrict__ bboxid,
                                   const int64_t* __restrict__ leaf_begin,
                                   const int32_t* __restrict__ leaf_count,
                                   uint64_t* __restrict__ lmask, const int64_t* __restrict__ roff_e,
                                   const int64_t* __restrict__ soff_e, const int64_t* __restrict__ eoff,
                                   int32_t* __restrict__ rbeg, int32_t* __restrict__ rpre,
                                   uint8_t* __restrict__ rcode, MonoDev mono,
                                   const int64_t* __restrict__ sizes, int64_t cap_range) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= F || e >= sizes[kNEntry]) return;    // F: the capacity of the entry buffer
    const FEntry E = ent[e];
    int32_t nr;
    int64_t tot;
    uint64_t m0;
    uint32_t m1;
    entry_ranges<true>(bd, tvs, nodes, E, e, bbox, bboxid, leaf_begin, leaf_count, lmask, rbeg, rpre,
                       rcode, mono, roff_e[e], soff_e[e] - soff_e[eoff[E.blk]], cap_range, nr, tot, m0, m1);
}

// First entry of every block (entries are sorted by block).
__global__ void block_entry_kernel(const FEntry* __restrict__ ent, const int64_t* __restrict__ sizes,
                                   int64_t cap_block, int64_t* __restrict__ eoff) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nblock = sizes[kNBlock], F = sizes[kNEntry];
    if (b > nblock || b > cap_block) return;
    int64_t lo = 0, hi = F;             // first e with ent[e].blk >= b
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (ent[mid].blk < b) lo = mid + 1;
        else hi = mid;
    }
    eoff[b] = lo;
}

// Listed sources in all (sum of the block list lengths) and the effective
// chunk: the requested one, or larger when the item partial sums (3 x 64
// floats per item) would pass max_items items.
__global__ void chunk_kernel(const int64_t* __restrict__ soff_e, int64_t* __restrict__ sizes,
                             int64_t chunk_req, int64_t max_items) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    const int64_t total = soff_e[sizes[kNEntry]];
    sizes[kTotalSrc] = total;
    int64_t chunk = chunk_req;
    const int64_t need = (total + max_items - 1) / max_items;
    if (need > chunk) chunk = ((need + kBlock - 1) / kBlock) * kBlock;
    if (chunk > INT32_MAX / 2) chunk = INT32_MAX / 2;
    sizes[kChunk] = chunk;
}

// Work items per block: its list in chunks (at least one item, so that every
// target is written); none for a block without an active target when flags
// are given.
__global__ void item_count_kernel(const int32_t* __restrict__ slen,
                                  const int32_t* __restrict__ bcount, int64_t* __restrict__ sizes,
                                  int64_t cap_block, const uint8_t* __restrict__ active,
                                  const int32_t* __restrict__ perm,
                                  const int32_t* __restrict__ bstart,
                                  int32_t* __restrict__ icount) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= cap_block) return;
    if (b >= sizes[kNBlock]) {
        icount[b] = 0;
        return;
    }
    if (active) {
        bool on = false;
        for (int32_t k = 0; k < bcount[b] && !on; ++k) on = active[perm[(int64_t)bstart[b] + k]] != 0;
        if (!on) {
            icount[b] = 0;
            return;
        }
    }
    const int32_t s = slen[b];
    const int64_t chunk = sizes[kChunk];
    icount[b] = s <= 0 ? 1 : (int32_t)((s + chunk - 1) / chunk);
    // (target, listed source) pairs; the kernel prunes some sources further
    atomicAdd(reinterpret_cast<unsigned long long*>(sizes + kCand),
              (unsigned long long)s * (unsigned long long)bcount[b]);
}

__global__ void item_fill_kernel(const int32_t* __restrict__ icount,
                                 const int64_t* __restrict__ ioff, const int64_t* __restrict__ sizes,
                                 int64_t cap_item, int32_t* __restrict__ iblock,
                                 int32_t* __restrict__ is0) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= sizes[kNBlock]) return;
    const int64_t o = ioff[b];
    const int64_t chunk = sizes[kChunk];
    for (int32_t c = 0; c < icount[b]; ++c) {
        if (o + c >= cap_item) return;
        iblock[o + c] = (int32_t)b;
        is0[o + c] = (int32_t)(c * chunk);
    }
}


// Item and range totals, and the flag that makes the PP kernels return.
__global__ void finish_sizes_kernel(int64_t* __restrict__ sizes, const int64_t* __restrict__ ioff,
                                    const int64_t* __restrict__ roff, int64_t cap_item,
                                    int64_t cap_range, const int* __restrict__ bad) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    const int64_t nb = sizes[kNBlock];
    const int64_t ni = ioff[nb], nr = roff[nb];
    sizes[kNeedItem] = ni;
    sizes[kNeedRange] = nr;
    sizes[kNItem] = ni < cap_item ? ni : cap_item;
    sizes[kNRange] = nr < cap_range ? nr : cap_range;
    if (ni > cap_item) sizes[kOverflow] |= 8;
    if (nr > cap_range) sizes[kOverflow] |= 4;
    sizes[kBad] = bad ? *bad : 0;
    sizes[kSkip] = (sizes[kOverflow] != 0 || sizes[kBad] != 0 || sizes[kMoved] != 0) ? 1 : 0;
}

// Per-pass slots of a pass that reuses the lists (the list counts stay; the
// overflow bits of the last pass go, since the lists' own buffers fitted).
__global__ void zero_sizes_reuse_kernel(int64_t* __restrict__ sizes, int* __restrict__ bad) {
    if (threadIdx.x != 0) return;
    sizes[kOverflow] = 0;
    sizes[kCand] = 0;
    sizes[kMoved] = 0;
    sizes[kSkip] = 0;
    sizes[kBad] = 0;
    *bad = 0;
}

__global__ void zero_sizes_kernel(int64_t* __restrict__ sizes, int* __restrict__ bad) {
    if (threadIdx.x < kSizeSlots) sizes[threadIdx.x] = 0;
    if (threadIdx.x == 0) *bad = 0;
}

}  // namespace

// A grid for a grid-stride loop over at most n items.
static unsigned stride_grid(int64_t n, int t) {
    const int64_t b = (n + t - 1) / t;
    return (unsigned)(b < 1 ? 1 : (b > 65536 ? 65536 : b));
}

// Nodes of the implicit trees over at most n leaves in nbox boxes: the
// leaves plus at most n / 7 + 1 nodes per level above them in every box.
static int64_t tree_node_bound(int64_t n, int nbox) {
    const int64_t m = n > 0 ? n : 1;
    return m + m / 7 + (int64_t)nbox * kTreeMaxLevels + 8;
}

// Levels of the implicit tree over at most n leaves.
static int levels_for(int64_t n) {
    int h = 1;
    int64_t c = n > 0 ? n : 1;
    while (c > 1 && h < kTreeMaxLevels) {
        c = (c + 7) / 8;
        ++h;
    }
    return h;
}

// Clears the count slots and the bad-input flag.
int reset_sizes(Work& w, hipStream_t s) {
    PP_TRY(w.sizes.reserve(sizeof(int64_t) * kSizeSlots));
    PP_TRY(w.bad.reserve(64));
    hipLaunchKernelGGL(zero_sizes_kernel, dim3(1), dim3(kSizeSlots), 0, s, w.sizes.as<int64_t>(),
                       w.bad.as<int>());
    PP_HIP(hipGetLastError());
    return PP_OK;
}

int reset_sizes_reuse(Work& w, hipStream_t s) {
    hipLaunchKernelGGL(zero_sizes_reuse_kernel, dim3(1), dim3(64), 0, s, w.sizes.as<int64_t>(),
                       w.bad.as<int>());
    PP_HIP(hipGetLastError());
    return PP_OK;
}

int stage_leaves(const BatchDev& bd, int64_t N, const uint64_t* sorted_keys, const double* pos_s,
                 Work& w, hipStream_t s) {
    PP_TRY(w.sizes.reserve(sizeof(int64_t) * kSizeSlots));
    PP_TRY(w.loff_dev.reserve(sizeof(int64_t) * (bd.nbox + 1)));
    const int M = bd.leaf_max;
    const int64_t len = N + M;
    const int64_t m = N > 0 ? N : 1;        // leaves: at most one per particle
    PP_TRY(w.lam.reserve(len + 1));
    PP_TRY(w.pmax.reserve(len + 1));
    PP_TRY(w.smax.reserve(len + 1));
    PP_TRY(w.level_p.reserve(N + 1));
    PP_TRY(w.flag.reserve(sizeof(int32_t) * (N + 1)));
    PP_TRY(w.flag_off.reserve(sizeof(int64_t) * (N + 2)));
    PP_TRY(w.lbegin.reserve(sizeof(int64_t) * (m + 1)));
    PP_TRY(w.lcount.reserve(sizeof(int32_t) * (m + 1)));
    PP_TRY(w.llevel.reserve(sizeof(int32_t) * (m + 1)));
    PP_TRY(w.lprefix.reserve(sizeof(uint64_t) * (m + 1)));
    // the leaf boxes are level 0 of the trees' node array (leaf a of the
    // batch is node a): the tree levels go after them
    PP_TRY(w.tree_boxes.reserve(sizeof(IBox) * tree_node_bound(N, bd.nbox)));
    if (N > 0) {
        hipLaunchKernelGGL(lam_kernel, dim3(blocks_for(len, 256)), dim3(256), 0, s, bd, sorted_keys, N,
                           w.lam.as<int8_t>());
        const int64_t nblk = (len + M) / (M + 1);
        hipLaunchKernelGGL(vhgw_kernel, dim3(blocks_for(nblk, 256)), dim3(256), 0, s,
                           w.lam.as<int8_t>(), len, M + 1, w.pmax.as<int8_t>(), w.smax.as<int8_t>());
        hipLaunchKernelGGL(level_kernel, dim3(blocks_for(N, 256)), dim3(256), 0, s, w.pmax.as<int8_t>(),
                           w.smax.as<int8_t>(), N, M, bd.bits, w.level_p.as<int8_t>());
        hipLaunchKernelGGL(flag_kernel, dim3(blocks_for(N, 256)), dim3(256), 0, s, bd, sorted_keys,
                           w.level_p.as<int8_t>(), N, w.flag.as<int32_t>());
        PP_HIP(hipGetLastError());
    }
    PP_TRY(launch_scan_i32_to_i64(w.flag.as<int32_t>(), w.flag_off.as<int64_t>(), N, w.scan_ws, s, w.sizes.as<int64_t>()));
    hipLaunchKernelGGL(leaf_offsets_kernel, dim3(blocks_for(bd.nbox + 1, 64)), dim3(64), 0, s, bd,
                       w.flag_off.as<int64_t>(), w.loff_dev.as<int64_t>(), w.sizes.as<int64_t>());
    PP_HIP(hipGetLastError());
    if (N > 0) {
        hipLaunchKernelGGL(leaf_fill_kernel, dim3(blocks_for(N, 256)), dim3(256), 0, s, sorted_keys,
                           w.level_p.as<int8_t>(), w.flag.as<int32_t>(), w.flag_off.as<int64_t>(), N,
                           bd.bits, w.lbegin.as<int64_t>(), w.llevel.as<int32_t>(),
                           w.lprefix.as<uint64_t>());
        hipLaunchKernelGGL(leaf_box_kernel, dim3(stride_grid(N, 128)), dim3(128), 0, s, bd, pos_s, N,
                           w.lbegin.as<int64_t>(), w.sizes.as<int64_t>(), w.lcount.as<int32_t>(),
                           w.tree_boxes.as<IBox>());
        PP_HIP(hipGetLastError());
    }
    return PP_OK;
}

int leaves_to_host(const BatchDev& bd, Work& w, hipStream_t s) {
    w.loff.assign(bd.nbox + 1, 0);
    PP_HIP(hipMemcpyAsync(w.loff.data(), w.loff_dev.p, sizeof(int64_t) * (bd.nbox + 1),
                          hipMemcpyDeviceToHost, s));
    PP_HIP(hipStreamSynchronize(s));
    w.nleaf = w.loff[bd.nbox];
    return PP_OK;
}

int stage_trees(const BatchDev& bd, int64_t N, Work& w, hipStream_t s) {
    const int nbox = bd.nbox;
    const int H = levels_for(N);
    w.max_levels = H;
    PP_TRY(w.tree_boxes.reserve(sizeof(IBox) * tree_node_bound(N, nbox)));
    PP_TRY(w.tviews.reserve(sizeof(TreeView) * nbox));
    PP_TRY(w.lvl_prefix.reserve(sizeof(int64_t) * (size_t)kTreeMaxLevels * (nbox + 1)));
    PP_TRY(w.tree_total.reserve(sizeof(int64_t) * 2));
    hipLaunchKernelGGL(tree_views_kernel, dim3(1), dim3(256), 0, s, w.loff_dev.as<int64_t>(), nbox,
                       w.tviews.as<TreeView>(), w.lvl_prefix.as<int64_t>(), w.tree_total.as<int64_t>());
    PP_HIP(hipGetLastError());
    IBox* nodes = w.tree_boxes.as<IBox>();       // level 0: the leaf boxes (stage_leaves)
    int64_t bound = N;
    for (int h = 1; h < H; ++h) {
        bound = (bound + 7) / 8 + nbox;
        hipLaunchKernelGGL(tree_level_kernel, dim3(stride_grid(bound, 256)), dim3(256), 0, s,
                           w.tviews.as<TreeView>(), w.lvl_prefix.as<int64_t>() + (size_t)h * (nbox + 1),
                           nbox, h, nodes);
    }
    PP_HIP(hipGetLastError());
    return PP_OK;
}

int trees_to_host(const BatchDev& bd, Work& w, hipStream_t s) {
    w.tv.assign(bd.nbox, TreeView{});
    PP_HIP(hipMemcpyAsync(w.tv.data(), w.tviews.p, sizeof(TreeView) * bd.nbox, hipMemcpyDeviceToHost, s));
    PP_HIP(hipStreamSynchronize(s));
    return PP_OK;
}

int stage_node_moments(const BatchDev& bd, int64_t N, Work& w, hipStream_t s) {
    const int nbox = bd.nbox;
    PP_TRY(w.tree_mc.reserve(sizeof(double4) * tree_node_bound(N, nbox)));
    if (N == 0) return PP_OK;
    double4* mc = w.tree_mc.as<double4>();
    hipLaunchKernelGGL(leaf_moment_kernel, dim3(stride_grid(N, 128)), dim3(128), 0, s,
                       w.pos_s.as<double>(), w.mass_s.as<float>(), w.pos_n, w.lbegin.as<int64_t>(),
                       w.sizes.as<int64_t>(), mc);
    int64_t bound = N;
    for (int h = 1; h < w.max_levels; ++h) {
        bound = (bound + 7) / 8 + nbox;
        hipLaunchKernelGGL(tree_moment_kernel, dim3(stride_grid(bound, 256)), dim3(256), 0, s,
                           w.tviews.as<TreeView>(), w.lvl_prefix.as<int64_t>() + (size_t)h * (nbox + 1),
                           nbox, h, mc);
    }
    PP_HIP(hipGetLastError());
    return PP_OK;
}

int build_canonical_pairs(const BatchDev& bd, const Work& w, int64_t W, int64_t T, DevBuf& row_cnt,
                          DevBuf& row_ptr, DevBuf& src, DevBuf& code, DevBuf& scan_ws,
                          int64_t* nentries, hipStream_t s) {
    (void)bd;
    const int64_t nleaf = w.nleaf;     // host copies: leaves_to_host, trees_to_host
    PP_TRY(row_cnt.reserve(sizeof(int32_t) * (nleaf + 1)));
    PP_TRY(row_ptr.reserve(sizeof(int64_t) * (nleaf + 1)));
    *nentries = 0;
    if (nleaf == 0) {
        PP_TRY(launch_scan_i32_to_i64(row_cnt.as<int32_t>(), row_ptr.as<int64_t>(), 0, scan_ws, s));
        PP_HIP(hipStreamSynchronize(s));
        return PP_OK;
    }
    const TreeView tv = w.tv[0];
    const IBox* nodes = w.tree_boxes.as<IBox>();
    hipLaunchKernelGGL(canon_kernel<false>, dim3(blocks_for(nleaf, 64)), dim3(64), 0, s, tv, nodes,
                       nleaf, W, T, row_cnt.as<int32_t>(), (const int64_t*)nullptr,
                       (int32_t*)nullptr, (uint8_t*)nullptr);
    PP_HIP(hipGetLastError());
    PP_TRY(launch_scan_i32_to_i64(row_cnt.as<int32_t>(), row_ptr.as<int64_t>(), nleaf, scan_ws, s));
    int64_t tot = 0;
    PP_TRY(read_back(row_ptr.as<int64_t>() + nleaf, &tot, s));
    PP_TRY(src.reserve(sizeof(int32_t) * (tot + 1)));
    PP_TRY(code.reserve(sizeof(uint8_t) * (tot + 1)));
    hipLaunchKernelGGL(canon_kernel<true>, dim3(blocks_for(nleaf, 64)), dim3(64), 0, s, tv, nodes,
                       nleaf, W, T, (int32_t*)nullptr, row_ptr.as<int64_t>(), src.as<int32_t>(),
                       code.as<uint8_t>());
    PP_HIP(hipGetLastError());
    *nentries = tot;
    return PP_OK;
}

// Capacities start from estimates and grow to 5/4 of what a pass needed
// whenever a buffer was too small (lists_to_host); the pass then runs again.
static int64_t grow_cap(int64_t cap, int64_t need) {
    if (need <= cap) return cap;
    return need + need / 4 + 1024;
}

// After a pass that fitted: a capacity well above the need comes down to it
// (plus the margin).  The grids and scans of the list builder span the
// capacities, so a first guess far above the need (the entry passes start
// from doublings) would otherwise keep costing time on every call.
static int64_t settle_cap(int64_t cap, int64_t need) {
    const int64_t want = need + need / 4 + 1024;
    return cap > want + want / 2 ? want : cap;
}

int stage_lists(const BatchDev& bd, const std::vector<int64_t>& poff, int chunk_req, Work& w,
                hipStream_t s, const MonoCfg& mcfg, const uint8_t* active) {
    const int nbox = bd.nbox;
    const int64_t N = poff[nbox];
    int64_t* sizes = w.sizes.as<int64_t>();
    // chunks of kBlock particles inside each box (offsets change only with
    // the box sizes; uploaded synchronously then)
    std::vector<int64_t> choff(nbox + 1, 0);
    for (int x = 0; x < nbox; ++x)
        choff[x + 1] = choff[x] + (poff[x + 1] - poff[x] + kBlock - 1) / kBlock;
    const int64_t nc = choff[nbox];
    w.nchunk = nc;
    PP_TRY(w.choff.reserve(sizeof(int64_t) * (nbox + 1)));
    if (choff != w.choff_h) {
        PP_HIP(hipMemcpy(w.choff.p, choff.data(), sizeof(int64_t) * (nbox + 1), hipMemcpyHostToDevice));
        w.choff_h = choff;
    }
    // capacities: blocks from the chunks, the rest from the last need
    if (w.cap_block < nc + nc / 8 + 64) w.cap_block = nc + nc / 8 + 64;
    const int64_t cb = w.cap_block;
    if (w.cap_ent[0] < 4 * cb) w.cap_ent[0] = 4 * cb;
    PP_TRY(w.ccount.reserve(sizeof(int32_t) * (nc + 1)));
    PP_TRY(w.coff.reserve(sizeof(int64_t) * (nc + 2)));
    PP_TRY(w.bstart.reserve(sizeof(int32_t) * cb));
    PP_TRY(w.bcount.reserve(sizeof(int32_t) * cb));
    PP_TRY(w.bbox.reserve(sizeof(IBox) * cb));
    PP_TRY(w.bboxid.reserve(sizeof(int32_t) * cb));
    PP_TRY(w.slen.reserve(sizeof(int32_t) * cb));
    PP_TRY(w.roff.reserve(sizeof(int64_t) * (cb + 2)));
    PP_TRY(w.icount.reserve(sizeof(int32_t) * (cb + 1)));
    PP_TRY(w.ioff.reserve(sizeof(int64_t) * (cb + 2)));
    PP_TRY(w.eoff.reserve(sizeof(int64_t) * (cb + 2)));
    // expansion passes (see below) and their entry capacities: the root pass
    // and H - 2 lowering passes, the last of which (level 2 to 1) is left
    // out when it would need too many entries
    const int H = w.max_levels;
    int nlower = H > 2 ? H - 2 : 0;
    const bool to_level1 = !w.stop_at_level2 || nlower == 0;
    if (!to_level1) nlower -= 1;
    const int npass = 1 + nlower;
    w.npass = npass;
    for (int p = 0; p < npass; ++p)
        if (w.cap_ent[p] < 1024) w.cap_ent[p] = p == 0 ? 4 * cb : w.cap_ent[p - 1] * 2;
    int64_t capcnt = cb;
    for (int p = 0; p < npass; ++p) capcnt = w.cap_ent[p] > capcnt ? w.cap_ent[p] : capcnt;
    // the scans' workspace for the largest scan of the pass, reserved before
    // the first one is enqueued
    PP_TRY(grow_scan(w.scan_ws, 2 * (capcnt > nc ? capcnt : nc), s));
    const double* pos_s = w.pos_s.as<double>();
    if (nc > 0) {
        hipLaunchKernelGGL(block_split_kernel<false>, dim3((unsigned)nc), dim3(kBlock), 0, s, bd,
                           pos_s, N, w.choff.as<int64_t>(), nc, w.ccount.as<int32_t>(),
                           (const int64_t*)nullptr, (int32_t*)nullptr, (int32_t*)nullptr,
                           (IBox*)nullptr, (int32_t*)nullptr, cb);
        PP_HIP(hipGetLastError());
    }
    {
        const ScanNote note{(int)kNBlock, (int)kNeedBlock, cb, 1ull, -1};
        PP_TRY(launch_scan_i32_to_i64(w.ccount.as<int32_t>(), w.coff.as<int64_t>(), nc, w.scan_ws, s, sizes,
                                      &note));
    }
    if (nc > 0)
        hipLaunchKernelGGL(block_split_kernel<true>, dim3((unsigned)nc), dim3(kBlock), 0, s, bd,
                           pos_s, N, w.choff.as<int64_t>(), nc, (int32_t*)nullptr,
                           w.coff.as<int64_t>(), w.bstart.as<int32_t>(), w.bcount.as<int32_t>(),
                           w.bbox.as<IBox>(), w.bboxid.as<int32_t>(), cb);
    PP_HIP(hipGetLastError());
    const TreeView* tvs = w.tviews.as<TreeView>();
    const IBox* nodes = w.tree_boxes.as<IBox>();
    const IBox* bbox = w.bbox.as<IBox>();
    const int32_t* bboxid = w.bboxid.as<int32_t>();
    MonoDev mono{mcfg.theta2, mcfg.alpha, mcfg.mc, nullptr};
    if (mcfg.alpha > 0.0) {
        PP_TRY(w.blk_amin2.reserve(sizeof(double) * (cb + 1)));
        hipLaunchKernelGGL(block_amin_kernel, dim3(blocks_for(cb, 128)), dim3(128), 0, s,
                           w.bstart.as<int32_t>(), w.bcount.as<int32_t>(), w.perm.as<int32_t>(),
                           mcfg.acc_ref, w.pos_n, sizes, w.blk_amin2.as<double>());
        PP_HIP(hipGetLastError());
        mono.amin2 = w.blk_amin2.as<double>();
    }
    // Breadth-first expansion from every box's root: pass 0 takes the roots,
    // every later pass lowers the entries above level 2 by one level and the
    // last pass lowers level 2 to level 1 (when it does not exceed the entry
    // budget), so that the depth-first walks cover at most 8 (else 64)
    // leaves each; passes beyond a box's depth carry its entries unchanged.
    // Entry buffers alternate between two arrays.
    int64_t cap_a = 0, cap_b = 0;
    for (int p = 0; p < npass; ++p) {
        int64_t& c = p % 2 == 0 ? cap_a : cap_b;
        c = w.cap_ent[p] > c ? w.cap_ent[p] : c;
    }
    PP_TRY(w.fent_a.reserve(sizeof(FEntry) * (cap_a + 1)));
    PP_TRY(w.fent_b.reserve(sizeof(FEntry) * (cap_b + 1)));
    PP_TRY(w.fcnt.reserve(sizeof(int32_t) * (capcnt + 1)));
    PP_TRY(w.foff.reserve(sizeof(int64_t) * (capcnt + 2)));
    PP_TRY(w.fmask.reserve(sizeof(uint16_t) * (capcnt + 1)));
    hipLaunchKernelGGL(bfs_root_kernel<false>, dim3(blocks_for(cb, 128)), dim3(128), 0, s, bd, tvs,
                       nodes, bbox, bboxid, (const int64_t*)sizes, cb, w.fcnt.as<int32_t>(),
                       (const int64_t*)nullptr, (FEntry*)nullptr, (int64_t)0, mono);
    PP_HIP(hipGetLastError());
    {
        const ScanNote note{(int)kEntry0, (int)kNeedEntry0, w.cap_ent[0], 2ull, npass == 1 ? (int)kNEntry : -1};
        PP_TRY(launch_scan_i32_to_i64(w.fcnt.as<int32_t>(), w.foff.as<int64_t>(), cb, w.scan_ws, s, sizes,
                                      &note));
    }
    hipLaunchKernelGGL(bfs_root_kernel<true>, dim3(blocks_for(cb, 128)), dim3(128), 0, s, bd, tvs,
                       nodes, bbox, bboxid, (const int64_t*)sizes, cb, (int32_t*)nullptr,
                       w.foff.as<int64_t>(), w.fent_a.as<FEntry>(), w.cap_ent[0], mono);
    PP_HIP(hipGetLastError());
    DevBuf* cur = &w.fent_a;
    DevBuf* nxt = &w.fent_b;
    for (int p = 1; p < npass; ++p) {
        const int stop = (p == npass - 1 && to_level1) ? kDfsLevel - 1 : kDfsLevel;
        const int64_t cin = w.cap_ent[p - 1], cout = w.cap_ent[p];
        hipLaunchKernelGGL(bfs_level_kernel<false>, dim3(blocks_for(cin, 128)), dim3(128), 0, s, bd,
                           tvs, nodes, bbox, bboxid, cur->as<FEntry>(),
                           (const int64_t*)(sizes + kEntry0 + p - 1), cin, stop, w.fcnt.as<int32_t>(),
                           (const int64_t*)nullptr, (FEntry*)nullptr, (int64_t)0, mono, w.fmask.as<uint16_t>());
        PP_HIP(hipGetLastError());
        const ScanNote note{(int)(kEntry0 + p), (int)(kNeedEntry0 + p), cout, 2ull,
                            p == npass - 1 ? (int)kNEntry : -1};
        PP_TRY(launch_scan_i32_to_i64(w.fcnt.as<int32_t>(), w.foff.as<int64_t>(), cin, w.scan_ws, s, sizes,
                                      &note));
        hipLaunchKernelGGL(bfs_level_kernel<true>, dim3(blocks_for(cin, 128)), dim3(128), 0, s, bd, tvs,
                           nodes, bbox, bboxid, cur->as<FEntry>(),
                           (const int64_t*)(sizes + kEntry0 + p - 1), cin, stop, (int32_t*)nullptr,
                           w.foff.as<int64_t>(), nxt->as<FEntry>(), cout, mono, w.fmask.as<uint16_t>());
        PP_HIP(hipGetLastError());
        DevBuf* t = cur;
        cur = nxt;
        nxt = t;
    }
    const int64_t F = w.cap_ent[npass - 1];    // the final entry buffer's capacity
    const FEntry* ent = cur->as<FEntry>();
    w.ent_final = ent;
    PP_TRY(w.lmask_e.reserve(sizeof(uint64_t) * (F + 1)));
    PP_TRY(w.rcnt_e.reserve(sizeof(int32_t) * (F + 1)));
    PP_TRY(w.scnt_e.reserve(sizeof(int32_t) * (F + 1)));
    PP_TRY(w.roff_e.reserve(sizeof(int64_t) * (F + 2)));
    PP_TRY(w.soff_e.reserve(sizeof(int64_t) * (F + 2)));
    const int64_t* lbegin = w.lbegin.as<int64_t>();
    const int32_t* lcount = w.lcount.as<int32_t>();
    uint64_t* mono0 = nullptr;
    uint8_t* mono1 = nullptr;
    if (mcfg.on()) {
        PP_TRY(w.mono0_e.reserve(sizeof(uint64_t) * (F + 1)));
        PP_TRY(w.mono1_e.reserve(sizeof(uint8_t) * (F + 1)));
        mono0 = w.mono0_e.as<uint64_t>();
        mono1 = w.mono1_e.as<uint8_t>();
    }
    w.mono0 = mono0;
    w.mono1 = mono1;
    if (w.cap_range < 1024) w.cap_range = 16 * cb;
    if (w.cap_item < 1024) w.cap_item = 2 * cb;
    hipLaunchKernelGGL(ranges_count_kernel, dim3(blocks_for(F, 128)), dim3(128), 0, s, bd, tvs, nodes, ent,
                       F, bbox, bboxid, lbegin, lcount, w.lmask_e.as<uint64_t>(), w.rcnt_e.as<int32_t>(),
                       w.scnt_e.as<int32_t>(), mono, mono0, mono1, (const int64_t*)sizes);
    PP_HIP(hipGetLastError());
    PP_TRY(launch_scan2_i32_to_i64(w.rcnt_e.as<int32_t>(), w.scnt_e.as<int32_t>(), w.roff_e.as<int64_t>(),
                                   w.soff_e.as<int64_t>(), F, w.scan_ws, s, sizes));
    hipLaunchKernelGGL(block_entry_kernel, dim3(blocks_for(cb + 1, 256)), dim3(256), 0, s, ent,
                       (const int64_t*)sizes, cb, w.eoff.as<int64_t>());
    hipLaunchKernelGGL(block_sum_kernel, dim3(blocks_for(cb + 1, 256)), dim3(256), 0, s,
                       (const int64_t*)w.eoff.as<int64_t>(), (const int64_t*)w.roff_e.as<int64_t>(),
                       (const int64_t*)w.soff_e.as<int64_t>(), sizes, cb, w.roff.as<int64_t>(),
                       w.slen.as<int32_t>());
    PP_HIP(hipGetLastError());
    constexpr int64_t kMaxItems = 1 << 21;
    hipLaunchKernelGGL(chunk_kernel, dim3(1), dim3(1), 0, s, (const int64_t*)w.soff_e.as<int64_t>(), sizes,
                       (int64_t)chunk_req, kMaxItems);
    PP_TRY(w.rbeg.reserve(sizeof(int32_t) * (w.cap_range + 1)));
    PP_TRY(w.rpre.reserve(sizeof(int32_t) * (w.cap_range + 1)));
    PP_TRY(w.rcode.reserve(sizeof(uint8_t) * (w.cap_range + 1)));
    hipLaunchKernelGGL(ranges_fill_kernel, dim3(blocks_for(F, 128)), dim3(128), 0, s, bd, tvs, nodes, ent,
                       F, bbox, bboxid, lbegin, lcount, w.lmask_e.as<uint64_t>(),
                       (const int64_t*)w.roff_e.as<int64_t>(), (const int64_t*)w.soff_e.as<int64_t>(),
                       (const int64_t*)w.eoff.as<int64_t>(), w.rbeg.as<int32_t>(), w.rpre.as<int32_t>(),
                       w.rcode.as<uint8_t>(), mono, (const int64_t*)sizes, w.cap_range);
    PP_HIP(hipGetLastError());
    return stage_items(bd, w, s, active);
}

int stage_items(const BatchDev& bd, Work& w, hipStream_t s, const uint8_t* active) {
    int64_t* sizes = w.sizes.as<int64_t>();
    const int64_t cb = w.cap_block;
    w.active = active;
    hipLaunchKernelGGL(item_count_kernel, dim3(blocks_for(cb, 256)), dim3(256), 0, s,
                       w.slen.as<int32_t>(), w.bcount.as<int32_t>(), sizes, cb, active,
                       w.perm.as<int32_t>(), w.bstart.as<int32_t>(), w.icount.as<int32_t>());
    PP_HIP(hipGetLastError());
    PP_TRY(launch_scan_i32_to_i64(w.icount.as<int32_t>(), w.ioff.as<int64_t>(), cb, w.scan_ws, s, sizes));
    PP_TRY(w.iblock.reserve(sizeof(int32_t) * (w.cap_item + 1)));
    PP_TRY(w.is0.reserve(sizeof(int32_t) * (w.cap_item + 1)));
    hipLaunchKernelGGL(item_fill_kernel, dim3(blocks_for(cb, 256)), dim3(256), 0, s,
                       w.icount.as<int32_t>(), w.ioff.as<int64_t>(), (const int64_t*)sizes, w.cap_item,
                       w.iblock.as<int32_t>(), w.is0.as<int32_t>());
    hipLaunchKernelGGL(finish_sizes_kernel, dim3(1), dim3(1), 0, s, sizes, w.ioff.as<int64_t>(),
                       w.roff.as<int64_t>(), w.cap_item, w.cap_range, w.bad.as<int>());
    PP_HIP(hipGetLastError());
    return PP_OK;
}

int lists_to_host(Work& w, hipStream_t s, bool* regrow, bool* moved) {
    *regrow = false;
    if (moved) *moved = false;
    PP_TRY(w.sizes_h.reserve(sizeof(int64_t) * kSizeSlots));
    int64_t* h = w.sizes_h.as<int64_t>();
    PP_HIP(hipMemcpyAsync(h, w.sizes.p, sizeof(int64_t) * kSizeSlots, hipMemcpyDeviceToHost, s));
    PP_HIP(hipStreamSynchronize(s));
    if (h[kBad]) return fail(PP_EINVAL, "non-finite position or mass");
    if (h[kMoved]) {                    // reused lists no longer cover every pair: rebuild
        if (moved) *moved = true;
        *regrow = true;
        return PP_OK;
    }
    if (h[kOverflow] & 64) return fail(PP_EDEVICE, "the list builder's single-pass scan did not complete");
    if (h[kOverflow] & 16) return fail(PP_ERANGE, "a target block lists more than 2^31 sources");
    if (h[kOverflow]) {
        w.cap_block = grow_cap(w.cap_block, h[kNeedBlock]);
        int np = w.npass;
        if (!w.stop_at_level2 && np >= 2 && h[kNeedEntry0 + np - 1] > kEntryBudget) {
            // the level-1 pass would be too large: stop at level 2 from now on
            w.stop_at_level2 = true;
            np -= 1;
        }
        for (int p = 0; p < np; ++p) w.cap_ent[p] = grow_cap(w.cap_ent[p], h[kNeedEntry0 + p]);
        w.cap_range = grow_cap(w.cap_range, h[kNeedRange]);
        w.cap_item = grow_cap(w.cap_item, h[kNeedItem]);
        *regrow = true;
        return PP_OK;
    }
    // capacities follow the needs (the buffers keep their size): scans and
    // grids then span little more than the data
    w.cap_block = settle_cap(w.cap_block, h[kNeedBlock]);
    for (int p = 0; p < w.npass; ++p) w.cap_ent[p] = settle_cap(w.cap_ent[p], h[kNeedEntry0 + p]);
    w.cap_range = settle_cap(w.cap_range, h[kNeedRange]);
    // the item count follows the active flags of each call: only a call
    // over every target brings the item capacity down
    if (!w.active) w.cap_item = settle_cap(w.cap_item, h[kNeedItem]);
    w.nleaf = h[kNLeaf];
    w.nblock = h[kNBlock];
    w.nentry = h[kNEntry];
    w.nrange = h[kNRange];
    w.nitem = h[kNItem];
    w.candidates = h[kCand];
    w.total_src = h[kTotalSrc];
    w.chunk = (int)h[kChunk];
    return PP_OK;
}

}  // namespace pp
