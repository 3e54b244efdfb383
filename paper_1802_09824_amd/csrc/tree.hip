// Octree leaves, the implicit tree over them, and the near-leaf lists.
//
// Leaves (sec. 3.2-3.3): with particles in Peano-Hilbert key order every
// octree node (the particles sharing the top 3l key bits) is a contiguous
// run.  A leaf is a maximal node holding at most M = leaf_max particles
// ("a leaf is a package of a given number of particles", sec. 3.3).  The
// level of the leaf of particle k is found without building the tree: the
// level-l node of k holds more than M particles iff some run of M + 1
// consecutive particles containing k shares its top 3l key bits, so
//   level(k) = 1 + max over s in [k - M, k] of lcp(key[s], key[s + M])
// (lcp in 3-bit digits, capped at b; 0 when no such run exists).  The
// sliding maximum uses the van Herk / Gil-Werman block prefix/suffix maxima.
//
// Near lists (sec. 3.3, the N-to-M leaf pairs of the dual tree traversal,
// restricted to the short range): an implicit 8-ary tree over the leaf
// array (leaves are in key order, so consecutive leaves are close in space)
// is walked depth-first without a stack, pruning subtrees whose integer
// bounding box is at least r_cut away.  The leaf test is exact integer
// arithmetic, identical for the canonical list and for the block lists.
#include "pp_internal.h"

namespace pp {
namespace {

inline unsigned blocks_for(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

#pragma clang fp contract(off)
// Grid cell of one coordinate: wrap into [0, L) as x - L floor(x / L) (an
// identity for already wrapped values), then floor(w 2^b / L) clamped, each
// operation rounded on its own exactly as in the key kernel.
__device__ __forceinline__ uint32_t quantise_w(double x, double L, double scale, uint32_t qmax) {
    double w = x - L * floor(x / L);
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

// lamp[s + M] = lcp(key[s], key[s + M]) for 0 <= s < n - M, else -1.
__global__ void lam_kernel(const uint64_t* __restrict__ keys, int64_t n, int M, int bits,
                           int8_t* __restrict__ lamp) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n + M) return;
    int64_t s = t - M;
    int8_t v = -1;
    if (s >= 0 && s + M < n) v = (int8_t)common_digits(keys[s], keys[s + M], bits);
    lamp[t] = v;
}

// Block prefix and suffix maxima over blocks of W = M + 1 entries.
__global__ void vhgw_kernel(const int8_t* __restrict__ a, int64_t len, int W,
                            int8_t* __restrict__ pmax, int8_t* __restrict__ smax) {
    int64_t blk = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t b0 = blk * W;
    if (b0 >= len) return;
    int64_t b1 = b0 + W < len ? b0 + W : len;
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
                             int64_t n, int M, int bits, int8_t* __restrict__ lev) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    // window of lamp indices [k, k + M]
    int8_t a = smax[k], b = pmax[k + M];
    int m = a > b ? a : b;
    lev[k] = (int8_t)(m < 0 ? 0 : (m + 1 < bits ? m + 1 : bits));
}

__global__ void flag_kernel(const uint64_t* __restrict__ keys, const int8_t* __restrict__ lev,
                            int64_t n, int bits, int32_t* __restrict__ flag) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    int f = 1;
    if (k > 0) {
        int l = lev[k - 1];
        f = key_prefix(keys[k], l, bits) != key_prefix(keys[k - 1], l, bits);
    }
    flag[k] = f;
}

__global__ void leaf_fill_kernel(const uint64_t* __restrict__ keys, const int8_t* __restrict__ lev,
                                 const int32_t* __restrict__ flag, const int64_t* __restrict__ off,
                                 int64_t n, int bits, int64_t* __restrict__ begin,
                                 int32_t* __restrict__ level, uint64_t* __restrict__ prefix) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n || !flag[k]) return;
    int64_t a = off[k];
    begin[a] = k;
    level[a] = lev[k];
    prefix[a] = key_prefix(keys[k], lev[k], bits);
}

__global__ void leaf_box_kernel(const double* __restrict__ pos_s, int64_t n,
                                const int64_t* __restrict__ begin, int64_t m, double L, double scale,
                                uint32_t qmax, int32_t* __restrict__ count,
                                IBox* __restrict__ box) {
    int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= m) return;
    int64_t b0 = begin[a], b1 = a + 1 < m ? begin[a + 1] : n;
    count[a] = (int32_t)(b1 - b0);
    IBox B;
    for (int ax = 0; ax < 3; ++ax) {
        uint32_t lo = 0xffffffffu, hi = 0;
        for (int64_t k = b0; k < b1; ++k) {
            uint32_t q = quantise_w(pos_s[ax * n + k], L, scale, qmax);
            lo = q < lo ? q : lo;
            hi = q > hi ? q : hi;
        }
        B.lo[ax] = (int32_t)lo;
        B.hi[ax] = (int32_t)hi + 1;
    }
    box[a] = B;
}

__global__ void tree_level_kernel(const IBox* __restrict__ child, int64_t nchild,
                                  IBox* __restrict__ parent, int64_t nparent) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nparent) return;
    IBox P = child[8 * i];
    int64_t e = 8 * i + 8 < nchild ? 8 * i + 8 : nchild;
    for (int64_t c = 8 * i + 1; c < e; ++c) {
        IBox C = child[c];
        for (int ax = 0; ax < 3; ++ax) {
            P.lo[ax] = C.lo[ax] < P.lo[ax] ? C.lo[ax] : P.lo[ax];
            P.hi[ax] = C.hi[ax] > P.hi[ax] ? C.hi[ax] : P.hi[ax];
        }
    }
    parent[i] = P;
}

// ------------------------------------------------------------ traversal --
// Gap along one axis between target [loA, hiA) and source [loB, hiB)
// shifted by s * W (grid units).
__device__ __forceinline__ int64_t axis_gap(int64_t loA, int64_t hiA, int64_t loB, int64_t hiB,
                                            int s, int64_t W) {
    int64_t sh = (int64_t)s * W;
    int64_t g1 = loB + sh - hiA, g2 = loA - hiB - sh;
    int64_t g = g1 > g2 ? g1 : g2;
    return g > 0 ? g : 0;
}

__device__ __forceinline__ int64_t gap2_shift(const IBox& A, const IBox& B, const int s[3],
                                              int64_t W) {
    int64_t r = 0;
    for (int ax = 0; ax < 3; ++ax) {
        int64_t g = axis_gap(A.lo[ax], A.hi[ax], B.lo[ax], B.hi[ax], s[ax], W);
        r += g * g;
    }
    return r;
}

// Allowed shifts per axis: bit 0 -> -1, bit 1 -> 0, bit 2 -> +1.
__device__ __forceinline__ void allowed_shifts(const IBox& A, int64_t W, int64_t T, int mask[3]) {
    for (int ax = 0; ax < 3; ++ax) {
        int64_t lo = A.lo[ax], up = W - A.hi[ax];
        mask[ax] = 2 | (lo * lo < T ? 1 : 0) | (up * up < T ? 4 : 0);
    }
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
            int64_t g = axis_gap(A.lo[ax], A.hi[ax], B.lo[ax], B.hi[ax], s, W);
            best = g < best ? g : best;
        }
        r += best * best;
    }
    return r;
}

// Depth-first walk of the implicit tree in ascending leaf order.  test(B)
// decides whether to descend into / visit node box B; visit(leaf) is called
// for every leaf that passes.
template <class Test, class Visit>
__device__ void walk(const TreeView& tv, Test&& test, Visit&& visit) {
    int h = tv.nlev - 1;
    int64_t i = 0;
    for (;;) {
        bool pass = test(tv.box[tv.off[h] + i]);
        if (pass && h == 0) visit(i);
        if (pass && h > 0) {
            h -= 1;
            i *= 8;
            continue;
        }
        for (;;) {
            if (h == tv.nlev - 1) return;
            int64_t nx = i + 1;
            if ((nx & 7) != 0 && nx < tv.cnt[h]) {
                i = nx;
                break;
            }
            i >>= 3;
            h += 1;
        }
    }
}

// Canonical list: one thread per target leaf, all shifts in one walk, leaf
// entries emitted in ascending (source, code) order.
template <bool FILL>
__global__ void canon_kernel(TreeView tv, int64_t nleaf, int64_t W, int64_t T,
                             int32_t* __restrict__ cnt, const int64_t* __restrict__ off,
                             int32_t* __restrict__ src, uint8_t* __restrict__ code) {
    int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= nleaf) return;
    const IBox A = tv.box[tv.off[0] + a];
    int mask[3];
    allowed_shifts(A, W, T, mask);
    int64_t k = FILL ? off[a] : 0;
    int32_t c = 0;
    walk(
        tv, [&](const IBox& B) { return gap2_min(A, B, mask, W) < T; },
        [&](int64_t b) {
            const IBox B = tv.box[tv.off[0] + b];
            for (int sc = 0; sc < 27; ++sc) {
                int s[3] = {sc / 9 - 1, (sc / 3) % 3 - 1, sc % 3 - 1};
                if (!(mask[0] >> (s[0] + 1) & 1) || !(mask[1] >> (s[1] + 1) & 1) ||
                    !(mask[2] >> (s[2] + 1) & 1))
                    continue;
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

__global__ void block_box_kernel(const double* __restrict__ pos_s, int64_t n, int64_t nblock,
                                 double L, double scale, uint32_t qmax, IBox* __restrict__ box) {
    int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nblock) return;
    int64_t k0 = b * kBlock, k1 = k0 + kBlock < n ? k0 + kBlock : n;
    IBox B;
    for (int ax = 0; ax < 3; ++ax) {
        uint32_t lo = 0xffffffffu, hi = 0;
        for (int64_t k = k0; k < k1; ++k) {
            uint32_t q = quantise_w(pos_s[ax * n + k], L, scale, qmax);
            lo = q < lo ? q : lo;
            hi = q > hi ? q : hi;
        }
        B.lo[ax] = (int32_t)lo;
        B.hi[ax] = (int32_t)hi + 1;
    }
    box[b] = B;
}

// Block lists: one thread per target block; one walk per allowed shift (in
// code order); consecutive leaves passing under the same shift merge into
// one range of source particles.
template <bool FILL>
__global__ void ranges_kernel(TreeView tv, const IBox* __restrict__ bbox, int64_t nblock,
                              const int64_t* __restrict__ leaf_begin,
                              const int32_t* __restrict__ leaf_count, int64_t W, int64_t T,
                              int32_t* __restrict__ rcount, int32_t* __restrict__ slen,
                              const int64_t* __restrict__ roff, int32_t* __restrict__ rbeg,
                              int32_t* __restrict__ rpre, uint8_t* __restrict__ rcode) {
    int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nblock) return;
    const IBox A = bbox[b];
    int mask[3];
    allowed_shifts(A, W, T, mask);
    int64_t k = FILL ? roff[b] : 0;
    int32_t nr = 0;
    int64_t tot = 0;
    for (int sc = 0; sc < 27; ++sc) {
        int s[3] = {sc / 9 - 1, (sc / 3) % 3 - 1, sc % 3 - 1};
        if (!(mask[0] >> (s[0] + 1) & 1) || !(mask[1] >> (s[1] + 1) & 1) ||
            !(mask[2] >> (s[2] + 1) & 1))
            continue;
        int64_t run0 = -1, run1 = -1;     // current run of leaves [run0, run1]
        auto flush = [&]() {
            if (run0 < 0) return;
            int64_t p0 = leaf_begin[run0];
            int64_t p1 = leaf_begin[run1] + leaf_count[run1];
            if (FILL) {
                rbeg[k] = (int32_t)p0;
                rpre[k] = (int32_t)tot;
                rcode[k] = (uint8_t)sc;
                ++k;
            }
            ++nr;
            tot += p1 - p0;
        };
        walk(
            tv, [&](const IBox& B) { return gap2_shift(A, B, s, W) < T; },
            [&](int64_t leaf) {
                if (run0 >= 0 && leaf == run1 + 1) {
                    run1 = leaf;
                } else {
                    flush();
                    run0 = run1 = leaf;
                }
            });
        flush();
    }
    if (!FILL) {
        rcount[b] = nr;
        slen[b] = (int32_t)(tot < INT32_MAX ? tot : INT32_MAX);
    }
}

__global__ void item_count_kernel(const int32_t* __restrict__ slen, int64_t nblock, int chunk,
                                  int32_t* __restrict__ icount,
                                  unsigned long long* __restrict__ cand) {
    int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nblock) return;
    int32_t s = slen[b];
    icount[b] = s <= 0 ? 1 : (s + chunk - 1) / chunk;
    atomicAdd(cand, (unsigned long long)s);
}

__global__ void item_fill_kernel(const int32_t* __restrict__ icount,
                                 const int64_t* __restrict__ ioff, int64_t nblock, int chunk,
                                 int32_t* __restrict__ iblock, int32_t* __restrict__ is0) {
    int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nblock) return;
    int64_t o = ioff[b];
    for (int32_t c = 0; c < icount[b]; ++c) {
        iblock[o + c] = (int32_t)b;
        is0[o + c] = c * chunk;
    }
}

template <class T>
int read_back(const T* dev, T* host, hipStream_t s) {
    PP_HIP(hipMemcpyAsync(host, dev, sizeof(T), hipMemcpyDeviceToHost, s));
    PP_HIP(hipStreamSynchronize(s));
    return PP_OK;
}

}  // namespace

int build_leaves_device(const uint64_t* sorted_keys, const double* pos_s, int64_t n, const Geo& g,
                        int leaf_max, LeafBuffers& lb, void* scan_ws, size_t scan_ws_bytes,
                        DevBuf& begin, DevBuf& count, DevBuf& level, DevBuf& prefix, DevBuf& boxes,
                        int64_t* nleaf_out, hipStream_t s) {
    *nleaf_out = 0;
    if (n == 0) return PP_OK;
    const int M = leaf_max;
    const int64_t len = n + M;
    hipLaunchKernelGGL(lam_kernel, dim3(blocks_for(len, 256)), dim3(256), 0, s, sorted_keys, n, M,
                       g.bits, lb.lam);
    const int64_t nblk = (len + M) / (M + 1);
    hipLaunchKernelGGL(vhgw_kernel, dim3(blocks_for(nblk, 256)), dim3(256), 0, s, lb.lam, len,
                       M + 1, lb.pmax, lb.smax);
    hipLaunchKernelGGL(level_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, lb.pmax, lb.smax,
                       n, M, g.bits, lb.level_p);
    hipLaunchKernelGGL(flag_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, sorted_keys,
                       lb.level_p, n, g.bits, lb.flag);
    PP_HIP(hipGetLastError());
    PP_TRY(launch_scan_i32_to_i64(lb.flag, lb.flag_off, n, scan_ws, scan_ws_bytes, s));
    int64_t m = 0;
    PP_TRY(read_back(lb.flag_off + n, &m, s));
    PP_TRY(begin.reserve(sizeof(int64_t) * (m + 1)));
    PP_TRY(count.reserve(sizeof(int32_t) * (m + 1)));
    PP_TRY(level.reserve(sizeof(int32_t) * (m + 1)));
    PP_TRY(prefix.reserve(sizeof(uint64_t) * (m + 1)));
    PP_TRY(boxes.reserve(sizeof(IBox) * (m + 1)));
    hipLaunchKernelGGL(leaf_fill_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, sorted_keys,
                       lb.level_p, lb.flag, lb.flag_off, n, g.bits, begin.as<int64_t>(),
                       level.as<int32_t>(), prefix.as<uint64_t>());
    hipLaunchKernelGGL(leaf_box_kernel, dim3(blocks_for(m, 128)), dim3(128), 0, s, pos_s, n,
                       begin.as<int64_t>(), m, g.L, g.qscale, (uint32_t)(g.W - 1), count.as<int32_t>(),
                       boxes.as<IBox>());
    PP_HIP(hipGetLastError());
    *nleaf_out = m;
    return PP_OK;
}

int build_tree(const IBox* leaf_boxes, int64_t nleaf, DevBuf& tree_boxes, TreeView* tv,
               hipStream_t s) {
    // level sizes
    int64_t cnt[kTreeMaxLevels], off[kTreeMaxLevels];
    int nlev = 0;
    int64_t c = nleaf, total = 0;
    for (;;) {
        if (nlev >= kTreeMaxLevels) return fail(PP_ERANGE, "tree too deep");
        cnt[nlev] = c;
        off[nlev] = total;
        total += c;
        ++nlev;
        if (c <= 1) break;
        c = (c + 7) / 8;
    }
    PP_TRY(tree_boxes.reserve(sizeof(IBox) * (total > 0 ? total : 1)));
    IBox* tb = tree_boxes.as<IBox>();
    if (nleaf > 0)
        PP_HIP(hipMemcpyAsync(tb, leaf_boxes, sizeof(IBox) * nleaf, hipMemcpyDeviceToDevice, s));
    for (int h = 1; h < nlev; ++h) {
        hipLaunchKernelGGL(tree_level_kernel, dim3(blocks_for(cnt[h], 256)), dim3(256), 0, s,
                           tb + off[h - 1], cnt[h - 1], tb + off[h], cnt[h]);
    }
    PP_HIP(hipGetLastError());
    tv->box = tb;
    tv->nlev = nlev;
    for (int h = 0; h < kTreeMaxLevels; ++h) {
        tv->cnt[h] = h < nlev ? cnt[h] : 0;
        tv->off[h] = h < nlev ? off[h] : 0;
    }
    return PP_OK;
}

int build_canonical_pairs(const TreeView& tv, int64_t nleaf, const Geo& g, DevBuf& row_cnt,
                          DevBuf& row_ptr, DevBuf& src, DevBuf& code, void* scan_ws,
                          size_t scan_ws_bytes, int64_t* nentries, hipStream_t s) {
    PP_TRY(row_cnt.reserve(sizeof(int32_t) * (nleaf + 1)));
    PP_TRY(row_ptr.reserve(sizeof(int64_t) * (nleaf + 1)));
    *nentries = 0;
    if (nleaf == 0) {
        int64_t z = 0;
        PP_HIP(hipMemcpyAsync(row_ptr.p, &z, sizeof(z), hipMemcpyHostToDevice, s));
        PP_HIP(hipStreamSynchronize(s));
        return PP_OK;
    }
    hipLaunchKernelGGL(canon_kernel<false>, dim3(blocks_for(nleaf, 64)), dim3(64), 0, s, tv,
                       nleaf, g.W, g.T, row_cnt.as<int32_t>(), (const int64_t*)nullptr,
                       (int32_t*)nullptr, (uint8_t*)nullptr);
    PP_HIP(hipGetLastError());
    PP_TRY(launch_scan_i32_to_i64(row_cnt.as<int32_t>(), row_ptr.as<int64_t>(), nleaf, scan_ws,
                                  scan_ws_bytes, s));
    int64_t tot = 0;
    PP_TRY(read_back(row_ptr.as<int64_t>() + nleaf, &tot, s));
    PP_TRY(src.reserve(sizeof(int32_t) * (tot + 1)));
    PP_TRY(code.reserve(sizeof(uint8_t) * (tot + 1)));
    hipLaunchKernelGGL(canon_kernel<true>, dim3(blocks_for(nleaf, 64)), dim3(64), 0, s, tv, nleaf,
                       g.W, g.T, (int32_t*)nullptr, row_ptr.as<int64_t>(), src.as<int32_t>(),
                       code.as<uint8_t>());
    PP_HIP(hipGetLastError());
    *nentries = tot;
    return PP_OK;
}

int build_block_lists(const double* pos_s, int64_t n, const int64_t* leaf_begin,
                      const int32_t* leaf_count, const TreeView& tv, int64_t nleaf, const Geo& g,
                      int chunk, BlockLists& bl, void* scan_ws, size_t scan_ws_bytes,
                      hipStream_t s) {
    const int64_t nb = (n + kBlock - 1) / kBlock;
    bl.nblock = nb;
    bl.nrange = bl.nitem = bl.candidates = 0;
    if (nb == 0) return PP_OK;
    PP_TRY(bl.box.reserve(sizeof(IBox) * nb));
    PP_TRY(bl.rcount.reserve(sizeof(int32_t) * nb));
    PP_TRY(bl.slen.reserve(sizeof(int32_t) * nb));
    PP_TRY(bl.roff.reserve(sizeof(int64_t) * (nb + 1)));
    PP_TRY(bl.icount.reserve(sizeof(int32_t) * nb));
    PP_TRY(bl.ioff.reserve(sizeof(int64_t) * (nb + 1) + sizeof(unsigned long long)));
    hipLaunchKernelGGL(block_box_kernel, dim3(blocks_for(nb, 128)), dim3(128), 0, s, pos_s, n, nb,
                       g.L, g.qscale, (uint32_t)(g.W - 1), bl.box.as<IBox>());
    hipLaunchKernelGGL(ranges_kernel<false>, dim3(blocks_for(nb, 64)), dim3(64), 0, s, tv,
                       bl.box.as<IBox>(), nb, leaf_begin, leaf_count, g.W, g.T,
                       bl.rcount.as<int32_t>(), bl.slen.as<int32_t>(), (const int64_t*)nullptr,
                       (int32_t*)nullptr, (int32_t*)nullptr, (uint8_t*)nullptr);
    PP_HIP(hipGetLastError());
    PP_TRY(launch_scan_i32_to_i64(bl.rcount.as<int32_t>(), bl.roff.as<int64_t>(), nb, scan_ws,
                                  scan_ws_bytes, s));
    // items per block (and the candidate total) while the range count is read
    unsigned long long* cand = reinterpret_cast<unsigned long long*>(bl.ioff.as<int64_t>() + nb + 1);
    PP_HIP(hipMemsetAsync(cand, 0, sizeof(unsigned long long), s));
    hipLaunchKernelGGL(item_count_kernel, dim3(blocks_for(nb, 256)), dim3(256), 0, s,
                       bl.slen.as<int32_t>(), nb, chunk, bl.icount.as<int32_t>(), cand);
    PP_HIP(hipGetLastError());
    PP_TRY(launch_scan_i32_to_i64(bl.icount.as<int32_t>(), bl.ioff.as<int64_t>(), nb, scan_ws,
                                  scan_ws_bytes, s));
    int64_t hostv[2];
    unsigned long long hc = 0;
    PP_HIP(hipMemcpyAsync(&hostv[0], bl.roff.as<int64_t>() + nb, sizeof(int64_t),
                          hipMemcpyDeviceToHost, s));
    PP_HIP(hipMemcpyAsync(&hostv[1], bl.ioff.as<int64_t>() + nb, sizeof(int64_t),
                          hipMemcpyDeviceToHost, s));
    PP_HIP(hipMemcpyAsync(&hc, cand, sizeof(hc), hipMemcpyDeviceToHost, s));
    PP_HIP(hipStreamSynchronize(s));
    bl.nrange = hostv[0];
    bl.nitem = hostv[1];
    bl.candidates = (int64_t)hc * kBlock;
    PP_TRY(bl.rbeg.reserve(sizeof(int32_t) * (bl.nrange + 1)));
    PP_TRY(bl.rpre.reserve(sizeof(int32_t) * (bl.nrange + 1)));
    PP_TRY(bl.rcode.reserve(sizeof(uint8_t) * (bl.nrange + 1)));
    PP_TRY(bl.iblock.reserve(sizeof(int32_t) * (bl.nitem + 1)));
    PP_TRY(bl.is0.reserve(sizeof(int32_t) * (bl.nitem + 1)));
    hipLaunchKernelGGL(ranges_kernel<true>, dim3(blocks_for(nb, 64)), dim3(64), 0, s, tv,
                       bl.box.as<IBox>(), nb, leaf_begin, leaf_count, g.W, g.T, (int32_t*)nullptr,
                       (int32_t*)nullptr, bl.roff.as<int64_t>(), bl.rbeg.as<int32_t>(),
                       bl.rpre.as<int32_t>(), bl.rcode.as<uint8_t>());
    hipLaunchKernelGGL(item_fill_kernel, dim3(blocks_for(nb, 256)), dim3(256), 0, s,
                       bl.icount.as<int32_t>(), bl.ioff.as<int64_t>(), nb, chunk,
                       bl.iblock.as<int32_t>(), bl.is0.as<int32_t>());
    PP_HIP(hipGetLastError());
    return PP_OK;
}

}  // namespace pp
