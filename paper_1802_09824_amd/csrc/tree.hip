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

template <class T>
int read_back(const T* dev, T* host, hipStream_t s) {
    PP_HIP(hipMemcpyAsync(host, dev, sizeof(T), hipMemcpyDeviceToHost, s));
    PP_HIP(hipStreamSynchronize(s));
    return PP_OK;
}

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

// Target blocks: one thread per chunk of kBlock consecutive particles walks
// the chunk and starts a new block whenever adding the next particle would
// make the bounding box wider than emax grid units along some axis.
template <bool FILL>
__global__ void block_split_kernel(const double* __restrict__ pos_s, int64_t n, int64_t nchunk,
                                   double L, double scale, uint32_t qmax, int64_t emax,
                                   int32_t* __restrict__ ccount, const int64_t* __restrict__ coff,
                                   int32_t* __restrict__ bstart, int32_t* __restrict__ bcount,
                                   IBox* __restrict__ box) {
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nchunk) return;
    const int64_t k0 = c * kBlock, k1 = k0 + kBlock < n ? k0 + kBlock : n;
    int64_t o = FILL ? coff[c] : 0;
    int32_t nb = 0;
    int64_t start = k0;
    IBox B;
    for (int64_t k = k0; k < k1; ++k) {
        int32_t q[3];
        for (int ax = 0; ax < 3; ++ax) q[ax] = (int32_t)quantise_w(pos_s[ax * n + k], L, scale, qmax);
        if (k == start) {
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
            wide |= (int64_t)(U.hi[ax] - U.lo[ax]) > emax;
        }
        if (wide) {
            if (FILL) {
                bstart[o + nb] = (int32_t)start;
                bcount[o + nb] = (int32_t)(k - start);
                box[o + nb] = B;
            }
            ++nb;
            start = k;
            for (int ax = 0; ax < 3; ++ax) {
                B.lo[ax] = q[ax];
                B.hi[ax] = q[ax] + 1;
            }
        } else {
            B = U;
        }
    }
    if (FILL) {
        bstart[o + nb] = (int32_t)start;
        bcount[o + nb] = (int32_t)(k1 - start);
        box[o + nb] = B;
    }
    ++nb;
    if (!FILL) ccount[c] = nb;
}

// Block lists.  A node passes for target box A under shift s when its box
// is closer than r_cut (gap^2 < T); it is *inside* when even its farthest
// point is (maxdist^2 < T), and then every leaf under it passes, so the
// node's whole leaf interval is listed without descending.  The walk is
// level-synchronous from the root down to the DFS level hd over all
// (block, shift, node) entries at once (one thread per entry, children
// written in order so entries stay sorted by block, shift, node), then one
// thread per entry walks its small subtree depth-first, testing the 8
// children of a node at once.  Leaves (or inside intervals) are visited in
// ascending order and consecutive ones merge into one range of source
// particles.
struct FEntry {
    int32_t blk;
    int32_t node;
    uint8_t sc;      // shift code
    uint8_t lev;     // tree level of node
    uint8_t inside;  // whole subtree within r_cut
    uint8_t pad;
};

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

__device__ __forceinline__ void decode_shift(int sc, int s[3]) {
    s[0] = sc / 9 - 1;
    s[1] = (sc / 3) % 3 - 1;
    s[2] = sc % 3 - 1;
}

// Test the children of (h, i): pass bits and inside bits (inside implies pass).
__device__ __forceinline__ void expand2(const TreeView& tv, int h, int64_t i, const IBox& A,
                                        const int s[3], int64_t W, int64_t T, uint32_t& pass,
                                        uint32_t& inside) {
    const int64_t c0 = 8 * i, nc = tv.cnt[h - 1];
    const IBox* base = tv.box + tv.off[h - 1];
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
__global__ void bfs_root_kernel(TreeView tv, const IBox* __restrict__ bbox, int64_t nb, int64_t W,
                                int64_t T, int32_t* __restrict__ cnt, const int64_t* __restrict__ off,
                                FEntry* __restrict__ out) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb) return;
    const IBox A = bbox[b];
    int mask[3];
    allowed_shifts(A, W, T, mask);
    const int top = tv.nlev - 1;
    const IBox R = tv.box[tv.off[top]];
    int64_t o = FILL ? off[b] : 0;
    int32_t c = 0;
    for (int sc = 0; sc < 27; ++sc) {
        int s[3];
        decode_shift(sc, s);
        if (!(mask[0] >> (s[0] + 1) & 1) || !(mask[1] >> (s[1] + 1) & 1) ||
            !(mask[2] >> (s[2] + 1) & 1))
            continue;
        if (!(gap2_shift(A, R, s, W) < T)) continue;
        if (FILL) {
            FEntry e;
            e.blk = (int32_t)b;
            e.node = 0;
            e.sc = (uint8_t)sc;
            e.lev = (uint8_t)top;
            e.inside = maxd2_shift(A, R, s, W) < T;
            e.pad = 0;
            out[o++] = e;
        } else {
            ++c;
        }
    }
    if (!FILL) cnt[b] = c;
}

// One level down: entries at level > hd that are not inside are replaced by
// their passing children; the others are carried unchanged.
template <bool FILL>
__global__ void bfs_level_kernel(TreeView tv, int hd, const IBox* __restrict__ bbox,
                                 const FEntry* __restrict__ in, int64_t F, int64_t W, int64_t T,
                                 int32_t* __restrict__ cnt, const int64_t* __restrict__ off,
                                 FEntry* __restrict__ out) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= F) return;
    const FEntry E = in[e];
    if (E.inside || E.lev <= hd) {
        if (FILL) out[off[e]] = E;
        else cnt[e] = 1;
        return;
    }
    int s[3];
    decode_shift(E.sc, s);
    uint32_t pass, inside;
    expand2(tv, E.lev, E.node, bbox[E.blk], s, W, T, pass, inside);
    if (!FILL) {
        cnt[e] = __popc(pass);
        return;
    }
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
        C.pad = 0;
        out[o++] = C;
    }
}

// Depth-first walk of one entry's subtree (at most 8^hd <= 64 leaves).  The
// count pass records which leaves of the subtree pass as a 64-bit mask
// (bit = leaf - first leaf of the subtree); the fill pass turns the mask
// back into runs without testing boxes again.  Inside entries and leaf
// entries are a single run and need no mask.
template <bool FILL>
__global__ void ranges_kernel(TreeView tv, const FEntry* __restrict__ ent, int64_t F,
                              const IBox* __restrict__ bbox, const int64_t* __restrict__ leaf_begin,
                              const int32_t* __restrict__ leaf_count, int64_t nleaf, int64_t W,
                              int64_t T, uint64_t* __restrict__ lmask, int32_t* __restrict__ rcnt,
                              int32_t* __restrict__ scnt, const int64_t* __restrict__ roff,
                              const int64_t* __restrict__ soff, const int64_t* __restrict__ eoff,
                              int32_t* __restrict__ rbeg, int32_t* __restrict__ rpre,
                              uint8_t* __restrict__ rcode) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= F) return;
    const FEntry E = ent[e];
    int64_t o = FILL ? roff[e] : 0;
    int64_t pos = FILL ? soff[e] - soff[eoff[E.blk]] : 0;
    int32_t nr = 0;
    int64_t tot = 0;
    // one run of leaves [l0, l1]
    auto emit = [&](int64_t l0, int64_t l1) {
        const int64_t p0 = leaf_begin[l0];
        const int64_t p1 = leaf_begin[l1] + leaf_count[l1];
        if (FILL) {
            rbeg[o] = (int32_t)p0;
            rpre[o] = (int32_t)pos;
            rcode[o] = E.sc;
            ++o;
        }
        ++nr;
        pos += p1 - p0;
        tot += p1 - p0;
    };
    const int64_t first = (int64_t)E.node << (3 * E.lev);
    int64_t last = (((int64_t)E.node + 1) << (3 * E.lev)) - 1;
    if (last > nleaf - 1) last = nleaf - 1;
    if (E.inside || E.lev == 0) {
        emit(first, last);
    } else {
        uint64_t mask = 0;
        if (FILL) {
            mask = lmask[e];
        } else {
            const IBox A = bbox[E.blk];
            int s[3];
            decode_shift(E.sc, s);
            // 16 bits per level: low byte pending children, high byte inside children
            uint64_t st = 0;
            int lev = E.lev;
            int64_t node = E.node;
            uint32_t pa, in;
            expand2(tv, lev, node, A, s, W, T, pa, in);
            st |= (uint64_t)(pa | (in << 8)) << (16 * (lev & 3));
            for (;;) {
                const uint32_t w = (uint32_t)(st >> (16 * (lev & 3))) & 0xffffu;
                const uint32_t m = w & 0xffu;
                if (m == 0) {
                    if (lev == E.lev) break;
                    ++lev;
                    node >>= 3;
                    continue;
                }
                const int c = __builtin_ctz(m);
                const uint32_t w2 = w & ~(1u << c);
                st = (st & ~(0xffffull << (16 * (lev & 3)))) | ((uint64_t)w2 << (16 * (lev & 3)));
                const int64_t child = 8 * node + c;
                if (lev == 1 || ((w >> 8) >> c & 1u)) {
                    const int64_t l0 = child << (3 * (lev - 1));
                    int64_t l1 = ((child + 1) << (3 * (lev - 1))) - 1;
                    if (l1 > nleaf - 1) l1 = nleaf - 1;
                    for (int64_t l = l0; l <= l1; ++l) mask |= 1ull << (l - first);
                } else {
                    --lev;
                    node = child;
                    expand2(tv, lev, node, A, s, W, T, pa, in);
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
    if (!FILL) {
        rcnt[e] = nr;
        scnt[e] = (int32_t)(tot < INT32_MAX ? tot : INT32_MAX);
    }
}

// First entry of every block (entries are sorted by block), then per-block
// range offsets and list lengths; flags a list longer than int32.
__global__ void block_entry_kernel(const FEntry* __restrict__ ent, int64_t F, int64_t nblock,
                                   int64_t* __restrict__ eoff) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b > nblock) return;
    int64_t lo = 0, hi = F;             // first e with ent[e].blk >= b
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (ent[mid].blk < b) lo = mid + 1;
        else hi = mid;
    }
    eoff[b] = lo;
}

__global__ void block_sum_kernel(const int64_t* __restrict__ eoff, const int64_t* __restrict__ roff_e,
                                 const int64_t* __restrict__ soff_e, int64_t nblock,
                                 int64_t* __restrict__ roff, int32_t* __restrict__ slen,
                                 int* __restrict__ overflow) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b > nblock) return;
    roff[b] = roff_e[eoff[b]];
    if (b == nblock) return;
    const int64_t len = soff_e[eoff[b + 1]] - soff_e[eoff[b]];
    if (len > INT32_MAX) atomicOr(overflow, 1);
    slen[b] = (int32_t)(len < INT32_MAX ? len : INT32_MAX);
}

__global__ void item_count_kernel(const int32_t* __restrict__ slen,
                                  const int32_t* __restrict__ bcount, int64_t nblock, int chunk,
                                  int32_t* __restrict__ icount,
                                  unsigned long long* __restrict__ cand) {
    int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nblock) return;
    int32_t s = slen[b];
    icount[b] = s <= 0 ? 1 : (s + chunk - 1) / chunk;
    // (target, listed source) pairs; the kernel prunes some sources further
    atomicAdd(cand, (unsigned long long)s * (unsigned long long)bcount[b]);
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


// Make sure the scan scratch holds an n-element scan.
int grow_scan(DevBuf& buf, int64_t n, void*& ws, size_t& bytes) {
    size_t need = 0;
    PP_TRY(scan_workspace(n, &need));
    PP_TRY(buf.reserve(need + 1));
    ws = buf.p;
    bytes = buf.bytes;
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
                      int chunk, double rcut, BlockLists& bl, DevBuf& scan_buf, hipStream_t s) {
    const int64_t nc = (n + kBlock - 1) / kBlock;
    void* scan_ws = nullptr;
    size_t scan_ws_bytes = 0;
    PP_TRY(grow_scan(scan_buf, nc + 1, scan_ws, scan_ws_bytes));
    bl.nchunk = nc;
    bl.nblock = bl.nrange = bl.nitem = bl.candidates = 0;
    if (nc == 0) return PP_OK;
    const int64_t emax = (int64_t)floor(2.0 * rcut * (double)g.W / g.L);
    PP_TRY(bl.ccount.reserve(sizeof(int32_t) * nc));
    PP_TRY(bl.coff.reserve(sizeof(int64_t) * (nc + 1)));
    hipLaunchKernelGGL(block_split_kernel<false>, dim3(blocks_for(nc, 128)), dim3(128), 0, s, pos_s,
                       n, nc, g.L, g.qscale, (uint32_t)(g.W - 1), emax, bl.ccount.as<int32_t>(),
                       (const int64_t*)nullptr, (int32_t*)nullptr, (int32_t*)nullptr,
                       (IBox*)nullptr);
    PP_HIP(hipGetLastError());
    PP_TRY(launch_scan_i32_to_i64(bl.ccount.as<int32_t>(), bl.coff.as<int64_t>(), nc, scan_ws,
                                  scan_ws_bytes, s));
    int64_t nb = 0;
    PP_TRY(read_back(bl.coff.as<int64_t>() + nc, &nb, s));
    bl.nblock = nb;
    PP_TRY(bl.bstart.reserve(sizeof(int32_t) * nb));
    PP_TRY(bl.bcount.reserve(sizeof(int32_t) * nb));
    PP_TRY(bl.box.reserve(sizeof(IBox) * nb));
    PP_TRY(bl.slen.reserve(sizeof(int32_t) * nb));
    PP_TRY(bl.roff.reserve(sizeof(int64_t) * (nb + 1)));
    PP_TRY(bl.icount.reserve(sizeof(int32_t) * nb));
    PP_TRY(bl.ioff.reserve(sizeof(int64_t) * (nb + 1) + 2 * sizeof(unsigned long long)));
    hipLaunchKernelGGL(block_split_kernel<true>, dim3(blocks_for(nc, 128)), dim3(128), 0, s, pos_s,
                       n, nc, g.L, g.qscale, (uint32_t)(g.W - 1), emax, (int32_t*)nullptr,
                       bl.coff.as<int64_t>(), bl.bstart.as<int32_t>(), bl.bcount.as<int32_t>(),
                       bl.box.as<IBox>());
    // breadth-first from the root down to the DFS level hd
    const int hd = tv.nlev - 1 < 2 ? tv.nlev - 1 : 2;
    DevBuf* cur = &bl.fent_a;
    DevBuf* nxt = &bl.fent_b;
    int64_t F = 0;
    {
        PP_TRY(bl.fcnt.reserve(sizeof(int32_t) * (nb + 1)));
        PP_TRY(bl.foff.reserve(sizeof(int64_t) * (nb + 2)));
        hipLaunchKernelGGL(bfs_root_kernel<false>, dim3(blocks_for(nb, 128)), dim3(128), 0, s, tv,
                           bl.box.as<IBox>(), nb, g.W, g.T, bl.fcnt.as<int32_t>(),
                           (const int64_t*)nullptr, (FEntry*)nullptr);
        PP_HIP(hipGetLastError());
        PP_TRY(grow_scan(scan_buf, nb + 1, scan_ws, scan_ws_bytes));
        PP_TRY(launch_scan_i32_to_i64(bl.fcnt.as<int32_t>(), bl.foff.as<int64_t>(), nb, scan_ws,
                                      scan_ws_bytes, s));
        PP_TRY(read_back(bl.foff.as<int64_t>() + nb, &F, s));
        PP_TRY(cur->reserve(sizeof(FEntry) * (F + 1)));
        hipLaunchKernelGGL(bfs_root_kernel<true>, dim3(blocks_for(nb, 128)), dim3(128), 0, s, tv,
                           bl.box.as<IBox>(), nb, g.W, g.T, (int32_t*)nullptr,
                           bl.foff.as<int64_t>(), cur->as<FEntry>());
        PP_HIP(hipGetLastError());
    }
    for (int h = tv.nlev - 1; h > hd; --h) {
        PP_TRY(bl.fcnt.reserve(sizeof(int32_t) * (F + 1)));
        PP_TRY(bl.foff.reserve(sizeof(int64_t) * (F + 2)));
        hipLaunchKernelGGL(bfs_level_kernel<false>, dim3(blocks_for(F, 128)), dim3(128), 0, s, tv,
                           hd, bl.box.as<IBox>(), cur->as<FEntry>(), F, g.W, g.T,
                           bl.fcnt.as<int32_t>(), (const int64_t*)nullptr, (FEntry*)nullptr);
        PP_HIP(hipGetLastError());
        PP_TRY(grow_scan(scan_buf, F + 1, scan_ws, scan_ws_bytes));
        PP_TRY(launch_scan_i32_to_i64(bl.fcnt.as<int32_t>(), bl.foff.as<int64_t>(), F, scan_ws,
                                      scan_ws_bytes, s));
        int64_t F2 = 0;
        PP_TRY(read_back(bl.foff.as<int64_t>() + F, &F2, s));
        PP_TRY(nxt->reserve(sizeof(FEntry) * (F2 + 1)));
        hipLaunchKernelGGL(bfs_level_kernel<true>, dim3(blocks_for(F, 128)), dim3(128), 0, s, tv, hd,
                           bl.box.as<IBox>(), cur->as<FEntry>(), F, g.W, g.T, (int32_t*)nullptr,
                           bl.foff.as<int64_t>(), nxt->as<FEntry>());
        PP_HIP(hipGetLastError());
        DevBuf* t = cur;
        cur = nxt;
        nxt = t;
        F = F2;
    }
    bl.nentry = F;
    const FEntry* ent = cur->as<FEntry>();
    PP_TRY(bl.rcnt_e.reserve(sizeof(int32_t) * (F + 1)));
    PP_TRY(bl.scnt_e.reserve(sizeof(int32_t) * (F + 1)));
    PP_TRY(bl.roff_e.reserve(sizeof(int64_t) * (F + 2)));
    PP_TRY(bl.soff_e.reserve(sizeof(int64_t) * (F + 2)));
    PP_TRY(bl.eoff.reserve(sizeof(int64_t) * (nb + 2)));
    PP_TRY(bl.lmask_e.reserve(sizeof(uint64_t) * (F + 1)));
    hipLaunchKernelGGL(ranges_kernel<false>, dim3(blocks_for(F, 128)), dim3(128), 0, s, tv, ent, F,
                       bl.box.as<IBox>(), leaf_begin, leaf_count, nleaf, g.W, g.T,
                       bl.lmask_e.as<uint64_t>(), bl.rcnt_e.as<int32_t>(), bl.scnt_e.as<int32_t>(),
                       (const int64_t*)nullptr,
                       (const int64_t*)nullptr, (const int64_t*)nullptr, (int32_t*)nullptr,
                       (int32_t*)nullptr, (uint8_t*)nullptr);
    hipLaunchKernelGGL(block_entry_kernel, dim3(blocks_for(nb + 1, 256)), dim3(256), 0, s, ent, F,
                       nb, bl.eoff.as<int64_t>());
    PP_HIP(hipGetLastError());
    PP_TRY(grow_scan(scan_buf, F + 1, scan_ws, scan_ws_bytes));
    PP_TRY(launch_scan_i32_to_i64(bl.rcnt_e.as<int32_t>(), bl.roff_e.as<int64_t>(), F, scan_ws,
                                  scan_ws_bytes, s));
    PP_TRY(launch_scan_i32_to_i64(bl.scnt_e.as<int32_t>(), bl.soff_e.as<int64_t>(), F, scan_ws,
                                  scan_ws_bytes, s));
    unsigned long long* cand = reinterpret_cast<unsigned long long*>(bl.ioff.as<int64_t>() + nb + 1);
    int* ovf = reinterpret_cast<int*>(cand + 1);
    PP_HIP(hipMemsetAsync(cand, 0, 2 * sizeof(unsigned long long), s));
    hipLaunchKernelGGL(block_sum_kernel, dim3(blocks_for(nb + 1, 256)), dim3(256), 0, s,
                       bl.eoff.as<int64_t>(), bl.roff_e.as<int64_t>(), bl.soff_e.as<int64_t>(), nb,
                       bl.roff.as<int64_t>(), bl.slen.as<int32_t>(), ovf);
    // items per block (and the candidate total)
    hipLaunchKernelGGL(item_count_kernel, dim3(blocks_for(nb, 256)), dim3(256), 0, s,
                       bl.slen.as<int32_t>(), bl.bcount.as<int32_t>(), nb, chunk,
                       bl.icount.as<int32_t>(), cand);
    PP_HIP(hipGetLastError());
    PP_TRY(launch_scan_i32_to_i64(bl.icount.as<int32_t>(), bl.ioff.as<int64_t>(), nb, scan_ws,
                                  scan_ws_bytes, s));
    int64_t hostv[2];
    unsigned long long hc[2] = {0, 0};
    PP_HIP(hipMemcpyAsync(&hostv[0], bl.roff.as<int64_t>() + nb, sizeof(int64_t),
                          hipMemcpyDeviceToHost, s));
    PP_HIP(hipMemcpyAsync(&hostv[1], bl.ioff.as<int64_t>() + nb, sizeof(int64_t),
                          hipMemcpyDeviceToHost, s));
    PP_HIP(hipMemcpyAsync(hc, cand, sizeof(hc), hipMemcpyDeviceToHost, s));
    PP_HIP(hipStreamSynchronize(s));
    if (hc[1] & 0xffffffffull) return fail(PP_ERANGE, "a target block lists more than 2^31 sources");
    bl.nrange = hostv[0];
    bl.nitem = hostv[1];
    bl.candidates = (int64_t)hc[0];
    PP_TRY(bl.rbeg.reserve(sizeof(int32_t) * (bl.nrange + 1)));
    PP_TRY(bl.rpre.reserve(sizeof(int32_t) * (bl.nrange + 1)));
    PP_TRY(bl.rcode.reserve(sizeof(uint8_t) * (bl.nrange + 1)));
    PP_TRY(bl.iblock.reserve(sizeof(int32_t) * (bl.nitem + 1)));
    PP_TRY(bl.is0.reserve(sizeof(int32_t) * (bl.nitem + 1)));
    hipLaunchKernelGGL(ranges_kernel<true>, dim3(blocks_for(F, 128)), dim3(128), 0, s, tv, ent, F,
                       bl.box.as<IBox>(), leaf_begin, leaf_count, nleaf, g.W, g.T,
                       bl.lmask_e.as<uint64_t>(), (int32_t*)nullptr, (int32_t*)nullptr,
                       bl.roff_e.as<int64_t>(),
                       bl.soff_e.as<int64_t>(), bl.eoff.as<int64_t>(), bl.rbeg.as<int32_t>(),
                       bl.rpre.as<int32_t>(), bl.rcode.as<uint8_t>());
    hipLaunchKernelGGL(item_fill_kernel, dim3(blocks_for(nb, 256)), dim3(256), 0, s,
                       bl.icount.as<int32_t>(), bl.ioff.as<int64_t>(), nb, chunk,
                       bl.iblock.as<int32_t>(), bl.is0.as<int32_t>());
    PP_HIP(hipGetLastError());
    return PP_OK;
}

}  // namespace pp
