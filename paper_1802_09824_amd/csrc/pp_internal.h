// Internal declarations shared by the library's translation units.
// Nothing here is part of the C ABI (include/photon_pp.h is).
//
// Every stage works on a *batch*: nbox independent periodic boxes whose
// particles are concatenated (box x owns particles [poff[x], poff[x+1])).
// A single box is a batch of one.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "photon_pp.h"

namespace pp {

// ---------------------------------------------------------------- errors --
void set_error(const std::string& msg);
int fail(int code, const std::string& msg);
int hip_fail(hipError_t e, const char* what, const char* file, int line);

#define PP_HIP(expr)                                                            \
    do {                                                                        \
        hipError_t _e = (expr);                                                 \
        if (_e != hipSuccess) return ::pp::hip_fail(_e, #expr, __FILE__, __LINE__); \
    } while (0)

#define PP_TRY(expr)                      \
    do {                                  \
        int _rc = (expr);                 \
        if (_rc != PP_OK) return _rc;     \
    } while (0)

// --------------------------------------------------------- device memory --
// Grow-only device buffer.  Contents are not preserved across growth; every
// growth bumps a global generation so cached graphs can notice.
// Bump region of device memory that DevBuf::reserve carves buffers from
// instead of calling hipMalloc while a ScratchScope is active on the thread
// (the allocation-free entry point); such buffers are never freed.
struct Arena {
    char* base = nullptr;
    size_t cap = 0, used = 0;
};
struct ScratchScope {
    explicit ScratchScope(Arena* a);
    ~ScratchScope();
    Arena* prev;
};

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    bool carved = false;     // carved from an Arena (not hipMalloc'ed)
    uint32_t tag = 0;        // free for the owner's bookkeeping; 0 after every reallocation
    int reserve(size_t need);
    void release();
    template <class T> T* as() const { return static_cast<T*>(p); }
    ~DevBuf() { release(); }
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
};
uint64_t alloc_generation();

inline unsigned blocks_for(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

template <class T>
int read_back(const T* dev, T* host, hipStream_t s) {
    PP_HIP(hipMemcpyAsync(host, dev, sizeof(T), hipMemcpyDeviceToHost, s));
    PP_HIP(hipStreamSynchronize(s));
    return PP_OK;
}

// Target blocks: runs of at most kBlock consecutive particles (key order)
// inside one kBlock-particle chunk of one box whose bounding box side stays
// within 2 r_cut (so FP32 offsets from the block centre stay small).
constexpr int kBlock = 64;
// The persistent kernel's 8 work queues (one per XCD), each counter on its
// own 256-byte stretch so that pops on different queues do not contend for
// one cache line.
constexpr int kQueueStride = 64;
constexpr size_t kQueueBytes = 8 * kQueueStride * sizeof(unsigned);

// Integer bounding box of grid cells, hi exclusive.  Grid units: the box is
// W = 2^b cells wide, coordinates fit int32.
struct IBox {
    int32_t lo[3];
    int32_t hi[3];
};

// Implicit 8-ary tree over one box's leaves: level 0 holds the leaf boxes,
// node i of level h covers nodes 8i..8i+7 of level h-1.  Node (h, i) is
// element off[h] + i of the shared node-box array; node indices are local
// to the box (leaf i of the box is global leaf loff + i).
constexpr int kTreeMaxLevels = 16;
struct TreeView {
    int64_t off[kTreeMaxLevels];
    int64_t cnt[kTreeMaxLevels];
    int64_t loff;
    int32_t nlev;
    int32_t pad;
};

// FP32 constants of the PP kernel for one box, in the kernel's length unit
// ell = 2 r_s sqrt(U_MAX / 2) (so that the split polynomial's variable is
// t = r2 - 1 and its coefficients are the same for every box).
struct PolyF32 {
    float eps2n;     // softening^2 / ell^2 (floored)
    float cut2;      // (rcut^2 + eps^2) / ell^2, the cut on r2
    float keep2;     // slightly widened (rcut / ell)^2, the staging test
    float pad;
};

// Per-box constants, resident on the device.
struct BoxDev {
    double L, qscale, cell, inv_len, scale;    // inv_len = 1 / ell, scale = G / ell^2
    double rs, rcut, eps, G;
    int64_t W, T, emax;
    int64_t poff, n;
    PolyF32 poly;
};

int make_poly(const pp_box_params& p, PolyF32* out);
// The FP32 kernel's length unit ell = 2 r_s sqrt(U_MAX / 2).
double pair_length_unit(const pp_box_params& p);
// skin > 0 widens the lists' cut to rcut + skin (the pair test keeps rcut)
BoxDev make_boxdev(const pp_box_params& p, int64_t poff, int64_t n, double skin = 0.0);
int validate_params(const pp_box_params* p, bool need_poly);

// Box of particle (or chunk, leaf, ...) k given ascending start offsets:
// the last x with off[x] <= k (empty boxes are skipped naturally).
__device__ __forceinline__ int box_of(const int64_t* __restrict__ off, int nbox, int64_t k) {
    int lo = 0, hi = nbox - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= k) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Device view of a batch shared by the kernels.
struct BatchDev {
    const BoxDev* box;       // [nbox]
    const int64_t* poff;     // [nbox + 1] particle offsets
    int nbox;
    int bits;                // key bits per axis (shared)
    int leaf_max;            // shared
};

// ------------------------------------------------------------- workspace --
// One entry of the near-list expansion: (target block, periodic image,
// source tree node at a level).
struct FEntry {
    int32_t blk;
    int32_t node;
    uint8_t sc;      // shift code
    uint8_t lev;     // tree level of node
    uint8_t inside;  // whole subtree within r_cut
    uint8_t mono;    // taken as a monopole (monopole acceptance on)
};

// Slots of Work::sizes (int64, device).  The list builder writes the counts
// of the current lists here and every later kernel reads them, so that no
// count has to come back to the host before the pass's last kernel.  Counts
// are clamped to the capacities the buffers were sized with; the kNeed
// slots keep the totals, from which the host grows the buffers when one was
// too small (and then runs the pass again).
enum SizeSlot : int {
    kNBlock = 0,        // target blocks
    kNItem = 1,         // work items
    kNRange = 2,        // source ranges
    kNEntry = 3,        // final entries of the list expansion
    kNLeaf = 4,         // leaves
    kTotalSrc = 5,      // listed sources summed over the blocks
    kChunk = 6,         // source-list positions per work item (the effective chunk)
    kSkip = 7,          // nonzero: a buffer was too small or an input not finite; the PP kernels return
    kCand = 8,          // (target, listed source) pairs
    kOverflow = 9,      // bit 0: blocks, 1: entries, 2: ranges, 3: items, 4: a list longer than int32,
                        // 6: a single-pass scan gave up waiting
    kBad = 10,          // a non-finite position or mass
    kNeedBlock = 11,
    kNeedRange = 12,
    kNeedItem = 13,
    kMoved = 14,        // a call reusing the lists met a particle that moved half the skin or more
    kEntry0 = 16,       // kEntry0 + p: entries after expansion pass p (clamped)
    kNeedEntry0 = 40,   // kNeedEntry0 + p: the same, unclamped
    kSizeSlots = 64
};
constexpr int kMaxPasses = kTreeMaxLevels + 1;
constexpr int64_t kEntryBudget = (int64_t)1 << 28;

// Page-locked host buffer (hipHostMalloc) for the counts read back at the
// end of a pass.
struct HostBuf {
    void* p = nullptr;
    size_t bytes = 0;
    bool pinned = false;     // hipHostMalloc'ed (else plain host memory, under a ScratchScope)
    int reserve(size_t need);
    template <class T> T* as() const { return static_cast<T*>(p); }
    ~HostBuf();
    HostBuf() = default;
    HostBuf(const HostBuf&) = delete;
    HostBuf& operator=(const HostBuf&) = delete;
};

struct Work {
    int64_t pos_n = 0;       // particles in the current batch (row stride of pos_s)
    // capacities the list buffers are sized with (grown when a pass reports
    // a larger need); entries per expansion pass
    int64_t cap_block = 0, cap_range = 0, cap_item = 0;
    int64_t cap_ent[kMaxPasses] = {};
    int npass = 0;                        // expansion passes of the current lists
    // the last pass lowers the entries from level 2 to level 1 unless that
    // would need more than kEntryBudget entries; then the depth-first walks
    // start at level 2 (64 leaves each) for the rest of the plan's life
    bool stop_at_level2 = false;
    HostBuf sizes_h;                      // host copy of sizes after a pass
    // particles
    DevBuf keys, keys_s, iota, perm, pos_s, mass_s, mass_sd, bad;
    DevBuf rec;              // double4 [N]: wrapped position and mass, input order (gather staging)
    DevBuf mass_flag;        // int32 [nbox]: 1 where the box's FP32 masses are not all equal
    DevBuf split_tab;        // float4 [128]: the interpolated split table (variant bit 8)
    DevBuf tree_mc;          // double4 per tree node: sum m x, sum m y, sum m z, sum m
    DevBuf blk_amin2;        // double per block: min |a_ref|^2 over its targets
    const FEntry* ent_final = nullptr;   // the list expansion's final entries (nentry)
    // monopoles accepted by the depth-first walk, per final entry (null when
    // acceptance is off): leaves (bit = leaf - the entry's first leaf) and
    // groups of 8 leaves (bit = group - the entry's first group)
    DevBuf mono0_e, mono1_e;
    const uint64_t* mono0 = nullptr;
    const uint8_t* mono1 = nullptr;
    const uint8_t* active = nullptr;     // the items' target flags (null: every target)
    DevBuf sort_ws, scan_ws, sort_tmp;
    // leaves
    DevBuf lam, pmax, smax, level_p, flag, flag_off;
    DevBuf lbegin, lcount, llevel, lprefix, loff_dev;   // leaf boxes: tree_boxes[0 .. nleaf)
    int64_t nleaf = 0;                    // host copies, valid after leaves_to_host
    std::vector<int64_t> loff;            //   or lists_to_host ([nbox + 1])
    // trees
    DevBuf tree_boxes, tviews, lvl_prefix, tree_total;
    std::vector<TreeView> tv;             // host copy [nbox], valid after trees_to_host
    int max_levels = 0;                   // bound on the tree levels of any box
    // blocks, lists, items (host copies, valid after lists_to_host)
    int64_t nchunk = 0, nblock = 0, nentry = 0, nrange = 0, nitem = 0;
    int64_t candidates = 0;
    int64_t total_src = 0;     // listed sources summed over the blocks
    int chunk = 0;           // effective chunk of the current items (>= the requested one)
    std::vector<int64_t> choff_h;         // chunk offsets of the boxes (host)
    DevBuf choff, ccount, coff;
    DevBuf bstart, bcount, bbox, bboxid;
    DevBuf fent_a, fent_b, fcnt, foff, fmask;
    DevBuf lmask_e, rcnt_e, scnt_e, roff_e, soff_e, eoff;
    DevBuf roff, slen, rbeg, rpre, rcode;
    DevBuf icount, ioff, iblock, is0;
    DevBuf sizes;      // int64 [kSizeSlots], see SizeSlot
    DevBuf misc;       // counters and flags
};

// ------------------------------------------------------------- launches --
// keys_sort.hip
int stage_keys(const BatchDev& bd, int64_t N, const double* pos, Work& w, hipStream_t s);
// per-box flag: masses not all equal (equal masses take a shorter pair loop)
int stage_mass_flags(const BatchDev& bd, int64_t N, Work& w, hipStream_t s);
// out = in wrapped into [0, L) per box (the form every later stage expects)
int stage_wrap_copy(const BatchDev& bd, int64_t N, const double* in, double* out, hipStream_t s);
int stage_sort(const BatchDev& bd, int64_t N, Work& w, hipStream_t s);
int stage_gather(const BatchDev& bd, int64_t N, const double* pos, const float* mass_f,
                 const double* mass_d, Work& w, hipStream_t s);
int sort_workspace(int64_t n, int nbox, int bits, size_t* bytes);
// workspace bytes of a single-pass scan over n counts (scan.hip)
int scan_workspace(int64_t n, size_t* bytes);
// reserves the workspace for n counts; fresh memory is cleared on stream s
int grow_scan(DevBuf& buf, int64_t n, hipStream_t s);
// Count slots a scan fills with its total (see launch_scan_i32_to_i64).
struct ScanNote {
    int slot, need_slot;
    int64_t cap;
    unsigned long long bit;
    int slot2;                  // >= 0: gets the clamped total as well
};
// exclusive scan of int32 counts into int64 offsets; off has n + 1 entries
// (off[n] = total); sizes, when given, gets overflow bit 6 if the scan gave
// up; with a note (needs sizes) also sizes[need_slot] = total,
// sizes[slot] = min(total, cap) and `bit` in the overflow slot when over
int launch_scan_i32_to_i64(const int32_t* in, int64_t* off, int64_t n, DevBuf& ws, hipStream_t s,
                           int64_t* sizes = nullptr, const ScanNote* note = nullptr);
// the same for two count arrays of equal length in one pass
int launch_scan2_i32_to_i64(const int32_t* a, const int32_t* b, int64_t* oa, int64_t* ob, int64_t n,
                            DevBuf& ws, hipStream_t s, int64_t* sizes = nullptr);
int launch_keys_raw(const double* pos, int64_t n, double L, int bits, uint64_t* keys,
                    hipStream_t s);
int launch_sort_raw(const uint64_t* keys, const int32_t* idx_in, uint64_t* keys_out,
                    int32_t* perm_out, int64_t n, int bits, void* ws, size_t ws_bytes,
                    hipStream_t s);

// tree.hip  (positions passed here are wrapped: x - L floor(x / L))
// These stages keep their counts on the device (Work::sizes, the leaf and
// tree offsets); nothing is read back until the *_to_host calls.
// Leaves of every box (buffers sized for N leaves).
int stage_leaves(const BatchDev& bd, int64_t N, const uint64_t* sorted_keys, const double* pos_s,
                 Work& w, hipStream_t s);
// w.loff and w.nleaf from the device.  Synchronises the stream.
int leaves_to_host(const BatchDev& bd, Work& w, hipStream_t s);
// The implicit 8-ary trees over every box's leaves (levels bounded from N).
int stage_trees(const BatchDev& bd, int64_t N, Work& w, hipStream_t s);
// w.tv from the device.  Synchronises the stream.
int trees_to_host(const BatchDev& bd, Work& w, hipStream_t s);
// Monopole acceptance settings of the list expansion (nodes of level >= 2):
// every enabled test must hold.  theta2 = theta^2 of the geometric test
// (0: off); alpha of Gadget-2's relative test against reference
// accelerations acc_ref (FP32 [3][N], input order; 0: off).  mc: node
// moments (stage_node_moments).
struct MonoCfg {
    double theta2 = 0.0;
    double alpha = 0.0;
    const double4* mc = nullptr;
    const float* acc_ref = nullptr;
    bool on() const { return theta2 > 0.0 || alpha > 0.0; }
};
// Target blocks, near lists and work items, counts on the device; buffers
// sized with the capacities in w (see lists_to_host).
// active: optional device flags per input particle; target blocks without an
// active target get no work items (their outputs are left alone).
int stage_lists(const BatchDev& bd, const std::vector<int64_t>& poff, int chunk_req, Work& w,
                hipStream_t s, const MonoCfg& mono = MonoCfg(), const uint8_t* active = nullptr);
// Work items of the current lists (after stage_lists, or on their own for a
// call that reuses the lists): items per block for the given active flags,
// their offsets, and the final counts.
int stage_items(const BatchDev& bd, Work& w, hipStream_t s, const uint8_t* active);
// Zero the count slots at the start of a pass.
int reset_sizes(Work& w, hipStream_t s);
// A pass that reuses the lists: clears the per-pass slots (candidates,
// moved, skip, bad) and keeps the list counts.
int reset_sizes_reuse(Work& w, hipStream_t s);
// Positions and masses of a call that reuses the lists, in the stored key
// order: every particle moves from its reference position (ref, [3][N], the
// positions the lists were built at) by its minimum-image displacement, so
// it keeps the periodic image the lists hold; a displacement of at least
// half_skin sets the kMoved slot, a non-finite value the bad flag.
int stage_regather(const BatchDev& bd, int64_t N, const double* pos, const float* mass,
                   const double* ref, double half_skin, Work& w, hipStream_t s);
// Reads the counts of the last pass back (synchronises the stream).  Sets
// *regrow and grows the capacities when a buffer was too small (the pass must
// then run again); sets *regrow and *moved when a pass that reused the lists
// met a particle that moved too far (the lists must be rebuilt); PP_EINVAL
// when an input was not finite.  Otherwise fills the host copies (nleaf,
// nblock, nentry, nrange, nitem, candidates, chunk).
int lists_to_host(Work& w, hipStream_t s, bool* regrow, bool* moved = nullptr);
// Mass and mass-weighted position sums of every tree node (after stage_trees;
// needs the FP32 masses in key order).
int stage_node_moments(const BatchDev& bd, int64_t N, Work& w, hipStream_t s);
// Adds the monopoles' forces to acc (input order), FP32 path.
int launch_monopole(const BatchDev& bd, const Work& w, float* acc, unsigned long long* counter,
                    hipStream_t s);
int build_canonical_pairs(const BatchDev& bd, const Work& w, int64_t W, int64_t T, DevBuf& row_cnt,
                          DevBuf& row_ptr, DevBuf& src, DevBuf& code, DevBuf& scan_ws,
                          int64_t* nentries, hipStream_t s);

// pp_kernels.hip
enum class Mode { kGrid = 0, kPersistent = 1 };
// variant bits: 1 = one Newton step after the hardware rsqrt, 2 = no Kahan
// compensation, 4 = no FP64 block-origin subtraction (box-origin offsets)
// Blocks with a single work item write acc directly; the reduction finishes
// the others.
int launch_pp_f32(const BatchDev& bd, const Work& w, int groups, Mode mode, int waves_per_cu,
                  int variant, float* partial, float* acc, unsigned long long* counters,
                  unsigned* queues, hipStream_t s);
int launch_reduce_f32(const BatchDev& bd, const Work& w, const float* partial, float* acc,
                      hipStream_t s);
int launch_pp_f64(const BatchDev& bd, const Work& w, double* partial, hipStream_t s);
int launch_reduce_f64(const BatchDev& bd, const Work& w, const double* partial, double* acc,
                      hipStream_t s);
int launch_count(const BatchDev& bd, const Work& w, int32_t* partial, hipStream_t s);
int launch_reduce_count(const BatchDev& bd, const Work& w, const int32_t* partial, int64_t* counts,
                        unsigned long long* total, hipStream_t s);
// Builds the interpolated split table (FP64 series, rounded to FP32).
int launch_split_table(Work& w, hipStream_t s);
int launch_reset_queues(unsigned* queues, hipStream_t s, unsigned long long* counters = nullptr);

}  // namespace pp
