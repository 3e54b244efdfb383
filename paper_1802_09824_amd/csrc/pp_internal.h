// Internal declarations shared by the library's translation units.
// Nothing here is part of the C ABI (include/photon_pp.h is).
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
// Grow-only device buffer.  Contents are not preserved across growth.
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    int reserve(size_t need);
    void release();
    template <class T> T* as() const { return static_cast<T*>(p); }
    ~DevBuf() { release(); }
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
};

// Integer bounding box of grid cells, hi exclusive.  Grid units: the box is
// W = 2^b cells wide, coordinates fit int32.
struct IBox {
    int32_t lo[3];
    int32_t hi[3];
};

// Implicit 8-ary tree over the leaf array: level 0 holds the leaf boxes,
// node i of level h covers nodes 8i..8i+7 of level h-1.
constexpr int kTreeMaxLevels = 16;
struct TreeView {
    const IBox* box;                 // all levels, level h at off[h]
    int64_t off[kTreeMaxLevels];
    int64_t cnt[kTreeMaxLevels];
    int nlev;
};

// ------------------------------------------------------- geometry params --
struct Geo {
    double L;           // box side
    int bits;           // key bits per axis
    int64_t W;          // 2^bits
    int64_t T;          // ceil(r^2), r = rcut * W / L (grid units)
    double qscale;      // 2^bits / L
};
Geo make_geo(const pp_box_params& p);

// Validation shared by the entry points; returns PP_OK or an error code.
int validate_params(const pp_box_params* p, bool need_poly);

// ------------------------------------------------------------- launches --
// keys_sort.hip
int launch_keys(const double* pos, int64_t n, double L, int bits, uint64_t* keys,
                int32_t* iota, int* bad_flag, hipStream_t s);
int sort_workspace(int64_t n, int bits, size_t* bytes);
int launch_sort(const uint64_t* keys, const int32_t* idx_in, uint64_t* keys_out,
                int32_t* perm_out, int64_t n, int bits, void* ws, size_t ws_bytes, hipStream_t s);
int launch_gather(const double* pos, const float* mass_f, const double* mass_d,
                  const int32_t* perm, int64_t n, double L, double* pos_s, float* mass_s_f,
                  double* mass_s_d, int* bad_flag, hipStream_t s);
int scan_workspace(int64_t n, size_t* bytes);
// exclusive scan of int32 counts into int64 offsets; off has n + 1 entries
int launch_scan_i32_to_i64(const int32_t* in, int64_t* off, int64_t n, void* ws, size_t ws_bytes,
                           hipStream_t s);

// tree.hip
struct LeafBuffers {           // device arrays sized for n particles
    int8_t* lam;               // n + leaf_max
    int8_t* pmax;              // n + leaf_max
    int8_t* smax;              // n + leaf_max
    int8_t* level_p;           // n  leaf level of each particle
    int32_t* flag;             // n  leaf-start flags
    int64_t* flag_off;         // n + 1
};
int build_leaves_device(const uint64_t* sorted_keys, const double* pos_s, int64_t n, const Geo& g,
                        int leaf_max, LeafBuffers& lb, void* scan_ws, size_t scan_ws_bytes,
                        DevBuf& begin, DevBuf& count, DevBuf& level, DevBuf& prefix, DevBuf& boxes,
                        int64_t* nleaf_out, hipStream_t s);
int build_tree(const IBox* leaf_boxes, int64_t nleaf, DevBuf& tree_boxes, TreeView* tv,
               hipStream_t s);
int build_canonical_pairs(const TreeView& tv, int64_t nleaf, const Geo& g, DevBuf& row_cnt,
                          DevBuf& row_ptr, DevBuf& src, DevBuf& code, void* scan_ws,
                          size_t scan_ws_bytes, int64_t* nentries, hipStream_t s);

// Target blocks: runs of at most kBlock consecutive particles (key order)
// inside one kBlock-particle chunk whose bounding box side stays within
// r_cut (so FP32 offsets from the block centre stay small).
constexpr int kBlock = 64;
struct BlockLists {
    int64_t nblock = 0, nrange = 0, nitem = 0, nchunk = 0;
    int64_t candidates = 0;
    DevBuf ccount;     // int32 [nchunk] blocks per chunk
    DevBuf coff;       // int64 [nchunk + 1]
    DevBuf bstart;     // int32 [nblock] first particle
    DevBuf bcount;     // int32 [nblock] particles (1..kBlock)
    DevBuf box;        // IBox [nblock]
    int64_t nentry = 0;
    DevBuf fent_a, fent_b;  // breadth-first entries (block, shift, node)
    DevBuf fcnt;       // int32 per entry: children / ranges
    DevBuf foff;       // int64 scan of fcnt
    DevBuf lmask_e;    // uint64 [nentry] passing leaves of the entry's subtree
    DevBuf rcnt_e;     // int32 [nentry] ranges per entry
    DevBuf scnt_e;     // int32 [nentry] listed sources per entry
    DevBuf roff_e;     // int64 [nentry + 1]
    DevBuf soff_e;     // int64 [nentry + 1]
    DevBuf eoff;       // int64 [nblock + 1] first entry of each block
    DevBuf roff;       // int64 [nblock + 1] first range of each block
    DevBuf rbeg;       // int32 [nrange] first source particle
    DevBuf rpre;       // int32 [nrange] exclusive prefix of lengths in the block list
    DevBuf rcode;      // uint8 [nrange] periodic shift code
    DevBuf slen;       // int32 [nblock] total sources in the block list
    DevBuf icount;     // int32 [nblock] work items per block
    DevBuf ioff;       // int64 [nblock + 1]
    DevBuf iblock;     // int32 [nitem]
    DevBuf is0;        // int32 [nitem] first list position of the item
};
int build_block_lists(const double* pos_s, int64_t n, const int64_t* leaf_begin,
                      const int32_t* leaf_count, const TreeView& tv, int64_t nleaf, const Geo& g,
                      int chunk, double rcut, BlockLists& bl, DevBuf& scan_ws, hipStream_t s);

// pp_kernels.hip
struct PolyF32 {
    float c[10];     // K * H coefficients in t, highest last
    float tscale;    // t = r2n * tscale - 1
    float eps2n;     // softening^2 / rcut^2 (floored)
    float cut2;      // 1 + eps2n
};
int make_poly(const pp_box_params& p, PolyF32* out);
int launch_pp_f32(const BlockLists& bl, const double* pos_s, const float* mass_s, int64_t n,
                  const pp_box_params& p, const PolyF32& poly, int chunk, float* partial,
                  unsigned long long* counters, hipStream_t s);
int launch_reduce_f32(const BlockLists& bl, const float* partial, const int32_t* perm, int64_t n,
                      double scale, float* acc, hipStream_t s);
int launch_pp_f64(const BlockLists& bl, const double* pos_s, const double* mass_s, int64_t n,
                  const pp_box_params& p, int chunk, double* partial, hipStream_t s);
int launch_reduce_f64(const BlockLists& bl, const double* partial, const int32_t* perm, int64_t n,
                      double* acc, hipStream_t s);
int launch_count(const BlockLists& bl, const double* pos_s, int64_t n, const pp_box_params& p,
                 int chunk, int32_t* partial_counts, hipStream_t s);
int launch_reduce_count(const BlockLists& bl, const int32_t* partial, const int32_t* perm,
                        int64_t n, int64_t* counts, unsigned long long* total, hipStream_t s);

}  // namespace pp
