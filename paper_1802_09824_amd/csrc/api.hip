// C ABI of the library (include/photon_pp.h): argument checks, plans and
// the order of the path's stages.  All compute runs in the HIP kernels of
// keys_sort.hip, tree.hip and pp_kernels.hip.
#include <cmath>
#include <cstring>
#include <new>
#include <string>

#include "pp_internal.h"
#include "split_poly.h"

namespace pp {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

int fail(int code, const std::string& msg) {
    set_error(msg);
    return code;
}

int hip_fail(hipError_t e, const char* what, const char* file, int line) {
    char buf[512];
    snprintf(buf, sizeof buf, "%s failed: %s (%s:%d)", what, hipGetErrorString(e), file, line);
    set_error(buf);
    return e == hipErrorOutOfMemory ? PP_ENOMEM : PP_EDEVICE;
}

int DevBuf::reserve(size_t need) {
    if (need <= bytes) return PP_OK;
    release();
    size_t want = need + need / 4 + 256;
    hipError_t e = hipMalloc(&p, want);
    if (e != hipSuccess) {
        p = nullptr;
        (void)hipGetLastError();
        char buf[160];
        snprintf(buf, sizeof buf, "hipMalloc of %zu bytes failed: %s", want, hipGetErrorString(e));
        set_error(buf);
        return e == hipErrorOutOfMemory ? PP_ENOMEM : PP_EDEVICE;
    }
    bytes = want;
    return PP_OK;
}

void DevBuf::release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
}

Geo make_geo(const pp_box_params& p) {
    Geo g;
    g.L = p.L;
    g.bits = p.key_bits;
    g.W = (int64_t)1 << p.key_bits;
    const double r = p.rcut * ldexp(1.0, p.key_bits) / p.L;
    g.T = (int64_t)ceil(r * r);
    g.qscale = ldexp(1.0, p.key_bits) / p.L;
    return g;
}

int validate_params(const pp_box_params* p, bool need_poly) {
    if (!p) return fail(PP_EINVAL, "params is NULL");
    if (!(std::isfinite(p->L) && p->L > 0)) return fail(PP_EINVAL, "L must be finite and > 0");
    if (!(std::isfinite(p->rs) && p->rs > 0)) return fail(PP_EINVAL, "rs must be finite and > 0");
    if (!(std::isfinite(p->rcut) && p->rcut > 0)) return fail(PP_EINVAL, "rcut must be finite and > 0");
    if (!(std::isfinite(p->eps) && p->eps >= 0)) return fail(PP_EINVAL, "eps must be finite and >= 0");
    if (!std::isfinite(p->G)) return fail(PP_EINVAL, "G must be finite");
    if (p->leaf_max < 1 || p->leaf_max > 1024) return fail(PP_EINVAL, "leaf_max must be in 1..1024");
    if (p->key_bits < 1 || p->key_bits > 21) return fail(PP_EINVAL, "key_bits must be in 1..21");
    if (!(p->rcut < 0.5 * p->L))
        return fail(PP_ERANGE, "rcut must be < L/2 (one periodic image at most within the cut)");
    if (need_poly) {
        const double xmax = sqrt(p->rcut * p->rcut + p->eps * p->eps) / (2.0 * p->rs);
        if (xmax > SPLIT_POLY_X_MAX)
            return fail(PP_ERANGE, "sqrt(rcut^2 + eps^2) / (2 rs) exceeds the fitted range of the "
                                   "split-factor polynomial (2.26)");
    }
    return PP_OK;
}

}  // namespace pp

using namespace pp;

// ----------------------------------------------------------- objects --
struct pp_leaves {
    int64_t n = 0, m = 0;
    pp_box_params p{};
    DevBuf begin, count, level, prefix, boxes;
};

struct pp_pairs {
    int64_t nrows = 0, nentries = 0;
    DevBuf row_cnt, row_ptr, src, code;
};

struct pp_plan {
    pp_box_params p{};
    Geo g{};
    PolyF32 poly{};
    int64_t n_max = 0;
    int chunk = 4096;
    // per-particle buffers
    DevBuf keys, keys_s, iota, perm, pos_s, mass_s, mass_sd, bad;
    DevBuf lam, pmax, smax, level_p, flag, flag_off;
    DevBuf sort_ws, scan_ws;
    size_t sort_ws_bytes = 0, scan_ws_bytes = 0;
    // leaves + tree
    DevBuf lbegin, lcount, llevel, lprefix, lboxes, tree_boxes;
    TreeView tv{};
    int64_t nleaf = 0;
    BlockLists bl;
    DevBuf partial, pcount, cnt_total;
    pp_stats st{};
    bool lists_valid = false;
    int64_t last_n = 0;
    bool timing = false, timed = false, evaluated_valid = false;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    ~pp_plan() {
        if (ev0) (void)hipEventDestroy(ev0);
        if (ev1) (void)hipEventDestroy(ev1);
    }
};

static hipStream_t S(void* s) { return reinterpret_cast<hipStream_t>(s); }

static int check_ptr(const void* p, int64_t n, const char* name) {
    if (n > 0 && !p) return fail(PP_EINVAL, std::string(name) + " is NULL");
    return PP_OK;
}

extern "C" {

const char* pp_strerror(int code) {
    switch (code) {
        case PP_OK: return "ok";
        case PP_EINVAL: return "invalid argument";
        case PP_ENOMEM: return "out of memory";
        case PP_EDEVICE: return "HIP device error";
        case PP_ERANGE: return "parameter out of supported range";
        case PP_EOVERFLOW: return "buffer too small";
        default: return "unknown error";
    }
}

const char* pp_last_error(void) { return g_last_error.c_str(); }

int pp_hilbert_keys(const double* pos, int64_t n, double L, int key_bits, uint64_t* keys,
                    void* stream) {
    if (n < 0) return fail(PP_EINVAL, "n < 0");
    PP_TRY(check_ptr(pos, n, "pos"));
    PP_TRY(check_ptr(keys, n, "keys"));
    if (!(std::isfinite(L) && L > 0)) return fail(PP_EINVAL, "L must be finite and > 0");
    if (key_bits < 1 || key_bits > 21) return fail(PP_EINVAL, "key_bits must be in 1..21");
    if (n == 0) return PP_OK;
    return launch_keys(pos, n, L, key_bits, keys, nullptr, nullptr, S(stream));
}

int pp_sort_workspace_size(int64_t n, size_t* bytes) {
    if (!bytes) return fail(PP_EINVAL, "bytes is NULL");
    if (n < 0 || n > INT32_MAX) return fail(PP_EINVAL, "n out of range");
    size_t b = 0;
    PP_TRY(sort_workspace(n, 21, &b));
    // plus the index sequence and key scratch the call fills itself
    *bytes = b + 256 + sizeof(int32_t) * (size_t)n + 256;
    return PP_OK;
}

namespace {
__global__ void iota_kernel(int32_t* p, int64_t n) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) p[k] = (int32_t)k;
}
}  // namespace

int pp_sort_by_key(const uint64_t* keys, int64_t n, int32_t* perm, uint64_t* sorted_keys, void* ws,
                   size_t ws_bytes, void* stream) {
    if (n < 0 || n > INT32_MAX) return fail(PP_EINVAL, "n out of range");
    PP_TRY(check_ptr(keys, n, "keys"));
    PP_TRY(check_ptr(perm, n, "perm"));
    if (n == 0) return PP_OK;
    size_t need = 0;
    PP_TRY(pp_sort_workspace_size(n, &need));
    if (!ws || ws_bytes < need) {
        char buf[128];
        snprintf(buf, sizeof buf, "sort workspace too small: need %zu bytes", need);
        return fail(PP_EOVERFLOW, buf);
    }
    size_t sb = 0;
    PP_TRY(sort_workspace(n, 21, &sb));
    char* w = static_cast<char*>(ws);
    int32_t* idx = reinterpret_cast<int32_t*>(w + ((sb + 255) / 256) * 256);
    hipLaunchKernelGGL(iota_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, S(stream), idx,
                       n);
    PP_HIP(hipGetLastError());
    DevBuf tmp;
    uint64_t* kout = sorted_keys;
    if (!kout) {
        PP_TRY(tmp.reserve(sizeof(uint64_t) * n));
        kout = tmp.as<uint64_t>();
    }
    PP_TRY(launch_sort(keys, idx, kout, perm, n, 21, w, sb, S(stream)));
    if (!sorted_keys) PP_HIP(hipStreamSynchronize(S(stream)));   // before tmp is freed
    return PP_OK;
}

int pp_build_leaves(const uint64_t* sorted_keys, const double* pos_sorted, int64_t n,
                    const pp_box_params* p, pp_leaves** out, void* stream) {
    if (!out) return fail(PP_EINVAL, "out is NULL");
    *out = nullptr;
    if (n < 0 || n > INT32_MAX) return fail(PP_EINVAL, "n out of range");
    PP_TRY(check_ptr(sorted_keys, n, "sorted_keys"));
    PP_TRY(check_ptr(pos_sorted, n, "pos_sorted"));
    PP_TRY(validate_params(p, false));
    pp_leaves* lv = new (std::nothrow) pp_leaves;
    if (!lv) return fail(PP_ENOMEM, "host allocation failed");
    lv->n = n;
    lv->p = *p;
    const Geo g = make_geo(*p);
    DevBuf lam, pmax, smax, level_p, flag, flag_off, scan_ws;
    size_t sw = 0;
    int rc = PP_OK;
    const int64_t len = n + p->leaf_max + 1;
    if ((rc = lam.reserve(len)) || (rc = pmax.reserve(len)) || (rc = smax.reserve(len)) ||
        (rc = level_p.reserve(n + 1)) || (rc = flag.reserve(4 * (n + 1))) ||
        (rc = flag_off.reserve(8 * (n + 2))) || (rc = scan_workspace(n, &sw)) ||
        (rc = scan_ws.reserve(sw + 1))) {
        delete lv;
        return rc;
    }
    LeafBuffers lb{lam.as<int8_t>(), pmax.as<int8_t>(), smax.as<int8_t>(), level_p.as<int8_t>(),
                   flag.as<int32_t>(), flag_off.as<int64_t>()};
    // wrapped copy of the sorted positions is what the boxes use; the input
    // is documented as already in key order, wrapping happens in quantise.
    rc = build_leaves_device(sorted_keys, pos_sorted, n, g, p->leaf_max, lb, scan_ws.p,
                             scan_ws.bytes, lv->begin, lv->count, lv->level, lv->prefix, lv->boxes,
                             &lv->m, S(stream));
    if (rc == PP_OK) {
        hipError_t e = hipStreamSynchronize(S(stream));
        if (e != hipSuccess) rc = hip_fail(e, "hipStreamSynchronize", __FILE__, __LINE__);
    }
    if (rc != PP_OK) {
        delete lv;
        return rc;
    }
    *out = lv;
    return PP_OK;
}

int pp_leaves_count(const pp_leaves* lv, int64_t* nleaf) {
    if (!lv || !nleaf) return fail(PP_EINVAL, "NULL argument");
    *nleaf = lv->m;
    return PP_OK;
}

int pp_leaves_export(const pp_leaves* lv, int64_t* begin, int32_t* count, int32_t* level,
                     uint64_t* prefix, int32_t* lo, int32_t* hi) {
    if (!lv) return fail(PP_EINVAL, "leaves is NULL");
    const int64_t m = lv->m;
    if (m == 0) return PP_OK;
    if (begin) PP_HIP(hipMemcpy(begin, lv->begin.p, 8 * m, hipMemcpyDefault));
    if (count) PP_HIP(hipMemcpy(count, lv->count.p, 4 * m, hipMemcpyDefault));
    if (level) PP_HIP(hipMemcpy(level, lv->level.p, 4 * m, hipMemcpyDefault));
    if (prefix) PP_HIP(hipMemcpy(prefix, lv->prefix.p, 8 * m, hipMemcpyDefault));
    if (lo || hi) {
        std::vector<IBox> hb(m);
        PP_HIP(hipMemcpy(hb.data(), lv->boxes.p, sizeof(IBox) * m, hipMemcpyDeviceToHost));
        std::vector<int32_t> t(3 * m);
        for (int w = 0; w < 2; ++w) {
            int32_t* dst = w == 0 ? lo : hi;
            if (!dst) continue;
            for (int64_t a = 0; a < m; ++a)
                for (int ax = 0; ax < 3; ++ax) t[ax * m + a] = w == 0 ? hb[a].lo[ax] : hb[a].hi[ax];
            PP_HIP(hipMemcpy(dst, t.data(), 4 * 3 * m, hipMemcpyDefault));
        }
    }
    return PP_OK;
}

void pp_leaves_free(pp_leaves* lv) { delete lv; }

int pp_near_pairs(const pp_leaves* lv, const pp_box_params* p, pp_pairs** out, void* stream) {
    if (!out) return fail(PP_EINVAL, "out is NULL");
    *out = nullptr;
    if (!lv) return fail(PP_EINVAL, "leaves is NULL");
    PP_TRY(validate_params(p, false));
    if (p->key_bits != lv->p.key_bits || p->L != lv->p.L)
        return fail(PP_EINVAL, "params do not match the leaves (L, key_bits)");
    pp_pairs* pr = new (std::nothrow) pp_pairs;
    if (!pr) return fail(PP_ENOMEM, "host allocation failed");
    const Geo g = make_geo(*p);
    DevBuf tree, scan_ws;
    TreeView tv{};
    size_t sw = 0;
    int rc = scan_workspace(lv->m, &sw);
    if (rc == PP_OK) rc = scan_ws.reserve(sw + 1);
    if (rc == PP_OK && lv->m > 0) rc = build_tree(lv->boxes.as<IBox>(), lv->m, tree, &tv, S(stream));
    if (rc == PP_OK)
        rc = build_canonical_pairs(tv, lv->m, g, pr->row_cnt, pr->row_ptr, pr->src, pr->code,
                                   scan_ws.p, scan_ws.bytes, &pr->nentries, S(stream));
    if (rc == PP_OK) {
        hipError_t e = hipStreamSynchronize(S(stream));
        if (e != hipSuccess) rc = hip_fail(e, "hipStreamSynchronize", __FILE__, __LINE__);
    }
    if (rc != PP_OK) {
        delete pr;
        return rc;
    }
    pr->nrows = lv->m;
    *out = pr;
    return PP_OK;
}

int pp_pairs_count(const pp_pairs* pr, int64_t* nrows, int64_t* nentries) {
    if (!pr) return fail(PP_EINVAL, "pairs is NULL");
    if (nrows) *nrows = pr->nrows;
    if (nentries) *nentries = pr->nentries;
    return PP_OK;
}

int pp_pairs_export(const pp_pairs* pr, int64_t* row_ptr, int32_t* src_leaf, uint8_t* shift_code) {
    if (!pr) return fail(PP_EINVAL, "pairs is NULL");
    if (row_ptr) PP_HIP(hipMemcpy(row_ptr, pr->row_ptr.p, 8 * (pr->nrows + 1), hipMemcpyDefault));
    if (pr->nentries > 0) {
        if (src_leaf) PP_HIP(hipMemcpy(src_leaf, pr->src.p, 4 * pr->nentries, hipMemcpyDefault));
        if (shift_code) PP_HIP(hipMemcpy(shift_code, pr->code.p, pr->nentries, hipMemcpyDefault));
    }
    return PP_OK;
}

void pp_pairs_free(pp_pairs* pr) { delete pr; }

int pp_plan_create(const pp_box_params* p, int64_t n_max, pp_plan** out) {
    if (!out) return fail(PP_EINVAL, "out is NULL");
    *out = nullptr;
    PP_TRY(validate_params(p, true));
    if (n_max < 0 || n_max > INT32_MAX - 2048) return fail(PP_EINVAL, "n_max out of range");
    int dev_count = 0;
    hipError_t e = hipGetDeviceCount(&dev_count);
    if (e != hipSuccess || dev_count == 0) {
        (void)hipGetLastError();
        return fail(PP_EDEVICE, "no HIP device available");
    }
    pp_plan* pl = new (std::nothrow) pp_plan;
    if (!pl) return fail(PP_ENOMEM, "host allocation failed");
    pl->p = *p;
    pl->g = make_geo(*p);
    make_poly(*p, &pl->poly);
    pl->n_max = n_max;
    const int64_t n = n_max > 0 ? n_max : 1;
    const int M = p->leaf_max;
    int rc = PP_OK;
    size_t sw = 0, cw = 0;
    if ((rc = pl->keys.reserve(8 * n)) || (rc = pl->keys_s.reserve(8 * n)) ||
        (rc = pl->iota.reserve(4 * n)) || (rc = pl->perm.reserve(4 * n)) ||
        (rc = pl->pos_s.reserve(24 * n)) || (rc = pl->mass_s.reserve(4 * n)) ||
        (rc = pl->bad.reserve(64)) || (rc = pl->lam.reserve(n + M + 1)) ||
        (rc = pl->pmax.reserve(n + M + 1)) || (rc = pl->smax.reserve(n + M + 1)) ||
        (rc = pl->level_p.reserve(n + 1)) || (rc = pl->flag.reserve(4 * (n + 1))) ||
        (rc = pl->flag_off.reserve(8 * (n + 2))) || (rc = sort_workspace(n, p->key_bits, &sw)) ||
        (rc = pl->sort_ws.reserve(sw + 1)) || (rc = scan_workspace(n + 1, &cw)) ||
        (rc = pl->scan_ws.reserve(cw + 1)) || (rc = pl->cnt_total.reserve(64))) {
        delete pl;
        return rc;
    }
    pl->sort_ws_bytes = pl->sort_ws.bytes;
    pl->scan_ws_bytes = pl->scan_ws.bytes;
    *out = pl;
    return PP_OK;
}

void pp_plan_destroy(pp_plan* plan) { delete plan; }

// Stages shared by the FP32 and FP64 paths: keys, sort, gather, leaves,
// tree and block lists.  Synchronises the stream.
static int prepare(pp_plan* pl, const double* pos, const float* mass_f, const double* mass_d,
                   int64_t n, hipStream_t s) {
    pl->lists_valid = false;
    pl->evaluated_valid = false;
    PP_HIP(hipMemsetAsync(pl->bad.p, 0, sizeof(int), s));
    PP_TRY(launch_keys(pos, n, pl->p.L, pl->p.key_bits, pl->keys.as<uint64_t>(),
                       pl->iota.as<int32_t>(), pl->bad.as<int>(), s));
    PP_TRY(launch_sort(pl->keys.as<uint64_t>(), pl->iota.as<int32_t>(), pl->keys_s.as<uint64_t>(),
                       pl->perm.as<int32_t>(), n, pl->p.key_bits, pl->sort_ws.p, pl->sort_ws_bytes,
                       s));
    if (mass_d) PP_TRY(pl->mass_sd.reserve(8 * (n > 0 ? n : 1)));
    PP_TRY(launch_gather(pos, mass_f, mass_d, pl->perm.as<int32_t>(), n, pl->p.L,
                         pl->pos_s.as<double>(), pl->mass_s.as<float>(),
                         mass_d ? pl->mass_sd.as<double>() : nullptr, pl->bad.as<int>(), s));
    LeafBuffers lb{pl->lam.as<int8_t>(), pl->pmax.as<int8_t>(), pl->smax.as<int8_t>(),
                   pl->level_p.as<int8_t>(), pl->flag.as<int32_t>(), pl->flag_off.as<int64_t>()};
    PP_TRY(build_leaves_device(pl->keys_s.as<uint64_t>(), pl->pos_s.as<double>(), n, pl->g,
                               pl->p.leaf_max, lb, pl->scan_ws.p, pl->scan_ws_bytes, pl->lbegin,
                               pl->lcount, pl->llevel, pl->lprefix, pl->lboxes, &pl->nleaf, s));
    int bad = 0;
    PP_HIP(hipMemcpyAsync(&bad, pl->bad.p, sizeof(int), hipMemcpyDeviceToHost, s));
    PP_HIP(hipStreamSynchronize(s));
    if (bad) return fail(PP_EINVAL, "non-finite position or mass");
    PP_TRY(build_tree(pl->lboxes.as<IBox>(), pl->nleaf, pl->tree_boxes, &pl->tv, s));
    PP_TRY(build_block_lists(pl->pos_s.as<double>(), n, pl->lbegin.as<int64_t>(),
                             pl->lcount.as<int32_t>(), pl->tv, pl->nleaf, pl->g, pl->chunk,
                             pl->p.rcut, pl->bl, pl->scan_ws, s));
    pl->scan_ws_bytes = pl->scan_ws.bytes;
    pl->st.n = n;
    pl->st.nleaf = pl->nleaf;
    pl->st.nblock = pl->bl.nblock;
    pl->st.nrange = pl->bl.nrange;
    pl->st.nitem = pl->bl.nitem;
    pl->st.candidates = pl->bl.candidates;
    pl->st.interactions = -1;
    pl->st.pp_kernel_ms = -1.0;
    pl->lists_valid = true;
    pl->last_n = n;
    return PP_OK;
}

static int check_accel_args(pp_plan* pl, const void* pos, const void* mass, int64_t n,
                            const void* acc) {
    if (!pl) return fail(PP_EINVAL, "plan is NULL");
    if (n < 0 || n > pl->n_max) return fail(PP_EINVAL, "n must be in 0..n_max of the plan");
    PP_TRY(check_ptr(pos, n, "pos"));
    PP_TRY(check_ptr(mass, n, "mass"));
    PP_TRY(check_ptr(acc, n, "acc"));
    return PP_OK;
}

int pp_accel(pp_plan* pl, const double* pos, const float* mass, int64_t n, float* acc,
             void* stream) {
    PP_TRY(check_accel_args(pl, pos, mass, n, acc));
    if (n == 0) return PP_OK;
    hipStream_t s = S(stream);
    PP_TRY(prepare(pl, pos, mass, nullptr, n, s));
    PP_TRY(pl->partial.reserve(sizeof(float) * 6 * kBlock * (pl->bl.nitem + 1)));
    unsigned long long* evald = reinterpret_cast<unsigned long long*>(pl->cnt_total.as<char>() + 8);
    PP_HIP(hipMemsetAsync(evald, 0, 2 * sizeof(unsigned long long), s));
    pl->evaluated_valid = true;
    if (pl->timing) PP_HIP(hipEventRecord(pl->ev0, s));
    PP_TRY(launch_pp_f32(pl->bl, pl->pos_s.as<double>(), pl->mass_s.as<float>(), n, pl->p, pl->poly,
                         pl->chunk, pl->partial.as<float>(), evald, s));
    if (pl->timing) {
        PP_HIP(hipEventRecord(pl->ev1, s));
        pl->timed = true;
    }
    const double scale = pl->p.G / (pl->p.rcut * pl->p.rcut);
    PP_TRY(launch_reduce_f32(pl->bl, pl->partial.as<float>(), pl->perm.as<int32_t>(), n, scale, acc,
                             s));
    return PP_OK;
}

int pp_accel_f64(pp_plan* pl, const double* pos, const double* mass, int64_t n, double* acc,
                 void* stream) {
    PP_TRY(check_accel_args(pl, pos, mass, n, acc));
    if (n == 0) return PP_OK;
    hipStream_t s = S(stream);
    PP_TRY(prepare(pl, pos, nullptr, mass, n, s));
    PP_TRY(pl->partial.reserve(sizeof(double) * 3 * kBlock * (pl->bl.nitem + 1)));
    if (pl->timing) PP_HIP(hipEventRecord(pl->ev0, s));
    PP_TRY(launch_pp_f64(pl->bl, pl->pos_s.as<double>(), pl->mass_sd.as<double>(), n, pl->p,
                         pl->chunk, pl->partial.as<double>(), s));
    if (pl->timing) {
        PP_HIP(hipEventRecord(pl->ev1, s));
        pl->timed = true;
    }
    PP_TRY(launch_reduce_f64(pl->bl, pl->partial.as<double>(), pl->perm.as<int32_t>(), n, acc, s));
    return PP_OK;
}

int pp_plan_stats(pp_plan* pl, pp_stats* out) {
    if (!pl || !out) return fail(PP_EINVAL, "NULL argument");
    pl->st.pp_kernel_ms = -1.0;
    if (pl->timing && pl->timed) {
        PP_HIP(hipEventSynchronize(pl->ev1));
        float ms = 0.f;
        PP_HIP(hipEventElapsedTime(&ms, pl->ev0, pl->ev1));
        pl->st.pp_kernel_ms = ms;
    }
    pl->st.evaluated = -1;
    pl->st.lane_pairs = -1;
    if (pl->evaluated_valid) {
        unsigned long long h[2] = {0, 0};
        PP_HIP(hipMemcpy(h, pl->cnt_total.as<char>() + 8, sizeof(h), hipMemcpyDeviceToHost));
        pl->st.evaluated = (int64_t)h[0];
        pl->st.lane_pairs = (int64_t)h[1];
    }
    *out = pl->st;
    return PP_OK;
}

int pp_plan_set_timing(pp_plan* pl, int on) {
    if (!pl) return fail(PP_EINVAL, "plan is NULL");
    if (on && !pl->ev0) {
        PP_HIP(hipEventCreate(&pl->ev0));
        PP_HIP(hipEventCreate(&pl->ev1));
    }
    pl->timing = on != 0;
    pl->timed = false;
    return PP_OK;
}

int pp_count_interactions(pp_plan* pl, int64_t* counts, int64_t* total, void* stream) {
    if (!pl || !total) return fail(PP_EINVAL, "NULL argument");
    if (!pl->lists_valid) return fail(PP_EINVAL, "no lists: call pp_accel first");
    const int64_t n = pl->last_n;
    hipStream_t s = S(stream);
    PP_TRY(pl->pcount.reserve(sizeof(int32_t) * kBlock * (pl->bl.nitem + 1)));
    PP_TRY(launch_count(pl->bl, pl->pos_s.as<double>(), n, pl->p, pl->chunk,
                        pl->pcount.as<int32_t>(), s));
    unsigned long long* tot = reinterpret_cast<unsigned long long*>(pl->cnt_total.p);
    PP_HIP(hipMemsetAsync(tot, 0, sizeof(unsigned long long), s));
    PP_TRY(launch_reduce_count(pl->bl, pl->pcount.as<int32_t>(), pl->perm.as<int32_t>(), n, counts,
                               tot, s));
    unsigned long long h = 0;
    PP_HIP(hipMemcpyAsync(&h, tot, sizeof(h), hipMemcpyDeviceToHost, s));
    PP_HIP(hipStreamSynchronize(s));
    *total = (int64_t)h;
    pl->st.interactions = (int64_t)h;
    return PP_OK;
}

}  // extern "C"
