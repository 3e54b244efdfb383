// C ABI of the library (include/photon_pp.h): argument checks, plans, the
// order of the path's stages, the batched persistent launch and its graph,
// and the autotuner.  All compute runs in the HIP kernels of keys_sort.hip,
// tree.hip and pp_kernels.hip (the PM force and the KDK driver have their
// own entry points in pm.hip and kdk.hip).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <mutex>
#include <new>
#include <sstream>
#include <string>

#include "pp_internal.h"
#include "split_poly.h"

namespace pp {

static thread_local std::string g_last_error;
static uint64_t g_alloc_generation = 1;

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

uint64_t alloc_generation() { return g_alloc_generation; }

static thread_local Arena* t_arena = nullptr;

ScratchScope::ScratchScope(Arena* a) : prev(t_arena) { t_arena = a; }
ScratchScope::~ScratchScope() { t_arena = prev; }

int DevBuf::reserve(size_t need) {
    if (need <= bytes) return PP_OK;
    release();
    if (t_arena) {
        const size_t want = (need + 255) & ~(size_t)255;
        if (t_arena->used + want > t_arena->cap)
            return fail(PP_ENOMEM, "the input needs more than the static device scratch of the "
                                   "allocation-free entry point holds");
        p = t_arena->base + t_arena->used;
        t_arena->used += want;
        bytes = want;
        carved = true;
        tag = 0;
        ++g_alloc_generation;
        return PP_OK;
    }
    const size_t want = need + need / 4 + 256;
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
    tag = 0;
    ++g_alloc_generation;
    return PP_OK;
}

void DevBuf::release() {
    if (p && !carved) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
    carved = false;
}

static void host_free(HostBuf& h) {
    if (h.p) {
        if (h.pinned) (void)hipHostFree(h.p);
        else std::free(h.p);
    }
    h.p = nullptr;
    h.bytes = 0;
}

int HostBuf::reserve(size_t need) {
    if (need <= bytes) return PP_OK;
    host_free(*this);
    if (t_arena) {                      // no HIP allocation at all: plain host memory
        p = std::malloc(need);
        if (!p) return fail(PP_ENOMEM, "host allocation failed");
        pinned = false;
        bytes = need;
        return PP_OK;
    }
    pinned = true;
    hipError_t e = hipHostMalloc(&p, need, hipHostMallocDefault);
    if (e != hipSuccess) {
        p = nullptr;
        (void)hipGetLastError();
        return fail(PP_ENOMEM, "hipHostMalloc failed");
    }
    bytes = need;
    return PP_OK;
}

HostBuf::~HostBuf() { host_free(*this); }

BoxDev make_boxdev(const pp_box_params& p, int64_t poff, int64_t n, double skin) {
    BoxDev b{};
    b.L = p.L;
    b.qscale = ldexp(1.0, p.key_bits) / p.L;
    b.cell = p.L / ldexp(1.0, p.key_bits);
    const double ell = pair_length_unit(p);
    b.inv_len = 1.0 / ell;
    b.scale = p.G / (ell * ell);
    b.rs = p.rs;
    b.rcut = p.rcut;
    b.eps = p.eps;
    b.G = p.G;
    b.W = (int64_t)1 << p.key_bits;
    const double r = (p.rcut + skin) * ldexp(1.0, p.key_bits) / p.L;
    b.T = (int64_t)ceil(r * r);
    b.emax = (int64_t)floor(2.0 * p.rcut * (double)b.W / p.L);
    b.poff = poff;
    b.n = n;
    make_poly(p, &b.poly);
    return b;
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

// ------------------------------------------------------------------ batch --
struct Batch {
    int nbox = 0;
    int64_t n_max = 0;                    // capacity (particles)
    std::vector<pp_box_params> params;
    std::vector<int64_t> poff;            // host [nbox + 1]
    int64_t N = 0;
    DevBuf box_dev, poff_dev;
    BatchDev bd{};
    Work w;
    pp_tuning tune{2048, 1, 20, 0, 0, 1};
    int64_t graph_variant = -1;
    bool table_ready = false;      // the interpolated split table is built
    double theta = 0.0;            // geometric monopole acceptance (0: off)
    double alpha = 0.0;            // relative monopole acceptance (0: off)
    DevBuf acc_ref;                // FP32 [3][acc_ref_n]: its reference accelerations
    int64_t acc_ref_n = 0;
    // lists built with the cut widened by `skin` are reused by later FP32
    // calls while every particle stays within skin / 2 of pos_ref (its
    // position, key order, when they were built)
    double skin = 0.0;
    DevBuf pos_ref;
    bool reuse_ready = false;      // the lists and pos_ref belong together
    bool lists_moved = false;      // the last pass reused the lists for moved particles
    int64_t list_builds = 0, list_reuses = 0;
    bool lists_mono = false;       // the current lists hold monopoles
    bool lists_active = false;     // the current items cover the active targets only
    pp_stats st{};
    bool lists_valid = false, evaluated_valid = false;
    bool timing = false, timed = false;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;   // around the PP kernel (or its graph)
    hipEvent_t ev2 = nullptr, ev3 = nullptr;   // around the whole PP stage
    DevBuf partial, pcount, counters, queues;
    // captured PP graph (persistent kernel + reduction)
    hipGraphExec_t gexec = nullptr;
    hipGraph_t graph = nullptr;
    hipStream_t cap_stream = nullptr;     // capture only (the null stream cannot be captured)
    uint64_t graph_gen = 0;
    const void* graph_acc = nullptr;
    const void* graph_active = nullptr;
    // the row stride of the SoA particle arrays, a kernel argument passed by
    // value (the chunk and the counts are read on the device)
    int64_t graph_n = -1;

    ~Batch() {
        if (gexec) (void)hipGraphExecDestroy(gexec);
        if (graph) (void)hipGraphDestroy(graph);
        if (ev0) (void)hipEventDestroy(ev0);
        if (ev1) (void)hipEventDestroy(ev1);
        if (ev2) (void)hipEventDestroy(ev2);
        if (ev3) (void)hipEventDestroy(ev3);
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
    }

    int init(int nb, const pp_box_params* p, const int64_t* n, bool need_poly = true) {
        if (nb < 1) return fail(PP_EINVAL, "need at least one box");
        for (int x = 0; x < nb; ++x) {
            PP_TRY(validate_params(&p[x], need_poly));
            if (n[x] < 0) return fail(PP_EINVAL, "negative particle count");
            if (p[x].key_bits != p[0].key_bits || p[x].leaf_max != p[0].leaf_max)
                return fail(PP_EINVAL, "all boxes of a batch must share key_bits and leaf_max");
        }
        int dev_count = 0;
        hipError_t e = hipGetDeviceCount(&dev_count);
        if (e != hipSuccess || dev_count == 0) {
            (void)hipGetLastError();
            return fail(PP_EDEVICE, "no HIP device available");
        }
        nbox = nb;
        params.assign(p, p + nb);
        poff.assign(nb + 1, 0);
        for (int x = 0; x < nb; ++x) poff[x + 1] = poff[x] + n[x];
        N = poff[nb];
        n_max = N;
        if (N > INT32_MAX - 4096) return fail(PP_EINVAL, "too many particles (int32 indices)");
        PP_TRY(box_dev.reserve(sizeof(BoxDev) * nb));
        PP_TRY(poff_dev.reserve(sizeof(int64_t) * (nb + 1)));
        PP_TRY(upload_boxes());
        PP_HIP(hipMemcpy(poff_dev.p, poff.data(), sizeof(int64_t) * (nb + 1), hipMemcpyHostToDevice));
        bd.box = box_dev.as<BoxDev>();
        bd.poff = poff_dev.as<int64_t>();
        bd.nbox = nb;
        bd.bits = p[0].key_bits;
        bd.leaf_max = p[0].leaf_max;
        const int64_t m = N > 0 ? N : 1;
        PP_TRY(w.keys.reserve(8 * m));
        PP_TRY(w.keys_s.reserve(8 * m));
        PP_TRY(w.iota.reserve(4 * m));
        PP_TRY(w.perm.reserve(4 * m));
        PP_TRY(w.pos_s.reserve(24 * m));
        PP_TRY(w.mass_s.reserve(4 * m));
        PP_TRY(w.bad.reserve(64));
        PP_TRY(w.misc.reserve(64));
        PP_TRY(counters.reserve(64));
        PP_TRY(queues.reserve(kQueueBytes));
        return PP_OK;
    }

    // The per-box constants, with the lists' cut widened by the skin.
    int upload_boxes() {
        std::vector<BoxDev> hb(nbox);
        for (int x = 0; x < nbox; ++x) hb[x] = make_boxdev(params[x], poff[x], poff[x + 1] - poff[x], skin);
        PP_HIP(hipMemcpy(box_dev.p, hb.data(), sizeof(BoxDev) * nbox, hipMemcpyHostToDevice));
        return PP_OK;
    }

    int set_skin(double sk) {
        if (!(std::isfinite(sk) && sk >= 0.0)) return fail(PP_EINVAL, "skin must be finite and >= 0");
        for (int x = 0; x < nbox; ++x)
            if (!(params[x].rcut + sk < 0.5 * params[x].L))
                return fail(PP_ERANGE, "rcut + skin must be < L/2");
        skin = sk;
        PP_TRY(upload_boxes());
        lists_valid = false;
        reuse_ready = false;
        return PP_OK;
    }

    // Reuse applies to the FP32 path without monopoles, with a kernel variant
    // whose source pruning uses the targets' current positions (not the
    // block boxes of the build).
    bool can_reuse() const {
        return skin > 0.0 && reuse_ready && (tune.variant & 4) == 0 && theta == 0.0 && alpha == 0.0;
    }

    // Stages shared by every entry point: keys, sort, gather, leaves, trees,
    // block lists.  Nothing is read back: the counts stay on the device until
    // finish() (see lists_to_host).
    int prepare(const double* pos, const float* mass_f, const double* mass_d, hipStream_t s,
                const uint8_t* active = nullptr) {
        lists_valid = false;
        evaluated_valid = false;
        reuse_ready = false;
        lists_moved = false;
        w.pos_n = N;
        PP_TRY(reset_sizes(w, s));
        PP_TRY(stage_keys(bd, N, pos, w, s));
        PP_TRY(stage_sort(bd, N, w, s));
        if (mass_d) PP_TRY(w.mass_sd.reserve(8 * (N > 0 ? N : 1)));
        PP_TRY(stage_gather(bd, N, pos, mass_f, mass_d, w, s));
        if (mass_f) PP_TRY(stage_mass_flags(bd, N, w, s));
        if (mass_f && !table_ready) {
            PP_TRY(launch_split_table(w, s));
            table_ready = true;
        }
        PP_TRY(stage_leaves(bd, N, w.keys_s.as<uint64_t>(), w.pos_s.as<double>(), w, s));
        PP_TRY(stage_trees(bd, N, w, s));
        // monopoles only on the FP32 path: the FP64 yardstick and the pair
        // count keep exact lists
        MonoCfg mc;
        if (mass_f != nullptr) {
            mc.theta2 = theta * theta;
            mc.alpha = alpha;
            mc.acc_ref = acc_ref.as<float>();
        }
        const bool mono = mc.on();
        if (mono && mc.alpha > 0.0 && acc_ref_n != N)
            return fail(PP_EINVAL, "the reference accelerations were given for another particle count");
        if (mono) {
            PP_TRY(stage_node_moments(bd, N, w, s));
            mc.mc = w.tree_mc.as<double4>();
        }
        PP_TRY(stage_lists(bd, poff, tune.chunk, w, s, mc, active));
        lists_mono = mono;
        lists_active = active != nullptr;
        return PP_OK;
    }

    // A pass that reuses the lists: the new positions and masses in the
    // stored key order, the equal-mass flags and the work items for the
    // given active flags; nothing else is rebuilt.
    int prepare_reuse(const double* pos, const float* mass, hipStream_t s, const uint8_t* active) {
        lists_valid = false;
        evaluated_valid = false;
        PP_TRY(reset_sizes_reuse(w, s));
        PP_TRY(stage_regather(bd, N, pos, mass, pos_ref.as<double>(), 0.5 * skin, w, s));
        PP_TRY(stage_mass_flags(bd, N, w, s));
        PP_TRY(stage_items(bd, w, s, active));
        lists_mono = false;
        lists_active = active != nullptr;
        lists_moved = true;
        return PP_OK;
    }

    // The end of a pass: reads the counts back (one synchronisation).  With
    // *again set, a buffer was too small or a reusing pass met a particle
    // that moved too far (the PP kernels did nothing), and the pass must run
    // again, with the grown capacities or rebuilt lists.
    int finish(hipStream_t s, bool* again, bool* moved = nullptr) {
        PP_TRY(lists_to_host(w, s, again, moved));
        if (*again) {
            evaluated_valid = false;
            return PP_OK;
        }
        st.n = N;
        st.nleaf = w.nleaf;
        st.nblock = w.nblock;
        st.nrange = w.nrange;
        st.nitem = w.nitem;
        st.candidates = w.candidates;
        st.interactions = -1;
        st.pp_kernel_ms = -1.0;
        lists_valid = true;
        return PP_OK;
    }

    // The FP32 short-range accelerations: prepare, PP, finish, repeated
    // while a buffer had to grow.
    int accel_f32(const double* pos, const float* mass, float* acc, hipStream_t s,
                  const uint8_t* active = nullptr) {
        for (int attempt = 0; attempt < 32; ++attempt) {
            const bool reuse = can_reuse();
            const int64_t cap_item0 = w.cap_item;
            if (reuse) PP_TRY(prepare_reuse(pos, mass, s, active));
            else PP_TRY(prepare(pos, mass, nullptr, s, active));
            PP_TRY(run_f32(acc, s));
            bool again = false, moved = false;
            PP_TRY(finish(s, &again, &moved));
            if (again) {
                // a particle moved too far: rebuild; a reusing pass that only
                // ran out of work items reuses again with more
                if (moved || !reuse) reuse_ready = false;
                continue;
            }
            if (reuse) {
                ++list_reuses;
                // the item count follows the active flags of each call: keep
                // the capacity a fuller call needed
                if (w.cap_item < cap_item0) w.cap_item = cap_item0;
            } else {
                ++list_builds;
                if (skin > 0.0 && !lists_mono) {
                    // the reference positions of the reuse test
                    PP_TRY(pos_ref.reserve(sizeof(double) * 3 * (N > 0 ? N : 1)));
                    PP_HIP(hipMemcpyAsync(pos_ref.p, w.pos_s.p, sizeof(double) * 3 * N, hipMemcpyDeviceToDevice, s));
                    reuse_ready = true;
                }
            }
            return PP_OK;
        }
        return fail(PP_ENOMEM, "the list buffers kept growing");
    }

    int run_pp_direct(float* acc, hipStream_t s) {
        unsigned long long* ctr = counters.as<unsigned long long>();
        PP_TRY(launch_reset_queues(tune.persistent ? queues.as<unsigned>() : nullptr, s, ctr));
        if (timing) PP_HIP(hipEventRecord(ev0, s));
        PP_TRY(launch_pp_f32(bd, w, tune.waves_per_block, tune.persistent ? Mode::kPersistent : Mode::kGrid,
                             tune.waves_per_cu, tune.variant, partial.as<float>(), acc, ctr,
                             queues.as<unsigned>(), s));
        if (timing) {
            PP_HIP(hipEventRecord(ev1, s));
            timed = true;
        }
        PP_TRY(launch_reduce_f32(bd, w, partial.as<float>(), acc, s));
        if (lists_mono) PP_TRY(launch_monopole(bd, w, acc, ctr + 2, s));
        evaluated_valid = true;
        return PP_OK;
    }

    // Records reset + persistent kernel + reduction on a private stream; the
    // graph is then launched on the caller's stream.  Nothing runs here.
    int capture(float* acc) {
        if (!cap_stream) PP_HIP(hipStreamCreateWithFlags(&cap_stream, hipStreamNonBlocking));
        hipStream_t s = cap_stream;
        if (gexec) {
            (void)hipGraphExecDestroy(gexec);
            gexec = nullptr;
        }
        if (graph) {
            (void)hipGraphDestroy(graph);
            graph = nullptr;
        }
        PP_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        int rc = launch_reset_queues(queues.as<unsigned>(), s);
        if (rc == PP_OK)
            rc = launch_pp_f32(bd, w, tune.waves_per_block, Mode::kPersistent, tune.waves_per_cu, tune.variant,
                               partial.as<float>(), acc, nullptr, queues.as<unsigned>(), s);
        if (rc == PP_OK) rc = launch_reduce_f32(bd, w, partial.as<float>(), acc, s);
        hipError_t e = hipStreamEndCapture(s, &graph);
        if (rc != PP_OK) return rc;
        if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture", __FILE__, __LINE__);
        PP_HIP(hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0));
        graph_gen = alloc_generation();
        graph_acc = acc;
        graph_active = w.active;
        graph_n = w.pos_n;
        graph_variant = graph_key();
        return PP_OK;
    }

    // what the captured launch depends on besides buffers: variant, waves per block and per CU
    int64_t graph_key() const {
        return ((int64_t)tune.variant << 32) | ((int64_t)tune.waves_per_block << 16) | (int64_t)tune.waves_per_cu;
    }

    // The PP stage: queue reset, PP kernel (or its graph), reduction and
    // monopoles; with timing on, events around the stage and the kernel.
    int run_f32(float* acc, hipStream_t s) {
        PP_TRY(partial.reserve(sizeof(float) * 3 * kBlock * (w.cap_item + 1)));
        if (timing) PP_HIP(hipEventRecord(ev2, s));
        PP_TRY(run_f32_stage(acc, s));
        if (timing) PP_HIP(hipEventRecord(ev3, s));
        return PP_OK;
    }

    int run_f32_stage(float* acc, hipStream_t s) {
        if (tune.persistent && tune.use_graph) {
            if (!gexec || graph_gen != alloc_generation() || graph_acc != acc ||
                graph_active != w.active || graph_variant != graph_key() || graph_n != w.pos_n)
                PP_TRY(capture(acc));
            if (timing) PP_HIP(hipEventRecord(ev0, s));
            PP_HIP(hipGraphLaunch(gexec, s));
            if (timing) {
                PP_HIP(hipEventRecord(ev1, s));
                timed = true;
            }
            if (lists_mono) PP_TRY(launch_monopole(bd, w, acc, nullptr, s));
            evaluated_valid = false;
            return PP_OK;
        }
        return run_pp_direct(acc, s);
    }

    int stats(pp_stats* out) {
        st.pp_kernel_ms = -1.0;
        st.pp_stage_ms = -1.0;
        if (timing && timed) {
            PP_HIP(hipEventSynchronize(ev3));
            float ms = 0.f;
            PP_HIP(hipEventElapsedTime(&ms, ev0, ev1));
            st.pp_kernel_ms = ms;
            PP_HIP(hipEventElapsedTime(&ms, ev2, ev3));
            st.pp_stage_ms = ms;
        }
        st.evaluated = st.lane_pairs = -1;
        st.monopoles = lists_mono ? -1 : 0;
        st.list_builds = list_builds;
        st.list_reuses = list_reuses;
        if (evaluated_valid) {
            unsigned long long h[3] = {0, 0, 0};
            PP_HIP(hipMemcpy(h, counters.p, sizeof(h), hipMemcpyDeviceToHost));
            st.evaluated = (int64_t)h[0];
            st.lane_pairs = (int64_t)h[1];
            if (lists_mono) st.monopoles = (int64_t)h[2];
        }
        *out = st;
        return PP_OK;
    }

    // Time the PP stage for the current tuning: events of its own around
    // everything run_f32 enqueues (queue reset, PP kernel or graph,
    // reduction), the same span for every launch shape; median of `reps`
    // runs after one warm run.
    int time_pp(const double* pos, const float* mass, float* acc, int reps, hipStream_t s,
                float* ms_out) {
        PP_TRY(accel_f32(pos, mass, acc, s));
        hipEvent_t a = nullptr, b = nullptr;
        PP_HIP(hipEventCreate(&a));
        hipError_t e = hipEventCreate(&b);
        if (e != hipSuccess) {
            (void)hipEventDestroy(a);
            return hip_fail(e, "hipEventCreate", __FILE__, __LINE__);
        }
        std::vector<float> t;
        int rc = PP_OK;
        for (int r = 0; r < reps && rc == PP_OK; ++r) {
            e = hipEventRecord(a, s);
            if (e == hipSuccess) rc = run_f32(acc, s);
            if (rc == PP_OK && e == hipSuccess) e = hipEventRecord(b, s);
            if (rc == PP_OK && e == hipSuccess) e = hipEventSynchronize(b);
            float ms = 0.f;
            if (rc == PP_OK && e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
            if (e != hipSuccess && rc == PP_OK) rc = hip_fail(e, "PP timing events", __FILE__, __LINE__);
            t.push_back(ms);
        }
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
        PP_TRY(rc);
        std::sort(t.begin(), t.end());
        *ms_out = t[t.size() / 2];
        return PP_OK;
    }

    std::string shape_key() const {
        int dev = 0;
        hipDeviceProp_t prop;
        std::string arch = "gpu";
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
            arch = prop.gcnArchName;
        const size_t colon = arch.find(':');
        if (colon != std::string::npos) arch = arch.substr(0, colon);
        int lg = 0;
        while ((int64_t(1) << (lg + 1)) <= (N > 0 ? N : 1)) ++lg;
        std::ostringstream k;
        k << arch << "/nbox" << nbox << "/n2^" << lg << "/leaf" << params[0].leaf_max;
        return k.str();
    }

    int autotune(const double* pos, const float* mass, float* acc, const char* cache_path,
                 hipStream_t s) {
        const std::string key = shape_key();
        // cache lookup: one line per shape, "key chunk persistent waves graph"
        if (cache_path) {
            std::ifstream in(cache_path);
            std::string line;
            while (std::getline(in, line)) {
                std::istringstream ls(line);
                std::string k;
                pp_tuning t{};
                t.variant = tune.variant;
                if (ls >> k >> t.chunk >> t.persistent >> t.waves_per_cu >> t.use_graph >> t.waves_per_block &&
                    k == key &&
                    check_tuning_ok(t)) {
                    tune = t;
                    lists_valid = false;
                    return PP_OK;
                }
            }
        }
        const bool batch = nbox > 1;
        const int variant = tune.variant;
        const bool multi = variant == 0 || variant == 8;      // K > 1 is built for these
        pp_tuning best = tune;
        float best_ms = 1e30f;
        auto trial = [&](const pp_tuning& t) -> int {
            tune = t;
            float ms = 0.f;
            PP_TRY(time_pp(pos, mass, acc, 3, s, &ms));
            if (ms < best_ms) {
                best_ms = ms;
                best = t;
            }
            return PP_OK;
        };
        // 1) the j tile: source-list positions per wave, and K waves per
        //    target block (a block's i tile of 64 targets swept by K waves),
        //    persistent at 20 waves per CU
        const int ks[] = {1, 2, 4, 8};
        for (int c : {1024, 2048, 4096})
            for (int k : ks) {
                if (k > 1 && !multi) continue;
                PP_TRY(trial(pp_tuning{c * k, 1, 20, batch ? 1 : 0, variant, k}));
            }
        // lists too short to give every SIMD several items at 1024 positions
        // per wave (small boxes): shorter j tiles too
        if (w.total_src < (int64_t)16384 * 1024)
            for (int c : {256, 512})
                for (int k : ks) {
                    if (k > 1 && !multi) continue;
                    PP_TRY(trial(pp_tuning{c * k, 1, 20, batch ? 1 : 0, variant, k}));
                }
        // 2) the launch shape at that tiling: resident waves per CU, or one
        //    workgroup per item
        const pp_tuning tiled = best;
        for (int wpc : {12, 24, 32})
            PP_TRY(trial(pp_tuning{tiled.chunk, 1, wpc, batch ? 1 : 0, variant, tiled.waves_per_block}));
        PP_TRY(trial(pp_tuning{tiled.chunk, 0, 20, 0, variant, tiled.waves_per_block}));
        tune = best;
        lists_valid = false;
        if (cache_path) {
            std::vector<std::string> keep;
            {
                std::ifstream in(cache_path);
                std::string line;
                while (std::getline(in, line))
                    if (line.compare(0, key.size() + 1, key + " ") != 0 && !line.empty()) keep.push_back(line);
            }
            std::ofstream out(cache_path, std::ios::trunc);
            if (!out) return fail(PP_EINVAL, std::string("cannot write tuning cache ") + cache_path);
            for (const std::string& l : keep) out << l << "\n";
            out << key << " " << best.chunk << " " << best.persistent << " " << best.waves_per_cu
                << " " << best.use_graph << " " << best.waves_per_block << "\n";
        }
        return PP_OK;
    }

    static bool check_tuning_ok(const pp_tuning& t) {
        return t.chunk >= 64 && t.chunk <= (1 << 24) && t.chunk % 64 == 0 && t.waves_per_cu >= 1 &&
               t.waves_per_cu <= 64 && !(t.use_graph && !t.persistent) && t.variant >= 0 &&
               t.variant <= 15 &&
               (t.waves_per_block == 1 ||
                ((t.waves_per_block == 2 || t.waves_per_block == 4 || t.waves_per_block == 8) &&
                 (t.variant == 0 || t.variant == 8)));
    }

    int set_timing(int on) {
        if (on && !ev0) {
            PP_HIP(hipEventCreate(&ev0));
            PP_HIP(hipEventCreate(&ev1));
            PP_HIP(hipEventCreate(&ev2));
            PP_HIP(hipEventCreate(&ev3));
        }
        timing = on != 0;
        timed = false;
        return PP_OK;
    }
};

static int check_tuning(const pp_tuning* t) {
    if (!t) return fail(PP_EINVAL, "tuning is NULL");
    if (t->chunk < 64 || t->chunk > (1 << 24) || (t->chunk % 64) != 0)
        return fail(PP_EINVAL, "chunk must be a multiple of 64 in 64..2^24");
    if (t->waves_per_cu < 1 || t->waves_per_cu > 64) return fail(PP_EINVAL, "waves_per_cu in 1..64");
    if (t->use_graph && !t->persistent) return fail(PP_EINVAL, "graph replay needs the persistent kernel");
    if (t->variant < 0 || t->variant > 15) return fail(PP_EINVAL, "variant must be in 0..15");
    if (t->waves_per_block != 1 && t->waves_per_block != 2 && t->waves_per_block != 4 && t->waves_per_block != 8)
        return fail(PP_EINVAL, "waves_per_block must be 1, 2, 4 or 8");
    if (t->waves_per_block > 1 && t->variant != 0 && t->variant != 8)
        return fail(PP_EINVAL, "more than one wave per block needs variant 0 or 8");
    return PP_OK;
}

}  // namespace pp

using namespace pp;

// ----------------------------------------------------------- objects --
struct pp_leaves {
    Batch b;
};

struct pp_pairs {
    int64_t nrows = 0, nentries = 0;
    DevBuf row_cnt, row_ptr, src, code, scan_ws;
};

struct pp_plan {
    Batch b;
};

struct pp_batch_plan {
    Batch b;
};

static hipStream_t S(void* s) { return reinterpret_cast<hipStream_t>(s); }

static int check_ptr(const void* p, int64_t n, const char* name) {
    if (n > 0 && !p) return fail(PP_EINVAL, std::string(name) + " is NULL");
    return PP_OK;
}

namespace {
__global__ void iota_kernel(int32_t* p, int64_t n) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) p[k] = (int32_t)k;
}
}  // namespace

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
    return launch_keys_raw(pos, n, L, key_bits, keys, S(stream));
}

int pp_sort_workspace_size(int64_t n, size_t* bytes) {
    if (!bytes) return fail(PP_EINVAL, "bytes is NULL");
    if (n < 0 || n > INT32_MAX) return fail(PP_EINVAL, "n out of range");
    size_t b = 0;
    PP_TRY(sort_workspace(n, 1, 21, &b));
    // plus the index sequence the call fills itself
    *bytes = ((b + 255) / 256) * 256 + sizeof(int32_t) * (size_t)n + 256;
    return PP_OK;
}

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
    PP_TRY(sort_workspace(n, 1, 21, &sb));
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
    PP_TRY(launch_sort_raw(keys, idx, kout, perm, n, 21, w, sb, S(stream)));
    if (!sorted_keys) PP_HIP(hipStreamSynchronize(S(stream)));   // before tmp is freed
    return PP_OK;
}

int pp_build_leaves(const uint64_t* sorted_keys, const double* pos_sorted, int64_t n,
                    const pp_box_params* p, pp_leaves** out, void* stream) {
    if (!out) return fail(PP_EINVAL, "out is NULL");
    *out = nullptr;
    if (n < 0 || n > INT32_MAX - 4096) return fail(PP_EINVAL, "n out of range");
    PP_TRY(check_ptr(sorted_keys, n, "sorted_keys"));
    PP_TRY(check_ptr(pos_sorted, n, "pos_sorted"));
    PP_TRY(validate_params(p, false));
    pp_leaves* lv = new (std::nothrow) pp_leaves;
    if (!lv) return fail(PP_ENOMEM, "host allocation failed");
    int rc = lv->b.init(1, p, &n, false);
    if (rc == PP_OK)
        rc = stage_wrap_copy(lv->b.bd, n, pos_sorted, lv->b.w.pos_s.as<double>(), S(stream));
    if (rc == PP_OK)
        rc = stage_leaves(lv->b.bd, n, sorted_keys, lv->b.w.pos_s.as<double>(), lv->b.w, S(stream));
    if (rc == PP_OK) rc = leaves_to_host(lv->b.bd, lv->b.w, S(stream));
    if (rc != PP_OK) {
        delete lv;
        return rc;
    }
    *out = lv;
    return PP_OK;
}

int pp_leaves_count(const pp_leaves* lv, int64_t* nleaf) {
    if (!lv || !nleaf) return fail(PP_EINVAL, "NULL argument");
    *nleaf = lv->b.w.nleaf;
    return PP_OK;
}

int pp_leaves_export(const pp_leaves* lv, int64_t* begin, int32_t* count, int32_t* level,
                     uint64_t* prefix, int32_t* lo, int32_t* hi) {
    if (!lv) return fail(PP_EINVAL, "leaves is NULL");
    const Work& w = lv->b.w;
    const int64_t m = w.nleaf;
    if (m == 0) return PP_OK;
    if (begin) PP_HIP(hipMemcpy(begin, w.lbegin.p, 8 * m, hipMemcpyDefault));
    if (count) PP_HIP(hipMemcpy(count, w.lcount.p, 4 * m, hipMemcpyDefault));
    if (level) PP_HIP(hipMemcpy(level, w.llevel.p, 4 * m, hipMemcpyDefault));
    if (prefix) PP_HIP(hipMemcpy(prefix, w.lprefix.p, 8 * m, hipMemcpyDefault));
    if (lo || hi) {
        std::vector<IBox> hb(m);
        PP_HIP(hipMemcpy(hb.data(), w.tree_boxes.p, sizeof(IBox) * m, hipMemcpyDeviceToHost));
        std::vector<int32_t> t(3 * m);
        for (int k = 0; k < 2; ++k) {
            int32_t* dst = k == 0 ? lo : hi;
            if (!dst) continue;
            for (int64_t a = 0; a < m; ++a)
                for (int ax = 0; ax < 3; ++ax) t[ax * m + a] = k == 0 ? hb[a].lo[ax] : hb[a].hi[ax];
            PP_HIP(hipMemcpy(dst, t.data(), 4 * 3 * m, hipMemcpyDefault));
        }
    }
    return PP_OK;
}

void pp_leaves_free(pp_leaves* lv) { delete lv; }

int pp_near_pairs(pp_leaves* lv, const pp_box_params* p, pp_pairs** out, void* stream) {
    if (!out) return fail(PP_EINVAL, "out is NULL");
    *out = nullptr;
    if (!lv) return fail(PP_EINVAL, "leaves is NULL");
    PP_TRY(validate_params(p, false));
    const pp_box_params& lp = lv->b.params[0];
    if (p->key_bits != lp.key_bits || p->L != lp.L)
        return fail(PP_EINVAL, "params do not match the leaves (L, key_bits)");
    pp_pairs* pr = new (std::nothrow) pp_pairs;
    if (!pr) return fail(PP_ENOMEM, "host allocation failed");
    const BoxDev g = make_boxdev(*p, 0, lv->b.N);
    int rc = stage_trees(lv->b.bd, lv->b.N, lv->b.w, S(stream));
    if (rc == PP_OK) rc = trees_to_host(lv->b.bd, lv->b.w, S(stream));
    if (rc == PP_OK)
        rc = build_canonical_pairs(lv->b.bd, lv->b.w, g.W, g.T, pr->row_cnt, pr->row_ptr, pr->src,
                                   pr->code, pr->scan_ws, &pr->nentries, S(stream));
    if (rc == PP_OK) {
        hipError_t e = hipStreamSynchronize(S(stream));
        if (e != hipSuccess) rc = hip_fail(e, "hipStreamSynchronize", __FILE__, __LINE__);
    }
    if (rc != PP_OK) {
        delete pr;
        return rc;
    }
    pr->nrows = lv->b.w.nleaf;
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

// ---------------------------------------------------------------- plans --
int pp_plan_create(const pp_box_params* p, int64_t n_max, pp_plan** out) {
    if (!out) return fail(PP_EINVAL, "out is NULL");
    *out = nullptr;
    PP_TRY(validate_params(p, true));
    if (n_max < 0 || n_max > INT32_MAX - 4096) return fail(PP_EINVAL, "n_max out of range");
    pp_plan* pl = new (std::nothrow) pp_plan;
    if (!pl) return fail(PP_ENOMEM, "host allocation failed");
    int rc = pl->b.init(1, p, &n_max);
    if (rc != PP_OK) {
        delete pl;
        return rc;
    }
    *out = pl;
    return PP_OK;
}

void pp_plan_destroy(pp_plan* plan) { delete plan; }

// A plan holds one box of up to n_max particles; a call with n < n_max
// describes the box again with n particles.
static int plan_resize(pp_plan* pl, int64_t n) {
    Batch& b = pl->b;
    if (b.poff[1] == n) return PP_OK;
    b.poff[1] = n;
    b.N = n;
    const BoxDev hb = make_boxdev(b.params[0], 0, n);
    PP_HIP(hipMemcpy(b.box_dev.p, &hb, sizeof(BoxDev), hipMemcpyHostToDevice));
    PP_HIP(hipMemcpy(b.poff_dev.p, b.poff.data(), sizeof(int64_t) * 2, hipMemcpyHostToDevice));
    return PP_OK;
}

static int check_accel_args(pp_plan* pl, const void* pos, const void* mass, int64_t n,
                            const void* acc) {
    if (!pl) return fail(PP_EINVAL, "plan is NULL");
    if (n < 0 || n > pl->b.n_max) return fail(PP_EINVAL, "n must be in 0..n_max of the plan");
    PP_TRY(check_ptr(pos, n, "pos"));
    PP_TRY(check_ptr(mass, n, "mass"));
    PP_TRY(check_ptr(acc, n, "acc"));
    return PP_OK;
}

int pp_accel(pp_plan* pl, const double* pos, const float* mass, int64_t n, float* acc,
             void* stream) {
    PP_TRY(check_accel_args(pl, pos, mass, n, acc));
    if (n == 0) return PP_OK;
    PP_TRY(plan_resize(pl, n));
    return pl->b.accel_f32(pos, mass, acc, S(stream));
}

// ------------------------------------------------- allocation-free path --
// Every buffer of pp_accel_scratch comes from one static device array of
// kScratchBytes (each device holds its own copy until the process ends).  In
// host code `scratch` is only a host-side stand-in: the device address is
// taken once per device with hipGetSymbolAddress, with that device current,
// and only that address reaches kernels and copies.
constexpr size_t kScratchBytes = (size_t)64 << 20;
constexpr int64_t kScratchMaxN = 65536;
constexpr int kScratchDevices = 64;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
static std::mutex g_scratch_mu[kScratchDevices];
static char* g_scratch_ptr[kScratchDevices];

// The device address of this device's scratch (g_scratch_mu[dev] held, dev current).
static int scratch_address(int dev, char** out) {
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)", __FILE__, __LINE__);
        if (!ptr) return fail(PP_EDEVICE, "hipGetSymbolAddress(scratch) gave no address");
        g_scratch_ptr[dev] = static_cast<char*>(ptr);
    }
    *out = g_scratch_ptr[dev];
    return PP_OK;
}

int pp_accel_active(pp_plan* pl, const double* pos, const float* mass, int64_t n,
                    const uint8_t* active, float* acc, void* stream) {
    PP_TRY(check_accel_args(pl, pos, mass, n, acc));
    PP_TRY(check_ptr(active, n, "active"));
    if (n == 0) return PP_OK;
    PP_TRY(plan_resize(pl, n));
    return pl->b.accel_f32(pos, mass, acc, S(stream), active);
}

int pp_accel_scratch(const pp_box_params* p, const double* pos, const float* mass, int64_t n,
                     float* acc, void* stream) {
    PP_TRY(validate_params(p, true));
    if (n < 0 || n > kScratchMaxN)
        return fail(PP_EINVAL, "pp_accel_scratch takes at most 65536 particles (the static scratch)");
    PP_TRY(check_ptr(pos, n, "pos"));
    PP_TRY(check_ptr(mass, n, "mass"));
    PP_TRY(check_ptr(acc, n, "acc"));
    if (n == 0) return PP_OK;
    int dev = 0;
    PP_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kScratchDevices) return fail(PP_EDEVICE, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu[dev]);
    char* base = nullptr;
    PP_TRY(scratch_address(dev, &base));
    Arena arena{base, kScratchBytes, 0};
    ScratchScope scope(&arena);
    hipStream_t s = S(stream);
    // the list capacities of the last attempt (a pass that overflowed runs
    // again, every buffer carved afresh from the start of the array)
    int64_t cap_block = 0, cap_range = 0, cap_item = 0;
    int64_t cap_ent[kMaxPasses] = {};
    bool stop2 = false;
    for (int attempt = 0; attempt < 32; ++attempt) {
        arena.used = 0;
        Batch b;
        PP_TRY(b.init(1, p, &n));
        b.w.cap_block = cap_block;
        b.w.cap_range = cap_range;
        b.w.cap_item = cap_item;
        for (int k = 0; k < kMaxPasses; ++k) b.w.cap_ent[k] = cap_ent[k];
        b.w.stop_at_level2 = stop2;
        PP_TRY(b.prepare(pos, mass, nullptr, s));
        PP_TRY(b.run_f32(acc, s));
        bool again = false;
        PP_TRY(b.finish(s, &again));
        if (!again) return PP_OK;
        cap_block = b.w.cap_block;
        cap_range = b.w.cap_range;
        cap_item = b.w.cap_item;
        for (int k = 0; k < kMaxPasses; ++k) cap_ent[k] = b.w.cap_ent[k];
        stop2 = b.w.stop_at_level2;
    }
    return fail(PP_ENOMEM, "the list buffers kept growing");
}

int pp_accel_f64(pp_plan* pl, const double* pos, const double* mass, int64_t n, double* acc,
                 void* stream) {
    PP_TRY(check_accel_args(pl, pos, mass, n, acc));
    if (n == 0) return PP_OK;
    PP_TRY(plan_resize(pl, n));
    hipStream_t s = S(stream);
    Batch& b = pl->b;
    for (int attempt = 0; attempt < 32; ++attempt) {
        PP_TRY(b.prepare(pos, nullptr, mass, s));
        PP_TRY(b.partial.reserve(sizeof(double) * 3 * kBlock * (b.w.cap_item + 1)));
        if (b.timing) PP_HIP(hipEventRecord(b.ev2, s));
        if (b.timing) PP_HIP(hipEventRecord(b.ev0, s));
        PP_TRY(launch_pp_f64(b.bd, b.w, reinterpret_cast<double*>(b.partial.p), s));
        if (b.timing) {
            PP_HIP(hipEventRecord(b.ev1, s));
            b.timed = true;
        }
        PP_TRY(launch_reduce_f64(b.bd, b.w, reinterpret_cast<double*>(b.partial.p), acc, s));
        if (b.timing) PP_HIP(hipEventRecord(b.ev3, s));
        bool again = false;
        PP_TRY(b.finish(s, &again));
        if (!again) return PP_OK;
    }
    return fail(PP_ENOMEM, "the list buffers kept growing");
}

int pp_plan_set_monopole(pp_plan* pl, double theta) {
    if (!pl) return fail(PP_EINVAL, "plan is NULL");
    if (!(theta >= 0.0 && theta < 1.0)) return fail(PP_EINVAL, "theta must be in [0, 1)");
    pl->b.theta = theta;
    pl->b.lists_valid = false;
    return PP_OK;
}

int pp_plan_set_skin(pp_plan* pl, double skin) {
    if (!pl) return fail(PP_EINVAL, "plan is NULL");
    return pl->b.set_skin(skin);
}

int pp_plan_set_monopole_relative(pp_plan* pl, double alpha, const float* acc_ref, int64_t n,
                                  void* stream) {
    if (!pl) return fail(PP_EINVAL, "plan is NULL");
    if (!(alpha >= 0.0) || !std::isfinite(alpha)) return fail(PP_EINVAL, "alpha must be finite and >= 0");
    Batch& b = pl->b;
    if (alpha > 0.0) {
        if (!acc_ref) return fail(PP_EINVAL, "acc_ref is NULL");
        if (n < 1 || n > b.n_max) return fail(PP_EINVAL, "n must be in 1..the plan's capacity");
        PP_TRY(b.acc_ref.reserve(sizeof(float) * 3 * n));
        PP_HIP(hipMemcpyAsync(b.acc_ref.p, acc_ref, sizeof(float) * 3 * n, hipMemcpyDeviceToDevice,
                              (hipStream_t)stream));
        b.acc_ref_n = n;
    } else {
        b.acc_ref_n = 0;
    }
    b.alpha = alpha;
    b.lists_valid = false;
    return PP_OK;
}

int pp_plan_stats(pp_plan* pl, pp_stats* out) {
    if (!pl || !out) return fail(PP_EINVAL, "NULL argument");
    return pl->b.stats(out);
}

int pp_plan_set_timing(pp_plan* pl, int on) {
    if (!pl) return fail(PP_EINVAL, "plan is NULL");
    return pl->b.set_timing(on);
}

int pp_plan_get_tuning(const pp_plan* pl, pp_tuning* t) {
    if (!pl || !t) return fail(PP_EINVAL, "NULL argument");
    *t = pl->b.tune;
    return PP_OK;
}

int pp_plan_set_tuning(pp_plan* pl, const pp_tuning* t) {
    if (!pl) return fail(PP_EINVAL, "plan is NULL");
    PP_TRY(check_tuning(t));
    pl->b.tune = *t;
    pl->b.lists_valid = false;
    pl->b.reuse_ready = false;
    return PP_OK;
}

static int lists_size(const Batch& b, int64_t* nblock, int64_t* nrange) {
    if (!b.lists_valid) return fail(PP_EINVAL, "no lists: call the accel function first");
    if (nblock) *nblock = b.w.nblock;
    if (nrange) *nrange = b.w.nrange;
    return PP_OK;
}

static int lists_export(const Batch& b, int32_t* perm, int32_t* bstart, int32_t* bcount, int32_t* blo,
                        int32_t* bhi, int64_t* roff, int32_t* slen, int32_t* rbeg, int32_t* rpre,
                        uint8_t* rcode) {
    PP_TRY(lists_size(b, nullptr, nullptr));
    const Work& w = b.w;
    const int64_t nb = w.nblock, nr = w.nrange, n = w.pos_n;
    PP_HIP(hipDeviceSynchronize());
    if (perm && n > 0) PP_HIP(hipMemcpy(perm, w.perm.p, 4 * n, hipMemcpyDefault));
    if (nb > 0) {
        if (bstart) PP_HIP(hipMemcpy(bstart, w.bstart.p, 4 * nb, hipMemcpyDefault));
        if (bcount) PP_HIP(hipMemcpy(bcount, w.bcount.p, 4 * nb, hipMemcpyDefault));
        if (slen) PP_HIP(hipMemcpy(slen, w.slen.p, 4 * nb, hipMemcpyDefault));
        if (blo || bhi) {
            std::vector<IBox> hb(nb);
            PP_HIP(hipMemcpy(hb.data(), w.bbox.p, sizeof(IBox) * nb, hipMemcpyDeviceToHost));
            std::vector<int32_t> t(3 * nb);
            for (int k = 0; k < 2; ++k) {
                int32_t* dst = k == 0 ? blo : bhi;
                if (!dst) continue;
                for (int64_t x = 0; x < nb; ++x)
                    for (int ax = 0; ax < 3; ++ax) t[ax * nb + x] = k == 0 ? hb[x].lo[ax] : hb[x].hi[ax];
                PP_HIP(hipMemcpy(dst, t.data(), 4 * 3 * nb, hipMemcpyDefault));
            }
        }
    }
    if (roff) PP_HIP(hipMemcpy(roff, w.roff.p, 8 * (nb + 1), hipMemcpyDefault));
    if (nr > 0) {
        if (rbeg) PP_HIP(hipMemcpy(rbeg, w.rbeg.p, 4 * nr, hipMemcpyDefault));
        if (rpre) PP_HIP(hipMemcpy(rpre, w.rpre.p, 4 * nr, hipMemcpyDefault));
        if (rcode) PP_HIP(hipMemcpy(rcode, w.rcode.p, nr, hipMemcpyDefault));
    }
    return PP_OK;
}

static int count_interactions(Batch& b, int64_t* counts, int64_t* total, hipStream_t s) {
    if (!b.lists_valid) return fail(PP_EINVAL, "no lists: call the accel function first");
    if (b.lists_mono)
        return fail(PP_EINVAL, "the lists hold monopoles: count after pp_accel_f64 or with theta 0");
    if (b.lists_active)
        return fail(PP_EINVAL, "the lists cover the active targets only: count after pp_accel or pp_accel_f64");
    if (b.lists_moved)
        return fail(PP_EINVAL, "the lists were reused for moved particles: count after pp_accel_f64");
    PP_TRY(b.pcount.reserve(sizeof(int32_t) * kBlock * (b.w.cap_item + 1)));
    PP_TRY(launch_count(b.bd, b.w, b.pcount.as<int32_t>(), s));
    unsigned long long* tot = b.w.misc.as<unsigned long long>() + 4;
    PP_HIP(hipMemsetAsync(tot, 0, sizeof(unsigned long long), s));
    PP_TRY(launch_reduce_count(b.bd, b.w, b.pcount.as<int32_t>(), counts, tot, s));
    unsigned long long h = 0;
    PP_HIP(hipMemcpyAsync(&h, tot, sizeof(h), hipMemcpyDeviceToHost, s));
    PP_HIP(hipStreamSynchronize(s));
    *total = (int64_t)h;
    b.st.interactions = (int64_t)h;
    return PP_OK;
}

int pp_plan_lists_size(const pp_plan* pl, int64_t* nblock, int64_t* nrange) {
    if (!pl) return fail(PP_EINVAL, "plan is NULL");
    return lists_size(pl->b, nblock, nrange);
}

int pp_plan_lists_export(const pp_plan* pl, int32_t* perm, int32_t* bstart, int32_t* bcount,
                         int32_t* blo, int32_t* bhi, int64_t* roff, int32_t* slen, int32_t* rbeg,
                         int32_t* rpre, uint8_t* rcode) {
    if (!pl) return fail(PP_EINVAL, "plan is NULL");
    return lists_export(pl->b, perm, bstart, bcount, blo, bhi, roff, slen, rbeg, rpre, rcode);
}

int pp_count_interactions(pp_plan* pl, int64_t* counts, int64_t* total, void* stream) {
    if (!pl || !total) return fail(PP_EINVAL, "NULL argument");
    return count_interactions(pl->b, counts, total, S(stream));
}

// -------------------------------------------------------------- batches --
int pp_batch_plan_create(int nbox, const pp_box_params* params, const int64_t* n,
                         pp_batch_plan** out) {
    if (!out) return fail(PP_EINVAL, "out is NULL");
    *out = nullptr;
    if (nbox < 1 || nbox > 65536) return fail(PP_EINVAL, "nbox must be in 1..65536");
    if (!params || !n) return fail(PP_EINVAL, "params or n is NULL");
    pp_batch_plan* bp = new (std::nothrow) pp_batch_plan;
    if (!bp) return fail(PP_ENOMEM, "host allocation failed");
    bp->b.tune.persistent = 1;
    bp->b.tune.use_graph = 1;
    int rc = bp->b.init(nbox, params, n);
    if (rc != PP_OK) {
        delete bp;
        return rc;
    }
    *out = bp;
    return PP_OK;
}

void pp_batch_plan_destroy(pp_batch_plan* bp) { delete bp; }

int pp_batch_accel(pp_batch_plan* bp, const double* pos, const float* mass, float* acc,
                   void* stream) {
    if (!bp) return fail(PP_EINVAL, "plan is NULL");
    Batch& b = bp->b;
    PP_TRY(check_ptr(pos, b.N, "pos"));
    PP_TRY(check_ptr(mass, b.N, "mass"));
    PP_TRY(check_ptr(acc, b.N, "acc"));
    if (b.N == 0) return PP_OK;
    return b.accel_f32(pos, mass, acc, S(stream));
}

int pp_batch_count_interactions(pp_batch_plan* bp, int64_t* counts, int64_t* total, void* stream) {
    if (!bp || !total) return fail(PP_EINVAL, "NULL argument");
    return count_interactions(bp->b, counts, total, S(stream));
}

int pp_batch_stats(pp_batch_plan* bp, pp_stats* out) {
    if (!bp || !out) return fail(PP_EINVAL, "NULL argument");
    return bp->b.stats(out);
}

int pp_batch_set_timing(pp_batch_plan* bp, int on) {
    if (!bp) return fail(PP_EINVAL, "plan is NULL");
    return bp->b.set_timing(on);
}

int pp_batch_get_tuning(const pp_batch_plan* bp, pp_tuning* t) {
    if (!bp || !t) return fail(PP_EINVAL, "NULL argument");
    *t = bp->b.tune;
    return PP_OK;
}

int pp_autotune(pp_plan* pl, const double* pos, const float* mass, int64_t n, const char* cache_path,
                void* stream) {
    if (!pl) return fail(PP_EINVAL, "plan is NULL");
    if (n <= 0 || n > pl->b.n_max) return fail(PP_EINVAL, "n must be in 1..n_max of the plan");
    PP_TRY(check_ptr(pos, n, "pos"));
    PP_TRY(check_ptr(mass, n, "mass"));
    PP_TRY(plan_resize(pl, n));
    DevBuf acc;
    PP_TRY(acc.reserve(sizeof(float) * 3 * n));
    return pl->b.autotune(pos, mass, acc.as<float>(), cache_path, S(stream));
}

int pp_batch_autotune(pp_batch_plan* bp, const double* pos, const float* mass,
                      const char* cache_path, void* stream) {
    if (!bp) return fail(PP_EINVAL, "plan is NULL");
    if (bp->b.N == 0) return PP_OK;
    PP_TRY(check_ptr(pos, bp->b.N, "pos"));
    PP_TRY(check_ptr(mass, bp->b.N, "mass"));
    DevBuf acc;
    PP_TRY(acc.reserve(sizeof(float) * 3 * bp->b.N));
    return bp->b.autotune(pos, mass, acc.as<float>(), cache_path, S(stream));
}

int pp_batch_set_tuning(pp_batch_plan* bp, const pp_tuning* t) {
    if (!bp) return fail(PP_EINVAL, "plan is NULL");
    PP_TRY(check_tuning(t));
    bp->b.tune = *t;
    bp->b.lists_valid = false;
    return PP_OK;
}

}  // extern "C"
