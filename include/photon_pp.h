/*
 * photon_pp — short-range particle-particle (PP) gravity on one MI355X GPU.
 *
 * The hot path of a PM + Tree + PP N-body solver (Wang et al. 2018,
 * "PHoToNs", arXiv:1802.09824): for every particle i of a periodic box,
 *
 *   a_i = sum_{j != i, s_ij < r_cut}  G m_j d_ij g(s_eps / (2 r_s)) / s_eps^3
 *
 * with d_ij = x_j - x_i at the minimum periodic image, s = |d_ij|,
 * s_eps = sqrt(s^2 + eps^2) (Plummer softening), and g the short-range factor
 * of the Gaussian PM split, sec. 3.1 Eq. (equ:split):
 *   g(x) = erfc(x) + (2 x / sqrt(pi)) exp(-x^2).
 * The pairs are found the way sec. 3.2-3.3 organise them: particles are
 * sorted along a Peano-Hilbert curve (sec. 4.1) so every octree node is one
 * contiguous run (sec. 3.2), leaves are nodes of at most leaf_max particles
 * (sec. 3.3, "a leaf is a package"), and the PP kernel runs over near
 * leaf pairs (the N-to-M case of the dual tree traversal, sec. 3.3).
 *
 * Conventions for every call:
 *  - return value: PP_OK (0) or a negative pp_status; nothing throws;
 *    pp_last_error() returns a message for the calling thread's last error.
 *  - buffers: device pointers owned by the caller, unless stated otherwise.
 *    Export calls accept host or device destinations.
 *  - layout: positions and accelerations are SoA [3][n] (x block, then y,
 *    then z), float64 positions, float32 masses/accelerations (float64 for
 *    the _f64 calls).
 *  - stream: a hipStream_t passed as void* (NULL = the null stream).  Work
 *    is enqueued on it.  Calls that must size library-owned buffers read a
 *    count back and therefore synchronise that stream; each says so.
 *  - objects: the library owns pp_leaves, pp_pairs, pp_plan and
 *    pp_batch_plan; free them with the matching *_free / *_destroy.
 *  - one object must not be used from two threads at once.
 */
#ifndef PHOTON_PP_H
#define PHOTON_PP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum pp_status {
    PP_OK = 0,
    PP_EINVAL = -1,     /* bad argument (size, pointer, parameter, NaN/Inf input) */
    PP_ENOMEM = -2,     /* device or host allocation failed */
    PP_EDEVICE = -3,    /* HIP runtime error (no device, launch failure, ...) */
    PP_ERANGE = -4,     /* parameter outside the supported range (e.g. r_cut >= L/2) */
    PP_EOVERFLOW = -5   /* caller buffer too small; the needed size is reported */
} pp_status;

/* Per-box parameters.  Lengths in any unit, consistent with the positions.
 *  L        periodic box side, > 0
 *  rs       split scale r_s of the PM/PP force split (sec. 3.1), > 0
 *  rcut     hard cut radius of the short-range sum, 0 < rcut < L/2 (so one
 *           periodic image at most lies within it); sec. 3.1 uses 4.5 r_s.
 *           The FP32 kernel's split-factor polynomial covers
 *           sqrt(rcut^2 + eps^2) <= 4.52 r_s; beyond that PP_ERANGE.
 *  eps      Plummer softening length, >= 0
 *  G        gravitational constant (any finite value)
 *  leaf_max maximum particles per octree leaf, 1..1024 (a leaf at the
 *           finest key level may hold more: its particles share a cell)
 *  key_bits bits per axis of the Peano-Hilbert grid, 1..21               */
typedef struct pp_box_params {
    double L, rs, rcut, eps, G;
    int32_t leaf_max, key_bits;
} pp_box_params;

typedef struct pp_leaves pp_leaves;
typedef struct pp_pairs pp_pairs;
typedef struct pp_plan pp_plan;
typedef struct pp_batch_plan pp_batch_plan;

/* Peano-Hilbert keys, sec. 4.1 (a 2^(3b) grid labelled along the curve).
 * Each coordinate is wrapped, w = x - L floor(x / L), and quantised,
 * q = floor(w * (2^b / L)) clamped to [0, 2^b - 1]; the key is the index of
 * cell q along J. Skilling's Hilbert curve ("Programming the Hilbert
 * curve", 2004), x taking the most significant bit of every 3-bit digit.
 *   pos   device SoA [3][n] float64;  keys  device [n] uint64 (out)
 * Errors: PP_EINVAL for n < 0, NULL pointers with n > 0, L <= 0, b out of
 * 1..21.  Asynchronous.                                                   */
int pp_hilbert_keys(const double* pos, int64_t n, double L, int key_bits,
                    uint64_t* keys, void* stream);

/* Scratch bytes pp_sort_by_key needs for n keys. */
int pp_sort_workspace_size(int64_t n, size_t* bytes);

/* Stable sort by key (sec. 3.2: all particles of a tree node become one
 * contiguous run).  Equal keys keep their input order, so the order is by
 * (key, index).  perm[k] is the input index of the k-th particle in key
 * order; sorted_keys (may be NULL) receives keys[perm[k]].
 *   keys device [n] uint64; perm device [n] int32 (out); ws device scratch
 *   of at least pp_sort_workspace_size(n) bytes.
 * Errors: PP_EINVAL (n < 0 or n > 2^31 - 1, NULL pointers), PP_EOVERFLOW
 * if ws_bytes is too small.  Asynchronous.                                 */
int pp_sort_by_key(const uint64_t* keys, int64_t n, int32_t* perm, uint64_t* sorted_keys,
                   void* ws, size_t ws_bytes, void* stream);

/* Octree leaves (sec. 3.2-3.3): maximal octree nodes holding at most
 * leaf_max particles, each a contiguous run of the key-sorted particles.
 * A node at level l is the set of particles sharing the top 3 l key bits.
 *   sorted_keys  device [n] uint64, ascending
 *   pos_sorted   device SoA [3][n] float64, the same particles in key order
 *                (used for the integer bounding boxes)
 *   p            box parameters (L, key_bits, leaf_max are used)
 *   out          receives a library-owned pp_leaves
 * Synchronises the stream (reads the leaf count back).
 * Errors: PP_EINVAL (bad sizes/params), PP_ENOMEM, PP_EDEVICE.             */
int pp_build_leaves(const uint64_t* sorted_keys, const double* pos_sorted, int64_t n,
                    const pp_box_params* p, pp_leaves** out, void* stream);
int pp_leaves_count(const pp_leaves* lv, int64_t* nleaf);
/* Copy the leaf table out (host or device destinations; any may be NULL):
 * begin [m] int64, count [m] int32, level [m] int32, prefix [m] uint64 (the
 * top 3*level key bits), lo/hi [3][m] int32 integer bounding box of the
 * particles' grid cells, hi exclusive (max q + 1).  Synchronous.           */
int pp_leaves_export(const pp_leaves* lv, int64_t* begin, int32_t* count, int32_t* level,
                     uint64_t* prefix, int32_t* lo, int32_t* hi);
void pp_leaves_free(pp_leaves* lv);

/* Near leaf pairs: the N-to-M leaf pairs of the dual tree traversal
 * (sec. 3.3) restricted to the short range.  In grid units (the box is
 * W = 2^b cells wide) target leaf A, source leaf B and periodic shift
 * s in {-1,0,1}^3 form a pair iff
 *   sum_k max(0, lo_B,k + s_k W - hi_A,k, lo_A,k - hi_B,k - s_k W)^2 < T,
 *   T = ceil(r^2),  r = rcut * W / L  (FP64, this operation order).
 * Every particle pair closer than rcut therefore appears.  Rows are target
 * leaves in key order; within a row entries ascend by (B, code) with
 * code = 9 (s_x + 1) + 3 (s_y + 1) + (s_z + 1).
 * Synchronises the stream (reads the entry count back).                    */
int pp_near_pairs(pp_leaves* lv, const pp_box_params* p, pp_pairs** out, void* stream);
int pp_pairs_count(const pp_pairs* pr, int64_t* nrows, int64_t* nentries);
/* Copy the canonical CSR out: row_ptr [nrows + 1] int64, src_leaf
 * [nentries] int32, shift_code [nentries] uint8.  Synchronous.             */
int pp_pairs_export(const pp_pairs* pr, int64_t* row_ptr, int32_t* src_leaf, uint8_t* shift_code);
void pp_pairs_free(pp_pairs* pr);

/* A plan validates the parameters, owns all scratch memory for boxes of
 * up to n_max particles and holds the kernel tiling.
 * Errors: PP_EINVAL / PP_ERANGE for parameters, PP_ENOMEM, PP_EDEVICE.     */
int pp_plan_create(const pp_box_params* p, int64_t n_max, pp_plan** out);
void pp_plan_destroy(pp_plan* plan);

/* Short-range accelerations (the whole path: keys, sort, leaves, near
 * lists, FP32 PP kernel, scatter back to input order).
 *   pos  device SoA [3][n] float64, input order, any values (wrapped)
 *   mass device [n] float32;  acc device SoA [3][n] float32 (out)
 * Arithmetic: positions relative to a per-block FP64 origin are rounded to
 * FP32; pair arithmetic is FP32 with a compensated per-target sum.
 * Synchronises the stream (list sizes).  PP_EINVAL for n > n_max, NaN/Inf
 * positions or masses.                                                     */
int pp_accel(pp_plan* plan, const double* pos, const float* mass, int64_t n, float* acc,
             void* stream);

/* pp_accel for the targets whose flag active[i] (device uint8 [n], input
 * order) is non-zero; acc[:, i] of the other targets is not written.  All n
 * particles are sources.  The active targets get exactly pp_accel's values
 * (the same lists, work items and summation order); the work saved is that
 * of the 64-particle target blocks (in key order) without an active target.
 * This is the force evaluation of the block time steps of sec. 3.4, where
 * only the particles whose step ends need new forces.  Synchronises the
 * stream like pp_accel.  pp_count_interactions refuses lists built by this
 * call (PP_EINVAL).  Errors as pp_accel, and PP_EINVAL for a NULL active
 * with n > 0. */
int pp_accel_active(pp_plan* plan, const double* pos, const float* mass, int64_t n,
                    const uint8_t* active, float* acc, void* stream);
/* pp_accel without any allocation, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  No plan: one box of p with at most 65536 particles,
 * the default tuning of a plan, every device buffer carved from one static
 * device array of 64 MiB that each device holds until the process ends (no
 * hipMalloc, hipFree or allocating library call; host bookkeeping only).
 * The results are those of pp_accel on a plan with the default tuning.
 * The array is shared by all calls on a device and keeps the last call's
 * contents (every buffer is written before it is read); calls on one device
 * from several host threads are serialised by a lock (unsynchronised they
 * would race on the array).  Synchronises the stream.
 * Errors: as pp_accel; PP_EINVAL for n > 65536; PP_ENOMEM when the input's
 * lists need more than the 64 MiB (possible for very clustered inputs near
 * the particle limit). */
int pp_accel_scratch(const pp_box_params* p, const double* pos, const float* mass, int64_t n,
                     float* acc, void* stream);
/* The same sum entirely in FP64 (accuracy yardstick).                     */
int pp_accel_f64(pp_plan* plan, const double* pos, const double* mass, int64_t n, double* acc,
                 void* stream);

/* Figures of the last pp_accel / pp_accel_f64 / pp_count_interactions call. */
typedef struct pp_stats {
    int64_t n, nleaf, nblock, nrange, nitem;
    int64_t candidates;     /* (target, listed source) pairs of the block lists */
    int64_t evaluated;      /* pairs the FP32 kernel evaluated (listed sources that survive
                               its bounding-box test, incl. pairs masked by the cut); -1 if
                               the last call was not pp_accel */
    int64_t lane_pairs;     /* lane-pair slots the FP32 kernel swept (64 per staged source,
                               idle lanes of partly filled blocks included); -1 likewise */
    int64_t interactions;   /* pairs with s < rcut, j != i (set by pp_count_interactions), else -1 */
    double pp_kernel_ms;    /* duration of the last PP kernel launch (HIP events on the
                               caller's stream) when timing is on, else -1 */
    int64_t monopoles;      /* (target, monopole) pairs of the last pp_accel with
                               monopole acceptance on (0 when off, -1 if unknown) */
    double pp_stage_ms;     /* the whole PP stage of that call (queue reset, kernel or
                               graph, reduction, monopoles) when timing is on, else -1 */
    int64_t list_builds;    /* FP32 calls (pp_accel, pp_accel_active) that built the lists */
    int64_t list_reuses;    /* FP32 calls that reused them (pp_plan_set_skin) */
} pp_stats;
/* Waits for the last PP kernel when timing is on.                          */
/* Monopole acceptance (sec. 3.3, the 1-to-N case of the dual tree walk) for
 * pp_accel on this plan.  The target block is kept (the policy sec. 3.3
 * takes on MIC) and the source tree is opened: a source node of any level
 * (a single leaf, a group of 8 consecutive leaves, or larger) whose box
 * satisfies (A + B) / R <= theta against the target block (A, B the longest
 * box sides, R the distance of the box centres; this implies
 * B / (R - A) <= theta) acts through its mass at its centre of mass, with
 * the same softened, split, cut pair force, instead of through its
 * particles.  theta = 0 (the default) keeps the exact pair sums; 0 <= theta
 * < 1.  Only the FP32 pp_accel uses it: pp_accel_f64 stays exact, and
 * pp_count_interactions refuses lists built with monopoles (PP_EINVAL). */
int pp_plan_set_monopole(pp_plan* plan, double theta);
/* Gadget-2's relative opening criterion (sec. 3.1) for the same monopole
 * acceptance: a node of mass M is taken only if G M B^2 / r^4 <= alpha |a|,
 * with B its longest box side, r the gap between its box and the target
 * block's box (0 for touching boxes, which are therefore always opened) and
 * |a| the smallest reference acceleration among the block's targets.
 * acc_ref: device FP32 [3][n] (x row, y row, z row) in input order, for
 * instance the accelerations of the previous step; it is copied on `stream`
 * (the caller may free it once the stream reaches this point) and must
 * describe the n particles of the following pp_accel calls (PP_EINVAL
 * otherwise).  When theta > 0 as well, a node must pass both tests.
 * alpha = 0 turns the test off (acc_ref may then be NULL).  Errors:
 * PP_EINVAL for alpha < 0 or non-finite, NULL acc_ref with alpha > 0, n
 * outside 1..the plan's capacity. */
int pp_plan_set_monopole_relative(pp_plan* plan, double alpha, const float* acc_ref, int64_t n,
                                  void* stream);
/* List reuse between calls on moving particles (for a time integrator's
 * substeps, sec. 3.4).  With skin > 0 the near lists are built with the cut
 * widened to rcut + skin (a length), and a later pp_accel or pp_accel_active
 * on the plan reuses them, without keys, sort, leaves or lists, while every
 * particle (same index in the input arrays) lies within skin / 2 of its
 * position at the last build (minimum image): no pair within rcut can then
 * be missing from them, and the pair test still uses rcut, so the forces are
 * those of a fresh build up to FP32 summation order.  A call that finds a
 * particle further away rebuilds the lists (one extra pass) and makes the
 * new positions the reference.  Reuse needs monopole acceptance off and a
 * kernel variant that prunes sources against the targets' current positions
 * (variants with bit 2 clear, the default included); otherwise every call
 * builds.  pp_count_interactions refuses lists reused for moved particles.
 * skin = 0 (the default) builds on every call.  Errors: PP_EINVAL for a
 * negative or non-finite skin, PP_ERANGE when rcut + skin >= L / 2. */
int pp_plan_set_skin(pp_plan* plan, double skin);
int pp_plan_stats(pp_plan* plan, pp_stats* out);

/* Turn HIP-event timing of the PP kernel on (1) or off (0).  With graph
 * replay the events bracket the whole replayed graph.                      */
int pp_plan_set_timing(pp_plan* plan, int on);

/* Launch shape of the FP32 PP kernel.
 *  chunk        source-list positions per work item (multiple of 64)
 *  persistent   0: one workgroup per work item (when the previous call's
 *               items give at most two waves per SIMD, a build of the
 *               kernel for two resident waves; same results); 1: a fixed
 *               grid of waves_per_cu waves per CU pulling items from
 *               per-XCD queues with stealing
 *  waves_per_cu used by the persistent form, 1..64
 *  use_graph    1: capture the persistent kernel and the reduction in a
 *               hipGraph once and replay it (needs persistent = 1)
 *  variant      arithmetic variants (bit flags): 1 = one Newton step after
 *               the hardware rsqrt, 2 = no Kahan compensation of the
 *               per-target sums, 4 = offsets from the box origin instead of
 *               the FP64 block centre (these three are precision
 *               ablations), 8 = the split factor from an interpolated
 *               table in LDS (128 quadratic pieces, the form sec. 3.1
 *               describes) instead of the polynomial.  0 is the production
 *               kernel.
 *  waves_per_block  1, 2, 4 or 8: waves sharing one work item.  A target block
 *               (the i tile: up to 64 targets, one per lane) is swept by
 *               waves_per_block waves, wave k taking the windows k, k + K,
 *               ... of 64 source-list positions of the item (the j tiles);
 *               their compensated sums are added in wave order in LDS.  So
 *               each wave sweeps about chunk / waves_per_block positions per
 *               item.  More than 1 needs variant 0 or 8.  Every lane of a
 *               wave sweeps every staged source; sources are pruned against
 *               four boxes around the block's runs of 16 targets first.
 * The chunk grows by itself when the lists are long enough that more than
 * 2^21 work items would be needed.  Results are reproducible for a given
 * tuning; a different chunk or waves_per_block changes the summation order.
 * Defaults: plans {2048, 1, 20, 0, 0, 1}; batch plans {2048, 1, 20, 1, 0, 1}. */
typedef struct pp_tuning {
    int32_t chunk, persistent, waves_per_cu, use_graph, variant, waves_per_block;
} pp_tuning;
int pp_plan_get_tuning(const pp_plan* plan, pp_tuning* t);
int pp_plan_set_tuning(pp_plan* plan, const pp_tuning* t);

/* Autotuner: times the PP stage (HIP events around the queue reset, the PP
 * kernel or its graph and the reduction; median of 3 after a warm run) on
 * the given particles and keeps the fastest tuning in the plan.  First the
 * tiles: 1024, 2048 or 4096 source-list positions per wave with 1, 2, 4 or 8
 * waves per target block (chunk = positions x waves_per_block), persistent
 * at 20 waves per CU, and 256 or 512 positions too when the lists hold
 * fewer than 2^24 positions in all (small boxes); then, at the best tiles, the launch shape: persistent
 * with 12, 24 or 32 waves per CU, or one workgroup per item.  The variant is
 * kept.  With cache_path (may be NULL) the choice is looked up first and
 * stored afterwards, one line "arch/nbox<k>/n2^<j>/leaf<m> chunk persistent
 * waves graph waves_per_block" per shape class.  The caller's inputs are not
 * modified.  Synchronises the stream.  */
int pp_autotune(pp_plan* plan, const double* pos, const float* mass, int64_t n,
                const char* cache_path, void* stream);

/* Count, per target, the pairs with s < rcut and j != i (FP64 test), using
 * the plan's lists from the last pp_accel call on the same positions.
 *   counts device [n] int64 (out, input order; may be NULL) ; total (host).
 * Synchronises the stream.                                                 */
int pp_count_interactions(pp_plan* plan, int64_t* counts, int64_t* total, void* stream);

/* The per-block source lists of the last pp_accel / pp_accel_active /
 * pp_accel_f64 call on this plan, as the PP kernels read them: the N-to-M
 * leaf lists of the dual tree traversal (sec. 3.3) gathered per target
 * block.  A target block is a run of consecutive particles in key order
 * (at most 64, inside one 64-particle chunk of the box, integer bounding box
 * at most floor(2 rcut 2^b / L) cells wide per axis); its list is a sequence
 * of ranges, each a run of whole consecutive leaves taken at one periodic
 * shift, holding every leaf whose integer box passes the near-pair test of
 * pp_near_pairs against the block's box, each (leaf, shift) once.
 *   pp_plan_lists_size: nblock, nrange (either may be NULL).
 *   pp_plan_lists_export (host or device destinations, any may be NULL):
 *     perm   [n] int32: input index of the k-th particle in key order
 *     bstart, bcount [nblock] int32: block b holds key-ordered particles
 *            bstart[b] .. bstart[b] + bcount[b] - 1
 *     blo, bhi [3][nblock] int32: its integer bounding box, hi exclusive
 *     roff   [nblock + 1] int64: block b's ranges are roff[b] .. roff[b+1]-1
 *     slen   [nblock] int32: the number of sources in block b's list
 *     rbeg   [nrange] int32: first particle (key order) of the range
 *     rpre   [nrange] int32: list position of the range's first particle
 *            within its block's list (ranges ascend; a range ends where the
 *            next one of its block starts, the last at slen[b])
 *     rcode  [nrange] uint8: shift code 9 (s_x + 1) + 3 (s_y + 1) + (s_z + 1)
 * Synchronous.  PP_EINVAL when the plan has no lists yet.                   */
int pp_plan_lists_size(const pp_plan* plan, int64_t* nblock, int64_t* nrange);
int pp_plan_lists_export(const pp_plan* plan, int32_t* perm, int32_t* bstart, int32_t* bcount,
                         int32_t* blo, int32_t* bhi, int64_t* roff, int32_t* slen, int32_t* rbeg,
                         int32_t* rpre, uint8_t* rcode);

/* ------------------------------------------------------------- batches --
 * Many independent periodic boxes of different N, L and split parameters in
 * one pass (the task-queue idea of sec. 4.3 taken to whole boxes): every
 * stage runs once over all boxes, and the PP kernel is one persistent,
 * work-stealing launch over the work items of all boxes, captured in a
 * hipGraph and replayed.  Boxes must share key_bits and leaf_max.
 *   params [nbox], n [nbox]: box x owns particles [off_x, off_x + n[x]) of
 *   the concatenated arrays, off_x = n[0] + ... + n[x-1].
 *   pos device SoA [3][N] float64 (N = sum n), mass [N] float32,
 *   acc SoA [3][N] float32 (out), all in the concatenated input order.
 * pp_batch_accel synchronises the stream (list sizes).                     */
int pp_batch_plan_create(int nbox, const pp_box_params* params, const int64_t* n,
                         pp_batch_plan** out);
void pp_batch_plan_destroy(pp_batch_plan* bp);
int pp_batch_accel(pp_batch_plan* bp, const double* pos, const float* mass, float* acc,
                   void* stream);
int pp_batch_count_interactions(pp_batch_plan* bp, int64_t* counts, int64_t* total, void* stream);
int pp_batch_stats(pp_batch_plan* bp, pp_stats* out);
int pp_batch_set_timing(pp_batch_plan* bp, int on);
int pp_batch_get_tuning(const pp_batch_plan* bp, pp_tuning* t);
int pp_batch_set_tuning(pp_batch_plan* bp, const pp_tuning* t);
/* Autotuner for a batch (same sweep; the persistent shapes use graph replay). */
int pp_batch_autotune(pp_batch_plan* bp, const double* pos, const float* mass,
                      const char* cache_path, void* stream);

/* ---------------------------------------------------------------------
 * Long-range force: particle-mesh (sec. 3.1)
 * ---------------------------------------------------------------------
 * The PM half of the force split of Eq. equ:split, on one periodic box:
 * cloud-in-cell assignment of the masses to an n_mesh^3 mesh; a forward
 * FFT; the 3-point difference Green function of sec. 3.1,
 *   phi_k = -pi G Delta^2 rho_k / (sin^2(pi l/N) + sin^2(pi m/N) + sin^2(pi n/N)),
 * times the long-range filter exp(-k^2 r_s^2) (k = 0 dropped); an inverse
 * FFT; -grad phi by a 4-point central difference; linear (CIC)
 * interpolation to the particles.  Mesh arithmetic is FP64 (the FFTs by
 * hipFFT); the output is FP32.  pp_accel + pp_pm_accel is the whole force.
 * The mass assignment uses no atomics (the particles are sorted by mesh
 * cell and every mesh point sums in a fixed order), so repeated calls on the
 * same input give identical bits.
 *
 * pp_pm_plan_create: p gives L, rs (the filter scale) and G (rcut, eps,
 *   leaf_max and key_bits are validated but unused); 4 <= n_mesh <= 2048.
 *   The plan owns its meshes (about 60 n_mesh^3 bytes), FFT plans, and
 *   per-particle sort buffers (about 90 bytes per particle plus up to
 *   64 bytes per occupied cell) that grow on the first call with a larger n.
 * pp_pm_accel: n < 2^31 particles; pos SoA FP64 [3][n] (any real values,
 *   wrapped into [0, L)),
 *   mass FP32 [n], acc FP32 [3][n] written (not added); device pointers,
 *   enqueued on the stream.  Non-finite positions are placed at the origin
 *   (they are not detected here; pp_accel reports them). */
typedef struct pp_pm_plan pp_pm_plan;
int pp_pm_plan_create(const pp_box_params* p, int32_t n_mesh, pp_pm_plan** out);
int pp_pm_accel(pp_pm_plan* plan, const double* pos, const float* mass, int64_t n, float* acc,
                void* stream);
void pp_pm_plan_destroy(pp_pm_plan* plan);

/* ---------------------------------------------------------------------
 * Adaptive Kick-Drift-Kick integration (sec. 3.4)
 * ---------------------------------------------------------------------
 * Drives the whole force, pp_accel + pp_pm_accel (n_mesh = 0: short range
 * only), for a non-expanding periodic box: kick v += a h, drift x += v h
 * (wrapped into [0, L)).  Each particle's step is dt / 2^k, with the
 * smallest k in [0, max_level] meeting dt / 2^k <= sqrt(2 eta eps / |a|)
 * (the Gadget-2 criterion that sec. 3.4 follows).  Levels are set from the
 * forces at the start of a top step.  A top step runs 2^K substeps (K the
 * deepest level in use): opening half kicks where a particle's step starts,
 * a drift of all particles, the forces, closing half kicks where a step
 * ends.  The short-range force is evaluated for the particles whose step
 * ends at the substep only (pp_accel_active), the PM force for all.
 *
 * pp_kdk_create: p as for pp_plan_create, with eps > 0 (it enters the step
 *   criterion); n particles; eta > 0; 0 <= max_level <= 15.  The object owns
 *   a PP plan, a PM plan (n_mesh > 0) and FP32 force buffers.
 * pp_kdk_init: the forces at the initial positions (needed once).
 * pp_kdk_step: one top step of length dt > 0 on pos (FP64 [3][n], updated
 *   in place), vel (FP64 [3][n], updated in place) with masses mass (FP32
 *   [n]); device pointers; enqueued on the stream.  Synchronises the stream
 *   once per step to read the level histogram.
 * pp_kdk_set_skin: pp_plan_set_skin on the object's PP plan: the substeps
 *   then reuse the short-range lists while no particle has moved skin / 2
 *   since they were built (0, the default: a build per force evaluation).
 * pp_kdk_get_info: counters of the object.
 * pp_kdk_levels: copies the levels of the last step (int8 [n], device).
 * pp_kdk_accel: copies the current forces (FP32 [3][n] short range, then
 *   with PM [3][n] long range: 6n floats), device. */
typedef struct pp_kdk pp_kdk;
typedef struct pp_kdk_info {
    int32_t deepest_level, pad;  /* K of the last top step */
    int64_t top_steps;           /* pp_kdk_step calls */
    int64_t force_evaluations;   /* including the one of pp_kdk_init */
    int64_t level_count[16];     /* particles per level in the last top step */
    int64_t short_range_targets; /* targets given new short-range forces, summed
                                    over the force evaluations */
    int64_t list_builds;         /* force evaluations that built the short-range
                                    lists (the others reused them) */
} pp_kdk_info;
int pp_kdk_create(const pp_box_params* p, int32_t n_mesh, int64_t n, double eta, int32_t max_level,
                  pp_kdk** out);
int pp_kdk_init(pp_kdk* k, const double* pos, const float* mass, void* stream);
int pp_kdk_step(pp_kdk* k, double* pos, double* vel, const float* mass, double dt, void* stream);
int pp_kdk_set_skin(pp_kdk* k, double skin);
int pp_kdk_get_info(const pp_kdk* k, pp_kdk_info* out);
int pp_kdk_levels(const pp_kdk* k, int8_t* level, void* stream);
int pp_kdk_accel(const pp_kdk* k, float* acc, void* stream);
void pp_kdk_destroy(pp_kdk* k);

#ifdef __cplusplus
}
#endif
#endif /* PHOTON_PP_H */
