/*
 * FP64 CPU oracle for the short-range PP gravity path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may call into this file.  It shares no code,
 * header, table or helper with the HIP library and must never be linked
 * into it.
 *
 * Everything here is the plain definition, written for a reader who checks
 * it against the paper (Wang et al. 2018, "PHoToNs"):
 *
 *  - oracle_split_factor: the short-range force factor of the PM-Tree split,
 *    sec. 3.1, Eq. (equ:split), written in x = s / (2 r_s).
 *  - oracle_accel: the short-range acceleration of every requested target,
 *    the direct sum over ALL other particles (no tree, no cell grid), each
 *    pair taken at its minimum periodic image, kept only if the unsoftened
 *    separation is below r_cut (sec. 3.1 sets r_cut = 4.5 r_s), with
 *    Plummer softening applied to the separation at which the split factor
 *    and the inverse cube are evaluated.  Sums are Neumaier-compensated.
 *  - oracle_hilbert_keys: the Peano-Hilbert key of sec. 4.1 on a 2^(3b)
 *    grid.  The curve is the one of J. Skilling, "Programming the Hilbert
 *    curve", AIP Conf. Proc. 707 (2004): the key is found digit by digit as
 *    the inverse of Skilling's index-to-axes map (a search; the axes-to-index
 *    direction is not used here).
 *  - oracle_leaves: octree leaves, sec. 3.2 (every node is one contiguous
 *    run of the key-sorted particles) and sec. 3.3 ("a leaf is a package"):
 *    maximal nodes holding at most leaf_max particles, found by recursive
 *    splitting of the sorted keys.
 *  - oracle_near_pairs: every (target leaf, source leaf, periodic shift)
 *    triple whose integer bounding boxes are closer than r_cut, by brute
 *    force over all leaf pairs and all 27 shifts (the N-to-M leaf pairs of
 *    the dual tree traversal, sec. 3.3, restricted to the short range).
 *
 * Readings where the paper is silent (documented with the design):
 *  - softening: Plummer, s_eps = sqrt(s^2 + eps^2), and the split factor is
 *    evaluated at s_eps;  a_i += G m_j d g(s_eps / 2 r_s) / s_eps^3, with
 *    d = x_j - x_i (attractive);
 *  - the cut uses the unsoftened s, strictly s < r_cut;
 *  - a pair at zero separation contributes nothing (self pairs are skipped);
 *  - positions are wrapped as x - L floor(x / L) before anything else.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_OK 0
#define ORACLE_EINVAL -1
#define ORACLE_ENOMEM -2

static const double ORACLE_SQRT_PI = 1.7724538509055160272981674833411;

/* Eq. (equ:split) with x = s / (2 r_s):  erfc(x) + (2 x / sqrt(pi)) exp(-x^2).
 * (s / (r_s sqrt(pi)) = 2 x / sqrt(pi) and s^2 / (4 r_s^2) = x^2.) */
double oracle_split_factor(double x)
{
    return erfc(x) + 2.0 * x / ORACLE_SQRT_PI * exp(-x * x);
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Position wrap into the periodic box [0, L). */
static double wrap(double x, double L)
{
    return x - L * floor(x / L);
}

/* Neumaier compensated accumulation. */
typedef struct { double s, c; } nsum;
static void nsum_add(nsum* a, double v)
{
    double t = a->s + v;
    if (fabs(a->s) >= fabs(v)) a->c += (a->s - t) + v;
    else a->c += (v - t) + a->s;
    a->s = t;
}
static double nsum_get(const nsum* a) { return a->s + a->c; }

/* Minimum-image separation along one axis for two wrapped coordinates. */
static double min_image(double d, double L)
{
    if (d > 0.5 * L) d -= L;
    else if (d < -0.5 * L) d += L;
    return d;
}

/*
 * Short-range accelerations by direct summation.
 *   pos      SoA [3][n] float64, any values (wrapped here)
 *   mass     [n] float64
 *   targets  indices of the targets to evaluate (NULL: all, nt must be n)
 *   acc      out [3][nt]
 *   band_in  out [3][nt] or NULL: summed contributions of kept pairs with
 *            |s^2 / r_cut^2 - 1| < 2^-20 (pairs an FP32 cut may drop)
 *   band_out out [3][nt] or NULL: same for dropped pairs in that band
 *   n_inter  out [nt] or NULL: number of kept pairs (j != i, s < r_cut)
 *   n_band   out [nt] or NULL: number of band pairs (kept or dropped)
 */
int oracle_accel(const double* pos, const double* mass, int64_t n,
                 double L, double rs, double rcut, double eps, double G,
                 const int64_t* targets, int64_t nt,
                 double* acc, double* band_in, double* band_out,
                 int64_t* n_inter, int64_t* n_band, double* pair_abs)
{
    if (n < 0 || nt < 0 || !(L > 0) || !(rs > 0) || !(rcut > 0) || !(rcut < 0.5 * L) || !(eps >= 0))
        return ORACLE_EINVAL;
    if (!targets && nt != n) return ORACLE_EINVAL;
    double* w = (double*)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
    if (!w) return ORACLE_ENOMEM;
    for (int64_t k = 0; k < 3 * n; ++k) w[k] = wrap(pos[k], L);
    const double* wx = w;
    const double* wy = w + n;
    const double* wz = w + 2 * n;
    const double rcut2 = rcut * rcut;
    const double eps2 = eps * eps;
    const double band = ldexp(1.0, -20);

#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < nt; ++t) {
        int64_t i = targets ? targets[t] : t;
        nsum ax = {0, 0}, ay = {0, 0}, az = {0, 0};
        nsum bix = {0, 0}, biy = {0, 0}, biz = {0, 0};
        nsum box = {0, 0}, boy = {0, 0}, boz = {0, 0};
        nsum sab = {0, 0};
        int64_t kept = 0, nb = 0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double dx = min_image(wx[j] - wx[i], L);
            double dy = min_image(wy[j] - wy[i], L);
            double dz = min_image(wz[j] - wz[i], L);
            double s2 = dx * dx + dy * dy + dz * dz;
            int in_band = fabs(s2 / rcut2 - 1.0) < band;
            int keep = s2 < rcut2;
            if (!keep && !in_band) continue;
            double fx = 0, fy = 0, fz = 0;
            if (s2 > 0) {
                double se = sqrt(s2 + eps2);
                double f = G * mass[j] * oracle_split_factor(se / (2.0 * rs)) / (se * se * se);
                fx = f * dx; fy = f * dy; fz = f * dz;
            }
            if (keep) {
                ++kept;
                nsum_add(&ax, fx); nsum_add(&ay, fy); nsum_add(&az, fz);
                if (pair_abs) nsum_add(&sab, sqrt(fx * fx + fy * fy + fz * fz));
                if (in_band) { nsum_add(&bix, fx); nsum_add(&biy, fy); nsum_add(&biz, fz); }
            } else {
                nsum_add(&box, fx); nsum_add(&boy, fy); nsum_add(&boz, fz);
            }
            if (in_band) ++nb;
        }
        acc[t] = nsum_get(&ax);
        acc[nt + t] = nsum_get(&ay);
        acc[2 * nt + t] = nsum_get(&az);
        if (band_in) { band_in[t] = nsum_get(&bix); band_in[nt + t] = nsum_get(&biy); band_in[2 * nt + t] = nsum_get(&biz); }
        if (band_out) { band_out[t] = nsum_get(&box); band_out[nt + t] = nsum_get(&boy); band_out[2 * nt + t] = nsum_get(&boz); }
        if (n_inter) n_inter[t] = kept;
        if (n_band) n_band[t] = nb;
        if (pair_abs) pair_abs[t] = nsum_get(&sab);
    }
    free(w);
    return ORACLE_OK;
}

/*
 * The in-cut neighbours of the requested targets: every j != i with FP64
 * s < r_cut at the minimum periodic image, decided exactly as oracle_accel
 * decides which pairs it keeps, with the image's shift code
 * c = 9 (s_x + 1) + 3 (s_y + 1) + (s_z + 1), where s = (x_j + s L) - x_i is
 * the minimum-image separation of the wrapped positions.
 *   row_ptr  out [nt + 1]: the neighbours of target t are entries
 *            row_ptr[t] .. row_ptr[t + 1] - 1, in ascending j
 *   nbr, code out [cap]: neighbour index and shift code
 * Returns the total number of neighbours (entries are written only when it
 * is at most cap), or a negative error.
 */
static int shift_of(double d, double L)
{
    if (d > 0.5 * L) return -1;
    if (d < -0.5 * L) return 1;
    return 0;
}

int64_t oracle_neighbours(const double* pos, int64_t n, double L, double rcut,
                          const int64_t* targets, int64_t nt, int64_t cap,
                          int64_t* row_ptr, int64_t* nbr, uint8_t* code)
{
    if (n < 0 || nt < 0 || !(L > 0) || !(rcut > 0) || !(rcut < 0.5 * L)) return ORACLE_EINVAL;
    if (!targets && nt != n) return ORACLE_EINVAL;
    double* w = (double*)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
    if (!w) return ORACLE_ENOMEM;
    for (int64_t k = 0; k < 3 * n; ++k) w[k] = wrap(pos[k], L);
    const double* wx = w;
    const double* wy = w + n;
    const double* wz = w + 2 * n;
    const double rcut2 = rcut * rcut;
    for (int pass = 0; pass < 2; ++pass) {
#pragma omp parallel for schedule(dynamic, 16)
        for (int64_t t = 0; t < nt; ++t) {
            int64_t i = targets ? targets[t] : t;
            int64_t k = pass ? row_ptr[t] : 0;
            for (int64_t j = 0; j < n; ++j) {
                if (j == i) continue;
                double ex = wx[j] - wx[i], ey = wy[j] - wy[i], ez = wz[j] - wz[i];
                double dx = min_image(ex, L);
                double dy = min_image(ey, L);
                double dz = min_image(ez, L);
                double s2 = dx * dx + dy * dy + dz * dz;
                if (!(s2 < rcut2)) continue;
                if (pass) {
                    nbr[k] = j;
                    code[k] = (uint8_t)(9 * (shift_of(ex, L) + 1) + 3 * (shift_of(ey, L) + 1) +
                                        (shift_of(ez, L) + 1));
                }
                ++k;
            }
            if (!pass) row_ptr[t + 1] = k;
        }
        if (!pass) {
            row_ptr[0] = 0;
            for (int64_t t = 0; t < nt; ++t) row_ptr[t + 1] += row_ptr[t];
            if (row_ptr[nt] > cap) break;
        }
    }
    free(w);
    return row_ptr[nt];
}

/* ---------------------------------------------------------------------------
 * Peano-Hilbert keys.
 *
 * Quantisation (sec. 4.1, a 2^(3b) grid): w = x - L floor(x / L) per axis,
 * q = floor(w * (2^b / L)) clamped to [0, 2^b - 1], the scale 2^b / L formed
 * once in FP64.
 *
 * The index-to-axes map follows Skilling's construction: the 3b-bit index is
 * dealt out bit by bit to the three axes (x takes the most significant bit of
 * every 3-bit digit), then Gray-decoded across axes, then the per-level
 * reflections and axis exchanges are undone from the coarsest level to the
 * finest.
 * ------------------------------------------------------------------------- */

static void index_to_axes(uint64_t h, int b, uint32_t X[3])
{
    /* deal the index out: bit (3 l + 2 - i) of h goes to bit l of X[i] */
    X[0] = X[1] = X[2] = 0;
    for (int l = 0; l < b; ++l)
        for (int i = 0; i < 3; ++i)
            X[i] |= (uint32_t)((h >> (3 * l + 2 - i)) & 1u) << l;
    const uint32_t N = 2u << (b - 1);
    /* Gray decode across the axes */
    uint32_t t = X[2] >> 1;
    for (int i = 2; i > 0; --i) X[i] ^= X[i - 1];
    X[0] ^= t;
    /* undo the excess work, coarsest level first */
    for (uint32_t Q = 2; Q != N; Q <<= 1) {
        uint32_t P = Q - 1;
        for (int i = 2; i >= 0; --i) {
            if (X[i] & Q) {
                X[0] ^= P;
            } else {
                uint32_t s = (X[0] ^ X[i]) & P;
                X[0] ^= s;
                X[i] ^= s;
            }
        }
    }
}

void oracle_hilbert_decode(const uint64_t* keys, int64_t n, int b, uint32_t* q /* [3][n] */)
{
    for (int64_t k = 0; k < n; ++k) {
        uint32_t X[3];
        index_to_axes(keys[k], b, X);
        q[k] = X[0]; q[n + k] = X[1]; q[2 * n + k] = X[2];
    }
}

void oracle_quantise(const double* pos, int64_t n, double L, int b, uint32_t* q /* [3][n] */)
{
    const double scale = ldexp(1.0, b) / L;
    const int64_t qmax = ((int64_t)1 << b) - 1;
    for (int64_t k = 0; k < 3 * n; ++k) {
        double w = wrap(pos[k], L);
        double f = floor(w * scale);
        int64_t v = f < 0 ? 0 : (f > (double)qmax ? qmax : (int64_t)f);
        q[k] = (uint32_t)v;
    }
}

/* Key of one grid cell: choose the digits from the top down; at each level
 * the chosen digit is the one whose sub-cube (all keys sharing a prefix fill
 * one aligned cube) contains the cell. */
static uint64_t key_of_cell(const uint32_t c[3], int b)
{
    uint64_t key = 0;
    for (int lev = 1; lev <= b; ++lev) {
        int shift = b - lev;               /* cube side at this level is 2^shift */
        int found = -1;
        for (int w = 0; w < 8 && found < 0; ++w) {
            uint64_t cand = ((key << 3) | (uint64_t)w) << (3 * shift);
            uint32_t X[3];
            index_to_axes(cand, b, X);
            if ((X[0] >> shift) == (c[0] >> shift) && (X[1] >> shift) == (c[1] >> shift) &&
                (X[2] >> shift) == (c[2] >> shift))
                found = w;
        }
        if (found < 0) return ~(uint64_t)0;   /* cannot happen for a valid curve */
        key = (key << 3) | (uint64_t)found;
    }
    return key;
}

int oracle_hilbert_keys(const double* pos, int64_t n, double L, int b, uint64_t* keys)
{
    if (n < 0 || !(L > 0) || b < 1 || b > 21) return ORACLE_EINVAL;
    uint32_t* q = (uint32_t*)malloc(sizeof(uint32_t) * 3 * (size_t)(n > 0 ? n : 1));
    if (!q) return ORACLE_ENOMEM;
    oracle_quantise(pos, n, L, b, q);
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int64_t k = 0; k < n; ++k) {
        uint32_t c[3] = {q[k], q[n + k], q[2 * n + k]};
        keys[k] = key_of_cell(c, b);
        if (keys[k] == ~(uint64_t)0) bad = 1;
    }
    free(q);
    return bad ? ORACLE_EINVAL : ORACLE_OK;
}

/* ---------------------------------------------------------------------------
 * Leaves: maximal octree nodes with at most leaf_max particles.
 * sorted_keys are the keys in ascending (key, original index) order.
 * A node at level l is the set of particles sharing the top 3 l key bits;
 * because every node is a contiguous run of the sorted keys, a node is a
 * range [begin, end).  The root is level 0.  Nodes at level b are never
 * split further (their particles share one grid cell).
 * Outputs are written up to cap rows; the return value is the leaf count
 * (negative on error).
 * ------------------------------------------------------------------------- */
typedef struct {
    const uint64_t* keys;
    int b, leaf_max;
    int64_t cap, count;
    int64_t* begin; int32_t* cnt; int32_t* level; uint64_t* prefix;
} leaf_ctx;

static void emit_leaf(leaf_ctx* c, int64_t b0, int64_t e0, int lev)
{
    if (c->count < c->cap) {
        c->begin[c->count] = b0;
        c->cnt[c->count] = (int32_t)(e0 - b0);
        c->level[c->count] = lev;
        c->prefix[c->count] = lev == 0 ? 0 : c->keys[b0] >> (3 * (c->b - lev));
    }
    c->count++;
}

static void split_node(leaf_ctx* c, int64_t b0, int64_t e0, int lev)
{
    if (e0 - b0 <= c->leaf_max || lev == c->b) {
        emit_leaf(c, b0, e0, lev);
        return;
    }
    /* children: runs of equal digit at level lev + 1 */
    int sh = 3 * (c->b - lev - 1);
    int64_t s = b0;
    while (s < e0) {
        uint64_t d = (c->keys[s] >> sh) & 7u;
        int64_t e = s;
        while (e < e0 && ((c->keys[e] >> sh) & 7u) == d) ++e;
        split_node(c, s, e, lev + 1);
        s = e;
    }
}

int64_t oracle_leaves(const uint64_t* sorted_keys, int64_t n, int b, int leaf_max,
                      int64_t cap, int64_t* begin, int32_t* cnt, int32_t* level, uint64_t* prefix)
{
    if (n < 0 || b < 1 || b > 21 || leaf_max < 1) return ORACLE_EINVAL;
    for (int64_t k = 1; k < n; ++k)
        if (sorted_keys[k] < sorted_keys[k - 1]) return ORACLE_EINVAL;
    leaf_ctx c = {sorted_keys, b, leaf_max, cap, 0, begin, cnt, level, prefix};
    if (n > 0) split_node(&c, 0, n, 0);
    return c.count;
}

/* Integer bounding boxes [lo, hi) of the leaves, hi = max q + 1. */
void oracle_leaf_boxes(const uint32_t* q_sorted /* [3][n] */, int64_t n, const int64_t* begin,
                       const int32_t* cnt, int64_t nleaf, int64_t* lo /* [3][nleaf] */,
                       int64_t* hi /* [3][nleaf] */)
{
    for (int64_t a = 0; a < nleaf; ++a)
        for (int ax = 0; ax < 3; ++ax) {
            int64_t mn = INT64_MAX, mx = INT64_MIN;
            for (int64_t k = begin[a]; k < begin[a] + cnt[a]; ++k) {
                int64_t v = q_sorted[(int64_t)ax * n + k];
                if (v < mn) mn = v;
                if (v > mx) mx = v;
            }
            lo[ax * nleaf + a] = mn;
            hi[ax * nleaf + a] = mx + 1;
        }
}

/* ---------------------------------------------------------------------------
 * Near leaf pairs by brute force.  Grid units throughout: the box is 2^b
 * cells wide.  For target A, source B and shift sigma in {-1,0,1}^3 the gap
 * along axis k is
 *     max(0, lo_B + sigma 2^b - hi_A, lo_A - hi_B - sigma 2^b)
 * and the triple is listed iff the sum of squared gaps is below
 * T = ceil(r^2), r = r_cut 2^b / L.  Rows are target leaves in order; each
 * row lists (B, code) in ascending B, then ascending code, with
 * code = 9 (sx + 1) + 3 (sy + 1) + (sz + 1).
 * row_ptr has nt + 1 entries; entries beyond cap are counted, not written.
 * Returns the total number of triples, or a negative error.
 * ------------------------------------------------------------------------- */
int64_t oracle_near_pairs(const int64_t* lo, const int64_t* hi, int64_t nleaf, double L,
                          double rcut, int b, const int64_t* rows, int64_t nt, int64_t cap,
                          int64_t* row_ptr, int32_t* src, uint8_t* code)
{
    if (nleaf < 0 || !(L > 0) || !(rcut > 0) || b < 1 || b > 21) return ORACLE_EINVAL;
    const double r = rcut * ldexp(1.0, b) / L;
    const int64_t T = (int64_t)ceil(r * r);
    const int64_t W = (int64_t)1 << b;
    int64_t total = 0;
    row_ptr[0] = 0;
    for (int64_t t = 0; t < nt; ++t) {
        int64_t A = rows ? rows[t] : t;
        for (int64_t B = 0; B < nleaf; ++B) {
            for (int c = 0; c < 27; ++c) {
                int sg[3] = {c / 9 - 1, (c / 3) % 3 - 1, c % 3 - 1};
                int64_t g2 = 0;
                for (int ax = 0; ax < 3; ++ax) {
                    int64_t loA = lo[ax * nleaf + A], hiA = hi[ax * nleaf + A];
                    int64_t loB = lo[ax * nleaf + B] + sg[ax] * W, hiB = hi[ax * nleaf + B] + sg[ax] * W;
                    int64_t g = 0;
                    if (loB - hiA > g) g = loB - hiA;
                    if (loA - hiB > g) g = loA - hiB;
                    g2 += g * g;
                }
                if (g2 < T) {
                    if (total < cap) { src[total] = (int32_t)B; code[total] = (uint8_t)c; }
                    ++total;
                }
            }
        }
        row_ptr[t + 1] = total;
    }
    return total;
}
