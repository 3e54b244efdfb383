// The long-range particle-mesh (PM) force of sec. 3.1, on one periodic box:
//   1. cloud-in-cell (CIC) assignment of the masses to an N^3 mesh, without
//      atomics: the particles are sorted by the mesh cell that holds them
//      (a stable radix sort, so ties keep the input order); each cell's run
//      is cut into chunks of 32 particles whose 8 corner sums are formed in
//      order, and every mesh point adds the matching corner sums of the 8
//      cells around it, cells and chunks in a fixed order; the result does
//      not depend on scheduling;
//   2. real-to-complex FFT (hipFFT, FP64);
//   3. the 3-point difference Green function of sec. 3.1,
//      phi_k = -pi G Delta^2 rho_k / (sin^2(pi l/N) + sin^2(pi m/N) + sin^2(pi n/N)),
//      times the long-range filter exp(-k^2 r_s^2) (the complement of the
//      short-range factor of Eq. equ:split), k = 0 dropped;
//   4. complex-to-real FFT to the mesh potential;
//   5. -grad phi on the mesh by the 4-point central difference;
//   6. linear (CIC) interpolation of the mesh acceleration to the particles,
//      taken in the sorted order (neighbouring threads read neighbouring
//      mesh points) and scattered back to the input order.
// Mesh arrays are x-major: point (i, j, k) at (i N + j) N + k, the layout
// hipFFT's 3-D transforms use with the last axis fastest.
#include <cmath>
#include <new>
#include <string>

#include <hipfft/hipfft.h>

#include "pp_internal.h"

namespace pp {
namespace {

__global__ void zero_f64_kernel(double* __restrict__ p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

__global__ void zero_i32x2_kernel(int32_t* __restrict__ a, int32_t* __restrict__ b, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        a[i] = 0;
        b[i] = 0;
    }
}

// Lower mesh corner and the weight of the upper corner per axis.
// A wrapped position that rounds to L itself, or a non-finite one, lands
// on point 0 with weight 0 for its upper neighbour, so every index stays in
// [0, N).
__device__ __forceinline__ void cic_corner(double x, double L, double inv_d, int N, int& i0, double& f) {
    double w = (x - L * floor(x / L)) * inv_d;      // wrap into [0, L), mesh units
    if (!(w >= 0.0 && w < (double)N)) w = 0.0;
    const double c = floor(w);
    f = w - c;
    const int i = (int)c;
    i0 = i < N ? i : N - 1;
}

// Cell of every particle (the key of the sort), the identity payload, and
// the particle's upper-corner weights and mass as one record (input order).
__global__ void __launch_bounds__(256) cic_cell_kernel(const double* __restrict__ pos,
                                                       const float* __restrict__ mass, int64_t n,
                                                       double L, double inv_d, int N,
                                                       uint64_t* __restrict__ key,
                                                       int32_t* __restrict__ idx,
                                                       double4* __restrict__ rec_in) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    int ix, iy, iz;
    double fx, fy, fz;
    cic_corner(pos[p], L, inv_d, N, ix, fx);
    cic_corner(pos[n + p], L, inv_d, N, iy, fy);
    cic_corner(pos[2 * n + p], L, inv_d, N, iz, fz);
    key[p] = ((uint64_t)ix * N + iy) * N + iz;
    idx[p] = (int32_t)p;
    rec_in[p] = make_double4(fx, fy, fz, (double)mass[p]);
}

// Per occupied cell, its run [cbeg, cend) of the sorted particles (cells
// that hold none keep the empty run [0, 0)); and the particle records in the
// sorted order.
__global__ void __launch_bounds__(256) cic_runs_kernel(const uint64_t* __restrict__ key_s,
                                                       const int32_t* __restrict__ perm,
                                                       const double4* __restrict__ rec_in, int64_t n,
                                                       int32_t* __restrict__ cbeg,
                                                       int32_t* __restrict__ cend,
                                                       double4* __restrict__ rec) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const uint64_t c = key_s[k];
    if (k == 0 || key_s[k - 1] != c) cbeg[c] = (int32_t)k;
    if (k == n - 1 || key_s[k + 1] != c) cend[c] = (int32_t)(k + 1);
    rec[k] = rec_in[perm[k]];
}

constexpr int kCicChunk = 32;         // particles per partial sum of a cell's run

// Chunks of at most kCicChunk particles per cell run.
__global__ void __launch_bounds__(256) cic_nchunk_kernel(const int32_t* __restrict__ cbeg,
                                                         const int32_t* __restrict__ cend,
                                                         int64_t cells, int32_t* __restrict__ nch) {
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < cells;
         c += (int64_t)gridDim.x * blockDim.x)
        nch[c] = (cend[c] - cbeg[c] + kCicChunk - 1) / kCicChunk;
}

// The 8 corner sums of one chunk (one thread per chunk; its cell found by
// bisection of the chunk offsets): corner (a, b, c) of the particle's cell
// gets m prod (a ? f : 1 - f), particles in the sorted order.
__global__ void __launch_bounds__(256) cic_chunk_kernel(const int32_t* __restrict__ cbeg,
                                                        const int32_t* __restrict__ cend,
                                                        const int64_t* __restrict__ choff,
                                                        const double4* __restrict__ rec,
                                                        int64_t cells, int64_t max_chunks,
                                                        double* __restrict__ part) {
    const int64_t nchunk = choff[cells];
    for (int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; o < nchunk && o < max_chunks;
         o += (int64_t)gridDim.x * blockDim.x) {
        int64_t lo = 0, hi = cells - 1;          // the last cell with choff[cell] <= o
        while (lo < hi) {
            const int64_t mid = (lo + hi + 1) >> 1;
            if (choff[mid] <= o) lo = mid;
            else hi = mid - 1;
        }
        const int32_t a0 = cbeg[lo] + (int32_t)(o - choff[lo]) * kCicChunk;
        const int32_t a1 = a0 + kCicChunk < cend[lo] ? a0 + kCicChunk : cend[lo];
        double w[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (int32_t q = a0; q < a1; ++q) {
            const double4 r = rec[q];
            const double x[2] = {1.0 - r.x, r.x}, y[2] = {1.0 - r.y, r.y}, z[2] = {1.0 - r.z, r.z};
#pragma unroll
            for (int k = 0; k < 8; ++k) w[k] += r.w * x[k >> 2] * y[(k >> 1) & 1] * z[k & 1];
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) part[8 * o + k] = w[k];
    }
}

// Mesh point (i, j, k) takes corner (a, b, c) of cell (i - a, j - b, k - c)
// (periodic): the CIC assignment seen from the mesh, with the cells and
// their chunks in a fixed order.
__global__ void __launch_bounds__(256) cic_gather_kernel(const int64_t* __restrict__ choff,
                                                         const double* __restrict__ part, int N,
                                                         double* __restrict__ rho) {
    const int64_t total = (int64_t)N * N * N;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int k = (int)(e % N);
        const int j = (int)((e / N) % N);
        const int i = (int)(e / ((int64_t)N * N));
        double sum = 0.0;
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    const int ci = i - a < 0 ? N - 1 : i - a;
                    const int cj = j - b < 0 ? N - 1 : j - b;
                    const int ck = k - c < 0 ? N - 1 : k - c;
                    const int64_t cell = ((int64_t)ci * N + cj) * N + ck;
                    const int corner = 4 * a + 2 * b + c;
                    for (int64_t o = choff[cell]; o < choff[cell + 1]; ++o) sum += part[8 * o + corner];
                }
        rho[e] = sum;
    }
}

// phi_k = -g_k rho_k e^{-k^2 r_s^2}; scale folds in the density 1/Delta^3
// and the 1/N^3 of the unnormalised inverse FFT.
__global__ void __launch_bounds__(256) green_kernel(hipfftDoubleComplex* __restrict__ rk, int N,
                                                    double L, double G, double rs, double scale) {
    const int nzh = N / 2 + 1;
    const int64_t total = (int64_t)N * N * nzh;
    const double pi = 3.14159265358979323846;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int kz = (int)(e % nzh);
        const int ky = (int)((e / nzh) % N);
        const int kx = (int)(e / ((int64_t)nzh * N));
        if (kx == 0 && ky == 0 && kz == 0) {
            rk[e].x = 0.0;
            rk[e].y = 0.0;
            continue;
        }
        const int lx = kx <= N / 2 ? kx : kx - N;
        const int ly = ky <= N / 2 ? ky : ky - N;
        const double sx = sin(pi * lx / N), sy = sin(pi * ly / N), sz = sin(pi * kz / N);
        const double S = sx * sx + sy * sy + sz * sz;
        const double d = L / N;
        const double k2 = (2.0 * pi / L) * (2.0 * pi / L) * (double)(lx * lx + ly * ly + kz * kz);
        const double f = -pi * G * d * d / S * exp(-k2 * rs * rs) * scale;
        rk[e].x *= f;
        rk[e].y *= f;
    }
}

// -grad phi by (8 (phi[i+1] - phi[i-1]) - (phi[i+2] - phi[i-2])) / (12 Delta).
__global__ void __launch_bounds__(256) gradient_kernel(const double* __restrict__ phi, int N,
                                                       double inv_12d, double* __restrict__ g) {
    const int64_t total = (int64_t)N * N * N;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int k = (int)(e % N);
        const int j = (int)((e / N) % N);
        const int i = (int)(e / ((int64_t)N * N));
        auto at = [&](int a, int b, int c) { return phi[((int64_t)a * N + b) * N + c]; };
        auto w = [&](int a) { return a >= N ? a - N : (a < 0 ? a + N : a); };
        g[e] = -(8.0 * (at(w(i + 1), j, k) - at(w(i - 1), j, k)) - (at(w(i + 2), j, k) - at(w(i - 2), j, k))) * inv_12d;
        g[total + e] = -(8.0 * (at(i, w(j + 1), k) - at(i, w(j - 1), k)) - (at(i, w(j + 2), k) - at(i, w(j - 2), k))) * inv_12d;
        g[2 * total + e] = -(8.0 * (at(i, j, w(k + 1)) - at(i, j, w(k - 1))) - (at(i, j, w(k + 2)) - at(i, j, w(k - 2)))) * inv_12d;
    }
}

__global__ void __launch_bounds__(256) cic_interp_kernel(const uint64_t* __restrict__ key_s,
                                                         const int32_t* __restrict__ perm,
                                                         const double4* __restrict__ rec, int64_t n,
                                                         int N, const double* __restrict__ g,
                                                         float* __restrict__ acc) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const uint64_t cell = key_s[k];
    const int iz = (int)(cell % N);
    const int iy = (int)((cell / N) % N);
    const int ix = (int)(cell / ((uint64_t)N * N));
    const double4 r = rec[k];
    const double fx = r.x, fy = r.y, fz = r.z;
    const int jx = ix + 1 == N ? 0 : ix + 1, jy = iy + 1 == N ? 0 : iy + 1, jz = iz + 1 == N ? 0 : iz + 1;
    const int xs[2] = {ix, jx}, ys[2] = {iy, jy}, zs[2] = {iz, jz};
    const double wx[2] = {1.0 - fx, fx}, wy[2] = {1.0 - fy, fy}, wz[2] = {1.0 - fz, fz};
    const int64_t total = (int64_t)N * N * N;
    double ax = 0, ay = 0, az = 0;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const double w = wx[a] * wy[b] * wz[c];
                const int64_t e = ((int64_t)xs[a] * N + ys[b]) * N + zs[c];
                ax += w * g[e];
                ay += w * g[total + e];
                az += w * g[2 * total + e];
            }
    const int64_t p = perm[k];
    acc[p] = (float)ax;
    acc[n + p] = (float)ay;
    acc[2 * n + p] = (float)az;
}

const char* fft_text(hipfftResult r) {
    switch (r) {
        case HIPFFT_SUCCESS: return "success";
        case HIPFFT_INVALID_PLAN: return "invalid plan";
        case HIPFFT_ALLOC_FAILED: return "allocation failed";
        case HIPFFT_INVALID_VALUE: return "invalid value";
        case HIPFFT_EXEC_FAILED: return "execution failed";
        case HIPFFT_SETUP_FAILED: return "setup failed";
        case HIPFFT_INVALID_SIZE: return "invalid size";
        default: return "hipFFT error";
    }
}

}  // namespace

int fft_fail(int code, const char* what) {
    return fail(code == HIPFFT_ALLOC_FAILED ? PP_ENOMEM : PP_EDEVICE,
                std::string(what) + " failed: " + fft_text((hipfftResult)code));
}

}  // namespace pp

using namespace pp;

struct pp_pm_plan {
    pp_box_params p{};
    int N = 0;
    hipfftHandle fwd = nullptr, inv = nullptr;
    DevBuf rho;        // FP64 [N^3]: density, then potential (in place of the real field)
    DevBuf rk;         // complex [N][N][N/2+1]
    DevBuf g;          // FP64 [3][N^3] mesh acceleration
    DevBuf key, key_s, idx, perm;   // particle cells and the sort by cell
    DevBuf rec_in, rec;             // double4 [n]: upper-corner weights, mass (input, sorted order)
    DevBuf cbeg, cend;              // int32 [N^3]: each cell's run of sorted particles
    DevBuf sort_ws;
    DevBuf nch, choff;              // chunks per cell run and their offsets [N^3 + 1]
    DevBuf part;                    // FP64 [chunks][8]: corner sums per chunk
    DevBuf scan_ws;
    ~pp_pm_plan() {
        if (fwd) hipfftDestroy(fwd);
        if (inv) hipfftDestroy(inv);
    }
};

#define PM_FFT(call)                                                   \
    do {                                                               \
        hipfftResult r_ = (call);                                      \
        if (r_ != HIPFFT_SUCCESS) return pp::fft_fail((int)r_, #call); \
    } while (0)

extern "C" {

int pp_pm_plan_create(const pp_box_params* p, int32_t n_mesh, pp_pm_plan** out) {
    if (!out) return fail(PP_EINVAL, "out is NULL");
    *out = nullptr;
    PP_TRY(validate_params(p, false));
    if (n_mesh < 4 || n_mesh > 2048) return fail(PP_EINVAL, "n_mesh must be in 4..2048");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) return fail(PP_EDEVICE, "no HIP device");
    pp_pm_plan* pl = new (std::nothrow) pp_pm_plan;
    if (!pl) return fail(PP_ENOMEM, "host allocation failed");
    pl->p = *p;
    pl->N = n_mesh;
    const int64_t N = n_mesh, cells = N * N * N, half = N * N * (N / 2 + 1);
    int rc = pl->rho.reserve(sizeof(double) * cells);
    if (rc == PP_OK) rc = pl->rk.reserve(sizeof(hipfftDoubleComplex) * half);
    if (rc == PP_OK) rc = pl->g.reserve(sizeof(double) * 3 * cells);
    if (rc == PP_OK) rc = pl->cbeg.reserve(sizeof(int32_t) * cells);
    if (rc == PP_OK) rc = pl->cend.reserve(sizeof(int32_t) * cells);
    if (rc == PP_OK) rc = pl->nch.reserve(sizeof(int32_t) * (cells + 1));
    if (rc == PP_OK) rc = pl->choff.reserve(sizeof(int64_t) * (cells + 1));
    if (rc == PP_OK) {
        hipfftResult r = hipfftPlan3d(&pl->fwd, n_mesh, n_mesh, n_mesh, HIPFFT_D2Z);
        if (r == HIPFFT_SUCCESS) r = hipfftPlan3d(&pl->inv, n_mesh, n_mesh, n_mesh, HIPFFT_Z2D);
        if (r != HIPFFT_SUCCESS) rc = pp::fft_fail((int)r, "hipfftPlan3d");
    }
    if (rc != PP_OK) {
        delete pl;
        return rc;
    }
    *out = pl;
    return PP_OK;
}

int pp_pm_accel(pp_pm_plan* pl, const double* pos, const float* mass, int64_t n, float* acc,
                void* stream) {
    if (!pl) return fail(PP_EINVAL, "plan is NULL");
    if (n < 0) return fail(PP_EINVAL, "n must be >= 0");
    if (n > 0 && (!pos || !mass || !acc)) return fail(PP_EINVAL, "NULL buffer");
    hipStream_t s = (hipStream_t)stream;
    const int N = pl->N;
    const int64_t cells = (int64_t)N * N * N;
    const double L = pl->p.L, d = L / N;
    if (n > INT32_MAX) return fail(PP_EINVAL, "n must be below 2^31");
    double* rho = pl->rho.as<double>();
    if (n > 0) {
        int mb = 0;                      // bits per axis of the cell key
        while ((1 << mb) < N) ++mb;
        size_t ws = 0;
        PP_TRY(sort_workspace(n, 1, mb, &ws));
        PP_TRY(pl->key.reserve(sizeof(uint64_t) * n));
        PP_TRY(pl->key_s.reserve(sizeof(uint64_t) * n));
        PP_TRY(pl->idx.reserve(sizeof(int32_t) * n));
        PP_TRY(pl->perm.reserve(sizeof(int32_t) * n));
        PP_TRY(pl->rec.reserve(sizeof(double4) * n));
        PP_TRY(pl->rec_in.reserve(sizeof(double4) * n));
        PP_TRY(pl->sort_ws.reserve(ws + 1));
        int32_t* cbeg = pl->cbeg.as<int32_t>();
        int32_t* cend = pl->cend.as<int32_t>();
        hipLaunchKernelGGL(zero_i32x2_kernel, dim3(2048), dim3(256), 0, s, cbeg, cend, cells);
        hipLaunchKernelGGL(cic_cell_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, pos, mass, n, L,
                           1.0 / d, N, pl->key.as<uint64_t>(), pl->idx.as<int32_t>(), pl->rec_in.as<double4>());
        PP_HIP(hipGetLastError());
        PP_TRY(launch_sort_raw(pl->key.as<uint64_t>(), pl->idx.as<int32_t>(), pl->key_s.as<uint64_t>(),
                               pl->perm.as<int32_t>(), n, mb, pl->sort_ws.p, pl->sort_ws.bytes, s));
        hipLaunchKernelGGL(cic_runs_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, pl->key_s.as<uint64_t>(),
                           pl->perm.as<int32_t>(), pl->rec_in.as<double4>(), n, cbeg, cend,
                           pl->rec.as<double4>());
        int32_t* nch = pl->nch.as<int32_t>();
        int64_t* choff = pl->choff.as<int64_t>();
        hipLaunchKernelGGL(cic_nchunk_kernel, dim3(2048), dim3(256), 0, s, cbeg, cend, cells, nch);
        PP_HIP(hipGetLastError());
        PP_TRY(launch_scan_i32_to_i64(nch, choff, cells, pl->scan_ws, s));
        // at most n / kCicChunk + (occupied cells) chunks
        const int64_t max_chunks = n / kCicChunk + (n < cells ? n : cells) + 1;
        PP_TRY(pl->part.reserve(sizeof(double) * 8 * max_chunks));
        hipLaunchKernelGGL(cic_chunk_kernel, dim3(4096), dim3(256), 0, s, cbeg, cend, choff,
                           pl->rec.as<double4>(), cells, max_chunks, pl->part.as<double>());
        hipLaunchKernelGGL(cic_gather_kernel, dim3(4096), dim3(256), 0, s, choff, pl->part.as<double>(), N,
                           rho);
    } else {
        hipLaunchKernelGGL(zero_f64_kernel, dim3(2048), dim3(256), 0, s, rho, cells);
    }
    PP_HIP(hipGetLastError());
    PM_FFT(hipfftSetStream(pl->fwd, s));
    PM_FFT(hipfftSetStream(pl->inv, s));
    hipfftDoubleComplex* rk = pl->rk.as<hipfftDoubleComplex>();
    PM_FFT(hipfftExecD2Z(pl->fwd, rho, rk));
    const double scale = 1.0 / (d * d * d) / (double)cells;
    hipLaunchKernelGGL(green_kernel, dim3(2048), dim3(256), 0, s, rk, N, L, pl->p.G, pl->p.rs, scale);
    PP_HIP(hipGetLastError());
    PM_FFT(hipfftExecZ2D(pl->inv, rk, rho));
    double* g = pl->g.as<double>();
    hipLaunchKernelGGL(gradient_kernel, dim3(2048), dim3(256), 0, s, rho, N, 1.0 / (12.0 * d), g);
    if (n > 0)
        hipLaunchKernelGGL(cic_interp_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s,
                           pl->key_s.as<uint64_t>(), pl->perm.as<int32_t>(), pl->rec.as<double4>(), n, N, g,
                           acc);
    PP_HIP(hipGetLastError());
    return PP_OK;
}

void pp_pm_plan_destroy(pp_pm_plan* pl) { delete pl; }

}  // extern "C"
