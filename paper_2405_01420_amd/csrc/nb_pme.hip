// Smooth particle-mesh Ewald: the reciprocal-space part that completes the real-space Ewald
// forces when the paper's runs use PME (section II-C; the PME spread / solve / gather kernels
// of Fig. 2).  The paper gives no algorithm; this follows the standard smooth-PME construction
// (cardinal B-spline interpolation of the charges, FFT convolution with the Ewald kernel):
//
//   u_i = K_a x_i,a / L_a (scaled coordinates), charges spread onto the K1 x K2 x K3 grid with
//   weights M_n(u_i,a - k_a) per axis (cardinal B-splines of order n, periodic in k);
//   phi = unnormalised inverse FFT of G(m) FFT(Q)(m), with
//   G(m) = fC / (pi V) exp(-pi^2 |m|^2 / beta^2) / |m|^2 |b1|^2 |b2|^2 |b3|^2 (G(0) = 0),
//   |b_a(m)|^-2 = |sum_{k=0}^{n-2} M_n(k + 1) exp(2 pi i m k / K_a)|^2;
//   E_rec = 1/2 sum_m G(m) |FFT(Q)(m)|^2, F_i = -q_i sum over the atom's grid points of
//   grad(weights) phi.
//
// MI355X layout: one thread per atom for the spread (FP64 atomics into the real grid, n^3 per
// atom) and the gather (FP64 sums, FP32 forces); the grid and both FFTs are FP64 (hipFFT,
// D2Z / Z2D); the solve runs over the half-complex grid and keeps per-block FP64 energy
// partials that one block adds in a fixed order.
#include <hip/hip_runtime.h>
#include <hipfft/hipfft.h>

#include <cmath>
#include <string>
#include <vector>

#include "nb.h"

#define NB_PME_BLOCK 256
#define NB_PME_MAX_ORDER 8

struct nb_pme {
    hipStream_t stream = nullptr;
    int device = 0;
    int natoms = 0, order = 0;
    int K[3] = {0, 0, 0};
    double L[3] = {0, 0, 0};
    double beta = 0, fc = 0;
    size_t nreal = 0, ncplx = 0;
    double *grid = nullptr;        // [K1][K2][K3] charges, then the potential phi
    double2 *cgrid = nullptr;      // [K1][K2][K3/2 + 1] transform
    double *infl = nullptr;        // [K1][K2][K3/2 + 1] G(m) times the Hermitian weight / 2
    double *part = nullptr;        // energy partials of the solve blocks
    int nsolve_blocks = 0;
    hipfftHandle fwd = 0, bwd = 0;
    bool have_fwd = false, have_bwd = false;
    std::string err;
};

namespace {

thread_local std::string g_pme_error;

int pfail(nb_pme *p, int code, const std::string &msg) {
    if (p) p->err = msg;
    else g_pme_error = msg;
    return code;
}

// Cardinal B-spline weights M_n(w + j), j = 0 .. n-1, for w in [0, 1), and their derivatives
// dM_n(w + j) / dx = M_{n-1}(w + j) - M_{n-1}(w + j - 1), by the recursion
// M_k(x) = x / (k-1) M_{k-1}(x) + (k - x) / (k-1) M_{k-1}(x - 1) evaluated on the n points at once.
__device__ __forceinline__ void pme_bspline(double w, int n, double *val, double *der) {
    // order-2 values on the points x_j = w + j: M_2(x) = 1 - |x - 1| on [0, 2]
    double m[NB_PME_MAX_ORDER + 1];
#pragma unroll
    for (int j = 0; j <= NB_PME_MAX_ORDER; ++j) m[j] = 0.0;
    m[0] = w;          // M_2(w), x in [0, 1)
    m[1] = 1.0 - w;    // M_2(w + 1)
    // m[j] holds M_k(w + j) for j = 0 .. k-1 (zero beyond)
    for (int k = 3; k <= n; ++k) {
        if (k == n) {
#pragma unroll
            for (int j = 0; j < NB_PME_MAX_ORDER; ++j)
                der[j] = (j < n) ? m[j] - (j > 0 ? m[j - 1] : 0.0) : 0.0;
        }
        const double inv = 1.0 / (k - 1);
        for (int j = k - 1; j >= 0; --j) {
            const double x = w + j;
            const double a = x * m[j];
            const double b = j > 0 ? (k - x) * m[j - 1] : 0.0;
            m[j] = (a + b) * inv;
        }
    }
#pragma unroll
    for (int j = 0; j < NB_PME_MAX_ORDER; ++j) val[j] = j < n ? m[j] : 0.0;
}

__device__ __forceinline__ int pme_wrap(int k, int K) {
    k %= K;
    return k < 0 ? k + K : k;
}

__global__ void k_pme_zero(size_t n, double *__restrict__ g) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) g[i] = 0.0;
}

__global__ void __launch_bounds__(NB_PME_BLOCK) k_pme_spread(int natoms, int n, int K1, int K2, int K3,
                                                              double L1, double L2, double L3,
                                                              const float *__restrict__ x,
                                                              const float *__restrict__ q,
                                                              double *__restrict__ grid) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= natoms) return;
    const double qi = q[i];
    if (qi == 0.0) return;
    double v[3][NB_PME_MAX_ORDER], d[3][NB_PME_MAX_ORDER];
    int base[3];
    const int K[3] = {K1, K2, K3};
    const double L[3] = {L1, L2, L3};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double u = (double)x[3 * i + a] / L[a] * K[a];
        const double fl = floor(u);
        pme_bspline(u - fl, n, v[a], d[a]);
        base[a] = pme_wrap((int)fl, K[a]);
    }
    for (int j1 = 0; j1 < n; ++j1) {
        const int k1 = pme_wrap(base[0] - j1, K1);
        const double w1 = qi * v[0][j1];
        for (int j2 = 0; j2 < n; ++j2) {
            const int k2 = pme_wrap(base[1] - j2, K2);
            const double w12 = w1 * v[1][j2];
            double *row = grid + ((size_t)k1 * K2 + k2) * K3;
            for (int j3 = 0; j3 < n; ++j3) atomicAdd(row + pme_wrap(base[2] - j3, K3), w12 * v[2][j3]);
        }
    }
}

// c(m) <- G(m) c(m) over the half-complex grid; energy partial sum of G |c|^2 with the
// Hermitian weights folded into infl (weight / 2, so that the sum is E_rec).
__global__ void __launch_bounds__(NB_PME_BLOCK) k_pme_solve(size_t ncplx, const double *__restrict__ infl,
                                                             const double *__restrict__ ewt,
                                                             double2 *__restrict__ c,
                                                             double *__restrict__ part) {
    __shared__ double s[NB_PME_BLOCK / 64];
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    double e = 0.0;
    if (i < ncplx) {
        const double g = infl[i];
        const double2 z = c[i];
        e = ewt[i] * g * (z.x * z.x + z.y * z.y);
        c[i] = make_double2(g * z.x, g * z.y);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) e += __shfl_xor(e, o, 64);
    if ((threadIdx.x & 63) == 0) s[threadIdx.x / 64] = e;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int k = 0; k < NB_PME_BLOCK / 64; ++k) t += s[k];
        part[blockIdx.x] = t;
    }
}

__global__ void __launch_bounds__(NB_PME_BLOCK) k_pme_energy(int nblk, const double *__restrict__ part,
                                                              double *__restrict__ e) {
    __shared__ double s[NB_PME_BLOCK / 64];
    double t = 0.0;
    for (int k = threadIdx.x; k < nblk; k += NB_PME_BLOCK) t += part[k];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
    if ((threadIdx.x & 63) == 0) s[threadIdx.x / 64] = t;
    __syncthreads();
    if (threadIdx.x == 0) {
        double r = 0.0;
        for (int k = 0; k < NB_PME_BLOCK / 64; ++k) r += s[k];
        e[0] = r;
    }
}

__global__ void __launch_bounds__(NB_PME_BLOCK) k_pme_gather(int natoms, int n, int K1, int K2, int K3,
                                                              double L1, double L2, double L3,
                                                              const float *__restrict__ x,
                                                              const float *__restrict__ q,
                                                              const double *__restrict__ phi,
                                                              float *__restrict__ f) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= natoms) return;
    const double qi = q[i];
    double v[3][NB_PME_MAX_ORDER], d[3][NB_PME_MAX_ORDER];
    int base[3];
    const int K[3] = {K1, K2, K3};
    const double L[3] = {L1, L2, L3};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double u = (double)x[3 * i + a] / L[a] * K[a];
        const double fl = floor(u);
        pme_bspline(u - fl, n, v[a], d[a]);
        base[a] = pme_wrap((int)fl, K[a]);
    }
    double gx = 0.0, gy = 0.0, gz = 0.0;
    if (qi != 0.0) {
        for (int j1 = 0; j1 < n; ++j1) {
            const int k1 = pme_wrap(base[0] - j1, K1);
            for (int j2 = 0; j2 < n; ++j2) {
                const int k2 = pme_wrap(base[1] - j2, K2);
                const double *row = phi + ((size_t)k1 * K2 + k2) * K3;
                double sv = 0.0, sd = 0.0;
                for (int j3 = 0; j3 < n; ++j3) {
                    const double p = row[pme_wrap(base[2] - j3, K3)];
                    sv += v[2][j3] * p;
                    sd += d[2][j3] * p;
                }
                gx += d[0][j1] * v[1][j2] * sv;
                gy += v[0][j1] * d[1][j2] * sv;
                gz += v[0][j1] * v[1][j2] * sd;
            }
        }
    }
    f[3 * i] = (float)(-qi * gx * K1 / L1);
    f[3 * i + 1] = (float)(-qi * gy * K2 / L2);
    f[3 * i + 2] = (float)(-qi * gz * K3 / L3);
}

// Host side: cardinal B-spline values M_n(k), k = 1 .. n-1, and the moduli |b(m)|^2.
std::vector<double> bspline_int(int n) {
    // M_n at the integers 0 .. n by the same recursion, from M_2(1) = 1
    std::vector<double> m(n + 1, 0.0);
    m[1] = 1.0;
    for (int k = 3; k <= n; ++k) {
        std::vector<double> nm(n + 1, 0.0);
        for (int x = 1; x < k; ++x) nm[x] = (x * m[x] + (k - x) * m[x - 1]) / (k - 1);
        m = nm;
    }
    return m;
}

std::vector<double> bmod2(int K, int n) {
    const std::vector<double> M = bspline_int(n);
    std::vector<double> out(K);
    for (int m = 0; m < K; ++m) {
        double re = 0.0, im = 0.0;
        for (int k = 0; k <= n - 2; ++k) {
            const double ph = 2.0 * M_PI * m * k / K;
            re += M[k + 1] * cos(ph);
            im += M[k + 1] * sin(ph);
        }
        out[m] = 1.0 / (re * re + im * im);
    }
    return out;
}

template <typename T>
int palloc(nb_pme *p, T **ptr, size_t count, const char *what) {
    if (hipMalloc((void **)ptr, sizeof(T) * std::max<size_t>(count, 1)) != hipSuccess) {
        *ptr = nullptr;
        return pfail(p, NB_ERR_OOM, std::string("hipMalloc ") + what);
    }
    return NB_OK;
}

void pme_free(nb_pme *p) {
    if (p->have_fwd) hipfftDestroy(p->fwd);
    if (p->have_bwd) hipfftDestroy(p->bwd);
    void *bufs[] = {p->grid, p->cgrid, p->infl, p->part};
    for (void *b : bufs)
        if (b) hipFree(b);
}

}  // namespace

extern "C" {

int nb_pme_setup(nb_pme **out, const nb_pme_params *prm, void *stream) {
    if (!out || !prm) return pfail(nullptr, NB_ERR_ARG, "NULL argument");
    *out = nullptr;
    for (int a = 0; a < 3; ++a) {
        if (!(std::isfinite(prm->box[a]) && prm->box[a] > 0.0)) return pfail(nullptr, NB_ERR_ARG, "box edges must be finite and > 0");
        if (prm->grid[a] < 2 * prm->order || prm->grid[a] > 1024) return pfail(nullptr, NB_ERR_ARG, "grid sizes must be in 2*order .. 1024");
    }
    if (prm->order < 4 || prm->order > NB_PME_MAX_ORDER || (prm->order & 1))
        return pfail(nullptr, NB_ERR_ARG, "order must be 4, 6 or 8");
    if (!(std::isfinite(prm->ewald_beta) && prm->ewald_beta > 0.0)) return pfail(nullptr, NB_ERR_ARG, "ewald_beta must be > 0");
    if (!(std::isfinite(prm->coulomb_const) && prm->coulomb_const > 0.0)) return pfail(nullptr, NB_ERR_ARG, "coulomb_const must be > 0");
    if (prm->natoms < 1 || prm->natoms > (1 << 27)) return pfail(nullptr, NB_ERR_ARG, "natoms must be in 1..2^27");
    nb_pme *p = new nb_pme();
    p->stream = (hipStream_t)stream;
    hipGetDevice(&p->device);
    p->natoms = prm->natoms;
    p->order = prm->order;
    for (int a = 0; a < 3; ++a) {
        p->K[a] = prm->grid[a];
        p->L[a] = prm->box[a];
    }
    p->beta = prm->ewald_beta;
    p->fc = prm->coulomb_const;
    const int K1 = p->K[0], K2 = p->K[1], K3 = p->K[2], K3h = K3 / 2 + 1;
    p->nreal = (size_t)K1 * K2 * K3;
    p->ncplx = (size_t)K1 * K2 * K3h;
    p->nsolve_blocks = (int)((p->ncplx + NB_PME_BLOCK - 1) / NB_PME_BLOCK);
    int r;
    if ((r = palloc(p, &p->grid, p->nreal, "grid")) != NB_OK ||
        (r = palloc(p, &p->cgrid, p->ncplx, "transform")) != NB_OK ||
        (r = palloc(p, &p->infl, 2 * p->ncplx, "influence function")) != NB_OK ||
        (r = palloc(p, &p->part, (size_t)p->nsolve_blocks, "energy partials")) != NB_OK) {
        g_pme_error = p->err;
        pme_free(p);
        delete p;
        return r;
    }
    // influence function G(m) and the Hermitian energy weights (1 for k3 = 0 and k3 = K3/2 of an
    // even K3, 2 for the other stored k3, since those stand for m and -m), both halved
    const std::vector<double> b1 = bmod2(K1, p->order), b2 = bmod2(K2, p->order), b3 = bmod2(K3, p->order);
    const double V = p->L[0] * p->L[1] * p->L[2];
    std::vector<double> g(2 * p->ncplx);
    for (int k1 = 0; k1 < K1; ++k1) {
        const double m1 = (k1 <= K1 / 2 ? k1 : k1 - K1) / p->L[0];
        for (int k2 = 0; k2 < K2; ++k2) {
            const double m2 = (k2 <= K2 / 2 ? k2 : k2 - K2) / p->L[1];
            for (int k3 = 0; k3 < K3h; ++k3) {
                const double m3 = k3 / p->L[2];
                const double msq = m1 * m1 + m2 * m2 + m3 * m3;
                const size_t i = ((size_t)k1 * K2 + k2) * K3h + k3;
                g[i] = msq > 0.0 ? p->fc / (M_PI * V) * exp(-M_PI * M_PI * msq / (p->beta * p->beta)) / msq *
                                       b1[k1] * b2[k2] * b3[k3]
                                 : 0.0;
                const double herm = (k3 == 0 || (K3 % 2 == 0 && k3 == K3 / 2)) ? 1.0 : 2.0;
                g[p->ncplx + i] = 0.5 * herm;
            }
        }
    }
    hipError_t e = hipMemcpy(p->infl, g.data(), sizeof(double) * g.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        pme_free(p);
        delete p;
        return pfail(nullptr, NB_ERR_HIP, std::string("upload influence function: ") + hipGetErrorString(e));
    }
    if (hipfftPlan3d(&p->fwd, K1, K2, K3, HIPFFT_D2Z) != HIPFFT_SUCCESS ||
        !(p->have_fwd = true) || hipfftPlan3d(&p->bwd, K1, K2, K3, HIPFFT_Z2D) != HIPFFT_SUCCESS) {
        pme_free(p);
        delete p;
        return pfail(nullptr, NB_ERR_HIP, "hipfftPlan3d");
    }
    p->have_bwd = true;
    if (hipfftSetStream(p->fwd, p->stream) != HIPFFT_SUCCESS || hipfftSetStream(p->bwd, p->stream) != HIPFFT_SUCCESS) {
        pme_free(p);
        delete p;
        return pfail(nullptr, NB_ERR_HIP, "hipfftSetStream");
    }
    *out = p;
    return NB_OK;
}

int nb_pme_forces(nb_pme *p, const float *x, const float *q, float *f, double *e) {
    if (!p || !x || !q || !f || !e) return pfail(p, NB_ERR_ARG, "NULL argument");
    hipSetDevice(p->device);
    const int K1 = p->K[0], K2 = p->K[1], K3 = p->K[2];
    const int ab = (p->natoms + NB_PME_BLOCK - 1) / NB_PME_BLOCK;
    hipLaunchKernelGGL(k_pme_zero, dim3((unsigned)((p->nreal + NB_PME_BLOCK - 1) / NB_PME_BLOCK)),
                       dim3(NB_PME_BLOCK), 0, p->stream, p->nreal, p->grid);
    hipLaunchKernelGGL(k_pme_spread, dim3(ab), dim3(NB_PME_BLOCK), 0, p->stream, p->natoms, p->order,
                       K1, K2, K3, p->L[0], p->L[1], p->L[2], x, q, p->grid);
    if (hipGetLastError() != hipSuccess) return pfail(p, NB_ERR_HIP, "spread launch");
    if (hipfftExecD2Z(p->fwd, (hipfftDoubleReal *)p->grid, (hipfftDoubleComplex *)p->cgrid) != HIPFFT_SUCCESS)
        return pfail(p, NB_ERR_HIP, "forward FFT");
    hipLaunchKernelGGL(k_pme_solve, dim3(p->nsolve_blocks), dim3(NB_PME_BLOCK), 0, p->stream, p->ncplx,
                       p->infl, p->infl + p->ncplx, p->cgrid, p->part);
    hipLaunchKernelGGL(k_pme_energy, dim3(1), dim3(NB_PME_BLOCK), 0, p->stream, p->nsolve_blocks, p->part, e);
    if (hipGetLastError() != hipSuccess) return pfail(p, NB_ERR_HIP, "solve launch");
    if (hipfftExecZ2D(p->bwd, (hipfftDoubleComplex *)p->cgrid, (hipfftDoubleReal *)p->grid) != HIPFFT_SUCCESS)
        return pfail(p, NB_ERR_HIP, "inverse FFT");
    hipLaunchKernelGGL(k_pme_gather, dim3(ab), dim3(NB_PME_BLOCK), 0, p->stream, p->natoms, p->order,
                       K1, K2, K3, p->L[0], p->L[1], p->L[2], x, q, p->grid, f);
    if (hipGetLastError() != hipSuccess) return pfail(p, NB_ERR_HIP, "gather launch");
    return NB_OK;
}

const char *nb_pme_last_error(nb_pme *p) { return p ? p->err.c_str() : g_pme_error.c_str(); }

int nb_pme_destroy(nb_pme *p) {
    if (!p) return NB_OK;
    hipSetDevice(p->device);
    hipStreamSynchronize(p->stream);
    pme_free(p);
    delete p;
    return NB_OK;
}

}  // extern "C"
