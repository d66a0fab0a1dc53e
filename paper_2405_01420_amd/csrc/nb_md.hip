// Molecular-dynamics loop around the short-range force path: leapfrog integration with the pair
// list rebuilt every nstlist steps and, between builds, the rolling prune of the list (the
// paper's prune-only kernel, section III-A) every nstprune steps.  The loop runs on the
// context's stream without host synchronisation except at list builds (none with
// NB_ASYNC_BUILD); each step is the force call (pack, force kernel, finalize), one update
// kernel and one single-block energy kernel.
//
// Leapfrog:  v(t + dt/2) = v(t - dt/2) + f(t) / m dt,   x(t + dt) = x(t) + v(t + dt/2) dt.
// The kinetic energy at t is the average of the two half-step kinetic energies,
// 1/2 m (|v(t - dt/2)|^2 + |v(t + dt/2)|^2) / 2, summed in FP64.
#include "nb_device.h"

namespace {

#define NB_MD_BLOCK 256

__global__ void __launch_bounds__(NB_MD_BLOCK) k_leapfrog(int n, float dt, const float *__restrict__ f,
                                                          const float *__restrict__ inv_m,
                                                          float *__restrict__ x, float *__restrict__ v,
                                                          double *__restrict__ kpart) {
    __shared__ double s[NB_MD_BLOCK / NB_WAVE];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    double ke = 0.0;
    if (i < n) {
        const float w = inv_m[i];
        double k2 = 0.0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const float v0 = v[3 * i + a];
            const float v1 = __builtin_fmaf(f[3 * i + a] * w, dt, v0);
            v[3 * i + a] = v1;
            x[3 * i + a] = __builtin_fmaf(v1, dt, x[3 * i + a]);
            k2 += (double)v0 * v0 + (double)v1 * v1;
        }
        ke = 0.25 * k2 / (double)w;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) ke += __shfl_xor(ke, o, NB_WAVE);
    if ((threadIdx.x & (NB_WAVE - 1)) == 0) s[threadIdx.x / NB_WAVE] = ke;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int k = 0; k < NB_MD_BLOCK / NB_WAVE; ++k) t += s[k];
        kpart[blockIdx.x] = t;
    }
}

// e[2] = kinetic energy (the block partials in order), e[3] = e[0] + e[1] + e[2].
__global__ void __launch_bounds__(NB_MD_BLOCK) k_md_energy(int nblk, const double *__restrict__ kpart,
                                                           double *__restrict__ e) {
    __shared__ double s[NB_MD_BLOCK / NB_WAVE];
    double t = 0.0;
    for (int b = threadIdx.x; b < nblk; b += blockDim.x) t += kpart[b];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, NB_WAVE);
    if ((threadIdx.x & (NB_WAVE - 1)) == 0) s[threadIdx.x / NB_WAVE] = t;
    __syncthreads();
    if (threadIdx.x == 0) {
        double k = 0.0;
        for (int w = 0; w < NB_MD_BLOCK / NB_WAVE; ++w) k += s[w];
        e[2] = k;
        e[3] = e[0] + e[1] + k;
    }
}

}  // namespace

hipError_t nb_launch_md_update(nb_ctx *c, float dt, const float *f, const float *inv_m, float *x,
                               float *v, double *e) {
    const int nblk = (c->natoms + NB_MD_BLOCK - 1) / NB_MD_BLOCK;
    if (!c->mdpart && hipMalloc((void **)&c->mdpart, sizeof(double) * nblk) != hipSuccess)
        return hipErrorOutOfMemory;
    hipLaunchKernelGGL(k_leapfrog, dim3(nblk), dim3(NB_MD_BLOCK), 0, c->stream, c->natoms, dt, f,
                       inv_m, x, v, c->mdpart);
    hipLaunchKernelGGL(k_md_energy, dim3(1), dim3(NB_MD_BLOCK), 0, c->stream, nblk, c->mdpart, e);
    return hipGetLastError();
}
