// Per-call force path: pack (gather positions/charges/types into cluster order), the
// cluster-pair force kernel (Lennard-Jones with potential shift + Ewald real-space Coulomb),
// and the finalize step (un-permute, f = f_i + f_j, FP64 energies with the shifts applied).
//
// This is the computation the paper identifies as the single-GPU rate limiter (section III-A;
// the flavour named in the Fig. 3 caption).  Kernel layout (a from-scratch design for a
// 64-wide wavefront, not the paper's SYCL layout):
//  * one wavefront per i-cluster; the C i-atoms are wave-uniform values, so every i-coordinate
//    is a scalar operand of the vector instructions;
//  * each lane owns one j-atom of one of the 64 / C j-clusters of the current batch and loops
//    over the C i-atoms, so the j-force of the lane's atom accumulates in registers and needs
//    one atomic add per component per batch (the only atomics);
//  * the i-forces accumulate per lane over the whole list and are reduced across the 64 lanes
//    once per i-cluster with cross-lane shuffles;
//  * erfc(beta r) = exp(-beta^2 r^2) P(r)/Q(r) with a (4,5) rational fit of the scaled
//    complementary error function (see fit_erfcx.py): one v_exp, one v_rcp, one v_rsq per pair;
//  * per-pair energies are rounded once to FP32 and accumulated in FP64; the Coulomb potential
//    shift is applied in FP64 at the end from the sum of q_i q_j over interacting pairs.
#include "nb_device.h"

namespace {

__global__ void k_pack(int npad_max, const int *__restrict__ perm, const float *__restrict__ x,
                       const float *__restrict__ q, const int32_t *__restrict__ type, int ntypes,
                       const float4 *__restrict__ off, const float *__restrict__ xbuild,
                       uint32_t checks, float stale2, float4 *__restrict__ xq,
                       int *__restrict__ tsort, float *__restrict__ fj, nb_meta *meta) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= npad_max || p >= meta->npad) return;
    int a = perm[p];
    if (a >= 0) {
        float x0 = x[3 * a], x1 = x[3 * a + 1], x2 = x[3 * a + 2];
        float4 o = off[a];
        if (checks & NB_CHECK_STALE) {
            float d0 = x0 - xbuild[3 * a], d1 = x1 - xbuild[3 * a + 1], d2 = x2 - xbuild[3 * a + 2];
            if (!(d0 * d0 + d1 * d1 + d2 * d2 < stale2)) atomicOr(&meta->flags, NB_F_STALE);
        }
        if ((checks & NB_CHECK_FINITE) && !(isfinite(x0) && isfinite(x1) && isfinite(x2)))
            atomicOr(&meta->flags, NB_F_NONFINITE);
        int t = type ? type[a] : 0;
        t = min(max(t, 0), ntypes - 1);
        xq[p] = make_float4(x0 + o.x, x1 + o.y, x2 + o.z, q ? q[a] : 0.0f);
        tsort[p] = t;
    } else {
        xq[p] = make_float4(-1e5f, -1e5f, -1e5f, 0.0f);
        tsort[p] = 0;
    }
    fj[p] = 0.0f;
    fj[npad_max + p] = 0.0f;
    fj[2 * npad_max + p] = 0.0f;
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, NB_WAVE);
    return v;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, NB_WAVE);
    return v;
}

template <int C>
__global__ void __launch_bounds__(256) k_force(nb_fparams fp, int cap, int npad_max,
                                               const float4 *__restrict__ xq,
                                               const int *__restrict__ tsort,
                                               const float4 *__restrict__ ljtab,
                                               const int *__restrict__ icount,
                                               const nb_entry *__restrict__ jl,
                                               float4 *__restrict__ fi_out, float *__restrict__ fj,
                                               double *__restrict__ epart, const nb_meta *meta) {
    constexpr int JPB = NB_WAVE / C;  // j-clusters per batch
    extern __shared__ float4 tab[];
    const int nt = fp.ntypes, ntt = nt * nt;
    for (int k = threadIdx.x; k < 2 * ntt; k += blockDim.x) tab[k] = ljtab[k];
    __syncthreads();
    const int lane = threadIdx.x & (NB_WAVE - 1);
    const int ci = __builtin_amdgcn_readfirstlane(blockIdx.x * (blockDim.x / NB_WAVE) +
                                                  threadIdx.x / NB_WAVE);
    if (ci >= meta->nclusters) return;
    const int b = lane % C, jsub = lane / C;

    float xi[C], yi[C], zi[C], qi[C];
    int ti[C];
#pragma unroll
    for (int k = 0; k < C; ++k) {
        float4 v = xq[ci * C + k];
        xi[k] = v.x;
        yi[k] = v.y;
        zi[k] = v.z;
        qi[k] = v.w * fp.fc;
        ti[k] = tsort[ci * C + k] * nt;
    }
    float fix[C], fiy[C], fiz[C];
#pragma unroll
    for (int k = 0; k < C; ++k) fix[k] = fiy[k] = fiz[k] = 0.0f;
    double elj = 0.0, ec = 0.0;
    float qqs = 0.0f;

    const int nj = icount[ci];
    const nb_entry *lst = jl + (size_t)ci * cap;
    for (int base = 0; base < nj; base += JPB) {
        const int e = base + jsub;
        const bool valid = e < nj;
        nb_entry en;
        if (valid) {
            en = lst[e];
        } else {
            en.cj = ci;
            en.shift = NB_SHIFT_ZERO;
            en.mlo = en.mhi = 0u;
        }
        const int s = en.shift;
        const int tx = nb_tx(s), ty = nb_ty(s), tz = nb_tz(s);
        const int jslot = en.cj * C + b;
        const float4 xj = xq[jslot];
        const int tj = tsort[jslot];
        const float xjs = xj.x + nb_dj(tx, fp.L[0]), yjs = xj.y + nb_dj(ty, fp.L[1]),
                    zjs = xj.z + nb_dj(tz, fp.L[2]);
        const float dix = nb_di(tx, fp.L[0]), diy = nb_di(ty, fp.L[1]), diz = nb_di(tz, fp.L[2]);
        const float qj = xj.w;
        const unsigned long long m = ((unsigned long long)en.mhi << 32) | en.mlo;
        unsigned mcol = 0;
#pragma unroll
        for (int k = 0; k < C; ++k) mcol |= (unsigned)((m >> (k * C + b)) & 1ull) << k;

        float fjx = 0.0f, fjy = 0.0f, fjz = 0.0f;
#pragma unroll
        for (int k = 0; k < C; ++k) {
            const float dx = (xi[k] + dix) - xjs;
            const float dy = (yi[k] + diy) - yjs;
            const float dz = (zi[k] + diz) - zjs;
            const float r2 = nb_r2(dx, dy, dz);
            const bool inc = (r2 < fp.rc2) && ((mcol >> k) & 1u);
            const float rinv = inc ? nb_rsq(r2) : 0.0f;
            const float rinv2 = rinv * rinv;
            const float rinv6 = rinv2 * rinv2 * rinv2;
            const float4 lj = tab[ti[k] + tj];   // (C6, C12, 6 C6, 12 C12)
            const float shv = tab[ntt + ti[k] + tj].x;
            const float m1 = inc ? 1.0f : 0.0f;
            // Lennard-Jones: energy C12 r^-12 - C6 r^-6 - shift, force factor
            // (12 C12 r^-6 - 6 C6) r^-6 r^-2
            const float u = __builtin_fmaf(lj.y, rinv6, -lj.x);
            const float elj_p = __builtin_fmaf(u, rinv6, -m1 * shv);
            const float tf = __builtin_fmaf(lj.w, rinv6, -lj.z);
            const float flj = tf * rinv6;
            // Ewald real space: erfc(beta r) = exp(-beta^2 r^2) P(r) / Q(r)
            const float r = r2 * rinv;
            const float ex = __builtin_amdgcn_exp2f(fp.cexp * r2);
            float P = fp.p[4];
            P = __builtin_fmaf(P, r, fp.p[3]);
            P = __builtin_fmaf(P, r, fp.p[2]);
            P = __builtin_fmaf(P, r, fp.p[1]);
            P = __builtin_fmaf(P, r, fp.p[0]);
            float Q = fp.q[5];
            Q = __builtin_fmaf(Q, r, fp.q[4]);
            Q = __builtin_fmaf(Q, r, fp.q[3]);
            Q = __builtin_fmaf(Q, r, fp.q[2]);
            Q = __builtin_fmaf(Q, r, fp.q[1]);
            Q = __builtin_fmaf(Q, r, fp.q[0]);
            const float R = P * nb_rcp(Q);
            const float qq = qi[k] * qj;
            const float qe = qq * ex;
            const float t1 = qe * rinv;               // fC q_i q_j exp(-b^2 r^2) / r
            const float ec_p = t1 * R;                // fC q_i q_j erfc(b r) / r
            const float uu = __builtin_fmaf(fp.kb, r, R);
            const float fs = __builtin_fmaf(t1, uu, flj) * rinv2;
            elj += (double)elj_p;
            ec += (double)ec_p;
            qqs = __builtin_fmaf(m1, qq, qqs);
            const float fx = fs * dx, fy = fs * dy, fz = fs * dz;
            fix[k] += fx;
            fiy[k] += fy;
            fiz[k] += fz;
            fjx -= fx;
            fjy -= fy;
            fjz -= fz;
        }
        if (valid) {
            atomicAdd(&fj[jslot], fjx);
            atomicAdd(&fj[npad_max + jslot], fjy);
            atomicAdd(&fj[2 * npad_max + jslot], fjz);
        }
    }
#pragma unroll
    for (int k = 0; k < C; ++k) {
        fix[k] = wave_sum(fix[k]);
        fiy[k] = wave_sum(fiy[k]);
        fiz[k] = wave_sum(fiz[k]);
    }
    elj = wave_sum(elj);
    ec = wave_sum(ec);
    double qqd = wave_sum((double)qqs);
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < C; ++k) fi_out[ci * C + k] = make_float4(fix[k], fiy[k], fiz[k], 0.0f);
        epart[4 * ci] = elj;
        epart[4 * ci + 1] = ec;
        epart[4 * ci + 2] = qqd;
    }
}

__global__ void k_finalize(int n, int npad_max, const int *__restrict__ slot_of,
                           const float4 *__restrict__ fi, const float *__restrict__ fj,
                           float *__restrict__ f) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int p = slot_of[i];
    float4 a = fi[p];
    f[3 * i] = a.x + fj[p];
    f[3 * i + 1] = a.y + fj[npad_max + p];
    f[3 * i + 2] = a.z + fj[2 * npad_max + p];
}

// FP64 sum of the per-cluster energy partials; the Coulomb shift is applied here.
__global__ void __launch_bounds__(1024) k_energy(const nb_meta *meta, const double *__restrict__ epart,
                                                  double shift_coul, double *__restrict__ e) {
    __shared__ double s[3][1024 / NB_WAVE];
    const int ncl = meta->nclusters;
    double a = 0.0, b = 0.0, c = 0.0;
    for (int k = threadIdx.x; k < ncl; k += blockDim.x) {
        a += epart[4 * k];
        b += epart[4 * k + 1];
        c += epart[4 * k + 2];
    }
    a = wave_sum(a);
    b = wave_sum(b);
    c = wave_sum(c);
    const int w = threadIdx.x / NB_WAVE;
    if ((threadIdx.x & (NB_WAVE - 1)) == 0) {
        s[0][w] = a;
        s[1][w] = b;
        s[2][w] = c;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double ta = 0.0, tb = 0.0, tc = 0.0;
        for (int k = 0; k < (int)(blockDim.x / NB_WAVE); ++k) {
            ta += s[0][k];
            tb += s[1][k];
            tc += s[2][k];
        }
        e[0] = ta;
        e[1] = tb - shift_coul * tc;
    }
}

}  // namespace

hipError_t nb_launch_pack(nb_ctx *c, const float *x, const float *q, const int32_t *type) {
    const int tb = 256;
    float stale2 = (float)(0.25 * c->rb * c->rb);
    hipLaunchKernelGGL(k_pack, dim3((c->npad_max + tb - 1) / tb), dim3(tb), 0, c->stream,
                       c->npad_max, c->perm, x, q, type, c->ntypes, c->off, c->xbuild, c->flags,
                       stale2, c->xq, c->tsort, c->fj, c->meta);
    return hipGetLastError();
}

hipError_t nb_launch_force(nb_ctx *c) {
    size_t shm = sizeof(float4) * 2 * c->ntypes * c->ntypes;
    dim3 grid((c->ncl_max + 3) / 4), block(256);
    if (c->C == 4)
        hipLaunchKernelGGL((k_force<4>), grid, block, shm, c->stream, c->fp, c->cap, c->npad_max,
                           c->xq, c->tsort, c->ljtab, c->icount, c->jl, c->fi, c->fj, c->epart,
                           c->meta);
    else
        hipLaunchKernelGGL((k_force<8>), grid, block, shm, c->stream, c->fp, c->cap, c->npad_max,
                           c->xq, c->tsort, c->ljtab, c->icount, c->jl, c->fi, c->fj, c->epart,
                           c->meta);
    return hipGetLastError();
}

hipError_t nb_launch_finalize(nb_ctx *c, float *f, double *e) {
    const int tb = 256;
    hipLaunchKernelGGL(k_finalize, dim3((c->natoms + tb - 1) / tb), dim3(tb), 0, c->stream,
                       c->natoms, c->npad_max, c->slot_of, c->fi, c->fj, f);
    hipLaunchKernelGGL(k_energy, dim3(1), dim3(1024), 0, c->stream, c->meta, c->epart,
                       c->shift_coul, e);
    return hipGetLastError();
}
