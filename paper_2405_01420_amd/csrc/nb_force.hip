// Per-call force path: pack (gather positions/charges/types into cluster order), the
// cluster-pair force kernel (Lennard-Jones with potential shift + Ewald real-space Coulomb),
// and the finalize step (un-permute, f = f_i + f_j, FP64 energies with the shifts applied).
//
// This is the computation the paper identifies as the single-GPU rate limiter (section III-A;
// the flavour named in the Fig. 3 caption).  The per-cluster body and its lane layout are in
// nb_force_body.h; here one wavefront is launched per work unit (an i-cluster's list or a part
// of a long one).
#include <hip/hip_ext.h>

#include <algorithm>

#include "nb_force_body.h"

namespace {

#define NB_FIN_BLOCK 512

// Positions (wrapped as at the build), charges and types into the cluster slots, one thread per
// atom in input order: every load is contiguous across the wave and independent of the others,
// and each store goes to the atom's slot.  Padding slots keep what the build's column sort wrote
// into them (far coordinates, type 0).  The fixed-point force sums are zero here already: the
// finalize clears every slot it reads, and no other slot receives anything (the sums that would
// reach padding slots are zero, and zero sums are skipped).
__global__ void k_pack(int n, const int *__restrict__ slot_of, const float *__restrict__ x,
                       const float *__restrict__ q, const int32_t *__restrict__ type, int ntypes,
                       const float4 *__restrict__ off, const float *__restrict__ xbuild,
                       uint32_t checks, float stale2, float4 *__restrict__ xq,
                       int *__restrict__ tsort, nb_meta *meta) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= n) return;
    // every load first, so that they are in flight together (the charge and type pointers are
    // null where only positions are packed)
    const int p = slot_of[a];
    const float x0 = x[3 * a], x1 = x[3 * a + 1], x2 = x[3 * a + 2];
    const float4 o = off[a];
    const float qa = q ? q[a] : 0.0f;
    int t = type ? type[a] : 0;
    if (checks & NB_CHECK_STALE) {
        float d0 = x0 - xbuild[3 * a], d1 = x1 - xbuild[3 * a + 1], d2 = x2 - xbuild[3 * a + 2];
        if (!(d0 * d0 + d1 * d1 + d2 * d2 < stale2)) atomicOr(&meta->flags, NB_F_STALE);
    }
    if ((checks & NB_CHECK_FINITE) && !(isfinite(x0) && isfinite(x1) && isfinite(x2)))
        atomicOr(&meta->flags, NB_F_NONFINITE);
    t = min(max(t, 0), ntypes - 1);
    xq[p] = make_float4(x0 + o.x, x1 + o.y, x2 + o.z, qa);
    tsort[p] = t;
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

// One work unit per wave, NB_FORCE_WAVES consecutive units per workgroup (neighbouring waves work
// on neighbouring clusters, whose j-atoms they share in the caches).  The energy sums of the
// workgroup's waves are combined in LDS by whichever wave finishes last, in wave order, and
// stored as the workgroup's partial (epart[4 blockIdx ..], virial vpart[6 blockIdx ..]; zeros
// from workgroups without a unit); waves do not wait for each other.  (Workgroups that take
// several units in turn, statically or from a shared counter, were measured slower: the former
// coarsen the tail of the launch, the latter serialise on the counter's atomics.)
#define NB_FORCE_WAVES 4

template <int C, bool EPREC, int FLAV, bool VIR>
__global__ void __launch_bounds__(NB_FORCE_WAVES * NB_WAVE) NB_FORCE_OCCUPANCY_VIR k_force(nb_fparams fp, int cap, int npad_max,
                                               const float4 *__restrict__ xq,
                                               const int *__restrict__ tsort,
                                               const float4 *__restrict__ ljtab,
                                               const double2 *__restrict__ etab, int etab_n,
                                               float etab_invh, const float4 *__restrict__ ftab,
                                               const int *__restrict__ icount,
                                               const nb_entry *__restrict__ jl,
                                               const int4 *__restrict__ units, float *__restrict__ fj,
                                               double *__restrict__ epart, double *__restrict__ vpart,
                                               nb_meta *meta) {
    extern __shared__ float4 tab[];
    __shared__ __attribute__((aligned(C * NB_WAVE * 4))) nb_wg_lds<C, EPREC, FLAV, NB_FORCE_WAVES> wl;
    __shared__ double esh[NB_FORCE_WAVES][VIR ? 9 : 3];
    __shared__ int edone;
    const int nunits = meta->nunits;
    if (blockIdx.x * NB_FORCE_WAVES >= nunits) {
        // an idle workgroup writes zero partials, so that the finalize can sum every
        // workgroup's row
        if (threadIdx.x < 4) epart[4 * blockIdx.x + threadIdx.x] = 0.0;
        if (VIR && threadIdx.x < 6) vpart[6 * blockIdx.x + threadIdx.x] = 0.0;
        return;
    }
    const int ntt = fp.ntypes * fp.ntypes;
    if (threadIdx.x == 0) edone = 0;
    nb_load_ljtab(tab, ljtab, ntt);
    nb_etab et;
    et.seg = reinterpret_cast<const double2 *>(tab + 2 * ntt);
    et.invh = etab_invh;
    et.n = etab_n;
    if (EPREC) {
        double2 *dst = reinterpret_cast<double2 *>(tab + 2 * ntt);
        for (int k = threadIdx.x; k < NB_ETAB_W * etab_n; k += blockDim.x) dst[k] = etab[k];
    }
    // tabulated Ewald: the force segments after the erfc table
    float4 *fdst = tab + 2 * ntt + NB_ETAB_W * etab_n;
    et.fseg = fdst;
    if (FLAV / 2 == NB_ELEC_EWALD_TAB)
        for (int k = threadIdx.x; k < NB_TAB_SEGMENTS; k += blockDim.x) fdst[k] = ftab[k];
    __syncthreads();
    const int lane = threadIdx.x & (NB_WAVE - 1);
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / NB_WAVE);
    const int u = __builtin_amdgcn_readfirstlane(blockIdx.x * NB_FORCE_WAVES + wv);
    nb_esum es{0.0, 0.0, 0.0, {0.0, 0.0, 0.0, 0.0, 0.0, 0.0}};
    if (u < nunits) {
        const int4 wu = units[u];
        es = nb_force_cluster<C, EPREC, FLAV, VIR>(
            fp, tab, et, nb_wave_view(wl, wv), __builtin_amdgcn_readfirstlane(wu.x),
            __builtin_amdgcn_readfirstlane(wu.y), __builtin_amdgcn_readfirstlane(wu.z), cap, npad_max,
            nb_g(xq), nb_g(tsort), nb_g(icount), nb_g(jl), nb_g(fj), nb_g(&meta->flags));
    }
    if (lane == 0) {
        esh[wv][0] = es.elj;
        esh[wv][1] = es.ec;
        esh[wv][2] = es.qq;
        if (VIR) {
#pragma unroll
            for (int m = 0; m < 6; ++m) esh[wv][3 + m] = es.v[m];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        const bool last = __hip_atomic_fetch_add(&edone, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) ==
                          NB_FORCE_WAVES - 1;
        if (last) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            double a = 0.0, b = 0.0, c = 0.0;
            for (int k = 0; k < NB_FORCE_WAVES; ++k) {
                a += esh[k][0];
                b += esh[k][1];
                c += esh[k][2];
            }
            epart[4 * blockIdx.x] = a;
            epart[4 * blockIdx.x + 1] = b;
            epart[4 * blockIdx.x + 2] = c;
            if (VIR) {
                for (int m = 0; m < 6; ++m) {
                    double v = 0.0;
                    for (int k = 0; k < NB_FORCE_WAVES; ++k) v += esh[k][3 + m];
                    vpart[6 * blockIdx.x + m] = v;
                }
            }
        }
    }
}

// Ewald exclusion correction and self term (NB_EWALD_CORR), run between the force kernel and
// the finalize, one thread per atom, all in FP64: for each excluded partner j of atom i at the
// minimum-image displacement d (r = |d|), the force fC q_i q_j (2 beta/sqrt(pi) exp(-beta^2 r^2)
// / r^2 - erf(beta r) / r^3) d is added to atom i's slot of fj (each slot has one owner, and the
// force kernel is complete), and the energy -fC q_i q_j erf(beta r) / r is counted at i < j;
// the self term is -fC beta / sqrt(pi) q_i^2.  The block sums (the two energies and the pair
// sums of f d_a d_b for the virial) go to cpart[NB_CORR_PART block ..].
__global__ void __launch_bounds__(NB_CORR_BLOCK) k_ewald_corr(int n, int npad_max,
                                                              const float *__restrict__ x,
                                                              const float *__restrict__ q,
                                                              const int *__restrict__ eoff,
                                                              const int *__restrict__ eidx,
                                                              const int *__restrict__ slot_of,
                                                              double3 box, double beta, double fc,
                                                              float *__restrict__ fj,
                                                              double *__restrict__ cpart) {
    constexpr double two_over_sqrt_pi = 1.1283791670955126;
    __shared__ double s[NB_CORR_PART][NB_CORR_BLOCK / NB_WAVE];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    double ex = 0.0, es = 0.0, v[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (i < n) {
        const double qi = q[i];
        es = -fc * beta * (0.5 * two_over_sqrt_pi) * qi * qi;
        if (eoff) {
            const double xi = x[3 * i], yi = x[3 * i + 1], zi = x[3 * i + 2];
            double fx = 0.0, fy = 0.0, fz = 0.0;
            for (int k = eoff[i]; k < eoff[i + 1]; ++k) {
                const int j = eidx[k];
                double dx = xi - (double)x[3 * j], dy = yi - (double)x[3 * j + 1], dz = zi - (double)x[3 * j + 2];
                dx -= box.x * rint(dx / box.x);
                dy -= box.y * rint(dy / box.y);
                dz -= box.z * rint(dz / box.z);
                const double r2 = dx * dx + dy * dy + dz * dz;
                const double qq = fc * qi * (double)q[j];
                double e, fs;
                if (r2 == 0.0) {
                    e = -qq * two_over_sqrt_pi * beta;
                    fs = 0.0;
                } else {
                    const double r = sqrt(r2), er = erf(beta * r);
                    e = -qq * er / r;
                    fs = qq * (two_over_sqrt_pi * beta * exp(-beta * beta * r2) / r2 - er / (r2 * r));
                }
                fx += fs * dx;
                fy += fs * dy;
                fz += fs * dz;
                if (i < j) {
                    ex += e;
                    v[0] += fs * dx * dx;
                    v[1] += fs * dy * dy;
                    v[2] += fs * dz * dz;
                    v[3] += fs * dx * dy;
                    v[4] += fs * dx * dz;
                    v[5] += fs * dy * dz;
                }
            }
            const int p = slot_of[i];
            // fixed-point accumulators (the force kernel's layout); this thread owns the slot
            reinterpret_cast<unsigned long long *>(fj)[p] += nb_fix_xy((float)fx, (float)fy);
            reinterpret_cast<int *>(fj + 2 * npad_max)[p] += nb_fix((float)fz);
        }
    }
    ex = nb_wave_sum_d(ex);
    es = nb_wave_sum_d(es);
#pragma unroll
    for (int m = 0; m < 6; ++m) v[m] = nb_wave_sum_d(v[m]);
    const int w = threadIdx.x / NB_WAVE;
    if ((threadIdx.x & (NB_WAVE - 1)) == 0) {
        s[0][w] = ex;
        s[1][w] = es;
        for (int m = 0; m < 6; ++m) s[2 + m][w] = v[m];
    }
    __syncthreads();
    if (threadIdx.x < NB_CORR_PART) {
        double a = 0.0;
        for (int k = 0; k < NB_CORR_BLOCK / NB_WAVE; ++k) a += s[threadIdx.x][k];
        cpart[NB_CORR_PART * blockIdx.x + threadIdx.x] = a;
    }
}

// Sum over the rows [0, nrow) of the first K columns of a row-major table of row stride S, by
// one block of NB_FIN_BLOCK threads: rows strided over the threads, then the wave and block
// trees.  Every thread gets the K sums; the order is fixed, so they are reproducible.
template <int K>
__device__ __forceinline__ void fin_block_sum(const double *__restrict__ tab, int nrow, int stride,
                                              double *out, double (*s)[NB_FIN_BLOCK / NB_WAVE]) {
    double a[K];
#pragma unroll
    for (int k = 0; k < K; ++k) a[k] = 0.0;
#pragma unroll 8
    for (int r = threadIdx.x; r < nrow; r += NB_FIN_BLOCK) {
#pragma unroll
        for (int k = 0; k < K; ++k) a[k] += tab[(size_t)stride * r + k];
    }
    const int w = threadIdx.x / NB_WAVE;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        a[k] = nb_wave_sum_d(a[k]);
        if ((threadIdx.x & (NB_WAVE - 1)) == 0) s[k][w] = a[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) {
        double t = 0.0;
        for (int j = 0; j < NB_FIN_BLOCK / NB_WAVE; ++j) t += s[k][j];
        out[k] = t;
    }
    __syncthreads();  // s is reused by the next call
}

// f[atom] in original order, and the FP64 energy sums.  Blocks 1 .. take one cluster slot per
// thread: its atom index and its fixed-point sums are loaded together (contiguous), the force
// goes to the atom's place, and the sums are cleared for the next call.  Block 0, dispatched
// first, adds the energy partials of all np force workgroups in order (strided per thread, then
// the wave and block trees) and applies the Coulomb shift, beside the other blocks' work and
// without inter-block synchronisation.
__global__ void __launch_bounds__(NB_FIN_BLOCK) k_finalize(int npad_max, int np,
                                                           const int *__restrict__ perm,
                                                           float *__restrict__ fj,
                                                           float *__restrict__ f,
                                                           const double *__restrict__ epart,
                                                           const double *__restrict__ cpart,
                                                           int ncpart, double shift_coul,
                                                           double coul_scale,
                                                           double *__restrict__ e,
                                                           const double *__restrict__ vpart,
                                                           double *__restrict__ vir) {
    __shared__ double s[8][NB_FIN_BLOCK / NB_WAVE];
    if (blockIdx.x != 0) {
        const int p = (blockIdx.x - 1) * blockDim.x + threadIdx.x;
        if (p >= npad_max) return;
        const int a = perm[p];
        // fixed-point sums: x in the low 32 bits of the xy word, y above it, z on its own
        unsigned long long *const wp = reinterpret_cast<unsigned long long *>(fj) + p;
        int *const zp = reinterpret_cast<int *>(fj + 2 * npad_max) + p;
        const unsigned long long w = *wp;
        const int iz = *zp;
        if (a < 0) return;
        *wp = 0ull;
        *zp = 0;
        const int ix = (int)(unsigned)w;
        const int iy = (int)((w - (unsigned long long)(long long)ix) >> 32);
        f[3 * a] = (float)ix * (1.0f / NB_FSCALE);
        f[3 * a + 1] = (float)iy * (1.0f / NB_FSCALE);
        f[3 * a + 2] = (float)iz * (1.0f / NB_FSCALE);
        return;
    }
    // energies: the force workgroups' partials; then the Ewald-correction and virial partials
    double en[3];
    fin_block_sum<3>(epart, np, 4, en, s);
    double cp[NB_CORR_PART] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (ncpart > 0) fin_block_sum<NB_CORR_PART>(cpart, ncpart, NB_CORR_PART, cp, s);
    double vp[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (vir) fin_block_sum<6>(vpart, np, 6, vp, s);
    if (threadIdx.x == 0) {
        e[0] = en[0];
        e[1] = coul_scale * (en[1] - shift_coul * en[2]);
        if (ncpart > 0) {
            e[2] = cp[0];
            e[3] = cp[1];
        }
        if (vir) {
            // Xi = -1/2 sum over pairs of d (x) F_ij with F_ij = f d (xx, yy, zz, xy, xz, yz)
            double v[6];
            for (int m = 0; m < 6; ++m) v[m] = -0.5 * (vp[m] + cp[2 + m]);
            vir[0] = v[0];
            vir[4] = v[1];
            vir[8] = v[2];
            vir[1] = vir[3] = v[3];
            vir[2] = vir[6] = v[4];
            vir[5] = vir[7] = v[5];
        }
    }
}

}  // namespace

hipError_t nb_launch_pack(nb_ctx *c, const float *x, const float *q, const int32_t *type) {
    const int tb = 256;
    float stale2 = (float)(0.25 * c->rb * c->rb);
    hipLaunchKernelGGL(k_pack, dim3((c->natoms + tb - 1) / tb), dim3(tb), 0, c->stream, c->natoms,
                       c->slot_of, x, q, type, c->ntypes, c->off, c->xbuild, c->flags, stale2, c->xq,
                       c->tsort, c->meta);
    return hipGetLastError();
}

template <int C, bool EPREC, int FLAV, bool VIR>
static void launch_force_t(nb_ctx *c, hipEvent_t ev0, hipEvent_t ev1) {
    const bool tabf = FLAV / 2 == NB_ELEC_EWALD_TAB;
    const size_t shm = sizeof(float4) * 2 * c->ntypes * c->ntypes +
                       (EPREC ? sizeof(double2) * NB_ETAB_W * c->etab_n : 0) +
                       (tabf ? sizeof(float4) * NB_TAB_SEGMENTS : 0);
    const dim3 grid((c->unit_cap + NB_FORCE_WAVES - 1) / NB_FORCE_WAVES), block(NB_FORCE_WAVES * NB_WAVE);
    hipExtLaunchKernelGGL((k_force<C, EPREC, FLAV, VIR>), grid, block, (uint32_t)shm, c->stream, ev0, ev1, 0u, c->fp, c->cap,
                       c->npad_max, c->xq, c->tsort, c->ljtab, c->etab, EPREC ? c->etab_n : 0,
                       c->etab_invh, c->ftab, c->icount, c->jl, c->units, c->fj, c->epart,
                       c->vpart, c->meta);
}

template <int C, int FLAV>
static void launch_force_f(nb_ctx *c, bool vir, hipEvent_t e0, hipEvent_t e1) {
    if constexpr (FLAV / 2 == NB_ELEC_EWALD_TAB) {
        // the tabulated flavour always evaluates its pair energies in FP64
        if (vir) launch_force_t<C, true, FLAV, true>(c, e0, e1);
        else launch_force_t<C, true, FLAV, false>(c, e0, e1);
    } else {
        const bool ep = (c->flags & NB_ENERGY_FP64) != 0;
        if (vir) {
            if (ep) launch_force_t<C, true, FLAV, true>(c, e0, e1);
            else launch_force_t<C, false, FLAV, true>(c, e0, e1);
        } else {
            if (ep) launch_force_t<C, true, FLAV, false>(c, e0, e1);
            else launch_force_t<C, false, FLAV, false>(c, e0, e1);
        }
    }
}

template <int C>
static void launch_force_c(nb_ctx *c, bool vir, hipEvent_t e0, hipEvent_t e1) {
    switch (NB_FLAV(c->elec, c->vdw)) {
    case NB_FLAV(NB_ELEC_EWALD, NB_VDW_SHIFT):
        launch_force_f<C, NB_FLAV(NB_ELEC_EWALD, NB_VDW_SHIFT)>(c, vir, e0, e1);
        break;
    case NB_FLAV(NB_ELEC_EWALD, NB_VDW_FSWITCH):
        launch_force_f<C, NB_FLAV(NB_ELEC_EWALD, NB_VDW_FSWITCH)>(c, vir, e0, e1);
        break;
    case NB_FLAV(NB_ELEC_RF, NB_VDW_SHIFT):
        launch_force_f<C, NB_FLAV(NB_ELEC_RF, NB_VDW_SHIFT)>(c, vir, e0, e1);
        break;
    case NB_FLAV(NB_ELEC_EWALD_TAB, NB_VDW_SHIFT):
        launch_force_f<C, NB_FLAV(NB_ELEC_EWALD_TAB, NB_VDW_SHIFT)>(c, vir, e0, e1);
        break;
    case NB_FLAV(NB_ELEC_EWALD_TAB, NB_VDW_FSWITCH):
        launch_force_f<C, NB_FLAV(NB_ELEC_EWALD_TAB, NB_VDW_FSWITCH)>(c, vir, e0, e1);
        break;
    default:
        launch_force_f<C, NB_FLAV(NB_ELEC_RF, NB_VDW_FSWITCH)>(c, vir, e0, e1);
        break;
    }
}

hipError_t nb_launch_force(nb_ctx *c, bool vir, hipEvent_t e0, hipEvent_t e1) {
    if (c->C == 4) launch_force_c<4>(c, vir, e0, e1);
    else launch_force_c<8>(c, vir, e0, e1);
    return hipGetLastError();
}

hipError_t nb_launch_ewald_corr(nb_ctx *c, const float *x, const float *q) {
    const int nblk = (c->natoms + NB_CORR_BLOCK - 1) / NB_CORR_BLOCK;
    hipLaunchKernelGGL(k_ewald_corr, dim3(nblk), dim3(NB_CORR_BLOCK), 0, c->stream, c->natoms,
                       c->npad_max, x, q, c->nnz_excl > 0 ? c->excl_off : nullptr, c->excl_idx,
                       c->slot_of, make_double3(c->box[0], c->box[1], c->box[2]), c->beta, c->fc,
                       c->fj, c->cpart);
    return hipGetLastError();
}

hipError_t nb_launch_finalize(nb_ctx *c, float *f, double *e, double *vir) {
    const int nblk = 1 + (c->npad_max + NB_FIN_BLOCK - 1) / NB_FIN_BLOCK;
    hipLaunchKernelGGL(k_finalize, dim3(nblk), dim3(NB_FIN_BLOCK), 0, c->stream, c->npad_max,
                       (c->unit_cap + NB_FORCE_WAVES - 1) / NB_FORCE_WAVES, c->perm, c->fj, f, c->epart, c->cpart,
                       (c->flags & NB_EWALD_CORR) ? (c->natoms + NB_CORR_BLOCK - 1) / NB_CORR_BLOCK : 0,
                       c->shift_coul, nb_energy_fp64(c) ? c->fc : 1.0, e, c->vpart, vir);
    return hipGetLastError();
}
