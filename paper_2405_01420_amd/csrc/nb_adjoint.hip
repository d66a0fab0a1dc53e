// Adjoint (vector-Jacobian product) of the short-range force computation, for force-matching
// losses L(F, E_LJ, E_C).  Given g = dL/dF per atom and (s_LJ, s_C) = dL/dE, every interacting
// pair with d = x_i - x_j, r = |d|, force F_ij = f(r) d on atom i, delta = g_i - g_j contributes
//   dL/dx_i += f delta + (f'(r)/r)(d . delta) d - (s_LJ f_LJ + s_C f_C) d     (-= for j)
//   dL/dq_i += q_j [H (d . delta) + s_C G],  H = fC erfc(b r)/r^3 + fC 2b/sqrt(pi) e^{-b^2 r^2}/r^2,
//              G = fC (erfc(b r)/r - erfc(b rc)/rc)                            (likewise for j)
//   dL/dC6  : G6  = -6 r^-8 (d . delta) - s_LJ (r^-6 - rc^-6)
//   dL/dC12 : G12 = 12 r^-14 (d . delta) + s_LJ (r^-12 - rc^-12)
// The LJ-parameter gradients are chained through Lorentz-Berthelot with per-atom sums
//   Su_i = sum_j (G6 C6 + G12 C12),  Sw_i = sum_j (6 G6 C6 + 12 G12 C12) / sigma_ab,
//   dL/deps_t = sum_{i of type t} Su_i / (2 eps_t),  dL/dsigma_t = sum_{i of type t} Sw_i / 2,
// because each pair's two type slots share d sigma_ab / d sigma_a = 1/2 and
// d eps_ab / d eps_a = eps_ab / (2 eps_a).  The traversal and lane layout are those of the
// force kernel; per-atom sums are FP32, the per-type reduction is FP64.
#include <mutex>

#include "nb_device.h"

namespace {

__global__ void k_pack_g(int npad_max, const int *__restrict__ perm, const float *__restrict__ g,
                         float4 *__restrict__ gs, float *__restrict__ adjj, const nb_meta *meta) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= npad_max) return;
    int a = p < meta->npad ? perm[p] : -1;
    gs[p] = a >= 0 ? make_float4(g[3 * a], g[3 * a + 1], g[3 * a + 2], 0.0f)
                   : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
#pragma unroll
    for (int k = 0; k < 6; ++k) adjj[k * npad_max + p] = 0.0f;
}

// One wavefront per i-cluster, the lanes of the force kernel (one j-atom each, 16 j-groups per
// batch).  A batch is worked through in halves of four i-atoms: a filter forms each lane's pairs
// with the half's i-atoms and appends the interacting ones (r < rc, unmasked) to a per-wave
// queue in LDS as (d, pair code); the queued pairs are then evaluated one per lane, each writing
// its six terms to its place (4-atom half index, lane) in LDS areas cleared for the half; and
// every lane adds the terms of its own pairs (zero where a pair does not interact) to the i- and
// j-side sums in registers, in the same order as a plain loop over the cluster's atoms.  So the
// pair arithmetic runs only on interacting pairs, with all lanes busy.  The pair code holds LDS
// byte addresses: (LJ table row << NB_ADJ_ROW) | (64 kk + lane) * 4 for i-atom 4 h + kk.
#define NB_ADJ_ROW 11
#define NB_ADJ_HALF 4            // i-atoms per half batch
#define NB_ADJ_SLOTS (NB_ADJ_HALF * NB_WAVE)

template <int C>
struct adj_lds {
    float out[6][NB_ADJ_SLOTS];  // per (kk, lane): v_x, v_y, v_z, A, u, w of the pair
    float4 rec[NB_ADJ_SLOTS];    // the half's interacting pairs: (d_x, d_y, d_z, code bits)
    float4 jg[NB_WAVE];          // per lane: the j-atom's (g_x, g_y, g_z, q)
    float4 id[C];                // per i-atom: (x, y, z, q) as loaded
    float4 ig[C];                // per i-atom: (g_x, g_y, g_z, -)
};

template <int C>
__global__ void __launch_bounds__(256) k_adjoint(nb_fparams fp, const double *__restrict__ ge, int cap,
                                                 int npad_max, const float4 *__restrict__ xq,
                                                 const int *__restrict__ tsort,
                                                 const float4 *__restrict__ gs,
                                                 const float4 *__restrict__ ljtab,
                                                 const int *__restrict__ icount,
                                                 const nb_entry *__restrict__ jl,
                                                 float *__restrict__ adj, float *__restrict__ adjj,
                                                 const nb_meta *meta) {
    static_assert(C % NB_ADJ_HALF == 0, "clusters of 4 or 8 atoms");
    extern __shared__ float4 tab[];
    __shared__ __attribute__((aligned(NB_ADJ_SLOTS * 4))) adj_lds<C> wls[256 / NB_WAVE];
    const int nt = fp.ntypes, ntt = nt * nt;
    for (int k = threadIdx.x; k < 2 * ntt; k += blockDim.x) tab[k] = ljtab[k];
    __syncthreads();
    const int lane = threadIdx.x & (NB_WAVE - 1);
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / NB_WAVE);
    const int ci = __builtin_amdgcn_readfirstlane(blockIdx.x * (blockDim.x / NB_WAVE) + wv);
    if (ci >= meta->nclusters) return;
    adj_lds<C> &w = wls[wv];
    const int b = lane % NB_JG, jsub = lane / NB_JG;
    const uint32_t lane4 = (uint32_t)lane * 4u;
    // energy cotangents (dL/dE_LJ, dL/dE_C), read on the device: no host round trip
    const float s_lj = (float)ge[0], s_c = (float)ge[1];

    // the i-atoms: coordinates, charges and cotangents (wave-uniform), and in LDS for the
    // evaluate phase; per i-atom the constant part of its pair codes (LJ row of its type)
    float xi[C], yi[C], zi[C], qi[C];
    uint32_t pci[C];
    const uint32_t tabrow = nb_laddr(tab);
#pragma unroll
    for (int k = 0; k < C; ++k) {
        const float4 v = xq[ci * C + k];
        xi[k] = v.x;
        yi[k] = v.y;
        zi[k] = v.z;
        qi[k] = v.w;
        pci[k] = ((tabrow + 32u * (uint32_t)(tsort[ci * C + k] * nt)) << NB_ADJ_ROW) |
                 ((uint32_t)(k % NB_ADJ_HALF) << 8);
    }
    if (lane < C) {
        w.id[lane] = xq[ci * C + lane];
        w.ig[lane] = gs[ci * C + lane];
    }
    const uint32_t out0 = nb_laddr(&w.out[0][0]);
    const uint32_t recb = nb_laddr(&w.rec[0]);
    float ax[C], ay[C], az[C], aq[C], aw[C], au[C];
#pragma unroll
    for (int k = 0; k < C; ++k) ax[k] = ay[k] = az[k] = aq[k] = aw[k] = au[k] = 0.0f;
    const int nj = icount[ci];
    const nb_entry *lst = jl + (size_t)ci * cap;
    for (int base = 0; base < nj; base += NB_JPB) {
        const int e = base + jsub;
        const bool valid = e < nj;
        const nb_entry en = valid ? lst[e] : nb_make_entry(ci * (C / NB_JG), NB_SHIFT_ZERO, 0u);
        const int s = nb_entry_shift(en);
        const int tx = nb_tx(s), ty = nb_ty(s), tz = nb_tz(s);
        const int jslot = nb_entry_group(en) * NB_JG + b;
        const float4 xj = xq[jslot];
        const float4 gj = gs[jslot];
        const int tj = tsort[jslot];
        const float xjs = xj.x + nb_dj(tx, fp.L[0]), yjs = xj.y + nb_dj(ty, fp.L[1]),
                    zjs = xj.z + nb_dj(tz, fp.L[2]);
        const float dix = nb_di(tx, fp.L[0]), diy = nb_di(ty, fp.L[1]), diz = nb_di(tz, fp.L[2]);
        const float qj = xj.w;
        const unsigned mcol = nb_mask_column<C>(en.mask, b);
        const uint32_t pcj = ((uint32_t)tj << (NB_ADJ_ROW + 5)) | lane4;
        nb_wave_lds_sync();  // the previous batch's reads of the work area are done
        w.jg[lane] = make_float4(gj.x, gj.y, gj.z, qj);
        float jx = 0.0f, jy = 0.0f, jz = 0.0f, jq = 0.0f, jw = 0.0f, ju = 0.0f;
#pragma unroll
        for (int h = 0; h < C / NB_ADJ_HALF; ++h) {
            // ---- filter: the lane's pairs with the half's i-atoms; interacting ones queued
#pragma unroll
            for (int a = 0; a < 6; ++a)
#pragma unroll
                for (int kk = 0; kk < NB_ADJ_HALF; ++kk) w.out[a][kk * NB_WAVE + lane] = 0.0f;
            int nq = 0;
#pragma unroll
            for (int kk = 0; kk < NB_ADJ_HALF; ++kk) {
                const int k = h * NB_ADJ_HALF + kk;
                const float dx = (xi[k] + dix) - xjs;
                const float dy = (yi[k] + diy) - yjs;
                const float dz = (zi[k] + diz) - zjs;
                const float r2 = nb_r2(dx, dy, dz);
                const bool inr = r2 < fp.rc2, inm = ((mcol >> k) & 1u) != 0u;
                const unsigned long long bal =
                    __builtin_amdgcn_ballot_w64(inr) & __builtin_amdgcn_ballot_w64(inm);
                uint32_t qb = recb + 16u * (uint32_t)nq;
                asm("" : "+s"(qb));
                if (inr && inm) {
                    const uint32_t pos = __builtin_amdgcn_mbcnt_hi((unsigned)(bal >> 32),
                                                                   __builtin_amdgcn_mbcnt_lo((unsigned)bal, 0u));
                    nb_lput<float4>(qb + 16u * pos, make_float4(dx, dy, dz, __uint_as_float(pci[k] + pcj)));
                }
                nq += __popcll(bal);
            }
            nb_wave_lds_sync();
            // ---- evaluate: the queued pairs, one per lane
            const int i0 = h * NB_ADJ_HALF;
            auto evaluate = [&](uint32_t qa) {
                const float4 rr = nb_lget<float4>(qa);
                const uint32_t code = __float_as_uint(rr.w);
                const uint32_t ta = code >> NB_ADJ_ROW;
                const float4 lj = nb_lget<float4>(ta);         // (C6, C12, 6 C6, 12 C12)
                const float4 lj2 = nb_lget<float4>(ta + 16u);  // (shift, 1/sigma_ab, -, -)
                const uint32_t kk = (code >> 8) & (NB_ADJ_HALF - 1);
                const float4 ip = w.id[i0 + kk];
                const float4 igk = w.ig[i0 + kk];
                const float4 jgl = nb_lget<float4>(nb_laddr(&w.jg[0]) + ((code & 0xFCu) << 2));
                const float dx = rr.x, dy = rr.y, dz = rr.z;
                const float r2 = nb_r2(dx, dy, dz);
                const float rinv = nb_rsq(r2);
                const float rinv2 = rinv * rinv;
                const float rinv4 = rinv2 * rinv2;
                const float rinv6 = rinv4 * rinv2;
                const float ddx = igk.x - jgl.x, ddy = igk.y - jgl.y, ddz = igk.z - jgl.z;
                const float dd = __builtin_fmaf(dz, ddz, __builtin_fmaf(dy, ddy, dx * ddx));
                // Lennard-Jones
                const float tf = __builtin_fmaf(lj.w, rinv6, -lj.z);      // 12 C12 r^-6 - 6 C6
                const float flj = tf * rinv6 * rinv2;                      // force factor
                const float dflj = __builtin_fmaf(-14.0f * lj.w, rinv6, 8.0f * lj.z) * rinv6 * rinv4;
                // Ewald real space
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
                const float R = P * nb_rcp(Q);             // erfcx(b r)
                const float fe = fp.fc * ex * rinv;                        // fC e^{-b^2r^2} / r
                const float H = fe * __builtin_fmaf(fp.kb, r, R) * rinv2;  // fC h(r)
                const float G = __builtin_fmaf(fe, R, -fp.fc * fp.shc);    // fC g(r)
                // d/dr of fC h(r), divided by r
                const float dH = -fe * rinv4 *
                                 __builtin_fmaf(fp.kb * r, __builtin_fmaf(2.0f * fp.b2, r2, 3.0f), 3.0f * R);
                const float qq = ip.w * jgl.w;
                const float fcl = qq * H;
                const float f = flj + fcl;
                const float dfr = dflj + qq * dH;
                const float coef = __builtin_fmaf(dfr, dd, -__builtin_fmaf(s_lj, flj, s_c * fcl));
                const float vx = __builtin_fmaf(f, ddx, coef * dx);
                const float vy = __builtin_fmaf(f, ddy, coef * dy);
                const float vz = __builtin_fmaf(f, ddz, coef * dz);
                const float A = __builtin_fmaf(H, dd, s_c * G);
                // LJ parameters
                const float r8 = rinv6 * rinv2;
                const float G6 = -6.0f * r8 * dd - s_lj * (rinv6 - fp.irc6);
                const float G12 = 12.0f * r8 * rinv6 * dd + s_lj * (rinv6 * rinv6 - fp.irc12);
                const float u = __builtin_fmaf(G6, lj.x, G12 * lj.y);
                const float wv6 = __builtin_fmaf(G6, lj.z, G12 * lj.w) * lj2.y;
                const uint32_t o = out0 + (code & 0x3FCu);
                nb_lput<float>(o, vx);
                nb_lput<float>(o + 4u * NB_ADJ_SLOTS, vy);
                nb_lput<float>(o + 8u * NB_ADJ_SLOTS, vz);
                nb_lput<float>(o + 12u * NB_ADJ_SLOTS, A);
                nb_lput<float>(o + 16u * NB_ADJ_SLOTS, u);
                nb_lput<float>(o + 20u * NB_ADJ_SLOTS, wv6);
            };
            uint32_t qa = recb + 16u * (uint32_t)lane;
            for (int p = 0; p < (nq >> 6); ++p, qa += 16u * NB_WAVE) evaluate(qa);
            if (lane < (nq & (NB_WAVE - 1))) evaluate(qa);
            nb_wave_lds_sync();
            // ---- accumulate: the terms of the lane's pairs of this half (zero where a pair does
            // not interact), in i-atom order
#pragma unroll
            for (int kk = 0; kk < NB_ADJ_HALF; ++kk) {
                const int k = h * NB_ADJ_HALF + kk;
                const float vx = w.out[0][kk * NB_WAVE + lane], vy = w.out[1][kk * NB_WAVE + lane];
                const float vz = w.out[2][kk * NB_WAVE + lane], A = w.out[3][kk * NB_WAVE + lane];
                const float u = w.out[4][kk * NB_WAVE + lane], wv6 = w.out[5][kk * NB_WAVE + lane];
                ax[k] += vx;
                ay[k] += vy;
                az[k] += vz;
                aq[k] = __builtin_fmaf(qj, A, aq[k]);
                au[k] += u;
                aw[k] += wv6;
                jx -= vx;
                jy -= vy;
                jz -= vz;
                jq = __builtin_fmaf(qi[k], A, jq);
                ju += u;
                jw += wv6;
            }
            nb_wave_lds_sync();  // the next half rewrites the work area
        }
        // lanes without an interacting pair in this batch skip the atomics, and lanes whose
        // LJ-parameter sums are zero (atoms of a type without LJ, such as water hydrogens) skip
        // those two
        if (valid && (jx != 0.0f || jy != 0.0f || jz != 0.0f || jq != 0.0f)) {
            atomicAdd(&adjj[jslot], jx);
            atomicAdd(&adjj[npad_max + jslot], jy);
            atomicAdd(&adjj[2 * npad_max + jslot], jz);
            atomicAdd(&adjj[3 * npad_max + jslot], jq);
        }
        if (valid && (jw != 0.0f || ju != 0.0f)) {
            atomicAdd(&adjj[4 * npad_max + jslot], jw);
            atomicAdd(&adjj[5 * npad_max + jslot], ju);
        }
    }
    // the i-side sums: a reduce-scatter across the wave leaves atom k's in the lanes with
    // lane / (64 / C) == k; the first lane of each group stores them
    const float sx = nb_wave_scatter_sum<C>(ax, lane), sy = nb_wave_scatter_sum<C>(ay, lane);
    const float sz = nb_wave_scatter_sum<C>(az, lane), sq = nb_wave_scatter_sum<C>(aq, lane);
    const float sw = nb_wave_scatter_sum<C>(aw, lane), su = nb_wave_scatter_sum<C>(au, lane);
    if (lane % (NB_WAVE / C) == 0) {
        const int p = ci * C + lane / (NB_WAVE / C);
        adj[p] = sx;
        adj[npad_max + p] = sy;
        adj[2 * npad_max + p] = sz;
        adj[3 * npad_max + p] = sq;
        adj[4 * npad_max + p] = sw;
        adj[5 * npad_max + p] = su;
    }
}

__global__ void k_adj_finalize(int n, int npad_max, const int *__restrict__ slot_of,
                               const float *__restrict__ adj, const float *__restrict__ adjj,
                               float *__restrict__ dx, float *__restrict__ dq) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int p = slot_of[i];
    dx[3 * i] = adj[p] + adjj[p];
    dx[3 * i + 1] = adj[npad_max + p] + adjj[npad_max + p];
    dx[3 * i + 2] = adj[2 * npad_max + p] + adjj[2 * npad_max + p];
    dq[i] = adj[3 * npad_max + p] + adjj[3 * npad_max + p];
}

// Per-type FP64 sums of the per-atom LJ-parameter terms, in two deterministic steps.  Step 1:
// each block takes NB_TYPE_SPAN consecutive slots per thread and reduces, type by type, the
// terms of its real atoms of that type (thread, wave and block trees in fixed order) into
// part[block][type][2].  Step 2: one block per type adds the block partials in block order.
#define NB_TYPE_SPAN 8

__global__ void __launch_bounds__(256) k_adj_types_part(int ntypes, int npad_max,
                                                        const int *__restrict__ perm,
                                                        const int *__restrict__ tsort,
                                                        const float *__restrict__ adj,
                                                        const float *__restrict__ adjj,
                                                        double *__restrict__ part) {
    __shared__ double sw[256 / NB_WAVE], su[256 / NB_WAVE];
    const int p0 = (blockIdx.x * blockDim.x + threadIdx.x) * NB_TYPE_SPAN;
    float w[NB_TYPE_SPAN], u[NB_TYPE_SPAN];
    int t[NB_TYPE_SPAN];
#pragma unroll
    for (int k = 0; k < NB_TYPE_SPAN; ++k) {
        const int p = p0 + k;
        const bool real = p < npad_max && perm[p] >= 0;
        t[k] = real ? tsort[p] : -1;
        w[k] = real ? adj[4 * npad_max + p] + adjj[4 * npad_max + p] : 0.0f;
        u[k] = real ? adj[5 * npad_max + p] + adjj[5 * npad_max + p] : 0.0f;
    }
    for (int ty = 0; ty < ntypes; ++ty) {
        double W = 0.0, U = 0.0;
#pragma unroll
        for (int k = 0; k < NB_TYPE_SPAN; ++k) {
            if (t[k] == ty) {
                W += (double)w[k];
                U += (double)u[k];
            }
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            W += __shfl_xor(W, o, NB_WAVE);
            U += __shfl_xor(U, o, NB_WAVE);
        }
        __syncthreads();  // the previous type's block sums have been read
        if ((threadIdx.x & (NB_WAVE - 1)) == 0) {
            sw[threadIdx.x / NB_WAVE] = W;
            su[threadIdx.x / NB_WAVE] = U;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double bw = 0.0, bu = 0.0;
            for (int k = 0; k < (int)(blockDim.x / NB_WAVE); ++k) {
                bw += sw[k];
                bu += su[k];
            }
            part[2 * (blockIdx.x * ntypes + ty)] = bw;
            part[2 * (blockIdx.x * ntypes + ty) + 1] = bu;
        }
    }
}

__global__ void __launch_bounds__(256) k_adj_types(nb_typeparams tp, int nblk,
                                                   const double *__restrict__ part,
                                                   double *__restrict__ dsig, double *__restrict__ deps) {
    __shared__ double sw[256 / NB_WAVE], su[256 / NB_WAVE];
    const int t = blockIdx.x;
    double w = 0.0, u = 0.0;
    for (int b = threadIdx.x; b < nblk; b += blockDim.x) {
        w += part[2 * (b * tp.ntypes + t)];
        u += part[2 * (b * tp.ntypes + t) + 1];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        w += __shfl_xor(w, o, NB_WAVE);
        u += __shfl_xor(u, o, NB_WAVE);
    }
    if ((threadIdx.x & (NB_WAVE - 1)) == 0) {
        sw[threadIdx.x / NB_WAVE] = w;
        su[threadIdx.x / NB_WAVE] = u;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double W = 0.0, U = 0.0;
        for (int k = 0; k < (int)(blockDim.x / NB_WAVE); ++k) {
            W += sw[k];
            U += su[k];
        }
        dsig[t] = 0.5 * W;
        deps[t] = tp.eps[t] > 0.0 ? U / (2.0 * tp.eps[t]) : 0.0;
    }
}

}  // namespace

// Work buffers of one adjoint call: per slot the i- and j-side sums (6 floats each) and the force
// cotangents in cluster order, and the per-block type partials.
struct nb_adj_bufs {
    float *adj, *adjj;
    float4 *gs;
    double *tpart;
};

static int adj_type_blocks(int npad_max) {
    return (npad_max + 256 * NB_TYPE_SPAN - 1) / (256 * NB_TYPE_SPAN);
}

static hipError_t launch_adjoint(nb_ctx *c, const nb_adj_bufs &b, const float *gf, const double *ge,
                                 float *dx, float *dq, double *dsig, double *deps) {
    const int tb = 256;
    hipLaunchKernelGGL(k_pack_g, dim3((c->npad_max + tb - 1) / tb), dim3(tb), 0, c->stream,
                       c->npad_max, c->perm, gf, b.gs, b.adjj, c->meta);
    size_t shm = sizeof(float4) * 2 * c->ntypes * c->ntypes;
    dim3 grid((c->ncl_max + 3) / 4), block(256);
    if (c->C == 4)
        hipLaunchKernelGGL((k_adjoint<4>), grid, block, shm, c->stream, c->fp, ge, c->cap,
                           c->npad_max, c->xq, c->tsort, b.gs, c->ljtab, c->icount, c->jl, b.adj,
                           b.adjj, c->meta);
    else
        hipLaunchKernelGGL((k_adjoint<8>), grid, block, shm, c->stream, c->fp, ge, c->cap,
                           c->npad_max, c->xq, c->tsort, b.gs, c->ljtab, c->icount, c->jl, b.adj,
                           b.adjj, c->meta);
    hipLaunchKernelGGL(k_adj_finalize, dim3((c->natoms + tb - 1) / tb), dim3(tb), 0, c->stream,
                       c->natoms, c->npad_max, c->slot_of, b.adj, b.adjj, dx, dq);
    nb_typeparams tp{};
    tp.ntypes = c->ntypes;
    for (int t = 0; t < c->ntypes; ++t) tp.eps[t] = c->epsilon[t];
    const int nblk = adj_type_blocks(c->npad_max);
    hipLaunchKernelGGL(k_adj_types_part, dim3(nblk), dim3(tb), 0, c->stream, c->ntypes, c->npad_max,
                       c->perm, c->tsort, b.adj, b.adjj, b.tpart);
    hipLaunchKernelGGL(k_adj_types, dim3(c->ntypes), dim3(256), 0, c->stream, tp, nblk, b.tpart,
                       dsig, deps);
    return hipGetLastError();
}

hipError_t nb_launch_adjoint(nb_ctx *c, const float *gf, const double *ge, float *dx, float *dq,
                             double *dsig, double *deps) {
    if (!c->adj) {
        if (hipMalloc((void **)&c->adj, sizeof(float) * 6 * (size_t)c->npad_max) != hipSuccess)
            return hipErrorOutOfMemory;
        if (hipMalloc((void **)&c->adjj, sizeof(float) * 6 * (size_t)c->npad_max) != hipSuccess)
            return hipErrorOutOfMemory;
        if (hipMalloc((void **)&c->gs, sizeof(float4) * (size_t)c->npad_max) != hipSuccess)
            return hipErrorOutOfMemory;
        if (hipMalloc((void **)&c->tpart, sizeof(double) * 2 * adj_type_blocks(c->npad_max) * c->ntypes) != hipSuccess)
            return hipErrorOutOfMemory;
    }
    return launch_adjoint(c, nb_adj_bufs{c->adj, c->adjj, c->gs, c->tpart}, gf, ge, dx, dq, dsig, deps);
}

// ---- allocation-free adjoint: the work buffers in a static device array -----------------------
//
// One array per device, holding the buffers of one call of at most NB_NOALLOC_MAX_SLOTS padded
// slots (64 bytes each) and the type partials.  Its host-side name is not a device address: the
// device address is looked up once per device (nb_noalloc_init, called by nb_setup with the
// context's device current) and only that address is handed to kernels.  Every call on a device
// shares its array, so calls that overlap on one device (other streams, other host threads)
// race; every buffer is fully written by the call before it is read.
#define NB_NOALLOC_TPART_BYTES \
    (2 * sizeof(double) * NB_MAX_TYPES * ((NB_NOALLOC_MAX_SLOTS + 256 * NB_TYPE_SPAN - 1) / (256 * NB_TYPE_SPAN)))
#define NB_NOALLOC_BYTES (64 * (size_t)NB_NOALLOC_MAX_SLOTS + NB_NOALLOC_TPART_BYTES)

static __device__ __align__(256) unsigned char scratch[NB_NOALLOC_BYTES];

#define NB_NOALLOC_MAX_DEVICES 64
static std::mutex g_scratch_mutex;
static void *g_scratch_dev[NB_NOALLOC_MAX_DEVICES];

hipError_t nb_noalloc_init(int device) {
    if (device < 0 || device >= NB_NOALLOC_MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (g_scratch_dev[device]) return hipSuccess;
    void *ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_dev[device] = ptr;
    return hipSuccess;
}

hipError_t nb_launch_adjoint_noalloc(nb_ctx *c, const float *gf, const double *ge, float *dx,
                                     float *dq, double *dsig, double *deps) {
    void *base = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mutex);
        if (c->device >= 0 && c->device < NB_NOALLOC_MAX_DEVICES) base = g_scratch_dev[c->device];
    }
    if (!base) return hipErrorNotInitialized;
    const size_t n = (size_t)c->npad_max;
    unsigned char *p = static_cast<unsigned char *>(base);
    nb_adj_bufs b;
    b.adj = reinterpret_cast<float *>(p);
    b.adjj = reinterpret_cast<float *>(p + 24 * n);
    b.gs = reinterpret_cast<float4 *>(p + 48 * n);
    b.tpart = reinterpret_cast<double *>(p + 64 * n);
    return launch_adjoint(c, b, gf, ge, dx, dq, dsig, deps);
}
