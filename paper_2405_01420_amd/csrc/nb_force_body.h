// Body of the short-range force computation for one i-cluster, shared by the single-box
// kernel and the persistent batched kernel.  Layout (a from-scratch design for a 64-wide
// wavefront):
//  * one wavefront per i-cluster; the C i-atoms are wave-uniform values, so every i-coordinate
//    is a scalar operand of the vector instructions;
//  * each lane owns one j-atom of one of the 16 four-atom j-groups of the current batch and
//    loops over the C i-atoms, so the j-force of the lane's atom accumulates in registers and
//    needs one atomic add per component per batch (the only atomics);
//  * batches whose entries share one periodic shift (the common case, since the list is grouped
//    by shift) use i-coordinates moved into that frame once and cached in scalar registers;
//    batches with no excluded or padding pair skip the mask test;
//  * the i-forces accumulate per lane over the whole list and are reduced across the 64 lanes
//    once per i-cluster with DPP row operations;
//  * erfc(beta r) = exp(-beta^2 r^2) P(r) / Q(r) with a (4,5) rational fit of the scaled
//    complementary error function (fit_erfcx.py), Newton-refined reciprocal square root and
//    reciprocal;
//  * per-pair energies are summed in FP32 over the C pairs of a lane's batch and accumulated in
//    FP64 from there on; the Coulomb potential
//    shift is applied in FP64 at the end from the sum of q_i q_j over interacting pairs;
//  * with EPREC the pair energies are instead evaluated in FP64 (exact displacement,
//    Newton-refined 1/r, erfc from an FP64 cubic Hermite table), forces staying FP32: the FP32
//    rounding noise of the pair energies is otherwise not averaged below 1e-6 of an energy
//    that is a 1e-4 .. 1e-3-conditioned sum, in boxes of a few thousand atoms.
#pragma once
#include "nb_device.h"

// Four waves per SIMD (at most 128 VGPRs) for the force kernels: the FP32 C = 8 body needs
// about that many, and the compiler's unconstrained choice lands just above, at three waves.
// The FP64-energy variant is register-bound either way and is left to the compiler.
#define NB_FORCE_OCCUPANCY __attribute__((amdgpu_waves_per_eu(EPREC ? 1 : 4)))
// With the virial sums (six more accumulators per lane) the FP32 body needs more than 128
// VGPRs: three waves per SIMD.
#define NB_FORCE_OCCUPANCY_VIR __attribute__((amdgpu_waves_per_eu(EPREC ? 1 : (VIR ? 3 : 4))))

__device__ __forceinline__ double nb_wave_sum_d(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, NB_WAVE);
    return v;
}

// Per-lane state of one batch: the lane's j-atom (shifted into the pair frame), its charge,
// type row offset and mask column; accumulators for its j-force.
struct nb_jlane {
    float x, y, z, q;   // q includes the Coulomb constant
    int t;
    unsigned mcol;
    float fx, fy, fz;
    double xd, yd, zd, qd;  // FP64 copies (exact) for the FP64 energy mode; qd without fC
};

// Erfc table of the FP64 energy mode: cubic Hermite segments of erfc(beta r) on
// [k h, (k+1) h] with h a power of two, coefficients (c0, c1), (c2, c3) in FP64.
struct nb_etab {
    const double2 *seg;
    float invh;
    int n;
};

// All C pairs (i-atom k, the lane's j-atom) of one batch.  xs/ys/zs hold the i-coordinates
// already moved into the pair frame (uniform over the wave in the fast path).  MASKED applies
// the topology mask; without it every unordered pair within rc interacts.  FLAV selects the
// electrostatics (Ewald real space or reaction field) and the Lennard-Jones cutoff treatment
// (potential shift or force switch), NB_FLAV(elec, vdw).
template <int C, bool MASKED, bool EPREC, int FLAV, bool VIR>
__device__ __forceinline__ void pair_block(const nb_fparams &fp, const float4 *tab, int ntt,
                                           const nb_etab &et, const float *xs, const float *ys,
                                           const float *zs, const float *qi, const int *ti,
                                           nb_jlane &j, float *fix, float *fiy, float *fiz,
                                           double &elj, double &ec, float &qqs, double &qqsd,
                                           double *vird, float p4v, float q5v) {
    constexpr bool RF = FLAV / 2 == NB_ELEC_RF;
    constexpr bool FSW = FLAV % 2 == NB_VDW_FSWITCH;
    // FP32 partial sums of the batch's C pair energies, added to the FP64 sums once per batch
    // (starting from -0 lets the first addition fold away)
    float eljb = -0.0f, ecb = -0.0f;
    // VIR: FP32 partial sums of f d_a d_b over the batch's pairs (xx, yy, zz, xy, xz, yz)
    float vb[6] = {-0.0f, -0.0f, -0.0f, -0.0f, -0.0f, -0.0f};
#pragma unroll
    for (int k = 0; k < C; ++k) {
        const float dx = xs[k] - j.x;
        const float dy = ys[k] - j.y;
        const float dz = zs[k] - j.z;
        const float r2 = nb_r2(dx, dy, dz);
        const bool inc = MASKED ? ((r2 < fp.rc2) && ((j.mcol >> k) & 1u)) : (r2 < fp.rc2);
        const float rinv = inc ? nb_rsq(r2) : 0.0f;
        const float rinv2 = rinv * rinv;
        const float rinv6 = rinv2 * rinv2 * rinv2;
        const float4 *ljp = tab + 2 * (ti[k] + j.t);
        const float4 lj = ljp[0];             // (C6, C12, 6 C6, 12 C12)
        const float shv = ljp[1].x;
        // Lennard-Jones: energy C12 r^-12 - C6 r^-6 - shift, force factor (12 C12 r^-6 - 6 C6) r^-8
        const float u = __builtin_fmaf(lj.y, rinv6, -lj.x);
        float elj_p = inc ? __builtin_fmaf(u, rinv6, -shv) : 0.0f;
        const float tf = __builtin_fmaf(lj.w, rinv6, -lj.z);
        float flj = tf * rinv6;
        const float r = r2 * rinv;            // zero for non-interacting pairs
        // FP64 pair energies (EPREC): exact displacement, 1/r refined in FP64 from the FP32 one
        double rid = 0.0, r2d = 0.0;
        if (EPREC) {
            const double dxd = (double)xs[k] - j.xd;
            const double dyd = (double)ys[k] - j.yd;
            const double dzd = (double)zs[k] - j.zd;
            r2d = __builtin_fma(dzd, dzd, __builtin_fma(dyd, dyd, dxd * dxd));
            const double y = (double)rinv;    // zero for non-interacting pairs
            const double ee = __builtin_fma(-(r2d * y), y, 1.0);
            rid = __builtin_fma(0.5 * y, ee, y);
            // Lennard-Jones pair energy in FP64 (C6, C12 are the FP32 instance values)
            const double c6d = lj.x, c12d = lj.y;
            const double rid2 = rid * rid, rid6 = rid2 * rid2 * rid2;
            double el = __builtin_fma(__builtin_fma(c12d, rid6, -c6d), rid6,
                                      -__builtin_fma(c12d, fp.lj_k12, -c6d * fp.lj_k6));
            if (FSW) {
                const double td = fmax(r2d * rid - fp.sw_r1_d, 0.0);
                const double e12 = __builtin_fma(fp.sw_eb12_d, td, fp.sw_ea12_d);
                const double e6 = __builtin_fma(fp.sw_eb6_d, td, fp.sw_ea6_d);
                el = __builtin_fma(-__builtin_fma(c12d, e12, -c6d * e6), td * td * td, el);
            }
            elj += inc ? el : 0.0;
        }
        if (FSW) {
            // force switch beyond sw_r1 (t = r - sw_r1 > 0; t = 0 for non-interacting pairs):
            // force (C12 (A12 + B12 t) - C6 (A6 + B6 t)) t^2 added to the magnitude, and
            // -(C12 (A12/3 + B12/4 t) - C6 (A6/3 + B6/4 t)) t^3 to the energy
            const float t = fmaxf(r - fp.sw_r1, 0.0f);
            const float t2 = t * t;
            const float p12 = __builtin_fmaf(fp.sw_b12, t, fp.sw_a12);
            const float p6 = __builtin_fmaf(fp.sw_b6, t, fp.sw_a6);
            const float sw = __builtin_fmaf(lj.y, p12, -lj.x * p6);
            flj = __builtin_fmaf(sw * t2, r, flj);  // the magnitude times r (the force factor carries r^-2)
            const float e12 = __builtin_fmaf(fp.sw_eb12, t, fp.sw_ea12);
            const float e6 = __builtin_fmaf(fp.sw_eb6, t, fp.sw_ea6);
            const float esw = __builtin_fmaf(lj.y, e12, -lj.x * e6);
            elj_p = __builtin_fmaf(-esw, t2 * t, elj_p);
        }
        const float qq = qi[k] * j.q;             // fC q_i q_j
        float fs;
        if (RF) {
            // reaction field: force factor fC q q (1/r^3 - 2 k_rf), energy fC q q (1/r + k_rf r^2);
            // c_rf is applied at the end to the sum of q_i q_j, accumulated exactly in FP64 (the
            // product of two FP32 charges is exact there): unlike erfc(beta rc)/rc, c_rf is not
            // small, and an FP32 running sum of the products would dominate the energy error
            const float cr = __builtin_fmaf(-2.0f * fp.krf, r2, rinv);
            fs = __builtin_fmaf(qq, cr, flj) * rinv2;
            const double qqd = (double)qi[k] * j.qd;
            qqsd += inc ? qqd : 0.0;
            if (EPREC) {
                // pair energy in FP64 without fC
                const double v = __builtin_fma(fp.krf_d, r2d, rid);
                ec = __builtin_fma(qqd, inc ? v : 0.0, ec);
            } else {
                const float r2m = inc ? r2 : 0.0f;
                ecb = __builtin_fmaf(qq, __builtin_fmaf(fp.krf, r2m, rinv), ecb);
            }
        } else {
            // Ewald real space: erfc(beta r) = exp(-beta^2 r^2) P(r) / Q(r)
            const float ex = __builtin_amdgcn_exp2f(fp.cexp * r2);
            float P = __builtin_fmaf(p4v, r, fp.p[3]);
            P = __builtin_fmaf(P, r, fp.p[2]);
            P = __builtin_fmaf(P, r, fp.p[1]);
            P = __builtin_fmaf(P, r, fp.p[0]);
            float Q = __builtin_fmaf(q5v, r, fp.q[4]);
            Q = __builtin_fmaf(Q, r, fp.q[3]);
            Q = __builtin_fmaf(Q, r, fp.q[2]);
            Q = __builtin_fmaf(Q, r, fp.q[1]);
            Q = __builtin_fmaf(Q, r, fp.q[0]);
            // refined reciprocal: the raw one's error pattern follows Q(r) and does not average out
            const float R = P * nb_rcp(Q);
            const float qe = qq * ex;
            const float t1 = qe * rinv;               // fC q_i q_j exp(-b^2 r^2) / r
            const float uu = __builtin_fmaf(fp.kb, r, R);
            fs = __builtin_fmaf(t1, uu, flj) * rinv2;
            if (EPREC) {
                // Coulomb pair energy in FP64 without fC, erfc(beta r) from the FP64 Hermite table
                // (segment found with the FP32 r)
                const double rd = r2d * rid;
                const int sg = min((int)(r * et.invh), et.n - 1);
                const double uq = __builtin_fma(rd, (double)et.invh, -(double)sg);
                const double2 c01 = et.seg[2 * sg], c23 = et.seg[2 * sg + 1];
                const double g = __builtin_fma(__builtin_fma(__builtin_fma(c23.y, uq, c23.x), uq, c01.y), uq, c01.x);
                const double qqd = (double)qi[k] * j.qd;
                ec = __builtin_fma(qqd * g, rid, ec);
                qqsd += inc ? qqd : 0.0;
            } else {
                ecb = __builtin_fmaf(t1, R, ecb);     // += fC q_i q_j erfc(b r) / r
                qqs += inc ? qq : 0.0f;
            }
        }
        if (!EPREC) eljb += elj_p;
        if (VIR) {
            const float tx = fs * dx, ty = fs * dy, tz = fs * dz;
            vb[0] = __builtin_fmaf(tx, dx, vb[0]);
            vb[1] = __builtin_fmaf(ty, dy, vb[1]);
            vb[2] = __builtin_fmaf(tz, dz, vb[2]);
            vb[3] = __builtin_fmaf(tx, dy, vb[3]);
            vb[4] = __builtin_fmaf(tx, dz, vb[4]);
            vb[5] = __builtin_fmaf(ty, dz, vb[5]);
        }
        fix[k] = __builtin_fmaf(fs, dx, fix[k]);
        fiy[k] = __builtin_fmaf(fs, dy, fiy[k]);
        fiz[k] = __builtin_fmaf(fs, dz, fiz[k]);
        j.fx = __builtin_fmaf(-fs, dx, j.fx);
        j.fy = __builtin_fmaf(-fs, dy, j.fy);
        j.fz = __builtin_fmaf(-fs, dz, j.fz);
    }
    if (!EPREC) {
        elj += (double)eljb;
        ec += (double)ecb;
    }
    if (VIR) {
#pragma unroll
        for (int m = 0; m < 6; ++m) vird[m] += (double)vb[m];
    }
}

// Whether the shift weight (sum of q_i q_j over interacting pairs) is accumulated in FP64
// without fC (FP64 energy mode, and reaction field) or in FP32 with fC (Ewald, FP32 energies).
template <bool EPREC, int FLAV>
constexpr bool nb_qq64() { return EPREC || FLAV / 2 == NB_ELEC_RF; }

__device__ __forceinline__ float nb_uniform(float v) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

// Fixed-point value of a force component (round to nearest; clamped so that the conversion is
// defined; values that large are flagged by the range check anyway).
__device__ __forceinline__ int nb_fix(float f) {
    return (int)__builtin_rintf(fminf(fmaxf(f * NB_FSCALE, -2147483520.0f), 2147483520.0f));
}

// x and y of one contribution as the 64-bit word x + 2^32 y (sums modulo 2^64 keep both).
__device__ __forceinline__ unsigned long long nb_fix_xy(float x, float y) {
    return (unsigned long long)(long long)nb_fix(x) + ((unsigned long long)(unsigned)nb_fix(y) << 32);
}

// Adds one atom's force contribution (lane-wise, where `on`) to the fixed-point accumulators
// fxy / fz, or to the FP32 ones (fj[3][npad_max]); the fixed-point form also raises the range
// flag if any active lane's component exceeds NB_FRANGE (or is not finite).
template <bool FIX>
__device__ __forceinline__ void nb_add_force(bool on, int slot, float fx, float fy, float fz,
                                             NB_G float *fj, int npad_max, NB_G unsigned *flags,
                                             int lane) {
    if (FIX) {
        const float m = fmaxf(fmaxf(fabsf(fx), fabsf(fy)), fabsf(fz));
        if (__ballot(on && !(m < NB_FRANGE)) != 0ull && lane == 0) atomicOr((unsigned *)flags, NB_F_RANGE);
        if (on) {
            atomicAdd((unsigned long long *)fj + slot, nb_fix_xy(fx, fy));
            atomicAdd((int *)(fj + 2 * npad_max) + slot, nb_fix(fz));
        }
    } else if (on) {
        atomicAdd((float *)(fj + slot), fx);
        atomicAdd((float *)(fj + npad_max + slot), fy);
        atomicAdd((float *)(fj + 2 * npad_max + slot), fz);
    }
}

// Energy sums of one work unit (every lane holds them): E_LJ, the Coulomb pair sum and the
// Coulomb shift weight (sum of q_i q_j over interacting pairs).
struct nb_esum {
    double elj, ec, qq;
    double v[6];  // with VIR: sum over pairs of f d_a d_b (xx, yy, zz, xy, xz, yz), F_ij = f d
};

// Forces and energy sums of one work unit, computed by one wavefront: the batches
// [b0, b0 + nbat) of i-cluster ci's j-list (all of them, or one part of a long list).  fp.L
// holds the box of the cluster.  Both the j-forces and the unit's i-force sums are added
// atomically to fj (several units may share an i-cluster), in fixed point with FIX (the layout
// of nb_add_force), in FP32 otherwise; the energy sums are returned.
template <int C, bool EPREC, int FLAV, bool VIR, bool FIX>
__device__ __forceinline__ nb_esum nb_force_cluster(const nb_fparams &fp, const float4 *tab,
                                                 const nb_etab &et, int ci, int b0, int nbat,
                                                 int cap, int npad_max,
                                                 const NB_G float4 *__restrict__ xq,
                                                 const NB_G int *__restrict__ tsort,
                                                 const NB_G int *__restrict__ icount,
                                                 const NB_G nb_entry *__restrict__ jl,
                                                 NB_G float *__restrict__ fj,
                                                 NB_G unsigned *__restrict__ flags) {
    constexpr unsigned FULL = (1u << C) - 1u;
    const int nt = fp.ntypes, ntt = nt * nt;
    const int lane = threadIdx.x & (NB_WAVE - 1);
    const int b = lane % NB_JG, jsub = lane / NB_JG;  // j-atom within the group, entry in batch

    float xi[C], yi[C], zi[C], qi[C], xs[C], ys[C], zs[C];
    int ti[C];
#pragma unroll
    for (int k = 0; k < C; ++k) {
        const float4 v = nb_ld(xq + ci * C + k);
        xi[k] = v.x;
        yi[k] = v.y;
        zi[k] = v.z;
        qi[k] = nb_uniform(v.w);
        ti[k] = nb_ld(tsort + ci * C + k) * nt;
        xs[k] = xi[k];
        ys[k] = yi[k];
        zs[k] = zi[k];
    }
    int cur_shift = NB_SHIFT_ZERO;  // shift the cached i-frame coordinates xs/ys/zs belong to
    float fix[C], fiy[C], fiz[C];
#pragma unroll
    for (int k = 0; k < C; ++k) fix[k] = fiy[k] = fiz[k] = 0.0f;
    double elj = 0.0, ec = 0.0, qqsd = 0.0;  // qqsd: FP64-energy mode sum of q_i q_j
    float qqs = 0.0f;                        // FP32 mode: sum of fC q_i q_j (shift weight)
    double vird[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};

    // the leading coefficients of the erfcx numerator and denominator live in vector registers
    // for the whole list: the first Horner step then reads one scalar register, which is all a
    // VOP3 instruction can take, instead of copying a constant into a VGPR for every pair
    float p4v, q5v;
    asm("v_mov_b32 %0, %1" : "=v"(p4v) : "s"(fp.p[4]));
    asm("v_mov_b32 %0, %1" : "=v"(q5v) : "s"(fp.q[5]));
    const int nj = min(nb_ld(icount + ci), (b0 + nbat) * NB_JPB);
    const NB_G nb_entry *lst = jl + (size_t)ci * cap;
    for (int base = b0 * NB_JPB; base < nj; base += NB_JPB) {
        const int e = base + jsub;
        const bool valid = e < nj;
        // lanes past the end of the list read the i-cluster's own first group with an empty mask
        const nb_entry en = valid ? nb_ld(lst + e) : nb_make_entry(ci * (C / NB_JG), NB_SHIFT_ZERO, 0u);
        const int s = nb_entry_shift(en);
        const int jslot = nb_entry_group(en) * NB_JG + b;
        const float4 xj = nb_ld(xq + jslot);
        nb_jlane jv;
        jv.q = xj.w * fp.fc;
        jv.qd = (double)xj.w;
        jv.t = nb_ld(tsort + jslot);
        jv.mcol = nb_mask_column<C>(en.mask, b);
        jv.fx = jv.fy = jv.fz = 0.0f;
        const int s0 = __builtin_amdgcn_readfirstlane(s);
        const bool uniform = __ballot(valid && s != s0) == 0ull;
        if (uniform) {
            // one periodic shift for the whole batch: i-coordinates of that frame are cached
            const int tx = nb_tx(s0), ty = nb_ty(s0), tz = nb_tz(s0);
            if (s0 != cur_shift) {
                cur_shift = s0;
                const float dix = nb_di(tx, fp.L[0]), diy = nb_di(ty, fp.L[1]), diz = nb_di(tz, fp.L[2]);
#pragma unroll
                for (int k = 0; k < C; ++k) {
                    xs[k] = nb_uniform(xi[k] + dix);
                    ys[k] = nb_uniform(yi[k] + diy);
                    zs[k] = nb_uniform(zi[k] + diz);
                }
            }
            jv.x = xj.x + nb_dj(tx, fp.L[0]);
            jv.y = xj.y + nb_dj(ty, fp.L[1]);
            jv.z = xj.z + nb_dj(tz, fp.L[2]);
            if (EPREC) {
                jv.xd = (double)jv.x;
                jv.yd = (double)jv.y;
                jv.zd = (double)jv.z;
            }
            const bool full = __ballot(!valid || jv.mcol != FULL) == 0ull;
            if (full)
                pair_block<C, false, EPREC, FLAV, VIR>(fp, tab, ntt, et, xs, ys, zs, qi, ti, jv, fix, fiy, fiz, elj, ec, qqs, qqsd, vird, p4v, q5v);
            else
                pair_block<C, true, EPREC, FLAV, VIR>(fp, tab, ntt, et, xs, ys, zs, qi, ti, jv, fix, fiy, fiz, elj, ec, qqs, qqsd, vird, p4v, q5v);
        } else {
            // shifts differ across the batch: per-lane frame offsets
            const int tx = nb_tx(s), ty = nb_ty(s), tz = nb_tz(s);
            const float dix = nb_di(tx, fp.L[0]), diy = nb_di(ty, fp.L[1]), diz = nb_di(tz, fp.L[2]);
            jv.x = xj.x + nb_dj(tx, fp.L[0]);
            jv.y = xj.y + nb_dj(ty, fp.L[1]);
            jv.z = xj.z + nb_dj(tz, fp.L[2]);
            if (EPREC) {
                jv.xd = (double)jv.x;
                jv.yd = (double)jv.y;
                jv.zd = (double)jv.z;
            }
            float xl[C], yl[C], zl[C];
#pragma unroll
            for (int k = 0; k < C; ++k) {
                xl[k] = xi[k] + dix;
                yl[k] = yi[k] + diy;
                zl[k] = zi[k] + diz;
            }
            pair_block<C, true, EPREC, FLAV, VIR>(fp, tab, ntt, et, xl, yl, zl, qi, ti, jv, fix, fiy, fiz, elj, ec, qqs, qqsd, vird, p4v, q5v);
        }
        // about 40% of the lanes of a batch have no pair within rc (their entry was kept for
        // another atom of the group, at rlist); they skip their atomics
        nb_add_force<FIX>(valid && (jv.fx != 0.0f || jv.fy != 0.0f || jv.fz != 0.0f), jslot, jv.fx,
                          jv.fy, jv.fz, fj, npad_max, flags, lane);
    }
#pragma unroll
    for (int k = 0; k < C; ++k) {
        fix[k] = nb_wave_sum_lane63(fix[k]);
        fiy[k] = nb_wave_sum_lane63(fiy[k]);
        fiz[k] = nb_wave_sum_lane63(fiz[k]);
    }
    elj = nb_wave_sum_d(elj);
    ec = nb_wave_sum_d(ec);
    const double qqd = nb_wave_sum_d(nb_qq64<EPREC, FLAV>() ? qqsd : (double)qqs);
    // the unit's i-force sums (in lane 63) go to lanes 0 .. C-1, one atom each, so that three
    // atomics of C lanes add them
    float vx = 0.0f, vy = 0.0f, vz = 0.0f;
#pragma unroll
    for (int k = 0; k < C; ++k) {
        const float sx = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(fix[k]), NB_WAVE - 1));
        const float sy = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(fiy[k]), NB_WAVE - 1));
        const float sz = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(fiz[k]), NB_WAVE - 1));
        vx = lane == k ? sx : vx;
        vy = lane == k ? sy : vy;
        vz = lane == k ? sz : vz;
    }
    nb_add_force<FIX>(lane < C, ci * C + lane, vx, vy, vz, fj, npad_max, flags, lane);
    nb_esum out{elj, ec, qqd, {0.0, 0.0, 0.0, 0.0, 0.0, 0.0}};
    if (VIR) {
#pragma unroll
        for (int m = 0; m < 6; ++m) out.v[m] = nb_wave_sum_d(vird[m]);
    }
    return out;
}
