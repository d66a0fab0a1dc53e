// Body of the short-range force computation for one i-cluster, shared by the single-box
// kernel and the persistent batched kernel.  Layout (a from-scratch design for a 64-wide
// wavefront):
//  * one wavefront per i-cluster; the C i-atoms are wave-uniform values, so every i-coordinate
//    is a scalar operand of the vector instructions;
//  * each lane owns one j-atom of one of the 16 four-atom j-groups of the current batch;
//  * a batch is processed in three phases.  Filter: every lane forms the displacements and
//    squared distances of its C pairs (i-atom k, its j-atom) and tests r < rc, and the topology
//    mask unless every listed pair of the batch is unmasked (the common case, checked with one
//    ballot); the pairs that interact (about a third of the listed ones) are appended to a
//    per-wave queue in LDS in (k, lane) order with a ballot and a lane count, as (r^2, pair
//    code), the code holding LDS byte addresses: of the pair's LJ table row, and of its force
//    factor, i-atom and j lane within the wave's parts of the work area (one shift or one
//    and-or each to decode).  Evaluate: the queue is worked through 64 pairs at a time, one pair
//    per lane, so the Lennard-Jones and Ewald arithmetic (the transcendental functions, the erfc
//    approximation, the energies) runs only on interacting pairs with all lanes busy; each
//    pair's scalar force factor goes to its place (64 k + lane) in a per-wave area cleared at the
//    start of the batch.  Accumulate: every lane reads the factors of its own C pairs (zero
//    where the pair does not interact) and adds f d to the i-force and j-force sums in
//    registers, in the same order as a plain loop over k;
//  * force factors come out in fixed-point units (the charge products and the table's force
//    coefficients carry the scale 2^12), so a sum converts to its integer with one rounding;
//  * batches whose entries share one periodic shift (the common case, since the list is grouped
//    by shift) use i-coordinates moved into that frame once and cached in scalar registers;
//  * the j-force of a lane's atom needs two atomic adds per batch (x and y in one 64-bit word,
//    z; the only atomics), skipped where the sum is zero; the i-forces accumulate per lane over
//    the whole list and are reduce-scattered across the 64 lanes once per work unit;
//  * erfc(beta r) = exp(-beta^2 r^2) P(r) / Q(r) with a (4,5) rational fit of the scaled
//    complementary error function (fit_erfcx.py), Newton-refined reciprocal square root and
//    reciprocal;
//  * per-pair energies (FP32) are added to per-lane FP64 sums one pair at a time (no FP32
//    partial sums, whose rounding would depend on how pairs are grouped); the Ewald potential
//    shift is part of each pair's energy, the reaction-field one (not small) is applied in FP64
//    at the end from the sum of q_i q_j over interacting pairs;
//  * with EPREC the pair energies are instead evaluated in FP64 (exact displacement,
//    Newton-refined 1/r, erfc from an FP64 quintic Hermite table), forces staying FP32: the FP32
//    rounding of the displacement and of erfc(beta r)/r is otherwise not averaged below 1e-6 of
//    an energy that is a 1e-4 .. 1e-3-conditioned sum, in boxes of a few thousand atoms.  The
//    FP64 work runs in the evaluate phase, i.e. on interacting pairs only.
#pragma once
#include "nb_device.h"

// Four waves per SIMD (at most 128 VGPRs) for the FP32-energy force kernels; the FP64-energy
// variant holds more state per lane and its workgroups more LDS (the erfc table and the j-atom
// frames), three waves.
#define NB_FORCE_OCCUPANCY __attribute__((amdgpu_waves_per_eu(EPREC ? 3 : 4)))
// With the virial sums (six more accumulators per lane) the FP32 body needs more than 128
// VGPRs: three waves per SIMD.
#define NB_FORCE_OCCUPANCY_VIR __attribute__((amdgpu_waves_per_eu(EPREC ? 3 : (VIR ? 3 : 4))))

__device__ __forceinline__ double nb_wave_sum_d(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, NB_WAVE);
    return v;
}

// LDS work areas of the force body for the NW wavefronts of a workgroup, one part per wave in
// every array.  RAWQ: the flavour needs the charges as loaded (exact FP64 products q_i q_j: FP64
// pair energies, and the reaction-field shift weight).  The evaluate phase addresses fsb, jqf and
// id from the bits of a pair code: each wave's part of these starts at a multiple of a power of
// two no smaller than the part (the struct is placed at a multiple of C * 256 bytes, the size of
// one fsb part), so the element offset is combined with the part's base by a bitwise or.
template <int C, bool EPREC, int FLAV, int NW>
struct nb_wg_lds {
    static constexpr bool RAWQ = EPREC || FLAV / 2 == NB_ELEC_RF;
    static constexpr int ALIGN = C * NB_WAVE * 4;
    float fsb[NW][C * NB_WAVE];     // force factor of pair (i-atom k, j lane) at 64 k + lane
    float jqf[NW][NB_WAVE];         // per j lane: fC NB_FSCALE q_j
    float4 id[NW][C];               // per i-atom: (x, y, z, q) as loaded (unshifted)
    uint2 q[NW][C * NB_WAVE];       // the batch's interacting pairs: (r^2 bits, pair code)
    float jq[NW][RAWQ ? NB_WAVE : 1];  // per j lane: q_j as loaded
    // FP64-energy mode, per j lane: x_j + dj - di in FP64 (exact), x, y and z in rows of 64, so
    // that x_i - (x_j + dj - di) is the exact displacement of the pair
    double jx[NW][EPREC ? 3 * NB_WAVE : 1];
};

// One wavefront's parts of the work area, as LDS byte addresses (wave-uniform).
struct nb_wv {
    uint32_t fsb, jqf, id, q, jq, jx;
};

template <int C, bool EPREC, int FLAV, int NW>
__device__ __forceinline__ nb_wv nb_wave_view(nb_wg_lds<C, EPREC, FLAV, NW> &g, int wv) {
    using G = nb_wg_lds<C, EPREC, FLAV, NW>;
    static_assert(offsetof(G, fsb) == 0 && offsetof(G, jqf) % (NB_WAVE * 4) == 0 &&
                      offsetof(G, id) % (C * 16) == 0,
                  "or-addressed parts must sit at multiples of their size");
    return nb_wv{nb_laddr(&g.fsb[wv][0]), nb_laddr(&g.jqf[wv][0]), nb_laddr(&g.id[wv][0]),
                 nb_laddr(&g.q[wv][0]),   nb_laddr(&g.jq[wv][0]),  nb_laddr(&g.jx[wv][0])};
}

// Pair code of a queued pair: (LDS byte address of its LJ table row << NB_PC_ROW) | (64 k + j
// lane) * 4 for i-atom k.  The low bits are the byte offset of the pair's force factor in its
// wave's fsb part; within them, bits 2-7 are 4 x the j lane and bits 8-10 the i-atom.
#define NB_PC_ROW 11
#define NB_PC_FSB 0x7FCu  // (64 k + lane) * 4
#define NB_PC_JQF 0xFCu   // lane * 4
#define NB_PC_ID 0x70u    // k * 16, from the code shifted right by 4

// The LJ table as the force body reads it: the force coefficients (6 C6, 12 C12) carry the
// fixed-point scale NB_FSCALE, so that force factors come out in fixed-point units.
__device__ __forceinline__ void nb_load_ljtab(float4 *tab, const float4 *ljtab, int ntt) {
    for (int k = threadIdx.x; k < 2 * ntt; k += blockDim.x) {
        float4 v = ljtab[k];
        if ((k & 1) == 0) {
            v.z *= NB_FSCALE;
            v.w *= NB_FSCALE;
        }
        tab[k] = v;
    }
}

// Erfc table of the FP64 energy mode: quintic Hermite segments of erfc(beta r) on
// [k h, (k+1) h] (value and first and second derivatives matched at both ends) with h a power of
// two, coefficients (c0, c1), (c2, c3), (c4, c5) in FP64.
struct nb_etab {
    const double2 *seg;
    float invh;
    int n;
    const float4 *fseg;  // tabulated Ewald: FP32 Hermite segments of G(r), NB_TAB_SEGMENTS of them
};

// erfc(beta r) in FP64 from the table, at the FP64 distance rd (segment chosen with the FP32 r).
__device__ __forceinline__ double nb_erfc_tab(const nb_etab &et, float r, double rd) {
    const int sg = min((int)(r * et.invh), et.n - 1);
    const double u = __builtin_fma(rd, (double)et.invh, -(double)sg);
    const double2 c01 = et.seg[3 * sg], c23 = et.seg[3 * sg + 1], c45 = et.seg[3 * sg + 2];
    double g = __builtin_fma(c45.y, u, c45.x);
    g = __builtin_fma(g, u, c23.y);
    g = __builtin_fma(g, u, c23.x);
    g = __builtin_fma(g, u, c01.y);
    return __builtin_fma(g, u, c01.x);
}

// Scalar force factor fs (F_ij = fs d) and the energies of one interacting pair at squared
// distance r2 with qq = fC q_i q_j and the LJ row lj (C6, C12, 6 C6, 12 C12) and shift shv (shd:
// the row's FP64 shift, used with EPREC).  The
// FP32 pair energies (the Ewald one shifted) are added to the FP64 sums elj / ec one pair at a
// time; the reaction field adds its shift weight as exact FP64 products qqd = q_i q_j to qqsd;
// with EPREC the FP64 energies of the pair, computed from the exact displacement (dxd, dyd,
// dzd), go to elj / ec and the products qqd to qqsd.
template <bool EPREC, int FLAV>
__device__ __forceinline__ float pair_eval(const nb_fparams &fp, const nb_etab &et, float r2,
                                           float qq, double qqd, const float4 &lj, float shv,
                                           double shd, double dxd, double dyd, double dzd,
                                           double &elj, double &ec, double &qqsd, float p4v,
                                           float q5v) {
    constexpr bool RF = FLAV / 2 == NB_ELEC_RF;
    constexpr bool TAB = FLAV / 2 == NB_ELEC_EWALD_TAB;
    constexpr bool FSW = FLAV % 2 == NB_VDW_FSWITCH;
    static_assert(!TAB || EPREC, "the tabulated flavour evaluates its pair energies in FP64");
    const float rinv = nb_rsq(r2);
    const float rinv2 = rinv * rinv;
    const float rinv6 = rinv2 * rinv2 * rinv2;
    // Lennard-Jones: energy C12 r^-12 - C6 r^-6 - shift, force factor (12 C12 r^-6 - 6 C6) r^-8
    const float u = __builtin_fmaf(lj.y, rinv6, -lj.x);
    float elj_p = __builtin_fmaf(u, rinv6, -shv);
    const float tf = __builtin_fmaf(lj.w, rinv6, -lj.z);
    float flj = tf * rinv6;
    const float r = r2 * rinv;
    // FP64 pair energies (EPREC): exact displacement, 1/r refined in FP64 from the FP32 one
    double rid = 0.0, r2d = 0.0;
    if (EPREC) {
        r2d = __builtin_fma(dzd, dzd, __builtin_fma(dyd, dyd, dxd * dxd));
        const double y = (double)rinv;
        const double ee = __builtin_fma(-(r2d * y), y, 1.0);
        rid = __builtin_fma(0.5 * y, ee, y);
        // Lennard-Jones pair energy in FP64 (C6, C12 are the FP32 instance values)
        const double c6d = lj.x, c12d = lj.y;
        const double rid2 = rid * rid, rid6 = rid2 * rid2 * rid2;
        double el = __builtin_fma(__builtin_fma(c12d, rid6, -c6d), rid6, -shd);
        if (FSW) {
            const double td = fmax(r2d * rid - fp.sw_r1_d, 0.0);
            const double e12 = __builtin_fma(fp.sw_eb12_d, td, fp.sw_ea12_d);
            const double e6 = __builtin_fma(fp.sw_eb6_d, td, fp.sw_ea6_d);
            el = __builtin_fma(-__builtin_fma(c12d, e12, -c6d * e6), td * td * td, el);
        }
        elj += el;
    }
    if (FSW) {
        // force switch beyond sw_r1 (t = r - sw_r1 > 0): force (C12 (A12 + B12 t) - C6 (A6 +
        // B6 t)) t^2 added to the magnitude, and -(C12 (A12/3 + B12/4 t) - C6 (A6/3 + B6/4 t))
        // t^3 to the energy
        const float t = fmaxf(r - fp.sw_r1, 0.0f);
        const float t2 = t * t;
        const float p12 = __builtin_fmaf(fp.fsw_b12, t, fp.fsw_a12);  // force terms: scaled
        const float p6 = __builtin_fmaf(fp.fsw_b6, t, fp.fsw_a6);
        const float sw = __builtin_fmaf(lj.y, p12, -lj.x * p6);
        flj = __builtin_fmaf(sw * t2, r, flj);  // the magnitude times r (the force factor carries r^-2)
        const float e12 = __builtin_fmaf(fp.sw_eb12, t, fp.sw_ea12);
        const float e6 = __builtin_fmaf(fp.sw_eb6, t, fp.sw_ea6);
        const float esw = __builtin_fmaf(lj.y, e12, -lj.x * e6);
        elj_p = __builtin_fmaf(-esw, t2 * t, elj_p);
    }
    float fs;
    if (RF) {
        // reaction field: force factor fC q q (1/r^3 - 2 k_rf), energy fC q q (1/r + k_rf r^2);
        // c_rf is applied at the end to the sum of q_i q_j, accumulated exactly in FP64 (the
        // product of two FP32 charges is exact there): unlike erfc(beta rc)/rc, c_rf is not
        // small, and an FP32 running sum of the products would dominate the energy error
        const float cr = __builtin_fmaf(-2.0f * fp.krf, r2, rinv);
        fs = __builtin_fmaf(qq, cr, flj) * rinv2;
        qqsd += qqd;
        if (EPREC) {
            // pair energy in FP64 without fC
            ec = __builtin_fma(qqd, __builtin_fma(fp.krf_d, r2d, rid), ec);
        } else {
            ec += (double)(qq * __builtin_fmaf(fp.krf, r2, rinv));
        }
    } else if (TAB) {
        // tabulated Ewald: force factor fC q q (1/r^3 - G(r)), G from its FP32 Hermite segment
        const float tr = r * fp.tinvh;
        const int sg = min((int)tr, NB_TAB_SEGMENTS - 1);
        const float uu = tr - (float)sg;
        const float4 c = et.fseg[sg];
        const float G = __builtin_fmaf(__builtin_fmaf(__builtin_fmaf(c.w, uu, c.z), uu, c.y), uu, c.x);
        fs = __builtin_fmaf(qq, __builtin_fmaf(-r2, G, rinv), flj) * rinv2;
        // Coulomb pair energy in FP64 without fC, erfc(beta r) from the FP64 table
        ec = __builtin_fma(qqd * nb_erfc_tab(et, r, r2d * rid), rid, ec);
        qqsd += qqd;
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
            // Coulomb pair energy in FP64 without fC, erfc(beta r) from the FP64 table
            ec = __builtin_fma(qqd * nb_erfc_tab(et, r, r2d * rid), rid, ec);
            qqsd += qqd;
        } else {
            // fC q_i q_j (erfc(b r) / r - erfc(b rc) / rc): the potential shift is about 1e-5 of
            // the pair's energy, so one FP32 rounding of the difference is all it adds (the
            // shift weight stays zero in this mode)
            ec += (double)__builtin_fmaf(t1, R, -qq * fp.shc);
        }
    }
    if (!EPREC) elj += (double)elj_p;
    return fs;
}

// Whether the shift weight (sum of q_i q_j over interacting pairs) is accumulated from exact
// FP64 products without fC (FP64 energy mode, and reaction field); otherwise (Ewald, FP32
// energies) it is zero, the shift being part of the pair energies.
template <bool EPREC, int FLAV>
constexpr bool nb_qq64() { return EPREC || FLAV / 2 == NB_ELEC_RF; }

// v where the wave-uniform c holds, else +0: an integer select kept on the scalar unit (the
// result is opaque to the compiler, which would otherwise move the select to the vector unit).
__device__ __forceinline__ float nb_sel_s(bool c, float v) {
    uint32_t r = c ? __float_as_uint(v) : 0u;
    asm("" : "+s"(r));
    return __uint_as_float(r);
}

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

// Fixed-point value of a force component that already carries the factor NB_FSCALE: rounded to
// the nearest integer, ties to even (FP32 values of 2^22 and above are multiples of 1/2, so ties
// are common, and rounding them all one way would bias the sums: the forces on the two atoms of
// a pair would no longer cancel), then converted by the hardware instruction, whose result is
// defined for every input (saturating; values that large raise the range flag anyway).
__device__ __forceinline__ int nb_rne(float v) {
    int r;
    asm("v_cvt_i32_f32 %0, %1" : "=v"(r) : "v"(__builtin_rintf(v)));
    return r;
}

// Adds one atom's force contribution, in units of 1 / NB_FSCALE (lane-wise, where `on` and not
// zero), to the fixed-point accumulators: x + 2^32 y in one 64-bit word (x sign-extended, so the
// high word is y - 1 for negative x), z in a 32-bit word.  Raises the range flag if an active
// lane's component reaches NB_FRANGE (or is not finite).  onmask: the ballot of `on`.
__device__ __forceinline__ void nb_add_fix(bool on, unsigned long long onmask, int slot, float fx,
                                           float fy, float fz, NB_G float *fj, int npad_max,
                                           NB_G unsigned *flags, int lane) {
    const float m = fmaxf(fmaxf(fabsf(fx), fabsf(fy)), fabsf(fz));
    if ((__builtin_amdgcn_ballot_w64(!(m < NB_FRANGE * NB_FSCALE)) & onmask) != 0ull &&
        lane == 0)
        atomicOr((unsigned *)flags, NB_F_RANGE);
    if (on && m != 0.0f) {
        const int ix = nb_rne(fx), iy = nb_rne(fy), iz = nb_rne(fz);
        const unsigned long long xy =
            ((unsigned long long)(unsigned)(iy + (ix >> 31)) << 32) | (unsigned long long)(unsigned)ix;
        atomicAdd((unsigned long long *)fj + slot, xy);
        atomicAdd((int *)(fj + 2 * npad_max) + slot, iz);
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
// holds the box of the cluster; w is the wavefront's part of the LDS work area and tab the LJ
// table in LDS (nb_load_ljtab).  Both the j-forces and the unit's i-force sums are added
// atomically to fj in fixed point (nb_add_fix; several units may share an i-cluster); the energy
// sums are returned.  Force factors are formed in units of 1 / NB_FSCALE (the charge products
// and the table's force coefficients carry the scale); the energy sums that inherit it are
// scaled back exactly (a power of two) at the end.
template <int C, bool EPREC, int FLAV, bool VIR>
__device__ __forceinline__ nb_esum nb_force_cluster(const nb_fparams &fp, const float4 *tab,
                                                 const nb_etab &et, const nb_wv &w, int ci,
                                                 int b0, int nbat, int cap, int npad_max,
                                                 const NB_G float4 *__restrict__ xq,
                                                 const NB_G int *__restrict__ tsort,
                                                 const NB_G int *__restrict__ icount,
                                                 const NB_G nb_entry *__restrict__ jl,
                                                 NB_G float *__restrict__ fj,
                                                 NB_G unsigned *__restrict__ flags) {
    constexpr bool RAWQ = EPREC || FLAV / 2 == NB_ELEC_RF;
    constexpr unsigned FULL = (1u << C) - 1u;
    const int nt = fp.ntypes;
    const int lane = threadIdx.x & (NB_WAVE - 1);
    const int b = lane % NB_JG, jsub = lane / NB_JG;  // j-atom within the group, entry in batch
    const uint32_t lane4 = (uint32_t)lane * 4u;

    // i-atoms: coordinates and charges in LDS (the evaluate phase, where a lane's i-atom varies,
    // and the frame changes read them); per i-atom the constant part of its pairs' codes, the
    // address of the LJ table row t_i * ntypes and k, wave-uniform
    // the wave's parts of the work area that are addressed by position
    float4 *const idp = (float4 *)(NB_L float4 *)(size_t)w.id;
    float *const fsbp = (float *)(NB_L float *)(size_t)w.fsb;
    float *const jqfp = (float *)(NB_L float *)(size_t)w.jqf;
    if (lane < C) idp[lane] = nb_ld(xq + ci * C + lane);
    const uint32_t tabrow = nb_laddr(tab);
    uint32_t pci[C];
#pragma unroll
    for (int k = 0; k < C; ++k)
        pci[k] = ((tabrow + 32u * (uint32_t)(__builtin_amdgcn_readfirstlane(nb_ld(tsort + ci * C + k)) * nt))
                  << NB_PC_ROW) | ((uint32_t)k << 8);
    // the code masks in vector registers, for single and-or address operations
    const uint32_t mfsb = nb_vreg(NB_PC_FSB), mjqf = nb_vreg(NB_PC_JQF), mid = nb_vreg(NB_PC_ID);
    nb_wave_lds_sync();
    // the cached i-frame coordinates xs/ys/zs and the shift they belong to: first the frame of
    // the zero shift (most lists start there), i.e. the coordinates as loaded, by scalar loads
    int cur_shift = NB_SHIFT_ZERO;
    float xs[C], ys[C], zs[C];
#pragma unroll
    for (int k = 0; k < C; ++k) {
        const float4 v = nb_ld(xq + ci * C + k);
        xs[k] = v.x;
        ys[k] = v.y;
        zs[k] = v.z;
    }
    float fix[C], fiy[C], fiz[C];
#pragma unroll
    for (int k = 0; k < C; ++k) fix[k] = fiy[k] = fiz[k] = 0.0f;
    // energy sums; qqsd: the shift weight, sum of q_i q_j over interacting pairs (exact FP64
    // products with FP64 energies or the reaction field; zero for Ewald with FP32 energies,
    // whose pair energies carry the shift)
    double elj = 0.0, ec = 0.0, qqsd = 0.0;
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
        // the lanes of entries below nj: the first nvl (formed on the scalar unit)
        const int nvl = min(NB_WAVE, NB_JG * (nj - base));
        const bool valid = lane < nvl;
        const unsigned long long vmask = nvl >= NB_WAVE ? ~0ull : (1ull << nvl) - 1ull;
        // lanes past the end of the list read the far group behind the last slot (coordinates
        // far outside any box) with an empty mask, so that none of their pairs is in range
        const nb_entry en = valid ? nb_ld(lst + e) : nb_make_entry(npad_max / NB_JG, NB_SHIFT_ZERO, 0u);
        const int s = nb_entry_shift(en);
        const int jslot = nb_entry_group(en) * NB_JG + b;
        const float4 xj = nb_ld(xq + jslot);
        const int tj = nb_ld(tsort + jslot);
        const unsigned mcol = nb_mask_column<C>(en.mask, b);
        const int s0 = __builtin_amdgcn_readfirstlane(s);
        // (ballots of single compares combined on the scalar unit: a ballot of a compound
        // condition costs two more vector instructions)
        const bool uniform = (__builtin_amdgcn_ballot_w64(s != s0) & vmask) == 0ull;
        // ---- filter: displacements of the lane's C pairs, interacting pairs queued in LDS
        float dx[C], dy[C], dz[C];
        float jx, jy, jz;     // the j-atom in the pair frame
        float dix, diy, diz;  // the i-frame offset of this lane's pairs
        if (uniform) {
            // one periodic shift for the whole batch: i-coordinates of that frame are cached, and
            // the frame offsets are scalar selects
            const int tx = nb_tx(s0), ty = nb_ty(s0), tz = nb_tz(s0);
            dix = nb_sel_s(tx > 0, fp.nL[0]);
            diy = nb_sel_s(ty > 0, fp.nL[1]);
            diz = nb_sel_s(tz > 0, fp.nL[2]);
            if (s0 != cur_shift) {
                cur_shift = s0;
#pragma unroll
                for (int k = 0; k < C; ++k) {
                    const float4 v = idp[k];
                    xs[k] = nb_uniform(v.x + dix);
                    ys[k] = nb_uniform(v.y + diy);
                    zs[k] = nb_uniform(v.z + diz);
                }
            }
            jx = xj.x + nb_sel_s(tx < 0, fp.nL[0]);
            jy = xj.y + nb_sel_s(ty < 0, fp.nL[1]);
            jz = xj.z + nb_sel_s(tz < 0, fp.nL[2]);
#pragma unroll
            for (int k = 0; k < C; ++k) {
                dx[k] = xs[k] - jx;
                dy[k] = ys[k] - jy;
                dz[k] = zs[k] - jz;
            }
        } else {
            // shifts differ across the batch: per-lane frame offsets
            const int tx = nb_tx(s), ty = nb_ty(s), tz = nb_tz(s);
            dix = nb_di(tx, fp.L[0]);
            diy = nb_di(ty, fp.L[1]);
            diz = nb_di(tz, fp.L[2]);
            jx = xj.x + nb_dj(tx, fp.L[0]);
            jy = xj.y + nb_dj(ty, fp.L[1]);
            jz = xj.z + nb_dj(tz, fp.L[2]);
#pragma unroll
            for (int k = 0; k < C; ++k) {
                const float4 v = idp[k];
                dx[k] = (v.x + dix) - jx;
                dy[k] = (v.y + diy) - jy;
                dz[k] = (v.z + diz) - jz;
            }
        }
        nb_wave_lds_sync();  // the previous batch's reads of the work area are done
        jqfp[lane] = xj.w * fp.fcs;
        if (RAWQ) nb_lput<float>(w.jq + lane4, xj.w);
        if (EPREC) {
            // x_j + dj (FP32, exact) minus the i-frame offset: exact in FP64
            nb_lput<double>(w.jx + 2u * lane4, (double)jx - (double)dix);
            nb_lput<double>(w.jx + 2u * lane4 + 8u * NB_WAVE, (double)jy - (double)diy);
            nb_lput<double>(w.jx + 2u * lane4 + 16u * NB_WAVE, (double)jz - (double)diz);
        }
#pragma unroll
        for (int k = 0; k < C; ++k) fsbp[k * NB_WAVE + lane] = 0.0f;
        // the lane's part of the pair codes: its type's table row offset and its lane
        const uint32_t pcj = ((uint32_t)tj << (NB_PC_ROW + 5)) | lane4;
        int nq = 0;  // interacting pairs of the batch (wave-uniform)
        // the record of a pair: the batch's next free record (qb, formed on the scalar unit before
        // the divergent branch) plus the rank of the lane among those that enqueue
        auto enqueue = [&](int k, uint32_t qb, float r2, unsigned long long bal) {
            const uint32_t pos = __builtin_amdgcn_mbcnt_hi((unsigned)(bal >> 32),
                                                           __builtin_amdgcn_mbcnt_lo((unsigned)bal, 0u));
            nb_lput<uint2>(qb + 8u * pos, make_uint2(__float_as_uint(r2), pci[k] + pcj));
        };
        if ((__builtin_amdgcn_ballot_w64(mcol != FULL) & vmask) == 0ull) {
            // every listed pair of the batch is unmasked (the common case): the range test alone
#pragma unroll
            for (int k = 0; k < C; ++k) {
                const float r2 = nb_r2(dx[k], dy[k], dz[k]);
                const bool in = r2 < fp.rc2;
                const unsigned long long bal = __builtin_amdgcn_ballot_w64(in);
                uint32_t qb = w.q + 8u * (uint32_t)nq;
                asm("" : "+s"(qb));
                if (in) enqueue(k, qb, r2, bal);
                nq += __popcll(bal);
            }
        } else {
#pragma unroll
            for (int k = 0; k < C; ++k) {
                const float r2 = nb_r2(dx[k], dy[k], dz[k]);
                const bool inr = r2 < fp.rc2, inm = (mcol & (1u << k)) != 0u;
                // two ballots of single compares, combined on the scalar unit
                const unsigned long long bal =
                    __builtin_amdgcn_ballot_w64(inr) & __builtin_amdgcn_ballot_w64(inm);
                uint32_t qb = w.q + 8u * (uint32_t)nq;
                asm("" : "+s"(qb));
                if (inr && inm) enqueue(k, qb, r2, bal);
                nq += __popcll(bal);
            }
        }
        nb_wave_lds_sync();
        // ---- evaluate: the queued pairs, one per lane; full passes of 64, then the rest
        auto evaluate = [&](uint32_t qa) {
            const uint2 qe = nb_lget<uint2>(qa);
            const uint32_t code = qe.y;
            const uint32_t ta = code >> NB_PC_ROW;  // the pair's LJ row
            const float4 lj = nb_lget<float4>(ta);
            const float shv = nb_lget<float>(ta + 16u);
            // the row's FP64 potential shift (FP64 pair energies only)
            const double shd = EPREC ? nb_lget<double>(ta + 24u) : 0.0;
            const uint32_t ia = ((code >> 4) & mid) | w.id;  // its i-atom's (x, y, z, q)
            const uint32_t jo = code & mjqf;                // 4 x its j lane
            const float qi = nb_lget<float>(ia + 12u);
            const float qq = qi * nb_lget<float>(jo | w.jqf);
            double qqd = 0.0, dxd = 0.0, dyd = 0.0, dzd = 0.0;
            if (RAWQ) qqd = (double)qi * (double)nb_lget<float>(w.jq + jo);
            if (EPREC) {
                // exact displacement: x_i - (x_j + dj - di), both terms exact in FP64 and their
                // difference too (a few tens of significant bits at most)
                const float4 idk = nb_lget<float4>(ia);
                const uint32_t ja = w.jx + 2u * jo;
                dxd = (double)idk.x - nb_lget<double>(ja);
                dyd = (double)idk.y - nb_lget<double>(ja + 8u * NB_WAVE);
                dzd = (double)idk.z - nb_lget<double>(ja + 16u * NB_WAVE);
            }
            const float fs = pair_eval<EPREC, FLAV>(fp, et, __uint_as_float(qe.x), qq, qqd, lj, shv, shd,
                                                    dxd, dyd, dzd, elj, ec, qqsd,
                                                    p4v, q5v);
            nb_lput<float>((code & mfsb) | w.fsb, fs);
        };
        uint32_t qa = w.q + 8u * (uint32_t)lane;
#pragma unroll 2
        for (int p = 0; p < (nq >> 6); ++p, qa += 8u * NB_WAVE) evaluate(qa);
        if (lane < (nq & (NB_WAVE - 1))) evaluate(qa);
        nb_wave_lds_sync();
        // ---- accumulate: f d of the lane's C pairs into the i- and j-force sums (the factor is
        // zero for pairs that do not interact)
        float vb[6] = {-0.0f, -0.0f, -0.0f, -0.0f, -0.0f, -0.0f};
        float jfx = 0.0f, jfy = 0.0f, jfz = 0.0f;
#pragma unroll
        for (int k = 0; k < C; ++k) {
            const float fs = fsbp[k * NB_WAVE + lane];
            if (VIR) {
                const float tx = fs * dx[k], ty = fs * dy[k], tz = fs * dz[k];
                vb[0] = __builtin_fmaf(tx, dx[k], vb[0]);
                vb[1] = __builtin_fmaf(ty, dy[k], vb[1]);
                vb[2] = __builtin_fmaf(tz, dz[k], vb[2]);
                vb[3] = __builtin_fmaf(tx, dy[k], vb[3]);
                vb[4] = __builtin_fmaf(tx, dz[k], vb[4]);
                vb[5] = __builtin_fmaf(ty, dz[k], vb[5]);
            }
            fix[k] = __builtin_fmaf(fs, dx[k], fix[k]);
            fiy[k] = __builtin_fmaf(fs, dy[k], fiy[k]);
            fiz[k] = __builtin_fmaf(fs, dz[k], fiz[k]);
            jfx = __builtin_fmaf(-fs, dx[k], jfx);
            jfy = __builtin_fmaf(-fs, dy[k], jfy);
            jfz = __builtin_fmaf(-fs, dz[k], jfz);
        }
        if (VIR) {
#pragma unroll
            for (int m = 0; m < 6; ++m) vird[m] += (double)vb[m];
        }
        // about 40% of the lanes of a batch have no pair within rc (their entry was kept for
        // another atom of the group, at rlist); their sums are zero and they skip the atomics
        nb_add_fix(valid, vmask, jslot, jfx, jfy, jfz, fj, npad_max, flags, lane);
    }
    // the unit's i-force sums: atom k's in the lanes with lane / (64 / C) == k, added by the
    // first lane of each group
    const float sx = nb_wave_scatter_sum<C>(fix, lane);
    const float sy = nb_wave_scatter_sum<C>(fiy, lane);
    const float sz = nb_wave_scatter_sum<C>(fiz, lane);
    elj = nb_wave_sum_d(elj);
    ec = nb_wave_sum_d(ec);
    double qqd = nb_wave_sum_d(qqsd);
    const bool head = lane % (NB_WAVE / C) == 0;
    nb_add_fix(head, __builtin_amdgcn_ballot_w64(head), ci * C + lane / (NB_WAVE / C), sx, sy, sz, fj,
               npad_max, flags, lane);
    // the FP32-energy Coulomb sums were formed from the scaled charge products, the virial from
    // the scaled force factors
    constexpr double unscale = 1.0 / NB_FSCALE;
    if (!EPREC) ec *= unscale;
    if (!nb_qq64<EPREC, FLAV>()) qqd *= unscale;
    nb_esum out{elj, ec, qqd, {0.0, 0.0, 0.0, 0.0, 0.0, 0.0}};
    if (VIR) {
#pragma unroll
        for (int m = 0; m < 6; ++m) out.v[m] = nb_wave_sum_d(vird[m]) * unscale;
    }
    nb_wave_lds_sync();  // the next unit of this wave rewrites the work area
    return out;
}
