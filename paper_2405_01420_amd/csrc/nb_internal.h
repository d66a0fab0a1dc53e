// Internal declarations shared by the host API and the HIP kernels of libnb.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "nb.h"

#define NB_WAVE 64
#define NB_MAX_TYPES 32
#define NB_SORT_MAX 4096   // largest column the LDS sort handles
#define NB_SHIFT_ZERO 13   // shift index of t = (0, 0, 0); index = 9 (tx+1) + 3 (ty+1) + (tz+1)

// Device-side status flags (nb_meta::flags)
#define NB_F_OVERFLOW 0x1u
#define NB_F_STALE 0x2u
#define NB_F_NONFINITE 0x4u
#define NB_F_COLUMN 0x8u
#define NB_F_RANGE 0x10u  // a pair force component beyond the fixed-point accumulators' check
#define NB_F_BUILD_NONFINITE 0x20u  // non-finite coordinates seen by a list build
// Conditions raised by force calls: kept across list builds until nb_check reports them.
#define NB_F_CALL_MASK (NB_F_STALE | NB_F_NONFINITE | NB_F_RANGE)

// Fixed-point force accumulation of the single-box path: a component f is added as the 32-bit
// integer rint(f * NB_FSCALE); x and y of an atom share one 64-bit word (x + 2^32 y, added
// modulo 2^64, which is exact for the two 32-bit sums as long as each stays within 32 bits),
// z is a 32-bit word.  Integer sums do not depend on the order of the atomics.  Net components
// up to 2^31 / NB_FSCALE = 524288 kJ mol^-1 nm^-1 per atom are represented; a contribution
// above NB_FRANGE (a quarter of that) in any component raises NB_F_RANGE.  (Stiff
// Lennard-Jones types at liquid density give single contributions above 3e4.)  The unit,
// 2^-12, adds a rounding error of about 7e-5 per contribution, ~6e-4 per atom component for
// the ~80 contributions an atom receives at 96k atoms: 1e-6 of typical water forces.
#define NB_FSCALE 4096.0f
#define NB_FRANGE 131072.0f

// Coordinates of padding slot p (also of the far j-group behind the last slot): far outside the
// box, and at least NB_PAD_SPACING from every other padding slot (the slot index spread over the
// three axes, 10 bits each, all values exact in FP32), so that no pair that involves padding lies
// within the list range (rc + rb < NB_PAD_SPACING is enforced): the topology masks leave padding
// unmasked and the distance test excludes it.
#define NB_PAD_SPACING 16.0f
__host__ __device__ __forceinline__ float4 nb_pad_coord(int p) {
    return make_float4(-1e5f - NB_PAD_SPACING * (float)(p & 1023),
                       -1e5f - NB_PAD_SPACING * (float)((p >> 10) & 1023),
                       -1e5f - NB_PAD_SPACING * (float)((p >> 20) & 1023), 0.0f);
}

// One j-entry of the cluster-pair list.  The j side of every entry is a group of NB_JG = 4
// consecutive slots: a whole cluster when C = 4, one half (lower or upper four in z order) of
// a cluster when C = 8, so an 8-atom i-cluster meets 4-atom j-groups (8 x 4 pairs per entry)
// and half-clusters with no atom pair in range are not listed.  gs packs the group index and
// the periodic shift of the j image (x_j + t L); mask bit (b * C + a) is set iff i-atom a and
// j-atom b of the group are distinct, not excluded and, for the self pair at t = 0, in
// increasing slot order.  Padding slots are not masked: they sit far outside the box and far
// apart (nb_pad_coord), so that the distance test excludes every pair that involves one.  The
// mask is column-major so that the lane holding j-atom b extracts its C bits with one shift.
#define NB_JG 4
#define NB_JPB (NB_WAVE / NB_JG)  // entries per batch of 64 lanes
struct nb_entry {
    uint32_t gs;    // (j-group << 5) | shift index
    uint32_t mask;
};
__host__ __device__ __forceinline__ int nb_entry_group(const nb_entry &e) { return (int)(e.gs >> 5); }
__host__ __device__ __forceinline__ int nb_entry_shift(const nb_entry &e) { return (int)(e.gs & 31u); }
__host__ __device__ __forceinline__ nb_entry nb_make_entry(int group, int shift, uint32_t mask) {
    nb_entry e;
    e.gs = ((uint32_t)group << 5) | (uint32_t)shift;
    e.mask = mask;
    return e;
}

// Counters written by the GPU during a build (read back by the host only when needed).
#define NB_HIST_BINS 8  // list-length classes floor(log2 batches): 1, 2-3, 4-7, ..., >= 128
struct nb_meta {
    int32_t nclusters;   // clusters of the current grid
    int32_t npad;        // nclusters * C
    uint32_t flags;      // NB_F_*
    int32_t maxcount;    // largest j-entry count of an overflowing i-cluster (for regrowing)
    int32_t maxcolumn;   // largest column population
    int32_t nunits;      // work units of the force kernel (i-cluster list parts)
    int32_t split;       // batches per work unit at most
    int32_t maxbatches;  // longest j-list, in 64-lane batches
    int32_t hist[NB_HIST_BINS];  // i-clusters per list-length class (non-empty lists)
    int32_t pad;
    uint64_t npairs_out; // pair-export counter
};

// Box geometry and the column grid, passed to kernels by value.
struct nb_geom {
    float L[3];
    float invw[2];      // 1 / column width in x and y
    float w[2];
    int ncx, ncy, ncol;
    float rl2;          // rlist^2 (search and prune)
    float rl;
    // z bins of the per-column cluster tables (k_colsort): bin k starts at k / zinv, nz bins
    // cover [0, L_z]
    float zinv;
    int nz;
};

// Force-kernel constants (FP32 values derived on the host in FP64).
struct nb_fparams {
    float L[3];
    float nL[3];        // -L (frame offsets selected on the scalar unit)
    float rc2;
    float fc;           // Coulomb constant
    float fcs;          // fC NB_FSCALE (the force body forms force factors in fixed-point units)
    float cexp;         // -beta^2 log2(e):  exp(-beta^2 r^2) = exp2(cexp r^2)
    float kb;           // 2 beta / sqrt(pi)
    // LJ table in LDS/global: per type pair (a * ntypes + b) two float4,
    // (C6, C12, 6 C6, 12 C12) and (potential shift, 1 / sigma_ab, FP64 potential shift as two
    // words: C12 lj_k12 - C6 lj_k6, for FP64 pair energies)
    float p[5];         // erfcx numerator coefficients scaled by beta^k (argument r)
    float q[6];         // erfcx denominator coefficients scaled by beta^k
    float b2;           // beta^2
    float irc6, irc12;  // rc^-6, rc^-12
    float shc;          // erfc(beta rc) / rc
    int ntypes;
    // reaction field: force factor 1/r^3 - 2 k_rf, energy 1/r + k_rf r^2 (c_rf applied at the end)
    float krf;
    // force switch from sw_r1 to rc: force terms A t^2 + B t^3, energy terms -(A/3) t^3 - (B/4) t^4
    // with t = r - sw_r1, for the r^-6 and r^-12 parts
    float sw_r1, sw_a6, sw_b6, sw_a12, sw_b12, sw_ea6, sw_eb6, sw_ea12, sw_eb12;
    float fsw_a6, fsw_b6, fsw_a12, fsw_b12;  // the force coefficients times NB_FSCALE
    // FP64 pair-energy constants: k_rf; LJ shift constants (value at rc of the r^-6 and r^-12
    // parts: rc^-a, or the force-switch constant); force-switch energy coefficients
    double krf_d, lj_k6, lj_k12, sw_r1_d, sw_ea6_d, sw_eb6_d, sw_ea12_d, sw_eb12_d;
    // tabulated Ewald force correction G(r): NB_TAB_SEGMENTS segments of width 1 / tinvh
    float tinvh;
};

// Flavour of a force kernel: electrostatics * 2 + van der Waals (NB_ELEC_*, NB_VDW_*).
#define NB_FLAV(elec, vdw) ((elec) * 2 + (vdw))

// Per-type constants for the LJ-parameter gradient reduction.
struct nb_typeparams {
    double eps[NB_MAX_TYPES];
    int ntypes;
};

struct nb_ctx {
    hipStream_t stream = nullptr;
    int device = 0;
    int natoms = 0, ntypes = 0, C = 8;
    double box[3] = {0, 0, 0};
    double rc = 0, rb = 0, beta = 0, fc = 0;
    int elec = NB_ELEC_EWALD, vdw = NB_VDW_SHIFT;
    double eps_rf = 0, rsw = 0;
    uint32_t flags = 0;
    nb_geom geom{};
    nb_fparams fp{};
    double shift_coul = 0;  // erfc(beta rc) / rc
    int npad_max = 0, ncl_max = 0;
    int cap = 0;            // j-entries per i-cluster
    int slots = 0;          // SIMDs of the device (4 per compute unit)
    int unit_cap = 0;       // work units at most: ncl_max + tail_n + 2 slots
    int tail_n = 0;         // clusters at the end of the unit order whose lists are split in halves
    bool have_list = false;
    bool pending_overflow_check = false;
    bool built_once = false;          // a build has completed (its capacity checked)
    nb_meta *host_meta = nullptr;     // pinned copy of the status block of the last async build
    hipEvent_t build_ev = nullptr;    // recorded after that copy
    std::vector<double> sigma, epsilon;
    std::string err;
    double build_ms = 0;

    // device buffers
    float4 *off = nullptr;      // [natoms] image offset added to x (-n L)
    float *xbuild = nullptr;    // [natoms*3] positions at the last build
    int *col = nullptr, *rank = nullptr, *tmp = nullptr, *slot_of = nullptr;  // [natoms]
    int *colcount = nullptr, *colstart = nullptr, *colcl = nullptr;           // [ncol(+1)]
    int2 *colz = nullptr;   // [ncol * (nz + 1)]: per column and z bin edge, the cluster bounds (k_colsort)
    int *perm = nullptr;        // [npad_max] slot -> atom (-1 = padding)
    float4 *xs = nullptr;       // [npad_max] build positions (wrapped), sorted
    float4 *xq = nullptr;       // [npad_max] per-call positions + charge, sorted
    int *tsort = nullptr;       // [npad_max] per-call type, sorted
    float *fj = nullptr;        // [3 * npad_max] words: fixed-point force sums in cluster order,
                                // x + 2^32 y as 64-bit words, then z; added to atomically by the
                                // force kernel, read and cleared by the finalize
    bool fj_clean = true;       // fj is all zero (false after a force call that failed part-way)
    float4 *bblo = nullptr, *bbhi = nullptr;  // [ncl_max]
    int *icount = nullptr;      // [ncl_max]
    nb_entry *jl = nullptr;     // [ncl_max * cap] the list the force calls use
    // rolling prune: while `pruned`, jl / icount hold the pruned list and jl_p / icount_p the
    // build's full list (swapped back by the next build); jl_p has room for jl_p_cap entries
    // per i-cluster
    nb_entry *jl_p = nullptr;
    int *icount_p = nullptr;
    int jl_p_cap = 0;
    bool pruned = false;
    float *xprune = nullptr;    // [natoms*3] positions at the last prune (with NB_CHECK_STALE)
    float stale2_prune = 0.0f;  // ((r_inner - rc) / 2)^2
    int4 *units = nullptr;      // [unit_cap] (i-cluster, first batch, batches, energy slot),
                                // longest first
    double *epart = nullptr;    // [unit_cap * 4] energy partials (one per force workgroup used)
    double *cpart = nullptr;    // [NB_CORR_PART * blocks] Ewald-correction partials (NB_EWALD_CORR)
    double *vpart = nullptr;    // [6 * force workgroups] virial pair sums (nb_forces_virial)
    nb_meta *meta = nullptr;
    float4 *ljtab = nullptr;    // [2 * nt * nt]: (C6, C12, 6 C6, 12 C12), (shift, 1/sigma_ab, 0, 0)
    double2 *etab = nullptr;    // [NB_ETAB_W * etab_n]: Hermite segments of erfc(beta r) (FP64 energy mode)
    float4 *ftab = nullptr;     // [NB_TAB_SEGMENTS]: FP32 Hermite segments of the tabulated Ewald
                                // force correction (NB_ELEC_EWALD_TAB)
    int etab_n = 0;
    float etab_invh = 0.0f;     // 1 / segment width, a power of two
    int *excl_off = nullptr, *excl_idx = nullptr;
    int nnz_excl = 0;
    int64_t *dbg_pairs = nullptr;
    int64_t dbg_cap = 0;
    // adjoint buffers (allocated on first use)
    float *adj = nullptr;       // [6 * npad_max]: i-side (dx, dy, dz, dq, Sw, Su) SoA
    float *adjj = nullptr;      // [6 * npad_max]: j-side, atomics
    float4 *gs = nullptr;       // [npad_max] force cotangents in cluster order
    double *tpart = nullptr;    // [adjoint type-sum blocks][ntypes][2] block partials
    double *mdpart = nullptr;   // [leapfrog blocks] kinetic-energy partials (allocated on first use)
    // kernel timing: every timing_every-th force launch (counted from nb_set_timing) is stamped
    bool timing = false;
    int timing_every = 1;
    int64_t timing_count = 0;
    std::vector<hipEvent_t> ev;  // pairs (start, stop)
    size_t ev_used = 0;          // pairs recorded
    double timed_ms = 0;
    int64_t timed_n = 0;
};

// Whether the force kernel evaluates the pair energies in FP64 (then the Coulomb sums carry no
// fC): NB_ENERGY_FP64, or the tabulated Ewald flavour, which always does.
inline bool nb_energy_fp64(const nb_ctx *c) {
    return (c->flags & NB_ENERGY_FP64) != 0 || c->elec == NB_ELEC_EWALD_TAB;
}

// ---- host helpers (nb_api.cpp) ----
int nb_read_meta(nb_ctx *c, nb_meta *m);
int nb_regrow_list(nb_ctx *c, int maxcount);
int nb_list_entries(nb_ctx *c, int nclusters, int64_t *total);  // sum of icount (synchronous)

// ---- launchers (nb_build.hip) ----
hipError_t nb_launch_build(nb_ctx *c, const float *x);
hipError_t nb_launch_debug_pairs(nb_ctx *c, int64_t cap);
hipError_t nb_launch_prune(nb_ctx *c, float rin2, const int *icount, const nb_entry *jl, int *icount_p,
                           nb_entry *jl_p);  // on the positions of the last pack
hipError_t nb_launch_prune_check(nb_ctx *c, const float *x);

// ---- launchers (nb_force.hip) ----
hipError_t nb_launch_pack(nb_ctx *c, const float *x, const float *q, const int32_t *type);
// ev0 / ev1 (or null): events that the dispatch itself stamps with the kernel's start and end
hipError_t nb_launch_force(nb_ctx *c, bool vir, hipEvent_t ev0, hipEvent_t ev1);
hipError_t nb_launch_finalize(nb_ctx *c, float *f, double *e, double *vir);
hipError_t nb_launch_ewald_corr(nb_ctx *c, const float *x, const float *q);

// Threads per block of the Ewald-correction kernel (one atom each), and its partial sums per
// block: the exclusion-correction and self energies, then six pair sums for the virial.
// double2 per segment of the FP64 erfc table (quintic: six coefficients)
#define NB_ETAB_W 3

#define NB_CORR_BLOCK 256
#define NB_CORR_PART 8

// ---- launchers (nb_md.hip) ----
hipError_t nb_launch_md_update(nb_ctx *c, float dt, const float *f, const float *inv_m, float *x,
                               float *v, double *e);

// ---- launchers (nb_adjoint.hip) ----
hipError_t nb_launch_adjoint(nb_ctx *c, const float *gf, const double *ge, float *dx, float *dq,
                             double *dsig, double *deps);
// The allocation-free form: the work buffers in the library's static device array (looked up
// per device by nb_noalloc_init); padded slots at most NB_NOALLOC_MAX_SLOTS.
hipError_t nb_noalloc_init(int device);
hipError_t nb_launch_adjoint_noalloc(nb_ctx *c, const float *gf, const double *ge, float *dx,
                                     float *dq, double *dsig, double *deps);
