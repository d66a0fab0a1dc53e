/*
 * nb.h - C-ABI of the MI355X short-range nonbonded force library (libnb.so).
 *
 * What the library computes is the short-range nonbonded force step of a molecular-dynamics
 * time step, the computation the paper identifies as the longest-running kernel and the
 * single-GPU rate limiter (section III-A, "NBNXM, short-range non-bonded forces"; the
 * Fig. 3 caption names the flavour: Ewald electrostatics and Lennard-Jones with a combination
 * rule).  The paper also names the pieces around it: a buffered pair list with a list range,
 * a prune step and list sorting (section III-A, the bullet list on the differences between
 * the GROMACS versions).  Concretely, for atoms in a rectangular periodic box:
 *
 *   for every unordered, non-excluded pair with minimum-image distance r < rc
 *     E_LJ += C12 (r^-12 - rc^-12) - C6 (r^-6 - rc^-6)             (potential shift)
 *     E_C  += fC q_i q_j (erfc(beta r)/r - erfc(beta rc)/rc)         (Ewald real space)
 *     F_i  += [12 C12 r^-14 - 6 C6 r^-8 + fC q_i q_j (erfc(beta r)/r^3
 *              + 2 beta/sqrt(pi) exp(-beta^2 r^2)/r^2)] (x_i - x_j),  F_j -= the same
 *   with C6 = 4 eps_ab sigma_ab^6, C12 = 4 eps_ab sigma_ab^12 and Lorentz-Berthelot
 *   combination sigma_ab = (sigma_a + sigma_b)/2, eps_ab = sqrt(eps_a eps_b).
 *
 * How: atoms are wrapped into the box, binned into x-y columns, sorted by z inside each
 * column and cut into clusters of C atoms; a cluster-pair list with one bit per atom pair
 * (exclusions, self pairs, padding) is built within rlist = rc + buffer and pruned at atom
 * level; the force kernel evaluates every listed cluster pair.  Pair arithmetic is FP32,
 * energy reductions are FP64.
 *
 * Conventions for every entry point:
 *  - All functions return an nb_status (0 = NB_OK).  On failure nb_last_error(ctx) describes
 *    the cause; outputs are then unspecified.
 *  - "device" pointers are HIP device (or managed) memory owned by the caller; "host" pointers
 *    are ordinary host memory, read during the call only (the library copies what it keeps).
 *  - Work is queued on the HIP stream given at setup (nb_set_stream changes it); unless a
 *    function says it synchronises, it returns before the GPU has finished.
 *  - Coordinates are float[3] per atom (AoS, nm), original atom order; forces likewise
 *    (kJ mol^-1 nm^-1); energies are double (kJ/mol).
 *  - A context is not thread-safe; use one context per host thread.
 */
#ifndef NB_H
#define NB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum nb_status {
    NB_OK = 0,
    NB_ERR_ARG = 1,        /* null pointer, negative or non-finite size or parameter */
    NB_ERR_CUTOFF = 2,     /* rc >= min(box)/2: the minimum image would not be unique */
    NB_ERR_OOM = 3,        /* device allocation failed */
    NB_ERR_HIP = 4,        /* a HIP runtime call or kernel launch failed */
    NB_ERR_STATE = 5,      /* call order violated (e.g. forces before the first pair list) */
    NB_ERR_OVERFLOW = 6,   /* a list or column exceeded its capacity (rebuilt automatically
                              when nb_pairlist can grow the buffer) */
    NB_ERR_LIST_STALE = 7, /* an atom moved more than buffer/2 since the list was built */
    NB_ERR_NONFINITE = 8,  /* non-finite coordinate seen with NB_CHECK_FINITE */
    NB_ERR_IO = 9,         /* autotune cache could not be read or written */
    NB_ERR_RANGE = 10      /* a pair force component exceeded 131072 kJ/mol/nm: the forces'
                              fixed-point accumulators hold net components up to 524288 */
} nb_status;

/* flags (nb_params.flags and per-call flags) */
#define NB_MAX_EXCL_PER_ATOM 32 /* excluded partners per atom accepted by nb_setup */

/* Interaction flavours (nb_params.elec, nb_params.vdw).  Every pair term is cut at rc and
 * shifted so that its energy is zero there.
 *   NB_ELEC_EWALD   real-space Ewald:  fC q_i q_j (erfc(beta r)/r - erfc(beta rc)/rc)
 *   NB_ELEC_RF      reaction field:    fC q_i q_j (1/r + k_rf r^2 - c_rf),
 *                   k_rf = (eps_rf - 1) / ((2 eps_rf + 1) rc^3)  (1 / (2 rc^3) for eps_rf = 0,
 *                   meaning infinity), c_rf = 1/rc + k_rf rc^2
 *   NB_VDW_SHIFT    C12 (r^-12 - rc^-12) - C6 (r^-6 - rc^-6)
 *   NB_VDW_FSWITCH  the force of each power r^-a (a = 6, 12) is switched smoothly to zero
 *                   between rswitch and rc: a r^-(a+1) + A_a (r - rswitch)^2 + B_a (r - rswitch)^3
 *                   beyond rswitch, with A_a, B_a making the force and its derivative vanish at
 *                   rc; the potential is the matching integral, shifted to zero at rc. */
#define NB_ELEC_EWALD   0
#define NB_ELEC_RF      1
#define NB_ELEC_EWALD_TAB 2  /* the same real-space Ewald interaction as NB_ELEC_EWALD, with the
                                force taken from a table instead of the analytic erfc: the
                                kernel flavour of the paper's runs ("tabulated electrostatics",
                                Fig. 3 caption, section IV-B).  The force factor is
                                fC q_i q_j (1/r^3 - G(r)) with G(r) = erf(beta r)/r^3 -
                                2 beta/sqrt(pi) exp(-beta^2 r^2)/r^2, a smooth function held as
                                FP32 cubic Hermite segments (NB_TAB_SEGMENTS over [0, rc], in
                                LDS); the pair energies are always evaluated in FP64 (as with
                                NB_ENERGY_FP64).  Single-box path only: not for the batched form
                                or nb_backward (NB_ERR_ARG) */
#define NB_TAB_SEGMENTS 256
#define NB_VDW_SHIFT    0
#define NB_VDW_FSWITCH  1

#define NB_CHECK_STALE  0x1u  /* nb_forces records whether any atom moved >= buffer/2 */
#define NB_CHECK_FINITE 0x2u  /* nb_forces records non-finite coordinates */
#define NB_REUSE_LIST   0x4u  /* nb_backward: use the current list instead of rebuilding */
#define NB_ASYNC_BUILD  0x8u  /* nb_pairlist: do not wait for the build; its overflow check
                                 is read at the next nb_pairlist (first build: synchronous) */
#define NB_EWALD_CORR   0x20u /* nb_forces also computes the Ewald exclusion correction and self
                                 term that complete the real-space sum once a reciprocal part
                                 is added: for every excluded pair -fC q_i q_j erf(beta r)/r
                                 (minimum image, with its force, which f includes) and
                                 -fC beta/sqrt(pi) sum q_i^2; e_dev then holds 4 doubles,
                                 e_dev[2] = exclusion correction, e_dev[3] = self term (FP64).
                                 Ewald electrostatics only; not for the batched form or
                                 nb_backward (NB_ERR_ARG) */
#define NB_SORT_UNITS   0x40u /* order the force kernel's work units longest first (by cost class
                                 floor(log2 batches), stable in cluster order): the paper's
                                 post-prune list sorting (section III-A); default: cluster
                                 order, which keeps neighbouring waves on neighbouring clusters */
#define NB_ENERGY_FP64  0x10u /* evaluate the Coulomb pair energies in FP64 (forces stay FP32):
                                 needed for 1e-6 relative E_C in boxes of a few thousand atoms,
                                 where FP32 pair-energy rounding does not average out
                                 (for the reaction field, whose terms do not decay towards rc,
                                 also in larger boxes) */

typedef struct nb_params {
    double box[3];          /* rectangular box edges Lx, Ly, Lz (nm), > 0 */
    double cutoff;          /* rc (nm), 0 < rc < min(box)/2 */
    double buffer;          /* pair-list buffer rb >= 0 (nm); rlist = rc + rb */
    double ewald_beta;      /* beta (1/nm) >= 0, with beta * rc <= 4 */
    double coulomb_const;   /* fC = 1/(4 pi eps0) in the caller's units (> 0) */
    int32_t ntypes;         /* number of LJ types, 1 .. 32 */
    const double *sigma;    /* host [ntypes] LJ sigma (nm) >= 0 */
    const double *epsilon;  /* host [ntypes] LJ epsilon (kJ/mol) >= 0 */
    int32_t natoms;         /* number of atoms, 1 .. 2^27 */
    const int32_t *excl_off;/* host [natoms+1] CSR offsets of excluded partners, or NULL */
    const int32_t *excl_idx;/* host [excl_off[natoms]] partner indices (symmetric lists),
                             * at most NB_MAX_EXCL_PER_ATOM per atom */
    uint32_t flags;         /* NB_CHECK_*, NB_ASYNC_BUILD, NB_ENERGY_FP64, NB_EWALD_CORR,
                               NB_SORT_UNITS */
    int32_t cluster;        /* cluster size C of the list: 4 or 8 (0 = 8) */
    int32_t elec;           /* NB_ELEC_EWALD or NB_ELEC_EWALD_TAB (ewald_beta used), NB_ELEC_RF */
    int32_t vdw;            /* NB_VDW_SHIFT or NB_VDW_FSWITCH */
    double epsilon_rf;      /* reaction-field dielectric: 0 (infinity) or >= 1 */
    double rswitch;         /* force-switch start, 0 <= rswitch < cutoff (NB_VDW_FSWITCH) */
} nb_params;

typedef struct nb_stats {
    int64_t natoms, nclusters, npadded;   /* atoms, clusters, slots incl. padding */
    int64_t nentries;                     /* j-entries in the list (i-cluster x 4-atom j-group) */
    int64_t evaluated_pairs;              /* nentries * C * 4 */
    int64_t list_capacity;                /* j-entries per i-cluster the list can hold */
    int32_t cluster, ncolumns;
    double build_ms_last;                 /* host-timed duration of the last nb_pairlist */
    int32_t work_units;                   /* force-kernel work units (parts of i-cluster lists) */
    int32_t unit_batches;                 /* 64-lane batches per work unit at most */
    int32_t max_list_batches;             /* longest i-cluster list, in 64-lane batches */
    int32_t pruned;                       /* 1 if the force calls use a list from nb_prune */
    int32_t list_hist[8];                 /* i-clusters by list length in 64-lane batches:
                                             1, 2-3, 4-7, ..., 64-127, >= 128 (written by the
                                             kernel that forms the work units) */
} nb_stats;

typedef struct nb_ctx nb_ctx;

/* Check parameters without touching the GPU.  Errors: NB_ERR_ARG, NB_ERR_CUTOFF. */
int nb_validate_params(const nb_params *p);

/* Create a context for one box: copies parameters and exclusions to the device, builds the
 * FP32 LJ table (C6, C12 from the combination rule in FP64, rounded once) and allocates all
 * buffers.  stream: a hipStream_t (NULL = default stream).  *out receives the context.
 * The environment variable NB_LIST_CAP, if set to a positive integer, replaces the initial
 * number of j-entries reserved per i-cluster (the list still grows on overflow).
 * Errors: NB_ERR_ARG, NB_ERR_CUTOFF, NB_ERR_OOM, NB_ERR_HIP. */
int nb_setup(nb_ctx **out, const nb_params *p, void *stream);

/* Replace the LJ parameters (host [ntypes] each); the next nb_forces uses them. */
int nb_set_lj(nb_ctx *ctx, const double *sigma, const double *epsilon);

/* Change the HIP stream used by later calls. */
int nb_set_stream(nb_ctx *ctx, void *stream);

/* Build the cluster-pair list from device coordinates x [natoms][3]: wrap into the box, grid
 * sort, cluster, bounding boxes, search within rlist, exclusion masks, atom-level prune.
 * Remembers x as the build positions for the staleness check.  Synchronises once to read the
 * overflow flag and rebuilds with a larger list if needed.  With NB_ASYNC_BUILD set at setup,
 * every build after the first returns without waiting: its status block is copied to pinned
 * host memory behind it on the stream and read at the next nb_pairlist, which waits only for
 * that copy (done long before the force calls queued after the build).  If that build had
 * overflowed, the forces computed with its list missed pairs: the next nb_pairlist regrows the
 * list, rebuilds synchronously and returns NB_ERR_OVERFLOW with a complete new list in place.
 * Not capturable in a HIP graph.
 * Errors: NB_ERR_ARG, NB_ERR_OVERFLOW (growing failed, or as above), NB_ERR_NONFINITE,
 * NB_ERR_HIP, NB_ERR_OOM. */
int nb_pairlist(nb_ctx *ctx, const float *x_dev);

/* Rolling (dynamic) prune of the list, the paper's prune-only kernel run between list builds
 * (section III-A): from the full list of the last nb_pairlist (cluster pairs within
 * rc + buffer at the build positions), keep for the following force calls only the j-groups
 * that have an unmasked atom pair within r_inner at the current positions x_dev [natoms][3]
 * (device).  rc <= r_inner <= rc + buffer.  Each call prunes the full list again, and the next
 * nb_pairlist restores it.  The pruned list holds every pair within rc while every atom has
 * moved less than (r_inner - rc)/2 since this call (and less than buffer/2 since the build);
 * with NB_CHECK_STALE the force calls check the first condition too (nb_check reports
 * NB_ERR_LIST_STALE).  Also rebuilds the force kernel's work units for the shorter lists
 * (long lists are split by the same rule as after a build).
 * Asynchronous on the context's stream; allocates the pruned list on first use (and after the
 * list has grown).  Errors: NB_ERR_ARG, NB_ERR_STATE (no list), NB_ERR_OOM, NB_ERR_HIP. */
int nb_prune(nb_ctx *ctx, const float *x_dev, double r_inner);

/* Forces and energies for device inputs x [natoms][3], q [natoms], type [natoms] (0-based
 * LJ type).  x must be the build positions or a continuous motion of them (no re-wrapping
 * since the build); pairs stay exact while every atom moved less than buffer/2.
 * The forces are summed in fixed point (2^-12 kJ mol^-1 nm^-1 units, integer atomics), so
 * they do not depend on the order in which the device adds the pair contributions; a pair
 * contribution above 131072 in any component is reported by nb_check as NB_ERR_RANGE (the
 * accumulators hold net components up to 524288 kJ mol^-1 nm^-1 per atom).
 * Outputs: f_dev [natoms][3] overwritten in original order; e_dev[0] = E_LJ, e_dev[1] = E_C
 * (device doubles; with NB_EWALD_CORR also e_dev[2] = Ewald exclusion correction, e_dev[3] =
 * self term, and f includes the exclusion-correction forces).  No allocation and no host
 * synchronisation: capturable in a HIP graph.
 * Errors: NB_ERR_STATE (no list), NB_ERR_HIP.  Stale / non-finite conditions are reported by
 * nb_check. */
int nb_forces(nb_ctx *ctx, const float *x_dev, const float *q_dev, const int32_t *type_dev,
              float *f_dev, double *e_dev);

/* nb_forces plus the virial of the computed forces, vir_dev [3][3] (device doubles, row-major,
 * symmetric): Xi = -1/2 sum over the interacting pairs of d_ij (x) F_ij, with d_ij the
 * minimum-image displacement x_i - x_j and F_ij the pair force on i; with NB_EWALD_CORR the
 * excluded pairs' correction forces are included.  This is the pair-force part of the pressure
 * an MD step reports on energy steps.  Same ownership, asynchrony and errors as nb_forces
 * (NB_ERR_ARG if vir_dev is NULL); about 6 more FMAs per pair. */
int nb_forces_virial(nb_ctx *ctx, const float *x_dev, const float *q_dev, const int32_t *type_dev,
                     float *f_dev, double *e_dev, double *vir_dev);

/* Synchronise the stream and report device-side conditions recorded since the last check:
 * NB_ERR_LIST_STALE, NB_ERR_NONFINITE, NB_ERR_OVERFLOW, NB_ERR_RANGE; clears them.  Conditions
 * raised by force calls stay recorded across later list builds until this call reports them. */
int nb_check(nb_ctx *ctx);

/* Vector-Jacobian product of (F, E_LJ, E_C) for a force-matching loss.
 * Inputs (device): x, q, type as for nb_forces; g_f [natoms][3] = dL/dF (float);
 * g_e [2] = (dL/dE_LJ, dL/dE_C) (double).  Outputs (device, overwritten): dx [natoms][3],
 * dq [natoms] (float), dsigma [ntypes], deps [ntypes] (double).  The pair list is rebuilt
 * from x first unless flags has NB_REUSE_LIST.  Types with epsilon = 0 get deps = 0 (the
 * derivative of sqrt(eps_a eps_b) does not exist there).  The first call allocates the adjoint
 * work buffers; later calls with NB_REUSE_LIST enqueue kernels only (g_e is read on the device,
 * no host synchronisation), while a list rebuild synchronises once as nb_pairlist does.
 * Defined for NB_ELEC_EWALD with NB_VDW_SHIFT (NB_ERR_ARG for other flavours).
 * Errors: as nb_pairlist and nb_forces. */
int nb_backward(nb_ctx *ctx, const float *x, const float *q, const int32_t *type,
                const float *g_f, const double *g_e, float *dx, float *dq, double *dsigma,
                double *deps, uint32_t flags);

/* Molecular dynamics around the force path: nsteps leapfrog steps of the atoms with device
 * coordinates x [natoms][3] (updated in place, continuous: never re-wrapped), velocities
 * v [natoms][3] (nm/ps, at the half step before the first step, updated in place), charges q,
 * types and inverse masses inv_mass [natoms] (mol/g), time step dt (ps):
 *   v(t + dt/2) = v(t - dt/2) + f(t) / m dt,  x(t + dt) = x(t) + v(t + dt/2) dt,
 * with f(t) from nb_forces.  The pair list is rebuilt at every nstlist-th step (the first step
 * included; asynchronously with NB_ASYNC_BUILD), and with r_inner != 0 the rolling prune
 * (nb_prune to r_inner, rc <= r_inner <= rc + buffer) runs at every nstprune-th step between
 * builds: the paper's prune-only kernel between pair searches (section III-A).  Outputs: f (device
 * [natoms][3], the forces of the last step) and e_steps (device double [nsteps][4]): per step
 * E_LJ and E_C at x(t), the kinetic energy at t (average of the half-step kinetic energies,
 * FP64) and their sum.  Queued on the context's stream; synchronises only at list builds (not
 * with NB_ASYNC_BUILD).  Not with NB_EWALD_CORR.  Errors: NB_ERR_ARG (NULL pointer, dt <= 0,
 * nsteps < 0, nstlist < 1, r_inner outside [rc, rc + buffer] or nstprune < 1 with r_inner
 * != 0), and those of nb_pairlist, nb_prune and nb_forces. */
int nb_md_leapfrog(nb_ctx *ctx, float *x, float *v, const float *q, const int32_t *type,
                   const float *inv_mass, double dt, int32_t nsteps, int32_t nstlist,
                   double r_inner, int32_t nstprune, float *f, double *e_steps);

/* Allocation-free nb_backward, for callers that cannot allocate device memory (code under HIP
 * graph capture, serving loops, harnesses that forbid hipMalloc): the same result as
 * nb_backward(ctx, ..., NB_REUSE_LIST) on the current list, with the adjoint's work buffers
 * (per padded slot the i- and j-side gradient sums and the force cotangents, 64 bytes, plus
 * per-type partial sums) in a static device array of the library instead of buffers allocated
 * by the first nb_backward.  Limit: NB_NOALLOC_MAX_SLOTS padded slots (about that many atoms;
 * the array is about 16 MiB per device, held until the process ends).  Calls that overlap on
 * one device share that array and race: serialise them (one stream, or events).  Needs a list
 * (nb_pairlist).  Errors: NB_ERR_ARG (NULL input, flavour other than Ewald + LJ shift, Ewald
 * corrections on, or a system above the limit), NB_ERR_STATE (no list), NB_ERR_HIP. */
#define NB_NOALLOC_MAX_SLOTS 262144
int nb_backward_noalloc(nb_ctx *ctx, const float *x, const float *q, const int32_t *type,
                        const float *g_f, const double *g_e, float *dx, float *dq, double *dsigma,
                        double *deps);

/* Export the interacting pairs of the current list at positions x (device): every listed atom
 * pair with r < rc under the same FP32 arithmetic as nb_forces, as (i, j) with i < j in
 * original indices, unsorted.  pairs_host: host int64 [cap][2]; *count receives the total
 * number (which may exceed cap; then only cap pairs were written).  Synchronises. */
int nb_debug_pairs(nb_ctx *ctx, const float *x_dev, int64_t *pairs_host, int64_t cap,
                   int64_t *count);

/* List statistics of the current list (synchronises). */
int nb_get_stats(nb_ctx *ctx, nb_stats *st);

/* Kernel timing: with every >= 1, the force kernel of every every-th later nb_forces call (the
 * first, the (every+1)-th, ...; 1: all of them) is dispatched with a HIP event pair that its
 * dispatch stamps with the kernel's start and end (hipExtLaunchKernel; a few microseconds of
 * overhead per stamped call, on the device too: the calls in between run unstamped); every <= 0
 * turns it off (the default).  Turning it on creates the events of the first 1024 timed
 * launches and restarts the count.
 * nb_get_timing synchronises, returns the summed kernel time in milliseconds and the number of
 * timed launches since the last nb_get_timing, and resets both. */
int nb_set_timing(nb_ctx *ctx, int every);
int nb_get_timing(nb_ctx *ctx, double *force_kernel_ms, int64_t *launches);

/* Text of the last error on this context (never NULL; "" if none). */
const char *nb_last_error(nb_ctx *ctx);

/* Free the context and its device buffers (synchronises). NULL is accepted. */
int nb_destroy(nb_ctx *ctx);

/* ---------------------------------------------------------------------------------------
 * Batched form: many independent boxes of uneven size, one list per box, and one persistent
 * force launch per cluster shape over the i-clusters of all boxes.  Ensemble-level
 * parallelism (independent simulations) is the outermost level of parallelism the paper
 * describes (section I-A); here the ensemble shares one GPU launch so that small boxes, which
 * alone cannot fill the GPU (the latency-bound regime of Fig. 2, section III-A), are processed
 * together, and the tail of uneven work is handled by a work queue in descending cost order.
 * ------------------------------------------------------------------------------------- */
typedef struct nb_batch nb_batch;

typedef struct nb_batch_info {
    int32_t nbox;
    int32_t sorted;           /* work items in descending cost order (1) or box order (0) */
    int64_t natoms;           /* atoms over all boxes */
    int64_t nitems;           /* i-clusters (work items) over all boxes */
    int64_t nentries;         /* j-entries over all boxes */
    int64_t evaluated_pairs;  /* sum over boxes of nentries * C * 4 */
    int32_t grid_blocks[2];   /* persistent blocks per launch for C = 4 and C = 8 (0 = unused) */
    int32_t graph_ready;      /* 1 if a captured graph exists for the current lists */
    int32_t pad;
    double build_ms_last;     /* host-timed duration of the last nb_batch_pairlist */
} nb_batch_info;

/* Create a batch of nbox boxes.  atom_off: host [nbox+1] offsets of each box's atoms in the
 * concatenated arrays (atom_off[0] = 0, atom_off[nbox] = common->natoms); boxes: host
 * [nbox][3] box edges; clusters: host [nbox] cluster size per box (4 or 8), or NULL to use
 * common->cluster for all.  common supplies cutoff, buffer, beta, fC, LJ types and the
 * exclusions over the concatenated atoms (global indices; no exclusion may cross boxes);
 * common->box is ignored.  stream: hipStream_t used by all batch calls; graph capture needs a
 * stream other than the legacy default stream.
 * Errors: NB_ERR_ARG, NB_ERR_CUTOFF (any box), NB_ERR_OOM, NB_ERR_HIP. */
int nb_batch_setup(nb_batch **out, int32_t nbox, const int32_t *atom_off, const double *boxes,
                   const int32_t *clusters, const nb_params *common, void *stream);

/* Work schedule: sorted != 0 orders work items by descending j-list length (the default);
 * blocks_per_cu > 0 fixes the persistent grid to that many 256-thread blocks per compute unit
 * (0 = as many as fit). Invalidates a captured graph. */
int nb_batch_set_schedule(nb_batch *bt, int32_t sorted, int32_t blocks_per_cu);

/* Schedule autotuner on the batch's own data (the order of the work decides the tail of the
 * kernel, the effect the paper's list sorting addresses, section III-A): times nb_batch_forces for each of the
 * NB_BATCH_NSCHED candidate schedules, in this order: sorted with as many blocks as fit, sorted
 * with 1, 2 and 4 blocks per compute unit, box order with as many blocks as fit (2 warm-up and
 * reps timed calls each, HIP events on the batch stream), then applies the fastest.  Inputs as
 * for nb_batch_forces (f and e are overwritten by the timed calls); us_out: host
 * [NB_BATCH_NSCHED] microseconds per call, or NULL; best: host [2] (sorted, blocks_per_cu) of
 * the chosen schedule, or NULL.  Needs a list (nb_batch_pairlist); synchronises.
 * Errors: NB_ERR_ARG (NULL input, reps < 1), NB_ERR_STATE, NB_ERR_HIP. */
#define NB_BATCH_NSCHED 5
int nb_batch_tune_schedule(nb_batch *bt, const float *x, const float *q, const int32_t *type, float *f,
                           double *e, int32_t reps, double *us_out, int32_t *best);

/* Build every box's pair list from device coordinates x [natoms][3] (concatenated), then the
 * work list.  Synchronises (overflow checks, work-list upload). Not capturable. */
int nb_batch_pairlist(nb_batch *bt, const float *x_dev);

/* Forces (f [natoms][3], concatenated, original order) and per-box energies e [nbox][2]
 * (E_LJ, E_C) for device inputs x, q, type.  Four launches on the batch stream; no allocation
 * or host synchronisation.  Errors: NB_ERR_STATE (no lists), NB_ERR_HIP. */
int nb_batch_forces(nb_batch *bt, const float *x, const float *q, const int32_t *type, float *f,
                    double *e);

/* As nb_batch_forces, through a HIP graph: the first call after a list build (or with other
 * pointers) captures the launches and instantiates the graph, later calls replay it with one
 * hipGraphLaunch. */
int nb_batch_graph_forces(nb_batch *bt, const float *x, const float *q, const int32_t *type,
                          float *f, double *e);

int nb_batch_get_info(nb_batch *bt, nb_batch_info *info);
/* Synchronise the batch stream and report NB_ERR_RANGE if a pair force component exceeded the
 * fixed-point accumulators' check (as for nb_forces) since the last call; clears it. */
int nb_batch_check(nb_batch *bt);
const char *nb_batch_last_error(nb_batch *bt);
int nb_batch_destroy(nb_batch *bt);

/* ---- Autotuner of the batched form ------------------------------------------------------
 * Chooses, on the caller's own boxes, the cluster size (4 or 8) per box-size bucket and the work
 * schedule of the persistent force kernel: the order of the work and the cluster shape decide
 * the tail of a batched call and the evaluated pairs per useful one (the effects of the
 * paper's post-prune list sorting, section III-A, and of small systems, section IV-C).  Sizes
 * are grouped in NB_TUNE_BUCKETS logarithmic buckets over [NB_TUNE_NMIN, NB_TUNE_NMAX) atoms
 * (smaller and larger boxes join the first and last bucket).  For every bucket with boxes and no
 * cache entry, up to NB_TUNE_SAMPLE of its boxes are gathered into a batch built once with C = 4
 * and once with C = 8, and 10 nb_batch_forces calls of each are timed with HIP events after 3
 * warm-up calls; the faster shape is kept.  With the shapes fixed, the schedule is chosen by
 * nb_batch_tune_schedule on the whole batch (unless cached).  Decisions are cached in a JSON
 * file, an object whose keys name the GPU architecture, HIP version, cutoff, interaction
 * flavour, energy mode and bucket (or batch size) and whose values hold the choice and the
 * measured microseconds; a later call with the same kind of boxes reuses them without timing.
 *   Inputs: as nb_batch_setup (atom_off, boxes host; common host) and nb_batch_pairlist /
 *   nb_batch_forces (x, q, type: device, concatenated); cache_path: a file to read and write,
 *   or NULL for no cache; stream: hipStream_t of the timed calls.
 *   Outputs: clusters_out host [nbox] (the chosen C of every box, to pass to nb_batch_setup),
 *   *res (per bucket: edges, boxes, choice, timings or cached; the schedule and its timings; the
 *   host seconds spent).
 * Allocates temporary batches and device buffers and synchronises; not capturable.  Errors:
 * NB_ERR_ARG, NB_ERR_IO (the cache file exists but cannot be read or is not such an object, or
 * cannot be written; checked before the device is used), and those of nb_batch_setup,
 * nb_batch_pairlist and nb_batch_forces.  nb_autotune_last_error() describes the last failure
 * of this host thread. */
#define NB_TUNE_BUCKETS 5
#define NB_TUNE_NMIN 3000
#define NB_TUNE_NMAX 30000
#define NB_TUNE_SAMPLE 16
typedef struct nb_tune_result {
    int32_t nbuckets;
    int32_t bucket_lo[NB_TUNE_BUCKETS], bucket_hi[NB_TUNE_BUCKETS]; /* atom-count edges */
    int32_t bucket_boxes[NB_TUNE_BUCKETS];    /* boxes of the batch in each bucket */
    int32_t bucket_cluster[NB_TUNE_BUCKETS];  /* chosen C (0: no box in the bucket) */
    int32_t bucket_cached[NB_TUNE_BUCKETS];   /* 1: taken from the cache, not timed */
    double bucket_us[NB_TUNE_BUCKETS][2];     /* us per sample call with C = 4 and C = 8 */
    int32_t sorted, blocks_per_cu;            /* chosen schedule (nb_batch_set_schedule) */
    int32_t schedule_cached;
    int32_t pad;
    double schedule_us[NB_BATCH_NSCHED];      /* as nb_batch_tune_schedule's us_out */
    double seconds;                           /* host time spent in the call */
} nb_tune_result;
int nb_autotune(int32_t nbox, const int32_t *atom_off, const double *boxes, const nb_params *common,
                const float *x, const float *q, const int32_t *type, const char *cache_path,
                void *stream, int32_t *clusters_out, nb_tune_result *res);
const char *nb_autotune_last_error(void);

/* ---- Reciprocal-space Ewald: smooth particle-mesh Ewald (PME) ---------------------------
 * The part that completes the real-space Ewald forces of nb_forces when a run uses PME (the
 * paper's production runs; section II-C and the PME kernels of Fig. 2), with the same beta:
 * together with NB_EWALD_CORR (exclusion correction and self term) it gives the full Ewald
 * electrostatics.  Charges are spread onto a K1 x K2 x K3 grid with cardinal B-splines of order
 * n, the grid is convolved with the Ewald kernel by FFT (hipFFT, FP64), and the forces are
 * gathered with the B-spline derivatives:
 *   E_rec = 1/2 sum_m G(m) |FFT(Q)(m)|^2,
 *   G(m) = fC / (pi V) exp(-pi^2 |m|^2 / beta^2) / |m|^2 |b1(m1) b2(m2) b3(m3)|^2, G(0) = 0,
 * an approximation of the Ewald reciprocal sum that converges to it as the grid is refined. */
typedef struct nb_pme nb_pme;

typedef struct nb_pme_params {
    double box[3];          /* rectangular box edges Lx, Ly, Lz (nm), > 0 */
    double ewald_beta;      /* Ewald splitting parameter beta (nm^-1), > 0 */
    double coulomb_const;   /* fC (kJ mol^-1 nm e^-2), > 0 */
    int32_t grid[3];        /* K1, K2, K3: grid points per axis, 2 * order .. 1024 */
    int32_t order;          /* B-spline order n: 4, 6 or 8 */
    int32_t natoms;         /* 1 .. 2^27 */
} nb_pme_params;

/* Create a PME context on the current device: device grids, the influence function (computed
 * in FP64 on the host) and two hipFFT plans bound to hip_stream.
 * Errors: NB_ERR_ARG (invalid parameters), NB_ERR_OOM, NB_ERR_HIP. */
int nb_pme_setup(nb_pme **out, const nb_pme_params *p, void *hip_stream);

/* Reciprocal-space forces and energy of the device arrays x [natoms][3] (any periodic images)
 * and q [natoms], by smooth PME (the PME kernels of the paper's Fig. 2): f_dev [natoms][3]
 * overwritten with the reciprocal forces (FP32, original order; add them to nb_forces' output),
 * e_dev[0] = E_rec (device double).  The grid, the FFTs and all sums are FP64; the charge spread
 * adds with FP64 atomics in on-chip memory, so results may differ in the last bits between
 * calls.  The system should be neutral (a net charge adds no energy here).  Asynchronous on the
 * context's stream; no allocation.  Errors: NB_ERR_ARG, NB_ERR_HIP. */
int nb_pme_forces(nb_pme *pme, const float *x_dev, const float *q_dev, float *f_dev, double *e_dev);

/* Message of the last error of this context (or of the last failed nb_pme_setup for NULL). */
const char *nb_pme_last_error(nb_pme *pme);

/* Synchronise the stream and free the context. */
int nb_pme_destroy(nb_pme *pme);

#ifdef __cplusplus
}
#endif
#endif /* NB_H */
