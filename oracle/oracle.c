/*
 * FP64 reference ("oracle") for the short-range nonbonded forces.
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the CPU-baseline leg of the
 * benchmark may load this library.  It shares no code, header, table or constant generator
 * with the HIP path; the product path never calls it.
 *
 * What it computes.  The paper names the computation (section III-A: the NBNXM kernel,
 * "short-range non-bonded forces", the longest-running kernel of the MD step; the Fig. 3
 * caption names the flavour "Ewald electrostatics, Lennard-Jones with combination rule") but
 * prints no formula.  The formulas below are the textbook definitions of that flavour as the
 * method specifies it: Lennard-Jones with a potential-shift cutoff plus the real-space part
 * of Ewald summation (Coulomb screened by erfc), both shifted to zero at the cutoff, summed
 * over minimum-image pairs of a rectangular periodic box.
 *
 *   For every unordered pair {i, j}, i != j, not excluded, with
 *     d = x_i - x_j - L * rint((x_i - x_j) / L)   (per component),  r = |d|,  r < rc:
 *   E_LJ,ij = C12 (r^-12 - rc^-12) - C6 (r^-6 - rc^-6)
 *   E_C,ij  = fC q_i q_j (erfc(beta r) / r - erfc(beta rc) / rc)
 *   F_ij    = [12 C12 r^-14 - 6 C6 r^-8
 *              + fC q_i q_j (erfc(beta r) / r^3 + 2 beta / sqrt(pi) exp(-beta^2 r^2) / r^2)] d
 *   F_i += F_ij,  F_j -= F_ij.
 *   Virial (also reported): Xi = -1/2 sum over the same pairs of d (x) F_ij (3 x 3, symmetric).
 *   C6 = 4 eps_ab sigma_ab^6, C12 = 4 eps_ab sigma_ab^12 with Lorentz-Berthelot combination
 *   sigma_ab = (sigma_a + sigma_b) / 2, eps_ab = sqrt(eps_a eps_b).
 *   Excluded pairs contribute nothing (no reciprocal-space exclusion correction here).
 *
 * Other flavours (oracle_set_flavor; the paper's runs also use reaction-field electrostatics and
 * force-switched Lennard-Jones, section IV):
 *   reaction field, dielectric eps_rf (0 = infinity):
 *     k_rf = (eps_rf - 1) / ((2 eps_rf + 1) rc^3)  (1 / (2 rc^3) for eps_rf = 0),
 *     c_rf = 1/rc + k_rf rc^2,
 *     E_C,ij = fC q_i q_j (1/r + k_rf r^2 - c_rf),  F_C,ij = fC q_i q_j (1/r^3 - 2 k_rf) d;
 *   force switch from r1 to rc, for each power r^-a of the LJ form (a = 6, 12) with t = r - r1:
 *     force  a r^-(a+1) + A_a t^2 + B_a t^3 for t > 0 (a r^-(a+1) otherwise),
 *     A_a = -a ((a+4) rc - (a+1) r1) / (rc^(a+2) (rc - r1)^2),
 *     B_a =  a ((a+3) rc - (a+1) r1) / (rc^(a+2) (rc - r1)^3),
 *     potential r^-a - (A_a/3) t^3 - (B_a/4) t^4 - K_a, K_a its value at rc without K_a;
 *     E_LJ,ij = C12 Phi_12 - C6 Phi_6,  F_LJ,ij = (C12 F_12 - C6 F_6) d / r.
 *
 * Ewald corrections (oracle_ewald_corrections), the terms that complete the real-space sum
 * once a reciprocal-space part is added (the paper's runs use PME, section II-C):
 *   every excluded pair {i, j}, at its minimum-image distance r (any r):
 *     E_excl,ij = -fC q_i q_j erf(beta r) / r,
 *     F_ij (on i) = fC q_i q_j [2 beta / sqrt(pi) exp(-beta^2 r^2) / r^2 - erf(beta r) / r^3] d,
 *     (r = 0: E = -fC q_i q_j 2 beta / sqrt(pi), F = 0);
 *   self term E_self = -fC beta / sqrt(pi) sum_i q_i^2 (no force).
 *
 * Everything is FP64 with libm erfc/exp.  Loops are plain: a full double loop over atoms
 * (each unordered pair visited twice, each visit adding only to atom i) or the same loop over
 * 27 neighbouring cells.  Parallelism is an OpenMP loop over i with no shared writes.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define TWO_OVER_SQRT_PI 1.1283791670955126

void oracle_set_threads(int nthreads) {
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

int oracle_get_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Lorentz-Berthelot table.  With round32 != 0 each entry is rounded once to FP32 and widened
 * back, which is how the instance's table is defined (the GPU receives the same FP32 values). */
void oracle_lj_table(int nt, const double *sigma, const double *eps, int round32,
                     double *c6, double *c12) {
    for (int a = 0; a < nt; ++a) {
        for (int b = 0; b < nt; ++b) {
            double s = 0.5 * (sigma[a] + sigma[b]);
            double e = sqrt(eps[a] * eps[b]);
            double s6 = s * s * s * s * s * s;
            double v6 = 4.0 * e * s6, v12 = 4.0 * e * s6 * s6;
            if (round32) {
                v6 = (double)(float)v6;
                v12 = (double)(float)v12;
            }
            c6[a * nt + b] = v6;
            c12[a * nt + b] = v12;
        }
    }
}

static void min_image(const double *xi, const double *xj, const double *box, double *d) {
    for (int c = 0; c < 3; ++c) {
        double v = xi[c] - xj[c];
        d[c] = v - box[c] * rint(v / box[c]);
    }
}

static int is_excluded(int i, int j, const int *off, const int *idx) {
    if (!off) return 0;
    for (int k = off[i]; k < off[i + 1]; ++k)
        if (idx[k] == j) return 1;
    return 0;
}

/* Interaction flavour: 0 = Ewald real space / LJ potential shift (the default); see above. */
static int g_elec = 0, g_vdw = 0;
static double g_eps_rf = 0.0, g_rswitch = 0.0;

void oracle_set_flavor(int elec, int vdw, double eps_rf, double rswitch) {
    g_elec = elec;
    g_vdw = vdw;
    g_eps_rf = eps_rf;
    g_rswitch = rswitch;
}

/* Force-switched power r^-a: potential (shifted to zero at rc) and force magnitude at r. */
static void switched_power(double a, double r, double r1, double rc, double *phi, double *force) {
    double d = rc - r1;
    double A = -a * ((a + 4.0) * rc - (a + 1.0) * r1) / (pow(rc, a + 2.0) * d * d);
    double B = a * ((a + 3.0) * rc - (a + 1.0) * r1) / (pow(rc, a + 2.0) * d * d * d);
    double K = pow(rc, -a) - A / 3.0 * d * d * d - B / 4.0 * d * d * d * d;
    double t = r > r1 ? r - r1 : 0.0;
    *phi = pow(r, -a) - A / 3.0 * t * t * t - B / 4.0 * t * t * t * t - K;
    *force = a * pow(r, -a - 1.0) + A * t * t + B * t * t * t;
}

/* Energies (shifted LJ, shifted and unshifted Coulomb) and the force factor f with
 * F_ij = f * d for one pair at distance r < rc. */
typedef struct {
    double elj, ec, ec_unshifted, fscal;
} pair_out;

static pair_out pair_terms(double r, double c6, double c12, double qq, double rc, double beta,
                           double fc) {
    pair_out o;
    double ir = 1.0 / r, ir2 = ir * ir, ir6 = ir2 * ir2 * ir2;
    double irc = 1.0 / rc, irc6 = irc * irc * irc * irc * irc * irc;
    double flj;
    if (g_vdw == 0) {
        o.elj = c12 * (ir6 * ir6 - irc6 * irc6) - c6 * (ir6 - irc6);
        flj = 12.0 * c12 * ir6 * ir6 * ir2 - 6.0 * c6 * ir6 * ir2;
    } else {
        double p6, f6, p12, f12;
        switched_power(6.0, r, g_rswitch, rc, &p6, &f6);
        switched_power(12.0, r, g_rswitch, rc, &p12, &f12);
        o.elj = c12 * p12 - c6 * p6;
        flj = (c12 * f12 - c6 * f6) * ir;
    }
    double fcoul;
    if (g_elec == 0) {
        double ercf = erfc(beta * r);
        o.ec_unshifted = fc * qq * ercf * ir;
        o.ec = fc * qq * (ercf * ir - erfc(beta * rc) * irc);
        fcoul = fc * qq * (ercf * ir2 * ir + TWO_OVER_SQRT_PI * beta * exp(-beta * beta * r * r) * ir2);
    } else {
        double krf = g_eps_rf == 0.0 ? 0.5 / (rc * rc * rc)
                                     : (g_eps_rf - 1.0) / ((2.0 * g_eps_rf + 1.0) * rc * rc * rc);
        double crf = 1.0 / rc + krf * rc * rc;
        o.ec_unshifted = fc * qq * (ir + krf * r * r);
        o.ec = fc * qq * (ir + krf * r * r - crf);
        fcoul = fc * qq * (ir2 * ir - 2.0 * krf);
    }
    o.fscal = flj + fcoul;
    return o;
}

/* Per-atom accumulation shared by both enumerations: the visit (i, j) adds F_ij to atom i and
 * half of each pair energy to atom i's energy.  Sums over atoms are done serially in atom order. */
typedef struct {
    double elj, ec, ecu, abs_lj, abs_c, qq_in;
    double vir[6]; /* xx, yy, zz, xy, xz, yz: a quarter of -d (x) F_ij per visit */
    int64_t npairs;
} atom_acc;

static void visit(int i, int j, const double *x, const double *q, const int *type, int nt,
                  const double *c6, const double *c12, const double *box, double rc, double beta,
                  double fc, const int *eoff, const int *eidx, double *fi, atom_acc *acc) {
    if (j == i) return;
    double d[3];
    min_image(&x[3 * i], &x[3 * j], box, d);
    double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    if (!(r2 < rc * rc)) return;
    if (is_excluded(i, j, eoff, eidx)) return;
    int tp = type[i] * nt + type[j];
    pair_out o = pair_terms(sqrt(r2), c6[tp], c12[tp], q[i] * q[j], rc, beta, fc);
    fi[0] += o.fscal * d[0];
    fi[1] += o.fscal * d[1];
    fi[2] += o.fscal * d[2];
    acc->elj += 0.5 * o.elj;
    acc->ec += 0.5 * o.ec;
    acc->ecu += 0.5 * o.ec_unshifted;
    acc->abs_lj += 0.5 * fabs(o.elj);
    acc->abs_c += 0.5 * fabs(o.ec);
    /* virial -1/2 sum over pairs of d (x) F_ij; each pair is visited twice with the same
     * product d (x) F_ij */
    acc->vir[0] -= 0.25 * o.fscal * d[0] * d[0];
    acc->vir[1] -= 0.25 * o.fscal * d[1] * d[1];
    acc->vir[2] -= 0.25 * o.fscal * d[2] * d[2];
    acc->vir[3] -= 0.25 * o.fscal * d[0] * d[1];
    acc->vir[4] -= 0.25 * o.fscal * d[0] * d[2];
    acc->vir[5] -= 0.25 * o.fscal * d[1] * d[2];
    if (i < j) {
        acc->npairs += 1;
        acc->qq_in += q[i] * q[j];
    }
}

static void finish(int n, const atom_acc *acc, double *eatom_lj, double *eatom_c, double *out) {
    double s[6] = {0, 0, 0, 0, 0, 0}, v[6] = {0, 0, 0, 0, 0, 0};
    int64_t np = 0;
    for (int i = 0; i < n; ++i) {
        for (int k = 0; k < 6; ++k) v[k] += acc[i].vir[k];
        s[0] += acc[i].elj;
        s[1] += acc[i].ec;
        s[2] += acc[i].ecu;
        s[3] += acc[i].abs_lj;
        s[4] += acc[i].abs_c;
        s[5] += acc[i].qq_in;
        np += acc[i].npairs;
        if (eatom_lj) eatom_lj[i] = acc[i].elj;
        if (eatom_c) eatom_c[i] = acc[i].ec;
    }
    /* out: E_LJ, E_C, E_C without the potential shift, sum |E_LJ,ij|, sum |E_C,ij|,
     *      number of interacting pairs, sum of q_i q_j over interacting pairs, and from out[7]
     *      the virial -1/2 sum d (x) F_ij as xx, yy, zz, xy, xz, yz */
    for (int k = 0; k < 6; ++k) out[7 + k] = v[k];
    out[0] = s[0];
    out[1] = s[1];
    out[2] = s[2];
    out[3] = s[3];
    out[4] = s[4];
    out[5] = (double)np;
    out[6] = s[5];
}

/* O(N^2) minimum-image brute force: the definition. */
int oracle_forces(int n, const double *x, const double *q, const int *type, int nt,
                  const double *c6, const double *c12, const double *box, double rc, double beta,
                  double fc, const int *eoff, const int *eidx, double *f, double *eatom_lj,
                  double *eatom_c, double *out) {
    atom_acc *acc = (atom_acc *)calloc((size_t)n, sizeof(atom_acc));
    if (!acc) return -1;
#pragma omp parallel for schedule(dynamic, 64)
    for (int i = 0; i < n; ++i) {
        double fi[3] = {0, 0, 0};
        for (int j = 0; j < n; ++j)
            visit(i, j, x, q, type, nt, c6, c12, box, rc, beta, fc, eoff, eidx, fi, &acc[i]);
        f[3 * i] = fi[0];
        f[3 * i + 1] = fi[1];
        f[3 * i + 2] = fi[2];
    }
    finish(n, acc, eatom_lj, eatom_c, out);
    free(acc);
    return 0;
}

/* Cells of edge >= rc along each axis; the same visits restricted to the 27 cells around
 * atom i's cell.  Needs at least 3 cells per axis so that the 27 neighbours are distinct. */
typedef struct {
    int nc[3];
    int *start, *atoms;
} cell_grid;

static int cell_of(const double *xi, const double *box, const int *nc, int c) {
    double w = xi[c] - box[c] * floor(xi[c] / box[c]);
    int k = (int)floor(w / box[c] * nc[c]);
    if (k >= nc[c]) k = nc[c] - 1;
    if (k < 0) k = 0;
    return k;
}

static int build_cells(int n, const double *x, const double *box, double rc, cell_grid *g) {
    for (int c = 0; c < 3; ++c) {
        g->nc[c] = (int)floor(box[c] / rc);
        if (g->nc[c] < 3) return -1;
    }
    int ncell = g->nc[0] * g->nc[1] * g->nc[2];
    g->start = (int *)calloc((size_t)ncell + 1, sizeof(int));
    g->atoms = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    int *cid = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    int *fill = (int *)calloc((size_t)ncell, sizeof(int));
    if (!g->start || !g->atoms || !cid || !fill) return -2;
    for (int i = 0; i < n; ++i) {
        int k0 = cell_of(&x[3 * i], box, g->nc, 0), k1 = cell_of(&x[3 * i], box, g->nc, 1),
            k2 = cell_of(&x[3 * i], box, g->nc, 2);
        cid[i] = (k0 * g->nc[1] + k1) * g->nc[2] + k2;
        g->start[cid[i] + 1]++;
    }
    for (int c = 0; c < ncell; ++c) g->start[c + 1] += g->start[c];
    for (int i = 0; i < n; ++i) g->atoms[g->start[cid[i]] + fill[cid[i]]++] = i;
    free(cid);
    free(fill);
    return 0;
}

int oracle_forces_cells(int n, const double *x, const double *q, const int *type, int nt,
                        const double *c6, const double *c12, const double *box, double rc,
                        double beta, double fc, const int *eoff, const int *eidx, double *f,
                        double *eatom_lj, double *eatom_c, double *out) {
    cell_grid g;
    if (build_cells(n, x, box, rc, &g) != 0)
        return oracle_forces(n, x, q, type, nt, c6, c12, box, rc, beta, fc, eoff, eidx, f,
                             eatom_lj, eatom_c, out);
    atom_acc *acc = (atom_acc *)calloc((size_t)n, sizeof(atom_acc));
    if (!acc) return -1;
#pragma omp parallel for schedule(dynamic, 64)
    for (int i = 0; i < n; ++i) {
        double fi[3] = {0, 0, 0};
        int k[3];
        for (int c = 0; c < 3; ++c) k[c] = cell_of(&x[3 * i], box, g.nc, c);
        for (int a = -1; a <= 1; ++a)
            for (int b = -1; b <= 1; ++b)
                for (int e = -1; e <= 1; ++e) {
                    int c0 = (k[0] + a + g.nc[0]) % g.nc[0];
                    int c1 = (k[1] + b + g.nc[1]) % g.nc[1];
                    int c2 = (k[2] + e + g.nc[2]) % g.nc[2];
                    int cell = (c0 * g.nc[1] + c1) * g.nc[2] + c2;
                    for (int s = g.start[cell]; s < g.start[cell + 1]; ++s)
                        visit(i, g.atoms[s], x, q, type, nt, c6, c12, box, rc, beta, fc, eoff,
                              eidx, fi, &acc[i]);
                }
        f[3 * i] = fi[0];
        f[3 * i + 1] = fi[1];
        f[3 * i + 2] = fi[2];
    }
    finish(n, acc, eatom_lj, eatom_c, out);
    free(acc);
    free(g.start);
    free(g.atoms);
    return 0;
}

/* Forces and per-atom energies of a subset of atoms only (brute force over all partners):
 * the same visits as oracle_forces restricted to the listed atoms i, so every listed row equals
 * the corresponding row of oracle_forces.  fs receives 3 values per listed atom; es_lj / es_c
 * (may be NULL) receive each listed atom's half of its pair energies (eatom_lj / eatom_c of
 * oracle_forces).  Used for finite differences of a loss where one perturbed coordinate or
 * charge changes only the rows of its neighbours. */
int oracle_forces_subset(int n, const double *x, const double *q, const int *type, int nt,
                         const double *c6, const double *c12, const double *box, double rc,
                         double beta, double fc, const int *eoff, const int *eidx, int nsub,
                         const int *sub, double *fs, double *es_lj, double *es_c) {
#pragma omp parallel for schedule(dynamic, 4)
    for (int s = 0; s < nsub; ++s) {
        int i = sub[s];
        double fi[3] = {0, 0, 0};
        atom_acc acc;
        memset(&acc, 0, sizeof(acc));
        for (int j = 0; j < n; ++j)
            visit(i, j, x, q, type, nt, c6, c12, box, rc, beta, fc, eoff, eidx, fi, &acc);
        fs[3 * s] = fi[0];
        fs[3 * s + 1] = fi[1];
        fs[3 * s + 2] = fi[2];
        if (es_lj) es_lj[s] = acc.elj;
        if (es_c) es_c[s] = acc.ec;
    }
    return 0;
}

/* The set of interacting pairs (i < j, original indices) with their FP64 distances, in
 * lexicographic order.  Returns the total count; at most cap entries are written. */
int64_t oracle_pairs(int n, const double *x, const double *box, double rc, const int *eoff,
                     const int *eidx, int64_t cap, int32_t *pi, int32_t *pj, double *pr) {
    int64_t *cnt = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    if (!cnt) return -1;
#pragma omp parallel for schedule(dynamic, 64)
    for (int i = 0; i < n; ++i) {
        int64_t c = 0;
        for (int j = i + 1; j < n; ++j) {
            double d[3];
            min_image(&x[3 * i], &x[3 * j], box, d);
            double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            if (r2 < rc * rc && !is_excluded(i, j, eoff, eidx)) ++c;
        }
        cnt[i + 1] = c;
    }
    for (int i = 0; i < n; ++i) cnt[i + 1] += cnt[i];
    int64_t total = cnt[n];
#pragma omp parallel for schedule(dynamic, 64)
    for (int i = 0; i < n; ++i) {
        int64_t w = cnt[i];
        for (int j = i + 1; j < n; ++j) {
            double d[3];
            min_image(&x[3 * i], &x[3 * j], box, d);
            double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            if (r2 < rc * rc && !is_excluded(i, j, eoff, eidx)) {
                if (w < cap) {
                    pi[w] = i;
                    pj[w] = j;
                    pr[w] = sqrt(r2);
                }
                ++w;
            }
        }
    }
    free(cnt);
    return total;
}

/*
 * Vector-Jacobian product of (F, E_LJ, E_C) for given cotangents gF = dL/dF (3 per atom) and
 * gE = (dL/dE_LJ, dL/dE_C).  Per interacting pair, with u = d / r, f the force factor
 * (F_ij = f d), f' = df/dr and delta = gF_i - gF_j:
 *   dL/dx_i += f delta + (f'/r)(d . delta) d - (gE_LJ f_LJ + gE_C f_C) d   (and minus for j),
 *     i.e. the Jacobian dF_ij/dd = f I + (f'/r) d d^T applied to delta, plus the energy term
 *     dE_ij/dd = -f d;
 *   dL/dq_i += fC q_j [h (delta . d) + gE_C g],  h = erfc(beta r)/r^3 + 2 beta/sqrt(pi)
 *     exp(-beta^2 r^2)/r^2,  g = erfc(beta r)/r - erfc(beta rc)/rc  (likewise for j);
 *   dL/dC6_ab  += -6 r^-8 (delta . d) - gE_LJ (r^-6 - rc^-6),
 *   dL/dC12_ab += 12 r^-14 (delta . d) + gE_LJ (r^-12 - rc^-12),
 *   chained to sigma and epsilon through Lorentz-Berthelot; each of the pair's two type slots
 *   receives half of d sigma_ab and a sqrt(eps_other / eps_self)/2 share of d eps_ab.
 * The table is built here in FP64 without rounding so that L is differentiable in sigma, eps.
 * Types with epsilon = 0 get epsilon gradient 0 (the derivative does not exist there).
 */
int oracle_vjp(int n, const double *x, const double *q, const int *type, int nt,
               const double *sigma, const double *eps, const double *box, double rc, double beta,
               double fc, const int *eoff, const int *eidx, const double *gF, const double *gE,
               double *dx, double *dq, double *dsig, double *deps) {
    if (g_elec != 0 || g_vdw != 0) return -2; /* defined for Ewald / potential shift only */
    double *c6 = (double *)malloc(sizeof(double) * (size_t)nt * nt);
    double *c12 = (double *)malloc(sizeof(double) * (size_t)nt * nt);
    /* per-atom partial type gradients: [n][nt] for sigma and eps, summed serially afterwards */
    double *ps = (double *)calloc((size_t)n * nt, sizeof(double));
    double *pe = (double *)calloc((size_t)n * nt, sizeof(double));
    if (!c6 || !c12 || !ps || !pe) return -1;
    oracle_lj_table(nt, sigma, eps, 0, c6, c12);
    const double irc = 1.0 / rc, irc6 = pow(irc, 6.0);
    const double shc = erfc(beta * rc) * irc;
#pragma omp parallel for schedule(dynamic, 64)
    for (int i = 0; i < n; ++i) {
        double gx[3] = {0, 0, 0}, gq = 0;
        for (int j = 0; j < n; ++j) {
            if (j == i) continue;
            double d[3];
            min_image(&x[3 * i], &x[3 * j], box, d);
            double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            if (!(r2 < rc * rc) || is_excluded(i, j, eoff, eidx)) continue;
            double r = sqrt(r2), ir = 1.0 / r, ir2 = ir * ir, ir6 = ir2 * ir2 * ir2;
            int tp = type[i] * nt + type[j];
            double C6 = c6[tp], C12 = c12[tp], qq = q[i] * q[j];
            double ercf = erfc(beta * r), ex = exp(-beta * beta * r2);
            double flj = 12.0 * C12 * ir6 * ir6 * ir2 - 6.0 * C6 * ir6 * ir2;
            double dflj = -168.0 * C12 * ir6 * ir6 * ir2 * ir + 48.0 * C6 * ir6 * ir2 * ir;
            double h = ercf * ir2 * ir + TWO_OVER_SQRT_PI * beta * ex * ir2;
            double dh = -3.0 * ercf * ir2 * ir2 -
                        TWO_OVER_SQRT_PI * beta * ex * (3.0 * ir2 * ir + 2.0 * beta * beta * ir);
            double fcl = fc * qq * h, dfcl = fc * qq * dh;
            double fsc = flj + fcl, dfsc_r = (dflj + dfcl) * ir;
            double del[3], dd = 0;
            for (int c = 0; c < 3; ++c) {
                del[c] = gF[3 * i + c] - gF[3 * j + c];
                dd += del[c] * d[c];
            }
            for (int c = 0; c < 3; ++c)
                gx[c] += fsc * del[c] + dfsc_r * dd * d[c] - (gE[0] * flj + gE[1] * fcl) * d[c];
            double g = ercf * ir - shc;
            gq += fc * q[j] * (h * dd + gE[1] * g);
            /* LJ parameters: this visit carries the type slot of atom i */
            double G6 = -6.0 * ir6 * ir2 * dd - gE[0] * (ir6 - irc6);
            double G12 = 12.0 * ir6 * ir6 * ir2 * dd + gE[0] * (ir6 * ir6 - irc6 * irc6);
            int ta = type[i], tb = type[j];
            double s = 0.5 * (sigma[ta] + sigma[tb]);
            double e = sqrt(eps[ta] * eps[tb]);
            double s5 = s * s * s * s * s, s6 = s5 * s, s11 = s6 * s5;
            /* d C6 / d sigma_ab = 24 e s^5, d C12 / d sigma_ab = 48 e s^11 ; slot share 1/2 */
            ps[(size_t)i * nt + ta] += 0.5 * (G6 * 24.0 * e * s5 + G12 * 48.0 * e * s11);
            /* d C6 / d eps_ab = 4 s^6, d C12 / d eps_ab = 4 s^12 ; d eps_ab / d eps_a slot share
             * = sqrt(eps_b / eps_a) / 2 */
            if (eps[ta] > 0.0)
                pe[(size_t)i * nt + ta] +=
                    (G6 * 4.0 * s6 + G12 * 4.0 * s6 * s6) * 0.5 * sqrt(eps[tb] / eps[ta]);
        }
        dx[3 * i] = gx[0];
        dx[3 * i + 1] = gx[1];
        dx[3 * i + 2] = gx[2];
        dq[i] = gq;
    }
    for (int t = 0; t < nt; ++t) {
        dsig[t] = 0;
        deps[t] = 0;
    }
    for (int i = 0; i < n; ++i)
        for (int t = 0; t < nt; ++t) {
            dsig[t] += ps[(size_t)i * nt + t];
            deps[t] += pe[(size_t)i * nt + t];
        }
    free(c6);
    free(c12);
    free(ps);
    free(pe);
    return 0;
}

/*
 * Ewald exclusion correction and self term (see the header): out[0] = sum over excluded pairs
 * of E_excl,ij, out[1] = E_self, out[2 ..] = the virial -1/2 sum d (x) F_ij of the exclusion
 * correction (xx, yy, zz, xy, xz, yz); f [n][3] receives the exclusion-correction forces
 * (overwritten).
 * Each excluded pair is visited from both atoms (the CSR lists are symmetric); each visit adds
 * the force on its own atom, and the pair energy is taken once, at i < j.
 */
int oracle_ewald_corrections(int n, const double *x, const double *q, const double *box,
                             double beta, double fc, const int *eoff, const int *eidx, double *f,
                             double *out) {
    double e_excl = 0.0, e_self = 0.0, vir[6] = {0, 0, 0, 0, 0, 0};
    for (int i = 0; i < n; ++i) {
        f[3 * i] = f[3 * i + 1] = f[3 * i + 2] = 0.0;
        e_self -= fc * beta * (0.5 * TWO_OVER_SQRT_PI) * q[i] * q[i];
        if (!eoff) continue;
        for (int k = eoff[i]; k < eoff[i + 1]; ++k) {
            const int j = eidx[k];
            double d[3];
            min_image(x + 3 * i, x + 3 * j, box, d);
            const double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            const double qq = fc * q[i] * q[j];
            double e, fs;
            if (r == 0.0) {
                e = -qq * TWO_OVER_SQRT_PI * beta;
                fs = 0.0;
            } else {
                const double er = erf(beta * r);
                e = -qq * er / r;
                fs = qq * (TWO_OVER_SQRT_PI * beta * exp(-beta * beta * r * r) / (r * r) - er / (r * r * r));
            }
            for (int c = 0; c < 3; ++c) f[3 * i + c] += fs * d[c];
            if (i < j) {
                e_excl += e;
                vir[0] -= 0.5 * fs * d[0] * d[0];
                vir[1] -= 0.5 * fs * d[1] * d[1];
                vir[2] -= 0.5 * fs * d[2] * d[2];
                vir[3] -= 0.5 * fs * d[0] * d[1];
                vir[4] -= 0.5 * fs * d[0] * d[2];
                vir[5] -= 0.5 * fs * d[1] * d[2];
            }
        }
    }
    out[0] = e_excl;
    out[1] = e_self;
    for (int k = 0; k < 6; ++k) out[2 + k] = vir[k];
    return 0;
}
