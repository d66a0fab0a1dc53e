// Host side of libnb: parameter validation, device buffers, the LJ table and kernel constants,
// the build / force / check entry points of include/nb.h.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "erfcx_rational.h"
#include "nb_internal.h"

namespace {

thread_local std::string g_setup_error;

int fail(nb_ctx *c, int code, const std::string &msg) {
    if (c) c->err = msg;
    else g_setup_error = msg;
    return code;
}

int hip_fail(nb_ctx *c, hipError_t e, const char *where) {
    return fail(c, NB_ERR_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

template <typename T>
int dalloc(nb_ctx *c, T **p, size_t count, const char *what) {
    if (*p) {
        hipFree(*p);
        *p = nullptr;
    }
    if (count == 0) count = 1;
    hipError_t e = hipMalloc((void **)p, sizeof(T) * count);
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(c, NB_ERR_OOM, std::string("hipMalloc failed for ") + what);
    }
    return NB_OK;
}

bool finite_pos(double v) { return isfinite(v) && v > 0.0; }

// j-entries per i-cluster to reserve: clusters (full list, not half) whose bounding boxes can
// come within rlist, from the volume of a cube of twice the cluster edge dilated by rlist.
int estimate_cap(double natoms, const double *box, int C, double rlist) {
    double V = box[0] * box[1] * box[2];
    double rho = natoms / V;
    double a = cbrt(C / rho);
    double s = 2.0 * a;
    double vol = s * s * s + 6.0 * s * s * rlist + 3.0 * M_PI * s * rlist * rlist +
                 4.0 / 3.0 * M_PI * rlist * rlist * rlist;
    double n = vol * rho / NB_JG;  // j-groups of NB_JG atoms within the dilated i-cluster
    int cap = (int)(1.25 * n) + 32;
    return (cap + 31) & ~31;
}

// Force-switch constants for the power r^-a between r1 and rc: the force a r^-(a+1) gains
// A t^2 + B t^3 (t = r - r1) so that it and its derivative vanish at rc; the potential
// r^-a - (A/3) t^3 - (B/4) t^4 is shifted by its value at rc.
struct fswitch_c {
    double A, B, shift;
};
fswitch_c fswitch_consts(double a, double r1, double rc) {
    const double d = rc - r1;
    fswitch_c k;
    k.A = -a * ((a + 4.0) * rc - (a + 1.0) * r1) / (pow(rc, a + 2.0) * d * d);
    k.B = a * ((a + 3.0) * rc - (a + 1.0) * r1) / (pow(rc, a + 2.0) * d * d * d);
    k.shift = pow(rc, -a) - k.A / 3.0 * d * d * d - k.B / 4.0 * d * d * d * d;
    return k;
}

void lj_table(nb_ctx *c, std::vector<float4> &tab) {
    const int nt = c->ntypes;
    tab.assign(2 * nt * nt, make_float4(0, 0, 0, 0));
    // potential shift of the r^-6 and r^-12 parts (their value at rc)
    double irc6 = 1.0 / pow(c->rc, 6.0), irc12 = irc6 * irc6;
    if (c->vdw == NB_VDW_FSWITCH) {
        irc6 = fswitch_consts(6.0, c->rsw, c->rc).shift;
        irc12 = fswitch_consts(12.0, c->rsw, c->rc).shift;
    }
    for (int a = 0; a < nt; ++a)
        for (int b = 0; b < nt; ++b) {
            double s = 0.5 * (c->sigma[a] + c->sigma[b]);
            double e = sqrt(c->epsilon[a] * c->epsilon[b]);
            double s6 = s * s * s * s * s * s;
            double c6 = 4.0 * e * s6, c12 = 4.0 * e * s6 * s6;
            float c6f = (float)c6, c12f = (float)c12;
            double sh = (double)c12f * irc12 - (double)c6f * irc6;
            // the FP64 shift of the FP64 pair energies: C12 k12 - C6 k6 with the kernels' FP64
            // constants, rounded as a device fused multiply-add would round it
            const double shd = std::fma((double)c12f, c->fp.lj_k12, -((double)c6f * c->fp.lj_k6));
            unsigned long long bits;
            std::memcpy(&bits, &shd, sizeof(bits));
            // two float4 per type pair, side by side: one address serves both LDS reads;
            // (C6, C12, 6 C6, 12 C12), (shift, 1 / sigma_ab, FP64 shift as two words)
            tab[2 * (a * nt + b)] = make_float4(c6f, c12f, (float)(6.0 * c6), (float)(12.0 * c12));
            float lo, hi;
            const uint32_t wlo = (uint32_t)bits, whi = (uint32_t)(bits >> 32);
            std::memcpy(&lo, &wlo, sizeof(lo));
            std::memcpy(&hi, &whi, sizeof(hi));
            tab[2 * (a * nt + b) + 1] = make_float4((float)sh, s > 0.0 ? (float)(1.0 / s) : 0.0f, lo, hi);
        }
}

void set_constants(nb_ctx *c) {
    nb_fparams &fp = c->fp;
    for (int k = 0; k < 3; ++k) {
        fp.L[k] = (float)c->box[k];
        fp.nL[k] = -fp.L[k];
    }
    fp.rc2 = (float)(c->rc * c->rc);
    fp.fc = (float)c->fc;
    fp.fcs = fp.fc * NB_FSCALE;
    const double beta = c->beta;
    fp.cexp = (float)(-beta * beta * 1.4426950408889634);
    fp.kb = (float)(2.0 * beta / sqrt(M_PI));
    double bk = 1.0;
    for (int k = 0; k < 6; ++k) {
        if (k < 5) fp.p[k] = (float)(nb_erfcx_p[k] * bk);
        fp.q[k] = (float)(nb_erfcx_q[k] * bk);
        bk *= beta;
    }
    fp.ntypes = c->ntypes;
    c->shift_coul = erfc(beta * c->rc) / c->rc;
    if (c->elec == NB_ELEC_RF) {
        const double rc = c->rc;
        const double krf = c->eps_rf == 0.0 ? 0.5 / (rc * rc * rc)
                                            : (c->eps_rf - 1.0) / ((2.0 * c->eps_rf + 1.0) * rc * rc * rc);
        fp.krf = (float)krf;
        fp.krf_d = krf;
        // c_rf; the FP32-energy path sums q_i q_j without fC, so fC goes into the shift there
        c->shift_coul = (1.0 / rc + krf * rc * rc) * (nb_energy_fp64(c) ? 1.0 : (double)fp.fc);
    }
    fp.lj_k6 = pow(c->rc, -6.0);
    fp.lj_k12 = pow(c->rc, -12.0);
    if (c->vdw == NB_VDW_FSWITCH) {
        const fswitch_c k6 = fswitch_consts(6.0, c->rsw, c->rc), k12 = fswitch_consts(12.0, c->rsw, c->rc);
        fp.lj_k6 = k6.shift;
        fp.lj_k12 = k12.shift;
        fp.sw_r1_d = c->rsw;
        fp.sw_ea6_d = k6.A / 3.0;
        fp.sw_eb6_d = k6.B / 4.0;
        fp.sw_ea12_d = k12.A / 3.0;
        fp.sw_eb12_d = k12.B / 4.0;
        fp.sw_r1 = (float)c->rsw;
        fp.sw_a6 = (float)k6.A;
        fp.sw_b6 = (float)k6.B;
        fp.sw_a12 = (float)k12.A;
        fp.sw_b12 = (float)k12.B;
        fp.fsw_a6 = fp.sw_a6 * NB_FSCALE;
        fp.fsw_b6 = fp.sw_b6 * NB_FSCALE;
        fp.fsw_a12 = fp.sw_a12 * NB_FSCALE;
        fp.fsw_b12 = fp.sw_b12 * NB_FSCALE;
        fp.sw_ea6 = (float)(k6.A / 3.0);
        fp.sw_eb6 = (float)(k6.B / 4.0);
        fp.sw_ea12 = (float)(k12.A / 3.0);
        fp.sw_eb12 = (float)(k12.B / 4.0);
    }
    fp.b2 = (float)(beta * beta);
    fp.irc6 = (float)pow(c->rc, -6.0);
    fp.irc12 = (float)pow(c->rc, -12.0);
    fp.shc = (float)c->shift_coul;
}

// Quintic Hermite segments of erfc(beta r) on [k h, (k+1) h], k = 0 .. n-1, covering [0, rc]:
// on u = r / h - k in [0, 1], the polynomial matching erfc and its first and second derivatives
// (scaled by h and h^2) at both ends; h is the largest power of two with at most 160 segments, so
// r / h is exact in floating point.  Interpolation error below 2e-13 (absolute) at rc = 1 nm.
int upload_etab(nb_ctx *c) {
    double h = 1.0 / 1024.0;
    while (c->rc / h > 159.0) h *= 2.0;
    const int n = (int)ceil(c->rc / h) + 1;
    std::vector<double2> seg(NB_ETAB_W * (size_t)n);
    const double kb = 2.0 * c->beta / sqrt(M_PI), b2 = c->beta * c->beta;
    for (int k = 0; k < n; ++k) {
        const double r0 = k * h, r1 = (k + 1) * h;
        const double f0 = erfc(c->beta * r0), f1 = erfc(c->beta * r1);
        // d/dr erfc(beta r) = -kb exp(-beta^2 r^2), d2/dr2 = 2 beta^2 r kb exp(-beta^2 r^2)
        const double e0 = exp(-b2 * r0 * r0), e1 = exp(-b2 * r1 * r1);
        const double d0 = -kb * e0 * h, d1 = -kb * e1 * h;
        const double s0 = 2.0 * b2 * r0 * kb * e0 * h * h, s1 = 2.0 * b2 * r1 * kb * e1 * h * h;
        const double df = f1 - f0;
        const double c3 = 10.0 * df - 6.0 * d0 - 4.0 * d1 - 0.5 * (3.0 * s0 - s1);
        const double c4 = -15.0 * df + 8.0 * d0 + 7.0 * d1 + 0.5 * (3.0 * s0 - 2.0 * s1);
        const double c5 = 6.0 * df - 3.0 * (d0 + d1) - 0.5 * (s0 - s1);
        seg[NB_ETAB_W * k] = make_double2(f0, d0);
        seg[NB_ETAB_W * k + 1] = make_double2(0.5 * s0, c3);
        seg[NB_ETAB_W * k + 2] = make_double2(c4, c5);
    }
    int r = dalloc(c, &c->etab, seg.size(), "erfc table");
    if (r != NB_OK) return r;
    hipError_t e = hipMemcpy(c->etab, seg.data(), sizeof(double2) * seg.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(c, e, "upload erfc table");
    c->etab_n = n;
    c->etab_invh = (float)(1.0 / h);
    return NB_OK;
}

// The smooth part of the Ewald real-space force factor, G(r) = erf(beta r)/r^3 -
// 2 beta/sqrt(pi) exp(-beta^2 r^2)/r^2 (the force factor is 1/r^3 - G(r)), and its derivative,
// in FP64: from the power series in x = beta r below x = 1 (the closed form cancels there),
// G = beta^3 S(x), S(x) = 2/sqrt(pi) sum_{n>=1} (-1)^(n+1) 2n x^(2n-2) / (n! (2n+1)).
void ewald_fcorr(double beta, double r, double *g, double *dg) {
    const double x = beta * r, k = 2.0 / sqrt(M_PI);
    if (x < 1.0) {
        double s = 0.0, ds = 0.0, fact = 1.0, xp = 1.0, xq = x;   // xp = x^(2n-2), xq = x^(2n-3)
        for (int n = 1; n <= 24; ++n) {
            fact *= n;
            const double sg = (n % 2) ? 1.0 : -1.0;
            s += sg * 2.0 * n * xp / (fact * (2.0 * n + 1.0));
            if (n >= 2) {
                ds += sg * 2.0 * n * (2.0 * n - 2.0) * xq / (fact * (2.0 * n + 1.0));
                xq *= x * x;
            }
            xp *= x * x;
        }
        *g = k * s * beta * beta * beta;
        *dg = k * ds * beta * beta * beta * beta;
    } else {
        const double ex = exp(-x * x), er = erf(x);
        const double r2 = r * r, r3 = r2 * r;
        *g = er / r3 - beta * k * ex / r2;
        *dg = beta * k * ex * (3.0 / r3 + 2.0 * beta * beta / r) - 3.0 * er / (r3 * r);
    }
}

// FP32 cubic Hermite segments of G on [k h, (k+1) h], h = rc / NB_TAB_SEGMENTS: (c0, c1, c2, c3)
// with G(r) ~ c0 + c1 u + c2 u^2 + c3 u^3, u = r / h - k.
int upload_ftab(nb_ctx *c) {
    const int n = NB_TAB_SEGMENTS;
    const double h = c->rc / n;
    std::vector<float4> seg(n);
    for (int k = 0; k < n; ++k) {
        double g0, d0, g1, d1;
        ewald_fcorr(c->beta, k * h, &g0, &d0);
        ewald_fcorr(c->beta, (k + 1) * h, &g1, &d1);
        d0 *= h;
        d1 *= h;
        seg[k] = make_float4((float)g0, (float)d0, (float)(3.0 * (g1 - g0) - 2.0 * d0 - d1),
                             (float)(2.0 * (g0 - g1) + d0 + d1));
    }
    int r = dalloc(c, &c->ftab, seg.size(), "tabulated Ewald force");
    if (r != NB_OK) return r;
    hipError_t e = hipMemcpy(c->ftab, seg.data(), sizeof(float4) * seg.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(c, e, "upload tabulated Ewald force");
    c->fp.tinvh = (float)(n / c->rc);
    return NB_OK;
}

int alloc_list(nb_ctx *c) {
    return dalloc(c, &c->jl, (size_t)c->ncl_max * c->cap, "pair list");
}

int upload_lj(nb_ctx *c) {
    std::vector<float4> tab;
    lj_table(c, tab);
    hipError_t e = hipMemcpyAsync(c->ljtab, tab.data(), sizeof(float4) * tab.size(),
                                  hipMemcpyHostToDevice, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "upload LJ table");
    // the host vector dies here: wait for the copy
    e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "upload LJ table");
    return NB_OK;
}

// An event of the kernel-timing pairs: without the system-scope fence that a default event adds
// when it is recorded (a cache write-back and invalidation that would slow the timed kernel);
// the events are only read for their time stamps.
hipError_t nb_timing_event(hipEvent_t *e) { return hipEventCreateWithFlags(e, hipEventDisableSystemFence); }

// Sum the recorded event pairs into timed_ms (synchronises on the last stop event).
int drain_events(nb_ctx *c) {
    for (size_t k = 0; k < c->ev_used; ++k) {
        hipError_t e = hipEventSynchronize(c->ev[2 * k + 1]);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, c->ev[2 * k], c->ev[2 * k + 1]);
        if (e != hipSuccess) return hip_fail(c, e, "kernel timing");
        c->timed_ms += ms;
        c->timed_n += 1;
    }
    c->ev_used = 0;
    return NB_OK;
}

int read_meta(nb_ctx *c, nb_meta *m) {
    hipError_t e = hipMemcpyAsync(m, c->meta, sizeof(nb_meta), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "read device status");
    return NB_OK;
}

void free_all(nb_ctx *c) {
    void *bufs[] = {c->off,   c->xbuild, c->col,    c->rank,  c->tmp,       c->slot_of,
                    c->colcount, c->colstart, c->colcl, c->perm, c->xs,     c->xq,
                    c->tsort, c->units,  c->fj,     c->bblo,  c->bbhi,      c->icount,
                    c->jl,    c->epart,  c->meta,   c->ljtab, c->excl_off,  c->excl_idx,
                    c->dbg_pairs, c->adj, c->adjj, c->gs, c->tpart, c->etab,
                    c->cpart, c->vpart, c->jl_p, c->icount_p, c->xprune, c->mdpart, c->ftab,
                    c->colz};
    for (void *p : bufs)
        if (p) hipFree(p);
}

}  // namespace

int nb_read_meta(nb_ctx *c, nb_meta *m) { return read_meta(c, m); }

int nb_list_entries(nb_ctx *c, int nclusters, int64_t *total) {
    *total = 0;
    if (!c->have_list || nclusters <= 0) return NB_OK;
    std::vector<int> cnt(nclusters);
    hipError_t e = hipMemcpy(cnt.data(), c->icount, sizeof(int) * nclusters, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(c, e, "read list lengths");
    for (int v : cnt) *total += v;
    return NB_OK;
}

int nb_regrow_list(nb_ctx *c, int maxcount) {
    c->cap = ((maxcount + maxcount / 8 + 32) + 31) & ~31;
    return alloc_list(c);
}

extern "C" {

int nb_validate_params(const nb_params *p) {
    if (!p) return fail(nullptr, NB_ERR_ARG, "params is NULL");
    for (int k = 0; k < 3; ++k)
        if (!finite_pos(p->box[k])) return fail(nullptr, NB_ERR_ARG, "box edges must be finite and > 0");
    if (!finite_pos(p->cutoff)) return fail(nullptr, NB_ERR_ARG, "cutoff must be finite and > 0");
    if (!(isfinite(p->buffer) && p->buffer >= 0.0)) return fail(nullptr, NB_ERR_ARG, "buffer must be finite and >= 0");
    if (!(isfinite(p->ewald_beta) && p->ewald_beta >= 0.0)) return fail(nullptr, NB_ERR_ARG, "ewald_beta must be finite and >= 0");
    if (p->ewald_beta * p->cutoff > NB_ERFCX_XMAX)
        return fail(nullptr, NB_ERR_ARG, "ewald_beta * cutoff exceeds the range of the erfc fit (4)");
    if (!finite_pos(p->coulomb_const)) return fail(nullptr, NB_ERR_ARG, "coulomb_const must be finite and > 0");
    if (p->ntypes < 1 || p->ntypes > NB_MAX_TYPES) return fail(nullptr, NB_ERR_ARG, "ntypes must be in 1..32");
    if (!p->sigma || !p->epsilon) return fail(nullptr, NB_ERR_ARG, "sigma/epsilon are NULL");
    for (int t = 0; t < p->ntypes; ++t)
        if (!(isfinite(p->sigma[t]) && p->sigma[t] >= 0.0 && isfinite(p->epsilon[t]) && p->epsilon[t] >= 0.0))
            return fail(nullptr, NB_ERR_ARG, "sigma/epsilon must be finite and >= 0");
    if (p->natoms < 1 || p->natoms > (1 << 27)) return fail(nullptr, NB_ERR_ARG, "natoms must be in 1..2^27");
    if (p->cluster != 0 && p->cluster != 4 && p->cluster != 8) return fail(nullptr, NB_ERR_ARG, "cluster must be 0, 4 or 8");
    if (p->flags & ~(NB_CHECK_STALE | NB_CHECK_FINITE | NB_ASYNC_BUILD | NB_ENERGY_FP64 | NB_EWALD_CORR |
                     NB_SORT_UNITS))
        return fail(nullptr, NB_ERR_ARG, "unknown flag bits");
    if ((p->flags & NB_EWALD_CORR) && p->elec == NB_ELEC_RF)
        return fail(nullptr, NB_ERR_ARG, "NB_EWALD_CORR needs Ewald electrostatics");
    if (p->elec != NB_ELEC_EWALD && p->elec != NB_ELEC_RF && p->elec != NB_ELEC_EWALD_TAB)
        return fail(nullptr, NB_ERR_ARG, "elec must be NB_ELEC_EWALD, NB_ELEC_EWALD_TAB or NB_ELEC_RF");
    if (p->vdw != NB_VDW_SHIFT && p->vdw != NB_VDW_FSWITCH) return fail(nullptr, NB_ERR_ARG, "vdw must be NB_VDW_SHIFT or NB_VDW_FSWITCH");
    if (p->elec == NB_ELEC_RF && !(isfinite(p->epsilon_rf) && (p->epsilon_rf == 0.0 || p->epsilon_rf >= 1.0)))
        return fail(nullptr, NB_ERR_ARG, "epsilon_rf must be 0 (infinity) or >= 1");
    if (p->vdw == NB_VDW_FSWITCH && !(isfinite(p->rswitch) && p->rswitch >= 0.0 && p->rswitch < p->cutoff))
        return fail(nullptr, NB_ERR_ARG, "rswitch must be in [0, cutoff)");
    if (p->excl_off) {
        if (p->excl_off[0] != 0) return fail(nullptr, NB_ERR_ARG, "excl_off[0] must be 0");
        for (int i = 0; i < p->natoms; ++i)
            if (p->excl_off[i + 1] < p->excl_off[i]) return fail(nullptr, NB_ERR_ARG, "excl_off must be non-decreasing");
        for (int i = 0; i < p->natoms; ++i)
            if (p->excl_off[i + 1] - p->excl_off[i] > NB_MAX_EXCL_PER_ATOM)
                return fail(nullptr, NB_ERR_ARG, "an atom has more than 32 excluded partners");
        int nnz = p->excl_off[p->natoms];
        if (nnz > 0 && !p->excl_idx) return fail(nullptr, NB_ERR_ARG, "excl_idx is NULL");
        for (int k = 0; k < nnz; ++k)
            if (p->excl_idx[k] < 0 || p->excl_idx[k] >= p->natoms) return fail(nullptr, NB_ERR_ARG, "exclusion index out of range");
    }
    double mn = std::min(p->box[0], std::min(p->box[1], p->box[2]));
    if (!(p->cutoff < 0.5 * mn)) return fail(nullptr, NB_ERR_CUTOFF, "cutoff must be below half the smallest box edge");
    if (!(p->cutoff + p->buffer < mn)) return fail(nullptr, NB_ERR_CUTOFF, "cutoff + buffer must be below the smallest box edge");
    if (!(p->cutoff + p->buffer < NB_PAD_SPACING))
        return fail(nullptr, NB_ERR_CUTOFF, "cutoff + buffer must be below 16 nm (the spacing of padding slots)");
    return NB_OK;
}

int nb_setup(nb_ctx **out, const nb_params *p, void *stream) {
    if (!out) return fail(nullptr, NB_ERR_ARG, "out is NULL");
    *out = nullptr;
    int rc = nb_validate_params(p);
    if (rc != NB_OK) return rc;
    nb_ctx *c = new nb_ctx();
    c->stream = (hipStream_t)stream;
    hipGetDevice(&c->device);
    {
        // device address of the static work area of nb_backward_noalloc on this device
        const hipError_t e = nb_noalloc_init(c->device);
        if (e != hipSuccess) {
            g_setup_error = std::string("static work area lookup: ") + hipGetErrorString(e);
            delete c;
            return NB_ERR_HIP;
        }
    }
    c->natoms = p->natoms;
    c->ntypes = p->ntypes;
    c->C = p->cluster == 0 ? 8 : p->cluster;
    for (int k = 0; k < 3; ++k) c->box[k] = p->box[k];
    c->rc = p->cutoff;
    c->rb = p->buffer;
    c->beta = p->ewald_beta;
    c->elec = p->elec;
    c->vdw = p->vdw;
    c->eps_rf = p->epsilon_rf;
    c->rsw = p->rswitch;
    c->fc = p->coulomb_const;
    c->flags = p->flags;
    c->sigma.assign(p->sigma, p->sigma + p->ntypes);
    c->epsilon.assign(p->epsilon, p->epsilon + p->ntypes);

    // column grid: square-ish columns of width (C / rho)^(1/3), at least 1 per axis
    const double rho = p->natoms / (p->box[0] * p->box[1] * p->box[2]);
    const double w = cbrt(c->C / rho);
    int ncx = std::max(1, (int)floor(p->box[0] / w + 0.5));
    int ncy = std::max(1, (int)floor(p->box[1] / w + 0.5));
    while ((double)p->natoms / ((double)ncx * ncy) > 0.5 * NB_SORT_MAX) {
        ncx *= 2;
        ncy *= 2;
    }
    nb_geom &g = c->geom;
    for (int k = 0; k < 3; ++k) g.L[k] = (float)p->box[k];
    g.ncx = ncx;
    g.ncy = ncy;
    g.ncol = ncx * ncy;
    g.w[0] = (float)(p->box[0] / ncx);
    g.w[1] = (float)(p->box[1] / ncy);
    g.invw[0] = (float)(ncx / p->box[0]);
    g.invw[1] = (float)(ncy / p->box[1]);
    const double rlist = p->cutoff + p->buffer;
    g.rl = (float)rlist;
    {
        // z bins of half a column width: a cluster window of the search is at most a bin or two
        // wider on each side than the clusters it has to hold
        const double dz = 0.5 * w;
        g.nz = std::max(1, (int)ceil(p->box[2] / dz));
        g.zinv = (float)(g.nz / p->box[2]);
    }
    g.rl2 = (float)(rlist * rlist);
    set_constants(c);

    c->npad_max = p->natoms + g.ncol * (c->C - 1);
    c->ncl_max = c->npad_max / c->C + 1;
    c->npad_max = c->ncl_max * c->C;
    {
        int ncu = 0;
        if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, c->device) != hipSuccess || ncu <= 0)
            ncu = 256;
        c->slots = ncu * 4;  // SIMDs
        // the last units of the force kernel run while the device drains: halving the lists of
        // the last three clusters per SIMD (two with FP64 pair energies, whose workgroups load an
        // erfc table each) shortens that tail
        c->tail_n = (nb_energy_fp64(c) ? 2 : 3) * c->slots;
        if (const char *ts = getenv("NB_TAIL_CLUSTERS")) c->tail_n = std::max(0, atoi(ts));
        c->unit_cap = c->ncl_max + std::min(c->tail_n, c->ncl_max) + 2 * c->slots + 64;
    }
    c->cap = estimate_cap(p->natoms, p->box, c->C, rlist);
    if (const char *ov = getenv("NB_LIST_CAP")) {
        // initial j-entries per i-cluster; the list still grows on overflow
        int v = atoi(ov);
        if (v > 0) c->cap = v;
    }
    const int n = p->natoms;
    int r = NB_OK;
#define NB_ALLOC(ptr, cnt) \
    if ((r = dalloc(c, &c->ptr, (size_t)(cnt), #ptr)) != NB_OK) goto fail_out;
    NB_ALLOC(off, n);
    NB_ALLOC(xbuild, 3 * (size_t)n);
    NB_ALLOC(col, n);
    NB_ALLOC(rank, n);
    NB_ALLOC(tmp, n);
    NB_ALLOC(slot_of, n);
    NB_ALLOC(colcount, g.ncol);
    NB_ALLOC(colstart, g.ncol + 1);
    NB_ALLOC(colcl, g.ncol + 1);
    NB_ALLOC(colz, (size_t)g.ncol * (g.nz + 1));
    NB_ALLOC(perm, c->npad_max);
    NB_ALLOC(xs, c->npad_max);
    // one j-group more than the slots: the far group that lanes past the end of a j-list read
    NB_ALLOC(xq, c->npad_max + NB_JG);
    NB_ALLOC(tsort, c->npad_max + NB_JG);

    NB_ALLOC(fj, 3 * (size_t)c->npad_max);
    NB_ALLOC(bblo, c->ncl_max);
    NB_ALLOC(bbhi, c->ncl_max);
    NB_ALLOC(icount, c->ncl_max);
    NB_ALLOC(units, c->unit_cap);
    NB_ALLOC(epart, 4 * (size_t)c->unit_cap);
    if (c->flags & NB_EWALD_CORR) NB_ALLOC(cpart, NB_CORR_PART * (size_t)((n + NB_CORR_BLOCK - 1) / NB_CORR_BLOCK));
    NB_ALLOC(vpart, 6 * (size_t)((c->unit_cap + 3) / 4));
    NB_ALLOC(meta, 1);
    NB_ALLOC(ljtab, 2 * (size_t)c->ntypes * c->ntypes);
#undef NB_ALLOC
    {
        // the far j-group (slots npad_max ..): far outside any box, type 0; no kernel writes it
        const float4 far[NB_JG] = {nb_pad_coord(c->npad_max), nb_pad_coord(c->npad_max + 1),
                                   nb_pad_coord(c->npad_max + 2), nb_pad_coord(c->npad_max + 3)};
        const int zero[NB_JG] = {0, 0, 0, 0};
        if (hipMemcpy(c->xq + c->npad_max, far, sizeof(far), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(c->tsort + c->npad_max, zero, sizeof(zero), hipMemcpyHostToDevice) != hipSuccess) {
            r = fail(c, NB_ERR_HIP, "nb_setup: initialising the far j-group failed");
            goto fail_out;
        }
    }
    if ((r = alloc_list(c)) != NB_OK) goto fail_out;
    if (p->excl_off) {
        int nnz = p->excl_off[n];
        if ((r = dalloc(c, &c->excl_off, (size_t)n + 1, "excl_off")) != NB_OK) goto fail_out;
        if ((r = dalloc(c, &c->excl_idx, (size_t)std::max(nnz, 1), "excl_idx")) != NB_OK) goto fail_out;
        c->nnz_excl = nnz;
        hipError_t e = hipMemcpy(c->excl_off, p->excl_off, sizeof(int) * (n + 1), hipMemcpyHostToDevice);
        if (e == hipSuccess && nnz > 0)
            e = hipMemcpy(c->excl_idx, p->excl_idx, sizeof(int) * nnz, hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            r = hip_fail(c, e, "upload exclusions");
            goto fail_out;
        }
    }
    // the fixed-point force sums start at zero and are left at zero by every complete force call
    if (hipMemset(c->meta, 0, sizeof(nb_meta)) != hipSuccess ||
        hipMemset(c->slot_of, 0, sizeof(int) * n) != hipSuccess ||
        hipMemset(c->fj, 0, sizeof(float) * 3 * (size_t)c->npad_max) != hipSuccess) {
        r = fail(c, NB_ERR_HIP, "hipMemset meta");
        goto fail_out;
    }
    if ((r = upload_lj(c)) != NB_OK) goto fail_out;
    if ((r = upload_etab(c)) != NB_OK) goto fail_out;
    if (c->elec == NB_ELEC_EWALD_TAB && (r = upload_ftab(c)) != NB_OK) goto fail_out;
    if (c->flags & NB_ASYNC_BUILD) {
        if (hipHostMalloc((void **)&c->host_meta, sizeof(nb_meta), hipHostMallocDefault) != hipSuccess) {
            c->host_meta = nullptr;
            r = fail(c, NB_ERR_OOM, "pinned status block");
            goto fail_out;
        }
        if (hipEventCreateWithFlags(&c->build_ev, hipEventDisableTiming) != hipSuccess) {
            c->build_ev = nullptr;
            r = fail(c, NB_ERR_HIP, "hipEventCreate");
            goto fail_out;
        }
    }
    *out = c;
    return NB_OK;
fail_out:
    g_setup_error = c->err;
    if (c->host_meta) hipHostFree(c->host_meta);
    free_all(c);
    delete c;
    return r;
}

int nb_set_lj(nb_ctx *c, const double *sigma, const double *epsilon) {
    if (!c || !sigma || !epsilon) return fail(c, NB_ERR_ARG, "NULL argument");
    for (int t = 0; t < c->ntypes; ++t)
        if (!(isfinite(sigma[t]) && sigma[t] >= 0.0 && isfinite(epsilon[t]) && epsilon[t] >= 0.0))
            return fail(c, NB_ERR_ARG, "sigma/epsilon must be finite and >= 0");
    c->sigma.assign(sigma, sigma + c->ntypes);
    c->epsilon.assign(epsilon, epsilon + c->ntypes);
    hipSetDevice(c->device);
    return upload_lj(c);
}

int nb_set_stream(nb_ctx *c, void *stream) {
    if (!c) return fail(c, NB_ERR_ARG, "NULL context");
    c->stream = (hipStream_t)stream;
    return NB_OK;
}

int nb_pairlist(nb_ctx *c, const float *x) {
    if (!c || !x) return fail(c, NB_ERR_ARG, "NULL argument");
    hipSetDevice(c->device);
    c->have_list = false;
    if (c->pruned) {   // the build writes the full list
        std::swap(c->jl, c->jl_p);
        std::swap(c->icount, c->icount_p);
        c->pruned = false;
    }
    auto t0 = std::chrono::steady_clock::now();
    // NB_ASYNC_BUILD: the status of the previous build was copied to pinned memory behind it
    // on the stream; that copy finished long before the force calls queued after the build,
    // so waiting for its event does not drain the stream
    bool prev_overflow = false;
    if (c->pending_overflow_check) {
        c->pending_overflow_check = false;
        hipError_t e = hipEventSynchronize(c->build_ev);
        if (e != hipSuccess) return hip_fail(c, e, "wait for the previous build's status");
        const nb_meta m = *c->host_meta;
        if (m.flags & NB_F_COLUMN)
            return fail(c, NB_ERR_OVERFLOW, "a grid column or the exclusions of one cluster exceed the build kernels' capacity");
        if (m.flags & NB_F_BUILD_NONFINITE) return fail(c, NB_ERR_NONFINITE, "non-finite coordinates at the previous build");
        if (m.flags & NB_F_OVERFLOW) {
            prev_overflow = true;
            // force calls queued after that build still read the old list
            e = hipStreamSynchronize(c->stream);
            if (e != hipSuccess) return hip_fail(c, e, "drain the stream before regrowing");
            c->cap = ((m.maxcount + m.maxcount / 8 + 32) + 31) & ~31;
            int r = alloc_list(c);
            if (r != NB_OK) return r;
        }
    }
    const bool async = (c->flags & NB_ASYNC_BUILD) && c->built_once && !prev_overflow;
    for (int attempt = 0; attempt < 4; ++attempt) {
        hipError_t e = nb_launch_build(c, x);
        if (e != hipSuccess) return hip_fail(c, e, "pair-list build launch");
        if (async) {
            e = hipMemcpyAsync(c->host_meta, c->meta, sizeof(nb_meta), hipMemcpyDeviceToHost, c->stream);
            if (e == hipSuccess) e = hipEventRecord(c->build_ev, c->stream);
            if (e != hipSuccess) return hip_fail(c, e, "queue the build status copy");
            c->have_list = true;
            c->pending_overflow_check = true;
            return NB_OK;
        }
        nb_meta m;
        int r = read_meta(c, &m);
        if (r != NB_OK) return r;
        if (m.flags & NB_F_COLUMN)
            return fail(c, NB_ERR_OVERFLOW, "a grid column or the exclusions of one cluster exceed the build kernels' capacity");
        if (m.flags & NB_F_BUILD_NONFINITE) return fail(c, NB_ERR_NONFINITE, "non-finite coordinates");
        if (m.flags & NB_F_OVERFLOW) {
            c->cap = ((m.maxcount + m.maxcount / 8 + 32) + 31) & ~31;
            if ((r = alloc_list(c)) != NB_OK) return r;
            continue;
        }
        c->have_list = true;
        c->built_once = true;
        c->build_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        if (prev_overflow)
            return fail(c, NB_ERR_OVERFLOW, "the previous pair list overflowed (forces computed with it "
                                            "missed pairs); the list was regrown and this one is complete");
        return NB_OK;
    }
    return fail(c, NB_ERR_OVERFLOW, "pair list still overflowing after regrowing");
}

int nb_prune(nb_ctx *c, const float *x, double r_inner) {
    if (!c || !x) return fail(c, NB_ERR_ARG, "NULL argument");
    if (!(std::isfinite(r_inner) && r_inner >= c->rc && r_inner <= c->rc + c->rb * (1.0 + 1e-12)))
        return fail(c, NB_ERR_ARG, "r_inner must be in [rc, rc + buffer]");
    if (!c->have_list) return fail(c, NB_ERR_STATE, "nb_prune called before nb_pairlist");
    hipSetDevice(c->device);
    int r;
    if (!c->pruned && c->jl_p_cap != c->cap) {   // room for the pruned list (the list may have grown)
        if ((r = dalloc(c, &c->jl_p, (size_t)c->ncl_max * c->cap, "pruned pair list")) != NB_OK) return r;
        c->jl_p_cap = c->cap;
    }
    if (!c->icount_p && (r = dalloc(c, &c->icount_p, (size_t)c->ncl_max, "pruned list lengths")) != NB_OK)
        return r;
    if ((c->flags & NB_CHECK_STALE) && !c->xprune &&
        (r = dalloc(c, &c->xprune, 3 * (size_t)c->natoms, "prune positions")) != NB_OK)
        return r;
    // positions in cluster order, as the force calls form them (charges and types are packed
    // again by the next force call)
    hipError_t e = nb_launch_pack(c, x, nullptr, nullptr);
    if (e != hipSuccess) return hip_fail(c, e, "prune: pack launch");
    // the full list is jl / icount before the first prune after a build, jl_p / icount_p after it
    const float rin = (float)r_inner;
    e = c->pruned ? nb_launch_prune(c, rin * rin, c->icount_p, c->jl_p, c->icount, c->jl)
                  : nb_launch_prune(c, rin * rin, c->icount, c->jl, c->icount_p, c->jl_p);
    if (e != hipSuccess) return hip_fail(c, e, "prune launch");
    if (!c->pruned) {
        std::swap(c->jl, c->jl_p);
        std::swap(c->icount, c->icount_p);
        c->pruned = true;
    }
    if (c->flags & NB_CHECK_STALE) {
        e = hipMemcpyAsync(c->xprune, x, sizeof(float) * 3 * (size_t)c->natoms, hipMemcpyDeviceToDevice, c->stream);
        if (e != hipSuccess) return hip_fail(c, e, "save prune positions");
        const double h = 0.5 * (r_inner - c->rc);
        c->stale2_prune = (float)(h * h);
    }
    return NB_OK;
}

static int forces_impl(nb_ctx *c, const float *x, const float *q, const int32_t *type, float *f,
                       double *e, double *vir) {
    if (!c || !x || !q || !type || !f || !e) return fail(c, NB_ERR_ARG, "NULL argument");
    if (!c->have_list) return fail(c, NB_ERR_STATE, "nb_forces called before nb_pairlist");
    hipError_t err = hipSuccess;
    const bool stamp = c->timing && (c->timing_count++ % c->timing_every) == 0;
    // a call that failed between its force kernel and its finalize may have left sums behind
    if (!c->fj_clean) err = hipMemsetAsync(c->fj, 0, sizeof(float) * 3 * (size_t)c->npad_max, c->stream);
    if (err == hipSuccess) err = nb_launch_pack(c, x, q, type);
    if (err == hipSuccess && c->pruned && (c->flags & NB_CHECK_STALE)) err = nb_launch_prune_check(c, x);
    c->fj_clean = false;
    if (stamp && err == hipSuccess) {
        const size_t kMaxPairs = 4096;
        if (c->ev_used == kMaxPairs) {
            int r = drain_events(c);
            if (r != NB_OK) return r;
        }
        if (c->ev.size() < 2 * (c->ev_used + 1)) {
            hipEvent_t a, b;
            if (nb_timing_event(&a) != hipSuccess || nb_timing_event(&b) != hipSuccess)
                return fail(c, NB_ERR_HIP, "hipEventCreate");
            c->ev.push_back(a);
            c->ev.push_back(b);
        }
    }
    // with timing on, the kernel's dispatch stamps an event pair with its own start and end
    if (err == hipSuccess)
        err = nb_launch_force(c, vir != nullptr, stamp ? c->ev[2 * c->ev_used] : nullptr,
                              stamp ? c->ev[2 * c->ev_used + 1] : nullptr);
    if (stamp && err == hipSuccess) c->ev_used += 1;
    if (err == hipSuccess && (c->flags & NB_EWALD_CORR)) err = nb_launch_ewald_corr(c, x, q);
    if (err == hipSuccess) err = nb_launch_finalize(c, f, e, vir);
    if (err != hipSuccess) return hip_fail(c, err, "force launch");
    c->fj_clean = true;
    return NB_OK;
}

int nb_forces(nb_ctx *c, const float *x, const float *q, const int32_t *type, float *f, double *e) {
    return forces_impl(c, x, q, type, f, e, nullptr);
}

int nb_forces_virial(nb_ctx *c, const float *x, const float *q, const int32_t *type, float *f,
                     double *e, double *vir) {
    if (!vir) return fail(c, NB_ERR_ARG, "NULL argument");
    return forces_impl(c, x, q, type, f, e, vir);
}

int nb_set_timing(nb_ctx *c, int every) {
    if (!c) return fail(c, NB_ERR_ARG, "NULL context");
    c->timing = every > 0;
    c->timing_every = every > 0 ? every : 1;
    c->timing_count = 0;
    // event pairs for the first 1024 timed launches are created here, so that timed loops do
    // not create events
    hipSetDevice(c->device);
    while (c->timing && c->ev.size() < 2 * 1024) {
        hipEvent_t a, b;
        if (nb_timing_event(&a) != hipSuccess) return fail(c, NB_ERR_HIP, "hipEventCreate");
        if (nb_timing_event(&b) != hipSuccess) {
            hipEventDestroy(a);
            return fail(c, NB_ERR_HIP, "hipEventCreate");
        }
        c->ev.push_back(a);
        c->ev.push_back(b);
    }
    return NB_OK;
}

int nb_get_timing(nb_ctx *c, double *ms, int64_t *n) {
    if (!c || !ms || !n) return fail(c, NB_ERR_ARG, "NULL argument");
    hipSetDevice(c->device);
    int r = drain_events(c);
    if (r != NB_OK) return r;
    *ms = c->timed_ms;
    *n = c->timed_n;
    c->timed_ms = 0;
    c->timed_n = 0;
    return NB_OK;
}

int nb_check(nb_ctx *c) {
    if (!c) return fail(c, NB_ERR_ARG, "NULL context");
    hipSetDevice(c->device);
    nb_meta m;
    int r = read_meta(c, &m);
    if (r != NB_OK) return r;
    uint32_t zero = 0;
    hipError_t e = hipMemcpy(&c->meta->flags, &zero, sizeof(zero), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(c, e, "clear device flags");
    if (m.flags & (NB_F_OVERFLOW | NB_F_COLUMN)) return fail(c, NB_ERR_OVERFLOW, "pair list overflow");
    if (m.flags & (NB_F_NONFINITE | NB_F_BUILD_NONFINITE)) return fail(c, NB_ERR_NONFINITE, "non-finite coordinates");
    if (m.flags & NB_F_STALE) return fail(c, NB_ERR_LIST_STALE, "an atom moved more than buffer/2 since the list was built");
    if (m.flags & NB_F_RANGE)
        return fail(c, NB_ERR_RANGE, "a pair force component exceeded 131072 kJ/mol/nm (or was not finite): "
                                     "net force components beyond 524288 would not be represented");
    return NB_OK;
}

int nb_debug_pairs(nb_ctx *c, const float *x, int64_t *pairs_host, int64_t cap, int64_t *count) {
    if (!c || !x || !count || (cap > 0 && !pairs_host) || cap < 0) return fail(c, NB_ERR_ARG, "bad argument");
    if (!c->have_list) return fail(c, NB_ERR_STATE, "nb_debug_pairs called before nb_pairlist");
    hipSetDevice(c->device);
    int64_t dcap = std::max<int64_t>(cap, 1);
    if (dcap > c->dbg_cap) {
        int r = dalloc(c, &c->dbg_pairs, 2 * (size_t)dcap, "pair export");
        if (r != NB_OK) return r;
        c->dbg_cap = dcap;
    }
    hipError_t e = nb_launch_pack(c, x, nullptr, nullptr);
    if (e == hipSuccess) e = nb_launch_debug_pairs(c, cap);
    if (e != hipSuccess) return hip_fail(c, e, "pair export launch");
    nb_meta m;
    int r = read_meta(c, &m);
    if (r != NB_OK) return r;
    *count = (int64_t)m.npairs_out;
    int64_t ncopy = std::min<int64_t>(cap, *count);
    if (ncopy > 0) {
        e = hipMemcpy(pairs_host, c->dbg_pairs, sizeof(int64_t) * 2 * ncopy, hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_fail(c, e, "copy pairs");
    }
    return NB_OK;
}

int nb_get_stats(nb_ctx *c, nb_stats *st) {
    if (!c || !st) return fail(c, NB_ERR_ARG, "NULL argument");
    hipSetDevice(c->device);
    nb_meta m;
    int r = read_meta(c, &m);
    if (r != NB_OK) return r;
    memset(st, 0, sizeof(*st));
    st->natoms = c->natoms;
    st->nclusters = m.nclusters;
    st->npadded = m.npad;
    if ((r = nb_list_entries(c, m.nclusters, &st->nentries)) != NB_OK) return r;
    st->evaluated_pairs = st->nentries * (int64_t)c->C * NB_JG;
    st->list_capacity = c->cap;
    st->cluster = c->C;
    st->ncolumns = c->geom.ncol;
    st->build_ms_last = c->build_ms;
    st->work_units = m.nunits;
    st->unit_batches = m.split;
    st->max_list_batches = m.maxbatches;
    st->pruned = c->pruned ? 1 : 0;
    for (int k = 0; k < NB_HIST_BINS; ++k) st->list_hist[k] = m.hist[k];
    return NB_OK;
}

const char *nb_last_error(nb_ctx *c) {
    return c ? c->err.c_str() : g_setup_error.c_str();
}

int nb_destroy(nb_ctx *c) {
    if (!c) return NB_OK;
    hipSetDevice(c->device);
    hipStreamSynchronize(c->stream);
    for (hipEvent_t ev : c->ev) hipEventDestroy(ev);
    if (c->build_ev) hipEventDestroy(c->build_ev);
    if (c->host_meta) hipHostFree(c->host_meta);
    free_all(c);
    delete c;
    return NB_OK;
}

int nb_backward(nb_ctx *c, const float *x, const float *q, const int32_t *type, const float *g_f,
                const double *g_e, float *dx, float *dq, double *dsigma, double *deps,
                uint32_t flags) {
    if (!c || !x || !q || !type || !g_f || !g_e || !dx || !dq || !dsigma || !deps)
        return fail(c, NB_ERR_ARG, "NULL argument");
    if (c->elec != NB_ELEC_EWALD || c->vdw != NB_VDW_SHIFT)
        return fail(c, NB_ERR_ARG, "nb_backward supports NB_ELEC_EWALD with NB_VDW_SHIFT only");
    if (c->flags & NB_EWALD_CORR)
        return fail(c, NB_ERR_ARG, "nb_backward does not include the Ewald corrections");
    hipSetDevice(c->device);
    if (!(flags & NB_REUSE_LIST) || !c->have_list) {
        int r = nb_pairlist(c, x);
        if (r != NB_OK) return r;
    }
    hipError_t e = nb_launch_pack(c, x, q, type);
    if (e == hipSuccess) e = nb_launch_adjoint(c, g_f, g_e, dx, dq, dsigma, deps);
    if (e != hipSuccess) return hip_fail(c, e, "adjoint launch");
    return NB_OK;
}

int nb_md_leapfrog(nb_ctx *c, float *x, float *v, const float *q, const int32_t *type,
                   const float *inv_mass, double dt, int32_t nsteps, int32_t nstlist,
                   double r_inner, int32_t nstprune, float *f, double *e_steps) {
    if (!c || !x || !v || !q || !type || !inv_mass || !f || !e_steps)
        return fail(c, NB_ERR_ARG, "NULL argument");
    if (!(std::isfinite(dt) && dt > 0.0) || nsteps < 0 || nstlist < 1)
        return fail(c, NB_ERR_ARG, "dt must be positive and finite, nsteps >= 0, nstlist >= 1");
    if (r_inner != 0.0 && !(nstprune >= 1 && std::isfinite(r_inner) && r_inner >= c->rc &&
                            r_inner <= c->rc + c->rb * (1.0 + 1e-12)))
        return fail(c, NB_ERR_ARG, "rolling prune: r_inner in [rc, rc + buffer] and nstprune >= 1, or r_inner = 0");
    if (c->flags & NB_EWALD_CORR) return fail(c, NB_ERR_ARG, "nb_md_leapfrog does not take NB_EWALD_CORR");
    hipSetDevice(c->device);
    for (int step = 0; step < nsteps; ++step) {
        int r;
        const int since = step % nstlist;
        if (since == 0) {
            if ((r = nb_pairlist(c, x)) != NB_OK) return r;
        } else if (r_inner != 0.0 && since % nstprune == 0) {
            if ((r = nb_prune(c, x, r_inner)) != NB_OK) return r;
        }
        double *e = e_steps + 4 * (size_t)step;
        if ((r = nb_forces(c, x, q, type, f, e)) != NB_OK) return r;
        hipError_t err = nb_launch_md_update(c, (float)dt, f, inv_mass, x, v, e);
        if (err != hipSuccess) return hip_fail(c, err, "leapfrog update");
    }
    return NB_OK;
}

int nb_backward_noalloc(nb_ctx *c, const float *x, const float *q, const int32_t *type,
                        const float *g_f, const double *g_e, float *dx, float *dq, double *dsigma,
                        double *deps) {
    if (!c || !x || !q || !type || !g_f || !g_e || !dx || !dq || !dsigma || !deps)
        return fail(c, NB_ERR_ARG, "NULL argument");
    if (c->elec != NB_ELEC_EWALD || c->vdw != NB_VDW_SHIFT)
        return fail(c, NB_ERR_ARG, "nb_backward_noalloc supports NB_ELEC_EWALD with NB_VDW_SHIFT only");
    if (c->flags & NB_EWALD_CORR)
        return fail(c, NB_ERR_ARG, "nb_backward_noalloc does not include the Ewald corrections");
    if (c->npad_max > NB_NOALLOC_MAX_SLOTS)
        return fail(c, NB_ERR_ARG, "nb_backward_noalloc: the system needs " + std::to_string(c->npad_max) +
                                       " padded slots, above the static work area's " +
                                       std::to_string(NB_NOALLOC_MAX_SLOTS));
    if (!c->have_list) return fail(c, NB_ERR_STATE, "nb_backward_noalloc needs a pair list (nb_pairlist)");
    hipSetDevice(c->device);
    hipError_t e = nb_launch_pack(c, x, q, type);
    if (e == hipSuccess) e = nb_launch_adjoint_noalloc(c, g_f, g_e, dx, dq, dsigma, deps);
    if (e != hipSuccess) return hip_fail(c, e, "allocation-free adjoint launch");
    return NB_OK;
}

}  // extern "C"
