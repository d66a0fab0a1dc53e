"""ctypes binding of the FP64 oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the CPU-baseline leg of
bench.py.  The product path (paper_2405_01420_amd) never imports this module, and this module
never imports the product.  Inputs are numpy arrays of an ``Instance`` from the shared seeded
generator; every FP32 input is widened exactly to FP64 before the oracle sees it.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SRC_PATH = os.path.join(HERE, "oracle.c")

_lib = None


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc (IEEE FP64, no contraction, OpenMP)."""
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC_PATH):
        tmp = LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
                               "-fno-fast-math", "-std=c99", "-o", tmp, SRC_PATH, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        i32p = ctypes.POINTER(ctypes.c_int32)
        c_i, c_d, c_i64 = ctypes.c_int, ctypes.c_double, ctypes.c_int64
        L.oracle_set_threads.argtypes = [c_i]
        L.oracle_get_threads.restype = c_i
        L.oracle_lj_table.argtypes = [c_i, dp, dp, c_i, dp, dp]
        fsig = [c_i, dp, dp, ip, c_i, dp, dp, dp, c_d, c_d, c_d, ip, ip, dp, dp, dp, dp]
        L.oracle_forces.argtypes = fsig
        L.oracle_forces_cells.argtypes = fsig
        L.oracle_forces.restype = L.oracle_forces_cells.restype = c_i
        L.oracle_forces_subset.argtypes = [c_i, dp, dp, ip, c_i, dp, dp, dp, c_d, c_d, c_d, ip, ip,
                                           c_i, ip, dp, dp, dp]
        L.oracle_pairs.argtypes = [c_i, dp, dp, c_d, ip, ip, c_i64, i32p, i32p, dp]
        L.oracle_pairs.restype = c_i64
        L.oracle_vjp.argtypes = [c_i, dp, dp, ip, c_i, dp, dp, dp, c_d, c_d, c_d, ip, ip, dp, dp,
                                 dp, dp, dp, dp]
        L.oracle_vjp.restype = c_i
        L.oracle_set_flavor.argtypes = [c_i, c_i, c_d, c_d]
        L.oracle_ewald_corrections.argtypes = [c_i, dp, dp, dp, c_d, c_d, ip, ip, dp, dp]
        L.oracle_ewald_corrections.restype = c_i
        _lib = L
    return _lib


def set_threads(n: int) -> None:
    lib().oracle_set_threads(int(n))


def get_threads() -> int:
    return int(lib().oracle_get_threads())


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _i(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def lj_table(sigma, epsilon, round32: bool = True):
    """Lorentz-Berthelot C6, C12 tables [nt, nt] in FP64 (optionally rounded once to FP32)."""
    s, sp = _d(sigma)
    e, ep = _d(epsilon)
    nt = len(s)
    c6, c6p = _d(np.zeros(nt * nt))
    c12, c12p = _d(np.zeros(nt * nt))
    lib().oracle_lj_table(nt, sp, ep, int(round32), c6p, c12p)
    return c6.reshape(nt, nt), c12.reshape(nt, nt)


class Result:
    """Forces [N,3] and energies from the oracle.

    e_lj, e_coul: potential-shifted energies; e_coul_unshifted: without the Coulomb shift;
    abs_lj, abs_coul: sums of |pair energy| (conditioning); npairs: interacting pairs;
    qq_sum: sum of q_i q_j over interacting pairs; eatom_*: per-atom halves of pair energies;
    virial: -1/2 sum over interacting pairs of d (x) F_ij (3 x 3)."""

    def __init__(self, f, out, eatom_lj, eatom_c):
        self.f = f
        self.e_lj, self.e_coul, self.e_coul_unshifted = out[0], out[1], out[2]
        self.abs_lj, self.abs_coul = out[3], out[4]
        self.npairs = int(round(out[5]))
        self.qq_sum = out[6]
        v = out[7:13]
        self.virial = np.array([[v[0], v[3], v[4]], [v[3], v[1], v[5]], [v[4], v[5], v[2]]])
        self.eatom_lj, self.eatom_c = eatom_lj, eatom_c


def _common(x, q, typ, sigma, epsilon, box, c6c12=None, round32=True):
    n = len(q)
    if c6c12 is None:
        c6, c12 = lj_table(sigma, epsilon, round32)
    else:
        c6, c12 = c6c12
    bx = np.array([box] * 3 if np.isscalar(box) else box, dtype=np.float64)
    return n, c6, c12, bx


class _flavor:
    """Sets the oracle's interaction flavour for the duration of one call (Ewald real space
    with LJ potential shift is the default state)."""

    def __init__(self, elec: int, vdw: int, epsilon_rf: float, rswitch: float):
        self.args = (int(elec), int(vdw), float(epsilon_rf), float(rswitch))

    def __enter__(self):
        lib().oracle_set_flavor(*self.args)

    def __exit__(self, *exc):
        lib().oracle_set_flavor(0, 0, 0.0, 0.0)
        return False


def forces(x, q, typ, sigma, epsilon, box, rc, beta, fc, excl_off=None, excl_idx=None,
           cells: bool = False, round32: bool = True, c6c12=None, elec: int = 0, vdw: int = 0,
           epsilon_rf: float = 0.0, rswitch: float = 0.0) -> Result:
    """elec: 0 Ewald real space, 1 reaction field (epsilon_rf, 0 = infinity); vdw: 0 potential
    shift, 1 force switch from rswitch."""
    n, c6, c12, bx = _common(x, q, typ, sigma, epsilon, box, c6c12, round32)
    xa, xp = _d(np.asarray(x, dtype=np.float64).reshape(-1))
    qa, qp = _d(q)
    ta, tp = _i(typ)
    c6a, c6p = _d(c6.reshape(-1))
    c12a, c12p = _d(c12.reshape(-1))
    ba, bp = _d(bx)
    if excl_off is not None:
        oa, op = _i(excl_off)
        ia, ipp = _i(excl_idx if len(excl_idx) else np.zeros(1, np.int32))
    else:
        op = ipp = None
    f, fp = _d(np.zeros(3 * n))
    el, elp = _d(np.zeros(n))
    ec, ecp = _d(np.zeros(n))
    out, outp = _d(np.zeros(16))
    fn = lib().oracle_forces_cells if cells else lib().oracle_forces
    with _flavor(elec, vdw, epsilon_rf, rswitch):
        rc_ = fn(n, xp, qp, tp, len(c6), c6p, c12p, bp, float(rc), float(beta), float(fc), op, ipp,
                 fp, elp, ecp, outp)
    if rc_ != 0:
        raise RuntimeError("oracle_forces failed")
    return Result(f.reshape(n, 3), out, el, ec)


def forces_subset(x, q, typ, sigma, epsilon, box, rc, beta, fc, excl_off, excl_idx, subset,
                  round32: bool = True):
    """Rows `subset` of the oracle's forces [len(subset), 3] and of its per-atom energy halves
    (eatom_lj, eatom_c), from visits restricted to those atoms."""
    n, c6, c12, bx = _common(x, q, typ, sigma, epsilon, box, None, round32)
    xa, xp = _d(np.asarray(x, dtype=np.float64).reshape(-1))
    qa, qp = _d(q)
    ta, tp = _i(typ)
    c6a, c6p = _d(c6.reshape(-1))
    c12a, c12p = _d(c12.reshape(-1))
    ba, bp = _d(bx)
    if excl_off is not None:
        oa, op = _i(excl_off)
        ia, ipp = _i(excl_idx if len(excl_idx) else np.zeros(1, np.int32))
    else:
        op = ipp = None
    sa, sp = _i(subset)
    fs, fsp = _d(np.zeros(3 * len(sa)))
    el, elp = _d(np.zeros(len(sa)))
    ec, ecp = _d(np.zeros(len(sa)))
    lib().oracle_forces_subset(n, xp, qp, tp, len(c6), c6p, c12p, bp, float(rc), float(beta),
                               float(fc), op, ipp, len(sa), sp, fsp, elp, ecp)
    return fs.reshape(-1, 3), el, ec


def pairs(x, box, rc, excl_off=None, excl_idx=None):
    """Interacting pairs (i < j, lexicographic) and their FP64 distances."""
    n = len(x)
    xa, xp = _d(np.asarray(x, dtype=np.float64).reshape(-1))
    bx = np.array([box] * 3 if np.isscalar(box) else box, dtype=np.float64)
    ba, bp = _d(bx)
    if excl_off is not None:
        oa, op = _i(excl_off)
        ia, ipp = _i(excl_idx)
    else:
        op = ipp = None
    L = lib()
    cnt = L.oracle_pairs(n, xp, bp, float(rc), op, ipp, 0, None, None, None)
    pi = np.zeros(max(cnt, 1), np.int32)
    pj = np.zeros(max(cnt, 1), np.int32)
    pr = np.zeros(max(cnt, 1), np.float64)
    L.oracle_pairs(n, xp, bp, float(rc), op, ipp, cnt,
                   pi.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                   pj.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                   pr.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return pi[:cnt], pj[:cnt], pr[:cnt]


def vjp(x, q, typ, sigma, epsilon, box, rc, beta, fc, excl_off, excl_idx, gF, gE):
    """dL/dx [N,3], dL/dq [N], dL/dsigma [nt], dL/deps [nt] for cotangents gF [N,3], gE [2]."""
    n = len(q)
    nt = len(sigma)
    xa, xp = _d(np.asarray(x, dtype=np.float64).reshape(-1))
    qa, qp = _d(q)
    ta, tp = _i(typ)
    sa, sp = _d(sigma)
    ea, ep = _d(epsilon)
    bx = np.array([box] * 3 if np.isscalar(box) else box, dtype=np.float64)
    ba, bp = _d(bx)
    oa, op = _i(excl_off)
    ia, ipp = _i(excl_idx)
    ga, gp = _d(np.asarray(gF, dtype=np.float64).reshape(-1))
    gea, gep = _d(gE)
    dx, dxp = _d(np.zeros(3 * n))
    dq, dqp = _d(np.zeros(n))
    ds, dsp = _d(np.zeros(nt))
    de, dep = _d(np.zeros(nt))
    rc_ = lib().oracle_vjp(n, xp, qp, tp, nt, sp, ep, bp, float(rc), float(beta), float(fc), op,
                           ipp, gp, gep, dxp, dqp, dsp, dep)
    if rc_ != 0:
        raise RuntimeError("oracle_vjp failed")
    return dx.reshape(n, 3), dq, ds, de


def ewald_corrections(x, q, box, beta, fc, excl_off=None, excl_idx=None):
    """Ewald exclusion correction and self term: returns (f [n][3] of the exclusion
    correction, E_excl, E_self, virial 3 x 3 of the exclusion correction)."""
    n = len(q)
    xa, xp = _d(np.asarray(x, dtype=np.float64).reshape(-1))
    qa, qp = _d(q)
    ba, bp = _d(np.array([box] * 3 if np.isscalar(box) else box, dtype=np.float64))
    if excl_off is not None:
        oa, op = _i(excl_off)
        ia, ipp = _i(excl_idx if len(excl_idx) else np.zeros(1, np.int32))
    else:
        op = ipp = None
    f, fp = _d(np.zeros(3 * n))
    out, outp = _d(np.zeros(8))
    lib().oracle_ewald_corrections(n, xp, qp, bp, float(beta), float(fc), op, ipp, fp, outp)
    v = out[2:8]
    vir = np.array([[v[0], v[3], v[4]], [v[3], v[1], v[5]], [v[4], v[5], v[2]]])
    return f.reshape(n, 3), float(out[0]), float(out[1]), vir


# ---- conveniences over an Instance ---------------------------------------------------------

def instance_forces(inst, cells: Optional[bool] = None, x=None, q=None, sigma=None,
                    epsilon=None, round32: bool = True, elec: int = 0, vdw: int = 0,
                    epsilon_rf: float = 0.0, rswitch: float = 0.0) -> Result:
    """Oracle forces/energies for an Instance (optionally with replaced x, q, sigma, eps, and
    another interaction flavour)."""
    if cells is None:
        cells = inst.natoms > 20000
    return forces(inst.x if x is None else x, inst.q if q is None else q, inst.type,
                  inst.sigma if sigma is None else sigma,
                  inst.epsilon if epsilon is None else epsilon, inst.box, inst.cutoff,
                  inst.beta, inst.coulomb_const, inst.excl_off, inst.excl_idx, cells=cells,
                  round32=round32, elec=elec, vdw=vdw, epsilon_rf=epsilon_rf, rswitch=rswitch)


def loss(inst, x, q, sigma, epsilon, f_target, e_target, cells: bool = False):
    """Force-matching loss sum |F - F_t|^2 + (E - E_t)^2 in FP64 (unrounded LJ table)."""
    r = forces(x, q, inst.type, sigma, epsilon, inst.box, inst.cutoff, inst.beta,
               inst.coulomb_const, inst.excl_off, inst.excl_idx, cells=cells, round32=False)
    e = r.e_lj + r.e_coul
    return float(np.sum((r.f - f_target) ** 2) + (e - e_target) ** 2), r


def useful_pair_estimate(natoms: int, box: float, rc: float, nmol: int) -> float:
    """N rho (4/3) pi rc^3 / 2 - 3 W: expected interacting pairs at uniform density."""
    rho = natoms / box ** 3
    return natoms * rho * (4.0 / 3.0) * math.pi * rc ** 3 / 2.0 - 3 * nmol
