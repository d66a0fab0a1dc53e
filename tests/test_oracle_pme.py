"""Pins of the FP64 reciprocal-space references (oracle/pme.py).

* Madelung: a rock-salt crystal of unit charges at nearest-neighbour distance r0 has the Ewald
  total energy (real space + reciprocal space + self term) -(N/2) M fC / r0 with the NaCl
  Madelung constant M = 1.747564594633182 (the textbook lattice sum); the real-space part comes
  from the C oracle (unshifted), the reciprocal part from ewald_recip_direct.  A wrong factor,
  sign or wave-vector scaling anywhere in the three parts fails it.
* The Ewald total does not depend on the splitting parameter beta.
* Reciprocal forces are minus the gradient of the reciprocal energy (central differences).
* Smooth PME converges to the direct sum as the grid and the B-spline order grow, to 1e-8 on a
  48^3 grid with order 8: two independent algorithms for the same quantity."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from oracle import pme

FC = 138.935458
MADELUNG_NACL = 1.747564594633182


def rock_salt(ncell, a):
    """ncell^3 conventional cells of edge a: 8 ncell^3 ions on a simple cubic lattice of spacing
    a/2 with charge (-1)^(i+j+k)."""
    s = 2 * ncell
    idx = np.stack(np.meshgrid(np.arange(s), np.arange(s), np.arange(s), indexing="ij"), -1).reshape(-1, 3)
    x = (idx + 0.25) * (a / 2.0)
    q = np.where(idx.sum(1) % 2 == 0, 1.0, -1.0)
    return x, q, ncell * a


def ewald_total(x, q, L, beta, rc):
    n = len(q)
    real = O.forces(x, q, np.zeros(n, np.int32), np.zeros(1), np.zeros(1), L, rc, beta, FC,
                    round32=False)
    e_rec, _ = pme.ewald_recip_direct(x, q, L, beta, FC)
    e_self = -FC * beta / math.sqrt(math.pi) * float(np.sum(q * q))
    return real.e_coul_unshifted + e_rec + e_self


def test_rock_salt_gives_the_madelung_energy():
    a = 0.5
    x, q, L = rock_salt(4, a)          # 512 ions, L = 2 nm
    rc = 0.99
    beta = 5.6 / rc                    # erfc(beta rc) ~ 1e-15
    e = ewald_total(x, q, L, beta, rc)
    ref = -0.5 * len(q) * MADELUNG_NACL * FC / (a / 2.0)
    assert abs(e - ref) <= 1e-9 * abs(ref)


def test_ewald_total_does_not_depend_on_beta():
    rng = np.random.default_rng(3)
    x, q, L = rock_salt(2, 0.5)
    x = x + rng.uniform(-0.05, 0.05, x.shape)   # off the lattice
    e1 = ewald_total(x, q, L, 5.6 / 0.49, 0.49)
    e2 = ewald_total(x, q, L, 7.0 / 0.49, 0.49)
    assert abs(e1 - e2) <= 1e-9 * abs(e1)


def small_system(n=48, L=1.8, seed=5):
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.0, L, (n, 3))
    q = rng.normal(0.0, 1.0, n)
    q -= q.mean()
    return x, q, L


def test_reciprocal_forces_are_minus_gradient():
    x, q, L = small_system()
    beta = 3.0
    _, f = pme.ewald_recip_direct(x, q, L, beta, FC)
    h = 1e-6
    for i in (0, 7, 31):
        for c in range(3):
            xp, xm = x.copy(), x.copy()
            xp[i, c] += h
            xm[i, c] -= h
            de = (pme.ewald_recip_direct(xp, q, L, beta, FC)[0] - pme.ewald_recip_direct(xm, q, L, beta, FC)[0]) / (2 * h)
            assert abs(f[i, c] + de) <= 1e-6 * np.abs(f).max()


def test_pme_converges_to_the_direct_sum():
    x, q, L = small_system()
    beta = 3.0
    e0, f0 = pme.ewald_recip_direct(x, q, L, beta, FC)
    errs = []
    for K, order in [(16, 4), (32, 6), (48, 8)]:
        e, f = pme.pme_reference(x, q, L, beta, FC, (K, K, K), order)
        errs.append((abs(e - e0) / abs(e0), float(np.sqrt(((f - f0) ** 2).sum() / (f0 ** 2).sum()))))
    assert errs[0][0] > errs[1][0] > errs[2][0] and errs[0][1] > errs[1][1] > errs[2][1]
    assert errs[2][0] <= 1e-8 and errs[2][1] <= 1e-8


def test_pme_forces_are_minus_gradient_of_pme_energy():
    """The PME forces are the exact gradient of the PME energy (the B-spline interpolation is
    differentiable), whatever the grid."""
    x, q, L = small_system(n=24)
    beta, grid, order = 3.0, (12, 14, 16), 4
    _, f = pme.pme_reference(x, q, L, beta, FC, grid, order)
    h = 1e-6
    for i in (0, 11):
        for c in range(3):
            xp, xm = x.copy(), x.copy()
            xp[i, c] += h
            xm[i, c] -= h
            de = (pme.pme_reference(xp, q, L, beta, FC, grid, order)[0] - pme.pme_reference(xm, q, L, beta, FC, grid, order)[0]) / (2 * h)
            assert abs(f[i, c] + de) <= 1e-6 * np.abs(f).max()
