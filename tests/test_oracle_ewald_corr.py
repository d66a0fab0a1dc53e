"""Pins of the oracle's Ewald exclusion correction and self term against facts outside their
code: for a large beta erf(beta r) = 1 and the exclusion correction is minus the bare Coulomb
interaction of the excluded pairs; for a small beta the self term and the exclusion correction
of a neutral molecule cancel up to the beta^3 term 2 beta^3 / (3 sqrt(pi)) fC sum q_i q_j r^2;
forces are minus the gradient (central differences); coincident excluded atoms take the r -> 0
limit; Newton's third law holds on a water box.

A dropped factor 2 / sqrt(pi), a wrong sign of either force term, a missing or doubled self term
or a pair counted twice fails at least one of them."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2405_01420_amd import synth

FC = 138.935458


def water(center=(2.0, 2.0, 2.0)):
    ang = math.radians(109.47)
    x = np.array([[0.0, 0.0, 0.0], [0.1, 0.0, 0.0], [0.1 * math.cos(ang), 0.1 * math.sin(ang), 0.0]])
    x += np.asarray(center)
    q = np.array([-0.82, 0.41, 0.41])
    off = np.array([0, 2, 4, 6], np.int32)
    idx = np.array([1, 2, 0, 2, 0, 1], np.int32)
    return x, q, off, idx


def corr(x, q, off, idx, beta, box=10.0):
    return O.ewald_corrections(x, q, box, beta, FC, off, idx)


def pair_list(x):
    return [(i, j, np.linalg.norm(x[i] - x[j])) for i in range(3) for j in range(i + 1, 3)]


def test_large_beta_gives_minus_bare_coulomb():
    x, q, off, idx = water()
    f, e_excl, _, _ = corr(x, q, off, idx, beta=50.0)
    bare = sum(FC * q[i] * q[j] / r for i, j, r in pair_list(x))
    assert abs(e_excl + bare) <= 1e-10 * abs(bare)
    fb = np.zeros((3, 3))
    for i, j, r in pair_list(x):
        fij = FC * q[i] * q[j] * (x[i] - x[j]) / r ** 3  # Coulomb force on i
        fb[i] += fij
        fb[j] -= fij
    assert np.allclose(f, -fb, rtol=1e-9, atol=0.0)


def test_small_beta_self_and_exclusion_cancel_to_beta_cubed():
    x, q, off, idx = water()
    beta = 1e-3
    _, e_excl, e_self, _ = corr(x, q, off, idx, beta)
    lead = FC * 2.0 * beta ** 3 / (3.0 * math.sqrt(math.pi)) * sum(q[i] * q[j] * r * r for i, j, r in pair_list(x))
    assert abs((e_excl + e_self) - lead) <= 1e-5 * abs(lead)
    # each term alone is far larger than the sum: the cancellation is what is checked
    assert abs(e_self) > 1e4 * abs(lead)


@pytest.mark.parametrize("beta", [1.0, 3.47])
def test_exclusion_forces_are_minus_gradient(beta):
    x, q, off, idx = water(center=(0.02, 9.97, 5.0))  # straddles two periodic faces
    f, _, _, _ = corr(x, q, off, idx, beta)
    h = 1e-6
    for a in range(3):
        for c in range(3):
            xp, xm = x.copy(), x.copy()
            xp[a, c] += h
            xm[a, c] -= h
            de = (corr(xp, q, off, idx, beta)[1] - corr(xm, q, off, idx, beta)[1]) / (2 * h)
            assert abs(f[a, c] + de) <= 1e-6 * np.abs(f).max()


def test_coincident_excluded_atoms_take_the_limit():
    x = np.array([[1.0, 1.0, 1.0], [1.0, 1.0, 1.0]])
    q = np.array([0.5, -0.3])
    off = np.array([0, 1, 2], np.int32)
    idx = np.array([1, 0], np.int32)
    beta = 3.0
    f, e0, _, _ = corr(x, q, off, idx, beta)
    assert abs(e0 + FC * q[0] * q[1] * 2.0 * beta / math.sqrt(math.pi)) <= 1e-12 * abs(e0)
    assert np.all(f == 0.0)
    x[1, 2] += 1e-6
    _, e1, _, _ = corr(x, q, off, idx, beta)
    assert abs(e1 - e0) <= 1e-9 * abs(e0)


def test_water_box_obeys_newtons_third_law():
    inst = synth.tiny()
    f, e_excl, e_self, _ = O.ewald_corrections(inst.x, inst.q, inst.box, inst.beta, inst.coulomb_const,
                                            inst.excl_off, inst.excl_idx)
    assert np.abs(f.sum(0)).max() <= 1e-12 * np.abs(f).sum()
    assert e_self < 0.0 < e_excl
