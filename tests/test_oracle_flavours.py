"""Pins of the oracle's reaction-field and force-switch flavours against facts that do not come
from the flavour code itself: the reduction of the reaction field with eps_rf = 1 to the plain
shifted Coulomb law (reached through the independent Ewald path with beta = 0), the vanishing
of energy and force at the cutoff, forces = -dE/dr by central differences, the identity of the
switched force with the plain Lennard-Jones force below the switch radius, the quadratic
vanishing of the switched force at rc, and Newton's third law on a water box.

A wrong k_rf or c_rf, a wrong sign or power in A_a or B_a, a wrong shift constant K_a or a
switch applied below r1 fails at least one of them."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2405_01420_amd import synth

FC = synth.f32(synth.COULOMB_CONST)
RC = 1.0
R1 = 0.8


def two_atoms(r, q=(0.7, -0.4), sigma=0.3166, eps=0.65):
    x = np.zeros((2, 3))
    x[0] = (1.0, 2.0, 3.0)
    x[1] = (1.0 + r, 2.0, 3.0)
    return x, np.array(q, dtype=np.float64), np.zeros(2, np.int32), np.array([sigma]), np.array([eps])


def run(r, coulomb=True, lj=True, **fl):
    """Two atoms r apart; coulomb/lj switch the charges and the LJ well off, so that a check
    sees one term alone."""
    x, q, t, s, e = two_atoms(r, q=(0.7, -0.4) if coulomb else (0.0, 0.0), eps=0.65 if lj else 0.0)
    return O.forces(x, q, t, s, e, 10.0, RC, 0.0, FC, round32=False, **fl)


def energy(r, **kw):
    res = run(r, **kw)
    return res.e_lj + res.e_coul


def test_rf_with_unit_dielectric_is_shifted_coulomb():
    """k_rf = 0 for eps_rf = 1: the reaction field reduces to fC q q (1/r - 1/rc), which the Ewald
    path gives with beta = 0 (erfc(0) = 1)."""
    for r in (0.15, 0.3, 0.55, 0.95):
        a = run(r, elec=1, epsilon_rf=1.0)
        b = run(r)  # Ewald, beta = 0
        assert abs(a.e_coul - b.e_coul) <= 1e-13 * abs(b.e_coul)
        assert np.allclose(a.f, b.f, rtol=1e-13, atol=0.0)


@pytest.mark.parametrize("eps_rf", [0.0, 78.0, 2.0])
def test_rf_energy_vanishes_at_cutoff_and_force_is_minus_gradient(eps_rf):
    fl = dict(elec=1, epsilon_rf=eps_rf, lj=False)
    scale = FC * 0.28 / RC
    e_edge = run(RC * (1.0 - 1e-9), **fl).e_coul
    assert abs(e_edge) <= 1e-7 * scale
    for r in (0.2, 0.5, 0.9):
        h = 1e-6
        de = (energy(r + h, **fl) - energy(r - h, **fl)) / (2 * h)
        f = run(r, **fl).f
        # force on atom 0 along x is -dE/dx0 = +dE/dr (atom 1 sits at larger x)
        assert abs(f[0, 0] - de) <= 1e-6 * abs(de) + 1e-9


def test_rf_force_vanishes_at_cutoff_for_conducting_boundary():
    """eps_rf = infinity gives k_rf = 1/(2 rc^3): dE/dr = fC q q (-1/r^2 + 2 k_rf r) = 0 at rc."""
    for d in (1e-3, 1e-4):
        f = run(RC - d, elec=1, epsilon_rf=0.0, lj=False).f[0, 0]
        f0 = run(0.5, elec=1, epsilon_rf=0.0, lj=False).f[0, 0]
        assert abs(f) <= 5.0 * d * abs(f0)


def test_force_switch_equals_plain_lj_below_r1():
    """Below r1 the switched force is the plain LJ force; the energies differ by one constant."""
    diffs = []
    for r in (0.3, 0.45, 0.7, R1 - 1e-6):
        a = run(r, coulomb=False, vdw=1, rswitch=R1)
        b = run(r, coulomb=False)
        assert np.allclose(a.f, b.f, rtol=1e-12, atol=0.0)
        diffs.append(a.e_lj - b.e_lj)
    # constant to FP64 rounding of energies up to ~1.4 (the offset itself is ~2e-3)
    assert np.ptp(diffs) <= 1e-11 * max(abs(d) for d in diffs)
    assert abs(diffs[0]) > 0.0


def test_force_switch_vanishes_quadratically_at_cutoff():
    """Energy zero at rc; force and its derivative zero at rc, so F(rc - d) ~ d^2."""
    eps_only = dict(vdw=1, rswitch=R1, coulomb=False)
    e_edge = run(RC * (1.0 - 1e-10), **eps_only).e_lj
    e_mid = run(0.35, **eps_only).e_lj
    assert abs(e_edge) <= 1e-9 * abs(e_mid)
    f1 = run(RC - 1e-3, **eps_only).f[0, 0]
    f2 = run(RC - 2e-3, **eps_only).f[0, 0]
    assert f1 != 0.0
    assert abs(f2 / f1 - 4.0) <= 0.05


@pytest.mark.parametrize("r", [0.32, 0.79, 0.81, 0.9, 0.99])
def test_force_switch_force_is_minus_gradient(r):
    h = 1e-6
    fl = dict(vdw=1, rswitch=R1, coulomb=False)
    de = (energy(r + h, **fl) - energy(r - h, **fl)) / (2 * h)
    f = run(r, **fl).f[0, 0]
    assert abs(f - de) <= 1e-6 * abs(de) + 1e-10


def test_force_switch_is_continuous_at_r1():
    fl = dict(vdw=1, rswitch=R1, coulomb=False)
    a, b = run(R1 - 1e-9, **fl), run(R1 + 1e-9, **fl)
    assert abs(a.f[0, 0] - b.f[0, 0]) <= 1e-6 * abs(a.f[0, 0])
    assert abs(a.e_lj - b.e_lj) <= 1e-6 * abs(a.e_lj)


@pytest.mark.parametrize("fl", [dict(elec=1, epsilon_rf=78.0), dict(vdw=1, rswitch=0.7),
                                dict(elec=1, vdw=1, rswitch=0.7)])
def test_flavoured_box_obeys_newtons_third_law(fl):
    inst = synth.tiny()
    r = O.instance_forces(inst, **fl)
    net = np.abs(r.f.sum(0)).max()
    assert net <= 1e-9 * np.abs(r.f).sum()


def test_vjp_rejects_other_flavours_cleanly():
    """The gradient oracle is defined for the default flavour only; the flavour state is reset
    after each flavoured call, so a later default call is unaffected."""
    inst = synth.tiny()
    a = O.instance_forces(inst)
    O.instance_forces(inst, elec=1)
    b = O.instance_forces(inst)
    assert a.e_coul == b.e_coul
