"""Pins of the oracle's virial Xi = -1/2 sum d (x) F_ij against the energy, which other pins
fix: stretching axis a of the box and every coordinate by (1 + h) changes the energy at the
rate 2 Xi_aa, and shearing an isolated cluster (x_a += g x_b) at the rate 2 Xi_ab.  Checked by
FP64 central differences for the default interactions, the force switch, the reaction field,
and for the Ewald exclusion correction.  A wrong sign, a missing factor 1/2 or a pair counted
twice fails them."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2405_01420_amd import synth

H = 1e-6


def energy(inst, x, box, **fl):
    r = O.forces(x, inst.q, inst.type, inst.sigma, inst.epsilon, box, inst.cutoff, inst.beta,
                 inst.coulomb_const, inst.excl_off, inst.excl_idx, **fl)
    return r.e_lj + r.e_coul, r


def stretched(inst, a, s):
    x = inst.x.astype(np.float64).copy()
    box = np.full(3, float(inst.box))
    x[:, a] *= s
    box[a] *= s
    return x, box


@pytest.mark.parametrize("fl", [dict(), dict(vdw=1, rswitch=0.7), dict(elec=1, epsilon_rf=0.0)])
def test_diagonal_is_half_the_stretch_derivative(fl):
    inst = synth.tiny()
    _, r0 = energy(inst, inst.x.astype(np.float64), float(inst.box), **fl)
    for a in range(3):
        ep, _ = energy(inst, *stretched(inst, a, 1.0 + H), **fl)
        em, _ = energy(inst, *stretched(inst, a, 1.0 - H), **fl)
        de = (ep - em) / (2 * H)
        assert abs(r0.virial[a, a] - 0.5 * de) <= 1e-6 * abs(de)


def cluster():
    """20 waters of the 648-atom box, moved to the middle of a 10 nm box (no images within rc)."""
    inst = synth.tiny()
    n = 60
    x = inst.x[:n].astype(np.float64) + 4.0
    sub = dict(q=inst.q[:n], type=inst.type[:n], sigma=inst.sigma, epsilon=inst.epsilon,
               excl_off=inst.excl_off[:n + 1], excl_idx=inst.excl_idx[:inst.excl_off[n]])
    return inst, x, sub


@pytest.mark.parametrize("a,b", [(0, 1), (0, 2), (1, 2)])
def test_off_diagonal_is_half_the_shear_derivative(a, b):
    inst, x, s = cluster()

    def e(g):
        xs = x.copy()
        xs[:, a] += g * x[:, b]
        r = O.forces(xs, s["q"], s["type"], s["sigma"], s["epsilon"], 10.0, inst.cutoff, inst.beta,
                     inst.coulomb_const, s["excl_off"], s["excl_idx"])
        return r.e_lj + r.e_coul, r

    _, r0 = e(0.0)
    de = (e(H)[0] - e(-H)[0]) / (2 * H)
    assert abs(r0.virial[a, b] - 0.5 * de) <= 1e-6 * abs(de)
    assert r0.virial[a, b] == r0.virial[b, a]


def test_exclusion_correction_virial():
    inst = synth.tiny()
    args = (inst.q, inst.beta, inst.coulomb_const, inst.excl_off, inst.excl_idx)

    def e_excl(x, box):
        q, beta, fc, eo, ei = args
        return O.ewald_corrections(x, q, box, beta, fc, eo, ei)

    _, _, _, vir = e_excl(inst.x, float(inst.box))
    for a in range(3):
        de = (e_excl(*stretched(inst, a, 1.0 + H))[1] - e_excl(*stretched(inst, a, 1.0 - H))[1]) / (2 * H)
        assert abs(vir[a, a] - 0.5 * de) <= 1e-6 * abs(de)
    inst2, x, s = cluster()
    xs_p, xs_m = x.copy(), x.copy()
    xs_p[:, 0] += H * x[:, 1]
    xs_m[:, 0] -= H * x[:, 1]
    ec = lambda xx: O.ewald_corrections(xx, s["q"], 10.0, inst.beta, inst.coulomb_const, s["excl_off"], s["excl_idx"])
    de = (ec(xs_p)[1] - ec(xs_m)[1]) / (2 * H)
    assert abs(ec(x)[3][0, 1] - 0.5 * de) <= 1e-6 * abs(de)
