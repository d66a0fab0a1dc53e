"""Pins of the FP64 oracle against facts that do not come from the oracle itself: printed
table values of erf, closed forms of the Lennard-Jones and Coulomb pair terms, Newton's third
law, forces = -grad E by central differences, exclusions, invariances under permutation,
translation and rotation of the periodic box, an explicit periodic-image enumeration, the
brute-force vs cell-list enumerations, and the expected pair count of a uniform fluid.

Each check is chosen so that a plausible slip in the oracle (a dropped term, a wrong sign, a
transposed index, a double-counted pair, a wrong image) fails at least one of them."""
import math
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2405_01420_amd import synth

HERE = os.path.dirname(os.path.abspath(__file__))
FC = synth.f32(synth.COULOMB_CONST)


def two_atoms(r, box=10.0, q=(1.0, -1.0), sigma=0.3166, eps=0.65, across=False, axis=0):
    """Two atoms r apart along `axis`; with across=True the pair straddles the periodic face."""
    x = np.zeros((2, 3))
    if across:
        x[0, axis] = 0.05
        x[1, axis] = box - (r - 0.05)
    else:
        x[0, axis] = 1.0
        x[1, axis] = 1.0 + r
    x[:, (axis + 1) % 3] += 2.0
    q = np.array(q, dtype=np.float64)
    typ = np.array([0, 0], dtype=np.int32)
    return x, q, typ, np.array([sigma]), np.array([eps])


def run(x, q, typ, sig, eps, box, rc, beta, fc=FC, off=None, idx=None, round32=False):
    return O.forces(x, q, typ, sig, eps, box, rc, beta, fc, off, idx, round32=round32)


# ---- closed forms ---------------------------------------------------------------------------

def test_erfc_matches_printed_table():
    """Two charges with beta chosen so that beta r hits the tabulated points; the shift term uses
    erfc(2) from the table as well (beta rc = 2).  E / (fC q1 q2) = erfc(beta r)/r - erfc(2)/rc."""
    tab = np.loadtxt(os.path.join(HERE, "golden", "erf_table.txt"))
    erfc2 = 1.0 - tab[tab[:, 0] == 2.0, 1][0]
    r = 0.4
    for xv, erfv in tab:
        if xv >= 2.0:
            continue
        beta = xv / r
        rc = 2.0 / beta
        if rc >= 5.0:
            continue
        xx, q, typ, s, e = two_atoms(r, q=(0.5, 0.8), eps=0.0)
        res = run(xx, q, typ, s, e, 10.0, rc, beta)
        expect = FC * 0.4 * ((1.0 - erfv) / r - erfc2 / rc)
        assert abs(res.e_coul - expect) <= 1e-12 * abs(expect), (xv, res.e_coul, expect)
        assert res.e_lj == 0.0


@pytest.mark.parametrize("across", [False, True])
def test_lj_minimum_and_zero_crossing(across):
    """q = 0: the LJ force vanishes at r* = 2^(1/6) sigma, where E = -eps - shift(rc); at
    r = sigma the unshifted LJ energy is zero, so E = -shift(rc)."""
    sig, eps, rc = 0.3166, 0.65, 1.0
    C6, C12 = 4 * eps * sig ** 6, 4 * eps * sig ** 12
    shift = C12 / rc ** 12 - C6 / rc ** 6
    rstar = 2 ** (1 / 6) * sig
    x, q, typ, s, e = two_atoms(rstar, q=(0.0, 0.0), across=across)
    res = run(x, q, typ, s, e, 10.0, rc, 3.0)
    assert abs(res.e_lj - (-eps - shift)) <= 1e-12 * eps
    assert np.abs(res.f).max() <= 1e-9
    x, q, typ, s, e = two_atoms(sig, q=(0.0, 0.0), across=across)
    res = run(x, q, typ, s, e, 10.0, rc, 3.0)
    assert abs(res.e_lj + shift) <= 1e-12 * eps
    # repulsive inside r*: the force on atom 0 points away from atom 1
    x, q, typ, s, e = two_atoms(0.9 * rstar, q=(0.0, 0.0))
    res = run(x, q, typ, s, e, 10.0, rc, 3.0)
    assert res.f[0, 0] < 0 and res.f[1, 0] > 0


def two_types(r, sig, eps):
    """Atom 0 of type 0 and atom 1 of type 1, r apart, no charges."""
    x = np.zeros((2, 3))
    x[:, 1] = 2.0
    x[0, 0] = 1.0
    x[1, 0] = 1.0 + r
    return x, np.zeros(2), np.array([0, 1], dtype=np.int32), np.array(sig), np.array(eps)


@pytest.mark.parametrize("sig,eps", [((0.25, 0.40), (0.10, 1.00)), ((0.3166, 0.28), (0.65, 0.2))])
def test_unlike_types_follow_lorentz_berthelot(sig, eps):
    """Two atoms of different types interact through sigma_ab = (sigma_a + sigma_b)/2 and
    eps_ab = sqrt(eps_a eps_b): the pair force vanishes at 2^(1/6) sigma_ab, where the energy is
    the well depth -eps_ab minus the shift, and the unshifted energy is zero at r = sigma_ab.
    (A geometric-mean sigma or an arithmetic-mean eps moves the minimum or changes its depth.)"""
    rc = 1.0
    sab = 0.5 * (sig[0] + sig[1])
    eab = math.sqrt(eps[0] * eps[1])
    shift = 4 * eab * ((sab / rc) ** 12 - (sab / rc) ** 6)
    x, q, typ, s, e = two_types(2 ** (1 / 6) * sab, sig, eps)
    res = run(x, q, typ, s, e, 10.0, rc, 3.0)
    assert abs(res.e_lj - (-eab - shift)) <= 1e-12 * eab
    assert np.abs(res.f).max() <= 1e-9 * eab / sab
    x, q, typ, s, e = two_types(sab, sig, eps)
    res = run(x, q, typ, s, e, 10.0, rc, 3.0)
    assert abs(res.e_lj + shift) <= 1e-12 * eab
    # the well is the deepest point: slightly off the minimum on either side the energy is higher
    for f in (0.999, 1.001):
        x, q, typ, s, e = two_types(f * 2 ** (1 / 6) * sab, sig, eps)
        assert run(x, q, typ, s, e, 10.0, rc, 3.0).e_lj > -eab - shift


def test_lj_table_hand_computed():
    """C6 = 4 eps_ab sigma_ab^6 and C12 = 4 eps_ab sigma_ab^12 for a three-type table whose
    combined parameters are exact decimals: sigma = (0.3, 0.5, 0.4), eps = (1, 4, 0.25) give
    sigma_01 = 0.4, eps_01 = 2; sigma_02 = 0.35, eps_02 = 0.5; sigma_12 = 0.45, eps_12 = 1."""
    c6, c12 = O.lj_table([0.3, 0.5, 0.4], [1.0, 4.0, 0.25], round32=False)
    expect6 = {(0, 0): 4 * 0.000729, (1, 1): 16 * 0.015625, (2, 2): 0.004096,
               (0, 1): 8 * 0.004096, (0, 2): 2 * 0.001838265625, (1, 2): 4 * 0.008303765625}
    expect12 = {(0, 0): 4 * 0.000729 ** 2, (1, 1): 16 * 0.015625 ** 2, (2, 2): 0.004096 ** 2,
                (0, 1): 8 * 0.004096 ** 2, (0, 2): 2 * 0.001838265625 ** 2,
                (1, 2): 4 * 0.008303765625 ** 2}
    for (a, b), v in expect6.items():
        for (i, j) in ((a, b), (b, a)):
            assert abs(c6[i, j] - v) <= 1e-14 * v, (i, j, c6[i, j], v)
            assert abs(c12[i, j] - expect12[(a, b)]) <= 1e-14 * expect12[(a, b)], (i, j)
    # rounded once to FP32: the instance's table
    r6, r12 = O.lj_table([0.3, 0.5, 0.4], [1.0, 4.0, 0.25], round32=True)
    assert np.array_equal(r6, c6.astype(np.float32).astype(np.float64))
    assert np.array_equal(r12, c12.astype(np.float32).astype(np.float64))


@pytest.mark.parametrize("across", [False, True])
def test_plain_coulomb_when_beta_is_zero(across):
    """beta = 0 reduces the Ewald real-space term to the shifted plain Coulomb law:
    E = fC q1 q2 (1/r - 1/rc), |F| = fC |q1 q2| / r^2, like charges repel."""
    rc = 1.2
    for r in (0.1, 0.35, 0.8, 1.19):
        x, q, typ, s, e = two_atoms(r, q=(0.7, 0.3), eps=0.0, across=across)
        res = run(x, q, typ, s, e, 10.0, rc, 0.0)
        assert abs(res.e_coul - FC * 0.21 * (1 / r - 1 / rc)) <= 1e-12 * FC * 0.21 / r
        assert abs(np.linalg.norm(res.f[0]) - FC * 0.21 / r ** 2) <= 1e-11 * FC * 0.21 / r ** 2
        sign = -1.0 if not across else 1.0  # atom 0 is left of atom 1 unless wrapped
        assert np.sign(res.f[0, 0]) == sign


def test_energy_vanishes_at_cutoff():
    rc, beta = 1.0, 3.1
    x, q, typ, s, e = two_atoms(rc - 1e-9, q=(0.8, -0.4))
    res = run(x, q, typ, s, e, 10.0, rc, beta)
    assert abs(res.e_lj) < 1e-9 and abs(res.e_coul) < 1e-9
    x, q, typ, s, e = two_atoms(rc + 1e-9, q=(0.8, -0.4))
    res = run(x, q, typ, s, e, 10.0, rc, beta)
    assert res.e_lj == 0.0 and res.e_coul == 0.0 and np.all(res.f == 0.0) and res.npairs == 0


def test_beta_meets_tolerance():
    for rc in (0.9, 1.0, 1.2):
        b = synth.ewald_beta(synth.f32(rc))
        assert abs(math.erfc(b * synth.f32(rc)) / 1e-5 - 1) < 1e-5


# ---- whole-box properties -------------------------------------------------------------------

@pytest.fixture(scope="module")
def tiny():
    return synth.tiny()


@pytest.fixture(scope="module")
def small_typed():
    """900 atoms, 4 LJ types on O, perturbed charges: a small stand-in of the gradient workload."""
    inst = synth.small_box(300, 0.9, 0.1, seed=11, ntypes_extra=4)
    return synth.perturb_charges(inst, 0.02, seed=12)


def test_newton_third_law(tiny, small_typed):
    for inst in (tiny, small_typed):
        r = O.instance_forces(inst)
        assert np.abs(r.f.sum(0)).max() <= 1e-10 * np.abs(r.f).sum()


def test_single_molecule_has_no_interaction():
    inst = synth.water_box(1, 3.0, 1.0, 0.0, seed=3)
    r = O.instance_forces(inst)
    assert r.e_lj == 0.0 and r.e_coul == 0.0 and np.all(r.f == 0.0) and r.npairs == 0


def test_forces_are_minus_energy_gradient(small_typed):
    """Central differences of the total energy (h = 1e-6 nm) against the oracle forces, on
    coordinates whose atom has no neighbour within 1e-4 nm of the cutoff."""
    inst = small_typed
    x0 = inst.x.astype(np.float64)
    ref = O.instance_forces(inst, round32=True)
    pi, pj, pr = O.pairs(x0, inst.box, inst.cutoff + 1e-3)
    near = np.unique(np.concatenate([pi[np.abs(pr - inst.cutoff) < 1e-4],
                                     pj[np.abs(pr - inst.cutoff) < 1e-4]]))
    rng = np.random.default_rng(7)
    h = 1e-6
    checked = 0
    for a in rng.permutation(inst.natoms):
        if a in near:
            continue
        c = rng.integers(3)
        xp, xm = x0.copy(), x0.copy()
        xp[a, c] += h
        xm[a, c] -= h
        ep = O.instance_forces(inst, x=xp)
        em = O.instance_forces(inst, x=xm)
        fd = -((ep.e_lj + ep.e_coul) - (em.e_lj + em.e_coul)) / (2 * h)
        assert abs(fd - ref.f[a, c]) <= 1e-6 * max(abs(ref.f[a, c]), 1e-3 * np.sqrt(np.mean(ref.f ** 2))), (a, c)
        checked += 1
        if checked == 24:
            break
    assert checked == 24


def test_exclusions_remove_exactly_the_intramolecular_pairs(tiny):
    with_ex = O.instance_forces(tiny)
    without = O.forces(tiny.x, tiny.q, tiny.type, tiny.sigma, tiny.epsilon, tiny.box, tiny.cutoff,
                       tiny.beta, tiny.coulomb_const)
    assert without.npairs - with_ex.npairs == 3 * (tiny.natoms // 3)


def test_permutation_invariance(small_typed):
    inst = small_typed
    rng = np.random.default_rng(5)
    p = rng.permutation(inst.natoms)
    inv = np.empty_like(p)
    inv[p] = np.arange(inst.natoms)
    # permuted exclusion lists
    lists = [inst.excl_idx[inst.excl_off[i]:inst.excl_off[i + 1]] for i in range(inst.natoms)]
    off = [0]
    idx = []
    for k in range(inst.natoms):
        part = sorted(inv[lists[p[k]]])
        idx += part
        off.append(len(idx))
    r0 = O.instance_forces(inst)
    r1 = O.forces(inst.x[p], inst.q[p], inst.type[p], inst.sigma, inst.epsilon, inst.box,
                  inst.cutoff, inst.beta, inst.coulomb_const, np.array(off), np.array(idx))
    assert np.allclose(r1.f, r0.f[p], rtol=0, atol=1e-10 * np.abs(r0.f).max())
    assert abs(r1.e_lj - r0.e_lj) <= 1e-12 * abs(r0.abs_lj)
    assert abs(r1.e_coul - r0.e_coul) <= 1e-12 * abs(r0.abs_coul)


def test_translation_invariance(tiny):
    rng = np.random.default_rng(9)
    t = rng.uniform(0, tiny.box, 3)
    x1 = np.mod(tiny.x.astype(np.float64) + t, tiny.box)
    r0 = O.instance_forces(tiny, x=tiny.x.astype(np.float64))
    r1 = O.instance_forces(tiny, x=x1)
    assert abs(r1.e_lj - r0.e_lj) <= 1e-12 * r0.abs_lj
    assert abs(r1.e_coul - r0.e_coul) <= 1e-12 * r0.abs_coul
    assert np.abs(r1.f - r0.f).max() <= 1e-10 * np.abs(r0.f).max()


def test_rotation_by_90_degrees(tiny):
    """(x, y, z) -> (L - y, x, z) maps the cubic box onto itself and rotates every force."""
    L = tiny.box
    x = tiny.x.astype(np.float64)
    xr = np.stack([np.mod(L - x[:, 1], L), x[:, 0], x[:, 2]], axis=1)
    r0 = O.instance_forces(tiny, x=x)
    r1 = O.instance_forces(tiny, x=xr)
    fr = np.stack([-r0.f[:, 1], r0.f[:, 0], r0.f[:, 2]], axis=1)
    assert np.abs(r1.f - fr).max() <= 1e-10 * np.abs(r0.f).max()
    assert abs(r1.e_coul - r0.e_coul) <= 1e-12 * r0.abs_coul


def test_explicit_image_enumeration(tiny):
    """Pairs found by scanning all 27 periodic images of every atom equal the minimum-image pair
    set, and no pair has two images inside the cutoff (rc < L/2)."""
    x = tiny.x.astype(np.float64)
    L, rc = tiny.box, tiny.cutoff
    n = len(x)
    found = {}
    for img in np.array(np.meshgrid([-1, 0, 1], [-1, 0, 1], [-1, 0, 1])).T.reshape(-1, 3):
        d = x[:, None, :] - (x[None, :, :] + img * L)
        r = np.sqrt((d * d).sum(-1))
        ii, jj = np.nonzero((r < rc) & (np.arange(n)[:, None] < np.arange(n)[None, :]))
        for a, b in zip(ii, jj):
            found[(a, b)] = found.get((a, b), 0) + 1
    assert max(found.values()) == 1
    excl = set()
    for i in range(n):
        for j in tiny.excl_idx[tiny.excl_off[i]:tiny.excl_off[i + 1]]:
            excl.add((min(i, j), max(i, j)))
    img_set = set(found) - excl
    pi, pj, _ = O.pairs(x, L, rc, tiny.excl_off, tiny.excl_idx)
    assert img_set == set(zip(pi.tolist(), pj.tolist()))


@pytest.mark.parametrize("which", ["tiny", "diff", "mid"])
def test_cell_list_equals_brute_force(which):
    """The cell-list enumeration (used for the 96k- and 3M-atom parity references) gives the same
    pair set, energies and forces as the O(N^2) definition on the 648-, 24k- and 96k-atom boxes."""
    inst = getattr(synth, which)()
    a = O.instance_forces(inst, cells=False)
    b = O.instance_forces(inst, cells=True)
    assert a.npairs == b.npairs
    assert abs(a.e_lj - b.e_lj) <= 1e-12 * a.abs_lj
    assert abs(a.e_coul - b.e_coul) <= 1e-12 * a.abs_coul
    assert abs(a.qq_sum - b.qq_sum) <= 1e-12 * np.abs(inst.q).max() ** 2 * a.npairs
    assert np.abs(a.f - b.f).max() <= 1e-10 * np.abs(a.f).max()
    if which != "mid":
        pi, pj, _ = O.pairs(inst.x, inst.box, inst.cutoff, inst.excl_off, inst.excl_idx)
        assert len(pi) == a.npairs


def test_subset_rows_equal_full_rows(small_typed):
    """oracle_forces_subset restricted to a few atoms reproduces those atoms' force rows and
    per-atom energy halves of the full O(N^2) sum."""
    inst = small_typed
    full = O.instance_forces(inst, cells=False)
    sub = np.array([0, 5, 17, 299, inst.natoms - 1], dtype=np.int32)
    fs, el, ec = O.forces_subset(inst.x, inst.q, inst.type, inst.sigma, inst.epsilon, inst.box,
                                 inst.cutoff, inst.beta, inst.coulomb_const, inst.excl_off,
                                 inst.excl_idx, sub)
    assert np.array_equal(fs, full.f[sub])
    assert np.array_equal(el, full.eatom_lj[sub]) and np.array_equal(ec, full.eatom_c[sub])


def test_unshifted_energy_consistency(tiny):
    r = O.instance_forces(tiny)
    sh = tiny.coulomb_const * math.erfc(tiny.beta * tiny.cutoff) / tiny.cutoff
    assert abs((r.e_coul_unshifted - r.e_coul) - sh * r.qq_sum) <= 1e-12 * r.abs_coul


def test_pair_count_matches_uniform_density():
    inst = synth.mid()
    r = O.instance_forces(inst, cells=True)
    est = O.useful_pair_estimate(inst.natoms, inst.box, inst.cutoff, inst.natoms // 3)
    assert abs(r.npairs / est - 1) < 0.01


@pytest.mark.parametrize("n", [4096, 4097, 1024])
def test_pair_count_of_an_evenly_spaced_periodic_line(n):
    """n atoms d = L / n apart on a line along z of a periodic box (L = 20 nm): every atom has
    exactly floor(rc / d) neighbours on each side within rc (none at rc exactly here), so the
    pair set holds n floor(rc / d) pairs, those across the periodic face included, and each
    pair's distance is a multiple of d."""
    L, rc = 20.0, np.float32(0.9)
    x = np.zeros((n, 3), dtype=np.float32)
    x[:, 0] = x[:, 1] = 1.0
    x[:, 2] = (np.arange(n) + 0.5) * (L / n)
    pi, pj, pr = O.pairs(x, np.float32(L), rc)
    d = L / n
    k = math.floor(float(rc) / d)
    assert abs(k * d - float(rc)) > 1e-4 and abs((k + 1) * d - float(rc)) > 1e-4
    assert len(pi) == n * k
    steps = np.rint(pr / d)
    assert np.all((steps >= 1) & (steps <= k)) and np.allclose(pr, steps * d, atol=1e-5)
    # every separation 1 .. k occurs n times, counting the pairs that wrap around the box
    assert np.array_equal(np.bincount(steps.astype(int), minlength=k + 1)[1:], np.full(k, n))
