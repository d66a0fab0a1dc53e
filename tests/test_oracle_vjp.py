"""Pin of the oracle's analytic VJP (dL/dx, dL/dq, dL/dsigma, dL/deps of the force-matching loss
L = sum |F - F_t|^2 + (E - E_t)^2) against FP64 central differences of the oracle loss.

Targets come from the oracle at parameters perturbed by 2% (sigma, epsilon, q).  Position
components whose atom has a neighbour within 1e-4 nm of the cutoff are skipped: the forces jump
there, so the loss is not differentiable.  Agreement: relative 1e-6 per component with magnitude
above 1e-3 of the RMS of its kind."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2405_01420_amd import synth


@pytest.fixture(scope="module")
def problem():
    inst = synth.small_box(300, 0.9, 0.1, seed=21, ntypes_extra=4)
    inst = synth.perturb_charges(inst, 0.02, seed=22)
    sig_t, eps_t, q_t = synth.perturbed_params(inst, 0.02, seed=23)
    tgt = O.forces(inst.x, q_t, inst.type, sig_t, eps_t, inst.box, inst.cutoff, inst.beta,
                   inst.coulomb_const, inst.excl_off, inst.excl_idx, round32=False)
    f_t, e_t = tgt.f, tgt.e_lj + tgt.e_coul
    x = inst.x.astype(np.float64)
    q = inst.q.astype(np.float64)
    L0, r0 = O.loss(inst, x, q, inst.sigma, inst.epsilon, f_t, e_t)
    e0 = r0.e_lj + r0.e_coul
    gF = 2.0 * (r0.f - f_t)
    gE = np.array([2.0 * (e0 - e_t)] * 2)
    dx, dq, ds, de = O.vjp(x, q, inst.type, inst.sigma, inst.epsilon, inst.box, inst.cutoff,
                           inst.beta, inst.coulomb_const, inst.excl_off, inst.excl_idx, gF, gE)
    return dict(inst=inst, f_t=f_t, e_t=e_t, x=x, q=q, dx=dx, dq=dq, ds=ds, de=de, L0=L0)


def fd(problem, which, index, h):
    inst = problem["inst"]
    args = dict(x=problem["x"].copy(), q=problem["q"].copy(), sigma=inst.sigma.copy(),
                epsilon=inst.epsilon.copy())
    vals = []
    for sgn in (1, -1):
        a = {k: v.copy() for k, v in args.items()}
        a[which][index] += sgn * h
        L, _ = O.loss(inst, a["x"], a["q"], a["sigma"], a["epsilon"], problem["f_t"], problem["e_t"])
        vals.append(L)
    return (vals[0] - vals[1]) / (2 * h)


def test_vjp_positions(problem):
    inst = problem["inst"]
    pi, pj, pr = O.pairs(problem["x"], inst.box, inst.cutoff + 1e-3)
    near = set(np.concatenate([pi[np.abs(pr - inst.cutoff) < 1e-4], pj[np.abs(pr - inst.cutoff) < 1e-4]]).tolist())
    rng = np.random.default_rng(7)
    rms = np.sqrt(np.mean(problem["dx"] ** 2))
    done = 0
    for a in rng.permutation(inst.natoms):
        if a in near:
            continue
        c = int(rng.integers(3))
        g = problem["dx"][a, c]
        if abs(g) < 1e-3 * rms:
            continue
        v = fd(problem, "x", (a, c), 1e-6)
        assert abs(v - g) <= 1e-6 * abs(g), (a, c, v, g)
        done += 1
        if done == 24:
            break
    assert done == 24


def test_vjp_charges(problem):
    inst = problem["inst"]
    rng = np.random.default_rng(8)
    rms = np.sqrt(np.mean(problem["dq"] ** 2))
    done = 0
    for a in rng.permutation(inst.natoms)[:60]:
        g = problem["dq"][a]
        if abs(g) < 1e-3 * rms:
            continue
        v = fd(problem, "q", a, 1e-6)
        assert abs(v - g) <= 1e-6 * abs(g), (a, v, g)
        done += 1
        if done == 16:
            break
    assert done == 16


def test_vjp_lj_parameters(problem):
    inst = problem["inst"]
    for t in range(inst.ntypes):
        if inst.epsilon[t] == 0.0:
            assert problem["de"][t] == 0.0
            continue
        for which, key in (("sigma", "ds"), ("epsilon", "de")):
            base = inst.sigma[t] if which == "sigma" else inst.epsilon[t]
            v = fd(problem, which, t, 1e-6 * base)
            g = problem[key][t]
            assert abs(v - g) <= 1e-6 * abs(g), (which, t, v, g)


def test_local_loss_difference_equals_full(problem):
    """The neighbour-row form of the loss difference used by the GPU gradient test at 24k atoms
    (tests/fd_local.py) equals the difference of the full loss, for coordinates and charges."""
    from tests.fd_local import loss_difference
    inst = problem["inst"]
    e0 = O.loss(inst, problem["x"], problem["q"], inst.sigma, inst.epsilon, problem["f_t"],
                problem["e_t"])[1]
    e0 = e0.e_lj + e0.e_coul
    rng = np.random.default_rng(31)
    for a in rng.permutation(inst.natoms)[:6]:
        c = int(rng.integers(3))
        loc = loss_difference(inst, problem["x"], problem["q"], e0, problem["f_t"], problem["e_t"], a, c)
        full = fd(problem, "x", (a, c), 1e-6)
        assert abs(loc - full) <= 1e-7 * max(abs(full), 1.0), (a, c, loc, full)
        loc = loss_difference(inst, problem["x"], problem["q"], e0, problem["f_t"], problem["e_t"], a)
        full = fd(problem, "q", a, 1e-6)
        assert abs(loc - full) <= 1e-7 * max(abs(full), 1.0), (a, loc, full)
