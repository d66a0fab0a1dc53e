"""Central differences of the force-matching loss L = sum_i |F_i - F_t,i|^2 + (E - E_t)^2 with
respect to one coordinate or one charge, computed from the oracle's rows of the atoms that the
perturbation touches (the perturbed atom and its neighbours within the cutoff): every other
row of F is unchanged bit for bit, and E changes by the change of those atoms' pair energies.
Oracle-only CPU helper of the gradient tests; equal to differencing the full loss (checked in
tests/test_oracle_vjp.py) at a small fraction of its cost."""
import numpy as np

from oracle import oracle as O


def neighbours(inst, x, a, margin=1e-3):
    d = x - x[a]
    d -= inst.box * np.rint(d / inst.box)
    r = np.sqrt((d * d).sum(1))
    return np.nonzero(r < inst.cutoff + margin)[0].astype(np.int32), r


def _rows(inst, x, q, sigma, epsilon, sub):
    f, el, ec = O.forces_subset(x, q, inst.type, sigma, epsilon, inst.box, inst.cutoff, inst.beta,
                                inst.coulomb_const, inst.excl_off, inst.excl_idx, sub,
                                round32=False)
    return f, float(np.sum(el) + np.sum(ec))


def loss_difference(inst, x0, q0, e0, f_t, e_t, a, coord=None, h=1e-6):
    """(L(+h) - L(-h)) / (2h) for coordinate `coord` of atom a, or for the charge of atom a when
    coord is None.  e0: the total energy at (x0, q0) (unrounded LJ table)."""
    sub, _ = neighbours(inst, x0, a)
    _, es0 = _rows(inst, x0, q0, inst.sigma, inst.epsilon, sub)
    out = []
    for sgn in (1.0, -1.0):
        x, q = x0, q0
        if coord is None:
            q = q0.copy()
            q[a] += sgn * h
        else:
            x = x0.copy()
            x[a, coord] += sgn * h
        f, es = _rows(inst, x, q, inst.sigma, inst.epsilon, sub)
        e = e0 + (es - es0)
        out.append(np.sum((f - f_t[sub]) ** 2) + (e - e_t) ** 2)
    # rows outside `sub` cancel exactly between the two states
    return (out[0] - out[1]) / (2 * h)
