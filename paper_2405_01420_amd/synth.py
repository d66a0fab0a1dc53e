"""Seeded synthetic water boxes: the inputs of every test, benchmark and parity check.

This module only *makes inputs*. It holds none of the short-range force arithmetic
(no pair potentials, no neighbour search, no forces): both the FP64 oracle and the
HIP path receive exactly the arrays produced here and compute independently.

The paper measures on uniform-density water/ethanol boxes of the Grappa family and on
biomolecular systems (paper section II-C); those input files are not available here, so
these boxes stand in for the uniform-density family.  Recipe (rigid 3-site water at about
100 atoms/nm^3 on a jittered cubic lattice with random orientations):

* geometry: O at the molecule origin, both H at 0.1 nm, H-O-H angle 109.47 degrees;
* charges: O -0.82 e, H +0.41 e;  Lennard-Jones on O only (sigma 0.3166 nm, epsilon
  0.650 kJ/mol); H carries a null LJ type (sigma = epsilon = 0);
* exclusions: the three intramolecular pairs of each molecule;
* lattice: n = ceil(W^(1/3)) sites per edge at (k + 1/2) L/n; when n^3 > W, W sites are
  chosen uniformly without replacement; each O is displaced by U(-0.02, 0.02) nm per axis;
  orientations are uniform on SO(3);
* guard: no two atoms of different molecules closer than 0.05 nm (an offending molecule
  gets a new orientation from a generator derived deterministically from its index);
* atom order O, H, H per molecule, molecules in lattice order; coordinates wrapped into
  [0, L);
* all floating-point inputs the GPU receives (x, q, L, rc, beta, f_C) are rounded to FP32;
  the oracle widens the same FP32 values exactly to FP64.

The Ewald splitting parameter beta is an *input* of the method; it is chosen here from
the usual real-space tolerance erfc(beta * rc) = 1e-5 by bisection.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

O_SIGMA = 0.3166          # nm
O_EPSILON = 0.650         # kJ/mol
Q_O = -0.82               # e
Q_H = 0.41                # e
OH_BOND = 0.1             # nm
HOH_ANGLE_DEG = 109.47
COULOMB_CONST = 138.935458  # kJ mol^-1 nm e^-2  (1 / (4 pi eps0))
DENSITY = 100.0           # atoms per nm^3 (batched boxes)
EWALD_RTOL = 1e-5


def f32(v: float) -> float:
    """Round a Python float to the nearest FP32 value (returned as a Python float)."""
    return float(np.float32(v))


def ewald_beta(rc: float, rtol: float = EWALD_RTOL) -> float:
    """beta with erfc(beta * rc) = rtol, by bisection in FP64 (then rounded to FP32)."""
    lo, hi = 0.0, 50.0 / rc
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if math.erfc(mid * rc) > rtol:
            lo = mid
        else:
            hi = mid
    return f32(0.5 * (lo + hi))


@dataclasses.dataclass
class Instance:
    """One periodic box.  Arrays are host numpy arrays in original atom order."""
    x: np.ndarray            # float32 [N, 3], in [0, L)
    q: np.ndarray            # float32 [N]
    type: np.ndarray         # int32 [N]
    box: float               # cubic edge L (FP32 value)
    cutoff: float            # rc (FP32 value)
    buffer: float            # rb, list buffer (FP32 value)
    beta: float              # Ewald beta (FP32 value)
    coulomb_const: float     # f_C (FP32 value)
    sigma: np.ndarray        # float64 [ntypes]
    epsilon: np.ndarray      # float64 [ntypes]
    excl_off: np.ndarray     # int32 [N + 1]  CSR offsets of excluded partners
    excl_idx: np.ndarray     # int32 [nnz]    excluded partner indices
    name: str = ""
    seed: int = 0

    @property
    def natoms(self) -> int:
        return int(self.x.shape[0])

    @property
    def ntypes(self) -> int:
        return int(self.sigma.shape[0])

    @property
    def rlist(self) -> float:
        return self.cutoff + self.buffer


def _random_rotations(rng: np.random.Generator, n: int) -> np.ndarray:
    """n rotation matrices uniform on SO(3) (Shoemake's unit-quaternion method)."""
    u1, u2, u3 = rng.random(n), rng.random(n), rng.random(n)
    a, b = np.sqrt(1 - u1), np.sqrt(u1)
    qw = a * np.sin(2 * np.pi * u2)
    qx = a * np.cos(2 * np.pi * u2)
    qy = b * np.sin(2 * np.pi * u3)
    qz = b * np.cos(2 * np.pi * u3)
    R = np.empty((n, 3, 3))
    R[:, 0, 0] = 1 - 2 * (qy * qy + qz * qz)
    R[:, 0, 1] = 2 * (qx * qy - qz * qw)
    R[:, 0, 2] = 2 * (qx * qz + qy * qw)
    R[:, 1, 0] = 2 * (qx * qy + qz * qw)
    R[:, 1, 1] = 1 - 2 * (qx * qx + qz * qz)
    R[:, 1, 2] = 2 * (qy * qz - qx * qw)
    R[:, 2, 0] = 2 * (qx * qz - qy * qw)
    R[:, 2, 1] = 2 * (qy * qz + qx * qw)
    R[:, 2, 2] = 1 - 2 * (qx * qx + qy * qy)
    return R


def _body_frame() -> np.ndarray:
    half = math.radians(HOH_ANGLE_DEG) / 2
    return np.array([[0.0, 0.0, 0.0],
                     [OH_BOND * math.sin(half), OH_BOND * math.cos(half), 0.0],
                     [-OH_BOND * math.sin(half), OH_BOND * math.cos(half), 0.0]])


def _close_molecules(pos: np.ndarray, L: float, dmin: float) -> np.ndarray:
    """Indices of molecules with an atom closer than dmin to an atom of another molecule."""
    from scipy.spatial import cKDTree
    flat = np.mod(pos.reshape(-1, 3), L)
    flat[flat >= L] = 0.0
    tree = cKDTree(flat, boxsize=L)
    pairs = tree.query_pairs(dmin, output_type="ndarray")
    if len(pairs) == 0:
        return np.zeros(0, dtype=np.int64)
    mi, mj = pairs[:, 0] // 3, pairs[:, 1] // 3
    inter = mi != mj
    return np.unique(np.concatenate([mi[inter], mj[inter]]))


def water_box(nwater: int, box: float, cutoff: float, buffer: float, seed: int,
              jitter: float = 0.02, name: str = "") -> Instance:
    """Rigid 3-site waters on a jittered lattice in a cubic periodic box (see module doc)."""
    rng = np.random.default_rng(seed)
    L = f32(box)
    n = int(math.ceil(round(nwater ** (1.0 / 3.0), 9)))
    while n ** 3 < nwater:
        n += 1
    sites = np.arange(n ** 3)
    if n ** 3 > nwater:
        sites = np.sort(rng.choice(n ** 3, size=nwater, replace=False))
    k = np.stack([sites // (n * n), (sites // n) % n, sites % n], axis=1).astype(np.float64)
    centres = (k + 0.5) * (L / n)
    centres += rng.uniform(-jitter, jitter, size=centres.shape)
    R = _random_rotations(rng, nwater)
    body = _body_frame()
    pos = centres[:, None, :] + np.einsum("mij,aj->mai", R, body)
    for attempt in range(1000):
        bad = _close_molecules(pos, L, 0.05)
        if len(bad) == 0:
            break
        for m in bad:
            r2 = np.random.default_rng([seed, int(m), attempt + 1])
            Rm = _random_rotations(r2, 1)[0]
            pos[m] = centres[m] + body @ Rm.T
    else:  # pragma: no cover - the guard always converges at these densities
        raise RuntimeError("could not place molecules without close contacts")
    x = np.mod(pos.reshape(-1, 3), L).astype(np.float32)
    x[x >= np.float32(L)] = 0.0
    x[x < 0] = 0.0
    natoms = 3 * nwater
    q = np.tile(np.array([Q_O, Q_H, Q_H], dtype=np.float32), nwater)
    typ = np.tile(np.array([0, 1, 1], dtype=np.int32), nwater)
    off = np.arange(0, 2 * natoms + 1, 2, dtype=np.int32)
    idx = np.empty(2 * natoms, dtype=np.int32)
    base = 3 * np.arange(nwater)
    for a in range(3):
        others = [b for b in range(3) if b != a]
        idx[2 * (base + a)] = base + others[0]
        idx[2 * (base + a) + 1] = base + others[1]
    return Instance(x=x, q=q, type=typ, box=L, cutoff=f32(cutoff), buffer=f32(buffer),
                    beta=ewald_beta(f32(cutoff)), coulomb_const=f32(COULOMB_CONST),
                    sigma=np.array([O_SIGMA, 0.0]), epsilon=np.array([O_EPSILON, 0.0]),
                    excl_off=off, excl_idx=idx, name=name, seed=seed)


def retype(inst: Instance, ntypes_extra: int, fraction_of_o: float, seed: int) -> Instance:
    """Assign extra LJ types to O atoms only (H keeps its null type).

    Type layout afterwards: 0 = the standard O type, 1 = null H type, 2.. = extra types with
    sigma ~ U(0.25, 0.40) nm and epsilon ~ U(0.1, 1.0) kJ/mol.  ``fraction_of_o`` of the O atoms
    (chosen without replacement) get one of the extra types uniformly.  With fraction 1 the
    standard O type disappears from the atoms but stays in the table.
    """
    rng = np.random.default_rng(seed)
    sig = np.concatenate([inst.sigma, rng.uniform(0.25, 0.40, ntypes_extra)])
    eps = np.concatenate([inst.epsilon, rng.uniform(0.1, 1.0, ntypes_extra)])
    typ = inst.type.copy()
    o_atoms = np.nonzero(typ == 0)[0]
    nsel = int(round(fraction_of_o * len(o_atoms)))
    chosen = np.sort(rng.choice(o_atoms, size=nsel, replace=False))
    typ[chosen] = 2 + rng.integers(0, ntypes_extra, size=nsel)
    return dataclasses.replace(inst, type=typ.astype(np.int32), sigma=sig, epsilon=eps)


# ----------------------------------------------------------------------------------------
# Named workloads (sizes of the five configurations the method is measured on)
# ----------------------------------------------------------------------------------------

def tiny() -> Instance:
    """216 waters (648 atoms), L = 1.862 nm, rc = 0.9 nm, no list buffer (one call)."""
    return water_box(216, 1.862, 0.9, 0.0, seed=1, name="tiny")


def mid() -> Instance:
    """32,000 waters (96,000 atoms), L = 9.87 nm, rc = 1.0 nm, rb = 0.1 nm."""
    return water_box(32000, 9.87, 1.0, 0.1, seed=2, name="mid")


def large() -> Instance:
    """1,000,000 waters (3,000,000 atoms), L = 31.1 nm, rc = 1.2 nm, rb = 0.1 nm;
    10% of all atoms (30% of the O atoms) get one of 4 extra LJ types."""
    inst = water_box(1000000, 31.1, 1.2, 0.1, seed=3, name="large")
    return retype(inst, 4, 0.3, seed=30)


def diff() -> Instance:
    """8,000 waters (24,000 atoms), L = 6.21 nm, rc = 1.0 nm, rb = 0.1 nm; every O gets one
    of 4 random LJ types; charges perturbed by N(0, 0.02 e) and re-neutralised per molecule."""
    inst = water_box(8000, 6.21, 1.0, 0.1, seed=5, name="diff")
    inst = retype(inst, 4, 1.0, seed=50)
    return perturb_charges(inst, 0.02, seed=51)


def perturb_charges(inst: Instance, sd: float, seed: int) -> Instance:
    rng = np.random.default_rng(seed)
    q = inst.q.astype(np.float64) + rng.normal(0.0, sd, inst.natoms)
    qm = q.reshape(-1, 3)
    qm -= qm.mean(axis=1, keepdims=True)
    return dataclasses.replace(inst, q=qm.reshape(-1).astype(np.float32))


def small_box(nwater: int, cutoff: float, buffer: float, seed: int, ntypes_extra: int = 0,
              name: str = "small") -> Instance:
    """A water box at 100 atoms/nm^3 with edge (3 W / 100)^(1/3)."""
    L = (3 * nwater / DENSITY) ** (1.0 / 3.0)
    inst = water_box(nwater, L, cutoff, buffer, seed=seed, name=name)
    if ntypes_extra:
        inst = retype(inst, ntypes_extra, 1.0, seed=seed + 7)
    return inst


def batch_sizes(nbox: int = 256, seed: int = 4) -> List[int]:
    """Atom counts log-uniform in [3000, 30000], multiples of 3."""
    rng = np.random.default_rng(seed)
    n = np.exp(rng.uniform(math.log(3000), math.log(30000), nbox))
    return [int(3 * round(v / 3)) for v in n]


def batch(nbox: int = 256, seed: int = 4, cutoff: float = 0.9, buffer: float = 0.1,
          sizes: Optional[List[int]] = None) -> List[Instance]:
    """Independent cubic boxes at 100 atoms/nm^3, one list each (box b uses seed 4000 + b)."""
    sizes = batch_sizes(nbox, seed) if sizes is None else sizes
    out = []
    for b, natoms in enumerate(sizes):
        w = natoms // 3
        L = (natoms / DENSITY) ** (1.0 / 3.0)
        out.append(water_box(w, L, cutoff, buffer, seed=1000 * seed + b, name=f"batch{b}"))
    return out


def jitter_stream(seed: int = 20):
    """Generator of per-call random-walk displacements N(0, 0.002 nm) (float32 [N,3])."""
    return np.random.default_rng(seed)


def perturbed_params(inst: Instance, rel: float, seed: int):
    """sigma, epsilon and q each multiplied by (1 + rel * xi), xi ~ N(0, 1); charges are then
    re-neutralised per molecule.  Null-type entries stay zero.  Returns (sigma, epsilon, q)."""
    rng = np.random.default_rng(seed)
    sig = inst.sigma * (1 + rel * rng.normal(size=inst.ntypes))
    eps = inst.epsilon * (1 + rel * rng.normal(size=inst.ntypes))
    q = inst.q.astype(np.float64) * (1 + rel * rng.normal(size=inst.natoms))
    qm = q.reshape(-1, 3)
    qm -= qm.mean(axis=1, keepdims=True)
    return sig, eps, qm.reshape(-1).astype(np.float32)


ION_Q = 0.5               # e, magnitude of the ion charges of the charged Lennard-Jones fluid
ION_MASS = 18.0           # g/mol
KB = 0.0083144626         # kJ mol^-1 K^-1


def ionic_fluid(nion: int, box: float, cutoff: float = 1.0, buffer: float = 0.1, seed: int = 8,
                temperature: float = 300.0, jitter: float = 0.02, name: str = "ionic"):
    """A single-site charged Lennard-Jones fluid for molecular dynamics without constraints:
    ions of charge +-ION_Q (alternating over a checkerboard of a jittered cubic lattice, signs of
    a few ions flipped where sites left empty unbalance it; neutral for an even number of ions),
    all of the water-oxygen Lennard-Jones type, mass
    ION_MASS, no exclusions; velocities drawn from the Maxwell-Boltzmann distribution at
    `temperature` with the net momentum removed.  Returns (Instance, v float32 [N, 3] nm/ps,
    inverse masses float32 [N])."""
    rng = np.random.default_rng(seed)
    L = f32(box)
    n = int(math.ceil(round(nion ** (1.0 / 3.0), 9)))
    while n ** 3 < nion:
        n += 1
    sites = np.arange(n ** 3)
    if n ** 3 > nion:
        sites = np.sort(rng.choice(n ** 3, size=nion, replace=False))
    k = np.stack([sites // (n * n), (sites // n) % n, sites % n], axis=1)
    pos = (k.astype(np.float64) + 0.5) * (L / n) + rng.uniform(-jitter, jitter, size=(nion, 3))
    x = np.mod(pos, L).astype(np.float32)
    x[x >= np.float32(L)] = 0.0
    sign = np.where(k.sum(1) % 2 == 0, 1.0, -1.0)
    excess = int(sign.sum())   # sites left out of the lattice can unbalance the checkerboard
    if excess != 0:
        major = np.nonzero(sign == np.sign(excess))[0]
        sign[rng.choice(major, size=abs(excess) // 2, replace=False)] *= -1.0
    q = (ION_Q * sign).astype(np.float32)
    typ = np.zeros(nion, dtype=np.int32)
    sd = math.sqrt(KB * temperature / ION_MASS)
    v = rng.normal(0.0, sd, size=(nion, 3))
    v -= v.mean(0)
    inst = Instance(x=x, q=q, type=typ, box=L, cutoff=f32(cutoff), buffer=f32(buffer),
                    beta=ewald_beta(f32(cutoff)), coulomb_const=f32(COULOMB_CONST),
                    sigma=np.array([O_SIGMA]), epsilon=np.array([O_EPSILON]),
                    excl_off=np.zeros(nion + 1, dtype=np.int32), excl_idx=np.zeros(0, dtype=np.int32),
                    name=name, seed=seed)
    return inst, v.astype(np.float32), np.full(nion, 1.0 / ION_MASS, dtype=np.float32)
