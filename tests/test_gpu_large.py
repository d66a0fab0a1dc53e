"""Parity at the largest size: 1,000,000 waters (3,000,000 atoms), L = 31.1 nm, rc = 1.2 nm,
rb = 0.1 nm, 30% of the O atoms re-typed to 4 extra LJ types.  The FP64 cell-list oracle
(checked equal to brute force on smaller boxes) gives all forces and energies; the pair set is
checked by its size (the full set has about 1.1e9 pairs), which may differ only by pairs whose
FP64 distance lies within 2^-22 L of the cutoff.  FP64 pair energies are used: with FP32 pair
energies the Coulomb energy of this box ends near 1e-6 relative (its conditioning is 1e-4)."""
import ctypes

import numpy as np
import pytest

from oracle import oracle as O
from paper_2405_01420_amd import nb, synth
from tests.gpu_helpers import ENERGY_TOL, FORCE_TOL, GpuBox, compare_forces

pytestmark = pytest.mark.gpu


def test_large_forces_energies_and_pair_count(torch_gpu):
    inst = synth.large()
    print("generated", inst.natoms, flush=True)
    box = GpuBox(torch_gpu, inst, flags=nb.NB_ENERGY_FP64)
    box.pairlist()
    f, e = box.forces()
    cnt = ctypes.c_int64(0)
    rc = nb.lib().nb_debug_pairs(box.ctx, box.x.data_ptr(), None, 0, ctypes.byref(cnt))
    assert rc == nb.NB_OK
    st = box.stats()
    box.close()
    print("gpu done", st, flush=True)
    ref = O.instance_forces(inst, cells=True)
    print(f"oracle pairs {ref.npairs} gpu pairs {cnt.value}", flush=True)
    fr, elj, ec = compare_forces(f, e, ref, "large")
    assert abs(cnt.value - ref.npairs) <= 200
    assert fr <= FORCE_TOL and elj <= ENERGY_TOL and ec <= ENERGY_TOL
