"""Parity at the largest size: 1,000,000 waters (3,000,000 atoms), L = 31.1 nm, rc = 1.2 nm,
rb = 0.1 nm, 30% of the O atoms re-typed to 4 extra LJ types.  The FP64 cell-list oracle
(checked equal to brute force on smaller boxes) gives all forces and energies; the pair set is
checked by its size (the full set has about 1.1e9 pairs), which may differ only by pairs whose
FP64 distance lies within 2^-22 L of the cutoff.  Both energy modes are checked against the same
oracle run: FP64 pair energies to the 1e-6 energy gate; the default FP32 pair energies (the mode
the benchmark times) to the force gate and 1e-6 on E_LJ, while its Coulomb energy, a sum
conditioned at 1e-4, ends at 1.05e-6 relative (the per-pair FP32 rounding) and is held to 2e-6."""
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
    # the default mode (FP32 pair energies), as the benchmark times it
    box = GpuBox(torch_gpu, inst)
    box.pairlist()
    f32, e32 = box.forces()
    box.close()
    ref = O.instance_forces(inst, cells=True)
    print(f"oracle pairs {ref.npairs} gpu pairs {cnt.value}", flush=True)
    fr, elj, ec = compare_forces(f, e, ref, "large")
    assert abs(cnt.value - ref.npairs) <= 200
    assert fr <= FORCE_TOL and elj <= ENERGY_TOL and ec <= ENERGY_TOL
    fr, elj, ec = compare_forces(f32, e32, ref, "large, FP32 pair energies")
    assert fr <= FORCE_TOL and elj <= ENERGY_TOL and ec <= 2 * ENERGY_TOL
