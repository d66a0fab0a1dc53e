"""Parity of the Ewald exclusion correction and self term (NB_EWALD_CORR) of the HIP path with
the FP64 oracle: forces (real-space + exclusion-correction forces) RMS relative <= 5e-6, the
real-space energies as in the plain parity tests, and the two correction energies, which both
sides compute in FP64: they differ by the order of an N-term sum of same-sign terms (the self
term) and libm erf against the device's, bounded by N u with u = 2^-53, i.e. 1.1e-11 for the
96,000-atom box; the bound used is 2^-53 N, at least 1e-12."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2405_01420_amd import nb, synth
from tests.gpu_helpers import ENERGY_TOL, FORCE_TOL, GpuBox, compare_forces

pytestmark = pytest.mark.gpu

CORR_TOL = 1e-12


def corr_tol(natoms):
    return max(CORR_TOL, natoms * 2.0 ** -53)


@pytest.mark.parametrize("name,flags", [("tiny", nb.NB_ENERGY_FP64), ("diff", 0), ("mid", 0)])
def test_ewald_corrections_match_oracle(torch_gpu, name, flags):
    """tiny, the 24k-atom box, and the 96k-atom box the benchmark times this call on."""
    inst = {"tiny": synth.tiny, "diff": synth.diff, "mid": synth.mid}[name]()
    box = GpuBox(torch_gpu, inst, flags=flags | nb.NB_EWALD_CORR)
    box.pairlist()
    f, e = box.forces()
    box.close()
    ref = O.instance_forces(inst, cells=name != "tiny")
    fcorr, e_excl, e_self, _ = O.ewald_corrections(inst.x, inst.q, inst.box, inst.beta,
                                                inst.coulomb_const, inst.excl_off, inst.excl_idx)
    ref.f = ref.f + fcorr
    fr, elj, ec = compare_forces(f, e, ref, f"{name} with Ewald corrections")
    rex = abs(e[2] - e_excl) / abs(e_excl)
    rse = abs(e[3] - e_self) / abs(e_self)
    print(f"E_excl {e[2]:.10e} ref {e_excl:.10e} rel {rex:.2e};  E_self rel {rse:.2e}", flush=True)
    assert fr <= FORCE_TOL and elj <= ENERGY_TOL and ec <= ENERGY_TOL
    assert rex <= corr_tol(inst.natoms) and rse <= corr_tol(inst.natoms)


def test_ewald_corrections_follow_the_positions(torch_gpu):
    """Atoms moved after the build (some across the periodic faces): the correction uses the
    minimum image of the current positions.  A 0.1 nm list buffer covers the motion (the
    648-atom box is otherwise built without one)."""
    inst = synth.tiny()
    box = GpuBox(torch_gpu, inst, flags=nb.NB_ENERGY_FP64 | nb.NB_EWALD_CORR, buffer=0.1)
    box.pairlist()
    x = inst.x.copy()
    rng = np.random.default_rng(11)
    x = (x + rng.normal(0.0, 0.002, x.shape)).astype(np.float32)
    box.set_x(x)
    f, e = box.forces()
    box.close()
    ref = O.instance_forces(inst, x=x)
    fcorr, e_excl, e_self, _ = O.ewald_corrections(x, inst.q, inst.box, inst.beta,
                                                inst.coulomb_const, inst.excl_off, inst.excl_idx)
    ref.f = ref.f + fcorr
    fr, elj, ec = compare_forces(f, e, ref, "tiny moved, with Ewald corrections")
    assert fr <= FORCE_TOL and elj <= ENERGY_TOL and ec <= ENERGY_TOL
    assert abs(e[2] - e_excl) <= CORR_TOL * abs(e_excl)
    assert abs(e[3] - e_self) <= CORR_TOL * abs(e_self)
