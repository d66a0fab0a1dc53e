"""Parity of the virial output (nb_forces_virial) with the FP64 oracle's
Xi = -1/2 sum d (x) F_ij.  Gate: Frobenius-norm relative error <= 5e-6, the force gate (the
virial is a sum of the same FP32 pair forces, weighted by the displacements); the 3 x 3 result
is symmetric by construction.  The forces and energies of the same call must still meet their
own gates, and with NB_EWALD_CORR the exclusion correction's virial is included."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2405_01420_amd import nb, synth
from tests.gpu_helpers import ENERGY_TOL, FORCE_TOL, GpuBox, compare_forces

pytestmark = pytest.mark.gpu

VIR_TOL = 5e-6


def run(torch, inst, flags=0, **fl):
    box = GpuBox(torch, inst, flags=flags, **fl)
    vir = torch.zeros(9, dtype=torch.float64, device="cuda:0")
    box.pairlist()
    nb.nb_forces_virial(box.ctx, box.x, box.q, box.t, box.f, box.e, vir)
    torch.cuda.synchronize()
    f = box.f.cpu().numpy().reshape(-1, 3).astype(np.float64)
    e = box.e.cpu().numpy()
    v = vir.cpu().numpy().reshape(3, 3)
    box.close()
    return f, e, v


def frob_rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("name,flags,fl", [
    ("tiny", nb.NB_ENERGY_FP64, {}),
    ("diff", 0, {}),
    ("diff", 0, dict(elec=nb.NB_ELEC_RF, epsilon_rf=0.0, vdw=nb.NB_VDW_FSWITCH, rswitch=0.8)),
    ("mid", 0, {}),   # the 96k-atom box the benchmark times nb_forces_virial on
])
def test_virial_matches_oracle(torch_gpu, name, flags, fl):
    inst = {"tiny": synth.tiny, "diff": synth.diff, "mid": synth.mid}[name]()
    f, e, v = run(torch_gpu, inst, flags, **fl)
    okw = dict(elec=fl.get("elec", 0), vdw=fl.get("vdw", 0), epsilon_rf=fl.get("epsilon_rf", 0.0),
               rswitch=fl.get("rswitch", 0.0))
    ref = O.instance_forces(inst, cells=name != "tiny", **okw)
    rel = frob_rel(v, ref.virial)
    print(f"{name} {okw} virial rel {rel:.2e}\n gpu {np.diag(v)}\n ref {np.diag(ref.virial)}", flush=True)
    fr, elj, ec = compare_forces(f, e, ref, f"{name} virial call")
    assert rel <= VIR_TOL
    assert np.array_equal(v, v.T)
    assert fr <= FORCE_TOL and elj <= ENERGY_TOL
    if fl.get("elec", 0) == 0:
        assert ec <= ENERGY_TOL


def test_virial_includes_the_exclusion_correction(torch_gpu):
    inst = synth.tiny()
    f, e, v = run(torch_gpu, inst, nb.NB_ENERGY_FP64 | nb.NB_EWALD_CORR)
    ref = O.instance_forces(inst)
    fc, e_excl, e_self, vc = O.ewald_corrections(inst.x, inst.q, inst.box, inst.beta,
                                                 inst.coulomb_const, inst.excl_off, inst.excl_idx)
    rel = frob_rel(v, ref.virial + vc)
    print(f"tiny + corrections virial rel {rel:.2e}", flush=True)
    assert rel <= VIR_TOL
    assert abs(e[2] - e_excl) <= 1e-12 * abs(e_excl)
