"""Parity of the reaction-field and force-switch flavours of the HIP path (through the C-ABI)
with the FP64 oracle: forces RMS relative <= 5e-6, energies relative <= 1e-6 per component.

Energies: the reaction-field pair terms do not decay towards rc (1/r + k_rf r^2 - c_rf), so the
Coulomb energy, a sum with |E_C| / sum |E_C,ij| ~ 1e-4, carries FP32 rounding noise of order
1e-6 even at 96k atoms; with FP32 pair energies it is held to the FP32 bound (1e-5) and the 1e-6
gate is checked in the FP64 pair-energy mode (NB_ENERGY_FP64), as for Ewald on small boxes.
Forces: with a finite eps_rf the reaction-field force does not vanish at rc, so a pair that the
FP32 and FP64 cutoff tests place on different sides of rc moves the force by a visible step; the
parity gates use eps_rf = infinity (force zero at rc) and a finite eps_rf is checked on the
648-atom box, which has no pair that close to rc."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2405_01420_amd import nb, synth
from tests.gpu_helpers import (ENERGY_TOL, FORCE_TOL, FP32_SMALL_BOX_EC_TOL, GpuBox,
                               compare_forces, rel_rms)

pytestmark = pytest.mark.gpu

FLAVOURS = {
    "rf": dict(elec=nb.NB_ELEC_RF, epsilon_rf=0.0),
    "rf-fsw": dict(elec=nb.NB_ELEC_RF, epsilon_rf=0.0, vdw=nb.NB_VDW_FSWITCH, rswitch=0.8),
    "ewald-fsw": dict(vdw=nb.NB_VDW_FSWITCH, rswitch=0.8),
}


def oracle_kw(fl):
    return dict(elec=fl.get("elec", 0), vdw=fl.get("vdw", 0), epsilon_rf=fl.get("epsilon_rf", 0.0),
                rswitch=fl.get("rswitch", 0.0))


def ec_gate(fl, flags, small):
    """The E_C bound: 1e-6 with FP64 pair energies; the FP32 bound for the reaction field and
    for Ewald on the 648-atom box."""
    if flags & nb.NB_ENERGY_FP64:
        return ENERGY_TOL
    if fl.get("elec", 0) == nb.NB_ELEC_RF or small:
        return FP32_SMALL_BOX_EC_TOL
    return ENERGY_TOL


@pytest.fixture(scope="module")
def inst_diff():
    return synth.diff()


@pytest.mark.parametrize("name", list(FLAVOURS))
@pytest.mark.parametrize("cluster", [8, 4])
@pytest.mark.parametrize("flags", [0, nb.NB_ENERGY_FP64])
def test_tiny_flavours(torch_gpu, name, cluster, flags):
    inst = synth.tiny()
    fl = dict(FLAVOURS[name])
    if "rswitch" in fl:
        fl["rswitch"] = 0.7  # rc = 0.9 here
    box = GpuBox(torch_gpu, inst, cluster=cluster, flags=flags, **fl)
    box.pairlist()
    f, e = box.forces()
    box.close()
    ref = O.instance_forces(inst, **oracle_kw(fl))
    fr, elj, ec = compare_forces(f, e, ref, f"tiny {name} C={cluster} flags={flags}")
    assert fr <= FORCE_TOL and elj <= ENERGY_TOL and ec <= ec_gate(fl, flags, True)


def test_tiny_rf_finite_dielectric(torch_gpu):
    inst = synth.tiny()
    fl = dict(elec=nb.NB_ELEC_RF, epsilon_rf=78.0, vdw=nb.NB_VDW_FSWITCH, rswitch=0.7)
    box = GpuBox(torch_gpu, inst, flags=nb.NB_ENERGY_FP64, **fl)
    box.pairlist()
    f, e = box.forces()
    box.close()
    ref = O.instance_forces(inst, **oracle_kw(fl))
    fr, elj, ec = compare_forces(f, e, ref, "tiny rf78-fsw")
    assert fr <= FORCE_TOL and elj <= ENERGY_TOL and ec <= ENERGY_TOL


@pytest.mark.parametrize("name", list(FLAVOURS))
@pytest.mark.parametrize("flags", [0, nb.NB_ENERGY_FP64])
def test_diff_flavours(torch_gpu, inst_diff, name, flags):
    """24,000 atoms, four LJ types, perturbed charges."""
    fl = FLAVOURS[name]
    box = GpuBox(torch_gpu, inst_diff, flags=flags, **fl)
    box.pairlist()
    f, e = box.forces()
    box.close()
    ref = O.instance_forces(inst_diff, cells=True, **oracle_kw(fl))
    fr, elj, ec = compare_forces(f, e, ref, f"diff {name} flags={flags}")
    assert fr <= FORCE_TOL and elj <= ENERGY_TOL and ec <= ec_gate(fl, flags, False)


@pytest.mark.parametrize("flags", [0, nb.NB_ENERGY_FP64])
def test_mid_rf_force_switch(torch_gpu, flags):
    inst = synth.mid()
    fl = FLAVOURS["rf-fsw"]
    box = GpuBox(torch_gpu, inst, flags=flags, **fl)
    box.pairlist()
    f, e = box.forces()
    box.close()
    ref = O.instance_forces(inst, cells=True, **oracle_kw(fl))
    fr, elj, ec = compare_forces(f, e, ref, f"mid rf-fsw flags={flags}")
    assert fr <= FORCE_TOL and elj <= ENERGY_TOL and ec <= ec_gate(fl, flags, False)


def test_batch_flavour_matches_oracle(torch_gpu):
    torch = torch_gpu
    boxes = synth.batch(6, sizes=[3000, 4503, 7500, 9999, 14001, 21000])
    fl = FLAVOURS["rf-fsw"]
    ao, bx, params, x, q, t = nb.concat_instances(boxes, flags=nb.NB_ENERGY_FP64, **fl)
    stream = torch.cuda.Stream()
    bt = nb.nb_batch_setup(ao, bx, params, stream=stream.cuda_stream)
    with torch.cuda.stream(stream):
        dx = torch.from_numpy(x.reshape(-1)).to("cuda:0")
        dq = torch.from_numpy(q).to("cuda:0")
        dt = torch.from_numpy(t).to("cuda:0")
        f = torch.zeros(len(q) * 3, dtype=torch.float32, device="cuda:0")
        e = torch.zeros(2 * len(boxes), dtype=torch.float64, device="cuda:0")
    stream.synchronize()
    nb.nb_batch_pairlist(bt, dx)
    nb.nb_batch_forces(bt, dx, dq, dt, f, e)
    stream.synchronize()
    fa = f.cpu().numpy().reshape(-1, 3).astype(np.float64)
    ea = e.cpu().numpy().reshape(-1, 2)
    nb.nb_batch_destroy(bt)
    for k, inst in enumerate(boxes):
        ref = O.instance_forces(inst, cells=True, **oracle_kw(fl))
        fr = rel_rms(fa[ao[k]:ao[k + 1]], ref.f)
        elj = abs(ea[k, 0] - ref.e_lj) / abs(ref.e_lj)
        ec = abs(ea[k, 1] - ref.e_coul) / abs(ref.e_coul)
        print(f"batch box {k} n={inst.natoms} f {fr:.2e} elj {elj:.2e} ec {ec:.2e}", flush=True)
        assert fr <= FORCE_TOL and elj <= ENERGY_TOL and ec <= ENERGY_TOL


def test_backward_rejects_other_flavours(torch_gpu):
    torch = torch_gpu
    inst = synth.tiny()
    box = GpuBox(torch, inst, **FLAVOURS["rf"])
    n = inst.natoms
    z3 = torch.zeros(3 * n, dtype=torch.float32, device="cuda:0")
    z1 = torch.zeros(n, dtype=torch.float32, device="cuda:0")
    ge = torch.zeros(2, dtype=torch.float64, device="cuda:0")
    dt = torch.zeros(inst.ntypes, dtype=torch.float64, device="cuda:0")
    with pytest.raises(nb.NbError) as ei:
        nb.nb_backward(box.ctx, box.x, box.q, box.t, z3, ge, z3.clone(), z1, dt, dt.clone())
    assert ei.value.code == nb.NB_ERR_ARG
    box.close()


@pytest.mark.parametrize("which", ["tiny", "diff", "mid"])
@pytest.mark.parametrize("vdw", [nb.NB_VDW_SHIFT, nb.NB_VDW_FSWITCH])
def test_tabulated_ewald_matches_oracle(torch_gpu, which, vdw):
    """NB_ELEC_EWALD_TAB: the Ewald real-space force from the FP32 table of its smooth part, the
    pair energies in FP64; the same interaction as the analytic flavour, so the oracle's Ewald
    definition is the reference (forces 5e-6, both energies 1e-6, also on the 648-atom box)."""
    inst = getattr(synth, which)()
    rsw = inst.cutoff - 0.2 if vdw == nb.NB_VDW_FSWITCH else 0.0
    box = GpuBox(torch_gpu, inst, elec=nb.NB_ELEC_EWALD_TAB, vdw=vdw, rswitch=rsw)
    box.pairlist()
    f, e = box.forces()
    box.close()
    ref = O.instance_forces(inst, vdw=vdw, rswitch=rsw)
    fr, elj, ec = compare_forces(f, e, ref, f"{which} tabulated Ewald vdw={vdw}")
    assert fr <= FORCE_TOL and elj <= ENERGY_TOL and ec <= ENERGY_TOL


def test_tabulated_ewald_rejected_where_not_built(torch_gpu):
    inst = synth.tiny()
    params = nb.Params.from_instance(inst, elec=nb.NB_ELEC_EWALD_TAB)
    ctx = nb.nb_setup(params)
    box = GpuBox(torch_gpu, inst, elec=nb.NB_ELEC_EWALD_TAB)
    box.pairlist()
    z = torch_gpu.zeros(3 * inst.natoms, dtype=torch_gpu.float32, device="cuda:0")
    with pytest.raises(nb.NbError) as ei:
        nb.nb_backward(box.ctx, box.x, box.q, box.t, z, box.e, z, z[:inst.natoms], box.e, box.e,
                       nb.NB_REUSE_LIST)
    assert ei.value.code == nb.NB_ERR_ARG
    box.close()
    nb.nb_destroy(ctx)
    insts = synth.batch(2, sizes=[3000, 3600])
    ao, bx, p, x, q, t = nb.concat_instances(insts, elec=nb.NB_ELEC_EWALD_TAB)
    with pytest.raises(nb.NbError) as ei:
        nb.nb_batch_setup(ao, bx, p)
    assert ei.value.code == nb.NB_ERR_ARG
