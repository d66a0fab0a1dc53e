"""Molecular dynamics around the force path (nb_md_leapfrog): leapfrog steps of a charged
Lennard-Jones fluid (4,096 ions of charge +-0.5 e at water-oxygen density, 300 K, dt 2 fs) with
the pair list rebuilt every 10 steps and the rolling prune to rc + 0.04 nm every 2 steps between
builds.  At sampled steps the forces and energies the loop computed are checked against the FP64
oracle at the positions of that step (forces RMS relative <= 5e-6, energies <= 1e-6, FP64 pair
energies); the total energy stays put over the run; the displacement check never fires."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2405_01420_amd import nb, synth
from tests.gpu_helpers import ENERGY_TOL, FORCE_TOL, rel_rms

pytestmark = pytest.mark.gpu

DT = 0.002


def setup_md(torch, inst, v0, im, flags):
    params = nb.Params.from_instance(inst, flags=flags)
    ctx = nb.nb_setup(params)
    dev = "cuda:0"
    x = torch.from_numpy(inst.x.reshape(-1).copy()).to(dev)
    v = torch.from_numpy(v0.reshape(-1).copy()).to(dev)
    q = torch.from_numpy(inst.q.copy()).to(dev)
    t = torch.from_numpy(inst.type.copy()).to(dev)
    m = torch.from_numpy(im.copy()).to(dev)
    f = torch.zeros(3 * inst.natoms, dtype=torch.float32, device=dev)
    return ctx, x, v, q, t, m, f


@pytest.mark.parametrize("prune", [True, False])
def test_md_steps_match_oracle(torch_gpu, prune):
    torch = torch_gpu
    inst, v0, im = synth.ionic_fluid(4096, 4.96)
    flags = nb.NB_ENERGY_FP64 | nb.NB_CHECK_STALE | nb.NB_ASYNC_BUILD
    ctx, x, v, q, t, m, f = setup_md(torch, inst, v0, im, flags)
    rin = inst.cutoff + 0.04 if prune else 0.0
    etot = []
    for chunk in range(4):
        e = torch.zeros((50, 4), dtype=torch.float64, device="cuda:0")
        nb.nb_md_leapfrog(ctx, x, v, q, t, m, DT, 50, 10, f, e, r_inner=rin, nstprune=2)
        xs = x.cpu().numpy().reshape(-1, 3).astype(np.float64)   # positions of the next step
        e1 = torch.zeros((1, 4), dtype=torch.float64, device="cuda:0")
        nb.nb_md_leapfrog(ctx, x, v, q, t, m, DT, 1, 10, f, e1, r_inner=rin, nstprune=2)
        torch.cuda.synchronize()
        etot.append(e.cpu().numpy()[:, 3])
        etot.append(e1.cpu().numpy()[:, 3])
        ref = O.instance_forces(inst, x=xs, cells=True)
        fg = f.cpu().numpy().reshape(-1, 3).astype(np.float64)
        eg = e1.cpu().numpy()[0]
        fr = rel_rms(fg, ref.f)
        elj = abs(eg[0] - ref.e_lj) / abs(ref.e_lj)
        ec = abs(eg[1] - ref.e_coul) / abs(ref.e_coul)
        print(f"step {51 * (chunk + 1) - 1}: force relRMS {fr:.2e} E_LJ {elj:.2e} E_C {ec:.2e}", flush=True)
        assert fr <= FORCE_TOL and elj <= ENERGY_TOL and ec <= ENERGY_TOL
    assert nb.nb_check(ctx) == nb.NB_OK
    etot = np.concatenate(etot)
    ke0 = float(e.cpu().numpy()[0, 2])
    drift = float(etot.max() - etot.min())
    print(f"total energy spread over {len(etot)} steps: {drift:.4f} kJ/mol (kinetic {ke0:.1f})", flush=True)
    assert np.all(np.isfinite(etot))
    assert drift <= 2e-3 * ke0
    nb.nb_destroy(ctx)


def test_md_pruned_and_full_lists_agree(torch_gpu):
    """The rolling prune changes only which listed pairs beyond r_inner are carried: the same
    trajectory to the force gate after 30 steps."""
    torch = torch_gpu
    inst, v0, im = synth.ionic_fluid(4096, 4.96)
    out = []
    for rin in (inst.cutoff + 0.04, 0.0):
        ctx, x, v, q, t, m, f = setup_md(torch, inst, v0, im, nb.NB_CHECK_STALE)
        e = torch.zeros((30, 4), dtype=torch.float64, device="cuda:0")
        nb.nb_md_leapfrog(ctx, x, v, q, t, m, DT, 30, 10, f, e, r_inner=rin, nstprune=2)
        torch.cuda.synchronize()
        assert nb.nb_check(ctx) == nb.NB_OK
        out.append((x.cpu().numpy().astype(np.float64), f.cpu().numpy().astype(np.float64)))
        nb.nb_destroy(ctx)
    assert np.abs(out[0][0] - out[1][0]).max() <= 1e-5
    assert rel_rms(out[0][1], out[1][1]) <= FORCE_TOL


def test_md_rejects_bad_arguments(torch_gpu):
    torch = torch_gpu
    inst, v0, im = synth.ionic_fluid(512, 2.48)
    ctx, x, v, q, t, m, f = setup_md(torch, inst, v0, im, 0)
    e = torch.zeros((4, 4), dtype=torch.float64, device="cuda:0")
    for kw in (dict(dt=-0.001, nsteps=4, nstlist=10), dict(dt=DT, nsteps=4, nstlist=0),
               dict(dt=DT, nsteps=4, nstlist=10, r_inner=inst.cutoff - 0.01)):
        with pytest.raises(nb.NbError) as ei:
            nb.nb_md_leapfrog(ctx, x, v, q, t, m, kw["dt"], kw["nsteps"], kw["nstlist"], f, e,
                              r_inner=kw.get("r_inner", 0.0), nstprune=2)
        assert ei.value.code == nb.NB_ERR_ARG
    nb.nb_destroy(ctx)
