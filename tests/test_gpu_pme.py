"""Parity of the GPU smooth PME (nb_pme_*) with the FP64 references of oracle/pme.py.

Gates: forces RMS relative <= 5e-6 (the force gate; FP32 output of FP64 sums), energies
relative <= 1e-9 against the FP64 PME reference (both sides FP64: grid, FFT, sums; they differ
by summation order and FFT algorithm only).  End to end, the GPU real-space energy (nb_forces),
self term (NB_EWALD_CORR) and PME energy of a rock-salt crystal reproduce the NaCl Madelung
energy to 1e-6 (the real-space cutoff at beta rc = 4 leaves ~1e-8)."""
import math

import numpy as np
import pytest

from oracle import pme as P
from paper_2405_01420_amd import nb, synth
from tests.gpu_helpers import FORCE_TOL, rel_rms

pytestmark = pytest.mark.gpu

FC = 138.935458
PME_E_TOL = 1e-9


def run_pme(torch, x, q, box, beta, grid, order, fc=FC):
    pm = nb.nb_pme_setup(nb.pme_params(box, beta, fc, grid, order, len(q)))
    dx = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32).reshape(-1)).to("cuda:0")
    dq = torch.from_numpy(np.ascontiguousarray(q, dtype=np.float32)).to("cuda:0")
    f = torch.zeros(len(q) * 3, dtype=torch.float32, device="cuda:0")
    e = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    nb.nb_pme_forces(pm, dx, dq, f, e)
    torch.cuda.synchronize()
    out = f.cpu().numpy().reshape(-1, 3).astype(np.float64), float(e.cpu().numpy()[0])
    nb.nb_pme_destroy(pm)
    return out


def random_system(n=96, L=(2.0, 2.2, 1.9), seed=7):
    rng = np.random.default_rng(seed)
    x = (rng.uniform(-0.5, 1.5, (n, 3)) * np.array(L)).astype(np.float32)  # some outside [0, L)
    q = rng.normal(0.0, 0.8, n)
    q -= q.mean()
    return x, q.astype(np.float32), L


@pytest.mark.parametrize("grid,order", [((20, 24, 28), 4), ((16, 18, 21), 6), ((24, 24, 24), 8),
                                        ((8, 13, 30), 4), ((16, 17, 20), 8)])
def test_pme_matches_fp64_reference(torch_gpu, grid, order):
    x, q, L = random_system()
    beta = 3.0
    f, e = run_pme(torch_gpu, x, q, L, beta, grid, order)
    e0, f0 = P.pme_reference(x.astype(np.float64), q.astype(np.float64), L, beta, FC, grid, order)
    fr, er = rel_rms(f, f0), abs(e - e0) / abs(e0)
    print(f"grid {grid} order {order}: force relRMS {fr:.2e}, energy rel {er:.2e}", flush=True)
    assert fr <= FORCE_TOL and er <= PME_E_TOL


def test_pme_clustered_atoms_and_repeated_calls(torch_gpu):
    """All atoms in a small cube (a few grid tiles hold every atom: several filter passes of
    1024 candidates and several staging passes per tile), then a second call on the same context
    with the atoms spread over the box: both match the reference."""
    torch = torch_gpu
    L, beta, grid, order = (2.0, 2.2, 1.9), 3.0, (20, 24, 18), 4
    rng = np.random.default_rng(11)
    n = 3000
    q = rng.normal(0.0, 0.8, n)
    q = (q - q.mean()).astype(np.float32)
    xa = (0.61 + rng.uniform(0.0, 0.15, (n, 3))).astype(np.float32)
    xb = (rng.uniform(0.0, 1.0, (n, 3)) * np.array(L)).astype(np.float32)
    pm = nb.nb_pme_setup(nb.pme_params(L, beta, FC, grid, order, n))
    dq = torch.from_numpy(q).to("cuda:0")
    for x in (xa, xb):
        dx = torch.from_numpy(x.reshape(-1)).to("cuda:0")
        f = torch.zeros(n * 3, dtype=torch.float32, device="cuda:0")
        e = torch.zeros(1, dtype=torch.float64, device="cuda:0")
        nb.nb_pme_forces(pm, dx, dq, f, e)
        torch.cuda.synchronize()
        e0, f0 = P.pme_reference(x.astype(np.float64), q.astype(np.float64), L, beta, FC, grid, order)
        fr = rel_rms(f.cpu().numpy().reshape(-1, 3).astype(np.float64), f0)
        er = abs(float(e.cpu().numpy()[0]) - e0) / abs(e0)
        print(f"force relRMS {fr:.2e}, energy rel {er:.2e}", flush=True)
        assert fr <= FORCE_TOL and er <= PME_E_TOL
    nb.nb_pme_destroy(pm)


def test_pme_on_the_water_box(torch_gpu):
    inst = synth.tiny()
    grid, order = (20, 20, 20), 4
    f, e = run_pme(torch_gpu, inst.x, inst.q, inst.box, inst.beta, grid, order, inst.coulomb_const)
    e0, f0 = P.pme_reference(inst.x.astype(np.float64), inst.q.astype(np.float64), inst.box, inst.beta,
                             inst.coulomb_const, grid, order)
    fr, er = rel_rms(f, f0), abs(e - e0) / abs(e0)
    print(f"water 648: force relRMS {fr:.2e}, energy rel {er:.2e}", flush=True)
    assert fr <= FORCE_TOL and er <= PME_E_TOL


def test_pme_at_the_benchmark_size(torch_gpu):
    """The configuration bench.py times: the 96,000-atom water box on a 96^3 grid with order-4
    B-splines, every atom and the energy against the FP64 reference."""
    inst = synth.mid()
    grid, order = (96, 96, 96), 4
    f, e = run_pme(torch_gpu, inst.x, inst.q, inst.box, inst.beta, grid, order, inst.coulomb_const)
    e0, f0 = P.pme_reference(inst.x.astype(np.float64), inst.q.astype(np.float64), inst.box, inst.beta,
                             inst.coulomb_const, grid, order)
    fr, er = rel_rms(f, f0), abs(e - e0) / abs(e0)
    print(f"96k atoms, 96^3, order 4: force relRMS {fr:.2e}, energy rel {er:.2e}", flush=True)
    assert fr <= FORCE_TOL and er <= PME_E_TOL


def test_fine_grid_pme_reaches_the_ewald_sum(torch_gpu):
    x, q, L = random_system(n=48)
    beta = 3.0
    f, e = run_pme(torch_gpu, x, q, L, beta, (48, 52, 46), 8)
    e0, f0 = P.ewald_recip_direct(x.astype(np.float64), q.astype(np.float64), L, beta, FC)
    fr, er = rel_rms(f, f0), abs(e - e0) / abs(e0)
    print(f"fine grid vs direct Ewald sum: force relRMS {fr:.2e}, energy rel {er:.2e}", flush=True)
    assert fr <= 1e-6 and er <= 1e-7


def test_rock_salt_madelung_energy_end_to_end(torch_gpu):
    """GPU real space + self term + PME of 512 unit charges on a rock-salt lattice."""
    torch = torch_gpu
    a, nc = 0.5, 4
    s = 2 * nc
    idx = np.stack(np.meshgrid(np.arange(s), np.arange(s), np.arange(s), indexing="ij"), -1).reshape(-1, 3)
    x = ((idx + 0.25) * (a / 2.0)).astype(np.float32)
    q = np.where(idx.sum(1) % 2 == 0, 1.0, -1.0).astype(np.float32)
    L, rc = nc * a, 0.99
    beta = 4.0 / rc
    n = len(q)
    params = nb.Params(n, [L] * 3, rc, 0.0, beta, FC, [0.0], [0.0],
                       flags=nb.NB_ENERGY_FP64 | nb.NB_EWALD_CORR)
    ctx = nb.nb_setup(params)
    dx = torch.from_numpy(x.reshape(-1).copy()).to("cuda:0")
    dq = torch.from_numpy(q).to("cuda:0")
    dt = torch.zeros(n, dtype=torch.int32, device="cuda:0")
    f = torch.zeros(3 * n, dtype=torch.float32, device="cuda:0")
    e = torch.zeros(4, dtype=torch.float64, device="cuda:0")
    nb.nb_pairlist(ctx, dx)
    nb.nb_forces(ctx, dx, dq, dt, f, e)
    torch.cuda.synchronize()
    er = e.cpu().numpy()
    nb.nb_destroy(ctx)
    _, e_rec = run_pme(torch, x, q, L, beta, (64, 64, 64), 8)
    total = er[1] + er[2] + er[3] + e_rec
    ref = -0.5 * n * 1.747564594633182 * FC / (a / 2.0)
    print(f"real {er[1]:.6f} excl {er[2]:.3e} self {er[3]:.6f} recip {e_rec:.6f} total {total:.8f} "
          f"Madelung {ref:.8f} rel {abs(total - ref) / abs(ref):.2e}", flush=True)
    assert abs(total - ref) <= 1e-6 * abs(ref)
