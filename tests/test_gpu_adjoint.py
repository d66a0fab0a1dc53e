"""GPU adjoint (nb_backward and the autograd Function) against the oracle's analytic VJP and
FP64 central differences of the oracle loss, on the 24,000-atom gradient workload (4 LJ types
on O, charges perturbed and re-neutralised per molecule, targets from the oracle at parameters
perturbed by 2%).

G1: fixed cotangents (the oracle's, rounded to FP32) -> dx, dq relative RMS <= 5e-6; each dsigma,
    deps relative <= 5e-6.
G2: end-to-end loss gradient through torch.autograd (cotangents from the GPU's own forces)
    against FP64 central differences of the oracle loss on 64 coordinates, 64 charges and all LJ
    parameters: relative <= 1e-3 (the 5e-6 force error is amplified ~50x in F - F_target)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2405_01420_amd import nb, synth
from tests.gpu_helpers import GpuBox, dev, rel_rms

pytestmark = pytest.mark.gpu

G1_TOL = 5e-6
G2_TOL = 1e-3


@pytest.fixture(scope="module")
def problem():
    inst = synth.diff()
    sig_t, eps_t, q_t = synth.perturbed_params(inst, 0.02, seed=6)
    tgt = O.forces(inst.x, q_t, inst.type, sig_t, eps_t, inst.box, inst.cutoff, inst.beta,
                   inst.coulomb_const, inst.excl_off, inst.excl_idx, cells=True, round32=False)
    f_t, e_t = tgt.f, tgt.e_lj + tgt.e_coul
    L0, r0 = O.loss(inst, inst.x, inst.q, inst.sigma, inst.epsilon, f_t, e_t, cells=True)
    gF = (2.0 * (r0.f - f_t)).astype(np.float32)
    s = 2.0 * ((r0.e_lj + r0.e_coul) - e_t)
    gE = np.array([s, s])
    vjp = O.vjp(inst.x, inst.q, inst.type, inst.sigma, inst.epsilon, inst.box, inst.cutoff,
                inst.beta, inst.coulomb_const, inst.excl_off, inst.excl_idx,
                gF.astype(np.float64), gE)
    return dict(inst=inst, f_t=f_t, e_t=e_t, gF=gF, gE=gE, vjp=vjp)


@pytest.mark.parametrize("cluster", [8, 4])
def test_adjoint_fixed_cotangents(torch_gpu, problem, cluster):
    torch = torch_gpu
    inst = problem["inst"]
    box = GpuBox(torch, inst, cluster=cluster)
    gf = dev(torch, problem["gF"].reshape(-1))
    ge = dev(torch, problem["gE"])
    dx = torch.empty(inst.natoms * 3, dtype=torch.float32, device="cuda:0")
    dq = torch.empty(inst.natoms, dtype=torch.float32, device="cuda:0")
    ds = torch.empty(inst.ntypes, dtype=torch.float64, device="cuda:0")
    de = torch.empty(inst.ntypes, dtype=torch.float64, device="cuda:0")
    nb.nb_backward(box.ctx, box.x, box.q, box.t, gf, ge, dx, dq, ds, de, 0)
    torch.cuda.synchronize()
    rdx, rdq, rds, rde = problem["vjp"]
    ex = rel_rms(dx.cpu().numpy().reshape(-1, 3).astype(np.float64), rdx)
    eq = rel_rms(dq.cpu().numpy().astype(np.float64), rdq)
    ds_, de_ = ds.cpu().numpy(), de.cpu().numpy()
    print(f"C={cluster} dx relRMS {ex:.2e} dq relRMS {eq:.2e}")
    present = np.unique(inst.type)
    for t in range(inst.ntypes):
        if t not in present or inst.epsilon[t] == 0.0:
            assert abs(de_[t]) == 0.0 or inst.epsilon[t] > 0.0
            continue
        es = abs(ds_[t] - rds[t]) / abs(rds[t])
        ee = abs(de_[t] - rde[t]) / abs(rde[t])
        print(f"  type {t}: dsigma rel {es:.2e}  deps rel {ee:.2e}")
        assert es <= G1_TOL and ee <= G1_TOL
    box.close()
    assert ex <= G1_TOL and eq <= G1_TOL


def test_autograd_end_to_end_vs_finite_differences(torch_gpu, problem):
    torch = torch_gpu
    from paper_2405_01420_amd.autograd import nonbonded
    inst = problem["inst"]
    params = nb.Params.from_instance(inst)
    ctx = nb.nb_setup(params)
    x = torch.tensor(inst.x, device="cuda:0", requires_grad=True)
    q = torch.tensor(inst.q, device="cuda:0", requires_grad=True)
    sig = torch.tensor(inst.sigma, device="cuda:0", requires_grad=True)
    eps = torch.tensor(inst.epsilon, device="cuda:0", requires_grad=True)
    types = torch.tensor(inst.type, device="cuda:0")
    f_t = torch.tensor(problem["f_t"], dtype=torch.float64, device="cuda:0")
    F, elj, ec = nonbonded(x, q, sig, eps, types, ctx)
    loss = ((F.double() - f_t) ** 2).sum() + (elj + ec - problem["e_t"]) ** 2
    loss.backward()
    torch.cuda.synchronize()
    gx = x.grad.cpu().numpy().astype(np.float64)
    gq = q.grad.cpu().numpy().astype(np.float64)
    gs = sig.grad.cpu().numpy()
    ge = eps.grad.cpu().numpy()
    nb.nb_destroy(ctx)

    def oloss(xv, qv, sv, ev):
        L, _ = O.loss(inst, xv, qv, sv, ev, problem["f_t"], problem["e_t"], cells=True)
        return L

    from tests.fd_local import loss_difference, neighbours
    x0 = inst.x.astype(np.float64)
    q0 = inst.q.astype(np.float64)
    r0 = O.loss(inst, x0, q0, inst.sigma, inst.epsilon, problem["f_t"], problem["e_t"], cells=True)[1]
    e0 = r0.e_lj + r0.e_coul
    rng = np.random.default_rng(7)
    worst = 0.0
    n_checked = 0
    rmsx = np.sqrt(np.mean(gx ** 2))
    for a in rng.permutation(inst.natoms):
        _, r = neighbours(inst, x0, a)
        if np.any(np.abs(r - inst.cutoff) < 1e-4):
            continue
        c = int(rng.integers(3))
        if abs(gx[a, c]) < 1e-2 * rmsx:
            continue
        fd = loss_difference(inst, x0, q0, e0, problem["f_t"], problem["e_t"], a, c)
        worst = max(worst, abs(gx[a, c] - fd) / abs(fd))
        n_checked += 1
        if n_checked == 64:
            break
    print(f"dx vs FD worst rel over {n_checked} coordinates", worst)
    assert n_checked == 64 and worst <= G2_TOL
    worst = 0.0
    rmsq = np.sqrt(np.mean(gq ** 2))
    for a in rng.permutation(inst.natoms)[:64]:
        fd = loss_difference(inst, x0, q0, e0, problem["f_t"], problem["e_t"], a)
        worst = max(worst, abs(gq[a] - fd) / max(abs(fd), 1e-3 * rmsq))
    print("dq vs FD worst rel over 64 charges", worst)
    assert worst <= G2_TOL
    for t in np.unique(inst.type):
        if inst.epsilon[t] == 0.0:
            continue
        for arr, g, nm in ((inst.sigma, gs, "sigma"), (inst.epsilon, ge, "eps")):
            hp = 1e-6 * arr[t]
            ap, am = arr.copy(), arr.copy()
            ap[t] += hp
            am[t] -= hp
            if nm == "sigma":
                fd = (oloss(x0, q0, ap, inst.epsilon) - oloss(x0, q0, am, inst.epsilon)) / (2 * hp)
            else:
                fd = (oloss(x0, q0, inst.sigma, ap) - oloss(x0, q0, inst.sigma, am)) / (2 * hp)
            rel = abs(g[t] - fd) / abs(fd)
            print(f"d{nm}[{t}] gpu {g[t]:.6e} fd {fd:.6e} rel {rel:.2e}")
            assert rel <= G2_TOL


def test_adjoint_on_a_pruned_list(torch_gpu, problem):
    """nb_backward with NB_REUSE_LIST on a list pruned by nb_prune (the pairs within rc are the
    same, so the VJP matches the oracle's to the G1 bound)."""
    torch = torch_gpu
    inst = problem["inst"]
    box = GpuBox(torch, inst)
    box.pairlist()
    nb.nb_prune(box.ctx, box.x, inst.cutoff + 0.02)
    assert box.stats()["pruned"] == 1
    gf = dev(torch, problem["gF"].reshape(-1))
    ge = dev(torch, problem["gE"])
    dx = torch.empty(inst.natoms * 3, dtype=torch.float32, device="cuda:0")
    dq = torch.empty(inst.natoms, dtype=torch.float32, device="cuda:0")
    ds = torch.empty(inst.ntypes, dtype=torch.float64, device="cuda:0")
    de = torch.empty(inst.ntypes, dtype=torch.float64, device="cuda:0")
    nb.nb_backward(box.ctx, box.x, box.q, box.t, gf, ge, dx, dq, ds, de, nb.NB_REUSE_LIST)
    torch.cuda.synchronize()
    rdx, rdq, _, _ = problem["vjp"]
    ex = rel_rms(dx.cpu().numpy().reshape(-1, 3).astype(np.float64), rdx)
    eq = rel_rms(dq.cpu().numpy().astype(np.float64), rdq)
    print(f"pruned list: dx relRMS {ex:.2e} dq relRMS {eq:.2e}")
    box.close()
    assert ex <= G1_TOL and eq <= G1_TOL
