"""The smallest systems the method accepts, through the C-ABI: one atom (no pair: zero forces and
energies, an empty pair set), two atoms inside the cutoff (directly and across a periodic face),
two atoms beyond it, an excluded pair, and a pair whose type has no Lennard-Jones term and no
charge.  Such boxes leave most columns of the grid empty and hold a single cluster.  Forces and
energies are compared with the oracle (interacting pairs) or are exactly zero (no pair).  Also
the limits the library states: a grid column of the largest size the build sorts (and one atom
more, reported as an overflow) and the largest LJ type table."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2405_01420_amd import nb, synth
from tests.gpu_helpers import ENERGY_TOL, FORCE_TOL, FP32_SMALL_BOX_EC_TOL, GpuBox, dev, rel_rms

pytestmark = pytest.mark.gpu

L, RC, RB = 2.5, 0.9, 0.1
SIGMA = np.array([0.3166, 0.0])   # an oxygen-like type and a null type (no LJ)
EPS = np.array([0.65, 0.0])


def make(x, q, types, excl=()):
    n = len(q)
    partners = [[] for _ in range(n)]
    for a, b in excl:
        partners[a].append(b)
        partners[b].append(a)
    off = np.zeros(n + 1, dtype=np.int32)
    off[1:] = np.cumsum([len(p) for p in partners])
    idx = np.array([b for p in partners for b in sorted(p)], dtype=np.int32)
    return synth.Instance(x=np.asarray(x, dtype=np.float32).reshape(n, 3),
                          q=np.asarray(q, dtype=np.float32), type=np.asarray(types, dtype=np.int32),
                          box=synth.f32(L), cutoff=synth.f32(RC), buffer=synth.f32(RB),
                          beta=synth.ewald_beta(RC), coulomb_const=synth.f32(138.935458),
                          sigma=SIGMA.copy(), epsilon=EPS.copy(), excl_off=off, excl_idx=idx,
                          name="degenerate")


CASES = {
    "one_atom": (make([[1.2, 0.7, 2.1]], [0.8], [0]), False),
    "pair_inside": (make([[0.6, 1.1, 1.3], [1.05, 1.3, 1.5]], [0.8, -0.8], [0, 0]), True),
    "pair_across_face": (make([[0.1, 1.2, 0.8], [2.25, 1.3, 0.7]], [0.8, -0.4], [0, 0]), True),
    "pair_beyond_cutoff": (make([[0.3, 0.3, 0.3], [1.25, 0.3, 0.3]], [0.8, -0.8], [0, 0]), False),
    "pair_excluded": (make([[0.6, 1.1, 1.3], [0.7, 1.1, 1.3]], [0.8, -0.8], [0, 0], excl=[(0, 1)]),
                      False),
    "pair_null_type": (make([[0.6, 1.1, 1.3], [0.9, 1.2, 1.3]], [0.0, 0.0], [1, 1]), False),
}


@pytest.mark.parametrize("cluster", [8, 4])
@pytest.mark.parametrize("flags", [0, nb.NB_ENERGY_FP64])
@pytest.mark.parametrize("name", list(CASES))
def test_smallest_systems(torch_gpu, name, cluster, flags):
    inst, interacting = CASES[name]
    print(f"case {name} C={cluster} flags={flags}", flush=True)
    box = GpuBox(torch_gpu, inst, cluster=cluster, flags=flags)
    try:
        box.pairlist()
        f, e = box.forces()
        pairs = np.asarray(box.pairs(), dtype=np.int64).reshape(-1, 2)
        assert nb.nb_check(box.ctx) == nb.NB_OK
    finally:
        box.close()
    pi, pj, _ = O.pairs(inst.x, inst.box, inst.cutoff, inst.excl_off, inst.excl_idx)
    assert sorted(map(tuple, pairs.tolist())) == sorted(zip(pi.tolist(), pj.tolist()))
    if not interacting:   # (the null-type pair is in the pair set, with zero force and energy)
        assert np.all(f == 0.0) and e[0] == 0.0 and e[1] == 0.0
        return
    ref = O.instance_forces(inst, cells=False)
    fr = rel_rms(f, ref.f)
    elj = abs(e[0] - ref.e_lj) / abs(ref.e_lj)
    ec = abs(e[1] - ref.e_coul) / abs(ref.e_coul)
    print(f"force relRMS {fr:.2e} E_LJ rel {elj:.2e} E_C rel {ec:.2e}", flush=True)
    assert fr <= FORCE_TOL and elj <= ENERGY_TOL and ec <= ENERGY_TOL
    assert np.abs(f.sum(0)).max() <= 1e-6 * np.abs(f).max()  # the two forces cancel


@pytest.mark.parametrize("graph", [False, True])
def test_smallest_systems_in_a_batch(torch_gpu, graph):
    """The same boxes between two water boxes in one batched launch (FP64 pair energies, the
    mode gated at 1e-6 on small boxes): each box's forces and energies against the oracle, or
    exactly zero where it has no interacting pair."""
    torch = torch_gpu
    water = [synth.small_box(300, RC, RB, 5), synth.small_box(400, RC, RB, 6)]
    insts = [water[0]] + [CASES[k][0] for k in CASES] + [water[1]]
    interacting = [True] + [CASES[k][1] for k in CASES] + [True]
    assert all(np.array_equal(i.sigma, SIGMA) and np.array_equal(i.epsilon, EPS) and i.beta == insts[0].beta
               for i in insts)
    print(f"batch of {len(insts)} boxes, graph={graph}", flush=True)
    ao, bx, params, x, q, t = nb.concat_instances(insts, clusters=[8] * len(insts), flags=nb.NB_ENERGY_FP64)
    stream = torch.cuda.Stream()
    bt = nb.nb_batch_setup(ao, bx, params, clusters=[8] * len(insts), stream=stream.cuda_stream)
    try:
        with torch.cuda.stream(stream):
            dx = torch.from_numpy(x.reshape(-1)).to("cuda:0")
            dq = torch.from_numpy(q).to("cuda:0")
            dt = torch.from_numpy(t).to("cuda:0")
            f = torch.zeros(len(q) * 3, dtype=torch.float32, device="cuda:0")
            e = torch.zeros(2 * len(insts), dtype=torch.float64, device="cuda:0")
        stream.synchronize()
        nb.nb_batch_pairlist(bt, dx)
        for _ in range(2):
            (nb.nb_batch_graph_forces if graph else nb.nb_batch_forces)(bt, dx, dq, dt, f, e)
        stream.synchronize()
        assert nb.nb_batch_check(bt) == nb.NB_OK
        fa = f.cpu().numpy().reshape(-1, 3).astype(np.float64)
        ea = e.cpu().numpy().reshape(-1, 2)
    finally:
        nb.nb_batch_destroy(bt)
    for k, inst in enumerate(insts):
        fk, ek = fa[ao[k]:ao[k + 1]], ea[k]
        if not interacting[k]:
            assert np.all(fk == 0.0) and ek[0] == 0.0 and ek[1] == 0.0, k
            continue
        ref = O.instance_forces(inst, cells=False)
        fr = rel_rms(fk, ref.f)
        elj = abs(ek[0] - ref.e_lj) / abs(ref.e_lj)
        ec = abs(ek[1] - ref.e_coul) / abs(ref.e_coul)
        print(f"box {k} n={inst.natoms} force relRMS {fr:.2e} E_LJ rel {elj:.2e} E_C rel {ec:.2e}", flush=True)
        assert fr <= FORCE_TOL and elj <= ENERGY_TOL and ec <= ENERGY_TOL, k


@pytest.mark.parametrize("name", list(CASES))
def test_smallest_systems_backward(torch_gpu, name):
    """The adjoint on the same boxes with seeded cotangents: dx, dq and the LJ-parameter
    gradients of the oracle's analytic VJP (relative <= 5e-6), or exactly zero without an
    interacting pair (also for the null-type pair, whose terms all carry a zero factor)."""
    torch = torch_gpu
    inst, interacting = CASES[name]
    print(f"case {name}", flush=True)
    rng = np.random.default_rng(11)
    gF = rng.standard_normal((inst.natoms, 3)).astype(np.float32)
    gE = np.array([0.7, -1.3])
    box = GpuBox(torch, inst)
    try:
        gf, ge = dev(torch, gF.reshape(-1)), dev(torch, gE)
        dx = torch.empty(inst.natoms * 3, dtype=torch.float32, device="cuda:0")
        dq = torch.empty(inst.natoms, dtype=torch.float32, device="cuda:0")
        ds = torch.empty(inst.ntypes, dtype=torch.float64, device="cuda:0")
        de = torch.empty(inst.ntypes, dtype=torch.float64, device="cuda:0")
        nb.nb_backward(box.ctx, box.x, box.q, box.t, gf, ge, dx, dq, ds, de, 0)
        torch.cuda.synchronize()
        assert nb.nb_check(box.ctx) == nb.NB_OK
        gx = dx.cpu().numpy().reshape(-1, 3).astype(np.float64)
        gq = dq.cpu().numpy().astype(np.float64)
        gs, ge_ = ds.cpu().numpy(), de.cpu().numpy()
    finally:
        box.close()
    if not interacting:
        assert np.all(gx == 0.0) and np.all(gq == 0.0) and np.all(gs == 0.0) and np.all(ge_ == 0.0)
        return
    rdx, rdq, rds, rde = O.vjp(inst.x, inst.q, inst.type, inst.sigma, inst.epsilon, inst.box,
                               inst.cutoff, inst.beta, inst.coulomb_const, inst.excl_off,
                               inst.excl_idx, gF.astype(np.float64), gE)
    ex, eq = rel_rms(gx, rdx), rel_rms(gq, rdq)
    es, ee = abs(gs[0] - rds[0]) / abs(rds[0]), abs(ge_[0] - rde[0]) / abs(rde[0])
    print(f"dx {ex:.2e} dq {eq:.2e} dsigma {es:.2e} deps {ee:.2e}", flush=True)
    assert ex <= FORCE_TOL and eq <= FORCE_TOL and es <= FORCE_TOL and ee <= FORCE_TOL
    assert gs[1] == 0.0 and ge_[1] == 0.0   # the null type has no pair here


def column_stack(n):
    """n atoms of the null type, uncharged, stacked along z in one grid column of a 20 nm box
    (the grid's column width there is 2.5 nm), 20 / n nm apart."""
    Lb = 20.0
    x = np.zeros((n, 3), dtype=np.float32)
    x[:, 0], x[:, 1] = 1.0, 1.0
    x[:, 2] = (np.arange(n) + 0.5) * (Lb / n)
    inst = make(x, np.zeros(n), np.ones(n, dtype=np.int32))
    inst.box = synth.f32(Lb)
    inst.name = f"column_{n}"
    return inst


@pytest.mark.parametrize("cluster", [8, 4])
def test_column_at_the_sort_limit(torch_gpu, cluster):
    """A column of the largest size the build sorts (4096 atoms): the pair set is the oracle's
    and the forces and energies of the null type are zero."""
    inst = column_stack(4096)
    print(f"column of {inst.natoms} atoms, C={cluster}", flush=True)
    box = GpuBox(torch_gpu, inst, cluster=cluster)
    try:
        box.pairlist()
        assert box.stats()["nclusters"] == 4096 // cluster   # all in one column
        f, e = box.forces()
        pairs = np.asarray(box.pairs(), dtype=np.int64).reshape(-1, 2)
        assert nb.nb_check(box.ctx) == nb.NB_OK
    finally:
        box.close()
    pi, pj, _ = O.pairs(inst.x, inst.box, inst.cutoff, inst.excl_off, inst.excl_idx)
    n = inst.natoms
    assert len(pairs) == len(pi) > 0
    assert np.array_equal(np.sort(pairs[:, 0] * n + pairs[:, 1]), np.sort(pi.astype(np.int64) * n + pj))
    assert np.all(f == 0.0) and e[0] == 0.0 and e[1] == 0.0


def test_column_over_the_sort_limit_is_reported(torch_gpu):
    """One atom more than the build sorts in a column: nb_pairlist reports NB_ERR_OVERFLOW."""
    inst = column_stack(4097)
    print(f"column of {inst.natoms} atoms", flush=True)
    box = GpuBox(torch_gpu, inst)
    try:
        with pytest.raises(nb.NbError) as ei:
            box.pairlist()
        assert ei.value.code == nb.NB_ERR_OVERFLOW
    finally:
        box.close()


@pytest.mark.parametrize("cluster", [8, 4])
@pytest.mark.parametrize("flags", [0, nb.NB_ENERGY_FP64])
def test_largest_type_table(torch_gpu, cluster, flags):
    """32 LJ types, the most the library takes (the type-pair table then fills 32 KB of the
    force kernel's LDS): the 648-atom water box with 30 extra types on 90% of its oxygens,
    against the oracle (E_C to the FP32 bound of so small a box with FP32 pair energies)."""
    inst = synth.retype(synth.tiny(), 30, 0.9, seed=3)
    assert inst.ntypes == 32 and len(np.unique(inst.type)) > 20
    print(f"32 types, C={cluster} flags={flags}", flush=True)
    box = GpuBox(torch_gpu, inst, cluster=cluster, flags=flags)
    try:
        box.pairlist()
        f, e = box.forces()
        assert nb.nb_check(box.ctx) == nb.NB_OK
    finally:
        box.close()
    ref = O.instance_forces(inst, cells=False)
    fr = rel_rms(f, ref.f)
    elj = abs(e[0] - ref.e_lj) / abs(ref.e_lj)
    ec = abs(e[1] - ref.e_coul) / abs(ref.e_coul)
    print(f"force relRMS {fr:.2e} E_LJ rel {elj:.2e} E_C rel {ec:.2e}", flush=True)
    assert fr <= FORCE_TOL and elj <= ENERGY_TOL
    assert ec <= (ENERGY_TOL if flags & nb.NB_ENERGY_FP64 else FP32_SMALL_BOX_EC_TOL)


def test_largest_type_table_tabulated_ewald_and_backward(torch_gpu):
    """32 LJ types with the kernels that hold more tables beside the type table in LDS: the
    tabulated Ewald flavour (its FP32 force table and the FP64 erfc table) against the oracle at
    the 1e-6 energy gate, and the adjoint against the oracle's VJP (normwise, 5e-6)."""
    torch = torch_gpu
    inst = synth.retype(synth.tiny(), 30, 0.9, seed=3)
    print("32 types: tabulated Ewald", flush=True)
    box = GpuBox(torch, inst, elec=nb.NB_ELEC_EWALD_TAB)
    try:
        box.pairlist()
        f, e = box.forces()
        assert nb.nb_check(box.ctx) == nb.NB_OK
    finally:
        box.close()
    ref = O.instance_forces(inst, cells=False)
    fr = rel_rms(f, ref.f)
    elj = abs(e[0] - ref.e_lj) / abs(ref.e_lj)
    ec = abs(e[1] - ref.e_coul) / abs(ref.e_coul)
    print(f"force relRMS {fr:.2e} E_LJ rel {elj:.2e} E_C rel {ec:.2e}", flush=True)
    assert fr <= FORCE_TOL and elj <= ENERGY_TOL and ec <= ENERGY_TOL
    print("32 types: backward", flush=True)
    rng = np.random.default_rng(12)
    gF = rng.standard_normal((inst.natoms, 3)).astype(np.float32)
    gE = np.array([0.7, -1.3])
    box = GpuBox(torch, inst)
    try:
        gf, ge = dev(torch, gF.reshape(-1)), dev(torch, gE)
        dx = torch.empty(inst.natoms * 3, dtype=torch.float32, device="cuda:0")
        dq = torch.empty(inst.natoms, dtype=torch.float32, device="cuda:0")
        ds = torch.empty(inst.ntypes, dtype=torch.float64, device="cuda:0")
        de = torch.empty(inst.ntypes, dtype=torch.float64, device="cuda:0")
        nb.nb_backward(box.ctx, box.x, box.q, box.t, gf, ge, dx, dq, ds, de, 0)
        torch.cuda.synchronize()
        assert nb.nb_check(box.ctx) == nb.NB_OK
        gx = dx.cpu().numpy().reshape(-1, 3).astype(np.float64)
        gq = dq.cpu().numpy().astype(np.float64)
        gs, ge_ = ds.cpu().numpy(), de.cpu().numpy()
    finally:
        box.close()
    rdx, rdq, rds, rde = O.vjp(inst.x, inst.q, inst.type, inst.sigma, inst.epsilon, inst.box,
                               inst.cutoff, inst.beta, inst.coulomb_const, inst.excl_off,
                               inst.excl_idx, gF.astype(np.float64), gE)
    ex, eq = rel_rms(gx, rdx), rel_rms(gq, rdq)
    print(f"dx {ex:.2e} dq {eq:.2e}", flush=True)
    assert ex <= FORCE_TOL and eq <= FORCE_TOL
    # the LJ-parameter gradients normwise over the types present, like dx and dq: with ~6 atoms
    # per type and random cotangents a single type's sum cancels to a few percent of its terms,
    # so its elementwise relative error says more about that cancellation than about the kernel
    present = [t for t in np.unique(inst.type) if inst.epsilon[t] > 0.0]
    es, ee = rel_rms(gs[present], rds[present]), rel_rms(ge_[present], rde[present])
    worst = max(max(abs(gs[t] - rds[t]) / abs(rds[t]), abs(ge_[t] - rde[t]) / abs(rde[t])) for t in present)
    print(f"{len(present)} LJ types present: dsigma {es:.2e} deps {ee:.2e} (worst single type "
          f"{worst:.2e})", flush=True)
    assert es <= FORCE_TOL and ee <= FORCE_TOL


@pytest.mark.parametrize("graph", [False, True])
def test_largest_type_table_in_a_batch(torch_gpu, graph):
    """32 LJ types in the batched kernel (FP64 pair energies): two water boxes whose oxygens take
    30 extra types, against the oracle."""
    torch = torch_gpu
    insts = [synth.retype(synth.small_box(300, RC, RB, 5), 30, 0.9, seed=3),
             synth.retype(synth.small_box(400, RC, RB, 6), 30, 0.9, seed=3)]
    assert np.array_equal(insts[0].sigma, insts[1].sigma) and insts[0].ntypes == 32
    print(f"32 types in a batch, graph={graph}", flush=True)
    ao, bx, params, x, q, t = nb.concat_instances(insts, clusters=[8, 8], flags=nb.NB_ENERGY_FP64)
    stream = torch.cuda.Stream()
    bt = nb.nb_batch_setup(ao, bx, params, clusters=[8, 8], stream=stream.cuda_stream)
    try:
        with torch.cuda.stream(stream):
            dx = torch.from_numpy(x.reshape(-1)).to("cuda:0")
            dq = torch.from_numpy(q).to("cuda:0")
            dt = torch.from_numpy(t).to("cuda:0")
            f = torch.zeros(len(q) * 3, dtype=torch.float32, device="cuda:0")
            e = torch.zeros(2 * len(insts), dtype=torch.float64, device="cuda:0")
        stream.synchronize()
        nb.nb_batch_pairlist(bt, dx)
        for _ in range(2):
            (nb.nb_batch_graph_forces if graph else nb.nb_batch_forces)(bt, dx, dq, dt, f, e)
        stream.synchronize()
        assert nb.nb_batch_check(bt) == nb.NB_OK
        fa = f.cpu().numpy().reshape(-1, 3).astype(np.float64)
        ea = e.cpu().numpy().reshape(-1, 2)
    finally:
        nb.nb_batch_destroy(bt)
    for k, inst in enumerate(insts):
        ref = O.instance_forces(inst, cells=False)
        fr = rel_rms(fa[ao[k]:ao[k + 1]], ref.f)
        elj = abs(ea[k, 0] - ref.e_lj) / abs(ref.e_lj)
        ec = abs(ea[k, 1] - ref.e_coul) / abs(ref.e_coul)
        print(f"box {k} n={inst.natoms} force relRMS {fr:.2e} E_LJ rel {elj:.2e} E_C rel {ec:.2e}", flush=True)
        assert fr <= FORCE_TOL and elj <= ENERGY_TOL and ec <= ENERGY_TOL, k
