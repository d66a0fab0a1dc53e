"""Parity of the HIP path (through the C-ABI) with the FP64 oracle on seeded water boxes.

Gates: pair set identical except pairs whose FP64 distance is within 2^-22 max(L, 1) nm of the
cutoff; forces RMS relative error <= 5e-6; each energy component relative error <= 1e-6.  The
96k- and 24k-atom boxes meet the energy gate with FP32 pair energies (the default); the
648-atom box needs FP64 pair energies (NB_ENERGY_FP64) for the Coulomb energy, whose
conditioning there leaves FP32 rounding noise near 1e-6 (checked in both modes)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2405_01420_amd import nb, synth
from tests.gpu_helpers import (ENERGY_TOL, FORCE_TOL, FP32_SMALL_BOX_EC_TOL, GpuBox,
                               compare_forces, pair_set_diff, rel_rms)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def inst_tiny():
    return synth.tiny()


@pytest.fixture(scope="module")
def inst_diff():
    return synth.diff()


@pytest.fixture(scope="module")
def inst_mid():
    return synth.mid()


@pytest.mark.parametrize("cluster", [8, 4])
@pytest.mark.parametrize("efp64", [True, False])
def test_tiny_pairs_and_forces(torch_gpu, inst_tiny, cluster, efp64):
    box = GpuBox(torch_gpu, inst_tiny, cluster=cluster, flags=nb.NB_ENERGY_FP64 if efp64 else 0)
    box.pairlist()
    bad, bnd, no, ng, dup = pair_set_diff(inst_tiny, box.pairs())
    print(f"tiny C={cluster}: oracle {no} pairs, gpu {ng}, mismatches {bad}, boundary {bnd}, dup {dup}")
    assert bad == 0
    f, e = box.forces()
    ref = O.instance_forces(inst_tiny)
    fr, elj, ec = compare_forces(f, e, ref, f"tiny C={cluster} efp64={efp64}")
    box.close()
    assert fr <= FORCE_TOL and elj <= ENERGY_TOL
    assert ec <= (ENERGY_TOL if efp64 else FP32_SMALL_BOX_EC_TOL)


@pytest.mark.parametrize("cluster", [8, 4])
def test_diff_pairs_and_forces(torch_gpu, inst_diff, cluster):
    box = GpuBox(torch_gpu, inst_diff, cluster=cluster)
    box.pairlist()
    bad, bnd, no, ng, dup = pair_set_diff(inst_diff, box.pairs())
    print(f"diff C={cluster}: oracle {no} pairs, gpu {ng}, mismatches {bad}, boundary {bnd}")
    assert bad == 0
    f, e = box.forces()
    ref = O.instance_forces(inst_diff, cells=True)
    fr, elj, ec = compare_forces(f, e, ref, f"diff C={cluster}")
    box.close()
    assert fr <= FORCE_TOL and elj <= ENERGY_TOL and ec <= ENERGY_TOL


@pytest.mark.parametrize("efp64", [False, True])
def test_mid_pairs_and_forces(torch_gpu, inst_mid, efp64):
    box = GpuBox(torch_gpu, inst_mid, flags=nb.NB_ENERGY_FP64 if efp64 else 0)
    box.pairlist()
    st = box.stats()
    print("mid stats", st)
    bad, bnd, no, ng, dup = pair_set_diff(inst_mid, box.pairs())
    print(f"mid: oracle {no} pairs, gpu {ng}, mismatches {bad}, boundary {bnd}")
    assert bad == 0
    f, e = box.forces()
    ref = O.instance_forces(inst_mid, cells=True)
    fr, elj, ec = compare_forces(f, e, ref, "mid")
    box.close()
    assert fr <= FORCE_TOL and elj <= ENERGY_TOL and ec <= ENERGY_TOL


def test_mid_jitter_rebuild_every_10(torch_gpu, inst_mid):
    """Random walk N(0, 0.002 nm) per call without re-wrapping, list rebuilt every 10 calls;
    checked against the oracle at calls 9, 19 and 29 (the last call before each rebuild, where
    atoms are farthest from the build positions)."""
    box = GpuBox(torch_gpu, inst_mid, flags=nb.NB_CHECK_STALE)
    rng = synth.jitter_stream(20)
    x = inst_mid.x.copy()
    for call in range(30):
        if call % 10 == 0:
            box.set_x(x)
            box.pairlist()
        else:
            box.set_x(x)
        f, e = box.forces()
        assert nb.nb_check(box.ctx) == nb.NB_OK
        if call % 10 == 9:
            ref = O.instance_forces(inst_mid, cells=True, x=x)
            pairs = box.pairs()
            bad, bnd, no, ng, dup = pair_set_diff(inst_mid, pairs, x=x)
            fr, elj, ec = compare_forces(f, e, ref, f"mid jitter call {call}")
            assert bad == 0
            assert fr <= FORCE_TOL and elj <= ENERGY_TOL and ec <= ENERGY_TOL
        x = (x + rng.normal(0.0, 0.002, x.shape)).astype(np.float32)
    box.close()


def test_newton_third_law(torch_gpu, inst_diff):
    box = GpuBox(torch_gpu, inst_diff)
    box.pairlist()
    f, _ = box.forces()
    box.close()
    net = np.abs(f.sum(0)).max()
    tot = np.abs(f).sum()
    print("net force", net, "sum |F|", tot)
    assert net <= 1e-8 * tot


def test_deterministic_pair_set(torch_gpu, inst_diff):
    box = GpuBox(torch_gpu, inst_diff)
    box.pairlist()
    p1 = box.pairs()
    box.pairlist()
    p2 = box.pairs()
    box.close()
    k1 = np.sort(p1[:, 0] * inst_diff.natoms + p1[:, 1])
    k2 = np.sort(p2[:, 0] * inst_diff.natoms + p2[:, 1])
    assert np.array_equal(k1, k2)


def test_list_regrows_after_overflow(torch_gpu, inst_tiny, monkeypatch):
    monkeypatch.setenv("NB_LIST_CAP", "2")
    box = GpuBox(torch_gpu, inst_tiny, flags=nb.NB_ENERGY_FP64)
    assert box.stats()["list_capacity"] == 2
    box.pairlist()  # overflows the 2-entry capacity, regrows and rebuilds
    st = box.stats()
    assert st["list_capacity"] > 2
    f, e = box.forces()
    ref = O.instance_forces(inst_tiny)
    fr, elj, ec = compare_forces(f, e, ref, "tiny after regrow")
    box.close()
    assert fr <= FORCE_TOL and elj <= ENERGY_TOL and ec <= ENERGY_TOL


def test_stale_list_is_reported(torch_gpu, inst_diff):
    box = GpuBox(torch_gpu, inst_diff, flags=nb.NB_CHECK_STALE)
    box.pairlist()
    box.forces()
    assert nb.nb_check(box.ctx) == nb.NB_OK
    x = inst_diff.x.copy()
    x[17, 0] += 0.06  # more than buffer / 2 = 0.05 nm
    box.set_x(x)
    box.forces()
    assert nb.nb_check(box.ctx) == nb.NB_ERR_LIST_STALE
    assert nb.nb_check(box.ctx) == nb.NB_OK  # cleared
    box.close()


@pytest.mark.parametrize("flags", [0, nb.NB_ASYNC_BUILD])
def test_stale_force_call_survives_a_rebuild(torch_gpu, inst_diff, flags):
    """A condition raised by a force call (stale list) is still reported by nb_check after a
    later list build: the build clears only its own status."""
    box = GpuBox(torch_gpu, inst_diff, flags=nb.NB_CHECK_STALE | flags)
    box.pairlist()
    box.forces()
    assert nb.nb_check(box.ctx) == nb.NB_OK
    x = inst_diff.x.copy()
    x[17, 0] += 0.06  # more than buffer / 2 = 0.05 nm
    box.set_x(x)
    box.forces()
    box.pairlist()   # rebuilt at the moved positions: the stale call happened before
    box.pairlist()
    box.forces()
    assert nb.nb_check(box.ctx) == nb.NB_ERR_LIST_STALE
    assert nb.nb_check(box.ctx) == nb.NB_OK
    box.close()


def test_nonfinite_is_reported(torch_gpu, inst_tiny):
    box = GpuBox(torch_gpu, inst_tiny, flags=nb.NB_CHECK_FINITE)
    x = inst_tiny.x.copy()
    x[5, 1] = np.nan
    box.set_x(x)
    with pytest.raises(nb.NbError) as ei:
        box.pairlist()
    assert ei.value.code == nb.NB_ERR_NONFINITE
    box.close()


def test_forces_before_list_is_state_error(torch_gpu, inst_tiny):
    box = GpuBox(torch_gpu, inst_tiny)
    with pytest.raises(nb.NbError) as ei:
        nb.nb_forces(box.ctx, box.x, box.q, box.t, box.f, box.e)
    assert ei.value.code == nb.NB_ERR_STATE
    box.close()


def test_async_builds_along_jitter(torch_gpu, inst_diff):
    """Asynchronous list builds (status read at the next build) on a random walk rebuilt every
    5 calls: forces and energies match the oracle at the last call before each rebuild (FP64
    pair energies: with FP32 ones the Coulomb energy of this 24k-atom box reaches 1.5e-6 on
    some of these configurations, a property of the energy precision, not of the list)."""
    box = GpuBox(torch_gpu, inst_diff, flags=nb.NB_ASYNC_BUILD | nb.NB_CHECK_STALE | nb.NB_ENERGY_FP64)
    rng = synth.jitter_stream(21)
    x = inst_diff.x.copy()
    for call in range(15):
        box.set_x(x)
        if call % 5 == 0:
            box.pairlist()
        f, e = box.forces()
        if call % 5 == 4:
            assert nb.nb_check(box.ctx) == nb.NB_OK
            ref = O.instance_forces(inst_diff, cells=True, x=x)
            fr, elj, ec = compare_forces(f, e, ref, f"diff async call {call}")
            assert fr <= FORCE_TOL and elj <= ENERGY_TOL and ec <= ENERGY_TOL
        x = (x + rng.normal(0.0, 0.002, x.shape)).astype(np.float32)
    box.pairlist()  # reads the last build's status: no overflow
    box.close()


def test_async_build_reports_overflow_of_previous_build(torch_gpu, inst_diff):
    """An asynchronous build whose lists overflow (4,000 atoms packed into a 0.6 nm cube) is
    reported by the next nb_pairlist, which regrows the list and rebuilds completely."""
    box = GpuBox(torch_gpu, inst_diff, flags=nb.NB_ASYNC_BUILD)
    box.pairlist()  # first build: synchronous
    cap0 = box.stats()["list_capacity"]
    xc = inst_diff.x.copy()
    c0 = 0.5 * inst_diff.box
    rng = np.random.default_rng(3)
    xc[:4000] = (c0 + rng.uniform(-0.3, 0.3, (4000, 3))).astype(np.float32)
    box.set_x(xc)
    box.pairlist()  # asynchronous: overflows
    box.set_x(inst_diff.x)
    with pytest.raises(nb.NbError) as ei:
        box.pairlist()
    assert ei.value.code == nb.NB_ERR_OVERFLOW
    assert box.stats()["list_capacity"] > cap0
    f, e = box.forces()
    ref = O.instance_forces(inst_diff, cells=True)
    fr, elj, ec = compare_forces(f, e, ref, "diff after async overflow")
    box.close()
    assert fr <= FORCE_TOL and elj <= ENERGY_TOL and ec <= ENERGY_TOL


def test_energies_do_not_depend_on_scheduling(torch_gpu, inst_diff):
    """Energy partials are summed per work unit, per finalize block and over blocks in fixed
    orders: repeated calls give bit-identical energies."""
    box = GpuBox(torch_gpu, inst_diff)
    box.pairlist()
    _, e1 = box.forces()
    for _ in range(5):
        _, e2 = box.forces()
        assert np.array_equal(e1, e2)
    box.close()


def test_forces_do_not_depend_on_scheduling(torch_gpu, inst_diff):
    """The forces are summed in fixed point with integer atomics: repeated calls give
    bit-identical forces, whatever order the device added the pair contributions in."""
    box = GpuBox(torch_gpu, inst_diff)
    box.pairlist()
    f1, _ = box.forces()
    for _ in range(5):
        f2, _ = box.forces()
        assert np.array_equal(f1, f2)
    box.close()


def test_force_beyond_the_fixed_point_range_is_reported(torch_gpu, inst_tiny):
    """Two oxygens 0.1 nm apart (a Lennard-Jones force of order 1e7 kJ/mol/nm) raise the range
    flag, which nb_check reports once and clears."""
    box = GpuBox(torch_gpu, inst_tiny, flags=nb.NB_ENERGY_FP64)
    x = inst_tiny.x.copy()
    x[0] = x[3] + np.array([0.1, 0.0, 0.0], np.float32)  # O of molecule 0 next to O of molecule 1
    box.set_x(x)
    box.pairlist()
    box.forces()
    assert nb.nb_check(box.ctx) == nb.NB_ERR_RANGE
    assert nb.nb_check(box.ctx) == nb.NB_OK
    box.set_x(inst_tiny.x)
    box.pairlist()
    box.forces()
    assert nb.nb_check(box.ctx) == nb.NB_OK
    box.close()


@pytest.mark.parametrize("which", ["tiny", "diff"])
def test_sorted_work_units_keep_results(torch_gpu, which):
    """NB_SORT_UNITS (work units longest first) only reorders the units: the same forces bit for
    bit (fixed-point sums of the same unit contributions) and the same energies up to summation
    order; the list-length histogram covers every non-empty list."""
    inst = getattr(synth, which)()
    out = []
    for flags in (0, nb.NB_SORT_UNITS):
        box = GpuBox(torch_gpu, inst, flags=flags | nb.NB_ENERGY_FP64)
        box.pairlist()
        f, e = box.forces()
        st = box.stats()
        out.append((f, e, st))
        box.close()
    (f0, e0, s0), (f1, e1, s1) = out
    assert np.array_equal(f0, f1)
    assert np.all(np.abs(e0 - e1) <= 1e-12 * np.abs(e0))
    assert s0["list_hist"] == s1["list_hist"] and s0["work_units"] == s1["work_units"]
    assert 0 < sum(s0["list_hist"]) <= s0["nclusters"]
    print(which, "list-length histogram (batches 1, 2-3, 4-7, ...):", s0["list_hist"])
