"""Rolling prune (nb_prune) of the HIP path, through the C-ABI: forces and energies stay equal to
the FP64 oracle along a random walk with the list pruned every other call, the pair set of a
list pruned to r_inner = rc is the oracle's, the next build restores the full list, the
displacement check covers the pruned list, and invalid calls are rejected.

Gates as for every parity test: forces RMS relative <= 5e-6, energies relative <= 1e-6 (FP64
pair energies, as in the asynchronous-build walk on this machine); pair sets exact up to pairs within
FP32 rounding of rc."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2405_01420_amd import nb, synth
from tests.gpu_helpers import ENERGY_TOL, FORCE_TOL, GpuBox, compare_forces, pair_set_diff

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def inst_diff():
    return synth.diff()


@pytest.mark.parametrize("cluster,extra", [(8, 0), (4, 0), (8, nb.NB_ASYNC_BUILD)])
def test_pruned_walk_matches_oracle(torch_gpu, inst_diff, cluster, extra):
    """24k atoms, built every 10 calls (also with asynchronous builds), pruned every 2 calls to
    rc + 0.04 nm (valid while atoms move less than 0.02 nm; the walk moves them ~0.003 nm per
    call)."""
    box = GpuBox(torch_gpu, inst_diff, cluster=cluster, flags=nb.NB_CHECK_STALE | nb.NB_ENERGY_FP64 | extra)
    rin = inst_diff.cutoff + 0.04
    rng = synth.jitter_stream(23)
    x = inst_diff.x.copy()
    box.pairlist()
    full = box.stats()["nentries"]
    for call in range(12):
        box.set_x(x)
        if call % 10 == 0:
            box.pairlist()
        if call % 2 == 0:
            nb.nb_prune(box.ctx, box.x, rin)
        f, e = box.forces()
        if call % 2 == 1:
            assert nb.nb_check(box.ctx) == nb.NB_OK
            st = box.stats()
            assert st["pruned"] == 1 and st["nentries"] < full
            ref = O.instance_forces(inst_diff, cells=True, x=x)
            fr, elj, ec = compare_forces(f, e, ref, f"C={cluster} pruned call {call} "
                                                    f"({st['nentries']} of {full} entries)")
            assert fr <= FORCE_TOL and elj <= ENERGY_TOL and ec <= ENERGY_TOL
        x = (x + rng.normal(0.0, 0.002, x.shape)).astype(np.float32)
    box.close()


def test_prune_to_cutoff_gives_the_oracle_pair_set(torch_gpu, inst_diff):
    box = GpuBox(torch_gpu, inst_diff)
    box.pairlist()
    full = box.stats()["nentries"]
    x = (inst_diff.x + synth.jitter_stream(5).normal(0.0, 0.004, inst_diff.x.shape)).astype(np.float32)
    box.set_x(x)
    nb.nb_prune(box.ctx, box.x, inst_diff.cutoff)
    st = box.stats()
    bad, bnd, no, ng, dup = pair_set_diff(inst_diff, box.pairs(), x=x)
    print(f"pruned to rc: {st['nentries']} of {full} entries; pairs oracle {no} gpu {ng} "
          f"boundary {bnd}", flush=True)
    assert bad == 0 and dup == 0
    f, e = box.forces()
    ref = O.instance_forces(inst_diff, cells=True, x=x)
    fr, elj, ec = compare_forces(f, e, ref, "pruned to rc")
    assert fr <= FORCE_TOL and elj <= ENERGY_TOL
    # the next build restores the full list
    box.set_x(inst_diff.x)
    box.pairlist()
    st2 = box.stats()
    assert st2["pruned"] == 0 and st2["nentries"] == full
    box.close()


def test_pruned_list_displacement_check(torch_gpu, inst_diff):
    """With NB_CHECK_STALE, an atom that moved more than (r_inner - rc)/2 since the prune (but less
    than buffer/2 since the build) is reported; smaller moves are not."""
    box = GpuBox(torch_gpu, inst_diff, flags=nb.NB_CHECK_STALE)
    box.pairlist()
    nb.nb_prune(box.ctx, box.x, inst_diff.cutoff + 0.02)
    x = inst_diff.x.copy()
    x[100, 0] += 0.008
    box.set_x(x)
    box.forces()
    assert nb.nb_check(box.ctx) == nb.NB_OK
    x[100, 0] += 0.01   # 0.018 from the prune positions: above 0.01, below buffer / 2
    box.set_x(x)
    box.forces()
    assert nb.nb_check(box.ctx) == nb.NB_ERR_LIST_STALE
    box.close()


def test_prune_rejects_invalid_calls(torch_gpu, inst_diff):
    box = GpuBox(torch_gpu, inst_diff)
    with pytest.raises(nb.NbError) as ei:
        nb.nb_prune(box.ctx, box.x, inst_diff.cutoff + 0.01)
    assert ei.value.code == nb.NB_ERR_STATE
    box.pairlist()
    for r in (inst_diff.cutoff - 0.01, inst_diff.cutoff + inst_diff.buffer + 0.01, float("nan")):
        with pytest.raises(nb.NbError) as ei:
            nb.nb_prune(box.ctx, box.x, r)
        assert ei.value.code == nb.NB_ERR_ARG
    box.close()
