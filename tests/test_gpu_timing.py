"""Kernel timing (nb_set_timing / nb_get_timing): with timing on, the force kernel is dispatched
with an event pair that the dispatch stamps; the results are the same bits as without timing (the
force sums are fixed point, the energies summed in a fixed order), every timed launch is counted,
more launches than the event pairs created up front are handled, and reading the timing resets
it."""
import numpy as np
import pytest

from paper_2405_01420_amd import nb, synth
from tests.gpu_helpers import GpuBox

pytestmark = pytest.mark.gpu


def test_timing_counts_launches_and_keeps_results(torch_gpu):
    inst = synth.tiny()
    box = GpuBox(torch_gpu, inst)
    try:
        box.pairlist()
        f0, e0 = box.forces()
        nb.nb_set_timing(box.ctx, True)
        ms, n = nb.nb_get_timing(box.ctx)
        assert n == 0 and ms == 0.0
        for _ in range(1100):  # more than the 1024 event pairs created when timing is turned on
            nb.nb_forces(box.ctx, box.x, box.q, box.t, box.f, box.e)
        f1, e1 = box.forces()  # one more timed launch
        ms, n = nb.nb_get_timing(box.ctx)
        print(f"timed launches {n}, mean {1e3 * ms / n:.2f} us", flush=True)
        assert n == 1101 and ms > 0.0
        assert np.array_equal(f0, f1) and np.array_equal(e0, e1)
        ms, n = nb.nb_get_timing(box.ctx)
        assert n == 0 and ms == 0.0
        nb.nb_set_timing(box.ctx, False)
        box.forces()
        assert nb.nb_get_timing(box.ctx)[1] == 0
    finally:
        box.close()
