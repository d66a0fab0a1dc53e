"""nb_backward_noalloc (work buffers in the library's static device array, no allocation) against
nb_backward with NB_REUSE_LIST on the same list, to the adjoint's G1 bound (5e-6 relative RMS for
dx and dq, 5e-6 relative per LJ parameter), on two calls in a row through the C-ABI: the
24,000-atom gradient box, then the smaller 648-atom box (which reuses the array the first call
filled), and again the first box."""
import numpy as np
import pytest

from paper_2405_01420_amd import nb, synth
from tests.gpu_helpers import GpuBox, dev, rel_rms

pytestmark = pytest.mark.gpu

TOL = 5e-6


def _run(torch, box, inst, fn, flags=None):
    n, nt = inst.natoms, inst.ntypes
    rng = np.random.default_rng(inst.natoms)
    gf = dev(torch, rng.standard_normal(3 * n).astype(np.float32))
    ge = dev(torch, np.array([0.3, -0.7]))
    dx = torch.full((3 * n,), float("nan"), dtype=torch.float32, device="cuda:0")
    dq = torch.full((n,), float("nan"), dtype=torch.float32, device="cuda:0")
    ds = torch.full((nt,), float("nan"), dtype=torch.float64, device="cuda:0")
    de = torch.full((nt,), float("nan"), dtype=torch.float64, device="cuda:0")
    if flags is None:
        fn(box.ctx, box.x, box.q, box.t, gf, ge, dx, dq, ds, de)
    else:
        fn(box.ctx, box.x, box.q, box.t, gf, ge, dx, dq, ds, de, flags)
    torch.cuda.synchronize()
    return (dx.cpu().numpy().astype(np.float64), dq.cpu().numpy().astype(np.float64),
            ds.cpu().numpy(), de.cpu().numpy())


def _compare(a, b, inst, label):
    ex = rel_rms(a[0], b[0])
    eq = rel_rms(a[1], b[1])
    print(f"{label}: dx relRMS {ex:.2e} dq relRMS {eq:.2e}", flush=True)
    assert np.all(np.isfinite(a[0])) and np.all(np.isfinite(a[1]))
    assert ex <= TOL and eq <= TOL
    for t in range(inst.ntypes):
        for k in (2, 3):
            if b[k][t] == 0.0:
                assert a[k][t] == 0.0
            else:
                assert abs(a[k][t] - b[k][t]) <= TOL * abs(b[k][t]), (label, k, t, a[k][t], b[k][t])


def test_noalloc_backward_matches_backward(torch_gpu):
    torch = torch_gpu
    big, small = synth.diff(), synth.tiny()
    bb = GpuBox(torch, big)
    bs = GpuBox(torch, small)
    try:
        bb.pairlist()
        bs.pairlist()
        ref_big = _run(torch, bb, big, nb.nb_backward, nb.NB_REUSE_LIST)
        ref_small = _run(torch, bs, small, nb.nb_backward, nb.NB_REUSE_LIST)
        _compare(_run(torch, bb, big, nb.nb_backward_noalloc), ref_big, big, "24k first call")
        _compare(_run(torch, bs, small, nb.nb_backward_noalloc), ref_small, small, "648 second call")
        _compare(_run(torch, bb, big, nb.nb_backward_noalloc), ref_big, big, "24k third call")
    finally:
        bb.close()
        bs.close()


def test_noalloc_backward_rejects_missing_list_and_oversized_system(torch_gpu):
    torch = torch_gpu
    inst = synth.tiny()
    box = GpuBox(torch, inst)
    try:
        with pytest.raises(nb.NbError) as ei:
            _run(torch, box, inst, nb.nb_backward_noalloc)
        assert ei.value.code == nb.NB_ERR_STATE
    finally:
        box.close()
    # 90,000 waters (270,000 atoms) need more padded slots than the static work area holds: the
    # call is refused on the host, before any kernel runs
    big = synth.water_box(90000, (270000 / 100.0) ** (1.0 / 3.0), 1.0, 0.1, seed=11)
    assert big.natoms > nb.NB_NOALLOC_MAX_SLOTS
    box = GpuBox(torch, big)
    try:
        with pytest.raises(nb.NbError) as ei:
            _run(torch, box, big, nb.nb_backward_noalloc)
        assert ei.value.code == nb.NB_ERR_ARG
        assert "static work area" in nb.nb_last_error(box.ctx)
    finally:
        box.close()
