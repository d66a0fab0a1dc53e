"""Autotuner of the batched form: the library's schedule tuner (nb_batch_tune_schedule) times
every candidate, applies the fastest and leaves the results unchanged (the forces are summed in
fixed point, so any schedule gives the same bits; the per-box FP64 energy sums may differ in
rounding order); the Python driver (tune.autotune) picks a cluster shape per size bucket and
reuses its JSON cache."""
import json

import numpy as np
import pytest

from paper_2405_01420_amd import nb, synth, tune

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def boxes():
    sizes = [3000, 9000, 4503, 15000, 6000, 24000]
    return synth.batch(len(sizes), sizes=sizes)


def test_schedule_tuner_keeps_results(torch_gpu, boxes):
    torch = torch_gpu
    clusters = [8, 4, 8, 8, 4, 8]
    ao, bx, params, x, q, t = nb.concat_instances(boxes, clusters=clusters)
    stream = torch.cuda.Stream()
    bt = nb.nb_batch_setup(ao, bx, params, clusters=clusters, stream=stream.cuda_stream)
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
    f0, e0 = f.cpu().numpy().copy(), e.cpu().numpy().copy()
    best, us = nb.nb_batch_tune_schedule(bt, dx, dq, dt, f, e, reps=3)
    print("schedule us", us, "->", best, flush=True)
    assert best in nb.BATCH_SCHEDULES
    assert all(v > 0.0 for v in us.values()) and us[best] == min(us.values())
    assert bool(nb.nb_batch_get_info(bt)["sorted"]) == best[0]
    f.zero_()
    nb.nb_batch_forces(bt, dx, dq, dt, f, e)
    stream.synchronize()
    assert np.array_equal(f.cpu().numpy(), f0)
    assert np.allclose(e.cpu().numpy(), e0, rtol=1e-12, atol=0.0)
    assert nb.nb_batch_check(bt) == nb.NB_OK
    nb.nb_batch_destroy(bt)


def test_schedule_tuner_needs_a_list(torch_gpu, boxes):
    torch = torch_gpu
    ao, bx, params, x, q, t = nb.concat_instances(boxes[:2], clusters=[8, 8])
    bt = nb.nb_batch_setup(ao, bx, params, clusters=[8, 8])
    z = torch.zeros(3 * len(q), dtype=torch.float32, device="cuda:0")
    with pytest.raises(nb.NbError) as ei:
        nb.nb_batch_tune_schedule(bt, z, z, z, z, z)
    assert ei.value.code == nb.NB_ERR_STATE
    nb.nb_batch_destroy(bt)


def test_autotune_caches_its_choices(torch_gpu, boxes, tmp_path):
    """nb_autotune through the C-ABI: every bucket with boxes gets a shape, the decisions go to
    the JSON cache, and a second call takes them from it without timing."""
    cache = tmp_path / "tune.json"
    r1 = tune.autotune(boxes, cache_path=str(cache))
    assert len(r1["clusters"]) == len(boxes) and set(r1["clusters"]) <= {4, 8}
    assert (r1["sorted"], r1["blocks_per_cu"]) in nb.BATCH_SCHEDULES
    used = [b for b in r1["buckets"] if b["boxes"] > 0]
    assert sum(b["boxes"] for b in used) == len(boxes)
    for b in used:
        assert not b["cached"] and b["cluster"] in (4, 8)
        assert b["us"][4] > 0 and b["us"][8] > 0
        assert b["cluster"] == (8 if b["us"][8] < b["us"][4] else 4)
    stored = json.loads(cache.read_text())
    assert any("schedule" in k for k in stored) and any("bucket" in k for k in stored)
    r2 = tune.autotune(boxes, cache_path=str(cache))
    assert r2["clusters"] == r1["clusters"]
    assert (r2["sorted"], r2["blocks_per_cu"]) == (r1["sorted"], r1["blocks_per_cu"])
    assert r2["schedule_cached"] and all(b["cached"] for b in r2["buckets"] if b["boxes"] > 0)
    assert json.loads(cache.read_text()) == stored
