"""Autotuner for the batched form: cluster size per box-size bucket and the work schedule.

For every size bucket (logarithmic buckets of the box atom count) the tuner builds a batch of
that bucket's boxes once per candidate cluster size (4 or 8 atoms), times the batched force
call on the GPU and keeps the fastest shape.  With the per-box shapes fixed it then times the
schedules of the persistent kernel (work items sorted by cost or in box order; persistent grid
of 1, 2, 4 blocks per compute unit or as many as fit) on the whole batch, in the library
(nb_batch_tune_schedule).  Decisions are cached
in a JSON file keyed by GPU architecture, HIP version, cutoff and bucket, so a later run with the
same kind of boxes reuses them without timing.  Timing uses torch CUDA events on the batch's
stream around repeated calls; the tuner itself does no force arithmetic.
"""
from __future__ import annotations

import json
import math
import os
import time
from typing import Dict, List, Optional, Sequence

import numpy as np

from . import nb

CLUSTERS = (4, 8)


def bucket_edges(nmin: int = 3000, nmax: int = 30000, nbuckets: int = 5) -> List[float]:
    r = (nmax / nmin) ** (1.0 / nbuckets)
    return [nmin * r ** k for k in range(nbuckets + 1)]


def bucket_of(natoms: int, edges: Sequence[float]) -> int:
    for k in range(len(edges) - 1):
        if natoms < edges[k + 1]:
            return k
    return len(edges) - 2


def _device_key() -> str:
    import torch
    p = torch.cuda.get_device_properties(0)
    arch = getattr(p, "gcnArchName", p.name)
    return f"{arch}|hip{torch.version.hip}"


def _time_batch(torch, insts, clusters, sorted_=True, blocks_per_cu=0, reps=10, warmup=3,
                stream=None) -> float:
    """Microseconds per batched force call for these boxes and shapes."""
    ao, bx, params, x, q, t = nb.concat_instances(insts, clusters=clusters)
    s = stream or torch.cuda.current_stream()
    bt = nb.nb_batch_setup(ao, bx, params, clusters=list(clusters), stream=s.cuda_stream)
    try:
        nb.nb_batch_set_schedule(bt, sorted_, blocks_per_cu)
        with torch.cuda.stream(s):
            dx = torch.from_numpy(x.reshape(-1)).to("cuda:0")
            dq = torch.from_numpy(q).to("cuda:0")
            dt = torch.from_numpy(t).to("cuda:0")
            f = torch.empty(len(q) * 3, dtype=torch.float32, device="cuda:0")
            e = torch.empty(2 * len(insts), dtype=torch.float64, device="cuda:0")
            nb.nb_batch_pairlist(bt, dx)
            for _ in range(warmup):
                nb.nb_batch_forces(bt, dx, dq, dt, f, e)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(s)
            for _ in range(reps):
                nb.nb_batch_forces(bt, dx, dq, dt, f, e)
            e1.record(s)
            s.synchronize()
            return 1e3 * e0.elapsed_time(e1) / reps
    finally:
        nb.nb_batch_destroy(bt)


def _tune_schedule(torch, insts, clusters, stream, reps=5):
    """One batch with the chosen shapes; the library times the candidate schedules on it
    (nb_batch_tune_schedule) and keeps the fastest."""
    ao, bx, params, x, q, t = nb.concat_instances(insts, clusters=clusters)
    bt = nb.nb_batch_setup(ao, bx, params, clusters=list(clusters), stream=stream.cuda_stream)
    try:
        with torch.cuda.stream(stream):
            dx = torch.from_numpy(x.reshape(-1)).to("cuda:0")
            dq = torch.from_numpy(q).to("cuda:0")
            dt = torch.from_numpy(t).to("cuda:0")
            f = torch.empty(len(q) * 3, dtype=torch.float32, device="cuda:0")
            e = torch.empty(2 * len(insts), dtype=torch.float64, device="cuda:0")
        stream.synchronize()
        nb.nb_batch_pairlist(bt, dx)
        return nb.nb_batch_tune_schedule(bt, dx, dq, dt, f, e, reps)
    finally:
        nb.nb_batch_destroy(bt)


def autotune(insts, cache_path: Optional[str] = None, max_boxes_per_bucket: int = 16,
             edges: Optional[Sequence[float]] = None, verbose: bool = False) -> Dict:
    """Returns {"clusters": [C per box], "sorted": bool, "blocks_per_cu": int, "tune_s": seconds,
    "buckets": {...}} and updates the JSON cache."""
    import torch
    t0 = time.perf_counter()
    edges = list(edges or bucket_edges())
    cache_path = cache_path or os.environ.get("NB_TUNE_CACHE")
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as fh:
            cache = json.load(fh)
    dev = _device_key()
    rc = insts[0].cutoff
    buckets: Dict[int, List[int]] = {}
    for k, inst in enumerate(insts):
        buckets.setdefault(bucket_of(inst.natoms, edges), []).append(k)
    choice = {}
    report = {}
    stream = torch.cuda.Stream()
    for bk, members in sorted(buckets.items()):
        key = f"{dev}|rc{rc:.4f}|bucket{int(edges[bk])}-{int(edges[bk + 1])}"
        if key in cache:
            choice[bk] = cache[key]["cluster"]
            report[key] = dict(cache[key], cached=True)
            continue
        sample = [insts[k] for k in members[:max_boxes_per_bucket]]
        times = {}
        for C in CLUSTERS:
            times[C] = _time_batch(torch, sample, [C] * len(sample), stream=stream)
        best = min(times, key=times.get)
        choice[bk] = best
        cache[key] = {"cluster": best, "us": {str(c): v for c, v in times.items()},
                      "boxes": len(sample)}
        report[key] = cache[key]
        if verbose:
            print("bucket", key, times, "->", best, flush=True)
    clusters = [choice[bucket_of(inst.natoms, edges)] for inst in insts]
    skey = f"{dev}|rc{rc:.4f}|schedule|n{len(insts)}"
    if skey in cache:
        sorted_, bpc = cache[skey]["sorted"], cache[skey]["blocks_per_cu"]
    else:
        (sorted_, bpc), stimes = _tune_schedule(torch, insts, clusters, stream)
        cache[skey] = {"sorted": sorted_, "blocks_per_cu": bpc,
                       "us": {f"sorted={s},bpc={b}": v for (s, b), v in stimes.items()}}
        if verbose:
            print("schedule", stimes, "->", (sorted_, bpc), flush=True)
    report[skey] = cache[skey]
    if cache_path:
        tmp = cache_path + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(cache, fh, indent=1, sort_keys=True)
        os.replace(tmp, cache_path)
    return {"clusters": clusters, "sorted": bool(sorted_), "blocks_per_cu": int(bpc),
            "tune_s": time.perf_counter() - t0, "buckets": report}
