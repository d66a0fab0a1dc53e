"""Autotuner of the batched form: a thin caller of the library's tuner (nb_autotune).

The library groups the boxes into logarithmic size buckets, times a sample batch of every
bucket with 4- and 8-atom clusters, then times the schedules of the persistent kernel on the
whole batch with the chosen shapes, and keeps its decisions in a JSON cache file.  This module
only moves the boxes to the GPU and passes pointers.
"""
from __future__ import annotations

import os
import time
from typing import Dict, List, Optional, Sequence

from . import nb


def bucket_edges(nmin: int = nb.NB_TUNE_NMIN, nmax: int = nb.NB_TUNE_NMAX,
                 nbuckets: int = nb.NB_TUNE_BUCKETS) -> List[float]:
    """The tuner's bucket edges (atoms): logarithmic over [nmin, nmax)."""
    r = (nmax / nmin) ** (1.0 / nbuckets)
    return [nmin * r ** k for k in range(nbuckets + 1)]


def bucket_of(natoms: int, edges: Sequence[float]) -> int:
    for k in range(len(edges) - 1):
        if natoms < edges[k + 1]:
            return k
    return len(edges) - 2


def autotune(insts, cache_path: Optional[str] = None, flags: int = 0, verbose: bool = False) -> Dict:
    """Returns {"clusters": [C per box], "sorted": bool, "blocks_per_cu": int, "tune_s": seconds,
    "buckets": [...], "schedule_us": {...}}; the cache file (cache_path, else $NB_TUNE_CACHE,
    else none) is read and updated by the library."""
    import torch
    t0 = time.perf_counter()
    cache_path = cache_path or os.environ.get("NB_TUNE_CACHE")
    ao, bx, params, x, q, t = nb.concat_instances(insts, flags=flags)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        dx = torch.from_numpy(x.reshape(-1)).to("cuda:0")
        dq = torch.from_numpy(q).to("cuda:0")
        dt = torch.from_numpy(t).to("cuda:0")
    stream.synchronize()
    clusters, res = nb.nb_autotune(ao, bx, params, dx, dq, dt, cache_path=cache_path,
                                   stream=stream.cuda_stream)
    if verbose:
        for b in res["buckets"]:
            print("bucket", b, flush=True)
        print("schedule", res["schedule_us"], "->", (res["sorted"], res["blocks_per_cu"]), flush=True)
    res.update(clusters=clusters, tune_s=time.perf_counter() - t0)
    return res
