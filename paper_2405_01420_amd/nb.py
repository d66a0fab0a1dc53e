"""Thin ctypes binding of libnb.so (include/nb.h): argument marshalling only.

Every function here has the name of the C entry point it calls.  Device buffers are passed as
torch tensors on the GPU (only their data pointers cross the boundary) and the HIP stream is
torch's current stream unless given.  There is no CPU fallback: if libnb.so is missing or
cannot be loaded, ``lib()`` raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libnb.so")

NB_OK, NB_ERR_ARG, NB_ERR_CUTOFF, NB_ERR_OOM, NB_ERR_HIP = 0, 1, 2, 3, 4
NB_ERR_STATE, NB_ERR_OVERFLOW, NB_ERR_LIST_STALE, NB_ERR_NONFINITE, NB_ERR_IO = 5, 6, 7, 8, 9
NB_ERR_RANGE = 10
NB_CHECK_STALE, NB_CHECK_FINITE, NB_REUSE_LIST, NB_ASYNC_BUILD = 0x1, 0x2, 0x4, 0x8
NB_ENERGY_FP64 = 0x10
NB_EWALD_CORR = 0x20
NB_SORT_UNITS = 0x40
NB_MAX_EXCL_PER_ATOM = 32
NB_NOALLOC_MAX_SLOTS = 262144  # padded slots nb_backward_noalloc handles at most
NB_ELEC_EWALD, NB_ELEC_RF, NB_ELEC_EWALD_TAB = 0, 1, 2
NB_TAB_SEGMENTS = 256
NB_VDW_SHIFT, NB_VDW_FSWITCH = 0, 1

STATUS_NAMES = {0: "NB_OK", 1: "NB_ERR_ARG", 2: "NB_ERR_CUTOFF", 3: "NB_ERR_OOM", 4: "NB_ERR_HIP",
                5: "NB_ERR_STATE", 6: "NB_ERR_OVERFLOW", 7: "NB_ERR_LIST_STALE",
                8: "NB_ERR_NONFINITE", 9: "NB_ERR_IO", 10: "NB_ERR_RANGE"}

EXPORTS = ["nb_validate_params", "nb_setup", "nb_set_lj", "nb_set_stream", "nb_pairlist", "nb_prune",
           "nb_forces", "nb_forces_virial", "nb_check", "nb_backward", "nb_backward_noalloc", "nb_md_leapfrog",
           "nb_debug_pairs", "nb_get_stats",
           "nb_last_error", "nb_destroy", "nb_set_timing", "nb_get_timing", "nb_batch_setup",
           "nb_batch_set_schedule", "nb_batch_tune_schedule", "nb_batch_pairlist", "nb_batch_forces",
           "nb_batch_graph_forces", "nb_batch_get_info", "nb_batch_check", "nb_batch_last_error",
           "nb_batch_destroy", "nb_autotune", "nb_autotune_last_error", "nb_pme_setup", "nb_pme_forces", "nb_pme_last_error", "nb_pme_destroy"]

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)
_vp = ctypes.c_void_p


class nb_params(ctypes.Structure):
    _fields_ = [("box", ctypes.c_double * 3), ("cutoff", ctypes.c_double),
                ("buffer", ctypes.c_double), ("ewald_beta", ctypes.c_double),
                ("coulomb_const", ctypes.c_double), ("ntypes", ctypes.c_int32),
                ("sigma", _dp), ("epsilon", _dp), ("natoms", ctypes.c_int32),
                ("excl_off", _ip), ("excl_idx", _ip), ("flags", ctypes.c_uint32),
                ("cluster", ctypes.c_int32), ("elec", ctypes.c_int32), ("vdw", ctypes.c_int32),
                ("epsilon_rf", ctypes.c_double), ("rswitch", ctypes.c_double)]


class nb_stats(ctypes.Structure):
    _fields_ = [("natoms", ctypes.c_int64), ("nclusters", ctypes.c_int64),
                ("npadded", ctypes.c_int64), ("nentries", ctypes.c_int64),
                ("evaluated_pairs", ctypes.c_int64), ("list_capacity", ctypes.c_int64),
                ("cluster", ctypes.c_int32), ("ncolumns", ctypes.c_int32),
                ("build_ms_last", ctypes.c_double), ("work_units", ctypes.c_int32),
                ("unit_batches", ctypes.c_int32), ("max_list_batches", ctypes.c_int32),
                ("pruned", ctypes.c_int32), ("list_hist", ctypes.c_int32 * 8)]


class nb_batch_info(ctypes.Structure):
    _fields_ = [("nbox", ctypes.c_int32), ("sorted", ctypes.c_int32), ("natoms", ctypes.c_int64),
                ("nitems", ctypes.c_int64), ("nentries", ctypes.c_int64),
                ("evaluated_pairs", ctypes.c_int64), ("grid_blocks", ctypes.c_int32 * 2),
                ("graph_ready", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("build_ms_last", ctypes.c_double)]


NB_TUNE_BUCKETS, NB_TUNE_NMIN, NB_TUNE_NMAX, NB_TUNE_SAMPLE = 5, 3000, 30000, 16


class nb_tune_result(ctypes.Structure):
    _fields_ = [("nbuckets", ctypes.c_int32), ("bucket_lo", ctypes.c_int32 * NB_TUNE_BUCKETS),
                ("bucket_hi", ctypes.c_int32 * NB_TUNE_BUCKETS),
                ("bucket_boxes", ctypes.c_int32 * NB_TUNE_BUCKETS),
                ("bucket_cluster", ctypes.c_int32 * NB_TUNE_BUCKETS),
                ("bucket_cached", ctypes.c_int32 * NB_TUNE_BUCKETS),
                ("bucket_us", (ctypes.c_double * 2) * NB_TUNE_BUCKETS),
                ("sorted", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32),
                ("schedule_cached", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("schedule_us", ctypes.c_double * 5), ("seconds", ctypes.c_double)]


class nb_pme_params(ctypes.Structure):
    _fields_ = [("box", ctypes.c_double * 3), ("ewald_beta", ctypes.c_double),
                ("coulomb_const", ctypes.c_double), ("grid", ctypes.c_int32 * 3),
                ("order", ctypes.c_int32), ("natoms", ctypes.c_int32)]


class NbError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


_lib = None


def lib():
    """Load libnb.so (built by paper_2405_01420_amd.build); raises if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2405_01420_amd.build` (no CPU fallback exists)")
        L = ctypes.CDLL(LIB_PATH)
        ci, cu, ci64 = ctypes.c_int, ctypes.c_uint32, ctypes.c_int64
        P = ctypes.POINTER
        L.nb_validate_params.argtypes = [P(nb_params)]
        L.nb_setup.argtypes = [P(_vp), P(nb_params), _vp]
        L.nb_set_lj.argtypes = [_vp, _dp, _dp]
        L.nb_set_stream.argtypes = [_vp, _vp]
        L.nb_pairlist.argtypes = [_vp, _vp]
        L.nb_prune.argtypes = [_vp, _vp, ctypes.c_double]
        L.nb_forces.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp]
        L.nb_forces_virial.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, _vp]
        L.nb_check.argtypes = [_vp]
        L.nb_backward.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, cu]
        L.nb_backward_noalloc.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]
        L.nb_md_leapfrog.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, ctypes.c_double, ctypes.c_int32,
                                     ctypes.c_int32, ctypes.c_double, ctypes.c_int32, _vp, _vp]
        L.nb_debug_pairs.argtypes = [_vp, _vp, _vp, ci64, P(ci64)]
        L.nb_get_stats.argtypes = [_vp, P(nb_stats)]
        L.nb_last_error.argtypes = [_vp]
        L.nb_last_error.restype = ctypes.c_char_p
        L.nb_destroy.argtypes = [_vp]
        L.nb_set_timing.argtypes = [_vp, ci]
        L.nb_batch_setup.argtypes = [P(_vp), ctypes.c_int32, _vp, _vp, _vp, P(nb_params), _vp]
        L.nb_batch_set_schedule.argtypes = [_vp, ctypes.c_int32, ctypes.c_int32]
        L.nb_batch_tune_schedule.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, ctypes.c_int32, _dp, _ip]
        L.nb_batch_pairlist.argtypes = [_vp, _vp]
        L.nb_batch_forces.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp]
        L.nb_batch_graph_forces.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp]
        L.nb_batch_get_info.argtypes = [_vp, P(nb_batch_info)]
        L.nb_batch_check.argtypes = [_vp]
        L.nb_batch_last_error.argtypes = [_vp]
        L.nb_batch_last_error.restype = ctypes.c_char_p
        L.nb_batch_destroy.argtypes = [_vp]
        L.nb_autotune.argtypes = [ctypes.c_int32, _vp, _vp, P(nb_params), _vp, _vp, _vp,
                                  ctypes.c_char_p, _vp, _vp, P(nb_tune_result)]
        L.nb_autotune_last_error.argtypes = []
        L.nb_autotune_last_error.restype = ctypes.c_char_p
        L.nb_get_timing.argtypes = [_vp, P(ctypes.c_double), P(ci64)]
        L.nb_pme_setup.argtypes = [P(_vp), P(nb_pme_params), _vp]
        L.nb_pme_forces.argtypes = [_vp, _vp, _vp, _vp, _vp]
        L.nb_pme_last_error.argtypes = [_vp]
        L.nb_pme_last_error.restype = ctypes.c_char_p
        L.nb_pme_destroy.argtypes = [_vp]
        for name in EXPORTS:
            fn = getattr(L, name, None)
            if fn is not None and name not in ("nb_last_error", "nb_batch_last_error", "nb_pme_last_error",
                                               "nb_autotune_last_error"):
                fn.restype = ci
        _lib = L
    return _lib


def _check(code: int, ctx=None):
    if code != NB_OK:
        msg = lib().nb_last_error(ctx).decode(errors="replace")
        raise NbError(code, msg)


def _ptr(t) -> int:
    """Device pointer of a torch tensor (or an int / None)."""
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _stream(stream) -> Optional[int]:
    if stream is not None:
        return int(stream)
    import torch
    return int(torch.cuda.current_stream().cuda_stream)


class Params:
    """Host-side parameter block (keeps the arrays alive while the C struct points at them)."""

    def __init__(self, natoms: int, box: Sequence[float], cutoff: float, buffer: float,
                 ewald_beta: float, coulomb_const: float, sigma, epsilon, excl_off=None,
                 excl_idx=None, flags: int = 0, cluster: int = 8, elec: int = 0, vdw: int = 0,
                 epsilon_rf: float = 0.0, rswitch: float = 0.0):
        self.sigma = np.ascontiguousarray(sigma, dtype=np.float64)
        self.epsilon = np.ascontiguousarray(epsilon, dtype=np.float64)
        self.excl_off = None if excl_off is None else np.ascontiguousarray(excl_off, dtype=np.int32)
        self.excl_idx = None if excl_idx is None else np.ascontiguousarray(excl_idx, dtype=np.int32)
        if self.excl_idx is not None and len(self.excl_idx) == 0:
            self.excl_idx = np.zeros(1, np.int32)
        b = list(box) if not np.isscalar(box) else [box] * 3
        self.c = nb_params()
        self.c.box = (ctypes.c_double * 3)(*[float(v) for v in b])
        self.c.cutoff, self.c.buffer = float(cutoff), float(buffer)
        self.c.ewald_beta, self.c.coulomb_const = float(ewald_beta), float(coulomb_const)
        self.c.ntypes = len(self.sigma)
        self.c.sigma = self.sigma.ctypes.data_as(_dp)
        self.c.epsilon = self.epsilon.ctypes.data_as(_dp)
        self.c.natoms = int(natoms)
        self.c.excl_off = None if self.excl_off is None else self.excl_off.ctypes.data_as(_ip)
        self.c.excl_idx = None if self.excl_idx is None else self.excl_idx.ctypes.data_as(_ip)
        self.c.flags = int(flags)
        self.c.cluster = int(cluster)
        self.c.elec, self.c.vdw = int(elec), int(vdw)
        self.c.epsilon_rf, self.c.rswitch = float(epsilon_rf), float(rswitch)

    @classmethod
    def from_instance(cls, inst, flags: int = 0, cluster: int = 8, buffer: Optional[float] = None,
                      elec: int = 0, vdw: int = 0, epsilon_rf: float = 0.0, rswitch: float = 0.0):
        return cls(inst.natoms, [inst.box] * 3, inst.cutoff,
                   inst.buffer if buffer is None else buffer, inst.beta, inst.coulomb_const,
                   inst.sigma, inst.epsilon, inst.excl_off, inst.excl_idx, flags, cluster,
                   elec, vdw, epsilon_rf, rswitch)


def nb_validate_params(params: Params) -> int:
    """Returns the status code (0 = valid); never touches the GPU."""
    return int(lib().nb_validate_params(ctypes.byref(params.c)))


def nb_setup(params: Params, stream=None) -> int:
    h = _vp()
    _check(lib().nb_setup(ctypes.byref(h), ctypes.byref(params.c), _stream(stream)))
    return h.value


def nb_set_lj(ctx: int, sigma, epsilon) -> None:
    s = np.ascontiguousarray(sigma, dtype=np.float64)
    e = np.ascontiguousarray(epsilon, dtype=np.float64)
    _check(lib().nb_set_lj(ctx, s.ctypes.data_as(_dp), e.ctypes.data_as(_dp)), ctx)


def nb_set_stream(ctx: int, stream=None) -> None:
    _check(lib().nb_set_stream(ctx, _stream(stream)), ctx)


def nb_pairlist(ctx: int, x) -> None:
    _check(lib().nb_pairlist(ctx, _ptr(x)), ctx)


def nb_prune(ctx: int, x, r_inner: float) -> None:
    """Rolling prune of the last build's list to the pairs within r_inner at positions x."""
    _check(lib().nb_prune(ctx, _ptr(x), ctypes.c_double(r_inner)), ctx)


def nb_forces(ctx: int, x, q, types, f, e) -> None:
    _check(lib().nb_forces(ctx, _ptr(x), _ptr(q), _ptr(types), _ptr(f), _ptr(e)), ctx)


def nb_forces_virial(ctx: int, x, q, types, f, e, vir) -> None:
    """nb_forces plus the virial -1/2 sum d (x) F_ij into vir (device float64, 9 values)."""
    _check(lib().nb_forces_virial(ctx, _ptr(x), _ptr(q), _ptr(types), _ptr(f), _ptr(e), _ptr(vir)),
           ctx)


def nb_check(ctx: int) -> int:
    """Returns the status code of the device-side checks (0 = none raised)."""
    return int(lib().nb_check(ctx))


def nb_backward(ctx: int, x, q, types, g_f, g_e, dx, dq, dsigma, deps, flags: int = 0) -> None:
    _check(lib().nb_backward(ctx, _ptr(x), _ptr(q), _ptr(types), _ptr(g_f), _ptr(g_e), _ptr(dx),
                             _ptr(dq), _ptr(dsigma), _ptr(deps), int(flags)), ctx)


def nb_md_leapfrog(ctx: int, x, v, q, types, inv_mass, dt: float, nsteps: int, nstlist: int,
                   f, e_steps, r_inner: float = 0.0, nstprune: int = 1) -> None:
    _check(lib().nb_md_leapfrog(ctx, _ptr(x), _ptr(v), _ptr(q), _ptr(types), _ptr(inv_mass),
                                float(dt), int(nsteps), int(nstlist), float(r_inner), int(nstprune),
                                _ptr(f), _ptr(e_steps)), ctx)


def nb_backward_noalloc(ctx: int, x, q, types, g_f, g_e, dx, dq, dsigma, deps) -> None:
    _check(lib().nb_backward_noalloc(ctx, _ptr(x), _ptr(q), _ptr(types), _ptr(g_f), _ptr(g_e),
                                     _ptr(dx), _ptr(dq), _ptr(dsigma), _ptr(deps)), ctx)


def nb_debug_pairs(ctx: int, x, cap: int, count_only: bool = False):
    """Interacting pairs as an int64 [count, 2] array (i < j, original indices, unsorted);
    with count_only, just the number of interacting pairs."""
    cnt = ctypes.c_int64(0)
    if count_only:
        _check(lib().nb_debug_pairs(ctx, _ptr(x), None, 0, ctypes.byref(cnt)), ctx)
        return int(cnt.value)
    buf = np.zeros((max(cap, 1), 2), dtype=np.int64)
    _check(lib().nb_debug_pairs(ctx, _ptr(x), buf.ctypes.data, int(cap), ctypes.byref(cnt)), ctx)
    if cnt.value > cap:
        return nb_debug_pairs(ctx, x, int(cnt.value))
    return buf[:cnt.value]


def nb_get_stats(ctx: int) -> dict:
    st = nb_stats()
    _check(lib().nb_get_stats(ctx, ctypes.byref(st)), ctx)
    out = {k: getattr(st, k) for k, _ in nb_stats._fields_}
    out["list_hist"] = list(st.list_hist)
    return out


def nb_last_error(ctx: Optional[int]) -> str:
    return lib().nb_last_error(ctx).decode(errors="replace")


def nb_destroy(ctx: int) -> None:
    _check(lib().nb_destroy(ctx))


def nb_set_timing(ctx: int, every) -> None:
    """Stamp every `every`-th force launch with a HIP event pair (True: all; False or 0: off)."""
    _check(lib().nb_set_timing(ctx, int(every)), ctx)


def nb_get_timing(ctx: int):
    """(summed force-kernel milliseconds, number of timed launches); resets the counters."""
    ms = ctypes.c_double(0)
    n = ctypes.c_int64(0)
    _check(lib().nb_get_timing(ctx, ctypes.byref(ms), ctypes.byref(n)), ctx)
    return ms.value, n.value


# ---- batched form ------------------------------------------------------------------------

def _bcheck(code: int, bt=None):
    if code != NB_OK:
        raise NbError(code, lib().nb_batch_last_error(bt).decode(errors="replace"))


def nb_batch_setup(atom_off, boxes, common: Params, clusters=None, stream=None) -> int:
    """atom_off: [nbox+1] ints, boxes: [nbox, 3] floats, common: Params over all atoms."""
    ao = np.ascontiguousarray(atom_off, dtype=np.int32)
    bx = np.ascontiguousarray(boxes, dtype=np.float64).reshape(-1, 3)
    cl = None if clusters is None else np.ascontiguousarray(clusters, dtype=np.int32)
    h = _vp()
    _bcheck(lib().nb_batch_setup(ctypes.byref(h), len(ao) - 1, ao.ctypes.data, bx.ctypes.data,
                                 None if cl is None else cl.ctypes.data, ctypes.byref(common.c),
                                 _stream(stream)))
    return h.value


def nb_batch_set_schedule(bt: int, sorted: bool = True, blocks_per_cu: int = 0) -> None:
    _bcheck(lib().nb_batch_set_schedule(bt, int(bool(sorted)), int(blocks_per_cu)), bt)


NB_BATCH_NSCHED = 5
# the candidate schedules of nb_batch_tune_schedule, in its order: (sorted, blocks_per_cu)
BATCH_SCHEDULES = [(True, 0), (True, 1), (True, 2), (True, 4), (False, 0)]


def nb_batch_tune_schedule(bt: int, x, q, types, f, e, reps: int = 5):
    """Times the candidate schedules on the batch's data and applies the fastest; returns
    ((sorted, blocks_per_cu), {schedule: us per call})."""
    us = (ctypes.c_double * NB_BATCH_NSCHED)()
    best = (ctypes.c_int32 * 2)()
    _bcheck(lib().nb_batch_tune_schedule(bt, _ptr(x), _ptr(q), _ptr(types), _ptr(f), _ptr(e), int(reps),
                                         ctypes.cast(us, _dp), ctypes.cast(best, _ip)), bt)
    return (bool(best[0]), int(best[1])), {s: us[k] for k, s in enumerate(BATCH_SCHEDULES)}


def nb_autotune_last_error() -> str:
    return lib().nb_autotune_last_error().decode(errors="replace")


def nb_autotune(atom_off, boxes, common: Params, x, q, types, cache_path: Optional[str] = None,
                stream=None):
    """Cluster size per box and schedule chosen by the library's tuner; returns
    (clusters [nbox], result dict)."""
    ao = np.ascontiguousarray(atom_off, dtype=np.int32)
    bx = np.ascontiguousarray(boxes, dtype=np.float64).reshape(-1, 3)
    nbox = len(ao) - 1
    cl = np.zeros(nbox, dtype=np.int32)
    res = nb_tune_result()
    code = lib().nb_autotune(nbox, ao.ctypes.data, bx.ctypes.data, ctypes.byref(common.c), _ptr(x),
                             _ptr(q), _ptr(types),
                             None if cache_path is None else os.fsencode(cache_path),
                             _stream(stream), cl.ctypes.data, ctypes.byref(res))
    if code != NB_OK:
        raise NbError(code, nb_autotune_last_error())
    out = {"sorted": bool(res.sorted), "blocks_per_cu": int(res.blocks_per_cu),
           "schedule_cached": bool(res.schedule_cached),
           "schedule_us": {s: res.schedule_us[k] for k, s in enumerate(BATCH_SCHEDULES)},
           "seconds": res.seconds, "buckets": []}
    for k in range(res.nbuckets):
        out["buckets"].append({"atoms": (int(res.bucket_lo[k]), int(res.bucket_hi[k])),
                               "boxes": int(res.bucket_boxes[k]),
                               "cluster": int(res.bucket_cluster[k]),
                               "cached": bool(res.bucket_cached[k]),
                               "us": {4: res.bucket_us[k][0], 8: res.bucket_us[k][1]}})
    return [int(c) for c in cl], out


def nb_batch_pairlist(bt: int, x) -> None:
    _bcheck(lib().nb_batch_pairlist(bt, _ptr(x)), bt)


def nb_batch_forces(bt: int, x, q, types, f, e) -> None:
    _bcheck(lib().nb_batch_forces(bt, _ptr(x), _ptr(q), _ptr(types), _ptr(f), _ptr(e)), bt)


def nb_batch_graph_forces(bt: int, x, q, types, f, e) -> None:
    _bcheck(lib().nb_batch_graph_forces(bt, _ptr(x), _ptr(q), _ptr(types), _ptr(f), _ptr(e)), bt)


def nb_batch_check(bt: int) -> int:
    """Status of the batch's device-side checks (0 = none raised); clears them."""
    return int(lib().nb_batch_check(bt))


def nb_batch_get_info(bt: int) -> dict:
    st = nb_batch_info()
    _bcheck(lib().nb_batch_get_info(bt, ctypes.byref(st)), bt)
    out = {k: getattr(st, k) for k, _ in nb_batch_info._fields_ if k != "pad"}
    out["grid_blocks"] = list(st.grid_blocks)
    return out


def nb_batch_last_error(bt: Optional[int]) -> str:
    return lib().nb_batch_last_error(bt).decode(errors="replace")


def nb_batch_destroy(bt: int) -> None:
    _bcheck(lib().nb_batch_destroy(bt))


def concat_instances(insts, cluster: int = 8, flags: int = 0, clusters=None, elec: int = 0,
                     vdw: int = 0, epsilon_rf: float = 0.0, rswitch: float = 0.0):
    """Concatenate independent boxes into (atom_off, boxes, Params, x, q, type) for the batch
    API: exclusions are shifted to global indices, every box shares the LJ table of the first."""
    n = [i.natoms for i in insts]
    ao = np.concatenate([[0], np.cumsum(n)]).astype(np.int32)
    boxes = np.array([[i.box] * 3 for i in insts], dtype=np.float64)
    eo = [np.zeros(1, np.int64)]
    ei = []
    base = 0
    for k, inst in enumerate(insts):
        eo.append(inst.excl_off[1:].astype(np.int64) + base)
        ei.append(inst.excl_idx.astype(np.int64) + ao[k])
        base += int(inst.excl_off[-1])
    excl_off = np.concatenate(eo).astype(np.int32)
    excl_idx = np.concatenate(ei).astype(np.int32)
    i0 = insts[0]
    params = Params(int(ao[-1]), [i0.box] * 3, i0.cutoff, i0.buffer, i0.beta, i0.coulomb_const,
                    i0.sigma, i0.epsilon, excl_off, excl_idx, flags, cluster, elec, vdw,
                    epsilon_rf, rswitch)
    x = np.concatenate([i.x for i in insts]).astype(np.float32)
    q = np.concatenate([i.q for i in insts]).astype(np.float32)
    t = np.concatenate([i.type for i in insts]).astype(np.int32)
    return ao, boxes, params, x, q, t


# ---- reciprocal-space Ewald (smooth PME) --------------------------------------------------

def _pcheck(code: int, pme=None):
    if code != NB_OK:
        raise NbError(code, lib().nb_pme_last_error(pme).decode(errors="replace"))


def pme_params(box, beta: float, coulomb_const: float, grid, order: int, natoms: int) -> nb_pme_params:
    p = nb_pme_params()
    b = [box] * 3 if np.isscalar(box) else list(box)
    for a in range(3):
        p.box[a] = float(b[a])
        p.grid[a] = int(grid[a])
    p.ewald_beta = float(beta)
    p.coulomb_const = float(coulomb_const)
    p.order = int(order)
    p.natoms = int(natoms)
    return p


def nb_pme_setup(params: nb_pme_params, stream=None) -> int:
    h = _vp()
    _pcheck(lib().nb_pme_setup(ctypes.byref(h), ctypes.byref(params), _stream(stream)))
    return h.value


def nb_pme_forces(pme: int, x, q, f, e) -> None:
    _pcheck(lib().nb_pme_forces(pme, _ptr(x), _ptr(q), _ptr(f), _ptr(e)), pme)


def nb_pme_last_error(pme: Optional[int]) -> str:
    return lib().nb_pme_last_error(pme).decode(errors="replace")


def nb_pme_destroy(pme: int) -> None:
    _pcheck(lib().nb_pme_destroy(pme))
