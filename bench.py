"""Benchmark of the short-range nonbonded force path on one MI355X.

Workload (the method's headline configuration): 32,000 rigid waters (96,000 atoms) in a
9.87 nm periodic box, rc = 1.0 nm, list buffer 0.1 nm, Ewald beta from erfc(beta rc) = 1e-5.
A step is one force + energy call (pack, cluster-pair force kernel, finalize) on positions that
follow a random walk N(0, 0.002 nm) per call without re-wrapping; every 10th step first rebuilds
the pair list (grid sort, search, masks, prune), so list construction is included amortised.
The whole trajectory is generated on the GPU before timing, so inputs are resident in HBM.

value = useful pair interactions per second (unordered, non-excluded pairs with r < rc,
counted at the start positions) over the timed steps.  The JSON line also carries the
force-kernel roofline (algorithmic FP32 flops per useful pair x useful pairs / the force
kernel's mean duration over the timed steps, from HIP event pairs that its dispatches stamp,
against the FP32 vector peak) and the FP64 oracle timed on the host as cpu_baseline.

Beside the headline line the JSON carries the two other forms against the plain kernel:
  batched - 256 independent boxes (3,000-30,000 atoms, log-uniform, rc 0.9 nm) in one persistent
            launch replayed from a HIP graph, with the autotuner's cluster sizes and schedule,
            against 256 sequential plain force calls on the same boxes;
  adjoint - the 24,000-atom four-type box: nb_backward (list reused, and with the list rebuilt
            from x) against nb_forces on the same box; and the adjoint on the 96k-atom box.
Further legs: small_boxes (the plain kernel on single 3,000-, 12,000- and 24,000-atom boxes with
its work units in cluster order and longest first, the post-prune list sorting); md (the
leapfrog loop nb_md_leapfrog on a 32,000-ion charged LJ fluid, with and without the rolling
prune); pme and ewald_step (the reciprocal part and the complete Ewald step).

With --large it also times single force calls on the 3,000,000-atom box (median of 20).

Usage: python bench.py [--gpus 1] [--steps 1000] [--warmup 20] [--cluster 8] [--cpu-seconds 12]
                       [--no-batch] [--no-adjoint] [--no-tune] [--no-pme] [--no-md] [--no-small]
                       [--no-cpu] [--large]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic FP32 work per useful pair (FMA = 2 flops, each transcendental = 1); see the
# breakdown in the design notes: displacement 3, r^2 5, rsq 1, r^-2/r^-6 3, LJ energy 4,
# LJ force 3, r 1, exp argument 1, exp 1, erfcx numerator 8, denominator 10, rcp + product 2,
# q_i q_j 1, Coulomb factor products 3, force factor 5, force vector 3, i/j force updates 6,
# energy sums 2, shift sums 3.
FLOPS_PER_PAIR = 65
# The other interaction flavours, counted the same way: the reaction field replaces the 27 flops
# of the Ewald Coulomb part (r, exp argument, exp, erfcx numerator and denominator, reciprocal
# and product, q_i q_j, Coulomb products) by 7 (q_i q_j 1, force factor 2, energy 4); the force
# switch adds 23 (t 2, t^2 1, force polynomials 4, combination 3, force update 3, energy
# polynomials 4, combination 3, energy update 3), plus r (1) where the reaction field left it out.
FLOPS_PER_PAIR_FLAVOUR = {("ewald", "shift"): 65, ("rf", "shift"): 45,
                          ("ewald", "fswitch"): 88, ("rf", "fswitch"): 69}
PEAK_FP32_VECTOR_TFLOPS = 157.3
REBUILD_EVERY = 10

# rocprofv3 counters of k_force on the 96k-atom box (profiles/k_force_water96k_counters.md):
# HBM bytes per launch from FETCH_SIZE and WRITE_SIZE, each scaled by the reading for a 256 MiB
# device copy (factors 2.0 and 1.0), and the counted FP32 VALU flops per launch
# (SQ_INSTS_VALU_FLOPS_FP32 x 64 lanes).  They describe the kernel built from the sources with
# this digest and are reported only while the sources are unchanged.
TIMING_EVERY = 7

K_FORCE_COUNTERS = {
    "sources": ["nb_force_body.h", "nb_force.hip", "nb_device.h", "nb_internal.h", "erfcx_rational.h"],
    "sha256": "d08835ff78032cc6dc476a7dc3da28a31d9828b70befb723d26c3a002154ea71",
    "read_bytes": 31.84e6, "write_bytes": 74.04e6,
    "counted_fp32_flop": 2580713401.7,
}


def _counters_current():
    import hashlib
    h = hashlib.sha256()
    for f in K_FORCE_COUNTERS["sources"]:
        with open(os.path.join(ROOT, "paper_2405_01420_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest() == K_FORCE_COUNTERS["sha256"]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--cluster", type=int, default=0, help="4 or 8 (0 = tuned or default 8)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-baseline-child", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--copy-probe", action="store_true",
                    help="end with one 256 MiB device-to-device copy (calibrates HBM byte counters)")
    ap.add_argument("--elec", choices=["ewald", "rf"], default="ewald",
                    help="electrostatics of the headline box (reaction field: eps_rf = infinity)")
    ap.add_argument("--vdw", choices=["shift", "fswitch"], default="shift",
                    help="Lennard-Jones cutoff treatment (force switch from --rswitch)")
    ap.add_argument("--rswitch", type=float, default=0.8)
    ap.add_argument("--large", action="store_true",
                    help="also time the 3,000,000-atom box (median of 20 force calls)")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-pme", action="store_true")
    ap.add_argument("--no-md", action="store_true")
    ap.add_argument("--no-small", action="store_true")
    ap.add_argument("--prune-every", type=int, default=0,
                    help="rolling-prune measurement: prune every this many calls (0: skip)")
    ap.add_argument("--prune-inner", type=float, default=0.05,
                    help="rolling-prune measurement: r_inner - rc (nm)")
    ap.add_argument("--no-tune", action="store_true", help="batched form with C = 8 everywhere")
    ap.add_argument("--energy-fp64", action="store_true",
                    help="evaluate Coulomb pair energies in FP64 (forces stay FP32)")
    return ap.parse_args()


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline_child(seconds):
    """Runs in a child process started by cpu_baseline (OpenMP placement set in its environment
    before the runtime starts): the FP64 oracle, cell-list enumeration on the 96,000-atom box
    repeated for about `seconds`, and the O(N^2) definition on the 648-atom box for about a
    tenth of that.  Prints one JSON object."""
    from oracle import oracle as O
    from paper_2405_01420_amd import synth
    inst = synth.mid()
    O.lib()
    r = O.instance_forces(inst, cells=True)  # warm
    useful = r.npairs
    t0 = time.perf_counter()
    calls = 0
    while True:
        O.instance_forces(inst, cells=True)
        calls += 1
        el = time.perf_counter() - t0
        if el >= seconds or calls >= 1000:
            break
    tiny = synth.tiny()
    rt = O.instance_forces(tiny, cells=False)
    t1 = time.perf_counter()
    ncalls_t = 0
    while True:
        O.instance_forces(tiny, cells=False)
        ncalls_t += 1
        el_t = time.perf_counter() - t1
        if el_t >= 0.1 * seconds or ncalls_t >= 10000:
            break
    print(json.dumps({"useful": useful, "calls": calls, "seconds": el, "threads": O.get_threads(),
                      "tiny_useful": rt.npairs, "tiny_calls": ncalls_t, "tiny_seconds": el_t}))


def cpu_baseline(seconds):
    """The FP64 oracle timed on all host cores in a child process with OMP_PLACES=cores and
    OMP_PROC_BIND=close (the parent's OpenMP runtime, loaded by torch, has already read its
    environment)."""
    import subprocess
    ncpu = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    env = dict(os.environ)
    env.setdefault("OMP_NUM_THREADS", str(ncpu))
    env["OMP_PLACES"] = "cores"
    env["OMP_PROC_BIND"] = "close"
    r = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-baseline-child",
                        "--cpu-seconds", str(seconds)], env=env, capture_output=True, text=True,
                       check=True)
    c = json.loads(r.stdout.strip().splitlines()[-1])
    per_call = c["seconds"] / c["calls"]
    per_tiny = c["tiny_seconds"] / c["tiny_calls"]
    return {"value": c["useful"] / per_call, "unit": "pair-interactions/s",
            "cores": c["threads"], "kind": "oracle",
            "sample": f"{c['calls']} full force+energy calls of the FP64 cell-list oracle on the "
                      f"96,000-atom box ({c['seconds']:.1f} s); per call {1e6 * per_call:.0f} us",
            "cpu_model": _cpu_model(), "nproc": ncpu, "omp_num_threads": env["OMP_NUM_THREADS"],
            "omp_places": env["OMP_PLACES"], "omp_proc_bind": env["OMP_PROC_BIND"],
            "us_per_call_cell_list_96k": 1e6 * per_call,
            "o_n2_tiny": {"workload": "648-atom water box, O(N^2) brute force (the definition)",
                          "us_per_call": 1e6 * per_tiny, "calls": c["tiny_calls"],
                          "pair_interactions_per_s": c["tiny_useful"] / per_tiny}}


def _event_us(torch, stream, fn, reps):
    """Average microseconds of fn() over reps calls, HIP events on `stream`."""
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    stream.synchronize()
    return 1e3 * e0.elapsed_time(e1) / reps


def bench_batched(torch, nb, synth, tune_on, reps=20):
    """256 uneven boxes: one persistent graph-replayed launch vs 256 sequential plain calls, in
    the FP64 pair-energy mode (the energy mode that holds 1e-6 on boxes of 3,000-30,000 atoms)
    and in the FP32 pair-energy mode (E_C held to 1e-5 on such boxes)."""
    from paper_2405_01420_amd import tune
    dev = "cuda:0"
    insts = synth.batch(256)
    stream = torch.cuda.Stream()
    out = {"workload": "256 water boxes, 3,000-30,000 atoms log-uniform (multiples of 3), "
                       "100 atoms/nm^3, rc 0.9 nm, rb 0.1 nm"}
    useful = None
    for mode, flags in (("fp64_energy", nb.NB_ENERGY_FP64), ("fp32_energy", 0)):
        tuned = None
        if tune_on:
            tuned = tune.autotune(insts, flags=flags)
            clusters, srt, bpc = tuned["clusters"], tuned["sorted"], tuned["blocks_per_cu"]
        else:
            clusters, srt, bpc = [8] * len(insts), True, 0
        ao, bx, params, x, q, t = nb.concat_instances(insts, clusters=clusters, flags=flags)
        n = int(ao[-1])
        bt = nb.nb_batch_setup(ao, bx, params, clusters=clusters, stream=stream.cuda_stream)
        nb.nb_batch_set_schedule(bt, srt, bpc)
        with torch.cuda.stream(stream):
            dx = torch.from_numpy(x.reshape(-1)).to(dev)
            dq = torch.from_numpy(q).to(dev)
            dt = torch.from_numpy(t).to(dev)
            f = torch.empty(3 * n, dtype=torch.float32, device=dev)
            e = torch.empty(2 * len(insts), dtype=torch.float64, device=dev)
        stream.synchronize()
        nb.nb_batch_pairlist(bt, dx)
        info = nb.nb_batch_get_info(bt)
        for _ in range(3):
            nb.nb_batch_graph_forces(bt, dx, dq, dt, f, e)
            nb.nb_batch_forces(bt, dx, dq, dt, f, e)
        us_graph = _event_us(torch, stream, lambda: nb.nb_batch_graph_forces(bt, dx, dq, dt, f, e), reps)
        us_eager = _event_us(torch, stream, lambda: nb.nb_batch_forces(bt, dx, dq, dt, f, e), reps)
        nb.nb_batch_destroy(bt)
        # the same boxes one after another through the plain path (C = 8, lists prebuilt)
        plain = []
        count = useful is None
        nuse = 0
        for k, inst in enumerate(insts):
            ctx = nb.nb_setup(nb.Params.from_instance(inst, flags=flags), stream=stream.cuda_stream)
            a, b = int(ao[k]), int(ao[k + 1])
            xs, qs, ts = dx[3 * a:3 * b], dq[a:b], dt[a:b]
            fs = f[3 * a:3 * b]
            es = e[2 * k:2 * k + 2]
            nb.nb_pairlist(ctx, xs)
            if count:
                nuse += nb.nb_debug_pairs(ctx, xs, 0, count_only=True)
            plain.append((ctx, xs, qs, ts, fs, es))
        if count:
            useful = nuse

        def seq():
            for ctx, xs, qs, ts, fs, es in plain:
                nb.nb_forces(ctx, xs, qs, ts, fs, es)
        seq()
        us_seq = _event_us(torch, stream, seq, max(3, reps // 4))
        for p in plain:
            nb.nb_destroy(p[0])
        r = {"energy_gate": "1e-6 (E_LJ, E_C)" if flags else "E_LJ 1e-6, E_C 1e-5",
             "us_per_batch_call_graph": us_graph, "us_per_batch_call_eager": us_eager,
             "us_256_sequential_plain_calls": us_seq,
             "pair_interactions_per_s_graph": useful / (us_graph * 1e-6),
             "pair_interactions_per_s_sequential": useful / (us_seq * 1e-6),
             "speedup_vs_sequential": us_seq / us_graph,
             "clusters": {"4": clusters.count(4), "8": clusters.count(8)},
             "schedule": {"sorted": bool(srt), "blocks_per_cu": int(bpc)},
             "evaluated_pairs": info["evaluated_pairs"]}
        if tuned is not None:
            r["tune_s"] = tuned["tune_s"]
            r["tuner_buckets"] = [{"atoms": list(b["atoms"]), "boxes": b["boxes"], "cluster": b["cluster"],
                                   "us_c4": b["us"][4], "us_c8": b["us"][8]}
                                  for b in tuned["buckets"] if b["boxes"] > 0]
            r["tuner_schedule_us"] = {f"sorted={k[0]},bpc={k[1]}": v for k, v in tuned["schedule_us"].items()}
        out[mode] = r
    out["natoms"] = n
    out["useful_pairs"] = useful
    return out


def bench_adjoint(torch, nb, synth, reps=50):
    """nb_backward vs nb_forces on the 24,000-atom differentiation box; the force call in the
    FP64 pair-energy mode (the mode that holds the 1e-6 energy gate on this machine along a walk)
    and in the FP32 mode.  The adjoint's gradients are held to 5e-6 (fixed cotangents)."""
    dev = "cuda:0"
    inst = synth.diff()
    stream = torch.cuda.current_stream()
    n = inst.natoms
    x = torch.from_numpy(inst.x.reshape(-1).copy()).to(dev)
    q = torch.from_numpy(inst.q.copy()).to(dev)
    t = torch.from_numpy(inst.type.copy()).to(dev)
    f = torch.empty(3 * n, dtype=torch.float32, device=dev)
    e = torch.empty(2, dtype=torch.float64, device=dev)
    g = torch.Generator(device=dev)
    g.manual_seed(7)
    gf = torch.randn(3 * n, generator=g, device=dev)
    ge = torch.tensor([0.3, -0.7], dtype=torch.float64, device=dev)
    ddx = torch.empty(3 * n, dtype=torch.float32, device=dev)
    ddq = torch.empty(n, dtype=torch.float32, device=dev)
    ds = torch.empty(inst.ntypes, dtype=torch.float64, device=dev)
    de = torch.empty(inst.ntypes, dtype=torch.float64, device=dev)
    us_f = {}
    for mode, flags in (("fp64_energy", nb.NB_ENERGY_FP64), ("fp32_energy", 0)):
        cf = nb.nb_setup(nb.Params.from_instance(inst, flags=flags), stream=stream.cuda_stream)
        nb.nb_pairlist(cf, x)
        nb.nb_forces(cf, x, q, t, f, e)
        us_f[mode] = _event_us(torch, stream, lambda: nb.nb_forces(cf, x, q, t, f, e), reps)
        nb.nb_destroy(cf)
    ctx = nb.nb_setup(nb.Params.from_instance(inst), stream=stream.cuda_stream)
    nb.nb_pairlist(ctx, x)
    useful = nb.nb_debug_pairs(ctx, x, 0, count_only=True)
    bw = lambda fl: nb.nb_backward(ctx, x, q, t, gf, ge, ddx, ddq, ds, de, fl)
    bw(nb.NB_REUSE_LIST)
    us_b = _event_us(torch, stream, lambda: bw(nb.NB_REUSE_LIST), reps)
    us_b_build = _event_us(torch, stream, lambda: bw(0), max(5, reps // 5))
    nb.nb_destroy(ctx)
    # the adjoint on the headline box (96k atoms), beside its force call
    mid = synth.mid()
    nm = mid.natoms
    xm = torch.from_numpy(mid.x.reshape(-1).copy()).to(dev)
    qm = torch.from_numpy(mid.q.copy()).to(dev)
    tm = torch.from_numpy(mid.type.copy()).to(dev)
    fm = torch.empty(3 * nm, dtype=torch.float32, device=dev)
    em = torch.empty(2, dtype=torch.float64, device=dev)
    gfm = torch.randn(3 * nm, generator=g, device=dev)
    dxm = torch.empty(3 * nm, dtype=torch.float32, device=dev)
    dqm = torch.empty(nm, dtype=torch.float32, device=dev)
    dsm = torch.empty(mid.ntypes, dtype=torch.float64, device=dev)
    dem = torch.empty(mid.ntypes, dtype=torch.float64, device=dev)
    cm = nb.nb_setup(nb.Params.from_instance(mid), stream=stream.cuda_stream)
    nb.nb_pairlist(cm, xm)
    useful_m = nb.nb_debug_pairs(cm, xm, 0, count_only=True)
    nb.nb_forces(cm, xm, qm, tm, fm, em)
    us_fm = _event_us(torch, stream, lambda: nb.nb_forces(cm, xm, qm, tm, fm, em), reps)
    bwm = lambda: nb.nb_backward(cm, xm, qm, tm, gfm, ge, dxm, dqm, dsm, dem, nb.NB_REUSE_LIST)
    bwm()
    us_bm = _event_us(torch, stream, bwm, reps)
    nb.nb_destroy(cm)
    return {"workload": "24,000-atom water box (8,000 waters, L 6.21 nm), 4 LJ types, "
                        "charges perturbed, rc 1.0 nm",
            "water_96k": {"useful_pairs": useful_m, "us_per_force_call_fp32_energy": us_fm,
                          "us_per_backward_call": us_bm, "backward_over_forces": us_bm / us_fm,
                          "pair_interactions_per_s_backward": useful_m / (us_bm * 1e-6)},
            "useful_pairs": useful,
            "us_per_force_call": us_f["fp64_energy"],
            "us_per_force_call_fp32_energy": us_f["fp32_energy"],
            "us_per_backward_call": us_b, "us_per_backward_call_with_list_rebuild": us_b_build,
            "backward_over_forces": us_b / us_f["fp64_energy"],
            "backward_over_forces_fp32_energy": us_b / us_f["fp32_energy"],
            "pair_interactions_per_s_backward": useful / (us_b * 1e-6)}


def bench_pme(torch, nb, synth, reps=50):
    """Reciprocal-space Ewald (smooth PME) of the 96k-atom water box: grid spacing ~0.1 nm,
    B-splines of order 4, event-timed calls (spread, FFTs, solve, gather)."""
    inst = synth.mid()
    dev = "cuda:0"
    K = 96
    pm = nb.nb_pme_setup(nb.pme_params(inst.box, inst.beta, inst.coulomb_const, (K, K, K), 4, inst.natoms))
    x = torch.from_numpy(inst.x.reshape(-1)).to(dev)
    q = torch.from_numpy(inst.q).to(dev)
    f = torch.zeros(inst.natoms * 3, dtype=torch.float32, device=dev)
    e = torch.zeros(1, dtype=torch.float64, device=dev)
    for _ in range(3):
        nb.nb_pme_forces(pm, x, q, f, e)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(reps):
        nb.nb_pme_forces(pm, x, q, f, e)
    ev1.record()
    torch.cuda.synchronize()
    nb.nb_pme_destroy(pm)
    return {"workload": "96k-atom water box, smooth PME, 96^3 grid (0.103 nm), B-spline order 4, FP64 grid and FFT",
            "us_per_call": 1e3 * ev0.elapsed_time(ev1) / reps}


def bench_ewald_step(torch, nb, synth, reps=50):
    """The complete Ewald force step of the 96k-atom box: real space with the exclusion
    correction and self term (nb_forces, NB_EWALD_CORR) and the reciprocal part (nb_pme_forces,
    96^3 grid, order 4).  Timed one after the other, and with the two on separate streams
    (default priority) joined at the end of every step, the way an MD step would overlap them."""
    inst = synth.mid()
    dev = "cuda:0"
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    ctx = nb.nb_setup(nb.Params.from_instance(inst, flags=nb.NB_EWALD_CORR), stream=s1.cuda_stream)
    pm = nb.nb_pme_setup(nb.pme_params(inst.box, inst.beta, inst.coulomb_const, (96, 96, 96), 4, inst.natoms),
                         stream=s2.cuda_stream)
    with torch.cuda.stream(s1):
        x = torch.from_numpy(inst.x.reshape(-1)).to(dev)
        q = torch.from_numpy(inst.q).to(dev)
        t = torch.from_numpy(inst.type).to(dev)
        fr = torch.zeros(inst.natoms * 3, dtype=torch.float32, device=dev)
        fk = torch.zeros(inst.natoms * 3, dtype=torch.float32, device=dev)
        er = torch.zeros(4, dtype=torch.float64, device=dev)
        ek = torch.zeros(1, dtype=torch.float64, device=dev)
    s1.synchronize()
    nb.nb_pairlist(ctx, x)

    def step(overlap):
        s2.wait_stream(s1)          # the step's inputs are ready on s1
        nb.nb_forces(ctx, x, q, t, fr, er)
        if not overlap:
            s2.wait_stream(s1)
        nb.nb_pme_forces(pm, x, q, fk, ek)
        s1.wait_stream(s2)          # both parts done before the next step

    out = {"workload": "96k-atom water box: real-space Ewald + exclusion correction + self term, "
                       "smooth PME 96^3 order 4 (FP64)"}
    for name, overlap in (("us_per_step_serial", False), ("us_per_step_two_streams", True)):
        for _ in range(3):
            step(overlap)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(s1)
        for _ in range(reps):
            step(overlap)
        ev1.record(s1)
        torch.cuda.synchronize()
        out[name] = 1e3 * ev0.elapsed_time(ev1) / reps
    nb.nb_pme_destroy(pm)
    nb.nb_destroy(ctx)
    return out


def bench_md(torch, nb, synth, nsteps=400):
    """Leapfrog MD of a charged Lennard-Jones fluid (32,000 ions of +-0.5 e at water-oxygen
    density, 9.87 nm box, rc 1.0 nm, rb 0.1 nm, dt 2 fs, 300 K): list rebuilt every 10 steps
    (asynchronous builds), with and without the rolling prune to rc + 0.04 nm every 2 steps;
    microseconds per MD step (event-timed) and the total-energy drift (FP64 pair energies)."""
    import numpy as np
    dev = "cuda:0"
    inst, v0, im = synth.ionic_fluid(32000, 9.87)
    out = {"workload": "charged LJ fluid, 32,000 ions +-0.5 e, L 9.87 nm, rc 1.0 nm, rb 0.1 nm, "
                       "dt 2 fs, 300 K, nstlist 10, FP64 pair energies"}
    stream = torch.cuda.current_stream()
    for name, rin in (("prune_every_2_rc+0.04", inst.cutoff + 0.04), ("no_prune", 0.0)):
        ctx = nb.nb_setup(nb.Params.from_instance(inst, flags=nb.NB_ENERGY_FP64 | nb.NB_ASYNC_BUILD),
                          stream=stream.cuda_stream)
        x = torch.from_numpy(inst.x.reshape(-1).copy()).to(dev)
        v = torch.from_numpy(v0.reshape(-1).copy()).to(dev)
        q = torch.from_numpy(inst.q.copy()).to(dev)
        t = torch.from_numpy(inst.type.copy()).to(dev)
        m = torch.from_numpy(im.copy()).to(dev)
        f = torch.zeros(3 * inst.natoms, dtype=torch.float32, device=dev)
        e = torch.zeros((nsteps, 4), dtype=torch.float64, device=dev)
        nb.nb_md_leapfrog(ctx, x, v, q, t, m, 0.002, 20, 10, f, e, r_inner=rin, nstprune=2)
        us = _event_us(torch, stream, lambda: nb.nb_md_leapfrog(ctx, x, v, q, t, m, 0.002, nsteps, 10, f, e,
                                                                r_inner=rin, nstprune=2), 1) / nsteps
        nb.nb_pairlist(ctx, x)   # reads the status of the last asynchronous build
        et = e.cpu().numpy()
        nb.nb_destroy(ctx)
        slope = float(np.polyfit(np.arange(nsteps) * 0.002, et[:, 3], 1)[0])  # kJ/mol/ps
        out[name] = {"us_per_md_step": us,
                     "energy_drift_kj_mol_per_ns_per_atom": 1e3 * slope / inst.natoms,
                     "total_energy_spread_kj_mol": float(et[:, 3].max() - et[:, 3].min()),
                     "kinetic_energy_kj_mol": float(et[-1, 2])}
    return out


def bench_small_boxes(torch, nb, synth, reps=200):
    """The plain force kernel on single small water boxes (3,000, 12,000 and 24,000 atoms,
    rc 0.9 nm, rb 0.1 nm), with its work units in cluster order and longest first
    (NB_SORT_UNITS, the post-prune list sorting): kernel microseconds (HIP events around each
    launch), the list-length histogram and the work-unit split."""
    dev = "cuda:0"
    out = {"workload": "single water boxes at 100 atoms/nm^3, rc 0.9 nm, rb 0.1 nm, FP32 pair energies"}
    for natoms in (3000, 12000, 24000):
        inst = synth.small_box(natoms // 3, 0.9, 0.1, seed=50 + natoms // 3000)
        x = torch.from_numpy(inst.x.reshape(-1).copy()).to(dev)
        q = torch.from_numpy(inst.q.copy()).to(dev)
        t = torch.from_numpy(inst.type.copy()).to(dev)
        f = torch.empty(3 * inst.natoms, dtype=torch.float32, device=dev)
        e = torch.empty(2, dtype=torch.float64, device=dev)
        row = {}
        for name, flags in (("cluster_order", 0), ("longest_first", nb.NB_SORT_UNITS)):
            ctx = nb.nb_setup(nb.Params.from_instance(inst, flags=flags))
            nb.nb_pairlist(ctx, x)
            for _ in range(5):
                nb.nb_forces(ctx, x, q, t, f, e)
            nb.nb_set_timing(ctx, True)
            nb.nb_get_timing(ctx)
            for _ in range(reps):
                nb.nb_forces(ctx, x, q, t, f, e)
            ms, nl = nb.nb_get_timing(ctx)
            st = nb.nb_get_stats(ctx)
            if name == "cluster_order":
                row["useful_pairs"] = nb.nb_debug_pairs(ctx, x, 0, count_only=True)
                row["list_hist_log2_batches"] = st["list_hist"]
                row["work_units"] = st["work_units"]
                row["max_batches_per_unit"] = st["unit_batches"]
                row["longest_list_batches"] = st["max_list_batches"]
            row["kernel_us_" + name] = 1e3 * ms / nl
            nb.nb_destroy(ctx)
        row["pair_interactions_per_s_kernel"] = row["useful_pairs"] / (1e-6 * min(
            row["kernel_us_cluster_order"], row["kernel_us_longest_first"]))
        out[str(natoms)] = row
    return out


def bench_large(torch, nb, synth, reps=20, warmup=3):
    """3,000,000-atom box (rc 1.2 nm, 5 LJ types): median and IQR of single force calls."""
    import numpy as np
    dev = "cuda:0"
    inst = synth.large()
    stream = torch.cuda.current_stream()
    ctx = nb.nb_setup(nb.Params.from_instance(inst), stream=stream.cuda_stream)
    n = inst.natoms
    x = torch.from_numpy(inst.x.reshape(-1).copy()).to(dev)
    q = torch.from_numpy(inst.q.copy()).to(dev)
    t = torch.from_numpy(inst.type.copy()).to(dev)
    f = torch.empty(3 * n, dtype=torch.float32, device=dev)
    e = torch.empty(2, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    tb = time.perf_counter()
    nb.nb_pairlist(ctx, x)
    torch.cuda.synchronize()
    build_ms = 1e3 * (time.perf_counter() - tb)
    useful = nb.nb_debug_pairs(ctx, x, 0, count_only=True)
    stats = nb.nb_get_stats(ctx)
    for _ in range(warmup):
        nb.nb_forces(ctx, x, q, t, f, e)
    us = [_event_us(torch, stream, lambda: nb.nb_forces(ctx, x, q, t, f, e), 1) for _ in range(reps)]
    nb.nb_destroy(ctx)
    med = float(np.median(us))
    q1, q3 = (float(v) for v in np.percentile(us, [25, 75]))
    return {"workload": "3,000,000 atoms (1,000,000 waters), L 31.1 nm, rc 1.2 nm, rb 0.1 nm, "
                        "10% of atoms on 4 extra LJ types",
            "useful_pairs": useful, "evaluated_pairs": stats["evaluated_pairs"],
            "us_per_force_call_median": med, "us_per_force_call_iqr": [q1, q3],
            "pair_interactions_per_s": useful / (med * 1e-6), "ms_list_build": build_ms}


def main():
    args = parse()
    if args.cpu_baseline_child:
        cpu_baseline_child(args.cpu_seconds)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the force path is "
              "single-GPU and multi-GPU sharding is not built.", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2405_01420_amd import nb, synth

    dev = "cuda:0"
    inst = synth.mid()
    cluster = args.cluster or 8
    flav = dict(elec=nb.NB_ELEC_RF if args.elec == "rf" else nb.NB_ELEC_EWALD,
                vdw=nb.NB_VDW_FSWITCH if args.vdw == "fswitch" else nb.NB_VDW_SHIFT,
                rswitch=args.rswitch if args.vdw == "fswitch" else 0.0)
    flops_per_pair = FLOPS_PER_PAIR_FLAVOUR[(args.elec, args.vdw)]
    # asynchronous list builds: a build's overflow status is read at the next build, so the
    # host never drains the stream (checked after the timed loop)
    params = nb.Params.from_instance(inst, cluster=cluster,
                                     flags=(nb.NB_ENERGY_FP64 if args.energy_fp64 else 0) | nb.NB_ASYNC_BUILD,
                                     **flav)
    ctx = nb.nb_setup(params)
    n = inst.natoms
    nsteps = args.warmup + args.steps
    # random-walk trajectory, generated on the GPU ahead of timing
    g = torch.Generator(device=dev)
    g.manual_seed(20)
    traj = torch.empty((nsteps + 1, n * 3), dtype=torch.float32, device=dev)
    traj[0] = torch.from_numpy(inst.x.reshape(-1)).to(dev)
    for k in range(1, nsteps + 1):
        traj[k] = traj[k - 1] + 0.002 * torch.randn(n * 3, generator=g, device=dev)
    q = torch.from_numpy(inst.q).to(dev)
    t = torch.from_numpy(inst.type).to(dev)
    f = torch.zeros(n * 3, dtype=torch.float32, device=dev)
    e = torch.zeros(2, dtype=torch.float64, device=dev)

    nb.nb_pairlist(ctx, traj[0])
    useful = len(nb.nb_debug_pairs(ctx, traj[0], 400 * n))
    stats = nb.nb_get_stats(ctx)

    def step(k):
        if k % REBUILD_EVERY == 0:
            nb.nb_pairlist(ctx, traj[k])
        nb.nb_forces(ctx, traj[k], q, t, f, e)

    # force-kernel time: HIP event pairs stamped by the dispatches of every TIMING_EVERY-th force
    # kernel of the timed region (a prime, so that every position in the rebuild period is
    # sampled), on the library's stream (nb_set_timing; its events are created before the
    # warm-up).  A stamped dispatch costs a few microseconds more, so the other calls run
    # unstamped.
    nb.nb_set_timing(ctx, TIMING_EVERY)
    for k in range(args.warmup):
        step(k)
    # HIP events on the stream at the start of every rebuild period inside the timed region
    # give the spread over periods (median and IQR of microseconds per call); they add no
    # synchronisation
    marks = []
    torch.cuda.synchronize()
    nb.nb_get_timing(ctx)  # drops the warm-up launches
    t0 = time.perf_counter()
    for k in range(args.warmup, nsteps):
        if k % REBUILD_EVERY == 0:
            ev = torch.cuda.Event(enable_timing=True)
            ev.record()
            marks.append((k, ev))
        step(k)
    end_ev = torch.cuda.Event(enable_timing=True)
    end_ev.record()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kms, klaunch = nb.nb_get_timing(ctx)
    nb.nb_set_timing(ctx, False)
    kernel_us = 1e3 * kms / klaunch
    ms_per_step = 1e3 * elapsed / args.steps
    value = useful * args.steps / elapsed
    marks.append((nsteps, end_ev))
    period_us = [1e3 * a[1].elapsed_time(b[1]) / (b[0] - a[0])
                 for a, b in zip(marks[:-1], marks[1:]) if b[0] - a[0] == REBUILD_EVERY]
    period_stats = None
    if period_us:
        p25, p50, p75 = (float(v) for v in np.percentile(period_us, [25, 50, 75]))
        period_stats = {"periods": len(period_us), "us_per_call_median": p50,
                        "us_per_call_iqr": [p25, p75],
                        "pair_interactions_per_s_median": useful / (p50 * 1e-6)}
    # the last asynchronous build's status (raises NB_ERR_OVERFLOW if any list had overflowed)
    nb.nb_pairlist(ctx, traj[nsteps - 1])

    # rolling prune: the same walk with the list pruned to rc + prune_inner every prune_every
    # calls (valid while atoms move less than prune_inner / 2 between prunes: the walk moves
    # them ~0.0035 nm per call)
    prune = None
    if args.prune_every > 0:
        rin = inst.cutoff + args.prune_inner

        def step_p(k):
            if k % REBUILD_EVERY == 0:
                nb.nb_pairlist(ctx, traj[k])
            if k % args.prune_every == 0:
                nb.nb_prune(ctx, traj[k], rin)
            nb.nb_forces(ctx, traj[k], q, t, f, e)

        for k in range(args.warmup):
            step_p(k)
        torch.cuda.synchronize()
        tp = time.perf_counter()
        for k in range(args.warmup, nsteps):
            step_p(k)
        torch.cuda.synchronize()
        elapsed_p = time.perf_counter() - tp
        nb.nb_pairlist(ctx, traj[nsteps - 1])
        nb.nb_prune(ctx, traj[nsteps - 1], rin)
        kept = nb.nb_get_stats(ctx)["nentries"]
        reps = 100
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for k in range(reps):
            nb.nb_prune(ctx, traj[nsteps - 1], rin)
        ev1.record()
        torch.cuda.synchronize()
        us_prune = 1e3 * ev0.elapsed_time(ev1) / reps
        ev0.record()
        for k in range(reps):
            nb.nb_forces(ctx, traj[nsteps - 1], q, t, f, e)
        ev1.record()
        torch.cuda.synchronize()
        prune = {"r_inner": rin, "prune_every": args.prune_every,
                 "pairs_per_s": useful * args.steps / elapsed_p,
                 "us_per_call_amortised": 1e6 * elapsed_p / args.steps,
                 "us_per_prune": us_prune,
                 "us_per_force_call_pruned": 1e3 * ev0.elapsed_time(ev1) / reps,
                 "list_entries_pruned": kept, "list_entries_full": stats["nentries"]}

    # force call alone (no rebuilds), event-timed on the current stream
    nb.nb_pairlist(ctx, traj[0])
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = max(100, args.steps // 2)
    ev0.record()
    for k in range(reps):
        nb.nb_forces(ctx, traj[0], q, t, f, e)
    ev1.record()
    torch.cuda.synchronize()
    us_force = 1e3 * ev0.elapsed_time(ev1) / reps

    # the same call with the virial output
    vir = torch.zeros(9, dtype=torch.float64, device=dev)
    ev0.record()
    for k in range(reps):
        nb.nb_forces_virial(ctx, traj[0], q, t, f, e, vir)
    ev1.record()
    torch.cuda.synchronize()
    us_force_virial = 1e3 * ev0.elapsed_time(ev1) / reps

    # the call with the Ewald exclusion correction and self term (a context with that flag)
    pc = nb.Params.from_instance(inst, cluster=cluster,
                                 flags=(nb.NB_ENERGY_FP64 if args.energy_fp64 else 0) | nb.NB_EWALD_CORR,
                                 **flav) if args.elec == "ewald" else None
    us_force_corr = None
    if pc is not None:
        ctx_c = nb.nb_setup(pc)
        e4 = torch.zeros(4, dtype=torch.float64, device=dev)
        nb.nb_pairlist(ctx_c, traj[0])
        nb.nb_forces(ctx_c, traj[0], q, t, f, e4)
        ev0.record()
        for k in range(reps):
            nb.nb_forces(ctx_c, traj[0], q, t, f, e4)
        ev1.record()
        torch.cuda.synchronize()
        us_force_corr = 1e3 * ev0.elapsed_time(ev1) / reps
        nb.nb_destroy(ctx_c)

    # the tabulated Ewald flavour (FP32 force table, FP64 pair energies) and, for comparison, the
    # analytic flavour with FP64 pair energies, on the same walk start
    us_tab = us_e64 = kernel_us_tab = kernel_us_e64 = None
    if args.elec == "ewald":
        for name, kw in (("tab", dict(elec=nb.NB_ELEC_EWALD_TAB, flags=0)),
                         ("e64", dict(elec=nb.NB_ELEC_EWALD, flags=nb.NB_ENERGY_FP64))):
            pt = nb.Params.from_instance(inst, cluster=cluster, flags=kw["flags"], elec=kw["elec"],
                                         vdw=flav["vdw"], rswitch=flav["rswitch"])
            ctx_t = nb.nb_setup(pt)
            nb.nb_pairlist(ctx_t, traj[0])
            nb.nb_forces(ctx_t, traj[0], q, t, f, e)
            ev0.record()
            for k in range(reps):
                nb.nb_forces(ctx_t, traj[0], q, t, f, e)
            ev1.record()
            torch.cuda.synchronize()
            us_call = 1e3 * ev0.elapsed_time(ev1) / reps
            nb.nb_set_timing(ctx_t, True)
            for k in range(reps):
                nb.nb_forces(ctx_t, traj[0], q, t, f, e)
            kms_t, kl_t = nb.nb_get_timing(ctx_t)
            nb.nb_destroy(ctx_t)
            if name == "tab":
                us_tab, kernel_us_tab = us_call, 1e3 * kms_t / kl_t
            else:
                us_e64, kernel_us_e64 = us_call, 1e3 * kms_t / kl_t

    # list build alone: each build waits for the previous one's status, so the interval between
    # the returns of successive calls spans one build; median and IQR of those intervals (the
    # host's wait varies from build to build)
    torch.cuda.synchronize()
    nbuild = 60
    stamps = []
    for k in range(nbuild + 1):
        nb.nb_pairlist(ctx, traj[k % len(traj)])
        stamps.append(time.perf_counter())
    torch.cuda.synchronize()
    b25, us_build, b75 = (float(v) for v in np.percentile(1e6 * np.diff(stamps), [25, 50, 75]))

    achieved = flops_per_pair * useful / (kernel_us * 1e-6) / 1e12
    traffic = counted = None
    default_flavour = args.elec == "ewald" and args.vdw == "shift"
    if cluster == 8 and not args.energy_fp64 and default_flavour and _counters_current():
        traffic = K_FORCE_COUNTERS["read_bytes"] + K_FORCE_COUNTERS["write_bytes"]
        counted = K_FORCE_COUNTERS["counted_fp32_flop"] / (kernel_us * 1e-6) / 1e12

    out = {
        "metric": "pair-interactions/s (96k-atom water box, force+energy call, list rebuilt every 10 calls)",
        "value": value,
        "unit": "pair-interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "water-96k: 32,000 rigid 3-site waters, L=9.87 nm, rc=1.0 nm, "
                               "rb=0.1 nm, beta=3.1234 nm^-1, random walk 0.002 nm/call, "
                               "rebuild every 10 calls",
                   "natoms": n, "cluster": cluster, "useful_pairs": useful,
                   "energy": "fp64 pair energies" if args.energy_fp64 else "fp32 pair energies, fp64 sums",
                   "list_build": "asynchronous (overflow status read at the next build)",
                   "interactions": ("Ewald real space" if args.elec == "ewald" else "reaction field (eps_rf inf)")
                   + (", LJ potential shift" if args.vdw == "shift" else f", LJ force switch from {args.rswitch} nm"),
                   "evaluated_pairs": stats["evaluated_pairs"], "list_entries": stats["nentries"]},
        "us_per_force_call": us_force,
        "us_per_force_call_with_virial": us_force_virial,
        "us_per_force_call_with_ewald_corrections": us_force_corr,
        "energy_modes": {"fp32_pair_energies": {"us_per_force_call": us_force, "kernel_us": kernel_us,
                                                "energy_gate": "1e-6 at 96k atoms"},
                         "fp64_pair_energies": {"us_per_force_call": us_e64, "kernel_us": kernel_us_e64,
                                                "energy_gate": "1e-6 at every size"},
                         "tabulated_ewald_fp64_energies": {"us_per_force_call": us_tab,
                                                           "kernel_us": kernel_us_tab,
                                                           "energy_gate": "1e-6 at every size"}},
        "us_per_list_build": us_build,
        "us_per_list_build_iqr": [b25, b75],
        "us_per_call_amortised": 1e3 * ms_per_step,
        "rebuild_periods": period_stats,
        "rolling_prune": prune,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_VECTOR_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_VECTOR_TFLOPS,
                     "traffic": traffic, "kernel": "k_force", "kernel_us": kernel_us,
                     "kernel_launches_timed": klaunch,
                     "kernel_timing": f"HIP event pairs stamped by every {TIMING_EVERY}th force kernel "
                                      "dispatch of the timed walk",
                     "flops_per_pair": flops_per_pair, "counted_fp32_tflops": counted},
    }
    nb.nb_destroy(ctx)
    if not args.no_adjoint:
        out["adjoint"] = bench_adjoint(torch, nb, synth)
    if not args.no_pme:
        out["pme"] = bench_pme(torch, nb, synth)
        out["ewald_step"] = bench_ewald_step(torch, nb, synth)
    if not args.no_md:
        out["md"] = bench_md(torch, nb, synth)
    if not args.no_batch:
        out["batched"] = bench_batched(torch, nb, synth, not args.no_tune)
    if not args.no_small:
        out["small_boxes"] = bench_small_boxes(torch, nb, synth)
    if args.large:
        out["large"] = bench_large(torch, nb, synth)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
    if args.copy_probe:
        src = torch.ones(64 << 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_probe_bytes"] = {"read": src.numel() * 4, "write": dst.numel() * 4}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
