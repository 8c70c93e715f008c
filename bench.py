#!/usr/bin/env python3
"""Benchmark of the operator-splitting reaction-diffusion hot path on one GPU.

Headline: the dendrite workload -- a seeded random branching tree of tapered
cylinders voxelised into 996,564 tets, a 15-species / 20-reaction calcium
buffer model with the calcium influx in 5% of the tets, 50 ms simulated at
tau = 7.2 us (about 6,950 windows).  A step is one 2.5 ms segment of that run
(Algorithm 1 to the segment end, the last window of a segment cut there), so
the default 20 timed steps are the whole 50 ms run, started from counts
resident in HBM.  Every window does the reaction SSA and the diffusion update
of every tet.

Prints one JSON line: voxel-steps/s (the value), SSA events/s, molecules and
face moves per second; the roofline of the main window kernel (its
algorithmic bytes per launch over its average launch time from HIP events
the library records on the launch stream, during the timed region when the
tuned launch shape uses plain launches, else in a second pass); the oracle
timed on the host's cores (serially, and its all-core build) on a bounded
sample of the same run; the exact serial SSA's event rate as the context of
the paper's speedup over serial SSA.  Secondary legs follow the headline:
the simple-model box (480,000 tets, 100 ms), the literal 1,296-tet 10 ms run,
the batched ensemble and the served request stream (each against the plain
path), the density/refinement series and forcing with recording.
``--no-extra`` leaves out the series and the forcing leg; ``--sweep``,
``--forcing`` and ``--simple`` print only that leg.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s
SEGMENT_S = 2.5e-3     # simulated time of one timed step of the headline run
KERNEL_SOURCE = os.path.join(ROOT, "paper_1610_02258_amd", "csrc", "rdx_kernels.hip")
COUNTERS = {
    "dendrite_calcium15": os.path.join(ROOT, "profiles", "window_main_kernel_dendrite_counters.txt"),
    "box20x20x200_simple10": os.path.join(ROOT, "profiles", "window_main_kernel_simple10_counters.txt"),
}
TRACES = {
    "dendrite_calcium15": os.path.join(ROOT, "profiles", "window_kernels_dendrite_kernel_trace.txt"),
    "box20x20x200_simple10": os.path.join(ROOT, "profiles", "window_kernels_simple10_kernel_trace.txt"),
}
SQ_COUNTERS = {
    "dendrite_calcium15": os.path.join(ROOT, "profiles", "window_kernels_dendrite_sq_counters.txt"),
    "box20x20x200_simple10": os.path.join(ROOT, "profiles", "window_kernels_simple10_sq_counters.txt"),
}
# VALU issue peak in wave64 instructions per second: 256 CUs x 4 SIMDs at
# 2.4 GHz, one wave64 instruction per SIMD every 4 cycles (times 64 lanes and
# 2 flops per FMA this is the published 78.6 TFLOP/s of fp64 vector work)
VALU_PEAK_PER_S = 256 * 4 * 2.4e9 / 4


def window_bytes(T: int, S: int, face_moves: float) -> float:
    """Algorithmic bytes of one window: per tet the counts read and written
    (8 S), the four neighbour ids (16), the couplings G, cum0..cum2 (32) and
    N_A V (8); per nonzero (tet, species, face) move one 4-byte
    read-modify-write of the neighbour's count (8)."""
    return float(T) * (8 * S + 16 + 32 + 8) + 8.0 * face_moves


def detect_kernel_bytes(T: int, S: int, n_regions: int) -> float:
    """Bytes the detect kernel must read in one window: the counts (4 S per
    tet), N_A V (8) and the region label when the model has regions (1)."""
    return float(T) * (4 * S + 8 + (1 if n_regions > 1 else 0))


def _summary(path):
    """key: value pairs of a committed profile summary, or None if the kernel
    source changed since it was taken."""
    try:
        kv = dict(line.split(":", 1) for line in open(path) if ":" in line and not line.startswith("#"))
        kv = {k.strip(): v.strip() for k, v in kv.items()}
        sha = hashlib.sha256(open(KERNEL_SOURCE, "rb").read()).hexdigest()
        return kv if kv.get("kernel_source_sha256") == sha else None
    except OSError:
        return None


def measured_traffic(workload: str = "dendrite_calcium15"):
    """HBM bytes per launch of the main kernel from the committed rocprofv3
    counter summary (FETCH_SIZE and WRITE_SIZE, each scaled by its copy-kernel
    calibration factor), or None if the kernel source changed since."""
    kv = _summary(COUNTERS[workload])
    try:
        fetch = float(kv["FETCH_SIZE_KiB_per_dispatch"]) * float(kv["fetch_factor"])
        write = float(kv["WRITE_SIZE_KiB_per_dispatch"]) * float(kv["write_factor"])
        return (fetch + write) * 1024.0
    except (TypeError, KeyError, ValueError):
        return None


def measured_valu(workload: str = "dendrite_calcium15"):
    """VALU wave instructions per launch of the main kernel from the
    committed rocprofv3 SQ counter summary (SQ_INSTS_VALU), or None if the
    kernel source changed since."""
    kv = _summary(SQ_COUNTERS[workload])
    try:
        return float(kv["window_main_kernel_SQ_INSTS_VALU_per_dispatch"])
    except (TypeError, KeyError, ValueError):
        return None


def rocprof_durations(workload: str):
    """Average main / detect kernel durations (us) from the committed
    rocprofv3 kernel-trace summary, or None if the source changed since."""
    kv = _summary(TRACES[workload])
    try:
        return {"main_us": float(kv["window_main_kernel_avg_us"]),
                "detect_us": float(kv["window_detect_kernel_avg_us"])}
    except (TypeError, KeyError, ValueError):
        return None


def host_info() -> dict:
    model = platform.processor()
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        affinity = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        affinity = os.cpu_count()
    return {"nproc": affinity, "cpu_count": os.cpu_count(), "cpu_model": model}


def cpu_baseline(workload, seconds: float = 12.0, par_seconds: float = 8.0) -> dict:
    """The oracle on the same mesh/model/seed/counts: serially for as many
    whole windows as fit in about `seconds` (the baseline proper), then its
    all-core build (the same code, the tet loop on every host core the
    process may use, bit-identical results) for about `par_seconds`."""
    from oracle import oracle as O

    inst = O.Instance(workload.mesh.as_dict(), workload.model.as_dict(), workload.seed)
    inst.reset(workload.counts)
    t0 = time.perf_counter()
    n = 0
    while time.perf_counter() - t0 < seconds:
        inst.step(1)
        n += 1
    dt = time.perf_counter() - t0
    host = host_info()
    threads = max(1, min(int(host["nproc"] or 1), 64))
    par = O.Instance(workload.mesh.as_dict(), workload.model.as_dict(), workload.seed, parallel=True)
    par.reset(workload.counts)
    t1 = time.perf_counter()
    m = 0
    while time.perf_counter() - t1 < par_seconds:
        par.step_parallel(1, threads)
        m += 1
    dtp = time.perf_counter() - t1
    return {"value": inst.tallies.voxel_steps / dt, "unit": "voxel-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"first {n} windows of the same run ({n * inst.T} voxel-steps, "
                      f"{inst.tallies.ssa_events} SSA events) in {dt:.1f} s on one host core",
            "ssa_events_per_s": inst.tallies.ssa_events / dt,
            "all_cores": {"value": par.tallies.voxel_steps / dtp, "unit": "voxel-steps/s", "cores": threads,
                          "kind": "oracle, all-core build (bit-identical)",
                          "sample": f"first {m} windows in {dtp:.1f} s on {threads} threads"},
            "host": host}


def ssa_context(workload, span_s: float, gpu_s_full: float, full_span_s: float) -> dict:
    """The exact serial SSA (Gillespie's direct method over every reaction and
    face jump, sum-tree selection) from the same counts for `span_s` of
    simulated time on one host core: events/s, and the time a serial exact
    SSA would need for the whole benchmarked span (events extrapolated
    linearly in simulated time), against the GPU's time for it -- the analogue
    of the paper's speedup over serial SSA (section 3)."""
    from oracle import oracle as O

    inst = O.Instance(workload.mesh.as_dict(), workload.model.as_dict(), workload.seed)
    t0 = time.perf_counter()
    _, ev = O.rdme_direct(inst, workload.counts, [span_s], seed=workload.seed, method="tree",
                          return_events=True)
    dt = time.perf_counter() - t0
    rate = ev / dt
    t_ssa_full = ev * (full_span_s / span_s) / rate
    return {"kind": "exact serial SSA (direct method, sum-tree selection), one host core",
            "simulated_s": span_s, "events": ev, "seconds": dt, "events_per_s": rate,
            "extrapolated_full_run_s": t_ssa_full, "gpu_full_run_s": gpu_s_full,
            "speedup_vs_serial_ssa": t_ssa_full / gpu_s_full}


def roofline(T: int, S: int, n_regions: int, windows: int, face_moves: int, kt: dict, source: str,
             workload: str) -> dict:
    """Roofline of the main window kernel: the window's algorithmic bytes
    per launch over its average launch time (HIP events on the launch
    stream), and the whole window (detect + main) beside it."""
    n = max(kt["windows"], 1)
    main_s, det_s = kt["main_ms"] * 1e-3 / n, kt["detect_ms"] * 1e-3 / n
    b = window_bytes(T, S, face_moves / max(windows, 1))
    achieved = b / main_s / 1e9
    out = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(workload),
           "kernel": "window_main_kernel", "bytes_per_launch": b,
           "bytes_per_voxel_step": b / T, "face_moves_per_window": face_moves / max(windows, 1),
           "avg_launch_us": main_s * 1e6, "duration_source": source,
           "window": {"detect_us": det_s * 1e6, "main_us": main_s * 1e6,
                      "achieved_GBs": b / (main_s + det_s) / 1e9,
                      "frac": b / (main_s + det_s) / 1e9 / HBM_PEAK_GBS},
           "detect_kernel": {"avg_launch_us": det_s * 1e6,
                             "bytes_per_launch": detect_kernel_bytes(T, S, n_regions),
                             "achieved_GBs": detect_kernel_bytes(T, S, n_regions) / det_s / 1e9}}
    rp = rocprof_durations(workload)
    if rp:
        out["rocprof"] = {"main_us": rp["main_us"], "detect_us": rp["detect_us"],
                          "frac_main": b / (rp["main_us"] * 1e-6) / 1e9 / HBM_PEAK_GBS}
    v = measured_valu(workload)
    if v:  # the issue side: counted VALU instructions over the same duration
        out["valu_issue"] = {"instructions_per_launch": v, "achieved_per_s": v / main_s,
                             "peak_per_s": VALU_PEAK_PER_S, "frac": v / main_s / VALU_PEAK_PER_S,
                             "unit": "wave64 VALU instructions/s", "source": "rocprofv3 SQ_INSTS_VALU"}
    return out


def _apply_shape(sim, shape: str):
    """Online tuning of the launch shape, or the fixed shape
    'div,graph,group[,claim]' (claim: diffusion tiles claimed at run time)."""
    if shape:
        v = [int(x) for x in shape.split(",")]
        d, g, e = v[:3]
        c = v[3] if len(v) > 3 else 0
        sim.set_exec_options(autotune=False, fast_grid_div=d, graph_windows=g, event_group=e, tile_claim=c)
    else:
        sim.set_exec_options(autotune=True)


def dendrite_headline(steps: int, warmup: int, shape: str = "") -> tuple:
    """The headline: `steps` consecutive segments of SEGMENT_S of one run of
    the dendrite workload, after `warmup` segments of a first run (the online
    tuner settles on a launch shape there) and a reset to t = 0."""
    import numpy as np
    import torch
    from paper_1610_02258_amd import inputs, rdx

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    w = inputs.config_dendrite()
    t0 = time.perf_counter()
    sim = rdx.Sim(w.mesh.as_dict(), w.model.as_dict(), w.seed)
    setup_s = time.perf_counter() - t0
    T, S = sim.T, sim.S
    c0 = torch.from_numpy(np.ascontiguousarray(w.counts)).to(dev)
    _apply_shape(sim, shape)  # tuned online in the warm-up unless fixed
    sim.set_counts(c0, stream=stream)
    k = 0
    while k < warmup or (sim.exec_options()["autotune"] and k < warmup + 8):
        sim.run((k + 1) * SEGMENT_S, stream=stream)
        torch.cuda.synchronize()
        k += 1
    shape = sim.exec_options()
    in_region = shape["graph_windows"] == 1  # events then cost no change of launch path
    sim.set_counts(c0, stream=stream)  # t = 0, window 0, tallies cleared
    sim.kernel_times(reset=True)
    sim.set_kernel_timing(in_region)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for k in range(steps):
        sim.run((k + 1) * SEGMENT_S, stream=stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    st = sim.stats(stream)
    if in_region:
        kt = sim.kernel_times(reset=True)
        source = "HIP events on the launch stream around each kernel, inside the timed region"
    else:
        sim.set_kernel_timing(True)
        sim.set_counts(c0, stream=stream)
        for k in range(steps):
            sim.run((k + 1) * SEGMENT_S, stream=stream)
        torch.cuda.synchronize()
        kt = sim.kernel_times(reset=True)
        source = "HIP events on the launch stream around each kernel, second pass of the same steps"
    sim.set_kernel_timing(False)
    n_regions = sim.n_regions
    out = {
        "value": T * st.windows / elapsed,
        "ms_per_step": elapsed * 1e3 / steps,
        "config": {"workload": w.name, "n_tets": T, "species": S, "reactions": sim.R, "regions": n_regions,
                   "molecules": int(w.counts.sum()), "t_end_s": steps * SEGMENT_S, "segment_s": SEGMENT_S,
                   "windows": st.windows, "tau_s": sim.tau, "launch_shape": shape,
                   "parallelism": "single GPU"},
        "ssa_events_per_s": st.ssa_events / elapsed,
        "moves_per_s": st.moves / elapsed,
        "face_moves_per_s": st.face_moves / elapsed,
        "setup_s": setup_s,
        "roofline": roofline(T, S, n_regions, st.windows, st.face_moves, kt, source, w.name),
    }
    sim.close()
    return out, w, elapsed


def simple_leg(steps: int, warmup: int, shape: str = "") -> dict:
    """The simple-model box: 10 x 10 x 100 um of 0.5 um cubes (480,000
    jittered tets), 10 species / 12 reactions, 1e6 molecules, 100 ms = 220
    windows per step, each step reset from device counts; timed on the
    production path (captured window graphs when tuned so), kernel durations
    from a second pass with per-kernel HIP events."""
    import numpy as np
    import torch
    from paper_1610_02258_amd import inputs, rdx

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    w = inputs.config_simple()
    sim = rdx.Sim(w.mesh.as_dict(), w.model.as_dict(), w.seed)
    c0 = torch.from_numpy(np.ascontiguousarray(w.counts)).to(dev)

    def one():
        sim.set_counts(c0, stream=stream)
        sim.run(w.t_end, stream=stream)

    _apply_shape(sim, shape)  # tuned online in the warm-up unless fixed
    k = 0
    while k < warmup or (sim.exec_options()["autotune"] and k < warmup + 8):
        one()
        torch.cuda.synchronize()
        k += 1
    t0 = time.perf_counter()
    for _ in range(steps):
        one()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    st = sim.stats(stream)
    sim.kernel_times(reset=True)
    sim.set_kernel_timing(True)
    for _ in range(steps):
        one()
    torch.cuda.synchronize()
    kt = sim.kernel_times(reset=True)
    sim.set_kernel_timing(False)
    out = {"workload": w.name, "n_tets": sim.T, "t_end_s": w.t_end, "windows_per_step": st.windows,
           "steps": steps, "voxel_steps_per_s": sim.T * st.windows * steps / el,
           "ssa_events_per_s": st.ssa_events * steps / el, "ms_per_step": el * 1e3 / steps,
           "window_us": el * 1e6 / (st.windows * steps), "launch_shape": sim.exec_options(),
           "roofline": roofline(sim.T, sim.S, sim.n_regions, st.windows, st.face_moves, kt,
                                "HIP events on the launch stream, second pass of the same steps", w.name)}
    sim.close()
    return out, w, el / steps


def literal_small_leg(reps: int = 200) -> dict:
    """The literal small-box run: 1,296 tets, A + B <-> C, 2,000 A and 2,000 B,
    10 ms = one window cut at t_end; per run on the GPU (reset from device
    counts + run, enqueued back to back), the oracle, and the exact serial
    SSA (sum-tree direct method) of the same 10 ms."""
    import numpy as np
    import torch
    from oracle import oracle as O
    from paper_1610_02258_amd import inputs, rdx

    stream = torch.cuda.current_stream()
    w = inputs.config_small()
    sim = rdx.Sim(w.mesh.as_dict(), w.model.as_dict(), w.seed)
    c0 = torch.from_numpy(np.ascontiguousarray(w.counts)).to("cuda:0")
    for _ in range(5):
        sim.set_counts(c0, stream=stream)
        sim.run(w.t_end, stream=stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        sim.set_counts(c0, stream=stream)
        sim.run(w.t_end, stream=stream)
    torch.cuda.synchronize()
    gpu_s = (time.perf_counter() - t0) / reps
    st = sim.stats(stream)
    T = sim.T
    sim.close()
    ref = O.Instance(w.mesh.as_dict(), w.model.as_dict(), w.seed)
    t0 = time.perf_counter()
    for _ in range(20):
        ref.reset(w.counts)
        ref.run(w.t_end)
    ora_s = (time.perf_counter() - t0) / 20
    t0 = time.perf_counter()
    ev = 0
    for r in range(20):
        _, e = O.rdme_direct(ref, w.counts, [w.t_end], seed=r, method="tree", return_events=True)
        ev += e
    ssa_s = (time.perf_counter() - t0) / 20
    return {"workload": w.name, "n_tets": T, "t_end_s": w.t_end,
            "windows": st.windows, "gpu_s_per_run": gpu_s, "oracle_s_per_run": ora_s,
            "exact_ssa_s_per_run": ssa_s, "exact_ssa_events_per_run": ev / 20,
            "speedup_vs_oracle": ora_s / gpu_s, "speedup_vs_serial_ssa": ssa_s / gpu_s}


def batched_leg(steps: int = 2) -> dict:
    """1024 realisations of uneven size (6 x 6 x n slabs of 1 um cubes,
    T ~ logU(1e3, 5e4)), A + B <-> C plus X -> Y -> Z with per-run rates
    x U(0.5, 1.5), 1 s each: all runs in one batch (shared window launches,
    launch shape tuned online, captured graphs) against the plain path (the
    same runs one simulation at a time).  Both reset every run's counts from
    device memory and run it to t_end inside the timed region; set-up is
    outside it."""
    import numpy as np
    import torch
    from paper_1610_02258_amd import inputs, rdx

    runs = inputs.ensemble_runs()
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    c0 = [torch.from_numpy(np.ascontiguousarray(w.counts)).to(dev) for w in runs]
    b = rdx.Batch([(w.mesh.as_dict(), w.model.as_dict(), w.seed) for w in runs])
    t_end = [w.t_end for w in runs]

    def batch_step():
        b.set_counts_all(c0, stream=stream)  # every run reset in one launch
        b.run(t_end, stream=stream)

    # warm-up, which also runs the online tuning of the launch shape (its
    # candidate shapes are timed on real windows; a step may not hold them all)
    for _ in range(20):
        batch_step()
        torch.cuda.synchronize()
        if not b.exec_options()["autotune"]:
            break
    t0 = time.perf_counter()
    for _ in range(steps):
        batch_step()
    torch.cuda.synchronize()
    tb = (time.perf_counter() - t0) / steps
    vs = sum(b.stats(i).voxel_steps for i in range(len(runs)))
    ev = sum(b.stats(i).ssa_events for i in range(len(runs)))
    shape = b.exec_options()
    b.close()

    sims = [rdx.Sim(w.mesh.as_dict(), w.model.as_dict(), w.seed) for w in runs]

    def plain_step():
        for s, c, w in zip(sims, c0, runs):
            s.set_counts(c, stream=stream)
            s.run(w.t_end, stream=stream)

    plain_step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plain_step()
    torch.cuda.synchronize()
    tp = (time.perf_counter() - t0) / steps
    vs_p = sum(s.stats().voxel_steps for s in sims)
    for s in sims:
        s.close()
    return {"workload": "ensemble1024_box6x6xn_abc_chain", "runs": len(runs),
            "total_tets": int(sum(w.mesh.n_tets for w in runs)),
            "voxel_steps_per_step": vs, "ssa_events_per_step": ev,
            "batched_voxel_steps_per_s": vs / tb, "batched_ssa_events_per_s": ev / tb,
            "plain_voxel_steps_per_s": vs_p / tp, "speedup_vs_plain": tp / tb,
            "batched_ms_per_step": tb * 1e3, "plain_ms_per_step": tp * 1e3,
            "launch_shape": shape, "steps": steps}


def serve_leg(n_requests: int = 400, rate: float = 200.0, submit_threads: int = 8) -> dict:
    """Poisson arrivals (rate per s) of box-mesh requests, T ~ logU(1296, 2e5)
    with the 10-species model, 100 ms each: the continuous-batching server
    against the plain path serving the same stream first-in first-out, one
    simulation at a time (create, set counts, run, read counts, destroy).
    Latency = completion - scheduled arrival; each request's host set-up is
    part of it in both."""
    import concurrent.futures as cf
    import numpy as np
    from paper_1610_02258_amd import inputs, rdx

    reqs = inputs.request_stream(n_requests=n_requests, rate_per_s=rate)
    model = reqs[0][1].model.as_dict()
    mesh_d = {}
    for _, w in reqs:
        mesh_d.setdefault(id(w.mesh), w.mesh.as_dict())

    def pct(x, q):
        return float(np.percentile(np.asarray(x), q, method="inverted_cdf"))

    # continuous batching
    srv = rdx.Server(model, hbm_budget_bytes=16 << 30, tick_windows=8)
    t0 = time.perf_counter()
    srv_t0 = t0

    def submit(j):
        arrival, w = reqs[j]
        delay = t0 + arrival - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        return srv.submit(mesh_d[id(w.mesh)], model, w.seed, w.counts, w.t_end)

    with cf.ThreadPoolExecutor(submit_threads) as pool:
        tickets = list(pool.map(submit, range(len(reqs))))
    lat_s, vs = [], 0
    for j, tk in enumerate(tickets):
        _, info = srv.wait(tk)
        lat_s.append(srv_t0 + info["t_done"] - (t0 + reqs[j][0]))
        vs += info["stats"].voxel_steps
    makespan_s = time.perf_counter() - t0
    sst = srv.stats()
    srv.close()

    # the same requests all at once: the server's throughput when it is never
    # short of work
    srv = rdx.Server(model, hbm_budget_bytes=16 << 30, tick_windows=8)
    t0 = time.perf_counter()

    def submit_now(j):
        w = reqs[j][1]
        return srv.submit(mesh_d[id(w.mesh)], model, w.seed, w.counts, w.t_end)

    with cf.ThreadPoolExecutor(submit_threads) as pool:
        tickets = list(pool.map(submit_now, range(len(reqs))))
    for tk in tickets:
        srv.wait(tk)
    burst_s = time.perf_counter() - t0
    bst = srv.stats()
    srv.close()

    # plain FIFO
    lat_p = []
    t0 = time.perf_counter()
    for arrival, w in reqs:
        delay = t0 + arrival - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        s = rdx.Sim(mesh_d[id(w.mesh)], model, w.seed)
        s.set_counts(w.counts)
        s.run(w.t_end)
        s.get_counts()
        s.close()
        lat_p.append(time.perf_counter() - (t0 + arrival))
    makespan_p = time.perf_counter() - t0
    return {"workload": f"poisson{int(rate)}_box5x5xn_simple10", "requests": len(reqs),
            "rate_per_s": rate, "mean_tets": float(np.mean([w.mesh.n_tets for _, w in reqs])),
            "served_p50_s": pct(lat_s, 50), "served_p99_s": pct(lat_s, 99),
            "plain_p50_s": pct(lat_p, 50), "plain_p99_s": pct(lat_p, 99),
            "served_voxel_steps_per_s": vs / makespan_s, "plain_voxel_steps_per_s": vs / makespan_p,
            "served_makespan_s": makespan_s, "plain_makespan_s": makespan_p,
            "server_ticks": sst["ticks"], "server_device_busy_s": sst["busy_s"],
            "server_device_busy_frac": sst["busy_s"] / makespan_s, "server_worker_s": sst["worker_s"],
            "burst_voxel_steps_per_s": vs / burst_s, "burst_makespan_s": burst_s,
            "burst_device_busy_frac": bst["busy_s"] / burst_s, "burst_ticks": bst["ticks"],
            "burst_worker_s": bst["worker_s"],
            "submit_threads": submit_threads}


SWEEP = [(0.1, 0.5), (1.0, 0.5), (10.0, 0.5), (1.0, 1.0), (1.0, 0.25)]


def sweep_leg(steps: int, windows: int = 200) -> list:
    """Density (0.1x, 1x, 10x molecules) and refinement (1, 0.5, 0.25 um
    cubes) series of the simple-model box, each run for a fixed number of
    windows: voxel-steps/s and SSA events/s on the graph path, then the two
    kernels' average durations from a pass with HIP events."""
    import numpy as np
    import torch
    from paper_1610_02258_amd import inputs, rdx

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    rows = []
    for density, h in SWEEP:
        w = inputs.config_simple_variant(density, h)
        print(f"bench: sweep {w.name}", file=sys.stderr, flush=True)
        sim = rdx.Sim(w.mesh.as_dict(), w.model.as_dict(), w.seed)
        sim.set_exec_options(autotune=True)
        t_end = windows * sim.tau
        c0 = torch.from_numpy(np.ascontiguousarray(w.counts)).to(dev)

        def run():
            sim.set_counts(c0, stream=stream)
            sim.run(t_end, stream=stream)

        # warm up until the online tuner has settled (it scores every
        # candidate shape three times, about 440 windows), so that the timed runs
        # and the per-kernel pass run the shape it picks
        for k in range(8):
            run()
            torch.cuda.synchronize()
            if k >= 1 and not sim.exec_options()["autotune"]:
                break
        shape = sim.exec_options()
        t0 = time.perf_counter()
        for _ in range(steps):
            run()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        st = sim.stats(stream)
        sim.kernel_times(reset=True)
        sim.set_kernel_timing(True)
        for _ in range(steps):
            run()
        torch.cuda.synchronize()
        kt = sim.kernel_times(reset=True)
        sim.set_kernel_timing(False)
        n = max(kt["windows"], 1)
        main_s, det_s = kt["main_ms"] * 1e-3 / n, kt["detect_ms"] * 1e-3 / n
        b_main = window_bytes(sim.T, sim.S, st.face_moves / st.windows)
        b_det = detect_kernel_bytes(sim.T, sim.S, w.model.kcst.shape[0])
        rows.append({"workload": w.name, "n_tets": sim.T, "molecules": int(w.counts.sum()),
                     "tau_s": sim.tau, "windows": st.windows,
                     "voxel_steps_per_s": sim.T * st.windows * steps / el,
                     "ssa_events_per_s": st.ssa_events * steps / el,
                     "events_per_window": st.ssa_events / st.windows,
                     "moves_per_s": st.moves * steps / el,
                     "window_us": el * 1e6 / (st.windows * steps),
                     "main_us": main_s * 1e6, "detect_us": det_s * 1e6,
                     "main_frac_of_hbm": b_main / main_s / 1e9 / HBM_PEAK_GBS,
                     "detect_frac_of_hbm": b_det / det_s / 1e9 / HBM_PEAK_GBS,
                     "launch_shape": shape})
        sim.close()
        del c0
    return rows


def record_kernel_bytes(T: int, S: int, n_regions: int) -> float:
    """Bytes the per-region count reduction must read: the counts (4 S per
    tet) and, with regions, the region labels (1 per tet)."""
    return float(T) * (4 * S + (1 if n_regions > 1 else 0))


def forcing_leg(sim_ms: float = 2.0, record_ms: float = 0.02, force_ms: float = 1.0) -> dict:
    """Time-varying forcing and recording as section 3.2 uses them, on the
    dendrite workload: the calcium influx redrawn every `force_ms` (x U(0.5,
    3)), per-region counts recorded every `record_ms` into a device ring
    (run to the record time, then the reduction writes the ring slot; no
    host sync), against the plain run of the same span.  Then the simple
    model recorded after every window against its graph path, and the
    reduction kernel alone, timed back to back with events on its stream."""
    import numpy as np
    import torch
    from paper_1610_02258_amd import inputs, rdx

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    out = {}
    w = inputs.config_dendrite()
    md = w.model.as_dict()
    sim = rdx.Sim(w.mesh.as_dict(), md, w.seed)
    c0 = torch.from_numpy(np.ascontiguousarray(w.counts)).to(dev)
    t_end = sim_ms * 1e-3
    n_rec = int(round(sim_ms / record_ms))
    per_force = int(round(force_ms / record_ms))
    ring = torch.zeros((n_rec, sim.n_regions, sim.S), dtype=torch.int64, device=dev)
    influx = np.flatnonzero(np.asarray(md["lhs"]).sum(axis=1) == 0)
    rng = np.random.default_rng(12)
    tables = []
    for _ in range((n_rec + per_force - 1) // per_force):
        k = np.array(md["kcst"], np.float64)
        k[:, influx] *= rng.uniform(0.5, 3.0)
        tables.append(k)

    def plain():
        sim.set_rate_constants(md["kcst"], stream=stream)
        sim.set_counts(c0, stream=stream)
        sim.run(t_end, stream=stream)

    def forced():
        sim.set_counts(c0, stream=stream)
        for r in range(n_rec):
            if r % per_force == 0:
                sim.set_rate_constants(tables[r // per_force], stream=stream)
            sim.run((r + 1) * record_ms * 1e-3, stream=stream)
            sim.region_counts(out=ring[r], stream=stream)

    res = {}
    for name, fn in (("plain", plain), ("forced_recorded", forced)):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        st = sim.stats(stream)
        res[name] = {"s": el, "windows": st.windows, "voxel_steps_per_s": st.voxel_steps / el,
                     "ssa_events_per_s": st.ssa_events / el}
    out["dendrite"] = {"workload": w.name, "n_tets": sim.T, "species": sim.S, "regions": sim.n_regions,
                       "tau_s": sim.tau, "simulated_s": t_end, "records": n_rec,
                       "rate_updates": len(tables), **{k: v for k, v in res.items()},
                       "overhead": res["forced_recorded"]["s"] / res["plain"]["s"] - 1.0}
    # the reduction alone at this size
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 200
    ev0.record(stream)
    for r in range(reps):
        sim.region_counts(out=ring[r % n_rec], stream=stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    us = ev0.elapsed_time(ev1) * 1e3 / reps
    b = record_kernel_bytes(sim.T, sim.S, sim.n_regions)
    out["record_kernel_dendrite"] = {"avg_us": us, "bytes": b, "GBs": b / us / 1e3,
                                     "frac_of_hbm": b / us / 1e3 / HBM_PEAK_GBS}
    sim.close()
    del c0, ring

    w = inputs.config_simple()
    sim = rdx.Sim(w.mesh.as_dict(), w.model.as_dict(), w.seed)
    c0 = torch.from_numpy(np.ascontiguousarray(w.counts)).to(dev)
    n_win = 220
    ring = torch.zeros((n_win, sim.n_regions, sim.S), dtype=torch.int64, device=dev)

    def every_window():
        sim.set_counts(c0, stream=stream)
        for r in range(n_win):
            sim.step(1, stream=stream)
            sim.region_counts(out=ring[r], stream=stream)

    def graph_path():
        sim.set_counts(c0, stream=stream)
        sim.step(n_win, stream=stream)

    def every_window_native():  # the same records, looped inside the library
        sim.set_counts(c0, stream=stream)
        sim.step_recorded(n_win, 1, ring, stream=stream)

    res = {}
    for name, fn in (("graph_path", graph_path), ("recorded_every_window", every_window),
                     ("recorded_every_window_native", every_window_native)):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) / 3
        res[name] = {"window_us": el * 1e6 / n_win, "voxel_steps_per_s": sim.T * n_win / el}
    ev0.record(stream)
    for r in range(reps):
        sim.region_counts(out=ring[r % n_win], stream=stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    us = ev0.elapsed_time(ev1) * 1e3 / reps
    b = record_kernel_bytes(sim.T, sim.S, sim.n_regions)
    out["simple"] = {"workload": w.name, "windows": n_win, **res}
    out["record_kernel_simple"] = {"avg_us": us, "bytes": b, "GBs": b / us / 1e3,
                                   "frac_of_hbm": b / us / 1e3 / HBM_PEAK_GBS}
    sim.close()
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="2.5 ms segments of the headline run (20 = 50 ms)")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-simple", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=400)
    ap.add_argument("--sweep", action="store_true",
                    help="instead of the headline line, print the density and refinement series")
    ap.add_argument("--forcing", action="store_true",
                    help="instead of the headline line, print the forcing and recording measurements")
    ap.add_argument("--simple", action="store_true",
                    help="instead of the headline line, print the simple-model leg (steps = its steps)")
    ap.add_argument("--shape", default="",
                    help="fixed launch shape 'grid_div,graph_windows,event_group[,tile_claim]' for the headline and the "
                         "simple leg instead of online tuning (for reproducible profiles)")
    ap.add_argument("--no-extra", action="store_true",
                    help="leave the density/refinement series and the forcing leg out of the line")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the workload is a single simulation on one "
              "device (multi-GPU sharding is a design note, not part of this build)", file=sys.stderr)
        return 2

    import torch
    from paper_1610_02258_amd import rdx

    rdx.lib()  # fails loudly if the HIP library is missing
    torch.cuda.init()
    if args.sweep:
        print(json.dumps({"sweep": sweep_leg(max(args.steps // 4, 2))}), flush=True)
        return 0
    if args.forcing:
        print(json.dumps({"forcing": forcing_leg()}), flush=True)
        return 0
    if args.simple:
        print(json.dumps({"simple": simple_leg(args.steps, args.warmup, args.shape)[0]}), flush=True)
        return 0
    print("bench: dendrite headline", file=sys.stderr, flush=True)
    head, w, gpu_s = dendrite_headline(args.steps, args.warmup, args.shape)
    out = {"metric": "voxel-steps/s & SSA events/s at 1 GPU; batched p50/p99 latency vs plain",
           "value": head["value"], "unit": "voxel-steps/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": head["ms_per_step"], "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64+i32", "data": "synthetic"}
    out.update({k: v for k, v in head.items() if k not in ("value", "ms_per_step")})
    secondary = []
    if not args.no_simple:
        secondary.append(("simple", lambda: simple_leg(10, 2, args.shape)))
    secondary.append(("literal_small", literal_small_leg))
    if not args.no_batched:
        secondary.append(("batched", batched_leg))
    if not args.no_serve:
        secondary.append(("served", lambda: serve_leg(args.serve_requests)))
    if not args.no_extra:
        secondary += [("sweep", lambda: sweep_leg(2)), ("forcing", forcing_leg)]
    simple_w = simple_step_s = None
    for key, fn in secondary:
        # measured after the headline; an exception is reported in the line
        # rather than losing the headline figures
        print(f"bench: {key} leg", file=sys.stderr, flush=True)
        try:
            r = fn()
            if key == "simple":
                r, simple_w, simple_step_s = r
            out[key] = r
        except Exception as e:  # noqa: BLE001
            out[key] = {"error": f"{type(e).__name__}: {e}"}
    if not args.no_cpu_baseline:
        print("bench: cpu baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
        ctx = {"dendrite": ssa_context(w, 2e-7, gpu_s, args.steps * SEGMENT_S)}
        if simple_w is not None:
            ctx["simple"] = ssa_context(simple_w, 2e-4, simple_step_s, simple_w.t_end)
        out["serial_ssa_context"] = ctx
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
