#!/usr/bin/env python3
"""Benchmark of the operator-splitting reaction-diffusion hot path on one GPU.

A step is one complete simulated run of the simple-model workload: a 10 x 10 x
100 um box of 0.5 um cubes (480,000 jittered tets), 10 species / 12 reactions,
1e6 molecules, 100 ms simulated = 220 windows (219 of tau, one truncated), every
window doing the reaction SSA and the diffusion update of every tet.  The
initial counts are resident in HBM before timing; each step resets the
simulation to them (device-to-device) and runs to t_end.

Prints one JSON line: voxel-steps/s (the value, timed on the production path
of captured window graphs), SSA events/s and molecules moved/s, the roofline
of the main window kernel (algorithmic bytes per launch over its average
launch time from HIP events on the launch stream, taken over a second pass of
the same steps with per-kernel events), and the oracle timed on host cores on
a bounded sample of the same workload.

The line also carries, measured after the headline figures, the density and
refinement series of the same box (``sweep``) and time-varying influx with
per-region recording on the dendrite workload (``forcing``); ``--no-extra``
leaves them out.  ``--sweep`` and ``--forcing`` print only that leg.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s
KERNEL_SOURCE = os.path.join(ROOT, "paper_1610_02258_amd", "csrc", "rdx_kernels.hip")
COUNTERS = os.path.join(ROOT, "profiles", "window_main_kernel_simple10_counters.txt")


def main_kernel_bytes(T: int, S: int, molecules_moved: float) -> float:
    """Bytes the main kernel must move in one window: the counts read and the
    next counts written (8 S per tet), the neighbour ids (16), the couplings
    G, cum0..cum2 (32), and one 4-byte read-modify-write per moved
    molecule's target count (8 each; moved molecules bound the nonzero face
    moves from above).  The listed tets' worklist traffic is left out (a few
    hundred tets of 480,000)."""
    return float(T) * (8 * S + 16 + 32) + 8.0 * molecules_moved


def detect_kernel_bytes(T: int, S: int, n_regions: int) -> float:
    """Bytes the detect kernel must read in one window: the counts (4 S per
    tet), N_A V (8) and the region label when the model has regions (1)."""
    return float(T) * (4 * S + 8 + (1 if n_regions > 1 else 0))


def measured_traffic():
    """HBM bytes per launch of the main kernel from the committed rocprofv3
    counter summary (FETCH_SIZE and WRITE_SIZE, each scaled by its copy-kernel
    calibration factor), or None if the kernel source changed since."""
    import hashlib
    try:
        kv = dict(line.split(":", 1) for line in open(COUNTERS) if ":" in line and not line.startswith("#"))
        kv = {k.strip(): v.strip() for k, v in kv.items()}
        sha = hashlib.sha256(open(KERNEL_SOURCE, "rb").read()).hexdigest()
        if kv.get("kernel_source_sha256") != sha:
            return None
        fetch = float(kv["FETCH_SIZE_KiB_per_dispatch"]) * float(kv["fetch_factor"])
        write = float(kv["WRITE_SIZE_KiB_per_dispatch"]) * float(kv["write_factor"])
        return (fetch + write) * 1024.0
    except (OSError, KeyError, ValueError):
        return None


def cpu_baseline(workload, seconds: float = 12.0) -> dict:
    """The oracle, single-threaded, on the same mesh/model/seed/counts for as
    many whole windows as fit in about `seconds`."""
    from oracle import oracle as O

    inst = O.Instance(workload.mesh.as_dict(), workload.model.as_dict(), workload.seed)
    inst.reset(workload.counts)
    t0 = time.perf_counter()
    n = 0
    while time.perf_counter() - t0 < seconds:
        inst.step(1)
        n += 1
    dt = time.perf_counter() - t0
    return {"value": inst.tallies.voxel_steps / dt, "unit": "voxel-steps/s", "cores": 1,
            "kind": "oracle",
            "sample": f"first {n} windows of the same run ({n * inst.T} voxel-steps, "
                      f"{inst.tallies.ssa_events} SSA events) in {dt:.1f} s on one host core",
            "ssa_events_per_s": inst.tallies.ssa_events / dt}


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
    for _ in range(6):
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
            "server_ticks": sst["ticks"], "server_busy_s": sst["busy_s"],
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
        t_end = windows * sim.tau
        c0 = torch.from_numpy(np.ascontiguousarray(w.counts)).to(dev)

        def run():
            sim.set_counts(c0, stream=stream)
            sim.run(t_end, stream=stream)

        run()
        torch.cuda.synchronize()
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
        b_main = main_kernel_bytes(sim.T, sim.S, st.moves / st.windows)
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
                     "detect_frac_of_hbm": b_det / det_s / 1e9 / HBM_PEAK_GBS})
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
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=400)
    ap.add_argument("--sweep", action="store_true",
                    help="instead of the headline line, print the density and refinement series")
    ap.add_argument("--forcing", action="store_true",
                    help="instead of the headline line, print the forcing and recording measurements")
    ap.add_argument("--no-extra", action="store_true",
                    help="leave the density/refinement series and the forcing leg out of the headline line")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the workload is a single simulation on one "
              "device (multi-GPU sharding is a design note, not part of this build)", file=sys.stderr)
        return 2

    import numpy as np
    import torch
    from paper_1610_02258_amd import inputs, rdx

    rdx.lib()  # fails loudly if the HIP library is missing
    torch.cuda.init()
    dev = torch.device("cuda:0")
    if args.sweep:
        print(json.dumps({"sweep": sweep_leg(max(args.steps // 4, 2))}), flush=True)
        return 0
    if args.forcing:
        print(json.dumps({"forcing": forcing_leg()}), flush=True)
        return 0
    w = inputs.config_simple()
    t0 = time.perf_counter()
    sim = rdx.Sim(w.mesh.as_dict(), w.model.as_dict(), w.seed)
    setup_s = time.perf_counter() - t0
    T, S = sim.T, sim.S
    n_regions = w.model.kcst.shape[0]
    counts0 = torch.from_numpy(np.ascontiguousarray(w.counts)).to(dev)
    stream = torch.cuda.current_stream()

    def one_step():
        sim.set_counts(counts0, stream=stream)
        sim.run(w.t_end, stream=stream)

    for _ in range(args.warmup):
        one_step()
    torch.cuda.synchronize()

    # timed region: K steps on the production path (windows replayed as
    # captured HIP graphs).
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for k in range(args.steps):
        sim.set_counts(counts0, stream=stream)
        sim.run(w.t_end, stream=stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    # kernel durations: the same steps again with the library recording HIP
    # events on the launch stream around each window's two kernels (detect
    # kernel, main kernel).  Events between kernels need plain launches, which
    # add a few microseconds of launch gaps per window, so this pass is kept
    # out of the throughput figure above.
    sim.kernel_times(reset=True)
    sim.set_kernel_timing(True)
    torch.cuda.synchronize()
    t_kt = time.perf_counter()
    for k in range(args.steps):
        sim.set_counts(counts0, stream=stream)
        sim.run(w.t_end, stream=stream)
    torch.cuda.synchronize()
    elapsed_timed = time.perf_counter() - t_kt
    kt = sim.kernel_times(reset=True)
    sim.set_kernel_timing(False)
    # tallies of the last step (each step restarts from the same counts)
    st = sim.stats(stream)
    windows_per_step = st.windows
    events_total = st.ssa_events * args.steps
    moves_total = st.moves * args.steps
    launches = kt["windows"]
    avg_main_s = kt["main_ms"] * 1e-3 / max(launches, 1)
    avg_detect_s = kt["detect_ms"] * 1e-3 / max(launches, 1)
    voxel_steps = T * windows_per_step * args.steps
    bytes_main = main_kernel_bytes(T, S, st.moves / windows_per_step)
    bytes_detect = detect_kernel_bytes(T, S, n_regions)
    achieved = bytes_main / avg_main_s / 1e9
    traffic = measured_traffic()

    out = {
        "metric": "voxel-steps/s & SSA events/s at 1 GPU; batched p50/p99 latency vs plain",
        "value": voxel_steps / elapsed,
        "unit": "voxel-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+i32",
        "data": "synthetic",
        "config": {"workload": w.name, "n_tets": T, "species": S, "reactions": sim.R,
                   "molecules": int(w.counts.sum()), "t_end_s": w.t_end,
                   "windows_per_step": windows_per_step, "tau_s": sim.tau,
                   "parallelism": "single GPU"},
        "ssa_events_per_s": events_total / elapsed,
        "moves_per_s": moves_total / elapsed,
        "setup_s": setup_s,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "window_main_kernel", "avg_launch_us": avg_main_s * 1e6,
                     "bytes_per_launch": bytes_main,
                     "detect_kernel": {"avg_launch_us": avg_detect_s * 1e6, "bytes_per_launch": bytes_detect,
                                       "achieved_GBs": bytes_detect / avg_detect_s / 1e9},
                     "window_us": elapsed * 1e6 / (windows_per_step * args.steps),
                     "window_us_with_kernel_events": elapsed_timed * 1e6 / (windows_per_step * args.steps),
                     "window_GBs": (bytes_main + bytes_detect) / (elapsed / (windows_per_step * args.steps)) / 1e9},
    }
    sim.close()
    if not args.no_batched:
        print("bench: batched ensemble leg", file=sys.stderr, flush=True)
        out["batched"] = batched_leg()
    if not args.no_serve:
        print("bench: serving leg", file=sys.stderr, flush=True)
        out["served"] = serve_leg(args.serve_requests)
    if not args.no_extra:
        # secondary measurements, outside the timed region; an exception here
        # is reported in the line rather than losing the headline figures
        for key, fn in (("sweep", lambda: sweep_leg(2)), ("forcing", forcing_leg)):
            print(f"bench: {key} leg", file=sys.stderr, flush=True)
            try:
                out[key] = fn()
            except Exception as e:  # noqa: BLE001
                out[key] = {"error": f"{type(e).__name__}: {e}"}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
