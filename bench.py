#!/usr/bin/env python3
"""Throughput of the in-situ macro-particle radiation sum on one MI355X.

Workload (default): the single-bunch FP32 case -- 65536 macro-particles, 100 time steps
(dt = 0.05 fs), 128 directions (8 x 16 within +-20 mrad) x 256 uniform frequencies up to
1e19 rad/s, CIC shape 0.1 um, betatron trajectories, FP32 particle input, FP64 phase.
One bench step = one complete spectrum: reset, 100 per-time-step pushes through the C ABI
(the in-situ evaluation, one push per simulation step) and the |S|^2 read-out on device.

Printed: ONE JSON line with updates/s, the roofline of the accumulate kernel (measured
live with HIP events recorded on the launch stream), per-push latency percentiles, the
FP64 CPU oracle's rate on a bounded sample of the same workload, and device-vs-oracle
parity on that sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FLOPS_PER_UPDATE = 20          # complex rotate 6 + form-factor scale 2 + 3 complex FMAs 12
FP32_PEAK_TFLOPS = 157.3       # MI355X FP32 vector peak (published)
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E bandwidth (published)


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="single_bunch_fp32",
                    choices=["single_bunch_fp32", "tiny_fp64", "batched_uneven", "serving", "precision_stress",
                             "fig3_analogue", "tracked"])
    ap.add_argument("--time-steps", type=int, default=0, help="batched_uneven: override the 200 time steps")
    ap.add_argument("--skip-per-bunch", action="store_true", help="batched_uneven: time only the batched launch")
    ap.add_argument("--skip-one-step", action="store_true",
                    help="tracked: time only the multi-step push (no one-step comparison)")
    ap.add_argument("--chunks", type=int, default=4000, help="serving: chunks in the arrival trace")
    ap.add_argument("--rate", type=float, default=2000.0, help="serving: Poisson arrival rate [chunks/s]")
    ap.add_argument("--distinct-steps", type=int, default=8,
                    help="batched_uneven: distinct generated steps per bunch, cycled over its 200 steps")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--latency-pushes", type=int, default=100)
    ap.add_argument("--omega-grid", choices=("uniform", "log", "blocklog"), default="uniform",
                    help="single_bunch_fp32: 'log' passes the frequencies as an explicit log-spaced list "
                         "(1e-4 * omega_max .. omega_max), evaluated with a per-term FP64 phase; 'blocklog' "
                         "spans the same range uniformly inside each block of 16 and log-like across "
                         "blocks (recurrence with a per-block step)")
    ap.add_argument("--shape", default="", help="single_bunch_fp32: override the macro-particle shape "
                                                "(e.g. cic3d for the direction-dependent cubic cell)")
    ap.add_argument("--tile", default="", help="override launch shape: w_per_lane,dir_per_wave,waves,wg_per_cu")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain streaming kernel (read MIB, write MIB) to scale HBM byte counters")
    return ap.parse_args()


def calibrate_copy(mib: int) -> int:
    """dst = src * 1 over `mib` MiB of float32: one read and one write of known size per
    dispatch, the reference for scaling FETCH_SIZE / WRITE_SIZE counter readings."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.rand(n, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(5):
        torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(20):
        torch.mul(src, 1.0, out=dst)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 20
    print(json.dumps({"calibration": "copy", "bytes_read_per_dispatch": n * 4, "bytes_written_per_dispatch": n * 4,
                      "dispatches": 25, "ms_per_dispatch": ms,
                      "copy_GB_per_s": 2 * n * 4 / (ms * 1e-3) / 1e9}), flush=True)
    return 0


def profiled_traffic(profile: str, tile: dict, files=None, suffix: str = ""):
    """HBM bytes per launch of the profiled kernel from the committed rocprofv3 summary, or
    None if the kernel source (the accumulate sources unless `files` names others) or the
    launch shape changed since those counters were taken.  `suffix` selects one of several
    entries of a summary (e.g. ".v1" for kernel variant 1)."""
    from paper_1802_03972_amd.build import ACCUMULATE_FILES, source_sha256
    if not tile:
        return None
    path = os.path.join(ROOT, "profiles", profile)
    try:
        text = open(path).read()
        sha = source_sha256(files or ACCUMULATE_FILES)
    except OSError:
        return None
    vals = {}
    for line in text.splitlines():
        if ":" not in line:
            continue
        k, v = line.split(":", 1)
        if k == "kernel_source_sha256":
            vals[k] = v.strip()
        elif k in ("traffic_bytes_per_launch" + suffix, "tile" + suffix):
            vals[k[:len(k) - len(suffix)]] = v.strip()
    tile_s = (",".join(str(tile[k]) for k in ("w_per_lane", "dir_per_wave", "waves", "wg_per_cu"))
              if isinstance(tile, dict) else str(tile))
    if vals.get("kernel_source_sha256") != sha or vals.get("tile") != tile_s or "traffic_bytes_per_launch" not in vals:
        return None
    return float(vals["traffic_bytes_per_launch"])


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def main() -> int:
    args = parse()
    if args.calibrate_copy:
        return calibrate_copy(args.calibrate_copy)
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py: this build measures one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}); "
              "the spectrum would shard by particles with one reduction of the complex spectrum, "
              "which is not part of this build.", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_1802_03972_amd as rad
    from workloads import SINGLE, TINY, flatten

    if args.workload == "batched_uneven":
        return bench_batched(args)
    if args.workload == "serving":
        return bench_serving(args)
    if args.workload == "precision_stress":
        return bench_precision(args)
    if args.workload == "fig3_analogue":
        return bench_fig3(args)
    if args.workload == "tracked":
        return bench_tracked(args)

    w = SINGLE if args.workload == "single_bunch_fp32" else TINY
    if args.shape:
        w = w.scaled(shape=args.shape)
    om_list = None
    if args.omega_grid == "log":
        om_list = np.geomspace(1e-4 * w.omega_max, w.omega_max, w.n_omega)
    elif args.omega_grid == "blocklog":
        from workloads import block_log_omegas
        om_list = block_log_omegas(1e-4 * w.omega_max, w.omega_max, w.n_omega)
    omegas = om_list if om_list is not None else w.omegas()
    big = args.workload == "single_bunch_fp32"
    dev_id = 0
    torch.cuda.set_device(dev_id)
    stream = torch.cuda.current_stream(dev_id)

    log(f"[bench] generating {w.name}: {w.n_particles} particles x {w.n_steps} steps")
    t_gen = time.perf_counter()
    st = w.steps()
    td = torch.float32 if w.in_dtype == "f32" else torch.float64
    dev = {k: torch.as_tensor(np.ascontiguousarray(st[k]).reshape(-1)).to(f"cuda:{dev_id}", td)
           for k in rad.FIELDS}
    torch.cuda.synchronize()
    log(f"[bench] inputs resident in HBM ({sum(v.numel() * v.element_size() for v in dev.values()) / 1e6:.1f} MB, "
        f"{time.perf_counter() - t_gen:.1f} s)")
    n = w.n_particles
    times = w.times()
    slices = [{k: v[j * n:(j + 1) * n] for k, v in dev.items()} for j in range(w.n_steps)]

    g = rad.Grid(w.directions(), w.omega0, w.domega, w.n_omega, shape=w.shape,
                 shape_len=w.shape_len, dt=w.dt, device=dev_id, omegas=om_list)
    if args.tile:
        a, b, c, d = (int(x) for x in args.tile.split(","))
        g.set_tile(w_per_lane=a, dir_per_wave=b, waves=c, wg_per_cu=d)
    tile = g.get_tile()
    I_dev = torch.empty(w.n_dir * w.n_omega, dtype=torch.float64, device=f"cuda:{dev_id}")
    updates_per_step = w.n_particles * w.n_steps * w.n_dir * w.n_omega

    def one_step():
        g.reset(stream)
        for j in range(w.n_steps):
            g.push_step(float(times[j]), slices[j], stream)
        g.spectrum_device(I_dev, stream)

    for i in range(args.warmup):
        one_step()
        log(f"[bench] warmup {i + 1}/{args.warmup} queued")
    torch.cuda.synchronize()
    log("[bench] warmup done")

    # ---- timed region (kernel events recorded on the launch stream while it runs)
    g.profile(True)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for i in range(args.steps):
        one_step()
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = g.profile_read()
    g.profile(False)
    gpu_s = ev0.elapsed_time(ev1) * 1e-3
    elapsed = max(wall, gpu_s)
    value = updates_per_step * args.steps / elapsed
    log(f"[bench] timed {args.steps} steps: {elapsed * 1e3:.2f} ms ({value:.4e} updates/s)")

    avg_ms = prof["accumulate_ms"] / max(1, prof["launches"])
    upd_per_launch = prof["updates"] / max(1, prof["launches"])
    achieved = upd_per_launch * FLOPS_PER_UPDATE / (avg_ms * 1e-3) / 1e12
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / FP32_PEAK_TFLOPS, 4),
                "traffic": (profiled_traffic("k_accumulate_single_bunch_fp32.md", tile) if not g.variant else
                            profiled_traffic("k_accumulate_variants_single_bunch.md", tile, suffix=f".v{g.variant}"))
                if big else None,
                "traffic_source": ("profiles/k_accumulate_single_bunch_fp32.md" if not g.variant else
                                   "profiles/k_accumulate_variants_single_bunch.md")
                + " (FETCH_SIZE x2.000 + WRITE_SIZE x1.000, bytes per launch)",
                "kernel": "k_accumulate", "avg_launch_ms": round(avg_ms, 4),
                "updates_per_launch": int(upd_per_launch), "flops_per_update": FLOPS_PER_UPDATE,
                "fold_ms_per_launch": round(prof["fold_ms"] / max(1, prof["launches"]), 4)}

    # ---- per-push latency (each push synchronised on its own)
    lat = []
    g.reset(stream)
    for i in range(args.latency_pushes):
        j = i % w.n_steps
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        g.push_step(float(times[j]), slices[j], stream)
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - t1) * 1e3)
    latency = None
    if lat:
        lat = np.array(lat)
        latency = {"p50": round(float(np.percentile(lat, 50)), 4), "p99": round(float(np.percentile(lat, 99)), 4),
                   "unit": "ms", "what": f"one time-step push of {n} particles (accumulate + fold), host-timed"}

    # ---- FP64 CPU oracle on a bounded sample, and device parity on the same sample
    cpu = None
    parity = None
    if not args.no_cpu_baseline:
        import oracle
        cores = len(os.sched_getaffinity(0))
        oracle.set_threads(cores)
        ns, kw = (8, 4) if big else (w.n_steps, 1)   # big: about 10 s on 16 host threads
        sel = np.arange(0, w.n_omega, kw)
        sub = {k: v[:ns] for k, v in st.items()}
        samples = flatten(sub, times[:ns])
        log(f"[bench] cpu oracle: {ns} steps x {n} particles x {w.n_dir} dirs x {len(sel)} omega on {cores} threads")
        tc = time.perf_counter()
        Iref = oracle.spectrum(samples, w.directions(), omegas[sel], w.shape, w.shape_len, w.dt)
        cpu_s = time.perf_counter() - tc
        cpu_updates = ns * n * w.n_dir * len(sel)
        cpu = {"value": cpu_updates / cpu_s, "unit": "updates/s", "cores": oracle.max_threads(), "kind": "oracle",
               "sample": f"first {ns} of {w.n_steps} steps, all {n} particles, all {w.n_dir} directions, "
                         f"every {kw}th of {w.n_omega} frequencies ({cpu_updates:.3e} updates, {cpu_s:.1f} s)",
               "extrapolated_full_run_s": updates_per_step / (cpu_updates / cpu_s)}
        g.reset(stream)
        for j in range(ns):
            g.push_step(float(times[j]), slices[j], stream)
        I = g.spectrum(stream)[:, sel]
        err = float(np.max(np.abs(I - Iref)) / np.max(Iref))
        parity = {"e_inf": err, "tolerance": 1e-4, "sample": "same as cpu_baseline"}
        log(f"[bench] parity on the sample: e_inf = {err:.3e}")

    out = {
        "metric": "particle*direction*frequency updates/s (vs FP32 peak); p50/p99 step latency",
        "value": value, "unit": "updates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": w.name, "particles": w.n_particles, "time_steps": w.n_steps,
                   "directions": w.n_dir, "frequencies": w.n_omega, "omega_max": w.omega_max,
                   "shape": w.shape, "shape_len": w.shape_len, "input_dtype": w.in_dtype,
                   "omega_grid": args.omega_grid if om_list is None else
                   f"{args.omega_grid} list {om_list[0]:.3e}..{om_list[-1]:.3e}",
                   "kernel_variant": g.variant,
                   "phase": "f64", "updates_per_step": updates_per_step, "tile": tile},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "latency_ms": latency,
        "parity": parity,
    }
    g.close()
    print(json.dumps(out), flush=True)
    return 0


def bench_batched(args) -> int:
    """12 independent bunches (log-uniform counts in [1e3, 5e5]), each with its own 8x8 x 256
    grid, 200 steps.  Per step: either 12 per-bunch pushes (one launch pair each) or one
    batched persistent launch over all 12 bunches.  Same data, same grids."""
    import numpy as np
    import torch

    import paper_1802_03972_amd as rad
    from workloads import batched_uneven

    mb = batched_uneven()
    ws = mb.bunches()
    if args.time_steps:
        ws = [w.scaled(n_steps=args.time_steps) for w in ws]
    n_steps = ws[0].n_steps
    kd = max(1, min(args.distinct_steps, n_steps))
    log(f"[bench] batched_uneven: counts {list(mb.counts)}, {n_steps} steps ({kd} distinct generated steps cycled)")
    devs, grids = [], []
    for w in ws:
        st = w.steps(0, kd)
        devs.append({k: torch.as_tensor(np.ascontiguousarray(st[k]).reshape(-1)).to("cuda:0", torch.float32)
                     for k in rad.FIELDS})
        grids.append(rad.Grid(w.directions(), w.omega0, w.domega, w.n_omega, shape=w.shape,
                              shape_len=w.shape_len, dt=w.dt))
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream(0)
    batcher = rad.Batcher(max_items=len(ws))
    gbatcher = rad.Batcher(max_items=len(ws), graph=True)
    slices = [[{k: v[j * w.n_particles:(j + 1) * w.n_particles] for k, v in d.items()} for j in range(kd)]
              for w, d in zip(ws, devs)]
    times = ws[0].times()
    updates = sum(w.n_particles for w in ws) * n_steps * ws[0].n_dir * ws[0].n_omega

    def per_bunch():
        for g in grids:
            g.reset(stream)
        for j in range(n_steps):
            for b, g in enumerate(grids):
                g.push_step(float(times[j]), slices[b][j % kd], stream)

    def batched(bt=batcher):
        for g in grids:
            g.reset(stream)
        for j in range(n_steps):
            bt.push([(g, float(times[j]), 1, slices[b][j % kd]) for b, g in enumerate(grids)], stream)

    def batched_graph():
        batched(gbatcher)

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    reps = max(1, args.steps)
    if args.skip_per_bunch:
        t_pb, I_pb = float("nan"), None
    else:
        t_pb = timed(per_bunch, reps)
        log(f"[bench] per-bunch launches: {t_pb * 1e3:.1f} ms per {n_steps} steps ({updates / t_pb:.4e} updates/s)")
        I_pb = [g.spectrum() for g in grids]
    batcher.profile(True)
    t_b = timed(batched, reps)
    prof = batcher.profile_read()
    batcher.profile(False)
    log(f"[bench] batched persistent: {t_b * 1e3:.1f} ms per {n_steps} steps ({updates / t_b:.4e} updates/s)")
    I_b = [g.spectrum() for g in grids]
    t_g = timed(batched_graph, reps)
    I_g = [g.spectrum() for g in grids]
    graph_equal = all(np.array_equal(a, b) for a, b in zip(I_b, I_g))
    log(f"[bench] batched persistent, graph replays: {t_g * 1e3:.1f} ms per {n_steps} steps "
        f"({updates / t_g:.4e} updates/s), bitwise equal to direct: {graph_equal}, {gbatcher.graph_stats()}")
    agree = None if I_pb is None else max(float(np.max(np.abs(a - b)) / np.max(a)) for a, b in zip(I_pb, I_b))
    # FP64 CPU oracle on the smallest bunch (all steps, every 2nd frequency), and the batched
    # spectrum of that bunch against it
    cpu = parity = None
    if not args.no_cpu_baseline:
        import oracle
        from workloads import flatten
        b = int(np.argmin([w.n_particles for w in ws]))
        w = ws[b]
        st = w.steps(0, kd)
        full = {k: np.stack([st[k][j % kd] for j in range(n_steps)]) for k in st}
        sel = np.arange(0, w.n_omega, 2)
        cores = len(os.sched_getaffinity(0))
        oracle.set_threads(cores)
        tc = time.perf_counter()
        Iref = oracle.spectrum(flatten(full, times[:n_steps]), w.directions(), w.omegas()[sel], w.shape,
                               w.shape_len, w.dt)
        cpu_s = time.perf_counter() - tc
        cu = w.n_particles * n_steps * w.n_dir * len(sel)
        cpu = {"value": cu / cpu_s, "unit": "updates/s", "cores": oracle.max_threads(), "kind": "oracle",
               "sample": f"bunch {b} ({w.n_particles} particles), all {n_steps} steps, all {w.n_dir} directions, "
                         f"every 2nd of {w.n_omega} frequencies ({cu:.3e} updates, {cpu_s:.1f} s)"}
        parity = {"e_inf": float(np.max(np.abs(I_b[b][:, sel] - Iref)) / np.max(Iref)), "tolerance": 1e-4,
                  "sample": "same as cpu_baseline (batched direct launches)"}
        log(f"[bench] batched parity on the sample: e_inf = {parity['e_inf']:.3e}")
    avg_ms = prof["accumulate_ms"] / max(1, prof["launches"])
    achieved = prof["updates"] / max(1, prof["launches"]) * FLOPS_PER_UPDATE / (avg_ms * 1e-3) / 1e12
    out = {
        "metric": "particle*direction*frequency updates/s (vs FP32 peak); p50/p99 step latency",
        "value": updates / t_b, "unit": "updates/s", "n_gpus": 1, "steps": reps, "warmup": 1,
        "ms_per_step": t_b * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "batched_uneven", "bunches": len(ws), "counts": list(mb.counts),
                   "time_steps": n_steps, "directions": ws[0].n_dir, "frequencies": ws[0].n_omega,
                   "distinct_generated_steps": kd, "updates_per_step": updates,
                   "tile": batcher.get_tile(), "per_bunch_tile": grids[0].get_tile()},
        "per_bunch_launches": {"value": updates / t_pb, "ms_per_step": t_pb * 1e3},
        "batched_graph": {"value": updates / t_g, "ms_per_step": t_g * 1e3, "bitwise_equal_to_direct": graph_equal},
        "speedup_vs_per_bunch": t_pb / t_b,
        "batched_vs_per_bunch_e_inf": agree,
        "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved / FP32_PEAK_TFLOPS, 4),
                     "traffic": profiled_traffic("k_accumulate_batch_batched_uneven.md", batcher.get_tile()),
                     "traffic_source": "profiles/k_accumulate_batch_batched_uneven.md (FETCH_SIZE and WRITE_SIZE "
                                       "scaled by the copy-kernel calibration, bytes per launch)",
                     "kernel": "k_accumulate_batch", "avg_launch_ms": round(avg_ms, 4),
                     "fold_ms_per_launch": round(prof["fold_ms"] / max(1, prof["launches"]), 4)},
        "cpu_baseline": cpu,
        "parity": parity,
    }
    print(json.dumps(out), flush=True)
    return 0


def bench_serving(args) -> int:
    """8 LWFA-like bunches (counts log-uniform in [1e4, 2e5], gamma ~ U(20, 500), CIC) on
    8x16 x 512 grids.  Chunks (one step of one bunch, FP32, pinned host memory) arrive as a
    Poisson process; the serving loop admits them by HBM footprint and batches them into
    persistent launches.  Reports throughput, p50/p99 arrival-to-completion latency and
    the backlog at the stated rate, then at 0.5x and 0.8x of the measured capacity."""
    import numpy as np
    import torch

    import paper_1802_03972_amd as rad
    from workloads import serving_bunches, poisson_trace

    sv = serving_bunches()
    ws = sv.bunches()
    kd = max(1, args.distinct_steps)
    log(f"[bench] serving: counts {list(sv.counts)}, {kd} distinct generated steps per bunch")
    host = []
    for w in ws:
        st = w.steps(0, kd)
        host.append([{k: torch.from_numpy(np.ascontiguousarray(st[k][j], dtype=np.float32)).pin_memory()
                      for k in rad.FIELDS} for j in range(kd)])
    grids = [rad.Grid(w.directions(), w.omega0, w.domega, w.n_omega, shape=w.shape,
                      shape_len=w.shape_len, dt=w.dt) for w in ws]
    per_chunk_updates = np.array([w.n_particles * w.n_dir * w.n_omega for w in ws], dtype=np.float64)

    server_tile = []
    served_steps = []

    def run(rate, n_chunks, seed):
        arrivals, which = poisson_trace(rate, n_chunks, len(ws), seed=seed)
        srv = rad.Server(hbm_budget=4 << 30, max_batch=64, max_inflight=2, max_admitted=256, poll_us=20)
        step_of = [0] * len(ws)
        t0 = srv.counters()["now"]
        wall0 = time.perf_counter()
        tickets = []
        max_backlog = 0
        for i in range(n_chunks):
            target = wall0 + arrivals[i]
            while True:
                d = target - time.perf_counter()
                if d <= 0:
                    break
                time.sleep(min(d, 0.002))
            b = int(which[i])
            j = step_of[b]
            step_of[b] += 1
            tickets.append((srv.submit(grids[b], float(j) * ws[b].dt, host[b][j % kd]), b, t0 + arrivals[i]))
            if i % 256 == 0:
                max_backlog = max(max_backlog, srv.counters()["pending"])
        srv.drain()
        cnt = srv.counters()
        lat, done, first, bsz = [], [], None, []
        for tk, b, t_arr in tickets:
            s = srv.wait(tk)
            lat.append(s["t_complete"] - t_arr)
            done.append(s["t_complete"])
            bsz.append(s["batch_size"])
        server_tile.append(srv.get_tile())
        served_steps.append(list(step_of))
        srv.close()
        total = float(sum(per_chunk_updates[b] for _, b, _ in tickets))
        span = max(done) - (t0 + arrivals[0])
        lat = np.array(lat) * 1e3
        return {"rate_chunks_per_s": rate, "chunks": n_chunks,
                "offered_updates_per_s": float(rate * per_chunk_updates.mean()),
                "achieved_updates_per_s": total / span, "span_s": span,
                "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                "max_pending_seen": int(max_backlog), "batches": int(cnt["batches"]),
                "mean_batch": float(np.mean(bsz))}

    full = run(args.rate, args.chunks, seed=0)
    log(f"[bench] serving at {args.rate:.0f}/s: {full}")
    # FP64 CPU oracle on the smallest bunch's served steps (16 directions x every 32nd
    # frequency), and its served spectrum against it (read before the load-scaled runs add
    # to the same grids)
    cpu = parity = None
    if not args.no_cpu_baseline:
        import oracle
        from workloads import flatten
        b = int(np.argmin([w.n_particles for w in ws]))
        w = ws[b]
        n_b = served_steps[0][b]
        st = w.steps(0, kd)
        stf = {k: np.stack([st[k][j % kd].astype(np.float32).astype(np.float64) for j in range(n_b)]) for k in st}
        dsel = np.arange(0, w.n_dir, max(1, w.n_dir // 16))
        osel = np.arange(0, w.n_omega, 32)
        cores = len(os.sched_getaffinity(0))
        oracle.set_threads(cores)
        tc = time.perf_counter()
        Iref = oracle.spectrum(flatten(stf, np.arange(n_b, dtype=np.float64) * w.dt), w.directions()[dsel],
                               w.omegas()[osel], w.shape, w.shape_len, w.dt)
        cpu_s = time.perf_counter() - tc
        cu = w.n_particles * n_b * len(dsel) * len(osel)
        cpu = {"value": cu / cpu_s, "unit": "updates/s", "cores": oracle.max_threads(), "kind": "oracle",
               "sample": f"bunch {b} ({w.n_particles} particles), its {n_b} served steps, {len(dsel)} of "
                         f"{w.n_dir} directions x {len(osel)} of {w.n_omega} frequencies ({cu:.3e} updates, "
                         f"{cpu_s:.1f} s)"}
        I = grids[b].spectrum()[np.ix_(dsel, osel)]
        parity = {"e_inf": float(np.max(np.abs(I - Iref)) / np.max(Iref)), "tolerance": 1e-4,
                  "sample": "same as cpu_baseline (served spectrum of that bunch)"}
        log(f"[bench] serving parity on the sample: e_inf = {parity['e_inf']:.3e}")
    cap = full["achieved_updates_per_s"] / per_chunk_updates.mean()
    scaled = []
    for f in (0.5, 0.8):
        r = run(f * cap, max(200, args.chunks // 4), seed=1)
        r["load_fraction"] = f
        log(f"[bench] serving at {f:.1f}x capacity ({f * cap:.0f}/s): {r}")
        scaled.append(r)
    out = {
        "metric": "particle*direction*frequency updates/s (vs FP32 peak); p50/p99 step latency",
        "value": full["achieved_updates_per_s"], "unit": "updates/s", "n_gpus": 1, "steps": args.chunks,
        "warmup": 0, "ms_per_step": full["span_s"] / args.chunks * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "serving", "bunches": len(ws), "counts": list(sv.counts),
                   "directions": ws[0].n_dir, "frequencies": ws[0].n_omega, "rate_chunks_per_s": args.rate,
                   "chunks": args.chunks, "distinct_generated_steps": kd, "batched_tile": server_tile[0]},
        "latency_ms": {"p50": full["p50_ms"], "p99": full["p99_ms"], "unit": "ms",
                       "what": "chunk arrival to completion"},
        "serving": full, "load_scaled": scaled,
        "cpu_baseline": cpu,
        "parity": parity,
    }
    print(json.dumps(out), flush=True)
    return 0


def error_report(I, Iref) -> dict:
    import numpy as np
    peak = float(np.max(Iref))
    diff = np.abs(I - Iref)
    big = Iref >= 1e-2 * peak
    col = np.maximum(np.max(Iref, axis=0), 1e-300)
    return {"e_inf": float(np.max(diff) / peak),
            "per_frequency_max": float(np.max(np.max(diff, axis=0) / col)),
            "per_frequency_max_top_quarter": float(np.max((np.max(diff, axis=0) / col)[-max(1, Iref.shape[1] // 4):])),
            "l2_rel": float(np.linalg.norm(I - Iref) / np.linalg.norm(Iref)),
            "per_direction_max": float(max(np.max(diff[d]) / max(np.max(Iref[d]), 1e-300)
                                           for d in range(Iref.shape[0]))),
            "per_point_rel_max_bins_ge_1e-2_peak": float(np.max(diff[big] / Iref[big])) if big.any() else 0.0,
            "abs_max": float(np.max(diff)), "peak": peak}


def bench_precision(args) -> int:
    """Precision stress: 16384 particles x 10000 steps from t0 = 1 ps, gamma ~ U(50, 1000),
    8x8 x 1024 frequencies to 1e20 rad/s, FP64 input.  Both arithmetic modes (FP64 geometry
    and phase with FP32 update; everything FP32) accumulate every step on the device; the
    FP64 oracle (the CPU-baseline leg) evaluates 4 directions x 9 frequencies of the same
    sum, and both device spectra are compared with it there.  Steps are generated, pushed
    and handed to the oracle in groups of 100."""
    import numpy as np
    import torch

    import paper_1802_03972_amd as rad
    from workloads import PRECISION, SINGLE, flatten

    w = PRECISION
    n_steps = args.time_steps or w.n_steps
    group = 100
    bunch = w.bunch()
    grids = {"fp64_phase": rad.Grid(w.directions(), w.omega0, w.domega, w.n_omega, shape=w.shape,
                                    shape_len=w.shape_len, dt=w.dt, precision=rad.PHASE_F64),
             "all_fp32": rad.Grid(w.directions(), w.omega0, w.domega, w.n_omega, shape=w.shape,
                                  shape_len=w.shape_len, dt=w.dt, precision=rad.ALL_F32)}
    for g in grids.values():
        g.profile(True)
    dsel = np.array([0, 9, 36, 63])
    osel = np.unique(np.concatenate([np.arange(0, w.n_omega, 128), [w.n_omega - 1]]))
    use_oracle = not args.no_cpu_baseline
    S_ref = None
    cpu_s = 0.0
    if use_oracle:
        import oracle
        oracle.set_threads(len(os.sched_getaffinity(0)))
    log(f"[bench] precision_stress: {w.n_particles} particles x {n_steps} steps from t0 = {w.t0:g} s")
    for j0 in range(0, n_steps, group):
        j1 = min(n_steps, j0 + group)
        st = w.steps(j0, j1, bunch=bunch)
        dev = {k: torch.as_tensor(np.ascontiguousarray(st[k]).reshape(-1)).to("cuda:0") for k in rad.FIELDS}
        t0 = float(w.times(j0, j0 + 1)[0])
        for g in grids.values():
            g.push_steps(t0, j1 - j0, dev)
        if use_oracle:   # cpu_baseline leg: the FP64 oracle on the direction x frequency subset
            tc = time.perf_counter()
            S = oracle.spectrum_complex(flatten(st, w.times(j0, j1)), w.directions()[dsel], w.omegas()[osel],
                                        w.shape, w.shape_len)
            cpu_s += time.perf_counter() - tc
            S_ref = S if S_ref is None else S_ref + S
        torch.cuda.synchronize()
        if j0 % 1000 == 0:
            log(f"[bench] steps {j1}/{n_steps}")
    out_modes = {}
    for name, g in grids.items():
        prof = g.profile_read()
        out_modes[name] = {"updates_per_s_kernel": prof["updates"] / (prof["accumulate_ms"] * 1e-3),
                           "accumulate_ms": prof["accumulate_ms"]}
    cpu = None
    if use_oracle:
        Iref = oracle.prefactor(w.dt) * np.sum(np.abs(S_ref) ** 2, axis=-1)
        for name, g in grids.items():
            out_modes[name]["errors_vs_oracle"] = error_report(g.spectrum()[np.ix_(dsel, osel)], Iref)
            log(f"[bench] {name}: {out_modes[name]}")
        upd = w.n_particles * n_steps * len(dsel) * len(osel)
        cpu = {"value": upd / cpu_s, "unit": "updates/s", "cores": oracle.max_threads(), "kind": "oracle",
               "sample": f"all {n_steps} steps x {w.n_particles} particles, directions {dsel.tolist()}, "
                         f"frequency indices {osel.tolist()} ({upd:.3e} updates, {cpu_s:.1f} s)",
               "extrapolated_full_run_s": w.n_particles * n_steps * w.n_dir * w.n_omega / (upd / cpu_s)}
        # input rounding of the FP32-input single-bunch workload: oracle on the FP64 trajectory
        # vs oracle on the FP32-rounded one (4 steps, every 16th frequency)
        ws = SINGLE.scaled(n_steps=4)
        b2 = ws.bunch()
        from workloads import stack_steps
        exact = stack_steps(b2, ws.times())
        rounded = {k: v.astype(np.float32).astype(np.float64) for k, v in exact.items()}
        om = ws.omegas()[::16]
        I_exact = oracle.spectrum(flatten(exact, ws.times()), ws.directions(), om, ws.shape, ws.shape_len, ws.dt)
        I_round = oracle.spectrum(flatten(rounded, ws.times()), ws.directions(), om, ws.shape, ws.shape_len, ws.dt)
        input_rounding = error_report(I_round, I_exact)
    out = {
        "metric": "particle*direction*frequency updates/s (vs FP32 peak); p50/p99 step latency",
        "value": out_modes["fp64_phase"]["updates_per_s_kernel"], "unit": "updates/s", "n_gpus": 1,
        "steps": n_steps, "warmup": 0, "ms_per_step": out_modes["fp64_phase"]["accumulate_ms"] / n_steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "precision_stress", "particles": w.n_particles, "time_steps": n_steps, "t0": w.t0,
                   "directions": w.n_dir, "frequencies": w.n_omega, "omega_max": w.omega_max, "input_dtype": "f64"},
        "modes": out_modes, "cpu_baseline": cpu,
        "input_rounding_single_bunch_fp32": input_rounding if use_oracle else None,
    }
    print(json.dumps(out), flush=True)
    return 0


def bench_tracked(args) -> int:
    """Post-processing variant: 1024 tracked particles x 100 steps of the single-bunch
    generator on its 128 x 256 grid; each step adds every particle's term into its own FP64
    time integral (read-modify-write of 32 B per particle and grid point), and the read-out
    applies weights and shape afterwards.  The timed push hands all 100 steps to one launch,
    which sums up to `Tracked.step_group()` (128) steps in registers before each
    read-modify-write of the integrals (64 B per particle and grid point per group);
    one-step pushes (64 B per update, HBM-bound) are timed beside it."""
    import numpy as np
    import torch

    import paper_1802_03972_amd as rad
    from paper_1802_03972_amd.build import AUX_FILES
    from workloads import SINGLE, flatten

    w = SINGLE.scaled(n_particles=1024, n_steps=100, seed=7)
    st = w.steps()
    n = w.n_particles
    dev = {k: torch.as_tensor(np.ascontiguousarray(st[k]).reshape(-1)).to("cuda:0", torch.float32)
           for k in rad.FIELDS}
    slices = [{k: v[j * n:(j + 1) * n] for k, v in dev.items()} for j in range(w.n_steps)]
    times = w.times()
    tr = rad.Tracked(w.directions(), w.omega0, w.domega, w.n_omega, n, dt=w.dt)
    stream = torch.cuda.current_stream(0)
    wts = st["w"][0]

    def pushes():
        tr.reset(stream)
        tr.push_steps(float(times[0]), w.n_steps, dev, stream)

    for _ in range(max(1, args.warmup)):
        pushes()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        pushes()
    ev1.record(stream)
    torch.cuda.synchronize()
    elapsed = max(time.perf_counter() - t0, ev0.elapsed_time(ev1) * 1e-3)
    updates = n * w.n_dir * w.n_omega * w.n_steps
    value = updates * args.steps / elapsed
    # duration of the accumulate kernel alone: the 100-step push (one launch) and, for
    # comparison, 100 one-step pushes (events bracket only the pushes; the reset fill runs
    # before the first event)
    def timed_push(multi):
        tr.reset(stream)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        if multi:
            tr.push_steps(float(times[0]), w.n_steps, dev, stream)
        else:
            for j in range(w.n_steps):
                tr.push_step(float(times[j]), slices[j], stream)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1)
    single_ms = None if args.skip_one_step else timed_push(False) / w.n_steps
    launch_ms = timed_push(True)
    group = rad.Tracked.step_group()
    groups = -(-w.n_steps // group)
    points = n * w.n_dir * w.n_omega
    bytes_per_launch = 64.0 * points * groups + 40.0 * n * w.n_steps
    hbm = bytes_per_launch / (launch_ms * 1e-3) / 1e9
    # the tracked update has no form-factor scale (weights and shape enter at read-out):
    # rotate 6 + three complex multiply-adds 12 = 18 flops in the 3-component form
    flops = FLOPS_PER_UPDATE - 2
    alu = points * w.n_steps * flops / (launch_ms * 1e-3) / 1e12
    tc = time.perf_counter()
    I = tr.spectrum(wts, w.shape, w.shape_len, stream)
    readout_ms = (time.perf_counter() - tc) * 1e3
    # the tracked kernel has one launch shape
    tile = f"fixed: 256 threads, 8 frequencies per thread, {group}-step groups"
    cpu = None
    parity = None
    if not args.no_cpu_baseline:
        import oracle
        cores = len(os.sched_getaffinity(0))
        oracle.set_threads(cores)
        sel = np.arange(0, w.n_omega, 4)
        tc = time.perf_counter()
        Iref = oracle.spectrum(flatten(st, times), w.directions(), w.omegas()[sel], w.shape, w.shape_len, w.dt)
        cpu_s = time.perf_counter() - tc
        cu = n * w.n_steps * w.n_dir * len(sel)
        cpu = {"value": cu / cpu_s, "unit": "updates/s", "cores": oracle.max_threads(), "kind": "oracle",
               "sample": f"all {w.n_steps} steps x {n} particles x {w.n_dir} directions x every 4th of "
                         f"{w.n_omega} frequencies ({cu:.3e} updates, {cpu_s:.1f} s)",
               "extrapolated_full_run_s": n * w.n_steps * w.n_dir * w.n_omega / (cu / cpu_s)}
        parity = {"e_inf": float(np.max(np.abs(I[:, sel] - Iref)) / np.max(Iref)), "tolerance": 1e-4,
                  "sample": "same as cpu_baseline"}
        log(f"[bench] tracked parity on the sample: e_inf = {parity['e_inf']:.3e}")
    tr.close()
    log(f"[bench] tracked: {value:.4e} updates/s; 100-step push {launch_ms:.3f} ms ({hbm:.0f} GB/s, "
        f"{alu:.1f} TFLOP/s)" + ("" if single_ms is None else
                                  f"; one-step pushes {single_ms:.4f} ms each "
                                  f"({64.0 * points / (single_ms * 1e-3) / 1e9:.0f} GB/s)"))
    out = {
        "metric": "particle*direction*frequency updates/s (vs FP32 peak); p50/p99 step latency",
        "value": value, "unit": "updates/s", "n_gpus": 1, "steps": args.steps, "warmup": max(1, args.warmup),
        "ms_per_step": elapsed / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "tracked", "particles": n, "time_steps": w.n_steps, "directions": w.n_dir,
                   "frequencies": w.n_omega, "shape_at_readout": w.shape, "integrals_bytes": 32 * n * w.n_dir * w.n_omega,
                   "step_group": group},
        "roofline": ({"bound": "alu", "achieved": round(alu, 3), "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                      "frac": round(alu / FP32_PEAK_TFLOPS, 4)}
                     if alu / FP32_PEAK_TFLOPS >= hbm / HBM_PEAK_GBS else
                     {"bound": "hbm", "achieved": round(hbm, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                      "frac": round(hbm / HBM_PEAK_GBS, 4)}) | {
                     "traffic": profiled_traffic("k_tracked_accumulate_tracked.md", tile, AUX_FILES),
                     "kernel": "k_tracked_accumulate", "avg_launch_ms": round(launch_ms, 4),
                     "algorithmic_hbm_GB_per_s": round(hbm, 1), "algorithmic_TFLOP_per_s": round(alu, 3),
                     "bytes_per_launch": bytes_per_launch, "flops_per_update": flops},
        "one_step_pushes": None if single_ms is None else {
            "ms_per_push": round(single_ms, 4), "hbm_GB_per_s": round(64.0 * points / (single_ms * 1e-3) / 1e9, 1),
            "updates_per_s": points / (single_ms * 1e-3)},
        "readout_ms": round(readout_ms, 3),
        "cpu_baseline": cpu,
        "parity": parity,
    }
    print(json.dumps(out), flush=True)
    return 0


def bench_fig3(args) -> int:
    """Synthetic analogue of the paper's Fig. 3: ONE macro-particle (N = 1e5 electrons) on a
    betatron trajectory (gamma 100, 100 fs), spectrum on axis and 10 mrad off axis over
    log-spaced frequencies 1e13 .. 1e19 rad/s, with three weightings evaluated on the device:
    point shape (all coherent, N^2), a shape so wide that g = 0 (all incoherent, N), and the
    Gaussian macro-particle shape sigma = 0.1 um (form factor, Eq. 12).  Reports the
    coherent -> incoherent transition frequency, where (N - 1) g = 1, measured from the
    device spectra and from the closed form (c / sigma) sqrt(ln(N - 1))."""
    import numpy as np
    import torch

    import paper_1802_03972_amd as rad
    from workloads import TINY

    N = 1e5
    sigma = 0.1e-6
    w = TINY.scaled(n_particles=1, n_steps=2000, gamma=("const", 100.0), seed=5)
    st = w.steps()
    one = dict(st)
    one["w"] = np.ones_like(st["w"])
    macro = dict(st)
    macro["w"] = np.full_like(st["w"], N)
    dirs = np.array([[0.0, 0.0, 1.0], [0.01, 0.0, np.sqrt(1 - 1e-4)]])
    om = np.geomspace(1e13, 1e19, 241)
    dev1 = {k: torch.as_tensor(np.ascontiguousarray(one[k]).reshape(-1)).to("cuda:0") for k in rad.FIELDS}
    devN = {k: torch.as_tensor(np.ascontiguousarray(macro[k]).reshape(-1)).to("cuda:0") for k in rad.FIELDS}

    def run(shape, length, parts):
        g = rad.Grid(dirs, 0.0, 0.0, 0, shape=shape, shape_len=length, dt=w.dt, omegas=om)
        g.profile(True)
        g.push_steps(w.t0, w.n_steps, parts)
        I = g.spectrum()
        prof = g.profile_read()
        return I, prof

    I1, _ = run("point", 0.0, dev1)
    Icoh, _ = run("point", 0.0, devN)
    Iinc, _ = run("gauss", 1.0, devN)
    Iff, prof = run("gauss", sigma, devN)
    ratio = Iff / I1
    g_ref = np.exp(-(om * sigma / 299792458.0) ** 2)
    F2 = N + (N * N - N) * g_ref
    dev_coh = float(np.max(np.abs(Icoh / I1 / N ** 2 - 1)))
    dev_inc = float(np.max(np.abs(Iinc / I1 / N - 1)))
    dev_ff = float(np.max(np.abs(ratio / F2 - 1)))
    # transition: F^2 = 2N, interpolated in log(omega) on the on-axis spectrum
    y = np.log(ratio[0] / (2 * N))
    k = int(np.argmax(y < 0))
    t = y[k - 1] / (y[k - 1] - y[k])
    om_t = float(np.exp(np.log(om[k - 1]) + t * (np.log(om[k]) - np.log(om[k - 1]))))
    om_t_ref = 299792458.0 / sigma * np.sqrt(np.log(N - 1))
    table = []
    for i in range(0, len(om), 20):
        table.append({"omega": float(om[i]), "I_single": float(I1[0, i]), "I_coherent": float(Icoh[0, i]),
                      "I_incoherent": float(Iinc[0, i]), "I_form_factor": float(Iff[0, i])})
    out = {
        "metric": "particle*direction*frequency updates/s (vs FP32 peak); p50/p99 step latency",
        "value": prof["updates"] / (prof["accumulate_ms"] * 1e-3), "unit": "updates/s", "n_gpus": 1,
        "steps": w.n_steps, "warmup": 0, "ms_per_step": prof["accumulate_ms"] / w.n_steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "fig3_analogue", "macro_particles": 1, "electrons": N, "gamma": 100.0,
                   "time_steps": w.n_steps, "directions": 2, "frequencies": len(om), "omega_grid": "log 1e13..1e19",
                   "shape": "gauss", "sigma": sigma},
        "transition_omega": {"measured": om_t, "closed_form": float(om_t_ref),
                             "rel_diff": float(abs(om_t / om_t_ref - 1))},
        "max_rel_dev": {"coherent_vs_N2": dev_coh, "incoherent_vs_N": dev_inc, "form_factor_vs_Eq12": dev_ff},
        "on_axis_table": table,
    }
    log(f"[bench] fig3 analogue: transition {om_t:.4e} (closed form {om_t_ref:.4e}); deviations "
        f"coh {dev_coh:.2e} inc {dev_inc:.2e} ff {dev_ff:.2e}")
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
