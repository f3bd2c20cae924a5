#!/usr/bin/env python3
"""Throughput of the in-situ macro-particle radiation sum on one MI355X.

Default run (no --workload): every workload, one JSON line.  The headline `value` is the
single-bunch FP32 case -- 65536 macro-particles, 100 time steps (dt = 0.05 fs), 128
directions (8 x 16 within +-20 mrad) x 256 uniform frequencies up to 1e19 rad/s, CIC shape
0.1 um, betatron trajectories, FP32 particle input, FP64 phase.  One bench step = one
complete spectrum: reset, 100 per-time-step pushes through the C ABI (the in-situ
evaluation, one push per simulation step) and the |S|^2 read-out on device.  The line also
carries, under "configs", the tiny FP64 case, the batched uneven bunches (12 bunches, 200
steps, batched vs per-bunch launches), the precision stress (16384 particles x 10000 steps
from 1 ps, both arithmetic modes) and the serving loop (8 bunches, Poisson arrivals, p50/p99
at the stated rate and at 0.5x / 0.8x of capacity), each with its kernel roofline (HIP
events on the launch stream), the FP64 CPU oracle's rate on a bounded sample and
device-vs-oracle parity on that sample (e_inf and the per-frequency error).

--workload NAME runs one workload and prints its line alone.
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
METRIC = "particle*direction*frequency updates/s (vs FP32 peak); p50/p99 step latency"
WORKLOADS = ["single_bunch_fp32", "tiny_fp64", "batched_uneven", "serving", "precision_stress",
             "fig3_analogue", "tracked"]


def parse(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="all", choices=["all"] + WORKLOADS)
    ap.add_argument("--time-steps", type=int, default=0,
                    help="batched_uneven / precision_stress: override the 200 / 10000 time steps")
    ap.add_argument("--skip-per-bunch", action="store_true", help="batched_uneven: time only the batched launch")
    ap.add_argument("--skip-one-step", action="store_true",
                    help="tracked: time only the multi-step push (no one-step comparison)")
    ap.add_argument("--chunks", type=int, default=4000, help="serving: chunks in the arrival trace")
    ap.add_argument("--rate", type=float, default=2000.0, help="serving: Poisson arrival rate [chunks/s]")
    ap.add_argument("--distinct-steps", type=int, default=8,
                    help="serving: generated steps per bunch, replayed (with their own times) over the trace")
    ap.add_argument("--batched-reps", type=int, default=2, help="batched_uneven: timed runs of the 200 steps per mode")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--latency-pushes", type=int, default=100)
    ap.add_argument("--omega-grid", choices=("uniform", "log", "blocklog"), default="uniform",
                    help="single_bunch_fp32: 'log' passes the frequencies as an explicit log-spaced list "
                         "(1e-4 * omega_max .. omega_max), evaluated with a per-term FP64 phase; 'blocklog' "
                         "spans the same range uniformly inside each block of 16 and log-like across "
                         "blocks (frequency walk with a per-block step)")
    ap.add_argument("--shape", default="", help="single_bunch_fp32: override the macro-particle shape "
                                                "(e.g. cic3d for the direction-dependent cubic cell)")
    ap.add_argument("--tile", default="", help="override launch shape: w_per_lane,dir_per_wave,waves,wg_per_cu")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain streaming kernel (read MIB, write MIB) to scale HBM byte counters")
    return ap.parse_args(argv)


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


def profile_values(profile: str, tile, files=None, suffix: str = "") -> dict:
    """Per-launch counter figures of the profiled kernel from the committed rocprofv3
    summary (traffic_bytes_per_launch, executed_fp32_flops_per_update), or {} if the kernel
    source (the accumulate sources unless `files` names others) or the launch shape changed
    since those counters were taken.  `suffix` selects one of several entries of a summary
    (e.g. ".v1" for kernel variant 1)."""
    from paper_1802_03972_amd.build import ACCUMULATE_FILES, source_sha256
    if not tile:
        return {}
    path = os.path.join(ROOT, "profiles", profile)
    try:
        text = open(path).read()
        sha = source_sha256(files or ACCUMULATE_FILES)
    except OSError:
        return {}
    vals = {}
    keys = ("traffic_bytes_per_launch", "executed_fp32_flops_per_update", "tile")
    for line in text.splitlines():
        if ":" not in line:
            continue
        k, v = line.split(":", 1)
        if k == "kernel_source_sha256":
            vals[k] = v.strip()
        elif k in tuple(x + suffix for x in keys):
            vals[k[:len(k) - len(suffix)]] = v.strip()
    tile_s = (",".join(str(tile[k]) for k in ("w_per_lane", "dir_per_wave", "waves", "wg_per_cu"))
              if isinstance(tile, dict) else str(tile))
    if vals.get("kernel_source_sha256") != sha or vals.get("tile") != tile_s:
        return {}
    return {k: float(vals[k]) for k in keys[:2] if k in vals}


def alu_roofline(updates_per_launch: float, avg_ms: float, kernel: str, profile: str = "", tile=None,
                 files=None, suffix: str = "", **extra) -> dict:
    """Roofline entry of an accumulate kernel: algorithmic FP32 flops (20 per update) per
    launch over the launch's measured average duration, against the FP32 vector peak.
    From the profile (while its kernel hash and launch shape match): HBM traffic per launch
    and the executed FP32 flops per update (SQ_INSTS_VALU_FLOPS_FP32), giving the executed
    fraction of the peak beside the algorithmic one."""
    achieved = updates_per_launch * FLOPS_PER_UPDATE / (avg_ms * 1e-3) / 1e12
    pv = profile_values(profile, tile, files, suffix) if profile else {}
    exe = pv.get("executed_fp32_flops_per_update")
    out = {"bound": "alu", "achieved": round(achieved, 3), "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
           "frac": round(achieved / FP32_PEAK_TFLOPS, 4), "traffic": pv.get("traffic_bytes_per_launch"),
           "kernel": kernel, "avg_launch_ms": round(avg_ms, 4), "updates_per_launch": int(updates_per_launch),
           "flops_per_update": FLOPS_PER_UPDATE,
           "frac_executed": None if exe is None else round(achieved / FLOPS_PER_UPDATE * exe / FP32_PEAK_TFLOPS, 4),
           "executed_fp32_flops_per_update": exe,
           "counters_source": f"profiles/{profile}" if pv else None}
    out.update(extra)
    return out


def parity_entry(I, Iref, ks, sample: str) -> dict:
    """Device vs oracle on a sample: the full error report and the gate (e_inf and the
    per-frequency error within 1e-4)."""
    from oracle.metrics import TOL, error_report, passes
    rep = error_report(I, Iref, ks)
    rep.update({"tolerance": TOL, "pass": passes(rep), "sample": sample})
    return rep


def rounding_entry(w, n_steps: int, om_stride: int) -> dict:
    """How much the FP32 rounding of the input trajectory alone moves the spectrum: the
    oracle on the FP64 trajectory against the oracle on its FP32 rounding (what the device
    ingests), over the first n_steps steps of bunch w and every om_stride-th frequency."""
    import numpy as np
    import oracle
    from oracle.metrics import error_report
    from workloads import flatten, stack_steps
    wn = w.scaled(n_steps=n_steps)
    exact = stack_steps(wn.bunch(), wn.times())
    rounded = {k: v.astype(np.float32).astype(np.float64) for k, v in exact.items()}
    om = wn.omegas()[::om_stride]
    I_exact = oracle.spectrum(flatten(exact, wn.times()), wn.directions(), om, wn.shape, wn.shape_len, wn.dt)
    I_round = oracle.spectrum(flatten(rounded, wn.times()), wn.directions(), om, wn.shape, wn.shape_len, wn.dt)
    rep = error_report(I_round, I_exact)
    rep["sample"] = (f"{wn.n_particles} particles x {n_steps} steps, {wn.n_dir} directions x every "
                     f"{om_stride}th of {w.n_omega} frequencies")
    return rep


def cpu_entry(updates: float, seconds: float, sample: str, **extra) -> dict:
    import oracle
    out = {"value": updates / seconds, "unit": "updates/s", "cores": oracle.max_threads(), "kind": "oracle",
           "sample": f"{sample} ({updates:.3e} updates, {seconds:.1f} s)"}
    out.update(extra)
    return out


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def host_threads() -> int:
    from workloads import host_workers
    return host_workers()


def set_oracle_threads() -> None:
    import oracle
    oracle.set_threads(len(os.sched_getaffinity(0)))


def main() -> int:
    args = parse()
    if args.calibrate_copy:
        return calibrate_copy(args.calibrate_copy)
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py: the library runs on one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}); "
              "the spectrum would shard by particles with one reduction of the complex spectrum, "
              "which is not implemented.", file=sys.stderr)
        return 2

    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    from paper_1802_03972_amd.build import ensure_built
    ensure_built()    # a built library is used as is; none in the tree: build it first
    import paper_1802_03972_amd  # noqa: F401

    runners = {"single_bunch_fp32": lambda: bench_single(args, "single_bunch_fp32"),
               "tiny_fp64": lambda: bench_single(args, "tiny_fp64"),
               "batched_uneven": lambda: bench_batched(args),
               "serving": lambda: bench_serving(args),
               "precision_stress": lambda: bench_precision(args),
               "fig3_analogue": lambda: bench_fig3(args),
               "tracked": lambda: bench_tracked(args)}
    if args.workload != "all":
        out = runners[args.workload]()
        print(json.dumps(out), flush=True)
        return 0 if (out.get("parity") or {}).get("pass", True) else 1

    t_all = time.perf_counter()
    head = runners["single_bunch_fp32"]()
    configs = {}
    for name in ("tiny_fp64", "batched_uneven", "precision_stress", "serving"):
        t0 = time.perf_counter()
        log(f"[bench] ---- {name}")
        configs[name] = runners[name]()
        configs[name]["bench_seconds"] = round(time.perf_counter() - t0, 1)
    head["configs"] = configs
    checks = {"single_bunch_fp32": head.get("parity")}
    for name, c in configs.items():
        if c.get("parity") is not None:
            checks[name] = c["parity"]
        for mode, m in (c.get("modes") or {}).items():
            if m.get("parity") is not None and mode != "all_fp32":
                checks[f"{name}/{mode}"] = m["parity"]
    head["parity_all_pass"] = (None if args.no_cpu_baseline else
                               all(p is not None and p["pass"] for p in checks.values()))
    head["bench_seconds"] = round(time.perf_counter() - t_all, 1)
    print(json.dumps(head), flush=True)
    return 0 if head["parity_all_pass"] in (True, None) else 1


def bench_single(args, name: str) -> dict:
    """Per-step pushes of one bunch: the headline (single_bunch_fp32) or the tiny FP64 case."""
    import numpy as np
    import torch

    import paper_1802_03972_amd as rad
    from workloads import SINGLE, TINY, flatten

    big = name == "single_bunch_fp32"
    w = SINGLE if big else TINY
    if big and args.shape:
        w = w.scaled(shape=args.shape)
    om_list = None
    if big and args.omega_grid == "log":
        om_list = np.geomspace(1e-4 * w.omega_max, w.omega_max, w.n_omega)
    elif big and args.omega_grid == "blocklog":
        from workloads import block_log_omegas
        om_list = block_log_omegas(1e-4 * w.omega_max, w.omega_max, w.n_omega)
    omegas = om_list if om_list is not None else w.omegas()
    dev_id = 0
    torch.cuda.set_device(dev_id)
    stream = torch.cuda.current_stream(dev_id)

    log(f"[bench] generating {w.name}: {w.n_particles} particles x {w.n_steps} steps")
    t_gen = time.perf_counter()
    st = w.steps(workers=host_threads())
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
    if big and args.tile:
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
    torch.cuda.synchronize()
    log("[bench] warmup done")

    # ---- timed region: kernel start/stop events stamped by every 10th accumulate launch
    # (and the fold after it) on the launch stream while it runs (events on every launch
    # cost 2 % of the whole-job time; every launch does the same work)
    g.profile(10)
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
    fold_ms = prof["fold_ms"] / max(1, prof["launches"])
    if not big:
        profile = ""
    elif not g.variant:
        profile = "k_accumulate_single_bunch_fp32.md"
    else:
        profile = "k_accumulate_variants_single_bunch.md"
    roofline = alu_roofline(upd_per_launch, avg_ms, "k_accumulate", profile, tile,
                            suffix=f".v{g.variant}" if g.variant else "",
                            fold_ms_per_launch=round(fold_ms, 4),
                            fold_share_of_accumulate=round(fold_ms / avg_ms, 4),
                            whole_job_over_accumulate=round(elapsed / args.steps / (avg_ms * 1e-3 * w.n_steps), 4))

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
    cpu = parity = rounding = None
    if not args.no_cpu_baseline:
        import oracle
        set_oracle_threads()
        if big:   # first 8 steps, all particles and directions, 5 frequencies per block of 16
            ns = 8
            ks = np.unique(np.concatenate([np.arange(o, w.n_omega, 16) for o in (0, 3, 7, 11, 15)]))
        else:
            ns, ks = w.n_steps, np.arange(w.n_omega)
        samples = flatten({k: v[:ns] for k, v in st.items()}, times[:ns])
        log(f"[bench] cpu oracle: {ns} steps x {n} particles x {w.n_dir} dirs x {len(ks)} omega")
        tc = time.perf_counter()
        Iref = oracle.spectrum(samples, w.directions(), omegas[ks], w.shape, w.shape_len, w.dt)
        cpu_s = time.perf_counter() - tc
        cpu_updates = ns * n * w.n_dir * len(ks)
        cpu = cpu_entry(cpu_updates, cpu_s,
                        f"first {ns} of {w.n_steps} steps, all {n} particles, all {w.n_dir} directions, "
                        f"{len(ks)} of {w.n_omega} frequencies (offsets 0, 3, 7, 11, 15 of every block of 16)"
                        if big else "the full run", extrapolated_full_run_s=updates_per_step / (cpu_updates / cpu_s))
        g.reset(stream)
        for j in range(ns):
            g.push_step(float(times[j]), slices[j], stream)
        parity = parity_entry(g.spectrum(stream)[:, ks], Iref, ks, "same as cpu_baseline")
        log(f"[bench] parity on the sample: e_inf {parity['e_inf']:.3e}, per-frequency "
            f"{parity['per_frequency_max']:.3e}, pass {parity['pass']}")
        if big and om_list is None and not args.shape:
            rounding = rounding_entry(w, 4, 16)

    g.close()
    return {
        "metric": METRIC,
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
        "input_rounding_fp32_vs_fp64_trajectory": rounding,
    }


def bench_batched(args) -> dict:
    """12 independent bunches (log-uniform counts in [1e3, 5e5]), each with its own 8x8 x 256
    grid, 200 distinct time steps (all generated, 9.3 GB of FP32 particles resident on the
    device).  Per step: either 12 per-bunch pushes (one launch pair each) or one batched
    persistent launch over all 12 bunches (directly, or replayed from a captured graph).
    Same data, same grids.  The oracle leg accumulates, group of steps by group of steps,
    every bunch's complex sum on 3 directions x 7 frequencies and the smallest bunch's on
    every direction x every 2nd frequency."""
    import numpy as np
    import torch

    import paper_1802_03972_amd as rad
    from workloads import batched_uneven, flatten

    mb = batched_uneven()
    ws = mb.bunches()
    if args.time_steps:
        ws = [w.scaled(n_steps=args.time_steps) for w in ws]
    n_steps = ws[0].n_steps
    times = ws[0].times()
    use_oracle = not args.no_cpu_baseline
    if use_oracle:
        import oracle
        set_oracle_threads()
    ds = np.array([0, 27, 63])
    ks = np.array([0, 7, 15, 100, 143, 200, 255])
    small = int(np.argmin([w.n_particles for w in ws]))
    sel = np.arange(0, ws[small].n_omega, 2)
    S_ref = [0.0] * len(ws)
    S_small = 0.0
    cpu_s = 0.0
    log(f"[bench] batched_uneven: counts {list(mb.counts)}, {n_steps} distinct steps")
    t_gen = time.perf_counter()
    bunches = [w.bunch() for w in ws]
    slices = [[None] * n_steps for _ in ws]
    group = 25
    for j0 in range(0, n_steps, group):
        j1 = min(n_steps, j0 + group)
        for b, w in enumerate(ws):
            st = w.steps(j0, j1, bunch=bunches[b], workers=host_threads())
            d = {k: torch.from_numpy(np.ascontiguousarray(st[k], dtype=np.float32).reshape(-1)).to("cuda:0")
                 for k in rad.FIELDS}
            n = w.n_particles
            for j in range(j1 - j0):
                slices[b][j0 + j] = {k: v[j * n:(j + 1) * n] for k, v in d.items()}
            if use_oracle:
                tc = time.perf_counter()
                fl = flatten(st, times[j0:j1])
                S_ref[b] = S_ref[b] + oracle.spectrum_complex(fl, w.directions()[ds], w.omegas()[ks], w.shape,
                                                              w.shape_len)
                if b == small:
                    S_small = S_small + oracle.spectrum_complex(fl, w.directions(), w.omegas()[sel], w.shape,
                                                                w.shape_len)
                cpu_s += time.perf_counter() - tc
        torch.cuda.synchronize()
    log(f"[bench] inputs resident in HBM, oracle sample accumulated ({time.perf_counter() - t_gen:.1f} s, "
        f"oracle {cpu_s:.1f} s)")
    grids = [rad.Grid(w.directions(), w.omega0, w.domega, w.n_omega, shape=w.shape,
                      shape_len=w.shape_len, dt=w.dt) for w in ws]
    stream = torch.cuda.current_stream(0)
    batcher = rad.Batcher(max_items=len(ws))
    gbatcher = rad.Batcher(max_items=len(ws), graph=True)
    updates = sum(w.n_particles for w in ws) * n_steps * ws[0].n_dir * ws[0].n_omega

    def per_bunch():
        for g in grids:
            g.reset(stream)
        for j in range(n_steps):
            for b, g in enumerate(grids):
                g.push_step(float(times[j]), slices[b][j], stream)

    def batched(bt=batcher):
        for g in grids:
            g.reset(stream)
        for j in range(n_steps):
            bt.push([(g, float(times[j]), 1, slices[b][j]) for b, g in enumerate(grids)], stream)

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

    reps = max(1, args.batched_reps)
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
    from oracle.metrics import error_report
    agree = None
    if I_pb is not None:
        reps_pb = [error_report(a, b) for a, b in zip(I_pb, I_b)]
        agree = {"e_inf": max(r["e_inf"] for r in reps_pb),
                 "per_frequency_max": max(r["per_frequency_max"] for r in reps_pb)}
    cpu = parity = None
    if use_oracle:
        worst = None
        for b, w in enumerate(ws):
            Iref = oracle.prefactor(w.dt) * np.sum(np.abs(S_ref[b]) ** 2, axis=-1)
            p = parity_entry(I_b[b][np.ix_(ds, ks)], Iref, ks, "")
            if I_pb is not None:
                p["per_bunch_launches_per_frequency_max"] = error_report(I_pb[b][np.ix_(ds, ks)], Iref)["per_frequency_max"]
            if worst is None or p["per_frequency_max"] > worst["per_frequency_max"]:
                worst = dict(p, bunch=b)
        w = ws[small]
        Iref = oracle.prefactor(w.dt) * np.sum(np.abs(S_small) ** 2, axis=-1)
        sm = dict(parity_entry(I_b[small][:, sel], Iref, sel, ""), bunch=small)
        cu = sum(w.n_particles for w in ws) * n_steps * len(ds) * len(ks) + \
            ws[small].n_particles * n_steps * ws[small].n_dir * len(sel)
        cpu = cpu_entry(cu, cpu_s, f"every bunch, all {n_steps} steps, directions {ds.tolist()} x frequency "
                                   f"indices {ks.tolist()}; plus bunch {small} ({ws[small].n_particles} particles) "
                                   f"on all {ws[small].n_dir} directions x every 2nd frequency")
        parity = dict(worst if worst["per_frequency_max"] >= sm["per_frequency_max"] else sm)
        parity["pass"] = worst["pass"] and sm["pass"]
        parity["sample"] = ("batched direct launches; the worse of (every bunch on 3 directions x 7 frequencies) "
                            f"and (bunch {small} on every direction x every 2nd frequency)")
        log(f"[bench] batched parity: e_inf {parity['e_inf']:.3e}, per-frequency {parity['per_frequency_max']:.3e}, "
            f"pass {parity['pass']}")
    avg_ms = prof["accumulate_ms"] / max(1, prof["launches"])
    fold_ms = prof["fold_ms"] / max(1, prof["launches"])
    roofline = alu_roofline(prof["updates"] / max(1, prof["launches"]), avg_ms, "k_accumulate_batch",
                            "k_accumulate_batch_batched_uneven.md", batcher.get_tile(),
                            fold_ms_per_launch=round(fold_ms, 4))
    return {
        "metric": METRIC,
        "value": updates / t_b, "unit": "updates/s", "n_gpus": 1, "steps": reps, "warmup": 1,
        "ms_per_step": t_b * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "batched_uneven", "bunches": len(ws), "counts": list(mb.counts),
                   "time_steps": n_steps, "directions": ws[0].n_dir, "frequencies": ws[0].n_omega,
                   "distinct_generated_steps": n_steps, "updates_per_step": updates,
                   "tile": batcher.get_tile(), "per_bunch_tile": grids[0].get_tile()},
        "per_bunch_launches": {"value": updates / t_pb, "ms_per_step": t_pb * 1e3},
        "batched_graph": {"value": updates / t_g, "ms_per_step": t_g * 1e3, "bitwise_equal_to_direct": graph_equal},
        "speedup_vs_per_bunch": t_pb / t_b,
        "graph_speedup_vs_per_bunch": t_pb / t_g,
        "batched_vs_per_bunch": agree,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "parity": parity,
        "input_rounding_fp32_vs_fp64_trajectory": (
            None if args.no_cpu_baseline else rounding_entry(ws[int(np.argmax([v.n_particles for v in ws]))], 2, 16)),
    }


def bench_serving(args) -> dict:
    """8 LWFA-like bunches (counts log-uniform in [1e4, 2e5], gamma ~ U(20, 500), CIC) on
    8x16 x 512 grids.  Chunks (one step of one bunch, FP32, pinned host memory) arrive as a
    Poisson process; the serving loop admits them by HBM footprint and batches them into
    persistent launches.  Reports throughput, p50/p99 arrival-to-completion latency and
    the backlog at the stated rate, then at 0.5x and 0.8x of the measured capacity.  Each
    bunch's chunks replay its `distinct_steps` generated steps, each with its own step time
    (distinct chunks for the whole trace would need 12 GB of pinned host memory; repeating
    positions at advancing times would instead create artificial cancellations in the sum)."""
    import numpy as np
    import torch

    import paper_1802_03972_amd as rad
    from workloads import serving_bunches, poisson_trace

    sv = serving_bunches()
    ws = sv.bunches()
    kd = max(1, args.distinct_steps)
    log(f"[bench] serving: counts {list(sv.counts)}, {kd} distinct generated steps per bunch")
    host, sts = [], []
    for w in ws:
        st = w.steps(0, kd, workers=host_threads())
        sts.append(st)
        host.append([{k: torch.from_numpy(np.ascontiguousarray(st[k][j], dtype=np.float32)).pin_memory()
                      for k in rad.FIELDS} for j in range(kd)])
    grids = [rad.Grid(w.directions(), w.omega0, w.domega, w.n_omega, shape=w.shape,
                      shape_len=w.shape_len, dt=w.dt) for w in ws]
    per_chunk_updates = np.array([w.n_particles * w.n_dir * w.n_omega for w in ws], dtype=np.float64)

    server_tile = []
    served_steps = []
    kernel = []

    def run(rate, n_chunks, seed):
        arrivals, which = poisson_trace(rate, n_chunks, len(ws), seed=seed)
        srv = rad.Server(hbm_budget=4 << 30, max_batch=64, max_inflight=2, max_admitted=256, poll_us=20)
        srv.profile(True)
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
            tickets.append((srv.submit(grids[b], float(j % kd) * ws[b].dt, host[b][j % kd]), b, t0 + arrivals[i]))
            if i % 256 == 0:
                max_backlog = max(max_backlog, srv.counters()["pending"])
        srv.drain()
        cnt = srv.counters()
        lat, done, bsz = [], [], []
        for tk, b, t_arr in tickets:
            s = srv.wait(tk)
            lat.append(s["t_complete"] - t_arr)
            done.append(s["t_complete"])
            bsz.append(s["batch_size"])
        kernel.append(srv.profile_read())
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
    # FP64 CPU oracle on the smallest bunch's served steps (16 directions x frequencies 0, 7,
    # 15 of every block of 64), and its served spectrum against it (read before the
    # load-scaled runs add to the same grids)
    cpu = parity = None
    if not args.no_cpu_baseline:
        import oracle
        from workloads import flatten
        set_oracle_threads()
        b = int(np.argmin([w.n_particles for w in ws]))
        w = ws[b]
        n_b = served_steps[0][b]
        stf = {k: np.stack([sts[b][k][j % kd] for j in range(n_b)]) for k in sts[b]}
        dsel = np.arange(0, w.n_dir, max(1, w.n_dir // 16))
        osel = np.unique(np.concatenate([np.arange(o, w.n_omega, 64) for o in (0, 7, 15)] + [[w.n_omega - 1]]))
        tc = time.perf_counter()
        Iref = oracle.spectrum(flatten(stf, (np.arange(n_b) % kd).astype(np.float64) * w.dt), w.directions()[dsel],
                               w.omegas()[osel], w.shape, w.shape_len, w.dt)
        cpu_s = time.perf_counter() - tc
        cu = w.n_particles * n_b * len(dsel) * len(osel)
        cpu = cpu_entry(cu, cpu_s, f"bunch {b} ({w.n_particles} particles), its {n_b} served steps, {len(dsel)} of "
                                   f"{w.n_dir} directions x {len(osel)} of {w.n_omega} frequencies")
        parity = parity_entry(grids[b].spectrum()[np.ix_(dsel, osel)], Iref, osel,
                              "same as cpu_baseline (served spectrum of that bunch)")
        log(f"[bench] serving parity: e_inf {parity['e_inf']:.3e}, per-frequency {parity['per_frequency_max']:.3e}, "
            f"pass {parity['pass']}")
    cap = full["achieved_updates_per_s"] / per_chunk_updates.mean()
    scaled = []
    for f in (0.5, 0.8):
        r = run(f * cap, max(200, args.chunks // 4), seed=1)
        r["load_fraction"] = f
        log(f"[bench] serving at {f:.1f}x capacity ({f * cap:.0f}/s): {r}")
        scaled.append(r)
    k0 = kernel[0]
    roofline = alu_roofline(k0["updates"] / max(1, k0["launches"]), k0["accumulate_ms"] / max(1, k0["launches"]),
                            "k_accumulate_batch (graph replays: plan upload, accumulate and fold timed together)",
                            launches=int(k0["launches"]))
    return {
        "metric": METRIC,
        "value": full["achieved_updates_per_s"], "unit": "updates/s", "n_gpus": 1, "steps": args.chunks,
        "warmup": 0, "ms_per_step": full["span_s"] / args.chunks * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "serving", "bunches": len(ws), "counts": list(sv.counts),
                   "directions": ws[0].n_dir, "frequencies": ws[0].n_omega, "rate_chunks_per_s": args.rate,
                   "chunks": args.chunks, "distinct_generated_steps": kd, "batched_tile": server_tile[0]},
        "latency_ms": {"p50": full["p50_ms"], "p99": full["p99_ms"], "unit": "ms",
                       "what": "chunk arrival to completion at the stated rate (offered load above capacity: "
                               "backlog); see load_scaled for 0.5x and 0.8x of capacity"},
        "serving": full, "load_scaled": scaled,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "parity": parity,
        "input_rounding_fp32_vs_fp64_trajectory": None if args.no_cpu_baseline else rounding_entry(ws[2], 8, 16),
    }


def bench_precision(args) -> dict:
    """Precision stress: 16384 particles x 10000 steps from t0 = 1 ps, gamma ~ U(50, 1000),
    8x8 x 1024 frequencies to 1e20 rad/s, FP64 input.  Both arithmetic modes (FP64 geometry
    and phase with FP32 update; everything FP32) accumulate every step on the device; the
    FP64 oracle (the CPU-baseline leg) evaluates 4 directions x 13 frequencies (seeded and
    walked bins) of the same sum, and both device spectra are compared with it there.
    Steps are generated, pushed and handed to the oracle in groups of 250."""
    import numpy as np
    import torch

    import paper_1802_03972_amd as rad
    from workloads import PRECISION, flatten

    w = PRECISION
    n_steps = args.time_steps or w.n_steps
    group = 250
    bunch = w.bunch()
    grids = {"fp64_phase": rad.Grid(w.directions(), w.omega0, w.domega, w.n_omega, shape=w.shape,
                                    shape_len=w.shape_len, dt=w.dt, precision=rad.PHASE_F64),
             "all_fp32": rad.Grid(w.directions(), w.omega0, w.domega, w.n_omega, shape=w.shape,
                                  shape_len=w.shape_len, dt=w.dt, precision=rad.ALL_F32)}
    for g in grids.values():
        g.profile(True)
    dsel = np.array([0, 9, 36, 63])
    osel = np.array([0, 1, 7, 15, 135, 271, 392, 519, 655, 776, 903, 1015, 1023])
    use_oracle = not args.no_cpu_baseline
    S_ref = None
    cpu_s = 0.0
    if use_oracle:
        import oracle
        set_oracle_threads()
    log(f"[bench] precision_stress: {w.n_particles} particles x {n_steps} steps from t0 = {w.t0:g} s")
    t_all = time.perf_counter()
    for j0 in range(0, n_steps, group):
        j1 = min(n_steps, j0 + group)
        st = w.steps(j0, j1, bunch=bunch, workers=host_threads())
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
        if j0 % 2000 == 0:
            log(f"[bench] steps {j1}/{n_steps} ({time.perf_counter() - t_all:.0f} s)")
    out_modes = {}
    for name, g in grids.items():
        prof = g.profile_read()
        avg_ms = prof["accumulate_ms"] / max(1, prof["launches"])
        out_modes[name] = {"updates_per_s_kernel": prof["updates"] / (prof["accumulate_ms"] * 1e-3),
                           "accumulate_ms": prof["accumulate_ms"], "launches": int(prof["launches"]),
                           "roofline": alu_roofline(prof["updates"] / max(1, prof["launches"]), avg_ms, "k_accumulate",
                                                    fold_ms_per_launch=round(prof["fold_ms"] / max(1, prof["launches"]), 4))}
    cpu = None
    if use_oracle:
        Iref = oracle.prefactor(w.dt) * np.sum(np.abs(S_ref) ** 2, axis=-1)
        for name, g in grids.items():
            out_modes[name]["parity"] = parity_entry(g.spectrum()[np.ix_(dsel, osel)], Iref, osel,
                                                     "same as cpu_baseline")
            p = out_modes[name]["parity"]
            log(f"[bench] {name}: e_inf {p['e_inf']:.3e}, per-frequency {p['per_frequency_max']:.3e}, "
                f"pass {p['pass']}")
        upd = w.n_particles * n_steps * len(dsel) * len(osel)
        cpu = cpu_entry(upd, cpu_s, f"all {n_steps} steps x {w.n_particles} particles, directions {dsel.tolist()}, "
                                    f"frequency indices {osel.tolist()}",
                        extrapolated_full_run_s=w.n_particles * n_steps * w.n_dir * w.n_omega / (upd / cpu_s))
    head = out_modes["fp64_phase"]
    return {
        "metric": METRIC,
        "value": head["updates_per_s_kernel"], "unit": "updates/s", "n_gpus": 1,
        "steps": n_steps, "warmup": 0, "ms_per_step": head["accumulate_ms"] / n_steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "value_is": "accumulate-kernel rate (kernel events; multi-step pushes of 250 steps)",
        "config": {"workload": "precision_stress", "particles": w.n_particles, "time_steps": n_steps, "t0": w.t0,
                   "directions": w.n_dir, "frequencies": w.n_omega, "omega_max": w.omega_max, "input_dtype": "f64"},
        "roofline": head["roofline"],
        "parity": head.get("parity"),
        "modes": out_modes, "cpu_baseline": cpu,
    }


def bench_tracked(args) -> dict:
    """Post-processing variant: 1024 tracked particles x 100 steps of the single-bunch
    generator on its 128 x 256 grid; each step adds every particle's term into its own FP64
    time integral (read-modify-write of 32 B per particle and grid point), and the read-out
    applies weights and shape afterwards.  Each timed push (a reset, then all 100 steps in one
    launch) sums up to `Tracked.step_group()` (128) steps in registers before each
    read-modify-write of the integrals (64 B per particle and grid point per group); the
    launches are timed one by one with events and averaged.  One-step pushes (64 B per
    update, HBM-bound) are timed first, for comparison."""
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

    # for comparison, 100 one-step pushes, timed first (events bracket only the pushes; the
    # reset fill runs before the first event); the read-out below is of the last 100-step push
    def timed_one_step_pushes():
        tr.reset(stream)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for j in range(w.n_steps):
            tr.push_step(float(times[j]), slices[j], stream)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1)
    single_ms = None if args.skip_one_step else timed_one_step_pushes() / w.n_steps

    def pushes():
        tr.reset(stream)
        tr.push_steps(float(times[0]), w.n_steps, dev, stream)

    for _ in range(max(1, args.warmup)):
        pushes()
    torch.cuda.synchronize()
    # the accumulate launch of every timed push is bracketed by its own events (the reset's
    # fill runs before the first one); the launches run back to back, as in the whole job
    kev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    for ka, kb in kev:
        tr.reset(stream)
        ka.record(stream)
        tr.push_steps(float(times[0]), w.n_steps, dev, stream)
        kb.record(stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    elapsed = max(time.perf_counter() - t0, ev0.elapsed_time(ev1) * 1e-3)
    updates = n * w.n_dir * w.n_omega * w.n_steps
    value = updates * args.steps / elapsed
    launch_ms = sum(ka.elapsed_time(kb) for ka, kb in kev) / len(kev)

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
        set_oracle_threads()
        sel = np.arange(0, w.n_omega, 4)
        tc = time.perf_counter()
        Iref = oracle.spectrum(flatten(st, times), w.directions(), w.omegas()[sel], w.shape, w.shape_len, w.dt)
        cpu_s = time.perf_counter() - tc
        cu = n * w.n_steps * w.n_dir * len(sel)
        cpu = cpu_entry(cu, cpu_s, f"all {w.n_steps} steps x {n} particles x {w.n_dir} directions x every 4th of "
                                   f"{w.n_omega} frequencies",
                        extrapolated_full_run_s=n * w.n_steps * w.n_dir * w.n_omega / (cu / cpu_s))
        parity = parity_entry(I[:, sel], Iref, sel, "same as cpu_baseline")
        log(f"[bench] tracked parity: e_inf {parity['e_inf']:.3e}, per-frequency {parity['per_frequency_max']:.3e}")
    tr.close()
    log(f"[bench] tracked: {value:.4e} updates/s; 100-step push {launch_ms:.3f} ms ({hbm:.0f} GB/s, "
        f"{alu:.1f} TFLOP/s)" + ("" if single_ms is None else
                                  f"; one-step pushes {single_ms:.4f} ms each "
                                  f"({64.0 * points / (single_ms * 1e-3) / 1e9:.0f} GB/s)"))
    pv = profile_values("k_tracked_accumulate_tracked.md", tile, AUX_FILES)
    return {
        "metric": METRIC,
        "value": value, "unit": "updates/s", "n_gpus": 1, "steps": args.steps, "warmup": max(1, args.warmup),
        "ms_per_step": elapsed / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "tracked", "particles": n, "time_steps": w.n_steps, "directions": w.n_dir,
                   "frequencies": w.n_omega, "shape_at_readout": w.shape, "integrals_bytes": 32 * n * w.n_dir * w.n_omega,
                   "step_group": group},
        "roofline": ({"bound": "alu", "achieved": round(alu, 3), "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                      "frac": round(alu / FP32_PEAK_TFLOPS, 4)}
                     if alu / FP32_PEAK_TFLOPS >= hbm / HBM_PEAK_GBS else
                     {"bound": "hbm", "achieved": round(hbm, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                      "frac": round(hbm / HBM_PEAK_GBS, 4)}) | {
                     "traffic": pv.get("traffic_bytes_per_launch"),
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


def bench_fig3(args) -> dict:
    """Synthetic analogue of the paper's Fig. 3: ONE macro-particle (N = 1e5 electrons) on a
    betatron trajectory (gamma 100, 100 fs), spectrum on axis and 10 mrad off axis over
    log-spaced frequencies 1e13 .. 1e19 rad/s, with four weightings evaluated on the device:
    a single electron, point shape (all coherent, N^2), a shape so wide that g = 0 (all
    incoherent, N), and the Gaussian macro-particle shape sigma = 0.1 um (form factor,
    Eq. 12).  Each device spectrum is compared with the oracle on the same inputs; the
    coherent -> incoherent transition frequency, where (N - 1) g = 1, is measured from the
    device spectra and compared with the closed form (c / sigma) sqrt(ln(N - 1))."""
    import numpy as np
    import torch

    import paper_1802_03972_amd as rad
    from workloads import Fig3Analogue, flatten

    f = Fig3Analogue()
    w = f.workload
    N, sigma = f.electrons, f.sigma
    dirs, om = f.directions(), f.omegas()
    runs = {"single_electron": ("point", 0.0, 1.0), "coherent": ("point", 0.0, N),
            "incoherent": ("gauss", 1.0, N), "form_factor": ("gauss", sigma, N)}
    I, parity, prof = {}, {}, None
    for name, (shape, length, weight) in runs.items():
        st = f.trajectory(weight)
        parts = {k: torch.as_tensor(np.ascontiguousarray(st[k]).reshape(-1)).to("cuda:0") for k in rad.FIELDS}
        g = rad.Grid(dirs, 0.0, 0.0, 0, shape=shape, shape_len=length, dt=w.dt, omegas=om)
        g.profile(True)
        g.push_steps(w.t0, w.n_steps, parts)
        I[name] = g.spectrum()
        prof = g.profile_read()
        g.close()
        if not args.no_cpu_baseline:
            import oracle
            Iref = oracle.spectrum(flatten(st, w.times()), dirs, om, shape, length, w.dt)
            parity[name] = parity_entry(I[name], Iref, None, "full grid (2 directions x 241 frequencies)")
    I1 = I["single_electron"]
    ratio = I["form_factor"] / I1
    g_ref = np.exp(-(om * sigma / 299792458.0) ** 2)
    F2 = N + (N * N - N) * g_ref
    dev_coh = float(np.max(np.abs(I["coherent"] / I1 / N ** 2 - 1)))
    dev_inc = float(np.max(np.abs(I["incoherent"] / I1 / N - 1)))
    dev_ff = float(np.max(np.abs(ratio / F2 - 1)))
    # transition: F^2 = 2N, interpolated in log(omega) on the on-axis spectrum
    y = np.log(ratio[0] / (2 * N))
    k = int(np.argmax(y < 0))
    t = y[k - 1] / (y[k - 1] - y[k])
    om_t = float(np.exp(np.log(om[k - 1]) + t * (np.log(om[k]) - np.log(om[k - 1]))))
    om_t_ref = 299792458.0 / sigma * np.sqrt(np.log(N - 1))
    table = []
    for i in range(0, len(om), 20):
        table.append({"omega": float(om[i]), "I_single": float(I1[0, i]), "I_coherent": float(I["coherent"][0, i]),
                      "I_incoherent": float(I["incoherent"][0, i]), "I_form_factor": float(I["form_factor"][0, i])})
    log(f"[bench] fig3 analogue: transition {om_t:.4e} (closed form {om_t_ref:.4e}); deviations "
        f"coh {dev_coh:.2e} inc {dev_inc:.2e} ff {dev_ff:.2e}")
    worst = max(parity.values(), key=lambda p: p["per_frequency_max"]) if parity else None
    return {
        "metric": METRIC,
        "value": prof["updates"] / (prof["accumulate_ms"] * 1e-3), "unit": "updates/s", "n_gpus": 1,
        "steps": w.n_steps, "warmup": 0, "ms_per_step": prof["accumulate_ms"] / w.n_steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "fig3_analogue", "macro_particles": 1, "electrons": N, "gamma": 100.0,
                   "time_steps": w.n_steps, "directions": 2, "frequencies": len(om), "omega_grid": "log 1e13..1e19",
                   "shape": "gauss", "sigma": sigma},
        "transition_omega": {"measured": om_t, "closed_form": float(om_t_ref),
                             "rel_diff": float(abs(om_t / om_t_ref - 1))},
        "max_rel_dev": {"coherent_vs_N2": dev_coh, "incoherent_vs_N": dev_inc, "form_factor_vs_Eq12": dev_ff},
        "parity_per_weighting": parity or None,
        "parity": None if worst is None else dict(worst, pass_all=all(p["pass"] for p in parity.values())),
        "on_axis_table": table,
    }


if __name__ == "__main__":
    sys.exit(main())
