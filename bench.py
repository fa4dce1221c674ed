"""Throughput benchmark of the M1 Lyman-alpha step on one MI355X.

Workload: the 512 x 1024 cylindrical (R, z) cloud (ionised bubble in a
log-normal neutral shell, radial outflow, dust, p_d = 1e-6, point source on
the axis), 194 frequency bins, synthetic seeded fields, stepped from a
developed radiation field (every cell and bin filled: inputs.filled_state).
A step is one full pass of the hot path: advection + emission/absorption,
force density, and the implicit frequency step, for every cell and bin.

value      : FP32-path cell-bin updates per second (N_cells x N_nu x steps / s)
             from the developed state, state resident in HBM before the timed
             region starts; from_empty gives the same path from E = F = 0
             (steps warmup..warmup+steps and near step 1000).
fp64_value : the FP64 plain path on the same workload and state.
errors     : FP32 and FP64 GPU paths against the FP64 oracle (and FP32
             against FP64) after 10 steps from the developed state: relative
             L2 and normalised L-infinity of E, F and the force.
roofline   : the dominant kernel (advection) is bound by vector-instruction
             issue: VALU lane-instructions per second (committed counters x
             cell-bins / HIP-event duration) against the issue peak, with its
             HBM figures (algorithmic bytes: E, F_x, F_y read and written once
             per cell-bin, 24 B FP32) beside them.
cpu_baseline : the FP64 oracle on the host cores (all threads and one), on a
             bounded sample: 10 (1) steps from the same developed state.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash():
    """Hash of the hot kernels' code (comments and blank lines ignored), which
    ties committed counter figures to the source they were taken on."""
    h = hashlib.sha256()
    for f in ("m1_step_kernels.hip", "m1_device.h"):
        with open(os.path.join(ROOT, "paper_2606_02711_amd", "csrc", f)) as fh:
            for line in fh:
                code = line.split("//", 1)[0].rstrip()
                if code:
                    h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def measured_traffic(kernel, prec):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they were
    taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "traffic_counters.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except Exception:
        return None
    if d.get("kernel_source_hash") != kernel_source_hash():
        return None
    rec = d.get("kernels", {}).get(f"{kernel}:{prec}")
    return rec.get("bytes_per_launch") if rec else None


VALU_PEAK = 1024 * 16 * 2.4e9      # lane-instructions/s: 1024 SIMDs x 16 lanes x 2.4 GHz


def measured_valu(kernel, prec):
    """VALU lane-instructions per cell-bin from the committed counter run, if
    it was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "valu_counters.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except Exception:
        return None
    if d.get("kernel_source_hash") != kernel_source_hash():
        return None
    rec = d.get("kernels", {}).get(f"{kernel}:{prec}")
    return rec.get("valu_per_cell_bin") if rec else None


def copy_bandwidth():
    """Streaming copy of 1 GiB (read 1 GiB + write 1 GiB), best of 5, in GB/s:
    the practical bandwidth the kernels' traffic is compared with.  It runs
    as dst = src * 1 through torch's vectorized elementwise kernel (16-byte
    accesses per lane), which streams at the rate of a float4 copy kernel;
    dst.copy_(src) goes through the runtime's copy path, about 20 % slower."""
    import torch
    src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(2):
        torch.mul(src, 1.0, out=dst)
    best = float("inf")
    for _ in range(5):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        torch.mul(src, 1.0, out=dst)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1))
    del src, dst
    torch.cuda.empty_cache()
    return 2.0 * (1 << 30) / (best * 1e-3) / 1e9


def e_peak(p, dt):
    """Peak energy density of the developed state: of the order of the first
    step's emission, c_tilde dt max(l) / (c 1e11 Hz)."""
    import numpy as np
    return p["c_tilde"] * dt * float(np.max(p["fields"]["emis"])) / (2.99792458e10 * 1.0e11)


def _timed(g, steps):
    """Times `steps` steps of grid g (wall clock, and HIP events around each
    kernel on the grid's stream)."""
    import torch
    g.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ms = [0.0, 0.0]
    left = steps
    while left > 0:
        n = min(left, 4096)
        a, b = g.step_profiled(n)
        ms[0] += a
        ms[1] += b
        left -= n
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    cell_bins = g.ncell * g.nb
    return dict(wall=wall, ms_advect=ms[0], ms_freq=ms[1], cell_bins=cell_bins, nb=g.nb,
                ncell=g.ncell, rate=cell_bins * steps / wall,
                ms_per_step=1e3 * wall / steps)


def run_path(p, prec, steps, warmup, fp64_tau=float("inf"), state=None, late=0, final=False):
    """Times `steps` steps after `warmup` untimed ones, from `state` (physical
    E, F_x, F_y) or from E = F = 0; with late > 0 also `steps` steps starting
    at step `late`, or right after the first window if that ends later.  With
    final, res["final"] holds E, F_x, F_y and the force after the timed
    window (host arrays, taken after the timing)."""
    import torch
    from paper_2606_02711_amd import m1
    log(f"[bench] init {prec} fp64_tau={fp64_tau} start={'developed' if state else 'empty'}")
    g = m1.M1Grid(p, prec=prec, fp64_tau=fp64_tau)
    if state is not None:
        g.set_state(*state)
    g.step(warmup)
    log(f"[bench] timing {steps} steps {prec}")
    res = _timed(g, steps)
    res["dt"] = g.dt
    if late > 0:                  # a later window: from step `late`, or right after this one
        first = max(late, warmup + steps)
        g.step(first - warmup - steps)
        res["late"] = dict(_timed(g, steps), first_step=first)
    if final:
        res["final"] = [t.cpu().numpy() for t in g.state()] + [g.force().cpu().numpy()]
    del g
    torch.cuda.empty_cache()
    return res


def run_batch(ps, steps, warmup):
    """64 uneven grids: FP32 in one persistent batch, against per-grid loops
    (FP32 and FP64) that launch each grid's kernels one after another."""
    import torch
    from paper_2606_02711_amd import m1
    cell_bins = 0
    out = {}
    stream = torch.cuda.Stream()
    for mode in ("fp32_batched", "fp32_loop", "fp64_loop"):
        prec = mode.split("_")[0]
        log(f"[bench] batch workload: {mode}, {len(ps)} grids")
        gs = [m1.M1Grid(p, prec=prec, stream=stream) for p in ps]
        cell_bins = sum(g.ncell * g.nb for g in gs)
        b = m1.M1Batch(gs, use_graph=True) if mode == "fp32_batched" else None
        tune = 5 * 3                           # steps the batch spends choosing its tiles
        for _ in range(max(warmup, tune if b else 0)):
            if b:
                b.step(1)
            else:
                for g in gs:
                    g.step(1)
        stream.synchronize()
        t0 = time.perf_counter()
        if b:
            b.step(steps)
        else:
            for _ in range(steps):
                for g in gs:
                    g.step(1)
        stream.synchronize()
        wall = time.perf_counter() - t0
        out[mode] = cell_bins * steps / wall
        if b:
            out["tile_bins"], ms = b.info()
            out["tuning_ms_per_step"] = ms
            b.free()
        for g in gs:
            g.free()
        del gs
        torch.cuda.empty_cache()
    out["cell_bins_per_step"] = cell_bins
    return out


def run_active(ps, steps, warmup, thr=1e-10):
    """Active-bin advection (the paper's threshold, 1e-10 of the total energy)
    on the 64-grid batch in FP32, after `warmup` steps beyond the tuning; the
    rate counts every cell and bin (inactive bins still take the emission/
    absorption and frequency steps).  Also the fraction of cell-bins in
    advected bins at the end, and one 512x1024 grid with the threshold."""
    import torch
    from paper_2606_02711_amd import inputs, m1
    log(f"[bench] active bins: {len(ps)} grids, threshold {thr}")
    stream = torch.cuda.Stream()
    gs = [m1.M1Grid(dict(p, active_frac=thr), prec="fp32", stream=stream) for p in ps]
    cell_bins = sum(g.ncell * g.nb for g in gs)
    b = m1.M1Batch(gs, use_graph=True)
    b.step(5 * 3 + warmup)
    stream.synchronize()
    t0 = time.perf_counter()
    b.step(steps)
    stream.synchronize()
    wall = time.perf_counter() - t0
    adv = sum(int(g.active_bins().sum()) * g.ncell for g in gs)
    out = {"batch_fp32": cell_bins * steps / wall, "advected_fraction": adv / cell_bins,
           "tile_bins": b.info()[0], "steps": steps, "warmup": warmup + 15}
    b.free()
    for g in gs:
        g.free()
    del gs
    torch.cuda.empty_cache()
    log("[bench] active bins: 512x1024 grid")
    g = m1.M1Grid(dict(inputs.config2(), active_frac=thr), prec="fp32")
    g.step(warmup)
    a, c = g.step_profiled(steps)
    out["config2_fp32_ms_per_step"] = (a + c) / steps
    out["config2_advected_bins"] = int(g.active_bins().sum())
    g.free()
    torch.cuda.empty_cache()
    return out


def run_substeps(steps, L=1.0e38):
    """The 10 % substep rule on the 512x1024 workload with its source at
    L erg/s (FP32, from an empty state, while the energy density grows and the
    rule splits steps), against one substep per step."""
    import torch
    from paper_2606_02711_amd import inputs, m1
    p = inputs.config2()
    p["fields"]["emis"] = p["fields"]["emis"] * L
    out = {"luminosity_erg_s": L, "steps": steps}
    for rule in (0, 1):
        log(f"[bench] substeps: rule {rule}")
        g = m1.M1Grid(dict(p, substep_rule=rule), prec="fp32")
        a, c = g.step_profiled(steps)
        out["ms_per_step_rule" if rule else "ms_per_step_one_substep"] = (a + c) / steps
        g.free()
        torch.cuda.empty_cache()
    return out


def band_bytes(nc, nb, prec):
    """Algorithmic HBM bytes of one band-step launch: per cell and band the
    state read and written and the three tables read once (9 values); per
    cell the force (4 doubles) written and the velocity data (4 gradients,
    2 face velocities) read."""
    rs = 4 if prec == "fp32" else 8
    return nc * (9 * rs * nb + 32 + 6 * rs)


def run_bands(steps, warmup):
    """Seven broad bands (IR, optical, FUV, LW, EUV1-3) on the 512 x 1024
    H II-region workload: one band-step kernel per step (advection,
    emission/absorption, force), FP32 and FP64."""
    import torch
    from paper_2606_02711_amd import inputs, m1
    p = inputs.band_hii_region()
    nc, nb = p["nx"] * p["ny"], p["n_band"]
    out = {"workload": "cylindrical 512x1024 (R,z) H II region: bubble + log-normal shell, "
                       "outflow 30 km/s, dust 0.01 solar, star on the axis (Gaussian, sigma 3 "
                       "cells); 7 bands", "steps": steps, "unit": "cell-band updates/s"}
    for prec in ("fp32", "fp64"):
        log(f"[bench] bands {prec}")
        g = m1.BandGrid(p, prec=prec)
        g.step(warmup)
        g.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        a, _ = g.step_profiled(steps)
        wall = time.perf_counter() - t0
        ms = a / steps
        alg = band_bytes(nc, nb, prec) / (ms * 1e-3) / 1e9
        rec = {"value": nc * nb * steps / wall, "ms_per_step": 1e3 * wall / steps,
               "kernel_ms": ms, "algorithmic_bytes": band_bytes(nc, nb, prec),
               "algorithmic_GBs": alg, "frac": alg / HBM_PEAK_GBS}
        t = measured_traffic("band_step", prec)
        if t is not None:
            rec.update(traffic_bytes=t, traffic_GBs=t / (ms * 1e-3) / 1e9)
        v = measured_valu("band_step", prec)
        if v is not None:
            rec.update(valu_per_cell_band=v,
                       valu_issue_frac=v * nc * nb / (ms * 1e-3) / VALU_PEAK)
        out[prec] = rec
        g.free()
        torch.cuda.empty_cache()
    return out


def run_large(steps, warmup):
    """4096 x 8192 cylindrical cloud in FP32, the force density copied out
    (to device arrays) after every step."""
    import torch
    from paper_2606_02711_amd import inputs, m1
    log("[bench] large grid: building inputs")
    p = inputs.config5()
    g = m1.M1Grid(p, prec="fp32")
    del p
    force = torch.empty((4, g.ny, g.nx), dtype=torch.float64, device="cuda")
    fp = [force[q].data_ptr() for q in range(4)]
    L = m1.lib()
    for _ in range(warmup):
        g.step(1)
        m1.check(L.m1_force(g.h, *fp))
    g.sync()
    log(f"[bench] large grid: timing {steps} steps")
    t0 = time.perf_counter()
    ms = [0.0, 0.0]
    for _ in range(steps):
        a, b = g.step_profiled(1)
        ms[0] += a
        ms[1] += b
        m1.check(L.m1_force(g.h, *fp))
    g.sync()
    wall = time.perf_counter() - t0
    cb = g.ncell * g.nb
    out = {"workload": "cylindrical 4096x8192 (R,z) turbulent log-normal cloud (sigma_ln 1.5), "
                       "HII region, velocities up to 50 km/s, dust 0.01 solar, p_d 1e-7, 16 ring "
                       "sources; FP32; force density output every step",
           "steps": steps, "cell_bins": cb, "value": cb * steps / wall, "unit": "cell-bin updates/s",
           "ms_per_step": 1e3 * wall / steps,
           "kernel_ms_per_step": {"advect_source": ms[0] / steps, "freq_step": ms[1] / steps},
           "algorithmic_GBps": 24.0 * cb * steps / wall / 1e9,
           "hbm_frac_algorithmic": 24.0 * cb * steps / wall / 1e9 / HBM_PEAK_GBS}
    g.free()
    del g, force
    torch.cuda.empty_cache()
    return out


def arena_bytes(gb):
    """The serving arena: gb GiB, or with gb <= 0 the device's free HBM less
    4 GiB (so admission is bounded by the memory the GPU really has)."""
    import torch
    if gb > 0:
        return int(gb) << 30
    free, _ = torch.cuda.mem_get_info()
    return int(free - (4 << 30)) & ~255


def run_serving(args):
    """Poisson stream of steady-state solves (uniform clouds, log N_HI 19..23,
    T 100..1e4 K, dust 0..0.01 solar) through the continuous-batching engine
    in FP32, and through the FP64 plain path (one request at a time)."""
    from paper_2606_02711_amd import inputs, serve
    reqs = inputs.config4_requests(rate=args.serve_rate, duration=args.serve_seconds,
                                   lo=args.serve_lo, hi=args.serve_hi)
    out = {"workload": f"Poisson {args.serve_rate} req/s for {args.serve_seconds} s, sides "
                       f"log-uniform {args.serve_lo}..{args.serve_hi}, uniform clouds log N_HI "
                       f"19..23, T 100..1e4 K, dust 0..0.01 solar; steady solve to relative "
                       f"residual 1e-6, at most {args.serve_max_steps} steps per request",
           "requests": len(reqs)}
    for name, prec, batched, slots in (("fp32_batched", "fp32", True, args.serve_slots),
                                       ("fp64_plain", "fp64", False, 1)):
        import torch
        torch.cuda.empty_cache()               # the previous run's arena back to the device
        arena = arena_bytes(args.serve_arena_gb)
        log(f"[bench] serving {name}: {len(reqs)} requests, arena {arena / 2**30:.1f} GiB")
        r = serve.run_stream(reqs, prec=prec, batched=batched, arena_bytes=arena,
                             max_resident=slots, check_every=32, rel_tol=1e-6,
                             max_steps=args.serve_max_steps, duration=args.serve_seconds,
                             drain=args.serve_drain, log=log)
        out[name] = r
    return out


def cpu_model():
    """Host CPU model and logical CPU count (from /proc/cpuinfo)."""
    model, n = "unknown", 0
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    n += 1
                    if model == "unknown":
                        model = line.split(":", 1)[1].strip()
    except OSError:
        pass
    return model, n


def gpu_after(p, prec, state, steps):
    """E, F_x, F_y and the force of the GPU path after `steps` steps from
    `state`, as host arrays."""
    import torch
    from paper_2606_02711_amd import m1
    g = m1.M1Grid(p, prec=prec)
    g.set_state(*state)
    g.step(steps)
    out = [t.cpu().numpy() for t in g.state()] + [g.force().cpu().numpy()]
    g.free()
    del g
    torch.cuda.empty_cache()
    return out


def error_figures(a, b):
    """Relative L2 and normalised L-infinity of E, F (vector) and the force
    (total, vector) of result a against reference b."""
    import numpy as np
    def pair(x, y):
        d = float(np.sqrt(sum(np.sum((u - v) ** 2) for u, v in zip(x, y))))
        n = float(np.sqrt(sum(np.sum(v ** 2) for v in y)))
        dm = float(np.max(np.sqrt(sum((u - v) ** 2 for u, v in zip(x, y)))))
        nm = float(np.max(np.sqrt(sum(v ** 2 for v in y))))
        return {"rel_l2": d / n if n > 0 else d, "linf": dm / nm if nm > 0 else dm}
    return {"E": pair([a[0]], [b[0]]), "F": pair(a[1:3], b[1:3]),
            "force": pair([a[3][0], a[3][1]], [b[3][0], b[3][1]])}


def cpu_baseline(p, state, steps=10, steps_1t=1):
    """The FP64 oracle on the host: `steps` steps from `state` with every
    thread (the reference of the error figures) and `steps_1t` with one."""
    from oracle import m1_oracle
    log(f"[bench] oracle sample: {steps} steps of the full workload on the host")
    o = m1_oracle.Oracle(p)
    o.set_state(*state)
    t0 = time.perf_counter()
    o.step(steps)
    dt = time.perf_counter() - t0
    ref = [o.E.copy(), o.Fx.copy(), o.Fy.copy(), o.force.copy()]
    n = o.s.nx * o.s.ny * o.s.nb * steps
    threads = m1_oracle.num_threads()
    log(f"[bench] oracle sample: {steps_1t} step(s) on one thread")
    o.set_state(*state)
    m1_oracle.set_num_threads(1)
    t1 = time.perf_counter()
    o.step(steps_1t)
    dt1 = time.perf_counter() - t1
    m1_oracle.set_num_threads(threads)
    n1 = o.s.nx * o.s.ny * o.s.nb * steps_1t
    model, ncpu = cpu_model()
    out = {"value": n / dt, "unit": "cell-bin updates/s", "cores": threads, "kind": "oracle",
           "sample": f"{steps} steps of the 512x1024 cylindrical workload from the developed "
                     f"state, all {o.s.nb} bins ({n:.3e} cell-bin updates, {dt:.1f} s, "
                     f"{threads} threads); one thread: {steps_1t} step ({n1:.3e}, {dt1:.1f} s)",
           "value_1_thread": n1 / dt1,
           "ns_per_cell_bin_per_core": 1e9 * dt1 / n1,
           "cpu_model": model, "host_logical_cpus": ncpu,
           "build": "gcc -O3, no fast-math, no FMA contraction"}
    del o
    return out, ref


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--batch-steps", type=int, default=500,
                    help="steps of the 64-grid batch workload (0 skips it)")
    ap.add_argument("--active-steps", type=int, default=200,
                    help="timed steps of the active-bin workload (0 skips it)")
    ap.add_argument("--substep-steps", type=int, default=200,
                    help="steps of the substep-rule workload (0 skips it)")
    ap.add_argument("--large-steps", type=int, default=20,
                    help="timed steps of the 4096 x 8192 grid (0 skips it)")
    ap.add_argument("--band-steps", type=int, default=500,
                    help="steps of the seven-band workload (0: skip)")
    ap.add_argument("--band-only", action="store_true",
                    help="only the seven-band workload")
    ap.add_argument("--serve-seconds", type=float, default=30.0,
                    help="length of the request stream (0 skips the serving workload)")
    ap.add_argument("--serve-rate", type=float, default=0.3, help="requests per second")
    ap.add_argument("--serve-lo", type=int, default=128)
    ap.add_argument("--serve-hi", type=int, default=160)
    ap.add_argument("--serve-slots", type=int, default=32, help="resident requests at most")
    ap.add_argument("--serve-arena-gb", type=int, default=0,
                    help="serving arena in GiB (0: the device's free HBM less 4 GiB)")
    ap.add_argument("--serve-max-steps", type=int, default=200000)
    ap.add_argument("--serve-drain", type=float, default=30.0,
                    help="seconds after the stream ends before the backlog is counted")
    ap.add_argument("--serve-only", action="store_true")
    ap.add_argument("--serve-config4", action="store_true",
                    help="only the serving workload as specified: 50 req/s for 120 s, sides "
                         "128..2048 (far beyond one GPU's capacity; reports the backlog)")
    ap.add_argument("--active-only", action="store_true",
                    help="run only the active-bin workload")
    ap.add_argument("--batch-only", action="store_true",
                    help="run only the 64-grid batch workload (profiling)")
    ap.add_argument("--profile", action="store_true",
                    help="only the FP32 (and, without --no-fp64, FP64) path on the 512 x 1024 "
                         "workload from the developed state (for counter runs)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run a plain 1 GiB device copy (counter calibration)")
    ap.add_argument("--fp64-tau", type=float, default=float("inf"),
                    help="FP32 path: cells above this line-centre depth use a double frequency step")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              f"(asked for --gpus {args.gpus}); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    from paper_2606_02711_amd import inputs
    if args.calibrate_copy:
        # known traffic: reads 2^30 B and writes 2^30 B per copy
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("[bench] copy calibration: 3 copies of 1 GiB")
        del src, dst
    if args.serve_config4:
        args.serve_rate, args.serve_seconds, args.serve_lo, args.serve_hi = 50.0, 120.0, 128, 2048
        print(json.dumps({"serving_config4": run_serving(args)}), flush=True)
        return
    if args.serve_only:
        print(json.dumps({"serving": run_serving(args)}), flush=True)
        return
    if args.batch_only:
        rb = run_batch(inputs.config3(), args.batch_steps, args.warmup)
        print(json.dumps({"batch_64_grids": rb}), flush=True)
        return
    if args.band_only:
        print(json.dumps({"bands": run_bands(args.band_steps, args.warmup)}), flush=True)
        return
    if args.active_only:
        print(json.dumps({"active_bins": run_active(inputs.config3(), args.active_steps, 100),
                          "substeps": run_substeps(args.substep_steps)}), flush=True)
        return
    if args.profile:
        from paper_2606_02711_amd import m1
        p = inputs.config2()
        g = m1.M1Grid(p, prec="fp32")          # its time step sets the state's scale
        state = inputs.filled_state(p, g.nb, e_peak(p, g.dt), seed=2)
        g.free()
        del g
        out = {"profile": {"fp32": run_path(p, "fp32", args.steps, args.warmup, state=state)}}
        if not args.no_fp64:
            out["profile"]["fp64"] = run_path(p, "fp64", args.steps, args.warmup, state=state)
        print(json.dumps(out), flush=True)
        return
    copy_gbs = copy_bandwidth()
    log(f"[bench] streaming copy: {copy_gbs:.0f} GB/s")
    p = inputs.config2()
    # FP32 from E = F = 0: the steps after the warm-up, and near step 1000
    r32e = run_path(p, "fp32", args.steps, args.warmup, args.fp64_tau, late=1000)
    # the developed state every timed and compared run below starts from
    state = inputs.filled_state(p, r32e["nb"], e_peak(p, r32e["dt"]), seed=2)
    r32 = run_path(p, "fp32", args.steps, args.warmup, args.fp64_tau, state=state,
                   final=not args.no_fp64)
    r64 = None if args.no_fp64 else run_path(p, "fp64", args.steps, args.warmup, state=state,
                                             final=True)
    # FP32 against FP64 after the whole timed window (both from the developed
    # state; the FP64 path meets the oracle step by step, see "errors")
    long_err = None
    if r64 is not None:
        long_err = {"steps": args.warmup + args.steps, "start": "developed state",
                    "fp32_vs_fp64": error_figures(r32.pop("final"), r64.pop("final"))}
    dom = "advect_source" if r32["ms_advect"] >= r32["ms_freq"] else "freq_step"
    dom_ms = (r32["ms_advect"] if dom == "advect_source" else r32["ms_freq"]) / args.steps
    alg_bytes = 24.0 * r32["cell_bins"]                    # per launch, FP32
    achieved = alg_bytes / (dom_ms * 1e-3) / 1e9
    traffic = measured_traffic(dom, "fp32")
    valu = measured_valu(dom, "fp32")
    if valu is not None:
        rate = valu * r32["cell_bins"] / (dom_ms * 1e-3)
        roof = {"bound": "alu", "kernel": dom, "achieved": rate, "peak": VALU_PEAK,
                "unit": "VALU lane-instr/s", "frac": rate / VALU_PEAK,
                "valu_per_cell_bin": valu, "traffic": traffic,
                "hbm_achieved": achieved, "hbm_peak": HBM_PEAK_GBS, "hbm_unit": "GB/s",
                "hbm_frac": achieved / HBM_PEAK_GBS, "copy_GBs": copy_gbs,
                "hbm_frac_of_copy": achieved / copy_gbs}
    else:                       # no counters for this source: the HBM figures alone
        roof = {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                "copy_GBs": copy_gbs, "frac_of_copy": achieved / copy_gbs}
    out = {
        "metric": "M1 Ly\u03b1 cell-updates/s (FP32 batched vs FP64 plain), %HBM roofline, p99 solve latency",
        "value": r32["rate"],
        "unit": "cell-bin updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * r32["wall"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "cylindrical 512x1024 (R,z) bubble + log-normal k^-2 shell, "
                               "radial outflow 30 km/s, dust 0.01 solar, p_d 1e-6, axis point "
                               "source; 194 frequency bins; FP32 path; stepped from a developed "
                               "radiation field (every cell and bin filled)",
                   "nx": 512, "ny": 1024, "n_nu": r32["nb"],
                   "spatial_cell_updates_per_s": r32["rate"] / r32["nb"]},
        "kernel_ms_per_step": {"advect_source": r32["ms_advect"] / args.steps,
                               "freq_step": r32["ms_freq"] / args.steps},
        "roofline": roof,
        "from_empty": {
            "first_timed_step": args.warmup, "value": r32e["rate"],
            "ms_per_step": r32e["ms_per_step"],
            "kernel_ms_per_step": {"advect_source": r32e["ms_advect"] / args.steps,
                                   "freq_step": r32e["ms_freq"] / args.steps},
            "late_window": {"first_timed_step": r32e["late"]["first_step"],
                               "value": r32e["late"]["rate"],
                               "ms_per_step": r32e["late"]["ms_per_step"],
                               "kernel_ms_per_step": {
                                   "advect_source": r32e["late"]["ms_advect"] / args.steps,
                                   "freq_step": r32e["late"]["ms_freq"] / args.steps}}},
    }
    # both kernels: algorithmic and (when the committed counters match the
    # source) measured HBM rates, against the nominal peak and the device copy
    kern = {}
    for name, ms_tot in (("advect_source", r32["ms_advect"]), ("freq_step", r32["ms_freq"])):
        ms = ms_tot / args.steps
        alg = alg_bytes / (ms * 1e-3) / 1e9
        rec = {"ms": ms, "algorithmic_GBs": alg, "algorithmic_frac": alg / HBM_PEAK_GBS}
        t = measured_traffic(name, "fp32")
        if t is not None:
            meas = t / (ms * 1e-3) / 1e9
            rec.update(traffic_bytes=t, traffic_GBs=meas, traffic_frac=meas / HBM_PEAK_GBS,
                       traffic_frac_of_copy=meas / copy_gbs)
        v = measured_valu(name, "fp32")
        if v is not None:
            rec.update(valu_per_cell_bin=v,
                       valu_issue_frac=v * r32["cell_bins"] / (ms * 1e-3) / VALU_PEAK)
        kern[name] = rec
    out["kernels_fp32"] = kern
    if r64 is not None:
        out["fp64_value"] = r64["rate"]
        out["fp64_ms_per_step"] = 1e3 * r64["wall"] / args.steps
        out["fp64_kernel_ms_per_step"] = {"advect_source": r64["ms_advect"] / args.steps,
                                          "freq_step": r64["ms_freq"] / args.steps}
    # errors after 10 steps from the developed state, and the oracle's timing
    log("[bench] error figures: FP32 and FP64 paths, 10 steps from the developed state")
    g32 = gpu_after(p, "fp32", state, 10)
    g64 = gpu_after(p, "fp64", state, 10)
    out["errors"] = {"steps": 10, "start": "developed state", "fp32_vs_fp64": error_figures(g32, g64)}
    if long_err is not None:
        out["errors"]["after_timed_window"] = long_err
    if not args.no_cpu:
        out["cpu_baseline"], ref = cpu_baseline(p, state, 10, 1)
        out["errors"]["fp32_vs_oracle"] = error_figures(g32, ref)
        out["errors"]["fp64_vs_oracle"] = error_figures(g64, ref)
        del ref
    del g32, g64, state
    if args.batch_steps > 0:
        rb = run_batch(inputs.config3(), args.batch_steps, args.warmup)
        out["batch_64_grids"] = {
            "workload": "64 uniform clouds, sides log-uniform 64..512, half Cartesian, half "
                        "cylindrical, log N_HI 19..23, T 100..1e4 K, dust 0..0.01 solar",
            "steps": args.batch_steps, "cell_bins_per_step": rb["cell_bins_per_step"],
            "fp32_batched": rb["fp32_batched"], "fp32_loop": rb["fp32_loop"],
            "fp64_loop": rb["fp64_loop"], "unit": "cell-bin updates/s",
            "batched_vs_fp64_loop": rb["fp32_batched"] / rb["fp64_loop"],
            "tile_bins": rb["tile_bins"], "tuning_ms_per_step": rb["tuning_ms_per_step"]}
    if args.active_steps > 0:
        out["active_bins"] = run_active(inputs.config3(), args.active_steps, 100)
    if args.substep_steps > 0:
        out["substeps"] = run_substeps(args.substep_steps)
    if args.large_steps > 0:
        out["large_grid"] = run_large(args.large_steps, 2)
    if args.band_steps > 0:
        out["bands"] = run_bands(args.band_steps, args.warmup)
    if args.serve_seconds > 0:
        out["serving"] = run_serving(args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
