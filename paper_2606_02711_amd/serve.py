"""Real-time request loop over the continuous-batching engine (M1Server).

Requests arrive at given times (seconds from the start); each is a
steady-state solve of a uniform cloud.  The loop submits every request whose
arrival time has passed, runs one engine round, and takes finished results
to the host (the force density), so a request's latency runs from its
arrival to its result on the host.
"""
import time

import numpy as np

from . import inputs, m1


def _cloud(prm):
    return inputs.uniform_cloud(prm["geom"], prm["n"], prm["log10_NHI"], prm["T"],
                                prm["dust_solar"])


def run_stream(requests, prec="fp32", batched=True, arena_bytes=64 << 30, max_resident=64,
               check_every=32, rel_tol=1e-6, max_steps=20000, duration=None, drain=30.0,
               max_bypass=8, log=None, sample_every=10.0):
    """requests: list of (arrival_s, params) with params as in
    inputs.config4_requests.  Stops when every request has finished, or at
    duration + drain seconds (what is still queued or resident then is the
    backlog).  Every finished request is released (failed and rejected ones
    too, so no arena block stays held).  Returns a dict of counts, latencies,
    throughput and a timeline of the queue (t, arrived, queued, resident,
    finished) every sample_every seconds."""
    duration = requests[-1][0] if duration is None else duration
    srv = m1.M1Server(arena_bytes, prec=prec, batched=batched, max_resident=max_resident,
                      check_every=check_every, max_bypass=max_bypass)
    arrival, size = {}, {}
    lat, states, steps = [], {}, []
    cell_bins = 0.0
    i = 0
    t0 = time.perf_counter()
    busy = 0
    next_log = 10.0
    next_sample = 0.0
    timeline = []
    admitted = 0
    while True:
        now = time.perf_counter() - t0
        while i < len(requests) and requests[i][0] <= now:
            a, prm = requests[i]
            meta = inputs.uniform_cloud(prm["geom"], prm["n"], prm["log10_NHI"], prm["T"],
                                        prm["dust_solar"], fields=False)
            rid = srv.submit(lambda prm=prm: _cloud(prm), rel_tol=rel_tol, max_steps=max_steps,
                             meta=meta, n_classes=1)
            arrival[rid] = a
            size[rid] = prm["n"] * prm["n"] * m1.num_bins(m1.make_config(meta, prec))
            i += 1
        if busy or i > 0:
            busy = srv.run(1)
        for rec in srv.poll():
            rid = rec["id"]
            states[rid] = rec["state"]
            admitted += rec["admit_round"] >= 0
            if rec["state"] in ("converged", "not_converged"):
                f = srv.force(rid).cpu().numpy()          # the result, on the host
                assert np.all(np.isfinite(f))
                lat.append(time.perf_counter() - t0 - arrival[rid])
                steps.append(rec["steps"])
                cell_bins += float(size[rid]) * rec["steps"]          # cells x bins x steps
            srv.release(rid)
        now = time.perf_counter() - t0
        if now >= next_sample:
            next_sample += sample_every
            st = srv.stats()
            timeline.append((round(now, 2), i, st["queued"], st["resident"], len(states)))
        if i == len(requests) and busy == 0:
            break
        if now > duration + drain:
            break
        if busy == 0 and i < len(requests):
            time.sleep(max(0.0, min(requests[i][0] - now, 0.05)))
        if log and now >= next_log:
            next_log += 10.0
            log(f"[serve] t={now:.0f}s arrived={i} done={len(states)} busy={busy}")
    elapsed = time.perf_counter() - t0
    # requests still waiting: their age so far bounds their latency from below
    waiting = [elapsed - arrival[k] for k in arrival if k not in states]
    st = srv.stats()
    timeline.append((round(elapsed, 2), i, st["queued"], st["resident"], len(states)))
    srv.free()
    lat_all = np.array(lat + waiting) if (lat or waiting) else np.array([np.nan])
    lat = np.array(lat) if lat else np.array([np.nan])
    cnt = {k: sum(1 for v in states.values() if v == k)
           for k in ("converged", "not_converged", "rejected", "failed")}
    return dict(
        prec=prec, batched=batched, arrived=i, offered=len(requests), elapsed_s=elapsed,
        arena_bytes=int(arena_bytes), admitted=admitted + st["resident"],
        completed=cnt["converged"] + cnt["not_converged"], **cnt,
        backlog=st["queued"] + st["resident"], backlog_queued=st["queued"],
        backlog_resident=st["resident"],
        p50_latency_s=float(np.percentile(lat, 50)), p99_latency_s=float(np.percentile(lat, 99)),
        p99_latency_incl_backlog_lower_bound_s=float(np.percentile(lat_all, 99)),
        solves_per_s=(cnt["converged"] + cnt["not_converged"]) / elapsed,
        mean_steps=float(np.mean(steps)) if steps else 0.0,
        cell_bin_updates_per_s=cell_bins / elapsed,
        timeline_t_arrived_queued_resident_finished=timeline)
