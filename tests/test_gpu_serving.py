"""GPU: the continuous-batching engine.  Every request's result (steps taken,
residual, E, F and force) must equal solving the same request alone with
m1_solve_steady, bitwise, whatever else is resident; admission must respect
the arena (HBM budget), and requests that can never fit are rejected."""
import numpy as np
import pytest

from paper_2606_02711_amd import inputs

pytestmark = pytest.mark.gpu

TOL = 1e-5
CHECK = 16


def problems():
    """Small uniform clouds (the serving workload's kind of request), which
    relax smoothly to a steady state."""
    out = []
    for g, n, lN, T in (("cart", 12, 19.0, 1.0e4), ("cyl", 16, 19.2, 8.0e3),
                        ("cart", 20, 19.1, 6.0e3), ("cyl", 12, 19.4, 9.0e3),
                        ("cart", 24, 19.0, 1.0e4), ("cyl", 20, 19.3, 7.0e3)):
        out.append(inputs.uniform_cloud(g, n, lN, T, 0.005))
    return out


MAX_STEPS = [20000, 20000, 20000, 20000, 37, 20000]   # one request stops at a cap off the check grid


def alone(ps, prec):
    from paper_2606_02711_amd import m1
    res = []
    for p, ms in zip(ps, MAX_STEPS):
        print(f"[gpu] alone {prec} {p['geom']} {p['nx']}x{p['ny']}", flush=True)
        g = m1.M1Grid(p, prec=prec)
        ok, steps, r = g.solve_steady(rel_tol=TOL, max_steps=ms, check_every=CHECK)
        E, Fx, Fy = [t.cpu().numpy() for t in g.state()]
        res.append(dict(ok=ok, steps=steps, r=r, E=E, Fx=Fx, Fy=Fy, f=g.force().cpu().numpy()))
        g.free()
    return res


def serve(ps, prec, batched, max_resident, arena_bytes):
    from paper_2606_02711_amd import m1
    print(f"[gpu] server {prec} batched={batched} resident<={max_resident}", flush=True)
    s = m1.M1Server(arena_bytes, prec=prec, batched=batched, max_resident=max_resident,
                    check_every=CHECK, max_bypass=2)
    ids = [s.submit(p, rel_tol=TOL, max_steps=ms) for p, ms in zip(ps, MAX_STEPS)]
    done, peak = {}, 0
    for _ in range(20000):
        busy = s.run(1)
        st = s.stats()
        peak = max(peak, st["resident"])
        assert st["arena_used"] <= arena_bytes
        for rec in s.poll():
            out = dict(rec)
            if rec["state"] in ("converged", "not_converged"):
                E, Fx, Fy = [t.cpu().numpy() for t in s.state(rec["id"])]
                out.update(E=E, Fx=Fx, Fy=Fy, f=s.force(rec["id"]).cpu().numpy())
                s.release(rec["id"])
            done[rec["id"]] = out
        if busy == 0 and len(done) == len(ids):
            break
    s.free()
    return ids, done, peak


def compare(ref, ids, done):
    for r, i in zip(ref, ids):
        d = done[i]
        assert d["state"] == ("converged" if r["ok"] else "not_converged"), (d["state"], r["ok"])
        assert d["steps"] == r["steps"] and d["residual"] == r["r"]
        for k in ("E", "Fx", "Fy", "f"):
            assert np.array_equal(d[k], r[k]), k


def test_server_fp32_batched_mix_equals_alone():
    from paper_2606_02711_amd import m1
    ps = problems()
    ref = alone(ps, "fp32")
    assert sum(r["ok"] for r in ref) >= 3 and not ref[4]["ok"]
    # an arena holding about four of the requests: admission waits for memory
    ws = [m1.workspace_bytes(m1.make_config(p, "fp32"),
                             m1.count_temperature_classes(p["fields"]["T"])) for p in ps]
    arena = 2 * max(ws) + 16384
    ids, done, peak = serve(ps, "fp32", True, 8, arena)
    assert 2 <= peak <= 5
    compare(ref, ids, done)


def test_server_fp64_plain_equals_alone():
    ps = problems()[:4]
    ref = alone(ps, "fp64")
    ids, done, peak = serve(ps, "fp64", False, 1, 1 << 30)
    assert peak == 1
    compare(ref, ids, done)


def test_server_rejects_request_larger_than_arena():
    from paper_2606_02711_amd import m1
    p = problems()[2]
    s = m1.M1Server(1 << 16, prec="fp32", max_resident=2, check_every=CHECK)
    rid = s.submit(p, rel_tol=TOL, max_steps=10)
    recs = s.poll()
    assert [r["state"] for r in recs] == ["rejected"] and recs[0]["id"] == rid
    assert s.run(1) == 0
    s.free()
