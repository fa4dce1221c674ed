"""GPU parity: the HIP library (through the C ABI) against the FP64 oracle.

Tolerances per result (E, F, force), element by element (parity.py):
  FP64 path : relative L2 1e-12 on E, F and the force (rounding-order
              differences only), with the normalised L-infinity, per-bin
              and per-cell bounds of parity.BOUNDS;
  FP32 path : relative L2 1e-5 on E and F, 1e-4 on the force (the stated
              target), with the FP32 element-wise bounds.
Every case prints its name before touching the GPU.
"""
import numpy as np
import pytest

import parity
from oracle import m1_oracle as M
from paper_2606_02711_amd import inputs

pytestmark = pytest.mark.gpu


def rel(a, b):
    nb = float(np.linalg.norm(b))
    return float(np.linalg.norm(a - b)) / nb if nb > 0 else float(np.linalg.norm(a))


def run_gpu(p, steps, prec, fp64_tau=float("inf")):
    from paper_2606_02711_amd import m1
    print(f"[gpu] {p['geom']} {p['nx']}x{p['ny']} steps={steps} prec={prec} fp64_tau={fp64_tau}",
          flush=True)
    g = m1.M1Grid(p, prec=prec, fp64_tau=fp64_tau)
    g.step(steps)
    E, Fx, Fy = [t.double().cpu().numpy() for t in g.state()]
    f = g.force().cpu().numpy()
    return g, E, Fx, Fy, f


def compare(p, steps, prec, tolE, tolF, oracle=None, fp64_tau=float("inf"), name=None,
            **bounds):
    g, E, Fx, Fy, f = run_gpu(p, steps, prec, fp64_tau)
    o = oracle if oracle is not None else M.run(p, steps=steps)
    assert g.dt == pytest.approx(o.dt, rel=1e-14)
    name = name or f"{p['geom']} {p['nx']}x{p['ny']} steps={steps} fp64_tau={fp64_tau}"
    errs = parity.check(name, prec, (E, Fx, Fy, f), (o.E, o.Fx, o.Fy, o.force),
                        l2=tolE, l2_force=tolF, **bounds)
    return g, errs


CASES = [("cart", 13, 9, 1, 1e3), ("cyl", 12, 10, 2, 1e3), ("cart", 70, 5, 3, 1e5),
         ("cyl", 4, 4, 4, 1e5), ("cyl", 67, 33, 5, 1e5)]


@pytest.mark.parametrize("geom,nx,ny,seed,hw", CASES)
def test_fp64_parity_random_heterogeneous(geom, nx, ny, seed, hw):
    p = inputs.random_small(geom, nx, ny, seed, half_width=hw, log_nHI=(-4.0, 1.0))
    compare(p, 8, "fp64", 1e-12, 1e-12)


@pytest.mark.parametrize("geom,nx,ny,seed,hw", CASES)
def test_fp32_parity_random_heterogeneous(geom, nx, ny, seed, hw):
    p = inputs.random_small(geom, nx, ny, seed, half_width=hw, log_nHI=(-4.0, 1.0))
    compare(p, 8, "fp32", 1e-5, 1e-4)


@pytest.mark.parametrize("fp64_tau", [0.0, 30.0])
def test_fp32_island_cells_parity(fp64_tau):
    """FP32 storage with double frequency-step coefficients in the cells whose
    line-centre depth reaches fp64_tau (all cells at 0)."""
    p = inputs.random_small("cyl", 67, 33, 5, half_width=1e5, log_nHI=(-4.0, 1.0))
    g, errs = compare(p, 8, "fp32", 1e-5, 1e-4, fp64_tau=fp64_tau)
    _, E0, _, _, _ = run_gpu(p, 8, "fp32")
    assert not np.array_equal(g.state()[0].cpu().numpy(), E0)   # the island path ran


def test_reflecting_box_and_line_off_cells():
    p = inputs.random_small("cart", 16, 12, 9, half_width=1e3, bc=("reflect",) * 4)
    p["fields"]["n_HI"][2:5, 3:9] = 0.0            # cells without line opacity
    compare(p, 6, "fp64", 1e-12, 1e-12)


@pytest.fixture(scope="module")
def config1_oracle():
    p = inputs.config1()
    return p, M.run(p)


def test_config1_fp64_full_run(config1_oracle):
    p, o = config1_oracle
    compare(p, p["steps"], "fp64", 1e-12, 1e-12, oracle=o)


def test_config1_fp32_full_run(config1_oracle):
    p, o = config1_oracle
    compare(p, p["steps"], "fp32", 1e-5, 1e-4, oracle=o)


@pytest.fixture(scope="module")
def config2_oracle():
    p = inputs.config2()
    print("[oracle] config 2, 2 steps", flush=True)
    return p, M.run(p, steps=2)


def test_config2_full_size_fp64(config2_oracle):
    p, o = config2_oracle
    compare(p, 2, "fp64", 1e-12, 1e-12, oracle=o)


def test_config2_full_size_fp32(config2_oracle):
    p, o = config2_oracle
    compare(p, 2, "fp32", 1e-5, 1e-4, oracle=o)


def test_linearity_bitwise_gpu():
    p = inputs.random_small("cyl", 20, 16, 11, half_width=1e3)
    _, E1, Fx1, _, f1 = run_gpu(p, 5, "fp32")
    p["fields"]["emis"] = p["fields"]["emis"] * 2.0 ** 37
    _, E2, Fx2, _, f2 = run_gpu(p, 5, "fp32")
    assert np.array_equal(E2, E1 * 2.0 ** 37)
    assert np.array_equal(Fx2, Fx1 * 2.0 ** 37)
    assert np.array_equal(f2, f1 * 2.0 ** 37)


def _alone(ps, steps, prec):
    out = []
    for p in ps:
        _, E, Fx, Fy, f = run_gpu(p, steps, prec)
        out.append((E, Fx, Fy, f))
    return out


def _assert_same(gs, ref):
    for g, (E, Fx, Fy, f) in zip(gs, ref):
        Eb, Fxb, Fyb = [t.double().cpu().numpy() for t in g.state()]
        assert np.array_equal(Eb, E) and np.array_equal(Fxb, Fx) and np.array_equal(Fyb, Fy)
        assert np.array_equal(g.force().cpu().numpy(), f)


def _mixed_problems():
    return [inputs.random_small(g, n, n + 3, s, half_width=1e3)
            for g, n, s in (("cart", 9, 1), ("cyl", 17, 2), ("cart", 33, 3), ("cyl", 70, 4))]


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_batched_equals_alone_bitwise(prec):
    """One batch of differently sized grids: the tuning steps (three per tile
    variant), then graph replays of step pairs and a single odd step."""
    from paper_2606_02711_amd import m1
    ps = _mixed_problems()
    steps = 5 * 3 + 7
    ref = _alone(ps, steps, prec)
    print(f"[gpu] batched {prec}", flush=True)
    import torch
    s = torch.cuda.Stream()              # a non-null stream: step pairs replay a graph
    gs = [m1.M1Grid(p, prec=prec, stream=s) for p in ps]
    b = m1.M1Batch(gs, use_graph=True)
    b.step(15)
    bk, ms = b.info()
    assert bk in (7, 14, 28, 49, -1) and all(t > 0 for t in ms)
    assert (ms[4] == float("inf")) == (prec == "fp64")      # fused: FP32 only
    b.step(7)
    _assert_same(gs, ref)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_batch_members_match_oracle(prec):
    """A batch of four grids of different sizes, geometries and media stepped
    together (the tuning steps over every tile variant, then graph replays of
    step pairs and an odd step): every member against the oracle run of its
    own problem, at the parity bounds of its precision."""
    from paper_2606_02711_amd import m1
    import torch
    ps = _mixed_problems()
    steps = 5 * 3 + 5
    print(f"[gpu] batch vs oracle {prec}", flush=True)
    s = torch.cuda.Stream()
    gs = [m1.M1Grid(p, prec=prec, stream=s) for p in ps]
    b = m1.M1Batch(gs, use_graph=True)
    b.step(steps)
    s.synchronize()
    for q, (p, g) in enumerate(zip(ps, gs)):
        o = M.run(p, steps=steps)
        assert g.dt == pytest.approx(o.dt, rel=1e-14)
        E, Fx, Fy = [t.double().cpu().numpy() for t in g.state()]
        parity.check(f"batch member {q} {p['geom']} {p['nx']}x{p['ny']}", prec,
                     (E, Fx, Fy, g.force().cpu().numpy()), (o.E, o.Fx, o.Fy, o.force))
    b.free()
    for g in gs:
        g.free()


def test_fused_kernel_equals_two_kernel_path_bitwise():
    """The fused kernel (frequency step inside the advection blocks) against
    the advection + frequency-step kernels, through batches with a fixed tile
    variant: identical bits after 11 steps, graph replays included."""
    from paper_2606_02711_amd import m1
    import torch
    ps = _mixed_problems()
    out = {}
    for bk in (-1, 28, 7):
        print(f"[gpu] batch with tile variant {bk}", flush=True)
        s = torch.cuda.Stream()
        gs = [m1.M1Grid(p, prec="fp32", stream=s) for p in ps]
        b = m1.M1Batch(gs, use_graph=True)
        b.set_tile(bk)
        b.step(11)
        b.free()
        out[bk] = [[t.cpu().numpy() for t in g.state()] + [g.force().cpu().numpy()] for g in gs]
    for bk in (28, 7):
        for ga, gb in zip(out[-1], out[bk]):
            for x, y in zip(ga, gb):
                assert np.array_equal(x, y), bk


def test_fused_variant_refused_with_island_cells():
    from paper_2606_02711_amd import m1
    p = _mixed_problems()[0]
    g = m1.M1Grid(p, prec="fp32", fp64_tau=30.0)
    b = m1.M1Batch([g], use_graph=False)
    with pytest.raises(m1.M1Error):
        b.set_tile(-1)
    b.free()


def test_batched_with_island_cells_equals_alone():
    from paper_2606_02711_amd import m1
    import torch
    ps = _mixed_problems()[:3]
    taus = (float("inf"), 30.0, 0.0)
    ref = []
    for p, t in zip(ps, taus):
        _, E, Fx, Fy, f = run_gpu(p, 9, "fp32", t)
        ref.append((E, Fx, Fy, f))
    print("[gpu] batched islands", flush=True)
    s = torch.cuda.Stream()
    gs = [m1.M1Grid(p, prec="fp32", fp64_tau=t, stream=s) for p, t in zip(ps, taus)]
    m1.M1Batch(gs, use_graph=True).step(9)
    _assert_same(gs, ref)


def test_batched_with_solo_steps_between():
    """A member stepped on its own between batch steps keeps its parity."""
    from paper_2606_02711_amd import m1
    ps = _mixed_problems()[:3]
    print("[gpu] batched + solo", flush=True)
    import torch
    s = torch.cuda.Stream()
    gs = [m1.M1Grid(p, prec="fp32", stream=s) for p in ps]
    b = m1.M1Batch(gs, use_graph=True)
    b.step(3)
    gs[1].step(1)
    b.step(5)
    gs[0].step(1)
    gs[2].step(1)
    b.step(1)
    gs[1].step(1)
    # steps taken: grid 0 3+5+1+1, grid 1 3+1+5+1+1, grid 2 3+5+1+1
    for g, n in zip(gs, (10, 11, 10)):
        assert g.t == pytest.approx(n * g.dt, rel=1e-12)
    ref = _alone(ps, 10, "fp32")
    _assert_same([gs[0], gs[2]], [ref[0], ref[2]])
    ref1 = _alone([ps[1]], 11, "fp32")
    _assert_same([gs[1]], ref1)


def test_solve_steady_matches_oracle():
    p = inputs.random_small("cart", 10, 10, 21, half_width=10.0, log_nHI=(-5.0, -3.0))
    p["c_tilde"] = 0.3 * inputs.C_LIGHT
    from paper_2606_02711_amd import m1
    print("[gpu] solve_steady", flush=True)
    g = m1.M1Grid(p, prec="fp64")
    ok, steps, r = g.solve_steady(rel_tol=1e-9, max_steps=20000, check_every=16)
    o = M.Oracle(p)
    ok2, steps2, r2 = o.solve_steady(rel_tol=1e-9, max_steps=20000, check_every=16)
    assert ok and ok2 and steps == steps2
    E = g.state()[0].cpu().numpy()
    assert rel(E, o.E) < 1e-10
    assert r == pytest.approx(r2, rel=1e-6)


def test_solve_steady_reports_not_converged():
    from paper_2606_02711_amd import m1
    p = inputs.random_small("cyl", 8, 8, 3, half_width=1e3)
    g = m1.M1Grid(p, prec="fp32")
    ok, steps, r = g.solve_steady(rel_tol=1e-12, max_steps=5, check_every=2)
    assert not ok and steps == 5 and r > 1e-12


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_two_bin_frequency_grid(prec, tol):
    """The smallest frequency grid (half-width 0.5 Doppler widths: 2 bins)."""
    p = inputs.random_small("cyl", 21, 13, 61, half_width=0.5, log_nHI=(-4.0, 1.0))
    g, _ = compare(p, 6, prec, tol, 10 * tol)
    assert g.nb == 2


def test_zero_emission_stays_zero():
    from paper_2606_02711_amd import m1
    p = inputs.random_small("cart", 19, 11, 62, half_width=1e3)
    p["fields"]["emis"] = np.zeros_like(p["fields"]["emis"])
    for prec in ("fp64", "fp32"):
        print(f"[gpu] zero emission {prec}", flush=True)
        g = m1.M1Grid(p, prec=prec)
        ok, steps, r = g.solve_steady(rel_tol=1e-6, max_steps=64, check_every=8)
        assert ok and steps == 8 and r == 0.0
        E, Fx, Fy = [t.cpu().numpy() for t in g.state()]
        assert not E.any() and not Fx.any() and not Fy.any()
        assert not g.force().cpu().numpy().any()


def test_dust_only_destruction_and_full_speed_of_light():
    """No line opacity anywhere, dust absorption, p_d = 1, c_tilde = c."""
    p = inputs.random_small("cyl", 23, 17, 63, half_width=1e3)
    f = p["fields"]
    f["n_HI"] = np.zeros_like(f["n_HI"])
    f["p_d"] = np.ones_like(f["p_d"])
    f["alpha_abs"] = f["alpha_abs"] + 1e-16
    f["alpha_flux"] = f["alpha_flux"] + 2e-16
    p["c_tilde"] = inputs.C_LIGHT
    compare(p, 7, "fp64", 1e-12, 1e-12)
    compare(p, 7, "fp32", 1e-5, 1e-4)


def test_batch_workload_full_size_equals_alone_bitwise():
    """The 64-grid workload the benchmark times as a batch (sides 64..512,
    6.3e8 cell-bins), FP32, in the benchmark's launch configuration: the
    15 tuning steps, a replayed step pair and an odd step, then every grid
    against the same grid stepped alone (whose path the parity tests pin to
    the oracle), bitwise, compared on the device."""
    import torch
    from paper_2606_02711_amd import m1
    ps = inputs.config3()
    print(f"[gpu] batch workload full size: {len(ps)} grids", flush=True)
    s = torch.cuda.Stream()
    gs = [m1.M1Grid(p, prec="fp32", stream=s) for p in ps]
    b = m1.M1Batch(gs, use_graph=True)
    b.step(15)
    b.step(3)
    s.synchronize()
    for q, (p, g) in enumerate(zip(ps, gs)):
        a = m1.M1Grid(p, prec="fp32")
        a.step(18)
        for x, y in zip(g.state(), a.state()):
            assert torch.equal(x, y), q
        assert torch.equal(g.force(), a.force()), q
        a.free()
    b.free()
    for g in gs:
        g.free()
    torch.cuda.empty_cache()


def test_residuals_of_many_grids_equal_one_by_one():
    """m1_residuals (one wait for all) gives m1_residual's values, including
    +inf for a grid that has not stepped."""
    import ctypes
    import torch
    from paper_2606_02711_amd import m1
    print("[gpu] m1_residuals", flush=True)
    s = torch.cuda.Stream()
    ps = [inputs.random_small(g, n, n + 2, q, half_width=1e3)
          for g, n, q in (("cart", 12, 21), ("cyl", 30, 22), ("cart", 45, 23))]
    gs = [m1.M1Grid(p, prec=pr, stream=s) for p, pr in zip(ps, ("fp32", "fp64", "fp32"))]
    gs[0].step(5)
    gs[1].step(7)
    hs = (ctypes.c_void_p * 3)(*[g.h.value for g in gs])
    out = (ctypes.c_double * 3)()
    m1.check(m1.lib().m1_residuals(hs, 3, out))
    assert list(out)[:2] == [gs[0].residual(), gs[1].residual()]
    assert out[2] == float("inf") and gs[2].residual() == float("inf")
    assert 0 < out[0] < float("inf") and 0 < out[1] < float("inf")
    for g in gs:
        g.free()
