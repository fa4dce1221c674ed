"""GPU parity at the full 512 x 1024 size of the cylindrical workload (ionised
bubble in a log-normal neutral shell, outflow, dust, p_d = 1e-6) from a
developed state instead of E = F = 0.

Every cell and bin starts filled (inputs.filled_state: a smooth spectrum over
~7 decades, a spatial envelope, |f| spanning [0, 1] and exactly 1 in the
outer far wings), set into the oracle and the GPU alike, so ten steps reach
the whole grid: the neutral shell, whose cells have line-centre depths
tau_cell,0 ~ 1e6-1e7, the outflow's Doppler term everywhere, the dust, and
the one-pass frequency kernel the benchmark times (grids of at least 2^16
cells).  FP64 against the oracle at 1e-12 (relative L2), FP32 at 1e-5 on E
and F and 1e-4 on the force, with the element-wise bounds of parity.py, with
float frequency-step coefficients everywhere (fp64_tau = inf) and with the
double ones in cells of depth above 1e6 (fp64_tau = 1e6).
"""
import numpy as np
import pytest

import parity
from oracle import m1_oracle as M
from paper_2606_02711_amd import inputs

pytestmark = pytest.mark.gpu

STEPS = 10


def e_peak(p, dt):
    """A peak energy density of the order of the first step's emission,
    c_tilde dt max(l) / (c 1e11 Hz), so the FP32 path's internal scale (taken
    from the first step's emission) suits the state."""
    return p["c_tilde"] * dt * float(np.max(p["fields"]["emis"])) / (M.C_LIGHT * 1.0e11)


@pytest.fixture(scope="module")
def developed():
    p = inputs.config2()
    o = M.Oracle(p)
    state = inputs.filled_state(p, o.s.nb, e_peak(p, o.dt), seed=2)
    o.set_state(*state)
    print(f"[oracle] config 2 from a filled state, {STEPS} steps", flush=True)
    o.step(STEPS)
    tau0 = o.s.alpha.reshape(p["ny"], p["nx"]) * (p["x1"] - p["x0"]) / p["nx"]
    return p, state, o, tau0


@pytest.mark.parametrize("prec,fp64_tau", [("fp64", float("inf")), ("fp32", float("inf")),
                                           ("fp32", 1.0e6)])
def test_config2_full_size_from_developed_state(developed, prec, fp64_tau):
    from paper_2606_02711_amd import m1
    p, state, o, tau0 = developed
    if fp64_tau < float("inf"):
        assert int((tau0 >= fp64_tau).sum()) > 100000        # the shell takes the island path
    print(f"[gpu] config 2 developed state {prec} fp64_tau={fp64_tau}", flush=True)
    g = m1.M1Grid(p, prec=prec, fp64_tau=fp64_tau)
    assert g.dt == pytest.approx(o.dt, rel=1e-14)
    g.set_state(*state)
    g.step(STEPS)
    E, Fx, Fy = [t.double().cpu().numpy() for t in g.state()]
    f = g.force().cpu().numpy()
    g.free()
    parity.check(f"config2 developed {STEPS} steps fp64_tau={fp64_tau}", prec,
                 (E, Fx, Fy, f), (o.E, o.Fx, o.Fy, o.force))


# Config 2 over 1000 steps, the FP32 path against the FP64 path (which meets
# the oracle step by step: the test above and test_gpu_parity.py), from
# E = F = 0 (the workload as stated) and from the developed state.  A step
# rounds the FP32 state once (source_update), so the error does not grow
# with the step count.  Measured on the MI355X, relative L2 on E / F / force:
# from E = F = 0 5.7e-8 / 1.8e-7 / 4.3e-8, per cell up to 3.2e-4 at the
# radiation front (whose position differs by a fraction of a cell); from the
# developed state 3.4e-7 / 3.1e-6 / 7.4e-7.  The usual FP32 bounds apply,
# except per bin from the developed state: there the largest per-bin errors
# are in the outermost dozen bins at each end of the frequency grid, which
# hold about 2e-8 of the peak energy, up to 1.1e-3 (E) and 1.3e-3 (F) of
# their own maxima (errors fall to ~3e-4 a dozen bins in); the bound for
# that check is 2e-3.
LONG_STEPS = 1000


@pytest.mark.parametrize("start", ["empty", "developed"])
def test_config2_fp32_against_fp64_over_1000_steps(start):
    import torch
    from paper_2606_02711_amd import m1
    p = inputs.config2()
    state = None
    out = {}
    for prec in ("fp64", "fp32"):
        print(f"[gpu] config 2, {LONG_STEPS} steps from {start}, {prec}", flush=True)
        g = m1.M1Grid(p, prec=prec)
        if start == "developed":
            if state is None:
                state = inputs.filled_state(p, g.nb, e_peak(p, g.dt), seed=2)
            g.set_state(*state)
        g.step(LONG_STEPS)
        out[prec] = [t.double().cpu().numpy() for t in g.state()] + [g.force().cpu().numpy()]
        g.free()
        del g
        torch.cuda.empty_cache()
    name = f"config2 {LONG_STEPS} steps from {start} fp32 vs fp64"
    if start == "empty":
        parity.check(name, "fp32", out["fp32"], out["fp64"])
    else:
        parity.check(name, "fp32", out["fp32"], out["fp64"], bin=2e-3)
