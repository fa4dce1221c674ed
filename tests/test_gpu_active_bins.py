"""GPU parity of active-bin advection (Section 2.2, active bins).

Bin k is advected when its energy in the volume, dnu_k sum_cells dV E_k,
exceeds active_frac times the total; the others keep their state through the
transport step.  The oracle takes the same selection in FP64.  Each case's
threshold keeps every nonzero share at least a factor e^0.005 away from it on
every step (checked on the oracle's state), so the FP32 state, ~1e-6 from the
oracle, cannot flip a bin: the advected sets are compared exactly, step by
step, and the states to the parity tolerances (relative L2 FP64 1e-12, FP32
1e-5 on E and F and 1e-4 on the force, with the element-wise bounds of
parity.py).
"""
import numpy as np
import pytest

import parity
from oracle import m1_oracle as M
from paper_2606_02711_amd import inputs

pytestmark = pytest.mark.gpu


def _volumes(o):
    s = o.s
    if s.geom == 1:
        return (np.pi * (s.xe[1:] ** 2 - s.xe[:-1] ** 2))[None, :] * np.diff(s.ye)[:, None]
    return np.diff(s.xe)[None, :] * np.diff(s.ye)[:, None]


def _oracle_steps(p, steps, margin=5e-3):
    """Oracle run recording the advected set of every step; asserts the margin."""
    o = M.Oracle(p)
    flags = []
    for _ in range(steps):
        W = o.s.grid["dnu"] * np.tensordot(o.E, _volumes(o), axes=([1, 2], [0, 1]))
        tot = W.sum()
        if tot > 0:
            sh = W[W > 0] / tot
            assert np.min(np.abs(np.log(sh / p["active_frac"]))) > margin
        o.step(1)
        flags.append(o.active.copy())
    return o, flags


CASES = [("cyl", 24, 20, 11, 1e-4), ("cart", 21, 18, 12, 1e-5), ("cyl", 70, 37, 13, 1e-3)]


@pytest.mark.parametrize("prec,tolE,tolF", [("fp64", 1e-12, 1e-12), ("fp32", 1e-5, 1e-4)])
@pytest.mark.parametrize("geom,nx,ny,seed,thr", CASES)
def test_active_bins_parity(geom, nx, ny, seed, thr, prec, tolE, tolF):
    from paper_2606_02711_amd import m1
    p = inputs.random_small(geom, nx, ny, seed, half_width=1e3, log_nHI=(-4.0, 1.0))
    p["active_frac"] = thr
    steps = 8
    o, flags = _oracle_steps(p, steps)
    print(f"[gpu] active bins {geom} {nx}x{ny} thr={thr} {prec}", flush=True)
    g = m1.M1Grid(p, prec=prec)
    assert int(g.active_bins().sum()) == 0                 # nothing selected before a step
    partial = 0
    for n in range(steps):
        g.step(1)
        fg = g.active_bins()
        assert np.array_equal(fg, flags[n]), n
        partial += 0 < int(fg.sum()) < g.nb
    assert partial >= steps - 1                           # the selection is not vacuous
    E, Fx, Fy = [t.double().cpu().numpy() for t in g.state()]
    f = g.force().cpu().numpy()
    parity.check(f"active bins {geom} {nx}x{ny} thr={thr}", prec, (E, Fx, Fy, f),
                 (o.E, o.Fx, o.Fy, o.force), l2=tolE, l2_force=tolF)
    g.free()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_tiny_threshold_equals_full_advection_bitwise(prec):
    """Emission in every cell fills every bin after the first step, so a
    threshold of 1e-300 advects every bin from then on (and none on the first
    step, whose state is empty): the selecting kernels give the same bits as
    the plain ones."""
    from paper_2606_02711_amd import m1
    p = inputs.random_small("cyl", 19, 23, 14, half_width=1e3)
    out = []
    for thr in (0.0, 1e-300):
        print(f"[gpu] threshold {thr} {prec}", flush=True)
        g = m1.M1Grid(dict(p, active_frac=thr), prec=prec)
        g.step(6)
        if thr > 0:
            assert g.active_bins().all()
        out.append([t.cpu().numpy() for t in g.state()] + [g.force().cpu().numpy()])
        g.free()
    for a, b in zip(*out):
        assert np.array_equal(a, b)


def test_active_bins_in_a_batch_equal_alone_bitwise():
    """A batch mixing grids with and without the selection (tuning over the
    five tile variants, the fused kernel included, then graph replays) gives
    the bits of each grid stepped alone."""
    from paper_2606_02711_amd import m1
    import torch
    ps = [dict(inputs.random_small(g, n, n + 3, s, half_width=1e3), active_frac=t)
          for g, n, s, t in (("cart", 9, 1, 1e-4), ("cyl", 17, 2, 0.0), ("cyl", 40, 3, 1e-5))]
    steps = 5 * 3 + 5
    ref = []
    for p in ps:
        print(f"[gpu] alone {p['geom']} {p['nx']} thr={p['active_frac']}", flush=True)
        g = m1.M1Grid(p, prec="fp32")
        g.step(steps)
        ref.append([t.cpu().numpy() for t in g.state()] + [g.force().cpu().numpy()])
        g.free()
    print("[gpu] batch with active bins", flush=True)
    s = torch.cuda.Stream()
    gs = [m1.M1Grid(p, prec="fp32", stream=s) for p in ps]
    b = m1.M1Batch(gs, use_graph=True)
    b.step(steps)
    for g, r in zip(gs, ref):
        got = [t.cpu().numpy() for t in g.state()] + [g.force().cpu().numpy()]
        for x, y in zip(got, r):
            assert np.array_equal(x, y)
    b.free()
