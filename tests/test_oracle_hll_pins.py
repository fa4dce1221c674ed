"""Pins of the oracle's M1 signal speeds and of its eigenvalue-HLL flux (the
HLL flux the paper reports having tried, Section 2.1, footnote on the GLF
solver; the speeds are not printed in the paper).

The speeds are the extreme eigenvalues of the Jacobian of the face flux
(F_n, P_nx, P_ny) with respect to (E, F_x, F_y) for the Levermore closure.
They are checked against facts independent of the oracle's cubic:
  * f = 0: the isotropic system has speeds -+1/sqrt(3);
  * f along the normal: the 2x2 system in (E, F_n) gives
    lambda = [chi' +- sqrt(chi'^2 + 4 (chi - f chi'))] / 2 (chi' = d chi/d f);
  * |f| = 1 (free streaming): every speed equals f . n;
  * random f: the eigenvalues numpy finds for a finite-difference Jacobian of
    the flux built from the closure;
  * symmetry: swapping x and y, and mirroring f.
The flux itself: a closed box conserves energy with it, and in a free-streaming
beam along x the rows do not exchange energy (every y-face speed is zero for
f = (1, 0), so no wave crosses those faces), unlike with the GLF flux.
"""
import math

import numpy as np
import pytest

from oracle import m1_oracle as M
from paper_2606_02711_amd import inputs


def _chi(f):
    return (3.0 + 4.0 * f * f) / (5.0 + 2.0 * math.sqrt(4.0 - 3.0 * f * f))


def _dchi(f):
    s = math.sqrt(4.0 - 3.0 * f * f)
    return (8.0 * f * (5.0 + 2.0 * s) + (3.0 + 4.0 * f * f) * 6.0 * f / s) / (5.0 + 2.0 * s) ** 2


def test_speeds_isotropic():
    for n in (0, 1):
        lo, hi = M.signal_speeds(0.0, 0.0, n)
        assert lo == pytest.approx(-1.0 / math.sqrt(3.0), rel=1e-15)
        assert hi == pytest.approx(1.0 / math.sqrt(3.0), rel=1e-15)


@pytest.mark.parametrize("f", [0.1, 0.3, 0.5, 0.7, 0.9, 0.97])
def test_speeds_along_the_normal_are_the_1d_ones(f):
    c, d = _chi(f), _dchi(f)
    root = math.sqrt(d * d + 4.0 * (c - f * d))
    lo, hi = M.signal_speeds(f, 0.0, 0)
    assert hi == pytest.approx(0.5 * (d + root), rel=1e-13, abs=1e-15)
    assert lo == pytest.approx(0.5 * (d - root), rel=1e-13, abs=1e-15)
    lo2, hi2 = M.signal_speeds(-f, 0.0, 0)                 # mirrored flux
    assert lo2 == pytest.approx(-hi, rel=1e-14) and hi2 == pytest.approx(-lo, rel=1e-14)


@pytest.mark.parametrize("ang", [0.0, 0.3, 1.0, 1.5707963267948966, 2.5, 4.0])
def test_speeds_free_streaming_equal_f_dot_n(ang):
    fx, fy = math.cos(ang), math.sin(ang)
    for n, fn in ((0, fx), (1, fy)):
        lo, hi = M.signal_speeds(fx, fy, n)
        # a triple root: the cubic's roots carry ~ (rounding)^(1/3)
        assert lo == pytest.approx(fn, abs=2e-6) and hi == pytest.approx(fn, abs=2e-6)


def _flux_x(U):
    """Face flux along x, (F_x, P_xx, P_xy), of U = (E, F_x, F_y) with the
    oracle's closure (pinned in test_oracle_pins)."""
    E, Fx, Fy = U
    Dxx, Dyy, Dxy, Dpp = M.eddington(E, Fx, Fy)
    return np.array([Fx, Dxx * E, Dxy * E])


def test_speeds_match_eigenvalues_of_a_numerical_jacobian():
    rng = np.random.default_rng(3)
    h = 1e-6
    worst = 0.0
    for _ in range(60):
        f = 0.95 * math.sqrt(rng.uniform())
        a = rng.uniform(0, 2 * math.pi)
        fx, fy = f * math.cos(a), f * math.sin(a)
        U = np.array([1.0, fx, fy])
        J = np.zeros((3, 3))
        for k in range(3):
            d = np.zeros(3)
            d[k] = h
            J[:, k] = (_flux_x(U + d) - _flux_x(U - d)) / (2 * h)
        ev = np.sort(np.linalg.eigvals(J).real)
        lo, hi = M.signal_speeds(fx, fy, 0)
        worst = max(worst, abs(lo - ev[0]), abs(hi - ev[-1]))
        assert lo <= fx <= hi or f < 1e-12                 # f . n lies between them
    assert worst < 1e-7, worst


def test_speeds_symmetry_between_directions():
    rng = np.random.default_rng(4)
    for _ in range(20):
        fx, fy = rng.uniform(-0.7, 0.7, size=2)
        assert np.allclose(M.signal_speeds(fx, fy, 0), M.signal_speeds(fy, fx, 1),
                           rtol=1e-14, atol=1e-15)
        lo, hi = M.signal_speeds(fx, fy, 0)
        lo2, hi2 = M.signal_speeds(fx, -fy, 0)             # tangential mirror: same speeds
        assert lo2 == pytest.approx(lo, rel=1e-13, abs=1e-15)
        assert hi2 == pytest.approx(hi, rel=1e-13, abs=1e-15)


def _box(geom, flux, n=10):
    p = inputs.random_small(geom, n, n, 41, with_velocity=False, half_width=10.0,
                            log_nHI=(-4.0, 0.0), bc=("reflect",) * 4)
    p["fields"]["emis"][:] = 0.0
    p["fields"]["alpha_abs"][:] = 0.0
    p["fields"]["p_d"][:] = 0.0
    p["flux"] = flux
    return p


@pytest.mark.parametrize("geom", ["cart", "cyl"])
def test_hll_eig_closed_box_conserves_energy(geom):
    """No sources, no absorption, reflecting walls: the bin-summed energy in
    the volume is conserved by a conservative flux."""
    p = _box(geom, "hll_eig")
    o = M.Oracle(p)
    s = o.s
    rng = np.random.default_rng(7)
    shape = (s.nb, s.ny, s.nx)
    E = rng.uniform(0.1, 1.0, shape)
    ang = rng.uniform(0, 2 * math.pi, shape)
    fr = rng.uniform(0.0, 0.99, shape)
    o.set_state(E, E * fr * np.cos(ang), E * fr * np.sin(ang))
    if geom == "cyl":
        vol = (math.pi * (s.xe[1:] ** 2 - s.xe[:-1] ** 2))[None, :] * np.diff(s.ye)[:, None]
    else:
        vol = np.diff(s.xe)[None, :] * np.diff(s.ye)[:, None]
    tot = lambda: float(np.sum(vol * np.tensordot(s.grid["dnu"], o.E, axes=(0, 0))))
    e0 = tot()
    o.step(6)
    assert tot() == pytest.approx(e0, rel=1e-13)
    assert np.all(o.E >= 0) and np.all(np.hypot(o.Fx, o.Fy) <= o.E * (1 + 1e-12))


def _beam(flux, amps):
    """A beam f = (1, 0) along x (rows of amplitude amps[j], a plateau over
    columns 2..7 of a 16-column slab; vacuum at the x ends, reflecting y
    walls, no opacity); returns the oracle after 4 steps."""
    ny = len(amps)
    p = inputs.base_problem("cart", 16, ny, 0.0, 16.0, 0.0, float(ny),
                            ("vacuum", "vacuum", "reflect", "reflect"))
    sh = (ny, 16)
    z = np.zeros(sh)
    p["fields"] = dict(n_HI=z.copy(), T=np.full(sh, 1e4), u_x=z.copy(), u_y=z.copy(),
                       alpha_abs=z.copy(), alpha_flux=z.copy(), p_d=z.copy(), emis=z.copy())
    p["half_width"] = 2.0
    p["flux"] = flux
    o = M.Oracle(p, dt=0.2)
    E = np.zeros((o.s.nb, ny, 16))
    E[:, :, 2:8] = np.asarray(amps, dtype=float)[None, :, None]
    o.set_state(E, E.copy(), np.zeros_like(E))
    o.step(4)
    return o


def test_hll_eig_beam_rows_do_not_exchange():
    """Free streaming along x with f = (1, 0) in every filled cell: across a
    y-face both states have f . n = 0 and |f| = 1, so every signal speed is
    zero and no wave crosses it; the face fluxes (F_y, P_yx, P_yy) vanish as
    well.  Each row therefore evolves as a one-dimensional beam: rows of
    different amplitude give exactly what a grid of identical rows gives, and
    F_y stays zero.  The GLF flux (speeds -+1) mixes the rows."""
    amps = [1.0, 3.0, 0.5, 2.0]
    o = _beam("hll_eig", amps)
    assert not o.Fy.any()
    for j, a in enumerate(amps):
        one = _beam("hll_eig", [a] * len(amps))
        assert np.allclose(o.E[:, j, :], one.E[:, j, :], rtol=1e-14, atol=0)
        assert np.allclose(o.Fx[:, j, :], one.Fx[:, j, :], rtol=1e-14, atol=0)
    assert o.E.max() > 0.1 and o.E[:, :, 8:].max() > 0.1      # the beam moved along x
    g = _beam("glf", amps)
    one = _beam("glf", [amps[0]] * len(amps))
    assert np.max(np.abs(g.E[:, 0, :] - one.E[:, 0, :])) > 1e-3
