"""Pins of the oracle's broad-band transport (Section 2.5; Appendix E).

The band step is the line step's advection and emission/absorption with
per-band opacities and no frequency step.  Each test compares the oracle with
something other than itself: the closed-form relaxation of a uniform closed
box (geometric series to E* = L/(c kappa_abs)), the closed-form update of the
interior of a uniform beam (which tells kappa_abs from kappa_F and fixes the
force sum_B kappa_F F_B), the energy a step in E moves across one face
(the corrected GLF flux with the blend eps(tau) from kappa_F), exact energy
conservation in a closed box, and equivariance under a permutation of the
bands.
"""
import numpy as np
import pytest

from oracle import m1_oracle as M
from paper_2606_02711_amd import inputs

C = M.C_LIGHT


def band_problem(geom, nx, ny, dx, bc, ka, kf, em, ux=0.0, uy=0.0, c_frac=0.01):
    """Uniform per-band tables ka, kf, em (sequences of n_band values)."""
    y0 = -0.5 * ny * dx if geom == "cyl" else 0.0
    p = inputs.base_problem(geom, nx, ny, 0.0, nx * dx, y0, y0 + ny * dx, bc, c_tilde_frac=c_frac)
    nb = len(ka)
    p = inputs.band_base(p, nb)
    sh = (nb, ny, nx)
    tab = lambda v: np.broadcast_to(np.asarray(v, dtype=np.float64)[:, None, None], sh).copy()
    p["fields"] = dict(u_x=np.full((ny, nx), float(ux)), u_y=np.full((ny, nx), float(uy)),
                       kappa_abs=tab(ka), kappa_flux=tab(kf), emis=tab(em))
    return p


def volumes(p):
    xe, ye = inputs.edges(p)
    if p["geom"] == "cyl":
        return (np.pi * (xe[1:] ** 2 - xe[:-1] ** 2))[None, :] * np.diff(ye)[:, None]
    return np.diff(xe)[None, :] * np.diff(ye)[:, None]


@pytest.mark.parametrize("geom", ["cart", "cyl"])
def test_uniform_closed_box_relaxes_geometrically(geom):
    """Closed reflecting box, uniform isotropic state: transport is exactly
    balanced (in (R, z) the hoop pressure cancels the divergence of the
    pressure), so each step is E <- (E + c dt L/c)/(1 + c dt kappa_abs):
    E_n = E*(1 - r^n), r = 1/(1 + c dt kappa_abs), E* = L/(c kappa_abs), F = 0."""
    dx = 1.0e16
    ka = [1.0e-17, 3.0e-16, 2.0e-15]
    kf = [5.0e-17, 9.0e-16, 2.0e-15]        # the flux opacity must not enter E
    em = [1.0e-20, 4.0e-22, 7.0e-21]
    p = band_problem(geom, 12, 10, dx, ("reflect",) * 4, ka, kf, em)
    o = M.BandOracle(p)
    n = 5
    o.step(n)
    ctdt = p["c_tilde"] * o.dt
    for b in range(3):
        Es = em[b] / (C * ka[b])
        r = 1.0 / (1.0 + ctdt * ka[b])
        want = Es * (1.0 - r ** n)
        np.testing.assert_allclose(o.E[b], want, rtol=1e-12, atol=0)
    if geom == "cart":
        assert np.all(o.Fx == 0) and np.all(o.Fy == 0) and np.all(o.force == 0)
    else:       # the cancellation holds up to the rounding of the two terms
        assert np.abs(o.Fx).max() <= 1e-14 * o.E.max() and np.all(o.Fy == 0)


def test_uniform_beam_interior_closed_form():
    """Uniform state E0, F = (0.5 E0, 0) in a Cartesian box: at least two cells
    away from the x walls every face carries the same flux, so one step gives
    E = (E0 + c dt L/c)/(1 + c dt kappa_abs), F_x = F0/(1 + c dt kappa_F) and
    force f_x = sum_B kappa_F,B F_x,B (gas share 0)."""
    dx = 1.0e16
    ka = [2.0e-17, 1.0e-16]
    kf = [8.0e-17, 3.0e-16]
    em = [3.0e-21, 0.0]
    nx, ny = 16, 6
    p = band_problem("cart", nx, ny, dx, ("reflect",) * 4, ka, kf, em)
    o = M.BandOracle(p)
    E0 = np.array([2.0e-8, 5.0e-9])
    sh = (2, ny, nx)
    E = np.broadcast_to(E0[:, None, None], sh).copy()
    o.set_state(E, 0.5 * E, np.zeros(sh))
    o.step(1)
    ctdt = p["c_tilde"] * o.dt
    inner = slice(2, nx - 2)
    fx = 0.0
    for b in range(2):
        wantE = (E0[b] + ctdt * em[b] / C) / (1.0 + ctdt * ka[b])
        wantF = 0.5 * E0[b] / (1.0 + ctdt * kf[b])
        np.testing.assert_allclose(o.E[b][:, inner], wantE, rtol=1e-13)
        np.testing.assert_allclose(o.Fx[b][:, inner], wantF, rtol=1e-13)
        assert np.all(o.Fy[b] == 0)
        fx += kf[b] * wantF
    np.testing.assert_allclose(o.force[0][:, inner], fx, rtol=1e-13)
    assert np.all(o.force[1] == 0) and np.all(o.force[2:] == 0)
    # the walls do change the two outer columns (the test above is not vacuous)
    assert not np.allclose(o.E[0][:, 0], o.E[0][:, nx // 2], rtol=1e-6, atol=0)


def test_step_exchange_follows_corrected_glf_flux():
    """A step in E (F = 0) across one face of a Cartesian row: MinMod gives
    zero slopes, so the face sees the cell values and the corrected GLF
    energy flux is -(E2 - E1) [eps/2 + (1 - eps)/(3 tau)] with
    eps = (0.2 + tau)/(0.2 + tau + tau^2) and tau = kappa_F dx (Section 2.1,
    the flux with the asymptotic diffusion fix); no other face carries
    energy.  Two bands, one thin and one thick in kappa_F, no absorption: a
    blend formed from any other opacity would move different energy."""
    dx, nx, ny = 1.0e16, 10, 4
    taus = [0.1, 30.0]
    kf = [t / dx for t in taus]
    p = band_problem("cart", nx, ny, dx, ("reflect",) * 4, [0.0, 0.0], kf, [0.0, 0.0])
    o = M.BandOracle(p)
    E1, E2, m = 3.0e-9, 1.0e-9, nx // 2
    E = np.full((2, ny, nx), E1)
    E[:, :, m:] = E2
    o.set_state(E, np.zeros_like(E), np.zeros_like(E))
    o.step(1)
    k = p["c_tilde"] * o.dt / dx
    for b, t in enumerate(taus):
        eps = (0.2 + t) / (0.2 + t + t * t)
        moved = k * (E1 - E2) * (0.5 * eps + (1.0 - eps) / (3.0 * t))
        np.testing.assert_allclose(o.E[b][:, m - 1], E1 - moved, rtol=1e-13)
        np.testing.assert_allclose(o.E[b][:, m], E2 + moved, rtol=1e-13)
        others = [i for i in range(nx) if i not in (m - 1, m)]
        np.testing.assert_array_equal(o.E[b][:, others], E[b][:, others])
    # the thick band moves far less energy than the thin one
    assert (E1 - o.E[1][0, m - 1]) < 0.2 * (E1 - o.E[0][0, m - 1])


@pytest.mark.parametrize("geom", ["cart", "cyl"])
def test_closed_box_conserves_energy(geom):
    """No absorption or emission, reflecting walls, gas at rest: the update
    is conservative, so sum_cells dV E of every band stays the same, whatever
    the (random) flux opacities that set the diffusion blend."""
    rng = np.random.default_rng(5)
    nx, ny, nb, dx = 20, 14, 3, 1.0e16
    p = band_problem(geom, nx, ny, dx, ("reflect",) * 4, [0.0] * nb, [0.0] * nb, [0.0] * nb)
    p["fields"]["kappa_flux"] = 10.0 ** rng.uniform(-3, 2, size=(nb, ny, nx)) / dx
    o = M.BandOracle(p)
    E = 1.0 + 0.5 * rng.uniform(size=(nb, ny, nx))
    Fx = 0.2 * E * rng.uniform(-1, 1, size=E.shape)
    Fy = 0.2 * E * rng.uniform(-1, 1, size=E.shape)
    o.set_state(E, Fx, Fy)
    V = volumes(p)
    before = (o.E * V).sum(axis=(1, 2))
    o.step(10)
    assert np.all(o.E > 0)                       # the clamp never acted
    after = (o.E * V).sum(axis=(1, 2))
    np.testing.assert_allclose(after, before, rtol=1e-13)
    # and the state did move
    assert np.abs(o.E - E).max() > 1e-3


def test_band_permutation_equivariance():
    """Bands are independent: permuting the band tables permutes the state
    (bitwise) and leaves the force unchanged up to the order of its sum."""
    p = inputs.band_random_small("cyl", 12, 10, seed=3, n_band=4)
    perm = [2, 0, 3, 1]
    q = dict(p)
    q["fields"] = dict(p["fields"])
    for k in ("kappa_abs", "kappa_flux", "emis"):
        q["fields"][k] = p["fields"][k][perm].copy()
    a = M.BandOracle(p).step(6)
    b = M.BandOracle(q).step(6)
    assert np.array_equal(a.E[perm], b.E)
    assert np.array_equal(a.Fx[perm], b.Fx)
    assert np.array_equal(a.Fy[perm], b.Fy)
    np.testing.assert_allclose(a.force, b.force, rtol=1e-13, atol=1e-300)
    assert np.abs(a.E).max() > 0 and np.abs(a.force).max() > 0


def test_band_refuses_runtime_controls():
    p = inputs.band_random_small("cart", 6, 6, seed=1, n_band=2)
    o = M.BandOracle(p)
    o.P.substep_rule = 1
    with pytest.raises(ValueError):
        o.step(1)


@pytest.mark.parametrize("geom,factor", [("cart", 8.0 / 3.0), ("cyl", 4.0)])
def test_isotropic_field_in_hubble_flow_cools_adiabatically(geom, factor):
    """Uniform isotropic radiation (F = 0) in a Hubble flow u = H r: the
    energy advected out of a cell, c dt E div(u)/c, plus the radiation
    pressure work, c dt (D : grad u / c) E with D = I/3, give one step's
    change E -> E (1 - k H c dt / c), k = 2 + 2/3 in the slab (div u = 2H)
    and 3 + 1 in (R, z) (div u = 3H, with the azimuthal u_R/R = H term) --
    radiation's adiabatic cooling dE/dt = -(4/3) E div u.  Cells away from
    the boundaries, no opacity or emission.  In (R, z) the face velocity,
    the mean of the two cells' centroid velocities, differs from H R_face
    by O((dR / R)^2), so there the factor approaches 4 outwards."""
    dx, nx, ny = 1.0e16, 16, 16
    p = band_problem(geom, nx, ny, dx, ("reflect", "vacuum", "vacuum", "vacuum") if geom == "cyl"
                     else ("vacuum",) * 4, [0.0], [0.0], [0.0], c_frac=0.01)
    xe, ye = inputs.edges(p)
    H = 3.0e-10                                   # 1/s: |u| <= 5e7 cm/s here
    xc = 0.5 * (xe[1:] + xe[:-1])
    if geom == "cyl":
        xc = (2.0 / 3.0) * (xe[1:] ** 3 - xe[:-1] ** 3) / (xe[1:] ** 2 - xe[:-1] ** 2)
    yc = 0.5 * (ye[1:] + ye[:-1])
    p["fields"]["u_x"] = np.broadcast_to(H * xc[None, :], (ny, nx)).copy()
    p["fields"]["u_y"] = np.broadcast_to(H * yc[:, None], (ny, nx)).copy()
    o = M.BandOracle(p)
    E0 = 1.0e-9
    o.set_state(np.full((1, ny, nx), E0), np.zeros((1, ny, nx)), np.zeros((1, ny, nx)))
    o.step(1)
    k1 = H * p["c_tilde"] * o.dt / C
    assert k1 > 1e-6                               # the effect is resolved
    fac = (1.0 - o.E[0][3:ny - 3, 3:nx - 3] / E0) / k1
    if geom == "cart":
        np.testing.assert_allclose(fac, factor, rtol=1e-9)
    else:
        err = np.abs(fac - factor)
        assert err.max() <= 1e-3 * factor
        assert np.all(np.diff(err[0]) < 0)          # converging outwards
