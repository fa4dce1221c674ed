"""Pins of the oracle's velocity terms against what the paper fixes.

Three parts of the step depend on the gas velocity, and each test below
checks it against a fact of the mathematics rather than against the oracle's
own formula:

  * the Doppler term of the frequency step, (1/c) d/dnu [nu (D : grad u) J]
    (Section 2.1 step 3; Appendix A): in an expanding flow the photon-weighted
    mean frequency falls at the rate (c_tilde / c) (D : grad u) while the
    photon number stays fixed (a redshift); with line opacity on, the
    exponential-scheme system assembled from C_k = K_k R_k + (nu_k / c)
    (D_k : grad u) is checked by a dense solve;
  * the cross term D_xy (d_y u_x + d_x u_y) of D : grad u (Appendix A), in
    the work term of the advection step and in the Doppler shift, with a
    shear flow where it is the only non-zero part;
  * the upwind velocity advection u J / c of the advection step (Section 2.1
    step 1): across a face between two plateaus the advective exchange
    carries the upstream cell's energy density.
"""
import math

import numpy as np
import pytest

from oracle import m1_oracle as M
from paper_2606_02711_amd import inputs

C = inputs.C_LIGHT


def _problem(nx, ny, dx, bc, ux, uy, n_HI=0.0, T=1.0e4):
    p = inputs.base_problem("cart", nx, ny, 0.0, nx * dx, 0.0, ny * dx, bc)
    sh = (ny, nx)
    z = np.zeros(sh)
    p["fields"] = dict(n_HI=np.full(sh, float(n_HI)), T=np.full(sh, float(T)),
                       u_x=np.broadcast_to(ux, sh).astype(np.float64).copy(),
                       u_y=np.broadcast_to(uy, sh).astype(np.float64).copy(),
                       alpha_abs=z.copy(), alpha_flux=z.copy(), p_d=z.copy(), emis=z.copy())
    return p


def _centred_spectrum(nb, width=8.0):
    """A spectrum over the narrow central bins (bin widths there are a few
    Doppler widths of 30 K, ~1e-5 of the line frequency)."""
    k = np.arange(nb)
    return np.exp(-0.5 * ((k - 0.5 * (nb - 1)) / width) ** 2)


def _levermore_D(fx, fy):
    """D = (1 - chi)/2 I + (3 chi - 1)/2 h h with chi = (3 + 4 f^2)/(5 + 2
    sqrt(4 - 3 f^2)) (Section 2.1, M1 closure): Dxx, Dyy, Dxy, Dphiphi."""
    f = math.hypot(fx, fy)
    chi = (3.0 + 4.0 * f * f) / (5.0 + 2.0 * math.sqrt(4.0 - 3.0 * f * f))
    iso, dirn = 0.5 * (1.0 - chi), 0.5 * (3.0 * chi - 1.0)
    hx, hy = (fx / f, fy / f) if f > 0 else (0.0, 0.0)
    return iso + dirn * hx * hx, iso + dirn * hy * hy, dirn * hx * hy, iso


def _mean_frequency_drop(o, Ess, E1, j, i):
    """Photon number before and after the frequency stage of cell (i, j), and
    the fall of sum_k nu_k dnu_k E_k (taken about line centre, which photon
    conservation makes the same fall without the cancellation)."""
    dnu = o.s.grid["dnu"]
    off = o.s.grid["nu_c"] - M.NU_LYA
    n0, n1 = float(dnu @ Ess[:, j, i]), float(dnu @ E1[:, j, i])
    drop = float((off * dnu) @ (Ess[:, j, i] - E1[:, j, i]))
    first = float((o.s.grid["nu_c"] * dnu) @ Ess[:, j, i])
    return n0, n1, drop, first


# ------------------------------------------------------------ Doppler term
def test_expanding_flow_redshifts_the_spectrum_line_off():
    """Uniform isotropic radiation in a Hubble flow u = H r (slab, no line
    opacity, so the frequency step is pure Doppler advection).  Integrating
    the Doppler term over frequency, d/dt int nu J dnu = -(c_tilde / c)
    (D : grad u) int nu J dnu and d/dt int J dnu = 0; with D = I/3 and
    grad u = H I (two dimensions), D : grad u = 2H/3 > 0.  Over one step the
    frequency stage must conserve photons exactly and lower sum nu dnu E by
    the fraction c_tilde dt (2H/3) / c.  On the discrete grid photons cross
    the interface k+1/2 over the centre distance nu_{k+1} - nu_k, which on a
    grid of growth factor q = 1.1 differs from the bin width by at most
    (q - 1)/2 = 5 %, with opposite signs on the two sides of the line; over a
    spectrum symmetric about the line the rate is the continuum one to a few
    1e-3, hence the 1 % bound.  A flipped sign raises the mean frequency, a
    missing factor nu or 1/3 misses by orders of magnitude."""
    n, dx = 12, 1.0e16
    xc = (np.arange(n) + 0.5) * dx - 0.5 * n * dx
    H = 2.0e5 / (0.5 * n * dx)                        # 2 km/s at the box edge
    p = _problem(n, n, dx, ("vacuum",) * 4, H * xc[None, :], H * xc[:, None])
    p["recoil"] = 0
    o = M.Oracle(p)
    s = o.s
    g = _centred_spectrum(s.nb)
    o.set_state(np.broadcast_to(g[:, None, None], (s.nb, n, n)).copy(),
                np.zeros((s.nb, n, n)), np.zeros((s.nb, n, n)))
    o.step(1)
    Ess, Xss, Yss = o.post_source_state()
    eps = p["c_tilde"] * o.dt * (2.0 * H / 3.0) / C
    for j in range(2, n - 2):
        for i in range(2, n - 2):
            assert not Xss[:, j, i].any() and not Yss[:, j, i].any()   # D = I/3 here
            n0, n1, drop, first = _mean_frequency_drop(o, Ess, o.E, j, i)
            assert n1 == pytest.approx(n0, rel=1e-13)
            assert drop > 0.0                                          # a redshift
            assert drop / (eps * first) == pytest.approx(1.0, abs=1e-2), (i, j)


def test_contracting_flow_blueshifts_the_spectrum_line_off():
    """The same with u = -H r: D : grad u = -2H/3, the mean frequency rises
    by the same fraction."""
    n, dx = 12, 1.0e16
    xc = (np.arange(n) + 0.5) * dx - 0.5 * n * dx
    H = 2.0e5 / (0.5 * n * dx)
    p = _problem(n, n, dx, ("vacuum",) * 4, -H * xc[None, :], -H * xc[:, None])
    p["recoil"] = 0
    o = M.Oracle(p)
    s = o.s
    g = _centred_spectrum(s.nb)
    o.set_state(np.broadcast_to(g[:, None, None], (s.nb, n, n)).copy(),
                np.zeros((s.nb, n, n)), np.zeros((s.nb, n, n)))
    o.step(1)
    Ess, _, _ = o.post_source_state()
    eps = p["c_tilde"] * o.dt * (2.0 * H / 3.0) / C
    for j, i in ((3, 3), (5, 7), (8, 4)):
        n0, n1, drop, first = _mean_frequency_drop(o, Ess, o.E, j, i)
        assert n1 == pytest.approx(n0, rel=1e-13)
        assert -drop / (eps * first) == pytest.approx(1.0, abs=1e-2)


def _face_velocities(p):
    """Face-normal and tangential velocities as the means of the two adjacent
    cell velocities; ghosts copy the boundary cell at a vacuum edge and mirror
    it (normal component negated) at a reflecting one."""
    f = p["fields"]
    ux, uy = f["u_x"], f["u_y"]
    bc = p["bc"]
    ny, nx = ux.shape
    gxl = np.where(bc[0] == "reflect", -1.0, 1.0)
    gxr = np.where(bc[1] == "reflect", -1.0, 1.0)
    ux_p = np.concatenate([gxl * ux[:, :1], ux, gxr * ux[:, -1:]], axis=1)
    uy_px = np.concatenate([uy[:, :1], uy, uy[:, -1:]], axis=1)
    un_x = 0.5 * (ux_p[:, :-1] + ux_p[:, 1:])            # [ny, nx+1]
    ut_x = 0.5 * (uy_px[:, :-1] + uy_px[:, 1:])
    gyl = np.where(bc[2] == "reflect", -1.0, 1.0)
    gyr = np.where(bc[3] == "reflect", -1.0, 1.0)
    uy_p = np.concatenate([gyl * uy[:1, :], uy, gyr * uy[-1:, :]], axis=0)
    ux_py = np.concatenate([ux[:1, :], ux, ux[-1:, :]], axis=0)
    un_y = 0.5 * (uy_p[:-1, :] + uy_p[1:, :])            # [ny+1, nx]
    ut_y = 0.5 * (ux_py[:-1, :] + ux_py[1:, :])
    return un_x, ut_x, un_y, ut_y


def _D_colon_grad_u(p, fx, fy, i, j):
    """D : grad u of cell (i, j) (Appendix A): D_RR d_R u_R + D_zz d_z u_z
    + D_phiphi <u_R / R> + D_Rz (d_z u_R + d_R u_z), the derivatives as
    differences of face velocities over the cell width and <u_R / R> as the
    sum of the two R-face velocities over the sum of their radii (the slab
    drops the phi term)."""
    un_x, ut_x, un_y, ut_y = _face_velocities(p)
    xe, ye = inputs.edges(p)
    hx, hy = xe[i + 1] - xe[i], ye[j + 1] - ye[j]
    dxux = (un_x[j, i + 1] - un_x[j, i]) / hx
    dxuy = (ut_x[j, i + 1] - ut_x[j, i]) / hx
    dyuy = (un_y[j + 1, i] - un_y[j, i]) / hy
    dyux = (ut_y[j + 1, i] - ut_y[j, i]) / hy
    Dxx, Dyy, Dxy, Dpp = _levermore_D(fx, fy)
    g = Dxx * dxux + Dyy * dyuy + Dxy * (dyux + dxuy)
    if p["geom"] == "cyl":
        g += Dpp * (un_x[j, i + 1] + un_x[j, i]) / (xe[i + 1] + xe[i])
    return g


@pytest.mark.parametrize("geom,seed", [("cart", 78), ("cyl", 79)])
def test_frequency_stage_with_doppler_matches_dense_solve_on_8x8(geom, seed):
    """Brute force with velocities on (random flows to 50 km/s, line opacity
    and recoil on): per cell the BDF1 system of Appendix A is assembled here
    from K_k = dnu_D^2 alpha <H>_k / 2 and C_k = K_k (h/kT - 2/nu_k) + (nu_k/c)
    (D_k : grad u), with D_k from the post-source state and the velocity
    gradients from the face velocities, and solved by a dense LU solve."""
    p = inputs.random_small(geom, 8, 8, seed, with_velocity=True, half_width=300.0,
                            log_nHI=(-3.0, 0.0))
    o = M.Oracle(p)
    s = o.s
    rng = np.random.default_rng(seed)
    shape = (s.nb, s.ny, s.nx)
    E0 = rng.uniform(0.5, 1.0, shape) * 1e-20
    ang = rng.uniform(0, 2 * np.pi, shape)
    fr = rng.uniform(0.0, 0.95, shape)
    o.set_state(E0, E0 * fr * np.cos(ang), E0 * fr * np.sin(ang))
    o.step(1)
    Ess, Xss, Yss = o.post_source_state()
    dnu = s.grid["dnu"]
    nu = s.grid["nu_c"]
    ct = p["c_tilde"] * o.dt
    worst, doppler_share = 0.0, 0.0
    for c in range(s.nx * s.ny):
        j, i = divmod(c, s.nx)
        h = s.hbar[s.cls[c]]
        K = 0.5 * s.dnuD[c] ** 2 * s.alpha[c] * h
        G = np.array([_D_colon_grad_u(p, Xss[k, j, i] / Ess[k, j, i],
                                      Yss[k, j, i] / Ess[k, j, i], i, j) for k in range(s.nb)])
        Cr = K * (s.hkT[c] - 2.0 / nu)
        Cd = nu / C * G
        doppler_share = max(doppler_share, float(np.max(np.abs(Cd) / (np.abs(Cr) + np.abs(Cd)))))
        Ck = Cr + Cd
        A = np.eye(s.nb)
        for k in range(s.nb - 1):
            gl, gr = M.interface_rates(K[k], Ck[k], 0.5 * dnu[k], K[k + 1], Ck[k + 1],
                                       0.5 * dnu[k + 1])
            A[k, k] += ct * gl / dnu[k]
            A[k, k + 1] -= ct * gr / dnu[k]
            A[k + 1, k + 1] += ct * gr / dnu[k + 1]
            A[k + 1, k] -= ct * gl / dnu[k + 1]
        Jn = np.linalg.solve(A, Ess[:, j, i])
        worst = max(worst, float(np.max(np.abs(Jn - o.E[:, j, i]) / np.abs(Jn).max())))
    assert doppler_share > 0.5           # the Doppler part matters in these cells
    assert worst < 1e-10, worst


# ------------------------------------------------------------- cross term
@pytest.mark.parametrize("s_sign,f_sign", [(1.0, 1.0), (1.0, -1.0), (-1.0, 1.0)])
def test_shear_flow_work_term_and_doppler_through_D_xy(s_sign, f_sign):
    """Uniform radiation with f at +-45 degrees (|f| = 0.6) in the shear flow
    u_y = s x (slab, no opacity).  Only d_x u_y = s is non-zero, so
    D : grad u = D_xy s.  In interior cells every flux difference vanishes
    (uniform state; the y-faces of a cell carry the same u_y), so the
    advection step is the work term alone: E** = E (1 - c_tilde dt D_xy s / c)
    with D_xy = (3 chi - 1)/2 h_x h_y.  The frequency stage then shifts the
    mean frequency by -c_tilde dt D_xy s / c (D from the post-source state).
    Either sign of D_xy s is tested."""
    n, dx = 12, 1.0e16
    xc = (np.arange(n) + 0.5) * dx - 0.5 * n * dx
    shear = s_sign * 2.0e5 / (0.5 * n * dx)
    p = _problem(n, n, dx, ("vacuum",) * 4, 0.0, shear * xc[None, :])
    p["recoil"] = 0
    o = M.Oracle(p)
    s = o.s
    g = _centred_spectrum(s.nb)
    E = np.broadcast_to(g[:, None, None], (s.nb, n, n)).copy()
    f = 0.6 / math.sqrt(2.0)
    o.set_state(E, f * E, f_sign * f * E)
    o.step(1)
    Ess, Xss, Yss = o.post_source_state()
    ct = p["c_tilde"] * o.dt
    Dxy = _levermore_D(f, f_sign * f)[2]
    work = ct * Dxy * shear / C
    assert abs(work) > 1e-8
    for j in range(2, n - 2):
        for i in range(2, n - 2):
            expect = E[:, j, i] * (1.0 - work)
            # to the rounding of E (1e-16) against a change of ~3e-8 of it
            assert np.all(np.abs(Ess[:, j, i] - expect) <= 1e-7 * abs(work) * E[:, j, i])
            fx, fy = Xss[96, j, i] / Ess[96, j, i], Yss[96, j, i] / Ess[96, j, i]
            eps = ct * _levermore_D(fx, fy)[2] * shear / C
            n0, n1, drop, first = _mean_frequency_drop(o, Ess, o.E, j, i)
            assert n1 == pytest.approx(n0, rel=1e-13)
            assert drop / (eps * first) == pytest.approx(1.0, abs=1e-2), (i, j)


# ------------------------------------------------------------- upwinding
@pytest.mark.parametrize("u", [3.0e6, -3.0e6])
def test_velocity_advection_is_upwind(u):
    """Two plateaus of E (f = 0) meet at the face between cells 3 and 4 of a
    row of 8; MinMod gives zero slopes there, so the reconstructed face
    states are the plateau values.  In a uniform flow (no gradients, so no
    work term; vacuum ghosts copy the velocity) the step with velocity u
    differs from the step with u = 0 (same dt) only by the advective fluxes
    (u / c) E_upwind: the cell downstream of the face gains (or the one
    upstream loses) c_tilde dt / dx (u / c) (E_R - E_L), and the other cell
    of the face is unchanged, because the faces of a cell inside a plateau
    carry equal states.  A downwind choice would swap the two cells."""
    nx, ny, dx = 8, 6, 1.0e16
    EL, ER = 1.0, 3.0
    res = {}
    for vel in (0.0, u):
        p = _problem(nx, ny, dx, ("vacuum",) * 4, vel, 0.0)
        p["recoil"] = 0
        o = M.Oracle(p, dt=0.2 * dx / p["c_tilde"])
        s = o.s
        E = np.zeros((s.nb, ny, nx))
        E[:, :, :4] = EL
        E[:, :, 4:] = ER
        o.set_state(E, np.zeros_like(E), np.zeros_like(E))
        o.step(1)
        res[vel] = (o.post_source_state()[0], p["c_tilde"] * o.dt)
    ct = res[u][1]
    d = res[u][0] - res[0.0][0]
    jump = ct / dx * (u / C) * (ER - EL)
    rows = slice(2, ny - 2)
    gain3, gain4 = d[:, rows, 3], d[:, rows, 4]
    if u > 0:   # face 3|4 carries (u/c) E_L: cell 4 changes by -ct/dx (u/c)(E_R - E_L)
        assert np.allclose(gain3, 0.0, atol=1e-12 * abs(jump))
        assert np.allclose(gain4, -jump, rtol=1e-9)
    else:       # it carries (u/c) E_R: cell 3 changes by -ct/dx (u/c)(E_R - E_L)
        assert np.allclose(gain3, -jump, rtol=1e-9)
        assert np.allclose(gain4, 0.0, atol=1e-12 * abs(jump))
