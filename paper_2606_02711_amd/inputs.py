"""Seeded synthetic inputs for the M1 Lyman-alpha transfer step.

This module only *builds problems*: grids, per-cell physical fields and run
parameters.  It holds none of the transfer method's arithmetic (no closure,
flux, source or frequency-step formula), so both the FP64 CPU oracle and the
GPU library can consume what it produces without sharing method code.

A problem is a plain dict:

  geom        "cart" (2D slab, unit depth) or "cyl" (axisymmetric R, z)
  nx, ny      cells along x (or R) and y (or z)
  x0,x1,y0,y1 domain edges [cm]
  bc          (x-, x+, y-, y+), each "vacuum" or "reflect"
  T_min, q, half_width   frequency-grid parameters (Section 2.1: 30 K, 1.1,
                         1e5 Doppler widths of T_min)
  c_tilde, cfl           reduced speed of light [cm/s], CFL factor
  recoil, doppler        0/1 switches for the recoil and Doppler terms
  steps                  number of explicit RT steps the workload runs
  fields      dict of float64 arrays of shape (ny, nx) (index [j, i]):
              n_HI [cm^-3], T [K], u_x, u_y [cm/s],
              alpha_abs  = continuum absorption alpha_c (1 - omega)  [cm^-1]
              alpha_flux = continuum flux opacity alpha_c (1 - omega g) [cm^-1]
              p_d        = Lya destruction probability per scattering
              emis       = Lya luminosity density [erg s^-1 cm^-3]

Workload recipes (the paper runs no public dataset on this path; these
seeded fields stand in for its test clouds and star-forming clouds):

  config 1  Cartesian 64^2 unit box, uniform neutral gas, line-centre depth
            1e4 across the box, T = 1e4 K, Gaussian source, 200 steps.
  config 2  cylindrical 512 x 1024 (R, z) = 1 pc x 2 pc, ionised bubble in a
            log-normal neutral shell with a k^-2 random field, radial outflow
            to 30 km/s, dust 0.01 solar, p_d = 1e-6, point source on the axis.
  config 3  64 uniform clouds of log-uniform size 64..512 cells per side.
  config 4  request stream of clouds of size 128..2048 per side.
  config 5  cylindrical 4096 x 8192 turbulent cloud with 16 ring sources.
"""
from __future__ import annotations

import math

import numpy as np

# Physical constants used to *construct* inputs (cgs).
PC = 3.0856775814913673e18          # parsec [cm]
KMS = 1.0e5                         # km/s [cm/s]
C_LIGHT = 2.99792458e10
M_H = 1.6735575e-24
# Line-centre cross-section scaling quoted in Section 2.1 (5.9e-14 T4^-1/2 cm^2);
# used only to turn a requested optical depth into a neutral density.
SIGMA0_1E4 = 5.9e-14
# Table 2, Lya row, mass-weighted over the three grain bins (f_Sil, f_C, f_PAH).
F_SIL, F_C, F_PAH = 0.7264, 0.2517, 0.0218
KAPPA_ABS_LYA = F_SIL * 1.84e4 + F_C * 2.48e4 + F_PAH * 3.31e5   # cm^2/g of dust
KAPPA_F_LYA = F_SIL * 2.22e4 + F_C * 2.84e4 + F_PAH * 3.31e5
DUST_TO_GAS_SOLAR = 1.0 / 162.0

SEED_BASE = 260602711

FIELD_NAMES = ("n_HI", "T", "u_x", "u_y", "alpha_abs", "alpha_flux", "p_d", "emis")


def rng_for(config_id: int, sub: int = 0) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([SEED_BASE + config_id, sub]))


# --------------------------------------------------------------------------
# geometry of the *input recipe* (cell volumes, used to normalise luminosity)
# --------------------------------------------------------------------------
def edges(p):
    xe = p["x0"] + (p["x1"] - p["x0"]) * np.arange(p["nx"] + 1) / p["nx"]
    ye = p["y0"] + (p["y1"] - p["y0"]) * np.arange(p["ny"] + 1) / p["ny"]
    return xe, ye


def cell_volumes(p) -> np.ndarray:
    xe, ye = edges(p)
    dy = np.diff(ye)
    if p["geom"] == "cyl":
        ring = math.pi * (xe[1:] ** 2 - xe[:-1] ** 2)
        return dy[:, None] * ring[None, :]
    return dy[:, None] * np.diff(xe)[None, :]


def cell_centres(p):
    """Plain midpoints: used only to place sources and density structure."""
    xe, ye = edges(p)
    return 0.5 * (xe[1:] + xe[:-1]), 0.5 * (ye[1:] + ye[:-1])


def gaussian_source(p, cx, cy, sigma, L=1.0) -> np.ndarray:
    """Gaussian luminosity density centred at (cx, cy), sigma in cm; its
    volume integral over the grid is L [erg/s]."""
    xc, yc = cell_centres(p)
    r2 = (xc[None, :] - cx) ** 2 + (yc[:, None] - cy) ** 2
    shape = np.exp(-0.5 * r2 / sigma ** 2)
    vol = cell_volumes(p)
    return shape * (L / float(np.sum(shape * vol)))


def point_source_cells(p, cells, L=1.0) -> np.ndarray:
    """Split luminosity L equally over the listed (i, j) cells."""
    vol = cell_volumes(p)
    em = np.zeros((p["ny"], p["nx"]))
    share = L / len(cells)
    for (i, j) in cells:
        em[j, i] += share / vol[j, i]
    return em


def dust_opacities(n_H, dust_solar):
    """Continuum opacities of dust at Lya (Table 2 Lya row; rho = n_H m_H/0.75,
    solar dust-to-gas ratio 1/162)."""
    rho = np.asarray(n_H) * M_H / 0.75
    D = np.asarray(dust_solar) * DUST_TO_GAS_SOLAR
    return D * rho * KAPPA_ABS_LYA, D * rho * KAPPA_F_LYA


def gaussian_random_field(rng, ny, nx, slope=-2.0) -> np.ndarray:
    """Zero-mean, unit-variance Gaussian random field on the index grid with
    power spectrum P(k) ~ k^slope (k = 0 removed)."""
    white = rng.standard_normal((ny, nx))
    ky = np.fft.fftfreq(ny)[:, None]
    kx = np.fft.rfftfreq(nx)[None, :]
    k = np.sqrt(kx * kx + ky * ky)
    amp = np.zeros_like(k)
    nz = k > 0
    amp[nz] = k[nz] ** (0.5 * slope)
    g = np.fft.irfft2(np.fft.rfft2(white) * amp, s=(ny, nx))
    g -= g.mean()
    g /= g.std()
    return g


def base_problem(geom, nx, ny, x0, x1, y0, y1, bc, c_tilde_frac=0.01, steps=1):
    return dict(
        geom=geom, nx=int(nx), ny=int(ny),
        x0=float(x0), x1=float(x1), y0=float(y0), y1=float(y1),
        bc=tuple(bc), T_min=30.0, q=1.1, half_width=1.0e5,
        c_tilde=c_tilde_frac * C_LIGHT, cfl=0.4, recoil=1, doppler=1,
        steps=int(steps), fields={},
    )


def uniform_fields(p, n_HI, T, dust_solar=0.0, p_d=0.0, n_H=None):
    sh = (p["ny"], p["nx"])
    n_H = n_HI if n_H is None else n_H
    a_abs, a_F = dust_opacities(np.full(sh, n_H), dust_solar)
    return dict(
        n_HI=np.full(sh, float(n_HI)), T=np.full(sh, float(T)),
        u_x=np.zeros(sh), u_y=np.zeros(sh),
        alpha_abs=a_abs, alpha_flux=a_F, p_d=np.full(sh, float(p_d)),
        emis=np.zeros(sh),
    )


# --------------------------------------------------------------------------
# the five workloads
# --------------------------------------------------------------------------
def config1():
    """64^2 Cartesian unit box, tau0 = 1e4 across, T = 1e4 K, Gaussian source."""
    p = base_problem("cart", 64, 64, 0.0, 1.0, 0.0, 1.0, ("vacuum",) * 4, steps=200)
    n_HI = 1.0e4 / SIGMA0_1E4          # alpha * 1 cm = 1e4 at T = 1e4 K
    f = uniform_fields(p, n_HI, 1.0e4)
    f["emis"] = gaussian_source(p, 0.5, 0.5, 2.0 / 64.0, 1.0)
    p["fields"] = f
    return p


def config2(nx=512, ny=1024, steps=1000):
    """Cylindrical (R, z) bubble + log-normal neutral shell, radial outflow."""
    p = base_problem("cyl", nx, ny, 0.0, PC, -PC, PC,
                     ("reflect", "vacuum", "vacuum", "vacuum"), steps=steps)
    rng = rng_for(2)
    R, Z = cell_centres(p)
    r = np.sqrt(R[None, :] ** 2 + Z[:, None] ** 2)
    g = gaussian_random_field(rng, ny, nx)
    sig = 1.0
    n_shell = 1.0e3 * np.exp(sig * g - 0.5 * sig * sig)
    bubble = r < 0.3 * PC
    n_H = np.where(bubble, 10.0, n_shell)
    n_HI = np.where(bubble, 10.0 * 1.0e-4, n_shell)
    T = np.where(bubble, 1.0e4, 100.0)
    a_abs, a_F = dust_opacities(n_H, 0.01)
    vr = 30.0 * KMS * np.minimum(r / PC, 1.0)
    with np.errstate(invalid="ignore", divide="ignore"):
        ux = np.where(r > 0, vr * R[None, :] / r, 0.0)
        uy = np.where(r > 0, vr * Z[:, None] / r, 0.0)
    jz = ny // 2
    em = point_source_cells(p, [(0, jz - 1), (0, jz)], 1.0)
    p["fields"] = dict(n_HI=n_HI, T=T, u_x=ux, u_y=uy, alpha_abs=a_abs,
                       alpha_flux=a_F, p_d=np.full(n_H.shape, 1.0e-6), emis=em)
    return p


def uniform_cloud(geom, n, log10_NHI, T, dust_solar, L_box=PC, steps=500, fields=True):
    """Uniform neutral cloud with a Gaussian sigma = 2 cells central source.
    Cartesian: [-L/2, L/2]^2, all vacuum.  Cylindrical: R, z in [0, L/2] with
    the axis and the z = 0 midplane reflecting.  fields=False returns the
    grid description only (empty "fields")."""
    half = 0.5 * L_box
    if geom == "cart":
        p = base_problem("cart", n, n, -half, half, -half, half,
                         ("vacuum",) * 4, steps=steps)
    else:
        p = base_problem("cyl", n, n, 0.0, half, 0.0, half,
                         ("reflect", "vacuum", "reflect", "vacuum"), steps=steps)
    if not fields:
        return p
    n_HI = 10.0 ** log10_NHI / half
    f = uniform_fields(p, n_HI, T, dust_solar=dust_solar, p_d=0.0)
    dx = (p["x1"] - p["x0"]) / n
    f["emis"] = gaussian_source(p, 0.0, 0.0, 2.0 * dx, 1.0)
    p["fields"] = f
    return p


def cone_cloud(n=256, R_cl=PC, tau_cl=1.0e8, tau_cone=1.0e5, T=1.0e4, mu_cone=2 ** -0.5,
               dmu=0.025):
    """Anisotropic-escape cloud of Section 3.2 (Test 6): a spherical cloud of
    radius R_cl at T with a bipolar low-density cone (half-opening angle
    acos(mu_cone), tanh transition of width dmu in mu = |Z|/r), neutral
    fraction 1 in the shell 0.5 R_cl < r <= R_cl and 1e-4 inside, uniform
    emission inside 0.5 R_cl, vacuum outside.  Densities from
    tau = n_H sigma0(T) R_cl.  Box [0, 1.1 R_cl]^2 in (R, Z): reflecting axis
    and midplane, outflow at the outer edges; c_tilde = c; recoil on, no
    continuum absorption, no destruction."""
    half = 1.1 * R_cl
    p = base_problem("cyl", n, n, 0.0, half, 0.0, half,
                     ("reflect", "vacuum", "reflect", "vacuum"), c_tilde_frac=1.0)
    R, Z = cell_centres(p)
    r = np.sqrt(R[None, :] ** 2 + Z[:, None] ** 2)
    mu = np.where(r > 0, np.abs(Z)[:, None] / np.where(r > 0, r, 1.0), 0.0)
    sig0 = SIGMA0_1E4 * (T / 1.0e4) ** -0.5
    n_cl, n_cone = tau_cl / (sig0 * R_cl), tau_cone / (sig0 * R_cl)
    n_H = n_cone + 0.5 * (n_cl - n_cone) * (1.0 - np.tanh((mu - mu_cone) / dmu))
    eps = np.where(r <= 0.5 * R_cl, 1.0e-4, 1.0)
    f = uniform_fields(p, 0.0, T)
    f["n_HI"] = np.where(r <= R_cl, eps * n_H, 0.0)
    src = (r <= 0.5 * R_cl).astype(float)
    f["emis"] = src / float(np.sum(src * cell_volumes(p)))      # 1 erg/s in the box
    p["fields"] = f
    p["R_cl"] = R_cl
    p["t_max"] = 4.0 * max((4.7e-4 * (T / 1.0e4) ** -0.5 * tau_cl) ** (1.0 / 3.0), 3.0) * R_cl / C_LIGHT
    return p


def static_sphere(n=64, R_cl=PC, tau_cl=1.0e6, T=1.0e4, tau_c=0.0, v_exp=0.0):
    """Uniform cloud of Section 3.1 (Tests 1, 2, 4 and 5): a uniform sphere of
    radius R_cl at T with line-centre depth tau_cl = n_HI sigma0(T) R_cl and
    uniform emission (1 erg/s in the box), vacuum outside; box
    [0, 1.1 R_cl]^2 in (R, Z) with reflecting axis and midplane, outflow at the
    outer edges; c_tilde = c; no recoil, no destruction.  tau_c: continuum
    (dust) absorption depth alpha_c R_cl inside the cloud, pure absorption
    (albedo 0, so the flux opacity equals it); 0 for the dust-free Test 1.
    v_exp: expansion rate dR_cl/dt [cm/s] of a Hubble-like flow
    u = (v_exp / R_cl) r r_hat inside the cloud (Test 2); gas at rest outside."""
    half = 1.1 * R_cl
    p = base_problem("cyl", n, n, 0.0, half, 0.0, half,
                     ("reflect", "vacuum", "reflect", "vacuum"), c_tilde_frac=1.0)
    p["recoil"] = 0
    R, Z = cell_centres(p)
    inside = np.sqrt(R[None, :] ** 2 + Z[:, None] ** 2) <= R_cl
    sig0 = SIGMA0_1E4 * (T / 1.0e4) ** -0.5
    f = uniform_fields(p, 0.0, T)
    f["n_HI"] = np.where(inside, tau_cl / (sig0 * R_cl), 0.0)
    f["alpha_abs"] = np.where(inside, tau_c / R_cl, 0.0)
    f["alpha_flux"] = f["alpha_abs"].copy()
    f["u_x"] = np.where(inside, (v_exp / R_cl) * R[None, :], 0.0)
    f["u_y"] = np.where(inside, (v_exp / R_cl) * Z[:, None], 0.0)
    src = inside.astype(float)
    f["emis"] = src / float(np.sum(src * cell_volumes(p)))
    p["fields"] = f
    p["R_cl"] = R_cl
    p["t_max"] = 4.0 * max((4.7e-4 * (T / 1.0e4) ** -0.5 * tau_cl) ** (1.0 / 3.0), 3.0) * R_cl / C_LIGHT
    return p


def config3(n_grids=64, lo=64, hi=512, config_id=3, steps=500):
    rng = rng_for(config_id)
    probs = []
    for g in range(n_grids):
        n = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        geom = "cart" if g < n_grids // 2 else "cyl"
        lN = rng.uniform(19.0, 23.0)
        T = 10.0 ** rng.uniform(2.0, 4.0)
        dust = rng.uniform(0.0, 0.01)
        probs.append(uniform_cloud(geom, n, lN, T, dust, steps=steps))
    return probs


def config4_requests(rate=50.0, duration=120.0, lo=128, hi=2048, seed_sub=0):
    """Poisson request stream: list of (arrival_time_s, problem_factory_args)."""
    rng = rng_for(4, seed_sub)
    t = 0.0
    reqs = []
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            break
        n = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        geom = "cart" if rng.uniform() < 0.5 else "cyl"
        lN = rng.uniform(19.0, 23.0)
        T = 10.0 ** rng.uniform(2.0, 4.0)
        dust = rng.uniform(0.0, 0.01)
        reqs.append((t, dict(geom=geom, n=n, log10_NHI=lN, T=T, dust_solar=dust)))
    return reqs


def config5(nx=4096, ny=8192, steps=10000):
    p = base_problem("cyl", nx, ny, 0.0, PC, -PC, PC,
                     ("reflect", "vacuum", "vacuum", "vacuum"), steps=steps)
    rng = rng_for(5)
    R, Z = cell_centres(p)
    r = np.sqrt(R[None, :] ** 2 + Z[:, None] ** 2)
    sig = 1.5
    g = gaussian_random_field(rng, ny, nx)
    n_H = 1.0e4 * np.exp(sig * g - 0.5 * sig * sig)
    del g
    hii = r < 0.2 * PC
    n_HI = np.where(hii, n_H * 1.0e-4, n_H)
    T = np.where(hii, 1.0e4, 100.0)
    a_abs, a_F = dust_opacities(n_H, 0.01)
    ux = gaussian_random_field(rng, ny, nx)
    uy = gaussian_random_field(rng, ny, nx)
    vmax = float(np.sqrt(ux * ux + uy * uy).max())
    ux *= 50.0 * KMS / vmax
    uy *= 50.0 * KMS / vmax
    cells = []
    dx = (p["x1"] - p["x0"]) / nx
    dy = (p["y1"] - p["y0"]) / ny
    while len(cells) < 16:
        rr = 0.2 * PC * math.sqrt(rng.uniform())
        th = rng.uniform(0.0, math.pi)
        sx, sz = rr * math.sin(th), rr * math.cos(th)
        i = min(int(sx / dx), nx - 1)
        j = min(int((sz - p["y0"]) / dy), ny - 1)
        if (i, j) not in cells:
            cells.append((i, j))
    em = point_source_cells(p, cells, 1.0)
    p["fields"] = dict(n_HI=n_HI, T=T, u_x=ux, u_y=uy, alpha_abs=a_abs,
                       alpha_flux=a_F, p_d=np.full(n_H.shape, 1.0e-7), emis=em)
    return p


def random_small(geom, nx, ny, seed, with_velocity=True, with_dust=True,
                 half_width=1.0e5, T_range=(100.0, 1.0e4), log_nHI=(-6.0, -2.0),
                 L_box=1.0e16, bc=None):
    """Small random heterogeneous problem for parity tests (all physics on)."""
    rng = np.random.default_rng(np.random.SeedSequence([SEED_BASE, 99, seed]))
    if geom == "cart":
        p = base_problem("cart", nx, ny, 0.0, L_box, 0.0, L_box * ny / nx,
                         bc or ("vacuum",) * 4)
    else:
        p = base_problem("cyl", nx, ny, 0.0, L_box, -0.5 * L_box * ny / nx,
                         0.5 * L_box * ny / nx,
                         bc or ("reflect", "vacuum", "vacuum", "vacuum"))
    p["half_width"] = half_width
    sh = (ny, nx)
    n_HI = 10.0 ** rng.uniform(*log_nHI, size=sh)
    T = 10.0 ** rng.uniform(math.log10(T_range[0]), math.log10(T_range[1]), size=sh)
    if with_dust:
        a_abs, a_F = dust_opacities(n_HI, rng.uniform(0.0, 0.05, size=sh))
    else:
        a_abs, a_F = np.zeros(sh), np.zeros(sh)
    if with_velocity:
        ux = rng.uniform(-50.0, 50.0, size=sh) * KMS
        uy = rng.uniform(-50.0, 50.0, size=sh) * KMS
    else:
        ux, uy = np.zeros(sh), np.zeros(sh)
    pd = 10.0 ** rng.uniform(-8.0, -3.0, size=sh)
    em = rng.uniform(0.0, 1.0, size=sh) ** 4
    em *= 1.0 / float(np.sum(em * cell_volumes(p)))
    p["fields"] = dict(n_HI=n_HI, T=T, u_x=ux, u_y=uy, alpha_abs=a_abs,
                       alpha_flux=a_F, p_d=pd, emis=em)
    return p


# --------------------------------------------------------------------------
# broad bands (stellar and IR transport of Section 2.5)
# --------------------------------------------------------------------------
# A band problem carries the line problem's geometry keys plus n_band and
# fields u_x, u_y (ny, nx) and, per band and cell (n_band, ny, nx):
#   kappa_abs  = absorption opacity [cm^-1]
#   kappa_flux = flux-mean opacity [cm^-1]
#   emis       = luminosity density [erg s^-1 cm^-3]
BANDS = ("IR", "opt", "FUV", "LW", "EUV1", "EUV2", "EUV3")
# Dust per band (Section 2.5 table of non-IR band properties): (kappa_abs,
# kappa_F) of silicate, graphite and PAH grains [cm^2 per g of dust in the
# bin].  IR: a grey stand-in (the paper's IR opacities are temperature
# dependent, Appendix E), used only to give the IR band a plausible depth.
DUST_BAND_KAPPA = {
    "IR": ((5.0, 5.0), (5.0, 5.0), (5.0, 5.0)),
    "opt": ((5.98e3, 1.69e4), (2.09e4, 2.61e4), (2.27e5, 2.27e5)),
    "FUV": ((1.71e4, 2.21e4), (2.29e4, 2.57e4), (2.86e5, 2.86e5)),
    "LW": ((1.80e4, 2.18e4), (3.88e4, 4.48e4), (5.92e5, 5.92e5)),
    "EUV1": ((1.53e4, 1.85e4), (5.60e4, 6.22e4), (1.08e6, 1.08e6)),
    "EUV2": ((1.37e4, 1.46e4), (1.90e4, 2.12e4), (2.83e5, 2.84e5)),
    "EUV3": ((1.30e4, 1.32e4), (1.04e4, 1.09e4), (8.81e4, 8.82e4)),
}
# Band-mean photoionisation cross-sections [cm^2] of H I, He I, He II:
# order-of-magnitude stand-ins (the paper takes them from its references),
# used only to shape the inputs.
GAS_BAND_SIGMA = {
    "EUV1": (3.0e-18, 0.0, 0.0),
    "EUV2": (5.7e-19, 4.5e-18, 0.0),
    "EUV3": (7.9e-20, 1.2e-18, 1.1e-18),
}
# Share of the stellar luminosity per band (a hot star; stand-in).
STAR_BAND_SHARE = {"IR": 0.0, "opt": 0.15, "FUV": 0.30, "LW": 0.10, "EUV1": 0.30,
                   "EUV2": 0.12, "EUV3": 0.03}


def band_opacities(n_H, x_HI, dust_solar, bands=BANDS):
    """(kappa_abs, kappa_F) [n_band, ...] of dust (mass fractions f_Sil, f_C,
    f_PAH of the dust) plus gas photoionisation (H I fraction x_HI, helium
    number ratio 0.08 with its neutral fraction following x_HI)."""
    n_H = np.asarray(n_H, dtype=np.float64)
    rho_d = np.asarray(dust_solar) * DUST_TO_GAS_SOLAR * n_H * M_H / 0.75
    n_HI = np.asarray(x_HI) * n_H
    n_He = 0.08 * n_H
    ka, kf = [], []
    for b in bands:
        d = DUST_BAND_KAPPA[b]
        da = sum(f * k[0] for f, k in zip((F_SIL, F_C, F_PAH), d)) * rho_d
        dF = sum(f * k[1] for f, k in zip((F_SIL, F_C, F_PAH), d)) * rho_d
        s = GAS_BAND_SIGMA.get(b, (0.0, 0.0, 0.0))
        gas = s[0] * n_HI + s[1] * n_He * np.asarray(x_HI) + s[2] * n_He * 0.5
        ka.append(da + gas)
        kf.append(dF + gas)
    return np.stack(ka), np.stack(kf)


def band_base(p, n_band):
    q = dict(p)
    q["n_band"] = int(n_band)
    for k in ("T_min", "q", "half_width", "recoil", "doppler"):
        q.pop(k, None)
    return q


def band_random_small(geom, nx, ny, seed, n_band=7, with_velocity=True, L_box=1.0e18,
                      log_tau_cell=(-4.0, 3.0), bc=None):
    """Small random band problem for parity tests: per-cell, per-band optical
    depths log-uniform over log_tau_cell, flux opacity >= absorption
    opacity, sparse random emission, velocities up to 50 km/s."""
    rng = np.random.default_rng(np.random.SeedSequence([SEED_BASE, 77, seed]))
    if geom == "cart":
        p = base_problem("cart", nx, ny, 0.0, L_box, 0.0, L_box * ny / nx,
                         bc or ("vacuum",) * 4)
    else:
        p = base_problem("cyl", nx, ny, 0.0, L_box, -0.5 * L_box * ny / nx,
                         0.5 * L_box * ny / nx,
                         bc or ("reflect", "vacuum", "vacuum", "vacuum"))
    p = band_base(p, n_band)
    dx = L_box / nx
    sh = (n_band, ny, nx)
    ka = 10.0 ** rng.uniform(*log_tau_cell, size=sh) / dx
    kf = ka * (1.0 + rng.uniform(0.0, 2.0, size=sh))
    em = rng.uniform(0.0, 1.0, size=sh) ** 8
    em *= 1.0 / float(np.sum(em[0] * cell_volumes(p)) + 1e-300)
    if with_velocity:
        ux = rng.uniform(-50.0, 50.0, size=sh[1:]) * KMS
        uy = rng.uniform(-50.0, 50.0, size=sh[1:]) * KMS
    else:
        ux, uy = np.zeros(sh[1:]), np.zeros(sh[1:])
    p["fields"] = dict(u_x=ux, u_y=uy, kappa_abs=ka, kappa_flux=kf, emis=em)
    return p


def band_hii_region(nx=512, ny=1024, L_star=1.0e39, steps=1000):
    """Seven-band workload: a cylindrical (R, z) = 1 pc x 2 pc cloud with the
    structure of the line workload (ionised bubble of 0.2 pc in a log-normal
    neutral shell, radial outflow to 30 km/s, dust 0.01 solar) and a star of
    L_star [erg/s] on the axis emitting in the non-IR bands with a Gaussian
    profile of sigma = 3 cells (Section 2.5, single star)."""
    rng = rng_for(6)
    p = base_problem("cyl", nx, ny, 0.0, PC, -PC, PC,
                     ("reflect", "vacuum", "vacuum", "vacuum"), steps=steps)
    p = band_base(p, len(BANDS))
    xc, yc = cell_centres(p)
    r = np.sqrt(xc[None, :] ** 2 + yc[:, None] ** 2)
    g = gaussian_random_field(rng, ny, nx)
    n_H = 100.0 * np.exp(0.8 * g)
    bubble = r < 0.2 * PC
    x_HI = np.where(bubble, 1.0e-4, 1.0)
    ka, kf = band_opacities(n_H, x_HI, 0.01)
    v = 30.0 * KMS * np.minimum(r / (0.2 * PC), 1.0)
    ux = v * xc[None, :] / np.maximum(r, 1e-30)
    uy = v * yc[:, None] / np.maximum(r, 1e-30)
    shape = gaussian_source(p, 0.0, 0.0, 3.0 * PC / nx, L_star)
    em = np.stack([STAR_BAND_SHARE[b] * shape for b in BANDS])
    p["fields"] = dict(u_x=ux, u_y=uy, kappa_abs=ka, kappa_flux=kf, emis=em)
    return p


def filled_state(p, nb, E_peak, seed=0):
    """A developed radiation field to start a run from (instead of E = F = 0),
    physical units: E [N_nu, ny, nx] and F_x, F_y, with

      * a smooth spectrum in the bin index, a core over the central bins and
        exponential wings, spanning ~7 decades over the grid;
      * a smooth spatial envelope exp(-r / 0.3 L) (r from the centre of the
        source plane: the axis mid-height in (R, z), the box centre in the
        slab; L the box diagonal) with a gentle seeded modulation, spanning
        about one more decade; the peak value is E_peak;
      * a reduced flux whose magnitude grows with r and towards the wings,
        |f| = min(1, (r / r_max) (0.4 + 1.2 |u_k|)), so it spans [0, 1] and is
        exactly 1 over the outer far-wing cell-bins, pointing away from the
        centre, turned by a bin-dependent angle.

    Only an input recipe (no part of the transfer method)."""
    rng = np.random.default_rng(np.random.SeedSequence([SEED_BASE, 77, seed]))
    xc, yc = cell_centres(p)
    if p["geom"] == "cyl":
        cx, cy = p["x0"], 0.5 * (p["y0"] + p["y1"])
    else:
        cx, cy = 0.5 * (p["x0"] + p["x1"]), 0.5 * (p["y0"] + p["y1"])
    L = math.hypot(p["x1"] - p["x0"], p["y1"] - p["y0"])
    X, Y = xc[None, :] - cx, yc[:, None] - cy
    r = np.hypot(X, Y)
    ph = rng.uniform(0.0, 2.0 * math.pi, size=2)
    env = np.exp(-r / (0.3 * L)) * (1.0 + 0.3 * np.sin(3.0 * X / L * 2.0 * math.pi + ph[0])
                                    * np.cos(2.0 * Y / L * 2.0 * math.pi + ph[1]))
    env *= 1.0 / float(env.max())
    u = (np.arange(nb) - 0.5 * (nb - 1)) / max(0.5 * nb, 1.0)
    spec = np.exp(-0.5 * (u / 0.08) ** 2) + 1.0e-3 * np.exp(-np.abs(u) / 0.1)
    spec *= 1.0 / float(spec.max())
    E = E_peak * spec[:, None, None] * env[None, :, :]
    rmax = float(r.max())
    fmag = np.minimum(1.0, (r[None, :, :] / rmax) * (0.4 + 1.2 * np.abs(u))[:, None, None])
    ang = np.arctan2(Y, X)[None, :, :] + 0.6 * np.sin(5.0 * u)[:, None, None]
    return E, E * fmag * np.cos(ang), E * fmag * np.sin(ang)


def get_config(cid: int, **kw):
    return {1: config1, 2: config2, 5: config5}[cid](**kw)
