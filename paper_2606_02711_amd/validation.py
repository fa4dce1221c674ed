"""Force multipliers of a run (Sections 3.1 and 3.2): M_F = (c/L) int dV |f| and
M_F,radial = (c/L) int dV f . r_hat, r_hat from the cloud centre at the
origin, and the static-cloud (Test 1) and anisotropic-escape (Test 6) runs on
the GPU."""
import time

import numpy as np

from . import inputs, m1


def force_multipliers(p, force):
    """force: [>=2][ny][nx] total force density (f_x, f_y) [dyn cm^-3]."""
    xc, yc = inputs.cell_centres(p)
    vol = inputs.cell_volumes(p)
    L = float(np.sum(p["fields"]["emis"] * vol))
    fx, fy = force[0], force[1]
    r = np.sqrt(xc[None, :] ** 2 + yc[:, None] ** 2)
    rx = np.where(r > 0, xc[None, :] / np.where(r > 0, r, 1.0), 0.0)
    ry = np.where(r > 0, yc[:, None] / np.where(r > 0, r, 1.0), 0.0)
    c = inputs.C_LIGHT
    mf = c / L * float(np.sum(np.hypot(fx, fy) * vol))
    mfr = c / L * float(np.sum((fx * rx + fy * ry) * vol))
    return mf, mfr


def run_cone(n=256, prec="fp32", t_max=None, log=None, checkpoints=4, problem=None,
             name="cone"):
    """Cone test to t_max (default 4 max((a tau)^1/3, 3) R_cl/c); returns the
    multipliers at evenly spaced checkpoints and the final ones.  `problem`
    runs another cloud (e.g. inputs.static_sphere) the same way."""
    p = inputs.cone_cloud(n) if problem is None else problem
    g = m1.M1Grid(p, prec=prec)
    t_end = p["t_max"] if t_max is None else t_max
    steps = int(np.ceil(t_end / g.dt))
    hist = []
    t0 = time.perf_counter()
    done = 0
    for q in range(1, checkpoints + 1):
        target = steps * q // checkpoints
        while done < target:
            k = min(target - done, 4096)
            g.step(k)
            done += k
        g.sync()
        f = g.force().cpu().numpy()
        mf, mfr = force_multipliers(p, f)
        hist.append((done, done * g.dt * inputs.C_LIGHT / p["R_cl"], mf, mfr))
        if log:
            log(f"[{name} {n}^2 {prec}] step {done}/{steps} t={hist[-1][1]:.1f} R_cl/c "
                f"M_F={mf:.3f} M_F,radial={mfr:.3f}")
    wall = time.perf_counter() - t0
    g.free()
    return dict(n=n, prec=prec, steps=steps, dt=g.dt, seconds=wall, M_F=hist[-1][2],
                M_F_radial=hist[-1][3], history=hist)


def energy_budget(p, g):
    """Steady-state energy budget of a grid g of problem p (Section 3.1, the
    escape-fraction test), over the emitted luminosity: (absorbed, escaped
    lower, escaped upper).  Absorbed: c alpha_abs int E dnu over the volume
    (alpha_abs the continuum absorption coefficient; no destruction).
    Escaped: the outflow through the vacuum faces x = x1 and y = y1 (the
    other sides must be reflecting), bracketed from the boundary cells'
    values: below by c F.n, above by the corrected GLF outflow with an empty
    ghost and no opacity, c (F.n + E)/2, at the cell centre (where E exceeds
    its face value).  An energy-conserving step has absorbed + escaped = 1
    inside the bracket."""
    nu, dnu = m1.frequency_grid(g.cfg)
    E, Fx, Fy = [t.cpu().numpy() for t in g.state()]
    Eint = np.tensordot(dnu, E, axes=(0, 0))
    Fxi = np.tensordot(dnu, Fx, axes=(0, 0))
    Fyi = np.tensordot(dnu, Fy, axes=(0, 0))
    vol = inputs.cell_volumes(p)
    L = float(np.sum(p["fields"]["emis"] * vol))
    c = inputs.C_LIGHT
    absorbed = c * float(np.sum(p["fields"]["alpha_abs"] * Eint * vol))
    xe, ye = inputs.edges(p)
    dz = np.diff(ye)
    if p["geom"] == "cyl":
        a_x = 2.0 * np.pi * xe[-1] * dz                      # outer cylinder, per row
        a_y = np.pi * (xe[1:] ** 2 - xe[:-1] ** 2)           # top annuli, per column
    else:
        a_x = dz
        a_y = np.diff(xe)
    fn = float(np.sum(Fxi[:, -1] * a_x)) + float(np.sum(Fyi[-1, :] * a_y))
    en = float(np.sum(Eint[:, -1] * a_x)) + float(np.sum(Eint[-1, :] * a_y))
    return absorbed / L, c * fn / L, 0.5 * c * (fn + en) / L
