"""Force multipliers of a run (Section 4): M_F = (c/L) int dV |f| and
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
