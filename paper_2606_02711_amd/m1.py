"""Python binding of libm1lya.so (argument marshalling only).

Every step of the method runs in the HIP library; PyTorch only provides the
device workspace, the output buffers and the stream.  Importing this module
without a built library, or using it without a GPU, raises: there is no CPU
fallback.

Names follow include/m1lya.h: m1_init, m1_step, m1_force, m1_solve_steady,
m1_residual, m1_get_state, m1_set_state, m1_batch_*, ...  The class
`M1Grid` wraps one handle for a problem dict built by `inputs`; `M1Batch`
wraps a batch of handles advanced together.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("M1LYA_LIB", os.path.join(HERE, "libm1lya.so"))

M1_OK, M1_EINVAL, M1_ENOMEM, M1_EDEVICE, M1_ENOTCONV, M1_ESTATE, M1_EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
M1_CART2D, M1_CYL_RZ = 0, 1
M1_BC_VACUUM, M1_BC_REFLECT = 0, 1
M1_FP64, M1_FP32 = 0, 1


class M1Error(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"m1 error {code}: {msg}")
        self.code = code


class m1_config(ctypes.Structure):
    _fields_ = [("geom", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("x0", ctypes.c_double), ("x1", ctypes.c_double), ("y0", ctypes.c_double),
                ("y1", ctypes.c_double), ("bc", ctypes.c_int32 * 4), ("T_min", ctypes.c_double),
                ("q", ctypes.c_double), ("half_width", ctypes.c_double),
                ("c_tilde", ctypes.c_double), ("cfl", ctypes.c_double),
                ("recoil", ctypes.c_int32), ("doppler", ctypes.c_int32),
                ("prec", ctypes.c_int32), ("fp64_tau", ctypes.c_double),
                ("active_frac", ctypes.c_double), ("substep_rule", ctypes.c_int32),
                ("flux", ctypes.c_int32)]


class m1_fields(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in
                ("n_HI", "T", "u_x", "u_y", "alpha_abs", "alpha_flux", "p_d", "emis")] + \
               [("on_device", ctypes.c_int32)]


class m1_band_fields(ctypes.Structure):
    _fields_ = [("u_x", ctypes.c_void_p), ("u_y", ctypes.c_void_p),
                ("kappa_abs", ctypes.c_void_p), ("kappa_flux", ctypes.c_void_p),
                ("emis", ctypes.c_void_p), ("on_device", ctypes.c_int32)]


class m1_server_config(ctypes.Structure):
    _fields_ = [("prec", ctypes.c_int32), ("batched", ctypes.c_int32),
                ("max_resident", ctypes.c_int32), ("check_every", ctypes.c_int32),
                ("use_graph", ctypes.c_int32), ("max_bypass", ctypes.c_int32)]


class m1_request_info(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int64), ("state", ctypes.c_int32), ("error", ctypes.c_int32),
                ("steps", ctypes.c_int64), ("residual", ctypes.c_double),
                ("admit_round", ctypes.c_int64), ("finish_round", ctypes.c_int64),
                ("ws_bytes", ctypes.c_size_t)]


FIELDS_CB = ctypes.CFUNCTYPE(ctypes.c_int32, ctypes.c_void_p, ctypes.c_int64,
                             ctypes.POINTER(m1_fields))
REQ_STATES = ("queued", "resident", "converged", "not_converged", "rejected", "failed")

_lib = None


def lib():
    """Load libm1lya.so; raises if it was not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: run __graft_entry__.build() first")
    L = ctypes.CDLL(LIB_PATH)
    P, I32, I64, D, VP = ctypes.POINTER, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
    sig = {
        "m1_default_config": (I32, [P(m1_config)]),
        "m1_num_bins": (I32, [P(m1_config), P(I32)]),
        "m1_frequency_grid": (I32, [P(m1_config), VP, VP]),
        "m1_workspace_bytes": (I32, [P(m1_config), I64, P(ctypes.c_size_t)]),
        "m1_count_temperature_classes": (I32, [VP, I64, P(I64)]),
        "m1_init": (I32, [P(m1_config), P(m1_fields), VP, ctypes.c_size_t, VP, P(VP)]),
        "m1_step": (I32, [VP, I32, P(D)]),
        "m1_force": (I32, [VP, VP, VP, VP, VP]),
        "m1_solve_steady": (I32, [VP, D, I64, I32, P(I64), P(D)]),
        "m1_residual": (I32, [VP, P(D)]),
        "m1_residuals": (I32, [P(VP), I32, VP]),
        "m1_get_state": (I32, [VP, VP, VP, VP]),
        "m1_set_state": (I32, [VP, VP, VP, VP]),
        "m1_get_state_region": (I32, [VP, I32, I32, I32, I32, VP, VP, VP]),
        "m1_get_info": (I32, [VP, P(D), P(I32), P(I32), P(I64), P(I32)]),
        "m1_active_bins": (I32, [VP, VP, P(I32)]),
        "m1_set_c_tilde": (I32, [VP, D]),
        "m1_dynamic_c_tilde": (I32, [P(m1_config), P(m1_fields), VP, D, VP, VP, P(D)]),
        "m1_dynamic_c_tilde_noalloc": (I32, [P(m1_config), P(m1_fields), VP, D, VP, P(D)]),
        "m1_band_workspace_bytes": (I32, [P(m1_config), I32, P(ctypes.c_size_t)]),
        "m1_band_init": (I32, [P(m1_config), I32, P(m1_band_fields), VP, ctypes.c_size_t, VP,
                               P(VP)]),
        "m1_batch_workspace_bytes": (I32, [P(VP), I32, P(ctypes.c_size_t)]),
        "m1_batch_init": (I32, [P(VP), I32, VP, ctypes.c_size_t, I32, P(VP)]),
        "m1_batch_step": (I32, [VP, I32]),
        "m1_batch_info": (I32, [VP, P(I32), P(D), I32]),
        "m1_batch_free": (I32, [VP]),
        "m1_batch_set_tile": (I32, [VP, I32]),
        "m1_batch_workspace_bound": (I32, [I32, I32, P(ctypes.c_size_t)]),
        "m1_server_create": (I32, [P(m1_server_config), VP, ctypes.c_size_t, VP, FIELDS_CB, VP,
                                   P(VP)]),
        "m1_server_submit": (I32, [VP, P(m1_config), I64, D, I64, P(I64)]),
        "m1_server_run": (I32, [VP, I32, P(I32)]),
        "m1_server_poll": (I32, [VP, P(m1_request_info), I32, P(I32)]),
        "m1_server_handle": (I32, [VP, I64, P(VP)]),
        "m1_server_release": (I32, [VP, I64]),
        "m1_server_stats": (I32, [VP, P(I64), P(I64), P(I64), P(I64), P(ctypes.c_size_t),
                                  P(ctypes.c_size_t)]),
        "m1_server_free": (I32, [VP]),
        "m1_step_profiled": (I32, [VP, I32, P(D)]),
        "m1_sync": (I32, [VP]),
        "m1_free": (I32, [VP]),
        "m1_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def exported_symbols():
    return ["m1_default_config", "m1_num_bins", "m1_frequency_grid", "m1_workspace_bytes",
            "m1_count_temperature_classes", "m1_init", "m1_step", "m1_force",
            "m1_solve_steady", "m1_residual", "m1_residuals", "m1_get_state", "m1_set_state", "m1_get_state_region", "m1_get_info",
            "m1_active_bins", "m1_set_c_tilde", "m1_dynamic_c_tilde",
            "m1_dynamic_c_tilde_noalloc", "m1_band_workspace_bytes", "m1_band_init",
            "m1_batch_workspace_bytes", "m1_batch_init", "m1_batch_step", "m1_batch_info",
            "m1_batch_free", "m1_batch_set_tile", "m1_batch_workspace_bound",
            "m1_server_create", "m1_server_submit", "m1_server_run", "m1_server_poll",
            "m1_server_handle", "m1_server_release", "m1_server_stats", "m1_server_free",
            "m1_step_profiled", "m1_sync", "m1_free", "m1_last_error"]


def check(code):
    if code != M1_OK:
        raise M1Error(code, lib().m1_last_error().decode())
    return code


# ----------------------------------------------------------------- config
BC = {"vacuum": M1_BC_VACUUM, "reflect": M1_BC_REFLECT}
FLUX = {"glf": 0, "hll_eig": 1}          # m1_flux


def make_config(p, prec="fp64", fp64_tau=float("inf")):
    c = m1_config()
    check(lib().m1_default_config(ctypes.byref(c)))
    c.geom = M1_CYL_RZ if p["geom"] == "cyl" else M1_CART2D
    c.nx, c.ny = int(p["nx"]), int(p["ny"])
    c.x0, c.x1, c.y0, c.y1 = float(p["x0"]), float(p["x1"]), float(p["y0"]), float(p["y1"])
    for s in range(4):
        c.bc[s] = BC[p["bc"][s]]
    c.T_min, c.q, c.half_width = float(p["T_min"]), float(p["q"]), float(p["half_width"])
    c.c_tilde, c.cfl = float(p["c_tilde"]), float(p["cfl"])
    c.recoil, c.doppler = int(p.get("recoil", 1)), int(p.get("doppler", 1))
    c.prec = M1_FP32 if prec == "fp32" else M1_FP64
    c.fp64_tau = float(fp64_tau)
    c.active_frac = float(p.get("active_frac", 0.0))
    c.substep_rule = int(p.get("substep_rule", 0))
    c.flux = FLUX[p.get("flux", "glf")]
    return c


def num_bins(cfg):
    n = ctypes.c_int32()
    check(lib().m1_num_bins(ctypes.byref(cfg), ctypes.byref(n)))
    return n.value


def frequency_grid(cfg):
    """(nu_centre, dnu) [Hz] of cfg's bins (m1_frequency_grid), numpy arrays."""
    n = num_bins(cfg)
    nu = np.zeros(n)
    dnu = np.zeros(n)
    check(lib().m1_frequency_grid(ctypes.byref(cfg), nu.ctypes.data, dnu.ctypes.data))
    return nu, dnu


def workspace_bytes(cfg, n_classes=0):
    b = ctypes.c_size_t()
    check(lib().m1_workspace_bytes(ctypes.byref(cfg), int(n_classes), ctypes.byref(b)))
    return b.value


def count_temperature_classes(T):
    T = np.ascontiguousarray(T, dtype=np.float64).ravel()
    n = ctypes.c_int64()
    check(lib().m1_count_temperature_classes(T.ctypes.data, T.size, ctypes.byref(n)))
    return n.value


FIELD_ORDER = ("n_HI", "T", "u_x", "u_y", "alpha_abs", "alpha_flux", "p_d", "emis")


def dynamic_c_tilde(p, cs, c_prev=0.0, noalloc=False):
    """The reduced speed of light the paper chooses for the medium of p with
    sound speeds cs [cm/s] (m1_dynamic_c_tilde, or with noalloc
    m1_dynamic_c_tilde_noalloc), the fields copied to the GPU."""
    torch = _torch()
    cfg = make_config(p)
    f = p["fields"]
    dev = [torch.as_tensor(np.ascontiguousarray(f[n], dtype=np.float64).ravel(), device="cuda")
           for n in FIELD_ORDER]
    d_cs = torch.as_tensor(np.ascontiguousarray(cs, dtype=np.float64).ravel(), device="cuda")
    work = torch.empty(1024, dtype=torch.float64, device="cuda")
    fl = m1_fields()
    for n, a in zip(FIELD_ORDER, dev):
        setattr(fl, n, a.data_ptr())
    fl.on_device = 1
    torch.cuda.current_stream().synchronize()      # inputs written on torch's stream
    out = ctypes.c_double()
    if noalloc:
        check(lib().m1_dynamic_c_tilde_noalloc(ctypes.byref(cfg), ctypes.byref(fl),
                                               d_cs.data_ptr(), float(c_prev), None,
                                               ctypes.byref(out)))
    else:
        check(lib().m1_dynamic_c_tilde(ctypes.byref(cfg), ctypes.byref(fl), d_cs.data_ptr(),
                                       float(c_prev), work.data_ptr(), None, ctypes.byref(out)))
    return out.value


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no GPU: the M1 library runs on the device only")
    return torch


class M1Grid:
    """One problem on the GPU: workspace, handle and outputs.

    p: problem dict (see inputs.py); prec: "fp64" or "fp32"."""

    def __init__(self, p, prec="fp64", fp64_tau=float("inf"), stream=None, workspace=None):
        torch = _torch()
        self.p = p
        self.prec = prec
        self.cfg = make_config(p, prec, fp64_tau)
        f = p["fields"]
        host = [np.ascontiguousarray(f[n], dtype=np.float64).ravel() for n in FIELD_ORDER]
        self._host = host
        self.ncls = count_temperature_classes(host[1])
        self.ws_bytes = workspace_bytes(self.cfg, self.ncls)
        self.nb = num_bins(self.cfg)
        self.nx, self.ny = self.cfg.nx, self.cfg.ny
        self.ncell = self.nx * self.ny
        if workspace is None:
            workspace = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device="cuda")
        self.ws = workspace
        base = workspace.data_ptr()
        self._ws_ptr = (base + 255) & ~255
        if self._ws_ptr + self.ws_bytes > base + workspace.numel():
            raise ValueError("workspace tensor too small")
        fl = m1_fields()
        for n, a in zip(FIELD_ORDER, host):
            setattr(fl, n, a.ctypes.data)
        fl.on_device = 0
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = ctypes.c_void_p()
        check(lib().m1_init(ctypes.byref(self.cfg), ctypes.byref(fl), self._ws_ptr,
                            self.ws_bytes, self.stream.cuda_stream, ctypes.byref(h)))
        self.h = h
        dt, nnu, pr, nc, e2 = (ctypes.c_double(), ctypes.c_int32(), ctypes.c_int32(),
                               ctypes.c_int64(), ctypes.c_int32())
        check(lib().m1_get_info(h, ctypes.byref(dt), ctypes.byref(nnu), ctypes.byref(pr),
                                ctypes.byref(nc), ctypes.byref(e2)))
        self.dt, self.scale_exp2 = dt.value, e2.value
        self.dtype = torch.float32 if prec == "fp32" else torch.float64
        self.t = 0.0

    # -- stepping
    def step(self, n=1):
        t = ctypes.c_double()
        check(lib().m1_step(self.h, int(n), ctypes.byref(t)))
        self.t = t.value
        return self

    def step_profiled(self, n):
        """Steps n times; returns summed device ms of (advection, frequency) kernels."""
        ms = (ctypes.c_double * 2)()
        check(lib().m1_step_profiled(self.h, int(n), ms))
        self.t += n * self.dt
        return ms[0], ms[1]

    def solve_steady(self, rel_tol=1e-6, max_steps=100000, check_every=16):
        done, r = ctypes.c_int64(), ctypes.c_double()
        code = lib().m1_solve_steady(self.h, float(rel_tol), int(max_steps), int(check_every),
                                     ctypes.byref(done), ctypes.byref(r))
        if code not in (M1_OK, M1_ENOTCONV):
            check(code)
        return code == M1_OK, done.value, r.value

    def residual(self):
        r = ctypes.c_double()
        check(lib().m1_residual(self.h, ctypes.byref(r)))
        return r.value

    def sync(self):
        check(lib().m1_sync(self.h))

    # -- outputs (torch tensors on the device)
    def state(self):
        torch = _torch()
        shape = (self.nb, self.ny, self.nx)
        E = torch.empty(shape, dtype=torch.float64, device="cuda")
        Fx = torch.empty_like(E)
        Fy = torch.empty_like(E)
        check(lib().m1_get_state(self.h, E.data_ptr(), Fx.data_ptr(), Fy.data_ptr()))
        return E, Fx, Fy

    def state_region(self, i0, i1, j0, j1):
        """E, Fx, Fy of cells i0 <= i < i1, j0 <= j < j1, all bins (float64)."""
        torch = _torch()
        E = torch.empty((self.nb, j1 - j0, i1 - i0), dtype=torch.float64, device="cuda")
        Fx = torch.empty_like(E)
        Fy = torch.empty_like(E)
        check(lib().m1_get_state_region(self.h, int(i0), int(i1), int(j0), int(j1), E.data_ptr(),
                                        Fx.data_ptr(), Fy.data_ptr()))
        return E, Fx, Fy

    def set_state(self, E, Fx, Fy):
        torch = _torch()
        conv = lambda a: torch.as_tensor(a, dtype=torch.float64, device="cuda").contiguous()
        self._set = (conv(E), conv(Fx), conv(Fy))
        torch.cuda.current_stream().synchronize()     # inputs written on torch's stream
        check(lib().m1_set_state(self.h, *[t.data_ptr() for t in self._set]))
        self.sync()

    def set_c_tilde(self, c_tilde):
        """New reduced speed of light, state kept (m1_set_c_tilde); updates dt."""
        check(lib().m1_set_c_tilde(self.h, float(c_tilde)))
        dt = ctypes.c_double()
        check(lib().m1_get_info(self.h, ctypes.byref(dt), None, None, None, None))
        self.dt = dt.value
        self.cfg.c_tilde = float(c_tilde)

    def active_bins(self):
        """Flags (int32 [N_nu]) of the bins the last step advected."""
        f = np.zeros(self.nb, dtype=np.int32)
        n = ctypes.c_int32()
        check(lib().m1_active_bins(self.h, f.ctypes.data, ctypes.byref(n)))
        return f

    def force(self, out=None):
        torch = _torch()
        if out is None:
            out = torch.empty((4, self.ny, self.nx), dtype=torch.float64, device="cuda")
        check(lib().m1_force(self.h, out[0].data_ptr(), out[1].data_ptr(), out[2].data_ptr(),
                             out[3].data_ptr()))
        self.sync()                                   # written on the handle's stream
        return out

    def free(self):
        if getattr(self, "h", None) is not None and self.h.value:
            lib().m1_sync(self.h)                     # work in flight uses the workspace
            lib().m1_free(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


BAND_FIELDS = ("u_x", "u_y", "kappa_abs", "kappa_flux", "emis")


def make_band_config(p, prec="fp64"):
    """Config of a band problem (geometry keys, c_tilde, cfl; the frequency
    grid fields keep their defaults)."""
    c = m1_config()
    check(lib().m1_default_config(ctypes.byref(c)))
    c.geom = M1_CYL_RZ if p["geom"] == "cyl" else M1_CART2D
    c.nx, c.ny = int(p["nx"]), int(p["ny"])
    c.x0, c.x1, c.y0, c.y1 = float(p["x0"]), float(p["x1"]), float(p["y0"]), float(p["y1"])
    for q in range(4):
        c.bc[q] = BC[p["bc"][q]]
    c.c_tilde, c.cfl = float(p["c_tilde"]), float(p["cfl"])
    c.prec = M1_FP32 if prec == "fp32" else M1_FP64
    return c


def band_workspace_bytes(cfg, n_band):
    b = ctypes.c_size_t()
    check(lib().m1_band_workspace_bytes(ctypes.byref(cfg), int(n_band), ctypes.byref(b)))
    return b.value


class BandGrid(M1Grid):
    """A grid of broad bands on the GPU (m1_band_init); stepping, state,
    force and residual as for M1Grid, with bands in place of bins.

    p: band problem dict (see inputs.band_random_small, inputs.band_hii_region)."""

    def __init__(self, p, prec="fp64", stream=None, workspace=None):
        torch = _torch()
        self.p = p
        self.prec = prec
        self.cfg = make_band_config(p, prec)
        self.nb = int(p["n_band"])
        self.nx, self.ny = self.cfg.nx, self.cfg.ny
        self.ncell = self.nx * self.ny
        f = p["fields"]
        host = [np.ascontiguousarray(f[n], dtype=np.float64).ravel() for n in BAND_FIELDS]
        if host[0].size != self.ncell or host[1].size != self.ncell or \
                any(h.size != self.nb * self.ncell for h in host[2:]):
            raise ValueError("band fields must be (ny, nx) velocities and (n_band, ny, nx) tables")
        self._host = host
        self.ws_bytes = band_workspace_bytes(self.cfg, self.nb)
        if workspace is None:
            workspace = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device="cuda")
        self.ws = workspace
        base = workspace.data_ptr()
        self._ws_ptr = (base + 255) & ~255
        if self._ws_ptr + self.ws_bytes > base + workspace.numel():
            raise ValueError("workspace tensor too small")
        fl = m1_band_fields()
        for n, a in zip(BAND_FIELDS, host):
            setattr(fl, n, a.ctypes.data)
        fl.on_device = 0
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = ctypes.c_void_p()
        check(lib().m1_band_init(ctypes.byref(self.cfg), self.nb, ctypes.byref(fl), self._ws_ptr,
                                 self.ws_bytes, self.stream.cuda_stream, ctypes.byref(h)))
        self.h = h
        dt, nnu, pr, nc, e2 = (ctypes.c_double(), ctypes.c_int32(), ctypes.c_int32(),
                               ctypes.c_int64(), ctypes.c_int32())
        check(lib().m1_get_info(h, ctypes.byref(dt), ctypes.byref(nnu), ctypes.byref(pr),
                                ctypes.byref(nc), ctypes.byref(e2)))
        self.dt, self.scale_exp2 = dt.value, e2.value
        self.dtype = torch.float32 if prec == "fp32" else torch.float64
        self.t = 0.0


class M1Batch:
    """Grids of one precision on one stream, advanced together by persistent
    launches (results bitwise identical to stepping each grid alone)."""

    def __init__(self, grids, use_graph=True):
        torch = _torch()
        self.grids = list(grids)
        n = len(self.grids)
        self._arr = (ctypes.c_void_p * n)(*[g.h.value for g in self.grids])
        b = ctypes.c_size_t()
        check(lib().m1_batch_workspace_bytes(self._arr, n, ctypes.byref(b)))
        self.ws = torch.empty(b.value + 256, dtype=torch.uint8, device="cuda")
        ptr = (self.ws.data_ptr() + 255) & ~255
        h = ctypes.c_void_p()
        check(lib().m1_batch_init(self._arr, n, ptr, b.value, int(bool(use_graph)),
                                  ctypes.byref(h)))
        self.h = h

    def step(self, n=1):
        check(lib().m1_batch_step(self.h, int(n)))
        for g in self.grids:
            g.t += n * g.dt
        return self

    def info(self):
        """(tile variant chosen: 7, 14, 28, 49 bins per block or -1 fused; 0 while
        tuning; ms per step of each of the five variants)."""
        bk = ctypes.c_int32()
        ms = (ctypes.c_double * 5)()
        check(lib().m1_batch_info(self.h, ctypes.byref(bk), ms, 5))
        return bk.value, list(ms)

    def set_tile(self, bins_per_block):
        check(lib().m1_batch_set_tile(self.h, int(bins_per_block)))

    def free(self):
        if getattr(self, "h", None) is not None and self.h.value:
            lib().m1_batch_free(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def step_batched(grids, nsteps, use_graph=True):
    """Advances the grids together by nsteps steps (one-off batch)."""
    b = M1Batch(grids, use_graph=use_graph)
    b.step(nsteps)
    for g in grids:
        g.sync()
    b.free()


class M1Server:
    """Continuous-batching engine for steady-state solves (m1_server_*).

    Requests are problem dicts, or zero-argument callables returning one
    (called at submission for the configuration and again at admission for
    the fields, so a long queue holds no field arrays)."""

    def __init__(self, arena_bytes, prec="fp32", batched=True, max_resident=64, check_every=16,
                 use_graph=True, max_bypass=8, stream=None):
        torch = _torch()
        self.prec = prec
        self.stream = stream if stream is not None else torch.cuda.Stream()
        self.arena = torch.empty(int(arena_bytes) + 256, dtype=torch.uint8, device="cuda")
        ptr = (self.arena.data_ptr() + 255) & ~255
        c = m1_server_config(M1_FP32 if prec == "fp32" else M1_FP64, int(bool(batched)),
                             int(max_resident), int(check_every), int(bool(use_graph)),
                             int(max_bypass))
        self._cb = FIELDS_CB(self._fields)
        self._source = {}        # id -> problem dict or factory, until admission
        self._meta = {}          # id -> (nb, ny, nx)
        self._keep = {}          # host arrays of requests admitted in the current run call
        self._cb_error = None
        h = ctypes.c_void_p()
        check(lib().m1_server_create(ctypes.byref(c), ptr, int(arena_bytes),
                                     self.stream.cuda_stream, self._cb, None, ctypes.byref(h)))
        self.h = h

    def _fields(self, user, rid, out):
        try:
            src = self._source.pop(rid)
            p = src() if callable(src) else src
            host = [np.ascontiguousarray(p["fields"][n], dtype=np.float64).ravel()
                    for n in FIELD_ORDER]
            self._keep[rid] = host
            fl = out.contents
            for n, a in zip(FIELD_ORDER, host):
                setattr(fl, n, a.ctypes.data)
            fl.on_device = 0
            return M1_OK
        except Exception as e:           # reported as a failed request
            self._cb_error = e
            return M1_EINVAL

    def submit(self, p, rel_tol=1e-6, max_steps=100000, meta=None, n_classes=None):
        """meta (a problem dict whose fields may be empty) and n_classes, when
        given, spare building the fields at submission."""
        if meta is None or n_classes is None:
            meta = p() if callable(p) else p
            n_classes = count_temperature_classes(meta["fields"]["T"])
        cfg = make_config(meta, self.prec)
        ncls = int(n_classes)
        rid = ctypes.c_int64()
        check(lib().m1_server_submit(self.h, ctypes.byref(cfg), ncls, float(rel_tol),
                                     int(max_steps), ctypes.byref(rid)))
        self._source[rid.value] = p
        self._meta[rid.value] = (num_bins(cfg), cfg.ny, cfg.nx)
        return rid.value

    def run(self, rounds=1):
        busy = ctypes.c_int32()
        try:
            check(lib().m1_server_run(self.h, int(rounds), ctypes.byref(busy)))
        finally:
            self._keep.clear()
        return busy.value

    def poll(self, cap=1024):
        arr = (m1_request_info * cap)()
        n = ctypes.c_int32()
        check(lib().m1_server_poll(self.h, arr, cap, ctypes.byref(n)))
        out = []
        for i in range(n.value):
            r = arr[i]
            out.append(dict(id=r.id, state=REQ_STATES[r.state], error=r.error, steps=r.steps,
                            residual=r.residual, admit_round=r.admit_round,
                            finish_round=r.finish_round, ws_bytes=r.ws_bytes))
            self._source.pop(r.id, None)
        return out

    def _handle(self, rid):
        h = ctypes.c_void_p()
        check(lib().m1_server_handle(self.h, int(rid), ctypes.byref(h)))
        return h

    def state(self, rid):
        torch = _torch()
        E = torch.empty(self._meta[rid], dtype=torch.float64, device="cuda")
        Fx, Fy = torch.empty_like(E), torch.empty_like(E)
        check(lib().m1_get_state(self._handle(rid), E.data_ptr(), Fx.data_ptr(), Fy.data_ptr()))
        return E, Fx, Fy

    def force(self, rid):
        torch = _torch()
        h = self._handle(rid)
        _, ny, nx = self._meta[rid]
        out = torch.empty((4, ny, nx), dtype=torch.float64, device="cuda")
        check(lib().m1_force(h, out[0].data_ptr(), out[1].data_ptr(), out[2].data_ptr(),
                             out[3].data_ptr()))
        check(lib().m1_sync(h))
        return out

    def release(self, rid):
        check(lib().m1_server_release(self.h, int(rid)))
        self._meta.pop(rid, None)

    def stats(self):
        v = [ctypes.c_int64() for _ in range(4)] + [ctypes.c_size_t(), ctypes.c_size_t()]
        check(lib().m1_server_stats(self.h, *[ctypes.byref(x) for x in v]))
        keys = ("queued", "resident", "finished", "rounds", "arena_used", "largest_free")
        return {k: x.value for k, x in zip(keys, v)}

    def free(self):
        if getattr(self, "h", None) is not None and self.h.value:
            lib().m1_server_free(self.h)
            self.h = ctypes.c_void_p()
        # the callback refers back to this object (a cycle): drop it and the
        # arena, so the arena's memory returns without waiting for the collector
        self._cb = None
        self.arena = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass
