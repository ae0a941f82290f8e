"""FP64 CPU oracle of the phase-field DUGKS step (arXiv:1810.07802).

TEST INFRASTRUCTURE. Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package. It shares no code
with the HIP path in ``paper_1810_07802_amd`` and neither imports the other.

The numerics live in ``dugks_oracle.c`` (plain C, IEEE double, built with
``-ffp-contract=off``); this module only builds and loads it and marshals
numpy arrays. Parameter dictionaries use the keys of ``PARAM_FIELDS``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dugks_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

VISC = {"uniform_nu": 0, "reciprocal": 1, "linear": 2}
GRAV = {"rho_g": 0, "buoyancy": 1}
VEL = {"uniform": 0, "rotation": 1, "shear": 2, "deform": 3}
RECON = {"central": 0, "upwind": 1}


class OrcParams(C.Structure):
    _fields_ = [
        ("phi_H", C.c_double), ("phi_L", C.c_double),
        ("rho_H", C.c_double), ("rho_L", C.c_double),
        ("mu_H", C.c_double), ("mu_L", C.c_double),
        ("nu", C.c_double),
        ("visc_mode", C.c_int),
        ("sigma", C.c_double), ("W", C.c_double), ("M", C.c_double),
        ("gx", C.c_double), ("gy", C.c_double),
        ("gravity_form", C.c_int),
        ("Gx", C.c_double), ("Gy", C.c_double),
        ("cfl", C.c_double),
        ("walls_y", C.c_int),
        ("vel_kind", C.c_int),
        ("U0", C.c_double), ("L0", C.c_double), ("T_period", C.c_double),
        ("recon", C.c_int),
        ("eps_n", C.c_double),
    ]


PARAM_DEFAULTS = dict(
    phi_H=1.0, phi_L=0.0, rho_H=1.0, rho_L=1.0, mu_H=0.1, mu_L=0.1, nu=0.1,
    visc="uniform_nu", sigma=0.0, W=4.0, M=0.1, gx=0.0, gy=0.0,
    gravity="rho_g", Gx=0.0, Gy=0.0, cfl=0.5, walls_y=False,
    vel="uniform", U0=0.0, L0=1.0, T_period=1.0, recon="central", eps_n=1e-6,
)


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (OpenMP over rows, strict IEEE)."""
    if force or not os.path.exists(_LIB_PATH) or (
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)):
        cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp",
               "-ffp-contract=off", "-fno-fast-math", "-Wall",
               "-o", _LIB_PATH + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_LIB_PATH)
        dp = C.POINTER(C.c_double)
        L.orc_create.restype = C.c_void_p
        L.orc_create.argtypes = [C.c_int, C.c_int, C.c_int, C.POINTER(OrcParams)]
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_set_params.argtypes = [C.c_void_p, C.POINTER(OrcParams)]
        L.orc_init.argtypes = [C.c_void_p, dp, dp, dp, dp]
        L.orc_step.argtypes = [C.c_void_p, C.c_int]
        L.orc_macros.argtypes = [C.c_void_p, dp, dp, dp, dp, dp]
        L.orc_cell_fields.argtypes = [C.c_void_p, dp, dp, dp, dp]
        L.orc_get_state.argtypes = [C.c_void_p, dp, dp, dp, C.POINTER(C.c_long)]
        L.orc_set_state.argtypes = [C.c_void_p, dp, dp, dp, C.c_long]
        L.orc_time.restype = C.c_double
        L.orc_time.argtypes = [C.c_void_p]
        L.orc_step_count.restype = C.c_long
        L.orc_step_count.argtypes = [C.c_void_p]
        L.orc_derived.argtypes = [C.c_void_p, dp]
        L.orc_feq.argtypes = [C.c_double] * 3 + [dp]
        L.orc_sf.argtypes = [C.c_double] * 5 + [dp]
        L.orc_geq.argtypes = [C.c_double] * 4 + [dp]
        L.orc_sg.argtypes = [C.c_double] * 6 + [dp]
        L.orc_bar_plus.argtypes = [C.c_double, C.c_double, dp, dp, dp, dp, dp]
        L.orc_face_df.argtypes = [C.c_double, C.c_double, dp, dp, dp, dp]
        L.orc_stencils.argtypes = [C.c_int, C.c_int, C.c_int, dp, dp, dp, dp, dp, dp]
        L.orc_recon.argtypes = [C.c_int] * 3 + [dp, dp, C.c_int, C.c_double, C.c_int, dp, dp, dp]
        L.orc_set_mesh.restype = C.c_int
        L.orc_set_mesh.argtypes = [C.c_void_p, dp, dp]
        _lib = L
    return _lib


def _ptr(a):
    if a is None:
        return None
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def make_params(d: dict) -> OrcParams:
    p = dict(PARAM_DEFAULTS)
    unknown = set(d) - set(p)
    if unknown:
        raise KeyError(f"unknown parameter keys: {sorted(unknown)}")
    p.update(d)
    s = OrcParams()
    for k in ("phi_H", "phi_L", "rho_H", "rho_L", "mu_H", "mu_L", "nu",
              "sigma", "W", "M", "gx", "gy", "Gx", "Gy", "cfl", "U0", "L0",
              "T_period", "eps_n"):
        setattr(s, k, float(p[k]))
    s.visc_mode = VISC[p["visc"]]
    s.gravity_form = GRAV[p["gravity"]]
    s.walls_y = int(bool(p["walls_y"]))
    s.vel_kind = VEL[p["vel"]]
    s.recon = RECON[p["recon"]]
    return s


class Sim:
    """One oracle simulation. ``model`` is "coupled" or "ac" (interface only)."""

    def __init__(self, nx: int, ny: int, params: dict, model: str = "coupled"):
        self.nx, self.ny = int(nx), int(ny)
        self.model = model
        self._p = make_params(params)
        self._h = lib().orc_create(self.nx, self.ny, 1 if model == "coupled" else 0,
                                   C.byref(self._p))
        if not self._h:
            raise ValueError("oracle rejected the grid/parameters")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_destroy(h)
            self._h = None

    @property
    def n(self):
        return self.nx * self.ny

    def init(self, phi, u=None, v=None, p=None):
        shape = (self.ny, self.nx)
        arrs = [_f64(a) for a in (phi, u, v, p)]
        for a in arrs:
            if a is not None and a.shape != shape:
                raise ValueError(f"field shape {a.shape} != {shape}")
        self._keep = arrs
        lib().orc_init(self._h, *[_ptr(a) for a in arrs])

    def set_mesh(self, dx=None, dy=None):
        """Stretched mesh of cell widths dx[nx], dy[ny] (None: unit widths on
        that axis; both None: the unit mesh)."""
        self._mesh = (_f64(dx), _f64(dy))
        if lib().orc_set_mesh(self._h, _ptr(self._mesh[0]), _ptr(self._mesh[1])) != 0:
            raise ValueError("mesh widths must be > 0")

    def set_params(self, params: dict):
        """New parameters from the next step on (the state is kept)."""
        self._p = make_params(params)
        lib().orc_set_params(self._h, C.byref(self._p))

    def step(self, nsteps: int = 1):
        lib().orc_step(self._h, int(nsteps))

    def macros(self):
        shape = (self.ny, self.nx)
        out = [np.empty(shape) for _ in range(5)]
        lib().orc_macros(self._h, *[_ptr(a) for a in out])
        return dict(zip(("phi", "u", "v", "p", "rho"), out))

    def cell_fields(self):
        shape = (self.ny, self.nx)
        out = [np.empty(shape) for _ in range(4)]
        lib().orc_cell_fields(self._h, *[_ptr(a) for a in out])
        return dict(zip(("gx", "gy", "lap", "mu"), out))

    def get_state(self):
        f = np.empty((9, self.ny, self.nx))
        g = np.empty((9, self.ny, self.nx))
        hist = np.empty((2, self.ny, self.nx))
        st = C.c_long(0)
        lib().orc_get_state(self._h, _ptr(f), _ptr(g), _ptr(hist), C.byref(st))
        return dict(f=f, g=g, hist=hist, step=int(st.value))

    def set_state(self, state):
        f, g, hist = (_f64(state[k]) for k in ("f", "g", "hist"))
        lib().orc_set_state(self._h, _ptr(f), _ptr(g), _ptr(hist), int(state["step"]))

    @property
    def time(self):
        return lib().orc_time(self._h)

    @property
    def steps_done(self):
        return int(lib().orc_step_count(self._h))

    def derived(self):
        out = np.empty(6)
        lib().orc_derived(self._h, _ptr(out))
        return dict(zip(("dt", "h", "kappa", "beta", "tau_f", "drho"), out))


# ------------------------------------------------------- point functions

def feq(phi, ux, uy):
    out = np.empty(9)
    lib().orc_feq(phi, ux, uy, _ptr(out))
    return out


def sf(theta, nx, ny, Dx, Dy):
    out = np.empty(9)
    lib().orc_sf(theta, nx, ny, Dx, Dy, _ptr(out))
    return out


def geq(p, rho, ux, uy):
    out = np.empty(9)
    lib().orc_geq(p, rho, ux, uy, _ptr(out))
    return out


def sg(ux, uy, drx, dry, Fx, Fy):
    out = np.empty(9)
    lib().orc_sg(ux, uy, drx, dry, Fx, Fy, _ptr(out))
    return out


def bar_plus(tau, dt, tilde, eq, S):
    tl, eq, S = (_f64(a) for a in (tilde, eq, S))
    bp, tp = np.empty(9), np.empty(9)
    lib().orc_bar_plus(tau, dt, _ptr(tl), _ptr(eq), _ptr(S), _ptr(bp), _ptr(tp))
    return bp, tp


def face_df(tau, h, bar, eq, S):
    bar, eq, S = (_f64(a) for a in (bar, eq, S))
    out = np.empty(9)
    lib().orc_face_df(tau, h, _ptr(bar), _ptr(eq), _ptr(S), _ptr(out))
    return out


def recon(a, q, h, mode="central", walls_y=False, dx=None, dy=None):
    """Bar values of population q of the cell field ``a`` ([ny][nx]) at the
    x-faces (east of each cell) and y-faces (north of each cell); ``dx``,
    ``dy``: cell widths of a stretched mesh (None: unit widths)."""
    a = np.ascontiguousarray(a, dtype=np.float64)
    ny, nx = a.shape
    dx, dy = _f64(dx), _f64(dy)
    xf, yf = np.empty_like(a), np.empty_like(a)
    lib().orc_recon(nx, ny, int(walls_y), _ptr(dx), _ptr(dy), RECON[mode], float(h), int(q),
                    _ptr(a), _ptr(xf), _ptr(yf))
    return xf, yf


def stencils(phi, walls_y=False, dx=None, dy=None):
    phi = _f64(phi)
    ny, nx = phi.shape
    dx, dy = _f64(dx), _f64(dy)
    gx, gy, lap = np.empty_like(phi), np.empty_like(phi), np.empty_like(phi)
    lib().orc_stencils(nx, ny, int(walls_y), _ptr(dx), _ptr(dy), _ptr(phi), _ptr(gx), _ptr(gy),
                       _ptr(lap))
    return gx, gy, lap


def run(nx, ny, params, model, phi, u=None, v=None, p=None, steps=0):
    """Convenience: init, advance ``steps`` and return the cell macros."""
    s = Sim(nx, ny, params, model)
    s.init(phi, u, v, p)
    if steps:
        s.step(steps)
    return s.macros()
