"""Python binding of libdugks, the gfx950 phase-field DUGKS library.

Argument marshalling only: every step of the method runs in the HIP kernels of
``csrc/``. The names follow the C ABI of ``include/dugks.h`` (``create``,
``set_params``, ``init_fields``, ``step``, ``get_macros``, ``destroy`` ...);
``Solver`` and ``Batch`` wrap a handle / batch with numpy or torch arrays.
Loading fails loudly when ``libdugks.so`` has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from .build import LIB as _LIB_PATH

OK, EINVAL, ENOMEM, EDEVICE, ENUMERIC, ESTATE, EBUSY = 0, -1, -2, -3, -4, -5, -6
FP32, FP64 = 0, 1
MODEL_AC, MODEL_COUPLED = 0, 1
_VISC = {"uniform_nu": 0, "reciprocal": 1, "linear": 2}
_GRAV = {"rho_g": 0, "buoyancy": 1}
_VEL = {"uniform": 0, "rotation": 1, "shear": 2, "deform": 3}
_RECON = {"central": 0, "upwind": 1}


class DugksError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libdugks error {code}: {msg}")
        self.code = code


class Params(C.Structure):
    _fields_ = [
        ("phi_H", C.c_double), ("phi_L", C.c_double),
        ("rho_H", C.c_double), ("rho_L", C.c_double),
        ("mu_H", C.c_double), ("mu_L", C.c_double),
        ("nu", C.c_double),
        ("visc_mode", C.c_int),
        ("sigma", C.c_double), ("W", C.c_double), ("M_phi", C.c_double),
        ("gx", C.c_double), ("gy", C.c_double),
        ("gravity_form", C.c_int),
        ("Gx", C.c_double), ("Gy", C.c_double),
        ("cfl", C.c_double),
        ("bc_y", C.c_int),
        ("vel_kind", C.c_int),
        ("U0", C.c_double), ("L0", C.c_double), ("T_period", C.c_double),
        ("recon", C.c_int),
        ("eps_n", C.c_double),
    ]


_DEFAULTS = dict(phi_H=1.0, phi_L=0.0, rho_H=1.0, rho_L=1.0, mu_H=0.1, mu_L=0.1,
                 nu=0.1, visc="uniform_nu", sigma=0.0, W=4.0, M=0.1, gx=0.0, gy=0.0,
                 gravity="rho_g", Gx=0.0, Gy=0.0, cfl=0.5, walls_y=False,
                 vel="uniform", U0=0.0, L0=1.0, T_period=1.0, recon="central", eps_n=1e-6)


def make_params(d: dict) -> Params:
    p = dict(_DEFAULTS)
    unknown = set(d) - set(p)
    if unknown:
        raise KeyError(f"unknown parameter keys: {sorted(unknown)}")
    p.update(d)
    s = Params()
    for k in ("phi_H", "phi_L", "rho_H", "rho_L", "mu_H", "mu_L", "nu", "sigma", "W",
              "gx", "gy", "Gx", "Gy", "cfl", "U0", "L0", "T_period", "eps_n"):
        setattr(s, k, float(p[k]))
    s.M_phi = float(p["M"])
    s.visc_mode = _VISC[p["visc"]]
    s.gravity_form = _GRAV[p["gravity"]]
    s.bc_y = 1 if p["walls_y"] else 0
    s.vel_kind = _VEL[p["vel"]]
    s.recon = _RECON[p["recon"]]
    return s


_lib = None


def _preload_torch_hip_runtime():
    """Bind libdugks to the HIP runtime that torch ships, so that a process
    holds one HIP runtime (device memory and streams are shared with torch).
    Both runtimes carry the same SONAME; the first one loaded wins."""
    try:
        import importlib.util
        spec = importlib.util.find_spec("torch")
        if spec is None or not spec.submodule_search_locations:
            return
        path = os.path.join(list(spec.submodule_search_locations)[0], "lib", "libamdhip64.so")
        if os.path.exists(path):
            C.CDLL(path, mode=C.RTLD_GLOBAL)
    except OSError:
        pass


def lib():
    """Load libdugks.so (built by ``build.py``); raise if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise ImportError(f"{_LIB_PATH} is missing: build it with "
                              "`python -m paper_1810_07802_amd.build`")
        _preload_torch_hip_runtime()
        L = C.CDLL(_LIB_PATH)
        vp, dp, i, ll, sz = C.c_void_p, C.POINTER(C.c_double), C.c_int, C.c_longlong, C.c_size_t
        sig = {
            "dugks_create": (i, [i, i, i, i, C.POINTER(vp)]),
            "dugks_set_params": (i, [vp, C.POINTER(Params)]),
            "dugks_set_stream": (i, [vp, vp]),
            "dugks_set_tile": (i, [vp, i]),
            "dugks_get_tile": (i, [vp]),
            "dugks_set_mesh": (i, [vp, dp, dp]),
            "dugks_autotune": (i, [vp, i, C.POINTER(i), dp]),
            "dugks_init_fields": (i, [vp, dp, dp, dp, dp]),
            "dugks_init_fields_device": (i, [vp, vp, vp, vp, vp]),
            "dugks_step": (i, [vp, i]),
            "dugks_sync": (i, [vp]),
            "dugks_get_macros": (i, [vp, dp, dp, dp, dp, dp]),
            "dugks_get_macros_device": (i, [vp, vp, vp, vp, vp, vp]),
            "dugks_get_diagnostics": (i, [vp, dp]),
            "dugks_get_diagnostics_noalloc": (i, [vp, vp]),
            "dugks_steps_done": (ll, [vp]),
            "dugks_time": (C.c_double, [vp]),
            "dugks_state_bytes": (sz, [vp]),
            "dugks_get_state": (i, [vp, vp, sz, C.POINTER(ll)]),
            "dugks_set_state": (i, [vp, vp, sz, ll]),
            "dugks_footprint_bytes": (sz, [i, i, i, i]),
            "dugks_last_error": (C.c_char_p, [vp]),
            "dugks_destroy": (i, [vp]),
            "dugks_batch_create": (i, [i, C.POINTER(i), C.POINTER(i), i, i, C.POINTER(vp)]),
            "dugks_batch_case": (vp, [vp, i]),
            "dugks_batch_create_from": (i, [i, C.POINTER(vp), C.POINTER(vp)]),
            "dugks_batch_step": (i, [vp, i, i]),
            "dugks_batch_set_budget": (i, [vp, i, ll]),
            "dugks_batch_set_stream": (i, [vp, vp]),
            "dugks_batch_sync": (i, [vp]),
            "dugks_batch_destroy": (i, [vp]),
            "dugks_batch_last_error": (C.c_char_p, [vp]),
            "dugks_batch_autotune": (i, [vp, i, C.POINTER(i), C.POINTER(i)]),
            "dugks_pool_create": (i, [sz, i, ll, i, i, C.POINTER(vp)]),
            "dugks_pool_set_stream": (i, [vp, vp]),
            "dugks_pool_case_bytes": (sz, [i, i, i, i]),
            "dugks_pool_admit": (i, [vp, i, i, C.POINTER(Params), dp, dp, dp, dp, ll, C.POINTER(i)]),
            "dugks_pool_admit_handle": (i, [vp, vp, ll, C.POINTER(i)]),
            "dugks_pool_status": (i, [vp, i]),
            "dugks_pool_step": (i, [vp, i, i]),
            "dugks_pool_steps_done": (ll, [vp, i]),
            "dugks_pool_remaining": (ll, [vp, i]),
            "dugks_pool_get_macros": (i, [vp, i, dp, dp, dp, dp, dp]),
            "dugks_pool_retire": (i, [vp, i]),
            "dugks_pool_bytes_free": (sz, [vp]),
            "dugks_pool_sync": (i, [vp]),
            "dugks_pool_last_error": (C.c_char_p, [vp]),
            "dugks_pool_destroy": (i, [vp]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype, f.argtypes = res, args
        _lib = L
    return _lib


def _check(rc, h=None, batch=False):
    if rc != OK:
        L = lib()
        msg = (L.dugks_batch_last_error(h) if batch else L.dugks_last_error(h)) or b""
        raise DugksError(rc, msg.decode())
    return rc


def _dptr(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_double))


def _host(a, shape):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.shape != shape:
        raise ValueError(f"field shape {a.shape} != {shape}")
    return a


# ---------------------------------------------------------------- C-ABI names

def create(nx, ny, precision=FP32, model=MODEL_COUPLED):
    h = C.c_void_p()
    _check(lib().dugks_create(int(nx), int(ny), int(precision), int(model), C.byref(h)))
    return h


def set_params(h, params: dict):
    p = make_params(params)
    _check(lib().dugks_set_params(h, C.byref(p)), h)


def set_stream(h, stream):
    _check(lib().dugks_set_stream(h, C.c_void_p(stream)), h)


def set_tile(h, seg_rows):
    _check(lib().dugks_set_tile(h, int(seg_rows)), h)


def init_fields(h, shape, phi, u=None, v=None, p=None):
    arrs = [_host(a, shape) for a in (phi, u, v, p)]
    _check(lib().dugks_init_fields(h, *[_dptr(a) for a in arrs]), h)


def step(h, nsteps=1):
    _check(lib().dugks_step(h, int(nsteps)), h)


def sync(h):
    _check(lib().dugks_sync(h), h)


def get_macros(h, shape):
    out = [np.empty(shape) for _ in range(5)]
    _check(lib().dugks_get_macros(h, *[_dptr(a) for a in out]), h)
    return dict(zip(("phi", "u", "v", "p", "rho"), out))


def get_diagnostics(h):
    out = np.empty(8)
    rc = lib().dugks_get_diagnostics(h, _dptr(out))
    if rc not in (OK, ENUMERIC):
        _check(rc, h)
    d = dict(zip(("sum_phi", "sum_rho_u", "sum_rho_v", "kinetic", "max_u", "sum_rho",
                  "nonfinite", "time"), out.tolist()))
    d["status"] = rc
    return d


def footprint_bytes(nx, ny, precision=FP32, model=MODEL_COUPLED):
    return int(lib().dugks_footprint_bytes(int(nx), int(ny), int(precision), int(model)))


def destroy(h):
    if h:
        lib().dugks_destroy(h)


# ------------------------------------------------------------------ wrappers

class Solver:
    """One grid: ``Solver(nx, ny, params, model="coupled", precision="fp32")``."""

    @classmethod
    def _view(cls, h, nx, ny, model, precision):
        """A Solver over a handle owned elsewhere (a batch's case)."""
        s = cls.__new__(cls)
        s.nx, s.ny, s.shape = int(nx), int(ny), (int(ny), int(nx))
        s.model, s.precision, s.h, s._owned = model, precision, C.c_void_p(h), False
        return s

    def __init__(self, nx, ny, params, model="coupled", precision="fp32", seg_rows=None):
        self._owned = True
        self.nx, self.ny = int(nx), int(ny)
        self.shape = (self.ny, self.nx)
        self.model = model
        self.precision = precision
        self.h = create(nx, ny, FP64 if precision == "fp64" else FP32,
                        MODEL_COUPLED if model == "coupled" else MODEL_AC)
        try:
            if seg_rows:
                set_tile(self.h, seg_rows)
            set_params(self.h, params)
        except Exception:
            destroy(self.h)
            self.h = None
            raise

    def __del__(self):
        h = getattr(self, "h", None)
        if h and getattr(self, "_owned", True):
            try:
                destroy(h)
            except Exception:  # interpreter shutdown: module globals may be gone
                pass
        self.h = None

    def set_stream(self, stream):
        set_stream(self.h, stream)

    def set_params(self, params):
        """New parameters from the next step on (the state is kept)."""
        set_params(self.h, params)

    def set_mesh(self, dx=None, dy=None):
        """Stretched mesh of cell widths dx[nx], dy[ny] (None: unit widths on
        that axis; both None: the unit mesh). Call before init."""
        ax = [None if a is None else np.ascontiguousarray(a, dtype=np.float64) for a in (dx, dy)]
        for a, n in zip(ax, (self.nx, self.ny)):
            if a is not None and a.shape != (n,):
                raise ValueError(f"widths must have shape ({n},)")
        _check(lib().dugks_set_mesh(self.h, *[_dptr(a) for a in ax]), self.h)
        self._mesh = ax

    def init(self, phi, u=None, v=None, p=None):
        init_fields(self.h, self.shape, phi, u, v, p)

    def init_device(self, phi, u=None, v=None, p=None):
        """Device tensors (torch, float64, contiguous, [ny][nx])."""
        ptr = [None if a is None else C.c_void_p(a.data_ptr()) for a in (phi, u, v, p)]
        _check(lib().dugks_init_fields_device(self.h, *ptr), self.h)

    def step(self, nsteps=1):
        step(self.h, nsteps)

    def sync(self):
        sync(self.h)

    def macros(self):
        return get_macros(self.h, self.shape)

    def macros_device(self, out):
        """Fill device tensors out['phi'|'u'|'v'|'p'|'rho'] (float64)."""
        ptr = [C.c_void_p(out[k].data_ptr()) if k in out else None
               for k in ("phi", "u", "v", "p", "rho")]
        _check(lib().dugks_get_macros_device(self.h, *ptr), self.h)

    def diagnostics(self):
        return get_diagnostics(self.h)

    def diagnostics_noalloc(self, out_ptr):
        """The seven diagnostics into device memory at `out_ptr` (7 doubles),
        asynchronously, with no device allocation."""
        _check(lib().dugks_get_diagnostics_noalloc(self.h, C.c_void_p(out_ptr)), self.h)

    @property
    def steps_done(self):
        return int(lib().dugks_steps_done(self.h))

    @property
    def time(self):
        return float(lib().dugks_time(self.h))

    @property
    def seg_rows(self):
        return int(lib().dugks_get_tile(self.h))

    def set_tile(self, seg_rows):
        set_tile(self.h, seg_rows)

    def autotune(self, probe_steps=20):
        """Time a few tiles on the current state, keep the fastest (the state
        is put back); returns (seg_rows, microseconds per step)."""
        seg, us = C.c_int(0), C.c_double(0.0)
        _check(lib().dugks_autotune(self.h, int(probe_steps), C.byref(seg), C.byref(us)), self.h)
        return int(seg.value), float(us.value)

    def get_state(self):
        n = int(lib().dugks_state_bytes(self.h))
        buf = np.empty(n, dtype=np.uint8)
        st = C.c_longlong(0)
        _check(lib().dugks_get_state(self.h, buf.ctypes.data_as(C.c_void_p), n, C.byref(st)), self.h)
        return buf, int(st.value)

    def set_state(self, buf, steps):
        buf = np.ascontiguousarray(buf, dtype=np.uint8)
        _check(lib().dugks_set_state(self.h, buf.ctypes.data_as(C.c_void_p), buf.nbytes,
                                     int(steps)), self.h)


class Batch:
    """Several solvers of one precision and model advanced together:
    ``Batch(solvers)`` over existing solvers (dugks_batch_create_from), or
    ``Batch.create(shapes, model, precision)`` with cases the batch owns
    (dugks_batch_create), reached as ``batch.case(k)``."""

    def __init__(self, solvers):
        self.solvers = list(solvers)
        arr = (C.c_void_p * len(self.solvers))(*[s.h.value for s in self.solvers])
        b = C.c_void_p()
        _check(lib().dugks_batch_create_from(len(self.solvers), arr, C.byref(b)), None, batch=True)
        self.b = b

    @classmethod
    def create(cls, shapes, model="coupled", precision="fp32"):
        """A batch owning len(shapes) new cases of (nx, ny) cells each."""
        n = len(shapes)
        nx = (C.c_int * n)(*[int(a) for a, _ in shapes])
        ny = (C.c_int * n)(*[int(b) for _, b in shapes])
        b = C.c_void_p()
        _check(lib().dugks_batch_create(n, nx, ny, FP64 if precision == "fp64" else FP32,
                                        MODEL_COUPLED if model == "coupled" else MODEL_AC,
                                        C.byref(b)), None, batch=True)
        self = cls.__new__(cls)
        self.b = b
        self.solvers = [Solver._view(lib().dugks_batch_case(b, k), shapes[k][0], shapes[k][1],
                                     model, precision) for k in range(n)]
        return self

    def case(self, k):
        """Case k as a Solver (set_params via ``set_params``, ``init``, ``macros``)."""
        return self.solvers[k]

    def __del__(self):
        b = getattr(self, "b", None)
        if b:
            try:
                lib().dugks_batch_destroy(b)
            except Exception:  # interpreter shutdown: module globals may be gone
                pass
            self.b = None

    def set_stream(self, stream):
        _check(lib().dugks_batch_set_stream(self.b, C.c_void_p(stream)), self.b, batch=True)

    def set_budget(self, k, steps):
        _check(lib().dugks_batch_set_budget(self.b, int(k), int(steps)), self.b, batch=True)

    def autotune(self, probe_steps=10):
        """Pick each boundary group's segment length by timing (states are
        put back); returns (periodic, walls) segment lengths (0: no case)."""
        a, w = C.c_int(0), C.c_int(0)
        _check(lib().dugks_batch_autotune(self.b, int(probe_steps), C.byref(a), C.byref(w)),
               self.b, batch=True)
        return int(a.value), int(w.value)

    def step(self, nsteps=1, use_graph=False):
        _check(lib().dugks_batch_step(self.b, int(nsteps), int(bool(use_graph))), self.b,
               batch=True)

    def sync(self):
        _check(lib().dugks_batch_sync(self.b), self.b, batch=True)


class Pool:
    """Serving pool (continuous batching): cases admitted by arena footprint
    while others run, advanced together, read out and retired one by one."""

    def __init__(self, hbm_bytes, max_cases, max_cells, precision="fp32", model="coupled"):
        self.precision = FP64 if precision == "fp64" else FP32
        self.model = MODEL_COUPLED if model == "coupled" else MODEL_AC
        p = C.c_void_p()
        rc = lib().dugks_pool_create(int(hbm_bytes), int(max_cases), int(max_cells),
                                     self.precision, self.model, C.byref(p))
        if rc != OK:
            raise DugksError(rc, (lib().dugks_pool_last_error(None) or b"").decode())
        self.p = p
        self.shapes = {}

    def _check(self, rc):
        if rc != OK:
            raise DugksError(rc, (lib().dugks_pool_last_error(self.p) or b"").decode())

    def __del__(self):
        p = getattr(self, "p", None)
        if p:
            try:
                lib().dugks_pool_destroy(p)
            except Exception:  # interpreter shutdown: module globals may be gone
                pass
            self.p = None

    def set_stream(self, stream):
        self._check(lib().dugks_pool_set_stream(self.p, C.c_void_p(stream)))

    def case_bytes(self, nx, ny):
        return int(lib().dugks_pool_case_bytes(int(nx), int(ny), self.precision, self.model))

    def admit(self, case, nsteps):
        """Admit a case dict (workloads format); returns its slot, or None
        when the pool has no free slot or no room (EBUSY)."""
        shape = (case["ny"], case["nx"])
        prm = make_params(case["params"])
        arrs = [_host(case.get(k), shape) for k in ("phi", "u", "v", "p")]
        slot = C.c_int(-1)
        rc = lib().dugks_pool_admit(self.p, case["nx"], case["ny"], C.byref(prm),
                                    *[_dptr(a) for a in arrs], int(nsteps), C.byref(slot))
        if rc == EBUSY:
            return None
        self._check(rc)
        self.shapes[slot.value] = shape
        return slot.value

    def admit_handle(self, solver, nsteps):
        """Admit a Solver's parameters and current state as a new case;
        returns its slot, or None when the pool has no room (EBUSY)."""
        slot = C.c_int(-1)
        rc = lib().dugks_pool_admit_handle(self.p, solver.h, int(nsteps), C.byref(slot))
        if rc == EBUSY:
            return None
        self._check(rc)
        self.shapes[slot.value] = solver.shape
        return slot.value

    def status(self, slot):
        """OK (0) or ENUMERIC as of the last ``sync``: a slot whose state
        went non-finite."""
        return int(lib().dugks_pool_status(self.p, int(slot)))

    def step(self, nsteps, use_graph=True):
        self._check(lib().dugks_pool_step(self.p, int(nsteps), 1 if use_graph else 0))

    def steps_done(self, slot):
        return int(lib().dugks_pool_steps_done(self.p, int(slot)))

    def remaining(self, slot):
        return int(lib().dugks_pool_remaining(self.p, int(slot)))

    def macros(self, slot):
        out = [np.empty(self.shapes[slot]) for _ in range(5)]
        self._check(lib().dugks_pool_get_macros(self.p, int(slot), *[_dptr(a) for a in out]))
        return dict(zip(("phi", "u", "v", "p", "rho"), out))

    def retire(self, slot):
        self._check(lib().dugks_pool_retire(self.p, int(slot)))
        self.shapes.pop(slot, None)

    def bytes_free(self):
        return int(lib().dugks_pool_bytes_free(self.p))

    def sync(self):
        self._check(lib().dugks_pool_sync(self.p))
