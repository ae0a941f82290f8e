"""Seeded synthetic inputs for the phase-field DUGKS step.

This module is shared by the tests, the benchmark, the oracle runs and the HIP
runs. It builds initial fields and parameter dictionaries for the benchmark
problems of the paper (arXiv:1810.07802, Sec. III and IV) and holds none of the
method's arithmetic: no equilibria, sources, stencils or fluxes, only problem
set-ups (grids, initial profiles, physical constants) and seeded random numbers.

A case is a dict with keys ``name, nx, ny, model ("coupled" | "ac"), params,
phi, u, v, p, steps``. ``params`` uses the keys of the parameter dictionary
understood by both the oracle and the HIP binding:

    phi_H, phi_L, rho_H, rho_L, mu_H, mu_L, nu, visc ("uniform_nu" |
    "reciprocal" | "linear"), sigma, W, M, gx, gy, gravity ("rho_g" |
    "buoyancy"), Gx, Gy, cfl, walls_y, vel ("uniform" | "rotation" | "shear" |
    "deform"), U0, L0, T_period
"""
from __future__ import annotations

import numpy as np


def _centres(nx, ny):
    x = np.arange(nx) + 0.5
    y = np.arange(ny) + 0.5
    return np.meshgrid(x, y)  # arrays of shape (ny, nx)


def tanh_profile(z, W, phi_H, phi_L):
    """Equilibrium interface profile of Sec. II.A (Eq. 7): phi_H where z >> 0."""
    return 0.5 * (phi_H + phi_L) + 0.5 * (phi_H - phi_L) * np.tanh(2.0 * z / W)


def _case(name, nx, ny, model, params, phi, u=None, v=None, p=None, steps=0):
    return dict(name=name, nx=int(nx), ny=int(ny), model=model, params=params,
                phi=np.ascontiguousarray(phi, dtype=np.float64),
                u=None if u is None else np.ascontiguousarray(u, dtype=np.float64),
                v=None if v is None else np.ascontiguousarray(v, dtype=np.float64),
                p=None if p is None else np.ascontiguousarray(p, dtype=np.float64),
                steps=int(steps))


# ---------------------------------------------------------------- configs

def diag_translation(L0=100, R=None, W=4.0, U0=0.02, M=0.01, cfl=0.5,
                     phi_H=1.0, phi_L=-1.0):
    """Interface-only diagonal translation (Sec. III.A, Eq. 40).

    Defaults: the 100x100 periodic case with R=25, W=4, U=0.02, M=0.01,
    CFL=0.5, phi=tanh(2(R-r)/W) in [-1, 1], one full period T = L0/U0.
    """
    R = L0 / 4.0 if R is None else R
    X, Y = _centres(L0, L0)
    r = np.hypot(X - 0.5 * L0, Y - 0.5 * L0)
    phi = tanh_profile(R - r, W, phi_H, phi_L)
    params = dict(phi_H=phi_H, phi_L=phi_L, W=W, M=M, cfl=cfl, vel="uniform",
                  U0=U0, L0=float(L0), T_period=L0 / U0)
    steps = int(round(L0 / U0 / cfl))
    return _case(f"diag_translation_{L0}", L0, L0, "ac", params, phi, steps=steps)


def zalesak(L0=256, R=100, slot=20, W=4.0, U0=None, Pe=128, M=0.02, cfl=0.5):
    """Zalesak's slotted disk in a rotation field (Sec. III.B, Eq. 41).

    The disk starts as a step (phi_H inside, phi_L outside); the slot is
    ``slot`` cells wide and reaches from the bottom of the disk to 60 % of its
    height above the centre. One period is T = 2 L0 / U0.
    """
    U0 = Pe * M / L0 if U0 is None else U0
    X, Y = _centres(L0, L0)
    xc = yc = 0.5 * L0
    inside = np.hypot(X - xc, Y - yc) <= R
    slot_cut = (np.abs(X - xc) <= 0.5 * slot) & (Y <= yc + 0.6 * R)
    phi = np.where(inside & ~slot_cut, 1.0, 0.0)
    T = 2.0 * L0 / U0
    params = dict(phi_H=1.0, phi_L=0.0, W=W, M=M, cfl=cfl, vel="rotation",
                  U0=U0, L0=float(L0), T_period=T)
    return _case(f"zalesak_{L0}", L0, L0, "ac", params, phi,
                 steps=int(round(T / cfl)))


def shear_elongation(L0=256, W=4.0, Pe=256, M=0.01, cfl=0.5):
    """Circle in the reversing shear flow (Sec. III.C, Eq. 42), R = L0/5 at
    (0.5 L0, 0.3 L0); the field reverses at T/2 with T = 2 L0 / U0."""
    U0 = Pe * M / L0
    X, Y = _centres(L0, L0)
    r = np.hypot(X - 0.5 * L0, Y - 0.3 * L0)
    phi = tanh_profile(L0 / 5.0 - r, W, 1.0, 0.0)
    T = 2.0 * L0 / U0
    params = dict(phi_H=1.0, phi_L=0.0, W=W, M=M, cfl=cfl, vel="shear",
                  U0=U0, L0=float(L0), T_period=T)
    return _case(f"shear_{L0}", L0, L0, "ac", params, phi,
                 steps=int(round(T / cfl)))


def smoothed_deformation(L0=512, W=4.0, Pe=512, M=0.02, cfl=0.5):
    """Circle R = L0/5 at the centre in the smoothed deformation field
    (Sec. III.D, Eq. 43) with period T = L0 / U0."""
    U0 = Pe * M / L0
    X, Y = _centres(L0, L0)
    r = np.hypot(X - 0.5 * L0, Y - 0.5 * L0)
    phi = tanh_profile(L0 / 5.0 - r, W, 1.0, 0.0)
    T = L0 / U0
    params = dict(phi_H=1.0, phi_L=0.0, W=W, M=M, cfl=cfl, vel="deform",
                  U0=U0, L0=float(L0), T_period=T)
    return _case(f"deform_{L0}", L0, L0, "ac", params, phi,
                 steps=int(round(T / cfl)))


def bubble(L=128, R=None, W=5.0, rho_H=1000.0, rho_L=1.0, sigma=1e-3,
           nu=0.1, M=0.1, cfl=0.5, steps=20000):
    """Stationary light bubble in a heavy liquid, periodic (Sec. IV.A, Eq. 45).

    Defaults: 128x128, R=32, density ratio 1000, sigma=1e-3, nu=0.1 in both
    phases, M=0.1, 20000 steps; centre at (L/2, L/2), u=0, p=0. The interface
    width is the paper's W=5 for this test: at W=4 the 1000:1 bubble diverges
    within a few hundred steps under the readings used here (the instability
    comes from the density-gradient terms of the g model on an under-resolved
    interface), while W=5 stays at rest with spurious |u| ~ 1e-7.
    """
    R = L / 4.0 if R is None else R
    X, Y = _centres(L, L)
    r = np.hypot(X - 0.5 * L, Y - 0.5 * L)
    phi = tanh_profile(r - R, W, 1.0, 0.0)
    params = dict(phi_H=1.0, phi_L=0.0, rho_H=rho_H, rho_L=rho_L, nu=nu,
                  visc="uniform_nu", sigma=sigma, W=W, M=M, cfl=cfl)
    return _case(f"bubble_{L}", L, L, "coupled", params, phi, steps=steps)


def hydrostatic_pressure(phi, params):
    """Initial pressure of a fluid at rest under gravity: the hydrostatic
    pressure of the row-averaged density profile, dp/dy = G_y with
    G = (rho - rho_ref) g (rho_ref the mean density in the buoyancy form, 0
    otherwise) and rho linear in phi between the phases, integrated along y
    by the trapezoid rule and shifted to zero mean. Shape of ``phi``."""
    p = params
    s = np.clip((phi - p["phi_L"]) / (p["phi_H"] - p["phi_L"]), 0.0, 1.0)
    rho = (p["rho_L"] + (p["rho_H"] - p["rho_L"]) * s).mean(axis=1)
    ref = 0.5 * (p["rho_H"] + p["rho_L"]) if p.get("gravity") == "buoyancy" else 0.0
    G = (rho - ref) * p.get("gy", 0.0)
    col = np.concatenate([[0.0], np.cumsum(0.5 * (G[1:] + G[:-1]))])
    return np.repeat((col - col.mean())[:, None], phi.shape[1], axis=1)


def rayleigh_taylor(L0=256, At=0.5, Re=3000.0, U=0.04, W=5.0, sigma=5e-5,
                    Pe=1000.0, cfl=0.25, steps=20000, rho_L=1.0):
    """Rayleigh-Taylor instability, L0 x 4L0, periodic in x, no-slip walls in
    y (Sec. IV.D, Eqs. 48-49). Heavy fluid above y = 2L0 + 0.1 L0 cos(2 pi x/L0).
    One dynamic viscosity mu = rho_H L0 U / Re; g = U^2 / L0 (U = sqrt(g L0));
    M = U L0 / Pe; buoyancy-form gravity. The fluids start at rest in the
    hydrostatic pressure of the mean (flat-interface) density profile, so
    that only the interface perturbation drives the flow: from p = 0 the
    weakly compressible g model first sets the whole column in motion, which
    moves phi off phi_H in the heavy bulk."""
    rho_H = rho_L * (1.0 + At) / (1.0 - At)
    mu = rho_H * L0 * U / Re
    g = U * U / L0
    nx, ny = L0, 4 * L0
    X, Y = _centres(nx, ny)
    H = 2.0 * L0 + 0.1 * L0 * np.cos(2.0 * np.pi * X / L0)
    phi = tanh_profile(Y - H, W, 1.0, 0.0)
    params = dict(phi_H=1.0, phi_L=0.0, rho_H=rho_H, rho_L=rho_L, mu_H=mu,
                  mu_L=mu, visc="linear", sigma=sigma, W=W, M=U * L0 / Pe,
                  gx=0.0, gy=-g, gravity="buoyancy", cfl=cfl, walls_y=True)
    return _case(f"rti_{nx}x{ny}", nx, ny, "coupled", params, phi,
                 p=hydrostatic_pressure(phi, params), steps=steps)


def spinodal(L=64, seed=1810, amp=0.01, rho_H=1000.0, rho_L=1.0, nu=0.1,
             M=0.1, W=4.0, sigma=0.1, cfl=0.5, steps=5000):
    """Spinodal decomposition (Sec. IV.C): phi uniform random in [-amp, amp]
    with (phi_H, phi_L) = (1, -1), density ratio 1000, periodic."""
    rng = np.random.default_rng(seed)
    phi = rng.uniform(-amp, amp, size=(L, L))
    params = dict(phi_H=1.0, phi_L=-1.0, rho_H=rho_H, rho_L=rho_L, nu=nu,
                  visc="uniform_nu", sigma=sigma, W=W, M=M, cfl=cfl)
    return _case(f"spinodal_{L}_s{seed}", L, L, "coupled", params, phi, steps=steps)


def spinodal_batch(n=64, seed=1810, sizes=(64, 128, 256, 512), steps=5000):
    """The batched spinodal workload: ``n`` cases whose sizes are drawn from
    ``sizes`` by ``default_rng(seed)``; case k uses seed ``seed + k``."""
    rng = np.random.default_rng(seed)
    Ls = rng.choice(np.asarray(sizes), size=n)
    return [spinodal(int(L), seed=seed + k, steps=steps) for k, L in enumerate(Ls)]


def poiseuille_analytic(ny, mu_H, mu_L, Gx):
    """Steady layered Poiseuille velocity (Sec. IV.B, Eq. 46) at cell centres.
    The channel y in [-h, h] maps to the grid with h = ny/2; the lower layer
    (y < 0) holds the phi_H fluid with viscosity mu_H."""
    h = 0.5 * ny
    y = np.arange(ny) + 0.5 - h
    a = (mu_L - mu_H) / (mu_L + mu_H)
    up = Gx * h * h / (2 * mu_L) * (-(y / h) ** 2 - (y / h) * a + 2 * mu_L / (mu_L + mu_H))
    lo = Gx * h * h / (2 * mu_H) * (-(y / h) ** 2 - (y / h) * a + 2 * mu_H / (mu_L + mu_H))
    return np.where(y > 0, up, lo)


def layered_poiseuille(nx=10, ny=100, mu_ratio=1000.0, mu_H=0.1, uc=1e-4,
                       W=4.0, sigma=1e-3, M=0.1, cfl=0.5, visc="reciprocal",
                       analytic_init=False, steps=20000):
    """Layered Poiseuille flow between no-slip walls, driven by G = (Gx, 0)
    with u_c = Gx h^2 / (mu_L + mu_H) (Sec. IV.B). rho_H = rho_L = 1."""
    mu_L = mu_H / mu_ratio
    h = 0.5 * ny
    Gx = uc * (mu_L + mu_H) / (h * h)
    X, Y = _centres(nx, ny)
    phi = tanh_profile(h - Y, W, 1.0, 0.0)
    u = None
    if analytic_init:
        u = np.repeat(poiseuille_analytic(ny, mu_H, mu_L, Gx)[:, None], nx, axis=1)
    params = dict(phi_H=1.0, phi_L=0.0, rho_H=1.0, rho_L=1.0, mu_H=mu_H,
                  mu_L=mu_L, visc=visc, sigma=sigma, W=W, M=M, Gx=Gx,
                  cfl=cfl, walls_y=True)
    c = _case(f"poiseuille_{nx}x{ny}_m{mu_ratio:g}", nx, ny, "coupled", params,
              phi, u=u, steps=steps)
    c["Gx"] = Gx
    return c


def served_stream(n=500, seed=7802, poiseuille_frac=0.5, nx_pois=64,
                  ny_range=(64, 1024), bubble_sizes=(64, 128, 256, 512, 1024),
                  steps_range=(1000, 20000)):
    """Request mix for the serving loop: half layered Poiseuille (viscosity
    ratio 100, analytic initial profile, nx=64, ny in 64..1024 step 64), half
    stationary bubbles (L in 64..1024, R = L/4, ratio 1000). Each request
    carries its step count. Arrival times are drawn by the caller."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n):
        steps = int(rng.integers(steps_range[0], steps_range[1] + 1))
        if rng.random() < poiseuille_frac:
            ny = int(rng.integers(ny_range[0] // 64, ny_range[1] // 64 + 1)) * 64
            c = layered_poiseuille(nx=nx_pois, ny=ny, mu_ratio=100.0,
                                   analytic_init=True, steps=steps)
        else:
            L = int(rng.choice(np.asarray(bubble_sizes)))
            c = bubble(L=L, steps=steps)
        c["name"] = f"req{k}_{c['name']}"
        out.append(c)
    return out


# --------------------------------------------------- generic test inputs

def smooth_field(nx, ny, seed, modes=3, amp=1.0, offset=0.0):
    """Periodic smooth random field: a few low Fourier modes."""
    rng = np.random.default_rng(seed)
    X, Y = _centres(nx, ny)
    out = np.full((ny, nx), float(offset))
    for _ in range(modes):
        kx, ky = rng.integers(0, 3, size=2)
        a, ph = rng.uniform(-1, 1), rng.uniform(0, 2 * np.pi)
        out += amp / modes * a * np.cos(2 * np.pi * (kx * X / nx + ky * Y / ny) + ph)
    return out


def random_coupled(nx, ny, seed=0, rho_ratio=10.0, sigma=1e-3, U=0.01,
                   visc="linear", walls_y=False, cfl=0.5):
    """A generic coupled case with a wavy interface and a smooth random
    velocity, for invariance and parity tests."""
    X, Y = _centres(nx, ny)
    rng = np.random.default_rng(seed)
    amp = 0.05 * ny
    wave = amp * np.sin(2 * np.pi * X / nx + rng.uniform(0, 2 * np.pi))
    if walls_y:  # one wavy interface, heavy fluid above
        phi = tanh_profile(Y - 0.5 * ny - wave, 4.0, 1.0, 0.0)
    else:  # a wavy band of heavy fluid, smooth across the periodic seam
        phi = tanh_profile(0.25 * ny - np.abs(Y - 0.5 * ny - wave), 4.0, 1.0, 0.0)
    if walls_y:  # a smooth shear flow that vanishes at the walls
        u = smooth_field(nx, ny, seed + 1, amp=U, offset=U) * np.sin(np.pi * Y / ny)
        v = None
    else:
        u = smooth_field(nx, ny, seed + 1, amp=U)
        v = smooth_field(nx, ny, seed + 2, amp=U)
    params = dict(phi_H=1.0, phi_L=0.0, rho_H=rho_ratio, rho_L=1.0,
                  mu_H=0.1 * rho_ratio, mu_L=0.1, visc=visc, sigma=sigma,
                  W=4.0, M=0.05, cfl=cfl, walls_y=walls_y,
                  gy=-1e-6 if walls_y else 0.0, gravity="buoyancy")
    return _case(f"random_coupled_{nx}x{ny}_s{seed}", nx, ny, "coupled", params,
                 phi, u=u, v=v)


# ------------------------------------------------------- stretched meshes

def stretched_widths(n, amp=0.3, length=None, phase=0.0, periods=1):
    """Cell widths of a smoothly stretched axis: w_i proportional to
    1 + amp sin(2 pi periods (i + 1/2) / n + phase), scaled to sum to
    ``length`` (default n)."""
    i = np.arange(n) + 0.5
    w = 1.0 + amp * np.sin(2 * np.pi * periods * i / n + phase)
    return w * ((n if length is None else length) / w.sum())


def random_widths(n, seed, lo=0.5, hi=1.5):
    """Cell widths drawn uniformly from [lo, hi] (a rough mesh)."""
    return np.random.default_rng(seed).uniform(lo, hi, n)


def clustered_widths(n, length, centres, fine=0.5, spread=None):
    """Widths that shrink to ``fine`` times the mean near each of ``centres``
    (positions along the axis) and grow away from them: w proportional to
    1 - (1 - fine) exp(-((x - c) / spread)^2) summed over the centres,
    iterated so that the widths follow their own centres."""
    spread = length / 8.0 if spread is None else spread
    w = np.full(n, length / n)
    for _ in range(20):
        x = np.cumsum(w) - 0.5 * w
        g = np.ones(n)
        for c in centres:
            g -= (1.0 - fine) * np.exp(-((x - c) / spread) ** 2)
        w = g * (length / g.sum())
    return w


def mesh_centres(w):
    """Centres of cells of widths ``w`` starting at 0."""
    return np.cumsum(w) - 0.5 * w
