"""Pins of oracle readings that the paper states only in words (-m "not gpu").

R7, the unit normal n of Sec. II.A: the oracle regularises it as
grad phi / sqrt(|grad phi|^2 + eps^2) (eps_n = 1e-6 by default) and takes the
plain unit normal with eps_n = 0. The two readings must give the same
paper-fixed outputs: the one-period interface error of Sec. III (Tables I,
III, V), the Laplace pressure jump of Sec. IV.A, the layered-Poiseuille error
of Sec. IV.B; the bounds below are a few times what was measured.

R16, the body force G of Eq. 8 (rho g, or (rho - mean rho) g): a stably
stratified fluid (heavy phase below a flat interface) between no-slip walls,
started from the hydrostatic pressure of its density profile, stays at rest,
its pressure gradient balances G in the bulk, and a perturbation at the
rounding level does not grow. A wrong sign, factor or reference density in G
breaks the balance and sets the fluid in motion.

R12, the linear viscosity interpolation of Sec. II.B (Eq. 36): the layered
Poiseuille flow with linear mu(s) reaches the steady profile of the momentum
balance d/dy (mu du/dy) = -G_x, u = 0 at both walls, solved by quadrature
for mu(y) of the initial tanh profile: at second order in the grid, and far
from the profile of the reciprocal interpolation (Eq. 35)."""
import numpy as np
import pytest

import oracle
import workloads as W


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _run(c, steps, **extra):
    o = oracle.Sim(c["nx"], c["ny"], dict(c["params"], **extra), c["model"])
    o.init(c["phi"], c.get("u"), c.get("v"), c.get("p"))
    o.step(steps)
    return o.macros()


def _sqrt_e(phi, phi0):
    # the printed one-period error: the root of sum |phi(T)-phi(0)|^2 / sum |phi(0)|^2
    return np.sqrt(np.sum((phi - phi0) ** 2) / np.sum(phi0 ** 2))


# ------------------------------------------------------------------- R7

@pytest.mark.parametrize("name", ["diag", "zalesak", "shear"])
def test_plain_and_regularised_normal_give_the_same_interface_error(name):
    c = {"diag": lambda: W.diag_translation(),
         "zalesak": lambda: W.zalesak(L0=64, R=25, slot=5),
         "shear": lambda: W.shear_elongation(L0=64)}[name]()
    a = _run(c, c["steps"])
    b = _run(c, c["steps"], eps_n=0.0)
    ea, eb = _sqrt_e(a["phi"], c["phi"]), _sqrt_e(b["phi"], c["phi"])
    print(f"{name}: sqrt E eps 1e-6 {ea:.6e}, plain {eb:.6e}, rel phi {rel(b['phi'], a['phi']):.2e}")
    # measured: relative field differences 0.9e-6 .. 6.9e-6
    assert rel(b["phi"], a["phi"]) < 3e-5
    assert abs(ea - eb) < 1e-3 * ea


def test_plain_and_regularised_normal_give_the_same_bubble_and_poiseuille():
    c = W.bubble(L=64, R=16, steps=0)
    a, b = _run(c, 1000), _run(c, 1000, eps_n=0.0)
    X, Y = np.meshgrid(np.arange(64) + 0.5, np.arange(64) + 0.5)
    r = np.hypot(X - 32, Y - 32)
    dp = [m["p"][r < 8].mean() - m["p"][r > 16 + 4 * 5].mean() for m in (a, b)]
    print(f"bubble: pressure jump {dp[0]:.6e} / {dp[1]:.6e}, rel phi {rel(b['phi'], a['phi']):.2e}")
    assert rel(b["phi"], a["phi"]) < 3e-6  # measured 5.5e-7
    assert abs(dp[0] - dp[1]) < 1e-3 * abs(dp[0])
    c = W.layered_poiseuille(analytic_init=True, steps=0)
    a, b = _run(c, 2000), _run(c, 2000, eps_n=0.0)
    ua = W.poiseuille_analytic(c["ny"], c["params"]["mu_H"], c["params"]["mu_L"], c["Gx"])
    ea, eb = (rel(m["u"][:, 0], ua) for m in (a, b))
    print(f"poiseuille: L2 error {ea:.6e} / {eb:.6e}, rel phi {rel(b['phi'], a['phi']):.2e}")
    assert rel(b["phi"], a["phi"]) < 3e-6  # measured 4.1e-7
    assert abs(ea - eb) < 1e-3 * ea


def test_plain_normal_is_zero_on_a_uniform_field():
    # eps_n = 0: n is undefined where grad phi = 0; the reading takes n = 0
    # there, so a uniform state stays uniform (no division by zero)
    c = W.bubble(L=32, R=8, steps=0)
    c["phi"] = np.full_like(c["phi"], 0.3)
    m = _run(c, 20, eps_n=0.0)
    assert np.all(np.isfinite(m["phi"])) and np.all(m["phi"] == m["phi"][0, 0])


# ------------------------------------------------------------------ R16

def _stratified(form, nx=16, ny=256):
    """Heavy phase below a flat interface at mid-height, no-slip walls, the
    Rayleigh-Taylor fluids (density 3:1, gravity g = 6.25e-6), at rest, with
    the hydrostatic pressure of the density profile (trapezoid rule)."""
    X, Y = np.meshgrid(np.arange(nx) + 0.5, np.arange(ny) + 0.5)
    prm = dict(W.rayleigh_taylor()["params"], gravity=form)
    phi = W.tanh_profile(ny / 2 - Y, prm["W"], 1.0, 0.0)
    rho = prm["rho_L"] + (prm["rho_H"] - prm["rho_L"]) * phi[:, 0]
    ref = 0.5 * (prm["rho_H"] + prm["rho_L"]) if form == "buoyancy" else 0.0
    G = (rho - ref) * prm["gy"]  # the body force the paper names (Eq. 8), per unit volume
    p = np.concatenate([[0.0], np.cumsum(0.5 * (G[1:] + G[:-1]))])
    p0 = np.repeat((p - p.mean())[:, None], nx, axis=1)
    return prm, phi, p0, G


@pytest.mark.parametrize("form", ["buoyancy", "rho_g"])
def test_stably_stratified_fluid_stays_at_rest_in_hydrostatic_balance(form):
    prm, phi, p0, G = _stratified(form)
    nx, ny = phi.shape[1], phi.shape[0]
    a = oracle.Sim(nx, ny, prm, "coupled")
    a.init(phi, None, None, p0)
    b = oracle.Sim(nx, ny, prm, "coupled")
    b.init(phi * (1 + 1e-13 * np.random.default_rng(2).standard_normal(phi.shape)), None, None, p0)
    a.step(1000)
    b.step(1000)
    ma, mb = a.macros(), b.macros()
    g = abs(prm["gy"])
    U = np.sqrt(g * ny)  # free-fall velocity scale of the column
    umax = max(np.abs(ma["u"]).max(), np.abs(ma["v"]).max())
    dpdy = np.gradient(ma["p"][:, nx // 2])
    bulk = np.r_[20:100, 156:236]  # away from the walls and the interface
    err = np.abs(dpdy[bulk] - G[bulk]).max()
    print(f"{form}: max|u| {umax:.2e} (U {U:.2e}), |dp/dy - G| {err:.2e} (|G| {np.abs(G[bulk]).min():.2e}), "
          f"perturbation {np.abs(ma['phi'] - mb['phi']).max():.2e}")
    assert umax < 1e-3 * U  # measured 1.3e-6 against U = 0.04
    assert err < 0.05 * np.abs(G[bulk]).min()
    assert np.abs(ma["phi"] - mb["phi"]).max() < 1e-11


def test_gravity_without_hydrostatic_start_compresses_the_column():
    """The same column from p = 0 is not in balance: the weakly compressible
    g model sets it in motion (the acoustic adjustment), which moves phi off
    phi_H in the heavy bulk; a rounding-level perturbation then grows there
    (the sharpening flux M theta n is anti-diffusive where phi is off phi_H
    and the gradient is flatter than theta). The hydrostatic start above has
    neither."""
    prm, phi, p0, G = _stratified("buoyancy")
    nx, ny = phi.shape[1], phi.shape[0]
    a = oracle.Sim(nx, ny, prm, "coupled")
    a.init(phi)
    b = oracle.Sim(nx, ny, prm, "coupled")
    b.init(phi * (1 + 1e-13 * np.random.default_rng(2).standard_normal(phi.shape)))
    a.step(750)
    b.step(750)
    ma, mb = a.macros(), b.macros()
    assert np.abs(ma["v"]).max() > 1e-5
    assert np.abs(ma["phi"][: ny // 2 - 20] - 1.0).max() > 1e-6
    assert np.abs(ma["phi"] - mb["phi"]).max() > 1e-8


# ------------------------------------------------------------------ R12

def _ode_profile(ny, phi_col, mu_H, mu_L, Gx, mode):
    """Steady velocity of a layered channel flow, d/dy (mu du/dy) = -Gx with
    u(0) = u(ny) = 0, by quadrature on a fine grid; mu(y) interpolated in s
    (linear or reciprocal) from the cell values of phi."""
    from scipy.integrate import cumulative_trapezoid as ct
    yf = np.linspace(0.0, ny, 400 * ny + 1)
    yc = np.arange(ny) + 0.5
    s = np.clip(np.interp(yf, yc, phi_col), 0.0, 1.0)
    mu = s * mu_H + (1 - s) * mu_L if mode == "linear" else 1.0 / (s / mu_H + (1 - s) / mu_L)
    i1, i0 = ct(yf / mu, yf, initial=0.0), ct(1.0 / mu, yf, initial=0.0)
    u = -Gx * (i1 - i1[-1] / i0[-1] * i0)
    return np.interp(yc, yf, u)


def test_linear_viscosity_poiseuille_converges_to_its_ode_profile():
    errs = []
    for ny, steps in ((32, 5000), (64, 20000)):
        c = W.layered_poiseuille(nx=4, ny=ny, mu_ratio=10.0, mu_H=1.0, uc=1e-4, visc="linear")
        m = _run(c, steps)
        phi_col = W.tanh_profile(0.5 * ny - (np.arange(ny) + 0.5), 4.0, 1.0, 0.0)
        prm = c["params"]
        lin = _ode_profile(ny, phi_col, prm["mu_H"], prm["mu_L"], c["Gx"], "linear")
        rec = _ode_profile(ny, phi_col, prm["mu_H"], prm["mu_L"], c["Gx"], "reciprocal")
        u = m["u"][:, 0]
        errs.append(rel(u, lin))
        print(f"ny {ny}: error to the linear-mu profile {errs[-1]:.2e}, to the reciprocal one {rel(u, rec):.2e}")
        assert rel(u, rec) > 5 * errs[-1]
    assert errs[0] < 0.03
    assert errs[0] / errs[1] > 3.3  # second order (measured 4.0)
