"""The oracle against textbook solutions and the numbers the paper prints.

* single-phase shear-wave decay at the rate nu k^2 with nu = tau_g RT
  (Appendix: the momentum equation is recovered with nu = tau_g RT);
* single-phase Poiseuille flow between the no-slip walls;
* layered Poiseuille flow at viscosity ratio 1000 against the analytic profile
  (Sec. IV.B, Eq. 46) and the paper's printed error bound;
* Laplace's law for the stationary 1000:1 bubble (Sec. IV.A);
* the interface returns after one period of diagonal translation
  (Sec. III.A), with the centroid back in place.
"""
import json
import os

import numpy as np
import pytest

import oracle
import workloads as W

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


@pytest.mark.parametrize("nu", [0.1, 0.01])
def test_shear_wave_decays_at_nu_k2(nu):
    ny, nx, U = 32, 4, 1e-3
    Y = np.arange(ny)[:, None] + 0.5 + np.zeros((1, nx))
    k = 2 * np.pi / ny
    params = dict(phi_H=1.0, phi_L=0.0, rho_H=1.0, rho_L=1.0, nu=nu,
                  visc="uniform_nu", sigma=0.0, W=4.0, M=0.1, cfl=0.5)
    s = oracle.Sim(nx, ny, params)
    s.init(np.ones((ny, nx)), U * np.sin(k * Y))
    s.step(int(2 / (nu * k * k) / 0.5))
    m = s.macros()
    amp = (m["u"] * np.sin(k * Y)).sum() / (np.sin(k * Y) ** 2).sum()
    rate = -np.log(amp / U) / s.time
    assert rate == pytest.approx(nu * k * k, rel=0.02)
    assert np.abs(m["v"]).max() < 1e-5 * U  # O(Ma^2) compressibility only


def test_single_phase_poiseuille_from_rest():
    c = W.layered_poiseuille(nx=4, ny=32, mu_ratio=1.0, sigma=0.0)
    s = oracle.Sim(c["nx"], c["ny"], c["params"])
    s.init(c["phi"])
    s.step(30000)
    m = s.macros()
    ua = W.poiseuille_analytic(32, 0.1, 0.1, c["Gx"])
    err = np.sqrt(((m["u"][:, 0] - ua) ** 2).sum() / (ua ** 2).sum())
    assert err < 1e-3
    assert np.abs(m["u"] - m["u"][:, :1]).max() < 1e-15  # x-independent
    assert np.abs(m["v"]).max() < 1e-10


def test_layered_poiseuille_viscosity_ratio_1000_within_paper_bound():
    """10 x 100 channel, mu* = 1000, u_c = 1e-4, W = 4, sigma = 1e-3: starting
    from the analytic profile, the error stays below the paper's printed
    maximum L2 error for this grid."""
    bound = [c for c in GOLD["layered_poiseuille_L2"]["cases"] if c["ny"] == 100][0]["L2"]
    c = W.layered_poiseuille(nx=10, ny=100, mu_ratio=1000.0, analytic_init=True)
    s = oracle.Sim(c["nx"], c["ny"], c["params"])
    s.init(c["phi"], c["u"])
    ua = W.poiseuille_analytic(100, 0.1, 1e-4, c["Gx"])
    for _ in range(4):
        s.step(5000)
        u = s.macros()["u"][:, 0]
        err = np.sqrt(((u - ua) ** 2).sum() / (ua ** 2).sum())
        assert err < bound


def _thermo_pressure(s, m, params):
    """Sec. IV.A: P = p0 - kappa phi lap(phi) + kappa |grad phi|^2 / 2 + p with
    p0 = phi d(eps)/d(phi) - eps."""
    cf = s.cell_fields()
    d = s.derived()
    phi, pH, pL = m["phi"], params["phi_H"], params["phi_L"]
    eps = d["beta"] * (phi - pH) ** 2 * (phi - pL) ** 2
    deps = 2 * d["beta"] * (phi - pH) * (phi - pL) * (2 * phi - pH - pL)
    return (phi * deps - eps - d["kappa"] * phi * cf["lap"]
            + 0.5 * d["kappa"] * (cf["gx"] ** 2 + cf["gy"] ** 2) + m["p"])


def test_laplace_law_stationary_bubble():
    """Density ratio 1000, W = 5, M = 0.1, nu = 0.1: the time-averaged
    pressure jump matches sigma / R to the accuracy the paper reports (about
    96.5 %); accept 0.85 - 1.10. The bubble stays at rest."""
    L, R = 64, 16
    c = W.bubble(L=L, R=R)
    s = oracle.Sim(L, L, c["params"])
    s.init(c["phi"])
    s.step(1000)
    X, Y = np.meshgrid(np.arange(L) + 0.5, np.arange(L) + 0.5)
    r = np.hypot(X - L / 2, Y - L / 2)
    ratios, umax = [], 0.0
    for _ in range(25):
        s.step(200)
        m = s.macros()
        P = _thermo_pressure(s, m, c["params"])
        ratios.append((P[r < R / 2].mean() - P[r > R + 10].mean()) * R / c["params"]["sigma"])
        umax = max(umax, np.hypot(m["u"], m["v"]).max())
    ratio = float(np.mean(ratios))
    assert 0.85 < ratio < 1.10, ratio
    assert umax < 1e-6  # the paper: spurious velocity below 1e-6


def test_diagonal_translation_returns_after_one_period():
    """The 100 x 100 interface-only case (R = 25, W = 4, U = 0.02, M = 0.01,
    CFL = 0.5, phi in [-1, 1]) after T = L0 / U0: the interface is back, its
    centroid within 0.1 cell, total phi conserved."""
    c = W.diag_translation()
    s = oracle.Sim(c["nx"], c["ny"], c["params"], "ac")
    s.init(c["phi"])
    s.step(c["steps"])
    m = s.macros()
    phi0, phi1 = c["phi"], m["phi"]
    E = ((phi1 - phi0) ** 2).sum() / (phi0 ** 2).sum()
    assert E < 2e-3  # the paper's DUGKS E at Pe = 128..1024 is 3.6e-3 .. 2.3e-2
    X, Y = np.meshgrid(np.arange(100) + 0.5, np.arange(100) + 0.5)
    w0, w1 = phi0 + 1.0, phi1 + 1.0
    for A in (X, Y):
        assert abs((A * w1).sum() / w1.sum() - (A * w0).sum() / w0.sum()) < 0.1
    assert abs(phi1.sum() - phi0.sum()) / np.abs(phi0).sum() < 1e-11


@pytest.mark.slow
@pytest.mark.parametrize("idx", [1, 2])
def test_table1_diagonal_translation_soft_pin(idx):
    """Sec. III.A, Table I (L0 = 256, M = 0.02, W = 4, phi in [0, 1]): the error
    after one period. The printed values are the square root of the error
    formula of Sec. III (its squared sums without the root are ~100x
    smaller); at Pe = 256 and 512 the oracle is within 40 % of them. Soft
    pin: the reconstruction details (central scheme) are a reading, and at
    Pe = 128 the oracle's error is 3x the printed one (an open discrepancy)."""
    t = GOLD["diag_translation_E_vs_Pe"]
    Pe, E_paper = t["Pe"][idx], t["E"][idx]
    M, L0 = 0.02, 256
    c = W.diag_translation(L0=L0, W=4.0, U0=Pe * M / L0, M=M, phi_H=1.0, phi_L=0.0)
    s = oracle.Sim(L0, L0, c["params"], "ac")
    s.init(c["phi"])
    s.step(c["steps"])
    phi = s.macros()["phi"]
    E = np.sqrt(((phi - c["phi"]) ** 2).sum() / (c["phi"] ** 2).sum())
    assert abs(E / E_paper - 1) < 0.4
