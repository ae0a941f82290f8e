"""The stationary bubble of Sec. IV.A at the benchmark's configuration
(128 x 128, R = 32, W = 5, density ratio 1000, sigma = 1e-3, nu = 0.1,
M = 0.1) run for the full 20000 steps on the HIP path: Laplace's law to the
accuracy the paper reports (numerical / analytical surface tension about
96.5 %), the spurious current below 1e-6 (the paper's statement), Sigma phi
conserved, and the FP32 run agreeing with the FP64 one."""
import json
import os

import numpy as np
import pytest

import paper_1810_07802_amd as D
import workloads as W

pytestmark = pytest.mark.gpu

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def thermo_pressure(phi, p, prm):
    """P = phi d(eps)/d(phi) - eps - kappa phi lap(phi) + kappa |grad phi|^2 / 2 + p
    (Sec. IV.A), with the isotropic stencils and the interface constants of the
    free energy (kappa = 3 sigma W / 2, beta = 12 sigma / W for phi in [0, 1])."""
    k = 1.5 * prm["sigma"] * prm["W"]
    b = 12.0 * prm["sigma"] / prm["W"]
    sh = lambda a, dx, dy: np.roll(np.roll(a, -dx, axis=1), -dy, axis=0)
    E, Wv, N, S = sh(phi, 1, 0), sh(phi, -1, 0), sh(phi, 0, 1), sh(phi, 0, -1)
    NE, NW, SE, SW = sh(phi, 1, 1), sh(phi, -1, 1), sh(phi, 1, -1), sh(phi, -1, -1)
    gx = (4 * (E - Wv) + (NE - NW) + (SE - SW)) / 12.0
    gy = (4 * (N - S) + (NE - SE) + (NW - SW)) / 12.0
    lap = (4 * (E + Wv + N + S) + (NE + NW + SE + SW) - 20 * phi) / 6.0
    eps = b * phi ** 2 * (phi - 1) ** 2
    deps = 2 * b * phi * (phi - 1) * (2 * phi - 1)
    return phi * deps - eps - k * phi * lap + 0.5 * k * (gx ** 2 + gy ** 2) + p


def run(prec):
    c = W.bubble()  # 128 x 128, R = 32, 20000 steps
    s = D.Solver(c["nx"], c["ny"], c["params"], "coupled", prec)
    s.init(c["phi"])
    L, R = c["nx"], 32.0
    X, Y = np.meshgrid(np.arange(L) + 0.5, np.arange(L) + 0.5)
    r = np.hypot(X - L / 2, Y - L / 2)
    s.step(15000)
    ratios = []
    for _ in range(10):  # time average over the last 5000 steps
        s.step(500)
        m = s.macros()
        P = thermo_pressure(m["phi"], m["p"], c["params"])
        ratios.append((P[r < R / 2].mean() - P[r > R + 10].mean()) * R / c["params"]["sigma"])
    d = s.diagnostics()
    return float(np.mean(ratios)), d, m, c


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_laplace_law_and_spurious_current_20000_steps(prec):
    ratio, d, m, c = run(prec)
    print(f"C2 bubble {prec}: Delta P R / sigma = {ratio:.4f} (paper ~{GOLD['laplace_ratio']['value']}), "
          f"max|u| = {d['max_u']:.3e}, nonfinite = {d['nonfinite']}", flush=True)
    assert d["nonfinite"] == 0
    assert 0.90 < ratio < 1.02
    assert d["max_u"] < 1e-6
    # Sigma phi: conserved to rounding, which accumulates over the 20000 steps.
    # FP64: about 5e-17 (relative) per step, 1.0e-12 after 20000 steps. FP32:
    # every step rounds each stored population to float; the total drifts by a
    # few 1e-10 per step on this case, 7e-6 after 20000 steps
    tol = 1e-11 if prec == "fp64" else 2e-5
    assert abs(m["phi"].sum() - c["phi"].sum()) / c["phi"].sum() < tol


def centroid(phi):
    w = 1.0 - phi  # the light phase (phi = 0) fills the bubble
    ny, nx = phi.shape
    X, Y = np.meshgrid(np.arange(nx) + 0.5, np.arange(ny) + 0.5)
    return np.array([(w * X).sum(), (w * Y).sum()]) / w.sum()


def test_fp32_agrees_with_fp64_after_20000_steps():
    """After 1000 steps the FP32 path is within 1e-5 of FP64 on phi
    (test_gpu_configs.py). Over 20000 steps float rounding of the interface
    profile accumulates: measured, phi differs by 2.7e-4 (relative L2) while
    the bubble's centroid agrees to 7e-5 cells and the Laplace ratios to
    4e-4. The bounds are on those three quantities."""
    r32, _, m32, _ = run("fp32")
    r64, _, m64, _ = run("fp64")
    e_phi = np.linalg.norm(m32["phi"] - m64["phi"]) / np.linalg.norm(m64["phi"])
    shift = np.hypot(*(centroid(m32["phi"]) - centroid(m64["phi"])))
    print(f"C2 fp32 vs fp64: phi rel L2 {e_phi:.2e}, centroid shift {shift:.2e} cells, "
          f"Laplace ratios {r32:.4f} / {r64:.4f}", flush=True)
    assert shift < 0.01
    assert e_phi < 1e-3
    assert abs(r32 - r64) < 0.01
