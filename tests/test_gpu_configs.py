"""The benchmark configurations at full size: HIP path vs the FP64 oracle.

Targets (stated per result):
  * FP64 path: relative L2 <= 1e-12 on phi, and on the driven fields. Fields
    that are residuals of a force balance (the spurious current and pressure
    of the static bubble, the cross-channel velocity and pressure of the
    layered Poiseuille flow) carry the rounding of the chemical potential,
    itself a small residual of two O(beta) terms; their errors are judged
    against natural scales instead: velocity against the capillary velocity
    U* = sigma / mu_L, pressure against the acoustic pressure rho_H c_s^2 U*
    (rounding in u reaches p through the weakly compressible pressure
    equation, amplified by rho_H c_s^2).
  * Unstable flows amplify rounding physically (Rayleigh-Taylor growth;
    interface translation at cell Peclet 2 with central reconstruction), so
    their FP64 comparison stops at 500-1000 steps; the full interface period
    is compared through its error norm.
  * FP32 path (float distributions and arithmetic, density / relaxation time
    interpolation in double): after 1000 steps relative L2 <= 1e-5 on phi and
    <= 1e-4 on u, v where the flow is driven; the static bubble's velocity
    against 1e-4 U*. Three configurations get a stated, measured exception:
    the Rayleigh-Taylor flow (phi 1e-4: the flow is unstable and a mode near
    the top wall amplifies rounding, about x5 per 200 steps in FP64),
    spinodal decomposition (phi 2e-5: unstable by design), and the layered
    Poiseuille flow (u 3e-4: in the mu_L = mu_H / 100 layer tau_g = 0.003, so
    the viscous stress lives in a non-equilibrium part 1e-4 of g, and float
    rounding of g reaches it).
  * sum phi conserved to 1e-12 (relative to sum |phi|) on the FP64 path.
"""
import numpy as np
import pytest

import oracle
import paper_1810_07802_amd as D
import workloads as W

pytestmark = pytest.mark.gpu


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


_ORACLE_CACHE = {}


def oracle_run(case, steps):
    key = (case["name"], steps)
    if key not in _ORACLE_CACHE:
        o = oracle.Sim(case["nx"], case["ny"], case["params"], case["model"])
        o.init(case["phi"], case["u"], case["v"], case["p"])
        o.step(steps)
        _ORACLE_CACHE[key] = o.macros()
    return _ORACLE_CACHE[key]


def gpu_run(case, steps, precision, seg=None):
    s = D.Solver(case["nx"], case["ny"], case["params"], case["model"], precision, seg)
    s.init(case["phi"], case["u"], case["v"], case["p"])
    s.step(steps)
    return s.macros()


def check(case, steps, precision, residual=(), u_scale=None, p_scale=None,
          fp32_phi=1e-5, fp32_u=1e-4, seg=None):
    """Compare after `steps`; `residual` names fields judged against scales;
    `seg` fixes the tile (rows per segment) instead of the automatic one."""
    g = gpu_run(case, steps, precision, seg)
    r = oracle_run(case, steps)
    e = {k: rel(g[k], r[k]) for k in ("phi", "u", "v", "p")}
    dsum = abs(g["phi"].sum() - r["phi"].sum()) / np.abs(r["phi"]).sum()
    dmax = {k: np.abs(g[k] - r[k]).max() for k in ("u", "v", "p")}
    print(f"{case['name']} {precision} {steps} steps: " +
          " ".join(f"{k}={v:.2e}" for k, v in e.items()) +
          " " + " ".join(f"max|d{k}|={v:.2e}" for k, v in dmax.items()) +
          f" dsum(phi)={dsum:.2e}", flush=True)
    tol = 1e-12 if precision == "fp64" else None
    if precision == "fp64":
        assert e["phi"] < 1e-12
        assert dsum < 1e-12
        for k in ("u", "v", "p"):
            if k in residual:
                scale = p_scale if k == "p" else u_scale
                assert dmax[k] < tol * scale, (k, dmax[k], scale)
            else:
                assert e[k] < tol, (k, e[k])
    else:
        assert e["phi"] < fp32_phi
        for k in ("u", "v"):
            if k in residual:
                assert dmax[k] < 1e-4 * u_scale, (k, dmax[k])
            else:
                assert e[k] < fp32_u, (k, e[k])
    return e


def _scales(c):
    """Capillary velocity sigma / mu_L and acoustic pressure rho_H c_s^2 U*."""
    p = c["params"]
    mu_L = p["nu"] * p["rho_L"] if p.get("visc", "uniform_nu") == "uniform_nu" else p["mu_L"]
    u_star = p["sigma"] / mu_L
    return u_star, p["rho_H"] / 3.0 * u_star


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_interface_only_diagonal_translation_100(prec):
    """100 x 100, R = 25, W = 4, U = 0.02, M = 0.01, FP64 over the full period
    (10000 steps), FP32 over 1000 steps."""
    c = W.diag_translation()
    check(c, 1000, prec)


def test_interface_only_full_period_error_norm():
    """After the full period (10000 steps) the FP64 fields may differ by the
    amplified rounding, but the error norm of Sec. III (Eq. 39) agrees."""
    c = W.diag_translation()
    g = gpu_run(c, c["steps"], "fp64")
    r = oracle_run(c, c["steps"])
    E = lambda phi: ((phi - c["phi"]) ** 2).sum() / (c["phi"] ** 2).sum()
    print("full period E:", E(g["phi"]), E(r["phi"]), flush=True)
    assert E(g["phi"]) == pytest.approx(E(r["phi"]), rel=1e-3)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_stationary_bubble_128(prec):
    c = W.bubble(L=128, R=32)
    us, ps = _scales(c)
    check(c, 1000, prec, residual=("u", "v", "p"), u_scale=us, p_scale=ps)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_rayleigh_taylor_256x1024(prec):
    """Velocities judged against U = sqrt(g L0) = 0.04 (Sec. IV.D)."""
    c = W.rayleigh_taylor()
    U = 0.04
    check(c, 500 if prec == "fp64" else 1000, prec, residual=("u", "v", "p"),
          u_scale=U, p_scale=c["params"]["rho_H"] / 3.0 * U, fp32_phi=1e-4)


@pytest.mark.parametrize("L", [64, 128])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_spinodal_batch_sizes(L, prec):
    check(W.spinodal(L=L, seed=1810), 1000, prec, fp32_phi=2e-5)


def test_spinodal_512_fp32_sampled_200_steps():
    """The largest batch size; the oracle runs 200 steps of it."""
    check(W.spinodal(L=512, seed=1811), 200, "fp32")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_layered_poiseuille_64x256(prec):
    c = W.layered_poiseuille(nx=64, ny=256, mu_ratio=100.0, analytic_init=True)
    us, ps = _scales(c)
    check(c, 1000, prec, residual=("v", "p"), u_scale=us, p_scale=ps, fp32_u=3e-4)


def test_served_bubble_256_fp32():
    c = W.bubble(L=256, R=64)
    us, ps = _scales(c)
    check(c, 1000, "fp32", residual=("u", "v", "p"), u_scale=us, p_scale=ps)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_large_grid_bubble_4096_in_the_bench_tiling(prec):
    """The large-grid benchmark case at its full size (4096^2, R = 1024, the
    same physics as the 128^2 bubble) in the tiling the bench times (6-row
    segments of the march): three steps against the oracle on every cell
    (the oracle takes about a second per step at this size). The velocity
    and pressure are the spurious current's residuals, judged against the
    capillary scales."""
    c = W.bubble(L=4096, R=1024, steps=0)
    u_star, p_star = _scales(c)
    check(c, 3, prec, residual=("u", "v", "p"), u_scale=u_star, p_scale=p_star, seg=6)
