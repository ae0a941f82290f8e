"""Pins of the oracle's upwind, limited face reconstruction.

Sec. III attributes the growth of the interface error with the Peclet number
to the numerical dissipation of the central reconstruction and names an
upwind reconstruction with a limiter as the remedy. The oracle's upwind mode
traces the population crossing a face back by h xi into its upwind cell and
evaluates it there with van Leer limited slopes. These tests fix it from
outside itself:

* exactness on linear data (the second-order property both reconstructions
  share), which a wrong sign, offset, axis or upwind cell breaks;
* the limiter's bound: every upwind face value lies between the smallest and
  largest of the cells its stencil reads, for any data (away from the
  unlimited one-sided slopes next to a wall), which the central
  reconstruction does not satisfy;
* zero slope at a local extremum (van Leer's defining property);
* the invariants of the full step (conservation of phi, uniform states,
  integer-shift, mirror and transpose equivariance);
* the paper's claim itself: at high Peclet number the upwind mode transports
  a drop with a smaller error than the central one.
"""
import numpy as np
import pytest

import oracle
import workloads as W

H = 0.25  # h = dt/2 at CFL 0.5
EX = [0, 1, 1, 0, -1, -1, -1, 0, 1]
EY = [0, 0, 1, 1, 1, 0, -1, -1, -1]


def _linear(nx, ny, c0=0.3, cx=0.07, cy=-0.11):
    y, x = np.mgrid[0:ny, 0:nx] + 0.5
    return c0 + cx * x + cy * y, (c0, cx, cy)


@pytest.mark.parametrize("mode", ["central", "upwind"])
@pytest.mark.parametrize("walls", [False, True])
def test_linear_data_is_reconstructed_exactly(mode, walls):
    """On a linear field the bar value at a face is the field at the point
    the population left from, x_f - h xi, in both reconstructions (on faces
    whose stencil does not cross the periodic seam)."""
    nx, ny = 12, 10
    a, (c0, cx, cy) = _linear(nx, ny)
    for q in range(9):
        xf, yf = oracle.recon(a, q, H, mode, walls_y=walls)
        # x-face east of (i, j) at (i + 1, j + 1/2)
        jr = range(ny) if walls else range(1, ny - 1)
        for j in jr:
            for i in range(1, nx - 3):
                exact = c0 + cx * (i + 1 - H * EX[q]) + cy * (j + 0.5 - H * EY[q])
                assert xf[j, i] == pytest.approx(exact, abs=1e-14), (q, i, j)
        # y-face north of (i, j) at (i + 1/2, j + 1)
        for j in range(1, ny - 3):
            for i in range(1, nx - 1):
                exact = c0 + cx * (i + 0.5 - H * EX[q]) + cy * (j + 1 - H * EY[q])
                assert yf[j, i] == pytest.approx(exact, abs=1e-14), (q, i, j)


def _nbhd(a, i, j, walls):
    """Values of cell (i, j) and its four neighbours (x periodic)."""
    ny, nx = a.shape
    out = [a[j, i], a[j, (i - 1) % nx], a[j, (i + 1) % nx]]
    for jj in (j - 1, j + 1):
        if walls and not 0 <= jj < ny:
            continue
        out.append(a[jj % ny, i])
    return out


def _stencil_range(a, q, i, j, axis, walls):
    ny, nx = a.shape
    if axis == "x":
        L, R = (i, j), ((i + 1) % nx, j)
        e = EX[q]
    else:
        L, R = (i, j), (i, (j + 1) % ny)
        e = EY[q]
    cells = [L] if e > 0 else [R] if e < 0 else [L, R]
    vals = [v for c in cells for v in _nbhd(a, c[0], c[1], walls)]
    return min(vals), max(vals)


@pytest.mark.parametrize("walls", [False, True])
def test_upwind_values_stay_within_their_stencil(walls):
    rng = np.random.default_rng(7)
    nx, ny = 11, 9
    viol_central = 0
    for trial in range(4):
        a = rng.standard_normal((ny, nx))
        for q in range(9):
            xf, yf = oracle.recon(a, q, H, "upwind", walls_y=walls)
            cx_, cy_ = oracle.recon(a, q, H, "central", walls_y=walls)
            for j in range(ny):
                for i in range(nx):
                    lo, hi = _stencil_range(a, q, i, j, "x", walls)
                    viol_central += not (lo <= cx_[j, i] <= hi)
                    # next to a wall the y-slope is the one-sided difference,
                    # unlimited: x-faces of the wall rows are exempt for
                    # populations with a y component
                    if not (walls and j in (0, ny - 1) and EY[q] != 0):
                        assert lo - 1e-14 <= xf[j, i] <= hi + 1e-14, ("x", q, i, j)
                    if walls and j == ny - 1:
                        continue
                    lo, hi = _stencil_range(a, q, i, j, "y", walls)
                    assert lo - 1e-14 <= yf[j, i] <= hi + 1e-14, ("y", q, i, j)
                    viol_central += not (lo <= cy_[j, i] <= hi)
    # the bound is a property of the limiter, not of any reconstruction
    assert viol_central > 0


def test_slope_vanishes_at_a_local_extremum():
    """At a strict local maximum the van Leer slopes are zero: a population
    leaving that cell carries the cell value to both faces."""
    nx, ny = 9, 9
    a, _ = _linear(nx, ny)
    a[4, 4] = 5.0
    for q in range(9):
        xf, yf = oracle.recon(a, q, H, "upwind")
        if EX[q] > 0:
            assert xf[4, 4] == 5.0
        if EX[q] < 0:
            assert xf[4, 3] == 5.0
        if EY[q] > 0:
            assert yf[4, 4] == 5.0
        if EY[q] < 0:
            assert yf[3, 4] == 5.0


def _upwind(c):
    c = dict(c)
    c["params"] = dict(c["params"], recon="upwind")
    return c


def _run(case, steps):
    s = oracle.Sim(case["nx"], case["ny"], case["params"], case["model"])
    s.init(case["phi"], case["u"], case["v"], case["p"])
    s.step(steps)
    return s


@pytest.mark.parametrize("which", ["coupled_periodic", "coupled_walls", "ac_deform"])
def test_phi_is_conserved(which):
    if which == "coupled_periodic":
        c = W.random_coupled(24, 20, seed=3, rho_ratio=100.0)
    elif which == "coupled_walls":
        c = W.random_coupled(16, 24, seed=4, rho_ratio=10.0, walls_y=True)
    else:
        c = W.smoothed_deformation(L0=32, Pe=256, M=0.02)
    c = _upwind(c)
    s = oracle.Sim(c["nx"], c["ny"], c["params"], c["model"])
    s.init(c["phi"], c["u"], c["v"], c["p"])
    t0 = s.macros()["phi"].sum()
    s.step(300)
    assert abs(s.macros()["phi"].sum() - t0) / np.abs(c["phi"]).sum() < 1e-12


def test_uniform_state_is_preserved():
    nx, ny = 7, 9
    phi = np.full((ny, nx), 0.37)
    params = dict(phi_H=1.0, phi_L=0.0, rho_H=50.0, rho_L=1.0, sigma=1e-3, visc="reciprocal",
                  mu_H=0.2, mu_L=0.02, M=0.05, recon="upwind")
    s = oracle.Sim(nx, ny, params)
    s.init(phi, np.full_like(phi, 0.013), np.full_like(phi, -0.007), np.full_like(phi, 2e-3))
    st0 = s.get_state()
    s.step(50)
    st1 = s.get_state()
    np.testing.assert_allclose(st1["f"], st0["f"], rtol=0, atol=1e-14)
    np.testing.assert_allclose(st1["g"], st0["g"], rtol=0, atol=2e-13)


@pytest.mark.parametrize("shift", [(3, 0), (0, 5), (7, 2)])
def test_integer_shift_equivariance_is_bitwise(shift):
    sx, sy = shift
    c = _upwind(W.random_coupled(20, 16, seed=11, rho_ratio=30.0))
    a = _run(c, 40).macros()
    c2 = dict(c)
    for k in ("phi", "u", "v"):
        c2[k] = np.roll(c[k], (sy, sx), axis=(0, 1))
    b = _run(c2, 40).macros()
    for k in ("phi", "u", "v", "p"):
        assert np.array_equal(np.roll(a[k], (sy, sx), axis=(0, 1)), b[k]), k


def test_mirror_x_equivariance():
    c = _upwind(W.random_coupled(18, 14, seed=21, rho_ratio=50.0))
    a = _run(c, 60).macros()
    c2 = dict(c)
    c2["phi"] = c["phi"][:, ::-1]
    c2["u"] = -c["u"][:, ::-1]
    c2["v"] = c["v"][:, ::-1]
    b = _run(c2, 60).macros()
    np.testing.assert_allclose(b["phi"], a["phi"][:, ::-1], rtol=0, atol=1e-12)
    np.testing.assert_allclose(b["u"], -a["u"][:, ::-1], rtol=0, atol=1e-13)
    np.testing.assert_allclose(b["v"], a["v"][:, ::-1], rtol=0, atol=1e-13)
    np.testing.assert_allclose(b["p"], a["p"][:, ::-1], rtol=0, atol=1e-12)


def test_mirror_y_equivariance_with_walls_and_gravity():
    c = _upwind(W.random_coupled(12, 16, seed=22, rho_ratio=10.0, walls_y=True))
    c["u"] = None
    a = _run(c, 60).macros()
    c2 = dict(c)
    c2["params"] = dict(c["params"], gy=-c["params"]["gy"])
    c2["phi"] = c["phi"][::-1, :]
    b = _run(c2, 60).macros()
    np.testing.assert_allclose(b["phi"], a["phi"][::-1, :], rtol=0, atol=1e-12)
    np.testing.assert_allclose(b["u"], a["u"][::-1, :], rtol=0, atol=1e-13)
    np.testing.assert_allclose(b["v"], -a["v"][::-1, :], rtol=0, atol=1e-13)


def test_transpose_equivariance():
    c = _upwind(W.random_coupled(16, 16, seed=31, rho_ratio=20.0))
    a = _run(c, 50).macros()
    c2 = dict(c)
    c2["phi"] = c["phi"].T.copy()
    c2["u"], c2["v"] = c["v"].T.copy(), c["u"].T.copy()
    b = _run(c2, 50).macros()
    np.testing.assert_allclose(b["phi"], a["phi"].T, rtol=0, atol=1e-12)
    np.testing.assert_allclose(b["u"], a["v"].T, rtol=0, atol=1e-13)
    np.testing.assert_allclose(b["v"], a["u"].T, rtol=0, atol=1e-13)


def test_central_is_the_default():
    c = W.random_coupled(12, 10, seed=5, rho_ratio=10.0)
    a = _run(c, 20).get_state()
    c2 = dict(c)
    c2["params"] = dict(c["params"], recon="central")
    b = _run(c2, 20).get_state()
    assert np.array_equal(a["f"], b["f"]) and np.array_equal(a["g"], b["g"])


@pytest.mark.parametrize("L0,Pe", [(32, 512), (48, 1024)])
def test_upwind_transports_a_drop_more_accurately_at_high_peclet(L0, Pe):
    """Sec. III: the central reconstruction's dissipation makes the error of
    a translated drop grow with Pe, which an upwind, limited reconstruction
    reduces. Diagonal translation over one period: the upwind error is at
    most 0.6 of the central one."""
    M = 0.02
    err = {}
    for mode in ("central", "upwind"):
        c = W.diag_translation(L0=L0, W=4.0, U0=Pe * M / L0, M=M, phi_H=1.0, phi_L=0.0)
        s = oracle.Sim(L0, L0, dict(c["params"], recon=mode), "ac")
        s.init(c["phi"])
        s.step(c["steps"])
        phi = s.macros()["phi"]
        err[mode] = np.sqrt(((phi - c["phi"]) ** 2).sum() / (c["phi"] ** 2).sum())
    assert err["upwind"] < 0.6 * err["central"], err
