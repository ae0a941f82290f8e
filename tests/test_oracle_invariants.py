"""Invariants of the oracle's full time step.

These hold for the exact method whatever the readings of the paper's silent
points, so they catch indexing, sign and transposition mistakes: conservation
of the order parameter (Sec. II.A: phi, not rho, is conserved), preservation
of uniform states, equivariance under integer shifts, reflections and the
x<->y transpose, conservation of momentum without forces, and bitwise
checkpoint/resume.
"""
import numpy as np
import pytest

import oracle
import workloads as W


def _run(case, steps):
    s = oracle.Sim(case["nx"], case["ny"], case["params"], case["model"])
    s.init(case["phi"], case["u"], case["v"], case["p"])
    s.step(steps)
    return s


def _total_phi(s):
    return s.macros()["phi"].sum()


@pytest.mark.parametrize("which", ["coupled_periodic", "coupled_walls", "ac_deform", "spinodal"])
def test_phi_is_conserved(which):
    if which == "coupled_periodic":
        c = W.random_coupled(24, 20, seed=3, rho_ratio=100.0)
    elif which == "coupled_walls":
        c = W.random_coupled(16, 24, seed=4, rho_ratio=10.0, walls_y=True)
    elif which == "ac_deform":
        c = W.smoothed_deformation(L0=32, Pe=64, M=0.02)
    else:
        c = W.spinodal(L=24, seed=5)
    s = oracle.Sim(c["nx"], c["ny"], c["params"], c["model"])
    s.init(c["phi"], c["u"], c["v"], c["p"])
    t0 = _total_phi(s)
    scale = np.abs(c["phi"]).sum()
    s.step(300)
    assert abs(_total_phi(s) - t0) / scale < 1e-12


@pytest.mark.parametrize("model", ["coupled", "ac"])
def test_uniform_state_is_preserved(model):
    nx, ny = 7, 9
    phi = np.full((ny, nx), 0.37)
    if model == "coupled":
        params = dict(phi_H=1.0, phi_L=0.0, rho_H=50.0, rho_L=1.0, sigma=1e-3,
                      visc="reciprocal", mu_H=0.2, mu_L=0.02, M=0.05)
        u, v, p = np.full_like(phi, 0.013), np.full_like(phi, -0.007), np.full_like(phi, 2e-3)
    else:
        params = dict(phi_H=1.0, phi_L=0.0, M=0.05, vel="uniform", U0=0.02)
        u = v = p = None
    s = oracle.Sim(nx, ny, params, model)
    s.init(phi, u, v, p)
    st0 = s.get_state()
    s.step(50)
    st1 = s.get_state()
    np.testing.assert_allclose(st1["f"], st0["f"], rtol=0, atol=1e-14)
    if model == "coupled":
        # the pressure round trip (Eq. 33 then Eq. 17) adds rounding each step
        np.testing.assert_allclose(st1["g"], st0["g"], rtol=0, atol=2e-13)


@pytest.mark.parametrize("shift", [(3, 0), (0, 5), (7, 2)])
def test_integer_shift_equivariance_is_bitwise(shift):
    sx, sy = shift
    c = W.random_coupled(20, 16, seed=11, rho_ratio=30.0)
    a = _run(c, 40).macros()
    c2 = dict(c)
    for k in ("phi", "u", "v"):
        c2[k] = np.roll(c[k], (sy, sx), axis=(0, 1))
    b = _run(c2, 40).macros()
    for k in ("phi", "u", "v", "p"):
        assert np.array_equal(np.roll(a[k], (sy, sx), axis=(0, 1)), b[k]), k


def test_x_shift_equivariance_with_walls_is_bitwise():
    c = W.random_coupled(12, 16, seed=12, rho_ratio=10.0, walls_y=True)
    a = _run(c, 40).macros()
    c2 = dict(c)
    for k in ("phi", "u", "v"):
        if c[k] is not None:
            c2[k] = np.roll(c[k], 5, axis=1)
    b = _run(c2, 40).macros()
    for k in ("phi", "u", "v", "p"):
        assert np.array_equal(np.roll(a[k], 5, axis=1), b[k]), k


def test_mirror_x_equivariance():
    """Reflecting x -> -x (u -> -u) commutes with the step."""
    c = W.random_coupled(18, 14, seed=21, rho_ratio=50.0)
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
    """Reflecting y -> -y with walls (v -> -v, g -> -g) commutes with the step."""
    c = W.random_coupled(12, 16, seed=22, rho_ratio=10.0, walls_y=True)
    c["u"] = W.smooth_field(12, 16, 5, amp=1e-3) * 0.0
    a = _run(c, 60).macros()
    c2 = dict(c)
    c2["params"] = dict(c["params"], gy=-c["params"]["gy"])
    c2["phi"] = c["phi"][::-1, :]
    c2["u"] = None
    b = _run(c2, 60).macros()
    np.testing.assert_allclose(b["phi"], a["phi"][::-1, :], rtol=0, atol=1e-12)
    np.testing.assert_allclose(b["u"], a["u"][::-1, :], rtol=0, atol=1e-13)
    np.testing.assert_allclose(b["v"], -a["v"][::-1, :], rtol=0, atol=1e-13)


@pytest.mark.parametrize("model", ["coupled", "ac"])
def test_transpose_equivariance(model):
    """Swapping x and y (u <-> v) commutes with the step on a square grid."""
    if model == "coupled":
        c = W.random_coupled(16, 16, seed=31, rho_ratio=20.0)
    else:
        c = W.smoothed_deformation(L0=16, Pe=32, M=0.02)
        c["params"] = dict(c["params"], vel="uniform", U0=0.01)
    a = _run(c, 50).macros()
    c2 = dict(c)
    c2["phi"] = c["phi"].T.copy()
    if model == "coupled":
        c2["u"], c2["v"] = c["v"].T.copy(), c["u"].T.copy()
    b = _run(c2, 50).macros()
    np.testing.assert_allclose(b["phi"], a["phi"].T, rtol=0, atol=1e-12)
    np.testing.assert_allclose(b["u"], a["v"].T, rtol=0, atol=1e-13)
    np.testing.assert_allclose(b["v"], a["u"].T, rtol=0, atol=1e-13)


def test_centred_bubble_keeps_d4_symmetry():
    """The centred bubble is symmetric under the dihedral group of the square;
    the step must keep it so up to rounding, which the 1000:1 density ratio
    amplifies (a wrong index or sign would break it at O(1e-4))."""
    c = W.bubble(L=32, R=8, steps=0)
    m = _run(c, 100).macros()
    phi = m["phi"]
    np.testing.assert_allclose(phi, phi.T, rtol=0, atol=1e-10)
    np.testing.assert_allclose(phi, phi[::-1, :], rtol=0, atol=1e-10)
    np.testing.assert_allclose(phi, phi[:, ::-1], rtol=0, atol=1e-10)
    umax = np.abs(m["u"]).max()
    assert umax > 0
    np.testing.assert_allclose(m["u"], -m["u"][:, ::-1], rtol=0, atol=1e-6 * umax)
    np.testing.assert_allclose(m["u"], m["v"].T, rtol=0, atol=1e-6 * umax)


def test_momentum_is_conserved_without_forces():
    """Single phase, no tension, no gravity: sum rho u is conserved."""
    nx, ny = 16, 12
    u = W.smooth_field(nx, ny, 40, amp=0.02)
    v = W.smooth_field(nx, ny, 41, amp=0.02)
    params = dict(phi_H=1.0, phi_L=0.0, rho_H=1.0, rho_L=1.0, sigma=0.0,
                  nu=0.05, visc="uniform_nu", M=0.1)
    s = oracle.Sim(nx, ny, params)
    s.init(np.ones((ny, nx)), u, v)
    m0 = s.macros()
    s.step(200)
    m1 = s.macros()
    assert abs(m1["u"].sum() - m0["u"].sum()) < 1e-13
    assert abs(m1["v"].sum() - m0["v"].sum()) < 1e-13
    assert np.abs(m1["u"]).max() < 0.8 * np.abs(m0["u"]).max()  # viscous decay


@pytest.mark.parametrize("walls", [False, True])
def test_checkpoint_resume_is_bitwise(walls):
    c = W.random_coupled(12, 16, seed=51, rho_ratio=10.0, walls_y=walls)
    a = _run(c, 30)
    st = a.get_state()
    a.step(30)
    b = oracle.Sim(c["nx"], c["ny"], c["params"], c["model"])
    b.set_state(st)
    b.step(30)
    sa, sb = a.get_state(), b.get_state()
    for k in ("f", "g", "hist"):
        assert np.array_equal(sa[k], sb[k])
    assert sa["step"] == sb["step"] == 60
