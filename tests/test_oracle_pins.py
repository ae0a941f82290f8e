"""Pins of the oracle's point functions against what the paper fixes.

Each test checks a closed-form property stated in the paper (moment identities
of the Chapman-Enskog appendix, the definitions of the auxiliary distributions,
exactness of the difference stencils on polynomials, the equilibrium interface
profile), not the oracle's own formulas retyped.
"""
import numpy as np
import pytest

import oracle

EX = np.array([0, 1, 1, 0, -1, -1, -1, 0, 1], dtype=float)
EY = np.array([0, 0, 1, 1, 1, 0, -1, -1, -1], dtype=float)
RT = 1.0 / 3.0
rng = np.random.default_rng(12345)


def _rand_states(n=16):
    """Random point states: 16 samples, the '4x4' brute-force grid."""
    for _ in range(n):
        yield dict(phi=rng.uniform(-1, 1.5), ux=rng.uniform(-0.1, 0.1),
                   uy=rng.uniform(-0.1, 0.1), p=rng.uniform(-0.1, 0.1),
                   rho=rng.uniform(0.5, 1000), theta=rng.uniform(-1, 1),
                   nang=rng.uniform(0, 2 * np.pi), Dx=rng.uniform(-1e-3, 1e-3),
                   Dy=rng.uniform(-1e-3, 1e-3), drx=rng.uniform(-300, 300),
                   dry=rng.uniform(-300, 300), Fx=rng.uniform(-1e-3, 1e-3),
                   Fy=rng.uniform(-1e-3, 1e-3))


def test_velocity_set_is_the_d2q9_tensor_product():
    """Eq. 14: the nine velocities are the tensor product of {-1,0,1} (times
    sqrt(3RT) = 1) and the weights are products of the 1-D Gauss-Hermite
    weights (2/3, 1/6, 1/6): check through the equilibrium at u = 0."""
    w1 = {0: 2 / 3, 1: 1 / 6, -1: 1 / 6}
    w = oracle.feq(1.0, 0.0, 0.0)
    for q in range(9):
        assert w[q] == pytest.approx(w1[int(EX[q])] * w1[int(EY[q])], rel=1e-15)
    assert sorted(zip(EX, EY)) == sorted((a, b) for a in (-1, 0, 1) for b in (-1, 0, 1))


def test_feq_moments():
    """Appendix: sum f^eq = phi, sum xi f^eq = phi u, sum xi xi f^eq = phi RT I."""
    for s in _rand_states():
        f = oracle.feq(s["phi"], s["ux"], s["uy"])
        assert f.sum() == pytest.approx(s["phi"], abs=1e-14)
        assert (EX * f).sum() == pytest.approx(s["phi"] * s["ux"], abs=1e-14)
        assert (EY * f).sum() == pytest.approx(s["phi"] * s["uy"], abs=1e-14)
        assert (EX * EX * f).sum() == pytest.approx(s["phi"] * RT, abs=1e-14)
        assert (EY * EY * f).sum() == pytest.approx(s["phi"] * RT, abs=1e-14)
        assert abs((EX * EY * f).sum()) < 1e-14


def test_sf_moments():
    """Appendix: sum S^f = 0 and sum xi S^f = theta RT n + d_t(phi u)."""
    for s in _rand_states():
        nx, ny = np.cos(s["nang"]), np.sin(s["nang"])
        S = oracle.sf(s["theta"], nx, ny, s["Dx"], s["Dy"])
        assert abs(S.sum()) < 1e-15
        assert (EX * S).sum() == pytest.approx(s["theta"] * RT * nx + s["Dx"], abs=1e-14)
        assert (EY * S).sum() == pytest.approx(s["theta"] * RT * ny + s["Dy"], abs=1e-14)


def test_geq_moments():
    """Appendix: sum g^eq = 0, sum xi g^eq = rho u, sum xi xi g^eq = p I + rho u u,
    third moment RT rho (delta u) symmetrised."""
    for s in _rand_states():
        p, rho, ux, uy = s["p"], s["rho"], s["ux"], s["uy"]
        g = oracle.geq(p, rho, ux, uy)
        tol = 1e-12 * max(1.0, rho)
        assert abs(g.sum()) < tol
        assert (EX * g).sum() == pytest.approx(rho * ux, abs=tol)
        assert (EY * g).sum() == pytest.approx(rho * uy, abs=tol)
        assert (EX * EX * g).sum() == pytest.approx(p + rho * ux * ux, abs=tol)
        assert (EY * EY * g).sum() == pytest.approx(p + rho * uy * uy, abs=tol)
        assert (EX * EY * g).sum() == pytest.approx(rho * ux * uy, abs=tol)
        # third moments: xxx -> 3 RT rho ux, xxy -> RT rho uy
        assert (EX ** 3 * g).sum() == pytest.approx(3 * RT * rho * ux, abs=tol)
        assert (EX * EX * EY * g).sum() == pytest.approx(RT * rho * uy, abs=tol)


def test_sg_moments():
    """Appendix: sum S^g = u . grad rho and sum xi S^g = F = F_s + G."""
    for s in _rand_states():
        ux, uy = s["ux"], s["uy"]
        S = oracle.sg(ux, uy, s["drx"], s["dry"], s["Fx"], s["Fy"])
        tol = 1e-12 * max(1.0, abs(s["drx"]) + abs(s["dry"]))
        assert S.sum() == pytest.approx(ux * s["drx"] + uy * s["dry"], abs=tol)
        assert (EX * S).sum() == pytest.approx(s["Fx"], abs=tol)
        assert (EY * S).sum() == pytest.approx(s["Fy"], abs=tol)


def test_sg_second_moment_to_order_u3():
    """Appendix: sum xi xi S^g = (uF + Fu) + RT (u grad rho + grad rho u +
    (u . grad rho) I) up to O(u^3): the residual must shrink as u^3."""
    res = []
    for scale in (1e-2, 5e-3):
        ux, uy = 0.7 * scale, -0.4 * scale
        drx, dry, Fx, Fy = 30.0, -12.0, 2e-3, 5e-4
        S = oracle.sg(ux, uy, drx, dry, Fx, Fy)
        udr = ux * drx + uy * dry
        exp_xx = 2 * ux * Fx + RT * (2 * ux * drx + udr)
        exp_xy = ux * Fy + uy * Fx + RT * (ux * dry + uy * drx)
        r = max(abs((EX * EX * S).sum() - exp_xx), abs((EX * EY * S).sum() - exp_xy))
        res.append(r)
    assert res[0] < 1e-4
    ratio = res[0] / res[1]
    assert 6.0 < ratio < 10.0  # cubic scaling: 2^3 = 8


def _rand9():
    return rng.uniform(-0.5, 0.5, 9)


@pytest.mark.parametrize("tau,dt", [(0.3, 0.5), (0.003, 0.5), (0.03, 0.25), (5.0, 1.0)])
def test_bar_plus_from_tilde_matches_definitions(tau, dt):
    """Eq. 29-30 must agree with the definitions of Eq. 23 and 26: start from
    an original distribution psi, form tilde psi by Eq. 23a, and compare the
    oracle's bar-plus / tilde-plus with Eq. 26b / 23b evaluated on psi."""
    h = 0.5 * dt
    psi, eq, S = _rand9(), _rand9(), _rand9()
    tilde = (2 * tau + dt) / (2 * tau) * psi - dt / (2 * tau) * eq - dt / 2 * S
    bp, tp = oracle.bar_plus(tau, dt, tilde, eq, S)
    bp_def = (2 * tau - h) / (2 * tau) * psi + h / (2 * tau) * eq + h / 2 * S
    tp_def = (2 * tau - dt) / (2 * tau) * psi + dt / (2 * tau) * eq + dt / 2 * S
    np.testing.assert_allclose(bp, bp_def, rtol=0, atol=1e-13)
    np.testing.assert_allclose(tp, tp_def, rtol=0, atol=1e-13)


@pytest.mark.parametrize("tau,h", [(0.3, 0.25), (0.003, 0.25), (2.0, 0.125)])
def test_face_df_inverts_bar_definition(tau, h):
    """Eq. 28 inverts Eq. 26a: psi -> bar psi -> psi."""
    psi, eq, S = _rand9(), _rand9(), _rand9()
    bar = (2 * tau + h) / (2 * tau) * psi - h / (2 * tau) * eq - h / 2 * S
    np.testing.assert_allclose(oracle.face_df(tau, h, bar, eq, S), psi, rtol=0, atol=1e-13)


def test_stencils_exact_on_quadratics_and_isotropic():
    """The gradient stencil is exact for quadratics and the nine-point
    Laplacian for quadratics (interior cells, away from the periodic seam)."""
    ny, nx = 12, 14
    X, Y = np.meshgrid(np.arange(nx) + 0.5, np.arange(ny) + 0.5)
    a, b, c, d, e, f = 0.3, -0.7, 0.11, -0.05, 0.08, 1.2
    phi = a * X + b * Y + c * X * X + d * X * Y + e * Y * Y + f
    gx, gy, lap = oracle.stencils(phi)
    sl = (slice(1, -1), slice(1, -1))
    np.testing.assert_allclose(gx[sl], (a + 2 * c * X + d * Y)[sl], atol=1e-12)
    np.testing.assert_allclose(gy[sl], (b + d * X + 2 * e * Y)[sl], atol=1e-12)
    np.testing.assert_allclose(lap[sl], 2 * (c + e), atol=1e-12)
    # isotropy of the Laplacian at fourth order: a plane wave along x and one
    # along the diagonal with the same |k| give the same discrete eigenvalue
    # to O(k^4) with an isotropic k^4 term; compare both to -k^2 (1 - k^2/12).
    n = 256
    X, Y = np.meshgrid(np.arange(n) + 0.5, np.arange(n) + 0.5)
    kk = 2 * np.pi * 4 / n
    p1 = np.cos(kk * X)
    p2 = np.cos(2 * np.pi * 4 / n * X + 2 * np.pi * 4 / n * Y)  # |k| = sqrt(2) kk
    _, _, l1 = oracle.stencils(p1)
    _, _, l2 = oracle.stencils(p2)
    e1 = (l1 / p1)[np.abs(p1) > 0.5].mean()
    e2 = (l2 / p2)[np.abs(p2) > 0.5].mean()
    k1, k2 = kk ** 2, 2 * kk ** 2
    assert e1 == pytest.approx(-k1 * (1 - k1 / 12), rel=1e-4)
    assert e2 == pytest.approx(-k2 * (1 - k2 / 12), rel=1e-4)


def test_stencils_wall_mirror():
    """At no-slip walls phi ghosts mirror the first interior row (neutral
    wetting), so a field even about the wall has zero normal gradient there."""
    ny, nx = 8, 6
    Y = np.arange(ny)[:, None] + 0.5 + np.zeros((1, nx))
    phi = np.cos(np.pi * Y / ny)  # even about y = 0 and y = ny
    gx, gy, lap = oracle.stencils(phi, walls_y=True)
    # row 0 sees phi(-1) = phi(0): central difference (phi1 - phi0)/... finite,
    # but a y-independent field must give exactly zero gradient and Laplacian
    gx0, gy0, lap0 = oracle.stencils(np.ones((ny, nx)) * 0.3, walls_y=True)
    assert np.abs(gy0).max() < 1e-15 and np.abs(lap0).max() < 1e-15 and np.abs(gx0).max() < 1e-15
    # mirrored ghost: gy at row 0 equals (phi1 - phi0)/2 for an x-constant field
    assert gy[0, 0] == pytest.approx((phi[1, 0] - phi[0, 0]) / 2.0, rel=1e-13)


@pytest.mark.parametrize("phi_H,phi_L", [(1.0, 0.0), (1.0, -1.0)])
def test_chemical_potential_vanishes_on_tanh_profile(phi_H, phi_L):
    """Eq. 4 with kappa, beta chosen for width W and tension sigma (Eq. 3,
    generalised to phi_H - phi_L != 1): mu_phi ~ 0 on the equilibrium profile
    of Eq. 7. With kappa, beta off by the factors that a wrong generalisation
    gives (Delta^2, Delta^4), mu_phi would be O(beta) instead."""
    W, sigma, ny, nx = 8.0, 1e-2, 64, 4
    Y = np.arange(ny)[:, None] + 0.5 + np.zeros((1, nx))
    z = Y - ny / 2
    phi = 0.5 * (phi_H + phi_L) + 0.5 * (phi_H - phi_L) * np.tanh(2 * z / W)
    params = dict(phi_H=phi_H, phi_L=phi_L, sigma=sigma, W=W, M=0.1)
    s = oracle.Sim(nx, ny, params, "ac")
    s.init(phi)
    mu = s.cell_fields()["mu"][8:-8]
    d = s.derived()
    scale = d["beta"] * (phi_H - phi_L) ** 3
    assert np.abs(mu).max() < 2e-2 * scale
    # and the interface tension recovered by quadrature of kappa |phi'|^2
    z1 = np.linspace(-40, 40, 40001)
    ph = 0.5 * (phi_H + phi_L) + 0.5 * (phi_H - phi_L) * np.tanh(2 * z1 / W)
    dph = np.gradient(ph, z1)
    assert d["kappa"] * np.trapezoid(dph ** 2, z1) == pytest.approx(sigma, rel=1e-6)


def test_theta_equals_gradient_on_profile():
    """theta(phi) (Eq. 6) equals |grad phi| on the tanh profile (Eq. 7), so a
    flat interface at rest is an equilibrium of the conservative Allen-Cahn
    model: the interface-only step leaves it almost unchanged, and it stays
    centred and keeps its width."""
    W, ny, nx = 4.0, 64, 4
    Y = np.arange(ny)[:, None] + 0.5 + np.zeros((1, nx))
    # a band of phi_H between two flat interfaces at ny/4 and 3ny/4
    phi = 0.5 + 0.5 * np.tanh(2 * (ny / 4 - np.abs(Y - ny / 2)) / W)
    params = dict(phi_H=1.0, phi_L=0.0, W=W, M=0.1, vel="uniform", U0=0.0)
    s = oracle.Sim(nx, ny, params, "ac")
    s.init(phi)
    s.step(1000)
    m1 = s.macros()["phi"]
    s.step(1000)
    m2 = s.macros()["phi"]
    # the discrete equilibrium sits within O(1/W^2) of the continuous profile
    # and does not move any more
    assert np.abs(m2 - phi).max() < 1e-2
    assert np.abs(m2 - m1).max() < 1e-5
    # a theta that is twice or half the profile gradient (wrong W in Eq. 6)
    # drives the interface to a visibly different width
    for Wp in (W / 2, 2 * W):
        s2 = oracle.Sim(nx, ny, dict(params, W=Wp), "ac")
        s2.init(phi)
        s2.step(1000)
        assert np.abs(s2.macros()["phi"] - phi).max() > 0.1
