"""Pins of the oracle on stretched (non-uniform tensor-product) meshes.

DUGKS is a finite-volume scheme (Sec. II.B, Eq. 21: the microflux is
integrated over the cell surface and divided by the cell volume), which the
introduction names as its advantage over the uniform lattice of LBM. The
paper's runs are all on uniform grids, so the stretched-mesh forms of the
stencils and of the face reconstruction are a reading (R27): derivatives over
the centre distances, linear interpolation to the face, the R8 / R9 stencils
as weighted sums of one-dimensional derivatives centred on the cell. These
tests fix that reading from outside the oracle:

* the stencils are exact on quadratics and the reconstruction on linear data,
  for random widths;
* on unit widths the general code gives the uniform path's results; on widths
  of 2 with the physical parameters scaled accordingly, the same solution;
* the step conserves the area integral of phi and keeps uniform states;
* mirror symmetry with a mirrored mesh;
* closed forms: a planar interface translated by a uniform velocity returns
  to its initial profile with a second-order error under refinement of a
  smoothly stretched mesh; a shear wave decays at nu k^2; the layered
  Poiseuille flow keeps its analytic profile on a mesh clustered at the walls
  and the interface.
"""
import numpy as np
import pytest

import oracle
import workloads as W

EX = [0, 1, 1, 0, -1, -1, -1, 0, 1]
EY = [0, 0, 1, 1, 1, 0, -1, -1, -1]


def _sim(c, dx=None, dy=None, params=None):
    s = oracle.Sim(c["nx"], c["ny"], params or c["params"], c["model"])
    if dx is not None or dy is not None:
        s.set_mesh(dx, dy)
    s.init(c["phi"], c["u"], c["v"], c["p"])
    return s


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def test_stencils_are_exact_on_quadratics():
    nx, ny = 14, 12
    dx, dy = W.random_widths(nx, 1), W.random_widths(ny, 2)
    X, Y = np.meshgrid(W.mesh_centres(dx), W.mesh_centres(dy))
    c0, b, c, d, e, f = 0.3, 0.7, -0.4, 0.11, -0.23, 0.07
    phi = c0 + b * X + c * Y + d * X * X + e * X * Y + f * Y * Y
    gx, gy, lap = oracle.stencils(phi, dx=dx, dy=dy)
    sl = (slice(1, ny - 1), slice(1, nx - 1))  # stencils that do not cross the seams
    np.testing.assert_allclose(gx[sl], (b + 2 * d * X + e * Y)[sl], rtol=0, atol=1e-11)
    np.testing.assert_allclose(gy[sl], (c + e * X + 2 * f * Y)[sl], rtol=0, atol=1e-11)
    np.testing.assert_allclose(lap[sl], 2 * d + 2 * f, rtol=0, atol=1e-11)


@pytest.mark.parametrize("walls", [False, True])
def test_stencils_on_unit_and_doubled_widths(walls):
    """Unit widths: the uniform stencils R8, R9. Widths 2: half the gradient,
    a quarter of the Laplacian."""
    nx, ny = 9, 8
    phi = np.random.default_rng(3).standard_normal((ny, nx))
    g0 = oracle.stencils(phi, walls_y=walls)
    g1 = oracle.stencils(phi, walls_y=walls, dx=np.ones(nx), dy=np.ones(ny))
    g2 = oracle.stencils(phi, walls_y=walls, dx=np.full(nx, 2.0), dy=np.full(ny, 2.0))
    for a, b in zip(g0, g1):
        np.testing.assert_allclose(b, a, rtol=0, atol=1e-14)
    for a, b, k in zip(g0, g2, (0.5, 0.5, 0.25)):
        np.testing.assert_allclose(b, k * a, rtol=0, atol=1e-14)


@pytest.mark.parametrize("mode", ["central", "upwind"])
@pytest.mark.parametrize("walls", [False, True])
def test_reconstruction_is_exact_on_linear_data(mode, walls):
    """The bar value at a face is the linear field at x_face - h xi."""
    nx, ny, h = 12, 10, 0.2
    dx, dy = W.random_widths(nx, 4), W.random_widths(ny, 5)
    xc, yc = W.mesh_centres(dx), W.mesh_centres(dy)
    X, Y = np.meshgrid(xc, yc)
    c0, cx, cy = 0.3, 0.07, -0.11
    a = c0 + cx * X + cy * Y
    for q in range(9):
        xf, yf = oracle.recon(a, q, h, mode, walls_y=walls, dx=dx, dy=dy)
        for j in (range(ny) if walls else range(1, ny - 1)):
            for i in range(1, nx - 3):
                x, y = xc[i] + 0.5 * dx[i] - h * EX[q], yc[j] - h * EY[q]
                assert xf[j, i] == pytest.approx(c0 + cx * x + cy * y, abs=1e-13), (q, i, j)
        for j in range(1, ny - 3):
            for i in range(1, nx - 1):
                x, y = xc[i] - h * EX[q], yc[j] + 0.5 * dy[j] - h * EY[q]
                assert yf[j, i] == pytest.approx(c0 + cx * x + cy * y, abs=1e-13), (q, i, j)


def test_upwind_values_stay_within_their_stencil():
    """Random data on a rough mesh: a population along an axis, or along the
    face, stays between the smallest and largest value its stencil reads. A
    diagonal one, traced to (w_n/2 - h, -h) from the upwind centre, may leave
    that range by at most (2h/w_t - 2h/w_n) times its width when the cell is
    narrower across the face (w_t) than along it (w_n): the capped slopes
    bound the two increments by (1 - 2h/w_n) and 2h/w_t of the range."""
    nx, ny, h = 11, 9, 0.2  # h below half the smallest width
    dx, dy = W.random_widths(nx, 6), W.random_widths(ny, 7)
    rng = np.random.default_rng(8)
    for _ in range(3):
        a = rng.standard_normal((ny, nx))
        for q in range(9):
            xf, yf = oracle.recon(a, q, h, "upwind", dx=dx, dy=dy)
            for j in range(ny):
                for i in range(nx):
                    for f, cells in ((xf, [(i, j), ((i + 1) % nx, j)]),
                                     (yf, [(i, j), (i, (j + 1) % ny)])):
                        en, et = (EX[q], EY[q]) if f is xf else (EY[q], EX[q])
                        up = cells[:1] if en > 0 else cells[1:] if en < 0 else cells
                        vals = [a[(jj + dj) % ny, (ii + di) % nx] for ii, jj in up
                                for di, dj in ((0, 0), (1, 0), (-1, 0), (0, 1), (0, -1))]
                        lo, hi = min(vals), max(vals)
                        slack = 0.0
                        if en != 0 and et != 0:
                            ii, jj = up[0]
                            wn, wt = (dx[ii], dy[jj]) if f is xf else (dy[jj], dx[ii])
                            slack = max(0.0, 2 * h / wt - 2 * h / wn) * (hi - lo)
                        assert lo - slack - 1e-13 <= f[j, i] <= hi + slack + 1e-13, (q, i, j)


CASES = {
    "coupled_periodic": lambda: W.random_coupled(20, 16, seed=3, rho_ratio=100.0),
    "coupled_walls": lambda: W.random_coupled(14, 18, seed=4, rho_ratio=10.0, walls_y=True),
    "ac_rotation": lambda: dict(W.smoothed_deformation(L0=24, Pe=64, M=0.02),
                                params=dict(W.smoothed_deformation(L0=24, Pe=64, M=0.02)["params"],
                                            vel="rotation", U0=0.02)),
    "upwind_periodic": lambda: dict(W.random_coupled(20, 16, seed=5, rho_ratio=100.0),
                                    params=dict(W.random_coupled(20, 16, seed=5, rho_ratio=100.0)["params"],
                                                recon="upwind")),
}


@pytest.mark.parametrize("which", sorted(CASES))
def test_unit_widths_reproduce_the_uniform_path(which):
    c = CASES[which]()
    a = _sim(c)
    b = _sim(c, np.ones(c["nx"]), np.ones(c["ny"]))
    a.step(100)
    b.step(100)
    ma, mb = a.macros(), b.macros()
    for k in ("phi", "u", "v", "p"):
        assert _rel(mb[k], ma[k]) < 1e-13 or np.abs(mb[k] - ma[k]).max() < 1e-16, k


@pytest.mark.parametrize("walls", [False, True])
def test_doubling_the_mesh_with_scaled_physics_gives_the_same_solution(walls):
    """Lengths x2 and times x2 (widths 2, so dt x2), with M, W, sigma, mu x2
    and body forces /2: the dimensionless problem is unchanged, so phi, u and
    p agree to rounding (the regularisation of the unit normal is in gradient
    units and scales too)."""
    c = W.random_coupled(16, 14, seed=9, rho_ratio=20.0, walls_y=walls)
    p = c["params"]
    p2 = dict(p, M=2 * p["M"], W=2 * p["W"], sigma=2 * p["sigma"], mu_H=2 * p["mu_H"],
              mu_L=2 * p["mu_L"], gx=p.get("gx", 0.0) / 2, gy=p.get("gy", 0.0) / 2,
              Gx=p.get("Gx", 0.0) / 2, Gy=p.get("Gy", 0.0) / 2)
    a = _sim(c)
    b = _sim(c, np.full(c["nx"], 2.0), np.full(c["ny"], 2.0), params=p2)
    a.step(60)
    b.step(60)
    assert b.time == pytest.approx(2 * a.time)
    ma, mb = a.macros(), b.macros()
    for k in ("phi", "u", "v", "p"):
        assert _rel(mb[k], ma[k]) < 1e-12, (k, _rel(mb[k], ma[k]))


@pytest.mark.parametrize("which", sorted(CASES))
def test_area_integral_of_phi_is_conserved(which):
    c = CASES[which]()
    dx, dy = W.random_widths(c["nx"], 11), W.random_widths(c["ny"], 12)
    area = np.outer(dy, dx)
    s = _sim(c, dx, dy)
    t0 = (s.macros()["phi"] * area).sum()
    s.step(200)
    t1 = (s.macros()["phi"] * area).sum()
    assert abs(t1 - t0) < 1e-12 * (np.abs(c["phi"]) * area).sum()


@pytest.mark.parametrize("phi0", [1.0, 0.0])
@pytest.mark.parametrize("walls", [False, True])
def test_uniform_state_is_preserved_on_a_rough_mesh(phi0, walls):
    """A uniform single-phase state in uniform motion stays put. (A uniform
    state between the phases is not used: there the conservative Allen-Cahn
    flux of the regularised normal (R7) is anti-diffusive for gradients below
    its regularisation, so the rounding of the interpolation weights of a
    stretched mesh seeds a phase separation, as a physical perturbation
    would.)"""
    nx, ny = 9, 8
    phi = np.full((ny, nx), phi0)
    params = dict(phi_H=1.0, phi_L=0.0, rho_H=50.0, rho_L=1.0, sigma=1e-3, visc="reciprocal",
                  mu_H=0.2, mu_L=0.02, M=0.05, walls_y=walls)
    s = oracle.Sim(nx, ny, params)
    s.set_mesh(W.random_widths(nx, 13), W.random_widths(ny, 14))
    u0, v0 = (0.0, 0.0) if walls else (0.013, -0.007)
    s.init(phi, np.full_like(phi, u0), np.full_like(phi, v0), np.full_like(phi, 2e-3))
    m0 = s.macros()
    s.step(200)
    m1 = s.macros()
    for k in ("phi", "u", "v"):
        np.testing.assert_allclose(m1[k], m0[k], rtol=0, atol=1e-13)
    np.testing.assert_allclose(m1["p"], m0["p"], rtol=0, atol=1e-12)


def test_mirror_x_with_the_mirrored_mesh():
    c = W.random_coupled(18, 14, seed=21, rho_ratio=50.0)
    dx, dy = W.random_widths(18, 15), W.random_widths(14, 16)
    a = _sim(c, dx, dy)
    a.step(60)
    ma = a.macros()
    c2 = dict(c, phi=c["phi"][:, ::-1], u=-c["u"][:, ::-1], v=c["v"][:, ::-1])
    b = _sim(c2, dx[::-1].copy(), dy)
    b.step(60)
    mb = b.macros()
    np.testing.assert_allclose(mb["phi"], ma["phi"][:, ::-1], rtol=0, atol=1e-12)
    np.testing.assert_allclose(mb["u"], -ma["u"][:, ::-1], rtol=0, atol=1e-13)
    np.testing.assert_allclose(mb["v"], ma["v"][:, ::-1], rtol=0, atol=1e-13)


def _translation_error(n, L=64.0, Wd=8.0, M=0.02, amp=0.35, recon="central"):
    """A slab of phi = 1 between two planar interfaces (the equilibrium tanh
    profile of the conservative Allen-Cahn equation) translated once around a
    periodic stretched x-axis: the exact solution returns to the start."""
    dx = W.stretched_widths(n, amp=amp, length=L)
    ny = 4
    xc = W.mesh_centres(dx)
    a, b = 0.25 * L, 0.65 * L
    prof = 0.5 * (np.tanh(2 * (xc - a) / Wd) - np.tanh(2 * (xc - b) / Wd))
    phi = np.repeat(prof[None, :], ny, axis=0)
    dt = 0.5 * min(dx.min(), 1.0)
    steps = int(round(L / (0.04 * dt)))
    U = L / (steps * dt)
    params = dict(phi_H=1.0, phi_L=0.0, W=Wd, M=M, cfl=0.5, vel="uniform", U0=U,
                  L0=L, T_period=L / U, recon=recon)
    s = oracle.Sim(n, ny, params, "ac")
    s.set_mesh(dx, np.ones(ny))
    s.init(phi)
    s.step(steps)
    assert s.time == pytest.approx(L / U)
    out = s.macros()["phi"][0]
    return np.sqrt((((out - prof) ** 2) * dx).sum() / ((prof ** 2) * dx).sum())


@pytest.mark.parametrize("recon", ["central", "upwind"])
def test_translation_on_a_stretched_mesh_converges_at_second_order(recon):
    """Both reconstructions: the limited one stays second order on this
    smooth, monotone profile (van Leer's slope is exact on linear data and
    only flattens at extrema, where the profile is flat)."""
    e1, e2 = _translation_error(64, recon=recon), _translation_error(128, recon=recon)
    print(f"planar translation, stretched mesh, {recon}: N=64 {e1:.3e}  N=128 {e2:.3e}  "
          f"ratio {e1 / e2:.2f}")
    assert e2 < e1 / 3.0


@pytest.mark.parametrize("nu", [0.05, 0.2])
def test_shear_wave_decays_at_nu_k2_on_a_stretched_mesh(nu):
    nx, ny, U = 4, 32, 1e-3
    dy = W.stretched_widths(ny, amp=0.3)
    yc = W.mesh_centres(dy)
    k = 2 * np.pi / ny
    Y = np.repeat(yc[:, None], nx, axis=1)
    params = dict(phi_H=1.0, phi_L=0.0, rho_H=1.0, rho_L=1.0, nu=nu, visc="uniform_nu",
                  sigma=0.0, W=4.0, M=0.1, cfl=0.5)
    s = oracle.Sim(nx, ny, params)
    s.set_mesh(np.ones(nx), dy)
    s.init(np.ones((ny, nx)), U * np.sin(k * Y))
    dt = 0.5 * dy.min()
    s.step(int(2 / (nu * k * k) / dt))
    m = s.macros()
    w = np.repeat(dy[:, None], nx, axis=1)
    amp = (m["u"] * np.sin(k * Y) * w).sum() / ((np.sin(k * Y) ** 2) * w).sum()
    rate = -np.log(amp / U) / s.time
    assert rate == pytest.approx(nu * k * k, rel=0.02)


def _poiseuille_at(y, h, mu_H, mu_L, Gx):
    """Steady layered Poiseuille velocity (Sec. IV.B) at heights y in [-h, h]."""
    a = (mu_L - mu_H) / (mu_L + mu_H)
    up = Gx * h * h / (2 * mu_L) * (-(y / h) ** 2 - (y / h) * a + 2 * mu_L / (mu_L + mu_H))
    lo = Gx * h * h / (2 * mu_H) * (-(y / h) ** 2 - (y / h) * a + 2 * mu_H / (mu_L + mu_H))
    return np.where(y > 0, up, lo)


def _poiseuille_errors(dy, nx=4, steps=(4000, 4000, 4000)):
    ny, L = len(dy), float(dy.sum())
    yc = W.mesh_centres(dy)
    c = W.layered_poiseuille(nx=nx, ny=ny, mu_ratio=100.0, analytic_init=True)
    p = c["params"]
    h = 0.5 * L
    phi = np.repeat(W.tanh_profile(h - yc, p["W"], 1.0, 0.0)[:, None], nx, axis=1)
    ua = _poiseuille_at(yc - h, h, p["mu_H"], p["mu_L"], c["Gx"])
    s = oracle.Sim(nx, ny, p)
    s.set_mesh(np.ones(nx), dy)
    s.init(phi, np.repeat(ua[:, None], nx, axis=1))
    out = []
    for n in steps:
        s.step(n)
        u = s.macros()["u"][:, 0]
        out.append(np.sqrt(((u - ua) ** 2 * dy).sum() / ((ua ** 2) * dy).sum()))
    return np.array(out)


def test_layered_poiseuille_on_a_mesh_clustered_at_walls_and_interface():
    """Sec. IV.B with mu* = 100 on 64 rows: started from the analytic profile,
    the error stays bounded, and 64 rows clustered at both walls and at the
    interface do better than 64 uniform rows at every check."""
    ny, L = 64, 64.0
    e_uni = _poiseuille_errors(np.ones(ny))
    e_clu = _poiseuille_errors(W.clustered_widths(ny, L, [0.0, 0.5 * L, L], fine=0.4))
    print("layered Poiseuille mu*=100, 64 rows: uniform", e_uni, "clustered", e_clu)
    assert np.all(e_clu < e_uni)
    assert np.all(e_clu < 2.5e-2)
