"""Edge cases of the HIP path: the smallest grids the C ABI accepts (one
strip far narrower than a wave, walls on the minimum height), ragged strips,
and the degenerate uniform state, against the FP64 oracle or exactly."""
import numpy as np
import pytest

import oracle
import paper_1810_07802_amd as D
import workloads as W

pytestmark = pytest.mark.gpu


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def both(c, steps, prec="fp64", seg=None):
    s = D.Solver(c["nx"], c["ny"], c["params"], c["model"], prec, seg)
    s.init(c["phi"], c["u"], c["v"], c["p"])
    s.step(steps)
    o = oracle.Sim(c["nx"], c["ny"], c["params"], c["model"])
    o.init(c["phi"], c["u"], c["v"], c["p"])
    o.step(steps)
    return s.macros(), o.macros()


@pytest.mark.parametrize("nx,ny,walls,seg", [(3, 3, False, None), (3, 3, False, 2), (5, 4, True, None),
                                              (5, 4, True, 3), (63, 7, False, None), (125, 5, True, 1)])
def test_small_and_ragged_grids_match_the_oracle(nx, ny, walls, seg):
    """Relative L2 <= 1e-12 per field, or, for fields that are residuals far
    below their scale on these grids (the velocity of a shear that vanishes
    at the walls, the pressure of a 3-cell periodic box, v where no force
    drives it), a maximum absolute difference <= 1e-15: rounding of values
    of 1e-4 and less."""
    c = W.random_coupled(nx, ny, seed=nx * 100 + ny, rho_ratio=10.0, walls_y=walls)
    g, r = both(c, 60, "fp64", seg)
    for k in ("phi", "u", "v", "p"):
        e, a = rel(g[k], r[k]), np.abs(g[k] - r[k]).max()
        print(f"{nx}x{ny} walls={walls} seg={seg} {k}: rel {e:.2e} abs {a:.2e}", flush=True)
        assert e < 1e-12 or a < 1e-15, (k, e, a)


@pytest.mark.parametrize("nx,ny", [(3, 3), (61, 3), (62, 9), (64, 5)])
def test_interface_only_small_grids(nx, ny):
    c = W.smoothed_deformation(L0=64, Pe=64, M=0.02)
    X, Y = np.meshgrid(np.arange(nx) + 0.5, np.arange(ny) + 0.5)
    c = dict(c, nx=nx, ny=ny, phi=np.ascontiguousarray(0.5 + 0.4 * np.sin(2 * np.pi * X / nx)
                                                       * np.cos(2 * np.pi * Y / ny)))
    c["params"] = dict(c["params"], vel="rotation", L0=float(max(nx, ny)))
    g, r = both(c, 40, "fp64")
    assert rel(g["phi"], r["phi"]) < 1e-12


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("walls", [False, True])
def test_uniform_state_is_preserved_bitwise(prec, walls):
    """No interface and no flow: every equilibrium equals its distribution,
    every source vanishes, every face reconstruction and flux difference is
    exact, so the state does not change by a single bit."""
    c = W.random_coupled(70, 36, seed=1, rho_ratio=10.0, walls_y=walls)
    c["params"] = dict(c["params"], gy=0.0)  # no gravity: a uniform state is at rest
    c["phi"] = np.full((36, 70), 0.3)
    s = D.Solver(70, 36, c["params"], "coupled", prec)
    s.init(c["phi"])
    s.step(1)  # the first step sets the history (phi u = 0 from the start)
    before = s.get_state()[0]
    s.step(25)
    assert np.array_equal(s.get_state()[0], before)


def test_empty_step_requests_change_nothing():
    """Zero steps (single handle, batch with and without graphs) leave the
    state and the step count as they were; a negative count is EINVAL."""
    import torch

    c = W.random_coupled(70, 36, seed=2, rho_ratio=10.0)
    s = D.Solver(70, 36, c["params"], "coupled", "fp32")
    s.init(c["phi"], c["u"], c["v"])
    s.step(3)
    before, n0 = s.get_state()[0], s.steps_done
    s.step(0)
    assert s.steps_done == n0 and np.array_equal(s.get_state()[0], before)
    with pytest.raises(D.DugksError) as e:
        s.step(-1)
    assert e.value.code == D.EINVAL
    st = torch.cuda.Stream()
    b = D.Batch([s])
    b.set_stream(st.cuda_stream)
    b.step(0)
    b.step(0, use_graph=True)
    b.sync()
    assert s.steps_done == n0 and np.array_equal(s.get_state()[0], before)


def _decode_state(buf, nx, ny, coupled, dtype):
    """Split a saved state by the layout dugks.h documents: ny rows, each the
    value groups of its nx cells (groups of four consecutive values,
    cell-interleaved, a last partial group of w values), then phi, padded
    to a multiple of 128 bytes."""
    es = np.dtype(dtype).itemsize
    nv = 20 if coupled else 11  # grouped values: f0..f8, [g0..g8], hist_x, hist_y
    rb = -(-(nv + 1) * nx * es // 128) * 128
    assert buf.nbytes == rb * ny
    rows = buf.reshape(ny, rb)
    vals = np.empty((nv, ny, nx), dtype=dtype)
    for v0 in range(0, nv, 4):
        w = min(4, nv - v0)
        blk = rows[:, v0 * nx * es:(v0 + w) * nx * es].copy().view(dtype).reshape(ny, nx, w)
        for k in range(w):
            vals[v0 + k] = blk[:, :, k]
    phi = rows[:, nv * nx * es:(nv + 1) * nx * es].copy().view(dtype).reshape(ny, nx)
    pad = rows[:, (nv + 1) * nx * es:]
    return vals, phi, pad


@pytest.mark.parametrize("prec,model,nx,ny", [("fp32", "coupled", 70, 9), ("fp64", "coupled", 37, 6),
                                              ("fp32", "ac", 5, 7), ("fp64", "ac", 64, 5)])
def test_saved_state_follows_the_documented_layout(prec, model, nx, ny):
    """A checkpoint decoded by the documented layout: the padding reads zero,
    the stored phi is the sum of the stored f in the order the kernels form
    it (bit for bit), and get_macros returns that phi."""
    dtype = np.float32 if prec == "fp32" else np.float64
    if model == "coupled":
        c = W.random_coupled(nx, ny, seed=nx, rho_ratio=10.0)
    else:
        c = W.smoothed_deformation(L0=64, Pe=64, M=0.02)
        c["params"] = dict(c["params"], vel="rotation", T_period=400.0, U0=0.02)
        c["phi"] = c["phi"][:ny, :nx]
    s = D.Solver(nx, ny, c["params"], model, prec)
    s.init(c["phi"])
    for steps in (0, 3):  # after init, then after 3 steps (the other buffer)
        if steps:
            s.step(steps)
        buf, _ = s.get_state()
        vals, phi, pad = _decode_state(buf, nx, ny, model == "coupled", dtype)
        assert not pad.any()
        acc = np.zeros((ny, nx), dtype=dtype)
        for q in range(9):
            acc = acc + vals[q]
        assert np.array_equal(acc, phi)
        assert np.array_equal(s.macros()["phi"], phi.astype(np.float64))


@pytest.mark.parametrize("prec,nx,ny,walls,mode", [("fp32", 1 << 26, 4, True, "march"),
                                                   ("fp32", 1 << 21, 128, False, "march"),
                                                   ("fp64", 1 << 25, 4, False, "march"),
                                                   ("fp32", 1 << 26, 4, True, "upwind"),
                                                   ("fp32", 1 << 21, 128, False, "mesh_y")])
def test_largest_grids_evolve_like_a_narrow_grid(prec, nx, ny, walls, mode):
    """Grids at the size limit of the C ABI (2^28 cells in FP32, 2^27 in
    FP64), as rows of up to 5.6 GB or as 22 GB buffers of many rows; the
    fused march, and the reconstruction march (upwind reconstruction, a mesh
    stretched along y). The initial state
    varies along y only, so every cell of a row sees the same inputs and must
    end with the bits of the same row of a 64-column grid (whose kernels give
    the march's bits): an address wrapped at 2^31 or 2^32 bytes, or a tile
    that misses cells, shows as a column that differs."""
    import torch

    c = W.random_coupled(64, ny, seed=3, rho_ratio=1000.0, walls_y=walls)
    p = dict(c["params"], recon="upwind") if mode == "upwind" else c["params"]
    dy = W.stretched_widths(ny, 0.3) if mode == "mesh_y" else None
    y = (np.arange(ny) + 0.5) / ny
    prof = p["phi_L"] + (p["phi_H"] - p["phi_L"]) * (0.5 + 0.45 * np.cos(2 * np.pi * y))
    steps = 3

    def run(width):
        s = D.Solver(width, ny, p, "coupled", prec)
        if dy is not None:
            s.set_mesh(None, dy)
        phi0 = torch.tensor(prof, device="cuda")[:, None].expand(ny, width).contiguous()
        out = {k: torch.empty((ny, width), dtype=torch.float64, device="cuda") for k in ("phi", "u", "v")}
        torch.cuda.synchronize()  # the library works on its own stream
        s.init_device(phi0)
        s.step(steps)
        s.macros_device(out)
        s.sync()
        del s, phi0
        return out

    ref = run(64)
    for k in ("phi", "u", "v"):  # the narrow grid is uniform along x itself
        assert torch.equal(ref[k], ref[k][:, :1].expand(ny, 64))
    assert torch.isfinite(ref["phi"]).all() and (ref["v"] != 0).any()
    big = run(nx)
    for k in ("phi", "u", "v"):
        same = big[k] == ref[k][:, :1]
        assert bool(same.all()), f"{k}: {int((~same).sum())} cells differ, first {torch.nonzero(~same)[:4].tolist()}"
    del big
    torch.cuda.empty_cache()
