"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle on
generic synthetic cases, plus the GPU-side invariants (tiling, checkpoint,
batch, diagnostics).

FP64 tolerance: relative L2 norm ||gpu - oracle|| / ||oracle|| <= 1e-12 for
every field after hundreds of steps; both sides evaluate the same double
formulas in a different order, so the difference is accumulated rounding.
Sizes span several 62-column strips with a ragged last strip and several row
segments, and cover periodic and wall-bounded y. The benchmark configurations
at full size, and the FP32 path, are in test_gpu_configs.py.
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


def run_both(case, steps, precision, seg_rows=None):
    s = D.Solver(case["nx"], case["ny"], case["params"], case["model"], precision, seg_rows)
    s.init(case["phi"], case["u"], case["v"], case["p"])
    s.step(steps)
    g = s.macros()
    o = oracle.Sim(case["nx"], case["ny"], case["params"], case["model"])
    o.init(case["phi"], case["u"], case["v"], case["p"])
    o.step(steps)
    r = o.macros()
    return g, r, s


def _report(tag, g, r):
    errs = {k: rel(g[k], r[k]) for k in ("phi", "u", "v", "p")}
    print(tag, " ".join(f"{k}={v:.2e}" for k, v in errs.items()), flush=True)
    return errs


@pytest.mark.parametrize("seg", [1, 4, 16])
def test_fp64_coupled_periodic(seg):
    c = W.random_coupled(100, 40, seed=3, rho_ratio=100.0)
    g, r, _ = run_both(c, 300, "fp64", seg)
    e = _report(f"fp64 periodic seg={seg}", g, r)
    for k in ("phi", "u", "v", "p"):
        assert e[k] < 1e-12, (k, e[k])


@pytest.mark.parametrize("seg", [1, 8])
def test_fp64_coupled_walls(seg):
    c = W.random_coupled(70, 36, seed=4, rho_ratio=10.0, walls_y=True)
    g, r, _ = run_both(c, 300, "fp64", seg)
    e = _report("fp64 walls", g, r)
    for k in ("phi", "u", "v", "p"):
        assert e[k] < 1e-12, (k, e[k])


@pytest.mark.parametrize("vel", ["uniform", "rotation", "shear", "deform"])
def test_fp64_interface_only(vel):
    c = W.smoothed_deformation(L0=96, Pe=96, M=0.02)
    c["params"] = dict(c["params"], vel=vel, T_period=400.0, U0=0.02)
    g, r, _ = run_both(c, 400, "fp64", 16)
    e = _report(f"fp64 ac {vel}", g, r)
    assert e["phi"] < 1e-12
    assert e["u"] < 1e-14 and e["v"] < 1e-14


def test_fp64_density_ratio_1000_driven_flow():
    """A well-conditioned flow (|u| ~ 1e-2) across a 1000:1 interface."""
    c = W.random_coupled(100, 40, seed=5, rho_ratio=1000.0, U=0.01)
    g, r, _ = run_both(c, 100, "fp64", 8)
    e = _report("fp64 ratio1000", g, r)
    for k in ("phi", "u", "v", "p"):
        assert e[k] < 1e-12, (k, e[k])


@pytest.mark.parametrize("walls", [False, True])
@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_tiling_does_not_change_bits(walls, prec):
    """Segments of 2, 7 and 64 rows (one wave marching each) and of 1 row
    (the three-wave row kernel) give the same state bit for bit."""
    c = W.random_coupled(130, 50, seed=7, rho_ratio=50.0, walls_y=walls)
    states = []
    for seg in (2, 1, 7, 64):
        s = D.Solver(c["nx"], c["ny"], c["params"], "coupled", prec, seg)
        s.init(c["phi"], c["u"], c["v"])
        s.step(50)
        states.append(s.get_state()[0])
    for k in range(1, 4):
        assert np.array_equal(states[0], states[k]), k


def test_row_kernel_interface_only_bits():
    c = W.smoothed_deformation(L0=96, Pe=96, M=0.02)
    c["params"] = dict(c["params"], vel="shear", T_period=400.0, U0=0.02)
    states = []
    for seg in (3, 1):
        s = D.Solver(c["nx"], c["ny"], c["params"], "ac", "fp64", seg)
        s.init(c["phi"])
        s.step(120)
        states.append(s.get_state()[0])
    assert np.array_equal(states[0], states[1])


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_checkpoint_resume_bitwise(prec):
    c = W.random_coupled(70, 36, seed=8, rho_ratio=10.0, walls_y=True)
    a = D.Solver(c["nx"], c["ny"], c["params"], "coupled", prec)
    a.init(c["phi"])
    a.step(31)
    buf, st = a.get_state()
    a.step(30)
    b = D.Solver(c["nx"], c["ny"], c["params"], "coupled", prec)
    b.set_state(buf, st)
    b.step(30)
    assert b.steps_done == a.steps_done == 61
    assert np.array_equal(a.get_state()[0], b.get_state()[0])


@pytest.mark.parametrize("created_stream", [False, True])
def test_autotune_restores_state_and_keeps_bits(created_stream):
    """The probes (direct launches on the null stream, captured graphs on a
    created one) leave the state and step counter as they were, and the
    chosen tile changes no bit."""
    import torch
    c = W.random_coupled(130, 50, seed=11, rho_ratio=50.0)
    ref = D.Solver(c["nx"], c["ny"], c["params"], "coupled", "fp32")
    ref.init(c["phi"], c["u"], c["v"])
    ref.step(25)
    s = D.Solver(c["nx"], c["ny"], c["params"], "coupled", "fp32")
    stream = torch.cuda.Stream()
    if created_stream:
        s.set_stream(stream.cuda_stream)
    s.init(c["phi"], c["u"], c["v"])
    s.step(10)
    before, n0 = s.get_state()
    seg, us = s.autotune(5)
    after, n1 = s.get_state()
    assert n0 == n1 == 10 and np.array_equal(before, after)
    assert s.seg_rows == seg and seg >= 1 and us > 0
    s.step(15)
    assert np.array_equal(s.get_state()[0], ref.get_state()[0])


def test_batch_matches_single_cases_bitwise():
    cases = [W.spinodal(L=L, seed=10 + k, steps=0) for k, L in enumerate((64, 100, 37))]
    alone, solvers = [], []
    for c in cases:
        s = D.Solver(c["nx"], c["ny"], c["params"], "coupled", "fp32")
        s.init(c["phi"])
        s.step(40)
        alone.append(s.get_state()[0])
        t = D.Solver(c["nx"], c["ny"], c["params"], "coupled", "fp32")
        t.init(c["phi"])
        solvers.append(t)
    import torch
    stream = torch.cuda.Stream()
    b = D.Batch(solvers)
    b.set_stream(stream.cuda_stream)
    b.step(15, use_graph=False)
    b.step(25, use_graph=True)
    b.sync()
    for k, s in enumerate(solvers):
        assert s.steps_done == 40
        assert np.array_equal(s.get_state()[0], alone[k]), k


@pytest.mark.parametrize("created_stream", [True, False])
def test_batch_autotune_restores_states_and_keeps_bits(created_stream):
    """The probes (captured graphs on a created stream, direct launches on
    the null stream) leave every state and step counter as it was, and the
    chosen tiles change no bit."""
    cases = [W.spinodal(L=64, seed=30, steps=0), W.random_coupled(70, 36, seed=31, walls_y=True),
             W.spinodal(L=100, seed=32, steps=0), W.random_coupled(130, 50, seed=33, walls_y=True)]
    solvers, alone = [], []
    for c in cases:
        a = D.Solver(c["nx"], c["ny"], c["params"], "coupled", "fp32")
        a.init(c["phi"], c.get("u"), c.get("v"))
        a.step(30)
        alone.append(a.get_state()[0])
        t = D.Solver(c["nx"], c["ny"], c["params"], "coupled", "fp32")
        t.init(c["phi"], c.get("u"), c.get("v"))
        solvers.append(t)
    import torch
    stream = torch.cuda.Stream()
    b = D.Batch(solvers)
    if created_stream:
        b.set_stream(stream.cuda_stream)
    b.step(10, use_graph=False)
    b.sync()
    before = [s.get_state()[0] for s in solvers]
    seg_p, seg_w = b.autotune(3)
    if not created_stream:
        b.set_stream(stream.cuda_stream)  # graphs need a created stream
    assert seg_p >= 1 and seg_w >= 1
    for k, s in enumerate(solvers):
        assert s.steps_done == 10
        assert np.array_equal(s.get_state()[0], before[k]), k
    b.step(20, use_graph=True)
    b.sync()
    for k, s in enumerate(solvers):
        assert np.array_equal(s.get_state()[0], alone[k]), k


def test_batch_budget_stops_a_case():
    cases = [W.spinodal(L=48, seed=20 + k, steps=0) for k in range(2)]
    solvers = []
    for c in cases:
        s = D.Solver(c["nx"], c["ny"], c["params"], "coupled", "fp32")
        s.init(c["phi"])
        solvers.append(s)
    ref = D.Solver(cases[1]["nx"], cases[1]["ny"], cases[1]["params"], "coupled", "fp32")
    ref.init(cases[1]["phi"])
    ref.step(7)
    b = D.Batch(solvers)
    b.set_budget(1, 7)
    b.step(20)
    b.sync()
    assert solvers[0].steps_done == 20 and solvers[1].steps_done == 7
    assert np.array_equal(solvers[1].get_state()[0], ref.get_state()[0])


def test_diagnostics_match_oracle_sums():
    c = W.random_coupled(100, 40, seed=9, rho_ratio=100.0)
    g, r, s = run_both(c, 100, "fp64")
    d = s.diagnostics()
    assert d["status"] == 0 and d["nonfinite"] == 0
    assert d["sum_phi"] == pytest.approx(r["phi"].sum(), rel=1e-12)
    # the momentum sums cancel; compare against the sum of magnitudes
    scale_u = np.abs(r["rho"] * r["u"]).sum()
    assert abs(d["sum_rho_u"] - (r["rho"] * r["u"]).sum()) < 1e-12 * scale_u
    assert d["sum_rho"] == pytest.approx(r["rho"].sum(), rel=1e-12)
    assert d["max_u"] == pytest.approx(np.hypot(r["u"], r["v"]).max(), rel=1e-10)
    ke = (0.5 * r["rho"] * (r["u"] ** 2 + r["v"] ** 2)).sum()
    assert d["kinetic"] == pytest.approx(ke, rel=1e-12)
    assert d["time"] == pytest.approx(100 * c["params"]["cfl"])
    # the wavefront and block reductions have a fixed order: same bits again
    assert s.diagnostics() == d


def test_graph_replays_match_direct_steps_with_eager_work_between():
    """A captured step sequence replayed four times, with direct launches,
    host readouts and torch work on the same stream between the replays:
    after every replay each case equals the same case stepped alone."""
    import torch
    cases = [W.spinodal(L=L, seed=40 + k, steps=0) for k, L in enumerate((64, 37))]
    solvers, refs = [], []
    for c in cases:
        for lst in (solvers, refs):
            s = D.Solver(c["nx"], c["ny"], c["params"], "coupled", "fp32")
            s.init(c["phi"])
            lst.append(s)
    stream = torch.cuda.Stream()
    b = D.Batch(solvers)
    b.set_stream(stream.cuda_stream)
    done = 0
    for rep in range(4):
        b.step(6, use_graph=True)
        b.step(2, use_graph=False)
        with torch.cuda.stream(stream):
            torch.ones(1 << 20, device="cuda").sum()  # unrelated eager work
        b.sync()
        done += 8
        for k, (s, r) in enumerate(zip(solvers, refs)):
            r.step(8)
            assert s.steps_done == done
            assert np.array_equal(s.get_state()[0], r.get_state()[0]), (rep, k)
            s.macros()


def test_graph_steps_need_a_stream():
    c = W.spinodal(L=40, seed=50, steps=0)
    s = D.Solver(c["nx"], c["ny"], c["params"], "coupled", "fp32")
    s.init(c["phi"])
    b = D.Batch([s])
    with pytest.raises(D.DugksError) as e:
        b.step(3, use_graph=True)  # no stream set: the null stream
    assert e.value.code == D.EINVAL and "stream" in str(e.value)
    b.step(3, use_graph=False)
    b.sync()
    assert s.steps_done == 3


@pytest.mark.parametrize("variant", ["central", "upwind", "mesh"])
def test_handle_graph_replays_match_direct_launches(variant):
    """Solver.step on a created stream replays captured graphs (8 or more
    steps); interleaved with short direct sequences, readouts and torch work,
    and with a change of reconstruction that drops the graphs, the state
    equals a handle stepped by direct launches on the null stream, bit for
    bit, after every call."""
    import torch
    c = W.random_coupled(70, 36, seed=60, rho_ratio=10.0, walls_y=(variant == "upwind"))
    recon = "upwind" if variant == "upwind" else "central"
    c["params"] = dict(c["params"], recon=recon)
    dx = W.stretched_widths(70, 0.3) if variant == "mesh" else None
    stream = torch.cuda.Stream()
    a = D.Solver(c["nx"], c["ny"], c["params"], "coupled", "fp32")
    b = D.Solver(c["nx"], c["ny"], c["params"], "coupled", "fp32")
    a.set_stream(stream.cuda_stream)
    for s in (a, b):
        if dx is not None:
            s.set_mesh(dx, None)
        s.init(c["phi"], c["u"], c["v"])
    for rep, n in enumerate((12, 3, 12, 12, 9)):
        if rep == 3:  # a new variant: the recorded sequences are dropped
            other = dict(c["params"], recon="central" if recon == "upwind" else "upwind")
            a.set_params(other)
            b.set_params(other)
        a.step(n)
        b.step(n)
        with torch.cuda.stream(stream):
            torch.ones(1 << 20, device="cuda").sum()
        torch.cuda.synchronize()
        assert a.steps_done == b.steps_done
        assert np.array_equal(a.get_state()[0], b.get_state()[0]), (variant, rep)
        a.macros()


@pytest.mark.parametrize("model,nx,ny", [("coupled", 130, 51), ("coupled", 3, 3), ("coupled", 64, 5),
                                         ("ac", 96, 37), ("coupled", 128, 128)])
def test_two_row_tiles_give_the_same_bits(model, nx, ny):
    """2-row tiles of periodic FP32 cases run the four-wave two-row kernel:
    the same state bit for bit as 1-row tiles (the row kernel) and 5-row
    segments (the march), odd heights (a last tile of one row) and grids
    smaller than one tile included."""
    if model == "coupled":
        c = W.random_coupled(nx, ny, seed=nx + ny, rho_ratio=100.0)
    else:
        c = W.smoothed_deformation(L0=96, Pe=96, M=0.02)
        c["params"] = dict(c["params"], vel="shear", T_period=400.0, U0=0.02)
        c["phi"] = np.ascontiguousarray(c["phi"][:ny, :nx])
        c["u"] = c["v"] = None
    states = []
    for seg in (2, 1, 5):
        s = D.Solver(nx, ny, c["params"], model, "fp32", seg)
        s.init(c["phi"], c["u"], c["v"])
        s.step(40)
        states.append(s.get_state()[0])
    assert np.array_equal(states[0], states[1])
    assert np.array_equal(states[0], states[2])
