"""The serving pool on the GPU (through the C ABI): every request's result is
the same alone and in the mix, bit for bit, whatever else runs beside it and
whenever it was admitted; the served layered Poiseuille flow keeps its
analytic profile (Sec. IV.B); arena memory is reused after retirement."""
import numpy as np
import pytest

import paper_1810_07802_amd as D
from paper_1810_07802_amd import serve
import workloads as W

pytestmark = pytest.mark.gpu


def _stream():
    import torch
    return torch.cuda.Stream()


def alone(case, steps, precision="fp32"):
    s = D.Solver(case["nx"], case["ny"], case["params"], "coupled", precision)
    s.init(case["phi"], case.get("u"), case.get("v"), case.get("p"))
    s.step(steps)
    return s.macros()


def mix():
    cases = [
        (W.bubble(L=48, R=12, steps=0), 120),
        (W.layered_poiseuille(nx=16, ny=64, mu_ratio=100.0, analytic_init=True, steps=0), 150),
        (W.spinodal(L=40, seed=5, steps=0), 60),
        (W.random_coupled(70, 36, seed=4, rho_ratio=10.0, walls_y=True), 90),
        (W.bubble(L=100, R=25, steps=0), 40),
        (W.random_coupled(130, 50, seed=7, rho_ratio=50.0), 75),
    ]
    return cases


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_results_are_the_same_alone_and_in_the_mix(precision):
    cases = mix()
    st = _stream()
    pool = D.Pool(1 << 30, max_cases=4, max_cells=100 * 100, precision=precision)
    pool.set_stream(st.cuda_stream)
    # staggered arrivals, fewer slots than requests: cases join and leave a
    # running set of changing composition
    reqs = [serve.Request(k, c, n, 0.002 * k) for k, (c, n) in enumerate(cases)]
    out = serve.run(pool, reqs, chunk=16)
    assert sorted(s.rid for s in out) == list(range(len(cases)))
    for s in out:
        c, n = cases[s.rid]
        ref = alone(c, n, precision)
        for k in ("phi", "u", "v", "p"):
            assert np.array_equal(s.macros[k], ref[k]), (s.rid, k)


def test_served_poiseuille_keeps_the_analytic_profile():
    c = W.layered_poiseuille(nx=64, ny=128, mu_ratio=100.0, analytic_init=True, steps=0)
    pool = D.Pool(1 << 28, max_cases=2, max_cells=64 * 128)
    pool.set_stream(_stream().cuda_stream)
    out = serve.run(pool, [serve.Request(0, c, 2000, 0.0)], chunk=500)
    u = out[0].macros["u"].mean(axis=1)
    ua = W.poiseuille_analytic(128, c["params"]["mu_H"], c["params"]["mu_L"], c["Gx"])
    err = np.linalg.norm(u - ua) / np.linalg.norm(ua)
    print(f"served Poiseuille 64x128 mu*=100, 2000 steps: relative L2 {err:.2e}", flush=True)
    assert err < 1e-2


def test_arena_memory_is_reused_after_retirement():
    c = W.bubble(L=64, R=16, steps=0)
    pool = D.Pool(1 << 30, max_cases=8, max_cells=64 * 64)
    one = pool.case_bytes(64, 64)
    pool = D.Pool(2 * one, max_cases=8, max_cells=64 * 64)
    pool.set_stream(_stream().cuda_stream)
    a = pool.admit(c, 10)
    b = pool.admit(c, 10)
    assert a is not None and b is not None and a != b
    assert pool.admit(c, 10) is None  # EBUSY: the arena is full
    pool.step(10)
    ref = pool.macros(a)
    pool.retire(a)
    pool.sync()
    assert pool.bytes_free() == one
    d = pool.admit(c, 10)
    assert d is not None
    pool.step(10)
    again = pool.macros(d)
    assert np.array_equal(again["phi"], ref["phi"]) and np.array_equal(again["u"], ref["u"])
    assert pool.remaining(b) == 0 and pool.steps_done(b) == 10
