"""Failure detection and the batch / pool boundary on the GPU (through the C
ABI).

A state that turns non-finite (here: a NaN planted in the initial phi, a bad
value and not a device fault) is reported as ENUMERIC at the next
synchronising call and stays reported (sticky) until the next init; in a
batch the message names the case, in the serving pool only that request
fails and every other result is the same as alone, bit for bit. Also the
batch whose cases the batch itself creates (dugks_batch_create +
dugks_batch_case) and the pool admission of an existing handle
(dugks_pool_admit_handle), both against single handles, bit for bit."""
import numpy as np
import pytest

import paper_1810_07802_amd as D
from paper_1810_07802_amd import serve
import workloads as W

pytestmark = pytest.mark.gpu


def _stream():
    import torch
    return torch.cuda.Stream()


def _poisoned(c):
    phi = c["phi"].copy()
    phi[c["ny"] // 3, c["nx"] // 2] = np.nan
    return phi


# every step kernel: one-row, two-row, march (periodic and walls), FP64, and
# the reconstruction march (upwind reconstruction)
KERNELS = [
    ("fp32", 1, "central", False), ("fp32", 2, "central", False), ("fp32", 6, "central", False),
    ("fp32", 6, "central", True), ("fp64", 4, "central", False), ("fp32", None, "upwind", False),
]


@pytest.mark.parametrize("prec,seg,recon,walls", KERNELS)
def test_nan_in_the_initial_phi_is_reported_at_the_next_sync(prec, seg, recon, walls):
    c = (W.random_coupled(70, 36, seed=4, rho_ratio=10.0, walls_y=True) if walls
         else W.bubble(L=48, R=12, steps=0))
    prm = dict(c["params"], recon=recon)
    print(f"numeric flag: {prec} seg={seg} {recon} walls={walls}", flush=True)
    s = D.Solver(c["nx"], c["ny"], prm, "coupled", prec, seg)
    s.set_stream(_stream().cuda_stream)
    s.init(_poisoned(c), c.get("u"), c.get("v"))
    s.step(3)  # asynchronous: nothing to report yet
    with pytest.raises(D.DugksError) as e:
        s.sync()
    assert e.value.code == D.ENUMERIC
    with pytest.raises(D.DugksError) as e:  # sticky: nothing more is enqueued
        s.step(1)
    assert e.value.code == D.ENUMERIC
    assert s.steps_done == 3
    assert s.diagnostics()["status"] == D.ENUMERIC
    # a fresh init clears it
    s.init(c["phi"], c.get("u"), c.get("v"))
    s.step(3)
    s.sync()
    d = s.diagnostics()
    assert d["status"] == D.OK and d["nonfinite"] == 0


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("recon", ["central", "upwind"])
def test_nan_on_a_stretched_mesh_is_reported(prec, recon):
    """The stretched-mesh marches flag a NaN in the initial phi the same way."""
    c = W.bubble(L=48, R=12, steps=0)
    print(f"numeric flag: {prec} {recon} stretched mesh", flush=True)
    s = D.Solver(c["nx"], c["ny"], dict(c["params"], recon=recon), "coupled", prec)
    s.set_stream(_stream().cuda_stream)
    s.set_mesh(W.stretched_widths(48, 0.3), W.stretched_widths(48, 0.3, phase=1.0))
    s.init(_poisoned(c))
    s.step(3)
    with pytest.raises(D.DugksError) as e:
        s.sync()
    assert e.value.code == D.ENUMERIC
    s.init(c["phi"])
    s.step(3)
    s.sync()
    assert s.diagnostics()["status"] == D.OK


def test_a_clean_run_never_reports():
    c = W.bubble(L=64, R=16, steps=0)
    s = D.Solver(c["nx"], c["ny"], c["params"], "coupled", "fp32")
    s.set_stream(_stream().cuda_stream)
    s.init(c["phi"])
    s.step(200)
    s.sync()
    s.autotune(2)  # the probes run on a copy and leave the flag as it was
    s.step(10)
    s.sync()


def test_batch_reports_the_case_and_leaves_the_others_unchanged():
    cases = [W.spinodal(L=48, seed=41, steps=0), W.bubble(L=64, R=16, steps=0),
             W.spinodal(L=40, seed=42, steps=0)]
    ref = []
    for k, c in enumerate(cases):
        if k == 1:
            ref.append(None)
            continue
        s = D.Solver(c["nx"], c["ny"], c["params"], "coupled", "fp32")
        s.init(c["phi"])
        s.step(20)
        ref.append(s.get_state()[0])
    b = D.Batch.create([(c["nx"], c["ny"]) for c in cases])
    b.set_stream(_stream().cuda_stream)
    for k, c in enumerate(cases):
        b.case(k).set_params(c["params"])
        b.case(k).init(_poisoned(c) if k == 1 else c["phi"])
    b.step(20, use_graph=True)
    with pytest.raises(D.DugksError) as e:
        b.sync()
    assert e.value.code == D.ENUMERIC and "case(s) 1" in str(e.value)
    with pytest.raises(D.DugksError) as e:
        b.step(1)
    assert e.value.code == D.ENUMERIC
    for k in (0, 2):
        assert np.array_equal(b.case(k).get_state()[0], ref[k]), k


def test_batch_owned_cases_match_single_handles_bitwise():
    cases = [W.spinodal(L=64, seed=51, steps=0), W.random_coupled(70, 36, seed=52, walls_y=True),
             W.spinodal(L=100, seed=53, steps=0)]
    alone = []
    for c in cases:
        s = D.Solver(c["nx"], c["ny"], c["params"], "coupled", "fp32")
        s.init(c["phi"], c.get("u"), c.get("v"))
        s.step(30)
        alone.append(s.get_state()[0])
    b = D.Batch.create([(c["nx"], c["ny"]) for c in cases])
    b.set_stream(_stream().cuda_stream)
    for k, c in enumerate(cases):
        b.case(k).set_params(c["params"])
        b.case(k).init(c["phi"], c.get("u"), c.get("v"))
    b.step(10, use_graph=False)
    b.step(20, use_graph=True)
    b.sync()
    for k in range(len(cases)):
        assert b.case(k).steps_done == 30
        assert np.array_equal(b.case(k).get_state()[0], alone[k]), k
    del b  # the batch destroys its own cases


def test_pool_fails_only_the_non_finite_request():
    good = [(W.bubble(L=48, R=12, steps=0), 60), (W.spinodal(L=40, seed=5, steps=0), 80)]
    bad = W.bubble(L=48, R=12, steps=0)
    bad = dict(bad, phi=_poisoned(bad))
    pool = D.Pool(1 << 28, max_cases=2, max_cells=64 * 64)
    pool.set_stream(_stream().cuda_stream)
    reqs = [serve.Request(0, good[0][0], good[0][1], 0.0), serve.Request(1, bad, 500, 0.0),
            serve.Request(2, good[1][0], good[1][1], 0.001)]
    out = {s.rid: s for s in serve.run(pool, reqs, chunk=20)}
    assert out[1].error == "ENUMERIC" and out[1].macros is None
    for rid, (c, n) in ((0, good[0]), (2, good[1])):
        s = D.Solver(c["nx"], c["ny"], c["params"], "coupled", "fp32")
        s.init(c["phi"])
        s.step(n)
        ref = s.macros()
        assert out[rid].error is None
        for k in ("phi", "u", "v", "p"):
            assert np.array_equal(out[rid].macros[k], ref[k]), (rid, k)
    # direct status and readout of a failed slot
    k = pool.admit(bad, 10)
    pool.step(10)
    pool.sync()
    assert pool.status(k) == D.ENUMERIC
    with pytest.raises(D.DugksError) as e:
        pool.macros(k)
    assert e.value.code == D.ENUMERIC
    pool.retire(k)


@pytest.mark.parametrize("kind", ["coupled", "deform"])
def test_pool_admits_a_handle_at_its_current_state_and_time(kind):
    if kind == "coupled":
        c = W.random_coupled(70, 36, seed=61, rho_ratio=10.0, walls_y=True)
        model, prec = "coupled", "fp32"
    else:  # time-dependent prescribed velocity: the slot must go on at the handle's time
        c = W.smoothed_deformation(L0=64, Pe=64, M=0.02)
        model, prec = "ac", "fp64"
    a = D.Solver(c["nx"], c["ny"], c["params"], model, prec)
    a.init(c["phi"], c.get("u"), c.get("v"))
    a.step(25)
    pool = D.Pool(1 << 28, max_cases=2, max_cells=c["nx"] * c["ny"], precision=prec, model=model)
    pool.set_stream(_stream().cuda_stream)
    k = pool.admit_handle(a, 35)
    assert k is not None
    a.step(35)  # the handle goes on by itself; the slot holds its own copy
    ref = a.macros()
    pool.step(40)
    assert pool.remaining(k) == 0
    got = pool.macros(k)
    for f in ("phi", "u", "v", "p"):
        assert np.array_equal(got[f], ref[f]), f
