"""Call splitting, through the C ABI: a lattice with fixed solids stepped in
calls of 1, 2, 3, 5 and 7 steps computes bit for bit what it computes in one
call of 18 steps.

Within one lbm_step call the sweep applies the bounce-back of the previous step
itself (fixed solids); the last step of a call is finished by the bounce-back
kernel, whose ghost values the first step of the next call pulls.  Splitting
therefore changes which route evaluates the bounce-back and the force of each
step.  Bar: identical bits for the state, the per-step force/torque history and
the macroscopic fields.  (The FP64 oracle comparisons in test_gpu_parity.py
cover both routes against the paper's method.)
"""
import numpy as np
import pytest

from paper_1906_05445_amd import workloads as W

pytestmark = pytest.mark.gpu

SPLIT = [1, 2, 3, 5, 7]


@pytest.fixture(scope="module")
def lbm():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1906_05445_amd import lbm as L

    return L


CASES = {
    # narrow gaps: nodes with links to two solids, missing x_ff / x_fff (fallback formulas)
    "d3q19_mrt_f32_quadratic_gaps": ("D3Q19", "MRT", "F32", (31, 29, 27), 0.7, (2e-6, 0.0, 1e-6),
                                     [W.solid("sphere", (9.5, 10.2, 9.9), 5.5),
                                      W.solid("sphere", (21.6, 10.4, 9.3), 5.2),
                                      W.solid("cylinder", (0.0, 22.3, 16.6), 3.1, axis=(1, 0, 0))],
                                     "QUADRATIC", None),
    "d3q19_bgk_f64_linear": ("D3Q19", "BGK", "F64", (37, 29, 23), 0.8, (3e-6, 1e-6, -5e-7),
                             [W.solid("sphere", (18.3, 14.1, 11.7), 7.6)], "LINEAR", None),
    "d3q19_mrt_f16_bounceback": ("D3Q19", "MRT", "F16", (33, 30, 26), 0.9, (1e-5, 0.0, 0.0),
                                 [W.solid("sphere", (16.2, 15.1, 12.8), 6.1)], "BB", None),
    "d3q19_general_rates_f32_quadratic": ("D3Q19", "MRT", "F32", (30, 28, 26), 0.8, (1.5e-6, 0.0, 0.0),
                                          [W.solid("sphere", (15.2, 13.9, 12.8), 4.9)], "QUADRATIC",
                                          np.array([0, 1.2, 1.4, 0, 1.1, 0, 1.1, 0, 1.1, 1.25, 1.3, 1.25, 1.3,
                                                    1.25, 1.25, 1.25, 1.5, 1.5, 1.5])),
    # rotating outer wall (wall velocity from the lever arm), inverted solid
    "d2q9_mrt_f64_couette": ("D2Q9", "MRT", "F64", (46, 46, 1), 1.0, (0.0, 0.0, 0.0),
                             [W.solid("cylinder", (23.31, 22.83, 0.0), 9.3),
                              W.solid("cylinder", (23.31, 22.83, 0.0), 20.1, inverted=True,
                                      omega=(0, 0, 0.01 / 20.1))], "QUADRATIC", None),
    "d2q9_bgk_f32_quadratic": ("D2Q9", "BGK", "F32", (61, 47, 1), 0.8, (1e-6, 2e-7, 0.0),
                               [W.solid("cylinder", (30.4, 23.7, 0.0), 7.3)], "QUADRATIC", None),
    # Yu's scheme (five populations per link) in the sweep and in the kernel, with gaps
    "d3q19_mrt_f32_yu_gaps": ("D3Q19", "MRT", "F32", (31, 29, 27), 0.7, (2e-6, 0.0, 1e-6),
                              [W.solid("sphere", (9.5, 10.2, 9.9), 5.5),
                               W.solid("sphere", (21.6, 10.4, 9.3), 5.2),
                               W.solid("cylinder", (0.0, 22.3, 16.6), 3.1, axis=(1, 0, 0))],
                              "YU", None),
    # Zhao & Yong's scheme stays with the bounce-back kernel after every sweep
    "d3q19_mrt_f16_zhao_yong": ("D3Q19", "MRT", "F16", (33, 30, 26), 0.9, (1e-5, 0.0, 0.0),
                                [W.solid("sphere", (16.2, 15.1, 12.8), 6.1)], "ZHAO_YONG", None),
    # FP16 with stochastic rounding: the link values of the sweep and of the bounce-back kernel take the
    # same dither (slot and step), so splitting calls changes nothing
    "d3q19_mrt_f16sr_quadratic": ("D3Q19", "MRT", "F16_SR", (33, 30, 26), 0.9, (1e-5, 0.0, 0.0),
                                  [W.solid("sphere", (16.2, 15.1, 12.8), 6.1)], "QUADRATIC", None),
    "d3q19_mrt_f16sr_zhao_yong": ("D3Q19", "MRT", "F16_SR", (33, 30, 26), 0.9, (1e-5, 0.0, 0.0),
                                  [W.solid("sphere", (16.2, 15.1, 12.8), 6.1)], "ZHAO_YONG", None),
}


def _make(lbm, case):
    lat, coll, storage, shape, tau, g, solids, method, rates = case
    ctx = lbm.Lattice(lat, coll, storage, shape, tau, rates=rates, g=g, max_solids=len(solids))
    ctx.set_solids(solids, method)
    return ctx


def _same(a, b, what):
    a, b = np.asarray(a), np.asarray(b)
    assert a.shape == b.shape, what
    assert np.array_equal(a.view(np.uint8), b.view(np.uint8)), f"{what} differs"


@pytest.mark.parametrize("name", sorted(CASES))
def test_split_calls_match_one_call(lbm, name):
    case = CASES[name]
    one = _make(lbm, case)
    one.step(sum(SPLIT))
    split = _make(lbm, case)
    for n in SPLIT:
        split.step(n)
    assert one.time == split.time == sum(SPLIT)
    _same(one.get_state(), split.get_state(), "state")
    _same(one.history(), split.history(), "force/torque history")
    for what, a, b in zip(("rho", "u", "node types"), one.macros(), split.macros()):
        _same(a, b, what)
    assert np.all(np.isfinite(one.history()))
    one.close()
    split.close()


def test_autotune_reports_policy(lbm):
    """After the tuning sweeps the context reports its sweep policy (non-temporal
    stores, tile order tuned) and the time of both tile orders; results do not
    depend on the policy (the split-call cases above tune in their first steps)."""
    ctx = _make(lbm, CASES["d3q19_bgk_f64_linear"])
    ctx.step(70)  # tuning: 8 sweeps skipped, then 4 runs of 12
    info = ctx.autotune_info()
    assert info["policy"] in ("nontemporal_linear", "nontemporal_xcd")
    assert info["sweep_us"]["nontemporal_linear"] > 0.0 and info["sweep_us"]["nontemporal_xcd"] > 0.0
    assert info["sweep_us"]["plain_linear"] == 0.0 and info["sweep_us"]["plain_xcd"] == 0.0
    assert info["nontemporal_stores"] == 1
    ctx.close()
