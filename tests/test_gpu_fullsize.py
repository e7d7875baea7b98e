"""Full-size workloads in the launch configuration bench.py times, through the C ABI.

* 256^3 box with 64 spheres (gaps down to 2 lattice units, 296k boundary links), FP64 storage,
  quadratic and single-node (Zhao-Yong) interpolated bounce-back, and FP32 storage with quadratic
  bounce-back (the bench line's configuration): node classification, link set and q bit-exact against
  the FP64 oracle, fields (max|du|/max|u|, max|drho|) and per-sphere force/torque after two steps at
  1e-12 (FP64) or the FP32 bars (the oracle needs about half a minute per step at this size).
* 512 lattices with translating spheres stepped as one FP32 batch (the batching workload, about
  1.7e8 cells): sampled members (the smallest, the largest and the median lattice) are bit for bit
  their lone runs after the batch's tuning steps.
"""
import os

import numpy as np
import pytest

from paper_1906_05445_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lbm():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1906_05445_amd import lbm as L

    return L


# FP32 storage (the configuration of the bench line): the FP32 bars of the periodic parity tests,
# relative 2e-5 in velocity and 1e-4 in force, density 1e-6 absolute
BARS = {"F64": {"u": 1e-12, "rho": 1e-12, "F": 1e-12}, "F32": {"u": 2e-5, "rho": 1e-6, "F": 1e-4}}


@pytest.mark.timeout(600)
@pytest.mark.parametrize("method,storage", [("QUADRATIC", "F64"), ("ZHAO_YONG", "F64"), ("QUADRATIC", "F32")])
def test_pack256_against_oracle(lbm, method, storage):
    from oracle import Oracle

    case = W.sphere_pack(storage=storage, method=method)
    bar = BARS[storage]
    print(f"pack256: {case.shape}, {len(case.solids)} spheres, {storage}", flush=True)
    gpu = lbm.Lattice(case.lattice, case.collision, storage, case.shape, case.tau, g=case.g,
                      max_solids=len(case.solids))
    gpu.set_solids(case.solids, case.method)
    orc = Oracle(case.lattice, case.collision, case.shape, case.tau, g=case.g, form="h",
                 threads=min(16, os.cpu_count() or 1))
    orc.set_solids(case.solids, case.method)
    Lg, Lo = gpu.links(), orc.links()
    assert len(Lg["cell"]) == len(Lo["cell"]) > 250000
    for k in ("cell", "dir", "sid"):
        assert np.array_equal(Lg[k], Lo[k]), k
    assert np.array_equal(Lg["q"].view(np.uint64), Lo["q"].view(np.uint64))
    assert (Lo["ff_ok"] == 0).sum() + (Lo["fff_ok"] == 0).sum() > 0  # narrow-gap fallbacks present
    gpu.step(2)
    orc.step(2)
    print("pack256: stepped", flush=True)
    rg, ug, tg = gpu.macros()
    ro, uo, to = orc.macros()
    assert np.array_equal(tg, to)
    fl = tg != 1
    du = np.max(np.abs(ug[:, fl] - uo[:, fl])) / np.max(np.abs(uo[:, fl]))
    drho = np.max(np.abs(rg[fl] - ro[fl]))
    assert du <= bar["u"] and drho <= bar["rho"], (du, drho)
    hg, ho = gpu.history(), orc.history()
    scale = max(np.max(np.abs(ho[-1, :, :3])), np.linalg.norm(case.g) * np.sum(fl))
    assert np.max(np.abs(hg[:, :, :3] - ho[:, :, :3])) / scale <= bar["F"]
    tscale = scale * max(case.shape)
    assert np.max(np.abs(hg[:, :, 3:] - ho[:, :, 3:])) / tscale <= bar["F"]
    gpu.close()


@pytest.mark.timeout(600)
def test_batch512_sampled_members_match_alone(lbm):
    cases = W.moving_sphere_batch(512)
    fps = [lbm.Batch.footprint(c.lattice, c.collision, c.storage, c.shape, c.tau, max_solids=1) for c in cases]
    pool = lbm.lbm_batch_table_bytes(512) + sum((f + 255) // 256 * 256 for f in fps) + (1 << 20)
    b = lbm.Batch("D3Q19", "F32", max_slots=512, pool_bytes=pool)
    members = []
    for c in cases:
        m = b.admit(c.collision, c.storage, c.shape, c.tau, g=c.g, max_solids=1)
        assert m is not None
        m.set_solids(c.solids, c.method)
        members.append(m)
    print(f"batch512: {sum(m.N for m in members)} cells admitted", flush=True)
    steps = 40  # the eager tuning steps (36) and the first graph replays
    b.step(steps)
    b.sync()
    sizes = np.array([m.N for m in members])
    order = np.argsort(sizes, kind="stable")
    picks = sorted({int(order[0]), int(order[-1]), int(order[len(order) // 2])})
    for k in picks:
        c = cases[k]
        ref = lbm.Lattice(c.lattice, c.collision, c.storage, c.shape, c.tau, g=c.g, max_solids=1)
        ref.set_solids(c.solids, c.method)
        ref.step(steps)
        m = members[k]
        assert np.array_equal(m.get_state().view(np.uint8), ref.get_state().view(np.uint8)), k
        assert np.array_equal(m.history().view(np.uint64), ref.history().view(np.uint64)), k
        ref.close()
    b.close()
