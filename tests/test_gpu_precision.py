"""Reduced-precision storage against FP64 storage on the same GPU (whose FP64 path matches the FP64
oracle to 1e-12, tests/test_gpu_parity.py).

Bars here, after 600 steps of reduced versions of the workloads (per-sphere relative drag error):
FP32 deviation storage 1e-4, FP16 deviation storage 2e-2 (round to nearest and stochastic rounding);
lattices stepped as an FP32 batch against the same lattices stepped alone with FP64 storage: force
error 1e-5 of the largest FP64 force.
The errors grow with the length of the run; bench.py reports them on the full workloads (256^3 with
64 spheres and 8 moving-sphere lattices, 10000 steps): FP32 6.4e-5; FP16 to nearest 4.3e-2 (a
systematic lag of the mean flow: per-step increments below half an FP16 unit are rounded away); FP16
with stochastic rounding 3.2e-4; batched FP32 vs plain FP64 1.8e-4; against stated full-length
tolerances of 2e-4, 1e-1, 2e-3 and 5e-4.
"""
import numpy as np
import pytest

from paper_1906_05445_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = {"F32": 1e-4, "F16": 2e-2, "F16_SR": 2e-2}


@pytest.fixture(scope="module")
def lbm():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1906_05445_amd import lbm as L

    return L


def _drag(lbm, case, storage, steps):
    g = lbm.Lattice(case.lattice, case.collision, storage, case.shape, case.tau, g=case.g,
                    max_solids=len(case.solids))
    g.set_solids(case.solids, case.method)
    g.step(steps)
    d = g.force_torque()[:, 0].copy()
    g.close()
    return d


def test_reduced_storage_drag_against_fp64(lbm):
    case = W.sphere_pack(n=96, count=8, R=8.0, seed=3)
    ref = _drag(lbm, case, "F64", 600)
    for storage, tol in TOL.items():
        d = _drag(lbm, case, storage, 600)
        rel = np.abs(d - ref) / np.abs(ref)
        assert rel.max() <= tol, f"{storage}: max per-sphere drag error {rel.max():.3e} > {tol}"


def test_fp32_batch_against_plain_fp64(lbm):
    cases = W.moving_sphere_batch(4, seed=11, edge=(32, 48))
    fps = [lbm.Batch.footprint(c.lattice, c.collision, "F32", c.shape, c.tau, max_solids=1) for c in cases]
    b = lbm.Batch("D3Q19", "F32", max_slots=4, pool_bytes=lbm.lbm_batch_table_bytes(4) + sum(fps) + (1 << 24))
    members = []
    for c in cases:
        m = b.admit(c.collision, "F32", c.shape, c.tau, g=c.g, max_solids=1)
        m.set_solids(c.solids, c.method)
        members.append(m)
    b.step(600)
    for c, m in zip(cases, members):
        ref = lbm.Lattice(c.lattice, c.collision, "F64", c.shape, c.tau, g=c.g, max_solids=1)
        ref.set_solids(c.solids, c.method)
        ref.step(600)
        f64 = ref.history()[:, 0, :3]
        f32 = m.history()[:, 0, :3]
        err = np.abs(f32 - f64).max() / np.abs(f64).max()
        ref.close()
        assert err <= 1e-5, f"{c.name}: batched FP32 force error {err:.3e}"
    b.close()
