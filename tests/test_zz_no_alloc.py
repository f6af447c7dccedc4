"""The allocation-free wall-shear entry point (fvib_loss_wall_shear_noalloc)
against fvib_loss_wall_shear, through the C ABI: same J and same adjoint,
bit for bit, on two calls in a row on one device, the second on a smaller
grid (fewer partial sums than the first left in the shared scratch)."""
import numpy as np
import pytest
import torch

import fvib_workloads as W
from gpu_util import make_grid, need_gpu

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_noalloc_wall_shear_matches_allocating_entry(precision):
    need_gpu()
    from oracle import Grid as OGrid
    from oracle.step import wall_shear as oracle_wall_shear
    # wall planes of 64 x 48 (12 blocks of partial sums) then 24 x 20 (2)
    cases = [W.channel(nx=64, ny=16, nz=48, steps=1), W.channel(nx=24, ny=12, nz=20, steps=1)]
    for n, w in enumerate(cases):
        g = make_grid(w, precision=precision)
        rng = np.random.default_rng(100 + n)
        shape = g.layouts[0][0]
        u0 = torch.tensor(rng.standard_normal(shape), dtype=g.dtype, device=g.device)
        seed = torch.tensor(rng.standard_normal(shape), dtype=g.dtype, device=g.device)
        ub_ref = seed.clone()
        ub_new = seed.clone()
        J_ref = g.loss_wall_shear(u0, ub_ref)
        J_new = torch.full((1,), float("nan"), dtype=torch.float64, device=g.device)
        g.loss_wall_shear_noalloc(u0, J_new, ub_new)
        torch.cuda.synchronize()
        assert float(J_new[0]) == float(J_ref[0]), (n, float(J_new[0]), float(J_ref[0]))
        assert torch.equal(ub_new, ub_ref), n
        # and the value itself: the oracle's loss on the same field
        og = OGrid(w)
        Jo = float(oracle_wall_shear(og, [torch.tensor(u0.double().cpu().numpy())]))
        tol = 1e-12 if precision == "fp64" else 1e-6
        assert abs(float(J_new[0]) - Jo) <= tol * max(1.0, abs(Jo)), (n, float(J_new[0]), Jo)
        print(f"{precision} grid {n}: J {float(J_new[0]):.12e} (oracle {Jo:.12e})")
