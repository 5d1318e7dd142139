"""Homogenised matrices from a loosely converged solve (GPU, through the C ABI).

For the exact discrete fluctuation the volume-averaged stress (flux) equals the
energy form (1/V) (x_i + u_i)^T K (x_k + u_k); for an iterate u = u* + e the
plain average is off by a term linear in e, the energy form by e_i^T K e_k
only.  The library reports the energy form (the average minus (1/V) u_i . r_k
with the final residual r_k), so a solve stopped at rtol = 1e-4 already meets
the 1e-6 target of the FP32-refined form (the hardest item here, 336 CG
steps, is at ~9e-7), and the reported matrices are symmetric to rounding (the
residual is taken after the solution is projected onto the constraints, so the
uniform-traction case is too).  Reference: the FP64 path solved to rtol = 1e-12.
"""
import numpy as np
import pytest

import chom_inputs as ci
from gpu_util import banner, require_gpu

pytestmark = pytest.mark.gpu


def _run(n, bc, precision, rtol, inner_rtol, params):
    from paper_1610_03484_amd import RVE, generate_plain_weave
    rve = RVE(*generate_plain_weave(n), ci.BASE_MATERIALS, bc=bc, precision=precision, rtol=rtol,
              inner_rtol=inner_rtol, max_iter=50000)
    C, K, D, rep = rve.homogenise(params)
    rve.close()
    return C, K, D, rep


@pytest.mark.parametrize("bc", ["dirichlet", "periodic", "neumann"])
def test_loose_solve_meets_target(bc):
    require_gpu()
    banner(f"energy form, 12^3 {bc}: FP32-refined at rtol 1e-4 vs FP64 at 1e-12")
    params = ci.draw_params(11, 2)
    C, K, D, rep = _run(12, bc, "fp32_refined", 1e-4, 1e-4, params)
    Cr, Kr, Dr, _ = _run(12, bc, "fp64", 1e-12, 1e-12, params)
    for i in range(len(params)):
        errs = [np.linalg.norm(a[i] - b[i]) / np.linalg.norm(b[i]) for a, b in ((C, Cr), (K, Kr), (D, Dr))]
        print(f"[energy] {bc} item {i}: errors C {errs[0]:.2e} K {errs[1]:.2e} D {errs[2]:.2e}; "
              f"iters {max(rep[i]['iters'])}; asym {rep[i]['asym']:.1e}")
        assert max(errs) <= 1e-6
        # the energy form is symmetric up to rounding for every BC: the final
        # residual is that of the projected (constraint-satisfying) solution
        assert rep[i]["asym"] <= 1e-12
        assert rep[i]["spd"] == 1
