"""Two concurrent CG chains per class (GPU, through the C ABI).

Large classes split their problems into two contiguous ranges solved on two
streams from two host threads; each problem's arithmetic is the same as in a
single chain, so the homogenised matrices agree to the solver tolerance.  The
split is forced here on small batches (CHOM_PCG_CHAINS=2), with odd and even
problem counts, both precisions and all BCs.  With the FP32 operator each chain
runs its own refinement loop, FP64 correction solves included (forced here with
CHOM_FORCE_FP64_FALLBACK in both chains at once).
"""
import os

import numpy as np
import pytest

import chom_inputs as ci
from gpu_util import banner, require_gpu

pytestmark = pytest.mark.gpu


def _solve(items, precision, chains, params, force_fp64=False):
    from paper_1610_03484_amd import RVE, Batch, generate_plain_weave
    os.environ["CHOM_PCG_CHAINS"] = str(chains)
    if force_fp64:
        os.environ["CHOM_FORCE_FP64_FALLBACK"] = "1"
    try:
        meshes = {n: generate_plain_weave(n) for n in {n for n, _ in items}}
        rves = [RVE(*meshes[n], ci.BASE_MATERIALS, bc=bc, precision=precision, rtol=1e-11, max_iter=50000)
                for n, bc in items]
        C, K, D, rep = Batch(rves).homogenise(params)
        for r in rves:
            r.close()
    finally:
        os.environ.pop("CHOM_PCG_CHAINS", None)
        os.environ.pop("CHOM_FORCE_FP64_FALLBACK", None)
    return np.concatenate([C, K, D], axis=1), rep


@pytest.mark.parametrize("precision", ["fp64", "fp32_refined"])
@pytest.mark.parametrize("items", [[(8, "dirichlet"), (9, "periodic"), (12, "neumann")],
                                   [(8, "periodic"), (10, "neumann"), (8, "dirichlet"), (12, "periodic")]])
def test_two_chains_match_one(items, precision):
    require_gpu()
    banner(f"CG chains 1 vs 2, {len(items)} items, {precision}")
    params = ci.draw_params(13, len(items))
    a, ra = _solve(items, precision, 1, params)
    b, rb = _solve(items, precision, 2, params)
    e = float(np.abs(a - b).max() / np.abs(a).max())
    print(f"[chains] {len(items)} items {precision}: max rel diff {e:.2e}")
    assert all(r["status"] == 0 for r in ra + rb)
    assert e <= 1e-9


def test_fp64_corrections_in_both_chains():
    """Every problem of both chains goes to an FP64 correction solve from the
    second refinement step on; the results match one chain without corrections."""
    require_gpu()
    items = [(8, "periodic"), (6, "neumann"), (8, "neumann"), (6, "periodic"), (8, "periodic")]
    banner(f"forced FP64 corrections, two chains, {len(items)} items")
    params = ci.draw_params(17, len(items))
    a, ra = _solve(items, "fp32_refined", 1, params)
    b, rb = _solve(items, "fp32_refined", 2, params, force_fp64=True)
    e = float(np.abs(a - b).max() / np.abs(a).max())
    print(f"[chains] forced FP64 corrections: max rel diff {e:.2e}")
    assert all(r["status"] == 0 for r in ra + rb)
    assert all(r["fp64_fallback"][0] == 1 for r in rb)
    assert e <= 1e-9
