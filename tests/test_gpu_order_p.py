"""GPU parity at orders 3 and 4 (hierarchic tables, matrix-core element operator)
against the CPU FP64 oracle (Lagrange P3/P4, exact integration).

Sizes: n = 2 and 3 cells per side (up to 13^3 lattice points at p = 4); the
operator gives each workgroup one cell (its six tets), so these sizes exercise
lattice wrap-around and boundary cells on every side.  Tolerances as at order 2: FP64 path 1e-9, FP32
operator with FP64 refinement 1e-6 (relative Frobenius error of each block).
"""
import numpy as np
import pytest

import chom_inputs as ci
from oracle import fem as ofem, mesh as omesh

from gpu_util import banner, rel, require_gpu, upper21, upper6

pytestmark = pytest.mark.gpu

BC_ID = {"dirichlet": ofem.BC_DIRICHLET, "periodic": ofem.BC_PERIODIC, "neumann": ofem.BC_NEUMANN}
_CACHE = {}


def oracle_result(n, p, bc, params, key):
    k = (n, p, bc, key)
    if k not in _CACHE:
        c, t, ph, ax = omesh.plain_weave(n)
        _CACHE[k] = ofem.homogenise(c, t, ph, ax, p, BC_ID[bc], ci.BASE_MATERIALS, params)
    return _CACHE[k]


def gpu_rve(n, bc, p, **opts):
    from paper_1610_03484_amd import RVE, generate_plain_weave
    coords, tets, phase, axis = generate_plain_weave(n, device="cuda")
    return RVE(coords, tets, phase, axis, ci.BASE_MATERIALS, bc=bc, order=p, **opts)


def errors(C, K, D, ref):
    return (rel(C, upper21(ref["C"])), rel(K, upper6(ref["K"])), rel(D, upper6(ref["D"])))


@pytest.mark.parametrize("p", [3, 4])
@pytest.mark.parametrize("bc", ["dirichlet", "periodic", "neumann"])
@pytest.mark.parametrize("n", [2, 3])
def test_order_p_fp64_matches_oracle(p, bc, n):
    require_gpu()
    params = ci.draw_params(13, 1)[0]
    banner(f"order {p} fp64 n={n} bc={bc}")
    rve = gpu_rve(n, bc, p, precision="fp64", rtol=1e-13, max_iter=20000)
    C, K, D, rep = rve.homogenise(params[None])
    ref = oracle_result(n, p, bc, params, "deg13")
    eC, eK, eD = errors(C[0], K[0], D[0], ref)
    banner(f"  errors C={eC:.2e} K={eK:.2e} D={eD:.2e} iters={rep[0]['iters']}")
    assert rep[0]["status"] == 0
    assert max(eC, eK, eD) < 1e-9


@pytest.mark.parametrize("p", [3, 4])
def test_order_p_fp32_refined_matches_oracle(p):
    require_gpu()
    params = ci.draw_params(14, 1)[0]
    banner(f"order {p} fp32 refined n=3 periodic")
    rve = gpu_rve(3, "periodic", p, precision="fp32_refined", rtol=1e-10, max_iter=20000)
    C, K, D, rep = rve.homogenise(params[None])
    ref = oracle_result(3, p, "periodic", params, "deg14")
    eC, eK, eD = errors(C[0], K[0], D[0], ref)
    banner(f"  errors C={eC:.2e} K={eK:.2e} D={eD:.2e} refine={rep[0]['refine_steps']}")
    assert rep[0]["status"] == 0
    assert max(eC, eK, eD) < 1e-6


def test_order_p_batch_of_mixed_sizes_equals_single_solves():
    require_gpu()
    from paper_1610_03484_amd import Batch
    banner("order 3 batch: n = 2, 3 mixed, periodic and Dirichlet")
    rves = [gpu_rve(2, "periodic", 3, precision="fp64", rtol=1e-13),
            gpu_rve(3, "dirichlet", 3, precision="fp64", rtol=1e-13),
            gpu_rve(3, "periodic", 3, precision="fp64", rtol=1e-13)]
    params = ci.draw_params(15, 3)
    C, K, D, rep = Batch(rves).homogenise(params)
    for i, r in enumerate(rves):
        c1, k1, d1, _ = r.homogenise(params[i:i + 1])
        # independent solves stopped at rtol = 1e-13: agree to well below 1e-10
        assert rel(C[i], c1[0]) < 1e-10 and rel(K[i], k1[0]) < 1e-10 and rel(D[i], d1[0]) < 1e-10


def test_batch_rejects_mixed_orders():
    require_gpu()
    from paper_1610_03484_amd import Batch
    from paper_1610_03484_amd import _lib as L
    with pytest.raises(L.ChomError):
        Batch([gpu_rve(2, "periodic", 3), gpu_rve(2, "periodic", 2)])


def _distorted_weave(n, seed, amount=0.2):
    """Plain-weave tags on a Kuhn mesh whose interior vertices are moved by up to amount * h."""
    c, t, ph, ax = omesh.plain_weave(n)
    u = ci.uniform_block(seed, 0, c.size).reshape(c.shape)
    ijk = np.rint(c * n).astype(int)
    interior = np.all((ijk > 0) & (ijk < n), axis=1)
    c = c.copy()
    c[interior] += amount / n * (2.0 * u[interior] - 1.0)
    return c, t, ph, ax


@pytest.mark.parametrize("p", [2, 3])
@pytest.mark.parametrize("bc", ["dirichlet", "periodic", "neumann"])
def test_distorted_mesh_matches_oracle(p, bc):
    """Per-tet geometry path (moved interior vertices) against the oracle on the same mesh."""
    require_gpu()
    from paper_1610_03484_amd import RVE
    n = 3
    c, t, ph, ax = _distorted_weave(n, 21)
    params = ci.draw_params(16, 1)[0]
    banner(f"distorted mesh order {p} bc={bc}")
    rve = RVE(c, t, ph, ax, ci.BASE_MATERIALS, bc=bc, order=p, precision="fp64", rtol=1e-13, max_iter=20000)
    C, K, D, rep = rve.homogenise(params[None])
    ref = ofem.homogenise(c, t, ph, ax, p, BC_ID[bc], ci.BASE_MATERIALS, params)
    eC, eK, eD = errors(C[0], K[0], D[0], ref)
    banner(f"  errors C={eC:.2e} K={eK:.2e} D={eD:.2e}")
    assert rep[0]["status"] == 0
    assert max(eC, eK, eD) < 1e-9


@pytest.mark.parametrize("p", [3, 4])
@pytest.mark.parametrize("bc", ["dirichlet", "periodic", "neumann"])
def test_homogeneous_rve_returns_its_material_at_order_p(bc, p):
    """Every tet matrix: the exact fluctuation is zero at any order and for every
    condition, so the homogenised tensors are the matrix's own."""
    require_gpu()
    from oracle import materials as M
    from paper_1610_03484_amd import RVE, generate_plain_weave
    coords, tets, phase, axis = generate_plain_weave(4, device="cuda")
    rec = ci.draw_params(14, 1)
    r = RVE(coords, tets, phase * 0, axis, ci.BASE_MATERIALS, bc=bc, order=p, precision="fp32_refined",
            rtol=1e-10, max_iter=20000)
    C, K, D, rep = r.homogenise(rec)
    r.close()
    m, _, _ = M.phase_materials(ci.BASE_MATERIALS, rec[0])
    Cm = M.isotropic_stiffness(m["E"], m["nu"])
    e = (np.abs(C[0] - upper21(Cm)).max() / np.abs(Cm).max(),
         np.abs(K[0] - m["k"] * np.array([1, 1, 1, 0, 0, 0])).max() / m["k"],
         np.abs(D[0] - m["D"] * np.array([1, 1, 1, 0, 0, 0])).max() / m["D"])
    banner(f"homogeneous 4^3 order {p} {bc}: errors {e}, status {rep[0]['status']}")
    assert rep[0]["status"] == 0
    assert max(e) <= 1e-9


@pytest.mark.parametrize("p", [3, 4])
def test_permuted_axes_give_the_permuted_tensors_at_order_p(p):
    """Orders 3 and 4 (element factors per tet type, basis tables, matrix-core
    products): renamed axes (x, y, z) -> (y, z, x) give the permuted tensors."""
    require_gpu()
    import torch
    from gpu_util import full3, full6, permuted_lattice, rotate_voigt
    from paper_1610_03484_amd import RVE, generate_plain_weave
    n = 4
    coords, tets, phase, axis = (x.cpu().numpy() for x in generate_plain_weave(n, device="cuda"))
    perm = [1, 2, 0]
    Q = np.eye(3)[perm]
    rec = ci.draw_params(20, 1)
    res = []
    for mesh in ((coords, tets, phase, axis), permuted_lattice(coords, tets, phase, axis, n, perm)):
        dev = [torch.as_tensor(np.ascontiguousarray(x), device="cuda") for x in mesh]
        r = RVE(*dev, ci.BASE_MATERIALS, bc="periodic", order=p, precision="fp32_refined", rtol=1e-9,
                max_iter=20000)
        res.append(r.homogenise(rec))
        r.close()
    (C, K, D, _), (Cp, Kp, Dp, _) = res
    exp_c = rotate_voigt(full6(C[0]), Q)
    err = np.abs(full6(Cp[0]) - exp_c).max() / np.abs(exp_c).max()
    for got, ref in ((Kp[0], K[0]), (Dp[0], D[0])):
        e3 = Q @ full3(ref) @ Q.T
        err = max(err, np.abs(full3(got) - e3).max() / np.abs(e3).max())
    banner(f"permuted axes 4^3 order {p}: max rel diff {err:.1e}")
    assert err <= 1e-7


@pytest.mark.parametrize("p", [3, 4])
def test_scaled_and_shifted_box_at_order_p(p):
    """Element factors and basis tables see the tet sizes: the weave on
    [lo, lo + 2.5] gives the tensors of the unit box at orders 3 and 4."""
    require_gpu()
    import torch
    from paper_1610_03484_amd import RVE, generate_plain_weave
    coords, tets, phase, axis = generate_plain_weave(4, device="cuda")
    lo = torch.tensor([1.0, -2.0, 0.5], dtype=coords.dtype, device=coords.device)
    rec = ci.draw_params(26, 1)
    out = []
    for c, a, b in ((coords, (0.0, 0.0, 0.0), (1.0, 1.0, 1.0)),
                    ((lo + 2.5 * coords).contiguous(), tuple(lo.tolist()), tuple((lo + 2.5).tolist()))):
        r = RVE(c, tets, phase, axis, ci.BASE_MATERIALS, bc="neumann", order=p, lo=a, hi=b,
                precision="fp64", rtol=1e-11, max_iter=20000)
        C, K, D, rep = r.homogenise(rec)
        r.close()
        assert rep[0]["status"] == 0
        out.append(np.concatenate([C, K, D], axis=1))
    e = float(np.abs(out[0] - out[1]).max() / np.abs(out[0]).max())
    banner(f"scaled and shifted box, 4^3 order {p} neumann: max rel diff {e:.1e}")
    assert e <= 1e-9
