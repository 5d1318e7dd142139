"""Potential-flow yarn directions on the GPU (chom_yarn_directions) against the oracle.

Both sides solve the same P1 Laplace problem per yarn (paper Sec. 6): the GPU
with Jacobi-preconditioned CG in FP64 to a relative residual of 1e-13, the
oracle with a sparse direct solve, so the directions agree to about the CG
tolerance times the conditioning.  Cases: the plain weave at n = 4, 8, 12 and
the 24^3 benchmark lattice; n = 3, where some yarn tets form a piece that
touches only one end face (zero gradient: the oracle's direction is undefined,
the library must refuse the mesh);
a straight prism (exact answer e_x) on a distorted lattice; and the directions
fed to the RVE solve, against the oracle homogenising with its own directions.
"""
import numpy as np
import pytest

import chom_inputs as ci
from oracle import fem as ofem, flow as oflow, mesh as omesh

from gpu_util import banner, require_gpu, result_errors

pytestmark = pytest.mark.gpu
AXES = [0, 0, 1, 1]


@pytest.mark.parametrize("n", [4, 8, 12, 24])
def test_directions_match_oracle(n):
    torch = require_gpu()
    from paper_1610_03484_amd import generate_plain_weave, yarn_directions
    banner(f"potential-flow directions, plain weave n={n}")
    coords, tets, phase, _ = generate_plain_weave(n, device="cuda")
    d_dev = yarn_directions(coords, tets, phase, AXES, rtol=1e-13).cpu().numpy()
    c, t, ph = coords.cpu().numpy(), tets.cpu().numpy(), phase.cpu().numpy()
    d_host = yarn_directions(c, t, ph, AXES, rtol=1e-13)
    ref = oflow.yarn_directions(c, t, ph, AXES)
    err = float(np.abs(d_dev - ref).max())
    banner(f"  max |direction difference| {err:.2e} over {int((ph > 0).sum())} yarn tets")
    assert err <= 1e-8
    assert np.array_equal(d_dev, d_host)
    assert np.all(d_dev[ph == 0] == 0.0)


def test_yarn_piece_without_a_gradient_is_refused():
    require_gpu()
    import warnings
    from paper_1610_03484_amd import generate_plain_weave, yarn_directions
    from paper_1610_03484_amd import _lib as L
    banner("potential-flow directions, n=3: yarn pieces at one end face only")
    coords, tets, phase, _ = generate_plain_weave(3, device="cuda")
    c, t, ph = coords.cpu().numpy(), tets.cpu().numpy(), phase.cpu().numpy()
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        ref = oflow.yarn_directions(c, t, ph, AXES)
    assert np.isnan(ref[ph > 0]).any()
    with pytest.raises(L.ChomError) as ei:
        yarn_directions(coords, tets, phase, AXES, rtol=1e-13)
    assert ei.value.status == L.CHOM_EMESH


def test_straight_prism_on_a_distorted_lattice():
    require_gpu()
    from paper_1610_03484_amd import yarn_directions
    n = 6
    coords, tets = omesh.kuhn_mesh(n)
    phase = np.zeros(6 * n ** 3, dtype=np.int8)
    for k in range(2, 4):
        for j in range(2, 4):
            for i in range(n):
                cell = i + n * (j + n * k)
                phase[6 * cell:6 * cell + 6] = 1
    ijk = np.stack(np.meshgrid(np.arange(n + 1), np.arange(n + 1), np.arange(n + 1), indexing="ij"),
                   axis=-1).reshape(-1, 3)[:, ::-1]
    inner = (ijk[:, 0] > 0) & (ijk[:, 0] < n) & (ijk[:, 1] == 3) & (ijk[:, 2] == 3)
    u = ci.uniform_block(5, 0, 3 * len(coords)).reshape(-1, 3)
    coords = coords.copy()
    coords[inner] += 0.2 / n * (2 * u[inner] - 1)
    banner("potential-flow directions, straight prism, distorted lattice")
    d = yarn_directions(coords, tets.astype(np.int32), phase, [0], rtol=1e-14)
    sel = phase == 1
    err = float(np.abs(d[sel] - np.array([1.0, 0.0, 0.0])).max())
    banner(f"  max |d - e_x| {err:.2e}")
    assert err <= 1e-10


def test_potential_flow_directions_drive_the_rve_solve():
    require_gpu()
    from paper_1610_03484_amd import RVE, generate_plain_weave, yarn_directions
    n = 6
    params = ci.draw_params(31, 1)
    banner(f"RVE solve with potential-flow directions, {n}^3 periodic FP64")
    coords, tets, phase, _ = generate_plain_weave(n, device="cuda")
    axis = yarn_directions(coords, tets, phase, AXES, rtol=1e-13)
    rve = RVE(coords, tets, phase, axis, ci.BASE_MATERIALS, bc="periodic", precision="fp64")
    C, K, D, rep = rve.homogenise(params)
    rve.close()
    c, t, ph = coords.cpu().numpy(), tets.cpu().numpy(), phase.cpu().numpy()
    ax = oflow.yarn_directions(c, t, ph, AXES)
    o = ofem.homogenise(c, t, ph, ax, 2, ofem.BC_PERIODIC, ci.BASE_MATERIALS, params[0])
    iu = np.triu_indices(6)
    sym3 = [(0, 0), (1, 1), (2, 2), (0, 1), (1, 2), (0, 2)]
    e = result_errors(C[0], K[0], D[0], o["C"][iu], [o["K"][a, b] for a, b in sym3],
                      [o["D"][a, b] for a, b in sym3])
    banner(f"  errors against the oracle {e}")
    assert rep[0]["status"] == 0
    assert max(e) <= 1e-9


def test_directions_ignore_the_box_size_and_position():
    """The potential of each yarn is fixed by its end faces, so scaling and
    shifting the box leaves every unit direction unchanged."""
    torch = require_gpu()
    from paper_1610_03484_amd import generate_plain_weave, yarn_directions
    coords, tets, phase, _ = generate_plain_weave(8, device="cuda")
    a = yarn_directions(coords, tets, phase, AXES, rtol=1e-13).cpu().numpy()
    lo = torch.tensor([2.0, -1.0, 0.5], dtype=coords.dtype, device=coords.device)
    b = yarn_directions((lo + 3.0 * coords).contiguous(), tets, phase, AXES, rtol=1e-13,
                        lo=tuple(lo.tolist()), hi=tuple((lo + 3.0).tolist())).cpu().numpy()
    err = float(np.abs(a - b).max())
    banner(f"directions on a scaled and shifted box: max difference {err:.1e}")
    assert err <= 1e-9
