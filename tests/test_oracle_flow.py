"""Pins of the potential-flow yarn directions of the oracle (paper Sec. 6).

* A yarn that is a straight prism of whole cells along x has the exact
  potential phi = x, which P1 elements reproduce on any mesh of the prism, so
  every direction is e_x to rounding, also with the prism's inner vertices
  moved (a wrong gradient, a transposed Jacobian or a swapped inlet fails this).
* Discrete maximum principle (Kuhn tetrahedra have no obtuse dihedral angle,
  so the P1 Laplacian is an M-matrix): 0 <= phi <= 1.
* Conservation: the flux entering at the inlet equals the flux leaving at the
  outlet (the reactions of the Dirichlet rows sum to zero).
* On the plain weave the directions approach the centreline tangent as the
  mesh is refined (the staircase yarn boundary is the only difference).
"""
import numpy as np
import pytest

import chom_inputs as ci
from oracle import flow, mesh


def _prism_phase(n, j0=2, j1=4, k0=2, k1=4):
    """Phase 1 on the six tets of every cell with j in [j0, j1), k in [k0, k1)."""
    phase = np.zeros(6 * n ** 3, dtype=np.int8)
    for k in range(k0, k1):
        for j in range(j0, j1):
            for i in range(n):
                cell = i + n * (j + n * k)
                phase[6 * cell:6 * cell + 6] = 1
    return phase


@pytest.mark.parametrize("distort", [False, True])
def test_straight_prism_gives_the_axis_exactly(distort):
    n = 6
    coords, tets = mesh.kuhn_mesh(n)
    phase = _prism_phase(n)
    if distort:
        # move only vertices strictly inside the prism (its faces stay planar)
        ijk = np.stack(np.meshgrid(np.arange(n + 1), np.arange(n + 1), np.arange(n + 1), indexing="ij"),
                       axis=-1).reshape(-1, 3)[:, ::-1]
        inner = (ijk[:, 0] > 0) & (ijk[:, 0] < n) & (ijk[:, 1] == 3) & (ijk[:, 2] == 3)
        u = ci.uniform_block(5, 0, 3 * len(coords)).reshape(-1, 3)
        coords = coords.copy()
        coords[inner] += 0.2 / n * (2 * u[inner] - 1)
    d = flow.yarn_directions(coords, tets, phase, [0])
    sel = phase == 1
    np.testing.assert_allclose(d[sel], np.tile([1.0, 0.0, 0.0], (sel.sum(), 1)), atol=1e-12)
    assert np.all(d[~sel] == 0.0)


def test_maximum_principle_and_flux_balance():
    coords, tets, phase, _ = mesh.plain_weave(8)
    for j, axis in enumerate([0, 0, 1, 1]):
        sel = np.flatnonzero(phase == j + 1)
        verts, phi, inlet, outlet, K = flow.yarn_potential(coords, tets, sel, axis, (0, 0, 0), (1, 1, 1))
        assert phi.min() >= -1e-12 and phi.max() <= 1 + 1e-12
        react = K @ phi
        fin, fout = react[inlet].sum(), react[outlet].sum()
        assert fout > 0 and abs(fin + fout) <= 1e-10 * fout
        free = np.setdiff1d(np.arange(len(verts)), np.r_[inlet, outlet])
        assert np.abs(react[free]).max() <= 1e-10 * fout


def test_directions_approach_the_centreline_tangent():
    means = []
    for n in (8, 12, 24):
        c, t, ph, ax = mesh.plain_weave(n)
        d = flow.yarn_directions(c, t, ph, [0, 0, 1, 1])
        y = ph > 0
        cosang = np.clip(np.abs((d[y] * ax[y]).sum(axis=1)), -1.0, 1.0)
        means.append(float(np.degrees(np.arccos(cosang)).mean()))
        assert np.allclose(np.linalg.norm(d[y], axis=1), 1.0)
    assert means[0] > means[1] > means[2] and means[2] < 10.0, means
