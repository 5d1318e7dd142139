"""Pins of the unstructured box meshes and of the oracle's RVE solve on them (CPU).

* The mesh is conforming: every interior triangle belongs to exactly two tets,
  every boundary triangle lies in a box face, the tets fill the box, and the
  triangles of opposite faces coincide after translation (periodic matching).
* The connectivity is not a lattice pattern: vertex valences vary.
* A homogeneous RVE returns its own material for every BC (zero fluctuation),
  on this mesh as on the lattice.
* Loewner order of the estimates on a heterogeneous unstructured weave:
  Voigt >= Dirichlet >= periodic >= Reuss.
"""
from collections import Counter

import numpy as np
import pytest

import chom_inputs as ci
from oracle import fem, materials as M, mesh


def _faces(tets):
    f = Counter()
    for t in tets:
        for q in range(4):
            f[tuple(sorted(int(v) for v in np.delete(t, q)))] += 1
    return f


@pytest.mark.parametrize("nc,seed", [(2, 0), (3, 1), (4, 2)])
def test_unstructured_box_is_conforming_and_periodic(nc, seed):
    coords, tets = ci.unstructured_box(nc, seed=seed)
    assert len(tets) == 12 * nc ** 3 and len(coords) == (nc + 1) ** 3 + nc ** 3
    vol = np.linalg.det(coords[tets][:, 1:] - coords[tets][:, :1]) / 6.0
    assert vol.min() > 0 and abs(vol.sum() - 1.0) < 1e-13
    f = _faces(tets)
    assert set(f.values()) <= {1, 2}
    bnd = [k for k, v in f.items() if v == 1]
    assert len(bnd) == 6 * 2 * nc * nc
    for tri in bnd:
        x = coords[list(tri)]
        assert any(np.allclose(x[:, d], 0.0) or np.allclose(x[:, d], 1.0) for d in range(3))
    # opposite faces: the same triangles after moving hi to lo
    key = lambda x: tuple(np.round(x, 12))
    for d in range(3):
        lo_tris, hi_tris = set(), set()
        for tri in bnd:
            x = coords[list(tri)].copy()
            if np.allclose(x[:, d], 0.0):
                lo_tris.add(frozenset(key(p) for p in x))
            elif np.allclose(x[:, d], 1.0):
                x[:, d] = 0.0
                hi_tris.add(frozenset(key(p) for p in x))
        assert lo_tris == hi_tris and len(lo_tris) == 2 * nc * nc
    # irregular connectivity: interior grid vertices do not all have the same valence
    val = Counter()
    for a, b in {tuple(sorted((int(t[i]), int(t[j])))) for t in tets for i in range(4) for j in range(i + 1, 4)}:
        val[a] += 1
        val[b] += 1
    n1 = nc + 1
    inner = [i + n1 * (j + n1 * k) for i in range(1, nc) for j in range(1, nc) for k in range(1, nc)]
    if len(inner) > 3:
        assert len({val[v] for v in inner}) > 1


@pytest.mark.parametrize("bc", [fem.BC_DIRICHLET, fem.BC_PERIODIC])
def test_homogeneous_unstructured_rve_returns_its_material(bc):
    coords, tets = ci.unstructured_box(2, seed=3)
    d = fem.Discretisation(coords, tets, 2)
    Cl = M.transiso_stiffness_local(55.0, 12.0, 4.5, 0.28, 0.4)
    C = M.rotate_stiffness(Cl, np.array([1.0, 0.2, 0.3]))
    r = fem.solve_rve(d, np.repeat(C[None], len(tets), axis=0), bc, 3)
    assert np.linalg.norm(r["hom"] - C) <= 1e-11 * np.linalg.norm(C)
    k = M.transverse_tensor(0.8, 0.3, [0.1, 1.0, -0.4])
    r = fem.solve_rve(d, np.repeat(k[None], len(tets), axis=0), bc, 1)
    assert np.linalg.norm(r["hom"] - k) <= 1e-11 * np.linalg.norm(k)


def test_loewner_order_on_an_unstructured_weave():
    coords, tets = ci.unstructured_box(3, seed=4)
    c = mesh.centroids(coords, tets)
    phase, axis = mesh.yarn_test(c[:, 0], c[:, 1], c[:, 2])
    assert 0 < (phase > 0).sum() < len(tets)
    d = fem.Discretisation(coords, tets, 2)
    m, y, _ = M.phase_materials(ci.BASE_MATERIALS, ci.draw_factors_only(2, 1)[0])
    Ce, Ke, De = M.element_tensors(phase, axis, m, y)
    for tens, nc_ in ((Ce, 3), (Ke, 1)):
        up, low = fem.voigt_reuss(d, tens)
        dh = fem.solve_rve(d, tens, fem.BC_DIRICHLET, nc_)["hom"]
        ph = fem.solve_rve(d, tens, fem.BC_PERIODIC, nc_)["hom"]
        s = np.linalg.norm(up)
        for a, b in ((up, dh), (dh, ph), (ph, low)):
            assert np.linalg.eigvalsh(0.5 * (a - b + (a - b).T)).min() > -1e-11 * s
