"""The algebra the two-level preconditioner rests on, checked on the CPU.

The GPU preconditioner (paper_1610_03484_amd/csrc/mg.hip) assumes
  1. the vertex functions of the order-2 hierarchic basis are the P1 hats, so
     the vertex-vertex block of the hierarchic stiffness matrix is the P1
     stiffness matrix of the same tets;
  2. the Kuhn split of an n-grid refines the Kuhn split of the n/2-grid: every
     vertex of the fine grid is a coarse vertex or the midpoint of a coarse
     Kuhn edge (directions e1, e2, e3, e1+e2, e1+e3, e2+e3, e1+e2+e3), so with
     the prolongation P (weight 1 at coarse vertices, 1/2 from the two ends of
     the edge otherwise) the Galerkin product P^T A_fine P is exactly the P1
     stiffness of the coarse grid;
  3. the coarse stencil is the 15-point Kuhn neighbourhood.
Each is checked here against matrices assembled by the oracle's own finite
element code (a wrong edge direction, weight or basis relation fails them).
"""
import numpy as np
import scipy.sparse as sp

from oracle import fem, mesh

KUHN_DIRS = [(1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 0), (1, 0, 1), (0, 1, 1), (1, 1, 1)]


def _spd(rng, count):
    a = rng.standard_normal((count, 3, 3))
    return np.einsum("eij,ekj->eik", a, a) + 0.5 * np.eye(3)


def _p1_laplace(n, kappa_of_tet):
    coords, tets = mesh.kuhn_mesh(n)
    disc = fem.Discretisation(coords, tets, 1)
    K = disc.stiffness_scalar(kappa_of_tet(coords, tets)).tocsr()
    # oracle node numbering -> lattice vertex (i, j, k)
    lat = np.rint(disc.nodes * n).astype(int)
    return K, lat


def _prolongation(nc, lat_f, lat_c):
    key_c = {tuple(v): i for i, v in enumerate(lat_c)}
    rows, cols, vals = [], [], []
    for f, v in enumerate(lat_f):
        o = v % 2
        if not o.any():
            rows.append(f); cols.append(key_c[tuple(v // 2)]); vals.append(1.0)
        else:
            assert tuple(o) in KUHN_DIRS
            for s in (-1, 1):
                rows.append(f); cols.append(key_c[tuple((v + s * o) // 2)]); vals.append(0.5)
    return sp.csr_matrix((vals, (rows, cols)), shape=(len(lat_f), len(lat_c)))


def test_galerkin_product_is_the_coarse_p1_matrix():
    rng = np.random.default_rng(3)
    nc = 3
    # one SPD conductivity per coarse tet, inherited by the fine tets inside it
    kap_c = _spd(rng, 6 * nc ** 3)
    coords_c, tets_c = mesh.kuhn_mesh(nc)

    def coarse_tet_of(points):
        x = coords_c[tets_c]                                    # [T, 4, 3]
        M = np.ones((len(tets_c), 4, 4))
        M[:, :3, :] = np.transpose(x, (0, 2, 1))
        Minv = np.linalg.inv(M)
        out = np.empty(len(points), dtype=int)
        for q, y in enumerate(points):
            lam = Minv @ np.append(y, 1.0)
            inside = np.all(lam >= -1e-12, axis=1)
            assert inside.sum() >= 1
            out[q] = int(np.argmax(inside))
        return out

    Kf, lat_f = _p1_laplace(2 * nc, lambda c, t: kap_c[coarse_tet_of(c[t].mean(axis=1))])
    Kc, lat_c = _p1_laplace(nc, lambda c, t: kap_c)
    P = _prolongation(nc, lat_f, lat_c)
    G = (P.T @ Kf @ P).toarray()
    assert np.abs(G - Kc.toarray()).max() <= 1e-12 * np.abs(Kc.toarray()).max()


def test_coarse_stencil_is_the_kuhn_neighbourhood():
    Kc, lat = _p1_laplace(4, lambda c, t: np.broadcast_to(np.diag([1.0, 2.0, 3.0]), (len(t), 3, 3)))
    offs = {(0, 0, 0)} | {d for d in KUHN_DIRS} | {tuple(-x for x in d) for d in KUHN_DIRS}
    Kc = Kc.tocoo()
    for i, j, v in zip(Kc.row, Kc.col, Kc.data):
        if abs(v) > 0.0:
            assert tuple(lat[j] - lat[i]) in offs


def test_hierarchic_vertex_block_is_the_p1_matrix():
    """Vertex functions lam_a = Lagrange vertex function + 1/2 (adjacent edge functions)."""
    rng = np.random.default_rng(5)
    n = 2
    coords, tets = mesh.kuhn_mesh(n)
    kap = _spd(rng, len(tets))
    d2 = fem.Discretisation(coords, tets, 2)
    d1 = fem.Discretisation(coords, tets, 1)
    K2 = d2.stiffness_scalar(kap).toarray()
    K1 = d1.stiffness_scalar(kap).toarray()
    lat2 = np.rint(d2.nodes * 2 * n).astype(int)
    lat1 = np.rint(d1.nodes * n).astype(int)
    key2 = {tuple(v): i for i, v in enumerate(lat2)}
    # hierarchic vertex function of vertex v, in the Lagrange P2 basis
    T = np.zeros((len(lat2), len(lat1)))
    for j, v in enumerate(lat1):
        T[key2[tuple(2 * v)], j] = 1.0
        for d in KUHN_DIRS:
            for s in (-1, 1):
                mid = tuple(2 * v + s * np.array(d))
                if mid in key2:
                    T[key2[mid], j] = 0.5
    assert np.abs(T.T @ K2 @ T - K1).max() <= 1e-12 * np.abs(K1).max()
