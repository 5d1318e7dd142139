"""Pins of the oracle's RVE solve against what the method and the mathematics fix (CPU).

Each test names the fact it checks; none re-types the oracle's own formulas.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import chom_inputs as ci
from oracle import fem, materials as M, mesh

BCS = (fem.BC_DIRICHLET, fem.BC_PERIODIC, fem.BC_NEUMANN)


def _transiso(axis=(1.0, 0.2, 0.3)):
    Cl = M.transiso_stiffness_local(55.0, 12.0, 4.5, 0.28, 0.4)
    return M.rotate_stiffness(Cl, np.asarray(axis, float))


def _uniform(C, T):
    return np.repeat(C[None], T, axis=0)


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _sym_eigmin(A):
    return np.linalg.eigvalsh(0.5 * (A + A.T)).min()


# ------------------------------------------------------------------ exact special cases
@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("p", [1, 2, 3])
def test_homogeneous_rve_returns_its_material(bc, p):
    """A homogeneous RVE has zero fluctuation, so C_bar = C and K_bar = k for every BC and p."""
    coords, tets = mesh.kuhn_mesh(2)
    d = fem.Discretisation(coords, tets, p)
    for C in (M.isotropic_stiffness(3.5, 0.35), _transiso()):
        r = fem.solve_rve(d, _uniform(C, len(tets)), bc, 3)
        assert _rel(r["hom"], C) < 1e-12
        assert _rel(r["hom_vol"], C) < 1e-12
    k = M.transverse_tensor(0.8, 0.3, [0.1, 1.0, -0.4])
    r = fem.solve_rve(d, _uniform(k, len(tets)), bc, 1)
    assert _rel(r["hom"], k) < 1e-12


def test_transiso_shear_order_pinned():
    """Fibre along x: G12 = G13 != G23 fixes the Voigt order [11,22,33,12,23,31]."""
    coords, tets = mesh.kuhn_mesh(2)
    d = fem.Discretisation(coords, tets, 2)
    C = _transiso((1.0, 0.0, 0.0))
    r = fem.solve_rve(d, _uniform(C, len(tets)), fem.BC_DIRICHLET, 3)
    Ch = r["hom"]
    assert np.isclose(Ch[3, 3], 4.5) and np.isclose(Ch[5, 5], 4.5)
    assert np.isclose(Ch[4, 4], 12.0 / (2 * 1.4))


@pytest.mark.parametrize("p", [1, 2, 3, 4])
@pytest.mark.parametrize("bc", BCS)
def test_patch_test_distorted_mesh(p, bc):
    """Distorted interior vertices, homogeneous material: the linear field is exact."""
    n = 3 if p < 4 else 2
    coords, tets = mesh.kuhn_mesh(n)
    u = ci.uniform01(7, np.arange(len(coords))[:, None], np.arange(3)[None, :])
    coords = mesh.distort_interior(coords, n, 0.2, u)
    assert np.all(np.abs(mesh.tet_volumes(coords, tets)) > 0)
    d = fem.Discretisation(coords, tets, p)
    C = _transiso((0.5, -0.3, 1.0))
    r = fem.solve_rve(d, _uniform(C, len(tets)), bc, 3)
    assert _rel(r["hom"], C) < 1e-11
    # total displacement equals the interpolated linear field: zero fluctuation
    X = fem.X_mech(d.nodes)                                  # [N, 3, 6]
    assert np.abs(r["u"].reshape(-1, 3, 6) - X).max() < 1e-11


def _laminate_closed_form(C1, C2, f1):
    """Exact periodic homogenisation of two layers normal to e3 (textbook laminate)."""
    Nn = [2, 4, 5]           # components that may jump across the interface (33, 23, 31)
    Pp = [0, 1, 3]           # in-plane components equal in both layers
    Cbar = np.zeros((6, 6))
    for k in range(6):
        eb = np.zeros(6)
        eb[k] = 1.0
        # unknowns: eps_N in layer 1 and 2 (6), equations: traction continuity + average
        A = np.zeros((6, 6))
        b = np.zeros(6)
        A[:3, :3] = C1[np.ix_(Nn, Nn)]
        A[:3, 3:] = -C2[np.ix_(Nn, Nn)]
        b[:3] = -(C1[np.ix_(Nn, Pp)] - C2[np.ix_(Nn, Pp)]) @ eb[Pp]
        A[3:, :3] = f1 * np.eye(3)
        A[3:, 3:] = (1 - f1) * np.eye(3)
        b[3:] = eb[Nn]
        x = np.linalg.solve(A, b)
        e1 = eb.copy()
        e2 = eb.copy()
        e1[Nn] = x[:3]
        e2[Nn] = x[3:]
        Cbar[:, k] = f1 * C1 @ e1 + (1 - f1) * C2 @ e2
    return Cbar


@pytest.mark.parametrize("p", [1, 2])
def test_periodic_laminate_closed_form(p):
    n = 4
    coords, tets = mesh.kuhn_mesh(n)
    d = fem.Discretisation(coords, tets, p)
    lower = d.centroid[:, 2] < 0.5
    C1 = M.isotropic_stiffness(3.5, 0.35)
    C2 = _transiso((1.0, 0.5, 0.0))      # fibre in the layer plane
    Ce = np.where(lower[:, None, None], C1[None], C2[None])
    r = fem.solve_rve(d, Ce, fem.BC_PERIODIC, 3)
    assert _rel(r["hom"], _laminate_closed_form(C1, C2, 0.5)) < 1e-11
    k1, k2 = 0.2, 0.8
    ke = np.where(lower[:, None, None], k1 * np.eye(3)[None], k2 * np.eye(3)[None])
    rk = fem.solve_rve(d, ke, fem.BC_PERIODIC, 1)
    arith, harm = 0.5 * (k1 + k2), 1.0 / (0.5 / k1 + 0.5 / k2)
    assert _rel(rk["hom"], np.diag([arith, arith, harm])) < 1e-12


# ------------------------------------------------------------------ invariants
@pytest.fixture(scope="module")
def weave_results():
    n, p = 3, 2
    coords, tets, phase, axis = mesh.plain_weave(n)
    d = fem.Discretisation(coords, tets, p)
    params = ci.draw_factors_only(1, 1)[0]
    m, y, _ = M.phase_materials(ci.BASE_MATERIALS, params)
    Ce, Ke, De = M.element_tensors(phase, axis, m, y)
    res = {bc: (fem.solve_rve(d, Ce, bc, 3), fem.solve_rve(d, Ke, bc, 1)) for bc in BCS}
    return d, Ce, Ke, res


def test_loewner_ordering_of_boundary_conditions(weave_results):
    """Voigt >= Dirichlet >= periodic >= Neumann >= Reuss (nested admissible spaces)."""
    d, Ce, Ke, res = weave_results
    for idx, tens in ((0, Ce), (1, Ke)):
        up, low = fem.voigt_reuss(d, tens)
        chain = [up] + [res[bc][idx]["hom"] for bc in BCS] + [low]
        scale = np.linalg.norm(up)
        for a, b in zip(chain[:-1], chain[1:]):
            assert _sym_eigmin(a - b) > -1e-11 * scale
        # and the orderings are strict for this heterogeneous RVE
        assert _sym_eigmin(chain[1] - chain[3]) > 1e-6 * scale or np.trace(chain[1] - chain[3]) > 1e-4 * scale


def test_hill_mandel_and_three_routes_agree(weave_results):
    """Multiplier, volume-average and energy routes of sigma_bar agree (Eqs. Hill_prin, eq_homo_stress)."""
    d, Ce, Ke, res = weave_results
    for bc in BCS:
        for r in res[bc]:
            assert _rel(r["hom_vol"], r["hom"]) < 1e-11
            assert _rel(r["hom_energy"], r["hom"]) < 1e-11


def test_symmetric_positive_definite(weave_results):
    d, Ce, Ke, res = weave_results
    for bc in BCS:
        for r in res[bc]:
            H = r["hom"]
            assert np.linalg.norm(H - H.T) / np.linalg.norm(H) < 1e-11
            assert np.linalg.eigvalsh(0.5 * (H + H.T)).min() > 0


def test_degree_one_homogeneity(weave_results):
    d, Ce, Ke, res = weave_results
    for bc in BCS:
        r = fem.solve_rve(d, 2.5 * Ce, bc, 3)
        assert _rel(r["hom"], 2.5 * res[bc][0]["hom"]) < 1e-12


def test_p_refinement_monotone():
    """Nested P_p spaces: C_bar(p+1) <= C_bar(p) for every BC."""
    coords, tets, phase, axis = mesh.plain_weave(2)
    m, y, _ = M.phase_materials(ci.BASE_MATERIALS)
    Ce, Ke, De = M.element_tensors(phase, axis, m, y)
    for bc in BCS:
        prev = None
        for p in (1, 2, 3):
            d = fem.Discretisation(coords, tets, p)
            H = fem.solve_rve(d, Ce, bc, 3)["hom"]
            if prev is not None:
                assert _sym_eigmin(prev - H) > -1e-10 * np.linalg.norm(H)
            prev = H


@pytest.mark.parametrize("n,p", [(1, 2), (2, 1)])
def test_sparse_lu_equals_dense_solve(n, p):
    coords, tets, phase, axis = mesh.plain_weave(n)
    d = fem.Discretisation(coords, tets, p)
    m, y, _ = M.phase_materials(ci.BASE_MATERIALS)
    Ce, Ke, De = M.element_tensors(phase, axis, m, y)
    for bc in BCS:
        r = fem.solve_rve(d, Ce, bc, 3)
        A = sp.bmat([[r["K"], r["C"].T], [r["C"], None]]).toarray()
        rhs = np.vstack([np.zeros((r["K"].shape[0], 6)), r["D"]])
        sol = np.linalg.solve(A, rhs)
        lam = sol[r["K"].shape[0]:]
        H = -(r["D"].T @ lam) / d.V
        assert _rel(r["hom"], H) < 1e-12


# ------------------------------------------------------------------ planted mistakes
def test_planted_mistakes_are_caught(monkeypatch):
    """Mistakes planted in the oracle (on the CPU) break at least one of the pins above."""
    coords, tets = mesh.kuhn_mesh(2)
    d = fem.Discretisation(coords, tets, 2)
    C = _transiso((1.0, 0.0, 0.0))

    def solve(bc=fem.BC_DIRICHLET):
        return fem.solve_rve(d, _uniform(C, len(tets)), bc, 3)["hom"]

    assert _rel(solve(), C) < 1e-12
    # (1) the matrix X exactly as printed (shear columns 13/23 swapped)
    orig = fem.X_mech

    def X_printed(y):
        X = orig(y)
        return X[..., [0, 1, 2, 3, 5, 4]]
    monkeypatch.setattr(fem, "X_mech", X_printed)
    assert _rel(solve(), C) > 1e-3
    monkeypatch.setattr(fem, "X_mech", orig)

    # (2) the shear halves of X dropped
    def X_noshear_half(y):
        X = orig(y)
        X[..., 3:] *= 2.0
        return X
    monkeypatch.setattr(fem, "X_mech", X_noshear_half)
    assert _rel(solve(), C) > 1e-3
    monkeypatch.setattr(fem, "X_mech", orig)

    # (3) transposed Voigt tensor map (only matters for anisotropic C): Hill-Mandel catches it
    orig_vt = M.voigt_to_tensor

    def bad_tensor(Cv):
        Ct = orig_vt(Cv)
        return np.transpose(Ct, (0, 2, 1, 3))
    monkeypatch.setattr(M, "voigt_to_tensor", bad_tensor)
    assert _rel(solve(), C) > 1e-3
    monkeypatch.setattr(M, "voigt_to_tensor", orig_vt)


@pytest.mark.parametrize("n,p", [(3, 2), (2, 3), (3, 1)])
def test_substitution_equals_multipliers(n, p):
    """Condensing the Dirichlet / periodic constraints gives the bordered system's answer (Sec. 2)."""
    c, t, ph, ax = mesh.plain_weave(n)
    prm = ci.draw_params(5, 1)[0]
    disc = fem.Discretisation(c, t, p)
    for bc in (fem.BC_DIRICHLET, fem.BC_PERIODIC):
        a = fem.homogenise(c, t, ph, ax, p, bc, ci.BASE_MATERIALS, prm, disc=disc)
        b = fem.homogenise(c, t, ph, ax, p, bc, ci.BASE_MATERIALS, prm, disc=disc, method="substitution")
        for k in "CKD":
            assert _rel(b[k], a[k]) < 1e-12, (bc, k)


def test_nested_dissection_is_a_permutation():
    c, t, ph, ax = mesh.plain_weave(3)
    disc = fem.Discretisation(c, t, 2)
    N = disc.n_nodes
    T, nn = disc.e2n.shape
    E2 = sp.csr_matrix((np.ones(T * nn), (np.repeat(np.arange(T), nn), disc.e2n.ravel())), shape=(T, N))
    order = fem.nested_dissection(disc.nodes, (E2.T @ E2).tocsr(), leaf=8)
    np.testing.assert_array_equal(np.sort(order), np.arange(N))


@pytest.mark.parametrize("bc", [fem.BC_PERIODIC, fem.BC_NEUMANN])
def test_permuted_axes_give_the_permuted_tensors(bc):
    """Renaming the axes (x, y, z) -> (y, z, x) of the lattice weave (tags and
    fibre axes with it) turns C_bar, K_bar, D_bar as tensors: pins the Voigt
    order, the engineering shear and the rotated transversely isotropic law
    against a transposed or mislabelled index anywhere in them."""
    from gpu_util import permuted_lattice, rotate_voigt
    n = 4
    c, t, ph, ax = mesh.plain_weave(n)
    c, t, ph, ax = (np.asarray(v) for v in (c, t, ph, ax))
    perm = [1, 2, 0]
    Q = np.eye(3)[perm]
    prm = np.r_[45.0, 1.0, 3.0, np.ones(8)]
    a = fem.homogenise(c, t, ph, ax, 2, bc, ci.BASE_MATERIALS, prm)
    b = fem.homogenise(*permuted_lattice(c, t, ph, ax, n, perm), 2, bc, ci.BASE_MATERIALS, prm)
    rc = rotate_voigt(a["C"], Q)
    assert np.abs(b["C"] - rc).max() <= 1e-12 * np.abs(rc).max()
    for k in ("K", "D"):
        r3 = Q @ a[k] @ Q.T
        assert np.abs(b[k] - r3).max() <= 1e-12 * np.abs(r3).max()
    assert np.abs(rc - a["C"]).max() > 1e-2 * np.abs(rc).max()   # the weave is not symmetric under it
