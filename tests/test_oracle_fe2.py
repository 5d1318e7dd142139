"""Pins of the oracle's FE^2 run on a synthetic macro box (paper Sec. 3-5).

* Mesh: the Kuhn split fills the box (volumes sum to lx ly lz, all positive).
* Elasticity of linear elements reproduces linear displacement fields exactly:
  for u = F x and a uniform anisotropic Voigt stiffness the strain energy
  u.K u / 2 equals the volume times eps.C eps / 2 with the engineering Voigt
  strain of F (a transposed strain operator or a shear factor fails this); with
  a uniform orthotropic stiffness the uniaxial test's reaction is
  ly lz strain / S_11, S = C^-1.
* Transport: the conductivity matrix (any symmetric coefficient) annihilates
  linear fields away from the boundary and the capacity matrix integrates one
  exactly; with a very long time step one implicit step reaches the
  exposure value everywhere (constants are in the kernel of K); a column
  heated from the top converges, as the mesh and step shrink, to the series
  solution of the one-dimensional problem (Fourier's law, insulated bottom).
* Damage: with the exposure equal to the initial state the fields stay
  uniform and (1 - omega) at every Gauss point follows the rate form's
  implicit Euler for that constant exposure.
"""
import numpy as np
import pytest

from oracle import fe2, materials


def _ortho_C(E=(3.0, 5.0, 7.0), nu=(0.2, 0.25, 0.3), G=(1.1, 1.3, 1.7)):
    S = np.zeros((6, 6))
    S[0, 0], S[1, 1], S[2, 2] = 1 / E[0], 1 / E[1], 1 / E[2]
    S[0, 1] = S[1, 0] = -nu[0] / E[0]
    S[1, 2] = S[2, 1] = -nu[1] / E[1]
    S[0, 2] = S[2, 0] = -nu[2] / E[0]
    S[3, 3], S[4, 4], S[5, 5] = 1 / G[0], 1 / G[1], 1 / G[2]
    return np.linalg.inv(S)


def _stub(C, k=0.5, d=0.3):
    return lambda params: {"C": C, "K": k * np.eye(3), "D": d * np.eye(3)}


def test_box_mesh_fills_the_box():
    coords, tets = fe2.box_mesh(3, 2, 2, 1.5, 1.0, 0.4)
    g, vol = fe2.p1_gradients(coords, tets)
    assert np.all(vol > 0) and abs(vol.sum() - 1.5 * 1.0 * 0.4) < 1e-14
    # barycentric gradients: sum to zero, and reproduce the coordinates' gradient
    x = coords[tets]
    assert np.allclose(g.sum(axis=1), 0.0, atol=1e-12)
    assert np.allclose(np.einsum("eai,eaj->eij", x, g), np.eye(3)[None], atol=1e-12)


def test_linear_fields_have_exact_energy():
    rng = np.random.default_rng(5)
    coords, tets = fe2.box_mesh(2, 3, 2, 1.0, 1.2, 0.7)
    A = rng.normal(size=(6, 6))
    C = A @ A.T + 6 * np.eye(6)                    # anisotropic, all couplings
    F = rng.normal(size=(3, 3))
    u = (coords @ F.T).ravel()
    K = fe2.elastic_matrix(coords, tets, np.repeat(C[None], len(tets), axis=0))
    eps = np.array([F[0, 0], F[1, 1], F[2, 2], F[0, 1] + F[1, 0], F[1, 2] + F[2, 1], F[2, 0] + F[0, 2]])
    vol = 1.0 * 1.2 * 0.7
    assert abs(u @ (K @ u) - vol * eps @ C @ eps) <= 1e-11 * vol * abs(eps @ C @ eps)


def test_uniaxial_reaction_of_a_uniform_orthotropic_box():
    C = _ortho_C()
    r = fe2.run(_stub(C), 2, 2, 2, lx=1.0, ly=0.8, lz=0.6, T0=20.0, T_top=20.0, c0=0.0, c_top=0.0, steps=1,
                strain_x=2e-3)
    S = np.linalg.inv(C)
    assert abs(r["reaction"][0] - 0.8 * 0.6 * 2e-3 / S[0, 0]) <= 1e-12 * abs(r["reaction"][0])
    # the displacement is the homogeneous uniaxial-stress field
    x = r["coords"]
    eps = S[:, 0] * 2e-3 / S[0, 0]
    assert np.allclose(r["u"], np.stack([eps[0] * x[:, 0], eps[1] * x[:, 1], eps[2] * x[:, 2]], axis=1),
                       atol=1e-14)


def test_long_step_reaches_the_exposure():
    r = fe2.run(_stub(_ortho_C()), 2, 2, 2, T0=20.0, T_top=45.0, c0=0.0, c_top=1.2, dt_years=1e9, steps=1)
    assert np.abs(r["T"][1] - 45.0).max() < 1e-6 and np.abs(r["c"][1] - 1.2).max() < 1e-6


def _series_bottom(t, L, kappa, T0, Ttop, terms=200):
    k = np.arange(terms)
    lam = (2 * k + 1) * np.pi / (2 * L)
    return Ttop + (T0 - Ttop) * np.sum(4 * (-1) ** k / ((2 * k + 1) * np.pi) * np.exp(-kappa * lam ** 2 * t))


def test_conductivity_matrix_is_exact_on_linear_fields():
    coords, tets = fe2.box_mesh(3, 3, 3, 1.0, 0.9, 0.8)
    kmat = np.array([[0.7, 0.1, 0.05], [0.1, 0.5, 0.02], [0.05, 0.02, 0.3]])
    M, K = fe2.scalar_matrices(coords, tets, kmat)
    a = np.array([0.3, -1.2, 0.8])
    r = K @ (coords @ a)
    inner = np.all((coords > 1e-9) & (coords < np.array([1.0, 0.9, 0.8]) - 1e-9), axis=1)
    assert np.abs(r[inner]).max() < 1e-13          # div(k grad(a.x)) = 0 away from the boundary
    assert abs(M.sum() - 1.0 * 0.9 * 0.8) < 1e-14   # the capacity matrix integrates one exactly


def test_heated_column_converges_to_the_series_solution():
    """A column whose top is held at T_top: the temperature of its insulated bottom
    against the series solution of the 1-D problem as cells and steps shrink (the
    Kuhn split is not symmetric, so the discrete field is only nearly independent
    of x and y; that difference shrinks with the cells too)."""
    L, kcond, cap, t_end = 0.5, 0.4, 2.0, 0.2
    exact = _series_bottom(t_end, L, kcond / cap, 20.0, 60.0)
    errs = []
    for nxy, nz, steps in ((1, 4, 4), (2, 8, 16), (4, 16, 64)):
        r = fe2.run(_stub(_ortho_C(), k=kcond), nxy, nxy, nz, lx=0.1, ly=0.1, lz=L, heat_capacity=cap, T0=20.0,
                    T_top=60.0, dt_years=t_end / steps, steps=steps)
        bottom = np.isclose(r["coords"][:, 2], 0.0)
        errs.append(float(np.abs(r["T"][-1][bottom] - exact).max()))
    assert errs[0] > 1.8 * errs[1] > 3.2 * errs[2], errs
    assert errs[2] < 0.01 * 40.0, errs


@pytest.mark.parametrize("steps", [1, 3])
def test_uniform_exposure_damages_every_point_alike(steps):
    T, c, dt = 50.0, 1.0, 0.5
    r = fe2.run(_stub(_ortho_C()), 2, 1, 1, T0=T, T_top=T, c0=c, c_top=c, dt_years=dt, steps=steps)
    ref = materials.damage_history(np.full((steps, 1), T), np.full((steps, 1), c), np.full(steps, dt))[:, 0]
    assert np.allclose(r["keep"], ref[:, None], rtol=1e-13, atol=0)
    assert np.allclose(r["T"], T) and np.allclose(r["c"], c)
