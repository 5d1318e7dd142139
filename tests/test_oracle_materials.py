"""Pins of the oracle's material laws and of the degradation model (CPU)."""
import os

import numpy as np
import pytest

from oracle import materials as M

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden():
    alphas = {}
    vals = {}
    with open(os.path.join(GOLDEN, "degradation_constants.txt")) as fh:
        for line in fh:
            tok = line.split("#")[0].split()
            if not tok:
                continue
            if tok[0] == "alpha":
                alphas[float(tok[1])] = float(tok[2])
            else:
                vals[tok[0]] = float(tok[1])
    return alphas, vals


def kelvin_form(C):
    w = np.array([1, 1, 1, np.sqrt(2), np.sqrt(2), np.sqrt(2)])
    return w[:, None] * C * w[None, :]


def test_isotropic_lame():
    E, nu = 3.5, 0.35
    C = M.isotropic_stiffness(E, nu)
    S = np.linalg.inv(C)
    assert np.isclose(1 / S[0, 0], E)
    assert np.isclose(-S[0, 1] / S[0, 0], nu)
    assert np.isclose(1 / S[3, 3], E / (2 * (1 + nu)))   # engineering shear


def test_transiso_engineering_constants():
    E1, E2, G12, nu12, nu23 = 55.0, 12.0, 4.5, 0.28, 0.4
    C = M.transiso_stiffness_local(E1, E2, G12, nu12, nu23)
    S = np.linalg.inv(C)
    assert np.isclose(1 / S[0, 0], E1) and np.isclose(1 / S[1, 1], E2) and np.isclose(1 / S[2, 2], E2)
    assert np.isclose(-S[0, 1] * E1, nu12) and np.isclose(-S[1, 2] * E2, nu23)
    assert np.isclose(1 / S[3, 3], G12) and np.isclose(1 / S[5, 5], G12)
    assert np.isclose(1 / S[4, 4], E2 / (2 * (1 + nu23)))
    # isotropy in the transverse plane: C44(23) = (C22 - C23) / 2
    assert np.isclose(C[4, 4], 0.5 * (C[1, 1] - C[1, 2]))
    assert np.all(np.linalg.eigvalsh(kelvin_form(C)) > 0)


def test_rotation_properties():
    Cl = M.transiso_stiffness_local(55, 12, 4.5, 0.28, 0.4)
    # axis e1 -> no change
    assert np.allclose(M.rotate_stiffness(Cl, [1, 0, 0]), Cl, atol=1e-12)
    a = np.array([0.3, -0.5, 0.8])
    Cg = M.rotate_stiffness(Cl, a)
    assert np.allclose(Cg, Cg.T, atol=1e-12)
    assert np.allclose(np.linalg.eigvalsh(kelvin_form(Cg)), np.linalg.eigvalsh(kelvin_form(Cl)), rtol=1e-12)
    # the fibre direction carries E1: uniaxial compliance along a equals 1/E1
    S = np.linalg.inv(Cg)
    a = a / np.linalg.norm(a)
    # uniaxial stress a(x)a in Voigt form; the normal strain along a is the same
    # contraction of the engineering strain vector
    sig_dir = np.array([a[0] ** 2, a[1] ** 2, a[2] ** 2, a[0] * a[1], a[1] * a[2], a[2] * a[0]])
    assert np.isclose(sig_dir @ S @ sig_dir, 1 / 55.0)
    # a 90 deg turn about z maps a fibre along x to a fibre along y: swaps 11<->22 and 23<->31
    Cy = M.rotate_stiffness(Cl, [0, 1, 0])
    P = [1, 0, 2, 3, 5, 4]
    assert np.allclose(Cy, Cl[np.ix_(P, P)], atol=1e-12)


def test_transverse_tensor():
    k = M.transverse_tensor(0.8, 0.3, [0, 0, 2.0])
    assert np.allclose(k, np.diag([0.3, 0.3, 0.8]))


def test_beta_reproduced_with_kelvin():
    """Eq. Eq_alphaT_LSF: printed beta lies in the band the 2-s.f. alphas allow (kelvin)."""
    alphas, vals = _golden()
    T = sorted(alphas)
    a = np.array([alphas[t] for t in T])
    beta_K = M.fit_beta(T, a, vals["Tg_C"], kelvin=True)
    lo = M.fit_beta(T, a + 0.00005, vals["Tg_C"], kelvin=True)
    hi = M.fit_beta(T, a - 0.00005, vals["Tg_C"], kelvin=True)
    assert lo <= vals["beta"] <= hi
    assert abs(beta_K - vals["beta"]) < 3e-5
    # the celsius reading of Eq. Eq_alphaT cannot reach the printed value
    beta_C = M.fit_beta(T, a, vals["Tg_C"], kelvin=False)
    lo_c = M.fit_beta(T, a + 0.00005, vals["Tg_C"], kelvin=False)
    hi_c = M.fit_beta(T, a - 0.00005, vals["Tg_C"], kelvin=False)
    assert not (lo_c <= vals["beta"] <= hi_c)
    assert abs(beta_C - vals["beta"]) > 1e-3
    assert np.isclose(M.BETA, vals["beta"]) and np.isclose(M.TG_CELSIUS, vals["Tg_C"])


def test_degradation_law_values_and_limits():
    alpha = M.alpha_of_T([25.0, 60.0, 80.0])
    assert np.allclose(alpha, [0.0023114, 0.0030271, 0.0036343], atol=5e-7)
    assert np.all(np.diff(alpha) > 0)                 # faster ageing when hotter
    assert abs(M.alpha_of_T(-M.KELVIN)) < 1e-15         # no degradation at 0 K
    # 112 days fully saturated (gamma = 1)
    keep = M.stiffness_factor([25.0, 60.0, 80.0], 1.5, 112 / M.DAYS_PER_YEAR, c_sat=1.5)
    assert np.allclose(keep, np.exp(-alpha * 112))
    assert np.allclose(keep, [0.7719, 0.7125, 0.6656], atol=1e-4)
    assert M.stiffness_factor(60.0, 1.0, 0.0) == 1.0
    assert M.stiffness_factor(60.0, 0.0, 7.0) == 1.0
    # the rate form d(1-w)/dt = -gamma alpha (1-w) holds for the closed form
    t = np.linspace(0.0, 5.0, 11)
    w = M.stiffness_factor(40.0, 0.9, t)
    rate = -M.gamma_of_c(0.9) * M.alpha_of_T(40.0) * M.DAYS_PER_YEAR
    num = np.gradient(np.log(w), t)
    assert np.allclose(num, rate, rtol=1e-10)


def test_phase_materials_groups():
    base = dict(E=3.5, nu=0.35, k=0.2, D=1.0, E1=55.0, E2=12.0, G12=4.5, nu12=0.28, nu23=0.4,
                k1=0.8, k2=0.3, D1=0.5, D2=0.2)
    f = [1.1, 0.9, 1.05, 0.95, 1.02, 0.98, 1.01, 0.99]
    params = np.array([60.0, 1.5, 1.0] + f)
    m, y, keep = M.phase_materials(base, params)
    assert np.isclose(keep, np.exp(-M.alpha_of_T(60.0) * M.DAYS_PER_YEAR))
    assert np.isclose(m["E"], 3.5 * 1.1 * keep) and np.isclose(m["nu"], 0.35 * 0.9)
    assert np.isclose(y["E1"], 55 * 1.02) and np.isclose(y["G12"], 4.5 * 1.02)
    assert np.isclose(y["nu23"], 0.4 * 0.98) and np.isclose(y["D2"], 0.2 * 0.99)


# ---------------------------------------------------------------- time-history degradation
def test_damage_history_converges_at_first_order_to_the_closed_form():
    """Constant exposure: backward Euler on the rate form approaches Eq.
    Eq_Model_final1 from above (implicit Euler over-estimates exp(-x)), with the
    error halving as the step halves; a forward step or a dropped moisture factor
    would fail one of these."""
    T, c, years = 60.0, 1.2, 3.0
    exact = float(M.stiffness_factor(T, c, years))
    errs = []
    for m in (50, 100, 200, 400):
        h = M.damage_history(np.full((m, 1), T), np.full((m, 1), c), np.full(m, years / m))
        assert h[-1, 0] > exact
        errs.append(h[-1, 0] - exact)
    ratios = [errs[i] / errs[i + 1] for i in range(3)]
    assert all(1.9 < r < 2.1 for r in ratios), ratios
    assert errs[-1] < 1e-2 * exact    # (lambda t)^2 / (2 m) relative: 0.9% at m = 400


def test_damage_history_piecewise_exposure_limit():
    """Two exposure phases: as the step shrinks the history tends to the exact
    solution of the rate form with piecewise-constant inputs,
    exp(-gamma1 alpha1 t1 - gamma2 alpha2 t2), not to a restart of the closed form."""
    (T1, c1, t1), (T2, c2, t2) = (40.0, 1.5, 2.0), (70.0, 0.5, 1.0)
    lam1 = M.gamma_of_c(c1) * M.alpha_of_T(T1) * t1 * M.DAYS_PER_YEAR
    lam2 = M.gamma_of_c(c2) * M.alpha_of_T(T2) * t2 * M.DAYS_PER_YEAR
    exact = np.exp(-lam1 - lam2)
    m = 4000
    T = np.r_[np.full(m, T1), np.full(m, T2)][:, None]
    c = np.r_[np.full(m, c1), np.full(m, c2)][:, None]
    dt = np.r_[np.full(m, t1 / m), np.full(m, t2 / m)]
    h = M.damage_history(T, c, dt)
    assert abs(h[m - 1, 0] - np.exp(-lam1)) < 1e-3 * np.exp(-lam1)
    assert abs(h[-1, 0] - exact) < 1e-3 * exact


def test_damage_history_invariants():
    """Dry material and absolute zero do not degrade (Sec. 4: degradation stops
    at 0 K); the factor never rises; the final value does not depend on the order
    of the steps (each step multiplies by its own factor); keep0 scales the result."""
    rng = np.random.default_rng(3)
    m, n = 30, 5
    T = rng.uniform(20, 60, (m, n))
    c = rng.uniform(0, 1.5, (m, n))
    dt = rng.uniform(0.01, 0.5, m)
    assert np.all(M.damage_history(T, np.zeros((m, n)), dt) == 1.0)
    assert np.all(M.damage_history(np.full((m, n), -M.KELVIN), c, dt) == 1.0)
    h = M.damage_history(T, c, dt)
    assert np.all(np.diff(np.vstack([np.ones(n), h]), axis=0) <= 0.0) and np.all(h > 0)
    perm = rng.permutation(m)
    hp = M.damage_history(T[perm], c[perm], dt[perm])
    np.testing.assert_allclose(hp[-1], h[-1], rtol=1e-13)
    keep0 = rng.uniform(0.2, 1.0, n)
    np.testing.assert_allclose(M.damage_history(T, c, dt, keep0=keep0), h * keep0, rtol=1e-13)


def test_equivalent_exposure_reproduces_the_factor():
    keep = np.array([1.0, 0.9, 0.3, 1e-3])
    t = M.equivalent_exposure_years(keep)
    np.testing.assert_allclose(M.stiffness_factor(60.0, 1.5, t, c_sat=1.5), keep, rtol=1e-12)
