"""Materials for the oracle: stiffness, conductivity, degradation (own implementation).

Voigt order follows the paper's text in Sec. 2 (definition of the macro-strain
vector): [11, 22, 33, 12, 23, 31] with engineering shear strains (2*eps_ij).

* Isotropic matrix: Lame form.
* Transversely isotropic yarn (paper Sec. 1 and Sec. 7, Table 2 uses the same
  class of material): compliance built from E1 (fibre), E2 = E3, G12 = G13,
  nu12 (major ratio, S12 = -nu12/E1), nu23 and G23 = E2 / (2 (1 + nu23)); the
  stiffness is its inverse, then rotated from the local frame (fibre along e1)
  to the fibre axis with the 6x6 Voigt (Bond) transformation.
* Conductivity / diffusivity of a yarn: k2 I + (k1 - k2) a a^T.
* Degradation (Sec. 4): alpha(T) = beta ln(1 - T/T_g) (Eq. Eq_alphaT), with the
  temperatures in kelvin, beta = -0.001682 per day, T_g = 126 C; the moisture
  factor gamma(c) is linear with gamma(0) = 0 and gamma(saturation) = 1 (Eq.
  Eq_Model3); for constant exposure the stiffness factor is
  (1 - omega) = exp(-gamma(c) alpha(T) t) (Eq. Eq_Model_final1), t in days;
  for time-varying exposure the rate form (Eq. Eq_Model_RateForm) is stepped
  with backward Euler, as the paper states.
  Only the matrix is degraded (Sec. 5, end of the FE^2 description).
"""
from __future__ import annotations

import numpy as np

BETA = -0.001682          # per day, Sec. 4 least-squares value
TG_CELSIUS = 126.0        # glass transition temperature, Sec. 4
KELVIN = 273.15
DAYS_PER_YEAR = 365.25

# Voigt index of a symmetric pair (i, j)
VOIGT = np.array([[0, 3, 5],
                  [3, 1, 4],
                  [5, 4, 2]])
VOIGT_PAIRS = [(0, 0), (1, 1), (2, 2), (0, 1), (1, 2), (2, 0)]


def isotropic_stiffness(E, nu):
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    C = np.zeros((6, 6))
    C[:3, :3] = lam
    C[0, 0] = C[1, 1] = C[2, 2] = lam + 2.0 * mu
    C[3, 3] = C[4, 4] = C[5, 5] = mu
    return C


def transiso_compliance(E1, E2, G12, nu12, nu23):
    """Local compliance, fibre along e1, Voigt [11,22,33,12,23,31], engineering shear."""
    G23 = E2 / (2.0 * (1.0 + nu23))
    S = np.zeros((6, 6))
    S[0, 0] = 1.0 / E1
    S[1, 1] = S[2, 2] = 1.0 / E2
    S[0, 1] = S[1, 0] = S[0, 2] = S[2, 0] = -nu12 / E1
    S[1, 2] = S[2, 1] = -nu23 / E2
    S[3, 3] = 1.0 / G12      # 12
    S[4, 4] = 1.0 / G23      # 23
    S[5, 5] = 1.0 / G12      # 31
    return S


def transiso_stiffness_local(E1, E2, G12, nu12, nu23):
    return np.linalg.inv(transiso_compliance(E1, E2, G12, nu12, nu23))


def frame_from_axis(a):
    """Rotation R whose first column is the unit vector a (rows: global axes)."""
    a = np.asarray(a, float)
    a = a / np.linalg.norm(a)
    helper = np.array([0.0, 0.0, 1.0]) if abs(a[2]) < 0.9 else np.array([1.0, 0.0, 0.0])
    b = np.cross(a, helper)
    b /= np.linalg.norm(b)
    c = np.cross(a, b)
    return np.stack([a, b, c], axis=1)


def voigt_rotation(R):
    """6x6 matrix T with eps_global = T eps_local for engineering-shear Voigt strains.

    Built by transforming each unit local strain as a tensor: eps_g = R eps_l R^T.
    """
    T = np.zeros((6, 6))
    for J in range(6):
        e = np.zeros((3, 3))
        i, j = VOIGT_PAIRS[J]
        if i == j:
            e[i, i] = 1.0
        else:                       # engineering shear 1 -> tensor components 1/2
            e[i, j] = e[j, i] = 0.5
        g = R @ e @ R.T
        for I in range(6):
            k, l = VOIGT_PAIRS[I]
            T[I, J] = g[k, l] if k == l else 2.0 * g[k, l]
    return T


def rotate_stiffness(C_local, axis):
    """Global stiffness for a local stiffness whose e1 is mapped to axis.

    Energy invariance: eps_l = T^-1 eps_g, so C_g = T^-T C_l T^-1.
    """
    T = voigt_rotation(frame_from_axis(axis))
    Ti = np.linalg.inv(T)
    return Ti.T @ C_local @ Ti


def voigt_to_tensor(C):
    """4th-order tensor C_ijkl from the 6x6 engineering-shear Voigt matrix."""
    Ct = np.empty((3, 3, 3, 3))
    for i in range(3):
        for j in range(3):
            for k in range(3):
                for l in range(3):
                    Ct[i, j, k, l] = C[VOIGT[i, j], VOIGT[k, l]]
    return Ct


def transverse_tensor(k_axial, k_trans, axis):
    a = np.asarray(axis, float)
    a = a / np.linalg.norm(a)
    return k_trans * np.eye(3) + (k_axial - k_trans) * np.outer(a, a)


# ---------------------------------------------------------------- degradation
def alpha_of_T(T_celsius, beta=BETA, Tg_celsius=TG_CELSIUS):
    """Degradation rate per day, Eq. Eq_alphaT with absolute temperatures."""
    TK = np.asarray(T_celsius, float) + KELVIN
    TgK = Tg_celsius + KELVIN
    return beta * np.log(1.0 - TK / TgK)


def gamma_of_c(c, c_sat=1.5):
    """Linear moisture factor, gamma(0) = 0 and gamma(c_sat) = 1 (Eq. Eq_Model3)."""
    return np.asarray(c, float) / c_sat


def stiffness_factor(T_celsius, c, t_years, c_sat=1.5):
    """(1 - omega) = exp(-gamma(c) alpha(T) t) for constant exposure (Eq. Eq_Model_final1)."""
    t_days = np.asarray(t_years, float) * DAYS_PER_YEAR
    return np.exp(-gamma_of_c(c, c_sat) * alpha_of_T(T_celsius) * t_days)


def damage_history(T_celsius, c, dt_years, keep0=1.0, c_sat=1.5):
    """(1 - omega) after every step of a time history (Sec. 4, Eq. Eq_Model_RateForm).

    The rate form d(1 - omega)/dt = -gamma(c) alpha(T) (1 - omega) is discretised
    with the implicit (backward) Euler method the paper names: over step k, of
    length dt_k (days) with exposure T_k, c_k,
        (1 - omega)_k - (1 - omega)_{k-1} = -dt_k gamma(c_k) alpha(T_k) (1 - omega)_k,
    solved for (1 - omega)_k (the equation is linear in it).
    T_celsius, c: [m, n] (step k of every point in row k); dt_years: [m];
    keep0: (1 - omega) before the first step, scalar or [n].  Returns [m, n].
    """
    T = np.atleast_2d(np.asarray(T_celsius, float))
    cc = np.atleast_2d(np.asarray(c, float))
    dt_days = np.asarray(dt_years, float).reshape(-1) * DAYS_PER_YEAR
    keep = np.broadcast_to(np.asarray(keep0, float), T.shape[1:]).copy()
    out = np.empty_like(T)
    for k in range(T.shape[0]):
        rate = gamma_of_c(cc[k], c_sat) * alpha_of_T(T[k])      # per day
        keep = keep / (1.0 + dt_days[k] * rate)
        out[k] = keep
    return out


def equivalent_exposure_years(keep, T_ref_celsius=60.0):
    """Time (years) of constant exposure at T_ref and full saturation (gamma = 1)
    after which Eq. Eq_Model_final1 gives the factor `keep`."""
    return -np.log(np.asarray(keep, float)) / (alpha_of_T(T_ref_celsius) * DAYS_PER_YEAR)


def fit_beta(T_celsius, alphas, Tg_celsius=TG_CELSIUS, kelvin=True):
    """Least-squares beta of Eq. Eq_alphaT_LSF (closed form of a 1-parameter fit)."""
    T = np.asarray(T_celsius, float)
    Tg = Tg_celsius
    if kelvin:
        T = T + KELVIN
        Tg = Tg + KELVIN
    L = np.log(1.0 - T / Tg)
    a = np.asarray(alphas, float)
    return float(np.dot(a, L) / np.dot(L, L))


# ---------------------------------------------------------------- per-RVE materials
def phase_materials(base, params=None, c_sat=1.5, degrade_yarn=False):
    """Per-phase properties for one parameter record.

    base: dict with E, nu, k, D (matrix) and E1, E2, G12, nu12, nu23, k1, k2, D1, D2.
    params: 11 numbers (T_celsius, c_wt, t_years, 8 factors) or None (no change).
    Factor groups: matrix {E, nu, k, D}; yarn {moduli E1, E2, G12}, {nu12, nu23},
    {k1, k2}, {D1, D2}.
    """
    b = dict(base)
    f = np.ones(8)
    omega_keep = 1.0
    if params is not None:
        params = np.asarray(params, float)
        f = params[3:11]
        omega_keep = float(stiffness_factor(params[0], params[1], params[2], c_sat))
    m = dict(E=b["E"] * f[0] * omega_keep, nu=b["nu"] * f[1], k=b["k"] * f[2], D=b["D"] * f[3])
    yscale = omega_keep if degrade_yarn else 1.0
    y = dict(E1=b["E1"] * f[4] * yscale, E2=b["E2"] * f[4] * yscale, G12=b["G12"] * f[4] * yscale,
             nu12=b["nu12"] * f[5], nu23=b["nu23"] * f[5],
             k1=b["k1"] * f[6], k2=b["k2"] * f[6], D1=b["D1"] * f[7], D2=b["D2"] * f[7])
    return m, y, omega_keep


def element_tensors(phase, axis, mat, yarn):
    """Per-element Voigt stiffness [T,6,6], conductivity [T,3,3], diffusivity [T,3,3]."""
    T = len(phase)
    C = np.empty((T, 6, 6))
    K = np.empty((T, 3, 3))
    D = np.empty((T, 3, 3))
    Cm = isotropic_stiffness(mat["E"], mat["nu"])
    Cy_loc = transiso_stiffness_local(yarn["E1"], yarn["E2"], yarn["G12"], yarn["nu12"], yarn["nu23"])
    for e in range(T):
        if phase[e] == 0:
            C[e] = Cm
            K[e] = mat["k"] * np.eye(3)
            D[e] = mat["D"] * np.eye(3)
        else:
            C[e] = rotate_stiffness(Cy_loc, axis[e])
            K[e] = transverse_tensor(yarn["k1"], yarn["k2"], axis[e])
            D[e] = transverse_tensor(yarn["D1"], yarn["D2"], axis[e])
    return C, K, D
