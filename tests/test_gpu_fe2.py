"""Fully nested FE^2 run on the GPU (chom_fe2_run) against the CPU oracle (oracle/fe2.py).

Both sides run the same macro box (Kuhn P1 tets, one Gauss point per tet), the
same implicit transport steps, the damage update per Gauss point and an RVE
solve per Gauss point and step; the oracle homogenises with its own FE solver
(Lagrange P2, sparse direct), the GPU with an FP64 RVE handle at rtol 1e-12, and
its macro systems with CG to 1e-13.  Cases: a 2 x 2 x 1 box (24 Gauss points) on
the 3^3 plain weave, two steps of one year with a hot, wet top face (damage
varies across the box); the same box with the exposure equal to the initial
state (no damage, one stiffness everywhere) against the oracle's macro solve
with that stiffness; argument errors.
"""
import numpy as np
import pytest

import chom_inputs as ci
from oracle import fe2 as ofe2, fem as ofem, mesh as omesh

from gpu_util import banner, require_gpu

pytestmark = pytest.mark.gpu
CASE = dict(nx=2, ny=2, nz=1, lx=1.0, ly=1.0, lz=0.5, heat_capacity=1.5, T0=20.0, c0=0.0, T_top=60.0, c_top=1.5,
            dt_years=1.0, steps=2, strain_x=1e-3)


def _full6(c21):
    C = np.zeros((len(c21), 6, 6))
    iu = np.triu_indices(6)
    C[:, iu[0], iu[1]] = c21
    C[:, iu[1], iu[0]] = c21
    return C


def _rve_pair(n=3):
    from paper_1610_03484_amd import RVE, generate_plain_weave
    c, t, ph, ax = omesh.plain_weave(n)
    disc = ofem.Discretisation(c, t, 2)

    def oracle_rve(params):
        return ofem.homogenise(c, t, ph, ax, 2, ofem.BC_PERIODIC, ci.BASE_MATERIALS, params, disc=disc)

    rve = RVE(*generate_plain_weave(n), ci.BASE_MATERIALS, bc="periodic", precision="fp64", rtol=1e-12,
              max_iter=50000)
    return rve, oracle_rve


def test_fe2_run_matches_oracle():
    require_gpu()
    from paper_1610_03484_amd import fe2_run
    banner("FE^2: 2x2x1 macro box, 24 Gauss points, 3^3 periodic RVE, two steps")
    rve, oracle_rve = _rve_pair()
    g = fe2_run(rve, macro_rtol=1e-13, **CASE)
    rve.close()
    o = ofe2.run(oracle_rve, **CASE)
    eT = np.abs(g["T"] - o["T"]).max() / 40.0
    ec = np.abs(g["c"] - o["c"]).max() / 1.5
    ek = np.abs(g["keep"] / o["keep"] - 1.0).max()
    eC = np.abs(_full6(g["C_bar"]) - o["C_bar"]).max() / np.abs(o["C_bar"]).max()
    eu = np.abs(g["u"] - o["u"]).max() / np.abs(o["u"]).max()
    eR = np.abs(g["reaction"] / o["reaction"] - 1.0).max()
    banner(f"  T {eT:.1e} c {ec:.1e} keep {ek:.1e} C_bar {eC:.1e} u {eu:.1e} reaction {eR:.1e}; "
           f"keep range {o['keep'].min():.3f}..{o['keep'].max():.3f}; macro CG steps {g['macro_iters']}")
    assert g["status"] == 0
    assert o["keep"].min() < 0.9 * o["keep"].max()        # the damage does vary across the box
    assert eT <= 1e-10 and ec <= 1e-10
    assert ek <= 1e-10
    assert eC <= 1e-9
    assert eu <= 1e-8 and eR <= 1e-8


def test_fe2_with_the_benchmark_rve_form_matches_oracle():
    """The RVE form the benchmark's FE^2 leg uses -- FP32 operator with FP64
    refinement at rtol 3e-5 (inner 2e-5), two-level preconditioner with its
    coarse grid (6^3 RVE: hierarchy 6 -> 3) -- on a 2 x 1 x 1 box over two steps:
    every output within the refined form's accuracy (C_bar about 1e-6 of the
    exact discrete values) of the oracle."""
    require_gpu()
    from paper_1610_03484_amd import RVE, fe2_run, generate_plain_weave
    banner("FE^2 with the FP32-refined two-level 6^3 RVE: 2x1x1 box, 12 Gauss points, two steps")
    n = 6
    c, t, ph, ax = omesh.plain_weave(n)
    disc = ofem.Discretisation(c, t, 2)

    def oracle_rve(params):
        return ofem.homogenise(c, t, ph, ax, 2, ofem.BC_PERIODIC, ci.BASE_MATERIALS, params, disc=disc,
                               method="substitution")

    rve = RVE(*generate_plain_weave(n), ci.BASE_MATERIALS, bc="periodic", precision="fp32_refined", rtol=3e-5,
              inner_rtol=2e-5, max_iter=50000)
    case = dict(CASE, nx=2, ny=1, nz=1)
    g = fe2_run(rve, macro_rtol=1e-12, **case)
    rve.close()
    o = ofe2.run(oracle_rve, **case)
    eT = np.abs(g["T"] - o["T"]).max() / 40.0
    ec = np.abs(g["c"] - o["c"]).max() / 1.5
    ek = np.abs(g["keep"] / o["keep"] - 1.0).max()
    eC = np.abs(_full6(g["C_bar"]) - o["C_bar"]).max() / np.abs(o["C_bar"]).max()
    eu = np.abs(g["u"] - o["u"]).max() / np.abs(o["u"]).max()
    eR = np.abs(g["reaction"] / o["reaction"] - 1.0).max()
    banner(f"  T {eT:.1e} c {ec:.1e} keep {ek:.1e} C_bar {eC:.1e} u {eu:.1e} reaction {eR:.1e}")
    assert g["status"] == 0
    assert eT <= 1e-6 and ec <= 1e-6 and ek <= 1e-6
    assert eC <= 2e-6 and eu <= 5e-6 and eR <= 5e-6


def test_fe2_undamaged_box_is_uniform():
    """No damage: every Gauss point gets the undamaged C_bar, the macro solution
    equals the oracle's macro solve with that uniform (anisotropic) stiffness, and
    the reaction is near ly lz strain / S_11 (exact only for an orthotropic
    stiffness; the weave's small shear couplings move it by about 2e-5)."""
    require_gpu()
    from paper_1610_03484_amd import fe2_run
    banner("FE^2: exposure equal to the initial state (no damage)")
    rve, _ = _rve_pair()
    case = dict(CASE, T_top=20.0, c_top=0.0, steps=1)
    g = fe2_run(rve, macro_rtol=1e-13, **case)
    rve.close()
    C = _full6(g["C_bar"])
    assert np.abs(C - C[0]).max() <= 1e-12 * np.abs(C[0]).max()   # one material everywhere
    assert np.all(g["keep"] == 1.0)
    o = ofe2.run(lambda p: {"C": C[0], "K": np.eye(3), "D": np.eye(3)}, **case)
    eu = np.abs(g["u"] - o["u"]).max() / np.abs(o["u"]).max()
    S = np.linalg.inv(C[0])
    ref = case["ly"] * case["lz"] * case["strain_x"] / S[0, 0]
    banner(f"  reaction {g['reaction'][0]:.10e} oracle {o['reaction'][0]:.10e} orthotropic closed form {ref:.10e}")
    assert eu <= 1e-9 and abs(g["reaction"][0] / o["reaction"][0] - 1.0) <= 1e-9
    assert abs(g["reaction"][0] / ref - 1.0) <= 1e-3


def _trained_surrogate(rve, members=2):
    """A small ensemble trained on 256 solves of the test RVE (its predictions are
    close to the RVE's, so the macro stiffness stays positive definite)."""
    from paper_1610_03484_amd import Surrogate
    p = ci.draw_params(41, 256)
    C, K, D, _ = rve.homogenise(p)
    s = Surrogate(members=members, seed=5)
    s.train(p, C, K, D, epochs=40, batch=64)
    return s


def test_fe2_surrogate_with_every_record_on_the_fallback_is_the_rve_path():
    require_gpu()
    from paper_1610_03484_amd import fe2_run
    banner("FE^2 with the surrogate, threshold 0 (every Gauss point re-solved by the RVE)")
    rve, _ = _rve_pair()
    s = _trained_surrogate(rve)
    g = fe2_run(rve, surrogate=s, surrogate_thresh=0.0, **CASE)
    r = fe2_run(rve, **CASE)
    s.close()
    rve.close()
    assert g["n_fallback"] == 6 * CASE["nx"] * CASE["ny"] * CASE["nz"] * CASE["steps"]
    for k in ("T", "c", "keep", "u", "reaction", "C_bar"):
        e = np.abs(g[k] - r[k]).max() / np.abs(r[k]).max()
        assert e <= 1e-9, (k, e)


def test_fe2_surrogate_network_matches_oracle():
    """Threshold infinity: the network's C_bar at every Gauss point.  The oracle runs
    the same FE^2 steps with the reference network (oracle/mlp.py) of the same
    weights and standardisation at the Gauss points; C_bar agrees to the
    surrogate's prediction tolerance (a few bfloat16 steps), the fields that do
    not depend on it (T, c, damage) to rounding."""
    require_gpu()
    from paper_1610_03484_amd import fe2_run
    from oracle import mlp as ref
    banner("FE^2 with the surrogate network at every Gauss point against the oracle")
    rve, oracle_rve = _rve_pair()
    s = _trained_surrogate(rve)
    g = fe2_run(rve, surrogate=s, surrogate_thresh=np.inf, **CASE)
    flats = [s.get_weights(m).astype(np.float64) for m in range(2)]
    nr = s.get_normalisation()
    s.close()
    rve.close()
    x_mu, x_sd, y_mu, y_sd = nr[:10], nr[10:20], nr[20:56], nr[56:92]

    def network(params):
        mean, _ = ref.predict(flats, x_mu, x_sd, y_mu, y_sd, np.asarray(params)[None, :], quant=True)
        return {"C": _full6(mean[:, :21])[0]}

    o = ofe2.run(oracle_rve, gauss=network, **CASE)
    assert g["n_fallback"] == 0
    for k in ("T", "c", "keep"):
        assert np.abs(g[k] - o[k]).max() <= 1e-9 * np.abs(o[k]).max(), k
    Cg, Co = _full6(g["C_bar"]), o["C_bar"]
    ec = np.linalg.norm(Cg - Co, axis=(1, 2)) / np.linalg.norm(Co, axis=(1, 2))
    eu = np.abs(g["u"] - o["u"]).max() / np.abs(o["u"]).max()
    er = np.abs(g["reaction"] / o["reaction"] - 1.0).max()
    banner(f"  C_bar block error max {ec.max():.1e}, u {eu:.1e}, reaction {er:.1e}")
    assert ec.max() <= 2e-3 and eu <= 3e-3 and er <= 3e-3


def test_fe2_rejects_bad_arguments():
    require_gpu()
    from paper_1610_03484_amd import fe2_run
    from paper_1610_03484_amd import _lib as L
    rve, _ = _rve_pair()
    with pytest.raises(L.ChomError) as ei:
        fe2_run(rve, **dict(CASE, nx=0))
    assert ei.value.status == L.CHOM_EINVAL
    with pytest.raises(L.ChomError) as ei:
        fe2_run(rve, **dict(CASE, T_top=130.0))     # above the glass transition: outside the law
    assert ei.value.status == L.CHOM_EINVAL
    with pytest.raises(L.ChomError) as ei:
        fe2_run(rve, **dict(CASE, c0=-0.1))         # negative moisture
    assert ei.value.status == L.CHOM_EINVAL
    with pytest.raises(L.ChomError) as ei:
        fe2_run(rve, **dict(CASE, dt_years=0.0))
    assert ei.value.status == L.CHOM_EINVAL
    # a valid call on the same handle still works after the rejections
    g = fe2_run(rve, **dict(CASE, steps=1))
    assert np.isfinite(g["reaction"]).all()
    rve.close()


def test_reaction_is_linear_in_the_applied_strain():
    """The macro problem is linear elasticity at the step's damage, and the
    damage does not depend on the load: doubling the prescribed strain doubles
    the reaction and the displacement and leaves T, c, (1 - omega) and C_bar
    unchanged (to the run-to-run rounding of atomic sums)."""
    require_gpu()
    from paper_1610_03484_amd import fe2_run
    rve, _ = _rve_pair()
    a = fe2_run(rve, macro_rtol=1e-13, **CASE)
    b = fe2_run(rve, macro_rtol=1e-13, **dict(CASE, strain_x=2 * CASE["strain_x"]))
    rve.close()
    eR = np.abs(b["reaction"] / (2 * a["reaction"]) - 1.0).max()
    eu = np.abs(b["u"] - 2 * a["u"]).max() / np.abs(2 * a["u"]).max()
    banner(f"FE^2 strain doubled: reaction {eR:.1e}, displacement {eu:.1e}")
    assert eR <= 1e-9 and eu <= 1e-9
    for k in ("T", "c", "keep", "C_bar"):   # equal up to the order of the solvers' FP64 atomic sums
        assert np.abs(a[k] - b[k]).max() <= 1e-12 * np.abs(a[k]).max(), k
