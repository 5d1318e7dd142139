"""Options of chom_options that change the inputs' meaning (GPU, through the
C ABI): the saturation content c_sat and yarn damage (degrade_yarn) against the
oracle; device-resident parameters and outputs (device_ptrs) and a caller's HIP
stream (hip_stream) against the default host-pointer call."""
import ctypes as ct

import numpy as np
import pytest

import chom_inputs as ci
from gpu_util import banner, require_gpu, result_errors, upper21, upper6
from oracle import fem as ofem, mesh as omesh

pytestmark = pytest.mark.gpu


def _rve(n, bc, **opts):
    from paper_1610_03484_amd import RVE, generate_plain_weave
    return RVE(*generate_plain_weave(n, device="cuda"), ci.BASE_MATERIALS, bc=bc, **opts)


@pytest.mark.parametrize("c_sat,degrade_yarn", [(1.0, 0), (1.5, 1), (2.5, 1)])
def test_c_sat_and_yarn_damage_match_oracle(c_sat, degrade_yarn):
    require_gpu()
    n = 4
    params = ci.draw_params(21, 2)
    r = _rve(n, "periodic", precision="fp64", rtol=1e-12, max_iter=20000, c_sat=c_sat, degrade_yarn=degrade_yarn)
    C, K, D, rep = r.homogenise(params)
    r.close()
    c, t, ph, ax = omesh.plain_weave(n)
    for i, p in enumerate(params):
        ref = ofem.homogenise(c, t, ph, ax, 2, ofem.BC_PERIODIC, ci.BASE_MATERIALS, p, c_sat=c_sat,
                              degrade_yarn=bool(degrade_yarn))
        e = result_errors(C[i], K[i], D[i], upper21(ref["C"]), upper6(ref["K"]), upper6(ref["D"]))
        banner(f"c_sat {c_sat} degrade_yarn {degrade_yarn} record {i}: keep {rep[i]['omega_keep']:.3e} errors {e}")
        assert rep[i]["status"] == 0 and max(e) <= 1e-9
        assert abs(rep[i]["omega_keep"] - ref["omega_keep"]) <= 1e-14


def test_yarn_damage_changes_the_result():
    """degrade_yarn really reaches the yarn moduli (a degraded record differs)."""
    require_gpu()
    params = ci.draw_params(22, 1)
    out = []
    for dy in (0, 1):
        r = _rve(4, "periodic", precision="fp64", rtol=1e-12, degrade_yarn=dy)
        out.append(r.homogenise(params)[0])
        r.close()
    assert np.abs(out[0] - out[1]).max() > 1e-3 * np.abs(out[0]).max()


def test_device_pointers_equal_host_pointers():
    require_gpu()
    import torch
    from paper_1610_03484_amd import _lib as L
    params = ci.draw_params(23, 3)
    host = _rve(6, "neumann", precision="fp32_refined", rtol=1e-8)
    Ch, Kh, Dh, _ = host.homogenise(params)
    host.close()
    dev = _rve(6, "neumann", precision="fp32_refined", rtol=1e-8, device_ptrs=1)
    B = len(params)
    p = torch.as_tensor(np.ascontiguousarray(params), dtype=torch.float64, device="cuda")
    C = torch.full((B, 21), float("nan"), dtype=torch.float64, device="cuda")
    K = torch.full((B, 6), float("nan"), dtype=torch.float64, device="cuda")
    D = torch.full((B, 6), float("nan"), dtype=torch.float64, device="cuda")
    reps = (L.ChomReport * B)()
    torch.cuda.synchronize()
    st = L.lib().chom_homogenise(dev._h, ct.c_void_p(p.data_ptr()), B, ct.c_void_p(C.data_ptr()),
                                 ct.c_void_p(K.data_ptr()), ct.c_void_p(D.data_ptr()), reps)
    torch.cuda.synchronize()
    dev.close()
    L.check(st, "chom_homogenise")
    e = max(float(np.abs(C.cpu().numpy() - Ch).max() / np.abs(Ch).max()),
            float(np.abs(K.cpu().numpy() - Kh).max() / np.abs(Kh).max()),
            float(np.abs(D.cpu().numpy() - Dh).max() / np.abs(Dh).max()))
    banner(f"device pointers vs host pointers, 6^3 neumann, {B} records: max rel diff {e:.1e}")
    assert e <= 1e-12


def test_caller_stream_gives_the_same_results():
    require_gpu()
    import torch
    params = ci.draw_params(24, 2)
    a = _rve(6, "periodic", precision="fp32_refined", rtol=1e-8)
    Ca, Ka, Da, _ = a.homogenise(params)
    a.close()
    s = torch.cuda.Stream()
    b = _rve(6, "periodic", precision="fp32_refined", rtol=1e-8, hip_stream=s.cuda_stream)
    Cb, Kb, Db, _ = b.homogenise(params)
    b.close()
    torch.cuda.synchronize()
    e = max(float(np.abs(Ca - Cb).max() / np.abs(Ca).max()), float(np.abs(Ka - Kb).max() / np.abs(Ka).max()),
            float(np.abs(Da - Db).max() / np.abs(Da).max()))
    banner(f"caller's stream vs the library's own: max rel diff {e:.1e}")
    assert e <= 1e-12


def test_general_mesh_device_pointers_equal_host_pointers():
    require_gpu()
    import torch
    from paper_1610_03484_amd import URVE, _lib as L
    from oracle import mesh as om
    coords, tets = ci.unstructured_box(3, seed=5)
    c = om.centroids(coords, tets)
    phase, axis = om.yarn_test(c[:, 0], c[:, 1], c[:, 2])
    params = ci.draw_params(25, 2)
    host = URVE(coords, tets, phase, axis, ci.BASE_MATERIALS, bc="neumann", rtol=1e-10, max_iter=20000)
    Ch, Kh, Dh, _ = host.homogenise(params)
    host.close()
    dev = URVE(coords, tets, phase, axis, ci.BASE_MATERIALS, bc="neumann", rtol=1e-10, max_iter=20000,
               device_ptrs=1)
    B = len(params)
    p = torch.as_tensor(np.ascontiguousarray(params), dtype=torch.float64, device="cuda")
    C = torch.full((B, 21), float("nan"), dtype=torch.float64, device="cuda")
    K = torch.full((B, 6), float("nan"), dtype=torch.float64, device="cuda")
    D = torch.full((B, 6), float("nan"), dtype=torch.float64, device="cuda")
    reps = (L.ChomReport * B)()
    torch.cuda.synchronize()
    st = L.lib().chom_urve_homogenise(dev._h, ct.c_void_p(p.data_ptr()), B, ct.c_void_p(C.data_ptr()),
                                      ct.c_void_p(K.data_ptr()), ct.c_void_p(D.data_ptr()), reps)
    torch.cuda.synchronize()
    dev.close()
    L.check(st, "chom_urve_homogenise")
    e = max(float(np.abs(C.cpu().numpy() - Ch).max() / np.abs(Ch).max()),
            float(np.abs(K.cpu().numpy() - Kh).max() / np.abs(Kh).max()),
            float(np.abs(D.cpu().numpy() - Dh).max() / np.abs(Dh).max()))
    banner(f"general mesh, device pointers vs host pointers: max rel diff {e:.1e}")
    assert e <= 1e-12
