"""ctypes view of include/chom.h (argument marshalling only).

Loading fails loudly when libchom.so has not been built: there is no fallback.
"""
from __future__ import annotations

import ctypes as ct
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libchom.so")

CHOM_OK, CHOM_EINVAL, CHOM_EMESH, CHOM_EMATERIAL, CHOM_ENOCONV, CHOM_EDEVICE, CHOM_ENOMEM = 0, -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "CHOM_OK", -1: "CHOM_EINVAL", -2: "CHOM_EMESH", -3: "CHOM_EMATERIAL",
                -4: "CHOM_ENOCONV", -5: "CHOM_EDEVICE", -6: "CHOM_ENOMEM"}
BC = {"dirichlet": 0, "periodic": 1, "neumann": 2}
FAIL_NONE, FAIL_CAP, FAIL_BREAKDOWN, FAIL_NONFINITE = 0, 1, 2, 3
PRECISION = {"fp64": 0, "fp32_refined": 1}
PRECOND = {"block_jacobi": 0, "two_level": 1}


class ChomMesh(ct.Structure):
    _fields_ = [("n_vertices", ct.c_int32), ("n_tets", ct.c_int32),
                ("coords", ct.c_void_p), ("tets", ct.c_void_p), ("phase", ct.c_void_p),
                ("fibre_axis", ct.c_void_p), ("lo", ct.c_double * 3), ("hi", ct.c_double * 3),
                ("on_device", ct.c_int32)]


class ChomMaterials(ct.Structure):
    _fields_ = [(k, ct.c_double) for k in
                ("E", "nu", "k", "D", "E1", "E2", "G12", "nu12", "nu23", "k1", "k2", "D1", "D2")]


class ChomParams(ct.Structure):
    _fields_ = [("T_celsius", ct.c_double), ("c_wt", ct.c_double), ("t_years", ct.c_double),
                ("factor", ct.c_double * 8)]


class ChomOptions(ct.Structure):
    _fields_ = [("precision", ct.c_int32), ("precond", ct.c_int32), ("max_iter", ct.c_int32),
                ("max_refine", ct.c_int32), ("rtol", ct.c_double), ("inner_rtol", ct.c_double),
                ("c_sat", ct.c_double), ("degrade_yarn", ct.c_int32), ("device_ptrs", ct.c_int32),
                ("hip_stream", ct.c_void_p)]


class ChomReport(ct.Structure):
    _fields_ = [("iters", ct.c_int32 * 12), ("refine_steps", ct.c_int32 * 3), ("status", ct.c_int32),
                ("resid", ct.c_double * 12), ("asym", ct.c_double), ("omega_keep", ct.c_double),
                ("fail", ct.c_int32 * 12), ("fp64_fallback", ct.c_int32 * 3), ("spd", ct.c_int32),
                ("hill_mandel_gap", ct.c_double)]


class ChomMlpOptions(ct.Structure):
    _fields_ = [("members", ct.c_int32), ("device_ptrs", ct.c_int32), ("seed", ct.c_uint64),
                ("c_sat", ct.c_double), ("hip_stream", ct.c_void_p)]


class ChomMlpTrainOptions(ct.Structure):
    _fields_ = [("epochs", ct.c_int32), ("batch", ct.c_int32), ("lr", ct.c_float), ("lr_final", ct.c_float),
                ("beta1", ct.c_float), ("beta2", ct.c_float), ("eps", ct.c_float),
                ("refit_normalisation", ct.c_int32)]


class ChomFe2Problem(ct.Structure):
    _fields_ = [("nx", ct.c_int32), ("ny", ct.c_int32), ("nz", ct.c_int32), ("lx", ct.c_double),
                ("ly", ct.c_double), ("lz", ct.c_double), ("heat_capacity", ct.c_double), ("T0", ct.c_double),
                ("c0", ct.c_double), ("T_top", ct.c_double), ("c_top", ct.c_double), ("dt_years", ct.c_double),
                ("steps", ct.c_int32), ("strain_x", ct.c_double), ("macro_rtol", ct.c_double),
                ("macro_max_iter", ct.c_int32), ("factors", ct.c_void_p), ("surrogate", ct.c_void_p),
                ("surrogate_thresh", ct.c_double)]


class ChomFe2Output(ct.Structure):
    _fields_ = [("T", ct.c_void_p), ("c", ct.c_void_p), ("keep", ct.c_void_p), ("reaction", ct.c_void_p),
                ("u", ct.c_void_p), ("C_bar", ct.c_void_p), ("macro_iters", ct.c_int32 * 3),
                ("n_fallback", ct.c_int64)]


# every exported symbol of include/chom.h with its ctypes signature
SIGNATURES = {
    "chom_default_options": (ct.c_int, [ct.POINTER(ChomOptions)]),
    "chom_mesh_sizes": (ct.c_int, [ct.c_int32, ct.POINTER(ct.c_int32), ct.POINTER(ct.c_int32)]),
    "chom_generate_plain_weave": (ct.c_int, [ct.c_int32, ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p,
                                             ct.c_void_p]),
    "chom_rve_create": (ct.c_int, [ct.POINTER(ChomMesh), ct.POINTER(ChomMaterials), ct.c_int32, ct.c_int32,
                                   ct.POINTER(ChomOptions), ct.POINTER(ct.c_void_p)]),
    "chom_homogenise": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_int32, ct.c_void_p, ct.c_void_p, ct.c_void_p,
                                   ct.POINTER(ChomReport)]),
    "chom_rve_destroy": (None, [ct.c_void_p]),
    "chom_urve_create": (ct.c_int, [ct.POINTER(ChomMesh), ct.POINTER(ChomMaterials), ct.c_int32,
                                    ct.POINTER(ChomOptions), ct.POINTER(ct.c_void_p)]),
    "chom_urve_sizes": (ct.c_int, [ct.c_void_p, ct.POINTER(ct.c_int64), ct.POINTER(ct.c_int64)]),
    "chom_urve_homogenise": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_int32, ct.c_void_p, ct.c_void_p,
                                        ct.c_void_p, ct.POINTER(ChomReport)]),
    "chom_urve_destroy": (None, [ct.c_void_p]),
    "chom_tag_plain_weave": (ct.c_int, [ct.c_void_p, ct.c_int64, ct.c_void_p, ct.c_int64, ct.c_int32, ct.c_void_p,
                                        ct.c_void_p]),
    "chom_yarn_directions": (ct.c_int, [ct.POINTER(ChomMesh), ct.c_int32, ct.c_void_p, ct.c_double, ct.c_int32,
                                        ct.c_void_p, ct.c_void_p]),
    "chom_damage_history": (ct.c_int, [ct.c_int64, ct.c_int32, ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p,
                                       ct.c_void_p, ct.c_double, ct.c_int32, ct.c_void_p, ct.c_void_p,
                                       ct.c_void_p]),
    "chom_fe2_run": (ct.c_int, [ct.c_void_p, ct.POINTER(ChomFe2Problem), ct.POINTER(ChomFe2Output)]),
    "chom_last_error": (ct.c_char_p, []),
    "chom_material_constants": (ct.c_int, [ct.POINTER(ChomMaterials), ct.POINTER(ChomParams), ct.c_double,
                                           ct.c_int32, ct.POINTER(ct.c_double), ct.POINTER(ct.c_double),
                                           ct.POINTER(ct.c_double), ct.POINTER(ct.c_double)]),
    "chom_version": (ct.c_char_p, []),
    "chom_batch_create": (ct.c_int, [ct.POINTER(ct.c_void_p), ct.c_int32, ct.POINTER(ChomOptions),
                                     ct.POINTER(ct.c_void_p)]),
    "chom_batch_homogenise": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p,
                                         ct.POINTER(ChomReport)]),
    "chom_batch_launch_config": (ct.c_int, [ct.c_void_p, ct.POINTER(ct.c_int32), ct.POINTER(ct.c_int32),
                                            ct.POINTER(ct.c_int32), ct.POINTER(ct.c_int32)]),
    "chom_batch_time_operator": (ct.c_int, [ct.c_void_p, ct.c_int32, ct.c_int32, ct.POINTER(ct.c_double),
                                            ct.POINTER(ct.c_int64), ct.POINTER(ct.c_int32)]),
    "chom_batch_destroy": (None, [ct.c_void_p]),
    "chom_time_operator": (ct.c_int, [ct.c_void_p, ct.c_int32, ct.c_int32, ct.POINTER(ct.c_double),
                                      ct.POINTER(ct.c_int64), ct.POINTER(ct.c_int32)]),
    "chom_element_apply_host": (ct.c_int, [ct.c_int32, ct.c_void_p, ct.c_double, ct.c_void_p, ct.c_void_p,
                                           ct.c_void_p, ct.c_void_p]),
    "chom_mlp_default_options": (ct.c_int, [ct.POINTER(ChomMlpOptions)]),
    "chom_mlp_default_train_options": (ct.c_int, [ct.POINTER(ChomMlpTrainOptions)]),
    "chom_mlp_create": (ct.c_int, [ct.POINTER(ChomMlpOptions), ct.POINTER(ct.c_void_p)]),
    "chom_mlp_sizes": (ct.c_int, [ct.c_void_p, ct.POINTER(ct.c_int64), ct.POINTER(ct.c_int32)]),
    "chom_mlp_set_weights": (ct.c_int, [ct.c_void_p, ct.c_int32, ct.c_void_p]),
    "chom_mlp_get_weights": (ct.c_int, [ct.c_void_p, ct.c_int32, ct.c_void_p]),
    "chom_mlp_set_normalisation": (ct.c_int, [ct.c_void_p, ct.c_void_p]),
    "chom_mlp_get_normalisation": (ct.c_int, [ct.c_void_p, ct.c_void_p]),
    "chom_mlp_train": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_int64,
                                  ct.POINTER(ChomMlpTrainOptions), ct.c_void_p]),
    "chom_mlp_loss_grad": (ct.c_int, [ct.c_void_p, ct.c_int32, ct.c_void_p, ct.c_void_p, ct.c_void_p,
                                      ct.c_void_p, ct.c_int64, ct.POINTER(ct.c_double), ct.c_void_p]),
    "chom_mlp_loss_grad_noalloc": (ct.c_int, [ct.c_void_p, ct.c_int32, ct.c_void_p, ct.c_void_p, ct.c_void_p,
                                              ct.c_void_p, ct.c_int64, ct.c_void_p, ct.c_void_p]),
    "chom_mlp_predict": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_int64, ct.c_void_p, ct.c_void_p, ct.c_void_p,
                                    ct.c_void_p]),
    "chom_homogenise_surrogate": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_int64, ct.c_double,
                                             ct.c_int32, ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p,
                                             ct.c_void_p, ct.POINTER(ct.c_int64)]),
    "chom_mlp_destroy": (None, [ct.c_void_p]),
    "chom_basis_tables_host": (ct.c_int, [ct.c_int32, ct.POINTER(ct.c_int32), ct.POINTER(ct.c_int32), ct.c_void_p,
                                          ct.c_void_p, ct.c_void_p, ct.c_void_p]),
    "chom_basis_eval_host": (ct.c_int, [ct.c_int32, ct.c_void_p, ct.c_void_p]),
}

_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "(the HIP library is required; there is no fallback path)")
        L = ct.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


class ChomError(RuntimeError):
    def __init__(self, status, where):
        msg = lib().chom_last_error().decode()
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def check(status, where):
    if status != CHOM_OK:
        raise ChomError(status, where)
    return status
