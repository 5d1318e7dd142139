"""MI355X-native RVE computational homogenisation (hot path of arXiv:1610.03484).

The compute path is libchom.so (hand-written HIP kernels for gfx950) behind the
C ABI declared in include/chom.h; this package is a thin binding over it.
"""
from .api import (  # noqa: F401
    RVE, URVE, Batch, Surrogate, damage_history, tag_plain_weave, yarn_directions, fe2_run, default_options, mlp_default_options, mlp_train_options, generate_plain_weave, material_constants, mesh_sizes,
    upper21_to_matrix, upper6_to_matrix,
)
