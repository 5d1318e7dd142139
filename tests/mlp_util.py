"""Seeded synthetic network weights and rows shared by the surrogate tests."""
import math

import numpy as np

import chom_inputs as ci
from oracle import mlp


def weights(seed, member=0, scale=1.0):
    """Member weights U(-a, a), a = scale * sqrt(3 / fan_in); biases U(-0.1, 0.1)."""
    u = ci.uniform_block(seed, member, mlp.n_params())
    out, k = [], 0
    for i, o in mlp.LAYERS:
        a = scale * math.sqrt(3.0 / i)
        W = (2.0 * u[k:k + o * i] - 1.0) * a
        k += o * i
        b = (2.0 * u[k:k + o] - 1.0) * 0.1
        k += o
        out.append(np.concatenate([W, b]))
    return np.concatenate(out)


def rows(seed, n, width, stream=0):
    return (2.0 * ci.uniform_block(seed, stream, n * width) - 1.0).reshape(n, width)


def norm_record(x_mu, x_sd, y_mu, y_sd):
    return np.concatenate([x_mu, x_sd, y_mu, y_sd])
