"""Helpers shared by the GPU tests (no arithmetic of the method here)."""
import numpy as np
import pytest


def require_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    return torch


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def upper21(C):
    iu = np.triu_indices(6)
    return np.asarray(C)[iu]


def upper6(K):
    K = np.asarray(K)
    return np.array([K[0, 0], K[1, 1], K[2, 2], K[0, 1], K[1, 2], K[0, 2]])


def banner(msg):
    print(f"[gpu-test] {msg}", flush=True)
