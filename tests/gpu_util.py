"""Helpers shared by the tests (no arithmetic of the method here)."""
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


def full6(c21):
    """Symmetric 6x6 from the 21 upper-triangle entries (row-major)."""
    M = np.zeros((6, 6))
    iu = np.triu_indices(6)
    M[iu] = np.asarray(c21)
    return M + np.triu(M, 1).T


def full3(k6):
    """Symmetric 3x3 from [xx, yy, zz, xy, yz, xz]."""
    a = np.asarray(k6)
    return np.array([[a[0], a[3], a[5]], [a[3], a[1], a[4]], [a[5], a[4], a[2]]])


def block_errors(got, ref):
    """Errors of a symmetric matrix `got` against the symmetric reference `ref`:
    relative Frobenius norm, largest entry error relative to ||ref||_F, and the
    energy-weighted error ||ref^-1/2 (got - ref) ref^-1/2||_2 (soft directions of
    a degraded material count as much as stiff ones)."""
    got, ref = np.asarray(got, float), np.asarray(ref, float)
    d = got - ref
    fro = float(np.linalg.norm(d) / np.linalg.norm(ref))
    elem = float(np.abs(d).max() / np.linalg.norm(ref))
    w, V = np.linalg.eigh(0.5 * (ref + ref.T))
    assert w.min() > 0, "reference not positive definite"
    h = V @ np.diag(w ** -0.5) @ V.T
    energy = float(np.abs(np.linalg.eigvalsh(h @ (0.5 * (d + d.T)) @ h)).max())
    return fro, elem, energy


def result_errors(C21, K6, D6, refC21, refK6, refD6):
    """max over the C, K, D blocks of each measure of block_errors (all three returned)."""
    out = np.zeros(3)
    for g, r in ((full6(C21), full6(refC21)), (full3(K6), full3(refK6)), (full3(D6), full3(refD6))):
        out = np.maximum(out, block_errors(g, r))
    return tuple(float(v) for v in out)


def rotate_voigt(C, Q):
    """C_bar (6x6 Voigt, [11, 22, 33, 12, 23, 31], engineering shear) of the
    rotated material: C'_ijkl = Q_ip Q_jq Q_kr Q_ls C_pqrs."""
    pairs = [(0, 0), (1, 1), (2, 2), (0, 1), (1, 2), (2, 0)]
    T = np.zeros((3, 3, 3, 3))
    for I, (i, j) in enumerate(pairs):
        for J, (k, l) in enumerate(pairs):
            for a, b in {(i, j), (j, i)}:
                for c, d in {(k, l), (l, k)}:
                    T[a, b, c, d] = C[I, J]
    Tr = np.einsum("ip,jq,kr,ls,pqrs->ijkl", Q, Q, Q, Q, T)
    return np.array([[Tr[i, j, k, l] for (k, l) in pairs] for (i, j) in pairs])


def permuted_lattice(coords, tets, phase, axis, n, perm):
    """The lattice mesh with axis perm[d] renamed d, in the canonical vertex and
    tet order: canonical vertex (i, j, k) takes the coordinates of the old
    vertex at the position whose axis perm[d] coordinate is the new d one, and
    each canonical tet takes the tags of the old tet on the same vertices."""
    n1 = n + 1
    idx = np.arange(n1 ** 3)
    pos = np.stack([idx % n1, (idx // n1) % n1, idx // (n1 * n1)], axis=1)   # new (i, j, k)
    old = np.zeros_like(pos)
    old[:, perm] = pos                                                       # old position
    vold = old[:, 0] + n1 * (old[:, 1] + n1 * old[:, 2])
    new_coords = coords[vold][:, perm]
    lookup = {tuple(sorted(t)): e for e, t in enumerate(tets.tolist())}
    src = np.array([lookup[tuple(sorted(vold[t]))] for t in tets.tolist()])
    return new_coords, tets, phase[src], axis[src][:, perm]
