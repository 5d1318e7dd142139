"""Yarn directions from a potential-flow solve on each yarn (oracle, test infrastructure only).

Sec. 6 of the paper obtains the fibre direction of a yarn from the potential
phi of a flow through that yarn alone: Laplace's equation on the yarn's
elements, and the direction is the gradient of phi.  The paper gives no
boundary data; the reading used here: phi = 0 on the yarn's vertices on the
inlet face of the cell (the coordinate plane lo[d], d the axis the yarn runs
along), phi = 1 on its vertices on the outlet face hi[d], and no flux through
the rest of the yarn's surface (the natural condition).  Discretisation:
linear (P1) elements on the yarn's tetrahedra, exact integration (the P1
stiffness of a tet is |e| g_a . g_b with g the gradients of the barycentric
coordinates), a direct sparse solve.  The direction of a tet is its constant
gradient of phi, normalised.

Everything here is plain assembly and a direct solve; it shares no code with
the GPU path.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def tet_gradients(coords, tets):
    """Barycentric gradients g [nt, 4, 3] and volumes [nt] of each tet."""
    x = np.asarray(coords, float)[np.asarray(tets)]
    J = np.stack([x[:, 1] - x[:, 0], x[:, 2] - x[:, 0], x[:, 3] - x[:, 0]], axis=2)   # columns: edges
    vol = np.abs(np.linalg.det(J)) / 6.0
    Jinv = np.linalg.inv(J)                     # rows: gradients of lambda_1..3
    g = np.empty((len(tets), 4, 3))
    g[:, 1:] = Jinv
    g[:, 0] = -Jinv.sum(axis=1)
    return g, vol


def yarn_potential(coords, tets, sel, axis, lo, hi, tol=1e-12):
    """phi at the vertices of the tets `sel` (one yarn).  Returns (vertex ids, phi,
    inlet ids, outlet ids, the assembled stiffness over those vertices)."""
    T = np.asarray(tets)[sel]
    verts, local = np.unique(T, return_inverse=True)
    local = local.reshape(T.shape)
    g, vol = tet_gradients(coords, T)
    Ke = vol[:, None, None] * np.einsum("eai,ebi->eab", g, g)
    rows = np.repeat(local, 4, axis=1).ravel()
    cols = np.tile(local, (1, 4)).ravel()
    K = sp.csr_matrix((Ke.ravel(), (rows, cols)), shape=(len(verts), len(verts)))
    xc = np.asarray(coords, float)[verts, axis]
    inlet = np.abs(xc - lo[axis]) <= tol * max(1.0, abs(hi[axis] - lo[axis]))
    outlet = np.abs(xc - hi[axis]) <= tol * max(1.0, abs(hi[axis] - lo[axis]))
    if not inlet.any() or not outlet.any():
        raise ValueError("yarn does not reach both end faces")
    fixed = inlet | outlet
    phi = np.zeros(len(verts))
    phi[outlet] = 1.0
    free = ~fixed
    rhs = -K[free][:, fixed] @ phi[fixed]
    phi[free] = spla.spsolve(K[free][:, free].tocsc(), rhs)
    return verts, phi, np.flatnonzero(inlet), np.flatnonzero(outlet), K


def yarn_directions(coords, tets, phase, yarn_axis, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0)):
    """Unit fibre axis [nt, 3] of every yarn tet (phase j + 1 runs along
    coordinate yarn_axis[j]); zero for matrix tets."""
    tets = np.asarray(tets)
    phase = np.asarray(phase)
    out = np.zeros((len(tets), 3))
    for j, d in enumerate(yarn_axis):
        sel = np.flatnonzero(phase == j + 1)
        if len(sel) == 0:
            continue
        verts, phi, _, _, _ = yarn_potential(coords, tets, sel, d, lo, hi)
        pos = {v: i for i, v in enumerate(verts)}
        g, _ = tet_gradients(coords, tets[sel])
        idx = np.vectorize(pos.get)(tets[sel])
        grad = np.einsum("ea,eai->ei", phi[idx], g)
        out[sel] = grad / np.linalg.norm(grad, axis=1, keepdims=True)
    return out
