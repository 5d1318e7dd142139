"""Seeded unstructured tet meshes of a box (input geometry only, no method arithmetic).

Every cell of an nc x nc x nc grid gets an extra vertex at the mean of its
eight corners and is cut into six pyramids (one per face, apex at that vertex),
each pyramid into two tets along the face diagonal through the face corner
with the smallest periodic id (the id of the corner's image in the lo cell).
Neighbouring cells then cut their shared face alike and opposite box faces are
cut alike, so the mesh is conforming and its opposite faces match vertex for
vertex and edge for edge.  Grid vertices are moved by a seeded jitter of up to
`jitter` cell sizes per axis, except along the axes on which they lie on the
box boundary; a vertex and its periodic images move alike.  Vertex valences
and tet shapes vary from cell to cell, so nothing in the mesh is a lattice
pattern.  Tets are oriented positively.
"""
from __future__ import annotations

import numpy as np

from .params import uniform_block

_FACES = (((0, 0, 0), (0, 1, 0), (0, 1, 1), (0, 0, 1)),
          ((1, 0, 0), (1, 1, 0), (1, 1, 1), (1, 0, 1)),
          ((0, 0, 0), (1, 0, 0), (1, 0, 1), (0, 0, 1)),
          ((0, 1, 0), (1, 1, 0), (1, 1, 1), (0, 1, 1)),
          ((0, 0, 0), (1, 0, 0), (1, 1, 0), (0, 1, 0)),
          ((0, 0, 1), (1, 0, 1), (1, 1, 1), (0, 1, 1)))


def unstructured_box(nc: int, seed: int = 0, jitter: float = 0.2, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0)):
    """(coords [(nc+1)^3 + nc^3, 3], tets [12 nc^3, 4] int32)."""
    if nc < 2:
        raise ValueError("nc must be at least 2")
    lo = np.asarray(lo, float)
    hi = np.asarray(hi, float)
    h = (hi - lo) / nc
    n1 = nc + 1
    ii, jj, kk = np.meshgrid(np.arange(n1), np.arange(n1), np.arange(n1), indexing="ij")
    ii, jj, kk = ii.ravel(order="F"), jj.ravel(order="F"), kk.ravel(order="F")   # vertex id i + n1 (j + n1 k)
    ijk = np.stack([ii, jj, kk], axis=1)
    master = (ii % nc) + nc * ((jj % nc) + nc * (kk % nc))
    u = uniform_block(seed, 0, 3 * nc ** 3).reshape(nc ** 3, 3)
    disp = (2.0 * u[master] - 1.0) * jitter * h
    on_bnd = (ijk == 0) | (ijk == nc)
    disp[on_bnd] = 0.0
    grid = lo + ijk * h + disp
    grid[ijk == nc] = np.broadcast_to(hi, grid.shape)[ijk == nc]        # exact box faces
    grid[ijk == 0] = np.broadcast_to(lo, grid.shape)[ijk == 0]
    vid = lambda i, j, k: i + n1 * (j + n1 * k)
    centres, tets = [], []
    nvg = n1 ** 3
    for k in range(nc):
        for j in range(nc):
            for i in range(nc):
                corners = {(a, b, c): vid(i + a, j + b, k + c) for a in (0, 1) for b in (0, 1) for c in (0, 1)}
                apex = nvg + len(centres)
                centres.append(grid[list(corners.values())].mean(axis=0))
                for face in _FACES:
                    q = [corners[f] for f in face]
                    m = [master[v] for v in q]
                    first = int(np.argmin(m))
                    if first in (0, 2):
                        tets += [(apex, q[0], q[1], q[2]), (apex, q[0], q[2], q[3])]
                    else:
                        tets += [(apex, q[1], q[2], q[3]), (apex, q[1], q[3], q[0])]
    coords = np.concatenate([grid, np.array(centres)])
    tets = np.array(tets, dtype=np.int32)
    x = coords[tets]
    det = np.linalg.det(x[:, 1:] - x[:, :1])
    flip = det < 0
    tets[flip, 1], tets[flip, 2] = tets[flip, 2].copy(), tets[flip, 1].copy()
    if np.abs(det).min() <= 1e-12 * np.prod(h):
        raise ValueError("degenerate tet: jitter too large")
    return coords, tets
