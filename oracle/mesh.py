"""Plain-weave RVE geometry for the oracle (own implementation).

Mesh: the unit cube [lo, hi]^3 split into n^3 cells, each cell cut into the six
Kuhn (Freudenthal) tetrahedra that share the cell's main diagonal.  For the
axis permutation (p0, p1, p2) the tet is
    (v0, v0 + e_p0, v0 + e_p0 + e_p1, v0 + (1,1,1)).
The paper meshes its RVE with tetrahedra (Sec. 7, 10,285 tets); this structured
mesh is the synthetic stand-in of the benchmark workload.

Tagging: a tet belongs to the first yarn whose elliptical cross-section
contains the tet centroid (two warp yarns along x, two weft yarns along y, with
sinusoidal centrelines); otherwise it is matrix.  The fibre axis of a yarn tet
is the unit tangent of the yarn centreline at the centroid's abscissa.  The
paper models yarns with elliptical sections along cubic-spline paths (Sec. 1,
Table 1) and takes the fibre directions from a potential-flow solve (Sec. 6);
the analytic tangent here replaces that solve.
"""
from __future__ import annotations

import itertools
import numpy as np

PERMS = list(itertools.permutations(range(3)))   # the 6 tets of a cell, fixed order

# Yarn description: (kind, offset, phase) in tagging order; kind 0 = warp (runs
# along x, section in the y-z plane), 1 = weft (runs along y, section in x-z).
YARNS = ((0, 0.25, 0.0), (0, 0.75, np.pi), (1, 0.25, 0.0), (1, 0.75, np.pi))
SEMI_IN_PLANE = 0.2
SEMI_Z = 0.06
AMPLITUDE = 0.12


def vertex_id(i, j, k, n):
    return i + (n + 1) * (j + (n + 1) * k)


def kuhn_mesh(n: int, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0)):
    """Coordinates [(n+1)^3, 3] and tets [6 n^3, 4] (cell-major, then PERMS order).

    Vertex (i, j, k) has id i + (n+1)(j + (n+1)k) and coordinate lo + (hi-lo)*i/n
    (computed as i/n for the unit cube).
    """
    r = np.arange(n + 1, dtype=np.float64) / n
    lo = np.asarray(lo, float)
    hi = np.asarray(hi, float)
    kk, jj, ii = np.meshgrid(r, r, r, indexing="ij")
    coords = np.stack([ii.ravel(), jj.ravel(), kk.ravel()], axis=1)
    if not (np.all(lo == 0.0) and np.all(hi == 1.0)):
        coords = lo + (hi - lo) * coords
    tets = np.empty((6 * n ** 3, 4), dtype=np.int64)
    ci = np.arange(n)
    K, J, I = np.meshgrid(ci, ci, ci, indexing="ij")
    I, J, K = I.ravel(), J.ravel(), K.ravel()
    for t, perm in enumerate(PERMS):
        corner = np.zeros((len(I), 3), dtype=np.int64)
        cols = [vertex_id(I, J, K, n)]
        for axis in perm[:2]:
            corner[:, axis] += 1
            cols.append(vertex_id(I + corner[:, 0], J + corner[:, 1], K + corner[:, 2], n))
        cols.append(vertex_id(I + 1, J + 1, K + 1, n))
        tets[t::6] = np.stack(cols, axis=1)
    return coords, tets


def tet_volumes(coords, tets):
    """Signed volumes det[x1-x0, x2-x0, x3-x0] / 6."""
    x = coords[tets]
    d = np.einsum("eij->eij", x[:, 1:, :] - x[:, :1, :])
    return np.linalg.det(d) / 6.0


def entity_counts(n: int):
    """Closed forms for the Kuhn mesh: vertices, edges, faces, tets."""
    V = (n + 1) ** 3
    E = 3 * n * (n + 1) ** 2 + 3 * n ** 2 * (n + 1) + n ** 3
    F = 6 * n ** 2 * (n + 1) + 6 * n ** 3
    T = 6 * n ** 3
    return V, E, F, T


def count_entities(tets):
    """Count distinct edges and faces of a tet list directly (brute force)."""
    edges = set()
    faces = set()
    for t in np.asarray(tets):
        t = sorted(int(v) for v in t)
        for a, b in itertools.combinations(t, 2):
            edges.add((a, b))
        for f in itertools.combinations(t, 3):
            faces.add(f)
    return len(edges), len(faces)


def yarn_test(cx, cy, cz):
    """Phase (0 matrix, 1..4 yarn) and unit fibre axis for centroid arrays."""
    cx, cy, cz = (np.asarray(a, float) for a in (cx, cy, cz))
    phase = np.zeros(cx.shape, dtype=np.int8)
    axis = np.zeros(cx.shape + (3,), dtype=np.float64)
    two_pi = 2.0 * np.pi
    for y_idx, (kind, off, ph) in enumerate(YARNS):
        if kind == 0:      # warp: centreline z = 0.5 + A sin(2 pi x + ph), section at y = off
            s = np.sin(two_pi * cx + ph)
            zc = 0.5 + AMPLITUDE * s
            d_in = (cy - off) / SEMI_IN_PLANE
            slope = AMPLITUDE * two_pi * np.cos(two_pi * cx + ph)
            tang = np.stack([np.ones_like(cx), np.zeros_like(cx), slope], axis=-1)
        else:              # weft: centreline z = 0.5 - A sin(2 pi y + ph), section at x = off
            s = np.sin(two_pi * cy + ph)
            zc = 0.5 - AMPLITUDE * s
            d_in = (cx - off) / SEMI_IN_PLANE
            slope = -AMPLITUDE * two_pi * np.cos(two_pi * cy + ph)
            tang = np.stack([np.zeros_like(cx), np.ones_like(cx), slope], axis=-1)
        d_z = (cz - zc) / SEMI_Z
        f = d_in * d_in + d_z * d_z
        hit = (f <= 1.0) & (phase == 0)
        phase[hit] = y_idx + 1
        tang = tang / np.linalg.norm(tang, axis=-1, keepdims=True)
        axis[hit] = tang[hit]
    return phase, axis


def yarn_test_values(cx, cy, cz):
    """Ellipse test value f of every yarn (f <= 1: inside), shape [..., 4] in tagging order."""
    cx, cy, cz = (np.asarray(a, float) for a in (cx, cy, cz))
    out = []
    for kind, off, ph in YARNS:
        if kind == 0:
            zc = 0.5 + AMPLITUDE * np.sin(2.0 * np.pi * cx + ph)
            d_in = (cy - off) / SEMI_IN_PLANE
        else:
            zc = 0.5 - AMPLITUDE * np.sin(2.0 * np.pi * cy + ph)
            d_in = (cx - off) / SEMI_IN_PLANE
        d_z = (cz - zc) / SEMI_Z
        out.append(d_in * d_in + d_z * d_z)
    return np.stack(out, axis=-1)


def yarn_tangents(cx, cy, cz):
    """Unit centreline tangent of every yarn at the centroid's abscissa, shape [..., 4, 3]."""
    cx, cy, cz = (np.asarray(a, float) for a in (cx, cy, cz))
    out = []
    for kind, off, ph in YARNS:
        if kind == 0:
            t = np.stack([np.ones_like(cx), np.zeros_like(cx),
                          AMPLITUDE * 2.0 * np.pi * np.cos(2.0 * np.pi * cx + ph)], axis=-1)
        else:
            t = np.stack([np.zeros_like(cx), np.ones_like(cx),
                          -AMPLITUDE * 2.0 * np.pi * np.cos(2.0 * np.pi * cy + ph)], axis=-1)
        out.append(t / np.linalg.norm(t, axis=-1, keepdims=True))
    return np.stack(out, axis=-2)


def yarn_margin(cx, cy, cz):
    """min over yarns of |f - 1| (ellipse test value), to spot near-ties."""
    cx, cy, cz = (np.asarray(a, float) for a in (cx, cy, cz))
    m = np.full(cx.shape, np.inf)
    two_pi = 2.0 * np.pi
    for kind, off, ph in YARNS:
        if kind == 0:
            zc = 0.5 + AMPLITUDE * np.sin(two_pi * cx + ph)
            d_in = (cy - off) / SEMI_IN_PLANE
        else:
            zc = 0.5 - AMPLITUDE * np.sin(two_pi * cy + ph)
            d_in = (cx - off) / SEMI_IN_PLANE
        d_z = (cz - zc) / SEMI_Z
        m = np.minimum(m, np.abs(d_in * d_in + d_z * d_z - 1.0))
    return m


def centroids(coords, tets):
    """Tet centroids, summed in vertex order then scaled by 1/4."""
    x = coords[tets]
    return (((x[:, 0] + x[:, 1]) + x[:, 2]) + x[:, 3]) * 0.25


def plain_weave(n: int):
    """Mesh + tags of the synthetic plain-weave RVE: (coords, tets, phase, axis)."""
    coords, tets = kuhn_mesh(n)
    c = centroids(coords, tets)
    phase, axis = yarn_test(c[:, 0], c[:, 1], c[:, 2])
    return coords, tets, phase, axis


def distort_interior(coords, n, amount, seed_u):
    """Move interior vertices by up to amount*h per coordinate.

    seed_u: array [(n+1)^3, 3] of numbers in [0, 1) supplied by the caller.
    Boundary vertices stay put, so the cube and its periodic faces are kept.
    """
    h = 1.0 / n
    out = coords.copy()
    ijk = np.stack(np.meshgrid(np.arange(n + 1), np.arange(n + 1), np.arange(n + 1),
                               indexing="ij"), axis=-1).reshape(-1, 3)[:, ::-1]
    interior = np.all((ijk > 0) & (ijk < n), axis=1)
    out[interior] += amount * h * (2.0 * seed_u[interior] - 1.0)
    return out
