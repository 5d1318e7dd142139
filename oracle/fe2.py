"""Fully nested multi-scale run (FE^2) on a synthetic macro box (oracle, test infrastructure only).

Sec. 3 of the paper: macro heat and moisture transport (Eq. Eq_field: capacity
times the rate equals the divergence of the conductivity (diffusivity) times
the gradient), discretised with linear shape functions into a capacity matrix C
and a conductivity matrix K (Eq. Eq_field_disc) and stepped in time here with
implicit Euler: (C/dt + K) psi_{n+1} = (C/dt) psi_n.  The conductivity and
diffusivity are the RVE's homogenised ones for the undamaged material (damage
only softens the matrix, Sec. 5, so they are homogenised once).  Sec. 4: the
damage (1 - omega) at every Gauss point by the rate form with implicit Euler
(materials.damage_history) and the step's end values of T and c.  Sec. 5 (fully
nested FE^2): at every Gauss point the RVE with that damage gives C_bar, and the
macro elasticity problem is solved with it.

Readings (the paper gives no macro mesh or loads): the box [0, lx] x [0, ly] x
[0, lz] split into nx x ny x nz cells of six Kuhn tets (linear elements), one
Gauss point -- the centroid -- per tet (exact for constant-strain elements; the
capacity matrix is the exact consistent P1 mass); T = T_top, c = c_top on the
face z = lz, no flux elsewhere, T0, c0 at t = 0; mechanics: u_x = 0 on x = 0,
u_x = strain_x * lx on x = lx, u_y = 0 on y = 0, u_z = 0 on z = 0, other faces
free; the reaction is the x-force on x = lx.  The Gauss-point values of T and c
are the means of the tet's vertex values.

Plain sparse assembly (scipy) and sparse direct solves; the RVE is a callable
(params record -> dict with C (6x6 Voigt, engineering shear), K, D (3x3)), e.g.
fem.homogenise on an RVE mesh.  Shares no code with the GPU path.
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import materials

PERMS = list(itertools.permutations(range(3)))


def box_mesh(nx, ny, nz, lx, ly, lz):
    """Vertices [(nx+1)(ny+1)(nz+1), 3] (x fastest) and tets [6 nx ny nz, 4]
    (cell-major, x fastest; six Kuhn tets per cell in PERMS order: corner, then
    one step along perm[0], then along perm[1], then the opposite corner)."""
    ii, jj, kk = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1), np.arange(nz + 1), indexing="ij")
    vid = lambda i, j, k: i + (nx + 1) * (j + (ny + 1) * k)
    coords = np.zeros(((nx + 1) * (ny + 1) * (nz + 1), 3))
    idx = vid(ii, jj, kk).ravel()
    coords[idx, 0] = ii.ravel() * lx / nx
    coords[idx, 1] = jj.ravel() * ly / ny
    coords[idx, 2] = kk.ravel() * lz / nz
    tets = []
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                for perm in PERMS:
                    c = [i, j, k]
                    row = [vid(*c)]
                    for axis in perm[:2]:
                        c[axis] += 1
                        row.append(vid(*c))
                    row.append(vid(i + 1, j + 1, k + 1))
                    tets.append(row)
    return coords, np.array(tets, dtype=np.int64)


def p1_gradients(coords, tets):
    """Gradients of the barycentric coordinates [ne, 4, 3] and volumes [ne]."""
    x = coords[tets]
    E = np.stack([x[:, 1] - x[:, 0], x[:, 2] - x[:, 0], x[:, 3] - x[:, 0]], axis=1)   # rows: edges
    vol = np.abs(np.linalg.det(E)) / 6.0
    G = np.linalg.inv(E).transpose(0, 2, 1)      # row a-1: gradient of lambda_a (E g_a = e_a)
    g = np.concatenate([-G.sum(axis=1, keepdims=True), G], axis=1)
    return g, vol


def _assemble(tets, blocks, ncomp, nv):
    ne = len(tets)
    dofs = (tets[:, :, None] * ncomp + np.arange(ncomp)[None, None, :]).reshape(ne, 4 * ncomp)
    rows = np.repeat(dofs, 4 * ncomp, axis=1).ravel()
    cols = np.tile(dofs, (1, 4 * ncomp)).ravel()
    return sp.csr_matrix((blocks.reshape(ne, -1).ravel(), (rows, cols)), shape=(nv * ncomp, nv * ncomp))


def scalar_matrices(coords, tets, kmat):
    """Consistent P1 capacity (unit capacity) and conductivity matrices."""
    g, vol = p1_gradients(coords, tets)
    Mloc = vol[:, None, None] * (np.ones((4, 4)) + np.eye(4))[None] / 20.0
    Kloc = vol[:, None, None] * np.einsum("eai,ij,ebj->eab", g, np.asarray(kmat, float), g)
    nv = len(coords)
    return _assemble(tets, Mloc, 1, nv), _assemble(tets, Kloc, 1, nv)


def strain_operator(g):
    """B [ne, 4, 6, 3]: engineering strain [11, 22, 33, 2*12, 2*23, 2*31] of a unit
    displacement of vertex a in direction d."""
    ne = len(g)
    B = np.zeros((ne, 4, 6, 3))
    B[:, :, 0, 0] = g[:, :, 0]
    B[:, :, 1, 1] = g[:, :, 1]
    B[:, :, 2, 2] = g[:, :, 2]
    B[:, :, 3, 0] = g[:, :, 1]
    B[:, :, 3, 1] = g[:, :, 0]
    B[:, :, 4, 1] = g[:, :, 2]
    B[:, :, 4, 2] = g[:, :, 1]
    B[:, :, 5, 0] = g[:, :, 2]
    B[:, :, 5, 2] = g[:, :, 0]
    return B


def elastic_matrix(coords, tets, Cvoigt):
    """Stiffness of linear elements with a Voigt stiffness [ne, 6, 6] per tet."""
    g, vol = p1_gradients(coords, tets)
    B = strain_operator(g)
    Kloc = vol[:, None, None, None, None] * np.einsum("eaip,eij,ebjq->eapbq", B, Cvoigt, B)
    return _assemble(tets, Kloc.reshape(len(tets), 12, 12), 3, len(coords))


def solve_dirichlet(A, b, fixed, values):
    """x with x[fixed] = values[fixed] and (A x - b)[free] = 0."""
    x = np.array(values, dtype=float)
    free = ~fixed
    rhs = b[free] - A[free][:, fixed] @ x[fixed]
    x[free] = spla.spsolve(A[free][:, free].tocsc(), rhs)
    return x


def run(rve, nx, ny, nz, lx=1.0, ly=1.0, lz=0.25, heat_capacity=1.0, T0=20.0, c0=0.0, T_top=60.0, c_top=1.5,
        dt_years=10.0 / 365.25, steps=10, strain_x=1e-3, factors=None, c_sat=1.5, gauss=None):
    """FE^2 steps; returns T, c [steps + 1, nv], keep [steps, ngp], reaction [steps],
    u [nv, 3] and C_bar [ngp, 6, 6] of the last step.  `gauss` (default: rve)
    gives C_bar at the Gauss points, e.g. a surrogate model; the transport
    coefficients always come from rve."""
    gauss = rve if gauss is None else gauss
    fac = np.ones(8) if factors is None else np.asarray(factors, float)
    coords, tets = box_mesh(nx, ny, nz, lx, ly, lz)
    nv, ne = len(coords), len(tets)
    top = np.isclose(coords[:, 2], lz)
    hom0 = rve(np.r_[20.0, 0.0, 0.0, fac])
    M, Kt = scalar_matrices(coords, tets, hom0["K"])
    _, Kc = scalar_matrices(coords, tets, hom0["D"])
    At = (heat_capacity / dt_years) * M + Kt
    Ac = (1.0 / dt_years) * M + Kc
    T = np.full(nv, float(T0))
    c = np.full(nv, float(c0))
    Ts, cs = [T.copy()], [c.copy()]
    fixed_u = np.zeros(3 * nv, dtype=bool)
    val_u = np.zeros(3 * nv)
    on_x0, on_x1 = np.isclose(coords[:, 0], 0.0), np.isclose(coords[:, 0], lx)
    fixed_u[3 * np.flatnonzero(on_x0 | on_x1)] = True
    val_u[3 * np.flatnonzero(on_x1)] = strain_x * lx
    fixed_u[3 * np.flatnonzero(np.isclose(coords[:, 1], 0.0)) + 1] = True
    fixed_u[3 * np.flatnonzero(np.isclose(coords[:, 2], 0.0)) + 2] = True
    keep = np.ones(ne)
    keeps, reactions = [], []
    u = Cs = None
    for _ in range(steps):
        T = solve_dirichlet(At, (heat_capacity / dt_years) * (M @ T), top, np.where(top, T_top, T))
        c = solve_dirichlet(Ac, (1.0 / dt_years) * (M @ c), top, np.where(top, c_top, c))
        Ts.append(T.copy())
        cs.append(c.copy())
        Tg = T[tets].mean(axis=1)
        cg = c[tets].mean(axis=1)
        keep = materials.damage_history(Tg[None, :], cg[None, :], [dt_years], keep0=keep, c_sat=c_sat)[0]
        keeps.append(keep.copy())
        t_eq = materials.equivalent_exposure_years(keep)
        Cs = np.array([gauss(np.r_[60.0, c_sat, t_eq[e], fac])["C"] for e in range(ne)])
        Ku = elastic_matrix(coords, tets, Cs)
        u = solve_dirichlet(Ku, np.zeros(3 * nv), fixed_u, val_u)
        reactions.append(float((Ku @ u)[3 * np.flatnonzero(on_x1)].sum()))
    return dict(T=np.array(Ts), c=np.array(cs), keep=np.array(keeps), reaction=np.array(reactions),
                u=u.reshape(nv, 3), C_bar=Cs, coords=coords, tets=tets)
