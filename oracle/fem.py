"""RVE problem of Sec. 2 solved exactly on the P_p Lagrange space (oracle).

Unknowns are the total micro displacement u (or field psi), not the
fluctuation.  The constraints are written in the unified form of Eqs.
eq_RVE_disc_Eqs / eq_mat_C_and_D,

    [K  C^T] [u     ]   [ 0           ]
    [C  0  ] [lambda] = [ D * eps_bar ],

with one choice of rows per boundary condition (the paper does not print its
H matrices; any rows spanning the same constraint set give the same answer):

  * linear Dirichlet (Sec. 2, item 1): one row per boundary node and component,
    u_b = X(y_b) eps_bar;
  * periodic (Sec. 2, item 2): per class of boundary nodes that coincide modulo
    the cell, u_s - u_m = (X(y_s) - X(y_m)) eps_bar for every non-master node,
    plus u = X(y) eps_bar at the lower corner to remove the translations;
  * uniform traction (Sec. 2, item 3): the 9 surface rows
    int_dOmega u_i n_j dS = int_dOmega (X eps_bar)_i n_j dS (their symmetric part
    is the kinematic form of t = sigma_bar n; the skew part removes rotations)
    and the 3 volume rows int_Omega u_i dV = int_Omega (X eps_bar)_i dV.

X is the matrix of Eq. eq_X_mech with its columns taken in the Voigt order of
the text ([11,22,33,12,23,31], engineering shear):
    X(y) = [[y1, 0, 0, y2/2, 0, y3/2], [0, y2, 0, y1/2, y3/2, 0], [0, 0, y3, 0, y2/2, y1/2]].
For the scalar problems (Eq. eq_X_psi) the linear field is y . grad(psi), so X is
the row [y1, y2, y3].

The system is factorised once (SuperLU) and solved for all load cases, as in
the text after Eq. Eq_C_stress.  Homogenised stress: testing the first block
row with the interpolant x_k of the linear field (C x_k = D e_k exactly) gives
V sigma_bar . e_k = x_k^T K u = -(D e_k)^T lambda, so sigma_bar = -D^T lambda / V
for the system exactly as printed (the paper prints +D^T lambda / V for its own
sign of lambda).  Columns of C_bar are the stresses of the six unit strains
(Eq. Eq_C_stress); K_bar and D_bar likewise from unit gradients (Eq.
eq_homo_flux).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import lagrange, materials as mats

BC_DIRICHLET, BC_PERIODIC, BC_NEUMANN = 0, 1, 2
BC_NAMES = {BC_DIRICHLET: "dirichlet", BC_PERIODIC: "periodic", BC_NEUMANN: "neumann"}


def X_mech(y):
    y = np.asarray(y, float)
    X = np.zeros(y.shape[:-1] + (3, 6))
    X[..., 0, 0] = y[..., 0]
    X[..., 1, 1] = y[..., 1]
    X[..., 2, 2] = y[..., 2]
    X[..., 0, 3] = 0.5 * y[..., 1]
    X[..., 1, 3] = 0.5 * y[..., 0]
    X[..., 1, 4] = 0.5 * y[..., 2]
    X[..., 2, 4] = 0.5 * y[..., 1]
    X[..., 0, 5] = 0.5 * y[..., 2]
    X[..., 2, 5] = 0.5 * y[..., 0]
    return X


def X_scalar(y):
    y = np.asarray(y, float)
    return y[..., None, :]          # [.., 1, 3]


class Discretisation:
    """Global P_p Lagrange nodes, element maps and geometry of a tet mesh."""

    def __init__(self, coords, tets, p):
        coords = np.asarray(coords, float)
        tets = np.asarray(tets, np.int64)
        self.p = p
        self.coords = coords
        self.tets = tets
        ref = lagrange.reference_tables(p)
        self.ref = ref
        alphas = ref["nodes"]
        nn = len(alphas)
        T = len(tets)
        # --- global node numbering: a node is identified by its support vertices
        # and their multiplicities, which two tets sharing it agree on.
        keymap = {}
        e2n = np.empty((T, nn), dtype=np.int64)
        node_xyz = []
        for e in range(T):
            tv = tets[e]
            for a, al in enumerate(alphas):
                key = tuple(sorted((int(tv[i]), int(al[i])) for i in range(4) if al[i]))
                idx = keymap.get(key)
                if idx is None:
                    idx = len(keymap)
                    keymap[key] = idx
                    node_xyz.append(sum(al[i] * coords[tv[i]] for i in range(4) if al[i]) / p)
                e2n[e, a] = idx
        self.e2n = e2n
        self.nodes = np.array(node_xyz)
        self.n_nodes = len(keymap)
        # --- geometry: gradients of barycentric coordinates and volumes
        x = coords[tets]                                  # [T, 4, 3]
        M = np.ones((T, 4, 4))
        M[:, :3, :] = np.transpose(x, (0, 2, 1))
        Minv = np.linalg.inv(M)                           # lam = Minv @ [x; 1]
        self.grad = Minv[:, :, :3]                        # [T, 4(i), 3(k)]
        self.vol = np.abs(np.linalg.det(M)) / 6.0
        self.V = float(self.vol.sum())
        self.centroid = x.mean(axis=1)
        # --- boundary faces (faces used by exactly one tet)
        faces = []
        for o in range(4):
            others = [i for i in range(4) if i != o]
            faces.append(np.sort(tets[:, others], axis=1))
        faces = np.stack(faces, axis=1).reshape(-1, 3)    # index e*4 + o
        _, inv, cnt = np.unique(faces, axis=0, return_inverse=True, return_counts=True)
        bmask = cnt[inv.ravel()] == 1
        bidx = np.nonzero(bmask)[0]
        self.bface_elem = bidx // 4
        self.bface_opp = bidx % 4
        fa, fn = [], []
        for e, o in zip(self.bface_elem, self.bface_opp):
            others = [i for i in range(4) if i != o]
            xa, xb, xc = x[e, others[0]], x[e, others[1]], x[e, others[2]]
            nrm = np.cross(xb - xa, xc - xa)
            area = 0.5 * np.linalg.norm(nrm)
            nrm = nrm / np.linalg.norm(nrm)
            if np.dot(x[e, o] - xa, nrm) > 0:
                nrm = -nrm
            fa.append(area)
            fn.append(nrm)
        self.bface_area = np.array(fa)
        self.bface_normal = np.array(fn).reshape(-1, 3)
        self.bface_centroid = np.array([
            x[e, [i for i in range(4) if i != o]].mean(axis=0)
            for e, o in zip(self.bface_elem, self.bface_opp)]).reshape(-1, 3)
        bnodes = set()
        for e, o in zip(self.bface_elem, self.bface_opp):
            for a, al in enumerate(alphas):
                if al[o] == 0:
                    bnodes.add(int(e2n[e, a]))
        self.boundary_nodes = np.array(sorted(bnodes), dtype=np.int64)

    # ------------------------------------------------------------ assembly
    def stiffness_scalar(self, kmat):
        """Sparse K_psi = sum_e int grad(phi)^T k_e grad(phi) dV (CSR)."""
        g = self.grad
        Q = np.einsum("eik,ekl,ejl->eij", g, kmat, g)
        Ke = self.vol[:, None, None] * np.einsum("eij,ijab->eab", Q, self.ref["S"])
        nn = Ke.shape[1]
        rows = np.repeat(self.e2n, nn, axis=1).ravel()
        cols = np.tile(self.e2n, (1, nn)).ravel()
        N = self.n_nodes
        return sp.coo_matrix((Ke.ravel(), (rows, cols)), shape=(N, N)).tocsr()

    def stiffness_mech(self, Cvoigt):
        """Sparse K = sum_e int B^T C_e B dV, DOF index 3*node + component (CSR)."""
        g = self.grad
        Ct = np.stack([mats.voigt_to_tensor(C) for C in Cvoigt])     # [T,3,3,3,3]
        Q = np.einsum("eik,eckdl,ejl->eijcd", g, Ct, g)
        Ke = self.vol[:, None, None, None, None] * np.einsum("ijab,eijcd->eacbd", self.ref["S"], Q)
        T, nn = self.e2n.shape
        Ke = Ke.reshape(T, 3 * nn, 3 * nn)
        dof = (3 * self.e2n[:, :, None] + np.arange(3)[None, None, :]).reshape(T, 3 * nn)
        rows = np.repeat(dof, 3 * nn, axis=1).ravel()
        cols = np.tile(dof, (1, 3 * nn)).ravel()
        N = 3 * self.n_nodes
        return sp.coo_matrix((Ke.ravel(), (rows, cols)), shape=(N, N)).tocsr()

    # ------------------------------------------------------------ constraints
    def periodic_classes(self, lo, hi, tol=1e-9):
        """(slave, master) pairs of boundary nodes equal modulo the cell, and the corner node."""
        lo = np.asarray(lo, float)
        hi = np.asarray(hi, float)
        y = self.nodes[self.boundary_nodes]
        w = y.copy()
        for k in range(3):
            w[np.abs(y[:, k] - hi[k]) < tol, k] = lo[k]
        keys = np.round((w - lo) / tol).astype(np.int64)
        groups = {}
        for node, key, on_hi in zip(self.boundary_nodes, map(tuple, keys),
                                    np.any(np.abs(y - hi) < tol, axis=1)):
            groups.setdefault(key, []).append((bool(on_hi), int(node)))
        pairs = []
        for members in groups.values():
            masters = [nd for hi_side, nd in members if not hi_side]
            if len(masters) != 1:
                raise ValueError("periodic class without a unique master node")
            m = masters[0]
            pairs.extend((nd, m) for hi_side, nd in members if hi_side)
        corner = int(self.boundary_nodes[np.argmin(np.linalg.norm(y - lo, axis=1))])
        return pairs, corner

    def constraints(self, bc, ncomp, lo=(0, 0, 0), hi=(1, 1, 1)):
        """Sparse constraint rows C [m, ncomp*N] and right sides D [m, ncase]."""
        Xf = X_mech if ncomp == 3 else X_scalar
        N = self.n_nodes
        rows, cols, vals, Drows = [], [], [], []

        def add_row(entries, drow):
            r = len(Drows)
            for c, v in entries:
                rows.append(r)
                cols.append(c)
                vals.append(v)
            Drows.append(drow)

        if bc == BC_DIRICHLET:
            for b in self.boundary_nodes:
                Xb = Xf(self.nodes[b])
                for c in range(ncomp):
                    add_row([(ncomp * b + c, 1.0)], Xb[c])
        elif bc == BC_PERIODIC:
            pairs, corner = self.periodic_classes(lo, hi)
            for s, m in pairs:
                dX = Xf(self.nodes[s]) - Xf(self.nodes[m])
                for c in range(ncomp):
                    add_row([(ncomp * s + c, 1.0), (ncomp * m + c, -1.0)], dX[c])
            Xc = Xf(self.nodes[corner])
            for c in range(ncomp):
                add_row([(ncomp * corner + c, 1.0)], Xc[c])
        elif bc == BC_NEUMANN:
            F = self.ref["F"]
            W = self.ref["W"]
            nn = self.e2n.shape[1]
            # surface moments int_dOmega phi_a n_j dS per node
            surf = np.zeros((N, 3))
            for e, o, A, nrm in zip(self.bface_elem, self.bface_opp, self.bface_area, self.bface_normal):
                for a in range(nn):
                    if F[o, a] != 0.0:
                        surf[self.e2n[e, a]] += A * F[o, a] * nrm
            volm = np.zeros(N)
            np.add.at(volm, self.e2n.ravel(), (self.vol[:, None] * W[None, :]).ravel())
            # right sides from the linear field (exact: it is linear on every face/tet)
            Xs = Xf(self.bface_centroid)                       # [nf, ncomp, ncase]
            Xv = Xf(self.centroid)
            nz = np.nonzero(np.any(surf != 0.0, axis=1))[0]
            for c in range(ncomp):
                for j in range(3):
                    drow = np.einsum("f,f,fk->k", self.bface_area, self.bface_normal[:, j], Xs[:, c, :])
                    add_row([(ncomp * a + c, surf[a, j]) for a in nz], drow)
            for c in range(ncomp):
                drow = np.einsum("e,ek->k", self.vol, Xv[:, c, :])
                add_row([(ncomp * a + c, volm[a]) for a in range(N)], drow)
        else:
            raise ValueError("unknown boundary condition")
        m = len(Drows)
        C = sp.coo_matrix((vals, (rows, cols)), shape=(m, ncomp * N)).tocsr()
        return C, np.array(Drows)

    # ------------------------------------------------------------ averages
    def grad_integrals(self, u, ncomp):
        """int_e grad(u) dV per element: [T, ncomp, 3] for each column of u [ncomp*N, ncase]."""
        Wd = self.ref["Wd"]                                   # [4, nn]
        ug = u.reshape(self.n_nodes, ncomp, -1)[self.e2n]     # [T, nn, ncomp, ncase]
        # int d(u_c)/dx_k = vol * sum_a sum_i Wd[i,a] g[e,i,k] u[a,c]
        return self.vol[:, None, None, None] * np.einsum("ia,eik,eacq->eckq", Wd, self.grad, ug)


def _voigt_strain(gint):
    """Engineering-shear Voigt vector from integrated displacement gradients [.., 3, 3(k), q]."""
    G = gint
    return np.stack([G[:, 0, 0], G[:, 1, 1], G[:, 2, 2],
                     G[:, 0, 1] + G[:, 1, 0], G[:, 1, 2] + G[:, 2, 1], G[:, 2, 0] + G[:, 0, 2]], axis=1)


def solve_rve(disc: Discretisation, physics_tensor, bc, ncomp, lo=(0, 0, 0), hi=(1, 1, 1)):
    """Solve the saddle-point system for all unit load cases.

    physics_tensor: per-element Voigt stiffness [T,6,6] (ncomp = 3) or conductivity [T,3,3] (ncomp = 1).
    Returns dict with the homogenised matrix from the multipliers ('hom'), from the
    volume average ('hom_vol'), from the energy ('hom_energy'), and the solution.
    """
    if ncomp == 3:
        K = disc.stiffness_mech(physics_tensor)
    else:
        K = disc.stiffness_scalar(physics_tensor)
    C, D = disc.constraints(bc, ncomp, lo, hi)
    n = K.shape[0]
    m = C.shape[0]
    A = sp.bmat([[K, C.T], [C, None]], format="csc")
    ncase = D.shape[1]
    rhs = np.zeros((n + m, ncase))
    rhs[n:] = D
    lu = spla.splu(A, permc_spec="MMD_AT_PLUS_A")           # factorised once
    sol = lu.solve(rhs)                                      # all load cases
    u, lam = sol[:n], sol[n:]
    V = disc.V
    hom = -(D.T @ lam) / V
    gint = disc.grad_integrals(u, ncomp)                     # [T, ncomp, 3, ncase]
    if ncomp == 3:
        eps = _voigt_strain(gint)                            # [T, 6, ncase]
        hom_vol = np.einsum("eij,ejq->iq", physics_tensor, eps) / V
    else:
        hom_vol = np.einsum("eij,ejq->iq", physics_tensor, gint[:, 0]) / V
    hom_energy = (u.T @ (K @ u)) / V
    return dict(hom=hom, hom_vol=hom_vol, hom_energy=hom_energy, u=u, lam=lam, K=K, C=C, D=D)


def nested_dissection(xyz, adj, leaf=48):
    """Fill-reducing elimination order (a permutation of the nodes) by geometric
    nested dissection: split at the median of the widest coordinate, take the
    left nodes coupled to the right half as the separator, recurse, order the
    separator last.  Wrap-around couplings of a periodic cell land in the
    separator too.  Only the factorisation cost depends on it, not the result.
    """
    parts = []

    def split(S):
        if S.size <= leaf:
            parts.append(S)
            return
        ax = int(np.argmax(xyz[S].max(axis=0) - xyz[S].min(axis=0)))
        med = np.median(xyz[S, ax])
        L, R = S[xyz[S, ax] < med], S[xyz[S, ax] >= med]
        if L.size == 0 or R.size == 0:
            parts.append(S)
            return
        on_sep = np.diff(adj[L][:, R].indptr) > 0
        split(L[~on_sep])
        split(R)
        parts.append(L[on_sep])

    split(np.arange(xyz.shape[0]))
    return np.concatenate(parts)


def solve_rve_substituted(disc: Discretisation, physics_tensor, bc, ncomp, lo=(0, 0, 0), hi=(1, 1, 1)):
    """Same discrete problem as solve_rve for the Dirichlet and periodic conditions,
    with the constraints eliminated by substitution instead of multipliers.

    Sec. 2 states that condensing the constrained DOFs and adding multipliers are two
    routes to one constrained system.  Here u = P w + g per load case: Dirichlet
    nodes take u = X(y) eps_bar; a periodic slave takes its master's value plus
    (X(y_s) - X(y_m)) eps_bar, and the lower corner's class is fixed to the linear
    field.  The reduced matrix P^T K P is SPD and factorised once; the homogenised
    matrix is the volume average of the fluxes (equal to the multiplier route,
    which this form has no multipliers for).
    """
    if bc not in (BC_DIRICHLET, BC_PERIODIC):
        raise ValueError("substitution is only written for the Dirichlet and periodic conditions")
    Xf = X_mech if ncomp == 3 else X_scalar
    K = disc.stiffness_mech(physics_tensor) if ncomp == 3 else disc.stiffness_scalar(physics_tensor)
    N = disc.n_nodes
    ncase = 6 if ncomp == 3 else 3
    rep = np.arange(N)                        # node whose unknowns a node copies
    fixed = np.zeros(N, dtype=bool)           # nodes whose value is prescribed outright
    g = np.zeros((N, ncomp, ncase))           # prescribed part of u per node
    if bc == BC_DIRICHLET:
        b = disc.boundary_nodes
        fixed[b] = True
        g[b] = Xf(disc.nodes[b])
    else:
        pairs, corner = disc.periodic_classes(lo, hi)
        for s, m in pairs:
            rep[s] = m
            g[s] = Xf(disc.nodes[s]) - Xf(disc.nodes[m])
        fixed[corner] = True
        g[corner] = Xf(disc.nodes[corner])
        for s, m in pairs:                    # slaves of the corner: linear field outright
            if m == corner:
                fixed[s] = True
                g[s] = Xf(disc.nodes[s])
    free_nodes = np.nonzero((rep == np.arange(N)) & ~fixed)[0]
    col_of = -np.ones(N, dtype=np.int64)
    col_of[free_nodes] = np.arange(free_nodes.size)
    node_col = np.where(fixed, -1, col_of[rep])
    rows = (ncomp * np.arange(N)[:, None] + np.arange(ncomp)[None, :])[node_col >= 0].ravel()
    cols = (ncomp * node_col[:, None] + np.arange(ncomp)[None, :])[node_col >= 0].ravel()
    P = sp.csr_matrix((np.ones(rows.size), (rows, cols)), shape=(ncomp * N, ncomp * free_nodes.size))
    G = g.reshape(ncomp * N, ncase)
    Kr = (P.T @ K @ P).tocsr()
    # fill-reducing order: nested dissection of the free nodes' coupling graph
    sel = np.nonzero(node_col >= 0)[0]
    Pn = sp.csr_matrix((np.ones(sel.size), (sel, node_col[sel])), shape=(N, free_nodes.size))
    T, nn = disc.e2n.shape
    E2 = sp.csr_matrix((np.ones(T * nn), (np.repeat(np.arange(T), nn), disc.e2n.ravel())), shape=(T, N))
    adj = (Pn.T @ (E2.T @ E2) @ Pn).tocsr()
    order = nested_dissection(disc.nodes[free_nodes], adj)
    perm = (ncomp * order[:, None] + np.arange(ncomp)[None, :]).ravel()
    lu = spla.splu(Kr[perm][:, perm].tocsc(), permc_spec="NATURAL", diag_pivot_thresh=0.0,
                   options=dict(SymmetricMode=True))
    rhs = -(P.T @ (K @ G))
    w = np.empty_like(rhs)
    w[perm] = lu.solve(rhs[perm])
    u = P @ w + G
    V = disc.V
    gint = disc.grad_integrals(u, ncomp)
    if ncomp == 3:
        hom_vol = np.einsum("eij,ejq->iq", physics_tensor, _voigt_strain(gint)) / V
    else:
        hom_vol = np.einsum("eij,ejq->iq", physics_tensor, gint[:, 0]) / V
    hom_energy = (u.T @ (K @ u)) / V
    return dict(hom=hom_vol, hom_vol=hom_vol, hom_energy=hom_energy, u=u, K=K)


def voigt_reuss(disc: Discretisation, tensors):
    w = disc.vol / disc.V
    upper = np.einsum("e,eij->ij", w, tensors)
    lower = np.linalg.inv(np.einsum("e,eij->ij", w, np.linalg.inv(tensors)))
    return upper, lower


def homogenise(coords, tets, phase, axis, p, bc, base, params=None, c_sat=1.5,
               degrade_yarn=False, lo=(0, 0, 0), hi=(1, 1, 1), disc=None, physics=("mech", "thermal", "moisture"),
               method="multipliers"):
    """C_bar (6x6), K_bar (3x3), D_bar (3x3) of one RVE and one parameter record.

    method: "multipliers" (the bordered system, every BC) or "substitution"
    (Dirichlet and periodic only; the same discrete solution, cheaper to factorise).
    """
    solve = solve_rve if method == "multipliers" else solve_rve_substituted
    disc = disc or Discretisation(coords, tets, p)
    m, y, keep = mats.phase_materials(base, params, c_sat, degrade_yarn)
    Ce, Ke, De = mats.element_tensors(phase, axis, m, y)
    out = {"omega_keep": keep}
    if "mech" in physics:
        out["C"] = solve(disc, Ce, bc, 3, lo, hi)["hom"]
    if "thermal" in physics:
        out["K"] = solve(disc, Ke, bc, 1, lo, hi)["hom"]
    if "moisture" in physics:
        out["D"] = solve(disc, De, bc, 1, lo, hi)["hom"]
    return out
