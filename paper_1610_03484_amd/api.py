"""Python binding of the C ABI (same names; marshalling only).

Device memory and streams come from PyTorch; every arithmetic step of the
homogenisation runs in libchom's HIP kernels.
"""
from __future__ import annotations

import ctypes as ct

import numpy as np

from . import _lib as L


def default_options(**kw) -> L.ChomOptions:
    o = L.ChomOptions()
    L.check(L.lib().chom_default_options(ct.byref(o)), "chom_default_options")
    if "precision" in kw and isinstance(kw["precision"], str):
        kw["precision"] = L.PRECISION[kw["precision"]]
    if "precond" in kw and isinstance(kw["precond"], str):
        kw["precond"] = L.PRECOND[kw["precond"]]
    for k, v in kw.items():
        if k == "hip_stream":
            v = ct.c_void_p(v)
        setattr(o, k, v)
    return o


def materials_struct(m: dict) -> L.ChomMaterials:
    s = L.ChomMaterials()
    for k, _ in L.ChomMaterials._fields_:
        setattr(s, k, float(m[k]))
    return s


def params_array(p: np.ndarray):
    p = np.ascontiguousarray(np.asarray(p, dtype=np.float64).reshape(-1, 11))
    arr = (L.ChomParams * len(p))()
    ct.memmove(arr, p.ctypes.data, p.nbytes)
    return arr


def mesh_sizes(n: int):
    nv, nt = ct.c_int32(), ct.c_int32()
    L.check(L.lib().chom_mesh_sizes(n, ct.byref(nv), ct.byref(nt)), "chom_mesh_sizes")
    return nv.value, nt.value


def generate_plain_weave(n: int, device="cuda"):
    """Device tensors (coords [V,3] f64, tets [T,4] i32, phase [T] i8, axis [T,3] f64)."""
    import torch
    nv, nt = mesh_sizes(n)
    coords = torch.empty((nv, 3), dtype=torch.float64, device=device)
    tets = torch.empty((nt, 4), dtype=torch.int32, device=device)
    phase = torch.empty((nt,), dtype=torch.int8, device=device)
    axis = torch.empty((nt, 3), dtype=torch.float64, device=device)
    stream = torch.cuda.current_stream(coords.device).cuda_stream
    L.check(L.lib().chom_generate_plain_weave(n, ct.c_void_p(coords.data_ptr()), ct.c_void_p(tets.data_ptr()),
                                              ct.c_void_p(phase.data_ptr()), ct.c_void_p(axis.data_ptr()),
                                              ct.c_void_p(stream)), "chom_generate_plain_weave")
    return coords, tets, phase, axis


def material_constants(materials: dict, params=None, c_sat=1.5, degrade_yarn=0):
    """Host-only: (mech[10], therm[4], moist[4], omega_keep) as the kernels use them."""
    m = materials_struct(materials)
    mech = (ct.c_double * 10)()
    th = (ct.c_double * 4)()
    mo = (ct.c_double * 4)()
    keep = ct.c_double()
    pp = None
    if params is not None:
        pp = params_array(params)
    L.check(L.lib().chom_material_constants(ct.byref(m), pp, c_sat, degrade_yarn, mech, th, mo, ct.byref(keep)),
            "chom_material_constants")
    return np.array(mech[:]), np.array(th[:]), np.array(mo[:]), keep.value


def yarn_directions(coords, tets, phase, yarn_axis=(0, 0, 1, 1), rtol=1e-12, max_iter=20000,
                    lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0)):
    """chom_yarn_directions: fibre axes [n_tets, 3] from the potential-flow solve of
    every yarn.  coords/tets/phase: all torch device tensors (result on the device)
    or all numpy arrays (result in host memory)."""
    mesh = L.ChomMesh()
    dev = hasattr(coords, "is_cuda") and coords.is_cuda
    if dev:
        import torch
        arrs = [coords.contiguous(), tets.contiguous(), phase.contiguous()]
        ptrs = [a.data_ptr() for a in arrs]
        out = torch.empty((arrs[1].shape[0], 3), dtype=torch.float64, device=coords.device)
        optr = out.data_ptr()
        stream = torch.cuda.current_stream(coords.device).cuda_stream
    else:
        arrs = [np.ascontiguousarray(coords, np.float64), np.ascontiguousarray(tets, np.int32),
                np.ascontiguousarray(phase, np.int8)]
        ptrs = [a.ctypes.data for a in arrs]
        out = np.zeros((arrs[1].shape[0], 3))
        optr = out.ctypes.data
        stream = None
    mesh.n_vertices, mesh.n_tets = arrs[0].shape[0], arrs[1].shape[0]
    mesh.coords, mesh.tets, mesh.phase = ptrs
    mesh.fibre_axis = None
    mesh.lo[:] = lo
    mesh.hi[:] = hi
    mesh.on_device = int(dev)
    ax = (ct.c_int32 * len(yarn_axis))(*yarn_axis)
    L.check(L.lib().chom_yarn_directions(ct.byref(mesh), len(yarn_axis), ax, rtol, max_iter, ct.c_void_p(optr),
                                         ct.c_void_p(stream) if stream else None), "chom_yarn_directions")
    return out


def damage_history(T_celsius, c_wt, dt_years, keep0=None, factors=None, c_sat=1.5, keep=True, params=True,
                   hip_stream=None):
    """chom_damage_history.  T_celsius, c_wt [m, n] (step-major), dt_years [m], keep0 [n],
    factors [n, 8]: all numpy arrays (host) or all contiguous torch device tensors
    (float64).  Returns (keep [m, n] or None, params [n, 11] or None) in the same
    kind of memory."""
    dev = hasattr(T_celsius, "data_ptr")
    m, n = T_celsius.shape
    if dev:
        import torch
        mk = lambda *s: torch.empty(s, dtype=torch.float64, device=T_celsius.device)
        conv = lambda a: a
        if hip_stream is None:
            hip_stream = torch.cuda.current_stream(T_celsius.device).cuda_stream
    else:
        mk = lambda *s: np.zeros(s)
        conv = lambda a: None if a is None else np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    T, c, dt, k0, f = (conv(a) for a in (T_celsius, c_wt, dt_years, keep0, factors))
    out_keep = mk(m, n) if keep else None
    out_par = mk(n, 11) if params else None
    L.check(L.lib().chom_damage_history(n, m, _ptr(T), _ptr(c), _ptr(dt), _ptr(k0), _ptr(f), c_sat, int(dev),
                                        ct.c_void_p(hip_stream) if hip_stream else None, _ptr(out_keep),
                                        _ptr(out_par)), "chom_damage_history")
    return out_keep, out_par


def fe2_run(rve, nx, ny, nz, lx=1.0, ly=1.0, lz=0.25, heat_capacity=1.0, T0=20.0, c0=0.0, T_top=60.0,
            c_top=1.5, dt_years=10.0 / 365.25, steps=10, strain_x=1e-3, macro_rtol=1e-10, macro_max_iter=20000,
            factors=None, surrogate=None, surrogate_thresh=1e-2, allow_noconv=False):
    """chom_fe2_run on an RVE handle (with `surrogate`, a Surrogate whose
    predictions replace the RVE solves, the RVE as fallback).  Returns a dict of
    numpy arrays: T, c [steps + 1, nv], keep [steps, ngp], reaction [steps],
    u [nv, 3] and C_bar [ngp, 21] of the last step, macro_iters [3],
    n_fallback, status."""
    nv = (nx + 1) * (ny + 1) * (nz + 1)
    ngp = 6 * nx * ny * nz
    fac = None if factors is None else np.ascontiguousarray(np.asarray(factors, dtype=np.float64).reshape(8))
    P = L.ChomFe2Problem(nx, ny, nz, lx, ly, lz, heat_capacity, T0, c0, T_top, c_top, dt_years, steps, strain_x,
                         macro_rtol, macro_max_iter, _ptr(fac), surrogate._h if surrogate is not None else None,
                         surrogate_thresh)
    res = dict(T=np.zeros((steps + 1, nv)), c=np.zeros((steps + 1, nv)), keep=np.zeros((steps, ngp)),
               reaction=np.zeros(steps), u=np.zeros((nv, 3)), C_bar=np.zeros((ngp, 21)))
    O = L.ChomFe2Output(*(_ptr(res[k]) for k in ("T", "c", "keep", "reaction", "u", "C_bar")))
    st = L.lib().chom_fe2_run(rve._h, ct.byref(P), ct.byref(O))
    if not (st == L.CHOM_OK or (allow_noconv and st == L.CHOM_ENOCONV)):
        L.check(st, "chom_fe2_run")
    res["macro_iters"] = list(O.macro_iters)
    res["n_fallback"] = int(O.n_fallback)
    res["status"] = st
    return res


class RVE:
    """Handle of chom_rve_create; homogenise() wraps chom_homogenise."""

    def __init__(self, coords, tets, phase, axis, materials: dict, bc="periodic", order=2,
                 lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), **options):
        self._h = ct.c_void_p()
        self.options = default_options(**options)
        mesh = L.ChomMesh()
        keep = []
        if hasattr(coords, "is_cuda") and coords.is_cuda:
            arrs = [coords.contiguous(), tets.contiguous(), phase.contiguous(), axis.contiguous()]
            keep = arrs
            mesh.on_device = 1
            ptrs = [a.data_ptr() for a in arrs]
            nv, nt = arrs[0].shape[0], arrs[1].shape[0]
        else:
            arrs = [np.ascontiguousarray(coords, np.float64), np.ascontiguousarray(tets, np.int32),
                    np.ascontiguousarray(phase, np.int8), np.ascontiguousarray(axis, np.float64)]
            keep = arrs
            mesh.on_device = 0
            ptrs = [a.ctypes.data for a in arrs]
            nv, nt = arrs[0].shape[0], arrs[1].shape[0]
        mesh.n_vertices, mesh.n_tets = nv, nt
        self.n = int(round((nt / 6) ** (1.0 / 3.0)))
        mesh.coords, mesh.tets, mesh.phase, mesh.fibre_axis = ptrs
        mesh.lo[:] = lo
        mesh.hi[:] = hi
        bc_id = L.BC[bc] if isinstance(bc, str) else int(bc)
        self.bc = bc_id
        self.materials = dict(materials)
        st = L.lib().chom_rve_create(ct.byref(mesh), ct.byref(materials_struct(materials)), bc_id, order,
                                     ct.byref(self.options), ct.byref(self._h))
        del keep
        L.check(st, "chom_rve_create")

    def homogenise(self, params, allow_noconv=False):
        """params [B, 11] -> (C21 [B,21], K6 [B,6], D6 [B,6], reports list)."""
        p = np.asarray(params, dtype=np.float64).reshape(-1, 11)
        B = len(p)
        C = np.zeros((B, 21))
        K = np.zeros((B, 6))
        D = np.zeros((B, 6))
        reps = (L.ChomReport * B)()
        st = L.lib().chom_homogenise(self._h, params_array(p), B, ct.c_void_p(C.ctypes.data),
                                     ct.c_void_p(K.ctypes.data), ct.c_void_p(D.ctypes.data), reps)
        if not (st == L.CHOM_OK or (allow_noconv and st == L.CHOM_ENOCONV)):
            L.check(st, "chom_homogenise")
        return C, K, D, [report_dict(r) for r in reps]

    def time_operator(self, physics=0, reps=50):
        """(ms per launch, tets per launch, problems per launch) of the operator kernel."""
        ms = ct.c_double()
        nt = ct.c_int64()
        npb = ct.c_int32()
        L.check(L.lib().chom_time_operator(self._h, physics, reps, ct.byref(ms), ct.byref(nt), ct.byref(npb)),
                "chom_time_operator")
        return ms.value, nt.value, npb.value

    def close(self):
        if self._h:
            L.lib().chom_rve_destroy(self._h)
            self._h = ct.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class URVE:
    """Handle of chom_urve_create (any conforming tet mesh of the box [lo, hi]);
    homogenise() wraps chom_urve_homogenise.  Host (numpy) mesh arrays."""

    def __init__(self, coords, tets, phase, axis, materials: dict, bc="periodic", lo=(0.0, 0.0, 0.0),
                 hi=(1.0, 1.0, 1.0), **options):
        self._h = ct.c_void_p()
        options.setdefault("precision", "fp64")
        self.options = default_options(**options)
        arrs = [np.ascontiguousarray(coords, np.float64), np.ascontiguousarray(tets, np.int32),
                np.ascontiguousarray(phase, np.int8), np.ascontiguousarray(axis, np.float64)]
        mesh = L.ChomMesh()
        mesh.on_device = 0
        mesh.n_vertices, mesh.n_tets = arrs[0].shape[0], arrs[1].shape[0]
        mesh.coords, mesh.tets, mesh.phase, mesh.fibre_axis = [a.ctypes.data for a in arrs]
        mesh.lo[:] = lo
        mesh.hi[:] = hi
        self.bc = L.BC[bc] if isinstance(bc, str) else int(bc)
        st = L.lib().chom_urve_create(ct.byref(mesh), ct.byref(materials_struct(materials)), self.bc,
                                      ct.byref(self.options), ct.byref(self._h))
        del arrs
        L.check(st, "chom_urve_create")

    def sizes(self):
        nn, nu = ct.c_int64(), ct.c_int64()
        L.check(L.lib().chom_urve_sizes(self._h, ct.byref(nn), ct.byref(nu)), "chom_urve_sizes")
        return nn.value, nu.value

    def homogenise(self, params, allow_noconv=False):
        """params [B, 11] -> (C21 [B,21], K6 [B,6], D6 [B,6], reports list)."""
        p = np.asarray(params, dtype=np.float64).reshape(-1, 11)
        B = len(p)
        C = np.zeros((B, 21))
        K = np.zeros((B, 6))
        D = np.zeros((B, 6))
        reps = (L.ChomReport * B)()
        st = L.lib().chom_urve_homogenise(self._h, params_array(p), B, ct.c_void_p(C.ctypes.data),
                                          ct.c_void_p(K.ctypes.data), ct.c_void_p(D.ctypes.data), reps)
        if not (st == L.CHOM_OK or (allow_noconv and st == L.CHOM_ENOCONV)):
            L.check(st, "chom_urve_homogenise")
        return C, K, D, [report_dict(r) for r in reps]

    def close(self):
        if self._h:
            L.lib().chom_urve_destroy(self._h)
            self._h = ct.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def tag_plain_weave(coords, tets):
    """chom_tag_plain_weave on host arrays: (phase [nt] int8, fibre_axis [nt, 3])."""
    c = np.ascontiguousarray(coords, np.float64)
    t = np.ascontiguousarray(tets, np.int32)
    ph = np.zeros(len(t), np.int8)
    ax = np.zeros((len(t), 3))
    L.check(L.lib().chom_tag_plain_weave(c.ctypes.data, len(c), t.ctypes.data, len(t), 0, ph.ctypes.data,
                                         ax.ctypes.data), "chom_tag_plain_weave")
    return ph, ax


def report_dict(r: L.ChomReport) -> dict:
    return dict(iters=list(r.iters), refine_steps=list(r.refine_steps), status=r.status,
                resid=list(r.resid), asym=r.asym, omega_keep=r.omega_keep, fail=list(r.fail),
                fp64_fallback=list(r.fp64_fallback), spd=r.spd, hill_mandel_gap=r.hill_mandel_gap)


def upper21_to_matrix(c21):
    """Upper-triangle vector (row-major) -> symmetric 6x6 (mirror of the upper triangle)."""
    c21 = np.asarray(c21)
    M = np.zeros(c21.shape[:-1] + (6, 6))
    iu = np.triu_indices(6)
    M[..., iu[0], iu[1]] = c21
    M[..., iu[1], iu[0]] = c21
    return M


def upper6_to_matrix(k6):
    k6 = np.asarray(k6)
    M = np.zeros(k6.shape[:-1] + (3, 3))
    idx = [(0, 0), (1, 1), (2, 2), (0, 1), (1, 2), (0, 2)]
    for q, (i, j) in enumerate(idx):
        M[..., i, j] = k6[..., q]
        M[..., j, i] = k6[..., q]
    return M


class Batch:
    """Handle of chom_batch_create: item i is homogenised on rves[i] (handles may repeat)."""

    def __init__(self, rves, **options):
        self._rves = list(rves)                # keep the handles alive
        self._h = ct.c_void_p()
        arr = (ct.c_void_p * len(self._rves))(*[r._h.value for r in self._rves])
        opt = default_options(**options) if options else self._rves[0].options
        self.options = opt
        L.check(L.lib().chom_batch_create(arr, len(self._rves), ct.byref(opt), ct.byref(self._h)),
                "chom_batch_create")

    def __len__(self):
        return len(self._rves)

    def homogenise(self, params, allow_noconv=False):
        """params [n, 11] -> (C21 [n,21], K6 [n,6], D6 [n,6], reports)."""
        p = np.asarray(params, dtype=np.float64).reshape(-1, 11)
        n = len(self._rves)
        if len(p) != n:
            raise ValueError(f"need {n} parameter records, got {len(p)}")
        C = np.zeros((n, 21))
        K = np.zeros((n, 6))
        D = np.zeros((n, 6))
        reps = (L.ChomReport * n)()
        st = L.lib().chom_batch_homogenise(self._h, params_array(p), ct.c_void_p(C.ctypes.data),
                                           ct.c_void_p(K.ctypes.data), ct.c_void_p(D.ctypes.data), reps)
        if not (st == L.CHOM_OK or (allow_noconv and st == L.CHOM_ENOCONV)):
            L.check(st, "chom_batch_homogenise")
        return C, K, D, [report_dict(r) for r in reps]

    def launch_config(self):
        v = [ct.c_int32() for _ in range(4)]
        L.check(L.lib().chom_batch_launch_config(self._h, *[ct.byref(x) for x in v]), "chom_batch_launch_config")
        return dict(rg_mech=v[0].value, rg_scal=v[1].value, nwg_mech=v[2].value, nwg_scal=v[3].value)

    def time_operator(self, physics=0, reps=50):
        ms = ct.c_double()
        nt = ct.c_int64()
        npb = ct.c_int32()
        L.check(L.lib().chom_batch_time_operator(self._h, physics, reps, ct.byref(ms), ct.byref(nt), ct.byref(npb)),
                "chom_batch_time_operator")
        return ms.value, nt.value, npb.value

    def close(self):
        if self._h:
            L.lib().chom_batch_destroy(self._h)
            self._h = ct.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mlp_default_options(**kw) -> L.ChomMlpOptions:
    o = L.ChomMlpOptions()
    L.check(L.lib().chom_mlp_default_options(ct.byref(o)), "chom_mlp_default_options")
    for k, v in kw.items():
        setattr(o, k, ct.c_void_p(v) if k == "hip_stream" else v)
    return o


def mlp_train_options(**kw) -> L.ChomMlpTrainOptions:
    o = L.ChomMlpTrainOptions()
    L.check(L.lib().chom_mlp_default_train_options(ct.byref(o)), "chom_mlp_default_train_options")
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def _ptr(x):
    """Data pointer of a torch tensor (device convention) or a C-contiguous numpy array (host)."""
    if x is None:
        return None
    if hasattr(x, "data_ptr"):
        if not x.is_contiguous():
            raise ValueError("tensor arguments must be contiguous")
        return ct.c_void_p(x.data_ptr())
    if not x.flags["C_CONTIGUOUS"]:
        raise ValueError("array arguments must be C-contiguous")
    return ct.c_void_p(x.ctypes.data)


class Surrogate:
    """Handle of chom_mlp_create: an ensemble of networks mapping parameter records to
    C_hom, K_hom, D_hom (see include/chom.h).  With device=True the bulk arrays are
    torch device tensors (float64, contiguous); otherwise numpy arrays."""

    def __init__(self, members=5, seed=0, c_sat=1.5, device=False, hip_stream=None):
        self.device = bool(device)
        opt = mlp_default_options(members=members, seed=seed, c_sat=c_sat, device_ptrs=int(self.device))
        if hip_stream is not None:
            opt.hip_stream = ct.c_void_p(hip_stream)
        self._h = ct.c_void_p()
        L.check(L.lib().chom_mlp_create(ct.byref(opt), ct.byref(self._h)), "chom_mlp_create")
        self.members = members

    def sizes(self):
        p, m = ct.c_int64(), ct.c_int32()
        L.check(L.lib().chom_mlp_sizes(self._h, ct.byref(p), ct.byref(m)), "chom_mlp_sizes")
        return p.value, m.value

    def set_weights(self, member, flat):
        w = np.ascontiguousarray(np.asarray(flat, dtype=np.float32))
        if w.size != self.sizes()[0]:
            raise ValueError("wrong number of weights")
        L.check(L.lib().chom_mlp_set_weights(self._h, member, _ptr(w)), "chom_mlp_set_weights")

    def get_weights(self, member):
        w = np.zeros(self.sizes()[0], dtype=np.float32)
        L.check(L.lib().chom_mlp_get_weights(self._h, member, _ptr(w)), "chom_mlp_get_weights")
        return w

    def set_normalisation(self, rec):
        r = np.ascontiguousarray(np.asarray(rec, dtype=np.float64))
        if r.size != 92:
            raise ValueError("the standardisation record has 92 numbers")
        L.check(L.lib().chom_mlp_set_normalisation(self._h, _ptr(r)), "chom_mlp_set_normalisation")

    def get_normalisation(self):
        r = np.zeros(92)
        L.check(L.lib().chom_mlp_get_normalisation(self._h, _ptr(r)), "chom_mlp_get_normalisation")
        return r

    def _bulk(self, p, C=None, K=None, D=None):
        if self.device:
            return p, C, K, D
        cv = lambda a, w: None if a is None else np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(-1, w))
        return cv(p, 11), cv(C, 21), cv(K, 6), cv(D, 6)

    def train(self, params, C, K, D, **train_opts):
        """Train every member; returns the loss history [members, epochs]."""
        p, C, K, D = self._bulk(params, C, K, D)
        n = len(p)
        o = mlp_train_options(**train_opts)
        hist = np.zeros((self.members, o.epochs), dtype=np.float32)
        L.check(L.lib().chom_mlp_train(self._h, _ptr(p), _ptr(C), _ptr(K), _ptr(D), n, ct.byref(o), _ptr(hist)),
                "chom_mlp_train")
        return hist

    def loss_grad(self, member, params, C, K, D):
        p, C, K, D = self._bulk(params, C, K, D)
        loss = ct.c_double()
        g = np.zeros(self.sizes()[0], dtype=np.float32)
        L.check(L.lib().chom_mlp_loss_grad(self._h, member, _ptr(p), _ptr(C), _ptr(K), _ptr(D), len(p),
                                           ct.byref(loss), _ptr(g)), "chom_mlp_loss_grad")
        return loss.value, g

    def loss_grad_noalloc(self, member, params, C, K, D, loss, grad):
        """chom_mlp_loss_grad_noalloc: every argument a contiguous torch device tensor
        (params [n,11], C [n,21], K [n,6], D [n,6] float64; loss [1] float64 and
        grad [143652] float32 written)."""
        n = params.shape[0]
        L.check(L.lib().chom_mlp_loss_grad_noalloc(self._h, member, _ptr(params), _ptr(C), _ptr(K), _ptr(D), n,
                                                   _ptr(loss), _ptr(grad)), "chom_mlp_loss_grad_noalloc")

    def _outputs(self, n):
        if self.device:
            import torch
            mk = lambda *s: torch.empty(s, dtype=torch.float64, device="cuda")
            return mk(n, 21), mk(n, 6), mk(n, 6), mk(n)
        return np.zeros((n, 21)), np.zeros((n, 6)), np.zeros((n, 6)), np.zeros(n)

    def predict(self, params):
        """(C21, K6, D6, disagreement) of the ensemble mean."""
        p = self._bulk(params)[0]
        n = len(p)
        C, K, D, dis = self._outputs(n)
        L.check(L.lib().chom_mlp_predict(self._h, _ptr(p), n, _ptr(C), _ptr(K), _ptr(D), _ptr(dis)),
                "chom_mlp_predict")
        return C, K, D, dis

    def homogenise(self, rve, params, thresh=1e-2, chunk=0, allow_noconv=False):
        """Surrogate with RVE fallback: (C21, K6, D6, disagreement, used_fallback, n_fallback)."""
        p = self._bulk(params)[0]
        n = len(p)
        C, K, D, dis = self._outputs(n)
        if self.device:
            import torch
            used = torch.empty(n, dtype=torch.uint8, device="cuda")
        else:
            used = np.zeros(n, dtype=np.uint8)
        nfb = ct.c_int64()
        st = L.lib().chom_homogenise_surrogate(self._h, rve._h, _ptr(p), n, thresh, chunk, _ptr(C), _ptr(K),
                                               _ptr(D), _ptr(dis), _ptr(used), ct.byref(nfb))
        if not (st == L.CHOM_OK or (allow_noconv and st == L.CHOM_ENOCONV)):
            L.check(st, "chom_homogenise_surrogate")
        return C, K, D, dis, used, nfb.value

    def close(self):
        if self._h:
            L.lib().chom_mlp_destroy(self._h)
            self._h = ct.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
