#!/usr/bin/env python
"""Benchmark: RVE homogenisations per second on one MI355X, plain vs batched vs surrogate.

Default workload ("c2"): 512 parameter records, one per macro Gauss point, each
on a synthetic plain-weave RVE whose size is drawn uniformly from
{8, 12, 16, 20, 24}^3 cells, order-2 hierarchic basis, periodic conditions,
degraded by the paper's law at T ~ U(20, 60) C, c ~ U(0, 1.5) wt%,
t ~ U(0, 10) years with seeded property factors; 6 mechanical + 3 thermal + 3
moisture load cases each; FP32 operator with FP64 reductions, projection,
refinement residual and averages.  One step = the whole batch in one
chom_batch_homogenise call (`value`).  Meshes, tags and element data are
resident on the GPU before timing starts.

Also measured, outside the timed region, into `config`:
  * plain GPU path: the same 512 records, one chom_homogenise call per record
    (same options), and the batched-over-plain speedup;
  * C0: the 8^3 linear-Dirichlet FP64 RVE, one call per record, with its error
    against a fresh oracle solve;
  * accuracy of the batch: items solved by the CPU oracle in this run (the 8^3
    items of the cpu_baseline sample), and one item of every size against the
    FP64 GPU path at rtol 1e-12 (labelled as such); relative Frobenius,
    largest-entry and energy-weighted errors;
  * surrogate (unless --no-surrogate): the ensemble trained on 12^3 solves, run
    on 1,000,000 records with fallback, its held-out error against stored
    oracle solves and its speedup over the plain and batched paths;
  * the damage-history kernel (time-varying exposure) on 1,000,000 points x
    100 steps, against the HBM peak;
  * the potential-flow yarn directions of the 24^3 RVE: time per call and the
    change of C_bar against the analytic centreline tangent;
  * the FE^2 outer loop on an 8 x 8 x 2 macro box (768 Gauss points, an 8^3
    RVE solve at each per step): time per macro step;
  * an RVE on a general (unstructured) tet mesh of 8,748 tets: time per
    homogenisation against the lattice path's 12^3 RVE;
  * roofline of the dominant kernel (the FP32 mechanical operator on the batch),
    from HIP events on the library's stream.
`cpu_baseline`: the oracle on host cores, on the 8^3 records of the batch.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c2|c1|c0|c3|c4|umesh|fe2]
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK = 8.0e12          # B/s, MI355X HBM3E
FP32_VEC_PEAK = 157.3e12   # flop/s, MI355X FP32 vector (published)
FP64_VEC_PEAK = 78.6e12
METRIC = "RVE homogenisations/s (12 load cases) @ stated C_hom error: plain vs batched vs MLP"

WORKLOADS = {
    "c2": dict(n=None, bcs=("periodic",), precision="fp32_refined",
               desc="512 RVEs (one per macro Gauss point) with sizes uniform over {8,12,16,20,24}^3 cells, "
                    "p=2, periodic, degraded (T~U(20,60) C, c~U(0,1.5) wt%, t~U(0,10) y, factors U(0.9,1.1)), "
                    "12 load cases each, FP32 operator + FP64 refinement, one batched call"),
    "c1": dict(n=24, bcs=("dirichlet", "periodic", "neumann"), precision="fp32_refined",
               desc="24^3 Kuhn plain-weave RVE (82,944 tets), p=2 (352,947 elastic DOFs), "
                    "Dirichlet+periodic+Neumann in one batch, 6+3+3 load cases each, FP32 operator + FP64 refinement"),
    "c0": dict(n=8, bcs=("dirichlet",), precision="fp64",
               desc="8^3 Kuhn plain-weave RVE (3,072 tets), p=2, linear Dirichlet, 6+3+3 load cases, FP64"),
    "c4": dict(n=12, bcs=("periodic",), precision="fp32_refined",
               desc="learned surrogate: 5-member ensemble of 10->256->256->256->36 GELU networks (BF16 MFMA, "
                    "FP32 accumulate) trained on 12^3 plain-weave RVE solves (p=2, periodic, degraded records "
                    "as in the batched workload), evaluated on 1,000,000 records with RVE fallback where the "
                    "ensemble disagreement exceeds 1e-2"),
    "umesh": dict(n=None, bcs=("periodic",), precision="fp64",
                  desc="general (unstructured) tet mesh: 9^3-cell box with a vertex per cell, 8,748 tets, synthetic "
                       "weave tags, periodic, FP64 PCG with point-block Jacobi, 12 load cases, sixteen degraded records "
                       "per call"),
    "fe2": dict(n=8, bcs=("periodic",), precision="fp32_refined",
                desc="FE^2 outer loop: 8 x 8 x 2 macro box (768 Gauss points), 8^3 periodic RVE solve per Gauss point "
                     "and step (FP32 operator + FP64 refinement), four implicit steps of 0.25 years"),
    "c3": dict(n=16, bcs=("periodic",), precision="fp32_refined",
               desc="p-refinement: batch of 16^3 Kuhn plain-weave RVEs (24,576 tets each) at order p (3: 352,947, "
                    "4: 823,875 elastic DOFs), periodic, degraded records as in the batched workload, element "
                    "operator on the FP32 matrix cores with FP64 refinement"),
}


# ---------------------------------------------------------------- algorithmic counts
def algorithmic_mech(n, nprob, fp32):
    """Bytes and flops of one mechanical operator launch (6 load cases) per problem:
    bytes = sum_RHS 2 ndof s + T (conn + n_A s), flops = T n_RHS 2 n_e^2, with
    conn = 40 B, n_A = 45, n_e = 30 at p = 2 (the dense element-block contraction)."""
    s = 4 if fp32 else 8
    T = 6 * n ** 3
    ndof = 3 * (2 * n + 1) ** 3
    bytes_ = 6 * 2 * ndof * s + T * (40 + 45 * s)
    flops = T * 6 * 2 * 30 ** 2
    return bytes_ * nprob, flops * nprob


def algorithmic_mech_order(n, p, nprob, fp32):
    """As algorithmic_mech at order p = 3, 4: n_e = 3 (p+1)(p+2)(p+3)/6 elastic element
    DOFs, conn = 60 / 64 B, n_A = 45, ndof = 3 (p n + 1)^3."""
    s = 4 if fp32 else 8
    T = 6 * n ** 3
    ne = 3 * (p + 1) * (p + 2) * (p + 3) // 6
    ndof = 3 * (p * n + 1) ** 3
    conn = 60 if p == 3 else 64
    bytes_ = 6 * 2 * ndof * s + T * (conn + 45 * s)
    flops = T * 6 * 2 * ne ** 2
    return bytes_ * nprob, flops * nprob


# HBM traffic of one all-active launch of op_p2_kernel<float,3,6,RG>, rocprofv3
# FETCH_SIZE + WRITE_SIZE scaled by the calibration copy, per workload and load-case
# grouping RG (profiles/op_p2_mech_fp32_*_traffic.md).  Must be re-measured (or the
# entry removed) whenever that kernel changes.
OP_TRAFFIC_BYTES = {
    "c1": {1: 124257650, 2: 128732682, 3: 108221564},
    "c2": {1: 7952610802, 2: 8208382168, 3: 7050862621},
}

# VALU wave-instructions of one all-active launch of op_p2_kernel<float,3,6,2> on the
# mixed batch (rocprofv3 SQ_INSTS_VALU, profiles/op_p2_mech_fp32_512_mixed_valu.md);
# re-measure (or remove) whenever that kernel changes.
OP_VALU_INSTS = {"c2": {2: 1.71849e9}}
SIMDS, CLOCK_HZ = 1024, 2.4e9

CAL_BYTES = 256 << 20


def calibration_copy(torch):
    """Three device-to-device copies of 256 MiB (outside the timed region): the plain
    copy of known size against which rocprofv3's FETCH_SIZE / WRITE_SIZE are scaled."""
    x = torch.ones(CAL_BYTES // 4, dtype=torch.float32, device="cuda:0")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    del x, y


# ---------------------------------------------------------------- errors
def _full6(c21):
    M = np.zeros((6, 6))
    M[np.triu_indices(6)] = c21
    return M + np.triu(M, 1).T


def _full3(k6):
    a = np.asarray(k6)
    return np.array([[a[0], a[3], a[5]], [a[3], a[1], a[4]], [a[5], a[4], a[2]]])


def result_errors(got, ref):
    """(relative Frobenius, largest entry / ||ref||_F, energy-weighted ||ref^-1/2 d ref^-1/2||_2),
    each the largest over the C, K, D blocks; got, ref: 33-vectors (C upper 21, K 6, D 6)."""
    out = np.zeros(3)
    for sl, full in ((slice(0, 21), _full6), (slice(21, 27), _full3), (slice(27, 33), _full3)):
        g, r = full(got[sl]), full(ref[sl])
        d = g - r
        w, V = np.linalg.eigh(r)
        h = V @ np.diag(w ** -0.5) @ V.T
        e = [np.linalg.norm(d) / np.linalg.norm(r), np.abs(d).max() / np.linalg.norm(r),
             np.abs(np.linalg.eigvalsh(h @ d @ h)).max()]
        out = np.maximum(out, e)
    return [float(v) for v in out]


def block_errors(pred, truth):
    """Per record, the largest over the C, K, D blocks of ||pred - truth||_F / ||truth||_F
    (full symmetric matrices: off-diagonal entries of the stored upper triangles count twice)."""
    w = np.array([1.0 if a == b else 2.0 for a in range(6) for b in range(a, 6)] + [1, 1, 1, 2, 2, 2] * 2)
    err = np.zeros(len(pred))
    for blk in (slice(0, 21), slice(21, 27), slice(27, 33)):
        num = np.sqrt((w[blk] * (pred[:, blk] - truth[:, blk]) ** 2).sum(axis=1))
        den = np.sqrt((w[blk] * truth[:, blk] ** 2).sum(axis=1))
        err = np.maximum(err, num / den)
    return err


def _stack(C, K, D):
    return np.concatenate([np.asarray(C), np.asarray(K), np.asarray(D)], axis=1)


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# ---------------------------------------------------------------- CPU oracle (host cores)
ORACLE_WORKER = r"""
import json, os, sys, time
sys.path.insert(0, {root!r})
import numpy as np
import chom_inputs as ci
from oracle import fem, mesh
n, bc, method = {n}, {bc}, {method!r}
recs = np.array(json.loads(sys.argv[1]))
c, t, ph, ax = mesh.plain_weave(n)
disc = fem.Discretisation(c, t, 2)
iu = np.triu_indices(6)
sym3 = [(0, 0), (1, 1), (2, 2), (0, 1), (1, 2), (0, 2)]
out = []
for p in recs:
    t0 = time.perf_counter()
    r = fem.homogenise(c, t, ph, ax, 2, bc, ci.BASE_MATERIALS, p, disc=disc, method=method)
    v = list(r["C"][iu]) + [r["K"][a, b] for a, b in sym3] + [r["D"][a, b] for a, b in sym3]
    out.append(dict(seconds=time.perf_counter() - t0, result=[float(x) for x in v]))
print(json.dumps(out))
"""


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def oracle_pool(n, bc, method, records, workers, timeout=900):
    """Solve `records` on the n^3 RVE with the CPU oracle in `workers` processes
    (one thread each; one record list per process).  Returns (results [k, 33],
    per-record seconds, wall seconds)."""
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1",
               CUDA_VISIBLE_DEVICES="", HIP_VISIBLE_DEVICES="")
    code = ORACLE_WORKER.format(root=ROOT, n=n, bc=bc, method=method)
    chunks = [records[i::workers] for i in range(workers)]
    t0 = time.perf_counter()
    procs = [subprocess.Popen([sys.executable, "-c", code, json.dumps(np.asarray(ch).tolist())],
                              stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True, env=env)
             for ch in chunks if len(ch)]
    outs = [p.communicate(timeout=timeout) for p in procs]
    wall = time.perf_counter() - t0
    res = [None] * len(records)
    secs = [None] * len(records)
    for w, (p, (so, se)) in enumerate(zip(procs, outs)):
        if p.returncode != 0:
            raise RuntimeError(f"oracle worker failed: {se[-2000:]}")
        for j, rec in enumerate(json.loads(so.strip().splitlines()[-1])):
            res[w + j * workers] = rec["result"]
            secs[w + j * workers] = rec["seconds"]
    return np.array(res), np.array(secs), wall


# ---------------------------------------------------------------- workloads
def bench_opts(args, precision):
    return dict(precision=precision, rtol=args.rtol, inner_rtol=args.inner_rtol, max_iter=50000,
                precond=args.precond)


def make_c2(args, torch):
    import chom_inputs as ci
    from paper_1610_03484_amd import RVE, generate_plain_weave
    sizes = ci.batch_sizes_c2(0, args.items)
    params = ci.draw_params(0, args.items)
    handles = {}
    for n_i in sorted(set(int(s) for s in sizes)):
        handles[n_i] = RVE(*generate_plain_weave(n_i, device="cuda:0"), ci.BASE_MATERIALS, bc="periodic",
                           **bench_opts(args, "fp32_refined"))
    rves = [handles[int(s)] for s in sizes]
    return sizes, params, handles, rves


def time_batch(batch, params, steps, warmup, torch):
    for _ in range(warmup):
        batch.homogenise(params)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        res = batch.homogenise(params)
    torch.cuda.synchronize()
    return time.perf_counter() - t0, res


def plain_path(handles, sizes, params, torch):
    """One chom_homogenise call per record on the record's own RVE handle (a warm-up
    call per size first): the plain GPU path on the same records."""
    first = {}
    for i, s in enumerate(sizes):
        first.setdefault(int(s), i)
    for s, i in first.items():
        handles[s].homogenise(params[i:i + 1])
    torch.cuda.synchronize()
    out = np.zeros((len(sizes), 33))
    t0 = time.perf_counter()
    for i, s in enumerate(sizes):
        C, K, D, _ = handles[int(s)].homogenise(params[i:i + 1])
        out[i] = _stack(C, K, D)[0]
    torch.cuda.synchronize()
    return time.perf_counter() - t0, out


def roofline_mech(batch, sizes_or_n, nprob_items, fp32, args, workload, order=2):
    ms, tets, nprob = batch.time_operator(0, args.op_reps)
    rg = batch.launch_config()["rg_mech"]
    if order != 2:
        bytes_, flops = algorithmic_mech_order(sizes_or_n, order, nprob, fp32)
    elif isinstance(sizes_or_n, (list, tuple, np.ndarray)):
        bytes_ = flops = 0
        for s_ in sizes_or_n:
            b1, f1 = algorithmic_mech(int(s_), 1, fp32)
            bytes_ += b1
            flops += f1
    else:
        bytes_, flops = algorithmic_mech(sizes_or_n, nprob, fp32)
    t = ms * 1e-3
    peak_alu = FP32_VEC_PEAK if fp32 else FP64_VEC_PEAK
    traffic = OP_TRAFFIC_BYTES.get(workload, {}).get(rg) if (fp32 and order == 2) else None
    if order != 2:
        roof = dict(bound="mfma", achieved=flops / t / 1e12, peak=FP32_VEC_PEAK / 1e12, unit="TFLOP/s",
                    frac=(flops / t) / FP32_VEC_PEAK, traffic=None,
                    note="FP32 matrix-core peak (157.3 TFLOP/s dense, equal to the packed FP32 vector peak)")
        kname = f"hp_op_kernel<float,{order},3,6,8>"
    elif flops / peak_alu >= bytes_ / HBM_PEAK:
        roof = dict(bound="alu", achieved=flops / t / 1e12, peak=peak_alu / 1e12, unit="TFLOP/s",
                    frac=(flops / t) / peak_alu, traffic=traffic)
        kname = f"op_p2_kernel<{'float' if fp32 else 'double'},3,6,{rg}>"
    else:
        roof = dict(bound="hbm", achieved=bytes_ / t / 1e9, peak=HBM_PEAK / 1e9, unit="GB/s",
                    frac=(bytes_ / t) / HBM_PEAK, traffic=traffic)
        kname = f"op_p2_kernel<{'float' if fp32 else 'double'},3,6,{rg}>"
    roof.update(kernel=kname, avg_launch_us=ms * 1e3, algorithmic_bytes=bytes_, algorithmic_flops=flops,
                hbm_frac=(bytes_ / t) / HBM_PEAK, problems_per_launch=nprob)
    valu = OP_VALU_INSTS.get(workload, {}).get(rg) if (fp32 and order == 2) else None
    if valu:
        # measured issue: a wave64 VALU instruction holds a SIMD for 4 cycles
        roof.update(valu_issue_frac=valu * 4 / (t * CLOCK_HZ * SIMDS),
                    valu_note="measured VALU issue against 1,024 SIMDs at 2.4 GHz; the kernel is issue bound, "
                              "the gap to frac 0.5 of the packed-FP32 peak is the dense-element flop count's "
                              "(packed FP32 is disabled at compile time)")
    log(f"operator: {ms * 1e3:.1f} us/launch, {bytes_ / t / 1e9:.0f} GB/s algorithmic, "
        f"{flops / t / 1e12:.2f} TFLOP/s algorithmic")
    return roof


def damage_history_kernel(torch):
    """chom_damage_history on 1,000,000 points x 100 steps (device arrays): per launch
    16 B read (T, c) and 8 B written per point and step."""
    import chom_inputs as ci
    from paper_1610_03484_amd import damage_history
    n, m = 1_000_000, 100
    u = torch.tensor(ci.uniform_block(71, 0, 2 * 4096), device="cuda:0")
    T = (20.0 + 40.0 * u[:4096]).repeat(m * n // 4096 + 1)[: m * n].reshape(m, n).contiguous()
    c = (1.5 * u[4096:]).repeat(m * n // 4096 + 1)[: m * n].reshape(m, n).contiguous()
    dt = torch.full((m,), 0.1, dtype=torch.float64, device="cuda:0")
    for _ in range(2):
        damage_history(T, c, dt, keep=True, params=False)
    torch.cuda.synchronize()
    reps = 5
    t0 = time.perf_counter()
    for _ in range(reps):
        damage_history(T, c, dt, keep=True, params=False)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / reps
    bytes_ = 24.0 * n * m
    del T, c
    return dict(points=n, steps=m, ms_per_call=t * 1e3, achieved_GBps=bytes_ / t / 1e9,
                hbm_frac=bytes_ / t / HBM_PEAK, bound="hbm",
                note="host-timed call (one kernel launch plus a 4-byte status read)")


def yarn_directions_leg(args, torch):
    """Potential-flow fibre directions of the 24^3 plain weave (four yarns, P1, FP64 CG):
    time per call, and the change of C_bar against the analytic centreline tangent."""
    import chom_inputs as ci
    from paper_1610_03484_amd import RVE, generate_plain_weave, yarn_directions
    coords, tets, phase, tangent = generate_plain_weave(24, device="cuda:0")
    yarn_directions(coords, tets, phase, (0, 0, 1, 1), rtol=1e-10)
    torch.cuda.synchronize()
    reps = 5
    t0 = time.perf_counter()
    for _ in range(reps):
        axis = yarn_directions(coords, tets, phase, (0, 0, 1, 1), rtol=1e-10)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / reps * 1e3
    y = phase > 0
    ang = torch.rad2deg(torch.arccos(torch.clamp((axis[y] * tangent[y]).sum(dim=1).abs(), max=1.0)))
    params = ci.draw_factors_only(0, 1)
    out = []
    for ax in (tangent, axis):
        rve = RVE(coords, tets, phase, ax, ci.BASE_MATERIALS, bc="periodic", precision="fp64", rtol=1e-12,
                  max_iter=50000)
        C, K, D, _ = rve.homogenise(params)
        rve.close()
        out.append(_stack(C, K, D)[0])
    e = result_errors(out[1], out[0])
    return dict(rve="24^3 plain weave, 4 yarns, 12,624 yarn tets", ms_per_call=ms,
                mean_angle_to_tangent_deg=float(ang.mean()), max_angle_to_tangent_deg=float(ang.max()),
                c_hom_change_vs_tangent=dict(fro=e[0], energy=e[2]),
                note="host-timed call: stencil assembly, one CG workgroup per yarn, per-tet gradients")


def fe2_leg(args, torch):
    """The FE^2 outer loop on an 8 x 8 x 2 macro box (768 Gauss points, one 8^3 periodic
    RVE solve each per step, FP32 operator + FP64 refinement), four implicit steps of
    0.25 years with the top face at 60 C and 1.5 wt%: time per macro step (transport,
    damage, 768 RVE solves, macro elasticity)."""
    import chom_inputs as ci
    from paper_1610_03484_amd import RVE, fe2_run, generate_plain_weave
    rve = RVE(*generate_plain_weave(8, device="cuda:0"), ci.BASE_MATERIALS, bc="periodic",
              **bench_opts(args, "fp32_refined"))
    box = dict(nx=8, ny=8, nz=2, lx=1.0, ly=1.0, lz=0.25, T0=20.0, c0=0.0, T_top=60.0, c_top=1.5,
               dt_years=0.25, strain_x=1e-3, macro_rtol=1e-10)
    fe2_run(rve, steps=1, **box)
    torch.cuda.synchronize()
    steps = 4
    t0 = time.perf_counter()
    g = fe2_run(rve, steps=steps, **box)
    dt = time.perf_counter() - t0
    rve.close()
    ngp = 6 * box["nx"] * box["ny"] * box["nz"]
    return dict(box="8x8x2 cells, 768 Gauss points (P1 Kuhn tets), 1.0 x 1.0 x 0.25",
                rve="8^3 plain weave, p=2, periodic, FP32 operator + FP64 refinement", steps=steps,
                dt_years=box["dt_years"], ms_per_macro_step=dt / steps * 1e3,
                rve_solves_per_s=ngp * steps / dt, macro_cg_iters=[int(v) for v in g["macro_iters"]],
                keep_range_last_step=[float(g["keep"][-1].min()), float(g["keep"][-1].max())],
                reaction=[float(v) for v in g["reaction"]],
                note="host-timed chom_fe2_run call (outputs copied to the host each step)")


def fe2_surrogate(rve, sur, torch):
    """The FE^2 box of the FE^2 leg on the 12^3 RVE: four macro steps with an RVE solve
    at every Gauss point, then with the trained ensemble (fallback threshold 1e-2)."""
    from paper_1610_03484_amd import fe2_run
    box = dict(nx=8, ny=8, nz=2, lx=1.0, ly=1.0, lz=0.25, T0=20.0, c0=0.0, T_top=60.0, c_top=1.5,
               dt_years=0.25, strain_x=1e-3, macro_rtol=1e-10)
    steps = 4
    out = {}
    for name, kw in (("rve", {}), ("surrogate", dict(surrogate=sur, surrogate_thresh=1e-2))):
        fe2_run(rve, steps=1, **box, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g = fe2_run(rve, steps=steps, **box, **kw)
        out[name] = (time.perf_counter() - t0) / steps * 1e3, g
    (t_rve, g_rve), (t_sur, g_sur) = out["rve"], out["surrogate"]
    rdiff = float(np.abs(g_sur["reaction"] / g_rve["reaction"] - 1.0).max())
    log(f"FE^2 12^3 RVE, 768 Gauss points: {t_rve:.1f} ms per macro step with RVE solves, {t_sur:.1f} ms with the "
        f"surrogate ({g_sur['n_fallback']} fallbacks), reactions {rdiff:.1e} apart")
    return dict(box="8x8x2 cells, 768 Gauss points", rve="12^3 plain weave, p=2, periodic, FP32 + FP64 refinement",
                steps=steps, ms_per_macro_step_rve=t_rve, ms_per_macro_step_surrogate=t_sur,
                speedup=t_rve / t_sur, fallbacks=int(g_sur["n_fallback"]), reaction_rel_diff=rdiff,
                note="host-timed chom_fe2_run calls")


def unstructured_leg(args, torch):
    """A general (unstructured) tet mesh of the paper's RVE size class: the 9 x 9 x 9
    cell box with a vertex per cell (8,748 tets, chom_inputs.unstructured_box), tagged
    by the synthetic weave on the GPU, periodic, FP64 PCG (point-block Jacobi) on the
    element-batched operator; time per homogenisation (12 load cases) over sixteen
    degraded records in one call (their load cases share every launch), against the
    lattice path's 12^3 RVE (10,368 tets) in FP64 with the same preconditioner and
    tolerance."""
    import chom_inputs as ci
    from paper_1610_03484_amd import RVE, URVE, generate_plain_weave, tag_plain_weave
    coords, tets = ci.unstructured_box(9, seed=0)
    phase, axis = tag_plain_weave(coords, tets)
    params = ci.draw_params(0, 16)
    u = URVE(coords, tets, phase, axis, ci.BASE_MATERIALS, bc="periodic", rtol=args.rtol, max_iter=50000)
    nn, nu = u.sizes()
    u.homogenise(params[:1])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, _, _, rep = u.homogenise(params)
    dt = (time.perf_counter() - t0) / len(params)
    u.close()
    lat = RVE(*generate_plain_weave(12, device="cuda:0"), ci.BASE_MATERIALS, bc="periodic", precision="fp64",
              precond="block_jacobi", rtol=args.rtol, max_iter=50000)
    lat.homogenise(params[:1])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, _, _, rep_l = lat.homogenise(params)
    dt_l = (time.perf_counter() - t0) / len(params)
    lat.close()
    its = [max(r["iters"][:6]) for r in rep]
    log(f"unstructured 8,748-tet periodic RVE: {dt * 1e3:.1f} ms per homogenisation (max mechanical CG steps "
        f"{max(its)}); lattice 12^3 FP64 block Jacobi {dt_l * 1e3:.1f} ms")
    return dict(mesh="unstructured box, 9^3 cells + a vertex per cell, 8,748 tets (seed 0), synthetic weave tags",
                p2_nodes=int(nn), free_nodes=int(nu), bc="periodic", precision="fp64", precond="block_jacobi",
                rtol=args.rtol, ms_per_homogenisation=dt * 1e3, rate=1.0 / dt, max_mech_cg_steps=int(max(its)),
                hill_mandel_gap_max=float(max(r["hill_mandel_gap"] for r in rep)),
                lattice_12cubed_fp64_block_jacobi_ms=dt_l * 1e3,
                lattice_12cubed_max_mech_cg_steps=int(max(max(r["iters"][:6]) for r in rep_l)),
                note="host-timed chom_urve_homogenise of 16 records (one chunk: every launch covers all their load "
                     "cases)")


def c0_plain(args, torch):
    """C0: 8^3 linear-Dirichlet FP64, one record per call; error against a fresh oracle solve."""
    import chom_inputs as ci
    from oracle import fem
    from paper_1610_03484_amd import RVE, generate_plain_weave
    params = ci.draw_factors_only(0, 1)
    rve = RVE(*generate_plain_weave(8, device="cuda:0"), ci.BASE_MATERIALS, bc="dirichlet", precision="fp64",
              rtol=1e-12, max_iter=50000)
    rve.homogenise(params)
    torch.cuda.synchronize()
    reps = 10
    t0 = time.perf_counter()
    for _ in range(reps):
        C, K, D, _ = rve.homogenise(params)
    torch.cuda.synchronize()
    rate = reps / (time.perf_counter() - t0)
    rve.close()
    ref, secs, _ = oracle_pool(8, fem.BC_DIRICHLET, "multipliers", params, 1)
    err = result_errors(_stack(C, K, D)[0], ref[0])
    return dict(rate=rate, err_vs_oracle=dict(fro=err[0], elem=err[1], energy=err[2]),
                oracle_seconds=float(secs[0]))


def surrogate_leg(args, torch, plain12_rate=None):
    """C4: train on 12^3 solves (outside timing), then the timed surrogate + fallback."""
    import chom_inputs as ci
    from paper_1610_03484_amd import RVE, Surrogate, generate_plain_weave
    n = 12
    rve = RVE(*generate_plain_weave(n, device="cuda:0"), ci.BASE_MATERIALS, bc="periodic",
              **bench_opts(args, "fp32_refined"))
    params = ci.draw_params(0, args.train)
    chunk = 512
    rve.homogenise(params[:chunk])
    t0 = time.perf_counter()
    parts = []
    for s0 in range(0, args.train, chunk):
        parts.append(rve.homogenise(params[s0:s0 + chunk])[:3])
        if (s0 // chunk) % 8 == 0:
            log(f"training solves {min(s0 + chunk, args.train)}/{args.train}")
    t_solve = time.perf_counter() - t0
    C = np.concatenate([q[0] for q in parts])
    K = np.concatenate([q[1] for q in parts])
    D = np.concatenate([q[2] for q in parts])
    batched12 = args.train / t_solve
    if plain12_rate is None:
        rve.homogenise(params[:1])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(32):
            rve.homogenise(params[i:i + 1])
        torch.cuda.synchronize()
        plain12_rate = 32 / (time.perf_counter() - t0)
    stream = torch.cuda.current_stream().cuda_stream
    sur = Surrogate(members=5, seed=11, device=True, hip_stream=stream)
    dev = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda:0")
    t0 = time.perf_counter()
    hist = sur.train(dev(params), dev(C), dev(K), dev(D), epochs=args.epochs, batch=256)
    t_train = time.perf_counter() - t0
    log(f"{args.train} solves in {t_solve:.1f} s ({batched12:.0f}/s); training {t_train:.1f} s, "
        f"final loss {hist[:, -1].mean():.2e}")
    pts = dev(ci.draw_params(3_000_000, args.points))
    sur.homogenise(rve, pts[:4096], thresh=1e-2, chunk=256)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, _, _, _, _, nfb = sur.homogenise(rve, pts, thresh=1e-2, chunk=256)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    rate = args.points / dt
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(5):
        sur.predict(pts)
    ev1.record()
    torch.cuda.synchronize()
    t_pred = ev0.elapsed_time(ev1) / 5 * 1e-3
    flops = 2 * (10 * 256 + 2 * 256 * 256 + 256 * 36) * 5 * args.points
    golden = os.path.join(ROOT, "tests", "golden", "surrogate_heldout_n12_periodic.txt")
    a = np.loadtxt(golden)
    hp, truth = a[:, 1:12], a[:, 12:45]
    Ch, Kh, Dh, _, _, nfbh = sur.homogenise(rve, dev(hp), thresh=1e-2, chunk=256)
    err = block_errors(_stack(Ch.cpu().numpy(), Kh.cpu().numpy(), Dh.cpu().numpy()), truth)
    Cp, Kp, Dp, _ = sur.predict(dev(hp))
    raw = block_errors(_stack(Cp.cpu().numpy(), Kp.cpu().numpy(), Dp.cpu().numpy()), truth)
    log(f"surrogate: {args.points} points in {dt:.2f} s ({rate:.3g}/s), {nfb} fallbacks; held-out max error "
        f"{err.max():.2e} (network alone {raw.max():.2e})")
    fe2 = None if args.no_fe2 else fe2_surrogate(rve, sur, torch)
    out = dict(rate=rate, points=args.points, fallbacks=int(nfb), training_solves=args.train,
               training_solve_s=t_solve, training_s=t_train, epochs=args.epochs,
               batched_rate_12cubed=batched12, plain_rate_12cubed=plain12_rate,
               speedup_vs_plain_12cubed=rate / plain12_rate, speedup_vs_batched_12cubed=rate / batched12,
               heldout_points=len(hp), heldout_reference="CPU FP64 oracle (stored)",
               heldout_max_err=float(err.max()), heldout_max_err_network_alone=float(raw.max()),
               heldout_fallbacks=int(nfbh),
               predict_kernel=dict(avg_launch_us=t_pred * 1e6, achieved_TFLOPs=flops / t_pred / 1e12,
                                   frac_bf16_peak=flops / t_pred / 2.5e15),
               fe2_outer_loop=fe2)
    sur.close()
    rve.close()
    return out


def run_c2(args, torch):
    import chom_inputs as ci
    from oracle import fem
    from paper_1610_03484_amd import RVE, Batch, generate_plain_weave
    wl = WORKLOADS["c2"]
    sizes, params, handles, rves = make_c2(args, torch)
    batch = Batch(rves)
    log(f"c2: {len(rves)} records, sizes {dict(zip(*np.unique(sizes, return_counts=True)))}")
    dt, (C, K, D, rep) = time_batch(batch, params, args.steps, args.warmup, torch)
    value = len(rves) * args.steps / dt
    launch = batch.launch_config()
    got = _stack(C, K, D)
    worst = max(range(len(rep)), key=lambda i: max(rep[i]["iters"]))
    log(f"batched: {value:.1f}/s; {sum(r['status'] == 0 for r in rep)}/{len(rep)} converged; max iters "
        f"{max(rep[worst]['iters'])} (item {worst}, n={sizes[worst]})")
    roof = roofline_mech(batch, list(sizes), len(rves), True, args, "c2")

    # ---- plain GPU path on the same records
    plain_rate, plain = None, None
    if not args.no_plain:
        t_plain, plain = plain_path(handles, sizes, params, torch)
        plain_rate = len(rves) / t_plain
        log(f"plain path (one record per call): {plain_rate:.1f}/s; batched/plain {value / plain_rate:.2f}")

    # ---- accuracy: FP64 GPU path (one item per size) and the oracle (8^3 items, with the cpu baseline)
    acc = {}
    if not args.no_accuracy:
        first = {}
        for i, s_ in enumerate(sizes):
            first.setdefault(int(s_), i)
        items = sorted(first.values())
        refs = [RVE(*generate_plain_weave(int(sizes[i]), device="cuda:0"), ci.BASE_MATERIALS, bc="periodic",
                    precision="fp64", rtol=1e-12, max_iter=50000) for i in items]
        rb = Batch(refs)
        Cr, Kr, Dr, _ = rb.homogenise(np.ascontiguousarray(params[items]))
        ref64 = _stack(Cr, Kr, Dr)
        e64 = np.array([result_errors(got[i], ref64[j]) for j, i in enumerate(items)])
        ep = (np.array([result_errors(plain[i], ref64[j]) for j, i in enumerate(items)]) if plain is not None
              else np.full((1, 3), np.nan))
        acc.update(vs_fp64_gpu=dict(items=items, sizes=[int(sizes[i]) for i in items],
                                    fro=float(e64[:, 0].max()), elem=float(e64[:, 1].max()),
                                    energy=float(e64[:, 2].max()), plain_path_fro=float(ep[:, 0].max()),
                                    plain_path_energy=float(ep[:, 2].max()),
                                    reference="FP64 GPU path at rtol 1e-12 (oracle-matched at 8^3 and 12^3 by tests)"))
        rb.close()
        for r in refs:
            r.close()
        log(f"batch vs FP64 GPU path: fro {e64[:, 0].max():.2e} energy {e64[:, 2].max():.2e}")

    # ---- C0 plain FP64
    c0 = None if args.no_c0 else c0_plain(args, torch)
    if c0:
        log(f"c0 plain FP64 8^3 Dirichlet: {c0['rate']:.1f}/s, error vs oracle {c0['err_vs_oracle']}")

    # ---- damage history kernel
    dmg = None
    if not args.no_damage:
        dmg = damage_history_kernel(torch)
        log(f"damage history: {dmg['ms_per_call']:.3f} ms per call, {dmg['achieved_GBps']:.0f} GB/s")

    # ---- potential-flow yarn directions
    flow = None if args.no_flow else yarn_directions_leg(args, torch)
    if flow:
        log(f"yarn directions 24^3: {flow['ms_per_call']:.2f} ms per call, mean angle to the tangent "
            f"{flow['mean_angle_to_tangent_deg']:.1f} deg, C_bar change {flow['c_hom_change_vs_tangent']}")

    # ---- general (unstructured) mesh
    umesh = None if args.no_umesh else unstructured_leg(args, torch)

    # ---- FE^2 outer loop
    fe2 = None if args.no_fe2 else fe2_leg(args, torch)
    if fe2:
        log(f"FE^2 8x8x2 box, 768 Gauss points: {fe2['ms_per_macro_step']:.1f} ms per macro step "
            f"({fe2['rve_solves_per_s']:.0f} RVE solves/s), macro CG steps {fe2['macro_cg_iters']}")

    # ---- surrogate
    sur = None
    if not args.no_surrogate:
        sur = surrogate_leg(args, torch)

    calibration_copy(torch)
    batch.close()

    # ---- cpu baseline: oracle on the 8^3 records of the batch, worker processes on the host cores
    cpu = None
    if not args.no_cpu_baseline:
        workers = max(1, min(16, os.cpu_count() or 1))
        idx8 = [i for i, s_ in enumerate(sizes) if int(s_) == 8][:workers]
        res, secs, wall = oracle_pool(8, fem.BC_PERIODIC, "substitution", params[idx8], workers)
        eo = np.array([result_errors(got[i], res[j]) for j, i in enumerate(idx8)])
        acc["vs_oracle"] = dict(items=idx8, size=8, fro=float(eo[:, 0].max()), elem=float(eo[:, 1].max()),
                                energy=float(eo[:, 2].max()),
                                reference="CPU FP64 oracle, solved in this run (substitution route)")
        log(f"batch vs oracle (8^3 items): fro {eo[:, 0].max():.2e} energy {eo[:, 2].max():.2e}")
        cpu = dict(value=len(idx8) / wall, unit="homogenisations/s", cores=len(idx8), kind="oracle",
                   sample=(f"CPU FP64 oracle (Lagrange P2, SuperLU, constraints by substitution) on the "
                           f"{len(idx8)} first 8^3 records of the batch, one per worker process ({len(idx8)} "
                           f"processes, one thread each) on {cpu_model()} ({os.cpu_count()} logical CPUs): "
                           f"{wall:.1f} s wall, {np.mean(secs):.1f} s per record; the larger records of the "
                           f"batch (12^3 to 24^3) are not run (a 12^3 periodic solve takes about two minutes on "
                           f"one core, 24^3 about 40 minutes), so this rate overstates the oracle on the mix"),
                   single_rve_latency_s=float(np.mean(secs)), cpu_model=cpu_model(),
                   logical_cpus=os.cpu_count())

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "homogenisations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": wl["desc"], "path": "batched", "rves_per_step": len(rves),
                   "sizes": {int(k): int(v) for k, v in zip(*np.unique(sizes, return_counts=True))},
                   "rtol": args.rtol, "inner_rtol": args.inner_rtol, "precond": args.precond,
                   "autotuned": os.environ.get("CHOM_AUTOTUNE") is not None, "launch": launch,
                   "converged": int(sum(r["status"] == 0 for r in rep)),
                   "max_cg_iters": int(max(rep[worst]["iters"])),
                   "plain_rate": plain_rate, "speedup_batched_over_plain": value / plain_rate if plain_rate else None,
                   "accuracy": acc, "c0_plain_fp64_8cubed": c0,
                   "surrogate": sur,
                   "speedup_surrogate_over_plain": (sur["speedup_vs_plain_12cubed"] if sur else None),
                   "damage_history_kernel": dmg, "yarn_directions_potential_flow": flow,
                   "fe2_outer_loop": fe2, "unstructured_rve": umesh},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))


def run_single(args, wl, torch):
    """c1 / c0 / c3: one batch of a few RVEs of one size (the earlier headline forms)."""
    import chom_inputs as ci
    from paper_1610_03484_amd import RVE, Batch, generate_plain_weave
    opts = bench_opts(args, wl["precision"])
    if args.workload == "c3":
        n = wl["n"]
        items = args.items if args.items != 512 else 64
        rve = RVE(*generate_plain_weave(n, device="cuda:0"), ci.BASE_MATERIALS, bc="periodic", order=args.order,
                  **opts)
        rves = [rve] * items
        params = ci.draw_params(0, items)
    else:
        n = wl["n"]
        mesh = generate_plain_weave(n, device="cuda:0")
        rves = [RVE(*mesh, ci.BASE_MATERIALS, bc=bc, **opts) for bc in wl["bcs"]]
        params = np.repeat(ci.draw_factors_only(0, 1), len(rves), axis=0)
    batch = Batch(rves)
    dt, (C, K, D, rep) = time_batch(batch, params, args.steps, args.warmup, torch)
    value = len(rves) * args.steps / dt
    for i, r in enumerate(rep[:6]):
        log(f"item {i}: iters={r['iters']} refine={r['refine_steps']} resid_max={max(r['resid']):.1e} "
            f"asym={r['asym']:.1e} HM gap={r['hill_mandel_gap']:.1e}")
    err = None
    if not args.no_accuracy and wl["precision"] != "fp64":
        acc_items = [0, 1] if args.workload == "c3" else list(range(len(rves)))
        if args.workload == "c3":
            r64 = RVE(*generate_plain_weave(n, device="cuda:0"), ci.BASE_MATERIALS, bc="periodic",
                      order=args.order, precision="fp64", rtol=1e-12, max_iter=50000)
            refs = [r64] * 2
        else:
            refs = [RVE(*mesh, ci.BASE_MATERIALS, bc=bc, precision="fp64", rtol=1e-12, max_iter=50000)
                    for bc in wl["bcs"]]
        rb = Batch(refs)
        Cr, Kr, Dr, _ = rb.homogenise(np.ascontiguousarray(params[acc_items]))
        got, ref = _stack(C, K, D), _stack(Cr, Kr, Dr)
        e = np.array([result_errors(got[i], ref[j]) for j, i in enumerate(acc_items)])
        err = dict(fro=float(e[:, 0].max()), elem=float(e[:, 1].max()), energy=float(e[:, 2].max()),
                   reference="FP64 GPU path at rtol 1e-12")
        rb.close()
    fp32 = wl["precision"] != "fp64"
    if args.workload == "c3":
        roof = roofline_mech(batch, n, len(rves), fp32, args, "c3", order=args.order)
    else:
        roof = roofline_mech(batch, n, len(rves), fp32, args, args.workload)
    calibration_copy(torch)
    line = {
        "metric": METRIC, "value": value, "unit": "homogenisations/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32+f64" if fp32 else "f64", "data": "synthetic",
        "config": {"workload": wl["desc"], "path": "batched", "rves_per_step": len(rves), "rtol": args.rtol,
                   "inner_rtol": args.inner_rtol, "precond": args.precond, "launch": batch.launch_config(),
                   "accuracy_vs_fp64_gpu": err, "converged": int(sum(r["status"] == 0 for r in rep))},
        "roofline": roof, "cpu_baseline": None,
    }
    print(json.dumps(line))


def run_c4(args, torch):
    sur = surrogate_leg(args, torch)
    line = {
        "metric": METRIC, "value": sur["rate"], "unit": "homogenisations/s", "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": args.points / sur["rate"] * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16+f32 (network), f32+f64 (fallback)", "data": "synthetic",
        "config": {"workload": WORKLOADS["c4"]["desc"], "path": "surrogate+fallback", **sur},
        "roofline": dict(bound="mfma", achieved=sur["predict_kernel"]["achieved_TFLOPs"], peak=2500.0,
                         unit="TFLOP/s", frac=sur["predict_kernel"]["frac_bf16_peak"], traffic=None,
                         kernel="predict_kernel (bf16 MFMA)",
                         avg_launch_us=sur["predict_kernel"]["avg_launch_us"]),
        "cpu_baseline": None,
    }
    print(json.dumps(line))


def run_leg(args, torch):
    """--workload umesh | fe2: the unstructured-mesh or FE^2 leg of the default line on its own."""
    if args.workload == "umesh":
        leg = unstructured_leg(args, torch)
        value, unit, metric = leg["rate"], "homogenisations/s", "RVE homogenisations/s (12 load cases), general tet mesh"
        ms = leg["ms_per_homogenisation"]
    else:
        leg = fe2_leg(args, torch)
        value, unit, metric = 1e3 / leg["ms_per_macro_step"], "macro steps/s", "FE^2 macro steps/s (768 Gauss points)"
        ms = leg["ms_per_macro_step"]
    line = {"metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": 1, "warmup": 1, "ms_per_step": ms,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f64" if args.workload == "umesh" else "f32+f64", "data": "synthetic",
            "config": {"workload": WORKLOADS[args.workload]["desc"], **leg}, "roofline": None, "cpu_baseline": None}
    print(json.dumps(line))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c2", choices=sorted(WORKLOADS))
    ap.add_argument("--op-reps", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true")
    ap.add_argument("--no-surrogate", action="store_true", help="c2: skip the surrogate leg")
    ap.add_argument("--no-c0", action="store_true", help="c2: skip the 8^3 FP64 plain (C0) leg")
    ap.add_argument("--no-plain", action="store_true", help="c2: skip the one-record-per-call leg")
    ap.add_argument("--no-damage", action="store_true", help="c2: skip the damage-history kernel leg")
    ap.add_argument("--no-flow", action="store_true", help="c2: skip the potential-flow yarn-direction leg")
    ap.add_argument("--no-fe2", action="store_true", help="skip the FE^2 outer-loop legs")
    ap.add_argument("--no-umesh", action="store_true", help="c2: skip the unstructured-mesh leg")
    ap.add_argument("--items", type=int, default=512, help="items of the c2 batch (c3: 64 unless set)")
    ap.add_argument("--precond", default="two_level", choices=["block_jacobi", "two_level"],
                    help="CG preconditioner (two_level: block Jacobi plus a P1 multigrid coarse correction)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="fixed launch shape instead of the library's autotuner (which runs in the warm-up)")
    ap.add_argument("--order", type=int, default=4, help="c3: polynomial order (3 or 4)")
    ap.add_argument("--rtol", type=float, default=3e-5,
                    help="stopping tolerance of each load case (relative to its own energy, in the metric of "
                         "the preconditioner); the errors against the FP64 path and the oracle are measured "
                         "and reported each run")
    ap.add_argument("--inner-rtol", type=float, default=2e-5,
                    help="FP32 inner solve tolerance per refinement pass (2/3 of rtol: an inner pass that stops "
                         "exactly at rtol misses the FP64 check by a hair on about 30%% of the mixed batch's "
                         "items and pays a restarted second pass)")
    ap.add_argument("--train", type=int, default=20000, help="surrogate: training solves")
    ap.add_argument("--epochs", type=int, default=300, help="surrogate: training epochs")
    ap.add_argument("--points", type=int, default=1_000_000, help="surrogate: evaluation points")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (the RVE batches would shard across GPUs without "
              f"communication, but no multi-GPU path is built); got --gpus {args.gpus}", file=sys.stderr)
        sys.exit(2)
    if not args.no_autotune:
        os.environ.setdefault("CHOM_AUTOTUNE", "1")
    import torch
    if not torch.cuda.is_available():
        print("bench.py: needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.workload == "c2":
        run_c2(args, torch)
    elif args.workload == "c4":
        run_c4(args, torch)
    elif args.workload in ("umesh", "fe2"):
        run_leg(args, torch)
    else:
        run_single(args, WORKLOADS[args.workload], torch)


if __name__ == "__main__":
    main()
