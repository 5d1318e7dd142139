#!/usr/bin/env python
"""Benchmark: RVE homogenisations per second on one MI355X.

Workload (default "c1"): the synthetic plain-weave RVE on a 24^3 Kuhn lattice
(82,944 tets), order-2 hierarchic basis (352,947 elastic DOFs), homogenised
under each of the three boundary conditions (linear Dirichlet, periodic,
uniform traction), 6 mechanical + 3 thermal + 3 moisture load cases each,
FP32 operator with FP64 CG reductions, constraint projection, refinement
residual and volume average.  One step = the three homogenisations.  The mesh,
tags and element data are resident on the GPU before timing starts.

Also reported (outside the timed region):
  * the error of the timed results against the FP64 GPU path on the same RVE
    (the FP64 path is checked against the CPU oracle at smaller sizes by tests);
  * the roofline record of the dominant kernel (the FP32 mechanical operator):
    HIP-event timing of its launches, algorithmic bytes/flops per launch;
  * the CPU oracle timed on the host on a bounded sample.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c1|c0]
"""
from __future__ import annotations

import argparse
import json
import os
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

WORKLOADS = {
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
    "c3": dict(n=16, bcs=("periodic",), precision="fp32_refined",
               desc="p-refinement: batch of 16^3 Kuhn plain-weave RVEs (24,576 tets each) at order p (3: 352,947, "
                    "4: 823,875 elastic DOFs), periodic, degraded records as in the batched workload, element "
                    "operator on the FP32 matrix cores with FP64 refinement"),
    "c2": dict(n=None, bcs=("periodic",), precision="fp32_refined",
               desc="batch of RVEs with sizes uniform over {8,12,16,20,24}^3 cells, p=2, periodic, degraded "
                    "(T~U(20,60) C, c~U(0,1.5) wt%, t~U(0,10) y, factors U(0.9,1.1)), 12 load cases each, "
                    "FP32 operator + FP64 refinement, one batch"),
}


def algorithmic_mech(n, nprob, fp32):
    """Bytes and flops of one mechanical operator launch (6 load cases) per the
    survey's definition: bytes = sum_RHS 2 ndof s + T (conn + n_A s),
    flops = T n_RHS 2 n_e^2, with conn = 40 B, n_A = 45, n_e = 30 at p = 2."""
    s = 4 if fp32 else 8
    T = 6 * n ** 3
    ndof = 3 * (2 * n + 1) ** 3
    bytes_ = 6 * 2 * ndof * s + T * (40 + 45 * s)
    flops = T * 6 * 2 * 30 ** 2
    return bytes_ * nprob, flops * nprob


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


# HBM traffic of one launch of op_p2_kernel<float,3,6,RG> on the default workload (three
# 24^3 items, all active) per load-case grouping RG, from rocprofv3 FETCH_SIZE and
# WRITE_SIZE scaled by the calibration copy
# (profiles/op_p2_mech_fp32_24cubed_three_bc_traffic.md).  Must be re-measured (or set
# to None) whenever that kernel changes.
C1_OP_TRAFFIC_BYTES = {1: 124257650, 2: 128732682, 3: 108221564}


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


CPU_SAMPLE_CODE = r"""
import sys, time, json
sys.path.insert(0, {root!r})
import chom_inputs as ci
from oracle import fem, mesh
n = {n}
params = ci.draw_factors_only(0, 1)[0]
c, t, ph, ax = mesh.plain_weave(n)
t0 = time.perf_counter()
count = 0
for bc in (fem.BC_DIRICHLET, fem.BC_PERIODIC, fem.BC_NEUMANN):
    fem.homogenise(c, t, ph, ax, 2, bc, ci.BASE_MATERIALS, params)
    count += 1
dt = time.perf_counter() - t0
print(json.dumps(dict(count=count, seconds=dt)))
"""


def cpu_baseline(n_sample=8):
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1",
               CUDA_VISIBLE_DEVICES="", HIP_VISIBLE_DEVICES="")
    code = CPU_SAMPLE_CODE.format(root=ROOT, n=n_sample)
    res = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, timeout=600)
    if res.returncode != 0:
        return None
    rec = json.loads(res.stdout.strip().splitlines()[-1])
    return dict(value=rec["count"] / rec["seconds"], unit="homogenisations/s", cores=1, kind="oracle",
                sample=(f"CPU FP64 oracle (Lagrange P2, SuperLU saddle point, factorised once per BC and "
                        f"physics) on the {n_sample}^3 plain-weave RVE, Dirichlet+periodic+Neumann x 12 load "
                        f"cases = {rec['count']} homogenisations in {rec['seconds']:.1f} s on 1 thread; the "
                        f"24^3 RVE is not run (about 40 min per mechanical factorisation), so this rate "
                        f"overstates the oracle's rate on the benchmark RVE"))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c1", choices=sorted(WORKLOADS))
    ap.add_argument("--op-reps", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true")
    ap.add_argument("--items", type=int, default=512, help="items of the c2 batch")
    ap.add_argument("--precond", default="two_level", choices=["block_jacobi", "two_level"],
                    help="CG preconditioner (two_level: block Jacobi plus a P1 multigrid coarse correction)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="fixed launch shape instead of the library's autotuner (which runs in the warm-up)")
    ap.add_argument("--order", type=int, default=4, help="c3: polynomial order (3 or 4)")
    ap.add_argument("--rtol", type=float, default=3e-5,
                    help="stopping tolerance of the FP64 residual (relative to the linear-field energy); with "
                         "the library's energy-form averages the default keeps C_hom >= 10x inside the 1e-6 "
                         "target of the FP32-refined form (the error against the FP64 path is measured and "
                         "reported each run)")
    ap.add_argument("--inner-rtol", type=float, default=3e-5, help="FP32 inner solve tolerance per refinement pass")
    ap.add_argument("--train", type=int, default=20000, help="c4: training solves")
    ap.add_argument("--epochs", type=int, default=300, help="c4: training epochs")
    ap.add_argument("--points", type=int, default=1_000_000, help="c4: surrogate evaluation points")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (the RVE batches would shard across GPUs without "
              f"communication, but no multi-GPU path is built); got --gpus {args.gpus}", file=sys.stderr)
        sys.exit(2)

    if not args.no_autotune:
        os.environ.setdefault("CHOM_AUTOTUNE", "1")
    import torch
    import chom_inputs as ci
    from paper_1610_03484_amd import RVE, generate_plain_weave

    if not torch.cuda.is_available():
        print("bench.py: needs a GPU", file=sys.stderr)
        sys.exit(1)
    wl = WORKLOADS[args.workload]
    if args.workload == "c4":
        return run_surrogate(args, wl)
    from paper_1610_03484_amd import Batch
    opts = dict(precision=wl["precision"], rtol=args.rtol, inner_rtol=args.inner_rtol, max_iter=50000,
                precond=args.precond)
    if args.workload == "c2":
        sizes = ci.batch_sizes_c2(0, args.items)
        params = ci.draw_params(0, args.items)
        handles = {}
        rves = []
        for n_i in sizes:
            if n_i not in handles:
                handles[n_i] = RVE(*generate_plain_weave(int(n_i), device="cuda:0"), ci.BASE_MATERIALS,
                                   bc="periodic", **opts)
            rves.append(handles[n_i])
        n = int(max(sizes))
        labels = [f"item {i} (n={int(s)})" for i, s in enumerate(sizes)]
    elif args.workload == "c3":
        n = wl["n"]
        items = args.items if args.items != 512 else 64
        rve = RVE(*generate_plain_weave(n, device="cuda:0"), ci.BASE_MATERIALS, bc="periodic", order=args.order, **opts)
        rves = [rve] * items
        params = ci.draw_params(0, items)
        labels = [f"item {i}" for i in range(items)]
    else:
        n = wl["n"]
        mesh = generate_plain_weave(n, device="cuda:0")
        rves = [RVE(*mesh, ci.BASE_MATERIALS, bc=bc, **opts) for bc in wl["bcs"]]
        params = np.repeat(ci.draw_factors_only(0, 1), len(rves), axis=0)
        labels = list(wl["bcs"])
    batch = Batch(rves)

    def step():
        return batch.homogenise(params)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res = step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    homs = len(rves) * args.steps
    value = homs / dt
    C, K, D, rep = res
    for i, lab in enumerate(labels[:6]):
        print(f"[bench] {lab}: iters={rep[i]['iters']} refine={rep[i]['refine_steps']} "
              f"resid_max={max(rep[i]['resid']):.1e} asym={rep[i]['asym']:.1e}", file=sys.stderr)
    worst = max(range(len(rep)), key=lambda i: max(rep[i]["iters"]))
    print(f"[bench] status: {sum(r['status'] == 0 for r in rep)}/{len(rep)} converged; "
          f"max iters {max(rep[worst]['iters'])} ({labels[worst]}: iters={rep[worst]['iters']} "
          f"refine={rep[worst]['refine_steps']})", file=sys.stderr)

    # accuracy against the FP64 GPU path solved to rtol 1e-12 (same RVEs, same
    # parameters): every item of the three-BC batch; for the mixed-size batch the
    # first item of each size; for the order-3/4 batch the first two items
    err = None
    acc_items = []
    if not args.no_accuracy and wl["precision"] != "fp64":
        if args.workload == "c2":
            first = {}
            for i, s_ in enumerate(sizes):
                first.setdefault(int(s_), i)
            acc_items = sorted(first.values())
            ref_rves = [RVE(*generate_plain_weave(int(sizes[i]), device="cuda:0"), ci.BASE_MATERIALS, bc="periodic",
                            precision="fp64", rtol=1e-12, max_iter=50000) for i in acc_items]
        elif args.workload == "c3":
            acc_items = [0, 1]
            r64 = RVE(*generate_plain_weave(n, device="cuda:0"), ci.BASE_MATERIALS, bc="periodic", order=args.order,
                      precision="fp64", rtol=1e-12, max_iter=50000)
            ref_rves = [r64] * len(acc_items)
        else:
            acc_items = list(range(len(rves)))
            ref_rves = [RVE(*mesh, ci.BASE_MATERIALS, bc=bc, precision="fp64", rtol=1e-12, max_iter=50000)
                        for bc in wl["bcs"]]
        ref = Batch(ref_rves)
        Cr, Kr, Dr, _ = ref.homogenise(np.ascontiguousarray(params[acc_items]))
        errs = [max(np.linalg.norm(C[i] - Cr[j]) / np.linalg.norm(Cr[j]),
                    np.linalg.norm(K[i] - Kr[j]) / np.linalg.norm(Kr[j]),
                    np.linalg.norm(D[i] - Dr[j]) / np.linalg.norm(Dr[j])) for j, i in enumerate(acc_items)]
        err = float(max(errs))
        ref.close()

    # dominant kernel: the mechanical operator launch of the batch
    ms, tets, nprob = batch.time_operator(0, args.op_reps)
    rg_mech = batch.launch_config()["rg_mech"]
    calibration_copy(torch)
    fp32 = wl["precision"] != "fp64"
    if args.workload == "c2":
        bytes_ = flops = 0
        for s_ in sizes:
            b1, f1 = algorithmic_mech(int(s_), 1, fp32)
            bytes_ += b1
            flops += f1
    elif args.workload == "c3":
        bytes_, flops = algorithmic_mech_order(n, args.order, nprob, fp32)
    else:
        bytes_, flops = algorithmic_mech(n, nprob, fp32)
    t = ms * 1e-3
    peak_alu = FP32_VEC_PEAK if fp32 else FP64_VEC_PEAK
    t_hbm, t_alu = bytes_ / HBM_PEAK, flops / peak_alu
    if t_alu >= t_hbm:
        roof = dict(bound="alu", achieved=flops / t / 1e12, peak=peak_alu / 1e12, unit="TFLOP/s",
                    frac=(flops / t) / peak_alu,
                    traffic=C1_OP_TRAFFIC_BYTES.get(rg_mech) if (args.workload == "c1" and fp32) else None)
    else:
        roof = dict(bound="hbm", achieved=bytes_ / t / 1e9, peak=HBM_PEAK / 1e9, unit="GB/s",
                    frac=(bytes_ / t) / HBM_PEAK, traffic=None)
    if args.workload == "c3":
        roof = dict(bound="mfma", achieved=flops / t / 1e12, peak=FP32_VEC_PEAK / 1e12, unit="TFLOP/s",
                    frac=(flops / t) / FP32_VEC_PEAK, traffic=None,
                    note="FP32 matrix-core peak (157.3 TFLOP/s dense, equal to the packed FP32 vector peak)")
        kname = f"hp_op_kernel<float,{args.order},3,6,8>"
    else:
        kname = f"op_p2_kernel<float,3,6,{rg_mech}>" if fp32 else f"op_p2_kernel<double,3,6,{rg_mech}>"
    roof.update(kernel=kname,
                avg_launch_us=ms * 1e3, algorithmic_bytes=bytes_, algorithmic_flops=flops)
    print(f"[bench] operator: {ms * 1e3:.1f} us/launch, {bytes_ / t / 1e9:.0f} GB/s algorithmic, "
          f"{flops / t / 1e12:.2f} TFLOP/s algorithmic", file=sys.stderr)

    cpu = None if args.no_cpu_baseline else cpu_baseline()
    line = {
        "metric": "RVE homogenisations/s (12 load cases) @ stated C_hom error",
        "value": value,
        "unit": "homogenisations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if fp32 else "f64",
        "data": "synthetic",
        "config": {"workload": wl["desc"], "path": "batched", "rves_per_step": len(rves),
                   "rtol": args.rtol, "inner_rtol": args.inner_rtol,
                   "autotuned": os.environ.get("CHOM_AUTOTUNE") is not None, "precond": args.precond,
                   "c_hom_rel_err_vs_fp64_gpu": err, "accuracy_items": acc_items,
                   "launch": batch.launch_config(),
                   "converged": int(sum(r["status"] == 0 for r in rep))},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))


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


MLP_FLOPS_PER_POINT = 2 * (10 * 256 + 2 * 256 * 256 + 256 * 36)   # one member, one record
BF16_PEAK = 2.5e15


def run_surrogate(args, wl):
    """C4: train the ensemble on RVE solves, then time surrogate + fallback on many records."""
    import torch
    import chom_inputs as ci
    from paper_1610_03484_amd import RVE, Surrogate, generate_plain_weave
    from paper_1610_03484_amd import _lib as L

    n = wl["n"]
    rve = RVE(*generate_plain_weave(n, device="cuda:0"), ci.BASE_MATERIALS, bc="periodic",
              precision="fp32_refined", rtol=args.rtol, inner_rtol=args.inner_rtol, max_iter=50000)
    # ---- training set: RVE solves of seeded degraded records
    params = ci.draw_params(0, args.train)
    chunk = 512
    t0 = time.perf_counter()
    parts = []
    for s0 in range(0, args.train, chunk):
        parts.append(rve.homogenise(params[s0:s0 + chunk])[:3])
        print(f"[bench] training solves {min(s0 + chunk, args.train)}/{args.train}", file=sys.stderr, flush=True)
    t_solve = time.perf_counter() - t0
    C = np.concatenate([q[0] for q in parts])
    K = np.concatenate([q[1] for q in parts])
    D = np.concatenate([q[2] for q in parts])
    batched_rate = args.train / t_solve
    stream = torch.cuda.current_stream().cuda_stream
    sur = Surrogate(members=5, seed=11, device=True, hip_stream=stream)
    dev = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda:0")
    t0 = time.perf_counter()
    hist = sur.train(dev(params), dev(C), dev(K), dev(D), epochs=args.epochs, batch=256)
    t_train = time.perf_counter() - t0
    print(f"[bench] {args.train} solves in {t_solve:.1f} s ({batched_rate:.0f}/s); training {t_train:.1f} s, "
          f"final loss {hist[:, -1].mean():.2e}", file=sys.stderr, flush=True)

    # ---- timed: surrogate with fallback on many records (inputs resident in HBM)
    pts = dev(ci.draw_params(3_000_000, args.points))
    sur.homogenise(rve, pts[:4096], thresh=1e-2, chunk=256)      # warm-up (also builds the fallback batch)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Cs, Ks, Ds, dis, used, nfb = sur.homogenise(rve, pts, thresh=1e-2, chunk=256)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    value = args.points / dt

    # ---- dominant kernel: the ensemble inference (HIP events on the stream it runs on)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 5
    ev0.record()
    for _ in range(reps):
        sur.predict(pts)
    ev1.record()
    torch.cuda.synchronize()
    t_pred = ev0.elapsed_time(ev1) / reps * 1e-3
    flops = MLP_FLOPS_PER_POINT * 5 * args.points
    roof = dict(bound="mfma", achieved=flops / t_pred / 1e12, peak=BF16_PEAK / 1e12, unit="TFLOP/s",
                frac=flops / t_pred / BF16_PEAK, traffic=None, kernel="predict_kernel (bf16 MFMA)",
                avg_launch_us=t_pred * 1e6, algorithmic_flops=flops,
                note="per-launch time includes the feature and output passes of the same kernel")

    # ---- accuracy on held-out records against the oracle's stored solves (else the FP64 GPU path)
    golden = os.path.join(ROOT, "tests", "golden", "surrogate_heldout_n12_periodic.txt")
    if os.path.exists(golden):
        a = np.loadtxt(golden)
        hp, truth, judge = a[:, 1:12], a[:, 12:45], "CPU FP64 oracle (stored)"
    else:
        hp = ci.draw_params(1_000_000, 256)
        fp64 = RVE(*generate_plain_weave(n, device="cuda:0"), ci.BASE_MATERIALS, bc="periodic", precision="fp64",
                   rtol=1e-12, max_iter=50000)
        c, k, d, _ = fp64.homogenise(hp)
        truth, judge = np.concatenate([c, k, d], axis=1), "FP64 GPU path"
        fp64.close()
    Ch, Kh, Dh, dish, usedh, nfbh = sur.homogenise(rve, dev(hp), thresh=1e-2, chunk=256)
    got = np.concatenate([Ch.cpu().numpy(), Kh.cpu().numpy(), Dh.cpu().numpy()], axis=1)
    err = block_errors(got, truth)
    Cp, Kp, Dp, _ = sur.predict(dev(hp))
    raw = block_errors(np.concatenate([Cp.cpu().numpy(), Kp.cpu().numpy(), Dp.cpu().numpy()], axis=1), truth)
    print(f"[bench] surrogate: {args.points} points in {dt:.2f} s, {nfb} fallbacks; held-out ({judge}) "
          f"max err {err.max():.2e} (network alone {raw.max():.2e}, median {np.median(raw):.2e})",
          file=sys.stderr, flush=True)
    line = {
        "metric": "RVE homogenisations/s (12 load cases) @ stated C_hom error",
        "value": value,
        "unit": "homogenisations/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 1,
        "ms_per_step": dt * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16+f32 (network), f32+f64 (fallback)",
        "data": "synthetic",
        "config": {"workload": wl["desc"], "path": "surrogate+fallback", "points": args.points,
                   "fallbacks": int(nfb), "training_solves": args.train, "training_solve_s": t_solve,
                   "training_s": t_train, "epochs": args.epochs, "batched_rate_12cubed": batched_rate,
                   "speedup_vs_batched": value / batched_rate, "heldout_points": len(hp),
                   "heldout_judge": judge, "heldout_max_err": float(err.max()),
                   "heldout_max_err_network_alone": float(raw.max()),
                   "heldout_fallbacks": int(nfbh)},
        "roofline": roof,
        "cpu_baseline": None,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
