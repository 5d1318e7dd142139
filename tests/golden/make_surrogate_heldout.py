#!/usr/bin/env python
"""Writes surrogate_heldout_n12_periodic.txt: oracle homogenisations of the
held-out set that judges the learned surrogate.

Points: draw_params(seed=1_000_000, n=256) (temperature, moisture, exposure
time and the eight property factors), each solved on the 12^3 plain-weave RVE,
order 2, periodic conditions, matrix-only degradation with c_sat = 1.5 wt%, by
the CPU oracle in its substitution form (the same discrete solution as the
bordered form; the tests pin the two against each other).

Each line: index, the 11 parameters, the 21 upper-triangle entries of C_bar
(row-major, Voigt order 11, 22, 33, 12, 23, 31), the 6 entries of K_bar and of
D_bar (xx, yy, zz, xy, yz, zx).  Every number is printed with repr().

Usage: python tests/golden/make_surrogate_heldout.py [--workers 6] [--count 256]
Resumable: finished points are kept in a .partial file beside the output.
"""
from __future__ import annotations

import argparse
import os
import sys

os.environ.setdefault("OMP_NUM_THREADS", "1")
os.environ.setdefault("OPENBLAS_NUM_THREADS", "1")
HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import chom_inputs as ci  # noqa: E402

N_CELLS = 12
SEED = 1_000_000
OUT = os.path.join(HERE, "surrogate_heldout_n12_periodic.txt")

_state = {}


def _init():
    from oracle import fem, mesh
    c, t, ph, ax = mesh.plain_weave(N_CELLS)
    _state.update(fem=fem, mesh=(c, t, ph, ax), disc=fem.Discretisation(c, t, 2))


def _solve(args):
    i, prm = args
    fem = _state["fem"]
    c, t, ph, ax = _state["mesh"]
    r = fem.homogenise(c, t, ph, ax, 2, fem.BC_PERIODIC, ci.BASE_MATERIALS, prm, c_sat=1.5,
                       degrade_yarn=False, disc=_state["disc"], method="substitution")
    iu = np.triu_indices(6)
    sym3 = [(0, 0), (1, 1), (2, 2), (0, 1), (1, 2), (2, 0)]
    vals = list(prm) + list(r["C"][iu]) + [r["K"][a, b] for a, b in sym3] + [r["D"][a, b] for a, b in sym3]
    return i, " ".join([str(i)] + [repr(float(v)) for v in vals])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workers", type=int, default=6)
    ap.add_argument("--count", type=int, default=256)
    args = ap.parse_args()
    params = ci.draw_params(SEED, args.count)
    partial = OUT + ".partial"
    done = {}
    if os.path.exists(partial):
        for line in open(partial):
            if line.strip():
                done[int(line.split()[0])] = line.rstrip("\n")
    todo = [(i, params[i]) for i in range(args.count) if i not in done]
    if todo:
        import multiprocessing as mp
        with mp.Pool(args.workers, initializer=_init) as pool, open(partial, "a") as fh:
            for i, line in pool.imap_unordered(_solve, todo):
                fh.write(line + "\n")
                fh.flush()
                done[i] = line
                print(f"[heldout] {len(done)}/{args.count}", flush=True)
    with open(OUT, "w") as fh:
        fh.write(f"# oracle homogenisations, 12^3 plain weave, p=2, periodic; params = draw_params({SEED}, "
                 f"{args.count}); columns: index, 11 params, 21 C_upper, 6 K, 6 D\n")
        for i in range(args.count):
            fh.write(done[i] + "\n")
    os.remove(partial)


if __name__ == "__main__":
    main()
