"""Writes batched_1024_flagged.json: the FP64 oracle's own outcome on the blocks of the 1024-block
batched workload (seed 4) that the batched GPU path leaves unconverged at GMRES(12).

Each block is solved alone by the oracle with its Dirichlet ghost data, in the linearised Picard
form (the library's default), GMRES(64), tight inner solves (relative 1e-12), at most 50 Picard
iterations and the step tolerance 1e-10.  The oracle stops a Picard iteration that makes no
progress two iterations in a row.  Recorded per block: whether it converged, its iteration counts
and scaled residual, and how many interior cells end with E < 0 and T at the T >= 0 bound (the
active set of the exchange solve of eq. PicardTemp, where the Picard map is not smooth).

Only the oracle and the seeded workload generator run here.  Several minutes per block on the
CPU; run from the repository root:  python tests/golden/make_batched_flagged.py [block ...]
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_2202_08778_amd import workloads as W  # noqa: E402

DEFAULT_BLOCKS = (280, 651, 670, 883)


def solve(batch, b):
    blk = batch["blocks"][b]
    ng = blk["ng"]
    s = (slice(ng - 1, -(ng - 1) or None),) * 3
    cut = lambda a: np.ascontiguousarray(a[(Ellipsis,) + s])
    P = oracle.Problem(cut(blk["rho"]), cut(blk["kP"]), cut(blk["kR"]), cut(blk["f"]), blk["dt"], blk["dx"],
                       "dirichlet", c=batch["c"], aR=batch["aR"], cv=batch["cv"], padded=True)
    t0 = time.time()
    E, F, T, st = P.step(cut(blk["E"]), cut(blk["F"]), cut(blk["T"]), tol=1e-10, mode="linearised",
                         max_picard=50, gmres_m=64, lin_rtol=1e-12, allow_unconverged=True)
    inner = (slice(1, -1),) * 3
    return {"block": b, "n": blk["n"], "crossings": blk["dt"] / blk["dx"], "kappa": float(blk["kP"].flat[0]),
            "converged": int(st["converged"]), "picard_iters": int(st["picard_iters"]),
            "krylov_iters": int(st["krylov_iters"]), "scaled_residual": float(st["scaled_residual"]),
            "cells_E_negative": int(np.sum(E[inner] < 0)), "cells_T_at_bound": int(np.sum(T[inner] <= 0)),
            "seconds": round(time.time() - t0, 1)}


def main():
    blocks = [int(a) for a in sys.argv[1:]] or list(DEFAULT_BLOCKS)
    batch = W.batched_blocks(nblocks=1024, seed=4)
    rows = []
    for b in blocks:
        rows.append(solve(batch, b))
        print(rows[-1], flush=True)
    out = {"workload": "batched_blocks(nblocks=1024, seed=4)",
           "oracle": "linearised Picard, GMRES(64), lin_rtol 1e-12, max_picard 50, tol 1e-10",
           "blocks": rows}
    with open(os.path.join(HERE, "batched_1024_flagged.json"), "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
