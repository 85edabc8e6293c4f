"""Writes tests/golden/cfg5_reference.npz: FP64 oracle outputs for the
32 x 2^18 FM-mixture workload (J=14, Q=(24,2), J_fr=5, Q_fr=2, T=2^14, F=2^4),
which the oracle needs several minutes per signal to produce (its own radix-2
FFT over 285 rows of 2^18 points), too long to recompute inside a GPU test.

Contents, for signals 0 and 31 of the seeded batch:
  s1_<b>     S1 [n1][N/T] (eq. (3) first order, every path)
  s2_<b>     S2 [len(alphas)][n_beta][2][L/F][N/T] at the temporal rates `alphas`
and for signal 0 the VJP `gx_0` of the cotangent (gS1, gS2 restricted to
`alphas`) drawn by synth.cotangents(seed=9), as float32 (the stored gradient's
rounding, 6e-8 relative, is far below the 1e-4 bar it serves).  `x_sha256`
fingerprints the FP32 inputs so that the test can tell a changed generator.

Only the oracle and the seeded generators are called.  Run from the repository
root:  python tests/golden/make_cfg5_reference.py   (several minutes, three
processes of about 6 GB each).
"""
from __future__ import annotations

import hashlib
import multiprocessing as mp
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import jtfs_oracle as O  # noqa: E402

CFG = 5
SIGNALS = (0, 31)
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "cfg5_reference.npz")


def plan():
    p = synth.PARAMS[CFG]
    return O.Plan(p["N"], p["J"], p["Q"][0], p["Q"][1], p["J_fr"], p["Q_fr"], p["T"], p["F"])


def sampled_alphas(P):
    """k2 = 0 (rows of 2^15 points), a middle rate and the shortest rate."""
    return [0, P.n_alpha // 2, P.n_alpha - 1]


def cotangent(P, alphas):
    gs1, gs2 = synth.cotangents((1,) + P.s1_shape(), (1,) + P.s2_shape(), seed=9)
    keep = np.zeros(P.n_alpha, bool)
    keep[alphas] = True
    gs2[:, ~keep] = 0.0
    return gs1[0], gs2[0]


def _job(args):
    kind, b = args
    P = plan()
    alphas = sampled_alphas(P)
    x = synth.batch(CFG)[b].astype(np.float64)
    if kind == "fwd":
        s1, s2 = O.jtfs(x, P, alphas=alphas)
        return kind, b, s1, s2[alphas]
    gs1, gs2 = cotangent(P, alphas)
    return kind, b, O.jtfs_vjp(x, gs1.astype(np.float64), gs2.astype(np.float64), P), None


def main():
    P = plan()
    xs = synth.batch(CFG)
    jobs = [("fwd", b) for b in SIGNALS] + [("vjp", 0)]
    with mp.get_context("fork").Pool(len(jobs)) as pool:
        res = pool.map(_job, jobs)
    out = {"alphas": np.array(sampled_alphas(P)), "signals": np.array(SIGNALS),
           "x_sha256": np.array(hashlib.sha256(np.ascontiguousarray(xs).tobytes()).hexdigest())}
    for kind, b, a, c in res:
        if kind == "fwd":
            out[f"s1_{b}"] = a
            out[f"s2_{b}"] = c
        else:
            out[f"gx_{b}"] = a.astype(np.float32)
    np.savez(OUT, **out)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
