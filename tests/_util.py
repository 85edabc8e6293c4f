"""Shared test helpers: oracle plans from workload parameters and the per-path
relative error metric (a path is one lambda row of S1, or one (alpha, beta,
theta) slice of S2, for one signal)."""
import numpy as np

from oracle import jtfs_oracle as O


def oracle_plan(p):
    return O.Plan(p["N"], p["J"], p["Q"][0], p["Q"][1], p["J_fr"], p["Q_fr"], p["T"], p["F"],
                  lowpass_pairs=p.get("lowpass_pairs", False), unpad=p.get("unpad", False))


def path_errors(got, ref, path_axes):
    """Relative L2 error of every path: ||d_p|| / max(||ref_p||, 1e-4 * rms_q ||ref_q||).

    got/ref: arrays for one signal; path_axes: number of leading axes that index
    paths (1 for S1, 3 for S2).  Returns (floored errors, unfloored errors)."""
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    shp = ref.shape[:path_axes]
    d = (got - ref).reshape(int(np.prod(shp)), -1)
    r = ref.reshape(int(np.prod(shp)), -1)
    nd = np.linalg.norm(d, axis=1)
    nr = np.linalg.norm(r, axis=1)
    rms = np.sqrt(np.mean(nr ** 2))
    floored = nd / np.maximum(nr, 1e-4 * rms)
    unfloored = nd / np.maximum(nr, 1e-300)
    return floored.reshape(shp), unfloored.reshape(shp)


def rel_l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
