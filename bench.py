"""Benchmark of the JTFS hot path on one MI355X.

One step = JTFS forward (S1, S2) plus the backward (VJP) of a fixed random
cotangent, over a batch of 64 synthetic chirps of 2^16 samples (J=12, Q=(16,1),
J_fr=4, Q_fr=1, T=2^11, F=2^3), inputs resident in HBM.  Prints one JSON line.

Also reported: batched forward-only and single-signal forward throughput, the
per-stage kernel times (HIP events on the launch stream), the roofline of the
dominant kernel, the FP64 oracle's parity on signal 0, and the oracle's own
speed on the host cores (a baseline only).
"""
from __future__ import annotations

import argparse
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

import synth  # noqa: E402

METRIC = "JTFS fwd+bwd Msamples/s (batched) vs plain fwd; % HBM roofline; rel err vs FP64"
CFG = 2
PEAK_FP32_MFMA = 157.3     # TFLOP/s, MI355X dense FP32 matrix
PEAK_F16_MFMA = 2500.0     # TFLOP/s, MI355X dense FP16 matrix
PEAK_HBM = 8000.0          # GB/s


# --------------------------------------------------------------------- CPU leg

def _oracle_worker(args):
    """Oracle forward + VJP of one signal restricted to a set of temporal rates
    (all first-order terms in the worker that has first=True)."""
    x, gs1, gs2, alphas, first = args
    from oracle import jtfs_oracle as O
    from tests._util import oracle_plan
    P = oracle_plan(synth.PARAMS[CFG])
    S1, S2 = O.jtfs(x, P, alphas=alphas)
    g = np.zeros_like(gs2)
    g[alphas] = gs2[alphas]
    gx = O.jtfs_vjp(x, gs1 if first else np.zeros_like(gs1), g, P)
    return alphas, S1, S2, gx


def cpu_baseline(x0, gs1, gs2, max_workers):
    """FP64 oracle, forward + VJP of one signal, the temporal rates split over a
    process pool (each worker runs the unmodified oracle on its rates)."""
    from tests._util import oracle_plan
    P = oracle_plan(synth.PARAMS[CFG])
    n_alpha = P.n_alpha
    workers = max(1, min(n_alpha, max_workers))
    groups = [list(range(i, n_alpha, workers)) for i in range(workers)]
    jobs = [(x0, gs1, gs2, g, i == 0) for i, g in enumerate(groups)]
    saved = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")}
    for k in saved:
        os.environ[k] = "1"
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(workers) as pool:
        res = pool.map(_oracle_worker, jobs)
    wall = time.perf_counter() - t0
    for k, v in saved.items():
        if v is None:
            os.environ.pop(k, None)
        else:
            os.environ[k] = v
    S1 = res[0][1]                      # every worker computes the same first order
    S2 = np.zeros(P.s2_shape())
    gx = np.zeros(P.N)
    for alphas, _, s2, g in res:
        S2[alphas] = s2[alphas]
        gx += g
    return dict(wall=wall, workers=workers, S1=S1, S2=S2, gx=gx)


# --------------------------------------------------------------------- GPU leg

def algorithmic_flops(info, shapes, B, split):
    """Dense-contraction flops of the frequential stage per step (unpadded sizes):
    forward 8 M_h n1 T_alpha + time lowpass 2 (2 M_h) T_alpha N/T per signal and
    rate; the backward recomputes both and adds the W^H product 8 M_h n1 T_alpha
    (one fused kernel in the split-FP16 mode, two kernels in the FP32 mode).  With
    the stored phase the backward recomputes neither the contraction nor the
    modulus: it does the lowpass adjoint and the W^H product only."""
    Mh, n1, NT = info.M_h, info.n1, info.out_t
    fwd = sum(8 * Mh * n1 * Ta + 4 * Mh * Ta * NT for Ta in shapes) * B
    lp = sum(4 * Mh * Ta * NT for Ta in shapes) * B
    wh = sum(8 * Mh * n1 * Ta for Ta in shapes) * B
    if split == "phase":
        return {"freq_fwd": fwd, "freq_adj_pq": lp + wh}
    if split:
        return {"freq_fwd": fwd, "freq_adj_pq": fwd + wh}
    return {"freq_fwd": fwd, "freq_adj_pq": fwd, "freq_adj_wh": wh}


def algorithmic_bytes(info, N, shapes, B):
    """Mandatory HBM bytes per step of the FFT-based stages: each stage's input
    plus output at their unpadded sizes, each read or written once (c64 = 8 B,
    f32 = 4 B).  x_hat has N/2+1 bins, X_hat n1 rows of N_X/2+1 bins, Y2 and
    its gradient n1 rows of T_alpha values per rate, gX n1 x N_X reals, the
    first-order gradient spectra n1 x N_X."""
    n1, NX, NT = info.n1, info.NX, info.out_t
    xh = 8 * (N // 2 + 1)
    Xh = 8 * n1 * (NX // 2 + 1)
    Y2 = 8 * n1 * sum(shapes)
    S1 = 4 * n1 * NT
    gX = 4 * n1 * NX
    g1 = 8 * n1 * NX
    # (S1 and the band accumulation read only band-limited bins of their inputs;
    # their mandatory bytes depend on the filter supports and they are not listed)
    per = {
        "input_fft": 4 * N + xh,
        "scalogram": xh + Xh,
        "second_order": Xh + Y2,
        "second_adj_fft": 2 * Y2,
        "second_adj": Y2 + S1 + gX,
        "first_adj": xh + gX + g1,
        "output_fft": xh + 4 * N,
    }
    return {k: v * B for k, v in per.items()}


# HBM bytes per launch of a stage's kernel from rocprofv3 FETCH_SIZE / WRITE_SIZE
# passes (scaled by the same counters on a copy of known size), kept beside the
# profiles with the hash of the kernel's source; stale once that source changes.
TRAFFIC_FILES = {("freq_fwd", "split16"): ("profiles/k_freq_fwd_h_64x65536_hbm_traffic.json",
                                         "paper_2204_08269_amd/csrc/split.hip"),
                 ("freq_adj_pq", "split16"): ("profiles/k_freq_bwd_h_64x65536_hbm_traffic.json",
                                            "paper_2204_08269_amd/csrc/split.hip"),
                 ("freq_fwd", "split16_phase"): ("profiles/k_freq_fwd_h_phase_64x65536_hbm_traffic.json",
                                               "paper_2204_08269_amd/csrc/split.hip"),
                 ("freq_adj_pq", "split16_phase"): ("profiles/k_freq_bwd_p_64x65536_hbm_traffic.json",
                                                  "paper_2204_08269_amd/csrc/split.hip")}


def measured_traffic(stage, contraction):
    import hashlib
    if (stage, contraction) not in TRAFFIC_FILES:
        return None
    rec_path, src = (os.path.join(HERE, v) for v in TRAFFIC_FILES[(stage, contraction)])
    if not os.path.exists(rec_path):
        return None
    rec = json.load(open(rec_path))
    if rec.get("source_sha256") != hashlib.sha256(open(src, "rb").read()).hexdigest():
        return None
    return {"bytes_per_launch": rec["bytes_per_launch"], "fetch_bytes_per_launch": rec["fetch_bytes_per_launch"],
            "write_bytes_per_launch": rec["write_bytes_per_launch"], "source": os.path.basename(rec_path)}


def ragged_batch(torch, dev, runs=3):
    """Forward + backward of the 256-signal ragged workload through the bucket API."""
    from paper_2204_08269_amd.jtfs import JTFSBucket
    p = synth.PARAMS[4]
    sigs = synth.cfg4_ragged(synth.BATCH[4])
    lengths = [len(v) for v in sigs]
    bk = JTFSBucket(lengths, p["J"], p["Q"], p["J_fr"], p["Q_fr"], p["T"], p["F"])
    x = torch.from_numpy(np.concatenate(sigs)).to(dev)
    g = torch.from_numpy(np.random.default_rng(4).standard_normal(bk.s_offset[-1]).astype(np.float32)).to(dev)
    out = torch.empty(bk.s_offset[-1], dtype=torch.float32, device=dev)
    gx = torch.empty(bk.x_offset[-1], dtype=torch.float32, device=dev)
    st = torch.cuda.Stream(device=dev)
    st.wait_stream(torch.cuda.current_stream(dev))
    with torch.cuda.stream(st):
        bk.run(x, g, out, gx)                    # capture + first replay
        st.synchronize()
        t0 = time.perf_counter()
        for _ in range(runs):
            bk.run(x, g, out, gx)
        st.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / runs
    real, padded = sum(lengths), sum(bk.pads)
    counts = {}
    for n in bk.pads:
        counts[str(n)] = counts.get(str(n), 0) + 1
    print(f"[bench] ragged batch: {ms:.2f} ms per fwd+bwd run", file=sys.stderr, flush=True)
    return {"workload": "256 harmonic tones + pink noise, lengths log-uniform in [2^13, 2^16], J=11, Q=(16,1), "
                        "J_fr=4, Q_fr=1, T=2^10, F=2^3; buckets of power-of-two pads, one HIP graph per run",
            "ms_per_run": round(ms, 3), "fwd_bwd_msamples_s_real": round(real / (ms * 1e-3) / 1e6, 3),
            "fwd_bwd_msamples_s_padded": round(padded / (ms * 1e-3) / 1e6, 3),
            "real_samples": real, "padded_samples": padded, "signals_per_pad": counts}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-workers", type=int, default=16)
    ap.add_argument("--contraction", choices=["split16", "split16_phase", "fp32"], default=None,
                    help="frequential contraction arithmetic (default: the plan's, split16 where available)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run one 1 GiB device copy first (calibrates HBM byte counters)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the plan's default launch choices (no autotuning before the timed steps)")
    ap.add_argument("--no-extras", action="store_true",
                    help="time the fwd+bwd step only (no forward-only or ragged-batch legs)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: this library has no multi-GPU path "
              "(signals shard across GPUs with no communication; see the design notes)", file=sys.stderr)
        sys.exit(2)

    p = synth.PARAMS[CFG]
    B = synth.BATCH[CFG]
    x_np = synth.batch(CFG)                                      # [64, 65536] float32
    from tests._util import oracle_plan
    Po = oracle_plan(p)
    gs1_np, gs2_np = synth.cotangents((B,) + Po.s1_shape(), (B,) + Po.s2_shape())

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(x_np[0].astype(np.float64), gs1_np[0].astype(np.float64),
                           gs2_np[0].astype(np.float64), args.cpu_workers)
        print(f"[bench] cpu baseline: {cpu['wall']:.1f} s on {cpu['workers']} processes", file=sys.stderr, flush=True)

    import torch
    from paper_2204_08269_amd import _lib
    from paper_2204_08269_amd.jtfs import JTFS

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.copy_probe:
        a = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    op = JTFS(p["N"], p["J"], p["Q"], p["J_fr"], p["Q_fr"], p["T"], p["F"], contraction=args.contraction)
    x = torch.from_numpy(x_np).to(dev)
    gs1 = torch.from_numpy(gs1_np).to(dev)
    gs2 = torch.from_numpy(gs2_np).to(dev)
    tuning = None
    if not args.no_autotune and args.contraction is None:
        tuning = op.autotune(B, x, reps=2)      # launch choices for this GPU and batch (before the workspace)
        torch.cuda.synchronize()
        print(f"[bench] autotune: {tuning['contraction']}, register rows {tuning['register_rows']}, "
              f"{tuning['step_ms']:.2f} ms/step", file=sys.stderr, flush=True)
    split = {"split16": True, "split16_phase": "phase"}.get(op.contraction, False)
    ws = op.new_workspace(B)

    def step():
        s1, s2 = op.forward(x, ws)
        gx = op.vjp(x, gs1, gs2, ws=ws, reuse_forward=True)
        return s1, s2, gx

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    _lib.timing_read()                           # clear
    _lib.timing_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        s1, s2, gx = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    _lib.timing_enable(False)
    stages = _lib.timing_read()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    print(f"[bench] {args.steps} timed steps: {ms_per_step:.2f} ms/step", file=sys.stderr, flush=True)
    samples = B * p["N"]
    value = samples / (ms_per_step * 1e-3) / 1e6

    fwd_ms = single_ms = None
    ragged = None
    if not args.no_extras:
        # forward only, batched
        for _ in range(2):
            op.forward(x, ws)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        nf = max(3, args.steps)
        for _ in range(nf):
            op.forward(x, ws)
        torch.cuda.synchronize()
        fwd_ms = (time.perf_counter() - t0) * 1e3 / nf

        # plain single-signal forward (B = 1, eager)
        x1 = x[:1].contiguous()
        ws1 = op.new_workspace(1)
        for _ in range(3):
            op.forward(x1, ws1)
        torch.cuda.synchronize()
        times = []
        for _ in range(20):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            op.forward(x1, ws1)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        single_ms = float(np.median(times)) * 1e3

        # ragged batch (bucketed to power-of-two pads, one graph per run): 256 harmonic
        # tones of log-uniform lengths in [2^13, 2^16], fwd+bwd
        ragged = ragged_batch(torch, dev)

    # rooflines from HIP-event times over the timed region: MFMA stages against
    # their algorithmic flops, FFT stages against their mandatory HBM bytes
    shapes = [Po.T_alpha(a) for a in range(Po.n_alpha)]
    flops = algorithmic_flops(op.info, shapes, B, split)
    nbytes = algorithmic_bytes(op.info, p["N"], shapes, B)
    peak = PEAK_F16_MFMA if split else PEAK_FP32_MFMA
    stage_roofline = {}
    for k, (ms, n) in stages.items():
        if n == 0 or ms <= 0:
            continue
        if k in flops:
            a = flops[k] * args.steps / (ms * 1e-3) / 1e12
            stage_roofline[k] = {"bound": "mfma", "achieved": round(a, 2), "peak": peak, "unit": "TFLOP/s",
                                 "frac": round(a / peak, 4)}
            if split and k != "freq_adj_wh":
                stage_roofline[k]["executed_frac"] = round(3 * a / peak, 4)
        elif k in nbytes:
            a = nbytes[k] * args.steps / (ms * 1e-3) / 1e9
            stage_roofline[k] = {"bound": "hbm", "achieved": round(a, 1), "peak": PEAK_HBM, "unit": "GB/s",
                                 "frac": round(a / PEAK_HBM, 4)}
    dom = max(stage_roofline, key=lambda k: stages[k][0])
    dom_ms, dom_n = stages[dom]
    roofline = dict(stage_roofline[dom])
    traffic = measured_traffic(dom, op.contraction)
    roofline.update({"kernel": dom, "traffic": traffic["bytes_per_launch"] if traffic else None,
                     "traffic_detail": traffic, "launches_per_step": dom_n // args.steps,
                     "avg_launch_ms": round(dom_ms / max(dom_n, 1), 4),
                     "per_launch_algorithmic": (flops[dom] if dom in flops else nbytes[dom]) // max(dom_n // args.steps, 1)})
    if dom in flops:
        roofline["dtype"] = "f16 operands (hi/lo split, 3 products), f32 accumulate" if split else "f32"

    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "Msamples/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic: seeded AM linear/exponential chirps 0.005-0.45 cycles/sample, 20 dB SNR",
        "config": {"workload": "JTFS fwd+bwd, 64 signals x 2^16 samples, J=12, Q=(16,1), J_fr=4, Q_fr=1, "
                               "T=2^11, F=2^3", "global_batch": B, "signal_length": p["N"],
                   "contraction": op.contraction},
        "batched_fwd_msamples_s": round(samples / (fwd_ms * 1e-3) / 1e6, 3) if fwd_ms else None,
        "plain_fwd_single_msamples_s": round(p["N"] / (single_ms * 1e-3) / 1e6, 3) if single_ms else None,
        "plain_fwd_single_ms": round(single_ms, 3) if single_ms else None,
        "tuning": tuning,
        "stage_ms_per_step": {k: round(v[0] / args.steps, 3) for k, v in stages.items()},
        "roofline": roofline,
        "stage_roofline": stage_roofline,
        "ragged_batch": ragged,
    }
    if cpu is not None:
        from tests._util import path_errors, rel_l2
        g1 = s1[0].cpu().numpy()
        g2 = s2[0].cpu().numpy()
        e1, _ = path_errors(g1, cpu["S1"], 1)
        e2, _ = path_errors(g2, cpu["S2"], 3)
        out["rel_err_vs_fp64"] = {"max_path_S1": float(e1.max()), "max_path_S2": float(e2.max()),
                                  "grad_rel_l2": rel_l2(gx[0].cpu().numpy(), cpu["gx"]),
                                  "sample": "signal 0 of the batch, every path"}
        out["cpu_baseline"] = {"value": round(p["N"] / cpu["wall"] / 1e6, 6), "unit": "Msamples/s",
                               "cores": cpu["workers"], "kind": "oracle",
                               "sample": "signal 0 of the batch: FP64 oracle forward + VJP, temporal rates "
                                         f"split over {cpu['workers']} processes; {cpu['wall']:.1f} s wall"}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
