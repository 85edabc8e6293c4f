"""Benchmark of the JTFS hot path on one MI355X.

One step = JTFS forward (S1, S2) plus the backward (VJP) of a fixed random
cotangent, over one batch of synthetic signals resident in HBM.  The headline
workload is the largest single-GPU one: 32 FM mixtures of 2^18 samples (J=14,
Q=(24,2), J_fr=5, Q_fr=2, T=2^14, F=2^4).  Prints one JSON line.

Also reported: batched forward-only and plain single-signal forward throughput,
the 64 x 2^16 chirp workload (fwd+bwd, forward), the 256-signal ragged batch,
100 texture-resynthesis iterations on 8 click trains of 2^17 samples,
per-stage kernel times from HIP events on the launch stream (a separate pass of
the same steps, so that the headline carries no event overhead), the roofline of
the dominant kernel, the FP64 oracle's parity on signal 0, and the oracle's own
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
PEAK_FP32_MFMA = 157.3     # TFLOP/s, MI355X dense FP32 matrix
PEAK_F16_MFMA = 2500.0     # TFLOP/s, MI355X dense FP16 matrix
PEAK_HBM = 8000.0          # GB/s

WORKLOADS = {
    5: dict(name="JTFS fwd+bwd, 32 signals x 2^18 samples, J=14, Q=(24,2), J_fr=5, Q_fr=2, T=2^14, F=2^4",
            tag="32x262144",
            data="synthetic: seeded mixtures of 4 FM sources (carrier 0.005-0.3, modulator 1e-4-5e-3 "
                 "cycles/sample, index 0-5) with random AM, plus Gaussian noise sigma=0.02"),
    2: dict(name="JTFS fwd+bwd, 64 signals x 2^16 samples, J=12, Q=(16,1), J_fr=4, Q_fr=1, T=2^11, F=2^3",
            tag="64x65536",
            data="synthetic: seeded AM linear/exponential chirps 0.005-0.45 cycles/sample, 20 dB SNR"),
}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


# --------------------------------------------------------------------- CPU leg

def _oracle_worker(args):
    """Oracle forward, or VJP, of one signal with the second order restricted to
    a set of temporal rates (first-order terms only where first=True)."""
    cfg, kind, x, gs1, gs2, alphas, first = args
    from oracle import jtfs_oracle as O
    from tests._util import oracle_plan
    P = oracle_plan(synth.PARAMS[cfg])
    if kind == "fwd":
        S1, S2 = O.jtfs(x, P, alphas=alphas)
        return kind, alphas, S1, S2
    g = np.zeros_like(gs2)
    g[alphas] = gs2[alphas]
    return kind, alphas, O.jtfs_vjp(x, gs1 if first else np.zeros_like(gs1), g, P), None


def cpu_baseline(cfg, x0, gs1, gs2, max_workers, sample_alphas=None):
    """FP64 oracle on one signal, forward + VJP, each worker running the unmodified
    oracle.  Without sample_alphas: every temporal rate, the rates split over a
    process pool (one forward and one VJP per worker).  With sample_alphas: the
    forward and the VJP in two processes, the second order restricted to those
    rates (the first order complete)."""
    from tests._util import oracle_plan
    P = oracle_plan(synth.PARAMS[cfg])
    if sample_alphas is None:
        workers = max(1, min(P.n_alpha, max_workers // 2))
        groups = [list(range(i, P.n_alpha, workers)) for i in range(workers)]
    else:
        groups = [list(sample_alphas)]
    jobs = []
    for i, g in enumerate(groups):
        jobs.append((cfg, "fwd", x0, gs1, gs2, g, i == 0))
        jobs.append((cfg, "vjp", x0, gs1, gs2, g, i == 0))
    saved = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")}
    for k in saved:
        os.environ[k] = "1"
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(len(jobs)) as pool:
        res = pool.map(_oracle_worker, jobs)
    wall = time.perf_counter() - t0
    for k, v in saved.items():
        if v is None:
            os.environ.pop(k, None)
        else:
            os.environ[k] = v
    S1 = next(r[2] for r in res if r[0] == "fwd")          # every forward computes the same first order
    S2 = np.full(P.s2_shape(), np.nan)
    gx = np.zeros(P.N)
    for kind, alphas, a, b in res:
        if kind == "fwd":
            S2[alphas] = b[alphas]
        else:
            gx += a
    return dict(wall=wall, processes=len(jobs), S1=S1, S2=S2, gx=gx,
                alphas=sorted(a for g in groups for a in g), n_alpha=P.n_alpha)


# --------------------------------------------------------------------- GPU leg

def algorithmic_flops(info, shapes, B, mode, fp32_backward):
    """Dense-contraction flops of the frequential stage per step (unpadded sizes):
    forward 8 M_h n1 T_alpha + time lowpass 2 (2 M_h) T_alpha N/T per signal and
    rate; the recomputing backward repeats both and adds the W^H product 8 M_h n1
    T_alpha (one fused kernel with split operands; two kernels, recompute and W^H,
    on the FP32 path).  With the stored phase the backward recomputes neither the
    contraction nor the modulus: it does the lowpass adjoint and the W^H product."""
    Mh, n1, NT = info.M_h, info.n1, info.out_t
    fwd = sum(8 * Mh * n1 * Ta + 4 * Mh * Ta * NT for Ta in shapes) * B
    lp = sum(4 * Mh * Ta * NT for Ta in shapes) * B
    wh = sum(8 * Mh * n1 * Ta for Ta in shapes) * B
    if fp32_backward:
        return {"freq_fwd": fwd, "freq_adj_pq": fwd, "freq_adj_wh": wh}
    if mode == "split16_phase":
        return {"freq_fwd": fwd, "freq_adj_pq": lp + wh}
    return {"freq_fwd": fwd, "freq_adj_pq": fwd + wh}


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
# Keyed by (stage, contraction mode, tile of that stage's kernel).
TRAFFIC_KERNELS = {("freq_fwd", "split16", 32): "k_freq_fwd_h", ("freq_adj_pq", "split16", 32): "k_freq_bwd_h",
                   ("freq_fwd", "split16_phase", 32): "k_freq_fwd_h_phase",
                   ("freq_adj_pq", "split16_phase", 32): "k_freq_bwd_p",
                   ("freq_fwd", "split16", 16): "k_freq_fwd_q",
                   ("freq_fwd", "split16_phase", 16): "k_freq_fwd_q_phase",
                   ("freq_adj_pq", "split16_phase", 16): "k_freq_bwd_q"}
TRAFFIC_SOURCE = "paper_2204_08269_amd/csrc/split.hip"


def measured_traffic(stage, contraction, tile, tag):
    import hashlib
    kern = TRAFFIC_KERNELS.get((stage, contraction, tile))
    if kern is None:
        return None
    rec_path = os.path.join(HERE, "profiles", f"{kern}_{tag}_hbm_traffic.json")
    if not os.path.exists(rec_path):
        return None
    rec = json.load(open(rec_path))
    src = os.path.join(HERE, TRAFFIC_SOURCE)
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
    bk = JTFSBucket(lengths, p["J"], p["Q"], p["J_fr"], p["Q_fr"], p["T"], p["F"], autotune=True)
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
    pads = list(bk.pads)
    del bk
    # each bucket alone (its signals as a ragged batch of one pad), for comparison
    # with the run that holds them all as parallel branches of one graph
    alone = {}
    for pad in sorted(set(pads)):
        idx = [i for i, n in enumerate(pads) if n == pad]
        b1 = JTFSBucket([lengths[i] for i in idx], p["J"], p["Q"], p["J_fr"], p["Q_fr"], p["T"], p["F"], autotune=True)
        x1 = torch.from_numpy(np.concatenate([sigs[i] for i in idx])).to(dev)
        g1 = torch.from_numpy(np.random.default_rng(5).standard_normal(b1.s_offset[-1]).astype(np.float32)).to(dev)
        o1 = torch.empty(b1.s_offset[-1], dtype=torch.float32, device=dev)
        gx1 = torch.empty(b1.x_offset[-1], dtype=torch.float32, device=dev)
        with torch.cuda.stream(st):
            b1.run(x1, g1, o1, gx1)
            st.synchronize()
            t0 = time.perf_counter()
            for _ in range(runs):
                b1.run(x1, g1, o1, gx1)
            st.synchronize()
            alone[str(pad)] = round((time.perf_counter() - t0) * 1e3 / runs, 3)
        del b1, x1, g1, o1, gx1
    print(f"[bench] ragged batch: buckets alone {alone} ms, sum {sum(alone.values()):.2f}", file=sys.stderr,
          flush=True)
    return {"workload": "256 harmonic tones + pink noise, lengths log-uniform in [2^13, 2^16], J=11, Q=(16,1), "
                        "J_fr=4, Q_fr=1, T=2^10, F=2^3; buckets of power-of-two pads, each bucket's plan autotuned, "
                        "one HIP graph per run",
            "ms_per_run": round(ms, 3), "fwd_bwd_msamples_s_real": round(real / (ms * 1e-3) / 1e6, 3),
            "fwd_bwd_msamples_s_padded": round(padded / (ms * 1e-3) / 1e6, 3),
            "real_samples": real, "padded_samples": padded, "signals_per_pad": counts,
            "bucket_alone_ms": alone, "sum_of_buckets_alone_ms": round(sum(alone.values()), 3)}


def texture_leg(torch, dev, iters=100, mu0=-0.05):
    """Texture resynthesis (sec. 5) of the 8 click-train targets of 2^17 samples
    (J=13, Q=(12,1), J_fr=4, Q_fr=2, T=2^13, F=2^3) from their white-noise starts:
    `iters` bold-driver iterations (one candidate forward + backward each, on
    the device), the normalised error ||Sx - Sy|| / ||Sx|| after 20 and after
    `iters` iterations, and the time per iteration (one recorded graph replayed;
    its capture included)."""
    from paper_2204_08269_amd.jtfs import JTFS, Texture
    p = synth.PARAMS[3]
    y, x0 = synth.cfg3_batch()
    op = JTFS(p["N"], p["J"], p["Q"], p["J_fr"], p["Q_fr"], p["T"], p["F"])
    tex = Texture(op, y.shape[0], mu0)
    yt, x0t = torch.from_numpy(y).to(dev), torch.from_numpy(x0).to(dev)
    tex.set_target(yt)
    tex.set_start(x0t)
    e0 = tex.read()[1].cpu().numpy()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hist = tex.iterate(iters)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / iters
    h = hist.cpu().numpy()
    print(f"[bench] texture: {ms:.2f} ms per iteration, median E {np.median(h[19]):.3f} after 20, "
          f"{np.median(h[-1]):.3f} after {iters}", file=sys.stderr, flush=True)
    del tex, op
    return {"workload": "texture resynthesis of 8 click trains x 2^17 samples (J=13, Q=(12,1), J_fr=4, Q_fr=2, "
                        "T=2^13, F=2^3) from white noise at the targets' RMS, bold driver, initial rate 0.05 "
                        "||y0|| / ||grad E(y0)||",
            "iterations": iters, "ms_per_iteration": round(ms, 3),
            "error_start": [round(float(v), 4) for v in e0],
            "error_after_20": [round(float(v), 4) for v in h[19]],
            f"error_after_{iters}": [round(float(v), 4) for v in h[-1]],
            "median_error_after_20": round(float(np.median(h[19])), 4),
            f"median_error_after_{iters}": round(float(np.median(h[-1])), 4),
            "paper_context": "about 10 % after 20 and 3 % after 100 iterations and 720 ms per iteration "
                             "(one bird-call recording of 2^16 samples, GPU not stated; sec. 5)"}


def _graph_ms(res):
    """Single-signal forward time from graph replays (ms, rounded), or the reason there is none."""
    v = res.get("single_graph_ms")
    return round(v, 3) if isinstance(v, float) else v


def _time_ms(torch, fn, n):
    """Mean wall time of fn over n calls (after one untimed call), GPU synchronised."""
    fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(n):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / n


def run_workload(torch, dev, cfg, args, extras=True, stage_pass=True):
    """Autotune, warm up and time `args.steps` fwd+bwd steps of workload cfg; then
    (optionally) the same steps again with per-stage HIP events, a batched
    forward-only run and the plain single-signal forward (B = 1, eager, split16
    without phase storage)."""
    from paper_2204_08269_amd import _lib
    from paper_2204_08269_amd.jtfs import JTFS
    from tests._util import oracle_plan
    p = synth.PARAMS[cfg]
    B = synth.BATCH[cfg]
    Po = oracle_plan(p)
    x_np = synth.batch(cfg)
    gs1_np, gs2_np = synth.cotangents((B,) + Po.s1_shape(), (B,) + Po.s2_shape())
    op = JTFS(p["N"], p["J"], p["Q"], p["J_fr"], p["Q_fr"], p["T"], p["F"], contraction=args.contraction)
    x = torch.from_numpy(x_np).to(dev)
    gs1 = torch.from_numpy(gs1_np).to(dev)
    gs2 = torch.from_numpy(gs2_np).to(dev)
    tuning = None
    if not args.no_autotune and args.contraction is None:
        tuning = op.autotune(B, x, reps=2)      # launch choices for this GPU and batch (before the workspace)
        torch.cuda.synchronize()
        print(f"[bench] cfg {cfg} autotune: {tuning['contraction']}, register rows {tuning['register_rows']}, "
              f"tiles {tuning['fwd_tile']}/{tuning['bwd_tile']}, {tuning['step_ms']:.2f} ms/step", file=sys.stderr,
              flush=True)
    elif args.fwd_tile or args.bwd_tile or args.radix8:
        mode, rows, ft, bt = op.tuning()
        r8 = [v for v in args.radix8.split(",") if v] if args.radix8 else []
        op.set_tuning(mode, rows, fwd_tile=args.fwd_tile or ft, bwd_tile=args.bwd_tile or bt, radix8=r8)
    ws = op.new_workspace(B)

    def step():
        s1, s2 = op.forward(x, ws)
        gx = op.vjp(x, gs1, gs2, ws=ws, reuse_forward=True)
        return s1, s2, gx

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        s1, s2, gx = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    samples = B * p["N"]
    print(f"[bench] cfg {cfg}: {args.steps} timed steps, {ms_per_step:.2f} ms/step", file=sys.stderr, flush=True)
    res = {"cfg": cfg, "B": B, "N": p["N"], "op": op, "x": x, "ws": ws, "s1": s1, "s2": s2, "gx": gx,
           "ms_per_step": ms_per_step, "value": samples / (ms_per_step * 1e-3) / 1e6, "tuning": tuning,
           "contraction": op.contraction, "Po": Po, "tiles": tuple(op.tuning()[2:])}
    if stage_pass:
        _lib.timing_read()                       # clear
        _lib.timing_enable(True)
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        _lib.timing_enable(False)
        res["stages"] = _lib.timing_read()
    if extras:
        for _ in range(2):
            op.forward(x, ws)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        nf = max(3, args.steps)
        for _ in range(nf):
            op.forward(x, ws)
        torch.cuda.synchronize()
        res["fwd_ms"] = (time.perf_counter() - t0) * 1e3 / nf
        # mu-log (sec. 4) fused into the output kernels, against the forward
        # followed by the separate mu-log pass; mu from this batch's path means
        mu1, mu2 = op.path_means(s1, s2)

        def separate():
            a1, a2 = op.forward(x, ws)
            op.mulog(a1, a2, mu1, mu2)

        res["mulog_ms"] = {"fused": _time_ms(torch, lambda: op.forward_mulog(x, mu1, mu2, ws=ws), nf),
                           "separate": _time_ms(torch, separate, nf)}
        # plain single-signal forward: no stored phase (a plain forward has no
        # backward to serve), same plan parameters
        plain = "split16" if op.contraction == "split16_phase" else op.contraction
        op1 = JTFS(p["N"], p["J"], p["Q"], p["J_fr"], p["Q_fr"], p["T"], p["F"], contraction=plain)   # a plan of its own
        x1 = x[:1].contiguous()
        if not args.no_autotune:
            # launch choices for one signal (the t-chunk above all), in the plain mode
            t1 = op1.autotune(1, x1, reps=3)
            op1.set_tuning(plain, t1["register_rows"], fwd_tile=t1["fwd_tile"], bwd_tile=t1["bwd_tile"],
                           radix8=t1["radix8"], lds_batch=t1["lds_batch"], t_chunk=t1["t_chunk"])
            res["single_tuning"] = {k: t1[k] for k in ("register_rows", "fwd_tile", "radix8", "lds_batch", "t_chunk")}
        ws1 = op1.new_workspace(1)
        for _ in range(3):
            op1.forward(x1, ws1)
        torch.cuda.synchronize()
        times = []
        for _ in range(20):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            op1.forward(x1, ws1)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        res["single_ms"] = float(np.median(times)) * 1e3
        res["single_contraction"] = plain
        # the same forward replayed from a captured HIP graph (no host launch cost
        # per kernel); reported only if a replay equals the eager forward bit for bit
        try:
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g):
                c1, c2 = op1.forward(x1, ws1)
            g.replay()
            torch.cuda.synchronize()
            e1, e2 = op1.forward(x1, ws1)
            torch.cuda.synchronize()
            if torch.equal(c1, e1) and torch.equal(c2, e2):
                times = []
                for _ in range(20):
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    g.replay()
                    torch.cuda.synchronize()
                    times.append(time.perf_counter() - t0)
                res["single_graph_ms"] = float(np.median(times)) * 1e3
            else:
                res["single_graph_ms"] = "replay differs from the eager forward"
            del g, c1, c2, e1, e2
        except RuntimeError as e:
            res["single_graph_ms"] = f"capture failed: {e}"
        del ws1, op1
    return res


def rooflines(res, steps):
    """Per-stage rates from the event pass (MFMA stages against their algorithmic
    flops, FFT stages against their mandatory HBM bytes) and the dominant stage's
    roofline object."""
    op, Po, B = res["op"], res["Po"], res["B"]
    stages = res["stages"]
    shapes = [Po.T_alpha(a) for a in range(Po.n_alpha)]
    mode = op.contraction
    split = mode != "fp32"
    fp32_bwd = stages.get("freq_adj_wh", (0, 0))[1] > 0          # the FP32 backward pair ran
    flops = algorithmic_flops(op.info, shapes, B, mode, fp32_bwd)
    nbytes = algorithmic_bytes(op.info, res["N"], shapes, B)
    out = {}
    for k, (ms, n) in stages.items():
        if n == 0 or ms <= 0:
            continue
        if k in flops:
            on_split = split and not (fp32_bwd and k != "freq_fwd")
            peak = PEAK_F16_MFMA if on_split else PEAK_FP32_MFMA
            a = flops[k] * steps / (ms * 1e-3) / 1e12
            out[k] = {"bound": "mfma", "achieved": round(a, 2), "peak": peak, "unit": "TFLOP/s",
                      "frac": round(a / peak, 4),
                      "dtype": "f16 operands (hi/lo split, 3 products), f32 accumulate" if on_split else "f32"}
            if on_split:
                out[k]["executed_frac"] = round(3 * a / peak, 4)
        elif k in nbytes:
            a = nbytes[k] * steps / (ms * 1e-3) / 1e9
            out[k] = {"bound": "hbm", "achieved": round(a, 1), "peak": PEAK_HBM, "unit": "GB/s",
                      "frac": round(a / PEAK_HBM, 4)}
    dom = max(out, key=lambda k: stages[k][0])
    dom_ms, dom_n = stages[dom]
    roof = dict(out[dom])
    tile = res["tiles"][0] if dom == "freq_fwd" else res["tiles"][1]
    traffic = measured_traffic(dom, mode, tile, WORKLOADS[res["cfg"]]["tag"])
    per_step = max(dom_n // steps, 1)
    roof.update({"kernel": dom, "tile": tile, "traffic": traffic["bytes_per_launch"] if traffic else None,
                 "traffic_detail": traffic, "launches_per_step": per_step,
                 "avg_launch_ms": round(dom_ms / max(dom_n, 1), 4),
                 "per_launch_algorithmic": (flops[dom] if dom in flops else nbytes[dom]) // per_step,
                 "timing": "HIP events on the launch stream around every launch, over a second pass of the "
                           "timed steps"})
    return roof, out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cfg", type=int, choices=sorted(WORKLOADS), default=5,
                    help="headline workload (5: 32 x 2^18, the largest single-GPU one; 2: 64 x 2^16)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-workers", type=int, default=16)
    ap.add_argument("--contraction", choices=["split16", "split16_phase", "fp32"], default=None,
                    help="frequential contraction arithmetic (default: autotuned)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run one 1 GiB device copy first (calibrates HBM byte counters)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the plan's default launch choices (no autotuning before the timed steps)")
    ap.add_argument("--fwd-tile", type=int, choices=[16, 32], default=None,
                    help="with --no-autotune: MFMA tile of the split forward contraction")
    ap.add_argument("--bwd-tile", type=int, choices=[16, 32], default=None,
                    help="with --no-autotune: MFMA tile of the stored-phase backward")
    ap.add_argument("--radix8", default="",
                    help="with --no-autotune: comma-separated stages whose register-resident transforms use "
                         "radix-8 passes (scalogram, second_order, row_fft, first_adj)")
    ap.add_argument("--no-extras", action="store_true",
                    help="time the fwd+bwd step only (no event pass, forward-only, second-workload or ragged legs)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: this library has no multi-GPU path "
              "(signals shard across GPUs with no communication; see the design notes)", file=sys.stderr)
        sys.exit(2)

    cfg = args.cfg
    p = synth.PARAMS[cfg]
    from tests._util import oracle_plan
    Po = oracle_plan(p)
    # the oracle needs minutes per 2^18 signal: its second order is sampled at
    # one temporal rate there (the first order is complete)
    sample_alphas = [Po.n_alpha // 2] if cfg == 5 else None
    cpu = None
    if not args.no_cpu_baseline:
        x0 = synth.batch(cfg, B=1)[0].astype(np.float64)
        B = synth.BATCH[cfg]
        g1, g2 = synth.cotangents((B,) + Po.s1_shape(), (B,) + Po.s2_shape())
        cpu = cpu_baseline(cfg, x0, g1[0].astype(np.float64), g2[0].astype(np.float64), args.cpu_workers,
                           sample_alphas)
        print(f"[bench] cpu baseline: {cpu['wall']:.1f} s on {cpu['processes']} processes", file=sys.stderr,
              flush=True)

    import torch

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.copy_probe:
        a = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    extras = not args.no_extras
    res = run_workload(torch, dev, cfg, args, extras=extras, stage_pass=extras)
    out = {
        "metric": METRIC, "value": round(res["value"], 3), "unit": "Msamples/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(res["ms_per_step"], 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 (frequential contraction: f16 hi/lo split, 3 products, f32 accumulate)"
                 if res["contraction"] != "fp32" else "f32",
        "data": WORKLOADS[cfg]["data"],
        "config": {"workload": WORKLOADS[cfg]["name"], "global_batch": res["B"], "signal_length": res["N"],
                   "contraction": res["contraction"]},
        "tuning": res["tuning"],
    }
    if extras:
        roof, stage_roof = rooflines(res, args.steps)
        out["batched_fwd_msamples_s"] = round(res["B"] * res["N"] / (res["fwd_ms"] * 1e-3) / 1e6, 3)
        out["plain_fwd_single_msamples_s"] = round(res["N"] / (res["single_ms"] * 1e-3) / 1e6, 3)
        out["plain_fwd_single_ms"] = round(res["single_ms"], 3)
        out["plain_fwd_single_contraction"] = res["single_contraction"]
        out["plain_fwd_single_graph_ms"] = _graph_ms(res)
        if "single_tuning" in res:
            out["plain_fwd_single_tuning"] = res["single_tuning"]
        out["mulog_fwd_ms"] = {k: round(v, 3) for k, v in res["mulog_ms"].items()}
        out["stage_ms_per_step"] = {k: round(v[0] / args.steps, 3) for k, v in res["stages"].items()}
        out["roofline"] = roof
        out["stage_roofline"] = stage_roof
    if cpu is not None:
        from tests._util import path_errors, rel_l2
        op = res["op"]
        alphas = cpu["alphas"]
        e1, _ = path_errors(res["s1"][0].cpu().numpy(), cpu["S1"], 1)
        e2, _ = path_errors(res["s2"][0].cpu().numpy()[alphas], cpu["S2"][alphas], 3)
        if sample_alphas is None:
            gx0 = res["gx"][0].cpu().numpy()
        else:
            # the gradient of the same cotangent restricted to the sampled rates (untimed)
            B = res["B"]
            g1, g2 = synth.cotangents((B,) + Po.s1_shape(), (B,) + Po.s2_shape())
            keep = np.zeros(Po.n_alpha, bool)
            keep[alphas] = True
            g2[:, ~keep] = 0.0
            gx0 = op.vjp(res["x"], torch.from_numpy(g1).to(dev), torch.from_numpy(g2).to(dev),
                         ws=res["ws"])[0].cpu().numpy()
        what = "every path" if sample_alphas is None else f"S1 every path, S2 every path at temporal rate(s) {alphas}"
        out["rel_err_vs_fp64"] = {"max_path_S1": float(e1.max()), "max_path_S2": float(e2.max()),
                                  "grad_rel_l2": rel_l2(gx0, cpu["gx"]),
                                  "sample": f"signal 0 of the batch, {what}"}
        covered = ("every temporal rate" if sample_alphas is None else
                   f"the first order complete and the second order at {len(alphas)} of {cpu['n_alpha']} "
                   "temporal rates, so the rate is an upper bound on the oracle's full-transform rate")
        out["cpu_baseline"] = {"value": round(res["N"] / cpu["wall"] / 1e6, 6), "unit": "Msamples/s",
                               "cores": cpu["processes"], "host_cpus": os.cpu_count(), "cpu_model": cpu_model(),
                               "kind": "oracle",
                               "sample": f"signal 0 of the batch: FP64 oracle forward + VJP in {cpu['processes']} "
                                         f"single-threaded processes, {covered}; {cpu['wall']:.1f} s wall"}
    # release the headline workload before the secondary ones
    for k in ("ws", "s1", "s2", "gx", "x"):
        res.pop(k, None)
    del res
    torch.cuda.empty_cache()
    if extras and cfg != 2:
        r2 = run_workload(torch, dev, 2, args, extras=True, stage_pass=False)
        out["cfg2"] = {"workload": WORKLOADS[2]["name"], "contraction": r2["contraction"],
                       "fwd_bwd_msamples_s": round(r2["value"], 3), "ms_per_step": round(r2["ms_per_step"], 3),
                       "batched_fwd_msamples_s": round(r2["B"] * r2["N"] / (r2["fwd_ms"] * 1e-3) / 1e6, 3),
                       "plain_fwd_single_msamples_s": round(r2["N"] / (r2["single_ms"] * 1e-3) / 1e6, 3),
                       "plain_fwd_single_ms": round(r2["single_ms"], 3),
                       "plain_fwd_single_contraction": r2["single_contraction"],
                       "plain_fwd_single_graph_ms": _graph_ms(r2)}
        del r2
        torch.cuda.empty_cache()
    if extras:
        out["ragged_batch"] = ragged_batch(torch, dev)
        torch.cuda.empty_cache()
        out["texture"] = texture_leg(torch, dev)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
