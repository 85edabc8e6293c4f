"""GPU parity: the HIP path through the C ABI against the FP64 oracle, on seeded
inputs, per coefficient path (relative L2 <= 1e-5 for the transform)."""
import numpy as np
import pytest
import torch

import synth
from oracle import jtfs_oracle as O
from tests._util import oracle_plan, path_errors, rel_l2

pytestmark = pytest.mark.gpu

TOL = 1e-5          # per-path relative L2 of S1 and S2 against FP64
TOL_VJP = 1e-4      # relative L2 of the gradient against the FP64 oracle's VJP
TOL_FD = 1e-3       # gradient against FP64 central finite differences


def gpu_op(p, contraction=None, average_fr=True, time_scattering=False):
    from paper_2204_08269_amd.jtfs import JTFS
    return JTFS(p["N"], p["J"], p["Q"], p["J_fr"], p["Q_fr"], p["T"], p["F"], contraction=contraction,
                average_fr=average_fr, time_scattering=time_scattering,
                lowpass_pairs=p.get("lowpass_pairs", False), unpad_lambda=p.get("unpad", False))


MODES = ["fp32", "split16"]
ALL_ROWS = ["scalogram", "second_order", "row_fft", "first_adj"]      # register-resident rows of 2^14 points


def run_forward(op, x):
    xt = torch.from_numpy(x).cuda()
    s1, s2 = op.forward(xt)
    torch.cuda.synchronize()
    return s1.cpu().numpy(), s2.cpu().numpy()


def check_paths(g1, g2, r1, r2, tol=TOL, alphas=None):
    e1, _ = path_errors(g1, r1, 1)
    if alphas is not None:
        g2 = g2[alphas]
        r2 = r2[alphas]
    e2, _ = path_errors(g2, r2, 3)
    assert e1.max() <= tol, f"S1 worst path error {e1.max():.3e} at {np.unravel_index(e1.argmax(), e1.shape)}"
    assert e2.max() <= tol, f"S2 worst path error {e2.max():.3e} at {np.unravel_index(e2.argmax(), e2.shape)}"
    return e1.max(), e2.max()


P1 = synth.PARAMS[1]
RAGGED = [
    dict(N=2048, J=6, Q=(8, 1), J_fr=3, Q_fr=1, T=2048, F=2),     # T = N: one frame; 224 rows (ragged tile)
    dict(N=1024, J=5, Q=(4, 1), J_fr=2, Q_fr=1, T=32, F=1),       # F = 1: no log-frequency decimation
    dict(N=4096, J=7, Q=(12, 2), J_fr=3, Q_fr=2, T=128, F=4),     # Q2 = 2, n1 = 70 (K tail)
    dict(N=8192, J=9, Q=(6, 1), J_fr=3, Q_fr=1, T=512, F=4),      # kX = 1
]


def test_filter_tables_match_oracle():
    for p in (P1, synth.PARAMS[2]):
        op = gpu_op(p)
        P = oracle_plan(p)
        t0 = op.table(0)
        ref0 = P.psi1_hat[:, : p["N"] // 2 + 1]
        assert np.max(np.abs(t0 - ref0)) <= 2e-7 * np.max(ref0)
        t1 = op.table(1)
        ref1 = P.psi2_hat[:, : P.NX // 2 + 1]
        assert np.max(np.abs(t1 - ref1)) <= 2e-7 * np.max(ref1)
        t2 = op.table(2)
        ref2 = np.concatenate([P.freq_wavelet_matrix(b, 0) for b in range(P.n_beta)])
        assert np.max(np.abs(t2 - ref2)) <= 2e-7 * np.max(np.abs(ref2))


@pytest.mark.parametrize("mode", MODES)
def test_forward_parity_cfg1_batch(mode):
    x = synth.batch(1, B=3)
    op = gpu_op(P1, mode)
    assert op.contraction == mode
    g1, g2 = run_forward(op, x)
    P = oracle_plan(P1)
    for b in range(3):
        r1, r2 = O.jtfs(x[b].astype(np.float64), P)
        check_paths(g1[b], g2[b], r1, r2)


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("p", RAGGED)
def test_forward_parity_ragged_shapes(p, mode):
    rng = np.random.default_rng(p["N"] + p["T"])
    x = (rng.standard_normal((2, p["N"])) * 0.5).astype(np.float32)
    op = gpu_op(p, mode)
    g1, g2 = run_forward(op, x)
    P = oracle_plan(p)
    for b in range(2):
        r1, r2 = O.jtfs(x[b].astype(np.float64), P)
        check_paths(g1[b], g2[b], r1, r2)


@pytest.mark.parametrize("mode", MODES)
def test_forward_parity_cfg2_full_batch_sampled(mode):
    """64 x 2^16 chirps in the benchmark's launch configuration; the oracle
    checks two signals on every S1 path and on three temporal rates of S2."""
    p = synth.PARAMS[2]
    x = synth.batch(2)
    op = gpu_op(p, mode)
    g1, g2 = run_forward(op, x)
    P = oracle_plan(p)
    alphas = [0, 6, P.n_alpha - 1]
    for b in (0, 63):
        r1, r2 = O.jtfs(x[b].astype(np.float64), P, alphas=alphas)
        check_paths(g1[b], g2[b], r1, r2, alphas=alphas)


@pytest.mark.parametrize("mode", MODES)
def test_pure_tone_closed_form_on_gpu(mode):
    """S1 of A cos(2 pi m n/N) is (A/2) |psi_hat_lambda(m/N)| and S2 vanishes."""
    N, m, A = P1["N"], 301, 0.7
    x = synth.tone(N, m, A, 0.3).astype(np.float32)[None]
    op = gpu_op(P1, mode)
    g1, g2 = run_forward(op, x)
    P = oracle_plan(P1)
    expect = 0.5 * A * np.abs(P.psi1_hat[:, m])
    assert np.max(np.abs(g1[0] - expect[:, None])) <= 1e-5 * expect.max()
    assert np.max(np.abs(g2)) <= 1e-5 * expect.max()


def test_zero_input_gives_zero_and_finite_gradient():
    op = gpu_op(P1)
    x = torch.zeros((2, P1["N"]), device="cuda")
    s1, s2 = op.forward(x)
    g = op.vjp(x, torch.ones_like(s1), torch.ones_like(s2))
    torch.cuda.synchronize()
    assert float(s1.abs().max()) == 0.0 and float(s2.abs().max()) == 0.0
    assert torch.isfinite(g).all() and float(g.abs().max()) == 0.0


@pytest.mark.parametrize("mode", MODES)
def test_batch_invariance_and_determinism(mode):
    x = synth.batch(1, B=4)
    op = gpu_op(P1, mode)
    a1, a2 = run_forward(op, x)
    b1, b2 = run_forward(op, x)
    assert np.array_equal(a1, b1) and np.array_equal(a2, b2)          # run to run
    for b in range(4):
        c1, c2 = run_forward(op, x[b:b + 1])
        assert np.array_equal(c1[0], a1[b]) and np.array_equal(c2[0], a2[b])   # batch = stacked singles


def test_vjp_parity_cfg1():
    x = synth.batch(1, B=2)
    P = oracle_plan(P1)
    gs1, gs2 = synth.cotangents((2,) + P.s1_shape(), (2,) + P.s2_shape())
    op = gpu_op(P1)
    xt = torch.from_numpy(x).cuda()
    g = op.vjp(xt, torch.from_numpy(gs1).cuda(), torch.from_numpy(gs2).cuda()).cpu().numpy()
    for b in range(2):
        ref = O.jtfs_vjp(x[b].astype(np.float64), gs1[b].astype(np.float64), gs2[b].astype(np.float64), P)
        err = rel_l2(g[b], ref)
        assert err <= TOL_VJP, f"signal {b}: relative L2 {err:.3e}"


@pytest.mark.parametrize("p", RAGGED[:2])
def test_vjp_parity_ragged(p):
    rng = np.random.default_rng(p["N"] + 7)
    x = (rng.standard_normal((1, p["N"])) * 0.5).astype(np.float32)
    P = oracle_plan(p)
    gs1, gs2 = synth.cotangents((1,) + P.s1_shape(), (1,) + P.s2_shape(), seed=3)
    op = gpu_op(p)
    g = op.vjp(torch.from_numpy(x).cuda(), torch.from_numpy(gs1).cuda(), torch.from_numpy(gs2).cuda()).cpu().numpy()
    ref = O.jtfs_vjp(x[0].astype(np.float64), gs1[0].astype(np.float64), gs2[0].astype(np.float64), P)
    assert rel_l2(g[0], ref) <= TOL_VJP


def test_gradient_matches_finite_differences():
    """GPU gradient of <gS, S(x)> against FP64 central differences of the
    transform along random directions (N = 2048 instance)."""
    x = synth.batch(1, B=1)
    P = oracle_plan(P1)
    gs1, gs2 = synth.cotangents((1,) + P.s1_shape(), (1,) + P.s2_shape())
    op = gpu_op(P1)
    g = op.vjp(torch.from_numpy(x).cuda(), torch.from_numpy(gs1).cuda(), torch.from_numpy(gs2).cuda())
    g = g.cpu().numpy()[0].astype(np.float64)
    x0 = x[0].astype(np.float64)
    rng = np.random.default_rng(9)
    for _ in range(3):
        v = rng.standard_normal(P1["N"])
        h = 1e-6
        fd = (O.loss(x0 + h * v, gs1[0], gs2[0], P) - O.loss(x0 - h * v, gs1[0], gs2[0], P)) / (2 * h)
        assert abs(g @ v - fd) <= TOL_FD * abs(fd)


def test_autograd_function_matches_vjp():
    x = torch.from_numpy(synth.batch(1, B=2)).cuda().requires_grad_(True)
    op = gpu_op(P1)
    P = oracle_plan(P1)
    gs1, gs2 = synth.cotangents((2,) + P.s1_shape(), (2,) + P.s2_shape())
    gs1, gs2 = torch.from_numpy(gs1).cuda(), torch.from_numpy(gs2).cuda()
    s1, s2 = op(x)
    ((s1 * gs1).sum() + (s2 * gs2).sum()).backward()
    g_ref = op.vjp(x.detach(), gs1, gs2)
    torch.cuda.synchronize()
    assert torch.equal(x.grad, g_ref)
    # without a graph to record, the call returns the same coefficients from the plan's workspace
    with torch.no_grad():
        n1, n2 = op(x)
    assert not n1.requires_grad and torch.equal(n1, s1.detach()) and torch.equal(n2, s2.detach())


def test_plan_create_signature_matches_ex():
    """jtfs_plan_create(N, J, Q[2], J_fr, Q_fr, T, F) builds the plan that
    jtfs_plan_create_ex builds with no flags: the same sizes, workspace sizes per
    signal that jtfs_workspace_size confirms, and bit-identical coefficients."""
    import ctypes
    from paper_2204_08269_amd import _lib
    L = _lib.load()
    p = P1
    plan = ctypes.c_void_p()
    _lib.check(L.jtfs_plan_create(ctypes.byref(plan), p["N"], p["J"], (ctypes.c_int * 2)(*p["Q"]), p["J_fr"],
                                  p["Q_fr"], p["T"], p["F"]))
    try:
        info = _lib.Info()
        _lib.check(L.jtfs_plan_info(plan, ctypes.byref(info)))
        op = gpu_op(p)
        for k in ("n1", "n_alpha", "n_beta", "L", "M_h", "out_t", "out_l", "s1_per_signal", "s2_per_signal",
                  "ws_fwd", "ws_bwd"):
            assert getattr(info, k) == getattr(op.info, k), k
        n = ctypes.c_size_t(0)
        _lib.check(L.jtfs_workspace_size(plan, 1, ctypes.byref(n)))
        assert n.value == info.ws_bwd
        _lib.check(L.jtfs_forward_workspace_size(plan, 1, ctypes.byref(n)))
        assert n.value == info.ws_fwd
        xt = torch.from_numpy(synth.batch(1, B=2)).cuda()
        _lib.check(L.jtfs_workspace_size(plan, 2, ctypes.byref(n)))
        ws = torch.empty(n.value, dtype=torch.uint8, device="cuda")
        s1 = torch.empty((2,) + op.s1_shape, dtype=torch.float32, device="cuda")
        s2 = torch.empty((2,) + op.s2_shape, dtype=torch.float32, device="cuda")
        _lib.check(L.jtfs_forward(plan, ctypes.c_void_p(xt.data_ptr()), 2, ctypes.c_void_p(s1.data_ptr()),
                                  ctypes.c_void_p(s2.data_ptr()), ctypes.c_void_p(ws.data_ptr()), n.value,
                                  ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))
        r1, r2 = op.forward(xt)
        torch.cuda.synchronize()
        assert torch.equal(s1, r1) and torch.equal(s2, r2)
        # its filterbanks and schedule (host FP64) against the oracle's own solve
        P = oracle_plan(p)
        n = P.n1 + P.n_alpha + P.n_beta
        xs = (ctypes.c_double * (2 * n))()
        sched = (ctypes.c_int32 * (1 + P.n_alpha + P.n_beta))()
        _lib.check(L.jtfs_plan_tables(plan, xs, sched))
        xs = np.array(xs).reshape(n, 2)
        ref = np.concatenate([np.stack([P.xi1, P.sigma1], 1), np.stack([P.xi2, P.sigma2], 1),
                              np.stack([P.xi_fr, P.sigma_fr], 1)])
        assert np.max(np.abs(xs - ref) / ref) <= 1e-13
        assert list(sched) == [P.kX] + list(P.k2) + list(P.k_fr)
    finally:
        L.jtfs_plan_destroy(plan)


def test_forward_captured_in_a_graph_replays_like_eager():
    """The forward allocates nothing and records no memset, so a caller can capture
    it in a HIP graph (torch.cuda.graph) on fixed buffers: three replays on new
    inputs, each followed by an eager forward on another workspace and a
    synchronisation, give the eager coefficients bit for bit."""
    op = gpu_op(P1, contraction="split16_phase")
    B = 2
    ws, ws_eager = op.new_workspace(B), op.new_workspace(B)
    static_x = torch.from_numpy(synth.batch(1, B=B)).cuda()
    op.forward(static_x, ws)                     # warm-up outside the capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        o1, o2 = op.forward(static_x, ws)
    for k in range(3):
        xk = torch.from_numpy(synth.batch(1, B=B, offset=2 * (k + 1))).cuda()
        static_x.copy_(xk)
        g.replay()
        r1, r2 = op.forward(xk, ws_eager)
        torch.cuda.synchronize()
        assert torch.equal(o1, r1) and torch.equal(o2, r2), f"replay {k}"


@pytest.mark.parametrize("autotune", [False, True])
def test_ragged_bucket_graph_matches_oracle_and_replays(autotune):
    """Uneven lengths, bucketed to powers of two and run as one HIP graph: every
    signal's coefficients equal the oracle's on the zero-padded signal, the
    gradient equals the oracle's VJP on the true samples, and replays of the
    graph (with eager work between them) are bitwise identical; also with each
    bucket's plan autotuned at creation."""
    from paper_2204_08269_amd.jtfs import JTFSBucket
    prm = dict(J=6, Q=(8, 1), J_fr=3, Q_fr=1, T=64, F=4)
    lengths = [3000, 2048, 5000, 1500, 8000, 2500]
    rng = np.random.default_rng(77)
    sigs = [(rng.standard_normal(L) * 0.5).astype(np.float32) for L in lengths]
    bk = JTFSBucket(lengths, **prm, autotune=autotune)
    x = torch.from_numpy(np.concatenate(sigs)).cuda()
    g = torch.from_numpy(rng.standard_normal(bk.s_offset[-1]).astype(np.float32)).cuda()
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        s_a, gx_a = bk.run(x, g)
    st.synchronize()
    s_a, gx_a = s_a.cpu().numpy(), gx_a.cpu().numpy()
    # the graph is keyed by pointers: the same output buffers give true replays
    out = torch.empty(bk.s_offset[-1], device="cuda")
    gxo = torch.zeros(bk.x_offset[-1], device="cuda")
    results = []
    for rep in range(3):
        torch.randn(1 << 20, device="cuda").sum()                # eager work between replays
        torch.cuda.synchronize()
        with torch.cuda.stream(st):
            bk.run(x, g, out=out, gx_out=gxo)
        st.synchronize()
        results.append((out.cpu().numpy().copy(), gxo.cpu().numpy().copy()))
    for r in results:
        assert np.array_equal(r[0], s_a) and np.array_equal(r[1], gx_a)
    for i, L in enumerate(lengths):
        N = bk.pads[i]
        p = dict(N=N, **prm)
        P = oracle_plan(p)
        xp = np.zeros(N)
        xp[:L] = sigs[i]
        s1n = int(np.prod(P.s1_shape()))
        seg = s_a[bk.s_offset[i]: bk.s_offset[i + 1]]
        r1, r2 = O.jtfs(xp, P)
        check_paths(seg[:s1n].reshape(P.s1_shape()), seg[s1n:].reshape(P.s2_shape()), r1, r2)
        gseg = g.cpu().numpy()[bk.s_offset[i]: bk.s_offset[i + 1]].astype(np.float64)
        ref = O.jtfs_vjp(xp, gseg[:s1n].reshape(P.s1_shape()), gseg[s1n:].reshape(P.s2_shape()), P)[:L]
        assert rel_l2(gx_a[bk.x_offset[i]: bk.x_offset[i + 1]], ref) <= TOL_VJP


# Scalogram rows and second-order rows of 2^15 points: each runs as two 2^14-point
# register transforms (decimation in frequency for the inverse, in time for the
# forward).  kX = 0 here, so N_X = N and the two fastest temporal rates keep 2^15.
LONG = dict(N=2 ** 15, J=5, Q=(1, 1), J_fr=2, Q_fr=1, T=2 ** 10, F=2)


@pytest.mark.parametrize("radix", [16, 8])
@pytest.mark.parametrize("mode", MODES)
def test_long_rows_forward_and_vjp(mode, radix):
    """(radix: the largest radix of the register-resident transforms' passes, a
    launch choice of the autotuner, applied to every stage.)"""
    P = oracle_plan(LONG)
    assert P.NX == 2 ** 15 and P.T_alpha(0) == 2 ** 15
    rng = np.random.default_rng(215)
    x = (rng.standard_normal((2, LONG["N"])) * 0.5).astype(np.float32)
    op = gpu_op(LONG, mode)
    if radix == 8:
        c, rows, ft, bt = op.tuning()
        op.set_tuning(c, rows, fwd_tile=ft, bwd_tile=bt, radix8=list(op.RADIX8_BITS))
        assert op.tuning_radix()[0] == list(op.RADIX8_BITS)
    g1, g2 = run_forward(op, x)
    gs1, gs2 = synth.cotangents((2,) + P.s1_shape(), (2,) + P.s2_shape(), seed=5)
    g = op.vjp(torch.from_numpy(x).cuda(), torch.from_numpy(gs1).cuda(), torch.from_numpy(gs2).cuda()).cpu().numpy()
    for b in range(2):
        xb = x[b].astype(np.float64)
        r1, r2 = O.jtfs(xb, P)
        check_paths(g1[b], g2[b], r1, r2)
        ref = O.jtfs_vjp(xb, gs1[b].astype(np.float64), gs2[b].astype(np.float64), P)
        err = rel_l2(g[b], ref)
        assert err <= TOL_VJP, f"signal {b}: gradient relative L2 {err:.3e}"


def test_cfg3_full_batch_sampled_forward_and_gradient():
    """8 x 2^17 click trains (N_X = 2^15): every S1 path and two temporal rates of
    S2 of the first and last target against the oracle, and the gradient at the
    first white-noise start (where texture synthesis differentiates) for a
    cotangent on S1 and on those two rates.  At the click trains themselves the
    gradient is ill-conditioned in any FP32 arithmetic: between clicks the
    high-frequency first-order outputs sit at the rounding floor, and the phase
    factor y/|y| of the modulus adjoint there is rounding noise (an input change
    of 1e-7 of its RMS moves the FP64 gradient by several percent at the target,
    by about 1e-7 at the start: test_click_train_gradient_is_ill_conditioned)."""
    p = synth.PARAMS[3]
    y, x0 = synth.cfg3_batch()
    P = oracle_plan(p)
    assert P.NX == 2 ** 15
    alphas = [P.n_alpha - 1, P.n_alpha - 4]
    op = gpu_op(p)
    g1, g2 = run_forward(op, y)
    for b in (0, y.shape[0] - 1):
        r1, r2 = O.jtfs(y[b].astype(np.float64), P, alphas=alphas)
        check_paths(g1[b], g2[b], r1, r2, alphas=alphas)
    gs1, gs2 = synth.cotangents((1,) + P.s1_shape(), (1,) + P.s2_shape(), seed=9)
    keep = np.zeros(P.n_alpha, bool)
    keep[alphas] = True
    gs2[:, ~keep] = 0.0
    g = op.vjp(torch.from_numpy(x0[:1]).cuda(), torch.from_numpy(gs1).cuda(), torch.from_numpy(gs2).cuda())
    ref = O.jtfs_vjp(x0[0].astype(np.float64), gs1[0].astype(np.float64), gs2[0].astype(np.float64), P)
    err = rel_l2(g.cpu().numpy()[0], ref)
    assert err <= TOL_VJP, f"gradient relative L2 {err:.3e}"


@pytest.mark.parametrize("mode", MODES)
def test_cfg5_full_batch_sampled_and_properties(mode):
    """32 x 2^18 FM mixtures (N_X = 2^15, 285 first-order and 24 second-order
    filters).  S1 rows that the oracle computes one at a time; exact equivariance
    to a shift by T and batch invariance, which hold at any size; the pure-tone
    closed form (S1 = (A/2)|psi_hat(m/N)|, S2 = 0)."""
    p = synth.PARAMS[5]
    T = p["T"]
    x = synth.batch(5)
    P = oracle_plan(p)
    assert P.NX == 2 ** 15
    op = gpu_op(p, mode)
    g1, g2 = run_forward(op, x)
    # S1 rows from the oracle's stage definitions, one row at a time
    for b in (0, x.shape[0] - 1):
        xb = x[b].astype(np.float64)[None, :]
        for lam in list(range(0, P.n1, 16)) + [P.n1 - 1]:
            Xr = np.abs(O.filt_decimate(xb, P.psi1_hat[lam], 1 << P.kX))
            ref = O.time_lowpass(Xr, P, P.kX)[0]
            err = rel_l2(g1[b, lam], ref)
            assert err <= TOL, f"signal {b} row {lam}: {err:.3e}"
    # shift by T moves every output frame by one
    xs = np.roll(x[:2], T, axis=1)
    h1, h2 = run_forward(op, xs)
    check_paths(h1[0], h2[0], np.roll(g1[0], 1, axis=-1), np.roll(g2[0], 1, axis=-1))
    check_paths(h1[1], h2[1], np.roll(g1[1], 1, axis=-1), np.roll(g2[1], 1, axis=-1))
    # a signal alone gives the same bits as in the batch
    c1, c2 = run_forward(op, x[5:6])
    assert np.array_equal(c1[0], g1[5]) and np.array_equal(c2[0], g2[5])
    # pure tone on an exact bin
    m, A = 9001, 0.6
    t1, t2 = run_forward(op, synth.tone(p["N"], m, A, 1.1).astype(np.float32)[None])
    expect = 0.5 * A * np.abs(P.psi1_hat[:, m])
    assert np.max(np.abs(t1[0] - expect[:, None])) <= 1e-5 * expect.max()
    assert np.max(np.abs(t2)) <= 1e-5 * expect.max()


CFG5_REF = None


def cfg5_reference():
    """FP64 oracle outputs of the 32 x 2^18 workload (signals 0 and 31; S2 at
    three temporal rates; the VJP of signal 0), written by
    tests/golden/make_cfg5_reference.py, which calls only the oracle."""
    global CFG5_REF
    if CFG5_REF is None:
        import hashlib
        import os
        path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "cfg5_reference.npz")
        ref = dict(np.load(path, allow_pickle=False))
        x = synth.batch(5)
        assert str(ref["x_sha256"]) == hashlib.sha256(np.ascontiguousarray(x).tobytes()).hexdigest(), \
            "the seeded 2^18 inputs differ from those the stored reference was computed on"
        ref["x"] = x
        CFG5_REF = ref
    return CFG5_REF


@pytest.mark.parametrize("mode,tile,btile", [("fp32", 32, 32), ("split16", 32, 32), ("split16_phase", 32, 32),
                                             ("split16", 16, 32), ("split16_phase", 16, 16),
                                             ("split16_phase", 32, 16)])
def test_cfg5_s2_and_gradient_match_oracle(mode, tile, btile):
    """32 x 2^18 FM mixtures (n1 = 285: K = 288, 18 k-steps of the split forward,
    9 i-blocks of the backward), in the launch configuration of the benchmark
    (the whole batch): every S1 path and every (beta, theta) path of S2 at the
    temporal rates k2 = 0 (rows of 2^15 points), a middle one and the shortest,
    for the first and last signal, against the FP64 oracle; the gradient of
    signal 0 for a cotangent on S1 and those rates against the oracle's VJP,
    after a forward on the same workspace (the stored-phase mode reads the
    phase it kept) and without one (that mode then takes the phase again);
    both tiles of the split forward and of the stored-phase backward (whose
    16 x 16 kernel holds the nine 32-row i-blocks in one pass)."""
    p = synth.PARAMS[5]
    ref = cfg5_reference()
    x = ref["x"]
    alphas = [int(a) for a in ref["alphas"]]
    op = gpu_op(p, mode)
    assert op.contraction == mode
    op.set_tuning(mode, ALL_ROWS, fwd_tile=tile, bwd_tile=btile)
    B = x.shape[0]
    xt = torch.from_numpy(x).cuda()
    ws = op.new_workspace(B)
    s1, s2 = op.forward(xt, ws)
    torch.cuda.synchronize()
    g1, g2 = s1.cpu().numpy(), s2.cpu().numpy()
    for b in (int(v) for v in ref["signals"]):
        e1, _ = path_errors(g1[b], ref[f"s1_{b}"], 1)
        e2, _ = path_errors(g2[b][alphas], ref[f"s2_{b}"], 3)
        assert e1.max() <= TOL, f"signal {b}: S1 worst path error {e1.max():.3e}"
        assert e2.max() <= TOL, f"signal {b}: S2 worst path error {e2.max():.3e} at {np.unravel_index(e2.argmax(), e2.shape)}"
    Po = oracle_plan(p)
    gs1 = np.zeros((B,) + Po.s1_shape(), np.float32)
    gs2 = np.zeros((B,) + Po.s2_shape(), np.float32)
    c1, c2 = synth.cotangents((1,) + Po.s1_shape(), (1,) + Po.s2_shape(), seed=9)
    keep = np.zeros(Po.n_alpha, bool)
    keep[alphas] = True
    c2[:, ~keep] = 0.0
    gs1[0], gs2[0] = c1[0], c2[0]
    gs1t, gs2t = torch.from_numpy(gs1).cuda(), torch.from_numpy(gs2).cuda()
    for reuse in (True, False):
        gx = op.vjp(xt, gs1t, gs2t, ws=ws, reuse_forward=reuse)
        torch.cuda.synchronize()
        err = rel_l2(gx[0].cpu().numpy(), ref["gx_0"])
        assert err <= TOL_VJP, f"reuse_forward={reuse}: gradient relative L2 {err:.3e}"
        assert float(gx[1:].abs().max()) == 0.0, "a signal with zero cotangent got a gradient"
    del ws
    torch.cuda.empty_cache()


# Eq. (4): no frequential averaging.  The packed (beta, theta) slices are spread
# to [n_alpha, n_beta, 2, L, N/T] (rows beyond L_beta zero) so that each
# (alpha, beta, theta) path is compared on its own.
def unpack_eq4(S2, P):
    out = np.zeros(S2.shape[:-2] + (P.n_beta, 2, P.L, P.out_t), S2.dtype)
    for b in range(P.n_beta):
        for s in range(2):
            out[..., b, s, :P.L_beta(b), :] = S2[..., P.s2_rows(b, s), :]
    return out


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("p", [P1, RAGGED[2], RAGGED[3]])
def test_unaveraged_forward_and_vjp(p, mode):
    P = oracle_plan(p)
    rng = np.random.default_rng(404 + p["N"])
    x = (rng.standard_normal((2, p["N"])) * 0.5).astype(np.float32)
    op = gpu_op(p, mode, average_fr=False)
    assert op.s2_shape == P.s2_shape(False)
    assert all(op.s2_rows(b, t) == P.s2_rows(b, t) for b in range(P.n_beta) for t in range(2))
    g1, g2 = run_forward(op, x)
    gs1, gs2 = synth.cotangents((2,) + P.s1_shape(), (2,) + P.s2_shape(False), seed=13)
    g = op.vjp(torch.from_numpy(x).cuda(), torch.from_numpy(gs1).cuda(), torch.from_numpy(gs2).cuda()).cpu().numpy()
    for b in range(2):
        xb = x[b].astype(np.float64)
        r1, r2 = O.jtfs(xb, P, average_fr=False)
        check_paths(g1[b], unpack_eq4(g2[b], P), r1, unpack_eq4(r2, P))
        ref = O.jtfs_vjp(xb, gs1[b].astype(np.float64), gs2[b].astype(np.float64), P, average_fr=False)
        err = rel_l2(g[b], ref)
        assert err <= TOL_VJP, f"signal {b}: gradient relative L2 {err:.3e}"


@pytest.mark.parametrize("average_fr", [True, False])
def test_mulog_matches_oracle(average_fr):
    """mu-log (sec. 4) end to end from x: path means over a batch of 3, the
    renormalised coefficients per path, and the adjoint with mu fixed."""
    P = oracle_plan(P1)
    x = synth.batch(1, B=3)
    op = gpu_op(P1, average_fr=average_fr)
    s1, s2 = op.forward(torch.from_numpy(x).cuda())
    mu1, mu2 = op.path_means(s1, s2)
    o1, o2 = op.mulog(s1, s2, mu1, mu2)
    gs1, gs2 = synth.cotangents(tuple(s1.shape), tuple(s2.shape), seed=17)
    d1, d2 = op.mulog_vjp(s1, s2, mu1, mu2, torch.from_numpy(gs1).cuda(), torch.from_numpy(gs2).cuda())
    refs = [O.jtfs(x[b].astype(np.float64), P, average_fr=average_fr) for b in range(3)]
    R1 = np.stack([r[0] for r in refs])
    R2 = np.stack([r[1] for r in refs])
    if average_fr:
        m1, m2 = O.path_means(R1, R2)
        R2u, G2 = R2, gs2
        g_o2, g_d2 = o2.cpu().numpy(), d2.cpu().numpy()
    else:
        m1 = np.float64(R1.mean())
        m2 = np.array([[[R2[:, a, P.s2_rows(b, t)].mean() for t in range(2)] for b in range(P.n_beta)]
                       for a in range(P.n_alpha)])
        R2u, G2 = unpack_eq4(R2, P), unpack_eq4(gs2.astype(np.float64), P)
        g_o2, g_d2 = unpack_eq4(o2.cpu().numpy(), P), unpack_eq4(d2.cpu().numpy(), P)
    assert abs(float(mu1.cpu()) - m1) <= 1e-5 * m1
    assert np.max(np.abs(mu2.cpu().numpy().reshape(m2.shape) - m2) / m2) <= 1e-5
    e1, e2 = O.mulog(R1, R2u, m1, m2)
    f1, f2 = O.mulog_vjp(R1, R2u, m1, m2, gs1, G2)
    for b in range(3):
        check_paths(o1.cpu().numpy()[b], g_o2[b], e1[b], e2[b])
        check_paths(d1.cpu().numpy()[b], g_d2[b], f1[b], f2[b])


def test_mulog_time_scattering_matches_oracle():
    """mu-log of a time-scattering transform: one path per (alpha, lambda1) row
    of S2 [n_alpha][n1][N/T], means over a batch of 3, the renormalised
    coefficients and the adjoint."""
    P = oracle_plan(P1)
    x = synth.batch(1, B=3)
    op = gpu_op(P1, time_scattering=True)
    s1, s2 = op.forward(torch.from_numpy(x).cuda())
    mu1, mu2 = op.path_means(s1, s2)
    assert tuple(mu2.shape) == (P.n_alpha * P.n1,)
    o1, o2 = op.mulog(s1, s2, mu1, mu2)
    gs1, gs2 = synth.cotangents(tuple(s1.shape), tuple(s2.shape), seed=19)
    d1, d2 = op.mulog_vjp(s1, s2, mu1, mu2, torch.from_numpy(gs1).cuda(), torch.from_numpy(gs2).cuda())
    refs = [O.scattering1d(x[b].astype(np.float64), P) for b in range(3)]
    R1 = np.stack([r[0] for r in refs])
    R2 = np.stack([r[1] for r in refs])
    m1, m2 = O.path_means(R1, R2, path_axes=1)
    assert abs(float(mu1.cpu()) - m1) <= 1e-5 * m1
    assert np.max(np.abs(mu2.cpu().numpy().reshape(m2.shape) - m2) / m2) <= 1e-5
    e1, e2 = O.mulog(R1, R2, m1, m2, path_axes=1)
    f1, f2 = O.mulog_vjp(R1, R2, m1, m2, gs1, gs2, path_axes=1)
    for b in range(3):
        for got, ref in ((o1.cpu().numpy()[b], e1[b]), (d1.cpu().numpy()[b], f1[b])):
            assert path_errors(got, ref, 1)[0].max() <= TOL
        for got, ref in ((o2.cpu().numpy()[b], e2[b]), (d2.cpu().numpy()[b], f2[b])):
            assert path_errors(got, ref, 2)[0].max() <= TOL


@pytest.mark.parametrize("variant,mode", [("eq3", None), ("eq3", "split16_phase"), ("eq4", None),
                                          ("time_scattering", None), ("eq3_lowpass_pairs", "split16_phase")])
def test_fused_mulog_matches_oracle(variant, mode):
    """mu-log fused into the transform's output kernels (sec. 4, eqs. (9)-(10)),
    mu given (here the oracle's path means of the batch): the outputs per path
    against the oracle's log(1 + S / (eps mu)), bit-identical to the unfused
    mulog(forward), and the gradient with mu fixed against the oracle's VJP of
    the mu-log adjoint, through the C ABI (eq. (3), eq. (4), time scattering) and
    through autograd with the stored phase."""
    lp = variant == "eq3_lowpass_pairs"
    p1 = dict(P1, lowpass_pairs=True) if lp else P1
    P = oracle_plan(p1)
    x = synth.batch(1, B=3)
    tsc = variant == "time_scattering"
    avg = variant.startswith("eq3")
    op = gpu_op(p1, contraction=mode, average_fr=avg or tsc, time_scattering=tsc)
    xt = torch.from_numpy(x).cuda()
    if tsc:
        refs = [O.scattering1d(x[b].astype(np.float64), P) for b in range(3)]
    else:
        refs = [O.jtfs(x[b].astype(np.float64), P, average_fr=avg) for b in range(3)]
    R1 = np.stack([r[0] for r in refs])
    R2 = np.stack([r[1] for r in refs])
    if avg:
        m1, m2 = O.path_means(R1, R2)
        m2_rows, axes = m2, 2                   # one mu per (alpha, beta, theta) slice
    elif tsc:
        m1, m2 = O.path_means(R1, R2, path_axes=1)
        m2_rows, axes = m2, 1
    else:
        m1 = np.float64(R1.mean())
        m2 = np.array([[[R2[:, a, P.s2_rows(b, t)].mean() for t in range(2)] for b in range(P.n_beta)]
                       for a in range(P.n_alpha)])
        m2_rows = np.zeros((P.n_alpha, R2.shape[2]))      # mu of each packed row's slice
        for a in range(P.n_alpha):
            for b in range(P.n_beta):
                for t in range(2):
                    m2_rows[a, P.s2_rows(b, t)] = m2[a, b, t]
        axes = 1
    mu1 = torch.tensor([m1], dtype=torch.float32, device="cuda")
    mu2 = torch.from_numpy(np.ascontiguousarray(m2, np.float32).reshape(-1)).cuda()
    e1, e2 = O.mulog(R1, R2, m1, m2_rows, path_axes=axes)
    go1, go2 = synth.cotangents((3,) + op.s1_shape, (3,) + op.s2_shape, seed=23)
    f1, f2 = O.mulog_vjp(R1, R2, m1, m2_rows, go1, go2, path_axes=axes)
    if mode == "split16_phase":
        xg = xt.clone().requires_grad_(True)
        o1, o2 = op(xg, mu=(mu1, mu2))
        (o1 * torch.from_numpy(go1).cuda()).sum().add((o2 * torch.from_numpy(go2).cuda()).sum()).backward()
        gx = xg.grad
    else:
        o1, o2 = op.forward_mulog(xt, mu1, mu2)
        gx = op.vjp_mulog(xt, o1, o2, mu1, mu2, torch.from_numpy(go1).cuda(), torch.from_numpy(go2).cuda())
    s1, s2 = op.forward(xt)
    u1, u2 = op.mulog(s1, s2, mu1, mu2)
    assert torch.equal(o1, u1) and torch.equal(o2, u2), "fused and unfused mu-log differ"
    o1, o2, gx = o1.detach().cpu().numpy(), o2.detach().cpu().numpy(), gx.cpu().numpy()
    for b in range(3):
        if avg:
            check_paths(o1[b], o2[b], e1[b], e2[b])
        else:
            assert path_errors(o1[b], e1[b], 1)[0].max() <= TOL
            assert path_errors(o2[b], e2[b], 2)[0].max() <= TOL
        xb = x[b].astype(np.float64)
        if tsc:
            ref = O.scattering1d_vjp(xb, f1[b], f2[b], P)
        else:
            ref = O.jtfs_vjp(xb, f1[b], f2[b], P, average_fr=avg)
        err = rel_l2(gx[b], ref)
        assert err <= TOL_VJP, f"signal {b}: gradient relative L2 {err:.3e}"


# Lowpass pairs: phi_T as one more temporal rate (its second-order rows are the S1
# rows) and phi_F as one more frequential scale, through every contraction mode.
LP_SHAPES = [P1, RAGGED[2], dict(N=4096, J=7, Q=(8, 1), J_fr=3, Q_fr=1, T=64, F=2),
             RAGGED[0], RAGGED[1]]      # T = N (one frame: phi_T's rate holds one column); F = 1


@pytest.mark.parametrize("mode", ["fp32", "split16", "split16_phase"])
@pytest.mark.parametrize("average_fr", [True, False])
@pytest.mark.parametrize("p", LP_SHAPES, ids=lambda p: f"N{p['N']}_T{p['T']}_Q{p['Q'][0]}")
def test_lowpass_pairs_forward_and_vjp(p, average_fr, mode):
    q = dict(p, lowpass_pairs=True)
    P = oracle_plan(q)
    rng = np.random.default_rng(606 + p["N"])
    x = (rng.standard_normal((2, p["N"])) * 0.5).astype(np.float32)
    op = gpu_op(q, contraction=mode, average_fr=average_fr)
    assert (op.info.n_alpha, op.info.n_beta) == (P.n_alpha, P.n_beta)
    xt = torch.from_numpy(x).cuda()
    ws = op.new_workspace(2)
    s1, s2 = op.forward(xt, ws)
    g1, g2 = s1.cpu().numpy(), s2.cpu().numpy()
    gs1, gs2 = synth.cotangents((2,) + P.s1_shape(), (2,) + P.s2_shape(average_fr), seed=37)
    g = op.vjp(xt, torch.from_numpy(gs1).cuda(), torch.from_numpy(gs2).cuda(), ws=ws,
               reuse_forward=(mode == "split16_phase")).cpu().numpy()
    for b in range(2):
        xb = x[b].astype(np.float64)
        r1, r2 = O.jtfs(xb, P, average_fr=average_fr)
        if average_fr:
            check_paths(g1[b], g2[b], r1, r2)
        else:
            check_paths(g1[b], unpack_eq4(g2[b], P), r1, unpack_eq4(r2, P))
        ref = O.jtfs_vjp(xb, gs1[b].astype(np.float64), gs2[b].astype(np.float64), P, average_fr=average_fr)
        err = rel_l2(g[b], ref)
        assert err <= TOL_VJP, f"signal {b}: gradient relative L2 {err:.3e}"


@pytest.mark.parametrize("mode", ["split16", "split16_phase"])
@pytest.mark.parametrize("p", [P1, RAGGED[2]], ids=lambda p: f"N{p['N']}_Q{p['Q'][0]}")
def test_unpadded_lambda_forward_and_vjp(p, mode):
    """S2 with the ceil(n1 / F) rows on first-order bands, with and without the
    lowpass pairs, and the gradient of a cotangent on those rows."""
    for lp in (False, True):
        q = dict(p, unpad=True, lowpass_pairs=lp)
        P = oracle_plan(q)
        x = (np.random.default_rng(77).standard_normal((2, p["N"])) * 0.5).astype(np.float32)
        op = gpu_op(q, contraction=mode)
        assert op.s2_shape[-2] == -(-P.n1 // p["F"]) < P.L // p["F"]
        xt = torch.from_numpy(x).cuda()
        ws = op.new_workspace(2)
        s1, s2 = op.forward(xt, ws)
        gs1, gs2 = synth.cotangents((2,) + P.s1_shape(), (2,) + P.s2_shape(), seed=41)
        g = op.vjp(xt, torch.from_numpy(gs1).cuda(), torch.from_numpy(gs2).cuda(), ws=ws,
                   reuse_forward=True).cpu().numpy()
        for b in range(2):
            xb = x[b].astype(np.float64)
            r1, r2 = O.jtfs(xb, P)
            check_paths(s1.cpu().numpy()[b], s2.cpu().numpy()[b], r1, r2)
            ref = O.jtfs_vjp(xb, gs1[b].astype(np.float64), gs2[b].astype(np.float64), P)
            assert rel_l2(g[b], ref) <= TOL_VJP


@pytest.mark.parametrize("p", [P1, RAGGED[0], synth.PARAMS[5]], ids=lambda p: f"N{p['N']}_T{p['T']}")
def test_zeroth_order_matches_oracle(p):
    """S0 = (x * phi_T)(tau T) and its adjoint (added to a given gx) against the
    oracle, up to T = N (one frame) and the 2^18-sample workload."""
    P = oracle_plan(p)
    rng = np.random.default_rng(55)
    x = rng.standard_normal((2, p["N"])).astype(np.float32)
    op = gpu_op(p)
    s0 = op.zeroth_order(torch.from_numpy(x).cuda()).cpu().numpy()
    g = rng.standard_normal((2, P.out_t)).astype(np.float32)
    gt = torch.from_numpy(g).cuda()
    gx = op.zeroth_order_vjp(gt).cpu().numpy()
    # the adjoint adds to what gx holds (one FP32 addition per sample)
    base = rng.standard_normal((2, p["N"])).astype(np.float32)
    acc = op.zeroth_order_vjp(gt, torch.from_numpy(base).cuda()).cpu().numpy()
    assert np.max(np.abs(acc - (base + gx))) <= 1e-6 * np.max(np.abs(base))
    for b in range(2):
        ref = O.zeroth_order(x[b].astype(np.float64), P)
        assert rel_l2(s0[b], ref) <= TOL, rel_l2(s0[b], ref)
        refg = O.zeroth_order_adj(g[b].astype(np.float64), P)
        assert rel_l2(gx[b], refg) <= TOL_VJP


@pytest.mark.parametrize("mode", ["split16", "split16_phase"])
def test_texture_loop_matches_oracle(mode):
    """Texture resynthesis (sec. 5), every step on the GPU, against the oracle's
    loop from the same start: the start's error, the best error after each of 8
    bold-driver iterations, the final iterate and rate, for 2 signals; and 3 + 5
    iterations in two calls (two graph captures) equal 8 in one.  With the stored
    phase each iteration's backward takes the modulus adjoint from its forward."""
    from paper_2204_08269_amd.jtfs import Texture
    P = oracle_plan(P1)
    x = synth.batch(1, B=2)
    rng = np.random.default_rng(55)
    y0 = (rng.standard_normal((2, P1["N"])) * x.std(axis=1, keepdims=True)).astype(np.float32)
    op = gpu_op(P1, mode)
    xt, yt = torch.from_numpy(x).cuda(), torch.from_numpy(y0).cuda()
    tex = Texture(op, 2, mu0=-0.05)
    tex.set_target(xt)
    tex.set_start(yt)
    _, e0, _ = tex.read()
    hist = tex.iterate(8).cpu().numpy()
    y, e, mu = (v.cpu().numpy() for v in tex.read())
    e0 = e0.cpu().numpy()
    for b in range(2):
        yo, ho, muo = O.texture_resynthesis(x[b].astype(np.float64), y0[b].astype(np.float64), P, 8, -0.05)
        assert abs(e0[b] - ho[0]) <= 1e-5 * ho[0]
        assert np.max(np.abs(hist[:, b] - ho[1:]) / ho[1:]) <= 1e-4, (hist[:, b], ho[1:])
        assert ho[-1] < ho[0]
        assert rel_l2(y[b], yo) <= 1e-4
        assert abs(mu[b] - muo) <= 1e-4 * muo
    tex2 = Texture(op, 2, mu0=-0.05)
    tex2.set_target(xt)
    tex2.set_start(yt)
    h1 = tex2.iterate(3).cpu().numpy()
    h2 = tex2.iterate(5).cpu().numpy()
    y2, _, _ = tex2.read()
    assert np.allclose(np.concatenate([h1, h2]), hist, rtol=1e-6, atol=0)
    assert rel_l2(y2.cpu().numpy(), y) <= 1e-6


def test_cfg4_ragged_full_batch_sampled():
    """The 256-signal ragged workload through the bucket graph: the shortest
    signal of every pad length against the oracle on the zero-padded signal (two temporal rates of S2, every S1 path), and the
    gradient of the shortest on its true samples."""
    from paper_2204_08269_amd.jtfs import JTFSBucket
    p = synth.PARAMS[4]
    sigs = synth.cfg4_ragged(synth.BATCH[4])
    lengths = [len(v) for v in sigs]
    bk = JTFSBucket(lengths, p["J"], p["Q"], p["J_fr"], p["Q_fr"], p["T"], p["F"])
    x = torch.from_numpy(np.concatenate(sigs)).cuda()
    g = torch.from_numpy(np.random.default_rng(12).standard_normal(bk.s_offset[-1]).astype(np.float32)).cuda()
    st = torch.cuda.Stream()
    st.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(st):
        s, gx = bk.run(x, g)
    st.synchronize()
    s, gx = s.cpu().numpy(), gx.cpu().numpy()
    picks = {}
    for j, n in enumerate(bk.pads):
        if n not in picks or lengths[j] < lengths[picks[n]]:
            picks[n] = j
    assert sorted(picks) == [2 ** 14, 2 ** 15, 2 ** 16]          # the shortest length is above 2^13
    for n, j in sorted(picks.items()):
        prm = dict(p, N=n)
        P = oracle_plan(prm)
        xp = np.zeros(n)
        xp[:lengths[j]] = sigs[j]
        alphas = [P.n_alpha - 1, P.n_alpha // 2]
        r1, r2 = O.jtfs(xp, P, alphas=alphas)
        n1 = int(np.prod(P.s1_shape()))
        got = s[bk.s_offset[j]:bk.s_offset[j + 1]]
        check_paths(got[:n1].reshape(P.s1_shape()), got[n1:].reshape(P.s2_shape()), r1, r2, alphas=alphas)
    j = picks[2 ** 14]
    P = oracle_plan(dict(p, N=2 ** 14))
    n1 = int(np.prod(P.s1_shape()))
    gs = g.cpu().numpy()[bk.s_offset[j]:bk.s_offset[j + 1]].astype(np.float64)
    xp = np.zeros(2 ** 14)
    xp[:lengths[j]] = sigs[j]
    ref = O.jtfs_vjp(xp, gs[:n1].reshape(P.s1_shape()), gs[n1:].reshape(P.s2_shape()), P)[:lengths[j]]
    err = rel_l2(gx[bk.x_offset[j]:bk.x_offset[j + 1]], ref)
    assert err <= TOL_VJP, f"gradient relative L2 {err:.3e}"


@pytest.mark.parametrize("p", [P1, RAGGED[3], LONG])
def test_time_scattering_forward_and_vjp(p):
    """Time scattering (sec. 4): S1 and |X * psi_alpha| * phi_T per (alpha, lambda)
    path against the oracle, and the gradient."""
    P = oracle_plan(p)
    rng = np.random.default_rng(808 + p["N"])
    x = (rng.standard_normal((2, p["N"])) * 0.5).astype(np.float32)
    op = gpu_op(p, time_scattering=True)
    assert op.s2_shape == (P.n_alpha, P.n1, P.out_t)
    g1, g2 = run_forward(op, x)
    gs1, gs2 = synth.cotangents((2,) + P.s1_shape(), (2, P.n_alpha, P.n1, P.out_t), seed=29)
    g = op.vjp(torch.from_numpy(x).cuda(), torch.from_numpy(gs1).cuda(), torch.from_numpy(gs2).cuda()).cpu().numpy()
    for b in range(2):
        xb = x[b].astype(np.float64)
        r1, r2 = O.scattering1d(xb, P)
        e1, _ = path_errors(g1[b], r1, 1)
        e2, _ = path_errors(g2[b], r2, 2)
        assert e1.max() <= TOL and e2.max() <= TOL, (e1.max(), e2.max())
        ref = O.scattering1d_vjp(xb, gs1[b].astype(np.float64), gs2[b].astype(np.float64), P)
        err = rel_l2(g[b], ref)
        assert err <= TOL_VJP, f"signal {b}: gradient relative L2 {err:.3e}"


# Stored phase: the forward also writes the unit phase of every contraction
# output, and a vjp that reuses its workspace takes the modulus adjoint from it
# instead of recomputing the contraction.  Shapes with 32- and 64-frame tiles,
# ragged row counts, 1 to 6 blocks of 32 lambda rows, and both eq. (3) and eq. (4).
PHASE_SHAPES = [P1, RAGGED[0], RAGGED[1], RAGGED[2], RAGGED[3],
                dict(N=4096, J=7, Q=(8, 1), J_fr=3, Q_fr=1, T=64, F=2),      # N/T = 64
                dict(N=4096, J=8, Q=(28, 1), J_fr=3, Q_fr=1, T=64, F=2),     # N/T = 64, n1 = 158: 5 i-blocks
                dict(N=4096, J=8, Q=(32, 1), J_fr=3, Q_fr=1, T=256, F=2)]    # n1 = 175: 6 i-blocks


@pytest.mark.parametrize("bwd_tile", [32, 16])
@pytest.mark.parametrize("average_fr", [True, False])
@pytest.mark.parametrize("p", PHASE_SHAPES, ids=lambda p: f"N{p['N']}_T{p['T']}_Q{p['Q'][0]}")
def test_stored_phase_vjp_matches_oracle(p, average_fr, bwd_tile):
    """(32 x 32 or 16 x 16 tiles of the stored-phase backward; the latter only
    where N/T <= 32, the former elsewhere.)"""
    P = oracle_plan(p)
    B = 3
    rng = np.random.default_rng(606 + p["N"] + p["T"])
    x = (rng.standard_normal((B, p["N"])) * 0.5).astype(np.float32)
    xt = torch.from_numpy(x).cuda()
    gs1, gs2 = synth.cotangents((B,) + P.s1_shape(), (B,) + P.s2_shape(average_fr), seed=17)
    gt1, gt2 = torch.from_numpy(gs1).cuda(), torch.from_numpy(gs2).cuda()
    res = {}
    for mode in ("split16", "split16_phase"):
        op = gpu_op(p, mode, average_fr=average_fr)
        assert op.contraction == mode
        if mode == "split16_phase":
            op.set_tuning(mode, ALL_ROWS, bwd_tile=bwd_tile)
        ws = op.new_workspace(B)
        s1, s2 = op.forward(xt, ws)
        g = op.vjp(xt, gt1, gt2, ws=ws, reuse_forward=True)
        g_alone = op.vjp(xt, gt1, gt2)          # no forward to reuse: recomputes the contraction
        torch.cuda.synchronize()
        res[mode] = [t.cpu().numpy() for t in (s1, s2, g, g_alone)]
    a, b_ = res["split16"], res["split16_phase"]
    # the phase store leaves the coefficients' bits alone, and without a forward
    # to reuse the two modes run the same recompute
    assert np.array_equal(a[0], b_[0]) and np.array_equal(a[1], b_[1])
    assert np.array_equal(a[3], b_[3])
    for b in range(B):
        xb = x[b].astype(np.float64)
        ref = O.jtfs_vjp(xb, gs1[b].astype(np.float64), gs2[b].astype(np.float64), P, average_fr=average_fr)
        err = rel_l2(b_[2][b], ref)
        assert err <= TOL_VJP, f"signal {b}: stored-phase gradient relative L2 {err:.3e}"
        assert rel_l2(a[2][b], ref) <= TOL_VJP


def test_stored_phase_zero_input_and_autograd():
    """Zero input: the stored phase is zero (|z| below eps), the gradient finite
    and zero.  Autograd through the object uses the stored phase and equals the
    explicit forward + vjp on one workspace."""
    op = gpu_op(P1, "split16_phase")
    x = torch.zeros((2, P1["N"]), device="cuda")
    ws = op.new_workspace(2)
    s1, s2 = op.forward(x, ws)
    g = op.vjp(x, torch.ones_like(s1), torch.ones_like(s2), ws=ws, reuse_forward=True)
    torch.cuda.synchronize()
    assert float(s1.abs().max()) == 0.0 and float(s2.abs().max()) == 0.0
    assert torch.isfinite(g).all() and float(g.abs().max()) == 0.0
    P = oracle_plan(P1)
    xs = torch.from_numpy(synth.batch(1, B=2)).cuda()
    gs1, gs2 = synth.cotangents((2,) + P.s1_shape(), (2,) + P.s2_shape(), seed=19)
    gs1, gs2 = torch.from_numpy(gs1).cuda(), torch.from_numpy(gs2).cuda()
    xr = xs.clone().requires_grad_(True)
    s1, s2 = op(xr)
    ((s1 * gs1).sum() + (s2 * gs2).sum()).backward()
    ws = op.new_workspace(2)
    op.forward(xs, ws)
    g_ref = op.vjp(xs, gs1, gs2, ws=ws, reuse_forward=True)
    torch.cuda.synchronize()
    assert torch.equal(xr.grad, g_ref)


# rows of 2^14 points (kX = 0): the autotuner's register-resident / in-LDS choice matters
MID = dict(N=2 ** 14, J=5, Q=(1, 1), J_fr=2, Q_fr=1, T=2 ** 9, F=2)


def test_autotune_then_every_row_choice_matches_oracle():
    """The autotuner returns a valid choice; and every combination of
    register-resident and in-LDS transforms for 2^14-point rows and of the
    forward contraction's tiles, in every contraction mode, gives the oracle's
    coefficients and gradient (the stored-phase mode's gradient after a forward
    on the same workspace)."""
    P = oracle_plan(MID)
    assert P.NX == 2 ** 14
    rng = np.random.default_rng(1414)
    x = (rng.standard_normal((2, MID["N"])) * 0.5).astype(np.float32)
    xt = torch.from_numpy(x).cuda()
    op = gpu_op(MID)
    choice = op.autotune(2, xt, reps=2)
    assert choice["contraction"] in ("split16", "split16_phase", "fp32") and choice["step_ms"] > 0
    assert not choice["from_cache"] and choice["fwd_tile"] in (16, 32)
    # every available mode was timed (the stored phase fits in memory at this size), both forward tiles
    c = choice["candidates_ms"]
    assert c["split16_register"] > 0 and c["fp32_register"] > 0 and c["split16_phase_register"] > 0
    assert c["split16_lds"] > 0 and choice["fwd_ms"]["tile16"] > 0
    assert op.tuning() == (choice["contraction"], choice["register_rows"], choice["fwd_tile"], choice["bwd_tile"])
    assert op.tuning_radix() == (choice["radix8"], choice["lds_batch"], choice["t_chunk"])
    gs1, gs2 = synth.cotangents((2,) + P.s1_shape(), (2,) + P.s2_shape(), seed=31)
    refs = [(O.jtfs(x[b].astype(np.float64), P),
             O.jtfs_vjp(x[b].astype(np.float64), gs1[b].astype(np.float64), gs2[b].astype(np.float64), P))
            for b in range(2)]
    for mode in MODES + ["split16_phase"]:
        # (register-resident stages, forward tile, backward tile, radix-8 stages, in-LDS batch, t-chunk)
        for rows, tile, btile, r8, lb, tc in (([], 16, 16, [], 8192, 1024), (ALL_ROWS, 32, 32, ALL_ROWS, 4096, 4096),
                                              (["scalogram", "row_fft"], 16, 32, ["scalogram", "row_fft"], 8192, 2048),
                                              (["second_order", "first_adj"], 32, 16, ["first_adj"], 4096, 1024),
                                              (ALL_ROWS, 16, 16, ["second_order", "row_fft"], 8192, 4096)):
            op.set_tuning(mode, rows, fwd_tile=tile, bwd_tile=btile, radix8=r8, lds_batch=lb, t_chunk=tc)
            assert op.tuning_radix() == (r8 if r8 != ALL_ROWS else list(op.RADIX8_BITS), lb, tc)
            ws = op.new_workspace(2)
            s1, s2 = op.forward(xt, ws)
            g = op.vjp(xt, torch.from_numpy(gs1).cuda(), torch.from_numpy(gs2).cuda(), ws=ws,
                       reuse_forward=True).cpu().numpy()
            g1, g2 = s1.cpu().numpy(), s2.cpu().numpy()
            for b in range(2):
                (r1, r2), rg = refs[b]
                check_paths(g1[b], g2[b], r1, r2)
                assert rel_l2(g[b], rg) <= TOL_VJP, (mode, rows, tile, btile, r8, lb, tc)


def test_autotune_cache_reuses_the_choice(tmp_path, monkeypatch):
    """With JTFS_TUNE_CACHE set, a second autotune of the same shape and batch on
    the same device applies the stored choice without timing it."""
    monkeypatch.setenv("JTFS_TUNE_CACHE", str(tmp_path / "tune.txt"))
    xt = torch.from_numpy(synth.batch(1, B=2)).cuda()
    first = gpu_op(P1).autotune(2, xt, reps=1)
    assert not first["from_cache"]
    assert (tmp_path / "tune.txt").read_text().count("B=2") == 1
    op = gpu_op(P1)
    second = op.autotune(2, xt, reps=1)
    assert second["from_cache"]
    for k in ("contraction", "register_rows", "fwd_tile", "bwd_tile"):
        assert second[k] == first[k], k
    assert op.tuning() == (first["contraction"], first["register_rows"], first["fwd_tile"], first["bwd_tile"])
    # another batch size is another key
    third = op.autotune(3, torch.from_numpy(synth.batch(1, B=3)).cuda(), reps=1)
    assert not third["from_cache"]
