"""Pins of the FP64 oracle against facts that do not come from the oracle itself:
library and textbook transforms, values the paper states, closed forms of the
operator on special inputs, exact symmetries, brute-force direct sums and
linear-algebra identities of the adjoint."""
import json
import math
import os

import numpy as np
import pytest

from oracle import jtfs_oracle as O
import synth

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def plan(cfg):
    p = synth.PARAMS[cfg]
    return O.Plan(p["N"], p["J"], p["Q"][0], p["Q"][1], p["J_fr"], p["Q_fr"], p["T"], p["F"])


@pytest.fixture(scope="module")
def P1():
    return plan(1)


@pytest.fixture(scope="module")
def x1():
    return synth.batch(1)[0].astype(np.float64)


# --------------------------------------------------------------------------- DFT

@pytest.mark.parametrize("n", [1, 2, 4, 8, 64, 256, 1024])
def test_fft_matches_defining_sum(n):
    rng = np.random.default_rng(n)
    a = rng.standard_normal((3, n)) + 1j * rng.standard_normal((3, n))
    for inv in (False, True):
        ref = O.dft_direct(a, inverse=inv)
        got = O.fft(a, inverse=inv)
        assert np.max(np.abs(got - ref)) <= 1e-13 * max(1.0, np.max(np.abs(ref)))


@pytest.mark.parametrize("n", [2 ** 11, 2 ** 16])
def test_fft_matches_numpy_fft(n):
    rng = np.random.default_rng(n)
    a = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    assert np.max(np.abs(O.fft(a) - np.fft.fft(a))) <= 1e-13 * np.max(np.abs(np.fft.fft(a)))
    assert np.max(np.abs(O.ifft(a) - np.fft.ifft(a))) <= 1e-13 * np.max(np.abs(np.fft.ifft(a)))


# -------------------------------------------------------------------- filterbank

def test_quality_factor_matches_paper():
    g = GOLDEN["quality_factor_Q1"]
    assert abs(O.quality_factor(1) - g["value"]) <= g["abs_tol"]


@pytest.mark.parametrize("Q", [1, 2, 8, 16, 24])
def test_wavelets_analytic_zero_mean_and_lp_bound(Q):
    M = 4096
    xi, sg = O.filterbank_centres(8, Q)
    hat, _ = O.morlet_family_hat(xi, sg, M)
    neg = O.signed_bins(M) < 0
    assert np.all(hat[:, neg] == 0.0)                 # analytic (sec. 2)
    assert np.all(hat[:, 0] == 0.0)                   # zero mean, exactly
    lp = np.sum(hat ** 2, axis=0)
    assert lp.max() <= 1.0 + 1e-12
    assert abs(lp[: M // 2 + 1].max() - 1.0) <= 1e-12
    f = np.arange(M // 2 + 1) / M
    band = (f >= xi.min()) & (f <= xi.max())
    floor = {1: 0.67, 2: 0.78}.get(Q, 0.86)
    assert lp[: M // 2 + 1][band].min() >= floor     # close to 1 in band


def test_filterbank_geometry():
    for Q in (1, 2, 8, 16):
        xi, sg = O.filterbank_centres(10, Q)
        Qf = O.quality_factor(Q)
        ncq = int(np.sum(np.isclose(xi / sg, Qf)))
        # constant-Q part: ratio 2^(1/Q) between neighbours
        r = xi[1:ncq] / xi[: ncq - 1]
        assert np.allclose(r, 2.0 ** (-1.0 / Q), rtol=1e-13)
        # neighbouring constant-Q filters cross at -3 dB (amplitude 1/sqrt 2)
        a, b = xi[0], xi[1]
        fx = (a * sg[1] + b * sg[0]) / (sg[0] + sg[1])
        g = math.exp(-(fx - a) ** 2 / (2 * sg[0] ** 2))
        assert abs(g - 1 / math.sqrt(2)) < 1e-12
        # linear part: minimum bandwidth, spacing 2 sqrt(ln 2) sigma_min
        smin = O.SIGMA0 / 2 ** 10
        assert np.allclose(sg[ncq:], smin)
        if len(xi) > ncq + 1:
            assert np.allclose(-np.diff(xi[ncq - 1:]), 2 * math.sqrt(math.log(2)) * smin)


def test_peak_response_at_centre(P1):
    """A tone at psi_lambda's centre frequency excites psi_lambda the most."""
    N = P1.N
    hits = 0
    for lam in range(P1.n1):
        m = int(round(P1.xi1[lam] * N))
        S1, _ = O.jtfs(synth.tone(N, m), P1)
        hits += int(np.argmax(S1[:, 0]) == lam)
    assert hits == P1.n1


# ------------------------------------------------------------ closed forms of S

def test_pure_tone_closed_form(P1):
    N, m, A = P1.N, 301, 0.7
    S1, S2 = O.jtfs(synth.tone(N, m, A, 0.3), P1)
    expect = 0.5 * A * np.abs(P1.psi1_hat[:, m])
    assert np.max(np.abs(S1 - expect[:, None])) <= 1e-12 * expect.max()
    assert np.max(np.abs(S2)) <= 1e-12 * expect.max()


def test_dc_gives_zero(P1):
    S1, S2 = O.jtfs(np.full(P1.N, 3.25), P1)
    assert np.max(np.abs(S1)) <= 1e-14 and np.max(np.abs(S2)) <= 1e-14


def test_homogeneity(P1, x1):
    S1, S2 = O.jtfs(x1, P1)
    c = -2.5
    T1, T2 = O.jtfs(c * x1, P1)
    assert np.max(np.abs(T1 - abs(c) * S1)) <= 1e-13 * np.max(np.abs(T1))
    assert np.max(np.abs(T2 - abs(c) * S2)) <= 1e-13 * np.max(np.abs(T2))


def test_shift_by_T_is_exact_frame_shift(P1, x1):
    S1, S2 = O.jtfs(x1, P1)
    T1, T2 = O.jtfs(np.roll(x1, P1.T), P1)
    assert np.max(np.abs(T1 - np.roll(S1, 1, axis=-1))) <= 1e-13 * np.max(S1)
    assert np.max(np.abs(T2 - np.roll(S2, 1, axis=-1))) <= 1e-13 * np.max(S2)


def test_shift_invariance_below_T(P1, x1):
    """Invariance to time shifts within the support T (sec. 2): the change grows
    with the shift and stays well below the coefficients' norm."""
    S1, S2 = O.jtfs(x1, P1)
    prev = 0.0
    for s in (1, 4, 16, 32):
        T1, T2 = O.jtfs(np.roll(x1, s), P1)
        d = np.linalg.norm(T2 - S2) / np.linalg.norm(S2)
        d1 = np.linalg.norm(T1 - S1) / np.linalg.norm(S1)
        assert d > prev
        assert d < 0.25 * s / P1.T + 1e-3 and d1 < 0.25 * s / P1.T + 1e-3
        prev = d


def test_frame_count_matches_paper():
    g = GOLDEN["frames_N65536_T2048"]
    P = plan(2)
    assert P.N == g["N"] and P.T == g["T"] and P.s1_shape()[1] == g["value"]
    assert P.s2_shape()[-1] == g["value"]


@pytest.mark.parametrize("kind", ["linear", "exp"])
def test_spin_direction(P1, kind):
    """Upward chirp -> energy on theta = -1 (spin index 0); downward -> theta = +1."""
    assert GOLDEN["spin_of_upward_chirp"]["value"] == -1
    N = P1.N
    rng = np.random.default_rng(5)
    up = synth.chirp_signal(rng, N, 0.02, 0.4, kind=kind, snr_db=None, am=False)
    down = synth.chirp_signal(rng, N, 0.4, 0.02, kind=kind, snr_db=None, am=False)
    eu = np.sum(O.jtfs(up, P1)[1] ** 2, axis=(0, 1, 3, 4))
    ed = np.sum(O.jtfs(down, P1)[1] ** 2, axis=(0, 1, 3, 4))
    assert eu[0] > 10 * eu[1]
    assert ed[1] > 10 * ed[0]


# ----------------------------------------------- brute force on tiny inputs

SMALL = [
    dict(N=128, J=3, Q=(2, 1), J_fr=2, Q_fr=1, T=16, F=2),
    dict(N=256, J=4, Q=(4, 1), J_fr=2, Q_fr=1, T=16, F=2),
    dict(N=256, J=5, Q=(8, 2), J_fr=3, Q_fr=2, T=32, F=4),
    dict(N=64, J=3, Q=(1, 1), J_fr=1, Q_fr=1, T=8, F=2),
]


@pytest.mark.parametrize("p", SMALL)
def test_cascade_matches_direct_sums(p):
    P = O.Plan(p["N"], p["J"], p["Q"][0], p["Q"][1], p["J_fr"], p["Q_fr"], p["T"], p["F"])
    x = np.random.default_rng(p["N"] + p["J"]).standard_normal(p["N"])
    a1, a2 = O.jtfs(x, P)
    b1, b2 = O.jtfs_direct(x, P)
    assert np.max(np.abs(a1 - b1)) <= 1e-12 * np.max(np.abs(b1))
    assert np.max(np.abs(a2 - b2)) <= 1e-12 * np.max(np.abs(b2))


@pytest.mark.parametrize("p", SMALL)
def test_unaveraged_cascade_matches_direct_sums(p):
    """Eq. (4) (no frequential averaging): FFT cascade against direct sums."""
    P = O.Plan(p["N"], p["J"], p["Q"][0], p["Q"][1], p["J_fr"], p["Q_fr"], p["T"], p["F"])
    x = np.random.default_rng(p["N"] + 5).standard_normal(p["N"])
    a1, a2 = O.jtfs(x, P, average_fr=False)
    b1, b2 = O.jtfs_direct(x, P, average_fr=False)
    assert a2.shape == (P.n_alpha, 2 * P.M_h, P.out_t)
    assert np.max(np.abs(a1 - b1)) <= 1e-12 * np.max(np.abs(b1))
    assert np.max(np.abs(a2 - b2)) <= 1e-12 * np.max(np.abs(b2))


def test_unaveraged_pure_tone_and_frame_shift(P1, x1):
    """Eq. (4) keeps the closed forms of eq. (3): a pure tone has no second order
    and a shift by T moves every frame by one."""
    m, A = 301, 0.7
    n = np.arange(P1.N)
    _, s2 = O.jtfs(A * np.cos(2 * np.pi * m * n / P1.N + 0.3), P1, average_fr=False)
    assert np.max(np.abs(s2)) <= 1e-12
    _, a2 = O.jtfs(x1, P1, average_fr=False)
    _, b2 = O.jtfs(np.roll(x1, P1.T), P1, average_fr=False)
    assert np.max(np.abs(np.roll(a2, 1, axis=-1) - b2)) <= 1e-12 * np.max(np.abs(a2))


# ---------------------------------------------------------------- adjoints

# ------------------------------------ lowpass pairs, unpadded lambda, zeroth order

def _plan_opts(p, **kw):
    return O.Plan(p["N"], p["J"], p["Q"][0], p["Q"][1], p["J_fr"], p["Q_fr"], p["T"], p["F"], **kw)


def test_lowpass_pairs_extend_the_wavelet_paths(P1, x1):
    """The lowpass pairs add one rate (phi_T) and one scale (phi_F): S1 and every
    wavelet-wavelet slice are those of the plain transform."""
    Pc = _plan_opts(synth.PARAMS[1], lowpass_pairs=True)
    S1, S2 = O.jtfs(x1, P1)
    C1, C2 = O.jtfs(x1, Pc)
    assert C2.shape == (P1.n_alpha + 1, P1.n_beta + 1, 2, P1.out_l, P1.out_t)
    assert np.array_equal(C1, S1)
    assert np.max(np.abs(C2[:-1, :-1] - S2)) <= 1e-14 * np.max(S2)
    assert Pc.k2[-1] == int(np.log2(Pc.T)) - Pc.kX and Pc.T_alpha(Pc.n_alpha - 1) == Pc.out_t
    assert Pc.k_fr[-1] == int(np.log2(Pc.F)) and Pc.L_beta(Pc.n_beta - 1) == Pc.L // Pc.F


def test_lowpass_pairs_spins_coincide(x1):
    """A lowpass along lambda (real and even) or along time (a real second-order
    row) leaves no orientation: both spin slots agree, while the wavelet pairs of
    a chirp signal differ between spins."""
    Pc = _plan_opts(synth.PARAMS[1], lowpass_pairs=True)
    _, C2 = O.jtfs(x1, Pc)
    ref = np.max(C2)
    assert np.max(np.abs(C2[:, -1, 0] - C2[:, -1, 1])) <= 1e-12 * ref
    assert np.max(np.abs(C2[-1, :, 0] - C2[-1, :, 1])) <= 1e-12 * ref
    assert np.max(np.abs(C2[:-1, :-1, 0] - C2[:-1, :-1, 1])) > 1e-2 * ref


@pytest.mark.parametrize("p", [synth.PARAMS[1], dict(N=256, J=5, Q=(8, 2), J_fr=3, Q_fr=2, T=32, F=4)])
def test_double_lowpass_pair_keeps_the_sum_of_s1(p):
    """(phi_T, phi_F) is positive and linear in S1: the time lowpass at the frame
    rate keeps sums (DC gain 1) and phi_F sampled at its critical rate F keeps 1/F
    of the sum up to aliasing of order exp(-50): F * sum S2[phi_T, phi_F] = sum S1."""
    Pc = _plan_opts(p, lowpass_pairs=True)
    x = np.random.default_rng(41).standard_normal(Pc.N)
    S1, S2 = O.jtfs(x, Pc, alphas=[Pc.n_alpha - 1])
    for th in range(2):
        assert abs(Pc.F * S2[-1, -1, th].sum() - S1.sum()) <= 1e-12 * S1.sum()


def test_lowpass_pairs_pure_tone(P1):
    """A pure tone has time-constant scalogram rows: the wavelet rates give zero
    in every pair, and phi_T's slices are constant along time and not zero."""
    Pc = _plan_opts(synth.PARAMS[1], lowpass_pairs=True)
    _, C2 = O.jtfs(synth.tone(Pc.N, 301, 0.7, 0.3), Pc)
    ref = np.max(np.abs(C2))
    assert ref > 0
    assert np.max(np.abs(C2[:-1])) <= 1e-12 * ref
    assert np.max(np.abs(C2[-1] - C2[-1][..., :1])) <= 1e-12 * ref


@pytest.mark.parametrize("p", SMALL)
@pytest.mark.parametrize("average_fr", [True, False])
def test_lowpass_pairs_cascade_matches_direct_sums(p, average_fr):
    P = _plan_opts(p, lowpass_pairs=True, unpad=average_fr)
    x = np.random.default_rng(p["N"] + 11).standard_normal(p["N"])
    a1, a2 = O.jtfs(x, P, average_fr=average_fr)
    b1, b2 = O.jtfs_direct(x, P, average_fr=average_fr)
    assert np.max(np.abs(a2 - b2)) <= 1e-12 * np.max(np.abs(b2))


def test_lowpass_pairs_vjp_matches_finite_differences(x1):
    Pc = _plan_opts(synth.PARAMS[1], lowpass_pairs=True)
    gS1, gS2 = synth.cotangents(Pc.s1_shape(), Pc.s2_shape(), seed=31)
    g = O.jtfs_vjp(x1, gS1, gS2, Pc)
    rng = np.random.default_rng(9)
    for _ in range(2):
        v = rng.standard_normal(Pc.N)
        h = 1e-6
        fd = (O.loss(x1 + h * v, gS1, gS2, Pc) - O.loss(x1 - h * v, gS1, gS2, Pc)) / (2 * h)
        assert abs(fd - g @ v) <= 1e-7 * abs(fd)


def test_unpadded_rows_are_the_leading_rows(P1, x1):
    """Unpadding keeps the rows m < ceil(n1 / F), whose log-frequency m F lies on
    a first-order band; the rest of the output is unchanged."""
    Pu = _plan_opts(synth.PARAMS[1], unpad=True)
    S1, S2 = O.jtfs(x1, P1)
    U1, U2 = O.jtfs(x1, Pu)
    nl = -(-P1.n1 // P1.F)
    assert Pu.out_l == nl < P1.out_l and (nl - 1) * P1.F < P1.n1 <= nl * P1.F
    assert np.array_equal(U1, S1) and np.max(np.abs(U2 - S2[..., :nl, :])) <= 1e-14 * np.max(S2)


def test_unpadded_rows_of_the_convnet_input():
    """Sec. 4.2 parametrises the transform for a 44 x 32 output (log-frequency x
    time).  The unpadded row count ceil(n1 / F) depends on n1, which follows the
    filterbank readings here (183 first-order bands where the paper's filterbank
    gives about 176): it lands within two rows of the stated 44, against 64 rows
    padded, and the frame count is the stated 32."""
    g = GOLDEN["convnet_input_lambda_rows"]
    P = O.Plan(g["N"], g["J"], g["Q1"], 1, 6, 1, g["T"], g["F"], unpad=True)
    assert P.out_l == -(-P.n1 // g["F"]) and abs(P.out_l - g["value"]) <= 2
    assert P.L // g["F"] == 64 and P.out_t == 32


def test_zeroth_order_closed_forms(P1):
    """S0 = x * phi_T at the frames: a constant passes unchanged (DC gain 1); a
    tone on bin m is scaled by phi_T_hat(m/N), the Gaussian of width 0.1/T."""
    N, T = P1.N, P1.T
    assert np.max(np.abs(O.zeroth_order(np.full(N, 2.5), P1) - 2.5)) <= 1e-13
    m, A, ph = 5, 0.7, 0.3
    s0 = O.zeroth_order(synth.tone(N, m, A, ph), P1)
    tau = np.arange(N // T)
    gain = np.exp(-(m / N) ** 2 / (2 * (0.1 / T) ** 2))
    assert 0.1 < gain < 0.9
    assert np.max(np.abs(s0 - A * gain * np.cos(2 * np.pi * m * tau * T / N + ph))) <= 1e-13


def test_zeroth_order_adjoint(P1):
    rng = np.random.default_rng(12)
    x = rng.standard_normal(P1.N)
    g = rng.standard_normal(P1.out_t)
    lhs = float(O.zeroth_order(x, P1) @ g)
    rhs = float(x @ O.zeroth_order_adj(g, P1))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def _rdot(a, b):
    return float(np.real(np.sum(np.conj(a) * b)))


def test_stage_adjoints_dot_product(P1):
    rng = np.random.default_rng(11)
    P = P1
    # first order: real x -> complex Y1d
    x = rng.standard_normal(P.N)
    g = rng.standard_normal((P.n1, P.NX)) + 1j * rng.standard_normal((P.n1, P.NX))
    lhs = _rdot(O.first_order_linear(x, P), g)
    rhs = _rdot(x, O.first_order_linear_adj(g, P))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    # second order: real X -> complex Y2
    X = rng.standard_normal((P.n1, P.NX))
    for a in range(P.n_alpha):
        g = rng.standard_normal((P.n1, P.T_alpha(a))) + 1j * rng.standard_normal((P.n1, P.T_alpha(a)))
        lhs = _rdot(O.second_order_linear(X, P, a), g)
        rhs = _rdot(X, O.second_order_linear_adj(g, P, a))
        assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    # time lowpass at each rate
    for k in sorted({P.kX} | {P.kX + k2 for k2 in P.k2}):
        M = P.N >> k
        U = rng.standard_normal((5, M))
        g = rng.standard_normal((5, P.out_t))
        lhs = _rdot(O.time_lowpass(U, P, k), g)
        rhs = _rdot(U, O.time_lowpass_adj(g, P, k, M))
        assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    # frequential wavelet matrices and lowpass: spin mirror and conjugation
    for b in range(P.n_beta):
        W0 = P.freq_wavelet_matrix(b, 0)
        W1 = P.freq_wavelet_matrix(b, 1)
        h0, h1 = P.psi_fr(b, 0), P.psi_fr(b, 1)
        assert np.allclose(h1, np.conj(h0), atol=1e-15)          # real spectrum -> mirror = conj
        assert W0.shape == (P.L_beta(b), P.n1) and W1.shape == W0.shape
        Pm = P.freq_lowpass_matrix(b)
        assert np.allclose(Pm.sum(axis=1), 1.0, atol=1e-12)       # DC gain 1


def test_vjp_matches_finite_differences(P1, x1):
    """FP64 central differences of <gS, S(x)> along random directions (N=2048)."""
    gS1, gS2 = synth.cotangents(P1.s1_shape(), P1.s2_shape())
    g = O.jtfs_vjp(x1, gS1, gS2, P1)
    rng = np.random.default_rng(3)
    for _ in range(3):
        v = rng.standard_normal(P1.N)
        h = 1e-6      # truncation error is O(h^2): 6e-5 at 1e-4, 6e-9 here
        fd = (O.loss(x1 + h * v, gS1, gS2, P1) - O.loss(x1 - h * v, gS1, gS2, P1)) / (2 * h)
        assert abs(fd - g @ v) <= 1e-7 * abs(fd)


def test_unaveraged_vjp_matches_finite_differences(P1, x1):
    """Eq. (4): FP64 central differences against the VJP."""
    gS1, gS2 = synth.cotangents(P1.s1_shape(), P1.s2_shape(False), seed=21)
    g = O.jtfs_vjp(x1, gS1, gS2, P1, average_fr=False)
    rng = np.random.default_rng(4)
    for _ in range(2):
        v = rng.standard_normal(P1.N)
        h = 1e-6
        fd = (O.loss(x1 + h * v, gS1, gS2, P1, False) - O.loss(x1 - h * v, gS1, gS2, P1, False)) / (2 * h)
        assert abs(fd - g @ v) <= 1e-7 * abs(fd)


def test_vjp_alpha_subset_consistent(P1, x1):
    gS1, gS2 = synth.cotangents(P1.s1_shape(), P1.s2_shape())
    full = O.jtfs_vjp(x1, gS1, gS2, P1)
    parts = O.jtfs_vjp(x1, gS1, np.zeros_like(gS2), P1)
    for a in range(P1.n_alpha):
        g = np.zeros_like(gS2)
        g[a] = gS2[a]
        parts = parts + O.jtfs_vjp(x1, np.zeros_like(gS1), g, P1)
    assert np.max(np.abs(parts - full)) <= 1e-12 * np.max(np.abs(full))


def test_plan_sizes_follow_readings():
    """Derived sizes obey the definitions: L = next pow2 of n1, every decimation
    divides T (resp. F), and the output grid is N/T x L/F."""
    for cfg in (1, 2, 3, 4, 5):
        P = plan(cfg)
        assert P.L >= P.n1 > P.L // 2
        assert P.kX <= int(math.log2(P.T))
        assert all(P.kX + k <= int(math.log2(P.T)) for k in P.k2)
        assert all(k <= int(math.log2(P.F)) for k in P.k_fr)
        assert list(P.k2) == sorted(P.k2) and list(P.k_fr) == sorted(P.k_fr)
        assert P.s2_shape() == (P.n_alpha, P.n_beta, 2, P.L // P.F, P.N // P.T)


# ----------------------------------------------------------------- mu-log

def test_mulog_means_and_closed_values():
    """mu is the plain average of each path (a brute-force loop); S = eps mu (e - 1)
    maps to exactly 1, S = 0 to 0; the map is increasing; the adjoint matches
    central differences of the elementwise log."""
    rng = np.random.default_rng(8)
    S1 = rng.random((3, 5, 4))
    S2 = rng.random((3, 2, 3, 2, 4, 4))
    mu1, mu2 = O.path_means(S1, S2)
    assert abs(mu1 - sum(S1.ravel()) / S1.size) <= 1e-15
    for a in range(2):
        for b in range(3):
            for t in range(2):
                vals = [S2[n, a, b, t, l, k] for n in range(3) for l in range(4) for k in range(4)]
                assert abs(mu2[a, b, t] - sum(vals) / len(vals)) <= 1e-15
    e = O.MULOG_EPS
    T1 = np.full_like(S1, e * mu1 * (math.e - 1.0))
    T2 = e * mu2[None, :, :, :, None, None] * (math.e - 1.0) * np.ones_like(S2)
    o1, o2 = O.mulog(T1, T2, mu1, mu2)
    assert np.allclose(o1, 1.0, atol=1e-15) and np.allclose(o2, 1.0, atol=1e-15)
    z1, z2 = O.mulog(np.zeros_like(S1), np.zeros_like(S2), mu1, mu2)
    assert not z1.any() and not z2.any()
    a1, _ = O.mulog(S1, S2, mu1, mu2)
    b1, _ = O.mulog(S1 + 1e-3, S2, mu1, mu2)
    assert np.all(b1 > a1)
    g1, g2 = rng.standard_normal(S1.shape), rng.standard_normal(S2.shape)
    v1, v2 = O.mulog_vjp(S1, S2, mu1, mu2, g1, g2)
    h = 1e-6
    p1, p2 = O.mulog(S1 + h, S2 + h, mu1, mu2)
    m1, m2 = O.mulog(S1 - h, S2 - h, mu1, mu2)
    assert np.allclose(v1, g1 * (p1 - m1) / (2 * h), rtol=1e-7, atol=1e-9)
    assert np.allclose(v2, g2 * (p2 - m2) / (2 * h), rtol=1e-7, atol=1e-9)


def test_mulog_time_scattering_paths():
    """Time scattering: one path per (alpha, lambda1) row, its mean over the
    signals and frames (a brute-force loop); S = eps mu (e - 1) maps to 1."""
    rng = np.random.default_rng(81)
    S1 = rng.random((3, 5, 4))
    S2 = rng.random((3, 2, 5, 4))
    mu1, mu2 = O.path_means(S1, S2, path_axes=1)
    assert mu2.shape == (2, 5)
    for a in range(2):
        for lam in range(5):
            vals = [S2[n, a, lam, k] for n in range(3) for k in range(4)]
            assert abs(mu2[a, lam] - sum(vals) / len(vals)) <= 1e-15
    T2 = O.MULOG_EPS * mu2[None, :, :, None] * (math.e - 1.0) * np.ones_like(S2)
    _, o2 = O.mulog(S1, T2, mu1, mu2, path_axes=1)
    assert np.allclose(o2, 1.0, atol=1e-15)
    g2 = rng.standard_normal(S2.shape)
    _, v2 = O.mulog_vjp(S1, S2, mu1, mu2, S1, g2, path_axes=1)
    assert np.allclose(v2, g2 / (O.MULOG_EPS * mu2[None, :, :, None] + S2), rtol=1e-15)


# ------------------------------------------------------- texture resynthesis

def test_texture_error_gradient_matches_finite_differences(P1, x1):
    """The gradient of E(y) = ||Sx - Sy|| / ||Sx|| against FP64 central differences."""
    rng = np.random.default_rng(31)
    y = rng.standard_normal(P1.N) * np.std(x1)
    target = O.texture_target(x1, P1)
    E, g = O.texture_error_grad(y, target, P1)
    for _ in range(2):
        v = rng.standard_normal(P1.N)
        h = 1e-6
        fd = (O.texture_error_grad(y + h * v, target, P1)[0] - O.texture_error_grad(y - h * v, target, P1)[0]) / (2 * h)
        assert abs(fd - g @ v) <= 1e-6 * abs(fd)


def test_texture_loop_bold_driver_rules(P1, x1):
    """Starting at the target the error is 0 and nothing moves; from noise the
    best error never increases, a small first step lowers E by about
    mu ||grad E||^2 (first order), and mu follows the accept/reject factors."""
    y, hist, mu = O.texture_resynthesis(x1, x1, P1, 3, 1e-3)
    assert hist.max() == 0.0 and np.array_equal(y, x1)
    rng = np.random.default_rng(32)
    y0 = rng.standard_normal(P1.N) * np.std(x1)
    target = O.texture_target(x1, P1)
    E0, g0 = O.texture_error_grad(y0, target, P1)
    mu0 = 1e-4 * np.linalg.norm(y0) / np.linalg.norm(g0)
    E1, _ = O.texture_error_grad(y0 - mu0 * g0, target, P1)
    pred = mu0 * float(g0 @ g0)
    assert abs((E0 - E1) - pred) <= 1e-2 * pred
    y, hist, mu = O.texture_resynthesis(x1, y0, P1, 12, -0.05)
    assert hist[0] == pytest.approx(E0, rel=1e-12)
    assert np.all(np.diff(hist) <= 0.0) and hist[-1] < 0.9 * hist[0]
    ups = int(np.sum(np.diff(hist) < 0))
    mu_start = 0.05 * np.linalg.norm(y0) / np.linalg.norm(g0)
    assert mu == pytest.approx(mu_start * O.BOLD_UP ** ups * O.BOLD_DOWN ** (12 - ups), rel=1e-12)


# ------------------------------------------------------------ time scattering

@pytest.mark.parametrize("p", SMALL)
def test_scattering1d_matches_direct_sums(p):
    P = O.Plan(p["N"], p["J"], p["Q"][0], p["Q"][1], p["J_fr"], p["Q_fr"], p["T"], p["F"])
    x = np.random.default_rng(p["N"] + 9).standard_normal(p["N"])
    a1, a2 = O.scattering1d(x, P)
    b1, b2 = O.scattering1d_direct(x, P)
    assert a2.shape == (P.n_alpha, P.n1, P.out_t)
    assert np.max(np.abs(a1 - b1)) <= 1e-12 * np.max(np.abs(b1))
    assert np.max(np.abs(a2 - b2)) <= 1e-12 * np.max(np.abs(b2))


def test_scattering1d_closed_forms_and_relation_to_jtfs(P1, x1):
    """A pure tone has no second order; a shift by T moves every frame by one; S1
    is that of jtfs, and each S2 row is the time lowpass of the modulus of the
    second-order row that jtfs passes to its frequential stage."""
    m, A = 301, 0.7
    n = np.arange(P1.N)
    _, s2 = O.scattering1d(A * np.cos(2 * np.pi * m * n / P1.N + 0.3), P1)
    assert np.max(np.abs(s2)) <= 1e-12
    a1, a2 = O.scattering1d(x1, P1)
    b1, b2 = O.scattering1d(np.roll(x1, P1.T), P1)
    assert np.max(np.abs(np.roll(a2, 1, axis=-1) - b2)) <= 1e-12 * np.max(np.abs(a2))
    j1, _, inter = O.jtfs(x1, P1, return_intermediates=True)
    assert np.array_equal(j1, a1)
    for a in range(P1.n_alpha):
        ref = O.time_lowpass(np.abs(inter["Y2"][a]), P1, P1.kX + P1.k2[a])
        assert np.allclose(a2[a], ref, rtol=0, atol=1e-14 * np.max(np.abs(ref)))


def test_scattering1d_vjp_matches_finite_differences(P1, x1):
    gS1, gS2 = synth.cotangents(P1.s1_shape(), (P1.n_alpha, P1.n1, P1.out_t), seed=23)
    g = O.scattering1d_vjp(x1, gS1, gS2, P1)
    f = lambda y: float(np.sum(gS1 * O.scattering1d(y, P1)[0]) + np.sum(gS2 * O.scattering1d(y, P1)[1]))
    rng = np.random.default_rng(5)
    for _ in range(2):
        v = rng.standard_normal(P1.N)
        h = 1e-6
        fd = (f(x1 + h * v) - f(x1 - h * v)) / (2 * h)
        assert abs(fd - g @ v) <= 1e-7 * abs(fd)


# ------------------------------------- subsampling schedule and stopping rules
#
# Decimating a complex band by 2^k keeps one period of width 2^-k of its
# spectrum: the band may be decimated without folding onto itself when the
# spectrum outside the interval of that width centred on its peak is negligible.
# The reading of the critical rate (sec. 1: each band's rate depends on its
# centre frequency) takes "negligible" as a Gaussian's value beyond five standard
# deviations, e^-12.5, and the rate as the lowest one that meets it (up to the
# caps that keep the output on the N/T and L/F grids).  These tests measure that
# property on the filter spectra themselves, so a change of the envelope
# constant, of a lowpass width or of a stopping rule fails one of them.

GAUSS_5SIGMA = math.exp(-12.5)


def _outside_band_ratio(hat, M, xi, halfwidth):
    """max |hat| over grid bins farther than halfwidth (cycles per grid sample)
    from xi, relative to the spectrum's peak (bin m has frequency m~/M)."""
    f = O.signed_bins(M) / M
    out = np.abs(f - xi) > halfwidth
    return float(np.max(np.abs(hat[out]), initial=0.0) / np.max(np.abs(hat)))


def _family_schedule(P, which):
    """(grid size, list of (xi, sigma, spectrum, k, cap)) of one wavelet family."""
    logT, logF = int(math.log2(P.T)), int(math.log2(P.F))
    if which == "first":
        return P.N, [(P.xi1[i], P.sigma1[i], P.psi1_hat[i], P.kX, logT) for i in range(P.n1)]
    if which == "second":
        return P.NX, [(P.xi2[a], P.sigma2[a], P.psi2_hat[a], P.k2[a], logT - P.kX) for a in range(P.n_alpha)]
    return P.L, [(P.xi_fr[b], P.sigma_fr[b], P.psi_fr_hat[b], P.k_fr[b], logF) for b in range(P.n_beta)]


@pytest.mark.parametrize("cfg", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("which", ["first", "second", "frequential"])
def test_decimation_keeps_each_band_within_its_alias_period(cfg, which):
    """Sufficient: every filter's spectrum outside the period kept by its
    decimation (width 2^-k, centred on xi) is at most e^-12.5 of its peak."""
    P = plan(cfg)
    M, fam = _family_schedule(P, which)
    for xi, sg, hat, k, cap in fam:
        r = _outside_band_ratio(hat, M, xi, 2.0 ** -(k + 1))
        assert r <= GAUSS_5SIGMA * (1 + 1e-9), (which, xi, k, r)


@pytest.mark.parametrize("cfg", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("which", ["first", "second", "frequential"])
def test_decimation_is_the_lowest_rate_that_keeps_the_band(cfg, which):
    """Minimal: one more halving of the rate (where the cap allows it) leaves
    part of the spectrum above e^-12.5 of the peak outside the kept period.  The
    first order uses one common rate set by its widest filter (the top one)."""
    P = plan(cfg)
    M, fam = _family_schedule(P, which)
    if which == "first":
        fam = fam[:1]
        assert np.argmax(P.sigma1) == 0
    for xi, sg, hat, k, cap in fam:
        if k == cap:
            continue
        h = 2.0 ** -(k + 2)
        # the continuous spectrum just outside the halved period, same normalisation
        c = np.max(np.abs(hat)) / float(O.morlet_hat(xi, sg, np.array([xi]))[0])
        edge = float(O.morlet_hat(xi, sg, np.array([xi + h]))[0]) * c
        grid = _outside_band_ratio(hat, M, xi, h)
        assert max(edge / np.max(np.abs(hat)), grid) > GAUSS_5SIGMA, (which, xi, k)


@pytest.mark.parametrize("cfg", [1, 2, 3, 4, 5])
def test_lowpass_at_output_nyquist(cfg):
    """phi_T at the output Nyquist 1/(2T) and phi_F at 1/(2F) are e^-12.5 of their
    DC gain of 1: the same five-deviation rule as the wavelets' rates, so the
    N/T and L/F output grids hold the lowpassed coefficients."""
    P = plan(cfg)
    phT = O.gauss_lowpass_hat(P.N, P.N, P.T)
    assert phT[0] == 1.0
    assert abs(phT[P.N // (2 * P.T)] - GAUSS_5SIGMA) <= 1e-15
    phF = O.gauss_lowpass_hat(P.L, P.L, P.F)
    assert phF[0] == 1.0
    assert abs(phF[P.L // (2 * P.F)] - GAUSS_5SIGMA) <= 1e-15
    # the same lowpass on every decimated grid the cascade uses: bin N/(2T) is the
    # output Nyquist at any rate 2^-k with k <= log2 T
    for k in sorted({P.kX} | {P.kX + k2 for k2 in P.k2}):
        M = P.N >> k
        ph = O.gauss_lowpass_hat(M, P.N, P.T)
        assert P.N // (2 * P.T) <= M // 2
        assert abs(ph[P.N // (2 * P.T)] - GAUSS_5SIGMA) <= 1e-15


def _cq_count(xi, Q):
    r = xi[1:] / xi[:-1]
    n = 1
    while n < len(xi) and abs(r[n - 1] - 2.0 ** (-1.0 / Q)) <= 1e-12:
        n += 1
    return n


@pytest.mark.parametrize("Jp,Q", [(6, 8), (12, 16), (13, 12), (11, 16), (14, 24), (4, 1), (10, 1), (3, 1),
                                  (4, 2), (5, 2), (12, 2)])
def test_filterbank_top_and_stopping_rules(Jp, Q):
    """The family's ends follow from the geometry alone:
    * top: the next filter up the geometric ladder, xi_0 2^(1/Q), would be the
      mirror of xi_0 about Nyquist, 1 - xi_0 (Q >= 2); for one filter per
      octave that mirror would leave xi_0 = 1/3 and the top sits at 0.35;
    * constant-Q part: the last filter's bandwidth sigma = xi/Q_f is still at
      least sigma_min = 0.1/2^J (its time support at most about 2^J), and the
      next one down would be narrower (longer than 2^J);
    * linear part: filters of bandwidth sigma_min, neighbours crossing at -3 dB;
      the lowest centre lies at least one spacing above DC and one more filter
      would not."""
    xi, sg = O.filterbank_centres(Jp, Q)
    if Q >= 2:
        assert abs(xi[0] * 2.0 ** (1.0 / Q) - (1.0 - xi[0])) <= 1e-15
    else:
        assert 1.0 / (1.0 + 2.0) < 0.35 and xi[0] == 0.35
    smin = 0.1 / 2.0 ** Jp
    n = _cq_count(xi, Q)
    Qf = O.quality_factor(Q)
    assert sg[n - 1] >= smin and np.all(sg[:n] >= smin)
    assert xi[n - 1] * 2.0 ** (-1.0 / Q) / Qf < smin
    lin = xi[n:]
    assert np.all(sg[n:] == smin)
    # spacing: Gaussians of width smin whose centres are `spacing` apart cross at -3 dB
    spacing = (xi[n - 1] - lin[0]) if len(lin) else None
    if spacing is not None:
        assert abs(math.exp(-(spacing / 2) ** 2 / (2 * smin ** 2)) - 1 / math.sqrt(2)) <= 1e-12
        assert np.allclose(-np.diff(xi[n - 1:]), spacing, rtol=0, atol=1e-15)
        assert lin[-1] >= spacing and lin[-1] - spacing < spacing
    else:
        # no linear filter fits: the last constant-Q centre is already within two spacings of DC
        d = 2 * math.sqrt(math.log(2)) * smin
        assert xi[n - 1] - d < d


@pytest.mark.parametrize("cfg", [1, 2, 3, 4, 5])
def test_first_order_family_covers_up_to_nyquist(cfg):
    """The first order reaches the top of the band: the LP sum is at least its
    in-band floor on [xi_0, 1/2] (where config 2's chirps end, at 0.45)."""
    P = plan(cfg)
    lp = np.sum(P.psi1_hat ** 2, axis=0)[: P.N // 2 + 1]
    f = np.arange(P.N // 2 + 1) / P.N
    band = (f >= P.xi1[-1]) & (f <= 0.45)
    assert lp[band].min() >= 0.86


# ------------------------------------------------------ conditioning (reading R24)

def _click_gradient_sensitivity(N, params):
    """Relative change of the FP64 oracle's gradient (cotangent on S1 and on two
    temporal rates) under a perturbation of the input of 1e-7 of its RMS (the
    size of FP32 rounding), at a click-train target and at its white-noise
    start."""
    P = O.Plan(N, params["J"], params["Q"][0], params["Q"][1], params["J_fr"], params["Q_fr"], params["T"],
               params["F"])
    y, x0 = synth.cfg3_pair(synth._rngs(3, 1)[0], N)
    gs1, gs2 = synth.cotangents((1,) + P.s1_shape(), (1,) + P.s2_shape(), seed=9)
    keep = np.zeros(P.n_alpha, bool)
    keep[[P.n_alpha - 1, P.n_alpha - 4]] = True
    gs2[:, ~keep] = 0.0
    g1, g2 = gs1[0].astype(np.float64), gs2[0].astype(np.float64)
    d = np.random.default_rng(5).standard_normal(N)
    out = {}
    for name, v in (("target", y), ("start", x0)):
        v = v.astype(np.float32).astype(np.float64)
        a = O.jtfs_vjp(v, g1, g2, P)
        b = O.jtfs_vjp(v + 1e-7 * np.linalg.norm(v) / math.sqrt(N) * d, g1, g2, P)
        out[name] = np.linalg.norm(b - a) / np.linalg.norm(a)
    return out


def test_click_train_gradient_is_ill_conditioned():
    """Reading R24, on the click-train family at 2^13 samples (J=9, T=2^9, the
    other parameters of the texture workload): between clicks the
    high-frequency first-order outputs are near zero, where the modulus
    Jacobian y/|y| turns with any perturbation, so an input change at FP32
    rounding size moves even the FP64 gradient by percents at the target, but
    by about that rounding size at the white-noise start.  This is why FP32
    gradients of that workload are checked at the start (where texture
    synthesis differentiates)."""
    p = dict(synth.PARAMS[3], J=9, T=2 ** 9)
    s = _click_gradient_sensitivity(2 ** 13, p)
    assert s["target"] > 1e-2, s
    assert s["start"] < 1e-6, s


@pytest.mark.slow
def test_click_train_gradient_is_ill_conditioned_full_size():
    """The same at the texture workload's own size (2^17 samples)."""
    s = _click_gradient_sensitivity(2 ** 17, synth.PARAMS[3])
    assert s["target"] > 1e-2, s
    assert s["start"] < 1e-6, s
