"""Plain FP64 CPU oracle for joint time-frequency scattering (JTFS) and its gradient.

TEST INFRASTRUCTURE ONLY.  Imported by ``tests/``, by ``__graft_entry__.smoke()``
and by the ``cpu_baseline`` leg of ``bench.py`` -- never by the GPU library or its
Python binding, and it shares no code with them (no kernels, tables or helpers).

It computes, in float64 and in the order the paper states them:

* the first-order scalogram  X(t, lambda) = |x * psi_lambda|(t)          (sec. 2)
* first-order coefficients   S1 = X *_t phi_T  (no frequential averaging; sec. 4.2)
* second order, eq. (3):     S2 = | X *_{t,lambda} Psi_{alpha,beta,theta} | *_{t,lambda} Phi_{T,F}
  with the separable joint wavelet of eq. (2), Psi = psi_alpha(t) psi_{beta,theta}(lambda),
  and the dilations of eq. (1)
* the variant of eq. (4) (``average_fr=False``): no frequential averaging, each
  (alpha, beta, theta) slice is |X *_{t,lambda} Psi| *_t phi_T on the lambda grid of
  its frequential wavelet
* the reverse-mode gradient by Hermitian adjoints of each stage in reverse order (sec. 5)
* time scattering (sec. 4, the Scattering1D comparison): the temporal wavelets
  alone applied to the scalogram, S2 = |X_lambda * psi_alpha| *_t phi_T for every
  (alpha, lambda) pair, no averaging along lambda
* the mu-log renormalisation of the convnet input (sec. 4): per-path means mu
  over a set of signals and log(1 + S / (eps mu))
* texture resynthesis (sec. 5): gradient descent on the normalised error
  ||Sx - Sy|| / ||Sx|| with the bold-driver learning rate
* the lowpass pairs that complete the joint filterbank of the cited transform
  (sec. 2): with ``lowpass_pairs`` the temporal rates gain phi_T and the
  frequential scales gain phi_F, each kept at its critical rate, and eq. (3)
  runs over every (alpha, beta, theta); the zeroth order S0 = x * phi_T
* the unpadded log-frequency output (``unpad``): the rows of S2 whose
  log-frequency m F falls on a first-order band, m < ceil(n1 / F)

The paper states the operator only as continuous equations.  The discretisation
used here (each item is a reading of the paper, listed in the design notes):

* all convolutions are circular on power-of-two grids; the DFT is
  X[m] = sum_n x[n] exp(-2 pi i m n / M), its inverse carries 1/M;
* Morlet wavelets are defined by their spectra: a Gaussian minus a corrective
  Gaussian at DC so that psi_hat(0) = 0 exactly, hard zero on negative
  frequencies (analytic, sec. 2) and the Nyquist bin kept;
* neighbouring wavelets cross at -3 dB, which gives a quality factor of about 2.5
  at one filter per octave (sec. 3.3); the lowest octave below the constant-Q range
  is tiled by linearly spaced filters of the minimum bandwidth;
* each family is normalised by one scalar so that its Littlewood-Paley sum peaks
  at exactly 1;
* lowpass filters are Gaussians of width sigma0/T (time) and sigma0/F (log-frequency),
  DC gain 1;
* every band is kept at a critical rate that depends on its bandwidth (sec. 1):
  decimate by 2^k with k the largest integer leaving a Nyquist of at least
  5 sigma, capped so that every output lands on the N/T (and L/F) grid;
* the log-frequency axis is zero-padded to the next power of two L and treated
  circularly; the lowest lambda index is the highest frequency, and the spin whose
  frequential wavelet is analytic along increasing index is theta = -1 (an upward
  chirp concentrates there, sec. 2);
* the modulus gradient is z / max(|z|, 1e-30).

Every intermediate is computed at full rate and then subsampled (the plain
definition); nothing is folded, fused or reordered.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SIGMA0 = 0.1      # lowpass width constant: phi_T has sigma = SIGMA0 / T cycles/sample
C_ENV = 5.0       # critical-rate rule: decimated Nyquist >= C_ENV * sigma
EPS_MOD = 1e-30   # modulus-gradient guard


# ---------------------------------------------------------------------------
# DFT: own radix-2 FFT plus a direct O(M^2) transform (used as its check and as
# the direct-convolution fallback)
# ---------------------------------------------------------------------------

def fft(a, inverse=False):
    """DFT along the last axis, power-of-two length, by iterative radix-2
    decimation in time.  Forward: sum_n a[n] e^{-2 pi i m n/M}; inverse
    divides by M and uses e^{+2 pi i m n/M}."""
    a = np.asarray(a, dtype=np.complex128)
    n = a.shape[-1]
    if n < 1 or n & (n - 1):
        raise ValueError("fft length must be a power of two")
    sign = 1.0 if inverse else -1.0
    lead = a.shape[:-1]
    # t[..., r, :] holds the length-m DFT of the samples a[..., r::n//m]
    t = a.reshape(lead + (n, 1))
    m = 1
    while m < n:
        half = t.shape[-2] // 2
        even = t[..., :half, :]
        odd = t[..., half:, :]
        k = np.arange(m, dtype=np.float64)
        ang = sign * 2.0 * np.pi * k / (2 * m)
        w = np.cos(ang) + 1j * np.sin(ang)
        wo = w * odd
        t = np.concatenate([even + wo, even - wo], axis=-1)
        m *= 2
    out = t.reshape(lead + (n,))
    return out / n if inverse else out


def ifft(a):
    return fft(a, inverse=True)


def dft_direct(a, inverse=False):
    """Textbook DFT by the defining sum (O(M^2)); same conventions as fft()."""
    a = np.asarray(a, dtype=np.complex128)
    n = a.shape[-1]
    idx = np.arange(n)
    sign = 1.0 if inverse else -1.0
    # reduce the product m*j modulo n first: keeps the angle small and exact
    ang = sign * 2.0 * np.pi * (np.outer(idx, idx) % n).astype(np.float64) / n
    mat = np.cos(ang) + 1j * np.sin(ang)
    out = a @ mat.T
    return out / n if inverse else out


def signed_bins(M):
    """m~ = m for m <= M/2, m - M otherwise (bin M/2 is taken as positive)."""
    m = np.arange(M)
    return np.where(m <= M // 2, m, m - M)


# ---------------------------------------------------------------------------
# Filterbanks (sec. 2, eq. (1))
# ---------------------------------------------------------------------------

def quality_factor(Q):
    """xi/sigma of a Gaussian-spectrum wavelet whose neighbours, 2^(1/Q) apart,
    cross at -3 dB.  Q = 1 gives 2.4977 (the paper quotes about 2.5, sec. 3.3)."""
    rho = 2.0 ** (-1.0 / Q)
    return (1.0 + rho) / (1.0 - rho) * math.sqrt(math.log(2.0))


def critical_log2(sigma, cap):
    """Largest k in [0, cap] with the decimated Nyquist 2^-(k+1) >= C_ENV*sigma."""
    v = 1.0 / (2.0 * C_ENV * sigma)
    k = math.floor(math.log2(v)) if v >= 1.0 else 0
    return int(min(max(k, 0), cap))


def filterbank_centres(Jp, Q):
    """(xi, sigma) of a Morlet family with Q filters per octave over Jp octaves.

    Constant-Q filters xi_n = xi_max 2^(-n/Q) with sigma = xi/Q_f while
    sigma >= SIGMA0/2^Jp; below, filters of the minimum bandwidth spaced by their
    -3 dB width down to xi >= that spacing."""
    Qf = quality_factor(Q)
    xi_max = max(1.0 / (1.0 + 2.0 ** (1.0 / Q)), 0.35)
    sigma_min = SIGMA0 / 2.0 ** Jp
    xis, sigmas = [], []
    n = 0
    while True:
        xi = xi_max * 2.0 ** (-n / Q)
        if xi / Qf < sigma_min:
            break
        xis.append(xi)
        sigmas.append(xi / Qf)
        n += 1
    if not xis:
        raise ValueError("no constant-Q filter: J too small")
    delta = 2.0 * math.sqrt(math.log(2.0)) * sigma_min
    xi_c = xis[-1]
    k = 1
    while xi_c - k * delta >= delta:
        xis.append(xi_c - k * delta)
        sigmas.append(sigma_min)
        k += 1
    return np.array(xis), np.array(sigmas)


def morlet_hat(xi, sigma, f):
    """Morlet spectrum at frequencies f: Gaussian at xi minus kappa times a
    Gaussian at 0 (so the value at f = 0 is exactly 0), zero for f < 0."""
    f = np.asarray(f, dtype=np.float64)
    # kappa e^{-f^2/2s^2} with kappa = e^{-xi^2/2s^2}, written as one exponential so
    # that both terms are the same rounded number at f = 0
    v = (np.exp(-(f - xi) ** 2 / (2.0 * sigma * sigma))
         - np.exp(-(f * f + xi * xi) / (2.0 * sigma * sigma)))
    return np.where(f >= 0.0, v, 0.0)


def morlet_family_hat(xis, sigmas, M):
    """Spectra of a family on an M-point grid (f = m~/M), normalised so that
    max over 0 <= f <= 1/2 of sum |psi_hat|^2 equals 1."""
    f = signed_bins(M) / M
    raw = np.stack([morlet_hat(a, b, f) for a, b in zip(xis, sigmas)])
    lp = np.sum(raw ** 2, axis=0)
    c = 1.0 / math.sqrt(np.max(lp[: M // 2 + 1]))
    return raw * c, c


def gauss_lowpass_hat(M, units_per_cycle, width):
    """Gaussian lowpass spectrum on an M-point grid whose bin m has frequency
    m~/units_per_cycle, with sigma = SIGMA0/width; DC gain 1, real and even."""
    f = signed_bins(M) / units_per_cycle
    s = SIGMA0 / width
    return np.exp(-f * f / (2.0 * s * s))


def is_pow2(v):
    return v >= 1 and (v & (v - 1)) == 0


@dataclass
class Plan:
    N: int
    J: int
    Q1: int
    Q2: int
    J_fr: int
    Q_fr: int
    T: int
    F: int
    lowpass_pairs: bool = False
    unpad: bool = False
    # derived
    xi1: np.ndarray = field(init=False)
    sigma1: np.ndarray = field(init=False)
    psi1_hat: np.ndarray = field(init=False)
    kX: int = field(init=False)
    NX: int = field(init=False)
    xi2: np.ndarray = field(init=False)
    sigma2: np.ndarray = field(init=False)
    psi2_hat: np.ndarray = field(init=False)
    k2: list = field(init=False)
    L: int = field(init=False)
    xi_fr: np.ndarray = field(init=False)
    sigma_fr: np.ndarray = field(init=False)
    psi_fr_hat: np.ndarray = field(init=False)
    k_fr: list = field(init=False)

    def __post_init__(self):
        N, T, F = self.N, self.T, self.F
        if not (is_pow2(N) and is_pow2(T) and is_pow2(F)):
            raise ValueError("N, T and F must be powers of two")
        if T > N:
            raise ValueError("T must not exceed N")
        logT = int(math.log2(T))
        # first-order filterbank on the N grid (cycles/sample)
        self.xi1, self.sigma1 = filterbank_centres(self.J, self.Q1)
        self.psi1_hat, self.c1 = morlet_family_hat(self.xi1, self.sigma1, N)
        # scalogram rate: common to every row so that lambda-columns align
        self.kX = min(logT, critical_log2(self.sigma1[0], int(math.log2(N))))
        self.NX = N >> self.kX
        # second-order temporal filterbank, in scalogram units
        if self.J - self.kX < 1:
            raise ValueError("J - kX must be >= 1")
        self.xi2, self.sigma2 = filterbank_centres(self.J - self.kX, self.Q2)
        self.psi2_hat, self.c2 = morlet_family_hat(self.xi2, self.sigma2, self.NX)
        self.k2 = [critical_log2(s, logT - self.kX) for s in self.sigma2]
        if self.lowpass_pairs:
            # phi_T as one more temporal rate: its spectrum on the scalogram grid (two-sided,
            # DC gain 1) at the rate the cap allows, so that its rows fall on the N/T frames
            self.psi2_hat = np.vstack([self.psi2_hat, gauss_lowpass_hat(self.NX, N, T)[None, :]])
            self.k2.append(logT - self.kX)
        # frequential filterbank on the zero-padded log-frequency axis
        n1 = len(self.xi1)
        self.L = 1 << int(math.ceil(math.log2(n1)))
        if not (1 <= self.J_fr <= int(math.log2(self.L))):
            raise ValueError("J_fr out of range")
        if F > self.L:
            raise ValueError("F must not exceed L")
        self.xi_fr, self.sigma_fr = filterbank_centres(self.J_fr, self.Q_fr)
        self.psi_fr_hat, self.c_fr = morlet_family_hat(self.xi_fr, self.sigma_fr, self.L)
        self.k_fr = [critical_log2(s, int(math.log2(F))) for s in self.sigma_fr]
        if self.lowpass_pairs:
            # phi_F as one more frequential scale, real and even along lambda, at its critical rate
            self.psi_fr_hat = np.vstack([self.psi_fr_hat, gauss_lowpass_hat(self.L, self.L, F)[None, :]])
            self.k_fr.append(critical_log2(SIGMA0 / F, int(math.log2(F))))

    # sizes ---------------------------------------------------------------
    @property
    def n1(self):
        return len(self.xi1)

    @property
    def n_alpha(self):
        return len(self.k2)

    @property
    def n_beta(self):
        return len(self.k_fr)

    def T_alpha(self, a):
        return self.NX >> self.k2[a]

    def L_beta(self, b):
        return self.L >> self.k_fr[b]

    @property
    def out_t(self):
        return self.N // self.T

    @property
    def out_l(self):
        if self.unpad:
            return -(-self.n1 // self.F)
        return self.L // self.F

    def s1_shape(self):
        return (self.n1, self.out_t)

    @property
    def M_h(self):
        """lambda rows of one spin summed over beta on the wavelets' own grids."""
        return sum(self.L_beta(b) for b in range(self.n_beta))

    def s2_shape(self, average_fr=True):
        """eq. (3): [n_alpha, n_beta, 2, L/F, N/T].  eq. (4) (no frequential
        averaging): the ragged slices packed as [n_alpha, sum_beta 2 L_beta, N/T],
        beta outer and theta inner (see s2_rows)."""
        if average_fr:
            return (self.n_alpha, self.n_beta, 2, self.out_l, self.out_t)
        return (self.n_alpha, 2 * self.M_h, self.out_t)

    def s2_rows(self, b, spin):
        """Rows of the (beta, theta) slice in the packed eq. (4) output."""
        o = 2 * sum(self.L_beta(q) for q in range(b)) + spin * self.L_beta(b)
        return slice(o, o + self.L_beta(b))

    # frequential wavelets and lowpass matrices ---------------------------
    def psi_fr(self, b, spin):
        """psi_{beta,theta}[j], j < L.  spin index 0 is theta = -1: the spectrum
        is analytic along increasing lambda index.  spin index 1 (theta = +1) is
        its mirror j -> -j, eq. (1) with theta = +1 instead of -1."""
        h = ifft(self.psi_fr_hat[b])
        if spin == 0:
            return h
        return h[(-np.arange(self.L)) % self.L]

    def freq_wavelet_matrix(self, b, spin):
        """Z = W Y along lambda: W[l, i] = psi_{beta,theta}[(l 2^kfr - i) mod L],
        l < L/2^kfr, i < n1 (rows beyond n1 of the padded axis are zero)."""
        h = self.psi_fr(b, spin)
        l = np.arange(self.L_beta(b))[:, None] << self.k_fr[b]
        i = np.arange(self.n1)[None, :]
        return h[(l - i) % self.L]

    def freq_lowpass_matrix(self, b):
        """S2 = P V along lambda on the 2^kfr-decimated grid:
        P[m, l] = phi_F[(m F/2^kfr - l) mod L_beta], m < L/F."""
        Lb = self.L_beta(b)
        phi = ifft(gauss_lowpass_hat(Lb, self.L, self.F)).real
        step = self.F >> self.k_fr[b]
        m = np.arange(self.out_l)[:, None] * step
        l = np.arange(Lb)[None, :]
        return phi[(m - l) % Lb]


# ---------------------------------------------------------------------------
# Stages (each a plain definition) and their adjoints
# ---------------------------------------------------------------------------

def upsample(g, d, M):
    """Transpose of keeping every d-th sample: zeros between the samples."""
    out = np.zeros(g.shape[:-1] + (M,), dtype=np.result_type(g, np.float64))
    out[..., ::d] = g
    return out


def filt_decimate(a, h_hat, d):
    """(a (*) h)[n d], circular convolution on the grid of a, h given by its spectrum."""
    return np.ascontiguousarray(ifft(fft(a) * h_hat)[..., ::d])


def filt_decimate_adj(g, h_hat, d, M):
    """Adjoint of filt_decimate: correlate the zero-upsampled g with h."""
    return ifft(fft(upsample(g, d, M)) * np.conj(h_hat))


def first_order_linear(x, P):
    """Y1d[lambda, n] = (x (*) psi_lambda)[n 2^kX]: the filtered signal at the scalogram rate."""
    return filt_decimate(np.asarray(x, np.float64)[None, :], P.psi1_hat, 1 << P.kX)


def first_order_linear_adj(g, P):
    """Real-input adjoint: Re sum_lambda of each band's adjoint."""
    out = np.zeros(P.N)
    for lam in range(P.n1):
        out += filt_decimate_adj(g[lam], P.psi1_hat[lam], 1 << P.kX, P.N).real
    return out


def time_lowpass(rows, P, k):
    """(rows (*) phi_T)[tau T/2^k] for rows sampled at 1/2^k of the input rate."""
    M = rows.shape[-1]
    phi_hat = gauss_lowpass_hat(M, P.N, P.T)
    return filt_decimate(rows, phi_hat, P.T >> k).real


def time_lowpass_adj(g, P, k, M):
    phi_hat = gauss_lowpass_hat(M, P.N, P.T)
    return filt_decimate_adj(g, phi_hat, P.T >> k, M).real


def second_order_linear(X, P, a):
    """Y2[lambda, t] = (X_lambda (*) psi_alpha)[t 2^k2(alpha)]."""
    return filt_decimate(X, P.psi2_hat[a], 1 << P.k2[a])


def second_order_linear_adj(g, P, a):
    return filt_decimate_adj(g, P.psi2_hat[a], 1 << P.k2[a], P.NX).real


def modulus_adj(gu, z):
    return gu * z / np.maximum(np.abs(z), EPS_MOD)


def jtfs(x, P: Plan, return_intermediates=False, alphas=None, average_fr=True):
    """S1 [n1, N/T] and S2 [n_alpha, n_beta, 2, L/F, N/T] of one real signal x
    (eq. (3)); with ``average_fr=False`` the eq. (4) variant, S2 packed as
    P.s2_shape(False).

    ``alphas`` restricts the second order to those temporal-rate indices (the
    other S2 slices are returned as NaN); used to sample very large cases."""
    x = np.asarray(x, dtype=np.float64)
    if x.shape != (P.N,):
        raise ValueError("x must have shape (N,)")
    Y1d = first_order_linear(x, P)
    X = np.abs(Y1d)
    S1 = time_lowpass(X, P, P.kX)
    S2 = np.zeros(P.s2_shape(average_fr))
    inter = {"Y1d": Y1d, "X": X, "Y2": [], "Z": {}}
    todo = range(P.n_alpha) if alphas is None else sorted(set(alphas))
    if alphas is not None:
        S2[:] = np.nan
    for a in todo:
        Y2 = second_order_linear(X, P, a)
        if return_intermediates:
            inter["Y2"].append(Y2)
        for b in range(P.n_beta):
            Pm = P.freq_lowpass_matrix(b)
            for s in range(2):
                Z = P.freq_wavelet_matrix(b, s) @ Y2
                if return_intermediates:
                    inter["Z"][(a, b, s)] = Z
                V = time_lowpass(np.abs(Z), P, P.kX + P.k2[a])
                if average_fr:
                    S2[a, b, s] = Pm @ V
                else:
                    S2[a, P.s2_rows(b, s)] = V
    if return_intermediates:
        return S1, S2, inter
    return S1, S2


def jtfs_vjp(x, gS1, gS2, P: Plan, average_fr=True):
    """Gradient of sum(gS1*S1) + sum(gS2*S2) with respect to x, by the
    Hermitian adjoint of every stage applied in reverse order (gS2 laid out as
    P.s2_shape(average_fr)).  Temporal-rate indices whose S2 cotangent is
    identically zero contribute nothing and are skipped."""
    x = np.asarray(x, dtype=np.float64)
    gS1 = np.asarray(gS1, dtype=np.float64)
    gS2 = np.asarray(gS2, dtype=np.float64)
    Y1d = first_order_linear(x, P)
    X = np.abs(Y1d)
    gX = time_lowpass_adj(gS1, P, P.kX, P.NX)
    for a in range(P.n_alpha):
        if not np.any(gS2[a]):
            continue
        Y2 = second_order_linear(X, P, a)
        Ta = P.T_alpha(a)
        gY2 = np.zeros((P.n1, Ta), dtype=np.complex128)
        for b in range(P.n_beta):
            Pm = P.freq_lowpass_matrix(b)
            for s in range(2):
                W = P.freq_wavelet_matrix(b, s)
                Z = W @ Y2
                gV = Pm.T @ gS2[a, b, s] if average_fr else gS2[a, P.s2_rows(b, s)]
                gU = time_lowpass_adj(gV, P, P.kX + P.k2[a], Ta)
                gZ = modulus_adj(gU, Z)
                gY2 += W.conj().T @ gZ
        gX += second_order_linear_adj(gY2, P, a)
    gY1d = modulus_adj(gX, Y1d)
    return first_order_linear_adj(gY1d, P)


def zeroth_order(x, P: Plan):
    """S0[tau] = (x (*) phi_T)[tau T], tau < N/T."""
    return time_lowpass(np.asarray(x, np.float64)[None, :], P, 0)[0]


def zeroth_order_adj(g, P: Plan):
    """Gradient of sum(g * S0) with respect to x."""
    return time_lowpass_adj(np.asarray(g, np.float64)[None, :], P, 0, P.N)[0]


def loss(x, gS1, gS2, P, average_fr=True):
    S1, S2 = jtfs(x, P, average_fr=average_fr)
    return float(np.sum(gS1 * S1) + np.sum(gS2 * S2))


# ---------------------------------------------------------------------------
# Direct (FFT-free) cascade for small N: every convolution as its defining sum
# ---------------------------------------------------------------------------

def _circ_direct(a, h, d):
    """out[..., n] = sum_j a[..., j] h[(n d - j) mod M] for n < M/d."""
    M = a.shape[-1]
    n = np.arange(M // d)[:, None] * d
    j = np.arange(M)[None, :]
    C = h[(n - j) % M]                    # (M/d, M)
    return a @ C.T


def jtfs_direct(x, P: Plan, average_fr=True):
    """Same operator as jtfs() with every convolution evaluated as a direct sum
    and every filter brought to the time domain by the defining DFT sum."""
    x = np.asarray(x, dtype=np.float64)
    psi1 = dft_direct(P.psi1_hat, inverse=True)
    X = np.abs(np.stack([_circ_direct(x[None, :].astype(complex), psi1[l], 1 << P.kX)[0]
                         for l in range(P.n1)]))
    phiX = dft_direct(gauss_lowpass_hat(P.NX, P.N, P.T), inverse=True)
    S1 = _circ_direct(X.astype(complex), phiX, P.T >> P.kX).real
    S2 = np.zeros(P.s2_shape(average_fr))
    psi2 = dft_direct(P.psi2_hat, inverse=True)
    for a in range(P.n_alpha):
        Ta = P.T_alpha(a)
        Y2 = _circ_direct(X.astype(complex), psi2[a], 1 << P.k2[a])
        Yp = np.zeros((P.L, Ta), dtype=complex)
        Yp[: P.n1] = Y2
        phiU = dft_direct(gauss_lowpass_hat(Ta, P.N, P.T), inverse=True)
        for b in range(P.n_beta):
            Lb = P.L_beta(b)
            h0 = dft_direct(P.psi_fr_hat[b], inverse=True)
            phiF = dft_direct(gauss_lowpass_hat(Lb, P.L, P.F), inverse=True).real
            for s in range(2):
                h = h0 if s == 0 else h0[(-np.arange(P.L)) % P.L]
                Z = _circ_direct(Yp.T, h, 1 << P.k_fr[b]).T          # along lambda
                V = _circ_direct(np.abs(Z).astype(complex), phiU, P.T >> (P.kX + P.k2[a])).real
                if average_fr:
                    S2[a, b, s] = _circ_direct(V.T, phiF, P.F >> P.k_fr[b]).T[: P.out_l]
                else:
                    S2[a, P.s2_rows(b, s)] = V
    return S1, S2


# ---------------------------------------------------------------------------
# mu-log (sec. 4): mean-based renormalisation and pointwise logarithm
# ---------------------------------------------------------------------------

MULOG_EPS = 0.1   # the constant epsilon of the paper, the same for every path


def path_means(S1s, S2s, path_axes=2):
    """mu per path over a set of signals.  S1s [n, n1, N/T] is one path (the
    first order); S2s [n, n_alpha, n_beta, 2, L/F, N/T] has one path per
    (alpha, beta, theta).  mu is the mean over the signals and over (lambda, t):
    the integral over the time-frequency plane divided by its area.  The last
    ``path_axes`` axes of S2s span one path: 2 for JTFS, 1 for time scattering,
    whose S2s [n, n_alpha, n1, N/T] has one path per (alpha, lambda1) pair,
    averaged over its frames."""
    S1s = np.asarray(S1s, np.float64)
    S2s = np.asarray(S2s, np.float64)
    mu1 = np.float64(S1s.mean())
    mu2 = S2s.mean(axis=(0,) + tuple(range(S2s.ndim - path_axes, S2s.ndim)))
    return mu1, mu2


def _per_coeff(mu2, path_axes):
    mu2 = np.asarray(mu2, np.float64)
    return mu2.reshape(mu2.shape + (1,) * path_axes)


def mulog(S1, S2, mu1, mu2, eps=MULOG_EPS, path_axes=2):
    """log(1 + S / (eps mu(path))) for one or several signals."""
    S1 = np.asarray(S1, np.float64)
    S2 = np.asarray(S2, np.float64)
    return np.log1p(S1 / (eps * mu1)), np.log1p(S2 / (eps * _per_coeff(mu2, path_axes)))


def mulog_vjp(S1, S2, mu1, mu2, g1, g2, eps=MULOG_EPS, path_axes=2):
    """Adjoint of mulog in S with mu held fixed: g / (eps mu + S)."""
    S1 = np.asarray(S1, np.float64)
    S2 = np.asarray(S2, np.float64)
    return np.asarray(g1) / (eps * mu1 + S1), np.asarray(g2) / (eps * _per_coeff(mu2, path_axes) + S2)


# ---------------------------------------------------------------------------
# Texture resynthesis (sec. 5)
# ---------------------------------------------------------------------------

BOLD_UP = 1.2      # learning-rate factor after an accepted (error-decreasing) step
BOLD_DOWN = 0.5    # factor after a rejected step; the iterate is kept


def texture_target(x, P, average_fr=True):
    """Coefficients Sx of the target and their norm ||Sx|| (S1 and S2 together)."""
    S1, S2 = jtfs(x, P, average_fr=average_fr)
    return S1, S2, math.sqrt(float(np.sum(S1 ** 2) + np.sum(S2 ** 2)))


def texture_error_grad(y, target, P, average_fr=True):
    """E(y) = ||Sx - Sy|| / ||Sx|| and its gradient, the VJP of the cotangent
    (Sy - Sx) / (||Sy - Sx|| ||Sx||) (zero where Sy = Sx)."""
    Sx1, Sx2, nx = target
    S1, S2 = jtfs(y, P, average_fr=average_fr)
    r1, r2 = S1 - Sx1, S2 - Sx2
    nr = math.sqrt(float(np.sum(r1 ** 2) + np.sum(r2 ** 2)))
    if nr == 0.0:
        return 0.0, np.zeros(P.N)
    g = jtfs_vjp(y, r1 / (nr * nx), r2 / (nr * nx), P, average_fr=average_fr)
    return nr / nx, g


def texture_resynthesis(x, y0, P, iters, mu0, average_fr=True):
    """Bold-driver gradient descent from y0 towards the coefficients of x.

    The start is evaluated first; each of the ``iters`` iterations then
    evaluates one candidate y - mu grad E(y): if its error is lower it is
    accepted and mu grows by BOLD_UP, otherwise it is rejected and mu shrinks
    by BOLD_DOWN.  mu0 > 0 is the initial rate; mu0 < 0 sets it relative to the
    start, |mu0| ||y0|| / ||grad E(y0)||.  Returns the best iterate, the best
    error after the start and after every iteration, and the final rate."""
    target = texture_target(x, P, average_fr)
    y = np.asarray(y0, np.float64)
    E, g = texture_error_grad(y, target, P, average_fr)
    gn = float(np.linalg.norm(g))
    mu = mu0 if mu0 > 0 else (-mu0 * float(np.linalg.norm(y)) / gn if gn > 0 else 0.0)
    hist = [E]
    for _ in range(iters):
        yc = y - mu * g
        Ec, gc = texture_error_grad(yc, target, P, average_fr)
        if Ec < E:
            y, E, g = yc, Ec, gc
            mu *= BOLD_UP
        else:
            mu *= BOLD_DOWN
        hist.append(E)
    return y, np.array(hist), mu


# ---------------------------------------------------------------------------
# Time scattering (sec. 4): the temporal filterbank alone on the scalogram
# ---------------------------------------------------------------------------

def scattering1d(x, P: Plan):
    """S1 [n1, N/T] (as jtfs) and S2 [n_alpha, n1, N/T] with
    S2[alpha, lambda] = (|X_lambda (*) psi_alpha| (*) phi_T) on the N/T frames."""
    x = np.asarray(x, dtype=np.float64)
    X = np.abs(first_order_linear(x, P))
    S1 = time_lowpass(X, P, P.kX)
    S2 = np.stack([time_lowpass(np.abs(second_order_linear(X, P, a)), P, P.kX + P.k2[a])
                   for a in range(P.n_alpha)])
    return S1, S2


def scattering1d_vjp(x, gS1, gS2, P: Plan):
    """Gradient of sum(gS1*S1) + sum(gS2*S2) of scattering1d by the stage adjoints."""
    x = np.asarray(x, dtype=np.float64)
    Y1d = first_order_linear(x, P)
    X = np.abs(Y1d)
    gX = time_lowpass_adj(np.asarray(gS1, np.float64), P, P.kX, P.NX)
    for a in range(P.n_alpha):
        Y2 = second_order_linear(X, P, a)
        gU = time_lowpass_adj(np.asarray(gS2[a], np.float64), P, P.kX + P.k2[a], P.T_alpha(a))
        gX += second_order_linear_adj(modulus_adj(gU, Y2), P, a)
    return first_order_linear_adj(modulus_adj(gX, Y1d), P)


def scattering1d_direct(x, P: Plan):
    """scattering1d with every convolution as a direct sum (small N)."""
    x = np.asarray(x, dtype=np.float64)
    psi1 = dft_direct(P.psi1_hat, inverse=True)
    X = np.abs(np.stack([_circ_direct(x[None, :].astype(complex), psi1[l], 1 << P.kX)[0]
                         for l in range(P.n1)]))
    phiX = dft_direct(gauss_lowpass_hat(P.NX, P.N, P.T), inverse=True)
    S1 = _circ_direct(X.astype(complex), phiX, P.T >> P.kX).real
    psi2 = dft_direct(P.psi2_hat, inverse=True)
    S2 = []
    for a in range(P.n_alpha):
        U = np.abs(_circ_direct(X.astype(complex), psi2[a], 1 << P.k2[a]))
        phiU = dft_direct(gauss_lowpass_hat(P.T_alpha(a), P.N, P.T), inverse=True)
        S2.append(_circ_direct(U.astype(complex), phiU, P.T >> (P.kX + P.k2[a])).real)
    return S1, np.stack(S2)
