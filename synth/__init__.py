"""Seeded synthetic inputs for the JTFS workloads.

This module is shared by the FP64 oracle's tests and by the GPU path's tests and
benchmark. It holds signal synthesis only -- none of the scattering arithmetic.
Every signal is generated in float64 and rounded to float32; the oracle consumes
the rounded values promoted back to float64, so both sides see identical inputs.

Workloads (sizes follow the paper's use of the transform; the audio the paper
uses is not available, so these stand in for it):

* ``cfg1`` -- N=2^11, J=6, Q=(8,1), J_fr=3, Q_fr=1, T=2^6, F=2^2: three
  amplitude-modulated sinusoids plus white noise (small parity case).
* ``cfg2`` -- N=2^16 (the clip length of the instrument-classification data,
  sec. 4.2), J=12, Q=(16,1), J_fr=4, Q_fr=1, T=2^11, F=2^3: AM linear or
  exponential chirps from 0.005 to 0.45 cycles/sample at 20 dB SNR.
* ``cfg3`` -- N=2^17, J=13, Q=(12,1), J_fr=4, Q_fr=2, T=2^13, F=2^3: damped
  resonant click trains (texture resynthesis target, sec. 5) and a white-noise
  starting point at the target's RMS.
* ``cfg4`` -- 256 harmonic tones with ADSR envelopes and pink noise at 30 dB SNR,
  lengths log-uniform in [2^13, 2^16]; J=11, Q=(16,1), J_fr=4, Q_fr=1, T=2^10, F=2^3.
* ``cfg5`` -- N=2^18, J=14, Q=(24,2), J_fr=5, Q_fr=2, T=2^14, F=2^4: mixtures of
  four FM sources with AM plus white noise.
"""
from __future__ import annotations

import numpy as np

SEED_BASE = 220408269

# Plan parameters of each workload: (N, J, (Q1, Q2), J_fr, Q_fr, T, F).
PARAMS = {
    1: dict(N=2 ** 11, J=6, Q=(8, 1), J_fr=3, Q_fr=1, T=2 ** 6, F=2 ** 2),
    2: dict(N=2 ** 16, J=12, Q=(16, 1), J_fr=4, Q_fr=1, T=2 ** 11, F=2 ** 3),
    3: dict(N=2 ** 17, J=13, Q=(12, 1), J_fr=4, Q_fr=2, T=2 ** 13, F=2 ** 3),
    4: dict(N=2 ** 16, J=11, Q=(16, 1), J_fr=4, Q_fr=1, T=2 ** 10, F=2 ** 3),
    5: dict(N=2 ** 18, J=14, Q=(24, 2), J_fr=5, Q_fr=2, T=2 ** 14, F=2 ** 4),
}
BATCH = {1: 1, 2: 64, 3: 8, 4: 256, 5: 32}


def _rngs(cfg: int, count: int, offset: int = 0):
    """One independent generator per signal: SeedSequence(base+cfg).spawn(count)."""
    children = np.random.SeedSequence(SEED_BASE + cfg).spawn(offset + count)
    return [np.random.default_rng(c) for c in children[offset:]]


def _am(rng, n, lo, hi):
    r = rng.uniform(lo, hi)
    psi = rng.uniform(0.0, 2 * np.pi)
    return 0.5 * (1.0 + np.sin(2 * np.pi * r * n + psi))


def _to_f32(x):
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64).astype(np.float32))


def cfg1_signal(rng, N=2 ** 11):
    n = np.arange(N, dtype=np.float64)
    s = np.zeros(N)
    for _ in range(3):
        f = rng.uniform(0.01, 0.4)
        ph = rng.uniform(0.0, 2 * np.pi)
        s += _am(rng, n, 0.001, 0.01) * np.sin(2 * np.pi * f * n + ph)
    s += 0.05 * rng.standard_normal(N)
    return s


def chirp_signal(rng, N, f0=0.005, f1=0.45, kind=None, snr_db=20.0, am=True):
    """AM chirp from f0 to f1 cycles/sample over N samples plus white noise."""
    n = np.arange(N, dtype=np.float64)
    if kind is None:
        kind = "linear" if rng.uniform() < 0.5 else "exp"
    if kind == "linear":
        phase = 2 * np.pi * (f0 * n + (f1 - f0) * n ** 2 / (2 * N))
    elif kind == "exp":
        k = np.log(f1 / f0)
        phase = 2 * np.pi * f0 * N / k * (np.exp(k * n / N) - 1.0)
    else:
        raise ValueError(kind)
    s = np.sin(phase + rng.uniform(0.0, 2 * np.pi))
    if am:
        s = s * _am(rng, n, 1e-4, 1e-2)
    if snr_db is not None:
        var = np.mean(s ** 2) / 10 ** (snr_db / 10)
        s = s + np.sqrt(var) * rng.standard_normal(N)
    return s


def cfg2_signal(rng, N=2 ** 16):
    return chirp_signal(rng, N)


def click_train(rng, N=2 ** 17):
    """Poisson clicks, each circularly convolved with a damped resonance."""
    rate = rng.uniform(20, 200) / 2 ** 14          # clicks per sample
    count = max(1, rng.poisson(rate * N))
    y = np.zeros(N)
    n = np.arange(N, dtype=np.float64)
    for _ in range(count):
        pos = rng.integers(0, N)
        amp = rng.uniform(0.5, 1.0) * (1 if rng.uniform() < 0.5 else -1)
        tau = rng.uniform(50, 500)
        f0 = rng.uniform(0.02, 0.3)
        h = np.exp(-n / tau) * np.sin(2 * np.pi * f0 * n)
        y += amp * np.roll(h, pos)
    return y


def cfg3_pair(rng, N=2 ** 17):
    """(target y, white-noise start x0 at y's RMS)."""
    y = click_train(rng, N)
    x0 = rng.standard_normal(N) * np.sqrt(np.mean(y ** 2))
    return y, x0


def pink_noise(rng, N):
    w = rng.standard_normal(N)
    spec = np.fft.rfft(w)                  # shaping only: not part of the transform
    m = np.arange(spec.shape[0], dtype=np.float64)
    scale = np.zeros_like(m)
    scale[1:] = 1.0 / np.sqrt(m[1:])
    return np.fft.irfft(spec * scale, n=N)


def harmonic_tone(rng, length, snr_db=30.0):
    n = np.arange(length, dtype=np.float64)
    f0 = rng.uniform(0.002, 0.05)
    s = np.zeros(length)
    for k in range(1, 11):
        if k * f0 >= 0.5:
            break
        s += np.sin(2 * np.pi * k * f0 * n + rng.uniform(0, 2 * np.pi)) / k
    a, d, r, sus = 0.05, 0.10, 0.20, 0.6
    u = n / length
    env = np.where(u < a, u / a,
          np.where(u < a + d, 1.0 - (1.0 - sus) * (u - a) / d,
          np.where(u < 1.0 - r, sus, sus * (1.0 - u) / r)))
    s = s * env
    p = pink_noise(rng, length)
    p *= np.sqrt(np.mean(s ** 2) / 10 ** (snr_db / 10) / max(np.mean(p ** 2), 1e-300))
    return s + p


def cfg4_lengths(count=256):
    rng = np.random.default_rng(np.random.SeedSequence(SEED_BASE + 4 + 1000))
    return np.round(2.0 ** rng.uniform(13, 16, size=count)).astype(np.int64)


def fm_mixture(rng, N=2 ** 18):
    n = np.arange(N, dtype=np.float64)
    s = np.zeros(N)
    for _ in range(4):
        fc = rng.uniform(0.005, 0.3)
        fm = rng.uniform(1e-4, 5e-3)
        I = rng.uniform(0, 5)
        s += _am(rng, n, 1e-4, 1e-2) * np.sin(
            2 * np.pi * fc * n + I * np.sin(2 * np.pi * fm * n + rng.uniform(0, 2 * np.pi))
            + rng.uniform(0, 2 * np.pi))
    s += 0.02 * rng.standard_normal(N)
    return s


def batch(cfg: int, B: int | None = None, offset: int = 0, N: int | None = None):
    """float32 array [B, N] of workload ``cfg`` (cfg 3 returns the targets y).

    ``offset`` skips the first signals of the seeded sequence so that a bounded
    sample of a large batch can be regenerated exactly.  ``N`` overrides the
    length (used for small parity cases of the same signal family).
    """
    if B is None:
        B = BATCH[cfg]
    if N is None:
        N = PARAMS[cfg]["N"]
    rngs = _rngs(cfg, B, offset)
    if cfg == 1:
        xs = [cfg1_signal(r, N) for r in rngs]
    elif cfg == 2:
        xs = [cfg2_signal(r, N) for r in rngs]
    elif cfg == 3:
        xs = [cfg3_pair(r, N)[0] for r in rngs]
    elif cfg == 4:
        xs = [harmonic_tone(r, N) for r in rngs]
    elif cfg == 5:
        xs = [fm_mixture(r, N) for r in rngs]
    else:
        raise ValueError(cfg)
    return _to_f32(np.stack(xs))


def cfg3_batch(B: int = 8, N: int = 2 ** 17, offset: int = 0):
    """(targets y [B,N], starts x0 [B,N]) as float32."""
    pairs = [cfg3_pair(r, N) for r in _rngs(3, B, offset)]
    return _to_f32(np.stack([p[0] for p in pairs])), _to_f32(np.stack([p[1] for p in pairs]))


def cfg4_ragged(count: int = 256, offset: int = 0):
    """List of float32 signals with log-uniform lengths in [2^13, 2^16]."""
    lengths = cfg4_lengths(offset + count)[offset:]
    rngs = _rngs(4, count, offset)
    return [_to_f32(harmonic_tone(r, int(L))) for r, L in zip(rngs, lengths)]


def cotangents(shape_s1, shape_s2, seed: int = 7):
    """Seeded float32 cotangents (gS1, gS2) for VJP parity tests."""
    rng = np.random.default_rng(np.random.SeedSequence(SEED_BASE + 100 + seed))
    return _to_f32(rng.standard_normal(shape_s1)), _to_f32(rng.standard_normal(shape_s2))


def tone(N: int, m: int, amp: float = 1.0, phase: float = 0.0):
    """A*cos(2*pi*m*n/N + phase): a pure tone exactly on DFT bin m."""
    n = np.arange(N, dtype=np.float64)
    return amp * np.cos(2 * np.pi * m * n / N + phase)
