"""Host-side tests of the C ABI (no GPU): the library loads and exports every
function include/jtfs.h declares, the host FP64 plan solve reproduces the
oracle's filterbanks and schedules, and invalid parameters are rejected."""
import ctypes
import os
import re

import numpy as np
import pytest

import synth
from oracle import jtfs_oracle as O
from tests._util import oracle_plan

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "jtfs.h")


@pytest.fixture(scope="module")
def L():
    from paper_2204_08269_amd import _lib
    return _lib


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(jtfs_\w+)\s*\(", text)))


def test_library_exports_every_declared_symbol(L):
    lib = L.load()
    names = declared_functions()
    assert len(names) >= 10
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(L.EXPORTS)


def test_library_is_built_for_gfx950(L):
    data = open(L.LIB_PATH, "rb").read()
    assert b"gfx950" in data


@pytest.mark.parametrize("cfg", [1, 2, 3, 4, 5])
def test_host_plan_matches_oracle(L, cfg):
    p = synth.PARAMS[cfg]
    P = oracle_plan(p)
    prm = L.params(p["N"], p["J"], p["Q"], p["J_fr"], p["Q_fr"], p["T"], p["F"])
    info = L.query(prm)
    assert (info.n1, info.n_alpha, info.n_beta, info.L, info.kX) == (P.n1, P.n_alpha, P.n_beta, P.L, P.kX)
    assert info.NX == P.NX and info.out_t == P.out_t and info.out_l == P.out_l
    assert info.M_h == sum(P.L_beta(b) for b in range(P.n_beta))
    assert info.sum_T == sum(P.T_alpha(a) for a in range(P.n_alpha))
    assert info.s1_per_signal == int(np.prod(P.s1_shape()))
    assert info.s2_per_signal == int(np.prod(P.s2_shape()))
    info4 = L.query(L.params(p["N"], p["J"], p["Q"], p["J_fr"], p["Q_fr"], p["T"], p["F"], average_fr=False))
    assert info4.s2_per_signal == int(np.prod(P.s2_shape(False)))      # eq. (4) packing
    assert info4.s1_per_signal == info.s1_per_signal and info4.M_h == info.M_h
    infot = L.query(L.params(p["N"], p["J"], p["Q"], p["J_fr"], p["Q_fr"], p["T"], p["F"], time_scattering=True))
    assert infot.s2_per_signal == P.n_alpha * P.n1 * P.out_t            # time scattering
    for fam, (xi, sg, ks) in enumerate([(P.xi1, P.sigma1, [P.kX] * P.n1), (P.xi2, P.sigma2, P.k2),
                                        (P.xi_fr, P.sigma_fr, P.k_fr)]):
        hx, hs, hk = L.query_filters(prm, fam)
        assert np.allclose(hx, xi, rtol=1e-14, atol=0) and np.allclose(hs, sg, rtol=1e-14, atol=0)
        assert list(hk) == list(ks)


BAD = [
    dict(N=3000, J=6, Q=(8, 1), J_fr=3, Q_fr=1, T=64, F=4),      # N not a power of two
    dict(N=2048, J=6, Q=(8, 1), J_fr=3, Q_fr=1, T=4096, F=4),    # T > N
    dict(N=2048, J=6, Q=(0, 1), J_fr=3, Q_fr=1, T=64, F=4),      # Q1 = 0
    dict(N=2048, J=6, Q=(8, 1), J_fr=9, Q_fr=1, T=64, F=4),      # J_fr > log2 L
    dict(N=2048, J=6, Q=(8, 1), J_fr=3, Q_fr=1, T=64, F=128),    # F > L
    dict(N=2048, J=20, Q=(8, 1), J_fr=3, Q_fr=1, T=64, F=4),     # J > log2 N
    dict(N=8, J=2, Q=(1, 1), J_fr=1, Q_fr=1, T=2, F=1),          # N < 16
    dict(N=2048, J=6, Q=(8, 1), J_fr=3, Q_fr=1, T=48, F=4),      # T not a power of two
]


@pytest.mark.parametrize("p", BAD)
def test_invalid_parameters_rejected_before_any_hip_call(L, p):
    prm = L.params(p["N"], p["J"], p["Q"], p["J_fr"], p["Q_fr"], p["T"], p["F"])
    info = L.Info()
    rc = L.load().jtfs_query(ctypes.byref(prm), ctypes.byref(info))
    assert rc == L.JTFS_EINVAL
    assert L.load().jtfs_last_error().decode() != ""
    plan = ctypes.c_void_p()
    assert L.load().jtfs_plan_create_ex(ctypes.byref(plan), ctypes.byref(prm)) == L.JTFS_EINVAL
    assert not plan.value


def test_unknown_flag_bits_rejected(L):
    p = synth.PARAMS[1]
    prm = L.params(p["N"], p["J"], p["Q"], p["J_fr"], p["Q_fr"], p["T"], p["F"])
    info = L.Info()
    # an unknown bit; both variants at once; lowpass pairs or unpadding with time
    # scattering; unpadding without frequential averaging
    for bad in (16, 3, 2 | 4, 2 | 8, 1 | 8):
        prm.flags = bad
        assert L.load().jtfs_query(ctypes.byref(prm), ctypes.byref(info)) == L.JTFS_EINVAL
    assert ctypes.sizeof(L.Params) == 48


@pytest.mark.parametrize("cfg", [1, 2, 5])
def test_lowpass_pairs_and_unpadded_sizes(L, cfg):
    """Sizes with the lowpass pairs (one more rate and scale, phi_F's rows at the
    L/F grid) and with the unpadded lambda axis (ceil(n1 / F) rows), against the
    oracle's plan with the same options."""
    p = synth.PARAMS[cfg]
    P = O.Plan(p["N"], p["J"], p["Q"][0], p["Q"][1], p["J_fr"], p["Q_fr"], p["T"], p["F"],
               lowpass_pairs=True, unpad=True)
    i = L.query(L.params(p["N"], p["J"], p["Q"], p["J_fr"], p["Q_fr"], p["T"], p["F"], lowpass_pairs=True,
                         unpad_lambda=True))
    assert (i.n_alpha, i.n_beta, i.M_h, i.out_l, i.sum_T) == (P.n_alpha, P.n_beta, P.M_h, P.out_l,
                                                             sum(P.T_alpha(a) for a in range(P.n_alpha)))
    assert i.out_l == -(-P.n1 // p["F"])
    assert i.s2_per_signal == int(np.prod(P.s2_shape()))
    j = L.query(L.params(p["N"], p["J"], p["Q"], p["J_fr"], p["Q_fr"], p["T"], p["F"]))
    assert (i.n_alpha, i.n_beta) == (j.n_alpha + 1, j.n_beta + 1)
    assert 0 < j.ws_fwd < j.ws_bwd and i.ws_bwd > j.ws_bwd       # one more rate and scale: more workspace
    assert i.M_h == j.M_h + j.L // p["F"]           # phi_F kept at its critical rate: L / F rows


def test_null_pointers_rejected(L):
    lib = L.load()
    assert lib.jtfs_query(None, None) == L.JTFS_EINVAL
    assert lib.jtfs_plan_create_ex(None, None) == L.JTFS_EINVAL
    assert lib.jtfs_forward(None, None, 1, None, None, None, 0, None) == L.JTFS_EINVAL
    assert lib.jtfs_backward(None, None, None, None, None, 1, None, 0, 0, None) == L.JTFS_EINVAL
    assert lib.jtfs_workspace_size(None, 1, None) == L.JTFS_EINVAL
    lib.jtfs_plan_destroy(None)


def test_timing_api_host_side(L):
    lib = L.load()
    ms = ctypes.c_double(1.0)
    n = ctypes.c_int64(5)
    assert lib.jtfs_timing_read(99, ctypes.byref(ms), ctypes.byref(n)) == L.JTFS_EINVAL
    assert lib.jtfs_timing_read(0, ctypes.byref(ms), ctypes.byref(n)) == L.JTFS_OK
    assert ms.value == 0.0 and n.value == 0
    assert lib.jtfs_timing_enable(0) == L.JTFS_OK
