"""PyTorch-facing JTFS module: torch supplies device memory and the stream; the
transform and its gradient run in libjtfs's HIP kernels (see include/jtfs.h)."""
from __future__ import annotations

import ctypes

import torch

from . import _lib


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _mode_name(mode):
    return {v: k for k, v in _lib.CONTRACTIONS.items()}[mode]


class JTFS:
    """Joint time-frequency scattering of real signals x [B, N] (float32, on the GPU).

    S1 [B, n1, N/T] and S2 [B, n_alpha, n_beta, 2, L/F, N/T] (spin index 0 is
    theta = -1), eq. (3).  With average_fr=False, the eq. (4) variant without
    frequential averaging: S2 [B, n_alpha, 2 M_h, N/T], the (beta, theta) slices
    of L/2^kfr(beta) rows packed beta-major (s2_rows gives a slice's rows).
    With time_scattering=True, the time-scattering variant of sec. 4 instead (no
    frequential stage): S2 [B, n_alpha, n1, N/T].
    lowpass_pairs=True adds phi_T as the last temporal rate and phi_F as the last
    frequential scale (the pairs (psi_alpha, phi_F), (phi_T, psi_beta) and
    (phi_T, phi_F) of the joint filterbank); unpad_lambda=True keeps the
    ceil(n1 / F) log-frequency rows of S2 that fall on first-order bands (eq. (3)
    only).  zeroth_order(x) gives S0 = (x * phi_T)(tau T).
    contraction: "split16" (FP16 matrix cores with split operands, the default
    where available), "split16_phase" (split16, and the forward stores the unit
    phase of the contraction so that a vjp that reuses the forward's workspace
    need not recompute it; a larger workspace) or "fp32" (FP32 matrix cores).  Calling the object is
    differentiable through torch.autograd; forward() and vjp() call the library
    directly."""

    def __init__(self, N, J, Q, J_fr, Q_fr, T, F, contraction=None, average_fr=True, time_scattering=False,
                 lowpass_pairs=False, unpad_lambda=False):
        if not torch.cuda.is_available():
            raise RuntimeError("JTFS needs a ROCm GPU (no CPU fallback)")
        self.lib = _lib.load()
        self.average_fr = bool(average_fr)
        self.time_scattering = bool(time_scattering)
        self.lowpass_pairs = bool(lowpass_pairs)
        self.params = _lib.params(N, J, Q, J_fr, Q_fr, T, F, average_fr, time_scattering, lowpass_pairs,
                                  unpad_lambda)
        self.device = torch.device("cuda", torch.cuda.current_device())
        plan = ctypes.c_void_p()
        _lib.check(self.lib.jtfs_plan_create_ex(ctypes.byref(plan), ctypes.byref(self.params)))
        self.plan = plan
        info = _lib.Info()
        _lib.check(self.lib.jtfs_plan_info(self.plan, ctypes.byref(info)))
        self.info = info
        if contraction is not None:
            _lib.check(self.lib.jtfs_plan_set_contraction(self.plan, _lib.CONTRACTIONS[contraction]))
        m = ctypes.c_int(0)
        _lib.check(self.lib.jtfs_plan_get_contraction(self.plan, ctypes.byref(m)))
        self.contraction = _mode_name(m.value)
        self.N = int(N)
        self.s1_shape = (info.n1, info.out_t)
        if self.time_scattering:
            self.s2_shape = (info.n_alpha, info.n1, info.out_t)
        elif self.average_fr:
            self.s2_shape = (info.n_alpha, info.n_beta, 2, info.out_l, info.out_t)
        else:
            self.s2_shape = (info.n_alpha, 2 * info.M_h, info.out_t)
        self._ws = {}

    def s2_rows(self, beta, theta):
        """Rows of the (beta, theta) slice in the eq. (4) layout (average_fr=False)."""
        _, _, k = _lib.query_filters(self.params, 2)
        Lb = [self.info.L >> int(v) for v in k]
        if self.lowpass_pairs:
            Lb.append(self.info.M_h - sum(Lb))     # phi_F's rows
        o = 2 * sum(Lb[:beta]) + theta * Lb[beta]
        return slice(o, o + Lb[beta])

    def __del__(self):
        try:
            if getattr(self, "plan", None) is not None and self.plan.value:
                self.lib.jtfs_plan_destroy(self.plan)
                self.plan = None
        except Exception:
            pass

    def workspace_bytes(self, B: int) -> int:
        n = ctypes.c_size_t(0)
        _lib.check(self.lib.jtfs_workspace_size(self.plan, int(B), ctypes.byref(n)))
        return n.value

    def forward_workspace_bytes(self, B: int) -> int:
        n = ctypes.c_size_t(0)
        _lib.check(self.lib.jtfs_forward_workspace_size(self.plan, int(B), ctypes.byref(n)))
        return n.value

    def new_workspace(self, B: int) -> torch.Tensor:
        return torch.empty(self.workspace_bytes(B), dtype=torch.uint8, device=self.device)

    def _workspace(self, B):
        ws = self._ws.get(B)
        if ws is None:
            ws = self._ws[B] = self.new_workspace(B)
        return ws

    def _check_x(self, x):
        if x.dim() != 2 or x.shape[1] != self.N or x.dtype != torch.float32 or not x.is_cuda:
            raise ValueError(f"x must be a float32 CUDA tensor of shape [B, {self.N}]")
        return x.contiguous()

    def forward(self, x, ws=None):
        x = self._check_x(x)
        B = x.shape[0]
        ws = self._workspace(B) if ws is None else ws
        s1 = torch.empty((B,) + self.s1_shape, dtype=torch.float32, device=x.device)
        s2 = torch.empty((B,) + self.s2_shape, dtype=torch.float32, device=x.device)
        _lib.check(self.lib.jtfs_forward(self.plan, _ptr(x), B, _ptr(s1), _ptr(s2), _ptr(ws), ws.numel(), _stream()))
        return s1, s2

    def zeroth_order(self, x):
        """S0 [B, N/T] = (x * phi_T)(tau T)."""
        x = self._check_x(x)
        s0 = torch.empty((x.shape[0], self.info.out_t), dtype=torch.float32, device=x.device)
        _lib.check(self.lib.jtfs_zeroth_order(self.plan, _ptr(x), x.shape[0], _ptr(s0), _stream()))
        return s0

    def zeroth_order_vjp(self, gs0, gx=None):
        """Gradient of sum(gs0 * S0) with respect to x, added to gx (zeros if None)."""
        gs0 = gs0.contiguous().float()
        B = gs0.shape[0]
        if gx is None:
            gx = torch.zeros((B, self.N), dtype=torch.float32, device=gs0.device)
        _lib.check(self.lib.jtfs_zeroth_order_backward(self.plan, _ptr(gs0), B, _ptr(gx), _stream()))
        return gx

    def vjp(self, x, gs1, gs2, ws=None, reuse_forward=False):
        x = self._check_x(x)
        B = x.shape[0]
        ws = self._workspace(B) if ws is None else ws
        gs1 = gs1.contiguous().float() if gs1 is not None else None
        gs2 = gs2.contiguous().float() if gs2 is not None else None
        gx = torch.empty_like(x)
        flags = _lib.JTFS_BWD_REUSE_FORWARD if reuse_forward else 0
        _lib.check(self.lib.jtfs_backward(self.plan, _ptr(x), _ptr(gs1), _ptr(gs2), _ptr(gx), B, _ptr(ws),
                                          ws.numel(), flags, _stream()))
        return gx

    # launch choices --------------------------------------------------------
    REG_BITS = {"scalogram": 1, "second_order": 2, "row_fft": 4, "first_adj": 8}
    FWD_TILE16 = 16
    BWD_TILE16 = 32
    RADIX8_BITS = {"scalogram": 64, "second_order": 128, "row_fft": 256, "first_adj": 512}
    LDS_BATCH8K = 1024
    TCHUNK_BITS = {1024: 2048, 2048: 4096, 4096: 0}

    def autotune(self, B, x=None, reps=3):
        """Times the candidate launch choices for B signals (x: [B, N] on the
        GPU, or None for zeros), keeps the fastest and returns what was chosen."""
        t = _lib.Tuning()
        xp = _ptr(self._check_x(x)) if x is not None else None
        _lib.check(self.lib.jtfs_plan_autotune(self.plan, xp, int(B), int(reps), _stream(), ctypes.byref(t)))
        self.contraction = _mode_name(t.contraction)
        self._ws = {}                          # the workspace size may have changed with the mode
        return {"contraction": self.contraction,
                "register_rows": [k for k, v in self.REG_BITS.items() if t.reg_rows & v],
                "fwd_tile": 16 if t.reg_rows & self.FWD_TILE16 else 32,
                "bwd_tile": 16 if t.reg_rows & self.BWD_TILE16 else 32,
                "radix8": [k for k, v in self.RADIX8_BITS.items() if t.reg_rows & v],
                "lds_batch": 8192 if t.reg_rows & self.LDS_BATCH8K else 4096,
                "t_chunk": self._chunk_of(t.reg_rows),
                "step_ms": t.step_ms, "from_cache": bool(t.from_cache),
                "fwd_ms": {"tile32": t.fwd_ms[0], "tile16": t.fwd_ms[1]},
                "bwd_ms": {"tile32": t.bwd_ms[0], "tile16": t.bwd_ms[1]},
                "candidates_ms": {"split16_register": t.candidates_ms[0], "split16_lds": t.candidates_ms[1],
                                  "fp32_register": t.candidates_ms[2], "fp32_lds": t.candidates_ms[3],
                                  "split16_phase_register": t.candidates_ms[4],
                                  "split16_phase_lds": t.candidates_ms[5]}}

    def _chunk_of(self, mask):
        return 1024 if mask & self.TCHUNK_BITS[1024] else 2048 if mask & self.TCHUNK_BITS[2048] else 4096

    def set_tuning(self, contraction, register_rows, fwd_tile=32, bwd_tile=32, radix8=(), lds_batch=4096,
                   t_chunk=4096):
        """Launch choices: contraction mode; stages whose 2^14-point rows are
        register-resident; contraction tiles; stages whose register-resident
        transforms use radix-8 passes (else radix 16); points per workgroup of
        the in-LDS row transforms (4096 or 8192); t-columns per workgroup of the
        forward contraction (1024, 2048 or 4096; the workspace size follows)."""
        mode = _lib.CONTRACTIONS[contraction]
        if lds_batch not in (4096, 8192):
            raise ValueError("lds_batch must be 4096 or 8192")
        if t_chunk not in self.TCHUNK_BITS:
            raise ValueError("t_chunk must be 1024, 2048 or 4096")
        mask = (sum(self.REG_BITS[k] for k in register_rows) | (self.FWD_TILE16 if fwd_tile == 16 else 0) |
                (self.BWD_TILE16 if bwd_tile == 16 else 0) | sum(self.RADIX8_BITS[k] for k in radix8) |
                (self.LDS_BATCH8K if lds_batch == 8192 else 0) | self.TCHUNK_BITS[t_chunk])
        _lib.check(self.lib.jtfs_plan_set_tuning(self.plan, mode, mask))
        self.contraction = contraction
        self._ws = {}

    def tuning_radix(self):
        """(stages in radix-8 passes, points per in-LDS workgroup, forward t-chunk) now set on the plan."""
        m, r = ctypes.c_int(0), ctypes.c_int(0)
        _lib.check(self.lib.jtfs_plan_get_tuning(self.plan, ctypes.byref(m), ctypes.byref(r)))
        return ([k for k, v in self.RADIX8_BITS.items() if r.value & v],
                8192 if r.value & self.LDS_BATCH8K else 4096, self._chunk_of(r.value))

    def tuning(self):
        """(contraction, register rows, forward tile, backward tile) now set on the plan."""
        m, r = ctypes.c_int(0), ctypes.c_int(0)
        _lib.check(self.lib.jtfs_plan_get_tuning(self.plan, ctypes.byref(m), ctypes.byref(r)))
        return (_mode_name(m.value), [k for k, v in self.REG_BITS.items() if r.value & v],
                16 if r.value & self.FWD_TILE16 else 32, 16 if r.value & self.BWD_TILE16 else 32)

    # mu-log renormalisation (sec. 4) -------------------------------------
    def _check_s(self, s1, s2):
        B = s1.shape[0]
        if tuple(s1.shape) != (B,) + self.s1_shape or tuple(s2.shape) != (B,) + self.s2_shape:
            raise ValueError("S1 / S2 shapes do not match the plan")
        return s1.contiguous(), s2.contiguous(), B

    def path_means(self, s1, s2):
        """mu per path over the batch: (mu1 [1], mu2 [n_alpha * n_beta * 2]); with
        time scattering one path per (alpha, lambda1): mu2 [n_alpha * n1]."""
        s1, s2, B = self._check_s(s1, s2)
        i = self.info
        n2 = i.n_alpha * i.n1 if self.time_scattering else i.n_alpha * i.n_beta * 2
        mu1 = torch.empty(1, dtype=torch.float32, device=s1.device)
        mu2 = torch.empty(n2, dtype=torch.float32, device=s1.device)
        _lib.check(self.lib.jtfs_path_means(self.plan, _ptr(s1), _ptr(s2), B, _ptr(mu1), _ptr(mu2), _stream()))
        return mu1, mu2

    def mulog(self, s1, s2, mu1, mu2, eps=0.1):
        """log(1 + S / (eps mu)) per path."""
        s1, s2, B = self._check_s(s1, s2)
        o1, o2 = torch.empty_like(s1), torch.empty_like(s2)
        _lib.check(self.lib.jtfs_mulog(self.plan, _ptr(s1), _ptr(s2), B, _ptr(mu1.contiguous()),
                                       _ptr(mu2.contiguous()), float(eps), _ptr(o1), _ptr(o2), _stream()))
        return o1, o2

    def mulog_vjp(self, s1, s2, mu1, mu2, g1, g2, eps=0.1):
        """Adjoint of mulog with mu fixed: g / (eps mu + S)."""
        s1, s2, B = self._check_s(s1, s2)
        g1, g2 = g1.contiguous().float(), g2.contiguous().float()
        d1, d2 = torch.empty_like(s1), torch.empty_like(s2)
        _lib.check(self.lib.jtfs_mulog_backward(self.plan, _ptr(s1), _ptr(s2), B, _ptr(mu1.contiguous()),
                                                _ptr(mu2.contiguous()), float(eps), _ptr(g1), _ptr(g2), _ptr(d1),
                                                _ptr(d2), _stream()))
        return d1, d2

    def forward_mulog(self, x, mu1, mu2, eps=0.1, ws=None):
        """log(1 + S / (eps mu)) per path, computed by the transform's own output
        kernels (S is not stored): (O1, O2) in the shapes of forward()."""
        x = self._check_x(x)
        B = x.shape[0]
        ws = self._workspace(B) if ws is None else ws
        o1 = torch.empty((B,) + self.s1_shape, dtype=torch.float32, device=x.device)
        o2 = torch.empty((B,) + self.s2_shape, dtype=torch.float32, device=x.device)
        _lib.check(self.lib.jtfs_forward_mulog(self.plan, _ptr(x), B, _ptr(mu1.contiguous()),
                                               _ptr(mu2.contiguous()), float(eps), _ptr(o1), _ptr(o2), _ptr(ws),
                                               ws.numel(), _stream()))
        return o1, o2

    def vjp_mulog(self, x, o1, o2, mu1, mu2, go1, go2, eps=0.1, ws=None, reuse_forward=False):
        """Gradient of <go, O(x)> with mu fixed, O = forward_mulog(x) (o1, o2 its outputs)."""
        x = self._check_x(x)
        B = x.shape[0]
        ws = self._workspace(B) if ws is None else ws
        go1 = go1.contiguous().float() if go1 is not None else None
        go2 = go2.contiguous().float() if go2 is not None else None
        gx = torch.empty_like(x)
        flags = _lib.JTFS_BWD_REUSE_FORWARD if reuse_forward else 0
        _lib.check(self.lib.jtfs_backward_mulog(self.plan, _ptr(x), _ptr(o1.contiguous()), _ptr(o2.contiguous()),
                                                _ptr(mu1.contiguous()), _ptr(mu2.contiguous()), float(eps),
                                                _ptr(go1), _ptr(go2), _ptr(gx), B, _ptr(ws), ws.numel(), flags,
                                                _stream()))
        return gx

    def table(self, which: int):
        """Device filter table copied to the host (0: psi1 dense, 1: psi2 dense, 2: W spin -1)."""
        import numpy as np
        i = self.info
        if which == 0:
            a = np.zeros((i.n1, self.N // 2 + 1), np.float32)
        elif which == 1:
            a = np.zeros((i.n_alpha, i.NX // 2 + 1), np.float32)
        else:
            a = np.zeros((i.M_h, i.n1), np.complex64)
        _lib.check(self.lib.jtfs_plan_table(self.plan, which, a.ctypes.data_as(ctypes.c_void_p), a.nbytes))
        return a

    def __call__(self, x, mu=None, eps=0.1):
        """(S1, S2), differentiable; with mu = (mu1, mu2) the mu-log outputs
        log(1 + S / (eps mu)) instead, differentiable with mu held fixed.  A call
        that records a graph gets a workspace of its own (kept for its backward);
        one that does not (no_grad, or x without requires_grad) reuses the plan's."""
        if not (torch.is_grad_enabled() and x.requires_grad):
            # no graph to serve: the plan's cached workspace, nothing kept for a backward
            if mu is None:
                return self.forward(x)
            return self.forward_mulog(x, mu[0], mu[1], eps)
        if mu is None:
            return _JTFSFunction.apply(x, self)
        return _JTFSMuLogFunction.apply(x, self, mu[0], mu[1], float(eps))


class _JTFSFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, op: JTFS):
        x = op._check_x(x)
        ws = op.new_workspace(x.shape[0])          # holds the intermediates for backward
        s1, s2 = op.forward(x, ws)
        ctx.op = op
        ctx.ws = ws
        ctx.save_for_backward(x)
        return s1, s2

    @staticmethod
    def backward(ctx, gs1, gs2):
        (x,) = ctx.saved_tensors
        ws = ctx.ws
        ctx.ws = None
        gx = ctx.op.vjp(x, gs1, gs2, ws=ws, reuse_forward=True)
        return gx, None


class _JTFSMuLogFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, op: JTFS, mu1, mu2, eps):
        x = op._check_x(x)
        ws = op.new_workspace(x.shape[0])
        o1, o2 = op.forward_mulog(x, mu1, mu2, eps, ws)
        ctx.op, ctx.ws, ctx.eps = op, ws, eps
        ctx.save_for_backward(x, o1, o2, mu1, mu2)
        return o1, o2

    @staticmethod
    def backward(ctx, go1, go2):
        x, o1, o2, mu1, mu2 = ctx.saved_tensors
        ws = ctx.ws
        ctx.ws = None
        gx = ctx.op.vjp_mulog(x, o1, o2, mu1, mu2, go1, go2, ctx.eps, ws=ws, reuse_forward=True)
        return gx, None, None, None, None


class JTFSBucket:
    """Ragged batch: signals of lengths `lengths` (zero-padded to powers of two,
    one plan per padded length), run as one recorded HIP graph.

    run(x_packed, g_packed=None) takes the signals back to back (float32, CUDA)
    and returns the packed coefficients (and the packed gradient with respect to
    the input samples when a packed cotangent is given).  Must be called on a
    non-default stream (graph capture)."""

    def __init__(self, lengths, J, Q, J_fr, Q_fr, T, F, autotune=False):
        """(autotune: tune each bucket's plan for its batch at creation.)"""
        if not torch.cuda.is_available():
            raise RuntimeError("JTFSBucket needs a ROCm GPU (no CPU fallback)")
        self.lib = _lib.load()
        self.lengths = [int(v) for v in lengths]
        n = len(self.lengths)
        arr = (ctypes.c_int64 * n)(*self.lengths)
        self.params = _lib.params(16, J, Q, J_fr, Q_fr, T, F)
        if autotune:
            self.params.flags |= _lib.JTFS_BUCKET_AUTOTUNE
        h = ctypes.c_void_p()
        _lib.check(self.lib.jtfs_bucket_create(ctypes.byref(h), arr, n, ctypes.byref(self.params)))
        self.h = h
        xo = (ctypes.c_int64 * (n + 1))()
        so = (ctypes.c_int64 * (n + 1))()
        _lib.check(self.lib.jtfs_bucket_offsets(self.h, xo, so))
        self.x_offset = list(xo)
        self.s_offset = list(so)
        self.pads = []
        for L in self.lengths:
            N = 16
            while N < L:
                N *= 2
            self.pads.append(N)

    def __del__(self):
        try:
            if getattr(self, "h", None) is not None and self.h.value:
                self.lib.jtfs_bucket_destroy(self.h)
                self.h = None
        except Exception:
            pass

    def run(self, x_packed, g_packed=None, out=None, gx_out=None):
        dev = x_packed.device
        s = out if out is not None else torch.empty(self.s_offset[-1], dtype=torch.float32, device=dev)
        gx = None
        if g_packed is not None:
            gx = gx_out if gx_out is not None else torch.zeros(self.x_offset[-1], dtype=torch.float32, device=dev)
        _lib.check(self.lib.jtfs_bucket_run(self.h, _ptr(x_packed), _ptr(s), _ptr(g_packed), _ptr(gx), _stream()))
        return s, gx


class Texture:
    """Texture resynthesis (sec. 5) of B signals with the plan of ``op``: bold-driver
    gradient descent on ||Sx - Sy|| / ||Sx||, every step on the GPU.  mu0 > 0 is
    the initial rate, mu0 < 0 a rate relative to the start (|mu0| ||y0|| / ||grad||)."""

    def __init__(self, op: JTFS, B: int, mu0: float = -0.05):
        self.op = op
        self.B = int(B)
        t = ctypes.c_void_p()
        _lib.check(op.lib.jtfs_texture_create(ctypes.byref(t), op.plan, self.B, float(mu0)))
        self.tex = t
        # iterations are replayed from a captured graph, which needs a stream of its own
        self.stream = torch.cuda.Stream(device=op.device)

    def _run(self, fn):
        cur = torch.cuda.current_stream(self.op.device)
        self.stream.wait_stream(cur)
        with torch.cuda.stream(self.stream):
            _lib.check(fn(ctypes.c_void_p(self.stream.cuda_stream)))
        cur.wait_stream(self.stream)

    def __del__(self):
        t = getattr(self, "tex", None)
        if t is not None and t.value:
            self.op.lib.jtfs_texture_destroy(t)
            self.tex = None

    def set_target(self, x):
        x = self.op._check_x(x)
        if x.shape[0] != self.B:
            raise ValueError(f"x must hold {self.B} signals")
        self._x = x                       # kept alive until the stream has used it
        self._run(lambda st: self.op.lib.jtfs_texture_set_target(self.tex, _ptr(x), st))

    def set_start(self, y0):
        y0 = self.op._check_x(y0)
        if y0.shape[0] != self.B:
            raise ValueError(f"y0 must hold {self.B} signals")
        self._y0 = y0
        self._run(lambda st: self.op.lib.jtfs_texture_set_start(self.tex, _ptr(y0), st))

    def iterate(self, iters: int, record: bool = True):
        """Runs ``iters`` iterations; returns the best error after each [iters, B] (if record)."""
        hist = torch.empty((max(int(iters), 1), self.B), dtype=torch.float32, device=self.op.device) if record else None
        cap = hist.shape[0] if record else 0
        self._run(lambda st: self.op.lib.jtfs_texture_iterate(self.tex, int(iters), _ptr(hist), cap, st))
        return hist[:iters] if record else None

    def read(self):
        """(best iterate [B, N], its error [B], current rate [B])."""
        y = torch.empty((self.B, self.op.N), dtype=torch.float32, device=self.op.device)
        e = torch.empty(self.B, dtype=torch.float32, device=self.op.device)
        m = torch.empty(self.B, dtype=torch.float32, device=self.op.device)
        self._run(lambda st: self.op.lib.jtfs_texture_read(self.tex, _ptr(y), _ptr(e), _ptr(m), st))
        return y, e, m
