/*
 * jtfs.h -- C ABI of libjtfs: joint time-frequency scattering (JTFS) and its
 * gradient on AMD Instinct MI355X (gfx950).
 *
 * Operator (arxiv 2204.08269, sec. 2): for a real signal x of N samples,
 *   first order   X(t,lambda) = |x * psi_lambda|(t)                 (scalogram)
 *                 S1 = X *_t phi_T                                   (sec. 4.2: no phi_F)
 *   second order  S2 = | X *_{t,lambda} Psi_{alpha,beta,theta} | *_{t,lambda} Phi_{T,F}   (eq. 3)
 *                 Psi_{alpha,beta,theta}(t,lambda) = psi_alpha(t) psi_{beta,theta}(lambda) (eq. 2)
 *                 psi_alpha(t) = 2^alpha psi(2^alpha t), psi_{beta,theta}(lambda) = 2^beta psi(theta 2^beta lambda) (eq. 1)
 * and the vector-Jacobian product of (S1, S2) with respect to x, formed by the
 * Hermitian adjoints of the stages in reverse order (sec. 5).
 *
 * Discretisation (the paper gives continuous equations only):
 *   - circular convolutions on power-of-two grids, Morlet wavelets defined by
 *     their spectra (analytic: zero on negative frequencies, zero at DC), Gaussian
 *     lowpasses of width 0.1/T and 0.1/F, neighbouring wavelets crossing at -3 dB
 *     (quality factor about 2.5 at Q = 1, sec. 3.3);
 *   - every band is computed at a critical rate set by its bandwidth (sec. 1);
 *   - the log-frequency axis (n1 first-order bands) is zero-padded to the next
 *     power of two L; its index 0 is the highest frequency;
 *   - spin index 0 is theta = -1 (positive slope: an upward chirp lands there),
 *     spin index 1 is theta = +1 (sec. 2, Fig. 1).
 *
 * Layouts (row-major, contiguous float32):
 *   x   [B][N]
 *   S1  [B][n1][N/T]
 *   S2  [B][n_alpha][n_beta][2][L/F][N/T]       (the paper's out_3D mode, sec. 4.2)
 *   gx  [B][N]
 *
 * Memory and streams: x, S1, S2, gS1, gS2, gx and the workspace are device
 * pointers owned by the caller.  The plan owns its filter tables (device memory
 * allocated at creation, freed by jtfs_plan_destroy).  All work is enqueued on the
 * given stream with no host synchronisation; a plan may be used from several
 * threads and streams at once as long as each call has its own workspace.
 *
 * Errors: functions return JTFS_OK (0) or a negative status; jtfs_last_error()
 * returns a thread-local description of the last failure.  Argument validation
 * happens before any HIP call.
 */
#ifndef JTFS_H
#define JTFS_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define JTFS_OK          0
#define JTFS_EINVAL     -1   /* invalid parameter, shape or null pointer          */
#define JTFS_ENOMEM     -2   /* device allocation of plan tables failed            */
#define JTFS_EHIP       -3   /* a HIP runtime call or kernel launch failed         */
#define JTFS_EWORKSPACE -4   /* workspace smaller than jtfs_workspace_size()       */
#define JTFS_ESHAPE     -5   /* a batch count outside [1, 65535], or a buffer size
                                that does not match the plan's shapes              */
#define JTFS_ENOTSUP    -6   /* valid parameters outside what this library supports */

/* Flags of jtfs_backward. */
#define JTFS_BWD_REUSE_FORWARD 1u  /* ws holds the intermediates of the immediately
                                      preceding jtfs_forward on the same x, B and plan:
                                      skip recomputing the first and second order */

typedef struct jtfs_plan jtfs_plan;

/* Transform parameters (sec. 2, sec. 4.2): N samples; J octaves of the temporal
 * filterbanks; Q1 / Q2 wavelets per octave at first / second order; J_fr octaves
 * and Q_fr wavelets per octave of the frequential filterbank; lowpass supports T
 * (time, samples) and F (log-frequency, bins).  N, T, F are powers of two with
 * 16 <= N <= 2^24, T <= N, F <= L.  flags: 0 or an OR of JTFS_NO_FREQ_AVERAGE,
 * JTFS_TIME_SCATTERING, JTFS_LOWPASS_PAIRS and JTFS_UNPAD_LAMBDA (unknown bits, or
 * combinations excluded below, give JTFS_EINVAL). */
typedef struct {
    int64_t N;
    int32_t J, Q1, Q2, J_fr, Q_fr;
    uint32_t flags;
    int64_t T, F;
} jtfs_params;

/* The variant of eq. (4): no frequential lowpass phi_F, so S2 keeps the lambda
 * grid of each frequential wavelet (L / 2^kfr(beta) rows, kfr capped by log2 F)
 * and stays equivariant to frequency transposition.  S2 layout then packs the
 * ragged (beta, theta) slices: [B][n_alpha][2 M_h][N/T] with beta outer, theta
 * inner: the slice (beta, theta) occupies rows 2 r(beta) + theta L_beta ..
 * + L_beta - 1, r(beta) = sum of L_beta' over beta' < beta.  S1 is unchanged. */
#define JTFS_NO_FREQ_AVERAGE 1u

/* Time scattering (sec. 4, the Scattering1D comparison): the temporal wavelets
 * alone applied to the scalogram, no frequential stage:
 *   S2[b][alpha][lambda1][tau] = (|X_lambda1 * psi_alpha| * phi_T)(tau T)
 * for every (alpha, lambda1) pair, layout [B][n_alpha][n1][N/T]; S1 unchanged.
 * Not combinable with JTFS_NO_FREQ_AVERAGE. */
#define JTFS_TIME_SCATTERING 2u

/* The lowpass pairs of the joint filterbank (the completion of the cited joint
 * time-frequency scattering, sec. 2): each axis gains its lowpass as one more
 * filter, so that
 *   alpha = n_alpha - 1 is phi_T (its second-order row is X *_t phi_T at N/T
 *     frames, i.e. the S1 rows, real), and
 *   beta = n_beta - 1 is phi_F (real and even along lambda, decimation
 *     log2 F as for the wavelets' critical rate),
 * and eq. (3) (or eq. (4)) runs over all (alpha, beta, theta): the slices
 * (psi_alpha, phi_F), (phi_T, psi_beta, theta) and (phi_T, phi_F) are
 * | X * Psi | * Phi_{T,F} with the lowpass in place of the wavelet.  Both spin
 * slots of a pair with a lowpass hold equal values (a real filter, or a real
 * input along lambda).  n_alpha and n_beta of jtfs_info count the lowpasses.
 * Not combinable with JTFS_TIME_SCATTERING. */
#define JTFS_LOWPASS_PAIRS 4u

/* Unpadded log-frequency output of eq. (3) (the out_3D input of sec. 4.2):
 * S2 keeps the rows m < ceil(n1 / F) whose log-frequency m F falls on a
 * first-order band, out_l = ceil(n1 / F) instead of L / F; the rows dropped are
 * the ones centred in the zero padding of the lambda axis.  Not combinable with
 * JTFS_NO_FREQ_AVERAGE or JTFS_TIME_SCATTERING. */
#define JTFS_UNPAD_LAMBDA 8u

/* Derived sizes. */
typedef struct {
    int32_t n1;        /* first-order wavelets (lambda rows of the scalogram)      */
    int32_t n_alpha;   /* second-order temporal wavelets (+ phi_T with JTFS_LOWPASS_PAIRS) */
    int32_t n_beta;    /* frequential wavelets, each with two spins (+ phi_F likewise)  */
    int32_t L;         /* zero-padded log-frequency length, next power of two >= n1 */
    int32_t kX;        /* scalogram decimation: X has N / 2^kX samples per row       */
    int32_t M_h;       /* frequential output rows per spin: sum_beta L / 2^kfr(beta) */
    int64_t NX;        /* N / 2^kX                                                   */
    int64_t out_t;     /* N / T frames                                               */
    int64_t out_l;     /* L / F log-frequency rows of S2 (ceil(n1 / F) unpadded)     */
    int64_t sum_T;     /* sum over alpha of the second-order lengths NX / 2^k2(alpha) */
    int64_t s1_per_signal;   /* n1 * out_t                                          */
    int64_t s2_per_signal;   /* n_alpha * n_beta * 2 * out_l * out_t; with
                                JTFS_NO_FREQ_AVERAGE n_alpha * 2 * M_h * out_t; with
                                JTFS_TIME_SCATTERING n_alpha * n1 * out_t            */
    int64_t ws_fwd;    /* workspace bytes of a forward of one signal (B = 1)        */
    int64_t ws_bwd;    /* ... of a forward and backward (jtfs_workspace_size at B = 1);
                          jtfs_query: the split contraction without the stored phase,
                          with the FP32 backward's buffers (an upper bound for the modes
                          without it); jtfs_plan_info: the plan's contraction mode now */
} jtfs_info;

/* Host-only queries (no GPU needed). */

/* Validate p and fill the derived sizes. */
int jtfs_query(const jtfs_params* p, jtfs_info* out);

/* Filter tables of one family, host FP64: family 0 = first-order temporal
 * (cycles/sample), 1 = second-order temporal (cycles per scalogram sample),
 * 2 = frequential (cycles per lambda bin).  xi and sigma are the centre and
 * Gaussian width of each wavelet; log2_decim is its critical decimation
 * exponent (family 0: kX for every row).  Arrays hold `cap` entries; the count
 * is returned through *count (a count above cap gives JTFS_EINVAL). */
int jtfs_query_filters(const jtfs_params* p, int family, int32_t cap,
                       double* xi, double* sigma, int32_t* log2_decim, int32_t* count);

/* Plan creation builds every filter table on the device in FP64 (spectra,
 * Littlewood-Paley normalisation, lambda-domain wavelet matrices, lowpass
 * matrices) and stores them as FP32.  Q = {Q1, Q2}. */
int jtfs_plan_create(jtfs_plan** out, int64_t N, int J, const int Q[2], int J_fr, int Q_fr,
                     int64_t T, int64_t F);
int jtfs_plan_create_ex(jtfs_plan** out, const jtfs_params* p);
int jtfs_plan_info(const jtfs_plan* plan, jtfs_info* out);
void jtfs_plan_destroy(jtfs_plan* plan);

/* Device bytes of workspace needed by jtfs_forward and jtfs_backward for a
 * batch of B signals (the same workspace serves both; the backward reuses the
 * forward's intermediates when called with JTFS_BWD_REUSE_FORWARD). */
int jtfs_workspace_size(const jtfs_plan* plan, int64_t B, size_t* bytes);
/* The leading part of that workspace which a forward alone uses (the forward's
 * intermediates; the backward's buffers follow it). */
int jtfs_forward_workspace_size(const jtfs_plan* plan, int64_t B, size_t* bytes);

/* S1 and S2 of B signals (layouts above).  ws: device workspace of ws_bytes, at
 * least jtfs_forward_workspace_size (its leading part; a backward that reuses
 * this forward's workspace needs the whole jtfs_workspace_size). */
int jtfs_forward(const jtfs_plan* plan, const float* x, int64_t B, float* s1, float* s2,
                 void* ws, size_t ws_bytes, hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation): jtfs_forward with its
 * workspace taken from a fixed array of JTFS_NOALLOC_SCRATCH_BYTES bytes that the
 * library keeps on every GPU it runs on until the process ends (256 MiB; e.g. up
 * to 128 signals of 2^11 samples or 1 signal of 2^16 samples with the
 * 64 x 2^16 chirp parameters).  x, s1, s2: caller-owned device buffers, layouts
 * of jtfs_forward.  The current device must be the plan's.  Calls no allocating
 * routine and records no stage events.  Every call on one GPU uses the same
 * array and leaves its last contents there (the transform writes every scratch
 * value it reads, so nothing needs clearing); calls that overlap on one GPU
 * (concurrent streams or threads) race on it and must be serialised by the
 * caller.  Errors: JTFS_EWORKSPACE if the plan's forward workspace for B
 * signals (jtfs_forward_workspace_size) exceeds the array, else those of
 * jtfs_forward. */
#define JTFS_NOALLOC_SCRATCH_BYTES (256ull << 20)
int jtfs_forward_noalloc(const jtfs_plan* plan, const float* x, int64_t B, float* s1, float* s2,
                         hipStream_t stream);

/* gx = d<gS1,S1(x)> + <gS2,S2(x)> / dx for B signals.  gx is overwritten.
 * Either of gs1 / gs2 may be NULL (a zero cotangent). */
int jtfs_backward(const jtfs_plan* plan, const float* x, const float* gs1, const float* gs2,
                  float* gx, int64_t B, void* ws, size_t ws_bytes, uint32_t flags,
                  hipStream_t stream);

/* Arithmetic of the frequential contraction (both accumulate in FP32 on MFMA):
 *   JTFS_CONTRACTION_FP32      FP32 operands on the FP32 matrix cores;
 *   JTFS_CONTRACTION_SPLIT_F16 each FP32 operand v (times a power of two) is split
 *                              as v = hi + lo with hi, lo FP16, and the product
 *                              formed as hi*hi + hi*lo + lo*hi on the FP16 matrix
 *                              cores (22-bit operand precision; products exact).
 *   JTFS_CONTRACTION_SPLIT_F16_PHASE  SPLIT_F16, and the forward also stores the
 *                              unit phase z / max(|z|, eps) of every contraction
 *                              output z (both spins; real and imaginary part each
 *                              as a snorm16, round(32767 x), so an absolute error
 *                              of at most 0.5 / 32767 = 1.5e-5) in the workspace,
 *                              so that a backward with JTFS_BWD_REUSE_FORWARD applies
 *                              the modulus adjoint (sec. 5) from it instead of
 *                              recomputing the contraction.  The gradient then
 *                              carries a relative error of order 1e-5 (the
 *                              recomputing modes: order 1e-6).  The workspace grows
 *                              by 8 * B * M_p * sum_alpha T_p(alpha) bytes (M_p: M_h
 *                              rounded up to 64; T_p: T_alpha rounded up to 128);
 *                              jtfs_workspace_size accounts for it.  A backward
 *                              without JTFS_BWD_REUSE_FORWARD recomputes as SPLIT_F16
 *                              where that backward holds the shapes, else it takes
 *                              the phase again with the forward contraction.
 * The default is SPLIT_F16 where the shapes allow it (n1 <= 304 and N/T <= 64),
 * else FP32.  The SPLIT_F16 backward holds n1 <= 192 (160 at N/T = 64); beyond
 * that a SPLIT_F16 plan differentiates with the FP32 kernels.  SPLIT_F16_PHASE
 * holds every shape of the split forward.
 * Returns JTFS_ENOTSUP if the requested mode is not available for the plan
 * (and SPLIT_F16_PHASE not with JTFS_TIME_SCATTERING, which has no
 * contraction). */
#define JTFS_CONTRACTION_FP32            0
#define JTFS_CONTRACTION_SPLIT_F16       1
#define JTFS_CONTRACTION_SPLIT_F16_PHASE 2
int jtfs_plan_set_contraction(jtfs_plan* plan, int mode);
int jtfs_plan_get_contraction(const jtfs_plan* plan, int* mode);

/* Copy a device filter table of the plan to host memory, for inspection in
 * tests.  which: 0 = first-order spectra as a dense [n1][N/2+1] FP32 array,
 * 1 = second-order spectra dense [n_alpha][NX/2+1], 2 = frequential wavelet
 * matrix, spin theta = -1, as interleaved complex FP32 [M_h][n1].
 * bytes must equal the table's size.  Synchronous. */
int jtfs_plan_table(const jtfs_plan* plan, int which, void* host_dst, size_t bytes);

/* Ragged batches (many signals of uneven lengths).  Each signal of length L_i
 * (16 <= L_i <= 2^24) is zero-padded to the next power of two N_i; the signals of
 * one padded length form a bucket with its own plan (the parameters p with N = N_i)
 * and workspace, owned by the bucket object.  Runs with a gradient use the
 * JTFS_CONTRACTION_SPLIT_F16_PHASE contraction where every bucket's plan allows it
 * and the larger workspaces fit in 80 % of the device memory free at creation
 * (else, and for forward-only runs, each plan's own contraction).
 *
 * Packed layouts (float32, device):
 *   x_packed  the signals back to back, signal i at x_offset[i], L_i samples;
 *   s_packed  per signal i at s_offset[i]: S1 [n1][N_i/T] then S2
 *             [n_alpha][n_beta][2][L/F][N_i/T] (layouts of jtfs_forward);
 *   g_packed  a cotangent in the layout of s_packed;
 *   gx_packed the gradient with respect to the L_i input samples, layout of x_packed.
 * jtfs_bucket_offsets fills x_offset[count+1] and s_offset[count+1] (the last
 * entries are the totals).
 *
 * jtfs_bucket_run computes S (and gx when g_packed and gx_packed are non-NULL).
 * The first call for a given (pointer set, stream) records all buckets' work as
 * one HIP graph (pack, forward, backward, unpack), each bucket on a branch of its
 * own (forked from and joined back to the stream, so that the buckets may run
 * concurrently); later calls with the same pointers replay it with a single
 * graph launch.  Not thread-safe per object.
 * With JTFS_BUCKET_AUTOTUNE in p->flags (jtfs_bucket_create only; the other bits
 * go to every bucket's plan), each bucket's plan is autotuned at creation for its
 * batch (jtfs_plan_autotune on zeros, on the null stream: seconds for large
 * buckets); the launch choices are kept and the contraction of each run is
 * chosen as without the flag. */
#define JTFS_BUCKET_AUTOTUNE 0x100u
typedef struct jtfs_bucket jtfs_bucket;
int jtfs_bucket_create(jtfs_bucket** out, const int64_t* lengths, int count, const jtfs_params* p);
int jtfs_bucket_offsets(const jtfs_bucket* bk, int64_t* x_offset, int64_t* s_offset);
int jtfs_bucket_run(jtfs_bucket* bk, const float* x_packed, float* s_packed, const float* g_packed,
                    float* gx_packed, hipStream_t stream);
void jtfs_bucket_destroy(jtfs_bucket* bk);

/* mu-log renormalisation (sec. 4, the input transform of the convnet): a path
 * is S1 as a whole or one (alpha, beta, theta) slice of S2 (either layout).
 * jtfs_path_means writes mu = the mean of each path over the B signals and over
 * (lambda, t): mu1 [1] for S1 and mu2 [n_alpha * n_beta * 2] (theta fastest),
 * device FP32, accumulated in FP64.  For a time-scattering plan a second-order
 * path is one (alpha, lambda1) row of S2 [n_alpha][n1][N/T], mu2 [n_alpha * n1]
 * (lambda1 fastest) its mean over the signals and frames.  jtfs_mulog writes log(1 + S / (eps mu)) for
 * every coefficient (o1, o2 may alias s1, s2); jtfs_mulog_backward writes
 * gS = g / (eps mu + S), the adjoint with mu held fixed (mu estimated beforehand
 * over a training set).  eps > 0 (the paper uses 0.1).  All pointers are device
 * memory in the layouts of jtfs_forward; 1 <= B <= 65535.  Stream-ordered. */
int jtfs_path_means(const jtfs_plan* plan, const float* s1, const float* s2, int64_t B, float* mu1, float* mu2,
                    hipStream_t stream);
int jtfs_mulog(const jtfs_plan* plan, const float* s1, const float* s2, int64_t B, const float* mu1,
               const float* mu2, float eps, float* o1, float* o2, hipStream_t stream);
int jtfs_mulog_backward(const jtfs_plan* plan, const float* s1, const float* s2, int64_t B, const float* mu1,
                        const float* mu2, float eps, const float* g1, const float* g2, float* gs1, float* gs2,
                        hipStream_t stream);

/* The filterbanks and the critical-rate schedule of a plan, host FP64 (sec. 2, eq. (1);
 * sec. 1 for the rates), for checks against an independent implementation:
 *   xi_sigma [2 (n1 + na + nb)]: (centre, width) of each wavelet, the first-order
 *     family (cycles per sample), then the second-order one (cycles per scalogram
 *     sample), then the frequential one (cycles per lambda bin);
 *   schedule [1 + na + nb]: kX, then k2 of each second-order wavelet, then kfr of
 *     each frequential wavelet (log2 decimations);
 * na, nb count the wavelets only (n_alpha, n_beta of jtfs_info less the lowpasses
 * that JTFS_LOWPASS_PAIRS adds).  Host pointers owned by the caller; either may be
 * NULL.  No GPU work. */
int jtfs_plan_tables(const jtfs_plan* plan, double* xi_sigma, int32_t* schedule);

/* Zeroth order: S0[b][tau] = (x * phi_T)(tau T), tau < N/T, the lowpass of the
 * signal itself that completes S1 and S2 (sec. 2's cited transform; with the
 * discretisation above: circular, phi_T the Gaussian lowpass of width 0.1/T, DC
 * gain 1).  x [B][N] and s0 [B][N/T] are device FP32; any plan (flags ignored).
 * jtfs_zeroth_order_backward ADDS the gradient of sum(gs0 * S0) to gx [B][N]
 * (so that it composes with jtfs_backward, which overwrites gx).  1 <= B <= 65535;
 * stream-ordered; no workspace. */
int jtfs_zeroth_order(const jtfs_plan* plan, const float* x, int64_t B, float* s0, hipStream_t stream);
int jtfs_zeroth_order_backward(const jtfs_plan* plan, const float* gs0, int64_t B, float* gx, hipStream_t stream);

/* The transform with the mu-log of sec. 4 (eqs. (9)-(10)) fused into its last
 * stage: o1, o2 (the layouts of s1, s2 in jtfs_forward) receive
 * log(1 + S / (eps mu)) per path, written by the kernels that produce S, so S
 * itself never reaches memory.  mu1, mu2 are device FP32 in the layouts of
 * jtfs_path_means (a statistic taken beforehand, e.g. over a training set);
 * eps > 0.  Workspace, stream and errors as for jtfs_forward.
 * jtfs_backward_mulog is the gradient with mu held fixed: go1, go2 are the
 * cotangents of o1, o2 (either may be null: zero), o1, o2 the outputs that
 * jtfs_forward_mulog wrote for the same x (needed where the matching cotangent
 * is given); the cotangent of S is go / (eps mu e^o), applied as the lowpass
 * adjoints read it.  flags and the rest as for jtfs_backward
 * (JTFS_BWD_REUSE_FORWARD after jtfs_forward_mulog on the same workspace). */
int jtfs_forward_mulog(const jtfs_plan* plan, const float* x, int64_t B, const float* mu1, const float* mu2,
                       float eps, float* o1, float* o2, void* ws, size_t ws_bytes, hipStream_t stream);
int jtfs_backward_mulog(const jtfs_plan* plan, const float* x, const float* o1, const float* o2, const float* mu1,
                        const float* mu2, float eps, const float* go1, const float* go2, float* gx, int64_t B,
                        void* ws, size_t ws_bytes, uint32_t flags, hipStream_t stream);

/* Texture resynthesis (sec. 5): from a start y0, gradient descent on the
 * normalised error E(y) = ||Sx - Sy|| / ||Sx|| (S1 and S2 of the plan's layout
 * together) towards the coefficients of a target x, for B independent signals,
 * with the bold-driver rate: each iteration evaluates the candidate
 * y - mu grad E(y) (one forward and one backward); a lower error accepts it and
 * multiplies mu by 1.2, otherwise it is rejected and mu is halved.
 *   create: the texture keeps `plan` (which must outlive it) and allocates its
 *     own device state (workspace, coefficients, iterates: about
 *     B * (workspace + 4 N + 6 coefficients) floats).  mu0 > 0 is the initial
 *     rate; mu0 < 0 sets it per signal to |mu0| ||y0|| / ||grad E(y0)||.
 *   set_target: x [B][N] device; computes and keeps Sx and ||Sx||.
 *   set_start: y0 [B][N] device; evaluates it (error and gradient).
 *   iterate: `iters` iterations, replayed from one captured HIP graph (the
 *     stream must not be the legacy null stream).  hist (device, optional):
 *     hist[i][b] = best error of signal b after iteration i of this call, for
 *     i < hist_cap.
 *   read: best iterate y [B][N], its error err [B] and the current rate mu [B]
 *     (device pointers, each optional).
 * All calls are stream-ordered.  Errors: JTFS_EINVAL (null pointers, B outside
 * [1, 65535], mu0 zero or not finite, calls out of order), JTFS_ENOMEM, JTFS_EHIP. */
typedef struct jtfs_texture jtfs_texture;
int jtfs_texture_create(jtfs_texture** out, const jtfs_plan* plan, int64_t B, float mu0);
int jtfs_texture_set_target(jtfs_texture* tex, const float* x, hipStream_t stream);
int jtfs_texture_set_start(jtfs_texture* tex, const float* y0, hipStream_t stream);
int jtfs_texture_iterate(jtfs_texture* tex, int iters, float* hist, int hist_cap, hipStream_t stream);
int jtfs_texture_read(const jtfs_texture* tex, float* y, float* err, float* mu, hipStream_t stream);
void jtfs_texture_destroy(jtfs_texture* tex);

/* Launch choices and their autotuning.  reg_rows is a bit mask over the four
 * stages that have both a register-resident and an in-LDS transform for rows of
 * 2^14 points (longer rows always use the register-resident one, shorter rows the
 * in-LDS one), plus JTFS_TUNE_FWD_TILE16 (the tile of the split forward
 * contraction).  jtfs_plan_autotune runs, for B signals x (device, [B][N]; NULL:
 * zeros), one untimed and `reps` timed fwd+bwd steps per candidate: each
 * available contraction mode, once with all four stages register-resident and
 * 32 x 32 contraction tiles and once with all four in LDS and 16 x 16 tiles in
 * the forward and the stored-phase backward (where these choices exist).  It
 * keeps the contraction whose own stages took least time (each contraction
 * kernel with its faster tile), per stage the faster transform, and the faster
 * tiles, then times the result (step_ms).  With the
 * environment variable JTFS_TUNE_CACHE naming a file, a result is appended to it
 * under a key of the device's architecture and name, the plan parameters and B,
 * and a later call with the same key applies the stored choice without timing
 * (from_cache = 1; candidates and fwd_ms then 0).  It
 * allocates its buffers itself (the largest workspace over the modes plus
 * coefficients and gradient for B signals), synchronises the stream, uses the
 * per-stage timers (JTFS_EINVAL if timing is enabled) and leaves their records
 * cleared.  SPLIT_F16_PHASE is a candidate only where its workspace fits in 80 %
 * of the device memory free at the call (the timed steps reuse the forward, so
 * where it is chosen, a backward that does not reuse its forward runs as
 * SPLIT_F16; a caller that wants the recomputing backward's gradient precision
 * sets the mode with jtfs_plan_set_tuning instead).  candidates_ms: fwd+bwd per step of
 * (split, first run), (split, second run), (FP32, first), (FP32, second), (split with
 * stored phase, first), (split with stored phase, second); 0 for candidates not run.
 * fwd_ms, bwd_ms: the chosen mode's forward contraction and backward contraction
 * per step with 32 x 32 and 16 x 16 tiles (0 where not run).  Then, for the chosen
 * mode and tiles, one run with every register-resident stage in radix-8 passes
 * (where rows of 2^14 points or more exist), one with 8192-point in-LDS
 * workgroups (where rows of 2^12 points or fewer exist) and one with 1024-column
 * t-chunks in the forward contraction (where a rate has more than 1024 columns)
 * settle those bits per stage (a stage must gain 1 % to take the other setting). */
#define JTFS_REG_SCALOGRAM    1
#define JTFS_REG_SECOND_ORDER 2
#define JTFS_REG_ROW_FFT      4
#define JTFS_REG_FIRST_ADJ    8
/* In the same mask: the split forward contraction in 16 x 16 MFMA tiles (each
 * wave 64 rows l x 16 columns t; available where N/T <= 32), else 32 x 32 tiles. */
#define JTFS_TUNE_FWD_TILE16  16
/* ... and the stored-phase backward in 16 x 16 tiles (each wave 16 columns t and
 * all rows i, one pass for any K; N/T <= 32), else 32 x 32 tiles. */
#define JTFS_TUNE_BWD_TILE16  32
/* ... the largest radix of the register-resident row transforms' passes, per
 * stage: radix 8 where the bit is set, else radix 16 (every pass of a 2^14-point
 * transform held as 16 values per thread). */
#define JTFS_TUNE_RADIX8_SCALOGRAM    64
#define JTFS_TUNE_RADIX8_SECOND_ORDER 128
#define JTFS_TUNE_RADIX8_ROW_FFT      256
#define JTFS_TUNE_RADIX8_FIRST_ADJ    512
/* ... and 8192 points per workgroup in the in-LDS second-order and gY2 row
 * transforms (rows shorter than 2^13: more rows per workgroup, fewer
 * workgroups of twice the LDS), else 4096. */
#define JTFS_TUNE_LDS_BATCH8K 1024
/* ... and the t-columns per workgroup of the forward contraction (its t-chunk):
 * 1024 or 2048 where one of these bits is set (1024 if both), else 4096.  Shorter
 * chunks give more workgroups to small batches and more partial V slots to sum;
 * the workspace size follows the choice (query it again after setting it).
 * Changing it rewrites two small device tables of the plan: not while work of
 * the plan is in flight. */
#define JTFS_TUNE_TCHUNK_1K   2048
#define JTFS_TUNE_TCHUNK_2K   4096
typedef struct {
    int32_t contraction;
    int32_t reg_rows;                 /* including JTFS_TUNE_FWD_TILE16 */
    double step_ms;
    double candidates_ms[6];
    double fwd_ms[2];
    double bwd_ms[2];
    int32_t from_cache;
} jtfs_tuning;
int jtfs_plan_autotune(jtfs_plan* plan, const float* x, int64_t B, int reps, hipStream_t stream, jtfs_tuning* out);
int jtfs_plan_set_tuning(jtfs_plan* plan, int contraction, int reg_rows);
int jtfs_plan_get_tuning(const jtfs_plan* plan, int* contraction, int* reg_rows);

/* Per-stage kernel timing (tracing).  While enabled, every launch of each stage
 * below is bracketed by a pair of HIP events recorded on the launch's stream.
 * jtfs_timing_read waits for the recorded events of one stage, returns their
 * summed duration in milliseconds and the number of launches, and clears that
 * stage.  Process-wide; thread-safe.  Disabled by default (no events recorded). */
#define JTFS_STAGE_INPUT_FFT      0  /* real FFT of x                                    */
#define JTFS_STAGE_SCALOGRAM      1  /* first order: fold, iFFT, modulus, real FFT of X   */
#define JTFS_STAGE_S1             2  /* time lowpass of the scalogram -> S1               */
#define JTFS_STAGE_SECOND_ORDER   3  /* second-order temporal wavelets -> Y2              */
#define JTFS_STAGE_OPERAND_SPLIT  4  /* Y2 -> scaled FP16 halves (split contraction only) */
#define JTFS_STAGE_FREQ_FWD       5  /* frequential contraction + modulus + time lowpass  */
#define JTFS_STAGE_FREQ_LOWPASS   6  /* frequency lowpass -> S2                           */
#define JTFS_STAGE_LOWPASS_ADJ    7  /* adjoint of the frequency lowpass                  */
#define JTFS_STAGE_FREQ_ADJ_PQ    8  /* contraction recompute, lowpass and modulus adj.
                                        (split mode: also the W^H product)                */
#define JTFS_STAGE_FREQ_ADJ_WH    9  /* adjoint of the contraction (W^H), FP32 mode       */
#define JTFS_STAGE_SECOND_ADJ_FFT 10 /* forward FFT of the gY2 rows                       */
#define JTFS_STAGE_SECOND_ADJ     11 /* second-order and S1 adjoints -> gX                */
#define JTFS_STAGE_FIRST_ADJ      12 /* modulus adjoint and FFT of each first-order row   */
#define JTFS_STAGE_BAND_ACCUM     13 /* band-limited accumulation over lambda1 -> gx_hat  */
#define JTFS_STAGE_OUTPUT_FFT     14 /* inverse real FFT to gx                            */
#define JTFS_NUM_STAGES           15
int jtfs_timing_enable(int on);
int jtfs_timing_read(int stage, double* ms, int64_t* launches);

/* Thread-local text of the last error ("" if none). */
const char* jtfs_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* JTFS_H */
