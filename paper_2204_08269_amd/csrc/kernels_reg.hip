// First- and second-order kernels for long rows (2^14 and 2^15 points) built on
// the register-resident FFT: 32 values per thread, LDS used only as a float
// exchange buffer of one row (64 KB at 2^14 -> two workgroups per CU; 128 KB at
// 2^15, which an in-LDS complex transform could not hold).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "plan.hpp"
#include "reg_fft.hpp"
#include "regk.hpp"

namespace jtfs {

constexpr int kRegE = 16;                            // values per thread
constexpr int kRegT = (1 << kRegMinLog) / kRegE;     // threads per row transform of 2^14 points

// fold of src * ps over the band [lo, hi] onto M = 2^logM bins, at bin p
__device__ __forceinline__ float2 fold_at(const float2* __restrict__ src, const float* __restrict__ ps, int lo, int hi,
                                          int logM, int p) {
    const int M = 1 << logM;
    float2 acc = make_float2(0.f, 0.f);
    for (int m = lo + ((p - lo) & (M - 1)); m <= hi; m += M) {
        const float2 v = src[m];
        const float g = ps[m - lo];
        acc.x += v.x * g;
        acc.y += v.y * g;
    }
    return acc;
}

// The thread's inputs of a register transform of 2^logM points (input layout
// of reg_fft), folded from src * ps over [lo, hi].  When the band fits the row
// every bin receives at most one band sample, and the loads go out four
// elements at a time with no loop between them.
template <int LOGM, int LRM = reg_lr_max(kRegE), int EE = kRegE>
__device__ __forceinline__ void fold_inputs(float2 (&v)[EE], const float2* __restrict__ src,
                                            const float* __restrict__ ps, int lo, int hi) {
    constexpr int M = 1 << LOGM;
    if (hi - lo < M) {
#pragma unroll
        for (int e0 = 0; e0 < EE; e0 += 4) {
            float g[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int p = reg_input_pos<LOGM, EE, LRM>(e0 + q);
                const int m = lo + ((p - lo) & (M - 1));
                const bool ok = m <= hi;
                v[e0 + q] = ok ? src[m] : make_float2(0.f, 0.f);
                g[q] = ok ? ps[m - lo] : 0.f;
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) v[e0 + q] = cscale(v[e0 + q], g[q]);
        }
        return;
    }
#pragma unroll
    for (int e = 0; e < EE; ++e) v[e] = fold_at(src, ps, lo, hi, LOGM, reg_input_pos<LOGM, EE, LRM>(e));
}

// Rows of 2^15 points run as two 2^14-point register transforms:
//  inverse (decimation in frequency):  y[2k] = IDFT_m(u[p] + u[p+m])[k],
//                                      y[2k+1] = IDFT_m((u[p] - u[p+m]) e^{+2 pi i p/n})[k];
//  forward (decimation in time):       G[k] = E[k] + e^{-2 pi i k/n} O[k], G[k+m] = E[k] - e^{-2 pi i k/n} O[k],
//                                      E, O the m-point DFTs of the even and odd samples (m = n/2).

// Inputs of one sub-transform of the inverse split (decimation in frequency),
// staged through LDS (real parts in A, imaginary parts in B, m = n/2 floats
// each) and loaded in the register transform's input layout.  half 0:
// u[p] + u[p+m]; half 1: (u[p] - u[p+m]) e^{+2 pi i p/n}.  Without the split
// (TWO false) each thread folds u at its own input positions; no LDS is used.
// (KU: positions whose loads a thread issues together in the batched fold.)
template <bool TWO, int KU = 4, int LRM = reg_lr_max(kRegE)>
__device__ __forceinline__ void load_dif(float2 (&v)[kRegE], float* A, float* B, const float2* __restrict__ src,
                                         const float* __restrict__ ps, int lo, int hi, int logn, int half,
                                         const float2* __restrict__ tw, int tw_log, bool zero) {
    if constexpr (!TWO) {
        // no staging: each thread folds its own inputs
        if (zero) {
#pragma unroll
            for (int e = 0; e < kRegE; ++e) v[e] = make_float2(0.f, 0.f);
        } else {
            fold_inputs<kRegMinLog, LRM>(v, src, ps, lo, hi);
        }
        return;
    }
    const int logS = logn - 1;
    const int m = 1 << logS;
    const int n = 1 << logn;
    __syncthreads();                                   // A, B free (2^logn floats)
    if (zero) {
        for (int p = threadIdx.x; p < m; p += blockDim.x) { A[p] = 0.f; B[p] = 0.f; }
    } else if (hi - lo < 2 * n) {
        // every bin of the row receives at most two band samples: a thread requests
        // all samples (and twiddles) of KU positions before forming any of them,
        // instead of waiting for each position's loads in turn
        for (int p0 = threadIdx.x; p0 < m; p0 += KU * (int)blockDim.x) {
            float2 sa[KU][2], sc[KU][2], w[KU];
            float ga[KU][2], gc[KU][2];
#pragma unroll
            for (int u = 0; u < KU; ++u) {
                const int p = p0 + u * (int)blockDim.x;
                const int ma = lo + ((p - lo) & (n - 1)), mc = lo + ((p + m - lo) & (n - 1));
#pragma unroll
                for (int k = 0; k < 2; ++k) {
                    const bool oka = p < m && ma + k * n <= hi, okc = p < m && mc + k * n <= hi;
                    sa[u][k] = oka ? src[ma + k * n] : make_float2(0.f, 0.f);
                    ga[u][k] = oka ? ps[ma + k * n - lo] : 0.f;
                    sc[u][k] = okc ? src[mc + k * n] : make_float2(0.f, 0.f);
                    gc[u][k] = okc ? ps[mc + k * n - lo] : 0.f;
                }
                w[u] = half == 1 && p < m ? twiddle(tw, p << (tw_log - logn), true) : make_float2(1.f, 0.f);
            }
#pragma unroll
            for (int u = 0; u < KU; ++u) {
                const int p = p0 + u * (int)blockDim.x;
                if (p >= m) continue;
                const float2 a = cadd(cscale(sa[u][0], ga[u][0]), cscale(sa[u][1], ga[u][1]));
                const float2 c = cadd(cscale(sc[u][0], gc[u][0]), cscale(sc[u][1], gc[u][1]));
                const float2 q = half == 0 ? cadd(a, c) : cmul(csub(a, c), w[u]);
                A[p] = q.x;
                B[p] = q.y;
            }
        }
    } else {
        for (int p = threadIdx.x; p < m; p += blockDim.x) {
            const float2 a = fold_at(src, ps, lo, hi, logn, p);
            const float2 c = fold_at(src, ps, lo, hi, logn, p + m);
            const float2 q = half == 0 ? cadd(a, c) : cmul(csub(a, c), twiddle(tw, p << (tw_log - logn), true));
            A[p] = q.x;
            B[p] = q.y;
        }
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < kRegE; ++e) {
        const int q = reg_input_pos<kRegMinLog, kRegE, LRM>(e);
        v[e] = make_float2(A[q], B[q]);
    }
}

// scalogram row -> X_hat (same computation as the in-LDS scalogram kernel)
template <bool TWO, int LRM>
__global__ void __launch_bounds__(kRegT) k_scalogram_r(const float2* __restrict__ xh, int64_t xh_pitch,
                                                     const float* __restrict__ psi1, const int* __restrict__ band1,
                                                     const int64_t* __restrict__ off1, float2* __restrict__ Xh,
                                                     int64_t Xh_pitch, int logNX, float invN,
                                                     const float2* __restrict__ tw, int tw_log) {
    extern __shared__ __align__(16) float xbuf[];          // NX floats (TWO: A = first NX/2, B = second NX/2)
    const int lam = blockIdx.x, n1 = gridDim.x;
    const int64_t b = blockIdx.y;
    const int NX = 1 << logNX, H = NX >> 1, logH = logNX - 1;
    const int logS = TWO ? logNX - 1 : logNX;
    float* A = xbuf;
    float* Bf = xbuf + (1 << logS);
    const float2* src = xh + b * xh_pitch;
    const float* ps = psi1 + off1[lam];
    const int lo = band1[2 * lam], hi = band1[2 * lam + 1];
    float2 v[kRegE];
    float even[TWO ? kRegE : 1];
    if constexpr (TWO) {
        load_dif<true, 4, LRM>(v, A, Bf, src, ps, lo, hi, logNX, 0, tw, tw_log, false);
        reg_fft<kRegE, kRegMinLog, LRM>(v, A, tw, tw_log, true);
#pragma unroll
        for (int e = 0; e < kRegE; ++e) even[e] = __builtin_amdgcn_sqrtf(v[e].x * v[e].x + v[e].y * v[e].y) * invN;   // X[2 pos]
        load_dif<true, 4, LRM>(v, A, Bf, src, ps, lo, hi, logNX, 1, tw, tw_log, false);
        reg_fft<kRegE, kRegMinLog, LRM>(v, A, tw, tw_log, true);
        __syncthreads();
#pragma unroll
        for (int e = 0; e < kRegE; ++e) {
            const int pos = reg_output_pos<kRegMinLog, kRegE, LRM>(e);
            xbuf[pos] = even[e];                                              // X[2 pos]
            xbuf[H + pos] = __builtin_amdgcn_sqrtf(v[e].x * v[e].x + v[e].y * v[e].y) * invN; // X[2 pos + 1]
        }
    } else {
        // the whole row fits one register transform; the exchange buffer is NX floats
        __syncthreads();
        fold_inputs<kRegMinLog, LRM>(v, src, ps, lo, hi);
        reg_fft<kRegE, kRegMinLog, LRM>(v, xbuf, tw, tw_log, true);
        __syncthreads();
#pragma unroll
        for (int e = 0; e < kRegE; ++e) {
            const int pos = reg_output_pos<kRegMinLog, kRegE, LRM>(e);
            xbuf[(pos & 1) * H + (pos >> 1)] = __builtin_amdgcn_sqrtf(v[e].x * v[e].x + v[e].y * v[e].y) * invN;
        }
    }
    __syncthreads();
    // real FFT of X through the complex FFT of z[k] = X[2k] + i X[2k+1] (H points)
    constexpr int EZ = TWO ? kRegE : kRegE / 2;
    constexpr int LH = TWO ? kRegMinLog : kRegMinLog - 1;      // log2 H
    float2 z[EZ];
#pragma unroll
    for (int e = 0; e < EZ; ++e) {
        const int k = reg_input_pos<LH, EZ>(e);
        z[e] = make_float2(xbuf[k], xbuf[H + k]);
    }
    reg_fft<EZ, LH>(z, xbuf, tw, tw_log, false);
    __syncthreads();
    float2* Z = (float2*)xbuf;               // H complex values = NX floats
#pragma unroll
    for (int e = 0; e < EZ; ++e) Z[reg_output_pos<LH, EZ>(e)] = z[e];
    __syncthreads();
    float2* out = Xh + (b * n1 + lam) * Xh_pitch;
    const int tws = tw_log - logNX;
    for (int m = threadIdx.x; m <= H / 2; m += blockDim.x) {
        if (m == 0) {
            const float2 q = Z[0];
            out[0] = make_float2(q.x + q.y, 0.f);
            out[H] = make_float2(q.x - q.y, 0.f);
            continue;
        }
        const float2 a = Z[m], c = Z[H - m];
        auto spec = [&](float2 p, float2 q, int k) {
            const float2 E = make_float2(0.5f * (p.x + q.x), 0.5f * (p.y - q.y));
            const float2 D = make_float2(p.x - q.x, p.y + q.y);
            const float2 O = make_float2(0.5f * D.y, -0.5f * D.x);
            return cadd(E, cmul(O, tw[k << tws]));
        };
        out[m] = spec(a, c, m);
        if (H - m != m) out[H - m] = spec(c, a, H - m);
    }
}

// one second-order row (T_alpha = 2^logTa >= 2^14): fold, inverse FFT, store, row max
template <bool TWO, int LRM>
__global__ void __launch_bounds__(kRegT) k_second_order_r(const float2* __restrict__ Xh, int64_t Xh_pitch, int n1,
                                                        const float* __restrict__ ps, int lo, int hi, int logTa,
                                                        int Tp, int Kp, float2* __restrict__ Y, int64_t y_bstride,
                                                        float invNX, const float2* __restrict__ tw, int tw_log,
                                                        float* __restrict__ rowmax, int alpha, int n_alpha) {
    extern __shared__ __align__(16) float xbuf[];
    __shared__ unsigned int rmx;
    const int lam = blockIdx.x;
    const int64_t b = blockIdx.y;
    const int logS = TWO ? logTa - 1 : logTa;
    float* A = xbuf;
    float* Bf = xbuf + (1 << logS);
    float2* out = Y + b * y_bstride + (int64_t)lam * Tp;
    if (lam >= n1) {
        // padding row: zeros (the contraction reads them), maximum 0
        for (int t = threadIdx.x; t < Tp; t += blockDim.x) out[t] = make_float2(0.f, 0.f);
        if (threadIdx.x == 0) rowmax[(b * n_alpha + alpha) * Kp + lam] = 0.f;
        return;
    }
    if (threadIdx.x == 0) rmx = 0u;
    const float2* row = Xh + (b * n1 + (lam < n1 ? lam : 0)) * Xh_pitch;
    float m = 0.f;
    float2 v[kRegE];
    // with two halves, the even outputs y[2 pos] stay in registers until the odd
    // ones y[2 pos + 1] are known, and each pair goes out as one 16-byte store
    float2 ev[TWO ? kRegE : 1];
#pragma unroll
    for (int half = 0; half < (TWO ? 2 : 1); ++half) {
        load_dif<TWO, 4, LRM>(v, A, Bf, row, ps, lo, hi, logTa, half, tw, tw_log, lam >= n1);
        reg_fft<kRegE, kRegMinLog, LRM>(v, A, tw, tw_log, true);
#pragma unroll
        for (int e = 0; e < kRegE; ++e) {
            const float2 y = cscale(v[e], invNX);
            const int pos = reg_output_pos<kRegMinLog, kRegE, LRM>(e);
            if constexpr (TWO) {
                if (half == 0) ev[e] = y;
                else *(float4*)(out + 2 * pos) = make_float4(ev[e].x, ev[e].y, y.x, y.y);
            } else {
                out[pos] = y;
            }
            m = fmaxf(m, fmaxf(fabsf(y.x), fabsf(y.y)));
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
    __syncthreads();
    if ((threadIdx.x & 63) == 0) atomicMax(&rmx, __float_as_uint(m));
    __syncthreads();
    if (threadIdx.x == 0) rowmax[(b * n_alpha + alpha) * Kp + lam] = __uint_as_float(rmx);
}

// in-place forward FFT of rows of 2^logn points (row r of batch b at base + b*bs + r*rs)
template <bool TWO, int LRM>
__global__ void __launch_bounds__(kRegT) k_rowfft_r(float2* __restrict__ base, int64_t bs, int64_t rs, int logn,
                                                  const float2* __restrict__ tw, int tw_log) {
    extern __shared__ __align__(16) float xbuf[];
    float2* row = base + (int64_t)blockIdx.y * bs + (int64_t)blockIdx.x * rs;
    const int logS = TWO ? logn - 1 : logn;
    float2 v[kRegE];
    if constexpr (!TWO) {
#pragma unroll
        for (int e = 0; e < kRegE; ++e) v[e] = row[reg_input_pos<kRegMinLog, kRegE, LRM>(e)];
        reg_fft<kRegE, kRegMinLog, LRM>(v, xbuf, tw, tw_log, false);
        __syncthreads();      // every thread has read its inputs before any output is stored
#pragma unroll
        for (int e = 0; e < kRegE; ++e) row[reg_output_pos<kRegMinLog, kRegE, LRM>(e)] = v[e];
    } else {
        const int m = 1 << logS;
        // E = DFT of the even samples, O = DFT of the odd ones, both held in registers:
        // each input position's even and odd samples arrive in one 16-byte load, the
        // row is read once and written once, and the combination pairs the two
        // transforms' outputs at the same position of the same thread (radix-8 passes:
        // with radix 16 the two halves' transforms need more registers than fit)
        float2 o[kRegE];
#pragma unroll
        for (int e = 0; e < kRegE; ++e) {
            const float4 q = ((const float4*)row)[reg_input_pos<kRegMinLog, kRegE, LRM>(e)];
            v[e] = make_float2(q.x, q.y);
            o[e] = make_float2(q.z, q.w);
        }
        reg_fft<kRegE, kRegMinLog, LRM>(v, xbuf, tw, tw_log, false);
        reg_fft<kRegE, kRegMinLog, LRM>(o, xbuf, tw, tw_log, false);
        __syncthreads();      // every thread has read its inputs before any output is stored
        const float2* twc = after(tw, o[0]);
#pragma unroll
        for (int e = 0; e < kRegE; ++e) {
            const int k = reg_output_pos<kRegMinLog, kRegE, LRM>(e);
            const float2 wo = cmul(o[e], twiddle(twc, k << (tw_log - logn), false));
            row[k] = cadd(v[e], wo);
            row[k + m] = csub(v[e], wo);
        }
    }
}

// Second-order rows of 2^LOGN points (2^11 to 2^13): the fold, inverse transform and
// row maximum of k_second_order_r with one register transform of 8 values per
// thread on 2^LOGN / 8 threads (72, 36 or 18 KB of exchange buffer and at most 64
// VGPRs: two, four or eight workgroups per CU).
template <int LOGN>
__global__ void __launch_bounds__((1 << LOGN) / 8, 8) k_second_order_rs(const float2* __restrict__ Xh, int64_t Xh_pitch, int n1,
                                                              const float* __restrict__ ps, int lo, int hi, int Tp,
                                                              int Kp, float2* __restrict__ Y, int64_t y_bstride,
                                                              float invNX, const float2* __restrict__ tw, int tw_log,
                                                              float* __restrict__ rowmax, int alpha, int n_alpha) {
    extern __shared__ __align__(16) float xbuf[];
    __shared__ unsigned int rmx;
    constexpr int E = 8;
    const int lam = blockIdx.x;
    const int64_t b = blockIdx.y;
    float2* out = Y + b * y_bstride + (int64_t)lam * Tp;
    if (lam >= n1) {
        for (int t = threadIdx.x; t < Tp; t += blockDim.x) out[t] = make_float2(0.f, 0.f);
        if (threadIdx.x == 0) rowmax[(b * n_alpha + alpha) * Kp + lam] = 0.f;
        return;
    }
    if (threadIdx.x == 0) rmx = 0u;
    float2 v[E];
    fold_inputs<LOGN, reg_lr_max(E), E>(v, Xh + (b * n1 + lam) * Xh_pitch, ps, lo, hi);
    reg_fft<E, LOGN>(v, xbuf, tw, tw_log, true);
    float m = 0.f;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const float2 y = cscale(v[e], invNX);
        out[reg_output_pos<LOGN, E>(e)] = y;
        m = fmaxf(m, fmaxf(fabsf(y.x), fabsf(y.y)));
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
    __syncthreads();
    if ((threadIdx.x & 63) == 0) atomicMax(&rmx, __float_as_uint(m));
    __syncthreads();
    if (threadIdx.x == 0) rowmax[(b * n_alpha + alpha) * Kp + lam] = __uint_as_float(rmx);
}

// Rows of 2^LOGN points (2^11 to 2^13): one register transform of 8 values per
// thread on 2^LOGN / 8 threads; its exchange buffer (72, 36 or 18 KB) and at most
// 64 VGPRs let two, four or eight workgroups share a CU.
template <int LOGN>
__global__ void __launch_bounds__((1 << LOGN) / 8, 8) k_rowfft_rs(float2* __restrict__ base, int64_t bs, int64_t rs,
                                                                 const float2* __restrict__ tw, int tw_log) {
    extern __shared__ __align__(16) float xbuf[];
    constexpr int E = 8;
    float2* row = base + (int64_t)blockIdx.y * bs + (int64_t)blockIdx.x * rs;
    float2 v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = row[reg_input_pos<LOGN, E>(e)];
    reg_fft<E, LOGN>(v, xbuf, tw, tw_log, false);
    __syncthreads();      // every thread has read its inputs before any output is stored
#pragma unroll
    for (int e = 0; e < E; ++e) row[reg_output_pos<LOGN, E>(e)] = v[e];
}

// adjoint of the modulus and first-order filter for one row: recompute y, weight
// gX by its phase, forward FFT -> g1[b][lambda][0..NX)
template <bool TWO, int LRM>
__global__ void __launch_bounds__(kRegT) k_scal_bwd_b_r(const float2* __restrict__ xh, int64_t xh_pitch,
                                                      const float* __restrict__ psi1, const int* __restrict__ band1,
                                                      const int64_t* __restrict__ off1, const float* __restrict__ gX,
                                                      float2* __restrict__ g1, int logNX, float invN,
                                                      const float2* __restrict__ tw, int tw_log) {
    extern __shared__ __align__(16) float xbuf[];
    const int lam = blockIdx.x, n1 = gridDim.x;
    const int64_t b = blockIdx.y;
    const int NX = 1 << logNX;
    const int logS = TWO ? logNX - 1 : logNX;
    float* A = xbuf;
    float* Bf = xbuf + (1 << logS);
    const float2* src = xh + b * xh_pitch;
    const float* ps = psi1 + off1[lam];
    const int lo = band1[2 * lam], hi = band1[2 * lam + 1];
    const float* gx = gX + (b * n1 + lam) * (int64_t)NX;
    float2* o = g1 + (b * n1 + lam) * (int64_t)NX;
    if constexpr (!TWO) {
        float2 v[kRegE];
        fold_inputs<kRegMinLog, LRM>(v, src, ps, lo, hi);
        reg_fft<kRegE, kRegMinLog, LRM>(v, A, tw, tw_log, true);
        const float* gxh = after(gx, v[0]);
#pragma unroll
        for (int e = 0; e < kRegE; ++e) {
            const float2 y = cscale(v[e], invN);
            const float sc = gxh[reg_output_pos<kRegMinLog, kRegE, LRM>(e)] *
                             __builtin_amdgcn_rcpf(fmaxf(__builtin_amdgcn_sqrtf(y.x * y.x + y.y * y.y), kEpsMod));
            v[e] = cscale(y, sc);
        }
        // from the last pass's output layout to the first pass's input layout
        reg_output_to_input<kRegMinLog, kRegE, LRM>(v, A);
        reg_fft<kRegE, kRegMinLog, LRM>(v, A, tw, tw_log, false);
#pragma unroll
        for (int e = 0; e < kRegE; ++e) o[reg_output_pos<kRegMinLog, kRegE, LRM>(e)] = v[e];
    } else {
        // the inverse transform by decimation in frequency gives the even time samples
        // (half 0) and the odd ones (half 1); both stay in registers, so that gX is
        // read once (one 8-byte load per position for the two halves) and the
        // forward transform by decimation in time combines the halves' spectra
        // without parking one of them in the output row
        const int m = 1 << logS;
        float2 v0[kRegE], v1[kRegE];
        load_dif<true, 4, LRM>(v0, A, Bf, src, ps, lo, hi, logNX, 0, tw, tw_log, false);
        reg_fft<kRegE, kRegMinLog, LRM>(v0, A, tw, tw_log, true);
        load_dif<true, 1, LRM>(v1, A, Bf, src, ps, lo, hi, logNX, 1, tw, tw_log, false);   // beside v0: fewer loads at once
        reg_fft<kRegE, kRegMinLog, LRM>(v1, A, tw, tw_log, true);
        const float2* gx2 = (const float2*)after(gx, v1[0]);
        const int tidw = opaque_tid();       // positions formed here, not kept from before
#pragma unroll
        for (int e = 0; e < kRegE; ++e) {
            const float2 g = gx2[reg_output_pos<kRegMinLog, kRegE, LRM>(e, tidw)];     // samples 2 pos, 2 pos + 1
            const float2 y0 = cscale(v0[e], invN), y1 = cscale(v1[e], invN);
            v0[e] = cscale(y0, g.x * __builtin_amdgcn_rcpf(
                                       fmaxf(__builtin_amdgcn_sqrtf(y0.x * y0.x + y0.y * y0.y), kEpsMod)));
            v1[e] = cscale(y1, g.y * __builtin_amdgcn_rcpf(
                                       fmaxf(__builtin_amdgcn_sqrtf(y1.x * y1.x + y1.y * y1.y), kEpsMod)));
        }
        reg_output_to_input<kRegMinLog, kRegE, LRM>(v0, A);
        reg_fft<kRegE, kRegMinLog, LRM>(v0, A, tw, tw_log, false);
        reg_output_to_input<kRegMinLog, kRegE, LRM>(v1, A);
        reg_fft<kRegE, kRegMinLog, LRM>(v1, A, tw, tw_log, false);
        const float2* twc = after(tw, v1[0]);
        const int tido = opaque_tid();
#pragma unroll
        for (int e = 0; e < kRegE; ++e) {
            const int k = reg_output_pos<kRegMinLog, kRegE, LRM>(e, tido);
            const float2 wo = cmul(v1[e], twiddle(twc, k << (tw_log - logNX), false));
            o[k] = cadd(v0[e], wo);
            o[k + m] = csub(v0[e], wo);
        }
    }
}

// Adjoint of the second order and of S1 for one scalogram row of NX = 2H points,
// with the inverse real FFT held in registers (the in-LDS kernel computes the same
// sums): the Hermitian half-spectrum of gX,
//   S[m] = 1/2 sum_alpha psi_hat_alpha[m] G_alpha[m mod Ta] (real part alone at m = 0, H)
//        + phi_hat[m] G1[m mod NT],   m = 0..H,
// G_alpha the FFT of the gY2 rows (taken beforehand), G1 the FFT of the S1
// cotangent row (plus the real part of phi_T's second-order rows with the lowpass
// pairs), is formed at the thread's input positions of the H-point transform and
// parked in LDS, so that each position k takes the packed spectrum
// Z[k] = S[k] + conj(S[H-k]) + i w^k (S[k] - conj(S[H-k])) (w = e^{2 pi i / NX});
// the inverse transform of Z gives gX[2n] + i gX[2n+1], scaled 1/NX.
template <int E, int LOGH, int LRM>
__global__ void __launch_bounds__(kRegT) k_scal_bwd_a_r(const float2* __restrict__ G, int64_t y_bstride,
                                                      const int64_t* __restrict__ yoff, const int* __restrict__ Tpv,
                                                      const int* __restrict__ Tav, const float* __restrict__ psi2,
                                                      const int* __restrict__ band2, const int64_t* __restrict__ off2,
                                                      int n_alpha, const float* __restrict__ gS1,
                                                      const float* __restrict__ phiX, int Mphi, int logNT,
                                                      float* __restrict__ gX, const float2* __restrict__ tw, int tw_log,
                                                      MuLogArg ml, const float2* __restrict__ gYphi, int Tphi) {
    extern __shared__ __align__(16) float xbuf[];
    constexpr int H = 1 << LOGH;
    const int lam = blockIdx.x, n1 = gridDim.x;
    const int64_t b = blockIdx.y;
    const int NT = 1 << logNT;
    float2* Sx = (float2*)xbuf;                                  // S[0..H] (H + 1 <= the exchange buffer)
    float2* g1 = (float2*)(xbuf + reg_xbuf_floats(LOGH));        // G1, lpad_len(NT) slots
    const float em = ml.mu1 ? ml.eps * ml.mu1[0] : 0.f;
    for (int t = threadIdx.x; t < NT; t += blockDim.x) {
        const int64_t i = (b * n1 + lam) * NT + t;
        float g = gS1 ? mulog_cot(gS1[i], ml.mu1, em, ml.mu1 ? ml.o1[i] : 0.f) : 0.f;
        if (gYphi) g += gYphi[b * y_bstride + (int64_t)lam * Tphi + t].x;
        g1[lpad(t)] = make_float2(g, 0.f);
    }
    __syncthreads();
    lds_fft<16>(g1, logNT, 1, NT, tw, tw_log, false);
    __syncthreads();
    // the half-spectrum at the thread's positions k (and at H on thread 0): the
    // temporal rates in the outer loop, so that a rate's loads for all positions
    // issue together
    const int extra = threadIdx.x == 0 ? 1 : 0;
    float2 c[E + 1];
#pragma unroll
    for (int e = 0; e <= E; ++e) c[e] = make_float2(0.f, 0.f);
    for (int a = 0; a < n_alpha; ++a) {
        const int lo = band2[2 * a], hi = band2[2 * a + 1];
        const float* pa = psi2 + off2[a] - lo;
        const float2* ga = G + b * y_bstride + yoff[a] + (int64_t)lam * Tpv[a];
        const int tmask = Tav[a] - 1;
#pragma unroll
        for (int e = 0; e <= E; ++e) {
            if (e == E && !extra) continue;
            const int m = e < E ? reg_input_pos<LOGH, E, LRM>(e) : H;
            if (m >= lo && m <= hi) {
                const float g = pa[m];
                const float2 v = ga[m & tmask];
                c[e].x += g * v.x;
                c[e].y += g * v.y;
            }
        }
    }
#pragma unroll
    for (int e = 0; e <= E; ++e) {
        if (e == E && !extra) continue;
        const int m = e < E ? reg_input_pos<LOGH, E, LRM>(e) : H;
        float2 hm = (m == 0 || m == H) ? make_float2(c[e].x, 0.f) : cscale(c[e], 0.5f);
        if (m <= Mphi) {
            const float2 v = g1[lpad(m & (NT - 1))];
            hm.x += phiX[m] * v.x;
            hm.y += phiX[m] * v.y;
        }
        Sx[m] = hm;
    }
    __syncthreads();
    const int tws = tw_log - (LOGH + 1);
    float2 v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int k = reg_input_pos<LOGH, E, LRM>(e);
        const float2 p = Sx[k], q = Sx[H - k];
        const float2 Sm = make_float2(p.x + q.x, p.y - q.y);
        const float2 D = make_float2(p.x - q.x, p.y + q.y);
        const float2 wD = cmulc(D, tw[k << tws]);
        v[e] = make_float2(Sm.x - wD.y, Sm.y + wD.x);
    }
    __syncthreads();                                             // S is read; the transform reuses the buffer
    reg_fft<E, LOGH, LRM>(v, xbuf, tw, tw_log, true);
    float2* o = (float2*)(gX + (b * n1 + lam) * (int64_t)(2 * H));
    const float sc = 1.f / (float)(2 * H);
#pragma unroll
    for (int e = 0; e < E; ++e) o[reg_output_pos<LOGH, E, LRM>(e)] = cscale(v[e], sc);
}

// Each long-row kernel in both row lengths and both largest radices of its
// transform passes (16, or 8 where the tuning asks for it): LRM = log2 of that radix.
#define JTFS_REG_VARIANTS(k)                                                          \
    (const void*)k<false, 4>, (const void*)k<true, 4>, (const void*)k<false, 3>, (const void*)k<true, 3>

int reg_attributes() {
    const void* ks[] = {JTFS_REG_VARIANTS(k_scalogram_r), JTFS_REG_VARIANTS(k_second_order_r),
                        JTFS_REG_VARIANTS(k_rowfft_r), JTFS_REG_VARIANTS(k_scal_bwd_b_r),
                        (const void*)k_scal_bwd_a_r<kRegE, kRegMinLog, 4>,
                        (const void*)k_scal_bwd_a_r<kRegE, kRegMinLog, 3>,
                        (const void*)k_scal_bwd_a_r<kRegE / 2, kRegMinLog - 1, 3>, (const void*)k_rowfft_rs<13>,
                        (const void*)k_rowfft_rs<12>, (const void*)k_rowfft_rs<11>,
                        (const void*)k_second_order_rs<13>, (const void*)k_second_order_rs<12>,
                        (const void*)k_second_order_rs<11>};
    for (const void* k : ks)
        if (hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, kMaxDynLds) != hipSuccess) {
            set_error("hipFuncSetAttribute failed for the long-row kernels");
            return JTFS_EHIP;
        }
    return JTFS_OK;
}

// rows of 2^14 points: one 512-thread register transform; 2^15: two of them
static inline bool two_of(int logn) { return logn == kRegMinLog + 1; }
// the variant of long-row kernel k for rows of 2^logn points, radix 8 passes if r8
#define JTFS_REG_PICK(k, logn, r8) \
    (two_of(logn) ? ((r8) ? k<true, 3> : k<true, 4>) : ((r8) ? k<false, 3> : k<false, 4>))
static inline unsigned reg_threads() { return (unsigned)((1 << kRegMinLog) / kRegE); }
// LDS of a long-row kernel: `floats` of its own use, and at least the padded
// exchange buffer of one 2^14-point transform
static inline size_t reg_lds(size_t floats) {
    return sizeof(float) * std::max(floats, (size_t)reg_xbuf_floats(kRegMinLog));
}

void launch_scalogram_r(const jtfs_plan* P, const float2* xh, int64_t xh_pitch, float2* Xh, int64_t Xh_pitch,
                        int64_t B, hipStream_t st) {
    const Shapes& s = P->s;
    auto k = JTFS_REG_PICK(k_scalogram_r, s.logNX, P->tune.r8_scalogram);
    hipLaunchKernelGGL(k, dim3(s.n1, (unsigned)B), dim3(reg_threads()), reg_lds(s.NX), st, xh, xh_pitch,
                       P->psi1, P->band1, P->off1, Xh, Xh_pitch, s.logNX, 1.0f / (float)s.N, P->tw, P->tw_log);
    // LDS: NX floats (the two staged halves at 2^15), at least one padded exchange buffer
}

void launch_second_order_r(const jtfs_plan* P, int a, const float2* Xh, int64_t Xh_pitch, float2* Y2, float* rowmax,
                           int64_t B, hipStream_t st) {
    const Shapes& s = P->s;
    const int logTa = s.logNX - s.k2[a];
    const Family& f2 = s.f2;
    if (logTa >= kRegMinLog - 3 && logTa <= kRegMinLog - 1) {
        auto k = logTa == kRegMinLog - 1   ? k_second_order_rs<kRegMinLog - 1>
                 : logTa == kRegMinLog - 2 ? k_second_order_rs<kRegMinLog - 2>
                                           : k_second_order_rs<kRegMinLog - 3>;
        hipLaunchKernelGGL(k, dim3(s.Kp, (unsigned)B), dim3((1u << logTa) / 8),
                           sizeof(float) * (size_t)reg_xbuf_floats(logTa), st, Xh, Xh_pitch, s.n1,
                           P->psi2 + f2.off[a], f2.lo[a], f2.hi[a], s.Tp[a], s.Kp, Y2 + s.yoff[a],
                           (int64_t)s.Kp * s.sumTp, 1.0f / (float)s.NX, P->tw, P->tw_log, rowmax, a, s.n_alpha);
        return;
    }
    auto k = JTFS_REG_PICK(k_second_order_r, logTa, P->tune.r8_second);
    hipLaunchKernelGGL(k, dim3(s.Kp, (unsigned)B), dim3(reg_threads()), reg_lds((size_t)1 << logTa), st, Xh, Xh_pitch,
                       s.n1, P->psi2 + f2.off[a], f2.lo[a], f2.hi[a], logTa, s.Tp[a], s.Kp, Y2 + s.yoff[a],
                       (int64_t)s.Kp * s.sumTp, 1.0f / (float)s.NX, P->tw, P->tw_log, rowmax, a, s.n_alpha);
}

void launch_rowfft_r(const jtfs_plan* P, float2* base, int64_t bs, int64_t rs, int rows, int logn, int64_t B,
                     hipStream_t st) {
    if (logn >= kRegMinLog - 3 && logn <= kRegMinLog - 1) {
        auto k = logn == kRegMinLog - 1   ? k_rowfft_rs<kRegMinLog - 1>
                 : logn == kRegMinLog - 2 ? k_rowfft_rs<kRegMinLog - 2>
                                          : k_rowfft_rs<kRegMinLog - 3>;
        hipLaunchKernelGGL(k, dim3((unsigned)rows, (unsigned)B), dim3((1u << logn) / 8),
                           sizeof(float) * (size_t)reg_xbuf_floats(logn), st, base, bs, rs, P->tw, P->tw_log);
        return;
    }
    auto k = JTFS_REG_PICK(k_rowfft_r, logn, P->tune.r8_rowfft);
    hipLaunchKernelGGL(k, dim3((unsigned)rows, (unsigned)B), dim3(reg_threads()), reg_lds(0), st,
                       base, bs, rs, logn, P->tw, P->tw_log);
}

void launch_scal_bwd_a_r(const jtfs_plan* P, const float2* G, int64_t y_bstride, const float* gS1, const MuLogArg& ml,
                         const float2* gYphi, int Tphi, float* gX, int64_t B, hipStream_t st) {
    const Shapes& s = P->s;
    const int logNT = s.logN - s.logT;
    // rows of 2^15 points: a 2^14-point transform of 16 values per thread; 2^14: 2^13 of 8
    auto k = s.logNX == kRegMinLog + 1
                 ? (P->tune.r8_first_adj ? k_scal_bwd_a_r<kRegE, kRegMinLog, 3> : k_scal_bwd_a_r<kRegE, kRegMinLog, 4>)
                 : k_scal_bwd_a_r<kRegE / 2, kRegMinLog - 1, 3>;
    const int logH = s.logNX - 1;
    const size_t lds = sizeof(float) * ((size_t)reg_xbuf_floats(logH) + 2 * (size_t)lpad_len(s.NT));
    hipLaunchKernelGGL(k, dim3(s.n1, (unsigned)B), dim3(reg_threads()), lds, st, G, y_bstride, P->d_yoff, P->d_Tp,
                       P->d_Ta, P->psi2, P->band2, P->off2, s.n_alpha_psi, gS1, P->phiX, s.Mphi, logNT, gX, P->tw,
                       P->tw_log, ml, gYphi, Tphi);
}

void launch_scal_bwd_b_r(const jtfs_plan* P, const float2* xh, int64_t xh_pitch, const float* gX, float2* g1,
                         int64_t B, hipStream_t st) {
    const Shapes& s = P->s;
    auto k = JTFS_REG_PICK(k_scal_bwd_b_r, s.logNX, P->tune.r8_first_adj);
    hipLaunchKernelGGL(k, dim3(s.n1, (unsigned)B), dim3(reg_threads()), reg_lds(s.NX), st, xh,
                       xh_pitch, P->psi1, P->band1, P->off1, gX, g1, s.logNX, 1.0f / (float)s.N, P->tw, P->tw_log);
}

}  // namespace jtfs
