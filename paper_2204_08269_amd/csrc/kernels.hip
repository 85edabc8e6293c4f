// JTFS forward and backward on gfx950: FFT passes in LDS, the fused scalogram
// and second-order kernels, the frequential contraction on FP32 MFMA with the
// modulus and time lowpass fused into its epilogue, and every stage's adjoint.
//
// Scaling conventions: all FFTs are unnormalised; every 1/M of an inverse DFT is
// applied explicitly where the stage's definition puts it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "fft_lds.hpp"
#include "plan.hpp"
#include "timing.hpp"
#include "split.hpp"
#include "regk.hpp"

namespace jtfs {

typedef float floatx16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ floatx16 mfma32(float a, float b, floatx16 c) {
    // D[i][j] += sum_k A[i][k] B[k][j], 32x32x2: lane (i + 32k) holds A[i][k] and
    // B[k][i]; D element (i, j) sits in lane j + 32*((i/4)%2), register (i%4) + 4*(i/8).
    return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ floatx16 zero16() {
    floatx16 z;
#pragma unroll
    for (int r = 0; r < 16; ++r) z[r] = 0.f;
    return z;
}
// row (within a 32x32 tile) held by register r of a lane in half h
__device__ __forceinline__ int crow(int r, int h) { return 8 * (r >> 2) + 4 * h + (r & 3); }

// ---------------------------------------------------------------------------
// Generic batched FFT over LDS: transform c of batch b has element e at
// in[b*ib + c*ics + e*ies]; the output X_c[k] (times w_n^{c k} when twl > 0, the
// four-step twist, and times scale) goes to out[b*ob + c*ocs + k*oes].
// Column mode (ics == 1): C = 2^logC adjacent transforms per workgroup, loaded
// with adjacent columns on adjacent threads.  Row mode: transforms contiguous.
// ---------------------------------------------------------------------------
template <typename CI, typename C>
__device__ __forceinline__ C to_cplx(CI v) {
    using R = typename cplx<C>::real;
    return cplx<C>::make((R)v.x, (R)v.y);
}

template <typename CI, typename C>
__global__ void __launch_bounds__(1024) k_fft_cols_t(const CI* in, C* out, int loglen, int ncols, int logC,
                                                    int64_t ib, int64_t ics, int64_t ies, int64_t ob, int64_t ocs,
                                                    int64_t oes, int twl, const C* __restrict__ tw, int tw_log, int inv,
                                                    typename cplx<C>::real scale) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    C* s = (C*)lds_raw;
    const int len = 1 << loglen, st = lpad_len(len) + 1;     // odd stride: columns in distinct banks
    const int Cn = 1 << logC;
    const int c0 = blockIdx.x * Cn;
    const int nc = min(Cn, ncols - c0);
    const int tot = nc * len;
    const int64_t b = blockIdx.y;
    in += b * ib;
    out += b * ob;
    // all of a thread's loads (at most 16: tot <= 16 blockDim, as the transform
    // requires) are issued before any LDS store, so that their latencies overlap
    // instead of following one another
    constexpr int kMaxPerThread = 16;
    C v[kMaxPerThread];
#pragma unroll
    for (int q = 0; q < kMaxPerThread; ++q) {
        const int e = threadIdx.x + q * blockDim.x;
        if (e < tot) {
            const int c = ics == 1 ? (e & (Cn - 1)) : (e >> loglen), k = ics == 1 ? (e >> logC) : (e & (len - 1));
            v[q] = to_cplx<CI, C>(in[(int64_t)(c0 + c) * ics + (int64_t)k * ies]);
        }
    }
#pragma unroll
    for (int q = 0; q < kMaxPerThread; ++q) {
        const int e = threadIdx.x + q * blockDim.x;
        if (e < tot) {
            const int c = ics == 1 ? (e & (Cn - 1)) : (e >> loglen), k = ics == 1 ? (e >> logC) : (e & (len - 1));
            s[c * st + lpad(k)] = v[q];
        }
    }
    __syncthreads();
    lds_fft<16>(s, loglen, nc, st, tw, tw_log, inv != 0);
    const int tws = tw_log - twl;
    if (ocs == 1) {
        for (int e = threadIdx.x; e < tot; e += blockDim.x) {
            const int c = e & (Cn - 1), k = e >> logC;
            C v = s[lpad(k) + c * st];
            if (twl) v = cmul(v, twiddle(tw, ((c0 + c) * k) << tws, inv != 0));
            out[(int64_t)(c0 + c) + (int64_t)k * oes] = cplx<C>::make(v.x * scale, v.y * scale);
        }
    } else {
        for (int e = threadIdx.x; e < tot; e += blockDim.x) {
            const int c = e >> loglen, k = e & (len - 1);
            C v = s[lpad(k) + c * st];
            if (twl) v = cmul(v, twiddle(tw, ((c0 + c) * k) << tws, inv != 0));
            out[(int64_t)(c0 + c) * ocs + (int64_t)k * oes] = cplx<C>::make(v.x * scale, v.y * scale);
        }
    }
}

// The FP32 transform used by the intermediate stages.
#define k_fft_cols k_fft_cols_t<float2, float2>

// Real-input spectrum in FP64 from the half-length complex FFT of
// z[k] = x[2k] + i x[2k+1] (z rows of pitch zp): X[m] = E[m] + w_n^m O[m], E/O the
// spectra of the even/odd samples; bins 0..H rounded once to FP32 into rows of
// pitch H+1 (H = n/2).
__global__ void k_rfft_post64(const double2* __restrict__ z, int64_t zp, float2* __restrict__ xh, int64_t pitch,
                              int logn, const double2* __restrict__ tw, int tw_log) {
    const int H = 1 << (logn - 1);
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m > H / 2) return;
    const double2* zr = z + (int64_t)blockIdx.y * zp;
    float2* row = xh + (int64_t)blockIdx.y * pitch;
    const int tws = tw_log - logn;
    if (m == 0) {
        const double2 q = zr[0];
        row[0] = make_float2((float)(q.x + q.y), 0.f);
        row[H] = make_float2((float)(q.x - q.y), 0.f);
        return;
    }
    const double2 a = zr[m], b = zr[H - m];
    auto spec = [&](double2 p, double2 q, int k) {
        const double2 E = make_double2(0.5 * (p.x + q.x), 0.5 * (p.y - q.y));
        const double2 D = make_double2(p.x - q.x, p.y + q.y);          // p - conj(q)
        const double2 O = make_double2(0.5 * D.y, -0.5 * D.x);      // D / (2i)
        const double2 X = cadd(E, cmul(O, tw[k << tws]));
        return make_float2((float)X.x, (float)X.y);
    };
    row[m] = spec(a, b, m);
    row[H - m] = spec(b, a, H - m);
}

// Inverse of the real-spectrum post-pass: Z'[k] = (X[k] + conj X[H-k]) + i w_n^{-k} (X[k] - conj X[H-k]),
// whose unnormalised inverse FFT is n times the interleaved real signal.
__global__ void k_irfft_pack(const float2* __restrict__ xh, int64_t pitch, float2* __restrict__ z, int64_t zpitch,
                             int logn, const float2* __restrict__ tw, int tw_log) {
    const int H = 1 << (logn - 1);
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k > H / 2) return;
    const float2* row = xh + (int64_t)blockIdx.y * pitch;
    float2* zr = z + (int64_t)blockIdx.y * zpitch;
    const int tws = tw_log - logn;
    auto pk = [&](float2 p, float2 q, int kk) {
        const float2 S = make_float2(p.x + q.x, p.y - q.y);          // p + conj q
        const float2 D = make_float2(p.x - q.x, p.y + q.y);          // p - conj q
        const float2 wD = cmulc(D, tw[kk << tws]);                   // w^{-k} D
        return make_float2(S.x - wD.y, S.y + wD.x);                  // S + i wD
    };
    const float2 a = row[k], b = row[H - k];
    zr[k] = pk(a, b, k);
    if (k > 0 && H - k != k) zr[H - k] = pk(b, a, H - k);
}

// ---------------------------------------------------------------------------
// First order (fused): fold x_hat * psi_hat_lambda over the band into NX bins,
// inverse FFT (the filtered signal at the scalogram rate), modulus, real FFT of
// the scalogram row; writes X_hat[b][lambda][0..NX/2].
// ---------------------------------------------------------------------------
__device__ __forceinline__ void fold_band(float2* s, const float2* __restrict__ src, const float* __restrict__ ps, int lo,
                                          int hi, int logM) {
    const int M = 1 << logM;
    if (hi - lo < M && M <= 16 * (int)blockDim.x) {
        // every bin receives at most one band sample: all of a thread's loads are
        // issued before any product is formed
        // (two rounds of eight keep the kernels within 64 VGPRs)
#pragma unroll
        for (int q0 = 0; q0 < 16; q0 += 8) {
            float2 v[8];
            float g[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int p = threadIdx.x + (q0 + q) * blockDim.x;
                const int m = lo + ((p - lo) & (M - 1));
                const bool ok = p < M && m <= hi;
                v[q] = ok ? src[m] : make_float2(0.f, 0.f);
                g[q] = ok ? ps[m - lo] : 0.f;
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int p = threadIdx.x + (q0 + q) * blockDim.x;
                if (p < M) s[lpad(p)] = make_float2(v[q].x * g[q], v[q].y * g[q]);
            }
        }
        return;
    }
    for (int p = threadIdx.x; p < M; p += blockDim.x) {
        float2 acc = make_float2(0.f, 0.f);
        for (int m = lo + ((p - lo) & (M - 1)); m <= hi; m += M) {
            const float2 v = src[m];
            const float g = ps[m - lo];
            acc.x += v.x * g;
            acc.y += v.y * g;
        }
        s[lpad(p)] = acc;
    }
}

__global__ void __launch_bounds__(1024, 8) k_scalogram(const float2* __restrict__ xh, int64_t xh_pitch,
                                                   const float* __restrict__ psi1, const int* __restrict__ band1,
                                                   const int64_t* __restrict__ off1, float2* __restrict__ Xh,
                                                   int64_t Xh_pitch, int logNX, float invN,
                                                   const float2* __restrict__ tw, int tw_log) {
    extern __shared__ float2 s[];
    const int lam = blockIdx.x, n1 = gridDim.x;
    const int64_t b = blockIdx.y;
    const int NX = 1 << logNX, H = NX >> 1;
    fold_band(s, xh + b * xh_pitch, psi1 + off1[lam], band1[2 * lam], band1[2 * lam + 1], logNX);
    __syncthreads();
    lds_fft<16>(s, logNX, 1, NX, tw, tw_log, true);
    // modulus of the scalogram-rate samples, packed as z[k] = X[2k] + i X[2k+1]
    {
        float2 v[8];   // H <= 8192 = 8 * blockDim
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int k = threadIdx.x + q * blockDim.x;
            if (k < H) {
                const float2 a = s[lpad(2 * k)], c = s[lpad(2 * k + 1)];
                v[q] = make_float2(__builtin_amdgcn_sqrtf(a.x * a.x + a.y * a.y) * invN,
                                   __builtin_amdgcn_sqrtf(c.x * c.x + c.y * c.y) * invN);
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int k = threadIdx.x + q * blockDim.x;
            if (k < H) s[lpad(k)] = v[q];
        }
        __syncthreads();
    }
    if (logNX > 1) lds_fft<16>(s, logNX - 1, 1, H, tw, tw_log, false);
    float2* out = Xh + (b * n1 + lam) * Xh_pitch;
    const int tws = tw_log - logNX;
    for (int m = threadIdx.x; m <= H / 2; m += blockDim.x) {
        if (m == 0) {
            const float2 z = s[0];
            out[0] = make_float2(z.x + z.y, 0.f);
            out[H] = make_float2(z.x - z.y, 0.f);
            continue;
        }
        const float2 a = s[lpad(m)], c = s[lpad(H - m)];
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

// S1[tau] = (X (*) phi_T)[tau T/2^kX]: fold X_hat * phi_hat over the N/T-bin grid
// (bins -Mneg..Mphi of the NX grid), inverse FFT, real part / NX.  One workgroup per
// (lambda, signal).  S1 may be null.  With the lowpass pairs, the same rows are also
// the second-order rows of alpha = phi_T: written to Yphi (real, zero beyond N/T
// frames and for the padding rows n1 <= lambda < Kp, which take the extra
// workgroups) with their row maxima for the operand split.
__global__ void __launch_bounds__(256) k_s1(const float2* __restrict__ Xh, int64_t Xh_pitch,
                                            const float* __restrict__ phiX, int Mphi, int logNX, int logNT, float invNX,
                                            float* __restrict__ S1, const float2* __restrict__ tw, int tw_log,
                                            const float* __restrict__ mu1, float eps, int n1,
                                            float2* __restrict__ Yphi, int64_t y_bstride, int Tp,
                                            float* __restrict__ rowmax, int alpha, int n_alpha, int Kp) {
    extern __shared__ float2 s[];
    __shared__ float red[256];
    const int lam = blockIdx.x;
    const int64_t b = blockIdx.y;
    const int NX = 1 << logNX, NT = 1 << logNT;
    if (lam >= n1) {                                 // padding rows of Yphi
        float2* y = Yphi + b * y_bstride + (int64_t)lam * Tp;
        for (int t = threadIdx.x; t < Tp; t += blockDim.x) y[t] = make_float2(0.f, 0.f);
        if (threadIdx.x == 0) rowmax[(b * n_alpha + alpha) * Kp + lam] = 0.f;
        return;
    }
    const float2* row = Xh + (b * n1 + lam) * Xh_pitch;
    const int Mneg = (Mphi == NX / 2) ? Mphi - 1 : Mphi;
    for (int p = threadIdx.x; p < NT; p += blockDim.x) {
        float2 acc = make_float2(0.f, 0.f);
        for (int mt = -Mneg + ((p + Mneg) & (NT - 1)); mt <= Mphi; mt += NT) {
            const float2 v = mt >= 0 ? row[mt] : conjf2(row[-mt]);
            const float g = phiX[mt >= 0 ? mt : -mt];
            acc.x += v.x * g;
            acc.y += v.y * g;
        }
        s[lpad(p)] = acc;
    }
    __syncthreads();
    lds_fft<64>(s, logNT, 1, NT, tw, tw_log, true);
    if (S1) {
        float* o = S1 + (b * n1 + lam) * NT;
        const float inv = mulog_inv(mu1, 0, eps);
        for (int t = threadIdx.x; t < NT; t += blockDim.x) o[t] = mulog_out(s[lpad(t)].x * invNX, mu1, inv);
    }
    if (Yphi) {
        float2* y = Yphi + b * y_bstride + (int64_t)lam * Tp;
        float mx = 0.f;
        for (int t = threadIdx.x; t < Tp; t += blockDim.x) {
            const float v = t < NT ? s[lpad(t)].x * invNX : 0.f;
            y[t] = make_float2(v, 0.f);
            mx = fmaxf(mx, fabsf(v));
        }
        red[threadIdx.x] = mx;
        __syncthreads();
        for (int w = blockDim.x / 2; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + w]);
            __syncthreads();
        }
        if (threadIdx.x == 0) rowmax[(b * n_alpha + alpha) * Kp + lam] = red[0];
    }
}

// Zeroth order: S0[b][tau] = (x (*) phi_T)[tau T] as the direct circular sum over the
// offsets where phi_T is stored, h[k] = phi_T[(k - H) mod N]:
//   S0[tau] = sum_{k < len} h[k] x[(tau T + H - k) mod N].
// grid (N/T, B); each thread sums a strided share of k, then the workgroup reduces.
__global__ void __launch_bounds__(256) k_s0(const float* __restrict__ x, int64_t N, int64_t T,
                                            const float* __restrict__ h, int64_t len, int64_t H,
                                            float* __restrict__ s0) {
    __shared__ float red[256];
    const int tau = blockIdx.x, NT = gridDim.x;
    const int64_t b = blockIdx.y;
    const float* xb = x + b * N;
    const int64_t base = (int64_t)tau * T + H;       // x index = (base - k) mod N
    float acc = 0.f;
    for (int64_t k = threadIdx.x; k < len; k += blockDim.x) {
        int64_t n = (base - k) % N;
        if (n < 0) n += N;
        acc += h[k] * xb[n];
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) s0[b * NT + tau] = red[0];
}

// Its adjoint, added to gx: gx[n] += sum_tau gS0[tau] h[(tau T - n + H) mod N] where
// that index is below len.  grid (ceil(N / 256), B).
__global__ void __launch_bounds__(256) k_s0_bwd(const float* __restrict__ gs0, int64_t N, int64_t T, int NT,
                                                const float* __restrict__ h, int64_t len, int64_t H,
                                                float* __restrict__ gx) {
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t b = blockIdx.y;
    if (n >= N) return;
    const float* g = gs0 + b * NT;
    float acc = 0.f;
    for (int tau = 0; tau < NT; ++tau) {
        int64_t k = ((int64_t)tau * T - n + H) % N;
        if (k < 0) k += N;
        if (k < len) acc += g[tau] * h[k];
    }
    gx[b * N + n] += acc;
}

// Second order: Y2[b][alpha][lambda][t] = (X_lambda (*) psi_alpha)[t 2^k2] for t < Ta,
// zero for Ta <= t < Tp and for lambda >= n1 (the K padding of the contraction).
__global__ void __launch_bounds__(1024) k_second_order(const float2* __restrict__ Xh, int64_t Xh_pitch, int n1,
                                                      const float* __restrict__ ps, int lo, int hi, int logTa, int Tp,
                                                      int rows, int Kp, float2* __restrict__ Y, int64_t y_bstride,
                                                      float invNX, const float2* __restrict__ tw, int tw_log,
                                                      float* __restrict__ rowmax, int alpha, int n_alpha) {
    extern __shared__ float2 s[];
    __shared__ unsigned int rmx[64];
    const int64_t b = blockIdx.y;
    const int r0 = blockIdx.x * rows;
    const int Ta = 1 << logTa, rs = lpad_len(Ta);    // row stride in LDS
    const int nr = min(rows, Kp - r0);
    if (r0 >= n1) {
        // padding rows lambda >= n1 only: zero rows (the contraction reads them), maxima 0
        float2* out = Y + b * y_bstride + (int64_t)r0 * Tp;
        for (int64_t e = threadIdx.x; e < (int64_t)nr * Tp; e += blockDim.x) out[e] = make_float2(0.f, 0.f);
        if ((int)threadIdx.x < nr) rowmax[(b * n_alpha + alpha) * Kp + r0 + threadIdx.x] = 0.f;
        return;
    }
    if (threadIdx.x < 64) rmx[threadIdx.x] = 0u;
    if (hi - lo < Ta && nr * Ta <= 16 * (int)blockDim.x) {
        // every bin receives at most one band sample: all of a thread's loads are
        // issued before any product is formed
#pragma unroll
        for (int q0 = 0; q0 < 16; q0 += 8) {
            float2 v[8];
            float g[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int e = threadIdx.x + (q0 + q) * blockDim.x;
                const int c = e >> logTa, p = e & (Ta - 1);
                const int lam = r0 + c;
                const int m = lo + ((p - lo) & (Ta - 1));
                const bool ok = e < nr * Ta && lam < n1 && m <= hi;
                v[q] = ok ? Xh[(b * n1 + lam) * Xh_pitch + m] : make_float2(0.f, 0.f);
                g[q] = ok ? ps[m - lo] : 0.f;
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int e = threadIdx.x + (q0 + q) * blockDim.x;
                if (e < nr * Ta) s[(e >> logTa) * rs + lpad(e & (Ta - 1))] = make_float2(v[q].x * g[q], v[q].y * g[q]);
            }
        }
    } else {
        for (int e = threadIdx.x; e < nr * Ta; e += blockDim.x) {
            const int c = e >> logTa, p = e & (Ta - 1);
            const int lam = r0 + c;
            float2 acc = make_float2(0.f, 0.f);
            if (lam < n1) {
                const float2* row = Xh + (b * n1 + lam) * Xh_pitch;
                for (int m = lo + ((p - lo) & (Ta - 1)); m <= hi; m += Ta) {
                    const float2 v = row[m];
                    const float g = ps[m - lo];
                    acc.x += v.x * g;
                    acc.y += v.y * g;
                }
            }
            s[c * rs + lpad(p)] = acc;
        }
    }
    __syncthreads();
    lds_fft<16>(s, logTa, nr, rs, tw, tw_log, true);
    float2* out = Y + b * y_bstride + (int64_t)r0 * Tp;
    for (int c = 0; c < nr; ++c) {
        float m = 0.f;
        for (int t = threadIdx.x; t < Tp; t += blockDim.x) {
            const float2 v = t < Ta ? cscale(s[c * rs + lpad(t)], invNX) : make_float2(0.f, 0.f);
            out[(int64_t)c * Tp + t] = v;
            m = fmaxf(m, fmaxf(fabsf(v.x), fabsf(v.y)));
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
        if ((threadIdx.x & 63) == 0) atomicMax(&rmx[c], __float_as_uint(m));
    }
    __syncthreads();
    if ((int)threadIdx.x < nr) rowmax[(b * n_alpha + alpha) * Kp + r0 + threadIdx.x] = __uint_as_float(rmx[threadIdx.x]);
}

// ---------------------------------------------------------------------------
// Frequential contraction (eq. 3 along lambda, both spins) on FP32 MFMA, fused
// with the modulus and the time lowpass:
//   Z_up^T[t][l]   = sum_k Y[k][t] W[l][k]        (theta = -1)
//   Z_down^T[t][l] = sum_k Y[k][t] conj W[l][k]   (theta = +1, the mirrored wavelet)
// from the four real products of (Yr, Yi) x (Wr, Wi); then
//   V^T[tau][l] += sum_t Phi[t][tau] |Z^T[t][l]|   (second MFMA, the C registers of
// the first serve directly as its B operand).  One workgroup: 64 l x one t-chunk,
// four waves on 32x32 sub-tiles; partial V per (t-chunk, t-half) slot.
// ---------------------------------------------------------------------------
template <int NTB>
__global__ void __launch_bounds__(256) k_freq_fwd(const float2* __restrict__ Y, int64_t y_bstride, int Tp, int chunk,
                                                  const float2* __restrict__ Wt, int Mp, int Kp,
                                                  const float* __restrict__ Phi, float* __restrict__ Vp,
                                                  int64_t vp_bstride, int slot0, int nlt) {
    constexpr int NTp = 32 * NTB;
    __shared__ float2 Ys[kKStep][kTileT];
    __shared__ float2 Ws[kKStep][kTileL];
    const int lt = blockIdx.x, ch = blockIdx.y;
    const int64_t b = blockIdx.z;
    const int l0 = lt * kTileL;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int h = lane >> 5, i32 = lane & 31;
    const int lw = (wave >> 1) * 32, twv = (wave & 1) * 32;
    const float2* Yb = Y + b * y_bstride;
    floatx16 vu[NTB], vd[NTB];
#pragma unroll
    for (int n = 0; n < NTB; ++n) { vu[n] = zero16(); vd[n] = zero16(); }

    for (int t0 = ch * chunk; t0 < (ch + 1) * chunk; t0 += kTileT) {
        floatx16 rr = zero16(), ir = zero16(), ri = zero16(), ii = zero16();
        for (int k0 = 0; k0 < Kp; k0 += kKStep) {
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int f = tid + q * 256, row = f >> 5, c = (f & 31) * 2;
                *(float4*)&Ys[row][c] = *(const float4*)(Yb + (int64_t)(k0 + row) * Tp + t0 + c);
                *(float4*)&Ws[row][c] = *(const float4*)(Wt + (int64_t)(k0 + row) * Mp + l0 + c);
            }
            __syncthreads();
#pragma unroll
            for (int ks = 0; ks < kKStep / 2; ++ks) {
                const float2 a = Ys[2 * ks + h][twv + i32];
                const float2 w = Ws[2 * ks + h][lw + i32];
                rr = mfma32(a.x, w.x, rr);
                ir = mfma32(a.y, w.x, ir);
                ri = mfma32(a.x, w.y, ri);
                ii = mfma32(a.y, w.y, ii);
            }
            __syncthreads();
        }
        floatx16 uu, ud;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const float ur = rr[r] - ii[r], ui = ir[r] + ri[r];
            const float dr = rr[r] + ii[r], di = ir[r] - ri[r];
            uu[r] = sqrtf(ur * ur + ui * ui);
            ud[r] = sqrtf(dr * dr + di * di);
        }
        const float* ph = Phi + (int64_t)(t0 + twv) * NTp;
#pragma unroll
        for (int n = 0; n < NTB; ++n) {
#pragma unroll
            for (int sidx = 0; sidx < 16; ++sidx) {
                const float p = ph[crow(sidx, h) * NTp + n * 32 + i32];
                vu[n] = mfma32(p, uu[sidx], vu[n]);
                vd[n] = mfma32(p, ud[sidx], vd[n]);
            }
        }
    }
    // partial V: [slot][lt][spin][tau][64 l]
    const int slot = slot0 + ch * 2 + (wave & 1);
    float* out = Vp + b * vp_bstride + ((int64_t)slot * nlt + lt) * 2 * NTp * kTileL;
#pragma unroll
    for (int n = 0; n < NTB; ++n) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int tau = n * 32 + crow(r, h);
            out[(int64_t)tau * kTileL + lw + i32] = vu[n][r];
            out[(int64_t)(NTp + tau) * kTileL + lw + i32] = vd[n][r];
        }
    }
}

// Frequency lowpass (eq. (3)): S2[b][alpha][beta][theta][m][tau] =
// sum_l PF_beta[m][l] V[theta][rowoff + l][tau], V summed over the partial slots
// of the contraction's t-chunks.  grid (n_beta, 2 n_alpha, B), every temporal rate
// in one launch.  The l axis runs in chunks of 64: the chunk's V (64 x TT columns
// tau, its partial slots summed on the way in) and its rows of PF^T (64 x 32 rows
// m, from the transposed table PFt) are staged in LDS, and each thread adds its
// TT / 8 outputs (rows m of one tau) over the chunk, l in order.  Rows m beyond 32
// and columns beyond TT take further passes.
template <int TT>
__global__ void __launch_bounds__(256) k_s2_out(const float* __restrict__ Vp, int64_t vp_bstride,
                                                const int64_t* __restrict__ vchoff, const int* __restrict__ nch,
                                                int slot_mult, int nlt, int NTp, int NT, const float* __restrict__ PFt,
                                                const int64_t* __restrict__ pfoff, const int* __restrict__ Lbv,
                                                const int* __restrict__ rowoffv, int NL, int NLo, int n_alpha,
                                                float* __restrict__ S2, const float* __restrict__ mu2, float eps) {
    // NLo <= NL output rows (the unpadded lambda axis keeps the first NLo)
    constexpr int LC = 64, MB = 32, NG = 256 / TT, RR = MB / NG;
    __shared__ float Vs[LC][TT + 1];
    __shared__ float Ps[LC][MB];
    const int beta = blockIdx.x, th = blockIdx.y & 1, alpha = blockIdx.y >> 1, n_beta = gridDim.x;
    const int slot0 = (int)vchoff[alpha] * slot_mult, nslots = nch[alpha] * slot_mult;
    const int64_t b = blockIdx.z;
    const int Lb = Lbv[beta], ro = rowoffv[beta];
    const float* PT = PFt + pfoff[beta];             // [Lb][NL]
    const float* Vb = Vp + b * vp_bstride;
    float* o = S2 + ((((b * n_alpha + alpha) * n_beta + beta) * 2 + th) * NLo) * (int64_t)NT;
    const int tau = threadIdx.x % TT, grp = threadIdx.x / TT;
    const float inv = mulog_inv(mu2, (alpha * n_beta + beta) * 2 + th, eps);
    for (int mb = 0; mb < NLo; mb += MB)
        for (int tb = 0; tb < NT; tb += TT) {
            float acc[RR];
#pragma unroll
            for (int r = 0; r < RR; ++r) acc[r] = 0.f;
            for (int l0 = 0; l0 < Lb; l0 += LC) {
                const int lc = Lb - l0 < LC ? Lb - l0 : LC;
                __syncthreads();                         // the previous chunk is read
                for (int e = threadIdx.x; e < LC * TT; e += 256) {
                    const int tt = e / LC, l = e - tt * LC;
                    float v = 0.f;
                    if (l < lc && tb + tt < NT) {
                        const int row = ro + l0 + l, lt = row / kTileL, lr = row % kTileL;
                        for (int sl = 0; sl < nslots; ++sl)
                            v += Vb[(((int64_t)(slot0 + sl) * nlt + lt) * 2 + th) * NTp * kTileL +
                                    (int64_t)(tb + tt) * kTileL + lr];
                    }
                    Vs[l][tt] = v;
                }
                for (int e = threadIdx.x; e < LC * MB; e += 256) {
                    const int l = e / MB, mm = e - l * MB;
                    Ps[l][mm] = l < lc && mb + mm < NLo ? PT[(int64_t)(l0 + l) * NL + mb + mm] : 0.f;
                }
                __syncthreads();
                for (int l = 0; l < lc; ++l) {
                    const float v = Vs[l][tau];
#pragma unroll
                    for (int r = 0; r < RR; ++r) acc[r] += Ps[l][grp * RR + r] * v;
                }
            }
            if (tb + tau < NT)
#pragma unroll
                for (int r = 0; r < RR; ++r) {
                    const int m = mb + grp * RR + r;
                    if (m < NLo) o[(int64_t)m * NT + tb + tau] = mulog_out(acc[r], mu2, inv);
                }
        }
}

// Eq. (4) (no frequential lowpass): V summed over its partial slots and stored per
// (beta, theta) at rows 2 rowoff(beta) + theta Lb + l of S2[b][alpha][2 Mh][NT].
// lambda runs fastest so that the partial-slot reads are contiguous.
__global__ void __launch_bounds__(256) k_v_out(const float* __restrict__ Vp, int64_t vp_bstride,
                                               const int64_t* __restrict__ vchoff, const int* __restrict__ nch,
                                               int slot_mult, int nlt, int NTp, int NT, const int* __restrict__ Lbv,
                                               const int* __restrict__ rowoffv, int Mh, int n_alpha,
                                               float* __restrict__ S2, const float* __restrict__ mu2, float eps) {
    // grid (n_beta, 2 n_alpha, B): every temporal rate in one launch
    const int beta = blockIdx.x, th = blockIdx.y & 1, alpha = blockIdx.y >> 1;
    const int slot0 = (int)vchoff[alpha] * slot_mult, nslots = nch[alpha] * slot_mult;
    const int64_t b = blockIdx.z;
    const int Lb = Lbv[beta], ro = rowoffv[beta];
    const float* Vb = Vp + b * vp_bstride;
    float* o = S2 + ((b * n_alpha + alpha) * 2 * (int64_t)Mh + 2 * ro + th * Lb) * NT;
    const float inv = mulog_inv(mu2, (alpha * (int)gridDim.x + beta) * 2 + th, eps);
    for (int e = threadIdx.x; e < Lb * NT; e += blockDim.x) {
        const int tau = e / Lb, l = e - tau * Lb;
        const int row = ro + l, lt = row / kTileL, lr = row % kTileL;
        float acc = 0.f;
        for (int sl = 0; sl < nslots; ++sl)
            acc += Vb[(((int64_t)(slot0 + sl) * nlt + lt) * 2 + th) * NTp * kTileL + (int64_t)tau * kTileL + lr];
        o[(int64_t)l * NT + tau] = mulog_out(acc, mu2, inv);
    }
}

// Time scattering (sec. 4): S2[b][alpha][lambda][tau] = sum_t |Y2[b][alpha][lambda][t]| Phi_alpha[t][tau]
// (modulus of the second-order row, then the time lowpass on the N/T frames).
// Threads are (tau, t-group) pairs; |Y2| of 256 samples at a time goes through LDS.
__global__ void __launch_bounds__(256) k_ts_out(const float2* __restrict__ Y, int64_t y_bstride, int Tp, int Ta,
                                                const float* __restrict__ Phi, int NTp, int NT, int alpha,
                                                int n_alpha, float* __restrict__ S2, const float* __restrict__ mu2,
                                                float eps) {
    __shared__ float mag[256];
    __shared__ float part[256];
    const int lam = blockIdx.x, n1 = gridDim.x;
    const int64_t b = blockIdx.y;
    const float2* row = Y + b * y_bstride + (int64_t)lam * Tp;
    const int tau = threadIdx.x % NTp, g = threadIdx.x / NTp, G = blockDim.x / NTp;
    float acc = 0.f;
    for (int t0 = 0; t0 < Ta; t0 += 256) {
        __syncthreads();
        const int t = t0 + threadIdx.x;
        if (t < Ta) {
            const float2 y = row[t];
            mag[threadIdx.x] = sqrtf(y.x * y.x + y.y * y.y);
        }
        __syncthreads();
        const int n = min(256, Ta - t0);
        for (int j = g; j < n; j += G) acc += mag[j] * Phi[(int64_t)(t0 + j) * NTp + tau];
    }
    part[threadIdx.x] = acc;
    __syncthreads();
    if (g == 0 && tau < NT) {
        float s = 0.f;
        for (int q = 0; q < G; ++q) s += part[q * NTp + tau];
        S2[((b * n_alpha + alpha) * n1 + lam) * (int64_t)NT + tau] =
            mulog_out(s, mu2, mulog_inv(mu2, alpha * n1 + lam, eps));
    }
}

// ---------------------------------------------------------------------------
// Backward.
// ---------------------------------------------------------------------------

// Time scattering adjoint: gY2[t] = (sum_tau gS2[tau] Phi_alpha[t][tau]) y_t / max(|y_t|, eps)
// for t < Ta, zero for Ta <= t < Tp (rows lambda < n1).
__global__ void __launch_bounds__(256) k_ts_bwd(const float2* __restrict__ Y, int64_t y_bstride, int Tp, int Ta,
                                                const float* __restrict__ Phi, int NTp, int NT, int alpha,
                                                int n_alpha, const float* __restrict__ gS2, float2* __restrict__ gY,
                                                MuLogArg ml) {
    __shared__ float gs[128];
    const int lam = blockIdx.x, n1 = gridDim.x;
    const int64_t b = blockIdx.y;
    const int64_t so = ((b * n_alpha + alpha) * n1 + lam) * (int64_t)NT;
    const float* src = gS2 ? gS2 + so : nullptr;
    const float em = ml.mu2 ? ml.eps * ml.mu2[alpha * n1 + lam] : 0.f;
    for (int i = threadIdx.x; i < NTp; i += blockDim.x)
        gs[i] = (src && i < NT) ? mulog_cot(src[i], ml.mu2, em, ml.mu2 ? ml.o2[so + i] : 0.f) : 0.f;
    __syncthreads();
    const float2* row = Y + b * y_bstride + (int64_t)lam * Tp;
    float2* out = gY + b * y_bstride + (int64_t)lam * Tp;
    for (int t = threadIdx.x; t < Tp; t += blockDim.x) {
        float2 r = make_float2(0.f, 0.f);
        if (t < Ta) {
            const float* ph = Phi + (int64_t)t * NTp;
            float gu = 0.f;
            for (int tau = 0; tau < NT; ++tau) gu += gs[tau] * ph[tau];
            const float2 y = row[t];
            const float sc = gu / fmaxf(sqrtf(y.x * y.x + y.y * y.y), kEpsMod);
            r = make_float2(y.x * sc, y.y * sc);
        }
        out[t] = r;
    }
}

// Sum over each aligned group of `width` lanes (32 or 64), returned to every lane of
// the group: rotations within rows of 16 lanes (DPP), then swaps between rows, all
// in registers (a butterfly of shuffles takes five round trips through LDS).
__device__ __forceinline__ float group_sum(float a, int width) {
    a += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(a), 0x128, 0xF, 0xF, false));   // row_ror:8
    a += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(a), 0x124, 0xF, 0xF, false));   // row_ror:4
    a += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(a), 0x122, 0xF, 0xF, false));   // row_ror:2
    a += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(a), 0x121, 0xF, 0xF, false));   // row_ror:1
    const unsigned u = __float_as_uint(a);
    const auto r16 = __builtin_amdgcn_permlane16_swap(u, u, false, false);   // rows 0+1, 2+3
    a = __uint_as_float(r16[0]) + __uint_as_float(r16[1]);
    if (width > 32) {
        const unsigned v = __float_as_uint(a);
        const auto r32 = __builtin_amdgcn_permlane32_swap(v, v, false, false);
        a = __uint_as_float(r32[0]) + __uint_as_float(r32[1]);
    }
    return a;
}

// gV[b][alpha][theta][rowoff+l][tau] = sum_m PF_beta[m][l] gS2[b][alpha][beta][theta][m][tau]
// (adjoint of the frequency lowpass), or with avg = 0 (eq. (4)) the gS2 row
// itself; block n_beta zeroes the padding rows.
// Also writes, per (signal, alpha, spin, beta), the largest row sum over tau of
// |gV| (a bound used to scale the split backward contraction).
// Adjoint of the frequency lowpass: gV[l][tau] = sum_m PF[m][l] gS2[m][tau] (or
// gS2 itself without frequential averaging), with the per-row sums of |gV| whose
// maximum sets the split scale of the backward contraction.  The gS2 tile and,
// with stage_pf, PF are held in LDS; row sums are reduced across the lanes of a
// row before one LDS atomic per row segment.
__global__ void __launch_bounds__(256) k_s2_bwd(const float* __restrict__ gS2, const float* __restrict__ PFall,
                                                const int64_t* __restrict__ pfoff, const int* __restrict__ Lbv,
                                                const int* __restrict__ rowoffv, int n_beta, int NL, int NLo, int NT, int NTp,
                                                int Mh, int Mp, int n_alpha, int avg, int stage_pf,
                                                float* __restrict__ gV, float* __restrict__ gvmax, MuLogArg ml) {
    extern __shared__ float sm[];      // rowsum [Lb] | gS2 tile [NL][NT] | (stage_pf) PF [NL][Lb]
    // grid (n_beta + 1, 2 n_alpha, B): every temporal rate in one launch
    const int beta = blockIdx.x, th = blockIdx.y & 1, alpha = blockIdx.y >> 1;
    const int64_t b = blockIdx.z;
    float* g = gV + (((b * n_alpha + alpha) * 2 + th) * (int64_t)Mp) * NTp;
    if (beta == n_beta) {
        for (int e = threadIdx.x; e < (Mp - Mh) * NTp; e += blockDim.x) g[(int64_t)Mh * NTp + e] = 0.f;
        return;
    }
    const int Lb = Lbv[beta], ro = rowoffv[beta];
    float* rowsum = sm;
    float* st = sm + Lb;
    float* pf = st + NL * NT;
    const float* PF = PFall + pfoff[beta];
    const int64_t so = avg ? ((((b * n_alpha + alpha) * n_beta + beta) * 2 + th) * NLo) * (int64_t)NT
                           : ((b * n_alpha + alpha) * 2 * (int64_t)Mh + 2 * ro + th * Lb) * NT;
    const float* src = gS2 ? gS2 + so : nullptr;
    const float* osrc = ml.mu2 ? ml.o2 + so : nullptr;
    const float em = ml.mu2 ? ml.eps * ml.mu2[(alpha * n_beta + beta) * 2 + th] : 0.f;
    for (int l = threadIdx.x; l < Lb; l += blockDim.x) rowsum[l] = 0.f;
    if (src && avg) {
        for (int e = threadIdx.x; e < NLo * NT; e += blockDim.x)
            st[e] = mulog_cot(src[e], ml.mu2, em, osrc ? osrc[e] : 0.f);
        if (stage_pf)
            for (int e = threadIdx.x; e < NL * Lb; e += blockDim.x) pf[e] = PF[e];
    }
    __syncthreads();
    const int width = NTp < 64 ? NTp : 64;           // lanes of one row segment within a wave
    for (int e0 = 0; e0 < Lb * NTp; e0 += blockDim.x) {
        const int e = e0 + (int)threadIdx.x;
        const bool valid = e < Lb * NTp;
        const int l = e / NTp, tau = e - l * NTp;
        float acc = 0.f;
        if (valid && src && tau < NT) {
            if (avg) {
                const float* pc = stage_pf ? pf + l : PF + l;
                for (int m = 0; m < NLo; ++m) acc += pc[m * Lb] * st[m * NT + tau];
            } else {
                acc = mulog_cot(src[(int64_t)l * NT + tau], ml.mu2, em, osrc ? osrc[(int64_t)l * NT + tau] : 0.f);
            }
        }
        if (valid) g[(int64_t)(ro + l) * NTp + tau] = acc;
        float a = fabsf(acc);
        a = group_sum(a, width);
        if (valid && (tau & (width - 1)) == 0) atomicAdd(&rowsum[l], a);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        float m = 0.f;
        for (int l = 0; l < Lb; ++l) m = fmaxf(m, rowsum[l]);
        gvmax[((b * n_alpha + alpha) * 2 + th) * n_beta + beta] = m;
    }
}

// Adjoint of the frequency lowpass of eq. (3): gV[rowoff + l][tau] =
// sum_m PF_beta[m][l] gS2[m][tau] over the NLo output rows m, with the row sums
// over tau of |gV| whose maximum sets the split scale of the backward
// contraction.  One lane per row l: the gS2 tile (after the mu-log adjoint when
// set) sits in LDS and every lane reads the same element of it at a time (a
// broadcast), PF[m][l] comes from global memory with consecutive lanes on
// consecutive l, and each lane keeps TT outputs of its row in registers, stores
// them as 16-byte writes and sums their moduli itself.  grid (n_beta + 1,
// 2 n_alpha, B); block n_beta zeroes the padding rows Mh..Mp.
template <int TT>
__global__ void __launch_bounds__(256) k_s2_bwd_avg(const float* __restrict__ gS2, const float* __restrict__ PFall,
                                                    const int64_t* __restrict__ pfoff, const int* __restrict__ Lbv,
                                                    const int* __restrict__ rowoffv, int n_beta, int NLo, int NT,
                                                    int NTp, int Mh, int Mp, int n_alpha, float* __restrict__ gV,
                                                    float* __restrict__ gvmax, MuLogArg ml) {
    extern __shared__ __align__(16) float st[];      // gS2 tile [NLo][NT]
    __shared__ float red[256];
    const int beta = blockIdx.x, th = blockIdx.y & 1, alpha = blockIdx.y >> 1;
    const int64_t b = blockIdx.z;
    float* g = gV + (((b * n_alpha + alpha) * 2 + th) * (int64_t)Mp) * NTp;
    if (beta == n_beta) {
        for (int e = threadIdx.x; e < (Mp - Mh) * NTp; e += blockDim.x) g[(int64_t)Mh * NTp + e] = 0.f;
        return;
    }
    const int Lb = Lbv[beta], ro = rowoffv[beta];
    const float* PF = PFall + pfoff[beta];           // [NL][Lb]
    const int64_t so = ((((b * n_alpha + alpha) * n_beta + beta) * 2 + th) * NLo) * (int64_t)NT;
    const float* src = gS2 ? gS2 + so : nullptr;
    const float* osrc = ml.mu2 ? ml.o2 + so : nullptr;
    const float em = ml.mu2 ? ml.eps * ml.mu2[(alpha * n_beta + beta) * 2 + th] : 0.f;
    for (int e = threadIdx.x; e < NLo * NT; e += blockDim.x)
        st[e] = src ? mulog_cot(src[e], ml.mu2, em, osrc ? osrc[e] : 0.f) : 0.f;
    __syncthreads();
    float mx = 0.f;
    for (int l = threadIdx.x; l < Lb; l += blockDim.x) {
        float* grow = g + (int64_t)(ro + l) * NTp;
        float rs = 0.f;
        for (int t0 = 0; t0 < NTp; t0 += TT) {
            float acc[TT];
#pragma unroll
            for (int j = 0; j < TT; ++j) acc[j] = 0.f;
            if (t0 < NT) {
                if (NT - t0 >= TT) {
                    for (int m = 0; m < NLo; ++m) {
                        const float p = PF[(int64_t)m * Lb + l];
                        const float4* s4 = (const float4*)(st + m * NT + t0);
#pragma unroll
                        for (int q = 0; q < TT / 4; ++q) {
                            const float4 v = s4[q];
                            acc[4 * q] += p * v.x;
                            acc[4 * q + 1] += p * v.y;
                            acc[4 * q + 2] += p * v.z;
                            acc[4 * q + 3] += p * v.w;
                        }
                    }
                } else {
                    for (int m = 0; m < NLo; ++m) {
                        const float p = PF[(int64_t)m * Lb + l];
#pragma unroll
                        for (int j = 0; j < TT; ++j)
                            if (t0 + j < NT) acc[j] += p * st[m * NT + t0 + j];
                    }
                }
            }
            float4* o4 = (float4*)(grow + t0);
#pragma unroll
            for (int q = 0; q < TT / 4; ++q) {
                o4[q] = make_float4(acc[4 * q], acc[4 * q + 1], acc[4 * q + 2], acc[4 * q + 3]);
                rs += fabsf(acc[4 * q]) + fabsf(acc[4 * q + 1]) + fabsf(acc[4 * q + 2]) + fabsf(acc[4 * q + 3]);
            }
        }
        mx = fmaxf(mx, rs);
    }
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) gvmax[((b * n_alpha + alpha) * 2 + th) * n_beta + beta] = red[0];
}

// Recompute Z = W Y (both spins) on a 64 l x 64 t tile, gU = gV Phi^T (adjoint of
// the time lowpass), gZ = gU Z / max(|Z|, eps) (modulus adjoint), and store
// P = gZ_up + gZ_down and Q' = i (gZ_down - gZ_up), so that the adjoint of the
// contraction is gY = Wr^T P + Wi^T Q'.  Non-transposed orientation: C rows = l.
template <int NTB>
__global__ void __launch_bounds__(256) k_bwd_pq(const float2* __restrict__ Y, int64_t y_bstride, int Tp,
                                                const float2* __restrict__ Wt, int Mp, int Kp,
                                                const float* __restrict__ Phi, const float* __restrict__ gV,
                                                int64_t gv_bstride, float2* __restrict__ PQ) {
    constexpr int NTp = 32 * NTB;
    constexpr int LDG = NTp + 1;
    __shared__ float2 Ys[kKStep][kTileT];
    __shared__ float2 Ws[kKStep][kTileL];
    __shared__ float gVs[2][kTileL][LDG];
    __shared__ float Phs[kTileT][LDG];
    const int lt = blockIdx.x, tt = blockIdx.y;
    const int64_t b = blockIdx.z;
    const int l0 = lt * kTileL, t0 = tt * kTileT;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int h = lane >> 5, i32 = lane & 31;
    const int lw = (wave >> 1) * 32, twv = (wave & 1) * 32;
    const float2* Yb = Y + b * y_bstride;
    const float* gvb = gV + b * gv_bstride;
    for (int e = tid; e < kTileL * NTp; e += 256) {
        const int l = e / NTp, tau = e - l * NTp;
        gVs[0][l][tau] = gvb[(int64_t)(l0 + l) * NTp + tau];
        gVs[1][l][tau] = gvb[(int64_t)(Mp + l0 + l) * NTp + tau];
        Phs[l][tau] = Phi[(int64_t)(t0 + l) * NTp + tau];
    }
    floatx16 rr = zero16(), ri = zero16(), ir = zero16(), ii = zero16();
    for (int k0 = 0; k0 < Kp; k0 += kKStep) {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int f = tid + q * 256, row = f >> 5, c = (f & 31) * 2;
            *(float4*)&Ys[row][c] = *(const float4*)(Yb + (int64_t)(k0 + row) * Tp + t0 + c);
            *(float4*)&Ws[row][c] = *(const float4*)(Wt + (int64_t)(k0 + row) * Mp + l0 + c);
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < kKStep / 2; ++ks) {
            const float2 w = Ws[2 * ks + h][lw + i32];   // A: rows l
            const float2 y = Ys[2 * ks + h][twv + i32];  // B: columns t
            rr = mfma32(w.x, y.x, rr);
            ri = mfma32(w.x, y.y, ri);
            ir = mfma32(w.y, y.x, ir);
            ii = mfma32(w.y, y.y, ii);
        }
        __syncthreads();
    }
    floatx16 gu = zero16(), gd = zero16();
#pragma unroll
    for (int n = 0; n < NTB; ++n) {
#pragma unroll
        for (int sidx = 0; sidx < 16; ++sidx) {
            const int tau = n * 32 + 2 * sidx + h;
            const float p = Phs[twv + i32][tau];
            gu = mfma32(gVs[0][lw + i32][tau], p, gu);
            gd = mfma32(gVs[1][lw + i32][tau], p, gd);
        }
    }
    float2* Pp = PQ + b * (2 * (int64_t)Mp * Tp);
    float2* Qp = Pp + (int64_t)Mp * Tp;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const float ur = rr[r] - ii[r], ui = ri[r] + ir[r];
        const float dr = rr[r] + ii[r], di = ri[r] - ir[r];
        const float su = gu[r] / fmaxf(sqrtf(ur * ur + ui * ui), kEpsMod);
        const float sd = gd[r] / fmaxf(sqrtf(dr * dr + di * di), kEpsMod);
        const float gur = su * ur, gui = su * ui, gdr = sd * dr, gdi = sd * di;
        const int l = l0 + lw + crow(r, h), t = t0 + twv + i32;
        Pp[(int64_t)l * Tp + t] = make_float2(gur + gdr, gui + gdi);
        Qp[(int64_t)l * Tp + t] = make_float2(-(gdi - gui), gdr - gur);
    }
}

// gY[i][t] = sum_l Wr[l][i] P[l][t] + Wi[l][i] Q'[l][t]  (adjoint of the contraction)
__global__ void __launch_bounds__(256) k_bwd_gy(const float2* __restrict__ PQ, int Tp, const float2* __restrict__ Wl,
                                                int Mp, int Kp, float2* __restrict__ gY, int64_t gy_bstride) {
    __shared__ float As[kKStep][kTileL];
    __shared__ float2 Bs[kKStep][kTileT];
    const int it = blockIdx.x, tt = blockIdx.y;
    const int64_t b = blockIdx.z;
    const int i0 = it * 64, t0 = tt * kTileT;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int h = lane >> 5, i32 = lane & 31;
    const int iw = (wave >> 1) * 32, twv = (wave & 1) * 32;
    const float2* PQb = PQ + b * (2 * (int64_t)Mp * Tp);
    floatx16 are = zero16(), aim = zero16();
    for (int plane = 0; plane < 2; ++plane) {
        const float2* Bsrc = PQb + (int64_t)plane * Mp * Tp;
        for (int k0 = 0; k0 < Mp; k0 += kKStep) {
            for (int e = tid; e < kKStep * 64; e += 256) {
                const int row = e >> 6, c = e & 63;
                float v = 0.f;
                if (i0 + c < Kp) {
                    const float2 w = Wl[(int64_t)(k0 + row) * Kp + i0 + c];
                    v = plane ? w.y : w.x;
                }
                As[row][c] = v;
            }
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int f = tid + q * 256, row = f >> 5, c = (f & 31) * 2;
                *(float4*)&Bs[row][c] = *(const float4*)(Bsrc + (int64_t)(k0 + row) * Tp + t0 + c);
            }
            __syncthreads();
#pragma unroll
            for (int ks = 0; ks < kKStep / 2; ++ks) {
                const float a = As[2 * ks + h][iw + i32];
                const float2 v = Bs[2 * ks + h][twv + i32];
                are = mfma32(a, v.x, are);
                aim = mfma32(a, v.y, aim);
            }
            __syncthreads();
        }
    }
    float2* o = gY + b * gy_bstride;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int i = i0 + iw + crow(r, h), t = t0 + twv + i32;
        if (i < Kp) o[(int64_t)i * Tp + t] = make_float2(are[r], aim[r]);
    }
}

// Adjoint of the second order and of S1 for one scalogram row: accumulates the
// Hermitian half-spectrum of gX,
//   H[m] = 1/2 sum_alpha psi_hat_alpha[m] G_alpha[m mod Ta] (real part at m = 0, NX/2)
//        + phi_hat[m] G1[m mod NT],
// G_alpha = FFT of gY2 rows (done beforehand), G1 = FFT of gS1 row, then the
// real inverse FFT gives gX[b][lambda][0..NX) (scaled 1/NX).
__global__ void __launch_bounds__(1024, 8) k_scal_bwd_a(const float2* __restrict__ G, int64_t y_bstride,
                                                    const int64_t* __restrict__ yoff, const int* __restrict__ Tpv,
                                                    const int* __restrict__ Tav, const float* __restrict__ psi2,
                                                    const int* __restrict__ band2, const int64_t* __restrict__ off2,
                                                    int n_alpha, const float* __restrict__ gS1,
                                                    const float* __restrict__ phiX, int Mphi, int logNT, int logNX,
                                                    float* __restrict__ gX, const float2* __restrict__ tw, int tw_log,
                                                    MuLogArg ml, const float2* __restrict__ gYphi, int Tphi) {
    extern __shared__ float2 s[];
    const int lam = blockIdx.x, n1 = gridDim.x;
    const int64_t b = blockIdx.y;
    const int NX = 1 << logNX, H = NX >> 1, NT = 1 << logNT;
    float2* g1 = s + lpad(H) + 1;
    const float em = ml.mu1 ? ml.eps * ml.mu1[0] : 0.f;
    for (int t = threadIdx.x; t < NT; t += blockDim.x) {
        const int64_t i = (b * n1 + lam) * NT + t;
        float g = gS1 ? mulog_cot(gS1[i], ml.mu1, em, ml.mu1 ? ml.o1[i] : 0.f) : 0.f;
        if (gYphi) g += gYphi[b * y_bstride + (int64_t)lam * Tphi + t].x;   // Re of phi_T's second-order rows
        g1[lpad(t)] = make_float2(g, 0.f);
    }
    __syncthreads();
    lds_fft<16>(g1, logNT, 1, NT, tw, tw_log, false);
    // bins m = m0 + tid + q blockDim, q < 5: the temporal rates in the outer loop,
    // so that a rate's loads for all of a thread's bins issue together
    for (int m0 = 0; m0 <= H; m0 += 5 * (int)blockDim.x) {
        float2 c[5];
#pragma unroll
        for (int q = 0; q < 5; ++q) c[q] = make_float2(0.f, 0.f);
        for (int a = 0; a < n_alpha; ++a) {
            const int lo = band2[2 * a], hi = band2[2 * a + 1];
            const float* pa = psi2 + off2[a] - lo;
            const float2* ga = G + b * y_bstride + yoff[a] + (int64_t)lam * Tpv[a];
            const int tmask = Tav[a] - 1;
#pragma unroll
            for (int q = 0; q < 5; ++q) {
                const int m = m0 + threadIdx.x + q * blockDim.x;
                if (m >= lo && m <= hi) {
                    const float g = pa[m];
                    const float2 v = ga[m & tmask];
                    c[q].x += g * v.x;
                    c[q].y += g * v.y;
                }
            }
        }
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            const int m = m0 + threadIdx.x + q * blockDim.x;
            if (m > H) continue;
            float2 hm = (m == 0 || m == H) ? make_float2(c[q].x, 0.f) : cscale(c[q], 0.5f);
            if (m <= Mphi) {
                const float2 v = g1[lpad(m & (NT - 1))];
                hm.x += phiX[m] * v.x;
                hm.y += phiX[m] * v.y;
            }
            s[lpad(m)] = hm;
        }
    }
    __syncthreads();
    const int tws = tw_log - logNX;
    for (int k = threadIdx.x; k <= H / 2; k += blockDim.x) {
        const float2 p = s[lpad(k)], q = s[lpad(H - k)];
        auto pk = [&](float2 pp, float2 qq, int kk) {
            const float2 S = make_float2(pp.x + qq.x, pp.y - qq.y);
            const float2 D = make_float2(pp.x - qq.x, pp.y + qq.y);
            const float2 wD = cmulc(D, tw[kk << tws]);
            return make_float2(S.x - wD.y, S.y + wD.x);
        };
        const float2 zk = pk(p, q, k);
        float2 zn = make_float2(0.f, 0.f);
        const bool two = k > 0 && H - k != k;
        if (two) zn = pk(q, p, H - k);
        s[lpad(k)] = zk;
        if (two) s[lpad(H - k)] = zn;
    }
    __syncthreads();
    if (logNX > 1) lds_fft<16>(s, logNX - 1, 1, H, tw, tw_log, true);
    float2* o = (float2*)(gX + (b * n1 + lam) * (int64_t)NX);
    const float sc = 1.f / (float)NX;
    for (int k = threadIdx.x; k < H; k += blockDim.x) o[k] = cscale(s[lpad(k)], sc);
}

// Adjoint of the modulus and of the first-order filter for one row: recompute the
// scalogram-rate filtered signal y, gY1 = gX y / max(|y|, eps), and its FFT
// (the spectrum that the decimation adjoint replicates): g1[b][lambda][0..NX).
__global__ void __launch_bounds__(1024, 8) k_scal_bwd_b(const float2* __restrict__ xh, int64_t xh_pitch,
                                                    const float* __restrict__ psi1, const int* __restrict__ band1,
                                                    const int64_t* __restrict__ off1, const float* __restrict__ gX,
                                                    float2* __restrict__ g1, int logNX, float invN,
                                                    const float2* __restrict__ tw, int tw_log) {
    extern __shared__ float2 s[];
    const int lam = blockIdx.x, n1 = gridDim.x;
    const int64_t b = blockIdx.y;
    const int NX = 1 << logNX;
    fold_band(s, xh + b * xh_pitch, psi1 + off1[lam], band1[2 * lam], band1[2 * lam + 1], logNX);
    __syncthreads();
    lds_fft<16>(s, logNX, 1, NX, tw, tw_log, true);
    const float* gx = gX + (b * n1 + lam) * (int64_t)NX;
    for (int n = threadIdx.x; n < NX; n += blockDim.x) {
        const float2 y = cscale(s[lpad(n)], invN);
        const float sc = gx[n] * __builtin_amdgcn_rcpf(fmaxf(__builtin_amdgcn_sqrtf(y.x * y.x + y.y * y.y), kEpsMod));
        s[lpad(n)] = cscale(y, sc);
    }
    __syncthreads();
    lds_fft<16>(s, logNX, 1, NX, tw, tw_log, false);
    float2* o = g1 + (b * n1 + lam) * (int64_t)NX;
    for (int n = threadIdx.x; n < NX; n += blockDim.x) o[n] = s[lpad(n)];
}

// Band-owned accumulation of the first-order adjoint over lambda for bins
// 0..N/2: K[m] = sum_lambda psi_hat_lambda[m] g1_lambda[m mod NX]; writes the
// Hermitian half-spectrum of gx (K/2, real part at m = 0 and N/2).
__global__ void __launch_bounds__(256) k_band_accum(const float2* __restrict__ g1, int n1, int logNX,
                                                    const float* __restrict__ psi1, const int* __restrict__ band1,
                                                    const int64_t* __restrict__ off1,
                                                    const int* __restrict__ lam_range, int Hn,
                                                    float2* __restrict__ gxh, int64_t pitch) {
    const int r = blockIdx.x;
    const int64_t b = blockIdx.y;
    const int m = r * 256 + threadIdx.x;
    if (m > Hn) return;
    const int la = lam_range[2 * r], lb = lam_range[2 * r + 1];
    const int mask = (1 << logNX) - 1;
    float2 k = make_float2(0.f, 0.f);
    for (int lam = la; lam <= lb; ++lam) {
        const int lo = band1[2 * lam], hi = band1[2 * lam + 1];
        if (m < lo || m > hi) continue;
        const float g = psi1[off1[lam] + m - lo];
        const float2 v = g1[(b * n1 + lam) * (int64_t)(mask + 1) + (m & mask)];
        k.x += g * v.x;
        k.y += g * v.y;
    }
    gxh[b * pitch + m] = (m == 0 || m == Hn) ? make_float2(k.x, 0.f) : cscale(k, 0.5f);
}

// ---------------------------------------------------------------------------
// Launch helpers
// ---------------------------------------------------------------------------
// LDS of the frequency lowpass and its adjoint: V tile (or row sums and the gS2
// tile), and the PF matrix when all of it fits kS2LdsCap (then held in LDS)
constexpr size_t kS2LdsCap = 96 * 1024;
static size_t s2_bwd_floats(const Shapes& s, bool stage) {
    return (size_t)s.L + (size_t)s.NL * s.NT + (stage ? (size_t)s.NL * s.L : 0);
}
static int s2_bwd_stage(const Shapes& s) { return sizeof(float) * s2_bwd_floats(s, true) <= kS2LdsCap ? 1 : 0; }
static size_t s2_bwd_lds(const Shapes& s) { return sizeof(float) * s2_bwd_floats(s, s2_bwd_stage(s)); }

static bool g_attr_done = false;

int setup_kernel_attributes() {
    if (g_attr_done) return JTFS_OK;
    const int lds = kMaxDynLds;
    const void* ks[] = {(const void*)k_fft_cols_t<float2, float2>, (const void*)k_fft_cols_t<float2, double2>,
                        (const void*)k_fft_cols_t<double2, double2>, (const void*)k_scalogram, (const void*)k_s1,
                        (const void*)k_s2_bwd, (const void*)k_s2_bwd_avg<16>, (const void*)k_s2_bwd_avg<32>,
                        (const void*)k_second_order, (const void*)k_scal_bwd_a, (const void*)k_scal_bwd_b};
    for (const void* k : ks) {
        hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
        if (e != hipSuccess) {
            set_error(std::string("hipFuncSetAttribute: ") + hipGetErrorString(e));
            return JTFS_EHIP;
        }
    }
    int rs = split_attributes();
    if (rs != JTFS_OK) return rs;
    rs = reg_attributes();
    if (rs != JTFS_OK) return rs;
    g_attr_done = true;
    return JTFS_OK;
}

// FFT of B rows of length n = 2^logn: in (row pitch ip) -> out (row pitch op),
// through scratch (pitch n) when n exceeds one LDS transform (four-step).
static void fft_rows(const float2* in, int64_t ip, float2* out, int64_t op, float2* scratch, int logn, int64_t B,
                     bool inv, float scale, const jtfs_plan* P, hipStream_t st) {
    if (logn <= kLdsFftMax) {
        const int logC = logn >= 12 ? 0 : 12 - logn;       // rows per workgroup
        const size_t lds = (size_t)(1 << logC) * (lpad_len(1 << logn) + 1) * sizeof(float2);
        hipLaunchKernelGGL((k_fft_cols), dim3((unsigned)((B + (1 << logC) - 1) >> logC)), dim3(1024), lds, st, in, out,
                           logn, (int)B, logC, (int64_t)0, ip, (int64_t)1, (int64_t)0, op, (int64_t)1, 0, P->tw,
                           P->tw_log, (int)inv, scale);
        return;
    }
    // n = P Q: input index a + P*bq (a < P columns, bq < Q), output k_b + Q*k_a
    const int lq = (logn + 1) / 2, lp = logn - lq;
    const int64_t Pn = (int64_t)1 << lp, Qn = (int64_t)1 << lq;
    int logC = std::max(0, 12 - lq);
    logC = std::min(logC, lp);
    size_t lds = (size_t)(1 << logC) * (lpad_len(Qn) + 1) * sizeof(float2);
    hipLaunchKernelGGL((k_fft_cols), dim3((unsigned)(Pn >> logC), (unsigned)B), dim3(1024), lds, st, in, scratch, lq,
                       (int)Pn, logC, ip, (int64_t)1, Pn, (int64_t)1 << logn, Qn, (int64_t)1, logn, P->tw, P->tw_log,
                       (int)inv, 1.0f);
    logC = std::min(std::max(0, 12 - lp), lq);
    lds = (size_t)(1 << logC) * (lpad_len(Pn) + 1) * sizeof(float2);
    hipLaunchKernelGGL((k_fft_cols), dim3((unsigned)(Qn >> logC), (unsigned)B), dim3(1024), lds, st, scratch, out, lp,
                       (int)Qn, logC, (int64_t)1 << logn, (int64_t)1, Qn, op, (int64_t)1, Qn, 0, P->tw, P->tw_log,
                       (int)inv, scale);
}

// Real FFT of the B input rows (N samples) in FP64: the complex FFT of the N/2
// interleaved pairs (one LDS transform up to 2^13 points, four-step above, the
// double-precision rows being twice as large), then the real-spectrum
// post-pass, which rounds each bin once to FP32.  Every later stage works on
// bands of x_hat, so the only transform that mixes all bands keeps its error
// below FP32 rounding of each bin (not of the whole spectrum).
static void input_fft64(const float* x, int64_t B, float2* xh, int64_t xh_pitch, double2* scratch, double2* z,
                        const jtfs_plan* P, hipStream_t st) {
    const int logn = P->s.logN - 1;
    const int64_t H = (int64_t)1 << logn;
    const float2* in = (const float2*)x;
    if (logn <= 13) {
        const int logC = logn >= 12 ? 0 : 12 - logn;
        const size_t lds = (size_t)(1 << logC) * (lpad_len(H) + 1) * sizeof(double2);
        hipLaunchKernelGGL((k_fft_cols_t<float2, double2>), dim3((unsigned)((B + (1 << logC) - 1) >> logC)), dim3(1024),
                           lds, st, in, z, logn, (int)B, logC, (int64_t)0, H, (int64_t)1, (int64_t)0, H, (int64_t)1, 0,
                           P->tw64, P->tw_log, 0, 1.0);
    } else {
        const int lq = (logn + 1) / 2, lp = logn - lq;
        const int64_t Pn = (int64_t)1 << lp, Qn = (int64_t)1 << lq;
        int logC = std::min(std::max(0, 12 - lq), lp);
        size_t lds = (size_t)(1 << logC) * (lpad_len(Qn) + 1) * sizeof(double2);
        hipLaunchKernelGGL((k_fft_cols_t<float2, double2>), dim3((unsigned)(Pn >> logC), (unsigned)B), dim3(1024), lds,
                           st, in, scratch, lq, (int)Pn, logC, H, (int64_t)1, Pn, H, Qn, (int64_t)1, logn, P->tw64,
                           P->tw_log, 0, 1.0);
        logC = std::min(std::max(0, 12 - lp), lq);
        lds = (size_t)(1 << logC) * (lpad_len(Pn) + 1) * sizeof(double2);
        hipLaunchKernelGGL((k_fft_cols_t<double2, double2>), dim3((unsigned)(Qn >> logC), (unsigned)B), dim3(1024), lds,
                           st, scratch, z, lp, (int)Qn, logC, H, (int64_t)1, Qn, H, (int64_t)1, Qn, 0, P->tw64,
                           P->tw_log, 0, 1.0);
    }
    hipLaunchKernelGGL(k_rfft_post64, dim3((unsigned)((H / 2 + 1 + 255) / 256), (unsigned)B), dim3(256), 0, st, z, H,
                       xh, xh_pitch, P->s.logN, P->tw64, P->tw_log);
}

}  // namespace jtfs

using namespace jtfs;

#define LAUNCHCHK(what)                                                                  \
    do {                                                                                 \
        hipError_t e_ = hipGetLastError();                                               \
        if (e_ != hipSuccess) {                                                          \
            set_error(std::string(what) + ": " + hipGetErrorString(e_));                 \
            return JTFS_EHIP;                                                            \
        }                                                                                \
    } while (0)

// Whether the backward of the plan's contraction mode runs on the split kernels
// (else the FP32 pair, which keeps P and Q' in the workspace).
static bool split_backward(const jtfs_plan* P) {
    if (P->contraction == JTFS_CONTRACTION_FP32 || P->s.tscat) return false;
    return P->contraction == JTFS_CONTRACTION_SPLIT_F16_PHASE ? P->split_bwdp_ok : P->split_bwd_ok;
}

// Workspace of a plan in its current contraction mode.
static Workspace plan_layout(const jtfs_plan* P, int64_t B) {
    const bool split = P->contraction != JTFS_CONTRACTION_FP32;          // SPLIT_F16 or SPLIT_F16_PHASE
    const bool phase = P->contraction == JTFS_CONTRACTION_SPLIT_F16_PHASE && !P->s.tscat;
    return layout(P->s, B, split, !(split && split_backward(P)), phase);
}

// forward_only: a forward needs the leading part of the layout only
static int check_common(const jtfs_plan* P, int64_t B, void* ws, size_t ws_bytes, bool forward_only) {
    if (!P) { set_error("null plan"); return JTFS_EINVAL; }
    if (B < 1 || B > 65535) { set_error("B must lie in [1, 65535]"); return JTFS_ESHAPE; }   // grid y / z
    if (!ws) { set_error("null workspace"); return JTFS_EINVAL; }
    const Workspace w = plan_layout(P, B);
    if (ws_bytes < (forward_only ? w.fwd_total : w.total)) { set_error("workspace too small"); return JTFS_EWORKSPACE; }
    return JTFS_OK;
}

extern "C" int jtfs_workspace_size(const jtfs_plan* P, int64_t B, size_t* bytes) {
    if (!P || !bytes) { set_error("null pointer"); return JTFS_EINVAL; }
    if (B < 1) { set_error("B must be >= 1"); return JTFS_ESHAPE; }
    *bytes = plan_layout(P, B).total;
    return JTFS_OK;
}

extern "C" int jtfs_forward_workspace_size(const jtfs_plan* P, int64_t B, size_t* bytes) {
    if (!P || !bytes) { set_error("null pointer"); return JTFS_EINVAL; }
    if (B < 1) { set_error("B must be >= 1"); return JTFS_ESHAPE; }
    *bytes = plan_layout(P, B).fwd_total;
    return JTFS_OK;
}

namespace {

// x -> x_hat -> X_hat -> S1, Y2
int forward_front(const jtfs_plan* P, const float* x, int64_t B, float* s1, char* base, const Workspace& w,
                  const MuLogArg& ml, hipStream_t st) {
    const Shapes& s = P->s;
    float2* xh = (float2*)(base + w.xh);
    float2* Xh = (float2*)(base + w.Xh);
    float2* Y2 = (float2*)(base + w.Y2);
    JTFS_TIMED(JTFS_STAGE_INPUT_FFT, st, input_fft64(x, B, xh, w.xh_pitch, (double2*)(base + w.tmp64),
                                                     (double2*)(base + w.z64), P, st));
    LAUNCHCHK("input FFT");
    if (use_reg_rows(s.logNX, P->tune.reg_scalogram)) {
        JTFS_TIMED(JTFS_STAGE_SCALOGRAM, st, launch_scalogram_r(P, xh, w.xh_pitch, Xh, w.Xh_pitch, B, st));
    } else {
        JTFS_TIMED(JTFS_STAGE_SCALOGRAM, st, hipLaunchKernelGGL(k_scalogram, dim3(s.n1, (unsigned)B), dim3(1024), sizeof(float2) * lpad_len(s.NX), st, xh, w.xh_pitch,
                       P->psi1, P->band1, P->off1, Xh, w.Xh_pitch, s.logNX, 1.0f / (float)s.N, P->tw, P->tw_log));
    }
    LAUNCHCHK("scalogram");
    if (s1 || s.complete) {
        // with the lowpass pairs the same launch fills the second-order rows of phi_T
        const int logNT = s.logN - s.logT;
        const int aphi = s.n_alpha_psi;
        float2* Yphi = s.complete ? Y2 + s.yoff[aphi] : nullptr;
        JTFS_TIMED(JTFS_STAGE_S1, st, hipLaunchKernelGGL(k_s1, dim3(s.complete ? s.Kp : s.n1, (unsigned)B), dim3(256), sizeof(float2) * lpad_len(s.NT), st, Xh, w.Xh_pitch,
                           P->phiX, s.Mphi, s.logNX, logNT, 1.0f / (float)s.NX, s1, P->tw, P->tw_log, ml.mu1, ml.eps,
                           s.n1, Yphi, (int64_t)s.Kp * s.sumTp, s.complete ? s.Tp[aphi] : 0,
                           (float*)(base + w.rowmax), aphi, s.n_alpha, s.Kp));
        LAUNCHCHK("first-order lowpass");
    }
    for (int a = 0; a < s.n_alpha_psi; ++a) {
        const int logTa = s.logNX - s.k2[a];
        // rows of 2^11 to 2^13 points take the register-resident transform with the same choice as 2^14
        if (use_reg_rows(logTa, P->tune.reg_second) ||
            (logTa >= kRegMinLogRows - 3 && logTa < kRegMinLogRows && P->tune.reg_second)) {
            JTFS_TIMED(JTFS_STAGE_SECOND_ORDER, st,
                       launch_second_order_r(P, a, Xh, w.Xh_pitch, Y2, (float*)(base + w.rowmax), B, st));
            LAUNCHCHK("second order");
            continue;
        }
        // <= 64 rows (row-maximum slots), and fewer where the grid would hold under ~1024 workgroups
        const int fill = (int)std::max<int64_t>(1, ((int64_t)s.Kp * B + 1023) / 1024);
        const int rows = std::min({64, std::max(1, (1 << lds_batch_log(P->tune)) >> logTa), fill});
        const size_t lds = sizeof(float2) * rows * lpad_len(s.Ta[a]);
        const Family& f2 = s.f2;
        // packed second-order spectrum of alpha: the plan's device table at its offset
        JTFS_TIMED(JTFS_STAGE_SECOND_ORDER, st, hipLaunchKernelGGL(k_second_order, dim3((unsigned)((s.Kp + rows - 1) / rows), (unsigned)B), dim3(1024), lds, st,
                           Xh, w.Xh_pitch, s.n1, P->psi2 + f2.off[a], f2.lo[a], f2.hi[a], logTa, s.Tp[a], rows, s.Kp,
                           Y2 + s.yoff[a], (int64_t)s.Kp * s.sumTp, 1.0f / (float)s.NX, P->tw, P->tw_log,
                           (float*)(base + w.rowmax), a, s.n_alpha));
        LAUNCHCHK("second order");
    }
    return JTFS_OK;
}

int forward_impl(const jtfs_plan* P, const float* x, int64_t B, float* s1, float* s2, void* ws, size_t ws_bytes,
                 const MuLogArg& ml, hipStream_t st) {
    int rc = check_common(P, B, ws, ws_bytes, true);
    if (rc != JTFS_OK) return rc;
    if (!x || !s1 || !s2) { set_error("null pointer"); return JTFS_EINVAL; }
    const Shapes& s = P->s;
    const Workspace w = plan_layout(P, B);
    char* base = (char*)ws;
    rc = forward_front(P, x, B, s1, base, w, ml, st);
    if (rc != JTFS_OK) return rc;
    float2* Y2 = (float2*)(base + w.Y2);
    float* Vp = (float*)(base + w.Vp);
    const int nlt = s.Mp / kTileL;
    for (int a = 0; a < s.n_alpha && s.tscat; ++a) {
        JTFS_TIMED(JTFS_STAGE_FREQ_FWD, st, hipLaunchKernelGGL(k_ts_out, dim3(s.n1, (unsigned)B), dim3(256), 0, st, Y2 + s.yoff[a],
                           (int64_t)s.Kp * s.sumTp, s.Tp[a], s.Ta[a], P->Phi + s.phioff[a], s.NTp, s.NT, a,
                           s.n_alpha, s2, ml.mu2, ml.eps));
        LAUNCHCHK("time-scattering lowpass");
    }
    const bool split = P->contraction != JTFS_CONTRACTION_FP32 && !s.tscat;
    unsigned* phase = P->contraction == JTFS_CONTRACTION_SPLIT_F16_PHASE && !s.tscat ? (unsigned*)(base + w.phase) : nullptr;
    for (int a = 0; a < s.n_alpha && split; ++a) {
        unsigned short* Yh = (unsigned short*)(base + w.Yh);
        float* ysc = (float*)(base + w.yscale);
        JTFS_TIMED(JTFS_STAGE_OPERAND_SPLIT, st,
                   rc = launch_ysplit(P, a, Y2, (const float*)(base + w.rowmax), Yh, ysc, B, st));
        if (rc != JTFS_OK) { set_error("operand split kernel failed"); return rc; }
        JTFS_TIMED(JTFS_STAGE_FREQ_FWD, st,
                   rc = launch_freq_fwd_split(P, a, Yh, ysc, Vp, w.vp_bstride, phase, w.ph_bstride, B, st));
        if (rc != JTFS_OK) { if (rc == JTFS_EHIP) set_error("split contraction launch failed"); return rc; }
    }
    for (int a = 0; a < s.n_alpha && !split && !s.tscat; ++a) {
        dim3 grid(nlt, s.nch[a], (unsigned)B);
        const int slot0 = (int)s.vchoff[a] * 2;
        const float2* Ya = Y2 + s.yoff[a];
        const float* Ph = P->Phi + s.phioff[a];
        const int64_t yb = (int64_t)s.Kp * s.sumTp;
        {
        TimedLaunch tl_fwd(JTFS_STAGE_FREQ_FWD, st);
        switch (s.NTp / 32) {
            case 1: hipLaunchKernelGGL(k_freq_fwd<1>, grid, dim3(256), 0, st, Ya, yb, s.Tp[a], s.chunk[a], P->Wt, s.Mp, s.Kp, Ph, Vp, w.vp_bstride, slot0, nlt); break;
            case 2: hipLaunchKernelGGL(k_freq_fwd<2>, grid, dim3(256), 0, st, Ya, yb, s.Tp[a], s.chunk[a], P->Wt, s.Mp, s.Kp, Ph, Vp, w.vp_bstride, slot0, nlt); break;
            case 4: hipLaunchKernelGGL(k_freq_fwd<4>, grid, dim3(256), 0, st, Ya, yb, s.Tp[a], s.chunk[a], P->Wt, s.Mp, s.Kp, Ph, Vp, w.vp_bstride, slot0, nlt); break;
            default: set_error("unsupported N/T"); return JTFS_ENOTSUP;
        }
        LAUNCHCHK("frequential contraction");
        }
    }
    if (!s.tscat) {
        // every temporal rate in one launch; the FP32 contraction writes two partial
        // slots per t-chunk (both halves of its row tile), the split one one
        const int mult = split ? 1 : 2;
        const dim3 grid((unsigned)s.n_beta, (unsigned)(2 * s.n_alpha), (unsigned)B);
        if (s.avg_fr) {
            auto k = s.NT <= 16 ? k_s2_out<16> : k_s2_out<32>;
            JTFS_TIMED(JTFS_STAGE_FREQ_LOWPASS, st, hipLaunchKernelGGL(k, grid, dim3(256), 0, st, Vp, w.vp_bstride, P->d_vchoff,
                               P->d_nch, mult, nlt, s.NTp, s.NT, P->PFt, P->d_pfoff, P->d_Lb, P->d_rowoff, s.NL, s.NLo, s.n_alpha, s2,
                               ml.mu2, ml.eps));
        } else {
            JTFS_TIMED(JTFS_STAGE_FREQ_LOWPASS, st, hipLaunchKernelGGL(k_v_out, grid, dim3(256), 0, st, Vp, w.vp_bstride, P->d_vchoff,
                               P->d_nch, mult, nlt, s.NTp, s.NT, P->d_Lb, P->d_rowoff, s.Mh, s.n_alpha, s2,
                               ml.mu2, ml.eps));
        }
        LAUNCHCHK("frequency lowpass");
    }
    return JTFS_OK;
}

}  // namespace

extern "C" int jtfs_forward(const jtfs_plan* P, const float* x, int64_t B, float* s1, float* s2, void* ws,
                            size_t ws_bytes, hipStream_t st) {
    return forward_impl(P, x, B, s1, s2, ws, ws_bytes, MuLogArg{}, st);
}

// forward FFT of every gY2 row of alpha (length T_alpha, rows lambda < n1), in place
static int gy2_row_fft(const jtfs_plan* P, int a, float2* gY2, int64_t yb, int64_t B, hipStream_t st) {
    const Shapes& s = P->s;
    if (a >= s.n_alpha_psi) return JTFS_OK;      // phi_T's rows go back through the S1 adjoint untransformed
    const int logTa = s.logNX - s.k2[a];
    const int lb = lds_batch_log(P->tune);
    const int logC = logTa >= lb ? 0 : lb - logTa;
    const size_t lds = (size_t)(1 << logC) * (lpad_len(s.Ta[a]) + 1) * sizeof(float2);
    // rows of 2^11 to 2^13 points take the register-resident transform with the same choice as 2^14
    if (use_reg_rows(logTa, P->tune.reg_rowfft) ||
        (logTa >= kRegMinLogRows - 3 && logTa < kRegMinLogRows && P->tune.reg_rowfft)) {
        JTFS_TIMED(JTFS_STAGE_SECOND_ADJ_FFT, st,
                   launch_rowfft_r(P, gY2 + s.yoff[a], yb, (int64_t)s.Tp[a], s.n1, logTa, B, st));
    } else {
        JTFS_TIMED(JTFS_STAGE_SECOND_ADJ_FFT, st, hipLaunchKernelGGL((k_fft_cols), dim3((unsigned)((s.n1 + (1 << logC) - 1) >> logC), (unsigned)B), dim3(1024), lds,
                       st, gY2 + s.yoff[a], gY2 + s.yoff[a], logTa, s.n1, logC, yb, (int64_t)s.Tp[a], (int64_t)1,
                       yb, (int64_t)s.Tp[a], (int64_t)1, 0, P->tw, P->tw_log, 0, 1.0f));
    }
    LAUNCHCHK("second-order adjoint FFT");
    return JTFS_OK;
}

namespace {

int backward_impl(const jtfs_plan* P, const float* x, const float* gs1, const float* gs2, float* gx, int64_t B,
                  void* ws, size_t ws_bytes, uint32_t flags, const MuLogArg& ml, hipStream_t st) {
    int rc = check_common(P, B, ws, ws_bytes, false);
    if (rc != JTFS_OK) return rc;
    if (!x || !gx) { set_error("null pointer"); return JTFS_EINVAL; }
    const Shapes& s = P->s;
    const Workspace w = plan_layout(P, B);
    char* base = (char*)ws;
    if (!(flags & JTFS_BWD_REUSE_FORWARD)) {
        rc = forward_front(P, x, B, nullptr, base, w, MuLogArg{}, st);
        if (rc != JTFS_OK) return rc;
    }
    float2* xh = (float2*)(base + w.xh);
    float2* tmp = (float2*)(base + w.tmp);
    float2* Y2 = (float2*)(base + w.Y2);
    float* gV = (float*)(base + w.gV);
    float2* PQ = (float2*)(base + w.PQ);
    float2* gY2 = (float2*)(base + w.gY2);
    float* gX = (float*)(base + w.gX);
    float2* g1 = (float2*)(base + w.g1);
    float2* gxh = (float2*)(base + w.gxh);
    const int64_t yb = (int64_t)s.Kp * s.sumTp;
    const int nlt = s.Mp / kTileL;
    // time scattering: the lowpass and modulus adjoints give gY2 directly
    for (int a = 0; a < s.n_alpha && s.tscat; ++a) {
        JTFS_TIMED(JTFS_STAGE_LOWPASS_ADJ, st, hipLaunchKernelGGL(k_ts_bwd, dim3(s.n1, (unsigned)B), dim3(256), 0, st, Y2 + s.yoff[a],
                           yb, s.Tp[a], s.Ta[a], P->Phi + s.phioff[a], s.NTp, s.NT, a, s.n_alpha, gs2,
                           gY2 + s.yoff[a], ml));
        LAUNCHCHK("time-scattering adjoint");
        rc = gy2_row_fft(P, a, gY2, yb, B, st);
        if (rc != JTFS_OK) return rc;
    }
    if (!s.tscat) {
        // every temporal rate in one launch
        const dim3 grid(s.n_beta + 1, 2 * s.n_alpha, (unsigned)B);
        if (s.avg_fr) {
            auto k = s.NTp % 32 == 0 && s.NT >= 32 ? k_s2_bwd_avg<32> : k_s2_bwd_avg<16>;
            JTFS_TIMED(JTFS_STAGE_LOWPASS_ADJ, st, hipLaunchKernelGGL(k, grid, dim3(256), sizeof(float) * s.NLo * s.NT, st, gs2,
                               P->PF, P->d_pfoff, P->d_Lb, P->d_rowoff, s.n_beta, s.NLo, s.NT, s.NTp, s.Mh, s.Mp,
                               s.n_alpha, gV, (float*)(base + w.gvmax), ml));
        } else {
            JTFS_TIMED(JTFS_STAGE_LOWPASS_ADJ, st, hipLaunchKernelGGL(k_s2_bwd, grid, dim3(256), s2_bwd_lds(s), st, gs2, P->PF, P->d_pfoff, P->d_Lb,
                               P->d_rowoff, s.n_beta, s.NL, s.NLo, s.NT, s.NTp, s.Mh, s.Mp, s.n_alpha, (int)s.avg_fr,
                               s2_bwd_stage(s), gV, (float*)(base + w.gvmax), ml));
        }
        LAUNCHCHK("frequency lowpass adjoint");
    }
    const bool split = split_backward(P);
    const bool phase_mode = split && P->contraction == JTFS_CONTRACTION_SPLIT_F16_PHASE;
    // the phase the forward stored, when this backward follows it on the same
    // workspace; without that forward, the phase is taken again by the forward
    // contraction where the recomputing kernel cannot hold the shapes
    const bool reuse = flags & JTFS_BWD_REUSE_FORWARD;
    const bool regen_phase = phase_mode && !reuse && !P->split_bwd_ok;
    const bool from_phase = phase_mode && (reuse || regen_phase);
    unsigned short* Yh = (unsigned short*)(base + w.Yh);
    float* ysc = (float*)(base + w.yscale);
    if (split && !reuse) {
        for (int a = 0; a < s.n_alpha; ++a) {
            JTFS_TIMED(JTFS_STAGE_OPERAND_SPLIT, st,
                       rc = launch_ysplit(P, a, Y2, (const float*)(base + w.rowmax), Yh, ysc, B, st));
            if (rc != JTFS_OK) { set_error("operand split kernel failed"); return rc; }
            if (regen_phase) {
                JTFS_TIMED(JTFS_STAGE_FREQ_FWD, st,
                           rc = launch_freq_fwd_split(P, a, Yh, ysc, (float*)(base + w.Vp), w.vp_bstride,
                                                      (unsigned*)(base + w.phase), w.ph_bstride, B, st));
                if (rc != JTFS_OK) { if (rc == JTFS_EHIP) set_error("split contraction launch failed"); return rc; }
            }
        }
    }
    if (from_phase) {
        JTFS_TIMED(JTFS_STAGE_OPERAND_SPLIT, st, rc = launch_gv_split(P, gV, (uint4*)(base + w.gvs), B, st));
        if (rc != JTFS_OK) { if (rc == JTFS_EHIP) set_error("gV split launch failed"); return rc; }
    }
    for (int a = 0; a < s.n_alpha && split; ++a) {
        if (from_phase) {
            // (one or two launches, each timed on its own)
            rc = launch_freq_bwd_phase(P, a, (const unsigned*)(base + w.phase), w.ph_bstride,
                                       (const uint4*)(base + w.gvs), w.gvs_bstride, (const float*)(base + w.gvmax),
                                       gY2, B, st);
        } else {
            JTFS_TIMED(JTFS_STAGE_FREQ_ADJ_PQ, st,
                       rc = launch_freq_bwd_split(P, a, Yh, ysc, gV, (const float*)(base + w.gvmax), gY2, B, st));
        }
        if (rc != JTFS_OK) { if (rc == JTFS_EHIP) set_error("split backward contraction launch failed"); return rc; }
        rc = gy2_row_fft(P, a, gY2, yb, B, st);
        if (rc != JTFS_OK) return rc;
    }
    for (int a = 0; a < s.n_alpha && !split && !s.tscat; ++a) {
        dim3 grid(nlt, s.Tp[a] / kTileT, (unsigned)B);
        const float2* Ya = Y2 + s.yoff[a];
        const float* Ph = P->Phi + s.phioff[a];
        const float* gVa = gV + (int64_t)a * 2 * s.Mp * s.NTp;
        const int64_t gvb = (int64_t)s.n_alpha * 2 * s.Mp * s.NTp;
        {
        TimedLaunch tl_pq(JTFS_STAGE_FREQ_ADJ_PQ, st);
        switch (s.NTp / 32) {
            case 1: hipLaunchKernelGGL(k_bwd_pq<1>, grid, dim3(256), 0, st, Ya, yb, s.Tp[a], P->Wt, s.Mp, s.Kp, Ph, gVa, gvb, PQ); break;
            case 2: hipLaunchKernelGGL(k_bwd_pq<2>, grid, dim3(256), 0, st, Ya, yb, s.Tp[a], P->Wt, s.Mp, s.Kp, Ph, gVa, gvb, PQ); break;
            case 4: hipLaunchKernelGGL(k_bwd_pq<4>, grid, dim3(256), 0, st, Ya, yb, s.Tp[a], P->Wt, s.Mp, s.Kp, Ph, gVa, gvb, PQ); break;
            default: set_error("unsupported N/T"); return JTFS_ENOTSUP;
        }
        LAUNCHCHK("contraction adjoint (recompute, modulus)");
        }
        JTFS_TIMED(JTFS_STAGE_FREQ_ADJ_WH, st, hipLaunchKernelGGL(k_bwd_gy, dim3((s.Kp + 63) / 64, s.Tp[a] / kTileT, (unsigned)B), dim3(256), 0, st, PQ,
                           s.Tp[a], P->Wl, s.Mp, s.Kp, gY2 + s.yoff[a], yb));
        LAUNCHCHK("contraction adjoint (W^H)");
        rc = gy2_row_fft(P, a, gY2, yb, B, st);
        if (rc != JTFS_OK) return rc;
    }
    const int logNT = s.logN - s.logT;
    const size_t lds_a = sizeof(float2) * (lpad_len(s.NX / 2) + 1 + lpad_len(s.NT));   // g1 at lpad(H) + 1
    const float2* gYphi = s.complete ? gY2 + s.yoff[s.n_alpha_psi] : nullptr;
    const int Tphi = s.complete ? s.Tp[s.n_alpha_psi] : 0;
    if (use_reg_rows(s.logNX, P->tune.reg_first_adj)) {
        JTFS_TIMED(JTFS_STAGE_SECOND_ADJ, st, launch_scal_bwd_a_r(P, gY2, yb, gs1, ml, gYphi, Tphi, gX, B, st));
    } else {
        JTFS_TIMED(JTFS_STAGE_SECOND_ADJ, st, hipLaunchKernelGGL(k_scal_bwd_a, dim3(s.n1, (unsigned)B), dim3(1024), lds_a, st, gY2, yb, P->d_yoff, P->d_Tp, P->d_Ta, P->psi2,
                           P->band2, P->off2, s.n_alpha_psi, gs1, P->phiX, s.Mphi, logNT, s.logNX, gX, P->tw, P->tw_log, ml,
                           gYphi, Tphi));
    }
    LAUNCHCHK("scalogram adjoint");
    if (use_reg_rows(s.logNX, P->tune.reg_first_adj)) {
        JTFS_TIMED(JTFS_STAGE_FIRST_ADJ, st, launch_scal_bwd_b_r(P, xh, w.xh_pitch, gX, g1, B, st));
    } else {
        JTFS_TIMED(JTFS_STAGE_FIRST_ADJ, st, hipLaunchKernelGGL(k_scal_bwd_b, dim3(s.n1, (unsigned)B), dim3(1024), sizeof(float2) * lpad_len(s.NX), st, xh, w.xh_pitch,
                       P->psi1, P->band1, P->off1, gX, g1, s.logNX, 1.0f / (float)s.N, P->tw, P->tw_log));
    }
    LAUNCHCHK("modulus and first-order adjoint");
    const int Hn = (int)(s.N / 2);
    JTFS_TIMED(JTFS_STAGE_BAND_ACCUM, st, hipLaunchKernelGGL(k_band_accum, dim3((unsigned)((Hn + 1 + 255) / 256), (unsigned)B), dim3(256), 0, st, g1, s.n1,
                       s.logNX, P->psi1, P->band1, P->off1, P->lam_range, Hn, gxh, w.xh_pitch));
    LAUNCHCHK("band accumulation");
    JTFS_TIMED(JTFS_STAGE_OUTPUT_FFT, st, hipLaunchKernelGGL(k_irfft_pack, dim3((unsigned)((Hn / 2 + 1 + 255) / 256), (unsigned)B), dim3(256), 0, st, gxh,
                       w.xh_pitch, tmp, (int64_t)Hn, s.logN, P->tw, P->tw_log));
    LAUNCHCHK("inverse real-FFT packing");
    JTFS_TIMED(JTFS_STAGE_OUTPUT_FFT, st, fft_rows(tmp, Hn, (float2*)gx, Hn, gxh, s.logN - 1, B, true, 1.0f / (float)s.N, P, st));
    LAUNCHCHK("output inverse FFT");
    return JTFS_OK;
}

int mulog_check(const jtfs_plan* P, const float* mu1, const float* mu2, float eps) {
    if (!P || !mu1 || !mu2) { set_error("null pointer"); return JTFS_EINVAL; }
    if (!(eps > 0.f)) { set_error("eps must be positive"); return JTFS_EINVAL; }
    return JTFS_OK;
}

}  // namespace

extern "C" int jtfs_backward(const jtfs_plan* P, const float* x, const float* gs1, const float* gs2, float* gx,
                             int64_t B, void* ws, size_t ws_bytes, uint32_t flags, hipStream_t st) {
    return backward_impl(P, x, gs1, gs2, gx, B, ws, ws_bytes, flags, MuLogArg{}, st);
}

extern "C" int jtfs_zeroth_order(const jtfs_plan* P, const float* x, int64_t B, float* s0, hipStream_t st) {
    if (!P || !x || !s0) { set_error("null pointer"); return JTFS_EINVAL; }
    if (B < 1 || B > 65535) { set_error("B must lie in [1, 65535]"); return JTFS_ESHAPE; }
    const Shapes& s = P->s;
    hipLaunchKernelGGL(k_s0, dim3((unsigned)s.NT, (unsigned)B), dim3(256), 0, st, x, s.N, s.T, P->phiN, P->phiN_len,
                       P->phiN_half, s0);
    LAUNCHCHK("zeroth order");
    return JTFS_OK;
}

extern "C" int jtfs_zeroth_order_backward(const jtfs_plan* P, const float* gs0, int64_t B, float* gx, hipStream_t st) {
    if (!P || !gs0 || !gx) { set_error("null pointer"); return JTFS_EINVAL; }
    if (B < 1 || B > 65535) { set_error("B must lie in [1, 65535]"); return JTFS_ESHAPE; }
    const Shapes& s = P->s;
    hipLaunchKernelGGL(k_s0_bwd, dim3((unsigned)((s.N + 255) / 256), (unsigned)B), dim3(256), 0, st, gs0, s.N, s.T, s.NT,
                       P->phiN, P->phiN_len, P->phiN_half, gx);
    LAUNCHCHK("zeroth-order adjoint");
    return JTFS_OK;
}

extern "C" int jtfs_forward_mulog(const jtfs_plan* P, const float* x, int64_t B, const float* mu1, const float* mu2,
                                  float eps, float* o1, float* o2, void* ws, size_t ws_bytes, hipStream_t st) {
    const int rc = mulog_check(P, mu1, mu2, eps);
    if (rc != JTFS_OK) return rc;
    return forward_impl(P, x, B, o1, o2, ws, ws_bytes, MuLogArg{mu1, mu2, eps, nullptr, nullptr}, st);
}

extern "C" int jtfs_backward_mulog(const jtfs_plan* P, const float* x, const float* o1, const float* o2,
                                   const float* mu1, const float* mu2, float eps, const float* go1, const float* go2,
                                   float* gx, int64_t B, void* ws, size_t ws_bytes, uint32_t flags, hipStream_t st) {
    const int rc = mulog_check(P, mu1, mu2, eps);
    if (rc != JTFS_OK) return rc;
    if ((go1 && !o1) || (go2 && !o2)) { set_error("null pointer"); return JTFS_EINVAL; }
    return backward_impl(P, x, go1, go2, gx, B, ws, ws_bytes, flags, MuLogArg{mu1, mu2, eps, o1, o2}, st);
}

