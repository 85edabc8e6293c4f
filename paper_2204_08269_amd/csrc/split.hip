// Frequential contraction on the FP16 matrix cores with split operands.
//
// Every FP32 operand value v, after multiplication by a power of two s that puts
// the operand block's maximum just below 2^14, is written as hi + lo with
// hi = fp16(v s) and lo = fp16(v s - hi) (22 significant bits).  A product is
// formed as hi*hi + hi*lo + lo*hi with v_mfma_f32_32x32x16_f16: the FP16 products
// are exact in FP32 and every sum accumulates in FP32, so the result carries the
// relative error of a 22-bit operand rounding (the dropped lo*lo term is of the
// same order) instead of FP32's 24 bits.  The scales are powers of two and are
// undone exactly.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "plan.hpp"
#include "split.hpp"
#include "timing.hpp"

namespace jtfs {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef _Float16 half8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ floatx16 z16() {
    floatx16 z;
#pragma unroll
    for (int r = 0; r < 16; ++r) z[r] = 0.f;
    return z;
}
__device__ __forceinline__ int crow(int r, int h) { return 8 * (r >> 2) + 4 * h + (r & 3); }

// D += A B with A 32x16, B 16x32 (FP16), D 32x32 FP32: lane (i + 32h) holds
// A[i][8h..8h+7] and B[8h..8h+7][i]; D as for the 32x32 FP32 instructions.
__device__ __forceinline__ floatx16 mfma16(half8 a, half8 b, floatx16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ half8 as_h8(uint4 v) { return __builtin_bit_cast(half8, v); }

__device__ __forceinline__ void split_h(float v, _Float16& hi, _Float16& lo) {
    hi = (_Float16)v;
    lo = (_Float16)(v - (float)hi);
}

// 2^(13 - e) with m < 2^e (frexp exponent): m * scale < 2^14; 1 for m == 0.
__device__ __forceinline__ float pow2_scale(float m) {
    if (!(m > 0.f)) return 1.f;
    int e;
    (void)frexpf(m, &e);
    return ldexpf(1.f, max(-120, min(120, 13 - e)));
}

// ---------------------------------------------------------------- plan tables

__global__ void k_absmax(const float* __restrict__ a, int64_t n, float* __restrict__ out) {
    __shared__ float red[256];
    float m = 0.f;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) m = fmaxf(m, fabsf(a[i]));
    red[threadIdx.x] = m;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

// Wsp[l][kb][p][j], k = 8 kb + j: p = 0 re hi, 1 re lo, 2 im hi, 3 im lo of W[l][k] * sw
__global__ void k_wsplit(const float2* __restrict__ Wl, int Mp, int Kp, float sw, unsigned short* __restrict__ Wsp) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)Mp * Kp) return;
    const int l = (int)(e / Kp), k = (int)(e % Kp);
    const float2 w = Wl[e];
    _Float16 a, b, c, d;
    split_h(w.x * sw, a, b);
    split_h(w.y * sw, c, d);
    _Float16* o = (_Float16*)Wsp + ((int64_t)l * (Kp / 8) + k / 8) * 32 + (k & 7);
    o[0] = a; o[8] = b; o[16] = c; o[24] = d;
}

// Phsp[t32][s][h][tau][p][j] = split(Phi[t32*32 + crow(8s+j, h)][tau] * sphi), p = hi, lo
__global__ void k_phsplit(const float* __restrict__ Phi, int Tp, int NTp, float sphi, unsigned short* __restrict__ Phsp) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)Tp * NTp) return;
    const int j = (int)(e & 7);
    int64_t r = e >> 3;
    const int tau = (int)(r % NTp); r /= NTp;
    const int h = (int)(r & 1); r >>= 1;
    const int s = (int)(r & 1); r >>= 1;
    const int t32 = (int)r;
    const int t = t32 * 32 + crow(8 * s + j, h);
    _Float16 hi, lo;
    split_h(Phi[(int64_t)t * NTp + tau] * sphi, hi, lo);
    _Float16* o = (_Float16*)Phsp + (((((int64_t)t32 * 2 + s) * 2 + h) * NTp + tau) * 2) * 8 + j;
    o[0] = hi;
    o[8] = lo;
}

// WTsp[c][i][s][h][p][j]: W[l][i] * sw split (p = re hi, re lo, im hi, im lo) for
// l = 32 c + crow(8 s + j, h): the rows of a 32-row chunk in the order in which the
// contraction's C registers hold them; chunk-major, so that the KpT x 32 block of
// one chunk is contiguous.  Rows i >= Kp are zero.
__global__ void k_wtsplit(const float2* __restrict__ Wl, int Mp, int Kp, int KpT, float sw,
                          unsigned short* __restrict__ WTsp) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)KpT * Mp) return;
    const int j = (int)(e & 7);
    int64_t r = e >> 3;
    const int h = (int)(r & 1); r >>= 1;
    const int s = (int)(r & 1); r >>= 1;
    const int i = (int)(r % KpT);
    const int c = (int)(r / KpT);
    const int l = 32 * c + crow(8 * s + j, h);
    const float2 w = i < Kp ? Wl[(int64_t)l * Kp + i] : make_float2(0.f, 0.f);
    _Float16 a, b, cc, d;
    split_h(w.x * sw, a, b);
    split_h(w.y * sw, cc, d);
    _Float16* o = (_Float16*)WTsp + ((((int64_t)c * KpT + i) * 2 + s) * 2 + h) * 32 + j;
    o[0] = a; o[8] = b; o[16] = cc; o[24] = d;
}

// PhTsp[t][g][p][j] = split(Phi[t][8 g + j] * sphi): tau-contiguous rows of Phi.
__global__ void k_phtsplit(const float* __restrict__ Phi, int Tp, int NTp, float sphi,
                           unsigned short* __restrict__ PhTsp) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)Tp * NTp) return;
    const int t = (int)(e / NTp), tau = (int)(e % NTp);
    _Float16 hi, lo;
    split_h(Phi[e] * sphi, hi, lo);
    _Float16* o = (_Float16*)PhTsp + (((int64_t)t * (NTp / 8) + tau / 8) * 2) * 8 + (tau & 7);
    o[0] = hi;
    o[8] = lo;
}

// ------------------------------------------------------------ Y2 conversion

// Yh[t][kb][p][j] = split(Y2[k][t] * sy) (k = 8 kb + j), transposed so that each
// lane of the contraction reads 8 consecutive lambda_1 of one t.  sy = 2^(13-e)
// from the block maximum (row maxima written by the second-order kernel).
// grid (Tp/64, B), 256 threads.
__global__ void __launch_bounds__(256) k_ysplit(const float2* __restrict__ Y, int64_t y_bstride, int Tp, int Kp,
                                                const float* __restrict__ rowmax, int alpha, int n_alpha,
                                                unsigned short* __restrict__ Yh, float* __restrict__ yscale) {
    __shared__ float2 tile[32][65];
    __shared__ float red[256];
    const int t0 = blockIdx.x * 64;
    const int64_t b = blockIdx.y;
    const float* rm = rowmax + (b * n_alpha + alpha) * Kp;
    float m = 0.f;
    for (int k = threadIdx.x; k < Kp; k += 256) m = fmaxf(m, rm[k]);
    red[threadIdx.x] = m;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    const float sy = pow2_scale(red[0]);
    if (blockIdx.x == 0 && threadIdx.x == 0) yscale[b * n_alpha + alpha] = sy;
    const float2* Yb = Y + b * y_bstride;
    _Float16* Ho = (_Float16*)Yh + b * y_bstride * 4;
    for (int k0 = 0; k0 < Kp; k0 += 32) {
        const int nk = min(32, Kp - k0);
        __syncthreads();
        for (int e = threadIdx.x; e < nk * 64; e += 256) {
            const int r = e >> 6, c = e & 63;
            tile[r][c] = Yb[(int64_t)(k0 + r) * Tp + t0 + c];
        }
        __syncthreads();
        const int nkb = nk / 8;
        for (int e = threadIdx.x; e < 64 * nkb; e += 256) {
            const int t = e / nkb, kb = e % nkb;
            half8 p0, p1, p2, p3;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const float2 v = tile[kb * 8 + j][t];
                _Float16 a, bb, c, d;
                split_h(v.x * sy, a, bb);
                split_h(v.y * sy, c, d);
                p0[j] = a; p1[j] = bb; p2[j] = c; p3[j] = d;
            }
            half8* o = (half8*)(Ho + ((int64_t)(t0 + t) * (Kp / 8) + k0 / 8 + kb) * 32);
            o[0] = p0; o[1] = p1; o[2] = p2; o[3] = p3;
        }
    }
}

// ------------------------------------------------------- forward contraction

// One workgroup: 64 rows l (W resident in LDS) x one t-chunk, in tiles of 128 t.
// Eight waves: wave (wl, wt) owns rows 32 wl.. and t 32 wt.. of each 128-t tile and
// streams its Y fragments from global memory (no barrier inside the K loop).
//   Z_up^T[t][l] = sum_k Y[k][t] W[l][k],   Z_down^T[t][l] = sum_k Y[k][t] conj W[l][k]
//   V^T[tau][l] += sum_t Phi[t][tau] |Z^T[t][l]|     (per spin)
// The modulus enters the second product split with a per-column power-of-two
// scale, removed from that tile's contribution before accumulation.
// Workgroups are mapped so that the row tiles sharing a t-chunk run on one XCD.
template <int NTB>
__global__ void __launch_bounds__(512) k_freq_fwd_h(const unsigned short* __restrict__ Yh, int64_t yh_bstride, int Tp,
                                                    int chunk, int nch, int nU, int nlt,
                                                    const unsigned short* __restrict__ Wsp, int Kp,
                                                    const unsigned short* __restrict__ Phsp, float unscale_wphi,
                                                    const float* __restrict__ yscale, int alpha, int n_alpha,
                                                    float* __restrict__ Vp, int64_t vp_bstride, int slot0) {
    constexpr int NTp = 32 * NTB;
    extern __shared__ __align__(16) unsigned char lds[];
    const int WS = Kp * 8 + 16;            // bytes per resident W row
    unsigned char* lw_ = lds;

    const int g = blockIdx.x;
    const int u = ((g >> 3) / nlt) * 8 + (g & 7);
    const int lt = (g >> 3) % nlt;
    if (u >= nU) return;
    const int64_t b = u / nch;
    const int ch = u % nch;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int h = lane >> 5, i32 = lane & 31;
    const int wl = wave & 1, wt = wave >> 1;
    const int nkb = Kp / 8;

    // resident W rows l0 .. l0+63
    {
        const uint4* src = (const uint4*)(Wsp + (int64_t)lt * 64 * Kp * 4);
        const int per_row = Kp / 2;        // uint4 per row
        for (int e = tid; e < 64 * per_row; e += 512) {
            const int r = e / per_row, c = e - r * per_row;
            *(uint4*)(lw_ + r * WS + c * 16) = src[e];
        }
    }
    const unsigned short* Yb = Yh + b * yh_bstride;
    floatx16 vu[NTB], vd[NTB];
#pragma unroll
    for (int n = 0; n < NTB; ++n) { vu[n] = z16(); vd[n] = z16(); }

    const int nK = Kp / 16;
    __syncthreads();                     // resident W complete
    const unsigned char* wbase = lw_ + (wl * 32 + i32) * WS + h * 64;
    for (int t0 = ch * chunk; t0 < (ch + 1) * chunk; t0 += kTileTh) {
        // each lane streams its own Y fragments (row t, k-group 2 kq + h) from global
        // memory two K-blocks ahead of use; W fragments come from the resident LDS rows.
        // One k-group is 4 planes x 8 halves = 4 uint4, one K-block (16 k) 8 uint4.
        const uint4* yrow = (const uint4*)(Yb + ((int64_t)(t0 + wt * 32 + i32) * nkb + h) * 32);
        uint4 a0 = yrow[0], a1 = yrow[1], a2 = yrow[2], a3 = yrow[3];
        uint4 b0 = a0, b1 = a1, b2 = a2, b3 = a3;
        if (nK > 1) { b0 = yrow[8]; b1 = yrow[9]; b2 = yrow[10]; b3 = yrow[11]; }
        floatx16 rr = z16(), ir = z16(), ri = z16(), ii = z16();
        auto block = [&](int kq, uint4 q0, uint4 q1, uint4 q2, uint4 q3) {
            const unsigned char* wr = wbase + kq * 128;
            const half8 w0 = as_h8(*(const uint4*)(wr + 0)), w1 = as_h8(*(const uint4*)(wr + 16));
            const half8 w2 = as_h8(*(const uint4*)(wr + 32)), w3 = as_h8(*(const uint4*)(wr + 48));
            const half8 y0 = as_h8(q0), y1 = as_h8(q1), y2 = as_h8(q2), y3 = as_h8(q3);
            rr = mfma16(y0, w0, rr); rr = mfma16(y0, w1, rr); rr = mfma16(y1, w0, rr);
            ir = mfma16(y2, w0, ir); ir = mfma16(y2, w1, ir); ir = mfma16(y3, w0, ir);
            ri = mfma16(y0, w2, ri); ri = mfma16(y0, w3, ri); ri = mfma16(y1, w2, ri);
            ii = mfma16(y2, w2, ii); ii = mfma16(y2, w3, ii); ii = mfma16(y3, w2, ii);
        };
        for (int kq = 0; kq < nK; kq += 2) {
            block(kq, a0, a1, a2, a3);
            if (kq + 2 < nK) {
                const uint4* p = yrow + 8 * (kq + 2);
                a0 = p[0]; a1 = p[1]; a2 = p[2]; a3 = p[3];
            }
            if (kq + 1 < nK) {
                block(kq + 1, b0, b1, b2, b3);
                if (kq + 3 < nK) {
                    const uint4* p = yrow + 8 * (kq + 3);
                    b0 = p[0]; b1 = p[1]; b2 = p[2]; b3 = p[3];
                }
            }
        }
        // modulus of both spins, per-column scale, split, second product with Phi
#pragma unroll
        for (int spin = 0; spin < 2; ++spin) {
            float uval[16];
            float m = 0.f;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const float zr = spin ? rr[r] + ii[r] : rr[r] - ii[r];
                const float zi = spin ? ir[r] - ri[r] : ir[r] + ri[r];
                uval[r] = sqrtf(zr * zr + zi * zi);
                m = fmaxf(m, uval[r]);
            }
            m = fmaxf(m, __shfl_xor(m, 32));
            const float su = pow2_scale(m);
            const float inv_su = 1.f / su;
            half8 uh[2], ul[2];
#pragma unroll
            for (int s = 0; s < 2; ++s)
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    _Float16 hi, lo;
                    split_h(uval[8 * s + j] * su, hi, lo);
                    uh[s][j] = hi;
                    ul[s][j] = lo;
                }
            const int t32 = (t0 >> 5) + wt;
#pragma unroll
            for (int n = 0; n < NTB; ++n) {
                floatx16 tmp = z16();
#pragma unroll
                for (int s = 0; s < 2; ++s) {
                    const uint4* ph = (const uint4*)(Phsp + (((((int64_t)t32 * 2 + s) * 2 + h) * NTp + n * 32 + i32) * 2) * 8);
                    const half8 phi = as_h8(ph[0]), plo = as_h8(ph[1]);
                    tmp = mfma16(phi, uh[s], tmp);
                    tmp = mfma16(phi, ul[s], tmp);
                    tmp = mfma16(plo, uh[s], tmp);
                }
                if (spin == 0) {
#pragma unroll
                    for (int r = 0; r < 16; ++r) vu[n][r] += tmp[r] * inv_su;
                } else {
#pragma unroll
                    for (int r = 0; r < 16; ++r) vd[n][r] += tmp[r] * inv_su;
                }
            }
        }
    }
    // sum the four t-quarter waves of each row half through LDS, unscale, store
    const float unscale = unscale_wphi / yscale[b * n_alpha + alpha];
    float* red = (float*)lds;                        // [wave][spin][64 lanes][16]
#pragma unroll
    for (int n = 0; n < NTB; ++n) {
        __syncthreads();
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            red[((wave * 2 + 0) * 64 + lane) * 16 + r] = vu[n][r];
            red[((wave * 2 + 1) * 64 + lane) * 16 + r] = vd[n][r];
        }
        __syncthreads();
        if (wt == 0) {
            float* o = Vp + b * vp_bstride;
#pragma unroll
            for (int spin = 0; spin < 2; ++spin) {
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    float acc = 0.f;
#pragma unroll
                    for (int q = 0; q < 4; ++q) acc += red[(((wl + 2 * q) * 2 + spin) * 64 + lane) * 16 + r];
                    const int tau = n * 32 + crow(r, h);
                    o[((((int64_t)(slot0 + ch) * nlt + lt) * 2 + spin) * NTp + tau) * kTileL + wl * 32 + i32] =
                        acc * unscale;
                }
            }
        }
    }
}


// ------------------------------------------------------ backward contraction

// Fused adjoint of the contraction, modulus and time lowpass for one signal and
// 128 columns t (four waves of 32).  The block loops over the 32-row chunks l of
// both spins and, per chunk:
//   Z[l][t] = sum_k W[l][k] Y[k][t]  (recomputed; both spins from four products)
//   gU[l][t] = sum_tau gV[l][tau] Phi[t][tau]       (adjoint of the time lowpass)
//   gZ = gU Z / max(|Z|, eps)                         (adjoint of the modulus)
//   P = gZ_up + gZ_down,  Q' = i (gZ_down - gZ_up)
//   gY[i][t] += sum_l Wr[l][i] P[l][t] + Wi[l][i] Q'[l][t]   (adjoint of W and conj W)
// P and Q' feed the last product straight from the C registers.  gV is split
// with a per-row scale (max over tau); P, Q' with one scale bounded by
// 2 max_l sum_tau |gV| max|Phi|; both are powers of two removed exactly.
//
// The chunks of split W (32 rows x Kp) and of split W^T (KpT rows x 32) are
// staged in LDS by direct global-to-LDS loads (no registers) and shared by the
// four waves: W^T double-buffered (the next chunk lands during the current
// one), W single-buffered (the next chunk lands during the W^T product, after
// every wave has finished the recompute).  The waits of a chunk never depend
// on those loads: they are issued after the chunk's last ordinary global loads.
// LDS slots are 16 bytes; a fragment segment is 32 consecutive slots (one per
// lane i32), which the MFMA fragment reads take conflict-free.
typedef __attribute__((address_space(3))) void lds_void_t;
typedef __attribute__((address_space(1))) void glob_void_t;

// one wave copies 64 slots: slot e = g * 64 + lane of the chunk's LDS layout
__device__ __forceinline__ void dma16(const uint4* src, uint4* lds_group) {
    __builtin_amdgcn_global_load_lds((glob_void_t*)src, (lds_void_t*)lds_group, 16, 0, 0);
}

// W chunk c (rows 32c..32c+31): LDS slot e = seg * 32 + r, seg = (2 kq + h) * 4 + p.
// Group g = wave + 4 j covers slots 64 g + lane: seg = 2 g + h, r = lane & 31, so a
// lane's source is its row's base plus 8 j slots.
__device__ __forceinline__ void stage_w(uint4* Ls, const uint4* Wsrc, int c, int nK, int nkb, int wave, int lane) {
    const uint4* src = Wsrc + (int64_t)c * (nK * 256) + (lane & 31) * (nkb * 4) + 2 * wave + (lane >> 5);
    uint4* dst = Ls + wave * 64;
    for (int j = 0; j < nK; ++j) dma16(src + 8 * j, dst + 256 * j);
}

// W^T chunk c (KpT = 32 NI rows): LDS slot e = seg * 32 + i32, seg = q * 16 + (sp * 2 + h) * 4 + p.
// Group g = wave + 4 k: seg = 8 k + 2 wave + h, i.e. q = k >> 1 and the segment
// inside q is 8 (k & 1) + 2 wave + h.
template <int NI>
__device__ __forceinline__ void stage_t(uint4* Ls, const uint4* Tsrc, int c, int wave, int lane) {
    const uint4* src = Tsrc + (int64_t)c * (NI * 512) + (lane & 31) * 16 + 2 * wave + (lane >> 5);
    uint4* dst = Ls + wave * 64;
#pragma unroll
    for (int k = 0; k < 2 * NI; ++k) dma16(src + (k >> 1) * 512 + 8 * (k & 1), dst + 256 * k);
}

template <int NTB, int NI>
__device__ __forceinline__ void bwd_chunk(int c, int nC, int nK, int nkb, int Mp, int wave, int lane, int h, int i32,
                                          const uint4* ycol, const uint4* phrow, const float* gvb, float inv_wy,
                                          float inv_phi, float spq, uint4* Ls_W, const uint4* Tcur, uint4* Tnext,
                                          const uint4* Wsrc, const uint4* Tsrc, floatx16 (&gyr)[NI],
                                          floatx16 (&gyi)[NI]) {
    constexpr int NTp = 32 * NTB;
    // ---- recompute Z for rows 32c.., columns tw0.. (four independent chains)
    const uint4* lw = Ls_W + h * 4 * 32 + i32;
    floatx16 rr = z16(), ri = z16(), ir = z16(), ii = z16();
    // Y fragments two k-steps ahead
    uint4 ya0 = ycol[0], ya1 = ycol[1], ya2 = ycol[2], ya3 = ycol[3];
    uint4 yb0 = ya0, yb1 = ya1, yb2 = ya2, yb3 = ya3;
    if (nK > 1) { yb0 = ycol[8]; yb1 = ycol[9]; yb2 = ycol[10]; yb3 = ycol[11]; }
    for (int kq = 0; kq < nK; ++kq) {
        const uint4* wk = lw + kq * 8 * 32;
        const half8 w0 = as_h8(wk[0]), w1 = as_h8(wk[32]), w2 = as_h8(wk[64]), w3 = as_h8(wk[96]);
        const half8 y0 = as_h8(ya0), y1 = as_h8(ya1), y2 = as_h8(ya2), y3 = as_h8(ya3);
        ya0 = yb0; ya1 = yb1; ya2 = yb2; ya3 = yb3;
        if (kq + 2 < nK) {
            const uint4* yp = ycol + 8 * (kq + 2);
            yb0 = yp[0]; yb1 = yp[1]; yb2 = yp[2]; yb3 = yp[3];
        }
        rr = mfma16(w0, y0, rr); ri = mfma16(w0, y2, ri); ir = mfma16(w2, y0, ir); ii = mfma16(w2, y2, ii);
        rr = mfma16(w0, y1, rr); ri = mfma16(w0, y3, ri); ir = mfma16(w2, y1, ir); ii = mfma16(w2, y3, ii);
        rr = mfma16(w1, y0, rr); ri = mfma16(w1, y2, ri); ir = mfma16(w3, y0, ir); ii = mfma16(w3, y2, ii);
    }
    // ---- gV rows of both spins, then the next W^T chunk (lands during this chunk)
    const int l0 = 32 * c;
    float4 v[2][NTB * 2][2];
#pragma unroll
    for (int spin = 0; spin < 2; ++spin) {
        const float* gr = gvb + ((int64_t)spin * Mp + l0 + i32) * NTp + 8 * h;
#pragma unroll
        for (int kb = 0; kb < NTB * 2; ++kb) {
            v[spin][kb][0] = *(const float4*)(gr + 16 * kb);
            v[spin][kb][1] = *(const float4*)(gr + 16 * kb + 4);
        }
    }
    // unconditional (the last chunk reloads itself into the idle buffer): with no
    // branch here the gV waits below count past these loads
    const int cn = c + 1 < nC ? c + 1 : c;
    stage_t<NI>(Tnext, Tsrc, cn, wave, lane);
    // ---- gU = gV Phi^T for both spins (gV split per row, Phi pre-split)
    floatx16 gu[2];
#pragma unroll
    for (int spin = 0; spin < 2; ++spin) {
        float mx = 0.f;
#pragma unroll
        for (int kb = 0; kb < NTB * 2; ++kb) {
            const float4 a0 = v[spin][kb][0], a1 = v[spin][kb][1];
            mx = fmaxf(mx, fmaxf(fmaxf(fabsf(a0.x), fabsf(a0.y)), fmaxf(fabsf(a0.z), fabsf(a0.w))));
            mx = fmaxf(mx, fmaxf(fmaxf(fabsf(a1.x), fabsf(a1.y)), fmaxf(fabsf(a1.z), fabsf(a1.w))));
        }
        mx = fmaxf(mx, __shfl_xor(mx, 32));
        const float sg = pow2_scale(mx);
        floatx16 acc = z16();
#pragma unroll
        for (int kb = 0; kb < NTB * 2; ++kb) {
            half8 ah, al;
            const float vv[8] = {v[spin][kb][0].x, v[spin][kb][0].y, v[spin][kb][0].z, v[spin][kb][0].w,
                                 v[spin][kb][1].x, v[spin][kb][1].y, v[spin][kb][1].z, v[spin][kb][1].w};
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                _Float16 hi, lo;
                split_h(vv[j] * sg, hi, lo);
                ah[j] = hi;
                al[j] = lo;
            }
            const uint4* pp = phrow + 4 * kb;       // k-group 2 kb + h: 32 bytes (hi, lo)
            const half8 bh = as_h8(pp[0]), bl = as_h8(pp[1]);
            acc = mfma16(ah, bh, acc);
            acc = mfma16(ah, bl, acc);
            acc = mfma16(al, bh, acc);
        }
        // row crow(r, h) of the C tile carries that row's gV scale (a power of
        // two: its reciprocal is exact)
        const float isg = inv_phi / sg;
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[r] *= __shfl(isg, crow(r, h));
        gu[spin] = acc;
    }
    // ---- modulus adjoint, P and Q' (FP32), split with the common scale
    half8 ph[2][4], pl[2][4];       // [s'][Pr, Pi, Qr, Qi]
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const float ur = (rr[r] - ii[r]) * inv_wy, ui = (ri[r] + ir[r]) * inv_wy;
        const float dr = (rr[r] + ii[r]) * inv_wy, di = (ri[r] - ir[r]) * inv_wy;
        // gU / |z| as gU * rsqrt(|z|^2), |z|^2 floored at a normal FP32 number
        // (kEpsMod2); z = 0 gives 0 as with the plain guard
        const float su = gu[0][r] * rsqrtf(fmaxf(ur * ur + ui * ui, kEpsMod2));
        const float sd = gu[1][r] * rsqrtf(fmaxf(dr * dr + di * di, kEpsMod2));
        const float gur = su * ur, gui = su * ui, gdr = sd * dr, gdi = sd * di;
        const float vals[4] = {gur + gdr, gui + gdi, -(gdi - gui), gdr - gur};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            _Float16 hi, lo;
            split_h(vals[q] * spq, hi, lo);
            ph[r >> 3][q][r & 7] = hi;
            pl[r >> 3][q][r & 7] = lo;
        }
    }
    // ---- every wave is done with this W chunk: stage the next one.  Only this
    // wave's LDS reads have to be complete (lgkmcnt 0; vmcnt and expcnt left at
    // their maxima in the gfx9 encoding), not the W^T staging just issued: a
    // fence would wait for that too, since it writes LDS through the vector
    // memory counter.
    __builtin_amdgcn_s_waitcnt(0xC07F);
    __builtin_amdgcn_s_barrier();
    stage_w(Ls_W, Wsrc, cn, nK, nkb, wave, lane);
    // ---- gY += Wr^T P + Wi^T Q' (A operand from the staged W^T chunk); two
    // i-blocks at a time, so that four independent accumulations alternate
#pragma unroll
    for (int q0 = 0; q0 < NI; q0 += 2) {
#pragma unroll
        for (int sp = 0; sp < 2; ++sp) {
            half8 wr[2][2], wi[2][2];             // [block][hi, lo]
#pragma unroll
            for (int d = 0; d < 2; ++d) {
                const int q = q0 + d < NI ? q0 + d : q0;
                const uint4* lt = Tcur + (q * 16 + (sp * 2 + h) * 4) * 32 + i32;
                wr[d][0] = as_h8(lt[0]); wr[d][1] = as_h8(lt[32]);
                wi[d][0] = as_h8(lt[64]); wi[d][1] = as_h8(lt[96]);
            }
#pragma unroll
            for (int term = 0; term < 6; ++term) {
                // (W part, P/Q' part): Wr hi*P hi, Wr hi*P lo, Wr lo*P hi, then the Wi terms with Q'
                const int wsel = term < 3 ? 0 : 1, whl = (term % 3) == 2 ? 1 : 0, phl = (term % 3) == 1 ? 1 : 0;
#pragma unroll
                for (int d = 0; d < 2; ++d) {
                    if (q0 + d >= NI) continue;
                    const half8 a = wsel ? wi[d][whl] : wr[d][whl];
                    const half8 br = phl ? pl[sp][wsel * 2] : ph[sp][wsel * 2];
                    const half8 bi = phl ? pl[sp][wsel * 2 + 1] : ph[sp][wsel * 2 + 1];
                    gyr[q0 + d] = mfma16(a, br, gyr[q0 + d]);
                    gyi[q0 + d] = mfma16(a, bi, gyi[q0 + d]);
                }
            }
        }
    }
    // ---- the next chunk's W and W^T have landed; every wave is done with this W^T chunk
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
}

template <int NTB, int NI>
__global__ void __launch_bounds__(256) k_freq_bwd_h(const unsigned short* __restrict__ Yh, int64_t yh_bstride,
                                                    int Tp, int nTt, int nU,
                                                    const unsigned short* __restrict__ Wsp,
                                                    const unsigned short* __restrict__ WTsp, int Kp, int Mp,
                                                    const unsigned short* __restrict__ PhTsp, float sphi,
                                                    const float* __restrict__ gV, int64_t gv_bstride,
                                                    const float* __restrict__ gvmax, int n_beta,
                                                    const float* __restrict__ yscale, int alpha, int n_alpha,
                                                    float sw, float2* __restrict__ gY, int64_t gy_bstride) {
    constexpr int NTp = 32 * NTB;
    __shared__ uint4 Ls_W[NI * 512];                // nK <= 2 NI k-steps x 8 segments x 32 slots
    __shared__ uint4 Ls_T0[NI * 512];               // 32 NI rows x 16 segments ... x 32 slots / 32
    __shared__ uint4 Ls_T1[NI * 512];
    const int u = blockIdx.x;
    if (u >= nU) return;                            // whole block
    const int64_t b = u / nTt;
    const int t0 = (u % nTt) * kTileTh;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int h = lane >> 5, i32 = lane & 31;
    const int tw0 = t0 + wave * 32;                 // this wave's columns
    const int nkb = Kp / 8, nK = Kp / 16, nC = Mp / 32;

    // scales
    float G = 0.f;
    for (int q = 0; q < 2 * n_beta; ++q) G = fmaxf(G, gvmax[(b * n_alpha + alpha) * 2 * n_beta + q]);
    const float spq = pow2_scale(2.f * G * 16384.f / sphi);
    const float sy = yscale[b * n_alpha + alpha];
    const float inv_wy = 1.f / (sw * sy);
    const float inv_phi = 1.f / sphi;

    floatx16 gyr[NI], gyi[NI];
#pragma unroll
    for (int q = 0; q < NI; ++q) { gyr[q] = z16(); gyi[q] = z16(); }

    const unsigned short* Yb = Yh + b * yh_bstride;
    const uint4* ycol = (const uint4*)(Yb + ((int64_t)(tw0 + i32) * nkb + h) * 32);   // B operand: column t
    const float* gvb = gV + b * gv_bstride;
    const uint4* phrow = (const uint4*)(PhTsp + ((int64_t)(tw0 + i32) * (NTp / 8) + h) * 16);
    const uint4* Wsrc = (const uint4*)Wsp;
    const uint4* Tsrc = (const uint4*)WTsp;

    stage_w(Ls_W, Wsrc, 0, nK, nkb, wave, lane);
    stage_t<NI>(Ls_T0, Tsrc, 0, wave, lane);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    for (int c = 0; c < nC; ++c) {
        uint4* Tc = (c & 1) ? Ls_T1 : Ls_T0;
        uint4* Tn = (c & 1) ? Ls_T0 : Ls_T1;
        bwd_chunk<NTB, NI>(c, nC, nK, nkb, Mp, wave, lane, h, i32, ycol, phrow, gvb, inv_wy, inv_phi, spq, Ls_W,
                           Tc, Tn, Wsrc, Tsrc, gyr, gyi);
    }
    // ---- store gY rows i < Kp, columns tw0.. (FP32 complex)
    const float inv = 1.f / (sw * spq);
    float2* o = gY + b * gy_bstride;
#pragma unroll
    for (int q = 0; q < NI; ++q)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int i = q * 32 + crow(r, h);
            if (i < Kp) o[(int64_t)i * Tp + tw0 + i32] = make_float2(gyr[q][r] * inv, gyi[q][r] * inv);
        }
}

}  // namespace jtfs

using namespace jtfs;

namespace jtfs {

size_t split_fwd_lds(const Shapes& s);

bool split_supported(const Shapes& s) { return split_fwd_lds(s) <= (size_t)kMaxDynLds && s.NTp <= 64; }

// LDS of k_freq_fwd_h: resident W rows during the main loop, then the cross-wave
// reduction buffer (8 waves x 2 spins x 64 lanes x 16 floats).
size_t split_fwd_lds(const Shapes& s) {
    const size_t main_loop = (size_t)64 * (s.Kp * 8 + 16);
    const size_t reduction = (size_t)8 * 2 * 64 * 16 * sizeof(float);
    return std::max(main_loop, reduction);
}

int build_split_tables(jtfs_plan* P, std::vector<void*>& owned) {
    const Shapes& s = P->s;
    P->split_ok = split_supported(s);
    if (!P->split_ok) return JTFS_OK;
    auto alloc = [&](size_t bytes) -> void* {
        void* p = nullptr;
        if (hipMalloc(&p, std::max<size_t>(bytes, 16)) != hipSuccess) return nullptr;
        owned.push_back(p);
        return p;
    };
    float* dmax = (float*)alloc(sizeof(float));
    P->Wsp = (unsigned short*)alloc(sizeof(float2) * s.Mp * s.Kp);
    P->Phsp = (unsigned short*)alloc(sizeof(float) * s.sumTp * s.NTp);
    if (!dmax || !P->Wsp || !P->Phsp) { set_error("device allocation failed"); return JTFS_ENOMEM; }
    float m = 0.f;
    hipLaunchKernelGGL(k_absmax, dim3(1), dim3(256), 0, 0, (const float*)P->Wl, (int64_t)2 * s.Mp * s.Kp, dmax);
    if (hipMemcpy(&m, dmax, sizeof(float), hipMemcpyDeviceToHost) != hipSuccess) {
        set_error("W maximum failed"); return JTFS_EHIP; }
    int e = 0;
    (void)std::frexp(m, &e);
    P->sw = m > 0.f ? std::ldexp(1.f, 13 - e) : 1.f;
    const int64_t nW = (int64_t)s.Mp * s.Kp;
    hipLaunchKernelGGL(k_wsplit, dim3((unsigned)((nW + 255) / 256)), dim3(256), 0, 0, P->Wl, s.Mp, s.Kp, P->sw, P->Wsp);
    P->sphi.assign(s.n_alpha, 1.f);
    for (int a = 0; a < s.n_alpha; ++a) {
        const int64_t n = (int64_t)s.Tp[a] * s.NTp;
        hipLaunchKernelGGL(k_absmax, dim3(1), dim3(256), 0, 0, P->Phi + s.phioff[a], n, dmax);
        if (hipMemcpy(&m, dmax, sizeof(float), hipMemcpyDeviceToHost) != hipSuccess) {
            set_error("Phi maximum failed"); return JTFS_EHIP; }
        (void)std::frexp(m, &e);
        P->sphi[a] = m > 0.f ? std::ldexp(1.f, 13 - e) : 1.f;
        hipLaunchKernelGGL(k_phsplit, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, 0, P->Phi + s.phioff[a],
                           s.Tp[a], s.NTp, P->sphi[a], P->Phsp + s.phioff[a] * 2);
    }
    P->KpT = (s.Kp + 31) / 32 * 32;
    P->WTsp = (unsigned short*)alloc(sizeof(float2) * (size_t)P->KpT * s.Mp);
    P->PhTsp = (unsigned short*)alloc(sizeof(float) * s.sumTp * s.NTp);
    if (!P->WTsp || !P->PhTsp) { set_error("device allocation failed"); return JTFS_ENOMEM; }
    {
        const int64_t n = (int64_t)P->KpT * s.Mp;
        hipLaunchKernelGGL(k_wtsplit, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, 0, P->Wl, s.Mp, s.Kp, P->KpT,
                           P->sw, P->WTsp);
    }
    for (int a = 0; a < s.n_alpha; ++a) {
        const int64_t n = (int64_t)s.Tp[a] * s.NTp;
        hipLaunchKernelGGL(k_phtsplit, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, 0, P->Phi + s.phioff[a],
                           s.Tp[a], s.NTp, P->sphi[a], P->PhTsp + s.phioff[a] * 2);
    }
    if (hipGetLastError() != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
        set_error("split-operand construction failed"); return JTFS_EHIP; }
    {
        const int NI = P->KpT / 32;
        // static LDS of the backward: W chunk + two W^T chunks, 24 NI KB (<= 160 KB)
        P->split_bwd_ok = (s.NTp == 32 && NI <= 6) || (s.NTp == 64 && NI <= 5);
    }
    P->contraction = JTFS_CONTRACTION_SPLIT_F16;
    return JTFS_OK;
}

int split_attributes() {
    // the backward kernels use static LDS only; the forward takes it dynamically
    const void* ks[] = {(const void*)k_freq_fwd_h<1>, (const void*)k_freq_fwd_h<2>};
    for (const void* k : ks)
        if (hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, kMaxDynLds) != hipSuccess) {
            set_error("hipFuncSetAttribute failed for the split contraction"); return JTFS_EHIP; }
    return JTFS_OK;
}

int launch_ysplit(const jtfs_plan* P, int a, const float2* Y2, const float* rowmax, unsigned short* Yh, float* yscale,
                  int64_t B, hipStream_t st) {
    const Shapes& s = P->s;
    const int64_t yb = (int64_t)s.Kp * s.sumTp;
    hipLaunchKernelGGL(k_ysplit, dim3(s.Tp[a] / 64, (unsigned)B), dim3(256), 0, st, Y2 + s.yoff[a], yb, s.Tp[a], s.Kp,
                       rowmax, a, s.n_alpha, Yh + s.yoff[a] * 4, yscale);
    return hipGetLastError() == hipSuccess ? JTFS_OK : JTFS_EHIP;
}

int launch_freq_fwd_split(const jtfs_plan* P, int a, const unsigned short* Yh, const float* yscale, float* Vp,
                          int64_t vp_bstride, int64_t B, hipStream_t st) {
    const Shapes& s = P->s;
    const int nlt = s.Mp / kTileL;
    const int nU = (int)(B * s.nch[a]);
    const unsigned grid = (unsigned)(((nU + 7) / 8) * 8 * nlt);
    const int64_t yhb = (int64_t)s.Kp * s.sumTp * 4;
    const float unscale = 1.f / (P->sw * P->sphi[a]);
    const size_t lds = split_fwd_lds(s);
    const unsigned short* Ya = Yh + s.yoff[a] * 4;
    const unsigned short* Ph = P->Phsp + s.phioff[a] * 2;
    const int slot0 = (int)s.vchoff[a];
    switch (s.NTp / 32) {
        case 1: hipLaunchKernelGGL(k_freq_fwd_h<1>, dim3(grid), dim3(512), lds, st, Ya, yhb, s.Tp[a], s.chunk[a], s.nch[a], nU, nlt, P->Wsp, s.Kp, Ph, unscale, yscale, a, s.n_alpha, Vp, vp_bstride, slot0); break;
        case 2: hipLaunchKernelGGL(k_freq_fwd_h<2>, dim3(grid), dim3(512), lds, st, Ya, yhb, s.Tp[a], s.chunk[a], s.nch[a], nU, nlt, P->Wsp, s.Kp, Ph, unscale, yscale, a, s.n_alpha, Vp, vp_bstride, slot0); break;
        case 4: hipLaunchKernelGGL(k_freq_fwd_h<4>, dim3(grid), dim3(512), lds, st, Ya, yhb, s.Tp[a], s.chunk[a], s.nch[a], nU, nlt, P->Wsp, s.Kp, Ph, unscale, yscale, a, s.n_alpha, Vp, vp_bstride, slot0); break;
        default: set_error("unsupported N/T"); return JTFS_ENOTSUP;
    }
    return hipGetLastError() == hipSuccess ? JTFS_OK : JTFS_EHIP;
}

template <int NTB>
static void launch_bwd_ni(int NI, dim3 grid, hipStream_t st, const unsigned short* Ya, int64_t yhb, int Tp, int nTt,
                          int nU, const jtfs_plan* P, const unsigned short* PhT, float sphi, const float* gVa,
                          int64_t gvb, const float* gvmax, const float* yscale, int a, float2* gYa, int64_t gyb) {
    const Shapes& s = P->s;
#define JTFS_BWD_CASE(ni)                                                                                      \
    case ni:                                                                                                   \
        hipLaunchKernelGGL((k_freq_bwd_h<NTB, ni>), grid, dim3(256), 0, st, Ya,                               \
                           yhb, Tp, nTt, nU, P->Wsp,                                                            \
                           P->WTsp, s.Kp, s.Mp, PhT, sphi, gVa, gvb, gvmax, s.n_beta, yscale, a, s.n_alpha,    \
                           P->sw, gYa, gyb);                                                                   \
        break;
    // LDS 24 NI KB and one wave per SIMD without scratch: NI <= 6 at N/T <= 32, NI <= 5 at N/T = 64
    if constexpr (NTB == 1) {
        switch (NI) {
            JTFS_BWD_CASE(1) JTFS_BWD_CASE(2) JTFS_BWD_CASE(3) JTFS_BWD_CASE(4)
            JTFS_BWD_CASE(5) JTFS_BWD_CASE(6)
            default: break;
        }
    } else {
        switch (NI) {
            JTFS_BWD_CASE(1) JTFS_BWD_CASE(2) JTFS_BWD_CASE(3) JTFS_BWD_CASE(4) JTFS_BWD_CASE(5)
            default: break;
        }
    }
#undef JTFS_BWD_CASE
}

int launch_freq_bwd_split(const jtfs_plan* P, int a, const unsigned short* Yh, const float* yscale, const float* gV,
                          const float* gvmax, float2* gY2, int64_t B, hipStream_t st) {
    const Shapes& s = P->s;
    const int NI = P->KpT / 32;
    if (!P->split_bwd_ok) { set_error("split backward not available for these shapes"); return JTFS_ENOTSUP; }
    const int nTt = s.Tp[a] / kTileTh;
    const int nU = (int)(B * nTt);
    const int64_t yhb = (int64_t)s.Kp * s.sumTp * 4;
    const int64_t yb = (int64_t)s.Kp * s.sumTp;
    const unsigned short* Ya = Yh + s.yoff[a] * 4;
    const unsigned short* PhT = P->PhTsp + s.phioff[a] * 2;
    const float* gVa = gV + (int64_t)a * 2 * s.Mp * s.NTp;
    const int64_t gvb = (int64_t)s.n_alpha * 2 * s.Mp * s.NTp;
    float2* gYa = gY2 + s.yoff[a];
    switch (s.NTp / 32) {
        case 1: launch_bwd_ni<1>(NI, dim3(nU), st, Ya, yhb, s.Tp[a], nTt, nU, P, PhT, P->sphi[a], gVa, gvb, gvmax, yscale, a, gYa, yb); break;
        case 2: launch_bwd_ni<2>(NI, dim3(nU), st, Ya, yhb, s.Tp[a], nTt, nU, P, PhT, P->sphi[a], gVa, gvb, gvmax, yscale, a, gYa, yb); break;
        default: set_error("unsupported N/T"); return JTFS_ENOTSUP;
    }
    return hipGetLastError() == hipSuccess ? JTFS_OK : JTFS_EHIP;
}

}  // namespace jtfs

extern "C" int jtfs_plan_set_contraction(jtfs_plan* P, int mode) {
    if (!P) { set_error("null plan"); return JTFS_EINVAL; }
    if (mode == JTFS_CONTRACTION_FP32) { P->contraction = mode; return JTFS_OK; }
    if (mode == JTFS_CONTRACTION_SPLIT_F16) {
        if (!P->split_ok) { set_error("split-FP16 contraction not available for these shapes"); return JTFS_ENOTSUP; }
        P->contraction = mode;
        return JTFS_OK;
    }
    set_error("unknown contraction mode");
    return JTFS_EINVAL;
}

extern "C" int jtfs_plan_get_contraction(const jtfs_plan* P, int* mode) {
    if (!P || !mode) { set_error("null pointer"); return JTFS_EINVAL; }
    *mode = P->contraction;
    return JTFS_OK;
}
