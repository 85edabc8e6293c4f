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

// s = 13 - e with m < 2^e (frexp exponent), so that m 2^s < 2^14; 0 for m == 0.
__device__ __forceinline__ int pow2_exp(float m) {
    if (!(m > 0.f)) return 0;
    int e;
    (void)frexpf(m, &e);
    return max(-120, min(120, 13 - e));
}
__device__ __forceinline__ float pow2_scale(float m) { return ldexpf(1.f, pow2_exp(m)); }

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

// WTsp[c][q][seg][i32][j], seg = (s * 2 + h) * 4 + p: W[l][i] * sw split (p = re hi,
// re lo, im hi, im lo) for i = 32 q + i32 and l = 32 c + crow(8 s + j, h): the rows of
// a 32-row chunk in the order in which the contraction's C registers hold them.  A
// chunk (KpT x 32) is contiguous and laid out exactly as the backward holds it in
// LDS, so that its staging copies contiguous 1 KB runs.  Rows i >= Kp are zero.
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
    _Float16* o = (_Float16*)WTsp +
                  ((int64_t)c * KpT * 16 + (i >> 5) * 512 + ((s * 2 + h) * 4) * 32 + (i & 31)) * 8 + j;
    o[0] = a; o[256] = b; o[512] = cc; o[768] = d;        // p = 0..3: 32 uint4 apart
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

// Yh[t / 32][kb][p][t % 32][j] = split(Y2[k][t] * sy) (k = 8 kb + j; p = re hi, re
// lo, im hi, im lo): each lane of the contraction reads 8 consecutive lambda_1 of
// one t as 16 bytes, and the 32 lanes of a column block read 512 contiguous bytes.
// sy = 2^(13-e) from the block maximum (row maxima written by the second-order
// kernel).  grid (Tp/64, B, Z), 256 threads: block z takes the 32-row chunks
// z, z + Z, ... (Z > 1 where Tp/64 x B alone would leave the GPU idle).
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
    if (blockIdx.x == 0 && blockIdx.z == 0 && threadIdx.x == 0) yscale[b * n_alpha + alpha] = sy;
    const float2* Yb = Y + b * y_bstride;
    _Float16* Ho = (_Float16*)Yh + b * y_bstride * 4;
    for (int k0 = 32 * (int)blockIdx.z; k0 < Kp; k0 += 32 * (int)gridDim.z) {
        const int nk = min(32, Kp - k0);
        __syncthreads();
        for (int e = threadIdx.x; e < nk * 64; e += 256) {
            const int r = e >> 6, c = e & 63;
            tile[r][c] = Yb[(int64_t)(k0 + r) * Tp + t0 + c];
        }
        __syncthreads();
        // one work item per (t, k-group, plane), t fastest: consecutive lanes store
        // consecutive 16-byte planes of one (k-group, plane)
        const int nkb = nk / 8;
        for (int e = threadIdx.x; e < 64 * nkb * 4; e += 256) {
            const int t = e & 63, g = e >> 6;
            const int pl = g & 3, kb = g >> 2;
            half8 out;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const float2 v = tile[kb * 8 + j][t];
                _Float16 hi, lo;
                split_h((pl < 2 ? v.x : v.y) * sy, hi, lo);
                out[j] = (pl & 1) ? lo : hi;
            }
            const int tt = t0 + t;
            half8* o = (half8*)Ho + ((((int64_t)(tt >> 5) * (Kp / 8) + k0 / 8 + kb) * 4 + pl) * 32 + (tt & 31));
            *o = out;
        }
    }
}

// A pointer the compiler cannot trace back to its (read-only, non-aliasing)
// kernel argument.  Loads through it are not taken as invariant, so the
// register allocator does not re-issue them next to their uses (possibly
// behind outstanding global-to-LDS loads, whose waits would then cover those
// too), and the Y loads, whose addresses are the same for every chunk, are not
// hoisted out of the chunk loop.
template <typename T>
using gptr = const __attribute__((address_space(1))) T*;
template <typename T>
__device__ __forceinline__ gptr<T> launder_v(const T* p) {
    gptr<T> g = (gptr<T>)p;
    asm volatile("" : "+v"(g));
    return g;
}
template <typename T>
__device__ __forceinline__ gptr<T> launder_s(const T* p) {
    gptr<T> g = (gptr<T>)p;
    asm volatile("" : "+s"(g));
    return g;
}

// Y fragments of k-step kq (k-groups 2 kq + h) of this lane's column: ycol points
// at plane 0 of k-group h of the lane's column; k-groups are 128 uint4 apart and
// planes 32
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void load_y(uint4 (&y)[4], gptr<uint4> ycol, int kq) {
    gptr<u32x4> p = (gptr<u32x4>)(ycol + 256 * kq);
#pragma unroll
    for (int j = 0; j < 4; ++j) y[j] = __builtin_bit_cast(uint4, p[32 * j]);
}

// The stored unit phase: two values in [-1, 1] as snorm16, round(x 32767), the
// first in the low half (absolute error at most 0.5 / 32767 per component).
__device__ __forceinline__ unsigned pack_snorm16(float a, float b) {
    return __builtin_bit_cast(unsigned, __builtin_amdgcn_cvt_pknorm_i16(a, b));
}
constexpr float kSnormInv = 1.f / 32767.f;

// ------------------------------------------------------- forward contraction

// rows t per pass of a wave's phase transpose in LDS: the whole 32-row tile where
// it fits beside the resident W rows (64 x (16 NK x 8 + 16) bytes), else 8 rows
template <int NK>
constexpr int kPhaseTrp = 64 * (16 * NK * 8 + 16) + 8 * 32 * 36 * 4 <= kMaxDynLds ? 32 : 8;

// One workgroup: 64 rows l (W resident in LDS) x one t-chunk, in tiles of 128 t.
// Eight waves: wave (wl, wt) owns rows 32 wl.. and t 32 wt.. of each 128-t tile and
// streams its Y fragments from global memory (no barrier inside the K loop).
//   Z_up^T[t][l] = sum_k Y[k][t] W[l][k],   Z_down^T[t][l] = sum_k Y[k][t] conj W[l][k]
//   V^T[tau][l] += sum_t Phi[t][tau] |Z^T[t][l]|     (per spin)
// The modulus enters the second product split with a per-column power-of-two
// scale, removed from that tile's contribution before accumulation.
// Workgroups are mapped so that the row tiles sharing a t-chunk run on one XCD.
template <int NTB, int NK>
__global__ void __launch_bounds__(512) k_freq_fwd_h(const unsigned short* __restrict__ Yh, int64_t yh_bstride, int Tp,
                                                    int chunk, int nch, int nU, int nlt,
                                                    const unsigned short* __restrict__ Wsp,
                                                    const unsigned short* __restrict__ Phsp, float unscale_wphi,
                                                    const float* __restrict__ yscale, int alpha, int n_alpha,
                                                    float* __restrict__ Vp, int64_t vp_bstride, int slot0,
                                                    unsigned* __restrict__ phase, int64_t ph_bstride, float sw) {
    constexpr int NTp = 32 * NTB;
    constexpr int Kp = 16 * NK;            // K = NK k-steps of 16 (compile time: the K loop is unrolled)
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
    // floor of |z|^2 in the scaled units of z (kEpsMod2 (sw sy)^2, kept a normal number)
    float eps2s = 0.f;
    if (phase) {
        const double wy = (double)sw * (double)yscale[b * n_alpha + alpha];
        eps2s = (float)fmax(fmin((double)kEpsMod2 * wy * wy, 1e30), 1.1754943508222875e-38);
    }
    floatx16 vu[NTB], vd[NTB];
#pragma unroll
    for (int n = 0; n < NTB; ++n) { vu[n] = z16(); vd[n] = z16(); }

    __syncthreads();                     // resident W complete
    const unsigned char* wbase = lw_ + (wl * 32 + i32) * WS + h * 64;
    // Each lane streams its own Y fragments (column t, k-group 2 kq + h; one
    // k-step is 4 uint4) from global memory through a ring of NR k-steps,
    // refilled as it drains; the next tile's first NR k-steps are requested
    // before the current tile's epilogue.  W fragments come from the resident
    // LDS rows.  The Phi fragments of a tile are requested before its Y loads,
    // so that waiting for them never waits for Y.
    const int tbeg = ch * chunk, tend = (ch + 1) * chunk;
    auto ycol_at = [&](int t0) {
        return launder_v((const uint4*)Yb + (((int64_t)((t0 >> 5) + wt) * nkb + h) * 128 + i32));
    };
    constexpr int NR0 = NTB == 1 ? 4 : 2;                     // ring depth within the register budget
    constexpr int NR = NK < NR0 ? NK : NR0;
    uint4 yr[NR][4];
    gptr<uint4> yc = ycol_at(tbeg);
#pragma unroll
    for (int s = 0; s < NR; ++s) load_y(yr[s], yc, s);
    for (int t0 = tbeg; t0 < tend; t0 += kTileTh) {
        const int t32 = (t0 >> 5) + wt;
        auto load_phi = [&](int n, int s, uint4 (&f)[2]) {
            gptr<u32x4> ph = (gptr<u32x4>)launder_v(
                (const uint4*)(Phsp + (((((int64_t)t32 * 2 + s) * 2 + h) * NTp + n * 32 + i32) * 2) * 8));
            f[0] = __builtin_bit_cast(uint4, ph[0]);
            f[1] = __builtin_bit_cast(uint4, ph[1]);
        };
        // with one 32-frame block the Phi fragments are held from here and the
        // next tile's Y is requested before the epilogue; wider frame counts
        // have no registers for that and request both where they are used
        constexpr bool early = NTB == 1;
        uint4 phf[2][2];                             // [s][hi, lo] of block n = 0
        if constexpr (early) {
            load_phi(0, 0, phf[0]);
            load_phi(0, 1, phf[1]);
        }
        // K loop, unrolled: k-step kq lives in ring slot kq % NR; W fragments are
        // read one k-step ahead, at the top of the k-step (a scheduling barrier
        // keeps them there: left to itself the compiler issues them after the
        // k-step's products, and the next k-step then waits for LDS), and a
        // scheduling barrier closes every k-step so that the LDS reads are not
        // all hoisted to the top
        floatx16 rr = z16(), ir = z16(), ri = z16(), ii = z16();
        uint4 wc[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) wc[j] = *(const uint4*)(wbase + 16 * j);
#pragma unroll
        for (int kq = 0; kq < NK; ++kq) {
            uint4 wn[4];
            if (kq + 1 < NK) {
#pragma unroll
                for (int j = 0; j < 4; ++j) wn[j] = *(const uint4*)(wbase + (kq + 1) * 128 + 16 * j);
            }
            __builtin_amdgcn_sched_barrier(0);
            const half8 w0 = as_h8(wc[0]), w1 = as_h8(wc[1]), w2 = as_h8(wc[2]), w3 = as_h8(wc[3]);
            uint4(&q)[4] = yr[kq % NR];
            const half8 y0 = as_h8(q[0]), y1 = as_h8(q[1]), y2 = as_h8(q[2]), y3 = as_h8(q[3]);
            // the four accumulators in turn (each keeps its own summation order)
            rr = mfma16(y0, w0, rr); ir = mfma16(y2, w0, ir); ri = mfma16(y0, w2, ri); ii = mfma16(y2, w2, ii);
            rr = mfma16(y0, w1, rr); ir = mfma16(y2, w1, ir); ri = mfma16(y0, w3, ri); ii = mfma16(y2, w3, ii);
            rr = mfma16(y1, w0, rr); ir = mfma16(y3, w0, ir); ri = mfma16(y1, w2, ri); ii = mfma16(y3, w2, ii);
            if (kq + NR < NK) load_y(q, yc, kq + NR);
            if (kq + 1 < NK) {
#pragma unroll
                for (int j = 0; j < 4; ++j) wc[j] = wn[j];
            }
            __builtin_amdgcn_sched_barrier(0);
        }
        auto next_tile = [&]() {
            if (t0 + kTileTh < tend) {
                yc = ycol_at(t0 + kTileTh);
#pragma unroll
                for (int s = 0; s < NR; ++s) load_y(yr[s], yc, s);
            }
        };
        if constexpr (early) next_tile();
        // modulus of both spins, per-column scale, split, second product with Phi;
        // with phase storage also u = z / max(|z|, eps) for the backward, as two
        // snorm16 (real in the low half), in groups of 8 rows l: element
        // ((spin, l / 32, (l % 32) / 8), t, l % 8); the floor is in the scaled
        // units of z
#pragma unroll
        for (int spin = 0; spin < 2; ++spin) {
            float uval[16];
            float m = 0.f;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const float zr = spin ? rr[r] + ii[r] : rr[r] - ii[r];
                const float zi = spin ? ir[r] - ri[r] : ir[r] + ri[r];
                uval[r] = __builtin_amdgcn_sqrtf(zr * zr + zi * zi);   // hardware square root (1 ulp)
                m = fmaxf(m, uval[r]);
            }
            // the wave's 32 x 32 tile of packed phases goes through its own LDS
            // area (rows t, 36-element pitch), so that each lane then stores 16
            // bytes (four rows l of one t) and a wave's store covers runs of TRP
            // consecutive t; TRP rows t per pass (32, or 8 where the resident W
            // tile leaves no room for the whole tile)
            if (phase) {
                unsigned* tb = (unsigned*)(lds + 64 * WS) + wave * (kPhaseTrp<NK> * 36);
                constexpr int TRP = kPhaseTrp<NK>, LTRP = TRP == 32 ? 5 : 3;
#pragma unroll
                for (int pass = 0; pass < 32 / TRP; ++pass) {
#pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        if (TRP == 8 && (r >> 2) != pass) continue;   // crow(r, h) / 8 = r / 4
                        const float zr = spin ? rr[r] + ii[r] : rr[r] - ii[r];
                        const float zi = spin ? ir[r] - ri[r] : ir[r] + ri[r];
                        const float q = __builtin_amdgcn_rsqf(fmaxf(zr * zr + zi * zi, eps2s));
                        tb[(crow(r, h) & (TRP - 1)) * 36 + i32] = pack_snorm16(zr * q, zi * q);
                    }
                    unsigned* pb = phase + b * ph_bstride + ((int64_t)(spin * nlt + lt) * 2 + wl) * 4 * Tp * 8 +
                                   (int64_t)(t0 + wt * 32 + pass * TRP) * 8;
#pragma unroll
                    for (int k = 0; k < TRP / 8; ++k) {
                        // element e of the pass: half hh of row group g at row tt
                        const int e = lane + 64 * k;
                        const int hh = e & 1, tt = (e >> 1) & (TRP - 1), g = e >> (1 + LTRP);
                        // read back only by the backward, long after: a streaming store, so
                        // that it does not evict the Y operand the row tiles share in L2
                        const u32x4 v = __builtin_bit_cast(u32x4, *(const uint4*)(tb + tt * 36 + 8 * g + 4 * hh));
                        __builtin_nontemporal_store(v, (u32x4*)(pb + (int64_t)g * Tp * 8 + tt * 8 + 4 * hh));
                    }
                }
            }
            m = fmaxf(m, __shfl_xor(m, 32));
            const int se = pow2_exp(m);
            const float su = ldexpf(1.f, se), inv_su = ldexpf(1.f, -se);
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
#pragma unroll
            for (int n = 0; n < NTB; ++n) {
                floatx16 tmp = z16();
#pragma unroll
                for (int s = 0; s < 2; ++s) {
                    uint4 f[2];
                    if constexpr (early) {
                        f[0] = phf[s][0];
                        f[1] = phf[s][1];
                    } else {
                        load_phi(n, s, f);
                    }
                    const half8 phi = as_h8(f[0]), plo = as_h8(f[1]);
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
        if constexpr (!early) next_tile();
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


// ---------------------------------------- forward contraction, 16 x 16 tiles

// D (16 x 16, FP32) += A (16 x 32) B (32 x 16) in FP16: lane j + 16 g holds
// A[j][8g .. 8g+7], B[8g .. 8g+7][j] and D[4g .. 4g+3][j].
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef _Float16 half4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ floatx4 mfma16q(half8 a, half8 b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}
// the same with K = 16: lane j + 16 g holds A[j][4g .. 4g+3] and B[4g .. 4g+3][j]
__device__ __forceinline__ floatx4 mfma16k(half4 a, half4 b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ floatx4 z4() { return floatx4{0.f, 0.f, 0.f, 0.f}; }

// Phq[t / 16][tau / 16][lane][p][r]: split(Phi[t][tau] * sphi) (p = hi, lo) for
// tau = 16 (tau / 16) + lane % 16, t = 16 (t / 16) + 4 (lane / 16) + r: the A operand
// of the 16 x 16 x 16 lowpass product, one 16-byte load per lane.
__global__ void k_phqsplit(const float* __restrict__ Phi, int Tp, int NTp, float sphi,
                           unsigned short* __restrict__ Phq) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)Tp * NTp) return;
    const int r = (int)(e & 3);
    int64_t q = e >> 2;
    const int lane = (int)(q & 63); q >>= 6;
    const int n = (int)(q % (NTp / 16));
    const int t16 = (int)(q / (NTp / 16));
    const int tau = 16 * n + (lane & 15), t = 16 * t16 + 4 * (lane >> 4) + r;
    _Float16 hi, lo;
    split_h(Phi[(int64_t)t * NTp + tau] * sphi, hi, lo);
    _Float16* o = (_Float16*)Phq + (((int64_t)t16 * (NTp / 16) + n) * 64 + lane) * 8 + r;
    o[0] = hi;
    o[4] = lo;
}

// Wq[lt][ks][lb][p][lane][j] = split(W[l][k] * sw), p = re hi, re lo, im hi, im lo,
// for l = 64 lt + 16 lb + lane % 16 and k = 32 ks + 8 (lane / 16) + j; zero for
// k >= Kp.  The A operands of the 16 x 16 x 32 forward products of a 64-row tile in
// the order in which the lanes read them: each fragment is 64 consecutive 16-byte
// slots, which an LDS read takes without bank conflicts.
__global__ void k_wqsplit(const float2* __restrict__ Wl, int Mp, int Kp, int NS, float sw,
                          unsigned short* __restrict__ Wq) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)Mp * NS * 128) return;        // Mp / 64 tiles x NS k-steps x 8192 halves
    const int j = (int)(e & 7);
    const int lane = (int)((e >> 3) & 63);
    const int p = (int)((e >> 9) & 3);
    const int lb = (int)((e >> 11) & 3);
    const int64_t r = e >> 13;
    const int ks = (int)(r % NS);
    const int lt = (int)(r / NS);
    const int l = 64 * lt + 16 * lb + (lane & 15);
    const int k = 32 * ks + 8 * (lane >> 4) + j;
    const float2 w = k < Kp ? Wl[(int64_t)l * Kp + k] : make_float2(0.f, 0.f);
    _Float16 hi, lo;
    split_h((p < 2 ? w.x : w.y) * sw, hi, lo);
    ((_Float16*)Wq)[e] = (p & 1) ? lo : hi;
}

// LDS of k_freq_fwd_q: the resident W tile (16 KB per k-step of 32) and a
// 16 x 20-word phase transpose area per wave, then the cross-wave reduction of V
// (8 waves x NTQ x 4 row blocks x 2 spins x 64 lanes x 4 floats).
constexpr size_t fwdq_lds(int Kp, int NTQ, bool with_phase) {
    const size_t main_loop = (size_t)((Kp / 16 + 1) / 2) * 16384 + (with_phase ? (size_t)8 * 16 * 20 * 4 : 0);
    const size_t reduction = (size_t)8 * NTQ * 4 * 2 * 64 * 4 * sizeof(float);
    return main_loop > reduction ? main_loop : reduction;
}

// One workgroup: 64 rows l (W resident in LDS) x one t-chunk, in tiles of 128 t.
// Eight waves; wave w owns t 16 w .. 16 w + 15 of each tile and all 64 rows, in
// four 16-row blocks: every Y fragment is loaded from global memory by exactly one
// wave, and each wave reads all W fragments of the tile from LDS.
//   Z_up^T[t][l] = sum_k Y[k][t] W[l][k],   Z_down^T[t][l] = sum_k Y[k][t] conj W[l][k]
//   V^T[tau][l] += sum_t Phi[t][tau] |Z^T[t][l]|     (per spin)
// The C registers of the first product (rows t) are the B operand of the second
// (K = t) as they stand.  The modulus enters the second product split with a
// per-column power-of-two scale, removed from that tile's contribution before
// accumulation.  NTQ blocks of 16 frames (N/T <= 32).  Workgroups are mapped as in
// k_freq_fwd_h.
template <int NK, int NTQ>
__global__ void __launch_bounds__(512) k_freq_fwd_q(const unsigned short* __restrict__ Yh, int64_t yh_bstride, int Tp,
                                                    int chunk, int nch, int nU, int nlt,
                                                    const unsigned short* __restrict__ Wq,
                                                    const unsigned short* __restrict__ Phq, float unscale_wphi,
                                                    const float* __restrict__ yscale, int alpha, int n_alpha,
                                                    float* __restrict__ Vp, int64_t vp_bstride, int slot0,
                                                    unsigned* __restrict__ phase, int64_t ph_bstride, float sw) {
    constexpr int NTp = 32;                  // tau slots of the partial-V layout
    constexpr int Kp = 16 * NK;
    constexpr int NS = (NK + 1) / 2;         // k-steps of 32
    constexpr bool TAIL = (NK & 1) != 0;     // the last k-step holds 16 k (k-groups 0, 1)
    constexpr int NR = NS < 2 ? NS : 2;      // Y ring depth (k-steps)
    extern __shared__ __align__(16) unsigned char lds[];

    const int g = blockIdx.x;
    const int u = ((g >> 3) / nlt) * 8 + (g & 7);
    const int lt = (g >> 3) % nlt;
    if (u >= nU) return;
    const int64_t b = u / nch;
    const int ch = u % nch;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int j16 = lane & 15, g4 = lane >> 4;
    constexpr int nkb = Kp / 8;

    // resident W tile of rows l0 .. l0+63, in read order (NS x 1024 slots)
    {
        const uint4* src = (const uint4*)Wq + (int64_t)lt * NS * 1024;
        uint4* dst = (uint4*)lds;
#pragma unroll
        for (int e = 0; e < 2 * NS; ++e) dst[e * 512 + tid] = src[e * 512 + tid];
    }
    const unsigned short* Yb = Yh + b * yh_bstride;
    float eps2s;                             // the floor of |z|^2 in the scaled units of Z
    {
        const double wy = (double)sw * (double)yscale[b * n_alpha + alpha];
        eps2s = (float)fmax(fmin((double)kEpsMod2 * wy * wy, 1e30), 1.1754943508222875e-38);
    }
    floatx4 vacc[NTQ][4][2];
#pragma unroll
    for (int n = 0; n < NTQ; ++n)
#pragma unroll
        for (int lb = 0; lb < 4; ++lb) { vacc[n][lb][0] = z4(); vacc[n][lb][1] = z4(); }
    __syncthreads();                         // resident W complete

    // this lane's W fragments: row 16 lb + j16, k-group 4 ks + g4, plane p
    const uint4* wfr = (const uint4*)lds + lane;
    auto load_w = [&](uint4 (&w)[4], int ks, int lb) {
#pragma unroll
        for (int p = 0; p < 4; ++p) w[p] = wfr[((ks * 4 + lb) * 4 + p) * 64];
    };
    // this lane's Y fragments: column t, k-group 4 ks + g4, plane p (uint4 units)
    const int tbeg = ch * chunk, tend = (ch + 1) * chunk;
    auto ycol_at = [&](int t0) {
        // the column offset formed from the thread index here, not kept live across
        // the tile loop (at 256 registers the compiler spilled it, and its reload
        // waited for every memory operation in flight)
        int tq = (int)threadIdx.x;
        asm volatile("" : "+v"(tq));
        const int t = t0 + (tq >> 6) * 16 + (tq & 15);
        return launder_v((const uint4*)Yb + (((int64_t)(t >> 5) * nkb + ((tq >> 4) & 3)) * 128 + (t & 31)));
    };
    auto load_yq = [&](uint4 (&y)[4], gptr<uint4> yc, int ks) {
        gptr<u32x4> p = (gptr<u32x4>)(yc + 512 * ks);
        const bool ok = !(TAIL && ks == NS - 1 && g4 >= 2);
#pragma unroll
        for (int j = 0; j < 4; ++j) y[j] = ok ? __builtin_bit_cast(uint4, p[32 * j]) : make_uint4(0, 0, 0, 0);
    };
    uint4 yr[NR][4];
    gptr<uint4> yc = ycol_at(tbeg);
#pragma unroll
    for (int s = 0; s < NR; ++s) load_yq(yr[s], yc, s);
    unsigned* tb = (unsigned*)(lds + NS * 16384) + wave * (16 * 20);   // phase transpose area
    for (int t0 = tbeg; t0 < tend; t0 += kTileTh) {
        const int t16 = (t0 >> 4) + wave;
        // Phi fragments of this tile (A operand of the lowpass product)
        uint4 phf[NTQ];
#pragma unroll
        for (int n = 0; n < NTQ; ++n)
            phf[n] = __builtin_bit_cast(uint4, ((gptr<u32x4>)launder_v((const uint4*)Phq))[((int64_t)t16 * (NTp / 16) + n) * 64 + lane]);
        floatx4 rr[4], ir[4], ri[4], ii[4];
#pragma unroll
        for (int lb = 0; lb < 4; ++lb) { rr[lb] = z4(); ir[lb] = z4(); ri[lb] = z4(); ii[lb] = z4(); }
        uint4 wc[4], wn[4];
        load_w(wc, 0, 0);
#pragma unroll
        for (int ks = 0; ks < NS; ++ks) {
            uint4(&q)[4] = yr[ks % NR];
            const half8 y0 = as_h8(q[0]), y1 = as_h8(q[1]), y2 = as_h8(q[2]), y3 = as_h8(q[3]);
#pragma unroll
            for (int lb = 0; lb < 4; ++lb) {
                // the next fragments (next row block, or the next k-step's first) are
                // requested before this block's products
                if (lb + 1 < 4) load_w(wn, ks, lb + 1);
                else if (ks + 1 < NS) load_w(wn, ks + 1, 0);
                __builtin_amdgcn_sched_barrier(0);
                // (the tile holds zeros beyond Kp, so a short last k-step needs no mask)
                const half8 w0 = as_h8(wc[0]), w1 = as_h8(wc[1]), w2 = as_h8(wc[2]), w3 = as_h8(wc[3]);
                // the four accumulators in turn, so that no product waits for the one
                // before it (each keeps its own summation order)
                rr[lb] = mfma16q(y0, w0, rr[lb]); ir[lb] = mfma16q(y2, w0, ir[lb]);
                ri[lb] = mfma16q(y0, w2, ri[lb]); ii[lb] = mfma16q(y2, w2, ii[lb]);
                rr[lb] = mfma16q(y0, w1, rr[lb]); ir[lb] = mfma16q(y2, w1, ir[lb]);
                ri[lb] = mfma16q(y0, w3, ri[lb]); ii[lb] = mfma16q(y2, w3, ii[lb]);
                rr[lb] = mfma16q(y1, w0, rr[lb]); ir[lb] = mfma16q(y3, w0, ir[lb]);
                ri[lb] = mfma16q(y1, w2, ri[lb]); ii[lb] = mfma16q(y3, w2, ii[lb]);
#pragma unroll
                for (int p = 0; p < 4; ++p) wc[p] = wn[p];
                __builtin_amdgcn_sched_barrier(0);
            }
            if (ks + NR < NS) load_yq(q, yc, ks + NR);
        }
        // the next tile's first Y k-steps go out before this tile's epilogue
        if (t0 + kTileTh < tend) {
            yc = ycol_at(t0 + kTileTh);
#pragma unroll
            for (int s = 0; s < NR; ++s) load_yq(yr[s], yc, s);
        }
        // modulus of both spins, per-column scale, split, lowpass product; with
        // phase storage also u = z / max(|z|, eps) as two snorm16 (real in the low
        // half) in the layout of k_freq_fwd_h: element ((spin, l / 32, (l % 32) / 8), t, l % 8)
#pragma unroll
        for (int spin = 0; spin < 2; ++spin) {
#pragma unroll
            for (int lb = 0; lb < 4; ++lb) {
                float uv[4];
                float m = 0.f;
                // |z| = |z|^2 rsq(|z|^2), with the reciprocal square root that the phase
                // uses (below the floor eps^2, |z|^2 / eps < eps: nothing the lowpass sees)
                float qn[4], zrs[4], zis[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const float zr = spin ? rr[lb][r] + ii[lb][r] : rr[lb][r] - ii[lb][r];
                    const float zi = spin ? ir[lb][r] - ri[lb][r] : ir[lb][r] + ri[lb][r];
                    const float m2 = zr * zr + zi * zi;
                    qn[r] = __builtin_amdgcn_rsqf(fmaxf(m2, eps2s));
                    uv[r] = m2 * qn[r];
                    zrs[r] = zr;
                    zis[r] = zi;
                    m = fmaxf(m, uv[r]);
                }
                if (phase) {
                    // rows t 4 g4 + r, column j16 of the wave's 16 x 16 block -> 16-byte
                    // runs of four rows l of one t
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        tb[(4 * g4 + r) * 20 + j16] = pack_snorm16(zrs[r] * qn[r], zis[r] * qn[r]);
                    const int tt = lane >> 2, jq = lane & 3;
                    const int ll = lb * 16 + 4 * jq;                 // first row of the quad in the 64-row tile
                    const int wl = ll >> 5, g8 = (ll & 31) >> 3;
                    unsigned* pb = phase + b * ph_bstride +
                                   ((((int64_t)(spin * nlt + lt) * 2 + wl) * 4 + g8) * Tp + t0 + wave * 16 + tt) * 8 +
                                   (ll & 7);
                    const u32x4 v = __builtin_bit_cast(u32x4, *(const uint4*)(tb + tt * 20 + 4 * jq));
                    // read back only by the backward, long after: a streaming store, so
                    // that it does not evict the Y operand the row tiles share in L2
                    __builtin_nontemporal_store(v, (u32x4*)pb);
                }
                {
                    // maximum over the four lane groups (16 lanes apart) by two lane swaps,
                    // without a round trip through LDS
                    const unsigned mb = __float_as_uint(m);
                    const auto r16 = __builtin_amdgcn_permlane16_swap(mb, mb, false, false);
                    m = fmaxf(__uint_as_float(r16[0]), __uint_as_float(r16[1]));
                    const unsigned mc = __float_as_uint(m);
                    const auto r32 = __builtin_amdgcn_permlane32_swap(mc, mc, false, false);
                    m = fmaxf(__uint_as_float(r32[0]), __uint_as_float(r32[1]));
                }
                const int se = pow2_exp(m);
                const float su = ldexpf(1.f, se), inv_su = ldexpf(1.f, -se);
                half4 uh, ul;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    _Float16 hi, lo;
                    split_h(uv[r] * su, hi, lo);
                    uh[r] = hi;
                    ul[r] = lo;
                }
#pragma unroll
                for (int n = 0; n < NTQ; ++n) {
                    const uint4 f = phf[n];
                    const half4 phi = __builtin_bit_cast(half4, make_uint2(f.x, f.y));
                    const half4 plo = __builtin_bit_cast(half4, make_uint2(f.z, f.w));
                    floatx4 tmp = z4();
                    tmp = mfma16k(phi, uh, tmp);
                    tmp = mfma16k(phi, ul, tmp);
                    tmp = mfma16k(plo, uh, tmp);
#pragma unroll
                    for (int r = 0; r < 4; ++r) vacc[n][lb][spin][r] += tmp[r] * inv_su;
                }
            }
        }
    }
    // sum the eight waves' partial V through LDS, unscale, store
    const float unscale = unscale_wphi / yscale[b * n_alpha + alpha];
    float* red = (float*)lds;                // [wave][n][lb][spin][64 lanes][4]
    __syncthreads();
#pragma unroll
    for (int n = 0; n < NTQ; ++n)
#pragma unroll
        for (int lb = 0; lb < 4; ++lb)
#pragma unroll
            for (int spin = 0; spin < 2; ++spin)
                *(float4*)(red + ((((wave * NTQ + n) * 4 + lb) * 2 + spin) * 64 + lane) * 4) =
                    make_float4(vacc[n][lb][spin][0], vacc[n][lb][spin][1], vacc[n][lb][spin][2],
                                vacc[n][lb][spin][3]);
    __syncthreads();
    float* o = Vp + b * vp_bstride + ((int64_t)(slot0 + ch) * nlt + lt) * 2 * NTp * kTileL;
    for (int e = tid; e < NTQ * 4 * 2 * 64 * 4; e += 512) {
        // e = (((n * 4 + lb) * 2 + spin) * 64 + ln) * 4 + r: element tau = 16 n + 4 (ln / 16) + r,
        // l = 16 lb + ln % 16
        const int r = e & 3, ln = (e >> 2) & 63, spin = (e >> 8) & 1, lb = (e >> 9) & 3, n = e >> 11;
        float acc = 0.f;
#pragma unroll
        for (int w = 0; w < 8; ++w) acc += red[(((w * NTQ * 4 * 2) * 64) * 4) + e];
        const int tau = 16 * n + 4 * (ln >> 4) + r, l = 16 * lb + (ln & 15);
        o[((int64_t)spin * NTp + tau) * kTileL + l] = acc * unscale;
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

// one wave copies 64 slots: slot e = g * 64 + lane of the chunk's LDS layout.
// The source is a block-uniform base plus this lane's byte offset (32 bits), the
// form the global-to-LDS load takes with the base in scalar registers, so that
// a staging sequence keeps one offset register instead of one 64-bit address
// per load.
__device__ __forceinline__ void dma16(const uint4* ubase, uint32_t lane_bytes, uint4* lds_group) {
    __builtin_amdgcn_global_load_lds((glob_void_t*)((const char*)ubase + lane_bytes), (lds_void_t*)lds_group, 16,
                                     0, 0);
}

// W chunk c (rows 32c..32c+31): LDS slot e = seg * 32 + r, seg = (2 kq + h) * 4 + p.
// Group g = wave + 4 j covers slots 64 g + lane: seg = 2 g + h, r = lane & 31, so a
// lane's source is its row's base plus 8 j slots.
__device__ __forceinline__ void stage_w(uint4* Ls, const uint4* Wsrc, int c, int nK, int nkb, int wave, int lane) {
    const uint4* base = Wsrc + (int64_t)c * (nK * 256);
    const uint32_t off = (uint32_t)((lane & 31) * (nkb * 4) + 2 * wave + (lane >> 5)) * 16u;
    uint4* dst = Ls + wave * 64;
    for (int j = 0; j < nK; ++j) dma16(base + 8 * j, off, dst + 256 * j);
}

// W^T chunk c (NI blocks of 32 rows i) into LDS, slot e = seg * 32 + i32 with
// seg = q * 16 + (sp * 2 + h) * 4 + p: the table holds the chunk in this order, so
// that the wave's 64 lanes copy 1 KB runs.  Chunks are cstride slots apart in the
// table (512 per i-block of the whole K); Tsrc points at the first staged block.
template <int NI>
__device__ __forceinline__ void stage_t(uint4* Ls, const uint4* Tsrc, int c, int64_t cstride, int wave, int lane) {
    const uint4* base = Tsrc + (int64_t)c * cstride;
    const uint32_t off = (uint32_t)(wave * 64 + lane) * 16u;
    uint4* dst = Ls + wave * 64;
#pragma unroll
    for (int k = 0; k < 2 * NI; ++k) dma16(base + 256 * k, off, dst + 256 * k);
}

// gV rows l0 + i32 of both spins, this lane's tau half (8 h.. of each 16)
template <int NTB>
__device__ __forceinline__ void load_gv(float4 (&v)[2][NTB * 2][2], gptr<float4> gvb, int Mp, int l0, int i32,
                                        int h) {
    constexpr int NTp = 32 * NTB;
#pragma unroll
    for (int spin = 0; spin < 2; ++spin) {
        gptr<f32x4> gr = (gptr<f32x4>)(gvb + (((int64_t)spin * Mp + l0 + i32) * NTp + 8 * h) / 4);
#pragma unroll
        for (int kb = 0; kb < NTB * 2; ++kb) {
            v[spin][kb][0] = __builtin_bit_cast(float4, gr[4 * kb]);
            v[spin][kb][1] = __builtin_bit_cast(float4, gr[4 * kb + 1]);
        }
    }
}

// One 32-row chunk c.  On entry the first min(NK, 4) k-steps of Y sit in the
// ring yr and the chunk's gV rows in v (both loaded during the previous chunk),
// and the chunk's W and W^T are in LDS.  On exit the same holds for chunk c + 1.
// Order of memory operations: the ring is refilled inside the recompute loop
// (ordinary loads, waited for there); the DMA staging of the next W and W^T is
// issued after that loop, and the next chunk's Y ring and gV after it, all of
// them waited for only at the chunk's end.  No wait for an ordinary load is
// therefore ever placed behind an outstanding global-to-LDS load.
template <int NTB, int NI, int NK>
__device__ __forceinline__ void bwd_chunk(int c, int nC, int Mp, int wave, int lane, int h, int i32,
                                          const uint4* ycol, const uint4 (&phv)[NTB * 2][2], const float* gvb,
                                          float eps2s,
                                          float ips, float spq, uint4* Ls_W, const uint4* Tcur, uint4* Tnext,
                                          const uint4* Wsrc, const uint4* Tsrc, floatx16 (&gyr)[NI],
                                          floatx16 (&gyi)[NI], uint4 (&yr)[4][4]) {
    constexpr int NR = NK < 4 ? NK : 4;                       // Y ring depth (k-steps in flight)
    // this chunk's gV rows (older than every Y load of the loop below, so the
    // loop's waits cover them)
    float4 v[2][NTB * 2][2];
    load_gv<NTB>(v, launder_s((const float4*)gvb), Mp, 32 * c, i32, h);
    // ---- recompute Z for rows 32c.., columns tw0.. (four independent chains)
    // (W fragments read one k-step ahead; a scheduling barrier closes every
    // k-step so that the reads are not all hoisted to the top)
    const uint4* lw = Ls_W + h * 4 * 32 + i32;
    gptr<uint4> yc = launder_v(ycol);
    floatx16 rr = z16(), ri = z16(), ir = z16(), ii = z16();
    uint4 wc[4] = {lw[0], lw[32], lw[64], lw[96]};
#pragma unroll
    for (int kq = 0; kq < NK; ++kq) {
        uint4 wn[4];
        if (kq + 1 < NK) {
            const uint4* wk = lw + (kq + 1) * 8 * 32;
            wn[0] = wk[0]; wn[1] = wk[32]; wn[2] = wk[64]; wn[3] = wk[96];
        }
        const half8 w0 = as_h8(wc[0]), w1 = as_h8(wc[1]), w2 = as_h8(wc[2]), w3 = as_h8(wc[3]);
        uint4(&ys)[4] = yr[kq % NR];
        const half8 y0 = as_h8(ys[0]), y1 = as_h8(ys[1]), y2 = as_h8(ys[2]), y3 = as_h8(ys[3]);
        rr = mfma16(w0, y0, rr); ri = mfma16(w0, y2, ri); ir = mfma16(w2, y0, ir); ii = mfma16(w2, y2, ii);
        rr = mfma16(w0, y1, rr); ri = mfma16(w0, y3, ri); ir = mfma16(w2, y1, ir); ii = mfma16(w2, y3, ii);
        rr = mfma16(w1, y0, rr); ri = mfma16(w1, y2, ri); ir = mfma16(w3, y0, ir); ii = mfma16(w3, y2, ii);
        if (kq + NR < NK) load_y(ys, yc, kq + NR);
        if (kq + 1 < NK) {
            wc[0] = wn[0]; wc[1] = wn[1]; wc[2] = wn[2]; wc[3] = wn[3];
        }
        __builtin_amdgcn_sched_barrier(0);
    }
    // gV is used from here on only: its wait lands here (long after the loads,
    // and ahead of the staging below), and nothing computed from it is moved
    // into the loop above
#pragma unroll
    for (int spin = 0; spin < 2; ++spin)
#pragma unroll
        for (int kb = 0; kb < NTB * 2; ++kb)
#pragma unroll
            for (int j = 0; j < 2; ++j)
                asm volatile("" : "+v"(v[spin][kb][j].x), "+v"(v[spin][kb][j].y), "+v"(v[spin][kb][j].z),
                             "+v"(v[spin][kb][j].w));
    // ---- every wave is done with this W chunk (only this wave's LDS reads must
    // be complete: lgkmcnt 0, vmcnt and expcnt at their maxima in the gfx9
    // encoding); stage the next W and W^T chunks (the last chunk reloads itself)
    __builtin_amdgcn_s_waitcnt(0xC07F);
    __builtin_amdgcn_s_barrier();
    const int cn = c + 1 < nC ? c + 1 : c;
    stage_w(Ls_W, Wsrc, cn, NK, 2 * NK, wave, lane);
    stage_t<NI>(Tnext, Tsrc, cn, (int64_t)NI * 512, wave, lane);
    // ---- gU = gV Phi^T for both spins (gV split per row, Phi pre-split), times spq
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
        const int se = pow2_exp(mx);
        const float sg = ldexpf(1.f, se);
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
            const half8 bh = as_h8(phv[kb][0]), bl = as_h8(phv[kb][1]);
            acc = mfma16(ah, bh, acc);
            acc = mfma16(ah, bl, acc);
            acc = mfma16(al, bh, acc);
        }
        // row crow(r, h) of the C tile carries that row's gV scale; every factor
        // is a power of two, so the rescaling is exact
        const float isg = ldexpf(ips, -se);
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[r] *= __shfl(isg, crow(r, h));
        gu[spin] = acc;
    }
    __builtin_amdgcn_sched_barrier(0);
    // ---- modulus adjoint, P and Q' (FP32, already carrying the scale spq).
    // gU z / |z| does not depend on the scale of z, so the scaled Z is used as
    // it is; |z|^2 is floored at kEpsMod2 on the unscaled value (eps2s)
    half8 ph[2][4], pl[2][4];       // [s'][Pr, Pi, Qr, Qi]
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        if (r == 8) __builtin_amdgcn_sched_barrier(0);
        const float ur = rr[r] - ii[r], ui = ri[r] + ir[r];
        const float dr = rr[r] + ii[r], di = ri[r] - ir[r];
        // (eps2s is a normal number: the hardware reciprocal square root needs no
        // denormal handling)
        const float su = gu[0][r] * __builtin_amdgcn_rsqf(fmaxf(ur * ur + ui * ui, eps2s));
        const float sd = gu[1][r] * __builtin_amdgcn_rsqf(fmaxf(dr * dr + di * di, eps2s));
        const float vals[4] = {su * ur + sd * dr, su * ui + sd * di, su * ui - sd * di, sd * dr - su * ur};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            _Float16 hi, lo;
            split_h(vals[q], hi, lo);
            ph[r >> 3][q][r & 7] = hi;
            pl[r >> 3][q][r & 7] = lo;
        }
    }
    __builtin_amdgcn_sched_barrier(0);
    // ---- the next chunk's Y ring (lands during the product below)
    gptr<uint4> yn = launder_v(ycol);
#pragma unroll
    for (int s = 0; s < NR; ++s) load_y(yr[s], yn, s);
    __builtin_amdgcn_sched_barrier(0);
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
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    // ---- the next chunk's operands have landed; every wave is done with this W^T chunk
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
}

template <int NTB, int NI, int NK>
__global__ void __launch_bounds__(256) k_freq_bwd_h(const unsigned short* __restrict__ Yh, int64_t yh_bstride,
                                                    int Tp, int nTt, int nU,
                                                    const unsigned short* __restrict__ Wsp,
                                                    const unsigned short* __restrict__ WTsp, int Mp,
                                                    const unsigned short* __restrict__ PhTsp, float sphi,
                                                    const float* __restrict__ gV, int64_t gv_bstride,
                                                    const float* __restrict__ gvmax, int n_beta,
                                                    const float* __restrict__ yscale, int alpha, int n_alpha,
                                                    float sw, float2* __restrict__ gY, int64_t gy_bstride) {
    constexpr int NTp = 32 * NTB;
    constexpr int Kp = 16 * NK, nkb = 2 * NK;
    __shared__ uint4 Ls_W[NI * 512];                // NK <= 2 NI k-steps x 8 segments x 32 slots
    __shared__ uint4 Ls_T0[NI * 512];               // 32 NI rows x 16 segments ... x 32 slots / 32
    __shared__ uint4 Ls_T1[NI * 512];
    const int u = blockIdx.x;
    if (u >= nU) return;                            // whole block
    const int64_t b = u / nTt;
    const int t0 = (u % nTt) * kTileTh;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int h = lane >> 5, i32 = lane & 31;
    const int tw0 = t0 + wave * 32;                 // this wave's columns
    const int nC = Mp / 32;

    // scales (all powers of two but the modulus floor)
    float G = 0.f;
    for (int q = 0; q < 2 * n_beta; ++q) G = fmaxf(G, gvmax[(b * n_alpha + alpha) * 2 * n_beta + q]);
    const float spq = pow2_scale(2.f * G * 16384.f / sphi);
    const float sy = yscale[b * n_alpha + alpha];
    const double wy = (double)sw * (double)sy;
    const float eps2s = (float)fmax(fmin((double)kEpsMod2 * wy * wy, 1e30), 1.1754943508222875e-38);
    const float ips = spq / sphi;

    floatx16 gyr[NI], gyi[NI];
#pragma unroll
    for (int q = 0; q < NI; ++q) { gyr[q] = z16(); gyi[q] = z16(); }

    const unsigned short* Yb = Yh + b * yh_bstride;
    const uint4* ycol = (const uint4*)Yb + (((int64_t)(tw0 >> 5) * nkb + h) * 128 + i32);   // B operand: column t
    const float* gvb = gV + b * gv_bstride;
    const uint4* phrow = (const uint4*)(PhTsp + ((int64_t)(tw0 + i32) * (NTp / 8) + h) * 16);
    const uint4* Wsrc = (const uint4*)Wsp;
    const uint4* Tsrc = (const uint4*)WTsp;

    // Phi^T fragments of the four columns (the same for every chunk): k-group
    // 2 kb + h, 32 bytes (hi, lo)
    uint4 phv[NTB * 2][2];
#pragma unroll
    for (int kb = 0; kb < NTB * 2; ++kb) {
        phv[kb][0] = phrow[4 * kb];
        phv[kb][1] = phrow[4 * kb + 1];
    }
    uint4 yr[4][4];
#pragma unroll
    for (int s = 0; s < (NK < 4 ? NK : 4); ++s) load_y(yr[s], (gptr<uint4>)ycol, s);
    stage_w(Ls_W, Wsrc, 0, NK, nkb, wave, lane);
    stage_t<NI>(Ls_T0, Tsrc, 0, (int64_t)NI * 512, wave, lane);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    // nC is even (Mp is a multiple of 64): the W^T buffers alternate at compile
    // time, so that the reads of one are not made to wait for the staging of the other
    for (int c = 0; c < nC; c += 2) {
        bwd_chunk<NTB, NI, NK>(c, nC, Mp, wave, lane, h, i32, ycol, phv, gvb, eps2s, ips, spq, Ls_W, Ls_T0, Ls_T1,
                               Wsrc, Tsrc, gyr, gyi, yr);
        bwd_chunk<NTB, NI, NK>(c + 1, nC, Mp, wave, lane, h, i32, ycol, phv, gvb, eps2s, ips, spq, Ls_W, Ls_T1,
                               Ls_T0, Wsrc, Tsrc, gyr, gyi, yr);
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

// ------------------------------------------ backward from the stored phase

// 16-byte units per 32-row chunk of the split gV: both spins' FP16 planes, then the
// rows' scales
template <int NTB>
constexpr int gvs_chunk() { return 512 * NTB + 16; }

// gV split once for the stored-phase backward (the recomputing backward splits it in
// registers, the same way).  Per (signal, rate) and 32-row chunk: planes
// [spin][kb][hl][h][i] of 8 halves, the values tau = 16 kb + 8 h + j of row 32 c + i
// times 2^se (se = pow2_exp of the row's largest |gV|), hi or lo; then 2^-se of the
// chunk's rows as [spin][32] floats.  One thread per (signal, rate, spin, row).
template <int NTB>
__global__ void k_gvsplit(const float* __restrict__ gV, int Mp, int64_t nrows, uint4* __restrict__ Gs) {
    constexpr int NTp = 32 * NTB;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nrows) return;
    const int l = (int)(e % Mp);
    const int spin = (int)((e / Mp) & 1);
    const int64_t ba = e / (2 * Mp);                 // signal x rate
    const float4* row = (const float4*)(gV + e * NTp);
    float4 v[NTp / 4];
    float mx = 0.f;
#pragma unroll
    for (int q = 0; q < NTp / 4; ++q) {
        v[q] = row[q];
        mx = fmaxf(mx, fmaxf(fmaxf(fabsf(v[q].x), fabsf(v[q].y)), fmaxf(fabsf(v[q].z), fabsf(v[q].w))));
    }
    const int se = pow2_exp(mx);
    const float sg = ldexpf(1.f, se);
    uint4* blk = Gs + (ba * (Mp / 32) + l / 32) * gvs_chunk<NTB>();
    const int i = l & 31;
#pragma unroll
    for (int kb = 0; kb < 2 * NTB; ++kb)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const float4 x0 = v[4 * kb + 2 * h], x1 = v[4 * kb + 2 * h + 1];
            const float vv[8] = {x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, x1.z, x1.w};
            half8 hi8, lo8;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                _Float16 hi, lo;
                split_h(vv[j] * sg, hi, lo);
                hi8[j] = hi;
                lo8[j] = lo;
            }
            blk[(((spin * 2 * NTB + kb) * 2 + 0) * 2 + h) * 32 + i] = __builtin_bit_cast(uint4, hi8);
            blk[(((spin * 2 * NTB + kb) * 2 + 1) * 2 + h) * 32 + i] = __builtin_bit_cast(uint4, lo8);
        }
    ((float*)(blk + 512 * NTB))[spin * 32 + i] = ldexpf(1.f, -se);
}

// Chunk c of the split gV into LDS (all 256 threads; lane order = source order).
template <int NTB>
__device__ __forceinline__ void stage_g(uint4* Ls, const uint4* Gb, int c, int tid) {
    const uint4* src = Gb + (int64_t)c * gvs_chunk<NTB>();
    uint4* dst = Ls + 64 * (tid >> 6);
#pragma unroll
    for (int k = 0; k < 2 * NTB; ++k) dma16(src + 256 * k, (uint32_t)tid * 16u, dst + 256 * k);
    if (tid < 16) dma16(src + 512 * NTB, (uint32_t)tid * 16u, Ls + 512 * NTB);
}

// Stored unit phase of rows crow(r, h), r = 8 s .. 8 s + 7 (g = 2 s, 2 s + 1), of one
// 32-row block, this lane's column t, both spins: one 16-byte load (four rows) per
// (spin, g); a wave's load is one contiguous 1 KB run.  pcol points at element 4 h
// of the lane's column in row group 0 of the block of spin 0; row groups are
// g_stride elements apart.
__device__ __forceinline__ void load_phase_half(uint4 (&pv)[2][4], int s, gptr<uint4> pcol, int64_t spin_stride,
                                                int64_t g_stride) {
#pragma unroll
    for (int spin = 0; spin < 2; ++spin)
#pragma unroll
        for (int gg = 0; gg < 2; ++gg) {
            const int g = 2 * s + gg;
            gptr<u32x4> p = (gptr<u32x4>)(pcol + (spin * spin_stride + g * g_stride) / 4);   // element offsets, % 4 = 0
            pv[spin][g] = __builtin_bit_cast(uint4, __builtin_nontemporal_load(p));   // read once
        }
}

// the two snorm16 of row crow(r, h) as integers in [-32767, 32767] (real, imaginary)
__device__ __forceinline__ float2 phase_at(const uint4 (&pv)[2][4], int spin, int r) {
    const uint4 q = pv[spin][r >> 2];
    const unsigned w = (r & 3) == 0 ? q.x : (r & 3) == 1 ? q.y : (r & 3) == 2 ? q.z : q.w;
    return make_float2((float)(int)(short)(w & 0xffffu), (float)((int)w >> 16));
}

// gU = gV Phi^T of one chunk for both spins (A operand from the split gV in LDS, Phi
// pre-split in registers); each row then scaled by its 2^-se times c0 (the scale of
// P and Q' over the snorm16 unit of the phase).
template <int NTB>
__device__ __forceinline__ void gu_chunk(const uint4* Lg, const uint4 (&phv)[NTB * 2][2], int h, int i32, float c0,
                                         floatx16 (&gu)[2]) {
    const float4* rs = (const float4*)(Lg + 512 * NTB);
#pragma unroll
    for (int spin = 0; spin < 2; ++spin) {
        floatx16 acc = z16();
#pragma unroll
        for (int kb = 0; kb < NTB * 2; ++kb) {
            const half8 ah = as_h8(Lg[(((spin * 2 * NTB + kb) * 2 + 0) * 2 + h) * 32 + i32]);
            const half8 al = as_h8(Lg[(((spin * 2 * NTB + kb) * 2 + 1) * 2 + h) * 32 + i32]);
            const half8 bh = as_h8(phv[kb][0]), bl = as_h8(phv[kb][1]);
            acc = mfma16(ah, bh, acc);
            acc = mfma16(ah, bl, acc);
            acc = mfma16(al, bh, acc);
        }
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            const float4 q = rs[spin * 8 + 2 * g + h];        // rows 8 g + 4 h .. + 3
            acc[4 * g + 0] *= q.x * c0;
            acc[4 * g + 1] *= q.y * c0;
            acc[4 * g + 2] *= q.z * c0;
            acc[4 * g + 3] *= q.w * c0;
        }
        gu[spin] = acc;
    }
}

// hi / lo FP16 split (as split_h) of two values, each packed as a pair: hp = (hi0,
// hi1) by one packed conversion, lp = (lo0, lo1) by two mixed-precision FMAs that
// form v - hi exactly in FP32 and round it once, writing the low and high halves.
__device__ __forceinline__ void split2(float v0, float v1, unsigned& hp, unsigned& lp) {
    typedef float f2v __attribute__((ext_vector_type(2)));
    typedef _Float16 h2v __attribute__((ext_vector_type(2)));
    hp = __builtin_bit_cast(unsigned, __builtin_convertvector((f2v){v0, v1}, h2v));
    asm("v_fma_mixlo_f16 %0, %1, 1.0, -%3 op_sel_hi:[0,0,1]\n\t"
        "v_fma_mixhi_f16 %0, %2, 1.0, -%3 op_sel:[0,0,1] op_sel_hi:[0,0,1]"
        : "=&v"(lp)
        : "v"(v0), "v"(v1), "v"(hp));
}

// Modulus adjoint of row pairs 8 s + 2 p0 .. 8 s + 2 p1 - 1 from the scaled gU and
// the stored phase: P and Q', split into FP16 hi / lo (lanes r - 8 s of ph[s],
// pl[s]).
__device__ __forceinline__ void modadj_pairs(int s, int p0, int p1, const floatx16 (&gu)[2], const uint4 (&pv)[2][4],
                                             half8 (&ph)[2][4], half8 (&pl)[2][4]) {
#pragma unroll
    for (int pr = 0; pr < 4; ++pr) {
        if (pr < p0 || pr >= p1) continue;
        float vals[2][4];
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const int r = 8 * s + 2 * pr + e;
            const float2 u = phase_at(pv, 0, r), d = phase_at(pv, 1, r);
            const float su = gu[0][r], sd = gu[1][r];
            vals[e][0] = su * u.x + sd * d.x;
            vals[e][1] = su * u.y + sd * d.y;
            vals[e][2] = su * u.y - sd * d.y;
            vals[e][3] = sd * d.x - su * u.x;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            unsigned hp, lp;
            split2(vals[0][q], vals[1][q], hp, lp);
            uint4 hv = __builtin_bit_cast(uint4, ph[s][q]), lv = __builtin_bit_cast(uint4, pl[s][q]);
            if (pr == 0) { hv.x = hp; lv.x = lp; }
            else if (pr == 1) { hv.y = hp; lv.y = lp; }
            else if (pr == 2) { hv.z = hp; lv.z = lp; }
            else { hv.w = hp; lv.w = lp; }
            ph[s][q] = __builtin_bit_cast(half8, hv);
            pl[s][q] = __builtin_bit_cast(half8, lv);
        }
    }
}
__device__ __forceinline__ void modadj_half(int s, const floatx16 (&gu)[2], const uint4 (&pv)[2][4],
                                            half8 (&ph)[2][4], half8 (&pl)[2][4]) {
    modadj_pairs(s, 0, 4, gu, pv, ph, pl);
}

// W^T fragments (hi, lo of Wr and Wi) of i-blocks q0 and q0 + 1 (clamped to q0 past
// NI) for the rows of half sp of the staged chunk.
struct WtFrag {
    half8 wr[2][2], wi[2][2];             // [block][hi, lo]
};
template <int NI>
__device__ __forceinline__ void load_wt(WtFrag& f, const uint4* Tcur, int sp, int q0, int h, int i32) {
#pragma unroll
    for (int d = 0; d < 2; ++d) {
        const int q = q0 + d < NI ? q0 + d : q0;
        const uint4* lt = Tcur + (q * 16 + (sp * 2 + h) * 4) * 32 + i32;
        f.wr[d][0] = as_h8(lt[0]); f.wr[d][1] = as_h8(lt[32]);
        f.wi[d][0] = as_h8(lt[64]); f.wi[d][1] = as_h8(lt[96]);
    }
}

// gY[q0], gY[q0 + 1] += Wr^T P + Wi^T Q' over the rows of half sp: the two i-blocks
// alternate, so that four accumulations are in flight.
template <int NI>
__device__ __forceinline__ void mma_group(const WtFrag& f, int sp, int q0, const half8 (&ph)[2][4],
                                          const half8 (&pl)[2][4], floatx16 (&gyr)[NI], floatx16 (&gyi)[NI]) {
#pragma unroll
    for (int term = 0; term < 6; ++term) {
        const int wsel = term < 3 ? 0 : 1, whl = (term % 3) == 2 ? 1 : 0, phl = (term % 3) == 1 ? 1 : 0;
#pragma unroll
        for (int d = 0; d < 2; ++d) {
            if (q0 + d >= NI) continue;
            const half8 a = wsel ? f.wi[d][whl] : f.wr[d][whl];
            const half8 br = phl ? pl[sp][wsel * 2] : ph[sp][wsel * 2];
            const half8 bi = phl ? pl[sp][wsel * 2 + 1] : ph[sp][wsel * 2 + 1];
            gyr[q0 + d] = mfma16(a, br, gyr[q0 + d]);
            gyi[q0 + d] = mfma16(a, bi, gyi[q0 + d]);
        }
    }
}

// Scheduling hint for a half: NM groups of one MFMA followed by NV VALU
// instructions, so that the vector work of the next rows issues while the matrix
// cores work (one wave per SIMD: nothing else would fill those cycles).
template <int NM, int NV>
__device__ __forceinline__ void interleave_mfma_valu() {
#pragma unroll
    for (int i = 0; i < NM; ++i) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
        __builtin_amdgcn_sched_group_barrier(0x002, NV, 0);
    }
}

// Values a half produces for the next half are pinned before its barrier (an empty
// asm that reads and writes them), so that the compiler cannot sink their
// arithmetic past the barrier into the next half, where it would not overlap with
// matrix work.
__device__ __forceinline__ void pin_pq(half8 (&ph)[2][4], half8 (&pl)[2][4], int s) {
#pragma unroll
    for (int q = 0; q < 4; ++q) asm volatile("" : "+v"(ph[s][q]), "+v"(pl[s][q]));
}
__device__ __forceinline__ void pin_gu(floatx16 (&gu)[2]) {
    asm volatile("" : "+v"(gu[0]), "+v"(gu[1]));
}

// One 32-row chunk c in two halves.  On entry: P/Q' of rows 0-15 in ph/pl[0], gU of
// the chunk (scaled) in gu, the phase of rows 16-31 in pv[.][2..3], W^T of the chunk
// in Tcur.  First half: the W^T product over rows 0-15 while the modulus adjoint of
// rows 16-31 runs; the next chunk's W^T, split gV and phase of rows 0-15 are
// requested at its start.  Second half: the product over rows 16-31 while gU of the
// next chunk and the modulus adjoint of its rows 0-15 run; the phase of its rows
// 16-31 is requested at its start.  Each half ends with a full wait and a barrier,
// so every request has a half chunk of matrix work to land.  Within a half, each
// pair of i-blocks is one scheduling region: the W^T fragments of the next pair are
// read from LDS at its top (they land while its products run) and a share of the
// rows' modulus adjoint is interleaved with its products.
template <int NTB, int NI>
__device__ __forceinline__ void bwd_phase_chunk(int c, int nC, int wave, int lane, int tid, int h, int i32,
                                                const uint4 (&phv)[NTB * 2][2], const uint4* Tsrc, const uint4* Gb,
                                                uint4* Ls_G, const unsigned* pbase, int64_t spin_stride,
                                                int64_t c_stride, float c0, int64_t cstride, const uint4* Tcur,
                                                uint4* Tnext,
                                                floatx16 (&gyr)[NI], floatx16 (&gyi)[NI], floatx16 (&gu)[2],
                                                uint4 (&pv)[2][4], half8 (&ph)[2][4], half8 (&pl)[2][4]) {
    constexpr int NG = (NI + 1) / 2;             // pairs of i-blocks
    const int cn = c + 1 < nC ? c + 1 : c;       // the last chunk reloads itself
    WtFrag f[2];
    // ---- first half
    stage_t<NI>(Tnext, Tsrc, cn, cstride, wave, lane);
    stage_g<NTB>(Ls_G, Gb, cn, tid);
    load_phase_half(pv, 0, launder_v((const uint4*)(pbase + cn * c_stride)), spin_stride, c_stride / 4);
    load_wt<NI>(f[0], Tcur, 0, 0, h, i32);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int g = 0; g < NG; ++g) {
        if (g + 1 < NG) load_wt<NI>(f[(g + 1) & 1], Tcur, 0, 2 * (g + 1), h, i32);
        __builtin_amdgcn_sched_barrier(0);
        mma_group<NI>(f[g & 1], 0, 2 * g, ph, pl, gyr, gyi);
        modadj_pairs(1, g * 4 / NG, (g + 1) * 4 / NG, gu, pv, ph, pl);
        interleave_mfma_valu<24, 4>();
        __builtin_amdgcn_sched_barrier(0);
    }
    pin_pq(ph, pl, 1);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    // ---- second half
    load_phase_half(pv, 1, launder_v((const uint4*)(pbase + cn * c_stride)), spin_stride, c_stride / 4);
    load_wt<NI>(f[0], Tcur, 1, 0, h, i32);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int g = 0; g < NG; ++g) {
        if (g + 1 < NG) load_wt<NI>(f[(g + 1) & 1], Tcur, 1, 2 * (g + 1), h, i32);
        __builtin_amdgcn_sched_barrier(0);
        mma_group<NI>(f[g & 1], 1, 2 * g, ph, pl, gyr, gyi);
        if (g == 0) {
            gu_chunk<NTB>(Ls_G, phv, h, i32, c0, gu);
            if (NG == 1) modadj_pairs(0, 0, 4, gu, pv, ph, pl);
            interleave_mfma_valu<24 + 6 * NTB, 2>();
        } else {
            modadj_pairs(0, (g - 1) * 4 / (NG - 1), g * 4 / (NG - 1), gu, pv, ph, pl);
            interleave_mfma_valu<24, 5>();
        }
        __builtin_amdgcn_sched_barrier(0);
    }
    pin_pq(ph, pl, 0);
    pin_gu(gu);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
}

// Backward contraction from the stored phase: one signal, 128 columns t (four
// waves of 32), all rows l in 32-row chunks; gY accumulated in registers for the
// NI i-blocks q_base .. q_base + NI - 1 of the nit blocks of W^T (the register
// budget holds at most 8 at 32 frames; larger K runs as several launches over
// disjoint i-ranges, each repeating the modulus adjoint).
template <int NTB, int NI>
__global__ void __launch_bounds__(256) k_freq_bwd_p(const unsigned* __restrict__ phase, int64_t ph_bstride, int Tp,
                                                    int nTt, int nU, const unsigned short* __restrict__ WTsp,
                                                    int q_base, int nit,
                                                    int Mp, int Kp, const unsigned short* __restrict__ PhTsp,
                                                    float sphi, const uint4* __restrict__ Gs, int64_t gs_bstride,
                                                    const float* __restrict__ gvmax, int n_beta, int alpha,
                                                    int n_alpha, float sw, float2* __restrict__ gY,
                                                    int64_t gy_bstride) {
    constexpr int NTp = 32 * NTB;
    __shared__ uint4 Ls_T0[NI * 512];
    __shared__ uint4 Ls_T1[NI * 512];
    __shared__ uint4 Ls_G[gvs_chunk<NTB>()];
    const int u = blockIdx.x;
    if (u >= nU) return;                            // whole block
    const int64_t b = u / nTt;
    const int t0 = (u % nTt) * kTileTh;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int h = lane >> 5, i32 = lane & 31;
    const int tw0 = t0 + wave * 32;                 // this wave's columns
    const int nC = Mp / 32;

    float G = 0.f;
    for (int q = 0; q < 2 * n_beta; ++q) G = fmaxf(G, gvmax[(b * n_alpha + alpha) * 2 * n_beta + q]);
    const float spq = pow2_scale(2.f * G * 16384.f / sphi);
    const float c0 = spq / sphi * kSnormInv;

    floatx16 gyr[NI], gyi[NI];
#pragma unroll
    for (int q = 0; q < NI; ++q) { gyr[q] = z16(); gyi[q] = z16(); }

    const uint4* phrow = (const uint4*)(PhTsp + ((int64_t)(tw0 + i32) * (NTp / 8) + h) * 16);
    const uint4* Tsrc = (const uint4*)WTsp + (int64_t)q_base * 512;
    const int64_t cstride = (int64_t)nit * 512;
    const uint4* Gb = Gs + b * gs_bstride;
    // this lane's column of the stored phase, rows 4h.. of each 8-row group
    // (blocks [spin][Mp / 32], each four row groups of Tp x 8 elements)
    const unsigned* pbase = phase + b * ph_bstride + (int64_t)(tw0 + i32) * 8 + 4 * h;
    const int64_t spin_stride = (int64_t)Tp * Mp, c_stride = (int64_t)Tp * 32;

    uint4 phv[NTB * 2][2];
#pragma unroll
    for (int kb = 0; kb < NTB * 2; ++kb) {
        phv[kb][0] = phrow[4 * kb];
        phv[kb][1] = phrow[4 * kb + 1];
    }
    uint4 pv[2][4];
    floatx16 gu[2];
    half8 ph[2][4], pl[2][4];
    // chunk 0: operands, gU and the P/Q' of its rows 0-15
    stage_t<NI>(Ls_T0, Tsrc, 0, cstride, wave, lane);
    stage_g<NTB>(Ls_G, Gb, 0, tid);
    load_phase_half(pv, 0, (gptr<uint4>)pbase, spin_stride, c_stride / 4);
    load_phase_half(pv, 1, (gptr<uint4>)pbase, spin_stride, c_stride / 4);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    gu_chunk<NTB>(Ls_G, phv, h, i32, c0, gu);
    modadj_half(0, gu, pv, ph, pl);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    // nC is even (Mp is a multiple of 64): the W^T buffers alternate at compile time
    for (int c = 0; c < nC; c += 2) {
        bwd_phase_chunk<NTB, NI>(c, nC, wave, lane, tid, h, i32, phv, Tsrc, Gb, Ls_G, pbase, spin_stride, c_stride,
                                 c0, cstride, Ls_T0, Ls_T1, gyr, gyi, gu, pv, ph, pl);
        bwd_phase_chunk<NTB, NI>(c + 1, nC, wave, lane, tid, h, i32, phv, Tsrc, Gb, Ls_G, pbase, spin_stride,
                                 c_stride, c0, cstride, Ls_T1, Ls_T0, gyr, gyi, gu, pv, ph, pl);
    }
    const float inv = 1.f / (sw * spq);
    float2* o = gY + b * gy_bstride;
#pragma unroll
    for (int q = 0; q < NI; ++q)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int i = (q_base + q) * 32 + crow(r, h);
            if (i < Kp) o[(int64_t)i * Tp + tw0 + i32] = make_float2(gyr[q][r] * inv, gyi[q][r] * inv);
        }
}


// ------------------------------ backward from the stored phase, 16 x 16 tiles

// Row of the 32-row chunk that k-slot j (0..7) of lane group g holds in the
// W^H product of k_freq_bwd_q: 4 g + j, then 16 + 4 g + j - 4 -- the rows whose
// gU a lane holds after the 16 x 16 lowpass-adjoint products of the chunk's two
// 16-row halves, and whose stored phase it loads.
__device__ __forceinline__ int qrow(int g, int j) { return j < 4 ? 4 * g + j : 12 + 4 * g + j; }

// WTq[c][it][p][lane][j] = split(W[l][i] * sw), p = re hi, re lo, im hi, im lo, for
// i = 16 it + lane % 16 and l = 32 c + qrow(lane / 16, j): the A operand of the
// 16 x 16 x 32 W^H product, a chunk (KpT x 32) contiguous.  Rows i >= Kp are zero.
__global__ void k_wtqsplit(const float2* __restrict__ Wl, int Mp, int Kp, int KpT, float sw,
                           unsigned short* __restrict__ WTq) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)KpT * Mp) return;
    const int j = (int)(e & 7);
    const int lane = (int)((e >> 3) & 63);
    const int64_t r = e >> 9;
    const int nq = KpT / 16;
    const int it = (int)(r % nq);
    const int c = (int)(r / nq);
    const int i = 16 * it + (lane & 15);
    const int l = 32 * c + qrow(lane >> 4, j);
    const float2 w = i < Kp ? Wl[(int64_t)l * Kp + i] : make_float2(0.f, 0.f);
    _Float16 a, bb, cc, d;
    split_h(w.x * sw, a, bb);
    split_h(w.y * sw, cc, d);
    _Float16* o = (_Float16*)WTq + ((((int64_t)c * nq + it) * 4) * 64 + lane) * 8 + j;
    o[0] = a; o[512] = bb; o[1024] = cc; o[1536] = d;      // planes 64 lanes x 8 halves apart
}

// Power-of-two scales of the lane's gV rows of one 32-row chunk, per spin and
// 16-row half: rows 16 hf + 4 g4 .. + 3.  Read straight from the split-gV table;
// the chunk's address goes through launder_v, so that the compiler issues these
// loads where they stand instead of repeating them next to their uses, where
// they would wait behind the global-to-LDS copies.
struct GvScaleQ {
    float4 q[2][2];       // [spin][hf]
};
__device__ __forceinline__ void bwdq_load_scales(GvScaleQ& g, const uint4* Gb, int c, int g4) {
    gptr<uint4> Lg = launder_v(Gb + (int64_t)c * gvs_chunk<1>() + 512);
#pragma unroll
    for (int spin = 0; spin < 2; ++spin)
#pragma unroll
        for (int hf = 0; hf < 2; ++hf)
            g.q[spin][hf] = __builtin_bit_cast(float4, ((gptr<u32x4>)Lg)[spin * 8 + 4 * hf + g4]);
}

// One lowpass-adjoint product: gU of rows 16 hf + 4 g4 + r at the lane's column
// from the split gV rows of the chunk staged in Lg (unscaled; the row scales are
// applied by the modulus adjoint).
__device__ __forceinline__ floatx4 bwdq_gu(const uint4* Lg, int g4, int j16, int spin, int hf, half8 fh, half8 fl) {
    const int base = (((spin * 2 + (g4 >> 1)) * 2) * 2 + (g4 & 1)) * 32 + 16 * hf + j16;
    const half8 ah = as_h8(Lg[base]), al = as_h8(Lg[base + 64]);
    floatx4 acc = z4();
    acc = mfma16q(ah, fh, acc);
    acc = mfma16q(ah, fl, acc);
    acc = mfma16q(al, fh, acc);
    return acc;
}

// Modulus adjoint of the rows 16 hf + 4 g4 + 2 pr, + 1 (k-slots 4 hf + 2 pr, + 1):
// P = gZ_up + gZ_down, Q' = i (gZ_down - gZ_up) with gZ = gU u from the stored unit
// phase, split into FP16 hi / lo; word 2 hf + pr of the B planes (P re, P im, Q' re,
// Q' im).
__device__ __forceinline__ void bwdq_modadj(int hf, int pr, const floatx4 (&gu)[2][2], const GvScaleQ& g, float c0,
                                            const uint4 (&pv)[2][2], half8 (&bh)[4], half8 (&bl)[4]) {
    float vals[2][4];
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        const int r = 2 * pr + e;
        const unsigned wu = r == 0 ? pv[0][hf].x : r == 1 ? pv[0][hf].y : r == 2 ? pv[0][hf].z : pv[0][hf].w;
        const unsigned wd = r == 0 ? pv[1][hf].x : r == 1 ? pv[1][hf].y : r == 2 ? pv[1][hf].z : pv[1][hf].w;
        const float qu = r == 0 ? g.q[0][hf].x : r == 1 ? g.q[0][hf].y : r == 2 ? g.q[0][hf].z : g.q[0][hf].w;
        const float qd = r == 0 ? g.q[1][hf].x : r == 1 ? g.q[1][hf].y : r == 2 ? g.q[1][hf].z : g.q[1][hf].w;
        const float ux = (float)(int)(short)(wu & 0xffffu), uy = (float)((int)wu >> 16);
        const float dx = (float)(int)(short)(wd & 0xffffu), dy = (float)((int)wd >> 16);
        const float su = gu[0][hf][r] * (qu * c0), sd = gu[1][hf][r] * (qd * c0);
        vals[e][0] = su * ux + sd * dx;
        vals[e][1] = su * uy + sd * dy;
        vals[e][2] = su * uy - sd * dy;
        vals[e][3] = sd * dx - su * ux;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        unsigned hp, lp;
        split2(vals[0][q], vals[1][q], hp, lp);
        const int w = 2 * hf + pr;
        uint4 hv = __builtin_bit_cast(uint4, bh[q]), lv = __builtin_bit_cast(uint4, bl[q]);
        if (w == 0) { hv.x = hp; lv.x = lp; }
        else if (w == 1) { hv.y = hp; lv.y = lp; }
        else if (w == 2) { hv.z = hp; lv.z = lp; }
        else { hv.w = hp; lv.w = lp; }
        bh[q] = __builtin_bit_cast(half8, hv);
        bl[q] = __builtin_bit_cast(half8, lv);
    }
}

// the lane's stored phase of a chunk: [spin][hf], four rows of one column each
__device__ __forceinline__ void bwdq_load_phase(uint4 (&pv)[2][2], const unsigned* pbase, int c, int g4,
                                                int64_t spin_stride, int64_t c_stride, int64_t g_stride) {
    gptr<uint4> base = launder_v((const uint4*)(pbase + c * c_stride));
#pragma unroll
    for (int spin = 0; spin < 2; ++spin)
#pragma unroll
        for (int hf = 0; hf < 2; ++hf) {
            gptr<u32x4> p = (gptr<u32x4>)(base + (spin * spin_stride + ((g4 >> 1) + 2 * hf) * g_stride) / 4);
            pv[spin][hf] = __builtin_bit_cast(uint4, __builtin_nontemporal_load(p));   // read once
        }
}

// Half h (i-tiles NI h .. NI h + NI - 1, NI x 4 KB) of the W^T chunk c into LDS by
// direct global-to-LDS loads: NI per thread of the 256.  A chunk's i-tiles are
// contiguous in the table, each [plane][lane].
// (wave is passed wave-uniform, so that the LDS destinations are scalar.)
template <int NI>
__device__ __forceinline__ void bwdq_stage_half(uint4* Ls, const uint4* WTq, int c, int h, int tid, int wave) {
    const uint4* src = WTq + (int64_t)c * (NI * 512) + h * (NI * 256);
    const uint32_t off = (uint32_t)tid * 16u;
#pragma unroll
    for (int k = 0; k < NI; ++k) dma16(src + k * 256, off, Ls + k * 256 + wave * 64);
}
// the split gV rows of chunk c (8 KB, without the scales) the same way
__device__ __forceinline__ void bwdq_stage_g(uint4* Ls, const uint4* Gb, int c, int tid, int wave) {
    const uint4* src = Gb + (int64_t)c * gvs_chunk<1>();
    const uint32_t off = (uint32_t)tid * 16u;
#pragma unroll
    for (int k = 0; k < 2; ++k) dma16(src + k * 256, off, Ls + k * 256 + wave * 64);
}

// The W^T products of i-tiles IT0 .. IT0 + NI - 1 (one half of the chunk, staged in
// Lh), one scheduling region per i-tile; the work of chunk c + 1 placed in this
// half (CHAINS: the four lowpass-adjoint chains from the gV rows in Lg; else the
// four modulus-adjoint shares) is spread over the regions.
template <int NI, int IT0, bool CHAINS>
__device__ __forceinline__ void bwdq_half(const uint4* Lh, const uint4* Lg, int lane, int g4, int j16, half8 fh,
                                          half8 fl, float c0, const half8 (&bh)[4], const half8 (&bl)[4],
                                          half8 (&nh)[4], half8 (&nl)[4], const uint4 (&pnext)[2][2],
                                          const GvScaleQ& snext, floatx4 (&gu)[2][2], floatx4 (&gyr)[2 * NI],
                                          floatx4 (&gyi)[2 * NI]) {
    const uint4* Lt = Lh + lane;
    uint4 wc[4], wn[4];
#pragma unroll
    for (int p = 0; p < 4; ++p) wc[p] = Lt[p * 64];
#pragma unroll
    for (int j = 0; j < NI; ++j) {
        const int it = IT0 + j;
        if (j + 1 < NI) {
#pragma unroll
            for (int p = 0; p < 4; ++p) wn[p] = Lt[((j + 1) * 4 + p) * 64];
        }
        const half8 wrh = as_h8(wc[0]), wrl = as_h8(wc[1]), wih = as_h8(wc[2]), wil = as_h8(wc[3]);
        gyr[it] = mfma16q(wrh, bh[0], gyr[it]); gyi[it] = mfma16q(wrh, bh[1], gyi[it]);
        gyr[it] = mfma16q(wrh, bl[0], gyr[it]); gyi[it] = mfma16q(wrh, bl[1], gyi[it]);
        gyr[it] = mfma16q(wrl, bh[0], gyr[it]); gyi[it] = mfma16q(wrl, bh[1], gyi[it]);
        gyr[it] = mfma16q(wih, bh[2], gyr[it]); gyi[it] = mfma16q(wih, bh[3], gyi[it]);
        gyr[it] = mfma16q(wih, bl[2], gyr[it]); gyi[it] = mfma16q(wih, bl[3], gyi[it]);
        gyr[it] = mfma16q(wil, bh[2], gyr[it]); gyi[it] = mfma16q(wil, bh[3], gyi[it]);
        // event k (chain (spin k & 1, half k >> 1), or share (half k >> 1, pair k & 1))
        // in region (k NI) / 4 of the half
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if ((k * NI) / 4 != j) continue;
            if constexpr (CHAINS) {
                gu[k & 1][k >> 1] = bwdq_gu(Lg, g4, j16, k & 1, k >> 1, fh, fl);
            } else {
                bwdq_modadj(k >> 1, k & 1, gu, snext, c0, pnext, nh, nl);
                interleave_mfma_valu<12, 4>();
            }
        }
#pragma unroll
        for (int p = 0; p < 4; ++p) wc[p] = wn[p];
        __builtin_amdgcn_sched_barrier(0);
    }
}

// Backward contraction from the stored phase in 16 x 16 tiles: one signal, 64
// columns t (four waves of 16, one per SIMD), all rows l in 32-row chunks, all NI
// pairs of 16-row i-tiles accumulated in registers (16 NI of them per lane), so
// that any K the split forward handles runs in one pass over the phase.
// Per chunk:
//   gU[l][t] = sum_tau gV[l][tau] Phi[t][tau]       (16 x 16 x 32, both spins, both row halves)
//   P, Q' from gU and the stored unit phase         (the lane's eight rows of its column)
//   gY[i][t] += sum_l Wr[l][i] P[l][t] + Wi[l][i] Q'[l][t]
// pipelined so that the first two steps of chunk c + 1 run during the third of
// chunk c.  The W^T chunk is staged in two halves by i-range, X (first NI
// i-tiles) and Y (the rest), and the split gV rows in G, each a distinct LDS array
// filled by direct global-to-LDS loads (8 NI + 8 KB in all):
//   chunk start: Y <- W^T(c) second half; phase of chunk c + 2 requested
//   first half:  products with X; lowpass-adjoint chains of chunk c + 1 from G
//   full wait, barrier
//   middle:      X <- W^T(c + 1) first half, G <- gV rows of chunk c + 2; their
//                scales requested
//   second half: products with Y; modulus adjoint of chunk c + 1
//   full wait, barrier
// Every copy thus has half a chunk of products to land, the arrays read in a half
// are never the ones being filled (so the compiler adds no wait for the copies
// before those reads), and nothing requested into registers is used before the
// next barrier (a wait for a register load while a copy is in flight is a wait
// for everything).  The last chunks request their own operands again.
template <int NI>
__global__ void __launch_bounds__(256) k_freq_bwd_q(const unsigned* __restrict__ phase, int64_t ph_bstride, int Tp,
                                                    int nTt, int nU, const unsigned short* __restrict__ WTq, int Mp,
                                                    int Kp, const unsigned short* __restrict__ PhTsp, float sphi,
                                                    const uint4* __restrict__ Gs, int64_t gs_bstride,
                                                    const float* __restrict__ gvmax, int n_beta, int alpha,
                                                    int n_alpha, float sw, float2* __restrict__ gY,
                                                    int64_t gy_bstride) {
    constexpr int NTp = 32, NQ = 2 * NI;
    __shared__ uint4 Ls_X[NI * 256];
    __shared__ uint4 Ls_Y[NI * 256];
    __shared__ uint4 Ls_G[512];
    const int u = blockIdx.x;
    if (u >= nU) return;                              // whole block
    const int64_t b = u / nTt;
    const int t0 = (u % nTt) * 64;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int j16 = lane & 15, g4 = lane >> 4;
    const int t = t0 + wave * 16 + j16;               // this lane's column
    const int nC = Mp / 32;

    float G = 0.f;
    for (int q = 0; q < 2 * n_beta; ++q) G = fmaxf(G, gvmax[(b * n_alpha + alpha) * 2 * n_beta + q]);
    const float spq = pow2_scale(2.f * G * 16384.f / sphi);
    const float c0 = spq / sphi * kSnormInv;

    floatx4 gyr[NQ], gyi[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) { gyr[q] = z4(); gyi[q] = z4(); }

    // Phi of the lane's column, tau 8 g4 .. 8 g4 + 7: hi and lo planes
    const uint4* phrow = (const uint4*)(PhTsp + ((int64_t)t * (NTp / 8) + g4) * 16);
    const half8 fh = as_h8(phrow[0]), fl = as_h8(phrow[1]);
    const uint4* Gb = Gs + b * gs_bstride;
    const uint4* Wt = (const uint4*)WTq;
    // the lane's phase rows: 4 (g4 % 2) .. of row group g4 / 2 (rows 4 g4 ..) and of
    // group 2 + g4 / 2 (rows 16 + 4 g4 ..)
    const unsigned* pbase = phase + b * ph_bstride + (int64_t)t * 8 + 4 * (g4 & 1);
    const int64_t spin_stride = (int64_t)Tp * Mp, c_stride = (int64_t)Tp * 32, g_stride = (int64_t)Tp * 8;
    const int one = 1 < nC ? 1 : 0;

    // chunk 0's B operands from its gV rows, scales and phase; then the gV rows of
    // chunk 1 into G, and the first half of W^T(0) into X
    half8 bh[4], bl[4];
    uint4 pnext[2][2];
    GvScaleQ snext;
    {
        uint4 p0[2][2];
        GvScaleQ s0;
        bwdq_load_phase(p0, pbase, 0, g4, spin_stride, c_stride, g_stride);
        bwdq_load_scales(s0, Gb, 0, g4);
        bwdq_stage_g(Ls_G, Gb, 0, tid, wave);
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        floatx4 gu[2][2];
#pragma unroll
        for (int k = 0; k < 4; ++k) gu[k & 1][k >> 1] = bwdq_gu(Ls_G, g4, j16, k & 1, k >> 1, fh, fl);
#pragma unroll
        for (int uu = 0; uu < 4; ++uu) bwdq_modadj(uu >> 1, uu & 1, gu, s0, c0, p0, bh, bl);
    }
    __syncthreads();                                  // every wave is done with chunk 0's gV rows
    bwdq_load_phase(pnext, pbase, one, g4, spin_stride, c_stride, g_stride);
    bwdq_load_scales(snext, Gb, one, g4);
    bwdq_stage_g(Ls_G, Gb, one, tid, wave);
    bwdq_stage_half<NI>(Ls_X, Wt, 0, 0, tid, wave);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();

    for (int c = 0; c < nC; ++c) {
        const int c1 = c + 1 < nC ? c + 1 : nC - 1, c2 = c + 2 < nC ? c + 2 : nC - 1;
        uint4 pfree[2][2];
        GvScaleQ sfree;
        half8 nh[4], nl[4];
        floatx4 gu[2][2];
        bwdq_stage_half<NI>(Ls_Y, Wt, c, 1, tid, wave);
        bwdq_load_phase(pfree, pbase, c2, g4, spin_stride, c_stride, g_stride);
        bwdq_half<NI, 0, true>(Ls_X, Ls_G, lane, g4, j16, fh, fl, c0, bh, bl, nh, nl, pnext, snext, gu, gyr, gyi);
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        bwdq_stage_half<NI>(Ls_X, Wt, c1, 0, tid, wave);
        bwdq_stage_g(Ls_G, Gb, c2, tid, wave);
        bwdq_load_scales(sfree, Gb, c2, g4);
        bwdq_half<NI, NI, false>(Ls_Y, Ls_G, lane, g4, j16, fh, fl, c0, bh, bl, nh, nl, pnext, snext, gu, gyr, gyi);
#pragma unroll
        for (int q = 0; q < 4; ++q) asm volatile("" : "+v"(nh[q]), "+v"(nl[q]));
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 4; ++q) { bh[q] = nh[q]; bl[q] = nl[q]; }
#pragma unroll
        for (int s2 = 0; s2 < 2; ++s2) { pnext[s2][0] = pfree[s2][0]; pnext[s2][1] = pfree[s2][1]; }
        snext = sfree;
    }
    const float inv = 1.f / (sw * spq);
    float2* o = gY + b * gy_bstride;
#pragma unroll
    for (int it = 0; it < NQ; ++it)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = 16 * it + 4 * g4 + r;
            if (i < Kp) o[(int64_t)i * Tp + t] = make_float2(gyr[it][r] * inv, gyi[it][r] * inv);
        }
}

}  // namespace jtfs

using namespace jtfs;

namespace jtfs {

size_t split_fwd_lds(const Shapes& s, bool with_phase);
int bwdp_max_ni(int NTp);

bool split_supported(const Shapes& s) { return split_fwd_lds(s, false) <= (size_t)kMaxDynLds && s.NTp <= 64; }

// LDS of k_freq_fwd_h: resident W rows during the main loop (with the stored phase
// also a transpose area of 32 or 8 rows of 36 elements per wave), then the
// cross-wave reduction buffer (8 waves x 2 spins x 64 lanes x 16 floats).
size_t split_fwd_lds(const Shapes& s, bool with_phase) {
    const size_t wres = (size_t)64 * (s.Kp * 8 + 16);
    const size_t trans = wres + (size_t)8 * 32 * 36 * 4 <= (size_t)kMaxDynLds ? 32 : 8;   // kPhaseTrp
    const size_t main_loop = wres + (with_phase ? (size_t)8 * trans * 36 * 4 : 0);
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
    if (s.NTp == 32) {
        // the W^T operand of the 16 x 16-tile stored-phase backward
        P->WTq = (unsigned short*)alloc(sizeof(float2) * (size_t)P->KpT * s.Mp);
        if (!P->WTq) { set_error("device allocation failed"); return JTFS_ENOMEM; }
        const int64_t n = (int64_t)P->KpT * s.Mp;
        hipLaunchKernelGGL(k_wtqsplit, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, 0, P->Wl, s.Mp, s.Kp, P->KpT,
                           P->sw, P->WTq);
    }
    if (s.NTp == 32) {
        // the W and lowpass operands of the 16 x 16-tile forward
        const int ns = (s.Kp / 16 + 1) / 2;
        const int64_t nq = (int64_t)s.Mp * ns * 128;     // halves: Mp / 64 tiles x ns k-steps x 16 KB
        P->Wq = (unsigned short*)alloc(sizeof(unsigned short) * nq);
        P->Phq = (unsigned short*)alloc(sizeof(float) * s.sumTp * s.NTp);
        if (!P->Wq || !P->Phq) { set_error("device allocation failed"); return JTFS_ENOMEM; }
        hipLaunchKernelGGL(k_wqsplit, dim3((unsigned)((nq + 255) / 256)), dim3(256), 0, 0, P->Wl, s.Mp, s.Kp, ns, P->sw,
                           P->Wq);
        for (int a = 0; a < s.n_alpha; ++a) {
            const int64_t n = (int64_t)s.Tp[a] * s.NTp;
            hipLaunchKernelGGL(k_phqsplit, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, 0, P->Phi + s.phioff[a],
                               s.Tp[a], s.NTp, P->sphi[a], P->Phq + s.phioff[a] * 2);
        }
    }
    if (hipGetLastError() != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
        set_error("split-operand construction failed"); return JTFS_EHIP; }
    {
        const int NI = P->KpT / 32;
        // recomputing backward: static LDS of a W chunk and two W^T chunks, 24 NI KB
        // (<= 160 KB), and one wave per SIMD without scratch
        P->split_bwd_ok = (s.NTp == 32 && NI <= 6) || (s.NTp == 64 && NI <= 5);
        // stored-phase backward: two W^T chunks (16 NI KB) per launch, at most two
        // launches over halves of the i-blocks; the forward must hold its phase
        // transpose area beside the resident W tile
        P->split_bwdp_ok = NI <= 2 * bwdp_max_ni(s.NTp) && split_fwd_lds(s, true) <= (size_t)kMaxDynLds;
    }
    P->contraction = JTFS_CONTRACTION_SPLIT_F16;
    return JTFS_OK;
}

// largest K (in k-steps of 16) whose resident W tile fits the dynamic LDS limit
constexpr int kMaxFwdNK = (kMaxDynLds / 64 - 16) / 8 / 16;

template <int NTB, int NK = 1>
static int fwd_attributes() {
    if constexpr (NK > kMaxFwdNK) {
        return JTFS_OK;
    } else {
        if (hipFuncSetAttribute((const void*)k_freq_fwd_h<NTB, NK>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                kMaxDynLds) != hipSuccess) {
            set_error("hipFuncSetAttribute failed for the split contraction");
            return JTFS_EHIP;
        }
        return fwd_attributes<NTB, NK + 1>();
    }
}

template <int NTQ, int NK = 1>
static int fwdq_attributes() {
    if constexpr (NK > kMaxFwdNK) {
        return JTFS_OK;
    } else {
        if (hipFuncSetAttribute((const void*)k_freq_fwd_q<NK, NTQ>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                kMaxDynLds) != hipSuccess) {
            set_error("hipFuncSetAttribute failed for the split contraction");
            return JTFS_EHIP;
        }
        return fwdq_attributes<NTQ, NK + 1>();
    }
}

int split_attributes() {
    // the backward kernels use static LDS only; the forward takes it dynamically
    int rc = fwd_attributes<1>();
    if (rc == JTFS_OK) rc = fwd_attributes<2>();
    if (rc == JTFS_OK) rc = fwdq_attributes<1>();
    if (rc == JTFS_OK) rc = fwdq_attributes<2>();
    return rc;
}

template <int NTQ, int NK = 1, typename... Args>
static void launch_fwdq_nk(int nk, dim3 grid, size_t lds, hipStream_t st, Args... args) {
    if constexpr (NK <= kMaxFwdNK) {
        if (nk == NK) hipLaunchKernelGGL((k_freq_fwd_q<NK, NTQ>), grid, dim3(512), lds, st, args...);
        else launch_fwdq_nk<NTQ, NK + 1>(nk, grid, lds, st, args...);
    }
}

// whether the 16 x 16-tile forward handles the plan's shapes (N/T <= 32, LDS)
bool fwdq_supported(const jtfs_plan* P, bool with_phase) {
    const Shapes& s = P->s;
    const int ntq = (s.NT + 15) / 16;
    return P->Phq && P->Wq && s.NTp == 32 && ntq <= 2 && s.Kp / 16 <= kMaxFwdNK &&
           fwdq_lds(s.Kp, ntq, with_phase) <= (size_t)kMaxDynLds;
}

template <int NTB, int NK = 1, typename... Args>
static void launch_fwd_nk(int nk, dim3 grid, size_t lds, hipStream_t st, Args... args) {
    if constexpr (NK <= kMaxFwdNK) {
        if (nk == NK) hipLaunchKernelGGL((k_freq_fwd_h<NTB, NK>), grid, dim3(512), lds, st, args...);
        else launch_fwd_nk<NTB, NK + 1>(nk, grid, lds, st, args...);
    }
}

int launch_ysplit(const jtfs_plan* P, int a, const float2* Y2, const float* rowmax, unsigned short* Yh, float* yscale,
                  int64_t B, hipStream_t st) {
    const Shapes& s = P->s;
    const int64_t yb = (int64_t)s.Kp * s.sumTp;
    // chunks of 32 rows spread over grid z until there are about 2048 workgroups
    const int64_t base = (int64_t)(s.Tp[a] / 64) * B;
    const int nchunk = (s.Kp + 31) / 32;
    const int z = (int)std::max<int64_t>(1, std::min<int64_t>(nchunk, (2048 + base - 1) / base));
    hipLaunchKernelGGL(k_ysplit, dim3(s.Tp[a] / 64, (unsigned)B, (unsigned)z), dim3(256), 0, st, Y2 + s.yoff[a], yb,
                       s.Tp[a], s.Kp, rowmax, a, s.n_alpha, Yh + s.yoff[a] * 4, yscale);
    return hipGetLastError() == hipSuccess ? JTFS_OK : JTFS_EHIP;
}

int launch_freq_fwd_split(const jtfs_plan* P, int a, const unsigned short* Yh, const float* yscale, float* Vp,
                          int64_t vp_bstride, unsigned* phase, int64_t ph_bstride, int64_t B, hipStream_t st) {
    const Shapes& s = P->s;
    const int nlt = s.Mp / kTileL;
    const int nU = (int)(B * s.nch[a]);
    const unsigned grid = (unsigned)(((nU + 7) / 8) * 8 * nlt);
    const int64_t yhb = (int64_t)s.Kp * s.sumTp * 4;
    const float unscale = 1.f / (P->sw * P->sphi[a]);
    const size_t lds = split_fwd_lds(s, phase != nullptr);
    if (lds > (size_t)kMaxDynLds) { set_error("K beyond the split contraction's LDS tile"); return JTFS_ENOTSUP; }
    const unsigned short* Ya = Yh + s.yoff[a] * 4;
    const unsigned short* Ph = P->Phsp + s.phioff[a] * 2;
    const int slot0 = (int)s.vchoff[a];
    const int nk = s.Kp / 16;
    if (nk < 1 || nk > kMaxFwdNK) { set_error("K beyond the split contraction's LDS tile"); return JTFS_ENOTSUP; }
    // this rate's block of the stored phase (2 Mp Tp elements) after the rates before it
    unsigned* pha = phase ? phase + (int64_t)2 * s.Mp * (s.yoff[a] / s.Kp) : nullptr;
    if (P->tune.fwd16 && fwdq_supported(P, phase != nullptr)) {
        const int ntq = (s.NT + 15) / 16;
        const size_t ldsq = fwdq_lds(s.Kp, ntq, phase != nullptr);
        const unsigned short* Pq = P->Phq + s.phioff[a] * 2;
        if (ntq == 1)
            launch_fwdq_nk<1>(nk, dim3(grid), ldsq, st, Ya, yhb, s.Tp[a], s.chunk[a], s.nch[a], nU, nlt, (const unsigned short*)P->Wq, Pq, unscale, yscale, a, s.n_alpha, Vp, vp_bstride, slot0, pha, ph_bstride, P->sw);
        else
            launch_fwdq_nk<2>(nk, dim3(grid), ldsq, st, Ya, yhb, s.Tp[a], s.chunk[a], s.nch[a], nU, nlt, (const unsigned short*)P->Wq, Pq, unscale, yscale, a, s.n_alpha, Vp, vp_bstride, slot0, pha, ph_bstride, P->sw);
        return hipGetLastError() == hipSuccess ? JTFS_OK : JTFS_EHIP;
    }
    switch (s.NTp / 32) {
        case 1: launch_fwd_nk<1>(nk, dim3(grid), lds, st, Ya, yhb, s.Tp[a], s.chunk[a], s.nch[a], nU, nlt, (const unsigned short*)P->Wsp, Ph, unscale, yscale, a, s.n_alpha, Vp, vp_bstride, slot0, pha, ph_bstride, P->sw); break;
        case 2: launch_fwd_nk<2>(nk, dim3(grid), lds, st, Ya, yhb, s.Tp[a], s.chunk[a], s.nch[a], nU, nlt, (const unsigned short*)P->Wsp, Ph, unscale, yscale, a, s.n_alpha, Vp, vp_bstride, slot0, pha, ph_bstride, P->sw); break;
        default: set_error("unsupported N/T"); return JTFS_ENOTSUP;
    }
    return hipGetLastError() == hipSuccess ? JTFS_OK : JTFS_EHIP;
}

template <int NTB>
static void launch_bwd_ni(int NI, int NK, dim3 grid, hipStream_t st, const unsigned short* Ya, int64_t yhb, int Tp,
                          int nTt, int nU, const jtfs_plan* P, const unsigned short* PhT, float sphi,
                          const float* gVa, int64_t gvb, const float* gvmax, const float* yscale, int a, float2* gYa,
                          int64_t gyb) {
    const Shapes& s = P->s;
    // NK = Kp / 16 k-steps is 2 NI - 1 or 2 NI (Kp is a multiple of 16, KpT = 32 NI)
#define JTFS_BWD_CASE(ni)                                                                                      \
    case ni:                                                                                                   \
        if (NK == 2 * ni)                                                                                      \
            hipLaunchKernelGGL((k_freq_bwd_h<NTB, ni, 2 * ni>), grid, dim3(256), 0, st, Ya, yhb, Tp, nTt, nU, \
                               P->Wsp, P->WTsp, s.Mp, PhT, sphi, gVa, gvb, gvmax, s.n_beta, yscale, a,         \
                               s.n_alpha, P->sw, gYa, gyb);                                                    \
        else                                                                                                   \
            hipLaunchKernelGGL((k_freq_bwd_h<NTB, ni, 2 * ni - 1>), grid, dim3(256), 0, st, Ya, yhb, Tp, nTt, \
                               nU, P->Wsp, P->WTsp, s.Mp, PhT, sphi, gVa, gvb, gvmax, s.n_beta, yscale, a,     \
                               s.n_alpha, P->sw, gYa, gyb);                                                    \
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
        case 1: launch_bwd_ni<1>(NI, s.Kp / 16, dim3(nU), st, Ya, yhb, s.Tp[a], nTt, nU, P, PhT, P->sphi[a], gVa, gvb, gvmax, yscale, a, gYa, yb); break;
        case 2: launch_bwd_ni<2>(NI, s.Kp / 16, dim3(nU), st, Ya, yhb, s.Tp[a], nTt, nU, P, PhT, P->sphi[a], gVa, gvb, gvmax, yscale, a, gYa, yb); break;
        default: set_error("unsupported N/T"); return JTFS_ENOTSUP;
    }
    return hipGetLastError() == hipSuccess ? JTFS_OK : JTFS_EHIP;
}

// i-blocks one phase-backward workgroup holds in registers without scratch
// (one wave per SIMD): 8 at 32 frames, 5 at 64
int bwdp_max_ni(int NTp) { return NTp == 32 ? 8 : NTp == 64 ? 5 : 0; }

template <int NTB>
static void launch_bwdp_ni(int NI, int q_base, int nit, dim3 grid, hipStream_t st, const unsigned* pha, int64_t phb,
                           int Tp, int nTt, int nU, const jtfs_plan* P, const unsigned short* PhT, float sphi,
                           const uint4* Gsa, int64_t gsb, const float* gvmax, int a, float2* gYa, int64_t gyb) {
    const Shapes& s = P->s;
#define JTFS_BWDP_CASE(ni)                                                                                    \
    case ni:                                                                                                  \
        hipLaunchKernelGGL((k_freq_bwd_p<NTB, ni>), grid, dim3(256), 0, st, pha, phb, Tp, nTt, nU, P->WTsp, \
                           q_base, nit, s.Mp, s.Kp, PhT, sphi, Gsa, gsb, gvmax, s.n_beta, a, s.n_alpha, P->sw, \
                           gYa, gyb);                                                                         \
        break;
    if constexpr (NTB == 1) {
        switch (NI) {
            JTFS_BWDP_CASE(1) JTFS_BWDP_CASE(2) JTFS_BWDP_CASE(3) JTFS_BWDP_CASE(4)
            JTFS_BWDP_CASE(5) JTFS_BWDP_CASE(6) JTFS_BWDP_CASE(7) JTFS_BWDP_CASE(8)
            default: break;
        }
    } else {
        switch (NI) {
            JTFS_BWDP_CASE(1) JTFS_BWDP_CASE(2) JTFS_BWDP_CASE(3) JTFS_BWDP_CASE(4) JTFS_BWDP_CASE(5)
            default: break;
        }
    }
#undef JTFS_BWDP_CASE
}

int launch_gv_split(const jtfs_plan* P, const float* gV, uint4* Gs, int64_t B, hipStream_t st) {
    const Shapes& s = P->s;
    const int64_t nrows = B * s.n_alpha * 2 * (int64_t)s.Mp;
    const unsigned grid = (unsigned)((nrows + 255) / 256);
    switch (s.NTp / 32) {
        case 1: hipLaunchKernelGGL(k_gvsplit<1>, dim3(grid), dim3(256), 0, st, gV, s.Mp, nrows, Gs); break;
        case 2: hipLaunchKernelGGL(k_gvsplit<2>, dim3(grid), dim3(256), 0, st, gV, s.Mp, nrows, Gs); break;
        default: set_error("unsupported N/T"); return JTFS_ENOTSUP;
    }
    return hipGetLastError() == hipSuccess ? JTFS_OK : JTFS_EHIP;
}

bool bwdq_supported(const jtfs_plan* P) {
    const int NI = P->KpT / 32;
    return P->WTq && P->s.NTp == 32 && NI >= 1 && NI <= 9;          // LDS: two W^T chunks of NI x 8 KB
}

template <int NI = 1>
static void launch_bwdq_ni(int ni, unsigned nU, hipStream_t st, const unsigned* pha, int64_t phb, int Tp, int nTt,
                           const jtfs_plan* P, const unsigned short* PhT, float sphi, const uint4* Gsa, int64_t gsb,
                           const float* gvmax, int a, float2* gYa, int64_t gyb) {
    if constexpr (NI <= 9) {
        if (ni != NI) {
            launch_bwdq_ni<NI + 1>(ni, nU, st, pha, phb, Tp, nTt, P, PhT, sphi, Gsa, gsb, gvmax, a, gYa, gyb);
            return;
        }
        const Shapes& s = P->s;
        hipLaunchKernelGGL((k_freq_bwd_q<NI>), dim3(nU), dim3(256), 0, st, pha, phb, Tp, nTt, (int)nU, P->WTq, s.Mp,
                           s.Kp, PhT, sphi, Gsa, gsb, gvmax, s.n_beta, a, s.n_alpha, P->sw, gYa, gyb);
    }
}

int launch_freq_bwd_phase(const jtfs_plan* P, int a, const unsigned* phase, int64_t ph_bstride, const uint4* Gs,
                          int64_t gs_bstride, const float* gvmax, float2* gY2, int64_t B, hipStream_t st) {
    const Shapes& s = P->s;
    const int NI = P->KpT / 32;
    if (P->tune.bwd16 && bwdq_supported(P)) {
        const int nTt = s.Tp[a] / 64;
        const unsigned nU = (unsigned)(B * nTt);
        const int64_t yb = (int64_t)s.Kp * s.sumTp;
        const unsigned* pha = phase + (int64_t)2 * s.Mp * (s.yoff[a] / s.Kp);
        const unsigned short* PhT = P->PhTsp + s.phioff[a] * 2;
        const uint4* Gsa = Gs + (int64_t)a * (s.Mp / 32) * (512 * (s.NTp / 32) + 16);
        JTFS_TIMED(JTFS_STAGE_FREQ_ADJ_PQ, st,
                   launch_bwdq_ni(NI, nU, st, pha, ph_bstride, s.Tp[a], nTt, P, PhT, P->sphi[a], Gsa, gs_bstride, gvmax,
                                  a, gY2 + s.yoff[a], yb));
        return hipGetLastError() == hipSuccess ? JTFS_OK : JTFS_EHIP;
    }
    if (!P->split_bwdp_ok) { set_error("stored-phase backward not available for these shapes"); return JTFS_ENOTSUP; }
    // one launch per range of i-blocks: a single one up to the register budget, else
    // two balanced halves
    const int nmax = bwdp_max_ni(s.NTp);
    const int ng = NI <= nmax ? 1 : 2;
    const int nia = (NI + ng - 1) / ng;
    const int nTt = s.Tp[a] / kTileTh;
    const int nU = (int)(B * nTt);
    const int64_t yb = (int64_t)s.Kp * s.sumTp;
    const unsigned* pha = phase + (int64_t)2 * s.Mp * (s.yoff[a] / s.Kp);
    const unsigned short* PhT = P->PhTsp + s.phioff[a] * 2;
    // this rate's chunks of the split gV
    const uint4* Gsa = Gs + (int64_t)a * (s.Mp / 32) * (512 * (s.NTp / 32) + 16);
    float2* gYa = gY2 + s.yoff[a];
    for (int g = 0, q0 = 0; g < ng; ++g) {
        const int ni = g == 0 ? nia : NI - nia;
        switch (s.NTp / 32) {
            case 1: JTFS_TIMED(JTFS_STAGE_FREQ_ADJ_PQ, st, launch_bwdp_ni<1>(ni, q0, NI, dim3(nU), st, pha, ph_bstride, s.Tp[a], nTt, nU, P, PhT, P->sphi[a], Gsa, gs_bstride, gvmax, a, gYa, yb)); break;
            case 2: JTFS_TIMED(JTFS_STAGE_FREQ_ADJ_PQ, st, launch_bwdp_ni<2>(ni, q0, NI, dim3(nU), st, pha, ph_bstride, s.Tp[a], nTt, nU, P, PhT, P->sphi[a], Gsa, gs_bstride, gvmax, a, gYa, yb)); break;
            default: set_error("unsupported N/T"); return JTFS_ENOTSUP;
        }
        q0 += ni;
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
    if (mode == JTFS_CONTRACTION_SPLIT_F16_PHASE) {
        if (!P->split_ok || !P->split_bwdp_ok || P->s.tscat) {
            set_error("split-FP16 contraction with stored phase not available for these shapes");
            return JTFS_ENOTSUP;
        }
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
