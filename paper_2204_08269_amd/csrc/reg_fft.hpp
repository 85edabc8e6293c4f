// Block-wide power-of-two FFT with the data resident in registers.
//
// Each of the T = 2^LOGN / E threads holds E complex values.  Passes are Stockham
// radix-16 where a thread holds 16 values, else radix-8 (then one shorter pass);
// between passes the values move to
// the thread that needs them through LDS as 8-byte complex values (one exchange
// and two barriers per pass), in a buffer of n complex slots plus at most four pad
// slots per 32.  Unnormalised in both directions; twiddles from the FP64-generated table
// tw[k] = exp(-2 pi i k / 2^tw_log).
//
// The length and the thread count are compile-time constants: every position a
// thread reads or writes is then its thread index plus a constant, so the LDS
// exchanges take immediate offsets instead of one address register per element.
#pragma once

#include <hip/hip_runtime.h>

#include "fft_lds.hpp"

namespace jtfs {

// radix (log2) of the full passes with E values per thread by default: 16 (one
// butterfly per thread and pass) when E >= 16, else 8
constexpr int reg_lr_max(int E) { return E >= 16 ? 4 : 3; }
// radix (log2) of pass i of a transform of 2^logn points with full passes of radix
// 2^lrm, and the pass count
constexpr int reg_pass_lr(int logn, int i, int lrm) { return i < logn / lrm ? lrm : logn - lrm * (logn / lrm); }
constexpr int reg_num_passes(int logn, int lrm) { return logn / lrm + (logn % lrm ? 1 : 0); }
// log2 of the sub-transform length after the passes before pass i
constexpr int reg_lns_before(int logn, int i, int lrm) {
    return i == 0 ? 0 : reg_lns_before(logn, i - 1, lrm) + reg_pass_lr(logn, i - 1, lrm);
}

// In-register 16-point DFT (sign -1 forward, +1 inverse), output in natural
// order: four 4-point DFTs over n1 (n = 4 n1 + n2), the twiddles W16^(n2 k1),
// four 4-point DFTs over n2 (k = k1 + 4 k2).
__device__ __forceinline__ void dft16(float2* a, bool inv) {
    constexpr float c1 = 0.92387953251128674f, s1 = 0.38268343236508977f, h = 0.70710678118654752f;
    float2 b[4][4];                          // [n2][k1]
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
        float2 t[4] = {a[n2], a[4 + n2], a[8 + n2], a[12 + n2]};
        dft4(t, inv);
#pragma unroll
        for (int k1 = 0; k1 < 4; ++k1) b[n2][k1] = t[k1];
    }
    // W16^m for m = n2 k1 in {1, 2, 3, 4, 6, 9} (conjugated for the inverse)
    auto tw16 = [&](float2 v, int m) -> float2 {
        if (m == 4) return inv ? make_float2(-v.y, v.x) : make_float2(v.y, -v.x);
        float c = 0.f, sn = 0.f;
        if (m == 1) { c = c1; sn = -s1; }
        else if (m == 2) { c = h; sn = -h; }
        else if (m == 3) { c = s1; sn = -c1; }
        else if (m == 6) { c = -h; sn = -h; }
        else { c = -c1; sn = s1; }          // m == 9
        if (inv) sn = -sn;
        return make_float2(v.x * c - v.y * sn, v.x * sn + v.y * c);
    };
#pragma unroll
    for (int n2 = 1; n2 < 4; ++n2)
#pragma unroll
        for (int k1 = 1; k1 < 4; ++k1) b[n2][k1] = tw16(b[n2][k1], n2 * k1);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
        float2 t[4] = {b[0][k1], b[1][k1], b[2][k1], b[3][k1]};
        dft4(t, inv);
#pragma unroll
        for (int k2 = 0; k2 < 4; ++k2) a[k1 + 4 * k2] = t[k2];
    }
}

// Twiddles w^r, r = 1..15, of one radix-16 butterfly: w, w^2, w^4, w^8 from the
// table, the others products of those (at most three roundings deep).
__device__ __forceinline__ void butterfly_twiddles16(float2 (&w)[16], const float2* __restrict__ tw, int k, bool inv) {
    butterfly_twiddles<8>(*(float2(*)[8])w, tw, k, inv);
    w[8] = twiddle(tw, 8 * k, inv);
#pragma unroll
    for (int r = 1; r < 8; ++r) w[8 + r] = cmul(w[r], w[8]);
}

// The thread index as a value the compiler cannot relate to any other copy of it.
// Positions are the thread index plus constants, the same in every pass; with
// one shared index the compiler keeps those sums for all passes at once (and
// spills them) instead of forming each where it is used.  Each pass takes its
// own copy.
__device__ __forceinline__ int opaque_tid() {
    int t = (int)threadIdx.x;
    asm volatile("" : "+v"(t));
    return t;
}

// position read by element e of thread tid in a pass of radix 2^LR
template <int LR, int LOGN, int E>
__device__ __forceinline__ int reg_in_pos(int e, int tid) {
    constexpr int R = 1 << LR, T = (1 << LOGN) / E;
    const int q = e >> LR, r = e & (R - 1);
    return tid + q * T + (r << (LOGN - LR));
}
// position written by element e of thread tid in a pass of radix 2^LR with
// sub-transform length 2^LNS
template <int LR, int LNS, int LOGN, int E>
__device__ __forceinline__ int reg_out_pos(int e, int tid) {
    constexpr int R = 1 << LR, T = (1 << LOGN) / E;
    const int q = e >> LR, r = e & (R - 1);
    const int j = tid + q * T;
    return ((j >> LNS) << (LNS + LR)) + (j & ((1 << LNS) - 1)) + (r << LNS);
}

// A pointer the compiler cannot see through, taken once v0 is known: loads from
// it are not issued before the code that produced v0.  Twiddle addresses depend
// only on the thread index; without this the loads of every pass are hoisted to
// the start of the transform (an LDS-only barrier does not hold back global
// loads) and their values occupy registers through all the passes before.
template <typename T>
__device__ __forceinline__ T* after(T* p, float2& v0) {
    asm volatile("" : "+s"(p), "+v"(v0.x));
    return p;
}

// Butterflies of one pass on the thread's E values (E / R butterflies).
template <int LR, int LNS, int LOGN, int E>
__device__ __forceinline__ void reg_butterflies(float2 (&v)[E], const float2* __restrict__ tw0, int tw_log, bool inv) {
    constexpr int R = 1 << LR, T = (1 << LOGN) / E;
    const int tws = tw_log - LNS - LR;
    const float2* tw = after(tw0, v[0]);
    const int tid = opaque_tid();
#pragma unroll
    for (int q = 0; q < E / R; ++q) {
        const int j = tid + q * T;
        const int k = j & ((1 << LNS) - 1);
        float2* a = v + q * R;
        float2 w[R];
        if constexpr (R == 16) butterfly_twiddles16(w, tw, k << tws, inv);
        else butterfly_twiddles<R>(w, tw, k << tws, inv);
#pragma unroll
        for (int r = 1; r < R; ++r) a[r] = cmul(a[r], w[r]);
        if constexpr (R == 16) {
            dft16(a, inv);
        } else {
            dft_small<R>(a, inv);
        }
    }
}

// Exchange-buffer slot of position i in the exchange after a pass of radix 2^LR
// over sub-transforms of 2^LNS points: 2^xpad_log(LR, LNS) unused slots after
// every 32 positions.  A half-wave's 32 eight-byte accesses then cover the 64 LDS
// banks once, both for the stores (positions R apart in the first exchange; runs
// of R consecutive positions, R^2 apart, in the second; runs of 2^LNS >= 32 after
// that) and for the contiguous reads of the next pass: one pad slot per 32 in
// general, and two (R = 16) or four (R = 8) in the second exchange, which put the
// stores' runs on distinct banks.  (One slot per eight, the earlier layout, left every exchange with 2-way
// conflicts on the stores or the reads.)  The pad is additive, so a thread's
// slots stay its own base plus immediate offsets.
// (at most four per 32, which the buffer size below allows)
constexpr int xpad_log(int lr, int lns) { return lns == lr && (lr == 3 || lr == 4) ? 5 - lr : 0; }
template <int LR, int LNS>
__device__ __forceinline__ int xpad(int i) { return i + ((i >> 5) << xpad_log(LR, LNS)); }

// floats of exchange buffer that reg_fft needs for 2^logn points (complex slots;
// at most four pad slots per 32)
constexpr int reg_xbuf_floats(int logn) { return 2 * ((1 << logn) + (1 << (logn - 3))); }

// Move the outputs of a radix-2^LR pass (sub-length 2^LNS) to the inputs of the
// next pass (radix 2^LR2) through `x` (reg_xbuf_floats(LOGN) floats, as complex
// slots).
// Each position is the bitwise OR of a part that depends on the thread only
// (element 0's position) and a compile-time part that depends on the element
// only (thread 0's): tid < T occupies the low bits that q T and r 2^k leave free,
// and the store map only inserts LR zero bits at bit LNS.  The pad, a multiple of
// the position's bits above bit 5, then splits over the two parts, so each thread
// pads one base per direction and every element is an immediate offset from it
// (the compiler does not split (tid + C) >> 5 by itself).
template <int LR, int LR2, int LNS, int LOGN, int E>
__device__ __forceinline__ void reg_exchange(float2 (&v)[E], float* x) {
    float2* xc = (float2*)x;
    const int tid = opaque_tid();
    float2* wb = xc + xpad<LR, LNS>(reg_out_pos<LR, LNS, LOGN, E>(0, tid));
    float2* rb = xc + xpad<LR, LNS>(reg_in_pos<LR2, LOGN, E>(0, tid));
    lds_sync();
#pragma unroll
    for (int e = 0; e < E; ++e) wb[xpad<LR, LNS>(reg_out_pos<LR, LNS, LOGN, E>(e, 0))] = v[e];
    lds_sync();
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = rb[xpad<LR, LNS>(reg_in_pos<LR2, LOGN, E>(e, 0))];
}

template <int E, int LOGN, int LRM, int I>
__device__ __forceinline__ void reg_fft_from(float2 (&v)[E], float* x, const float2* __restrict__ tw, int tw_log,
                                             bool inv) {
    constexpr int NP = reg_num_passes(LOGN, LRM);
    if constexpr (I < NP) {
        constexpr int LR = reg_pass_lr(LOGN, I, LRM), LNS = reg_lns_before(LOGN, I, LRM);
        reg_butterflies<LR, LNS, LOGN, E>(v, tw, tw_log, inv);
        if constexpr (I + 1 < NP) {
            reg_exchange<LR, reg_pass_lr(LOGN, I + 1, LRM), LNS, LOGN, E>(v, x);
            reg_fft_from<E, LOGN, LRM, I + 1>(v, x, tw, tw_log, inv);
        }
    }
}

// Full transform of 2^LOGN points by (2^LOGN / E)-thread blocks (x:
// reg_xbuf_floats(LOGN) floats of LDS).  On entry element e of the thread holds
// the input at reg_input_pos<LOGN, E>(e); on exit it holds the output at
// reg_output_pos<LOGN, E>(e).  Needs LOGN >= 6.
template <int E, int LOGN, int LRM = reg_lr_max(E)>
__device__ __forceinline__ void reg_fft(float2 (&v)[E], float* x, const float2* __restrict__ tw, int tw_log,
                                        bool inv) {
    static_assert(LOGN >= 6 && (1 << LOGN) % E == 0 && (1 << LRM) <= E, "transform shape");
    reg_fft_from<E, LOGN, LRM, 0>(v, x, tw, tw_log, inv);
}

// input position of element e (that of the first pass)
template <int LOGN, int E, int LRM = reg_lr_max(E)>
__device__ __forceinline__ int reg_input_pos(int e) {
    return reg_in_pos<reg_pass_lr(LOGN, 0, LRM), LOGN, E>(e, (int)threadIdx.x);
}

// output position of element e after reg_fft (of thread tid)
template <int LOGN, int E, int LRM = reg_lr_max(E)>
__device__ __forceinline__ int reg_output_pos(int e, int tid = (int)threadIdx.x) {
    constexpr int NP = reg_num_passes(LOGN, LRM);
    constexpr int LR = reg_pass_lr(LOGN, NP - 1, LRM);
    return reg_out_pos<LR, LOGN - LR, LOGN, E>(e, tid);
}

// Exchange from the last pass's output layout to the first pass's input layout
template <int LOGN, int E, int LRM = reg_lr_max(E)>
__device__ __forceinline__ void reg_output_to_input(float2 (&v)[E], float* x) {
    constexpr int NP = reg_num_passes(LOGN, LRM);
    constexpr int LR = reg_pass_lr(LOGN, NP - 1, LRM);
    reg_exchange<LR, reg_pass_lr(LOGN, 0, LRM), LOGN - LR, LOGN, E>(v, x);
}

}  // namespace jtfs
