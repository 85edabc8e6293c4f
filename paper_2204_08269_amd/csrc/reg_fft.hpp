// Block-wide power-of-two FFT with the data resident in registers.
//
// Each of the T = blockDim.x threads holds E = n / T complex values.  Passes are
// Stockham radix-8 (then one radix-4 or radix-2 pass); between passes the values
// move to the thread that needs them through LDS, the real parts first and the
// imaginary parts second, so the exchange buffer holds only n floats plus one pad
// float per eight (a little over half of an in-LDS complex transform).  Unnormalised in both directions; twiddles from the
// FP64-generated table tw[k] = exp(-2 pi i k / 2^tw_log).
#pragma once

#include <hip/hip_runtime.h>

#include "fft_lds.hpp"

namespace jtfs {

// radix (log2) of pass `i` for a transform of 2^logn points
__device__ __forceinline__ int reg_pass_lr(int logn, int i) {
    const int full = logn / 3;
    return i < full ? 3 : logn - 3 * full;
}
__device__ __forceinline__ int reg_num_passes(int logn) { return logn / 3 + (logn % 3 ? 1 : 0); }

// position read by element e of the thread in a pass of radix 2^LR
template <int LR>
__device__ __forceinline__ int reg_in_pos(int e, int logn) {
    constexpr int R = 1 << LR;
    const int q = e >> LR, r = e & (R - 1);
    return (int)threadIdx.x + q * (int)blockDim.x + (r << (logn - LR));
}
// position written by element e in a pass of radix 2^LR with sub-transform length 2^lNs
template <int LR>
__device__ __forceinline__ int reg_out_pos(int e, int lNs) {
    constexpr int R = 1 << LR;
    const int q = e >> LR, r = e & (R - 1);
    const int j = (int)threadIdx.x + q * (int)blockDim.x;
    return ((j >> lNs) << (lNs + LR)) + (j & ((1 << lNs) - 1)) + (r << lNs);
}

// Butterflies of one pass on the thread's E values (E / R butterflies).
template <int LR, int E>
__device__ __forceinline__ void reg_butterflies(float2 (&v)[E], int lNs, const float2* __restrict__ tw, int tw_log,
                                                bool inv) {
    constexpr int R = 1 << LR;
    const int tws = tw_log - lNs - LR;
#pragma unroll
    for (int q = 0; q < E / R; ++q) {
        const int j = (int)threadIdx.x + q * (int)blockDim.x;
        const int k = j & ((1 << lNs) - 1);
        float2* a = v + q * R;
        float2 w[R];
        butterfly_twiddles<R>(w, tw, k << tws, inv);
#pragma unroll
        for (int r = 1; r < R; ++r) a[r] = cmul(a[r], w[r]);
        if constexpr (R == 2) {
            const float2 a0 = a[0], a1 = a[1];
            a[0] = cadd(a0, a1);
            a[1] = csub(a0, a1);
        } else if constexpr (R == 4) {
            dft4(a, inv);
        } else {
            float2 b[4], c[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                b[r] = cadd(a[r], a[r + 4]);
                c[r] = csub(a[r], a[r + 4]);
            }
            const float h = 0.70710678118654752f;
            c[1] = inv ? make_float2(h * (c[1].x - c[1].y), h * (c[1].x + c[1].y))
                       : make_float2(h * (c[1].x + c[1].y), h * (c[1].y - c[1].x));
            c[2] = inv ? make_float2(-c[2].y, c[2].x) : make_float2(c[2].y, -c[2].x);
            c[3] = inv ? make_float2(-h * (c[3].x + c[3].y), h * (c[3].x - c[3].y))
                       : make_float2(h * (c[3].y - c[3].x), -h * (c[3].x + c[3].y));
            dft4(b, inv);
            dft4(c, inv);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                a[2 * r] = b[r];
                a[2 * r + 1] = c[r];
            }
        }
    }
}

// Exchange-buffer slot of position i: one unused float after every eight.  The
// stores of the first passes go to positions R apart across the lanes (R = 8);
// with the pad those become 9 floats apart, an odd stride, so that consecutive
// lanes fall into distinct LDS banks.  Contiguous reads gain at most a 2-way
// conflict where a run crosses a pad.
__device__ __forceinline__ int xpad(int i) { return i + (i >> 3); }

// floats of exchange buffer that reg_fft needs for 2^logn points
constexpr int reg_xbuf_floats(int logn) { return (1 << logn) + (1 << (logn - 3)); }

// Move the outputs of a radix-2^LR pass (sub-length 2^lNs) to the inputs of the
// next pass (radix 2^LR2) through `x` (reg_xbuf_floats(logn) floats): real
// parts, then imaginary.
template <int LR, int LR2, int E>
__device__ __forceinline__ void reg_exchange(float2 (&v)[E], float* x, int logn, int lNs) {
    lds_sync();
#pragma unroll
    for (int e = 0; e < E; ++e) x[xpad(reg_out_pos<LR>(e, lNs))] = v[e].x;
    lds_sync();
#pragma unroll
    for (int e = 0; e < E; ++e) v[e].x = x[xpad(reg_in_pos<LR2>(e, logn))];
    lds_sync();
#pragma unroll
    for (int e = 0; e < E; ++e) x[xpad(reg_out_pos<LR>(e, lNs))] = v[e].y;
    lds_sync();
#pragma unroll
    for (int e = 0; e < E; ++e) v[e].y = x[xpad(reg_in_pos<LR2>(e, logn))];
}

// Full transform (x: reg_xbuf_floats(logn) floats of LDS).  On entry element e of the thread holds the input at
// reg_in_pos<first radix>(e) (use reg_input_pos below); on exit it holds the
// output at reg_output_pos(e, logn).  Needs 2^logn = E * blockDim.x and logn >= 6.
template <int E>
__device__ __forceinline__ void reg_fft(float2 (&v)[E], float* x, int logn, const float2* __restrict__ tw,
                                        int tw_log, bool inv) {
    const int np = reg_num_passes(logn);
    int lNs = 0;
    for (int i = 0; i < np; ++i) {
        const int lr = reg_pass_lr(logn, i);
        const bool last = i + 1 == np;
        const int lr2 = last ? 0 : reg_pass_lr(logn, i + 1);
        if (lr == 3) {
            reg_butterflies<3, E>(v, lNs, tw, tw_log, inv);
            if (!last) {
                if (lr2 == 3) reg_exchange<3, 3, E>(v, x, logn, lNs);
                else if (lr2 == 2) reg_exchange<3, 2, E>(v, x, logn, lNs);
                else reg_exchange<3, 1, E>(v, x, logn, lNs);
            }
        } else if (lr == 2) {
            reg_butterflies<2, E>(v, lNs, tw, tw_log, inv);
        } else {
            reg_butterflies<1, E>(v, lNs, tw, tw_log, inv);
        }
        lNs += lr;
    }
}

// input position of element e (the first pass is radix 8 for logn >= 3)
__device__ __forceinline__ int reg_input_pos(int e, int logn) { return reg_in_pos<3>(e, logn); }

// output position of element e after reg_fft
__device__ __forceinline__ int reg_output_pos(int e, int logn) {
    const int np = reg_num_passes(logn);
    const int lr = reg_pass_lr(logn, np - 1);
    const int lNs = logn - lr;
    if (lr == 3) return reg_out_pos<3>(e, lNs);
    if (lr == 2) return reg_out_pos<2>(e, lNs);
    return reg_out_pos<1>(e, lNs);
}

}  // namespace jtfs
