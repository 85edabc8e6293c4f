// Batched power-of-two complex FFT held in LDS (Stockham autosort, radix 4 with
// one radix-2 pass for odd log2 sizes).  Every pass reads all of a thread's
// butterfly inputs, waits at a barrier, and writes the outputs back in place, so
// a single LDS buffer suffices.  Twiddles come from an FP64-generated table
// tw[k] = exp(-2 pi i k / 2^tw_log) (no recurrences), conjugated for the inverse.
// Transforms are unnormalised in both directions.
#pragma once

#include <hip/hip_runtime.h>

namespace jtfs {

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {  // a * conj(b)
    return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ float2 conjf2(float2 a) { return make_float2(a.x, -a.y); }

// twiddle e^{sign 2 pi i k / 2^tw_log}, sign = -1 (forward) or +1 (inverse)
__device__ __forceinline__ float2 twiddle(const float2* __restrict__ tw, int k, bool inv) {
    float2 w = tw[k];
    if (inv) w.y = -w.y;
    return w;
}

// One Stockham pass of radix R = 2^LR over `count` transforms of length 2^logn
// located at s + t*stride.  Ns = 2^lNs is the length of the sub-transforms
// already combined.  MAXE bounds the elements each thread holds.
template <int LR, int MAXE>
__device__ __forceinline__ void fft_pass(float2* s, int logn, int count, int stride, int lNs,
                                         const float2* __restrict__ tw, int tw_log, bool inv) {
    constexpr int R = 1 << LR;
    constexpr int MAXB = MAXE / R;
    const int nb_log = logn - LR;            // butterflies per transform = 2^nb_log
    const int total = count << nb_log;
    const int Ns = 1 << lNs;
    const int tws = tw_log - lNs - LR;       // table step of the angle unit 1/(Ns R)
    float2 v[MAXB][R];
#pragma unroll
    for (int q = 0; q < MAXB; ++q) {
        const int g = threadIdx.x + q * blockDim.x;
        if (g < total) {
            const int t = g >> nb_log;
            const int j = g & ((1 << nb_log) - 1);
            const float2* src = s + t * stride;
            const int k = j & (Ns - 1);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                float2 a = src[j + (r << nb_log)];
                if (r) a = cmul(a, twiddle(tw, (r * k) << tws, inv));
                v[q][r] = a;
            }
            if constexpr (R == 2) {
                const float2 a0 = v[q][0], a1 = v[q][1];
                v[q][0] = cadd(a0, a1);
                v[q][1] = csub(a0, a1);
            } else {
                const float2 a0 = v[q][0], a1 = v[q][1], a2 = v[q][2], a3 = v[q][3];
                const float2 t0 = cadd(a0, a2), t1 = csub(a0, a2), t2 = cadd(a1, a3);
                const float2 d = csub(a1, a3);
                // (a1 - a3) times (s i), s = -1 forward, +1 inverse
                const float2 t3 = inv ? make_float2(-d.y, d.x) : make_float2(d.y, -d.x);
                v[q][0] = cadd(t0, t2);
                v[q][2] = csub(t0, t2);
                v[q][1] = cadd(t1, t3);
                v[q][3] = csub(t1, t3);
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < MAXB; ++q) {
        const int g = threadIdx.x + q * blockDim.x;
        if (g < total) {
            const int t = g >> nb_log;
            const int j = g & ((1 << nb_log) - 1);
            float2* dst = s + t * stride;
            const int idx = ((j >> lNs) << (lNs + LR)) + (j & (Ns - 1));
#pragma unroll
            for (int r = 0; r < R; ++r) dst[idx + r * Ns] = v[q][r];
        }
    }
    __syncthreads();
}

// count transforms of length 2^logn at s + t*stride, all threads of the block
// taking part; count * 2^logn <= MAXE * blockDim.x.  Starts and ends with the
// data in LDS; the caller must __syncthreads() before calling.
template <int MAXE>
__device__ void lds_fft(float2* s, int logn, int count, int stride, const float2* __restrict__ tw,
                        int tw_log, bool inv) {
    int lNs = 0;
    if (logn & 1) {
        fft_pass<1, MAXE>(s, logn, count, stride, lNs, tw, tw_log, inv);
        lNs += 1;
    }
    while (lNs < logn) {
        fft_pass<2, MAXE>(s, logn, count, stride, lNs, tw, tw_log, inv);
        lNs += 2;
    }
}

}  // namespace jtfs
