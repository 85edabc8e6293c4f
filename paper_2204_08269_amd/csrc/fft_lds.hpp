// Batched power-of-two complex FFT held in LDS (Stockham autosort: radix-8 passes,
// then one radix-4 or radix-2 pass).  Every pass reads all of a thread's
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

// the same operations in FP64 (the input transform runs in double precision)
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }

template <typename C> struct cplx;
template <> struct cplx<float2> {
    using real = float;
    static __device__ __forceinline__ float2 make(float x, float y) { return make_float2(x, y); }
};
template <> struct cplx<double2> {
    using real = double;
    static __device__ __forceinline__ double2 make(double x, double y) { return make_double2(x, y); }
};

// twiddle e^{sign 2 pi i k / 2^tw_log}, sign = -1 (forward) or +1 (inverse)
template <typename C>
__device__ __forceinline__ C twiddle(const C* __restrict__ tw, int k, bool inv) {
    C w = tw[k];
    if (inv) w.y = -w.y;
    return w;
}

// LDS slot of element j of one transform: the low five bits of j are XORed with
// bits 3..7.  A half-wave's 8-byte accesses cover the 64 four-byte banks once, so
// a pass's loads (32 consecutive elements, permuted inside their aligned block
// of 32) and its stores (8 apart in the first pass, runs of 8 spaced 64 apart in
// the second, longer runs after) meet no bank twice for transforms of 256 points
// or more.  For j < n (n a power of two) the slot stays below n; element n of a
// half spectrum lands at n + n/8 below 256 points and at n from there on.  Every
// kernel that fills or reads an LDS transform buffer indexes it through lpad.
__device__ __forceinline__ int lpad(int j) { return j ^ ((j >> 3) & 31); }
// slots one transform of n points occupies, with element n of a half spectrum;
// even from 16 points on, so that a column stride of lpad_len + 1 is odd
constexpr int lpad_len(int n) { return n + (n < 256 ? n / 8 : 0) + 2; }

// Workgroup barrier that orders LDS only: it waits for this wave's LDS accesses
// (not for its global loads and stores, which may stay in flight across it).
__device__ __forceinline__ void lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Twiddles w^r, r = 1..R-1, of one radix-R butterfly, w = twiddle(tw, k, inv): w,
// w^2 and w^4 come from the table, the others are products of those (at most
// two roundings deep), so a radix-8 butterfly loads three twiddles, not seven.
template <int R, typename C>
__device__ __forceinline__ void butterfly_twiddles(C (&w)[R], const C* __restrict__ tw, int k, bool inv) {
    if constexpr (R >= 2) w[1] = twiddle(tw, k, inv);
    if constexpr (R >= 4) {
        w[2] = twiddle(tw, 2 * k, inv);
        w[3] = cmul(w[1], w[2]);
    }
    if constexpr (R >= 8) {
        w[4] = twiddle(tw, 4 * k, inv);
        w[5] = cmul(w[1], w[4]);
        w[6] = cmul(w[2], w[4]);
        w[7] = cmul(w[3], w[4]);
    }
}

// In-register 4-point DFT (sign -1 forward, +1 inverse).
template <typename C>
__device__ __forceinline__ void dft4(C* a, bool inv) {
    const C t0 = cadd(a[0], a[2]), t1 = csub(a[0], a[2]), t2 = cadd(a[1], a[3]);
    const C d = csub(a[1], a[3]);
    const C t3 = inv ? cplx<C>::make(-d.y, d.x) : cplx<C>::make(d.y, -d.x);   // d * (s i)
    a[0] = cadd(t0, t2);
    a[2] = csub(t0, t2);
    a[1] = cadd(t1, t3);
    a[3] = csub(t1, t3);
}

// In-register DFT of R = 2, 4 or 8 points (sign -1 forward, +1 inverse), output
// in natural order.  Eight points as two 4-point DFTs: X[2q] = DFT4(a_r + a_{r+4}),
// X[2q+1] = DFT4((a_r - a_{r+4}) w8^r).  Shared by the in-LDS Stockham passes and
// the register-resident transforms.
template <int R, typename C>
__device__ __forceinline__ void dft_small(C* a, bool inv) {
    static_assert(R == 2 || R == 4 || R == 8, "radix");
    using Rl = typename cplx<C>::real;
    if constexpr (R == 2) {
        const C a0 = a[0], a1 = a[1];
        a[0] = cadd(a0, a1);
        a[1] = csub(a0, a1);
    } else if constexpr (R == 4) {
        dft4(a, inv);
    } else {
        C b[4], c[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            b[r] = cadd(a[r], a[r + 4]);
            c[r] = csub(a[r], a[r + 4]);
        }
        const Rl h = (Rl)0.70710678118654752440;
        // c1 *= w8, c2 *= w8^2 = -/+ i, c3 *= w8^3
        c[1] = inv ? cplx<C>::make(h * (c[1].x - c[1].y), h * (c[1].x + c[1].y))
                   : cplx<C>::make(h * (c[1].x + c[1].y), h * (c[1].y - c[1].x));
        c[2] = inv ? cplx<C>::make(-c[2].y, c[2].x) : cplx<C>::make(c[2].y, -c[2].x);
        c[3] = inv ? cplx<C>::make(-h * (c[3].x + c[3].y), h * (c[3].x - c[3].y))
                   : cplx<C>::make(h * (c[3].y - c[3].x), -h * (c[3].x + c[3].y));
        dft4(b, inv);
        dft4(c, inv);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            a[2 * r] = b[r];
            a[2 * r + 1] = c[r];
        }
    }
}

// One Stockham pass of radix R = 2^LR over `count` transforms of length 2^logn
// located at s + t*stride.  Ns = 2^lNs is the length of the sub-transforms
// already combined.  MAXE bounds the elements each thread holds.
template <int LR, int MAXE, typename C>
__device__ __forceinline__ void fft_pass(C* s, int logn, int count, int stride, int lNs,
                                         const C* __restrict__ tw, int tw_log, bool inv) {
    using Rl = typename cplx<C>::real;
    constexpr int R = 1 << LR;
    constexpr int MAXB = MAXE / R;
    const int nb_log = logn - LR;            // butterflies per transform = 2^nb_log
    const int total = count << nb_log;
    const int Ns = 1 << lNs;
    const int tws = tw_log - lNs - LR;       // table step of the angle unit 1/(Ns R)
    C v[MAXB][R];
#pragma unroll
    for (int q = 0; q < MAXB; ++q) {
        const int g = threadIdx.x + q * blockDim.x;
        if (g < total) {
            const int t = g >> nb_log;
            const int j = g & ((1 << nb_log) - 1);
            const C* src = s + t * stride;
            const int k = j & (Ns - 1);
            C w[R];
            butterfly_twiddles<R>(w, tw, k << tws, inv);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                C a = src[lpad(j + (r << nb_log))];
                if (r) a = cmul(a, w[r]);
                v[q][r] = a;
            }
            dft_small<R>(v[q], inv);
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < MAXB; ++q) {
        const int g = threadIdx.x + q * blockDim.x;
        if (g < total) {
            const int t = g >> nb_log;
            const int j = g & ((1 << nb_log) - 1);
            C* dst = s + t * stride;
            const int idx = ((j >> lNs) << (lNs + LR)) + (j & (Ns - 1));
#pragma unroll
            for (int r = 0; r < R; ++r) dst[lpad(idx + r * Ns)] = v[q][r];
        }
    }
    __syncthreads();
}

// count transforms of length 2^logn at s + t*stride (element j of a transform at
// slot lpad(j); stride >= lpad_len(2^logn)), all threads of the block taking
// part; count * 2^logn <= MAXE * blockDim.x.  Starts and ends with the data in
// LDS; the caller must __syncthreads() before calling.
template <int MAXE, typename C>
__device__ __forceinline__ void lds_fft(C* s, int logn, int count, int stride, const C* __restrict__ tw,
                        int tw_log, bool inv) {
    int lNs = 0;
    // radix-8 passes while three or more stages remain, then one radix-4 or radix-2
    while (logn - lNs >= 3) {
        fft_pass<3, MAXE>(s, logn, count, stride, lNs, tw, tw_log, inv);
        lNs += 3;
    }
    if (logn - lNs == 2) fft_pass<2, MAXE>(s, logn, count, stride, lNs, tw, tw_log, inv);
    if (logn - lNs == 1) fft_pass<1, MAXE>(s, logn, count, stride, lNs, tw, tw_log, inv);
}

}  // namespace jtfs
