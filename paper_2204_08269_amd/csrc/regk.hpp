// Launchers of the long-row kernels (kernels_reg.hip), and the mu-log arguments
// that the coefficient writers and cotangent readers share.
#pragma once
#include <hip/hip_runtime.h>

#include "plan.hpp"

namespace jtfs {
// mu-log of sec. 4 (eqs. (9)-(10)) fused into the coefficient writers and the
// cotangent readers.  With mu set, a writer stores O = log(1 + S / (eps mu)) of its
// path instead of S, and a reader takes the cotangent g of O to the cotangent of
// S, g / (eps mu + S) = g / (eps mu e^O), from O itself (mu held fixed).
struct MuLogArg {
    const float* mu1;   // [1]: the S1 path; null: no mu-log
    const float* mu2;   // one per second-order path (the layouts of the mu-log entry points)
    float eps;
    const float* o1;    // backward: the forward's outputs O1, O2
    const float* o2;
};

__device__ __forceinline__ float mulog_inv(const float* mu, int p, float eps) {
    return mu ? 1.f / (eps * mu[p]) : 0.f;
}
__device__ __forceinline__ float mulog_out(float v, const float* mu, float inv) {
    return mu ? log1pf(v * inv) : v;
}
__device__ __forceinline__ float mulog_cot(float g, const float* mu, float em, float o) {
    return mu ? g / (em * expf(o)) : g;
}

constexpr int kRegMinLog = kRegMinLogRows;   // shortest row length (log2) of the register-resident FFT
int reg_attributes();
void launch_scalogram_r(const jtfs_plan* P, const float2* xh, int64_t xh_pitch, float2* Xh, int64_t Xh_pitch,
                        int64_t B, hipStream_t st);
void launch_second_order_r(const jtfs_plan* P, int a, const float2* Xh, int64_t Xh_pitch, float2* Y2, float* rowmax,
                           int64_t B, hipStream_t st);
void launch_rowfft_r(const jtfs_plan* P, float2* base, int64_t bs, int64_t rs, int rows, int logn, int64_t B,
                     hipStream_t st);
// adjoint of the second order and of S1 for rows of N_X = 2^14 or 2^15 points
void launch_scal_bwd_a_r(const jtfs_plan* P, const float2* G, int64_t y_bstride, const float* gS1, const MuLogArg& ml,
                         const float2* gYphi, int Tphi, float* gX, int64_t B, hipStream_t st);
void launch_scal_bwd_b_r(const jtfs_plan* P, const float2* xh, int64_t xh_pitch, const float* gX, float2* g1,
                         int64_t B, hipStream_t st);
}  // namespace jtfs
