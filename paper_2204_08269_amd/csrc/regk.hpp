// Launchers of the long-row kernels (kernels_reg.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "plan.hpp"

namespace jtfs {
constexpr int kRegMinLog = kRegMinLogRows;   // shortest row length (log2) of the register-resident FFT
int reg_attributes();
void launch_scalogram_r(const jtfs_plan* P, const float2* xh, int64_t xh_pitch, float2* Xh, int64_t Xh_pitch,
                        int64_t B, hipStream_t st);
void launch_second_order_r(const jtfs_plan* P, int a, const float2* Xh, int64_t Xh_pitch, float2* Y2, float* rowmax,
                           int64_t B, hipStream_t st);
void launch_rowfft_r(const jtfs_plan* P, float2* base, int64_t bs, int64_t rs, int rows, int logn, int64_t B,
                     hipStream_t st);
void launch_scal_bwd_b_r(const jtfs_plan* P, const float2* xh, int64_t xh_pitch, const float* gX, float2* g1,
                         int64_t B, hipStream_t st);
}  // namespace jtfs
