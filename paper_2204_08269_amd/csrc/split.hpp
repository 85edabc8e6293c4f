// Launchers of the split-FP16 frequential contraction (split.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

#include "plan.hpp"

namespace jtfs {
bool split_supported(const Shapes& s);
int build_split_tables(jtfs_plan* P, std::vector<void*>& owned);
int split_attributes();
int launch_ysplit(const jtfs_plan* P, int a, const float2* Y2, const float* rowmax, unsigned short* Yh, float* yscale,
                  int64_t B, hipStream_t st);
int launch_freq_bwd_split(const jtfs_plan* P, int a, const unsigned short* Yh, const float* yscale, const float* gV,
                          const float* gvmax, float2* gY2, int64_t B, hipStream_t st);
// phase: NULL, or the stored-phase buffer of the workspace (ph_bstride packed snorm16
// pairs per signal)
int launch_freq_fwd_split(const jtfs_plan* P, int a, const unsigned short* Yh, const float* yscale, float* Vp,
                          int64_t vp_bstride, unsigned* phase, int64_t ph_bstride, int64_t B, hipStream_t st);
// backward contraction from the phase the forward stored (no recomputation of Z)
int launch_freq_bwd_phase(const jtfs_plan* P, int a, const unsigned* phase, int64_t ph_bstride, const uint4* Gs,
                          int64_t gs_bstride, const float* gvmax, float2* gY2, int64_t B, hipStream_t st);
// gV of every rate split into the FP16 planes and row scales the stored-phase
// backward reads (Gs: gs_bstride 16-byte units per signal)
int launch_gv_split(const jtfs_plan* P, const float* gV, uint4* Gs, int64_t B, hipStream_t st);
// whether the 16 x 16-tile forward contraction handles the plan's shapes
bool fwdq_supported(const jtfs_plan* P, bool with_phase);
// whether the 16 x 16-tile stored-phase backward handles the plan's shapes
bool bwdq_supported(const jtfs_plan* P);
}  // namespace jtfs
