// Host-side plan of the JTFS transform: parameter validation, the FP64 solve of
// every filterbank's centre frequencies and widths, the critical-rate schedule,
// padded shapes, device table handles and the workspace layout.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/jtfs.h"

namespace jtfs {

constexpr double kSigma0 = 0.1;    // lowpass width: phi_T has sigma = kSigma0 / T
constexpr double kCEnv = 5.0;      // critical rate: decimated Nyquist >= kCEnv * sigma
constexpr double kSupportTol = 1e-13;  // spectra below this (after normalisation) are not stored
constexpr float kEpsMod = 1e-30f;  // modulus-gradient guard: z / max(|z|, eps)
// The same guard on |z|^2 where the gradient takes rsqrt(|z|^2): the floor must
// stay a normal FP32 number, so it acts at |z| = 1e-18 (z = 0 still gives 0).
constexpr float kEpsMod2 = 1e-36f;

constexpr int kTileL = 64;         // frequential GEMM: rows (l) per tile
constexpr int kTileT = 64;         // frequential GEMM: columns (t) per tile
constexpr int kTileTh = 128;       // split-FP16 contraction: columns (t) per tile (t padding unit)
constexpr int kKStep = 16;         // frequential GEMM: K (lambda_1) per LDS stage
constexpr int kChunkT = 4096;      // frequential GEMM: t-range reduced by one workgroup
constexpr int kLdsFftMax = 14;     // log2 of the largest complex FFT held in LDS
constexpr int kMaxLogNX = 15;      // longest scalogram row
constexpr int kRegMinLogRows = 14; // shortest row length (log2) with a register-resident kernel
constexpr int kMaxDynLds = 159 * 1024;  // dynamic LDS limit set on kernels (1 KB left for static LDS)

void set_error(const std::string& s);

// One Morlet family (sec. 2): centres, widths and band supports on its grid.
struct Family {
    int M = 0;                       // grid length (spectrum bins 0..M-1)
    std::vector<double> xi, sigma;   // centre / Gaussian width in cycles per grid sample
    std::vector<int> lo, hi;         // stored support [lo, hi], 0 <= lo <= hi <= M/2
    std::vector<int64_t> off;        // offset of each filter in the packed value table
    int64_t total = 0;               // packed table length
    int n() const { return (int)xi.size(); }
};

struct Shapes {
    jtfs_params p{};
    int logN = 0, logT = 0, logF = 0;
    int n1 = 0, kX = 0, logNX = 0, n_alpha = 0, n_beta = 0, L = 0, logL = 0;
    int64_t N = 0, NX = 0, T = 0, F = 0;
    bool avg_fr = true;              // eq. (3); false: eq. (4), no frequency lowpass
    bool tscat = false;              // time scattering: no frequential stage
    bool complete = false;           // lowpass pairs: alpha = n_alpha_psi is phi_T, beta = n_beta_psi is phi_F
    int n_alpha_psi = 0, n_beta_psi = 0;   // wavelets among the n_alpha / n_beta rates and scales
    int NT = 0, NTp = 0, NL = 0;     // N/T, padded to 32, L/F
    int NLo = 0;                     // lambda rows of the S2 output: NL, or ceil(n1 / F) unpadded
    int Kp = 0;                      // n1 padded to kKStep
    int Mh = 0, Mp = 0;              // frequential rows per spin, padded to kTileL
    std::vector<int> k2, Ta, Tp, nch, chunk;   // per alpha: decimation, length, padded length, t-chunks
    std::vector<int64_t> yoff, phioff, vchoff; // per alpha offsets
    int64_t sumTp = 0, sumch = 0, sumT = 0;
    std::vector<int> kfr, Lb, rowoff;          // per beta
    std::vector<int64_t> pfoff;
    int Mphi = 0;                    // phi_T support on the NX grid (bins 0..Mphi)
    Family f1, f2, ffr;
};

// Validate and solve; returns JTFS_OK or JTFS_EINVAL with the error set.
int solve_shapes(const jtfs_params& p, Shapes* s);
// t-chunks of the forward contraction: chunk[a] = min(Tp[a], chunk) columns per
// workgroup, nch[a] partial-V slots per rate, their offsets and total (sumch).
void set_chunks(Shapes* s, int chunk);
// JTFS_OK if the device path of this library handles the shapes, else JTFS_ENOTSUP.
int check_supported(const Shapes& s);
const char* last_error();

// Workspace layout for B signals (byte offsets from the workspace base).
struct Workspace {
    size_t xh = 0, tmp = 0, tmp64 = 0, z64 = 0, Xh = 0, Y2 = 0, Vp = 0;   // forward
    size_t Yh = 0, rowmax = 0, yscale = 0, gvmax = 0;          // split-FP16 operands
    size_t gV = 0, PQ = 0, gY2 = 0, gX = 0, g1 = 0, gxh = 0;   // backward
    size_t phase = 0;              // stored unit phase of the contraction output (SPLIT_F16_PHASE)
    int64_t ph_bstride = 0;        // stored-phase elements (two snorm16) per signal: 2 spins x sum Tp x Mp
    size_t gvs = 0;                // gV split into FP16 planes for the stored-phase backward
    int64_t gvs_bstride = 0;       // 16-byte units of gvs per signal
    int64_t vp_bstride = 0;        // floats of partial V per signal
    size_t total = 0;
    size_t fwd_total = 0;          // leading part of the layout that the forward uses
    int64_t xh_pitch = 0, Xh_pitch = 0;
};
// with_split: the split-FP16 operand copy of Y2; with_pq: the FP32 backward's P/Q';
// with_phase: the stored unit phase of the contraction output, per signal and rate
// [spin][Mp / 32][4][Tp][8] elements of two snorm16.
Workspace layout(const Shapes& s, int64_t B, bool with_split, bool with_pq, bool with_phase);

}  // namespace jtfs

namespace jtfs {
// Launch choices an autotuner may change (defaults: register-resident 2^14-point rows).
struct Tuning {
    bool reg_scalogram = true;   // scalogram rows of 2^14 points
    bool reg_second = true;      // second-order rows of 2^14 points
    bool reg_rowfft = true;      // FFT of the gY2 rows of 2^14 points
    bool reg_first_adj = true;   // first-order adjoint rows of 2^14 points
    bool fwd16 = false;          // forward contraction in 16 x 16 tiles (else 32 x 32)
    bool bwd16 = false;          // stored-phase backward in 16 x 16 tiles (else 32 x 32)
    // register-resident rows: radix-8 passes instead of radix-16 ones, per stage
    bool r8_scalogram = false, r8_second = false, r8_rowfft = false, r8_first_adj = false;
    bool batch8k = false;        // in-LDS row transforms: 8192 points per workgroup (else 4096)
    int chunk = kChunkT;         // t-columns per workgroup of the forward contraction (1024, 2048 or 4096)
};
// points per workgroup of the in-LDS second-order and gY2 row transforms
inline int lds_batch_log(const Tuning& t) { return t.batch8k ? 13 : 12; }
// rows of 2^logn points take the register-resident kernels above 2^14 always, at
// 2^14 when the tuning says so, and the in-LDS kernels below
inline bool use_reg_rows(int logn, bool knob) { return logn > kRegMinLogRows || (logn == kRegMinLogRows && knob); }
}  // namespace jtfs

struct jtfs_plan {
    jtfs::Shapes s;
    jtfs::Tuning tune;
    int device = 0;
    int tw_log = 0;
    float2* tw = nullptr;          // e^{-2 pi i k / 2^tw_log}
    double2* tw64 = nullptr;       // the same in FP64 (input transform)
    float* psi1 = nullptr;         // packed first-order spectra (real)
    int* band1 = nullptr;          // [n1][2] lo, hi
    int64_t* off1 = nullptr;
    float* psi2 = nullptr;         // packed second-order spectra
    int* band2 = nullptr;
    int64_t* off2 = nullptr;
    float2* Wt = nullptr;          // frequential wavelet matrix, theta=-1, [Kp][Mp] (k-major)
    float2* Wl = nullptr;          // same, [Mp][Kp] (row-major)
    float* Phi = nullptr;          // per alpha [Tp][NTp]: phi_alpha[(tau d - t) mod T_alpha]
    float* PF = nullptr;           // per beta [NL][Lb]: phi_F[(m F/2^kfr - l) mod Lb]
    float* PFt = nullptr;          // per beta [Lb][NL]: PF transposed (the forward lowpass reads rows l)
    float* phiX = nullptr;         // phi_T spectrum on the NX grid, bins 0..Mphi
    float* phiN = nullptr;         // zeroth order: phi_T on the N grid, phiN[k] = phi_T[(k - phiN_half) mod N]
    int64_t phiN_len = 0, phiN_half = 0;
    int* lam_range = nullptr;      // per 256-bin range of 0..N/2: first and last lambda touching it
    int64_t* d_yoff = nullptr;     // per alpha: offset of its Y2 block
    int* d_Tp = nullptr;           // per alpha: padded length
    int* d_Ta = nullptr;           // per alpha: length NX / 2^k2
    int64_t* d_vchoff = nullptr;   // per alpha: first partial-V slot
    int* d_nch = nullptr;          // per alpha: partial-V slots (t-chunks)
    int64_t* d_pfoff = nullptr;    // per beta: offset of its frequency-lowpass matrix
    int* d_Lb = nullptr;           // per beta: L / 2^kfr
    int* d_rowoff = nullptr;       // per beta: first row of the contraction
    double c1 = 0, c2 = 0, cfr = 0;  // Littlewood-Paley normalisations
    // split-FP16 contraction operands (hi + lo halves of power-of-two scaled FP32 values)
    int contraction = 0;           // JTFS_CONTRACTION_FP32, _SPLIT_F16 or _SPLIT_F16_PHASE
    bool split_ok = false;         // shapes allow the split kernels (W tile fits in LDS)
    bool split_bwd_ok = false;     // ... and the recomputing split backward (register budget)
    bool split_bwdp_ok = false;    // ... and the stored-phase split backward
    unsigned short* Wsp = nullptr; // [Mp][Kp/8][4][8]: re_hi, re_lo, im_hi, im_lo of W * sw
    float sw = 1.f;
    unsigned short* Phsp = nullptr;  // per alpha [Tp/32][2][2][NTp][2][8]: Phi * sphi[alpha]
    int KpT = 0;                   // Kp rounded up to 32 (rows of WTsp)
    unsigned short* WTsp = nullptr;  // [Mp/32][KpT/32][16][32][8]: W^T * sw, chunks in LDS order
    unsigned short* PhTsp = nullptr; // per alpha [Tp][NTp/8][2][8]: Phi * sphi[alpha], tau contiguous
    unsigned short* Phq = nullptr;   // per alpha [Tp/16][NTp/16][64][2][4]: Phi * sphi[alpha] (N/T <= 32)
    unsigned short* WTq = nullptr;   // [Mp/32][KpT/16][4][64][8]: W^T * sw in the 16 x 16 backward's k order
    unsigned short* Wq = nullptr;    // [Mp/64][ceil(Kp/32)][4][4][64][8]: W * sw in the 16 x 16 forward's read order
    std::vector<float> sphi;
    void* owned = nullptr;         // list of device allocations released by destroy
};
