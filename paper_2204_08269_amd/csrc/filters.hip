// Plan creation: every filter table is built on the device in FP64 (Morlet and
// Gaussian spectra, the Littlewood-Paley normalisation, the lambda-domain
// frequential wavelet matrix, the time and frequency lowpass matrices, FFT
// twiddles) and stored as FP32 for the transform kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "plan.hpp"
#include "split.hpp"

namespace jtfs {

// Un-normalised Morlet spectrum at f >= 0 (sec. 2): Gaussian at xi minus the
// corrective Gaussian that makes the value at f = 0 exactly zero.
__device__ __forceinline__ double morlet_raw(double xi, double sg, double f) {
    if (f < 0.0) return 0.0;
    const double d = 2.0 * sg * sg;
    return exp(-(f - xi) * (f - xi) / d) - exp(-(f * f + xi * xi) / d);
}

// max over bins 0..M/2 of sum_lambda psi_hat_lambda^2 (single workgroup).
__global__ void __launch_bounds__(1024) k_fb_lp(const double* __restrict__ xi, const double* __restrict__ sg,
                                                const int* __restrict__ band, int n, int M, double* __restrict__ out) {
    __shared__ double red[1024];
    double best = 0.0;
    for (int m = threadIdx.x; m <= M / 2; m += blockDim.x) {
        const double f = (double)m / (double)M;
        double acc = 0.0;
        for (int i = 0; i < n; ++i) {
            if (m < band[2 * i] || m > band[2 * i + 1]) continue;
            const double v = morlet_raw(xi[i], sg[i], f);
            acc += v * v;
        }
        best = fmax(best, acc);
    }
    red[threadIdx.x] = best;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = 1.0 / sqrt(red[0]);
}

// packed[off_i + j] = c * psi_hat_i(lo_i + j)
__global__ void k_fb_pack(const double* __restrict__ xi, const double* __restrict__ sg, const int* __restrict__ band,
                          const int64_t* __restrict__ off, int n, int M, int64_t total, const double* __restrict__ cnorm,
                          float* __restrict__ out) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= total) return;
    int a = 0, b = n - 1;                       // last i with off[i] <= e
    while (a < b) {
        const int mid = (a + b + 1) / 2;
        if (off[mid] <= e) a = mid; else b = mid - 1;
    }
    const int m = band[2 * a] + (int)(e - off[a]);
    out[e] = (float)(cnorm[0] * morlet_raw(xi[a], sg[a], (double)m / (double)M));
}

// psi_{beta,-1}[j] = (c/L) sum_{m=0}^{L/2} psi_hat_beta(m/L) e^{2 pi i m j / L}
__global__ void k_fb_psi_fr(const double* __restrict__ xi, const double* __restrict__ sg, int L,
                            const double* __restrict__ cnorm, double2* __restrict__ out) {
    const int beta = blockIdx.y;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= L) return;
    double re = 0.0, im = 0.0;
    for (int m = 0; m <= L / 2; ++m) {
        const double v = morlet_raw(xi[beta], sg[beta], (double)m / L);
        double s, c;
        sincospi(2.0 * (double)((int64_t)m * j % L) / L, &s, &c);
        re += v * c;
        im += v * s;
    }
    out[(int64_t)beta * L + j] = make_double2(re * cnorm[0] / L, im * cnorm[0] / L);
}

// W[row=(beta,l)][i] = psi_{beta,-1}[(l 2^kfr - i) mod L] for i < n1, 0 for padding,
// stored k-major (Wt[i][row]) and row-major (Wl[row][i]).
__global__ void k_fb_W(const double2* __restrict__ psi, const int* __restrict__ row_beta, const int* __restrict__ row_l,
                       const int* __restrict__ kfr, int Mh, int Mp, int n1, int Kp, int L,
                       float2* __restrict__ Wt, float2* __restrict__ Wl) {
    const int row = blockIdx.y;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= Kp) return;
    float2 w = make_float2(0.f, 0.f);
    if (row < Mh && i < n1) {
        const int beta = row_beta[row], l = row_l[row];
        const int j = (((l << kfr[beta]) - i) % L + L) % L;
        const double2 v = psi[(int64_t)beta * L + j];
        w = make_float2((float)v.x, (float)v.y);
    }
    Wt[(int64_t)i * Mp + row] = w;
    Wl[(int64_t)row * Kp + i] = w;
}

// Gaussian lowpass spectrum exp(-f^2 / (2 s^2)), f = mt / units.
__device__ __forceinline__ double gauss_hat(double mt, double units, double s) {
    const double f = mt / units;
    return exp(-f * f / (2.0 * s * s));
}

// Phi_alpha[t][tau] = phi_alpha[(tau d - t) mod Ta] (0 outside t < Ta, tau < NT),
// phi_alpha = inverse DFT on the Ta grid of the phi_T spectrum (bin m~ at m~/N).
__global__ void k_fb_phi(float* __restrict__ Phi, int Ta, int Tp, int NT, int NTp, int d, double N, double sgT,
                         int Mphi) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)Tp * NTp) return;
    const int t = (int)(e / NTp), tau = (int)(e % NTp);
    float val = 0.f;
    if (t < Ta && tau < NT) {
        const int j = (int)((((int64_t)tau * d - t) % Ta + Ta) % Ta);
        const int Mx = min(Mphi, Ta / 2);
        double acc = gauss_hat(0.0, N, sgT);
        for (int m = 1; m <= Mx; ++m) {
            const double g = gauss_hat((double)m, N, sgT);
            double s, c;
            sincospi(2.0 * (double)((int64_t)m * j % Ta) / Ta, &s, &c);
            acc += (m == Ta / 2 ? 1.0 : 2.0) * g * c;    // bins +m and -m (Nyquist once)
        }
        val = (float)(acc / Ta);
    }
    Phi[e] = val;
}

// PF_beta[m][l] = phi_F[(m step - l) mod Lb], phi_F = inverse DFT on the Lb grid of
// the phi_F spectrum (bin m~ at m~/L cycles per lambda bin).
__global__ void k_fb_pf(float* __restrict__ PF, int NL, int Lb, int step, double L, double sgF) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= NL * Lb) return;
    const int m = e / Lb, l = e % Lb;
    const int j = ((m * step - l) % Lb + Lb) % Lb;
    double acc = 0.0;
    for (int q = 0; q < Lb; ++q) {
        const int mt = q <= Lb / 2 ? q : q - Lb;
        double s, c;
        sincospi(2.0 * (double)((int64_t)q * j % Lb) / Lb, &s, &c);
        acc += gauss_hat((double)mt, L, sgF) * c;
    }
    PF[e] = (float)(acc / Lb);
}

// PFt_beta[l][m] = PF_beta[m][l]
__global__ void k_fb_pft(const float* __restrict__ PF, float* __restrict__ PFt, int NL, int Lb) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= NL * Lb) return;
    const int l = e / NL, m = e % NL;
    PFt[e] = PF[(int64_t)m * Lb + l];
}

// The lowpass as the last row block of the frequential matrix (lowpass pairs):
// phi_F[j] = (1/L) sum over the L bins of phi_F_hat(m~/L) e^{2 pi i m j / L}, real
// and even, so its two spins coincide.
__global__ void k_fb_phi_fr(double2* __restrict__ out, int L, double sgF) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= L) return;
    double acc = 0.0;
    for (int q = 0; q < L; ++q) {
        const int mt = q <= L / 2 ? q : q - L;
        double s, c;
        sincospi(2.0 * (double)((int64_t)q * j % L) / L, &s, &c);
        acc += gauss_hat((double)mt, L, sgF) * c;
    }
    out[j] = make_double2(acc / L, 0.0);
}

// Zeroth order: phi_T on the N-sample grid around offset 0,
// h[k] = phi_T[(k - H) mod N] for k < len, phi_T[j] = (1/N) sum over bins |m| <= Mx
// of phi_hat_T(m/N) e^{2 pi i m j / N} (the Nyquist bin once).
__global__ void k_fb_phin(float* __restrict__ h, int64_t len, int64_t H, int64_t N, double sgT, int64_t Mx) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= len) return;
    const int64_t j = ((k - H) % N + N) % N;
    double acc = gauss_hat(0.0, (double)N, sgT);
    for (int64_t m = 1; m <= Mx; ++m) {
        double s, c;
        sincospi(2.0 * (double)(m * j % N) / (double)N, &s, &c);
        acc += (2 * m == N ? 1.0 : 2.0) * gauss_hat((double)m, (double)N, sgT) * c;
    }
    h[k] = (float)(acc / (double)N);
}

__global__ void k_fb_phix(float* __restrict__ phiX, int Mphi, double N, double sgT) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m <= Mphi) phiX[m] = (float)gauss_hat((double)m, N, sgT);
}

__global__ void k_fb_twiddle(float2* __restrict__ tw, int tw_log) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= ((int64_t)1 << tw_log)) return;
    double s, c;
    sincospi(2.0 * (double)k / (double)((int64_t)1 << tw_log), &s, &c);
    tw[k] = make_float2((float)c, (float)-s);
}

__global__ void k_fb_twiddle64(double2* __restrict__ tw, int tw_log) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= ((int64_t)1 << tw_log)) return;
    double s, c;
    sincospi(2.0 * (double)k / (double)((int64_t)1 << tw_log), &s, &c);
    tw[k] = make_double2(c, -s);
}

}  // namespace jtfs

using namespace jtfs;

namespace {

struct DevAlloc {
    std::vector<void*> ptrs;
    bool failed = false;
    template <class T> T* get(size_t count) {
        void* p = nullptr;
        if (hipMalloc(&p, std::max<size_t>(count, 1) * sizeof(T)) != hipSuccess) { failed = true; return nullptr; }
        ptrs.push_back(p);
        return (T*)p;
    }
    void release() { for (void* p : ptrs) (void)hipFree(p); ptrs.clear(); }
};

template <class T> T* upload(DevAlloc& A, const std::vector<T>& v) {
    T* d = A.get<T>(v.size());
    if (d && !v.empty()) {
        if (hipMemcpy(d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess) A.failed = true;
    }
    return d;
}

#define HIPCHK(x)                                                         \
    do {                                                                  \
        hipError_t e_ = (x);                                              \
        if (e_ != hipSuccess) {                                           \
            set_error(std::string(#x) + ": " + hipGetErrorString(e_));    \
            return JTFS_EHIP;                                             \
        }                                                                 \
    } while (0)

int build_family(DevAlloc& A, const Family& f, float** vals, int** band, int64_t** off, double* cval) {
    std::vector<int> bd(2 * f.n());
    for (int i = 0; i < f.n(); ++i) { bd[2 * i] = f.lo[i]; bd[2 * i + 1] = f.hi[i]; }
    double* dxi = upload(A, f.xi);
    double* dsg = upload(A, f.sigma);
    *band = upload(A, bd);
    *off = upload(A, f.off);
    double* dc = A.get<double>(1);
    *vals = A.get<float>(f.total);
    if (A.failed) { set_error("device allocation failed"); return JTFS_ENOMEM; }
    hipLaunchKernelGGL(k_fb_lp, dim3(1), dim3(1024), 0, 0, dxi, dsg, *band, f.n(), f.M, dc);
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(k_fb_pack, dim3((unsigned)((f.total + 255) / 256)), dim3(256), 0, 0, dxi, dsg, *band, *off, f.n(),
                       f.M, f.total, dc, *vals);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpy(cval, dc, sizeof(double), hipMemcpyDeviceToHost));
    return JTFS_OK;
}

}  // namespace

namespace jtfs {
int setup_kernel_attributes();  // kernels.hip
}

extern "C" int jtfs_plan_create_ex(jtfs_plan** out, const jtfs_params* p) {
    if (!out || !p) { set_error("null pointer"); return JTFS_EINVAL; }
    *out = nullptr;
    Shapes s;
    int st = solve_shapes(*p, &s);
    if (st != JTFS_OK) return st;
    st = check_supported(s);
    if (st != JTFS_OK) return st;
    if (s.NTp > 128) { set_error("N/T above 128 frames is not supported by this library"); return JTFS_ENOTSUP; }
    if ((s.NX / 2 + 1 + s.NT) * sizeof(float2) > 160 * 1024 || (size_t)33 * s.L * sizeof(float) > 160 * 1024) {
        set_error("LDS needs of these shapes exceed 160 KB"); return JTFS_ENOTSUP; }
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    st = setup_kernel_attributes();
    if (st != JTFS_OK) return st;

    jtfs_plan* P = new (std::nothrow) jtfs_plan();
    if (!P) { set_error("host allocation failed"); return JTFS_ENOMEM; }
    P->s = s;
    P->device = dev;
    DevAlloc A;
    auto fail = [&](int code) { A.release(); delete P; return code; };

    // twiddles for every FFT length up to N
    P->tw_log = s.logN;
    P->tw = A.get<float2>((size_t)1 << P->tw_log);
    P->tw64 = A.get<double2>((size_t)1 << P->tw_log);
    if (A.failed) { set_error("device allocation failed"); return fail(JTFS_ENOMEM); }
    hipLaunchKernelGGL(k_fb_twiddle, dim3((unsigned)((((int64_t)1 << P->tw_log) + 255) / 256)), dim3(256), 0, 0, P->tw,
                       P->tw_log);
    hipLaunchKernelGGL(k_fb_twiddle64, dim3((unsigned)((((int64_t)1 << P->tw_log) + 255) / 256)), dim3(256), 0, 0,
                       P->tw64, P->tw_log);
    if (hipGetLastError() != hipSuccess) { set_error("twiddle kernel failed"); return fail(JTFS_EHIP); }

    if ((st = build_family(A, s.f1, &P->psi1, &P->band1, &P->off1, &P->c1)) != JTFS_OK) return fail(st);
    if ((st = build_family(A, s.f2, &P->psi2, &P->band2, &P->off2, &P->c2)) != JTFS_OK) return fail(st);

    // frequential family: normalisation on the L grid, then lambda-domain wavelets
    {
        float* dummy_vals; int* band; int64_t* off;
        if ((st = build_family(A, s.ffr, &dummy_vals, &band, &off, &P->cfr)) != JTFS_OK) return fail(st);
        double* dxi = upload(A, s.ffr.xi);
        double* dsg = upload(A, s.ffr.sigma);
        double* dc = upload(A, std::vector<double>{P->cfr});
        double2* psi = A.get<double2>((size_t)s.n_beta * s.L);
        std::vector<int> rb(s.Mh), rl(s.Mh);
        for (int b = 0; b < s.n_beta; ++b)
            for (int l = 0; l < s.Lb[b]; ++l) { rb[s.rowoff[b] + l] = b; rl[s.rowoff[b] + l] = l; }
        int* drb = upload(A, rb);
        int* drl = upload(A, rl);
        int* dkfr = upload(A, s.kfr);
        P->Wt = A.get<float2>((size_t)s.Kp * s.Mp);
        P->Wl = A.get<float2>((size_t)s.Mp * s.Kp);
        if (A.failed) { set_error("device allocation failed"); return fail(JTFS_ENOMEM); }
        hipLaunchKernelGGL(k_fb_psi_fr, dim3((s.L + 127) / 128, s.n_beta_psi), dim3(128), 0, 0, dxi, dsg, s.L, dc, psi);
        if (s.complete)
            hipLaunchKernelGGL(k_fb_phi_fr, dim3((s.L + 127) / 128), dim3(128), 0, 0, psi + (size_t)s.n_beta_psi * s.L,
                               s.L, kSigma0 / (double)s.F);
        hipLaunchKernelGGL(k_fb_W, dim3((s.Kp + 63) / 64, s.Mp), dim3(64), 0, 0, psi, drb, drl, dkfr, s.Mh, s.Mp, s.n1,
                           s.Kp, s.L, P->Wt, P->Wl);
        if (hipGetLastError() != hipSuccess) { set_error("frequential wavelet kernels failed"); return fail(JTFS_EHIP); }
    }
    // lowpass matrices
    {
        const double sgT = kSigma0 / (double)s.T, sgF = kSigma0 / (double)s.F;
        P->Phi = A.get<float>((size_t)s.sumTp * s.NTp);
        int64_t pf_total = 0;
        for (int b = 0; b < s.n_beta; ++b) pf_total += (int64_t)s.NL * s.Lb[b];
        P->PF = A.get<float>((size_t)pf_total);
        P->PFt = A.get<float>((size_t)pf_total);
        P->phiX = A.get<float>((size_t)s.Mphi + 1);
        if (A.failed) { set_error("device allocation failed"); return fail(JTFS_ENOMEM); }
        for (int a = 0; a < s.n_alpha; ++a) {
            const int64_t cnt = (int64_t)s.Tp[a] * s.NTp;
            const int d = (int)(s.T >> (s.kX + s.k2[a]));
            hipLaunchKernelGGL(k_fb_phi, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, 0, P->Phi + s.phioff[a], s.Ta[a],
                               s.Tp[a], s.NT, s.NTp, d, (double)s.N, sgT, s.Mphi);
        }
        for (int b = 0; b < s.n_beta; ++b) {
            const int cnt = s.NL * s.Lb[b];
            hipLaunchKernelGGL(k_fb_pf, dim3((cnt + 255) / 256), dim3(256), 0, 0, P->PF + s.pfoff[b], s.NL, s.Lb[b],
                               (int)(s.F >> s.kfr[b]), (double)s.L, sgF);
            hipLaunchKernelGGL(k_fb_pft, dim3((cnt + 255) / 256), dim3(256), 0, 0, P->PF + s.pfoff[b],
                               P->PFt + s.pfoff[b], s.NL, s.Lb[b]);
        }
        hipLaunchKernelGGL(k_fb_phix, dim3((s.Mphi + 256) / 256), dim3(256), 0, 0, P->phiX, s.Mphi, (double)s.N, sgT);
        // zeroth order: phi_T in time, within the offsets where it exceeds kSupportTol of its peak
        {
            const double R = std::sqrt(2.0 * std::log(1.0 / kSupportTol));
            const double sg_t = 1.0 / (2.0 * M_PI * sgT);                 // its width in samples
            const int64_t H = (int64_t)std::ceil(R * sg_t);
            if (2 * H + 1 >= s.N) { P->phiN_len = s.N; P->phiN_half = s.N / 2; }
            else { P->phiN_len = 2 * H + 1; P->phiN_half = H; }
            const double mm = (double)s.N * sgT * R;
            const int64_t Mx = std::min<int64_t>(s.N / 2, (int64_t)std::floor(mm) + 1);
            P->phiN = A.get<float>((size_t)P->phiN_len);
            if (A.failed) { set_error("device allocation failed"); return fail(JTFS_ENOMEM); }
            hipLaunchKernelGGL(k_fb_phin, dim3((unsigned)((P->phiN_len + 255) / 256)), dim3(256), 0, 0, P->phiN,
                               P->phiN_len, P->phiN_half, s.N, sgT, Mx);
        }
        if (hipGetLastError() != hipSuccess) { set_error("lowpass kernels failed"); return fail(JTFS_EHIP); }
    }
    // first-order bands touching each 256-bin range of 0..N/2 (gradient accumulation)
    {
        const int64_t nb = s.N / 2 + 1, nr = (nb + 255) / 256;
        std::vector<int> rng(2 * nr);
        for (int64_t r = 0; r < nr; ++r) {
            const int64_t m0 = r * 256, m1 = std::min<int64_t>(nb - 1, m0 + 255);
            int a = -1, b = -2;
            for (int i = 0; i < s.n1; ++i)
                if (s.f1.lo[i] <= m1 && s.f1.hi[i] >= m0) { if (a < 0) a = i; b = i; }
            rng[2 * r] = a; rng[2 * r + 1] = b;
        }
        P->lam_range = upload(A, rng);
        P->d_yoff = upload(A, s.yoff);
        P->d_Tp = upload(A, s.Tp);
        P->d_Ta = upload(A, s.Ta);
        P->d_vchoff = upload(A, s.vchoff);
        P->d_nch = upload(A, s.nch);
        P->d_pfoff = upload(A, s.pfoff);
        P->d_Lb = upload(A, s.Lb);
        P->d_rowoff = upload(A, s.rowoff);
        if (A.failed) { set_error("device allocation failed"); return fail(JTFS_ENOMEM); }
    }
    if (hipDeviceSynchronize() != hipSuccess) { set_error("plan construction failed on the device"); return fail(JTFS_EHIP); }
    if ((st = build_split_tables(P, A.ptrs)) != JTFS_OK) return fail(st);
    // the plan keeps every allocation; stash the list for destroy
    auto* keep = new (std::nothrow) std::vector<void*>(A.ptrs);
    if (!keep) return fail(JTFS_ENOMEM);
    P->owned = keep;
    *out = P;
    return JTFS_OK;
}

extern "C" int jtfs_plan_create(jtfs_plan** out, int64_t N, int J, const int Q[2], int J_fr, int Q_fr, int64_t T,
                                int64_t F) {
    if (!Q) { set_error("null pointer"); return JTFS_EINVAL; }
    jtfs_params p{};
    p.N = N; p.J = J; p.Q1 = Q[0]; p.Q2 = Q[1]; p.J_fr = J_fr; p.Q_fr = Q_fr; p.T = T; p.F = F; p.flags = 0;
    return jtfs_plan_create_ex(out, &p);
}

extern "C" void jtfs_plan_destroy(jtfs_plan* P) {
    if (!P) return;
    if (P->owned) {
        auto* v = (std::vector<void*>*)P->owned;
        for (void* p : *v) (void)hipFree(p);
        delete v;
    }
    delete P;
}

extern "C" int jtfs_plan_info(const jtfs_plan* P, jtfs_info* out) {
    if (!P) { set_error("null plan"); return JTFS_EINVAL; }
    const int rc = jtfs_query(&P->s.p, out);
    if (rc != JTFS_OK) return rc;
    size_t f = 0, t = 0;
    jtfs_forward_workspace_size(P, 1, &f);
    jtfs_workspace_size(P, 1, &t);
    out->ws_fwd = (int64_t)f;
    out->ws_bwd = (int64_t)t;
    return JTFS_OK;
}

extern "C" int jtfs_plan_tables(const jtfs_plan* P, double* xi_sigma, int32_t* schedule) {
    if (!P) { set_error("null plan"); return JTFS_EINVAL; }
    const Shapes& s = P->s;
    const Family* fams[3] = {&s.f1, &s.f2, &s.ffr};
    int64_t o = 0;
    for (const Family* f : fams)
        for (int i = 0; i < f->n(); ++i, ++o)
            if (xi_sigma) { xi_sigma[2 * o] = f->xi[i]; xi_sigma[2 * o + 1] = f->sigma[i]; }
    if (schedule) {
        int q = 0;
        schedule[q++] = s.kX;
        for (int a = 0; a < s.n_alpha_psi; ++a) schedule[q++] = s.k2[a];
        for (int b = 0; b < s.n_beta_psi; ++b) schedule[q++] = s.kfr[b];
    }
    return JTFS_OK;
}

extern "C" int jtfs_plan_table(const jtfs_plan* P, int which, void* host_dst, size_t bytes) {
    if (!P || !host_dst) { set_error("null pointer"); return JTFS_EINVAL; }
    const Shapes& s = P->s;
    if (which == 0 || which == 1) {
        const Family& f = which == 0 ? s.f1 : s.f2;
        const int64_t W = f.M / 2 + 1;
        if (bytes != sizeof(float) * W * f.n()) { set_error("table size mismatch"); return JTFS_ESHAPE; }
        std::vector<float> packed(f.total);
        HIPCHK(hipMemcpy(packed.data(), which == 0 ? P->psi1 : P->psi2, sizeof(float) * f.total, hipMemcpyDeviceToHost));
        float* dst = (float*)host_dst;
        std::memset(dst, 0, bytes);
        for (int i = 0; i < f.n(); ++i)
            for (int m = f.lo[i]; m <= f.hi[i]; ++m) dst[(int64_t)i * W + m] = packed[f.off[i] + m - f.lo[i]];
        return JTFS_OK;
    }
    if (which == 2) {
        if (bytes != sizeof(float2) * s.Mh * s.n1) { set_error("table size mismatch"); return JTFS_ESHAPE; }
        std::vector<float2> Wl((size_t)s.Mp * s.Kp);
        HIPCHK(hipMemcpy(Wl.data(), P->Wl, sizeof(float2) * Wl.size(), hipMemcpyDeviceToHost));
        float2* dst = (float2*)host_dst;
        for (int r = 0; r < s.Mh; ++r)
            for (int i = 0; i < s.n1; ++i) dst[(int64_t)r * s.n1 + i] = Wl[(int64_t)r * s.Kp + i];
        return JTFS_OK;
    }
    set_error("unknown table");
    return JTFS_EINVAL;
}
