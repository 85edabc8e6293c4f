// mu-log renormalisation of the scattering coefficients (sec. 4): per-path means
// mu over a batch and log(1 + S / (eps mu)), with its adjoint for mu held fixed.
//
// A path is S1 as a whole (every lambda1 and frame of a signal) or one
// (alpha, beta, theta) slice of S2.  In both S2 layouts (eq. (3) and the packed
// eq. (4) layout) a slice is one contiguous block per signal, so every kernel
// runs one workgroup per (path, signal) over that block; block index n_paths
// stands for S1.  In time scattering (S2 [n_alpha][n1][N/T]) a second-order
// path is one (alpha, lambda1) pair, its N/T frames a contiguous row: the same
// geometry as eq. (3) with one row per path.
#include <hip/hip_runtime.h>

#include "plan.hpp"

namespace jtfs {

struct PathGeom {
    int n_paths, n_beta, NL, NT, Mh, avg;
    int64_t s1_per, s2_per;
    const int* rowoff;
    const int* Lb;
};

// offset (within one signal's S2, or S1 for p == n_paths) and length of path p
__device__ __forceinline__ void path_span(const PathGeom& g, int p, int64_t* off, int64_t* len) {
    if (p == g.n_paths) { *off = 0; *len = g.s1_per; return; }
    if (g.avg) { *off = (int64_t)p * g.NL * g.NT; *len = (int64_t)g.NL * g.NT; return; }
    const int a = p / (2 * g.n_beta), be = (p >> 1) % g.n_beta, th = p & 1;
    *off = ((int64_t)a * 2 * g.Mh + 2 * g.rowoff[be] + th * g.Lb[be]) * g.NT;
    *len = (int64_t)g.Lb[be] * g.NT;
}

__global__ void __launch_bounds__(256) k_path_mean(PathGeom g, const float* __restrict__ s1,
                                                   const float* __restrict__ s2, int64_t B, float* __restrict__ mu1,
                                                   float* __restrict__ mu2) {
    __shared__ double red[256];
    const int p = blockIdx.x;
    int64_t off, len;
    path_span(g, p, &off, &len);
    const float* base = p == g.n_paths ? s1 : s2;
    const int64_t per = p == g.n_paths ? g.s1_per : g.s2_per;
    double acc = 0.0;
    for (int64_t b = 0; b < B; ++b)
        for (int64_t j = threadIdx.x; j < len; j += blockDim.x) acc += (double)base[b * per + off + j];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const float m = (float)(red[0] / ((double)B * (double)len));
        if (p == g.n_paths) mu1[0] = m;
        else mu2[p] = m;
    }
}

// out = log1p(S / (eps mu)); out may alias S
__global__ void __launch_bounds__(256) k_mulog(PathGeom g, const float* s1, const float* s2,
                                               const float* __restrict__ mu1, const float* __restrict__ mu2, float eps,
                                               float* o1, float* o2) {
    const int p = blockIdx.x;
    const int64_t b = blockIdx.y;
    int64_t off, len;
    path_span(g, p, &off, &len);
    const bool first = p == g.n_paths;
    const int64_t o = b * (first ? g.s1_per : g.s2_per) + off;
    const float* S = (first ? s1 : s2) + o;
    float* O = (first ? o1 : o2) + o;
    const float inv = 1.f / (eps * (first ? mu1[0] : mu2[p]));
    for (int64_t j = threadIdx.x; j < len; j += blockDim.x) O[j] = log1pf(S[j] * inv);
}

// gS = g / (eps mu + S); gS may alias g
__global__ void __launch_bounds__(256) k_mulog_bwd(PathGeom g, const float* __restrict__ s1,
                                                   const float* __restrict__ s2, const float* __restrict__ mu1,
                                                   const float* __restrict__ mu2, float eps, const float* g1,
                                                   const float* g2, float* gs1, float* gs2) {
    const int p = blockIdx.x;
    const int64_t b = blockIdx.y;
    int64_t off, len;
    path_span(g, p, &off, &len);
    const bool first = p == g.n_paths;
    const int64_t o = b * (first ? g.s1_per : g.s2_per) + off;
    const float* S = (first ? s1 : s2) + o;
    const float* G = (first ? g1 : g2) + o;
    float* D = (first ? gs1 : gs2) + o;
    const float em = eps * (first ? mu1[0] : mu2[p]);
    for (int64_t j = threadIdx.x; j < len; j += blockDim.x) D[j] = G[j] / (em + S[j]);
}

static PathGeom geom(const jtfs_plan* P) {
    const Shapes& s = P->s;
    PathGeom g;
    if (s.tscat) {
        g.n_paths = s.n_alpha * s.n1;
        g.n_beta = 0;
        g.NL = 1;
        g.NT = s.NT;
        g.Mh = 0;
        g.avg = 1;
        g.s1_per = (int64_t)s.n1 * s.NT;
        g.s2_per = (int64_t)g.n_paths * s.NT;
        g.rowoff = nullptr;
        g.Lb = nullptr;
        return g;
    }
    g.n_paths = s.n_alpha * s.n_beta * 2;
    g.n_beta = s.n_beta;
    g.NL = s.NLo;
    g.NT = s.NT;
    g.Mh = s.Mh;
    g.avg = s.avg_fr ? 1 : 0;
    g.s1_per = (int64_t)s.n1 * s.NT;
    g.s2_per = s.avg_fr ? (int64_t)g.n_paths * s.NLo * s.NT : (int64_t)s.n_alpha * 2 * s.Mh * s.NT;
    g.rowoff = P->d_rowoff;
    g.Lb = P->d_Lb;
    return g;
}

}  // namespace jtfs

using namespace jtfs;

static int launch_status(const char* what) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error(std::string(what) + ": " + hipGetErrorString(e));
        return JTFS_EHIP;
    }
    return JTFS_OK;
}

extern "C" int jtfs_path_means(const jtfs_plan* P, const float* s1, const float* s2, int64_t B, float* mu1,
                               float* mu2, hipStream_t st) {
    if (!P || !s1 || !s2 || !mu1 || !mu2) { set_error("null pointer"); return JTFS_EINVAL; }
    if (B < 1 || B > 65535) { set_error("B must lie in [1, 65535]"); return JTFS_ESHAPE; }
    const PathGeom g = geom(P);
    hipLaunchKernelGGL(k_path_mean, dim3((unsigned)(g.n_paths + 1)), dim3(256), 0, st, g, s1, s2, B, mu1, mu2);
    return launch_status("path means");
}

extern "C" int jtfs_mulog(const jtfs_plan* P, const float* s1, const float* s2, int64_t B, const float* mu1,
                          const float* mu2, float eps, float* o1, float* o2, hipStream_t st) {
    if (!P || !s1 || !s2 || !mu1 || !mu2 || !o1 || !o2) { set_error("null pointer"); return JTFS_EINVAL; }
    if (B < 1 || B > 65535) { set_error("B must lie in [1, 65535]"); return JTFS_ESHAPE; }
    if (!(eps > 0.f)) { set_error("eps must be positive"); return JTFS_EINVAL; }
    const PathGeom g = geom(P);
    hipLaunchKernelGGL(k_mulog, dim3((unsigned)(g.n_paths + 1), (unsigned)B), dim3(256), 0, st, g, s1, s2, mu1, mu2,
                       eps, o1, o2);
    return launch_status("mu-log");
}

extern "C" int jtfs_mulog_backward(const jtfs_plan* P, const float* s1, const float* s2, int64_t B,
                                   const float* mu1, const float* mu2, float eps, const float* g1, const float* g2,
                                   float* gs1, float* gs2, hipStream_t st) {
    if (!P || !s1 || !s2 || !mu1 || !mu2 || !g1 || !g2 || !gs1 || !gs2) { set_error("null pointer"); return JTFS_EINVAL; }
    if (B < 1 || B > 65535) { set_error("B must lie in [1, 65535]"); return JTFS_ESHAPE; }
    if (!(eps > 0.f)) { set_error("eps must be positive"); return JTFS_EINVAL; }
    const PathGeom g = geom(P);
    hipLaunchKernelGGL(k_mulog_bwd, dim3((unsigned)(g.n_paths + 1), (unsigned)B), dim3(256), 0, st, g, s1, s2, mu1,
                       mu2, eps, g1, g2, gs1, gs2);
    return launch_status("mu-log adjoint");
}
