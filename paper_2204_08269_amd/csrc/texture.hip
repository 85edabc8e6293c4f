// Texture resynthesis (sec. 5): gradient descent from a start y0 on the
// normalised error E(y) = ||Sx - Sy|| / ||Sx|| (S1 and S2 together), with the
// bold-driver learning rate, for a batch of independent signals.
//
// Every signal keeps its own state on the device (best iterate, its gradient,
// best error, learning rate); an iteration evaluates one candidate
// y_c = y_best - mu grad E(y_best): forward, residual and cotangent, backward,
// accept (E lower: y_best = y_c, mu *= 1.2) or reject (mu *= 0.5), next
// candidate.  The decision is taken on the device, so one iteration is a fixed
// sequence of launches, captured once as a HIP graph and replayed.
#include <hip/hip_runtime.h>

#include <cmath>
#include <new>
#include <vector>

#include "plan.hpp"

namespace jtfs {

constexpr float kBoldUp = 1.2f;
constexpr float kBoldDown = 0.5f;

// block-wide sum of one double per thread (blockDim.x = 1024)
__device__ __forceinline__ double block_sum(double v, double* red) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[w];
    return t;
}

// nx[b] = ||Sx_b|| over S1 and S2
__global__ void __launch_bounds__(1024) k_tex_norm(const float* __restrict__ s1, const float* __restrict__ s2,
                                                   int64_t n1, int64_t n2, float* __restrict__ nx) {
    __shared__ double red[16];
    const int64_t b = blockIdx.x;
    double acc = 0.0;
    for (int64_t j = threadIdx.x; j < n1; j += blockDim.x) { const double v = s1[b * n1 + j]; acc += v * v; }
    for (int64_t j = threadIdx.x; j < n2; j += blockDim.x) { const double v = s2[b * n2 + j]; acc += v * v; }
    const double t = block_sum(acc, red);
    if (threadIdx.x == 0) nx[b] = (float)sqrt(t);
}

// Ec[b] = ||Sc - Sx|| / ||Sx||; cotangent G = (Sc - Sx) / (||Sc - Sx|| ||Sx||) (0 if Sc = Sx)
__global__ void __launch_bounds__(1024) k_tex_resid(const float* __restrict__ c1, const float* __restrict__ c2,
                                                    const float* __restrict__ x1, const float* __restrict__ x2,
                                                    int64_t n1, int64_t n2, const float* __restrict__ nx,
                                                    float* __restrict__ Ec, float* __restrict__ g1,
                                                    float* __restrict__ g2) {
    __shared__ double red[16];
    const int64_t b = blockIdx.x;
    double acc = 0.0;
    for (int64_t j = threadIdx.x; j < n1; j += blockDim.x) {
        const double v = (double)c1[b * n1 + j] - (double)x1[b * n1 + j];
        acc += v * v;
    }
    for (int64_t j = threadIdx.x; j < n2; j += blockDim.x) {
        const double v = (double)c2[b * n2 + j] - (double)x2[b * n2 + j];
        acc += v * v;
    }
    const double nr = sqrt(block_sum(acc, red));
    const double den = nr * (double)nx[b];
    const float sc = den > 0.0 ? (float)(1.0 / den) : 0.f;
    if (threadIdx.x == 0) Ec[b] = nx[b] > 0.f ? (float)(nr / (double)nx[b]) : 0.f;
    for (int64_t j = threadIdx.x; j < n1; j += blockDim.x) g1[b * n1 + j] = (c1[b * n1 + j] - x1[b * n1 + j]) * sc;
    for (int64_t j = threadIdx.x; j < n2; j += blockDim.x) g2[b * n2 + j] = (c2[b * n2 + j] - x2[b * n2 + j]) * sc;
}

// Accept or reject the candidate of each signal.  init: the start itself (always
// kept; mu from mu0, or relative to the start when mu0 < 0).  Appends the best
// error to hist[count][b] when hist is given.
__global__ void __launch_bounds__(1024) k_tex_decide(const float* __restrict__ yc, const float* __restrict__ gc,
                                                     int64_t N, const float* __restrict__ Ec, float* __restrict__ Eb,
                                                     float* __restrict__ mu, int* __restrict__ acc, float mu0, int init,
                                                     float* __restrict__ hist, const int* __restrict__ count, int cap,
                                                     int64_t B) {
    __shared__ double red[16];
    const int64_t b = blockIdx.x;
    // relative initial rate |mu0| ||y0|| / ||grad E(y0)||: block-wide norms
    double ny = 0.0, ng = 0.0;
    if (init && !(mu0 > 0.f)) {
        double sy = 0.0, sg = 0.0;
        for (int64_t j = threadIdx.x; j < N; j += blockDim.x) {
            const double y = yc[b * N + j], g = gc[b * N + j];
            sy += y * y;
            sg += g * g;
        }
        ny = sqrt(block_sum(sy, red));
        ng = sqrt(block_sum(sg, red));
    }
    if (threadIdx.x != 0) return;
    float m = mu[b], e = Eb[b];
    int a;
    if (init) {
        a = 1;
        e = Ec[b];
        m = mu0 > 0.f ? mu0 : (ng > 0.0 ? (float)(-(double)mu0 * ny / ng) : 0.f);
    } else {
        a = Ec[b] < e ? 1 : 0;
        if (a) { e = Ec[b]; m *= kBoldUp; }
        else { m *= kBoldDown; }
    }
    acc[b] = a;
    Eb[b] = e;
    mu[b] = m;
    if (hist) {
        const int c = *count;
        if (c < cap) hist[(int64_t)c * B + b] = e;
    }
}

__global__ void k_tex_tick(int* count) { if (threadIdx.x == 0) *count += 1; }
__global__ void k_tex_zero(int* count) { if (threadIdx.x == 0) *count = 0; }

// accepted: y_best = y_c, g_best = g_c; then y_c = y_best - mu g_best
__global__ void __launch_bounds__(256) k_tex_update(float* __restrict__ yc, const float* __restrict__ gc,
                                                    float* __restrict__ yb, float* __restrict__ gb, int64_t N,
                                                    const int* __restrict__ acc, const float* __restrict__ mu) {
    const int64_t b = blockIdx.y;
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    const int64_t i = b * N + n;
    float y, g;
    if (acc[b]) {
        y = yc[i];
        g = gc[i];
        yb[i] = y;
        gb[i] = g;
    } else {
        y = yb[i];
        g = gb[i];
    }
    yc[i] = y - mu[b] * g;
}

}  // namespace jtfs

using namespace jtfs;

struct jtfs_texture {
    const jtfs_plan* plan = nullptr;
    jtfs_info info{};
    int64_t B = 0, N = 0, n1 = 0, n2 = 0;
    float mu0 = 0.f;
    void* ws = nullptr;
    size_t ws_bytes = 0;
    float *x1 = nullptr, *x2 = nullptr, *c1 = nullptr, *c2 = nullptr, *g1 = nullptr, *g2 = nullptr;
    float *yc = nullptr, *gc = nullptr, *yb = nullptr, *gb = nullptr;
    float *nx = nullptr, *Ec = nullptr, *Eb = nullptr, *mu = nullptr;
    int *acc = nullptr, *count = nullptr;
    bool have_target = false, have_start = false;
    std::vector<void*> owned;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    const void* key[3] = {nullptr, nullptr, nullptr};
};

static void tex_release(jtfs_texture* t) {
    if (!t) return;
    if (t->exec) (void)hipGraphExecDestroy(t->exec);
    if (t->graph) (void)hipGraphDestroy(t->graph);
    for (void* q : t->owned) (void)hipFree(q);
    delete t;
}

static int tex_status(const char* what) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) { set_error(std::string(what) + ": " + hipGetErrorString(e)); return JTFS_EHIP; }
    return JTFS_OK;
}

// forward of the candidate, residual and cotangent, backward, decision, update
static int tex_evaluate(jtfs_texture* t, int init, float* hist, int cap, hipStream_t st) {
    const unsigned B = (unsigned)t->B;
    int rc = jtfs_forward(t->plan, t->yc, t->B, t->c1, t->c2, t->ws, t->ws_bytes, st);
    if (rc != JTFS_OK) return rc;
    hipLaunchKernelGGL(k_tex_resid, dim3(B), dim3(1024), 0, st, t->c1, t->c2, t->x1, t->x2, t->n1, t->n2, t->nx,
                       t->Ec, t->g1, t->g2);
    rc = jtfs_backward(t->plan, t->yc, t->g1, t->g2, t->gc, t->B, t->ws, t->ws_bytes, JTFS_BWD_REUSE_FORWARD, st);
    if (rc != JTFS_OK) return rc;
    hipLaunchKernelGGL(k_tex_decide, dim3(B), dim3(1024), 0, st, t->yc, t->gc, t->N, t->Ec, t->Eb, t->mu, t->acc,
                       t->mu0, init, hist, t->count, cap, t->B);
    if (hist) hipLaunchKernelGGL(k_tex_tick, dim3(1), dim3(64), 0, st, t->count);
    hipLaunchKernelGGL(k_tex_update, dim3((unsigned)((t->N + 255) / 256), B), dim3(256), 0, st, t->yc, t->gc, t->yb,
                       t->gb, t->N, t->acc, t->mu);
    return tex_status("texture iteration");
}

extern "C" int jtfs_texture_create(jtfs_texture** out, const jtfs_plan* plan, int64_t B, float mu0) {
    if (!out || !plan) { set_error("null pointer"); return JTFS_EINVAL; }
    *out = nullptr;
    if (B < 1 || B > 65535) { set_error("B must lie in [1, 65535]"); return JTFS_ESHAPE; }
    if (!(mu0 != 0.f) || !std::isfinite(mu0)) { set_error("mu0 must be finite and non-zero"); return JTFS_EINVAL; }
    auto* t = new (std::nothrow) jtfs_texture();
    if (!t) { set_error("host allocation failed"); return JTFS_ENOMEM; }
    t->plan = plan;
    jtfs_plan_info(plan, &t->info);
    t->B = B;
    t->N = t->info.NX << t->info.kX;
    t->n1 = t->info.s1_per_signal;
    t->n2 = t->info.s2_per_signal;
    t->mu0 = mu0;
    jtfs_workspace_size(plan, B, &t->ws_bytes);
    bool ok = true;
    auto get = [&](size_t bytes) -> void* {
        void* q = nullptr;
        if (hipMalloc(&q, bytes < 256 ? 256 : bytes) != hipSuccess) { ok = false; return nullptr; }
        t->owned.push_back(q);
        return q;
    };
    t->ws = get(t->ws_bytes);
    const size_t f = sizeof(float);
    t->x1 = (float*)get(f * B * t->n1); t->x2 = (float*)get(f * B * t->n2);
    t->c1 = (float*)get(f * B * t->n1); t->c2 = (float*)get(f * B * t->n2);
    t->g1 = (float*)get(f * B * t->n1); t->g2 = (float*)get(f * B * t->n2);
    t->yc = (float*)get(f * B * t->N); t->gc = (float*)get(f * B * t->N);
    t->yb = (float*)get(f * B * t->N); t->gb = (float*)get(f * B * t->N);
    t->nx = (float*)get(f * B); t->Ec = (float*)get(f * B); t->Eb = (float*)get(f * B); t->mu = (float*)get(f * B);
    t->acc = (int*)get(sizeof(int) * B);
    t->count = (int*)get(sizeof(int));
    if (!ok) { tex_release(t); set_error("device allocation failed"); return JTFS_ENOMEM; }
    *out = t;
    return JTFS_OK;
}

extern "C" int jtfs_texture_set_target(jtfs_texture* t, const float* x, hipStream_t st) {
    if (!t || !x) { set_error("null pointer"); return JTFS_EINVAL; }
    int rc = jtfs_forward(t->plan, x, t->B, t->x1, t->x2, t->ws, t->ws_bytes, st);
    if (rc != JTFS_OK) return rc;
    hipLaunchKernelGGL(k_tex_norm, dim3((unsigned)t->B), dim3(1024), 0, st, t->x1, t->x2, t->n1, t->n2, t->nx);
    rc = tex_status("target norms");
    if (rc == JTFS_OK) t->have_target = true;
    return rc;
}

extern "C" int jtfs_texture_set_start(jtfs_texture* t, const float* y0, hipStream_t st) {
    if (!t || !y0) { set_error("null pointer"); return JTFS_EINVAL; }
    if (!t->have_target) { set_error("set the target first"); return JTFS_EINVAL; }
    if (hipMemcpyAsync(t->yc, y0, sizeof(float) * t->B * t->N, hipMemcpyDeviceToDevice, st) != hipSuccess) {
        set_error("copy of the start failed"); return JTFS_EHIP; }
    hipLaunchKernelGGL(k_tex_zero, dim3(1), dim3(64), 0, st, t->count);
    const int rc = tex_evaluate(t, 1, nullptr, 0, st);
    if (rc == JTFS_OK) t->have_start = true;
    return rc;
}

extern "C" int jtfs_texture_iterate(jtfs_texture* t, int iters, float* hist, int hist_cap, hipStream_t st) {
    if (!t) { set_error("null texture"); return JTFS_EINVAL; }
    if (!t->have_start) { set_error("set the start first"); return JTFS_EINVAL; }
    if (iters < 0 || (hist && hist_cap < 1)) { set_error("invalid iteration count or history capacity"); return JTFS_EINVAL; }
    if (iters == 0) return JTFS_OK;
    // the graph bakes in the history pointer, its capacity and the stream
    const void* key[3] = {hist, st, (const void*)(intptr_t)(hist ? hist_cap : 0)};
    if (!(t->exec && key[0] == t->key[0] && key[1] == t->key[1] && key[2] == t->key[2])) {
        if (t->exec) { (void)hipGraphExecDestroy(t->exec); t->exec = nullptr; }
        if (t->graph) { (void)hipGraphDestroy(t->graph); t->graph = nullptr; }
        if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) {
            set_error("hipStreamBeginCapture failed (the stream must not be the legacy null stream)");
            return JTFS_EHIP;
        }
        const int rc = tex_evaluate(t, 0, hist, hist_cap, st);
        hipGraph_t g = nullptr;
        const hipError_t ec = hipStreamEndCapture(st, &g);
        if (rc != JTFS_OK) { if (g) (void)hipGraphDestroy(g); return rc; }
        if (ec != hipSuccess || !g) { set_error("hipStreamEndCapture failed"); return JTFS_EHIP; }
        t->graph = g;
        if (hipGraphInstantiate(&t->exec, g, nullptr, nullptr, 0) != hipSuccess) {
            set_error("hipGraphInstantiate failed"); return JTFS_EHIP; }
        t->key[0] = key[0];
        t->key[1] = key[1];
        t->key[2] = key[2];
    }
    if (hist) hipLaunchKernelGGL(k_tex_zero, dim3(1), dim3(64), 0, st, t->count);
    for (int i = 0; i < iters; ++i)
        if (hipGraphLaunch(t->exec, st) != hipSuccess) { set_error("hipGraphLaunch failed"); return JTFS_EHIP; }
    return tex_status("texture iterations");
}

extern "C" int jtfs_texture_read(const jtfs_texture* t, float* y, float* err, float* mu, hipStream_t st) {
    if (!t) { set_error("null texture"); return JTFS_EINVAL; }
    if (!t->have_start) { set_error("set the start first"); return JTFS_EINVAL; }
    const auto cp = [&](void* d, const void* s, size_t n) {
        return !d || hipMemcpyAsync(d, s, n, hipMemcpyDeviceToDevice, st) == hipSuccess;
    };
    if (!cp(y, t->yb, sizeof(float) * t->B * t->N) || !cp(err, t->Eb, sizeof(float) * t->B) ||
        !cp(mu, t->mu, sizeof(float) * t->B)) {
        set_error("copy failed"); return JTFS_EHIP; }
    return JTFS_OK;
}

extern "C" void jtfs_texture_destroy(jtfs_texture* t) { tex_release(t); }
