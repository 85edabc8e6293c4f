// Ragged batches: signals bucketed by padded power-of-two length, one plan and
// workspace per bucket, pack / forward / backward / unpack recorded once as a HIP
// graph and replayed.  Each bucket's work is recorded on a stream of its own,
// forked from and joined back to the caller's stream, so that the graph holds
// one independent branch per bucket and the buckets' launches can overlap (the
// short launches of one bucket's low temporal rates fill the GPU with another's).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <new>
#include <vector>

#include "plan.hpp"

namespace jtfs {

// xb[j][n] = x_packed[xoff[j] + n] for n < len[j], 0 up to N
__global__ void k_pack(const float* __restrict__ xp, const int64_t* __restrict__ xoff, const int64_t* __restrict__ len,
                       int64_t N, float* __restrict__ xb) {
    const int j = blockIdx.y;
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    xb[(int64_t)j * N + n] = n < len[j] ? xp[xoff[j] + n] : 0.f;
}

// Copies `per` floats of each signal j between a bucket array [B][per] (at column
// `col` of a row of `row` floats) and the packed array at soff[j] + col.
__global__ void k_copy_rows(const float* __restrict__ src, float* __restrict__ dst, const int64_t* __restrict__ soff,
                            int64_t per, int64_t row, int64_t col, int to_packed) {
    const int j = blockIdx.y;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= per) return;
    if (to_packed) dst[soff[j] + col + e] = src[(int64_t)j * row + e];
    else dst[(int64_t)j * row + e] = src[soff[j] + col + e];
}

// gx_packed[xoff[j] + n] = gxb[j][n] for n < len[j]
__global__ void k_unpack_grad(const float* __restrict__ gxb, const int64_t* __restrict__ xoff,
                              const int64_t* __restrict__ len, int64_t N, float* __restrict__ gxp) {
    const int j = blockIdx.y;
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= len[j]) return;
    gxp[xoff[j] + n] = gxb[(int64_t)j * N + n];
}

}  // namespace jtfs

using namespace jtfs;

struct Bucket {
    int64_t N = 0;
    std::vector<int> members;           // signal indices
    jtfs_plan* plan = nullptr;
    jtfs_info info{};
    void* ws = nullptr;
    size_t ws_bytes = 0;
    hipStream_t stream = nullptr;             // the bucket's branch while the graph is recorded
    hipEvent_t done = nullptr;
    int mode_plain = JTFS_CONTRACTION_FP32;   // the plan's own contraction (forward-only runs)
    bool phase = false;                       // runs with a gradient store the phase
    float *xb = nullptr, *s1 = nullptr, *s2 = nullptr, *g1 = nullptr, *g2 = nullptr, *gxb = nullptr;
    int64_t *d_xoff = nullptr, *d_len = nullptr, *d_soff = nullptr;
};

struct jtfs_bucket {
    jtfs_params p{};
    std::vector<int64_t> lengths, xoff, soff;
    std::vector<Bucket> buckets;
    std::vector<void*> owned;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t fork = nullptr;
    const void* key[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
};

static void release(jtfs_bucket* bk) {
    if (!bk) return;
    if (bk->exec) (void)hipGraphExecDestroy(bk->exec);
    if (bk->graph) (void)hipGraphDestroy(bk->graph);
    if (bk->fork) (void)hipEventDestroy(bk->fork);
    for (auto& b : bk->buckets) {
        if (b.plan) jtfs_plan_destroy(b.plan);
        if (b.stream) (void)hipStreamDestroy(b.stream);
        if (b.done) (void)hipEventDestroy(b.done);
    }
    for (void* q : bk->owned) (void)hipFree(q);
    delete bk;
}

extern "C" int jtfs_bucket_create(jtfs_bucket** out, const int64_t* lengths, int count, const jtfs_params* p) {
    if (!out || !lengths || !p || count < 1) { set_error("invalid arguments"); return JTFS_EINVAL; }
    *out = nullptr;
    auto* bk = new (std::nothrow) jtfs_bucket();
    if (!bk) { set_error("host allocation failed"); return JTFS_ENOMEM; }
    bk->p = *p;
    const bool tune = (p->flags & JTFS_BUCKET_AUTOTUNE) != 0;
    bk->p.flags &= ~JTFS_BUCKET_AUTOTUNE;           // the plans' own flags
    std::map<int64_t, std::vector<int>> groups;
    for (int i = 0; i < count; ++i) {
        if (lengths[i] < 16 || lengths[i] > (int64_t(1) << 24)) { release(bk); set_error("length out of range"); return JTFS_EINVAL; }
        int64_t N = 16;
        while (N < lengths[i]) N <<= 1;
        groups[N].push_back(i);
        bk->lengths.push_back(lengths[i]);
    }
    bk->xoff.resize(count + 1);
    bk->xoff[0] = 0;
    for (int i = 0; i < count; ++i) bk->xoff[i + 1] = bk->xoff[i] + lengths[i];
    std::vector<int64_t> s_per(count);
    for (auto& kv : groups) {
        Bucket b;
        b.N = kv.first;
        b.members = kv.second;
        jtfs_params q = bk->p;
        q.N = b.N;
        int st = jtfs_plan_create_ex(&b.plan, &q);
        if (st != JTFS_OK) { release(bk); return st; }
        bk->buckets.push_back(b);
        Bucket& bb = bk->buckets.back();
        if (tune) {
            // launch choices for this bucket's batch; the contraction of each run is
            // chosen below (the stored phase when a gradient is asked for)
            jtfs_tuning t;
            st = jtfs_plan_autotune(bb.plan, nullptr, (int64_t)bb.members.size(), 2, nullptr, &t);
            int mode = 0, mask = 0;
            if (st == JTFS_OK) st = jtfs_plan_get_tuning(bb.plan, &mode, &mask);
            if (st == JTFS_OK)
                st = jtfs_plan_set_tuning(bb.plan, bb.plan->split_ok ? JTFS_CONTRACTION_SPLIT_F16 : JTFS_CONTRACTION_FP32,
                                          mask);
            if (st != JTFS_OK) { release(bk); return st; }
        }
        jtfs_plan_info(bb.plan, &bb.info);
        for (int i : bb.members) s_per[i] = bb.info.s1_per_signal + bb.info.s2_per_signal;
    }
    bk->soff.resize(count + 1);
    bk->soff[0] = 0;
    for (int i = 0; i < count; ++i) bk->soff[i + 1] = bk->soff[i] + s_per[i];
    // Runs with a gradient use the split-FP16 contraction with the phase stored by
    // the forward (the backward reuses the forward's workspace) where every
    // bucket's plan allows it and the larger workspaces fit in 80 % of the free
    // device memory; forward-only runs keep each plan's own contraction.
    {
        bool all = true;
        size_t need = 0;
        for (auto& b : bk->buckets) jtfs_plan_get_contraction(b.plan, &b.mode_plain);
        for (auto& b : bk->buckets) {
            const int64_t B = (int64_t)b.members.size();
            all = all && b.plan->split_ok && b.plan->split_bwdp_ok && !b.plan->s.tscat;
            if (!all) break;
            b.plan->contraction = JTFS_CONTRACTION_SPLIT_F16_PHASE;
            size_t w = 0;
            jtfs_workspace_size(b.plan, B, &w);
            b.plan->contraction = b.mode_plain;
            need += w + sizeof(float) * B * (2 * b.N + 2 * (b.info.s1_per_signal + b.info.s2_per_signal));
        }
        size_t free_b = 0, total_b = 0;
        const bool fits = all && hipMemGetInfo(&free_b, &total_b) == hipSuccess && (double)need <= 0.8 * (double)free_b;
        for (auto& b : bk->buckets) b.phase = fits;
    }
    // per-bucket device buffers (the workspace sized for the contraction with a gradient)
    for (auto& b : bk->buckets) {
        const int64_t B = (int64_t)b.members.size();
        size_t wsb = 0;
        if (b.phase) b.plan->contraction = JTFS_CONTRACTION_SPLIT_F16_PHASE;
        jtfs_workspace_size(b.plan, B, &wsb);
        b.plan->contraction = b.mode_plain;
        auto get = [&](size_t bytes) -> void* {
            void* q = nullptr;
            if (hipMalloc(&q, std::max<size_t>(bytes, 16)) != hipSuccess) return nullptr;
            bk->owned.push_back(q);
            return q;
        };
        b.ws = get(wsb);
        b.ws_bytes = wsb;
        b.xb = (float*)get(sizeof(float) * B * b.N);
        b.gxb = (float*)get(sizeof(float) * B * b.N);
        b.s1 = (float*)get(sizeof(float) * B * b.info.s1_per_signal);
        b.s2 = (float*)get(sizeof(float) * B * b.info.s2_per_signal);
        b.g1 = (float*)get(sizeof(float) * B * b.info.s1_per_signal);
        b.g2 = (float*)get(sizeof(float) * B * b.info.s2_per_signal);
        std::vector<int64_t> xo(B), ln(B), so(B);
        for (int64_t j = 0; j < B; ++j) {
            xo[j] = bk->xoff[b.members[j]];
            ln[j] = bk->lengths[b.members[j]];
            so[j] = bk->soff[b.members[j]];
        }
        b.d_xoff = (int64_t*)get(sizeof(int64_t) * B);
        b.d_len = (int64_t*)get(sizeof(int64_t) * B);
        b.d_soff = (int64_t*)get(sizeof(int64_t) * B);
        if (!b.ws || !b.xb || !b.gxb || !b.s1 || !b.s2 || !b.g1 || !b.g2 || !b.d_xoff || !b.d_len || !b.d_soff) {
            release(bk); set_error("device allocation failed"); return JTFS_ENOMEM;
        }
        if (hipMemcpy(b.d_xoff, xo.data(), sizeof(int64_t) * B, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(b.d_len, ln.data(), sizeof(int64_t) * B, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(b.d_soff, so.data(), sizeof(int64_t) * B, hipMemcpyHostToDevice) != hipSuccess) {
            release(bk); set_error("upload failed"); return JTFS_EHIP;
        }
        // the branch's stream (default priority) and its join event
        if (hipStreamCreateWithFlags(&b.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&b.done, hipEventDisableTiming) != hipSuccess) {
            release(bk); set_error("stream or event creation failed"); return JTFS_EHIP;
        }
    }
    if (hipEventCreateWithFlags(&bk->fork, hipEventDisableTiming) != hipSuccess) {
        release(bk); set_error("event creation failed"); return JTFS_EHIP;
    }
    *out = bk;
    return JTFS_OK;
}

extern "C" int jtfs_bucket_offsets(const jtfs_bucket* bk, int64_t* x_offset, int64_t* s_offset) {
    if (!bk) { set_error("null bucket"); return JTFS_EINVAL; }
    if (x_offset) std::memcpy(x_offset, bk->xoff.data(), sizeof(int64_t) * bk->xoff.size());
    if (s_offset) std::memcpy(s_offset, bk->soff.data(), sizeof(int64_t) * bk->soff.size());
    return JTFS_OK;
}

// Records every bucket's work on its own stream, forked from st and joined back
// (called while st is being captured: the branches become parallel in the graph).
static int enqueue(jtfs_bucket* bk, const float* xp, float* sp, const float* gp, float* gxp, hipStream_t st0) {
    if (hipEventRecord(bk->fork, st0) != hipSuccess) { set_error("fork event failed"); return JTFS_EHIP; }
    for (auto& b : bk->buckets) {
        const hipStream_t st = b.stream;
        if (hipStreamWaitEvent(st, bk->fork, 0) != hipSuccess) { set_error("fork wait failed"); return JTFS_EHIP; }
        const unsigned B = (unsigned)b.members.size();
        const int64_t s1n = b.info.s1_per_signal, s2n = b.info.s2_per_signal, row = s1n + s2n;
        hipLaunchKernelGGL(k_pack, dim3((unsigned)((b.N + 255) / 256), B), dim3(256), 0, st, xp, b.d_xoff, b.d_len,
                           b.N, b.xb);
        // the contraction is fixed when the work is recorded
        b.plan->contraction = (gp && gxp && b.phase) ? JTFS_CONTRACTION_SPLIT_F16_PHASE : b.mode_plain;
        int rc = jtfs_forward(b.plan, b.xb, B, b.s1, b.s2, b.ws, b.ws_bytes, st);
        if (rc != JTFS_OK) return rc;
        hipLaunchKernelGGL(k_copy_rows, dim3((unsigned)((s1n + 255) / 256), B), dim3(256), 0, st, b.s1, sp, b.d_soff,
                           s1n, s1n, (int64_t)0, 1);
        hipLaunchKernelGGL(k_copy_rows, dim3((unsigned)((s2n + 255) / 256), B), dim3(256), 0, st, b.s2, sp, b.d_soff,
                           s2n, s2n, s1n, 1);
        if (gp && gxp) {
            hipLaunchKernelGGL(k_copy_rows, dim3((unsigned)((s1n + 255) / 256), B), dim3(256), 0, st, gp, b.g1,
                               b.d_soff, s1n, s1n, (int64_t)0, 0);
            hipLaunchKernelGGL(k_copy_rows, dim3((unsigned)((s2n + 255) / 256), B), dim3(256), 0, st, gp, b.g2,
                               b.d_soff, s2n, s2n, s1n, 0);
            rc = jtfs_backward(b.plan, b.xb, b.g1, b.g2, b.gxb, B, b.ws, b.ws_bytes, JTFS_BWD_REUSE_FORWARD, st);
            if (rc != JTFS_OK) return rc;
            hipLaunchKernelGGL(k_unpack_grad, dim3((unsigned)((b.N + 255) / 256), B), dim3(256), 0, st, b.gxb,
                               b.d_xoff, b.d_len, b.N, gxp);
        }
        (void)row;
        if (hipGetLastError() != hipSuccess) { set_error("bucket kernel launch failed"); return JTFS_EHIP; }
        if (hipEventRecord(b.done, st) != hipSuccess || hipStreamWaitEvent(st0, b.done, 0) != hipSuccess) {
            set_error("join failed"); return JTFS_EHIP; }
    }
    return JTFS_OK;
}

extern "C" int jtfs_bucket_run(jtfs_bucket* bk, const float* xp, float* sp, const float* gp, float* gxp,
                               hipStream_t st) {
    if (!bk || !xp || !sp) { set_error("null pointer"); return JTFS_EINVAL; }
    if ((gp == nullptr) != (gxp == nullptr)) { set_error("g_packed and gx_packed go together"); return JTFS_EINVAL; }
    const void* key[5] = {xp, sp, gp, gxp, st};
    const bool same = bk->exec && std::equal(key, key + 5, bk->key);
    if (!same) {
        if (bk->exec) { (void)hipGraphExecDestroy(bk->exec); bk->exec = nullptr; }
        if (bk->graph) { (void)hipGraphDestroy(bk->graph); bk->graph = nullptr; }
        if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) {
            set_error("hipStreamBeginCapture failed (the stream must not be the legacy null stream)");
            return JTFS_EHIP;
        }
        const int rc = enqueue(bk, xp, sp, gp, gxp, st);
        hipGraph_t g = nullptr;
        const hipError_t ec = hipStreamEndCapture(st, &g);
        if (rc != JTFS_OK) { if (g) (void)hipGraphDestroy(g); return rc; }
        if (ec != hipSuccess || !g) { set_error("hipStreamEndCapture failed"); return JTFS_EHIP; }
        bk->graph = g;
        if (hipGraphInstantiate(&bk->exec, g, nullptr, nullptr, 0) != hipSuccess) {
            set_error("hipGraphInstantiate failed"); return JTFS_EHIP; }
        std::copy(key, key + 5, bk->key);
    }
    if (hipGraphLaunch(bk->exec, st) != hipSuccess) { set_error("hipGraphLaunch failed"); return JTFS_EHIP; }
    return JTFS_OK;
}

extern "C" void jtfs_bucket_destroy(jtfs_bucket* bk) { release(bk); }
