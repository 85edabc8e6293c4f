// Autotuning of a plan's launch choices on the caller's GPU and batch size.
//
// Candidates: the contraction arithmetic (split FP16, split FP16 with the phase
// stored by the forward, or FP32 matrix cores); the tile of the split forward
// contraction (32 x 32 or 16 x 16 MFMA tiles); and, for rows of 2^14 points, the
// register-resident or the in-LDS transform in each of the four stages that have
// both (scalogram, second order, gY2 row FFTs, first-order adjoint).  Every
// candidate runs whole fwd+bwd steps; the per-stage HIP-event timers attribute
// the time, so these binary choices are settled from two runs per contraction
// mode (all register-resident with 32 x 32 tiles, all in LDS with 16 x 16 tiles)
// rather than from thirty-two.  For the chosen mode, one more run each settles
// the largest radix of the register-resident transforms' passes (16 or 8, per
// stage), the points per workgroup of the in-LDS row transforms (4096 or
// 8192, i.e. how many workgroups share a CU's LDS) and the forward contraction's
// t-chunk (1024 or 4096 columns per workgroup).  Results can be kept in a
// text file keyed by the device and the plan's shape (JTFS_TUNE_CACHE).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "plan.hpp"
#include "split.hpp"

namespace jtfs {
bool timing_on();
}
using namespace jtfs;

namespace {

struct DevBuf {
    void* p = nullptr;
    ~DevBuf() { if (p) (void)hipFree(p); }
    bool alloc(size_t n) { return hipMalloc(&p, std::max<size_t>(n, 256)) == hipSuccess; }
};

void set_rows(jtfs_plan* P, int mask) {
    P->tune.reg_scalogram = (mask & JTFS_REG_SCALOGRAM) != 0;
    P->tune.reg_second = (mask & JTFS_REG_SECOND_ORDER) != 0;
    P->tune.reg_rowfft = (mask & JTFS_REG_ROW_FFT) != 0;
    P->tune.reg_first_adj = (mask & JTFS_REG_FIRST_ADJ) != 0;
    P->tune.fwd16 = (mask & JTFS_TUNE_FWD_TILE16) != 0;
    P->tune.bwd16 = (mask & JTFS_TUNE_BWD_TILE16) != 0;
    P->tune.r8_scalogram = (mask & JTFS_TUNE_RADIX8_SCALOGRAM) != 0;
    P->tune.r8_second = (mask & JTFS_TUNE_RADIX8_SECOND_ORDER) != 0;
    P->tune.r8_rowfft = (mask & JTFS_TUNE_RADIX8_ROW_FFT) != 0;
    P->tune.r8_first_adj = (mask & JTFS_TUNE_RADIX8_FIRST_ADJ) != 0;
    P->tune.batch8k = (mask & JTFS_TUNE_LDS_BATCH8K) != 0;
    const int chunk = (mask & JTFS_TUNE_TCHUNK_1K) ? 1024 : (mask & JTFS_TUNE_TCHUNK_2K) ? 2048 : kChunkT;
    if (chunk != P->tune.chunk) {
        // the partial-V slot tables of the shapes and their device copies
        P->tune.chunk = chunk;
        set_chunks(&P->s, chunk);
        (void)hipMemcpy(P->d_vchoff, P->s.vchoff.data(), sizeof(int64_t) * P->s.n_alpha, hipMemcpyHostToDevice);
        (void)hipMemcpy(P->d_nch, P->s.nch.data(), sizeof(int) * P->s.n_alpha, hipMemcpyHostToDevice);
    }
}

constexpr int kRadix8Bits = JTFS_TUNE_RADIX8_SCALOGRAM | JTFS_TUNE_RADIX8_SECOND_ORDER | JTFS_TUNE_RADIX8_ROW_FFT |
                            JTFS_TUNE_RADIX8_FIRST_ADJ;

int get_rows(const jtfs_plan* P) {
    return (P->tune.reg_scalogram ? JTFS_REG_SCALOGRAM : 0) | (P->tune.reg_second ? JTFS_REG_SECOND_ORDER : 0) |
           (P->tune.reg_rowfft ? JTFS_REG_ROW_FFT : 0) | (P->tune.reg_first_adj ? JTFS_REG_FIRST_ADJ : 0) |
           (P->tune.fwd16 ? JTFS_TUNE_FWD_TILE16 : 0) | (P->tune.bwd16 ? JTFS_TUNE_BWD_TILE16 : 0) |
           (P->tune.r8_scalogram ? JTFS_TUNE_RADIX8_SCALOGRAM : 0) |
           (P->tune.r8_second ? JTFS_TUNE_RADIX8_SECOND_ORDER : 0) | (P->tune.r8_rowfft ? JTFS_TUNE_RADIX8_ROW_FFT : 0) |
           (P->tune.r8_first_adj ? JTFS_TUNE_RADIX8_FIRST_ADJ : 0) | (P->tune.batch8k ? JTFS_TUNE_LDS_BATCH8K : 0) |
           (P->tune.chunk == 1024 ? JTFS_TUNE_TCHUNK_1K : P->tune.chunk == 2048 ? JTFS_TUNE_TCHUNK_2K : 0);
}

// Cache key: the device's architecture and name, the plan parameters and B.
std::string cache_key(const jtfs_plan* P, int64_t B) {
    hipDeviceProp_t prop;
    std::string dev = "unknown";
    if (hipGetDeviceProperties(&prop, P->device) == hipSuccess) dev = std::string(prop.gcnArchName) + "/" + prop.name;
    for (char& c : dev)
        if (c == ' ' || c == '\t') c = '_';
    const jtfs_params& p = P->s.p;
    char buf[256];
    std::snprintf(buf, sizeof buf, "N=%lld,J=%d,Q=%d/%d,Jfr=%d,Qfr=%d,T=%lld,F=%lld,flags=%u,B=%lld", (long long)p.N,
                  p.J, p.Q1, p.Q2, p.J_fr, p.Q_fr, (long long)p.T, (long long)p.F, p.flags, (long long)B);
    return dev + "|" + buf;
}

const char* cache_path() {
    const char* f = std::getenv("JTFS_TUNE_CACHE");
    return f && *f ? f : nullptr;
}

// the last entry for key in the cache file: contraction, choice mask, step ms
bool cache_lookup(const std::string& key, int* mode, int* mask, double* ms) {
    const char* path = cache_path();
    if (!path) return false;
    FILE* f = std::fopen(path, "r");
    if (!f) return false;
    char line[512];
    bool found = false;
    while (std::fgets(line, sizeof line, f)) {
        char k[400];
        int m = 0, r = 0;
        double t = 0.0;
        if (std::sscanf(line, "%399s %d %d %lf", k, &m, &r, &t) == 4 && key == k) {
            *mode = m; *mask = r; *ms = t;
            found = true;
        }
    }
    std::fclose(f);
    return found;
}

void cache_store(const std::string& key, int mode, int mask, double ms) {
    const char* path = cache_path();
    if (!path) return;
    FILE* f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "%s %d %d %.4f\n", key.c_str(), mode, mask, ms);
    std::fclose(f);
}

// reps timed fwd+bwd steps after one untimed one: total ms per step and ms per stage per step
int run_steps(jtfs_plan* P, const float* x, int64_t B, float* s1, float* s2, float* gx, void* ws, size_t wsb,
              int reps, hipStream_t st, double* step_ms, double* stage_ms) {
    auto step = [&]() -> int {
        int rc = jtfs_forward(P, x, B, s1, s2, ws, wsb, st);
        if (rc != JTFS_OK) return rc;
        return jtfs_backward(P, x, s1, s2, gx, B, ws, wsb, JTFS_BWD_REUSE_FORWARD, st);
    };
    int rc = step();
    if (rc != JTFS_OK) return rc;
    if (hipStreamSynchronize(st) != hipSuccess) { set_error("autotune: stream synchronisation failed"); return JTFS_EHIP; }
    double ms = 0.0;
    int64_t n = 0;
    for (int k = 0; k < JTFS_NUM_STAGES; ++k) jtfs_timing_read(k, &ms, &n);       // clear
    jtfs_timing_enable(1);
    hipEvent_t a = nullptr, b = nullptr;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
        jtfs_timing_enable(0);
        set_error("autotune: event creation failed");
        return JTFS_EHIP;
    }
    (void)hipEventRecord(a, st);
    for (int r = 0; r < reps && rc == JTFS_OK; ++r) rc = step();
    (void)hipEventRecord(b, st);
    const hipError_t es = hipEventSynchronize(b);
    jtfs_timing_enable(0);
    float total = 0.f;
    if (rc == JTFS_OK && es == hipSuccess) (void)hipEventElapsedTime(&total, a, b);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (rc != JTFS_OK) return rc;
    if (es != hipSuccess) { set_error("autotune: event synchronisation failed"); return JTFS_EHIP; }
    *step_ms = total / reps;
    for (int k = 0; k < JTFS_NUM_STAGES; ++k) {
        jtfs_timing_read(k, &ms, &n);
        stage_ms[k] = ms / reps;
    }
    return JTFS_OK;
}

}  // namespace

extern "C" int jtfs_plan_set_tuning(jtfs_plan* P, int contraction, int reg_rows) {
    if (!P) { set_error("null plan"); return JTFS_EINVAL; }
    if (reg_rows & ~(JTFS_REG_SCALOGRAM | JTFS_REG_SECOND_ORDER | JTFS_REG_ROW_FFT | JTFS_REG_FIRST_ADJ |
                     JTFS_TUNE_FWD_TILE16 | JTFS_TUNE_BWD_TILE16 | kRadix8Bits | JTFS_TUNE_LDS_BATCH8K |
                     JTFS_TUNE_TCHUNK_1K | JTFS_TUNE_TCHUNK_2K)) {
        set_error("unknown row-kernel bits"); return JTFS_EINVAL; }
    const int rc = jtfs_plan_set_contraction(P, contraction);
    if (rc != JTFS_OK) return rc;
    set_rows(P, reg_rows);
    return JTFS_OK;
}

extern "C" int jtfs_plan_get_tuning(const jtfs_plan* P, int* contraction, int* reg_rows) {
    if (!P || !contraction || !reg_rows) { set_error("null pointer"); return JTFS_EINVAL; }
    *contraction = P->contraction;
    *reg_rows = get_rows(P);
    return JTFS_OK;
}

extern "C" int jtfs_plan_autotune(jtfs_plan* P, const float* x, int64_t B, int reps, hipStream_t st,
                                  jtfs_tuning* out) {
    if (!P || !out) { set_error("null pointer"); return JTFS_EINVAL; }
    if (B < 1 || B > 65535) { set_error("B must lie in [1, 65535]"); return JTFS_ESHAPE; }
    if (reps < 1 || reps > 100) { set_error("reps must lie in [1, 100]"); return JTFS_EINVAL; }
    if (timing_on()) { set_error("autotune uses the stage timers: disable jtfs timing first"); return JTFS_EINVAL; }
    std::memset(out, 0, sizeof(*out));
    const Shapes& s = P->s;
    const int saved_mode = P->contraction, saved_rows = get_rows(P);
    const std::string key = cache_key(P, B);
    {
        int cm = 0, cr = 0;
        double cms = 0.0;
        if (cache_lookup(key, &cm, &cr, &cms) && jtfs_plan_set_tuning(P, cm, cr) == JTFS_OK) {
            out->contraction = cm;
            out->reg_rows = cr;
            out->step_ms = cms;
            out->from_cache = 1;
            return JTFS_OK;
        }
        P->contraction = saved_mode;
        set_rows(P, saved_rows);
    }
    // candidates
    std::vector<int> modes;
    if (P->split_ok) modes.push_back(JTFS_CONTRACTION_SPLIT_F16);
    modes.push_back(JTFS_CONTRACTION_FP32);
    jtfs_info info;
    jtfs_plan_info(P, &info);
    const size_t coef_bytes = sizeof(float) * B * (info.s1_per_signal + info.s2_per_signal + 2 * s.N);
    if (P->split_ok && P->split_bwdp_ok && !s.tscat) {
        // the stored phase only where the whole candidate set fits in 80 % of free memory
        P->contraction = JTFS_CONTRACTION_SPLIT_F16_PHASE;
        size_t b = 0;
        jtfs_workspace_size(P, B, &b);
        size_t free_b = 0, total_b = 0;
        if (hipMemGetInfo(&free_b, &total_b) == hipSuccess && (double)(b + coef_bytes) <= 0.8 * (double)free_b)
            modes.push_back(JTFS_CONTRACTION_SPLIT_F16_PHASE);
        P->contraction = saved_mode;
    }
    bool has14 = s.logNX == kRegMinLogRows;
    // (2^11- to 2^13-point rows of the second order and row FFT stages follow the same choice)
    for (int a = 0; a < s.n_alpha_psi; ++a)
        has14 = has14 || (s.logNX - s.k2[a] <= kRegMinLogRows && s.logNX - s.k2[a] >= kRegMinLogRows - 3);
    const int all_rows = JTFS_REG_SCALOGRAM | JTFS_REG_SECOND_ORDER | JTFS_REG_ROW_FFT | JTFS_REG_FIRST_ADJ;
    // second run: rows in LDS and the 16 x 16 contraction tiles, where any of these choices exists
    const bool tile16 = P->split_ok && !s.tscat && fwdq_supported(P, false);
    const bool btile16 = P->split_ok && P->split_bwdp_ok && !s.tscat && bwdq_supported(P);
    std::vector<int> row_opts{all_rows};
    if (has14 || tile16 || btile16)
        row_opts.push_back((has14 ? 0 : all_rows) | (tile16 ? JTFS_TUNE_FWD_TILE16 : 0) |
                           (btile16 ? JTFS_TUNE_BWD_TILE16 : 0));
    // buffers: the largest workspace over the modes (at the shortest t-chunk, whose
    // partial V is largest); the coefficients double as cotangents
    size_t wsb = 0;
    set_rows(P, saved_rows | JTFS_TUNE_TCHUNK_1K);
    for (int m : modes) {
        P->contraction = m;
        size_t b = 0;
        jtfs_workspace_size(P, B, &b);
        wsb = std::max(wsb, b);
    }
    set_rows(P, saved_rows);
    DevBuf ws, s1, s2, gx, xz;
    if (!ws.alloc(wsb) || !s1.alloc(sizeof(float) * B * info.s1_per_signal) ||
        !s2.alloc(sizeof(float) * B * info.s2_per_signal) || !gx.alloc(sizeof(float) * B * s.N)) {
        P->contraction = saved_mode;
        set_error("autotune: device allocation failed");
        return JTFS_ENOMEM;
    }
    if (!x) {
        if (!xz.alloc(sizeof(float) * B * s.N) || hipMemsetAsync(xz.p, 0, sizeof(float) * B * s.N, st) != hipSuccess) {
            P->contraction = saved_mode;
            set_error("autotune: device allocation failed");
            return JTFS_ENOMEM;
        }
        x = (const float*)xz.p;
    }
    // measure
    double stage[3][2][JTFS_NUM_STAGES] = {};
    double total[3][2] = {};
    for (size_t mi = 0; mi < modes.size(); ++mi) {
        for (size_t ri = 0; ri < row_opts.size(); ++ri) {
            P->contraction = modes[mi];
            set_rows(P, row_opts[ri]);
            const int rc = run_steps(P, x, B, (float*)s1.p, (float*)s2.p, (float*)gx.p, ws.p, wsb, reps, st,
                                     &total[mi][ri], stage[mi][ri]);
            if (rc != JTFS_OK) {
                P->contraction = saved_mode;
                set_rows(P, saved_rows);
                return rc;
            }
            const int slot = (modes[mi] == JTFS_CONTRACTION_FP32             ? 2
                              : modes[mi] == JTFS_CONTRACTION_SPLIT_F16_PHASE ? 4
                                                                              : 0) +
                             (int)ri;
            out->candidates_ms[slot] = total[mi][ri];
        }
    }
    // contraction: the stages it owns (each contraction kernel with the faster of its tiles)
    const int cstages[] = {JTFS_STAGE_OPERAND_SPLIT, JTFS_STAGE_FREQ_LOWPASS, JTFS_STAGE_LOWPASS_ADJ,
                           JTFS_STAGE_FREQ_ADJ_WH};
    auto fwd_ms = [&](size_t mi, size_t ri) { return stage[mi][ri][JTFS_STAGE_FREQ_FWD]; };
    auto bwd_ms = [&](size_t mi, size_t ri) { return stage[mi][ri][JTFS_STAGE_FREQ_ADJ_PQ]; };
    auto tile_ok = [&](size_t mi) {
        return tile16 && row_opts.size() == 2 && modes[mi] != JTFS_CONTRACTION_FP32 &&
               fwdq_supported(P, modes[mi] == JTFS_CONTRACTION_SPLIT_F16_PHASE);
    };
    auto btile_ok = [&](size_t mi) {
        return btile16 && row_opts.size() == 2 && modes[mi] == JTFS_CONTRACTION_SPLIT_F16_PHASE;
    };
    size_t best_m = 0;
    double best_c = 1e300;
    for (size_t mi = 0; mi < modes.size(); ++mi) {
        double c = tile_ok(mi) ? std::min(fwd_ms(mi, 0), fwd_ms(mi, 1)) : fwd_ms(mi, 0);
        c += btile_ok(mi) ? std::min(bwd_ms(mi, 0), bwd_ms(mi, 1)) : bwd_ms(mi, 0);
        for (int k : cstages) c += stage[mi][0][k];
        if (c < best_c) { best_c = c; best_m = mi; }
    }
    const bool use16 = tile_ok(best_m) && fwd_ms(best_m, 1) < fwd_ms(best_m, 0);
    const bool buse16 = btile_ok(best_m) && bwd_ms(best_m, 1) < bwd_ms(best_m, 0);
    out->fwd_ms[0] = fwd_ms(best_m, 0);
    out->fwd_ms[1] = tile_ok(best_m) ? fwd_ms(best_m, 1) : 0.0;
    out->bwd_ms[0] = bwd_ms(best_m, 0);
    out->bwd_ms[1] = btile_ok(best_m) ? bwd_ms(best_m, 1) : 0.0;
    // rows of 2^14 points: per stage, the faster of the two runs of the chosen mode
    int rows = all_rows;
    if (has14) {
        const int kstage[4] = {JTFS_STAGE_SCALOGRAM, JTFS_STAGE_SECOND_ORDER, JTFS_STAGE_SECOND_ADJ_FFT,
                               JTFS_STAGE_FIRST_ADJ};
        const int kbit[4] = {JTFS_REG_SCALOGRAM, JTFS_REG_SECOND_ORDER, JTFS_REG_ROW_FFT, JTFS_REG_FIRST_ADJ};
        rows = 0;
        for (int q = 0; q < 4; ++q) {
            // the first-order adjoint's bit also chooses the kernel of the second-order adjoint
            const double r0 = stage[best_m][0][kstage[q]] + (q == 3 ? stage[best_m][0][JTFS_STAGE_SECOND_ADJ] : 0.0);
            const double r1 = stage[best_m][1][kstage[q]] + (q == 3 ? stage[best_m][1][JTFS_STAGE_SECOND_ADJ] : 0.0);
            if (r0 <= r1) rows |= kbit[q];
        }
    }
    if (use16) rows |= JTFS_TUNE_FWD_TILE16;
    if (buse16) rows |= JTFS_TUNE_BWD_TILE16;
    P->contraction = modes[best_m];
    set_rows(P, rows);
    auto fail = [&](int rc) {
        P->contraction = saved_mode;
        set_rows(P, saved_rows);
        return rc;
    };
    // radix of the register-resident passes and points per in-LDS workgroup: one
    // run each against the choice so far, settled per stage
    bool has_long = s.logNX >= kRegMinLogRows, has_short = false, has_chunks = false;
    for (int a = 0; a < s.n_alpha_psi; ++a) {
        has_long = has_long || s.logNX - s.k2[a] >= kRegMinLogRows;
        has_short = has_short || s.logNX - s.k2[a] <= 12;
    }
    for (int a = 0; a < s.n_alpha; ++a) has_chunks = has_chunks || s.Tp[a] > 1024;
    if (has_long || has_short || has_chunks) {
        double base_ms = 0.0, base_st[JTFS_NUM_STAGES];
        int rc = run_steps(P, x, B, (float*)s1.p, (float*)s2.p, (float*)gx.p, ws.p, wsb, reps, st, &base_ms, base_st);
        if (rc != JTFS_OK) return fail(rc);
        int next = rows;
        if (has_long) {
            double ms = 0.0, st8[JTFS_NUM_STAGES];
            set_rows(P, rows | kRadix8Bits);
            rc = run_steps(P, x, B, (float*)s1.p, (float*)s2.p, (float*)gx.p, ws.p, wsb, reps, st, &ms, st8);
            if (rc != JTFS_OK) return fail(rc);
            const int kstage[4] = {JTFS_STAGE_SCALOGRAM, JTFS_STAGE_SECOND_ORDER, JTFS_STAGE_SECOND_ADJ_FFT,
                                   JTFS_STAGE_FIRST_ADJ};
            const int kbit[4] = {JTFS_TUNE_RADIX8_SCALOGRAM, JTFS_TUNE_RADIX8_SECOND_ORDER, JTFS_TUNE_RADIX8_ROW_FFT,
                                 JTFS_TUNE_RADIX8_FIRST_ADJ};
            for (int q = 0; q < 4; ++q) {
                const double r16 = base_st[kstage[q]] + (q == 3 ? base_st[JTFS_STAGE_SECOND_ADJ] : 0.0);
                const double r8 = st8[kstage[q]] + (q == 3 ? st8[JTFS_STAGE_SECOND_ADJ] : 0.0);
                if (r8 < 0.99 * r16) next |= kbit[q];
            }
        }
        if (has_short) {
            double ms = 0.0, stb[JTFS_NUM_STAGES];
            set_rows(P, rows | JTFS_TUNE_LDS_BATCH8K);
            rc = run_steps(P, x, B, (float*)s1.p, (float*)s2.p, (float*)gx.p, ws.p, wsb, reps, st, &ms, stb);
            if (rc != JTFS_OK) return fail(rc);
            const double a0 = base_st[JTFS_STAGE_SECOND_ORDER] + base_st[JTFS_STAGE_SECOND_ADJ_FFT];
            const double a1 = stb[JTFS_STAGE_SECOND_ORDER] + stb[JTFS_STAGE_SECOND_ADJ_FFT];
            if (a1 < 0.99 * a0) next |= JTFS_TUNE_LDS_BATCH8K;
        }
        if (has_chunks) {
            // 1024 t-columns per forward workgroup instead of 4096: the forward contraction
            // and the frequency lowpass that sums its partial slots
            double ms = 0.0, stc[JTFS_NUM_STAGES];
            set_rows(P, rows | JTFS_TUNE_TCHUNK_1K);
            rc = run_steps(P, x, B, (float*)s1.p, (float*)s2.p, (float*)gx.p, ws.p, wsb, reps, st, &ms, stc);
            if (rc != JTFS_OK) return fail(rc);
            const double a0 = base_st[JTFS_STAGE_FREQ_FWD] + base_st[JTFS_STAGE_FREQ_LOWPASS];
            const double a1 = stc[JTFS_STAGE_FREQ_FWD] + stc[JTFS_STAGE_FREQ_LOWPASS];
            if (a1 < 0.99 * a0) next |= JTFS_TUNE_TCHUNK_1K;
        }
        rows = next;
        set_rows(P, rows);
    }
    double stage_final[JTFS_NUM_STAGES];
    const int rc = run_steps(P, x, B, (float*)s1.p, (float*)s2.p, (float*)gx.p, ws.p, wsb, reps, st, &out->step_ms,
                             stage_final);
    if (rc != JTFS_OK) return fail(rc);
    out->contraction = P->contraction;
    out->reg_rows = rows;
    cache_store(key, out->contraction, rows, out->step_ms);
    return JTFS_OK;
}
