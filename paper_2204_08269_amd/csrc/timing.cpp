// Per-stage kernel timing with HIP events recorded on the launch stream.
#include "timing.hpp"

#include <mutex>
#include <vector>

namespace jtfs {
namespace {
struct Rec { int stage; hipEvent_t a, b; };
std::mutex g_mu;
bool g_on = false;
std::vector<Rec> g_recs;
std::vector<hipEvent_t> g_pool;

hipEvent_t take() {
    if (!g_pool.empty()) { hipEvent_t e = g_pool.back(); g_pool.pop_back(); return e; }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}
}  // namespace

static thread_local int t_quiet = 0;

bool timing_on() { std::lock_guard<std::mutex> l(g_mu); return g_on; }

TimingSuppressed::TimingSuppressed() { ++t_quiet; }
TimingSuppressed::~TimingSuppressed() { --t_quiet; }

TimedLaunch::TimedLaunch(int stage, hipStream_t st) : stage_(stage), st_(st) {
    if (t_quiet) return;
    std::lock_guard<std::mutex> l(g_mu);
    if (!g_on) return;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st_, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;  // no events in graphs
    a_ = take(); b_ = take();
    if (a_ && b_) (void)hipEventRecord(a_, st_);
}

TimedLaunch::~TimedLaunch() {
    std::lock_guard<std::mutex> l(g_mu);
    if (!a_ || !b_) return;
    (void)hipEventRecord(b_, st_);
    g_recs.push_back({stage_, a_, b_});
}

}  // namespace jtfs

extern "C" int jtfs_timing_enable(int on) {
    std::lock_guard<std::mutex> l(jtfs::g_mu);
    jtfs::g_on = on != 0;
    return JTFS_OK;
}

extern "C" int jtfs_timing_read(int stage, double* ms, int64_t* launches) {
    if (!ms || !launches || stage < 0 || stage >= JTFS_NUM_STAGES) {
        jtfs::set_error("invalid stage or null pointer");
        return JTFS_EINVAL;
    }
    std::lock_guard<std::mutex> l(jtfs::g_mu);
    double total = 0.0;
    int64_t n = 0;
    std::vector<jtfs::Rec> keep;
    for (auto& r : jtfs::g_recs) {
        if (r.stage != stage) { keep.push_back(r); continue; }
        float t = 0.f;
        if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&t, r.a, r.b) != hipSuccess) {
            jtfs::set_error("event timing failed");
            return JTFS_EHIP;
        }
        total += t;
        ++n;
        jtfs::g_pool.push_back(r.a);
        jtfs::g_pool.push_back(r.b);
    }
    jtfs::g_recs.swap(keep);
    *ms = total;
    *launches = n;
    return JTFS_OK;
}
