// Launch measurement behind ttsg_stats_enable / ttsg_stats_read.
#include <mutex>

#include "ttsg_internal.h"

namespace ttsg {
namespace {

struct Rec {
    hipEvent_t a, b;
    int cls;
    double flops, bytes;
};

std::mutex g_mu;
std::vector<Rec> g_recs;
bool g_on = false;

}  // namespace

bool stats_on() { return g_on; }

StatScope::StatScope(int cls, double flops, double bytes, hipStream_t st)
    : cls_(cls), flops_(flops), bytes_(bytes), st_(st) {
    if (!g_on) return;
    hipEvent_t a, b;
    TTSG_HIP(hipEventCreate(&a));
    TTSG_HIP(hipEventCreate(&b));
    TTSG_HIP(hipEventRecord(a, st));
    a_ = a;
    b_ = b;
}

StatScope::~StatScope() {
    if (a_ == nullptr) return;
    hipEvent_t a = static_cast<hipEvent_t>(a_), b = static_cast<hipEvent_t>(b_);
    if (hipEventRecord(b, st_) != hipSuccess) return;
    std::lock_guard<std::mutex> lk(g_mu);
    g_recs.push_back(Rec{a, b, cls_, flops_, bytes_});
}

}  // namespace ttsg

extern "C" {

int ttsg_stats_enable(int32_t on) {
    std::lock_guard<std::mutex> lk(ttsg::g_mu);
    for (auto& r : ttsg::g_recs) {
        (void)hipEventSynchronize(r.b);
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    ttsg::g_recs.clear();
    ttsg::g_on = on != 0;
    return 0;
}

int ttsg_stats_read(ttsg_stats* out) {
    if (out == nullptr) return -TTSG_ERR_ARG;
    std::lock_guard<std::mutex> lk(ttsg::g_mu);
    for (int c = 0; c < TTSG_ST_CLASSES; ++c) {
        out->launches[c] = 0;
        out->flops[c] = out->bytes[c] = out->seconds[c] = 0.0;
    }
    int rc = 0;
    for (auto& r : ttsg::g_recs) {
        float ms = 0.0f;
        if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) rc = -TTSG_ERR_HIP;
        const int c = r.cls;
        out->launches[c] += 1;
        out->flops[c] += r.flops;
        out->bytes[c] += r.bytes;
        out->seconds[c] += 1e-3 * (double)ms;
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    ttsg::g_recs.clear();
    return rc;
}

}  // extern "C"
