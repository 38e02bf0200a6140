// Launch measurement behind ttsg_stats_enable / ttsg_stats_read.
//
// Every measured launch gets one DevSlot in a device array; its workgroups
// record the earliest start and latest end of the GPU wall clock.  The
// duration of a launch is therefore the time its kernel actually ran, not the
// gap between host-side events (which would include submission latency
// whenever the stream had drained).
#include <mutex>

#include "ttsg_internal.h"

namespace ttsg {
namespace {

struct Rec {
    int cls;
    double flops, bytes;
    int64_t slot;
};

constexpr int64_t kSlots = 1 << 20;
std::mutex g_mu;
std::vector<Rec> g_recs;
bool g_on = false;
DevSlot* g_slots = nullptr;
int64_t g_next = 0;

}  // namespace

bool stats_on() { return g_on; }

StatScope::StatScope(int cls, double flops, double bytes, hipStream_t st) {
    (void)st;
    if (!g_on) return;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_next >= kSlots) return;           // beyond the slot budget: not measured
    const int64_t id = g_next++;
    slot_ = g_slots + id;
    g_recs.push_back(Rec{cls, flops, bytes, id});
}

StatScope::~StatScope() = default;

}  // namespace ttsg

extern "C" {

int ttsg_stats_enable(int32_t on) {
    std::lock_guard<std::mutex> lk(ttsg::g_mu);
    ttsg::g_recs.clear();
    ttsg::g_next = 0;
    if (on) {
        if (ttsg::g_slots == nullptr) {
            if (hipMalloc(&ttsg::g_slots, ttsg::kSlots * sizeof(ttsg::DevSlot)) != hipSuccess) return -TTSG_ERR_HIP;
        }
        if (hipMemset(ttsg::g_slots, 0, ttsg::kSlots * sizeof(ttsg::DevSlot)) != hipSuccess) return -TTSG_ERR_HIP;
        if (hipDeviceSynchronize() != hipSuccess) return -TTSG_ERR_HIP;
    }
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
    if (hipDeviceSynchronize() != hipSuccess) return -TTSG_ERR_HIP;
    int rate_khz = 0;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || rate_khz <= 0)
        return -TTSG_ERR_HIP;
    std::vector<ttsg::DevSlot> h(ttsg::g_next);
    if (ttsg::g_next > 0 &&
        hipMemcpy(h.data(), ttsg::g_slots, ttsg::g_next * sizeof(ttsg::DevSlot), hipMemcpyDeviceToHost) != hipSuccess)
        return -TTSG_ERR_HIP;
    for (const auto& r : ttsg::g_recs) {
        const ttsg::DevSlot& s = h[r.slot];
        if (s.end == 0 || s.start_inv == 0) continue;      // launch without workgroups
        const unsigned long long t0 = ~s.start_inv;
        const double sec = s.end > t0 ? (double)(s.end - t0) / (1e3 * rate_khz) : 0.0;
        const int c = r.cls;
        out->launches[c] += 1;
        out->flops[c] += r.flops;
        out->bytes[c] += r.bytes;
        out->seconds[c] += sec;
        if (c == TTSG_ST_SVD && s.aux > (unsigned long long)out->flops[7]) out->flops[7] = (double)s.aux;
    }
    ttsg::g_recs.clear();
    ttsg::g_next = 0;
    if (hipMemset(ttsg::g_slots, 0, ttsg::kSlots * sizeof(ttsg::DevSlot)) != hipSuccess) return -TTSG_ERR_HIP;
    return 0;
}

}  // extern "C"
