// Launch measurement behind ttsg_stats_enable / ttsg_stats_read.
//
// Every measured launch gets one DevSlot in a device array; its workgroups
// record the earliest start and latest end of the GPU wall clock.  The
// duration of a launch is therefore the time its kernel actually ran, not the
// gap between host-side events (which would include submission latency
// whenever the stream had drained).  A class's busy time is the union of its
// launches' intervals: below the summed durations when launches of the class
// overlap on several streams.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <mutex>
#include <utility>
#include <vector>

#include "ttsg_internal.h"

namespace ttsg {
namespace {

struct Rec {
    int cls;
    double flops, bytes;
    int64_t slot;
    int shp[5];
};

constexpr int64_t kSlots = 1 << 18;
std::mutex g_mu;
std::vector<Rec> g_recs;
bool g_on = false;
DevSlot* g_slots = nullptr;
int64_t g_next = 0;

}  // namespace

bool stats_on() { return g_on; }

int64_t g_events[TTSG_ST_CLASSES] = {};
void stats_event(int cls) {
    if (!g_on || cls < 0 || cls >= TTSG_ST_CLASSES) return;
    std::lock_guard<std::mutex> lk(g_mu);
    ++g_events[cls];
}

StatScope::StatScope(int cls, double flops, double bytes, hipStream_t st) {
    (void)st;
    if (!g_on) return;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_next >= kSlots) return;           // beyond the slot budget: not measured
    const int64_t id = g_next++;
    slot_ = g_slots + id;
    rec_ = (int64_t)g_recs.size();
    g_recs.push_back(Rec{cls, flops, bytes, id, {0, 0, 0, 0, 0}});
}

void StatScope::shape(int a, int b, int c, int d, int e) {
    if (rec_ < 0) return;
    std::lock_guard<std::mutex> lk(g_mu);
    if (rec_ >= (int64_t)g_recs.size()) return;
    int* p = g_recs[rec_].shp;
    p[0] = a;
    p[1] = b;
    p[2] = c;
    p[3] = d;
    p[4] = e;
}

StatScope::~StatScope() = default;

}  // namespace ttsg

extern "C" {

int ttsg_stats_enable(int32_t on) {
    std::lock_guard<std::mutex> lk(ttsg::g_mu);
    ttsg::g_recs.clear();
    ttsg::g_next = 0;
    for (auto& e : ttsg::g_events) e = 0;
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
        out->flops[c] = out->bytes[c] = out->seconds[c] = out->busy[c] = 0.0;
    }
    std::vector<std::vector<std::pair<unsigned long long, unsigned long long>>> spans(TTSG_ST_CLASSES);
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
    const char* logp = std::getenv("TTSG_SHAPE_LOG");
    FILE* log = (logp != nullptr && logp[0] != 0) ? std::fopen(logp, "a") : nullptr;
    for (const auto& r : ttsg::g_recs) {
        const ttsg::DevSlot& s = h[r.slot];
        unsigned long long t0 = ~0ull, t1 = 0;
        for (int l = 0; l < ttsg::kSlotLanes; ++l) {
            if (s.start_inv[l] != 0) t0 = std::min(t0, ~s.start_inv[l]);
            t1 = std::max(t1, s.end[l]);
        }
        if (t1 == 0 || t0 == ~0ull) continue;      // launch without workgroups
        const double sec = t1 > t0 ? (double)(t1 - t0) / (1e3 * rate_khz) : 0.0;
        if (log != nullptr)
            std::fprintf(log, "%d %d %d %d %d %d %.9f %.6e %llu\n", r.cls, r.shp[0], r.shp[1], r.shp[2], r.shp[3],
                         r.shp[4], sec, r.flops, (unsigned long long)s.aux);
        const int c = r.cls;
        out->launches[c] += 1;
        // a Jacobi launch records one sweep's rotations; it ran aux sweeps
        out->flops[c] += (c == TTSG_ST_SVD && s.aux > 0) ? r.flops * (double)s.aux : r.flops;
        out->bytes[c] += r.bytes;
        out->seconds[c] += sec;
        if (t1 > t0) spans[c].emplace_back(t0, t1);
        if (c == TTSG_ST_SVD && s.aux > (unsigned long long)out->flops[7]) out->flops[7] = (double)s.aux;
    }
    if (log != nullptr) std::fclose(log);
    for (int c = 0; c < TTSG_ST_CLASSES; ++c) {
        auto& v = spans[c];
        std::sort(v.begin(), v.end());
        unsigned long long cov = 0, a = 0, b = 0;
        bool open = false;
        for (const auto& iv : v) {
            if (!open || iv.first > b) {
                if (open) cov += b - a;
                a = iv.first;
                b = iv.second;
                open = true;
            } else if (iv.second > b) {
                b = iv.second;
            }
        }
        if (open) cov += b - a;
        out->busy[c] = (double)cov / (1e3 * rate_khz);
    }
    for (int c = 0; c < TTSG_ST_CLASSES; ++c) {
        out->launches[c] += ttsg::g_events[c];
        ttsg::g_events[c] = 0;
    }
    ttsg::g_recs.clear();
    ttsg::g_next = 0;
    if (hipMemset(ttsg::g_slots, 0, ttsg::kSlots * sizeof(ttsg::DevSlot)) != hipSuccess) return -TTSG_ERR_HIP;
    return 0;
}

}  // extern "C"
