// Per-kernel timing with HIP events (dmcr_profile_start / dmcr_profile_stop).
// Each recorded launch carries an event pair that the runtime stamps with the
// dispatch's begin and end; totals are aggregated by kernel name when recording
// stops.
#include <string.h>

#include <map>
#include <string>
#include <vector>

#include "dmcr_internal.h"

namespace dmcr {

namespace {

struct Rec {
    const char *name;
    double bytes;
    hipEvent_t a, b;
};

bool g_on = false;
std::vector<Rec> g_recs;
std::vector<hipEvent_t> g_pool;
size_t g_next = 0;

hipEvent_t take_event()
{
    if (g_next == g_pool.size()) {
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        g_pool.push_back(e);
    }
    return g_pool[g_next++];
}

}  // namespace

bool prof_on() { return g_on; }

void prof_pair(const char *name, double bytes, hipEvent_t *start, hipEvent_t *stop)
{
    Rec r{name, bytes, take_event(), take_event()};
    *start = r.a;
    *stop = r.b;
    g_recs.push_back(r);
}

}  // namespace dmcr

using namespace dmcr;

extern "C" {

dmcr_status dmcr_profile_start(void)
{
    g_recs.clear();
    g_next = 0;
    g_on = true;
    return DMCR_OK;
}

int32_t dmcr_profile_stop(dmcr_kernel_stat *out, int32_t max)
{
    g_on = false;
    struct Agg {
        int launches = 0;
        double ms = 0, bytes = 0;
    };
    std::map<std::string, Agg> agg;
    std::vector<std::string> order;
    for (const Rec &r : g_recs) {
        if (!r.a || !r.b) return DMCR_EDEVICE;
        if (hipEventSynchronize(r.b) != hipSuccess) return DMCR_EDEVICE;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) return DMCR_EDEVICE;
        if (!agg.count(r.name)) order.push_back(r.name);
        Agg &a = agg[r.name];
        a.launches += 1;
        a.ms += ms;
        a.bytes += r.bytes;
    }
    g_recs.clear();
    g_next = 0;
    int32_t n = 0;
    for (const std::string &k : order) {
        if (out && n < max) {
            memset(&out[n], 0, sizeof(dmcr_kernel_stat));
            strncpy(out[n].name, k.c_str(), sizeof(out[n].name) - 1);
            out[n].launches = agg[k].launches;
            out[n].total_ms = agg[k].ms;
            out[n].bytes = agg[k].bytes;
        }
        ++n;
    }
    return n;
}

}  // extern "C"
