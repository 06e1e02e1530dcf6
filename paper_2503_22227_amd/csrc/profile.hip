// Kernel timing with HIP events, for measurement runs.  When enabled, every
// kernel launch of the library is bracketed by two events recorded on the
// launch's own stream; rf_profile_read() waits for the recorded events and
// reports the launch count and the summed elapsed time per kernel name.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "rf_internal.hpp"

namespace rf {

namespace {
struct Rec {
    const char *name;
    hipEvent_t start, stop;
};
std::mutex g_mu;
bool g_on = false;
std::vector<Rec> g_recs;
std::vector<hipEvent_t> g_pool;

hipEvent_t take_event() {
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}
}  // namespace

ProfScope::ProfScope(const char *name, hipStream_t s) : idx_(-1), s_(s) {
    if (!name) return;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_on) return;
    Rec r{name, take_event(), take_event()};
    if (!r.start || !r.stop) return;
    if (hipEventRecord(r.start, s) != hipSuccess) return;
    g_recs.push_back(r);
    idx_ = (int)g_recs.size() - 1;
}

ProfScope::~ProfScope() {
    if (idx_ < 0) return;
    std::lock_guard<std::mutex> lk(g_mu);
    if (idx_ < (int)g_recs.size()) (void)hipEventRecord(g_recs[idx_].stop, s_);
}

}  // namespace rf

extern "C" int rf_profile_enable(int on) {
    std::lock_guard<std::mutex> lk(rf::g_mu);
    rf::g_on = on != 0;
    return RF_OK;
}

extern "C" int rf_profile_read(char *buf, size_t len) {
    using namespace rf;
    std::map<std::string, std::pair<long, double>> acc;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        for (Rec &r : g_recs) {
            if (hipEventSynchronize(r.stop) != hipSuccess) return fail(RF_EHIP, "rf_profile_read: event");
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, r.start, r.stop) != hipSuccess) return fail(RF_EHIP, "rf_profile_read: elapsed");
            auto &a = acc[r.name];
            a.first += 1;
            a.second += ms;
            g_pool.push_back(r.start);
            g_pool.push_back(r.stop);
        }
        g_recs.clear();
    }
    std::string out;
    for (auto &kv : acc)
        out += kv.first + " " + std::to_string(kv.second.first) + " " + std::to_string(kv.second.second) + "\n";
    if (buf && len) {
        size_t n = out.size() < len - 1 ? out.size() : len - 1;
        out.copy(buf, n);
        buf[n] = 0;
    }
    return (int)out.size();
}
