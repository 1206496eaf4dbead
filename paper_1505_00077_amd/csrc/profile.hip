// Stage timing: optional HIP-event pairs around every kernel launch, summed per
// kernel name.  Off by default; when off, prof_begin/prof_end cost one load.
#include <string.h>

#include <mutex>
#include <string>
#include <vector>

#include "../../include/bfgp.h"
#include "launch.hpp"

namespace bfgp {
namespace {

constexpr int kMaxPairs = 16384;

struct Prof {
    std::mutex mu;
    bool on = false;
    std::vector<hipEvent_t> ev;        // 2 * kMaxPairs events, created once
    std::vector<const char *> name;    // per recorded pair
    std::vector<long long> threads;    // per recorded pair: grid size in threads
    int used = 0;
    bool open = false;
};

Prof &prof() {
    static Prof p;
    return p;
}

}  // namespace

void prof_begin(hipStream_t s, const char *name, long long threads) {
    Prof &p = prof();
    if (!p.on) return;
    std::lock_guard<std::mutex> g(p.mu);
    if (!p.on || p.used >= kMaxPairs) return;
    if (hipEventRecord(p.ev[2 * p.used], s) != hipSuccess) return;
    p.name[p.used] = name;
    p.threads[p.used] = threads;
    p.open = true;
}

void prof_end(hipStream_t s) {
    Prof &p = prof();
    if (!p.on) return;
    std::lock_guard<std::mutex> g(p.mu);
    if (!p.open) return;
    if (hipEventRecord(p.ev[2 * p.used + 1], s) == hipSuccess) ++p.used;
    p.open = false;
}

}  // namespace bfgp

using namespace bfgp;

extern "C" {

int bf_profile_enable(int on) {
    Prof &p = prof();
    std::lock_guard<std::mutex> g(p.mu);
    if (on && p.ev.empty()) {
        p.ev.resize(2 * kMaxPairs);
        p.name.resize(kMaxPairs);
        p.threads.resize(kMaxPairs);
        for (auto &e : p.ev)
            if (hipEventCreate(&e) != hipSuccess) {
                p.ev.clear();
                return BF_EHIP;
            }
    }
    p.used = 0;
    p.open = false;
    p.on = on != 0;
    return BF_OK;
}

int bf_profile_collect(int max, const char **names, int *counts, double *total_ms, long long *threads) {
    Prof &p = prof();
    std::lock_guard<std::mutex> g(p.mu);
    if (max < 0 || (max > 0 && (!names || !counts || !total_ms || !threads))) return BF_EINVAL;
    int n = 0;
    for (int i = 0; i < p.used; ++i) {
        if (hipEventSynchronize(p.ev[2 * i + 1]) != hipSuccess) return BF_EHIP;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, p.ev[2 * i], p.ev[2 * i + 1]) != hipSuccess) return BF_EHIP;
        int j = 0;
        while (j < n && strcmp(names[j], p.name[i]) != 0) ++j;
        if (j == n) {
            if (n >= max) continue;
            names[n] = p.name[i];
            counts[n] = 0;
            total_ms[n] = 0.0;
            ++n;
        }
        counts[j] += 1;
        total_ms[j] += ms;
        threads[j] = p.threads[i];
    }
    return n;
}

}  // extern "C"
