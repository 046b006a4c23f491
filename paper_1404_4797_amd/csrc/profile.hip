// Per-kernel HIP-event timing (see profile.hpp).
#include "profile.hpp"

namespace sclap {

Profiler& profiler() {
    thread_local Profiler p;
    return p;
}

int Profiler::begin(const char* name, double bytes, hipStream_t s) {
    if (!only.empty() && only != name) return -1;
    size_t idx = stats.size();
    for (size_t i = 0; i < stats.size(); ++i)
        if (stats[i].name == name) idx = i;
    if (idx == stats.size()) {
        stats.push_back(KernelStat());
        stats.back().name = name;
    }
    Pending p;
    for (hipEvent_t* e : {&p.a, &p.b}) {
        if (!pool.empty()) {
            *e = pool.back();
            pool.pop_back();
        } else {
            HIPCHK(hipEventCreate(e));
        }
    }
    p.idx = idx;
    p.bytes = bytes;
    HIPCHK(hipEventRecord(p.a, s));
    pending.push_back(p);
    return static_cast<int>(pending.size() - 1);
}

void Profiler::end(int token, hipStream_t s) { HIPCHK(hipEventRecord(pending[token].b, s)); }

void Profiler::collect() {
    for (Pending& p : pending) {
        float ms = 0;
        HIPCHK(hipEventSynchronize(p.b));
        HIPCHK(hipEventElapsedTime(&ms, p.a, p.b));
        KernelStat& k = stats[p.idx];
        k.launches += 1;
        k.ms += ms;
        k.bytes += p.bytes;
        pool.push_back(p.a);
        pool.push_back(p.b);
    }
    pending.clear();
}

void Profiler::reset() {
    collect();
    stats.clear();
}

}  // namespace sclap
