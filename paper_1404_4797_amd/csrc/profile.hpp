// Optional per-kernel timing with HIP events on the launching stream, and the
// algorithmic bytes each launch must move.  Off unless the caller enables it
// (sclap_profile_begin); per thread.
#pragma once

#include <string>
#include <vector>

#include "common.hpp"

namespace sclap {

struct KernelStat {
    std::string name;
    int64_t launches = 0;
    double ms = 0;
    double bytes = 0;
};

struct Profiler {
    bool on = false;
    std::string only;  // when set, only scopes of this name are timed
    std::vector<KernelStat> stats;
    struct Pending {
        hipEvent_t a, b;
        size_t idx;
        double bytes;
    };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> pool;

    int begin(const char* name, double bytes, hipStream_t s);
    void end(int token, hipStream_t s);
    // Adds up finished launches; call after the stream has been synchronised.
    void collect();
    void reset();
};

Profiler& profiler();

// RAII helper: times the launches issued while it lives (when profiling is on).
struct ProfScope {
    int token;
    hipStream_t s;
    ProfScope(const char* name, double bytes, hipStream_t st) : s(st) {
        token = profiler().on ? profiler().begin(name, bytes, st) : -1;
    }
    ~ProfScope() {
        if (token >= 0) profiler().end(token, s);
    }
};

}  // namespace sclap
