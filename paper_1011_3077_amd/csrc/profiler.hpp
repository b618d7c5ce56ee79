// Opt-in per-launch timing of the hot kernels with HIP events recorded on the
// launch stream, together with each launch's algorithmic flops and bytes.
// Enabled per handle (sdc_profile_enable); the engine installs the handle's
// profiler for the duration of a call.
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

namespace sdc {

enum ProfKernel { PROF_UPDATE = 0, PROF_PANEL = 1, PROF_GEMM = 2, PROF_LA = 3, PROF_NKERNELS = 4 };

struct Profiler {
    bool on = false;
    struct Rec {
        int kernel;
        hipEvent_t a, b;
        double flops, bytes;
    };
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;
    size_t used = 0;
    // accumulated after resolve()
    long long launches[PROF_NKERNELS] = {0, 0, 0, 0};
    double ms[PROF_NKERNELS] = {0, 0, 0, 0};
    double flops[PROF_NKERNELS] = {0, 0, 0, 0};
    double bytes[PROF_NKERNELS] = {0, 0, 0, 0};

    hipEvent_t next_event() {
        if (used == pool.size()) {
            hipEvent_t e;
            if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
            pool.push_back(e);
        }
        return pool[used++];
    }
    // bracket a launch: begin() before, end() after
    int begin(hipStream_t s) {
        if (!on) return -1;
        hipEvent_t a = next_event();
        if (!a || hipEventRecord(a, s) != hipSuccess) return -1;
        recs.push_back(Rec{0, a, nullptr, 0, 0});
        return (int)recs.size() - 1;
    }
    void end(int id, hipStream_t s, int kernel, double fl, double by) {
        if (id < 0) return;
        hipEvent_t b = next_event();
        if (!b || hipEventRecord(b, s) != hipSuccess) return;
        recs[id].b = b;
        recs[id].kernel = kernel;
        recs[id].flops = fl;
        recs[id].bytes = by;
    }
    // fold recorded launches into the totals (stream must be synchronized)
    void resolve() {
        for (const Rec& r : recs) {
            if (!r.b) continue;
            float t = 0;
            if (hipEventElapsedTime(&t, r.a, r.b) != hipSuccess) continue;
            launches[r.kernel] += 1;
            ms[r.kernel] += t;
            flops[r.kernel] += r.flops;
            bytes[r.kernel] += r.bytes;
        }
        recs.clear();
        used = 0;
    }
    void reset() {
        recs.clear();
        used = 0;
        for (int k = 0; k < PROF_NKERNELS; ++k) launches[k] = 0, ms[k] = flops[k] = bytes[k] = 0;
    }
    ~Profiler() {
        for (hipEvent_t e : pool) (void)hipEventDestroy(e);
    }
};

// The profiler of the call in progress (null when profiling is off).
extern thread_local Profiler* g_prof;

}  // namespace sdc
