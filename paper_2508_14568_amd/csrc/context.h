// Device context of liblvs.
#pragma once

#include <hip/hip_runtime_api.h>

#include <vector>

#include "launch.h"
#include "lvs_internal.h"

namespace lvs {

struct Context : Handle {
    lvs_params p{};
    int device = 0;
    hipStream_t stream = nullptr;
    hipStream_t capture_stream = nullptr;   // created on first graph capture
    uint8_t* arena = nullptr;
    size_t arena_bytes = 0;
    uint32_t* bsk = nullptr;      // NTT domain
    uint64_t* ksk = nullptr;
    uint32_t* tw = nullptr;       // forward pairs, inverse pairs, scale, scale companion
    uint64_t* luts = nullptr;     // [LVS_LUT_SLOTS][N]
    DevTables tables{};
    int cus = 0;                  // compute units of the device
    // launch shape of the blind rotation (lvs_context_set_tuning / lvs_autotune)
    int br_grid = 0;              // persistent grid (0: one workgroup per job)
    int latency_form_max = 0;     // batches up to this size take the one-workgroup-per-CU form
    int latency_waves = 8;        // that form's wavefronts per bootstrap: 8 or 16
    int throughput_waves = 8;     // larger batches: two workgroups per CU of 8 (or 4) wavefronts
    int ks_tile = 8;              // key switch: ciphertexts per workgroup (4, 8 or 16)
    size_t refresh_every = LVS_REFRESH_DEFAULT;   // noise-refresh interval in anti-diagonals (0: off)
    // kernel timing (lvs_profile_*): event pairs recorded around launches
    bool profiling = false;
    struct Timed {
        hipEvent_t start, end;
        int kernel;
        uint64_t units;
    };
    std::vector<Timed> timed;
    std::vector<hipEvent_t> spare;
};

inline hipEvent_t take_event(Context* C) {
    hipEvent_t e = nullptr;
    if (!C->spare.empty()) {
        e = C->spare.back();
        C->spare.pop_back();
    } else if (hipEventCreate(&e) != hipSuccess) {
        e = nullptr;
    }
    return e;
}

// Profile ids (lvs_profile_read): 0 sums the blind-rotation forms, which are
// recorded as 3 (eight-wave workgroup, one per CU), 4 (four-wave workgroups,
// two per CU), 5 (sixteen-wave workgroup, one per CU) and 6 (eight-wave
// workgroups, two per CU).
constexpr int kProfBlindRotate = 0, kProfKeySwitch = 1, kProfGraph = 2, kProfBrLatency = 3, kProfBrThroughput = 4,
              kProfBrW16 = 5, kProfBrPair = 6;

inline int br_profile_id(const Context* C, int B) {
    if (B > C->latency_form_max) return C->throughput_waves == 8 ? kProfBrPair : kProfBrThroughput;
    return C->latency_waves == 16 ? kProfBrW16 : kProfBrLatency;
}

// Brackets one launch with events when profiling is on.
struct TimedLaunch {
    Context* C;
    hipEvent_t a = nullptr;
    int kernel;
    uint64_t units;
    // an event that cannot be recorded goes back to the spares and the launch
    // is left untimed
    TimedLaunch(Context* c, int k, uint64_t u) : C(c), kernel(k), units(u) {
        if (k >= 0 && C->profiling && (a = take_event(C)) && hipEventRecord(a, C->stream) != hipSuccess) {
            C->spare.push_back(a);
            a = nullptr;
        }
    }
    ~TimedLaunch() {
        if (!a) return;
        hipEvent_t b = take_event(C);
        if (!b || hipEventRecord(b, C->stream) != hipSuccess) {
            C->spare.push_back(a);
            if (b) C->spare.push_back(b);
            return;
        }
        C->timed.push_back({a, b, kernel, units});
    }
};

}  // namespace lvs
