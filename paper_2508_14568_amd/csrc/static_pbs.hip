// Programmable bootstraps that allocate nothing: the job list and the key
// switch's partial sums of lvs_pbs_batch live in a file-scope device array
// instead of a caller workspace, for callers that cannot allocate device
// memory (code under stream capture, serving loops, harnesses that forbid it).
//
// Every device the library runs on holds its own copy of the array until the
// process ends.  Its address on a device is taken once, with that device
// current, when a context is created there (lvs_context_create); host code
// uses only that address, never the array's name, which on the host is a
// stand-in and not a device address.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <string>

#include "context.h"
#include "launch.h"
#include "lvs_internal.h"

namespace lvs {
namespace {

constexpr size_t kStaticMaxB = LVS_PBS_STATIC_MAX;
constexpr size_t kAlignStatic = 256;
constexpr size_t kJobArea = (sizeof(Job) * kStaticMaxB + kAlignStatic - 1) / kAlignStatic * kAlignStatic;
// Rows of n + 1 partial-sum words: splits x ciphertexts of one call.  The
// split count is capped so that it fits (a full batch of kStaticMaxB takes
// two splits; narrow batches keep up to 64).
constexpr size_t kPartRows = 2 * kStaticMaxB;
constexpr size_t kScratchBytes = kJobArea + sizeof(uint64_t) * kPartRows * kSmallWords;
constexpr int kMaxDevices = 64;

std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

// Job of ciphertext b: input d_in[b] (coefficient 1), table ids[b] or lut,
// output M to d_out[b] (the job's third destination, written as is).
struct StaticJobsArgs {
    const uint64_t* in;
    uint64_t* out;
    Job* jobs;
    uint32_t B;
    uint32_t lut;
    uint32_t per_ct;
    uint8_t ids[kStaticMaxB];
};

}  // namespace

static __device__ __align__(256) uint8_t scratch[kScratchBytes];

namespace {

__global__ void __launch_bounds__(256) static_jobs_kernel(StaticJobsArgs a) {
    const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= a.B) return;
    Job J{};
    J.src[0] = a.in + size_t(b) * kCtWords;
    J.coef[0] = 1;
    J.lut = a.per_ct ? uint32_t(a.ids[b]) : a.lut;
    J.dst[2] = a.out + size_t(b) * kCtWords;
    a.jobs[b] = J;
}

// Largest power-of-two split count up to the launcher's own choice whose
// partial sums fit the array's rows.
int static_splits(int B, int tile) {
    int s = keyswitch_splits(B, tile);
    while (s > 1 && size_t(s) * size_t(B) > kPartRows) s /= 2;
    return s;
}

}  // namespace

// Set-up of the calling thread's current device: records the array's address
// there (once per device).  Returns hipSuccess or the lookup's error.
hipError_t static_scratch_setup(int device) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (g_scratch[device]) return hipSuccess;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_scratch[device] = ptr;
    return hipSuccess;
}

size_t static_scratch_bytes() { return kScratchBytes; }

}  // namespace lvs

using namespace lvs;

extern "C" {

int lvs_pbs_batch_static(lvs_context* ctx, const uint64_t* d_in, const uint8_t* lut_ids, int lut_id, size_t B,
                         uint64_t* d_out) {
    auto* C = reinterpret_cast<Context*>(ctx);
    auto fail = [](int code, const std::string& msg) {
        set_error(msg);
        return code;
    };
    if (!C || C->kind != kContext) return fail(LVS_E_INVAL, "lvs_pbs_batch_static: bad context");
    if (B == 0) return LVS_OK;
    if (B > kStaticMaxB)
        return fail(LVS_E_INVAL, "lvs_pbs_batch_static: B = " + std::to_string(B) + " exceeds LVS_PBS_STATIC_MAX (" +
                                     std::to_string(kStaticMaxB) + ")");
    if (!d_in || !d_out) return fail(LVS_E_INVAL, "lvs_pbs_batch_static: NULL buffer");
    StaticJobsArgs a{};
    if (lut_ids) {
        for (size_t k = 0; k < B; ++k) {
            if (lut_ids[k] >= LVS_LUT_SLOTS) return fail(LVS_E_INVAL, "lvs_pbs_batch_static: bad lut id");
            a.ids[k] = lut_ids[k];
        }
    } else if (lut_id < 0 || lut_id >= LVS_LUT_SLOTS) {
        return fail(LVS_E_INVAL, "lvs_pbs_batch_static: bad lut id");
    }
    if (!(d_out + B * kCtWords <= d_in || d_in + B * kCtWords <= d_out))
        return fail(LVS_E_INVAL, "lvs_pbs_batch_static: in and out overlap");
    if (C->device < 0 || C->device >= kMaxDevices) return fail(LVS_E_DEVICE, "lvs_pbs_batch_static: bad device");
    uint8_t* base;
    {
        std::lock_guard<std::mutex> lock(g_mu);
        base = reinterpret_cast<uint8_t*>(g_scratch[C->device]);
    }
    if (!base) return fail(LVS_E_DEVICE, "lvs_pbs_batch_static: device scratch not set up");
    hipError_t e = hipSetDevice(C->device);
    a.in = d_in;
    a.out = d_out;
    a.jobs = reinterpret_cast<Job*>(base);
    a.B = uint32_t(B);
    a.lut = uint32_t(lut_id);
    a.per_ct = lut_ids ? 1u : 0u;
    uint64_t* part = reinterpret_cast<uint64_t*>(base + kJobArea);
    const int nB = int(B);
    const int ns = static_splits(nB, C->ks_tile);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(static_jobs_kernel, dim3((nB + 255) / 256), dim3(256), 0, C->stream, a);
        e = hipGetLastError();
    }
    if (e == hipSuccess) {
        TimedLaunch t(C, kProfKeySwitch, uint64_t(nB));
        e = launch_keyswitch_jobs(a.jobs, nB, C->ksk, part, C->stream, ns, C->ks_tile);
    }
    if (e == hipSuccess) {
        TimedLaunch t(C, br_profile_id(C, nB), uint64_t(nB));
        e = launch_blind_rotate_jobs(a.jobs, nB, part, C->luts, C->bsk, C->tables, C->br_grid, C->latency_form_max,
                                     C->latency_waves, C->stream, ns, C->throughput_waves);
    }
    if (e != hipSuccess) return fail(LVS_E_DEVICE, std::string("lvs_pbs_batch_static: ") + hipGetErrorString(e));
    return LVS_OK;
}

}  // extern "C"
