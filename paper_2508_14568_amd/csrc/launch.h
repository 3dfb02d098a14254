// Host-side launchers of the device kernels (kernels.hip).
#pragma once

#include <hip/hip_runtime_api.h>

#include "lvs_internal.h"

namespace lvs {

// One bootstrap of a step.  Its input ciphertext is the linear combination
// sum_k coef[k] * src[k] (+ delta on the body), so the key of a cell and the
// differences of the equality test are formed while the key switch reads
// them; its output M (the sample-extracted result) is written to every
// non-null dst[k] as M - sub[k] - sub_delta[k] (sub[k] may be null; sub_delta
// is subtracted from the body only), which applies the difference update of
// a cell in the same pass; dst[2] receives M itself and dst[3] a second copy
// of output copy_of (0 or 1), which collects the differences of a band path.
// A thread reads every sub[] word before writing the dst[] words of the same
// index, so dst and sub may alias; dst[2] may alias src[0] (an in-place
// refresh), since the key switch reads the mask in an earlier launch and the
// blind rotation reads the body before it writes any output.
struct Job {
    const uint64_t* src[3];
    int32_t coef[3];
    uint32_t lut;
    uint64_t delta;
    uint64_t* dst[4];
    const uint64_t* sub[2];
    uint64_t sub_delta[2];
    uint32_t copy_of;
};

struct DevTables {
    const uint32_t* fwd;      // [kPrimes][N][2] forward twiddles psi^brv(k) with Shoup companions
    const uint32_t* inv;      // [kPrimes][N][2] inverse twiddles psi^-brv(k) with Shoup companions
    const uint32_t* scale;    // [kPrimes] (1/N) 2^32 mod p
    const uint32_t* scale_s;
};

hipError_t launch_fill_u64(uint64_t* p, size_t count, uint64_t v, hipStream_t st);
// Key switch of B job inputs in tiles of `tile` ciphertexts per workgroup (4,
// 8 or 16) into partial sums part[split][B][n+1]; keyswitch_splits gives the
// number of splits of the input coefficients (the blind rotation sums them),
// at most kKsPartRows / B (rounded down to a power of two) when B > 1, so
// that keyswitch_part_words(B) words hold the partials of any batch up to B
// at any tile.
constexpr size_t kKsPartRows = 16384;
int keyswitch_splits(int B, int tile = 8);
size_t keyswitch_part_words(int B);
// nsplit > 0 overrides keyswitch_splits(B, tile) (a power of two, at most
// 64); the blind rotation that sums the partials must be given the same count.
hipError_t launch_keyswitch_jobs(const Job* jobs, int B, const uint64_t* ksk, uint64_t* part, hipStream_t st,
                                 int nsplit = 0, int tile = 8);
// Batches of at most latency_form_max bootstraps take the one-workgroup-per-CU
// form of the blind rotation (latency_waves 8 or 16 wavefronts), larger ones
// a two-per-CU form (throughput_waves 8: the eight-wave form with one LDS
// buffer; 4: the four-wave form).
hipError_t launch_blind_rotate_jobs(const Job* jobs, int B, const uint64_t* part, const uint64_t* luts,
                                    const uint32_t* bsk, const DevTables& t, int grid, int latency_form_max,
                                    int latency_waves, hipStream_t st, int nsplit = 0, int throughput_waves = 8);
hipError_t prepare_kernels();
// Records the address of the no-allocation entry point's device array on
// `device`, which must be current (static_pbs.hip); once per device.
hipError_t static_scratch_setup(int device);
size_t static_scratch_bytes();
hipError_t launch_bsk_convert(const uint64_t* bsk_u64, uint32_t* out, const DevTables& t, hipStream_t st);
hipError_t launch_trivial(uint64_t* out, int count, uint32_t mu, hipStream_t st);
// out[item][g] = sum_{k in group g} in[item][k] for items x cnt ciphertexts in
// groups of `group` (the last may be shorter); groups = ceil(cnt / group).
hipError_t launch_group_sum(const uint64_t* in, uint64_t* out, size_t items, int cnt, int groups, int group,
                            int cus, hipStream_t st);
// Microbenchmarks: the forward butterfly's instruction mix from registers
// (blocks of 256 threads, iters rounds) and a 16-byte vector copy.
hipError_t launch_modmul_probe(uint32_t* out, int blocks, int iters, hipStream_t st);
int modmul_probe_muls_per_thread_iter();
hipError_t launch_copy_probe(const void* src, void* dst, size_t bytes, int cus, hipStream_t st);

}  // namespace lvs
