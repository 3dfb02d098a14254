// Host-side launchers of the device kernels (kernels.hip).
#pragma once

#include <hip/hip_runtime_api.h>

#include "lvs_internal.h"

namespace lvs {

struct DevTables {
    const uint32_t* fwd;      // [kPrimes][N] forward twiddles psi^brv(k)
    const uint32_t* fwd_s;    // Shoup companions
    const uint32_t* inv;      // [kPrimes][N] inverse twiddles psi^-brv(k)
    const uint32_t* inv_s;
    const uint32_t* scale;    // [kPrimes] (1/N) 2^32 mod p
    const uint32_t* scale_s;
};

hipError_t launch_fill_u64(uint64_t* p, size_t count, uint64_t v, hipStream_t st);
hipError_t launch_keyswitch(const uint64_t* in, const uint64_t* ksk, uint64_t* ks_out, int B, hipStream_t st);
hipError_t launch_blind_rotate(const uint64_t* ks, const uint8_t* lut_ids, int lut_id, const uint64_t* luts,
                               const uint32_t* bsk, const DevTables& t, uint64_t* out, int B, int grid,
                               hipStream_t st);
hipError_t launch_bsk_convert(const uint64_t* bsk_u64, uint32_t* out, const DevTables& t, hipStream_t st);
hipError_t launch_pair(const uint64_t* A, int a_stride, int sa, const uint64_t* B, int b_stride, int sb,
                       const uint8_t* clear_syms, const uint64_t* E, uint64_t alpha, uint64_t delta, uint64_t* out,
                       int n, long c0, long count, hipStream_t st);
hipError_t launch_key(const uint64_t* V, const uint64_t* H, const uint64_t* EQ, size_t eq_si, size_t eq_sj,
                      const int32_t* col, uint64_t* key, int i0, int s, int count, hipStream_t st);
hipError_t launch_update(uint64_t* V, uint64_t* H, const uint64_t* M, int i0, int s, int count, uint64_t* trace,
                         int n, hipStream_t st);
hipError_t launch_trivial(uint64_t* out, int count, uint32_t mu, hipStream_t st);
hipError_t launch_table_scatter(const uint64_t* src, uint64_t* dst, int m, int alen, long c0, long count,
                                hipStream_t st);

}  // namespace lvs
