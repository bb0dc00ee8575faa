// Cost loads with the non-temporal cache policy, for kernels that read each cost once and whose
// other data should keep the caches (the scanline DP sweeps).
#pragma once
#include "edp_device.hpp"

namespace edp {

constexpr int CPOL_NT = 2;   // buffer instruction cache policy: non-temporal

// load_cost_words with non-temporal loads
template <class CK, int N>
__device__ __forceinline__ void load_cost_words_nt(__amdgpu_buffer_rsrc_t r, int32_t off, int32_t* w) {
    if constexpr (sizeof(CK) == 4) {
        load_vec<N, CPOL_NT>(r, off, w);
    } else if constexpr (std::is_same<CK, Pair16>::value && N % 2 == 0) {
        load_vec<N / 2, CPOL_NT>(r, off, w);
    } else {
#pragma unroll
        for (int k = 0; k < N; ++k)
            w[k] = (int32_t)(int16_t)__builtin_amdgcn_raw_buffer_load_b16(r, off + 2 * k, 0, CPOL_NT);
    }
}

}  // namespace edp
