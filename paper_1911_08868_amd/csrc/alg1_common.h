// alg1_common.h -- what the two Algorithm 1 kernels share: their arguments,
// the bounded draws of the event parameters and the check function.
#pragma once

#include "bp_core.h"
#include "internal.h"

namespace pbp {

struct Alg1Args {
    const float *llr;
    int64_t F;
    uint8_t *msg;
    int32_t *iters;
    uint8_t *ok;
    float *soft;
    const uint32_t *syn;
    const int32_t *meta;
    uint32_t *counter;
    int32_t K_msg, max_iter, it_min, stop;
    float alpha;
    int32_t P_range, P_level, D, N_min, first_reset;
    uint64_t seed;
    uint64_t *hist;  // [F][H] decision hashes, or NULL
    int32_t H;
    float noise_sigma;  // > 0: channel level y + sigma g(frame, e, j) after event e
    uint64_t noise_seed;
};

// uniform integer in [0, m): the high 32 bits of the next output, scaled by m
__device__ __forceinline__ uint32_t draw_below(uint64_t &s, uint32_t m) {
    const uint64_t hi = splitmix64_next(s) >> 32;
    return (uint32_t)((hi * (uint64_t)m) >> 32);
}

// Check function of the processing elements: CN 0 min-sum, 1 scaled min-sum
// (the clamp form: equal to the FP32 oracle's values, a zero possibly with
// the other sign; x is the bound, an L operand as in the fixed-schedule
// kernels), 2 the exact boxplus (FP32 on the hardware exp2/log2).
template <int CN>
__device__ __forceinline__ float alg1_check(float x, float y, float alpha) {
    if constexpr (CN == 2) return cnode_exact(x, y);
    else return cnode_clamp<CN>(x, y, alpha);
}

// iteration after which a frame's first event comes: first_reset, or the
// spacing Eq. 2 gives a permutation of the whole graph (N_zero = N (n-1)),
// at most half the iteration budget
__device__ __forceinline__ int alg1_first_event(const Alg1Args &a, int N, int n) {
    if (a.first_reset > 0) return a.first_reset;
    const int full = a.D > 0 ? (N * (n - 1)) / a.D : 0;
    const int v = full > a.N_min ? full : a.N_min;
    return v < a.max_iter / 2 ? v : a.max_iter / 2;
}

// the kernel of Algorithm 1 under the original-graph reading, for n = 4..10
int run_alg1_orig(const Alg1Args &a, int n, int cn, hipStream_t s);

}  // namespace pbp
