// decode_inst.h -- launch of the decode kernel for one block length.  Each
// decode_nXX.hip includes this with its own NLOG so the instantiations build
// in parallel translation units.
#pragma once

#include "decode_kernel.h"
#include "internal.h"

namespace pbp {

struct DecodeLaunch {
    DecodeArgs args;
    int kp = 0;
    bool scaled = false, gmode = false;
    // kernel family: 0 min-sum, 1 min-sum with decision history, 2 exact
    // boxplus, 3 min-sum with noise injected at the events (1..3 are built
    // with two rows per thread only)
    int variant = 0;
    int rho = 2, slots = 0, grid = 0;
    int64_t F = 0;
    hipStream_t stream = nullptr;
};

template <int NLOG, int KP, int RHO, int CN, bool GM, bool TR, bool NZ>
int run_decode(const DecodeLaunch &L) {
    using P = Plan<NLOG, KP, RHO>;
    const int TPS = P::TPS;
    int S = L.slots;
    if (S <= 0) S = TPS >= 256 ? 1 : 256 / TPS;
    constexpr int LB = TPS > 256 ? TPS : 256;  // the kernel's launch bound
    if (S * TPS > LB) return fail(PC_EINVAL, "slots * threads per frame exceeds the launch bound");
    const size_t lds = DecodeLds<P>::bytes(S);
    if (lds > 160 * 1024) return fail(PC_EINVAL, "LDS budget exceeded for this launch shape");
    auto kern = k_decode<NLOG, KP, RHO, CN, GM, TR, NZ>;
    int grid = L.grid;
    if (grid <= 0) {
        int per_cu = 0;
        hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, S * TPS, lds);
        if (e != hipSuccess) return hip_fail(e, "occupancy query");
        if (per_cu < 1) per_cu = 1;
        grid = per_cu * device_cu_count();
    }
    const int64_t need = (L.F + S - 1) / S;
    if (grid > need) grid = (int)need;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(S * TPS), lds, L.stream, L.args);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "decode launch");
    return PC_OK;
}

template <int NLOG, int KP, int RHO, int V, bool GM>
int run_decode_check(const DecodeLaunch &L) {
    if constexpr (V == 2) {
        return run_decode<NLOG, KP, RHO, 2, GM, false, false>(L);
    } else {
        return L.scaled ? run_decode<NLOG, KP, RHO, 1, GM, V == 1, V == 3>(L)
                        : run_decode<NLOG, KP, RHO, 0, GM, V == 1, V == 3>(L);
    }
}

template <int NLOG, int KP, int RHO, int V>
int run_decode_flags(const DecodeLaunch &L) {
    if constexpr (KP == 0) {
        return L.gmode ? run_decode_check<NLOG, KP, RHO, V, true>(L) : run_decode_check<NLOG, KP, RHO, V, false>(L);
    } else {
        if (L.gmode) return fail(PC_ENOTSUP, "the G test is only built for the original graph");
        return run_decode_check<NLOG, KP, RHO, V, false>(L);
    }
}

template <int NLOG, int RHO, int V>
int run_decode_kp(const DecodeLaunch &L) {
    if (L.kp == 0) return run_decode_flags<NLOG, 0, RHO, V>(L);
    if (L.kp == NLOG) {
        if constexpr (NLOG >= 2) return run_decode_flags<NLOG, NLOG, RHO, V>(L);
    }
    switch (L.kp) {
        case 2: if constexpr (NLOG > 2) return run_decode_flags<NLOG, 2, RHO, V>(L); break;
        case 3: if constexpr (NLOG > 3) return run_decode_flags<NLOG, 3, RHO, V>(L); break;
        case 4: if constexpr (NLOG > 4) return run_decode_flags<NLOG, 4, RHO, V>(L); break;
        case 5: if constexpr (NLOG > 5) return run_decode_flags<NLOG, 5, RHO, V>(L); break;
        default: break;
    }
    return fail(PC_ENOTSUP, "permuted range k must be 2..5 or n in this library");
}

// V: kernel family (DecodeLaunch::variant)
template <int NLOG, int V>
int run_decode_n(const DecodeLaunch &L) {
    if constexpr (NLOG == 1) {
        return run_decode_kp<1, 1, V>(L);
    } else {
        if (L.rho == 3) {
            if constexpr (NLOG >= 3 && V == 0) return run_decode_kp<NLOG, 3, V>(L);
            return fail(V ? PC_ENOTSUP : PC_EINVAL,
                        V ? "decision history, exact boxplus and noise injection are built for rho 2"
                          : "rho exceeds log2 N");
        }
        if (L.rho != 2) return fail(PC_EINVAL, "rho must be 2 or 3");
        return run_decode_kp<NLOG, 2, V>(L);
    }
}

}  // namespace pbp

namespace pbp {
// dispatch on log2 N to the per-length translation units
int launch_decode_n(int n, const DecodeLaunch &L);
}  // namespace pbp
