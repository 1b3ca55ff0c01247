// wbp_inst.h -- launches of the weighted-BP kernels for one block length.
#pragma once

#include "internal.h"
#include "wbp_kernel.h"

namespace pbp {

struct WbpLaunch {
    WbpArgs args;
    int kp = 0;
    bool backward = false;
    int slots = 0, bslots = 0, grid = 0, bgrid = 0;
    hipStream_t stream = nullptr;
};

// frames per workgroup of the weighted forward for block length 2^n
inline int wbp_slots(int n) {
    const int tps = 1 << (n - 2);
    return tps >= 256 ? 1 : 256 / tps;
}
// and of the adjoint (wbp_bwd_slots in wbp_kernel.h, two rows per thread)
inline int wbp_bwd_slots_n(int n) {
    const int tps = 1 << (n - 2);
    return tps <= 64 ? 512 / tps : wbp_slots(n);
}

// Block lengths from 2^kWbpBigLog on (wbp_kernel.h) run the adjoint with its
// arrays in a per-workgroup scratch (k_wbp_bwd_big) on a persistent grid of
// this many workgroups (one per CU at N = 4096, two at N = 2048); fixed, so
// that the order of the gradient sums does not depend on the device.
inline int wbp_big_grid(int n) { return n >= 12 ? 256 : 512; }
// Below that the adjoint's grid is fixed too: as many workgroups as the chip
// holds at once at N <= 256 (one per CU: their frames fill its LDS) and twice
// that above; each walks batches of its slot count, adding into its partial.
inline int wbp_small_grid(int n) { return n <= 8 ? 256 : 512; }
size_t wbp_big_scratch_floats(int n);

template <int NLOG, int KP>
int run_wbp(const WbpLaunch &L) {
    using P = Plan<NLOG, KP, 2>;
    const int S = L.backward ? L.bslots : L.slots;
    if (L.backward && NLOG < kWbpBigLog && S != wbp_bwd_slots<NLOG, 2>())
        return fail(PC_EINVAL, "adjoint slot count does not match the kernel");
    const size_t lds = L.backward && NLOG < kWbpBigLog ? WbpLds<P, true>::bytes(S) : WbpLds<P, false>::bytes(S);
    if (lds > 160 * 1024) return fail(PC_EINVAL, "LDS budget exceeded for weighted BP");
    if (L.backward) {
        if constexpr (NLOG >= kWbpBigLog) {
            constexpr size_t big_lds = BigLds<P>::bytes;
            static_assert(big_lds <= 160 * 1024, "large-frame adjoint exceeds the LDS");
            hipLaunchKernelGGL((k_wbp_bwd_big<NLOG, KP>), dim3(L.grid), dim3(P::TPS), big_lds, L.stream, L.args);
        } else {
            hipLaunchKernelGGL((k_wbp_bwd<NLOG, KP, 2>), dim3(L.grid), dim3(S * P::TPS), lds, L.stream, L.args);
        }
    } else
        hipLaunchKernelGGL((k_wbp_fwd<NLOG, KP, 2>), dim3(L.grid), dim3(S * P::TPS), lds, L.stream, L.args);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "weighted BP launch");
    return PC_OK;
}

template <int NLOG>
int run_wbp_n(const WbpLaunch &L) {
    switch (L.kp) {
        case 0: return run_wbp<NLOG, 0>(L);
        case 2: if constexpr (NLOG > 2) return run_wbp<NLOG, 2>(L); break;
        case 3: if constexpr (NLOG > 3) return run_wbp<NLOG, 3>(L); break;
        case 4: if constexpr (NLOG > 4) return run_wbp<NLOG, 4>(L); break;
        case 5: if constexpr (NLOG > 5) return run_wbp<NLOG, 5>(L); break;
        default: break;
    }
    return fail(PC_ENOTSUP, "weighted BP supports permuted ranges k = 2..5 below n");
}

int launch_wbp_n(int n, const WbpLaunch &L);

}  // namespace pbp
