// diag.hip -- error classes of decoded frames (Sec. II-C) from the decided
// and transmitted messages, the stop verdict and the decision-hash history
// that the trace decoders record.
//
// One wave per frame: its lanes compare the message bytes, and lane p-1
// tests whether the last W = min(H, iters) hashes repeat with period p
// (h_i = h_{i+p} for i = 1..W-p, p <= W/2); the smallest such p is the
// frame's decision period (0 if none).  Classes: 0 correct (message equal),
// 1 false converged (wrong, and accepted by the stop test or stationary,
// p = 1), 2 oscillation (wrong, not accepted, p >= 2), 3 unconverged (the
// rest).
#include "bp_core.h"
#include "internal.h"

namespace pbp {

__global__ void __launch_bounds__(256) k_classify(const uint8_t *msg_hat, const uint8_t *msg,
                                                  const uint8_t *ok, const int32_t *iters,
                                                  const uint64_t *hist, int32_t H, int64_t F,
                                                  int32_t K_msg, uint8_t *cls, int32_t *period) {
    const int lane = threadIdx.x & 63;
    const int64_t f = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (f >= F) return;  // uniform over the wave
    const uint8_t *a = msg_hat + f * K_msg, *b = msg + f * K_msg;
    bool diff = false;
    for (int i = lane; i < K_msg; i += 64) diff |= a[i] != b[i];
    const bool wrong = __ballot(diff) != 0ull;
    const int it = iters[f];
    const int W = it < H ? it : H;
    const uint64_t *h = hist + f * H;
    // hash number i (0 = oldest of the window) sits at (it - W + i) mod H
    auto at = [&](int i) { return h[(it - W + i) % H]; };
    const int p = lane + 1;
    bool periodic = false;
    if (W > 0 && 2 * p <= W) {
        periodic = true;
        for (int i = 0; i + p < W && periodic; ++i) periodic = at(i) == at(i + p);
    }
    const uint64_t m = __ballot(periodic);
    if (lane == 0) {
        const int per = m ? __ffsll((long long)m) : 0;
        uint8_t c;
        if (!wrong) c = 0;
        else if (ok[f] || per == 1) c = 1;
        else if (per >= 2) c = 2;
        else c = 3;
        cls[f] = c;
        if (period) period[f] = per;
    }
}

int launch_classify(const uint8_t *d_msg_hat, const uint8_t *d_msg, const uint8_t *d_ok,
                    const int32_t *d_iters, const uint64_t *d_hist, int32_t H, int64_t F,
                    int32_t K_msg, uint8_t *d_class, int32_t *d_period, hipStream_t s) {
    constexpr int kFramesPerBlock = 4;  // one wave each
    const int64_t grid = (F + kFramesPerBlock - 1) / kFramesPerBlock;
    hipLaunchKernelGGL(k_classify, dim3((unsigned)grid), dim3(64 * kFramesPerBlock), 0, s, d_msg_hat,
                       d_msg, d_ok, d_iters, d_hist, H, F, K_msg, d_class, d_period);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? PC_OK : hip_fail(e, "classification launch");
}

}  // namespace pbp
