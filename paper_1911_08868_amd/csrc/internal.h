// internal.h -- shared declarations of the polarbp library (host side).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/polarbp.h"

namespace pbp {

constexpr int kMaxN = 4096;
constexpr int kMaxLog = 12;
constexpr int kMaxPool = 8;

// Device-side per-row tables of one code.  meta[j]: >= 0 message index of
// row j, -1 CRC position, -2 frozen.  syn[j]: CRC syndrome contribution of a
// decided 1 at row j (0 for frozen rows); the syndrome of a decision vector
// is the xor of syn over its ones and is 0 exactly when the CRC matches.
struct DeviceTables {
    uint32_t *syn = nullptr;
    int32_t *meta = nullptr;
    int32_t *info = nullptr;   // K information rows, ascending
    uint32_t *crc_of_msg_bit = nullptr;  // [K_msg] CRC of the unit message e_i
};

}  // namespace pbp

struct pc_code {
    int32_t N = 0, n = 0, K = 0, crc_width = 0, K_msg = 0;
    uint32_t crc_poly = 0;
    int device = 0;
    std::vector<int32_t> info;
    std::vector<uint8_t> frozen;
    std::vector<uint32_t> syn;
    std::vector<int32_t> meta;
    std::vector<uint32_t> crc_of_msg_bit;
    pbp::DeviceTables d;
};

namespace pbp {

void set_error(const std::string &msg);
int fail(int rc, const std::string &msg);
int hip_fail(hipError_t e, const char *what);

// trellis pool (SplitMix64 + Fisher-Yates); returns number of entries
int make_pool(int n, int k, int Q, uint64_t seed, int8_t *orders);

// number of compute units of the current device (cached)
int device_cu_count();

// per-call queue counters (16 lines of 64 bytes, one counter per line) from
// library-owned device memory: a recycled ring for eager calls, a block kept
// for good for a call under graph capture; NULL (error set) on failure
uint32_t *counter_block(int device, hipStream_t stream);
__global__ void k_reset_queues(uint32_t *c, int k);

// ---- decode ----------------------------------------------------------------
struct DecodeConfig {
    int n = 0, kp = 0;         // log2 N, permuted stages (0 = none)
    bool scaled = false;       // alpha != 1
    bool gmode = false;        // G-matrix test machinery
    int rho = 2, slots = 1, grid = 0;
};

int launch_decode(const pc_code *code, const float *d_llr, int64_t F, const pc_bp_params &bp,
                  int pp_mode, int kp, int T, int Q, const int8_t *orders, uint8_t *d_msg,
                  int32_t *d_iters, uint8_t *d_ok, float *d_soft, const pc_launch_cfg *cfg,
                  hipStream_t stream);

// x = u G_N into d_x (or NULL), and u on the information rows into d_ua
// [F][K] (or NULL)
int launch_encode(const pc_code *code, const uint8_t *d_msg, uint8_t *d_x, uint8_t *d_ua, int64_t F,
                  hipStream_t stream);

// Algorithm 1 with random subgraphs (per-row stage orders, messages in LDS)
int launch_alg1(const pc_code *code, const float *d_llr, int64_t F, const pc_bp_params &bp,
                const pc_pp_params &pp, uint8_t *d_msg, int32_t *d_iters, uint8_t *d_ok, float *d_soft,
                uint64_t *d_hist, int32_t H, hipStream_t stream);

// error classes from the decision history (one wave per frame)
int launch_classify(const uint8_t *d_msg_hat, const uint8_t *d_msg, const uint8_t *d_ok,
                    const int32_t *d_iters, const uint64_t *d_hist, int32_t H, int64_t F,
                    int32_t K_msg, uint8_t *d_class, int32_t *d_period, hipStream_t stream);

size_t batched_ws_bytes(int64_t F);
// resolve the current device's copy of the allocation-free entry point's
// scratch (batched.hip); PC_OK or PC_EHIP
int noalloc_scratch_init();

size_t wbp_ws_bytes(const pc_code *code, int64_t F, int T);
int launch_wbp_forward(const pc_code *code, const float *d_llr, int64_t F, const float *d_w,
                       int T, int kp, int Tev, int Q, const int8_t *orders, float *d_out,
                       void *d_ws, size_t ws_bytes, hipStream_t stream);
int launch_wbp_backward(const pc_code *code, const float *d_llr, int64_t F, const float *d_w,
                        int T, int kp, int Tev, int Q, const int8_t *orders,
                        const float *d_gout, float *d_gw, void *d_ws, size_t ws_bytes,
                        hipStream_t stream);

}  // namespace pbp
