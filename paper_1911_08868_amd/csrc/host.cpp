// host.cpp -- C ABI of the polarbp library: code construction, tables,
// argument validation and kernel dispatch.  Compiled by hipcc for gfx950.
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <numeric>

#include "decode_inst.h"
#include "internal.h"

namespace pbp {

// ---------------------------------------------------------------------------
// errors
static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

int fail(int rc, const std::string &msg) {
    set_error(msg);
    return rc;
}

int hip_fail(hipError_t e, const char *what) {
    set_error(std::string(what) + ": " + hipGetErrorString(e));
    return PC_EHIP;
}

// ---------------------------------------------------------------------------
// device helpers
int device_cu_count() {
    static int cached[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (cached[dev] == 0) {
        int cu = 0;
        if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            cu <= 0)
            cu = 256;
        cached[dev] = cu;
    }
    return cached[dev];
}

// Library-owned queue counters, per device: blocks of kBlockLines 64-byte
// lines (one counter per line).  An eager call takes the next block of a
// ring of kRing blocks and resets it with a kernel on its own stream before
// its decode launch, so eager calls in flight on different streams use
// different counters unless more than kRing of them overlap.  A call made
// while its stream is being captured into a HIP graph takes a block that is
// never handed out again: the graph may be replayed at any time, beside any
// later eager call or another graph.  Both regions are allocated by the first
// call on the device (which must not be under capture).
static constexpr int kRing = 1024, kHeld = 1024, kBlockLines = 16;

__global__ void k_reset_queues(uint32_t *c, int k) {
    if ((int)threadIdx.x < k) c[16 * threadIdx.x] = 0u;
}

uint32_t *counter_block(int device, hipStream_t stream) {
    static std::mutex mu;
    static uint32_t *base[64] = {nullptr};
    static unsigned ring_pos[64] = {0}, held_used[64] = {0};
    if (device < 0 || device >= 64) {
        set_error("device index out of range");
        return nullptr;
    }
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(stream, &cs) != hipSuccess) cs = hipStreamCaptureStatusNone;
    const bool capturing = cs == hipStreamCaptureStatusActive;
    std::lock_guard<std::mutex> lk(mu);
    if (!base[device]) {
        if (capturing) {
            set_error("the first decode call on a device must not be captured (it allocates the queue counters)");
            return nullptr;
        }
        void *p = nullptr;
        if (hipMalloc(&p, (size_t)(kRing + kHeld) * kBlockLines * 64) != hipSuccess) {
            set_error("queue counter allocation");
            return nullptr;
        }
        base[device] = static_cast<uint32_t *>(p);
    }
    size_t blk;
    if (capturing) {
        if (held_used[device] >= (unsigned)kHeld) {
            set_error("more than 1024 captured decode calls on this device (each keeps its counters)");
            return nullptr;
        }
        blk = kRing + held_used[device]++;
    } else {
        blk = ring_pos[device]++ % kRing;
    }
    return base[device] + blk * kBlockLines * 16;
}

// ---------------------------------------------------------------------------
// SplitMix64 (Steele, Lea, Flood 2014) and the trellis pool.
static uint64_t splitmix64(uint64_t &s) {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static uint32_t below(uint64_t &s, uint32_t m) {
    return (uint32_t)(((splitmix64(s) >> 32) * (uint64_t)m) >> 32);
}

// Pool of stage orders for the fixed multi-trellis schedules: entry 0 is the
// original graph; entries 1.. give the last k stages distinct non-identity
// orders of bits n-k..n-1, each a Fisher-Yates shuffle of the identity
// (position from k-1 down to 1 swapped with a uniform position at or below
// it); an identity or repeated draw is drawn again.
int make_pool(int n, int k, int Q, uint64_t seed, int8_t *orders) {
    if (n < 1 || n > kMaxLog || k < 0 || k > n || Q < 1 || Q > kMaxPool || !orders)
        return fail(PC_EINVAL, "pool parameters out of range");
    int64_t fact = 1;
    for (int i = 2; i <= k && fact < Q; ++i) fact *= i;
    const int qeff = (int)std::min<int64_t>(Q, fact);
    uint64_t st = seed;
    for (int s = 0; s < n; ++s) orders[s] = (int8_t)s;
    int8_t cand[kMaxLog];
    for (int q = 1; q < qeff; ++q) {
        for (;;) {
            for (int i = 0; i < k; ++i) cand[i] = (int8_t)(n - k + i);
            for (int i = k - 1; i >= 1; --i) {
                const uint32_t j = below(st, (uint32_t)(i + 1));
                std::swap(cand[i], cand[j]);
            }
            bool ident = true;
            for (int i = 0; i < k; ++i) ident &= cand[i] == n - k + i;
            if (ident) continue;
            bool dup = false;
            for (int p = 1; p < q && !dup; ++p)
                dup = std::equal(cand, cand + k, orders + p * n + (n - k));
            if (dup) continue;
            break;
        }
        for (int s = 0; s < n - k; ++s) orders[q * n + s] = (int8_t)s;
        for (int i = 0; i < k; ++i) orders[q * n + n - k + i] = cand[i];
    }
    return qeff;
}

// ---------------------------------------------------------------------------
// Construction (Sec. II-A).  Successive cancellation on this factor graph
// (level 1 = channel, stage s pairing rows 2^(s-1) apart) combines last on
// the most significant bit, so bit channel i is reached from z0 by one
// polarising step per bit of i, least significant bit first: bit 0 degrades
// (2z - z^2), bit 1 upgrades (z^2).  ln z, z0 = exp(-(K/N) Eb/N0).
static void construct_info(int N, int K, double ebn0_db, std::vector<int32_t> &info) {
    int n = 0;
    while ((1 << n) < N) ++n;
    const double lz0 = -((double)K / N) * std::pow(10.0, ebn0_db / 10.0);
    std::vector<double> lz(N);
    for (int i = 0; i < N; ++i) {
        double v = lz0;
        for (int b = 0; b < n; ++b) v = ((i >> b) & 1) ? 2.0 * v : v + std::log1p(-std::expm1(v));
        lz[i] = v;
    }
    std::vector<int32_t> idx(N);
    std::iota(idx.begin(), idx.end(), 0);
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) {
        if (lz[a] != lz[b]) return lz[a] < lz[b];
        return a > b;  // ties: larger index is taken first
    });
    info.assign(idx.begin(), idx.begin() + K);
    std::sort(info.begin(), info.end());
}

// CRC contribution of each message position: the CRC of the unit message
// e_i.  With init 0 and no final xor the CRC is linear; the register after a
// single 1 is the generator, and every further zero bit is one more shift, so
// crc(e_i) = step^(K_msg-1-i)(g).
static void crc_unit_table(int kmsg, int width, uint32_t poly, std::vector<uint32_t> &tab) {
    tab.assign(kmsg, 0u);
    if (width <= 0 || kmsg <= 0) return;
    const uint32_t mask = width == 32 ? 0xFFFFFFFFu : ((1u << width) - 1u);
    const uint32_t g = poly & mask;
    uint32_t r = g;
    for (int i = kmsg - 1; i >= 0; --i) {
        tab[i] = r;
        const uint32_t top = (r >> (width - 1)) & 1u;
        r = (r << 1) & mask;
        if (top) r ^= g;
    }
}

template <class T>
static int upload(T **dst, const std::vector<T> &src) {
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, std::max<size_t>(1, src.size()) * sizeof(T));
    if (e != hipSuccess) return hip_fail(e, "device table allocation");
    if (!src.empty()) {
        e = hipMemcpy(p, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            (void)hipFree(p);
            return hip_fail(e, "device table upload");
        }
    }
    *dst = static_cast<T *>(p);
    return PC_OK;
}

static void free_tables(pc_code *c) {
    if (c->d.syn) (void)hipFree(c->d.syn);
    if (c->d.meta) (void)hipFree(c->d.meta);
    if (c->d.info) (void)hipFree(c->d.info);
    if (c->d.crc_of_msg_bit) (void)hipFree(c->d.crc_of_msg_bit);
    c->d = DeviceTables{};
}

}  // namespace pbp

using namespace pbp;

// ---------------------------------------------------------------------------
extern "C" {

const char *polar_strerror(int rc) {
    switch (rc) {
        case PC_OK: return "success";
        case PC_EINVAL: return "invalid argument";
        case PC_ENOTSUP: return "not supported by this library";
        case PC_EHIP: return "HIP runtime error";
        case PC_ENOMEM: return "out of memory or workspace too small";
        default: return "unknown error";
    }
}

const char *polar_last_error(void) { return g_last_error.c_str(); }

int polar_construct(int32_t N, int32_t K, int32_t crc_width, uint32_t crc_poly,
                    double design_ebn0_db, pc_code **out) {
    if (!out) return fail(PC_EINVAL, "out is NULL");
    *out = nullptr;
    if (N < 2 || N > kMaxN || (N & (N - 1))) return fail(PC_EINVAL, "N must be a power of two in [2, 4096]");
    if (crc_width < 0 || crc_width > 32) return fail(PC_EINVAL, "crc_width must be 0..32");
    if (K < 1 || K > N || crc_width >= K) return fail(PC_EINVAL, "need 1 <= K <= N and crc_width < K");
    if (!std::isfinite(design_ebn0_db) && !(std::isinf(design_ebn0_db) && design_ebn0_db < 0))
        return fail(PC_EINVAL, "design Eb/N0 must be finite or -inf");
    pc_code *c = new (std::nothrow) pc_code();
    if (!c) return fail(PC_ENOMEM, "host allocation");
    c->N = N;
    while ((1 << c->n) < N) c->n++;
    c->K = K;
    c->crc_width = crc_width;
    c->crc_poly = crc_poly;
    c->K_msg = K - crc_width;
    if (hipGetDevice(&c->device) != hipSuccess) c->device = 0;
    construct_info(N, K, design_ebn0_db, c->info);
    c->frozen.assign(N, 1);
    for (int32_t j : c->info) c->frozen[j] = 0;
    crc_unit_table(c->K_msg, crc_width, crc_poly, c->crc_of_msg_bit);
    c->syn.assign(N, 0u);
    c->meta.assign(N, -2);
    for (int i = 0; i < K; ++i) {
        const int j = c->info[i];
        if (i < c->K_msg) {
            c->meta[j] = i;
            c->syn[j] = crc_width ? c->crc_of_msg_bit[i] : 0u;
        } else {
            c->meta[j] = -1;
            c->syn[j] = 1u << (crc_width - 1 - (i - c->K_msg));
        }
    }
    int rc = upload(&c->d.syn, c->syn);
    if (!rc) rc = upload(&c->d.meta, c->meta);
    if (!rc) rc = upload(&c->d.info, c->info);
    if (!rc) rc = upload(&c->d.crc_of_msg_bit, c->crc_of_msg_bit);
    if (rc) {
        free_tables(c);
        delete c;
        return rc;
    }
    // per-device set-up of the allocation-free batched entry point: the
    // address of this device's scratch (a failure here is reported by that
    // entry point, which resolves it again)
    (void)noalloc_scratch_init();
    *out = c;
    return PC_OK;
}

int polar_code_free(pc_code *code) {
    if (!code) return PC_OK;
    free_tables(code);
    delete code;
    return PC_OK;
}

int polar_code_query(const pc_code *code, int32_t *info_idx, uint8_t *frozen) {
    if (!code) return fail(PC_EINVAL, "code is NULL");
    if (info_idx) std::memcpy(info_idx, code->info.data(), code->info.size() * sizeof(int32_t));
    if (frozen) std::memcpy(frozen, code->frozen.data(), code->frozen.size());
    return PC_OK;
}

int polar_trellis_pool(int32_t n, int32_t k, int32_t Q, uint64_t seed, int8_t *orders) {
    return make_pool(n, k, Q, seed, orders);
}

int polar_encode(const pc_code *code, const uint8_t *d_msg, uint8_t *d_x, int64_t F, void *stream) {
    if (!code) return fail(PC_EINVAL, "code is NULL");
    if (F < 0) return fail(PC_EINVAL, "F < 0");
    if (F == 0) return PC_OK;
    if (!d_msg || !d_x) return fail(PC_EINVAL, "null buffer");
    return launch_encode(code, d_msg, d_x, nullptr, F, static_cast<hipStream_t>(stream));
}

int polar_info_bits(const pc_code *code, const uint8_t *d_msg, uint8_t *d_u_info, int64_t F,
                    void *stream) {
    if (!code) return fail(PC_EINVAL, "code is NULL");
    if (F < 0) return fail(PC_EINVAL, "F < 0");
    if (F == 0) return PC_OK;
    if (!d_msg || !d_u_info) return fail(PC_EINVAL, "null buffer");
    return launch_encode(code, d_msg, nullptr, d_u_info, F, static_cast<hipStream_t>(stream));
}

static int check_bp(const pc_code *code, const pc_bp_params *bp) {
    if (!bp) return fail(PC_EINVAL, "bp params are NULL");
    if (bp->max_iter < 1) return fail(PC_EINVAL, "max_iter must be >= 1");
    if (bp->it_min < 1) return fail(PC_EINVAL, "it_min must be >= 1");
    if (bp->stop < PC_STOP_NONE || bp->stop > PC_STOP_CRC) return fail(PC_EINVAL, "unknown stop test");
    if (bp->stop == PC_STOP_CRC && code->crc_width == 0) return fail(PC_EINVAL, "CRC stop on a code without CRC");
    if (!(bp->alpha > 0.f) || !std::isfinite(bp->alpha)) return fail(PC_EINVAL, "alpha must be finite and > 0");
    if (bp->check != PC_CHECK_MINSUM && bp->check != PC_CHECK_EXACT) return fail(PC_EINVAL, "unknown check function");
    if (bp->check == PC_CHECK_EXACT && bp->alpha != 1.0f) return fail(PC_EINVAL, "the exact boxplus takes no scale (alpha = 1)");
    return PC_OK;
}

static int decode_common(const pc_code *code, const float *d_llr, int64_t F, const pc_bp_params *bp,
                         const pc_pp_params *pp, uint8_t *d_msg, int32_t *d_iters, uint8_t *d_ok,
                         float *d_soft, const pc_launch_cfg *cfg, void *stream,
                         uint64_t *d_hist = nullptr, int32_t H = 0) {
    if (!code) return fail(PC_EINVAL, "code is NULL");
    if (F < 0 || F > INT32_MAX) return fail(PC_EINVAL, "F must be in [0, 2^31)");
    int rc = check_bp(code, bp);
    if (rc) return rc;
    if (F == 0) return PC_OK;
    if (!d_llr || !d_msg) return fail(PC_EINVAL, "null buffer");
    if (reinterpret_cast<uintptr_t>(d_llr) % 4) return fail(PC_EINVAL, "LLR pointer not 4-byte aligned");
    int mode = pp ? pp->mode : PC_PP_NONE;
    int kp = 0, T = 1, Q = 1;
    int8_t orders[kMaxPool * kMaxLog] = {0};
    const int n = code->n;
    const bool exact = bp->check == PC_CHECK_EXACT;
    if (exact && d_hist) return fail(PC_ENOTSUP, "the decision history is built for min-sum");
    const float sigma = pp ? pp->noise_sigma : 0.f;
    if (!(sigma >= 0.f) || !std::isfinite(sigma)) return fail(PC_EINVAL, "noise_sigma must be finite and >= 0");
    if (sigma > 0.f) {
        if (mode != PC_PP_LASTK && mode != PC_PP_FULL && mode != PC_PP_ALG1 && mode != PC_PP_ALG1_ORIG)
            return fail(PC_EINVAL, "noise is injected at the trellis events (LASTK, FULL, ALG1, ALG1_ORIG)");
        if (exact || d_hist) return fail(PC_ENOTSUP, "noise injection is built for min-sum without history");
    }
    if (mode == PC_PP_ALG1 || mode == PC_PP_ALG1_ORIG) {
        if (cfg && (cfg->rho || cfg->slots || cfg->grid))
            return fail(PC_EINVAL, "Algorithm 1 takes no launch shape (one frame per workgroup)");
        return launch_alg1(code, d_llr, F, *bp, *pp, d_msg, d_iters, d_ok, d_soft, d_hist, H,
                           static_cast<hipStream_t>(stream));
    }
    if (mode != PC_PP_NONE && mode != PC_PP_LASTK && mode != PC_PP_FULL)
        return fail(PC_EINVAL, "unknown multi-trellis mode");
    if (mode == PC_PP_LASTK || mode == PC_PP_FULL) {
        kp = (mode == PC_PP_FULL) ? n : pp->k;
        if (kp < 2 || kp > n) return fail(PC_EINVAL, "k must satisfy 2 <= k <= n");
        if (pp->period_T < 1) return fail(PC_EINVAL, "period T must be >= 1");
        if (pp->pool_Q < 1 || pp->pool_Q > kMaxPool) return fail(PC_EINVAL, "pool Q must be 1..8");
        T = pp->period_T;
        Q = make_pool(n, kp, pp->pool_Q, pp->seed, orders);
        if (Q < 0) return Q;
        if (Q == 1) kp = 0;  // the identity pool is the original graph
    } else {
        for (int s = 0; s < n; ++s) orders[s] = (int8_t)s;
    }
    hipStream_t hs = static_cast<hipStream_t>(stream);
    uint32_t *ctr = counter_block(code->device, hs);
    if (!ctr) return PC_ENOMEM;
    hipLaunchKernelGGL(k_reset_queues, dim3(1), dim3(64), 0, hs, ctr, kQueues);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "counter reset launch");

    DecodeLaunch L;
    DecodeArgs &a = L.args;
    std::memset(&a, 0, sizeof(a));
    a.llr = d_llr;
    a.F = F;
    a.msg = d_msg;
    a.iters = d_iters;
    a.ok = d_ok;
    a.soft = d_soft;
    a.syn = code->d.syn;
    a.meta = code->d.meta;
    a.counter = ctr;
    a.K_msg = code->K_msg;
    a.max_iter = bp->max_iter;
    a.it_min = bp->it_min;
    a.stop = bp->stop;
    a.alpha = bp->alpha;
    a.T = T;
    a.Q = Q;
    a.hist = d_hist;
    a.H = H;
    for (int q = 0; q < Q; ++q)
        for (int s = 0; s < n; ++s) a.orders[q][s] = orders[q * n + s];
    L.kp = kp;
    L.variant = d_hist ? 1 : exact ? 2 : sigma > 0.f ? 3 : 0;
    a.noise_sigma = sigma;
    a.noise_seed = pp ? pp->seed : 0;
    L.scaled = bp->alpha != 1.0f;
    L.gmode = bp->stop == PC_STOP_G || (bp->stop == PC_STOP_NONE && code->crc_width == 0);
    L.F = F;
    L.stream = hs;
    // default shape: two rows per thread, except N = 512 and 4096, where
    // eight rows per thread measured faster (one-wave frames at 512); the
    // side kernel families are built for two rows only
    L.rho = cfg && cfg->rho ? cfg->rho : (L.variant == 0 && (n == 9 || n == 12)) ? 3 : (n >= 2 ? 2 : 1);
    L.slots = cfg ? cfg->slots : 0;
    L.grid = cfg ? cfg->grid : 0;
    return launch_decode_n(n, L);
}

int bp_decode(const pc_code *code, const float *d_llr, int64_t F, const pc_bp_params *bp,
              uint8_t *d_msg_hat, int32_t *d_iters, uint8_t *d_ok, void *stream) {
    return decode_common(code, d_llr, F, bp, nullptr, d_msg_hat, d_iters, d_ok, nullptr, nullptr,
                         stream);
}

int pp_mt_bp_decode(const pc_code *code, const float *d_llr, int64_t F, const pc_bp_params *bp,
                    const pc_pp_params *pp, uint8_t *d_msg_hat, int32_t *d_iters, uint8_t *d_ok,
                    void *stream) {
    return decode_common(code, d_llr, F, bp, pp, d_msg_hat, d_iters, d_ok, nullptr, nullptr, stream);
}

int pp_mt_bp_decode_ex(const pc_code *code, const float *d_llr, int64_t F,
                       const pc_bp_params *bp, const pc_pp_params *pp, uint8_t *d_msg_hat,
                       int32_t *d_iters, uint8_t *d_ok, float *d_soft_u,
                       const pc_launch_cfg *cfg, void *stream) {
    return decode_common(code, d_llr, F, bp, pp, d_msg_hat, d_iters, d_ok, d_soft_u, cfg, stream);
}

int pp_mt_bp_decode_trace(const pc_code *code, const float *d_llr, int64_t F, const pc_bp_params *bp,
                          const pc_pp_params *pp, uint8_t *d_msg_hat, int32_t *d_iters, uint8_t *d_ok,
                          uint64_t *d_hist, int32_t H, void *stream) {
    if (H < 1 || H > 64) return fail(PC_EINVAL, "history length H must be 1..64");
    if (F > 0 && !d_hist) return fail(PC_EINVAL, "null history buffer");
    if (F > 0 && reinterpret_cast<uintptr_t>(d_hist) % 8) return fail(PC_EINVAL, "history pointer not 8-byte aligned");
    return decode_common(code, d_llr, F, bp, pp, d_msg_hat, d_iters, d_ok, nullptr, nullptr, stream,
                         d_hist, H);
}

int polar_classify_errors(const uint8_t *d_msg_hat, const uint8_t *d_msg, const uint8_t *d_ok,
                          const int32_t *d_iters, const uint64_t *d_hist, int32_t H, int64_t F,
                          int32_t K_msg, uint8_t *d_class, int32_t *d_period, void *stream) {
    if (F < 0 || F > INT32_MAX) return fail(PC_EINVAL, "F must be in [0, 2^31)");
    if (H < 1 || H > 64) return fail(PC_EINVAL, "history length H must be 1..64");
    if (K_msg < 1) return fail(PC_EINVAL, "K_msg must be >= 1");
    if (F == 0) return PC_OK;
    if (!d_msg_hat || !d_msg || !d_ok || !d_iters || !d_hist || !d_class)
        return fail(PC_EINVAL, "null buffer");
    if (reinterpret_cast<uintptr_t>(d_hist) % 8 || reinterpret_cast<uintptr_t>(d_iters) % 4 ||
        reinterpret_cast<uintptr_t>(d_period) % 4)
        return fail(PC_EINVAL, "misaligned history, iteration or period buffer");
    return launch_classify(d_msg_hat, d_msg, d_ok, d_iters, d_hist, H, F, K_msg, d_class, d_period,
                           static_cast<hipStream_t>(stream));
}

}  // extern "C"
