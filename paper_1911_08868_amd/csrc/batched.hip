// batched.hip -- mixed-length, mixed-rate PP-MT-BP decoding from a device
// work queue in one persistent launch.
//
// A round is five launches on the caller's stream, all device-side so the
// whole round can be captured in a HIP graph and replayed:
//   1. clear the queue counters in the workspace (a kernel, no memset node);
//   2. count the frames of each block length (n = 6..10);
//   3. lay out one contiguous frame list per length, longest codes first;
//   4. scatter frame indices into their lists;
//   5. the persistent decoder: each workgroup walks the lists from N = 1024
//      down to N = 64; for each length it runs the lock-step slot loop of
//      the single-code kernel, taking frames from that list with one atomic
//      per frame and reading each frame's own code tables, so frames of
//      different rates share a workgroup and a frame that stops early frees
//      its slot for the next one.  Longest codes go first so the short, cheap
//      frames fill the tail.
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <mutex>

#include "decode_kernel.h"
#include "internal.h"

namespace pbp {

constexpr int kBatchMaxCodes = 32;
constexpr int kBuckets = 5;  // n = 6 .. 10
constexpr int kBatchBlock = 256;

struct BatchCode {
    const uint32_t *syn;
    const int32_t *meta;
    int32_t n, K_msg;
};

struct BatchedArgs {
    BatchCode codes[kBatchMaxCodes];
    const int32_t *code_id;
    const int64_t *llr_off;
    const float *llr_pool;
    const int64_t *bits_off;
    uint8_t *bits_pool;
    int32_t *iters;
    uint8_t *ok;
    int64_t F;
    int32_t n_codes;
    int32_t *ctl;   // [0..4] counts, [8..12] starts, [16..20] cursors, [24..28] queue heads
    int32_t *list;  // [F]
    int32_t max_iter, it_min, stop;
    float alpha;
    int32_t T, Q;
    int8_t orders[kBuckets][8 * 16];
};

template <int N_>
struct BatchSrc {
    static constexpr bool kTrace = false;
    static constexpr bool kNoise = false;
    const BatchedArgs &a;
    int64_t F;
    int b, count, start;
    ChunkClaim<N_> claim;
    __device__ BatchSrc(const BatchedArgs &args, int bucket)
        : a(args), F(args.F), b(bucket), count(args.ctl[bucket]), start(args.ctl[8 + bucket]) {}
    __device__ int64_t pop() {
        const int64_t idx = claim.take(count, [&](int k) { return (int64_t)atomicAdd(&a.ctl[24 + b], k); });
        return idx < count ? (int64_t)a.list[start + idx] : F;
    }
    __device__ const float *llr(int64_t f) const { return a.llr_pool + a.llr_off[f]; }
    __device__ const uint32_t *syn(int64_t f) const { return a.codes[a.code_id[f]].syn; }
    __device__ const int32_t *meta(int64_t f) const { return a.codes[a.code_id[f]].meta; }
    __device__ uint8_t *msg(int64_t f) const { return a.bits_pool + a.bits_off[f]; }
    __device__ bool want_soft() const { return false; }
    __device__ void soft(int64_t, int, float) const {}
    __device__ void finish(int64_t f, int iters, bool pass) const {
        if (a.iters) a.iters[f] = iters;
        if (a.ok) a.ok[f] = pass ? 1 : 0;
    }
    __device__ void trace(int64_t, int, uint64_t) const {}
};

__global__ void k_batch_clear(int32_t *ctl) {
    if (threadIdx.x < 32) ctl[threadIdx.x] = 0;
}

// Bucket of frame f (code length 2^(6+b)), or -1 for a skipped frame.
__device__ __forceinline__ int frame_bucket(const BatchedArgs &a, int64_t f) {
    if (f >= a.F) return -1;
    const int c = a.code_id[f];
    return (c >= 0 && c < a.n_codes) ? a.codes[c].n - 6 : -1;
}

// The queue preparation aggregates per wave: one ballot per bucket and one
// atomic per bucket and wave instead of one per frame (a single address took
// one atomic per frame of a one-length stream, about 1e8 per second).  Every
// wave runs the same number of trips, so the ballots see all 64 lanes.
__global__ void __launch_bounds__(256) k_batch_count(BatchedArgs a) {
    const int lane = threadIdx.x & 63;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t f0 = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63); f0 < a.F; f0 += stride) {
        const int b = frame_bucket(a, f0 + lane);
        for (int k = 0; k < kBuckets; ++k) {
            const uint64_t m = __ballot(b == k);
            if (lane == 0 && m) atomicAdd(&a.ctl[k], (int)__popcll(m));
        }
    }
}

__global__ void k_batch_layout(int32_t *ctl) {
    if (threadIdx.x != 0) return;
    int start = 0;
    for (int b = kBuckets - 1; b >= 0; --b) {  // longest codes first
        ctl[8 + b] = start;
        ctl[16 + b] = start;
        ctl[24 + b] = 0;
        start += ctl[b];
    }
}

// Each wave reserves, per bucket, one range of the bucket's list for its
// frames of that bucket and writes them there in lane order.
__global__ void __launch_bounds__(256) k_batch_scatter(BatchedArgs a) {
    const int lane = threadIdx.x & 63;
    const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t f0 = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63); f0 < a.F; f0 += stride) {
        const int64_t f = f0 + lane;
        const int b = frame_bucket(a, f);
        for (int k = 0; k < kBuckets; ++k) {
            const uint64_t m = __ballot(b == k);
            if (!m) continue;
            int base = 0;
            if (lane == 0) base = atomicAdd(&a.ctl[16 + k], (int)__popcll(m));
            base = __shfl(base, 0, 64);
            if (b == k) a.list[base + (int)__popcll(m & below)] = (int32_t)f;
        }
    }
}

template <int NLOG, int KPQ, int RHO, bool SCALED>
__device__ __forceinline__ void run_bucket(const BatchedArgs &a, float *smem) {
    constexpr int KP = KPQ == 0 ? 0 : (KPQ < NLOG ? KPQ : NLOG - 1);
    constexpr int TPS = Plan<NLOG, KP, RHO>::TPS;
    const int S = blockDim.x / TPS;
    BatchSrc<(1 << NLOG)> src(a, NLOG - 6);
    DecodeCtl c{a.max_iter, a.it_min, a.stop, a.alpha, a.T, a.Q, a.orders[NLOG - 6]};
    // The thread index goes through an empty asm so that nothing derived
    // from it is shared with (and kept live across) the other lengths'
    // loops: each loop alone fits 128 VGPRs, all five together spilled.
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    decode_loop<NLOG, KP, RHO, SCALED, false>(src, c, smem, S, tid);
}

// MASK selects the buckets (bit b = length 2^(b+6)) this launch decodes, so
// that one length can run under another rho in a launch of its own.
template <int KPQ, int RHO, bool SCALED, int MASK>
__global__ void __launch_bounds__(512, (RHO <= 2 ? 4 : 2)) k_batched(BatchedArgs a) {
    extern __shared__ __align__(16) float smem[];
    for (int b = kBuckets - 1; b >= 0; --b) {
        if (!((MASK >> b) & 1) || a.ctl[b] == 0) continue;
        switch (b) {
            case 4: if constexpr ((MASK >> 4) & 1) run_bucket<10, KPQ, RHO, SCALED>(a, smem); break;
            case 3: if constexpr ((MASK >> 3) & 1) run_bucket<9, KPQ, RHO, SCALED>(a, smem); break;
            case 2: if constexpr ((MASK >> 2) & 1) run_bucket<8, KPQ, RHO, SCALED>(a, smem); break;
            case 1: if constexpr ((MASK >> 1) & 1) run_bucket<7, KPQ, RHO, SCALED>(a, smem); break;
            default: if constexpr (MASK & 1) run_bucket<6, KPQ, RHO, SCALED>(a, smem); break;
        }
        __syncthreads();
    }
}

template <int KPQ, int RHO, int MASK>
static size_t batched_lds(int block) {
    size_t m = 0;
    auto one = [&](auto P, int n) {
        using PP = decltype(P);
        if (!((MASK >> (n - 6)) & 1)) return;
        const int S = block / PP::TPS;
        m = std::max(m, DecodeLds<PP>::bytes(S < 1 ? 1 : S));
    };
    one(Plan<10, (KPQ == 0 ? 0 : (KPQ < 10 ? KPQ : 9)), RHO>{}, 10);
    one(Plan<9, (KPQ == 0 ? 0 : (KPQ < 9 ? KPQ : 8)), RHO>{}, 9);
    one(Plan<8, (KPQ == 0 ? 0 : (KPQ < 8 ? KPQ : 7)), RHO>{}, 8);
    one(Plan<7, (KPQ == 0 ? 0 : (KPQ < 7 ? KPQ : 6)), RHO>{}, 7);
    one(Plan<6, (KPQ == 0 ? 0 : (KPQ < 6 ? KPQ : 5)), RHO>{}, 6);
    return m;
}

template <int KPQ, int RHO, bool SC, int MASK>
static int launch_batched_kernel(const BatchedArgs &a, int block, int grid, hipStream_t s) {
    auto kern = k_batched<KPQ, RHO, SC, MASK>;
    const size_t lds = batched_lds<KPQ, RHO, MASK>(block);
    if (grid <= 0) {
        // occupancy is a property of the kernel and launch shape: cache it
        // (one cache per kernel instance)
        static std::mutex mu;
        static int cached[2] = {0, 0};
        const int bi = block == 512 ? 1 : 0;
        std::lock_guard<std::mutex> lk(mu);
        int &per_cu = cached[bi];
        if (per_cu == 0) {
            hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, block, lds);
            if (e != hipSuccess) return hip_fail(e, "occupancy query");
            if (per_cu < 1) per_cu = 1;
        }
        grid = per_cu * device_cu_count();
    }
    hipLaunchKernelGGL(kern, dim3(grid), dim3(block), lds, s, a);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? PC_OK : hip_fail(e, "batched decode launch");
}

// rho 2 or 3 decodes every length in one launch; rho 0 decodes the 512-bit
// frames under rho 3 in a launch of their own (at n = 9 rho 2 leaves half of
// each 128-thread slot's lanes to the two-slot lock step) and the other
// lengths under rho 2 in a second launch on the same stream.
template <int KPQ, bool SC>
static int launch_batched_rho(const BatchedArgs &a, int rho, int block, int grid, hipStream_t s) {
    if (rho == 2) return launch_batched_kernel<KPQ, 2, SC, 0x1f>(a, block, grid, s);
    if (rho == 3) return launch_batched_kernel<KPQ, 3, SC, 0x1f>(a, block, grid, s);
    const int r = launch_batched_kernel<KPQ, 3, SC, 0x08>(a, block, grid, s);
    if (r != PC_OK) return r;
    return launch_batched_kernel<KPQ, 2, SC, 0x17>(a, block, grid, s);
}

size_t batched_ws_bytes(int64_t F) { return 256 + (size_t)std::max<int64_t>(F, 1) * sizeof(int32_t); }

// Scratch of the allocation-free batched entry point: the queue control
// words and the frame list of one call, for at most kNoAllocMaxFrames frames
// (4 MiB + 256 bytes, held by every device the library runs on until the
// process ends).  Host code never passes `scratch` itself to a kernel: its
// name is a host-side stand-in, and the device address of each device's copy
// comes from hipGetSymbolAddress with that device current.
constexpr int64_t kNoAllocMaxFrames = int64_t(1) << 20;
constexpr size_t kNoAllocBytes = 256 + (size_t)kNoAllocMaxFrames * sizeof(int32_t);
static __device__ __align__(256) uint8_t scratch[kNoAllocBytes];

static std::mutex g_scratch_mu;
static void *g_scratch_ptr[64] = {nullptr};

// Resolve the current device's copy of the scratch (once per device).
// Called by polar_construct, and by the entry point if a call comes first on
// a device that constructed nothing.  Returns PC_OK or PC_EHIP.
int noalloc_scratch_init() {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= 64) return fail(PC_ENOTSUP, "device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[dev]) return PC_OK;
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!p) return fail(PC_EHIP, "hipGetSymbolAddress(scratch) gave NULL");
    g_scratch_ptr[dev] = p;
    return PC_OK;
}

static void *noalloc_scratch(int dev) {
    if (dev < 0 || dev >= 64) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch_ptr[dev];
}

}  // namespace pbp

using namespace pbp;

extern "C" {

size_t polar_batched_workspace_bytes(int64_t F) { return F < 0 ? 0 : batched_ws_bytes(F); }

}  // extern "C"

static int decode_batched_impl(const pc_code *const *codes, int32_t n_codes, const int32_t *d_code_id,
                               const int64_t *d_llr_off, const float *d_llr_pool, int64_t F,
                               const pc_bp_params *bp, const pc_pp_params *pp, uint8_t *d_bits_pool,
                               const int64_t *d_bits_off, int32_t *d_iters, uint8_t *d_ok, void *d_ws,
                               size_t ws_bytes, const pc_launch_cfg *cfg, void *stream) {
    if (!codes || n_codes < 1 || n_codes > kBatchMaxCodes) return fail(PC_EINVAL, "need 1..32 codes");
    if (!bp) return fail(PC_EINVAL, "bp params are NULL");
    if (F < 0 || F > INT32_MAX) return fail(PC_EINVAL, "F must be in [0, 2^31)");
    if (bp->max_iter < 1 || bp->it_min < 1) return fail(PC_EINVAL, "max_iter and it_min must be >= 1");
    if (bp->stop != PC_STOP_CRC && bp->stop != PC_STOP_NONE)
        return fail(PC_ENOTSUP, "batched decoding uses the CRC test (or none)");
    if (!(bp->alpha > 0.f) || !std::isfinite(bp->alpha)) return fail(PC_EINVAL, "alpha must be finite and > 0");
    if (bp->check != PC_CHECK_MINSUM) return fail(PC_ENOTSUP, "the batched decoder is built for min-sum");
    if (pp && pp->noise_sigma != 0.f) return fail(PC_ENOTSUP, "the batched decoder injects no noise");
    BatchedArgs a;
    std::memset(&a, 0, sizeof(a));
    for (int i = 0; i < n_codes; ++i) {
        const pc_code *c = codes[i];
        if (!c) return fail(PC_EINVAL, "null code");
        if (c->n < 6 || c->n > 10) return fail(PC_ENOTSUP, "batched codes must have N in [64, 1024]");
        if (c->crc_width == 0) return fail(PC_EINVAL, "batched codes need a CRC");
        a.codes[i] = BatchCode{c->d.syn, c->d.meta, c->n, c->K_msg};
    }
    if (F == 0) return PC_OK;
    if (!d_code_id || !d_llr_off || !d_llr_pool || !d_bits_pool || !d_bits_off)
        return fail(PC_EINVAL, "null buffer");
    if (!d_ws || ws_bytes < batched_ws_bytes(F)) return fail(PC_ENOMEM, "workspace too small");
    int kq = 0;
    if (pp && pp->mode != PC_PP_NONE) {
        if (pp->mode != PC_PP_LASTK) return fail(PC_ENOTSUP, "batched decoding uses the fixed last-k schedule");
        if (pp->k != 4) return fail(PC_ENOTSUP, "batched decoding is built for k = 4 (k = n-1 when n <= 4)");
        if (pp->period_T < 1 || pp->pool_Q < 1 || pp->pool_Q > kMaxPool)
            return fail(PC_EINVAL, "period T >= 1 and pool Q in 1..8");
        kq = 4;
        a.T = pp->period_T;
        int qq = 0;
        for (int b = 0; b < kBuckets; ++b) {
            const int n = b + 6;
            int8_t ord[kMaxPool * kMaxLog];
            const int q = make_pool(n, std::min(4, n - 1), pp->pool_Q, pp->seed, ord);
            if (q < 0) return q;
            qq = q;
            for (int p = 0; p < q; ++p)
                for (int s = 0; s < n; ++s) a.orders[b][p * 16 + s] = ord[p * n + s];
        }
        a.Q = qq;
    } else {
        a.T = 1;
        a.Q = 1;
        for (int b = 0; b < kBuckets; ++b)
            for (int s = 0; s < b + 6; ++s) a.orders[b][s] = (int8_t)s;
    }
    a.code_id = d_code_id;
    a.llr_off = d_llr_off;
    a.llr_pool = d_llr_pool;
    a.bits_off = d_bits_off;
    a.bits_pool = d_bits_pool;
    a.iters = d_iters;
    a.ok = d_ok;
    a.F = F;
    a.n_codes = n_codes;
    a.ctl = static_cast<int32_t *>(d_ws);
    a.list = reinterpret_cast<int32_t *>(static_cast<char *>(d_ws) + 256);
    a.max_iter = bp->max_iter;
    a.it_min = bp->it_min;
    a.stop = bp->stop;
    a.alpha = bp->alpha;
    const int rho = cfg ? cfg->rho : 0;
    const int block = cfg && cfg->slots == 2 ? 512 : kBatchBlock;
    const int grid = cfg ? cfg->grid : 0;
    if (rho != 0 && rho != 2 && rho != 3) return fail(PC_EINVAL, "rho must be 0, 2 or 3");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int prep_grid = (int)std::min<int64_t>((F + 255) / 256, (int64_t)device_cu_count() * 4);
    hipLaunchKernelGGL(k_batch_clear, dim3(1), dim3(64), 0, s, a.ctl);
    hipLaunchKernelGGL(k_batch_count, dim3(prep_grid), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_batch_layout, dim3(1), dim3(64), 0, s, a.ctl);
    hipLaunchKernelGGL(k_batch_scatter, dim3(prep_grid), dim3(256), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "batched queue preparation");
    const bool sc = bp->alpha != 1.0f;
    if (kq == 4) return sc ? launch_batched_rho<4, true>(a, rho, block, grid, s)
                           : launch_batched_rho<4, false>(a, rho, block, grid, s);
    return sc ? launch_batched_rho<0, true>(a, rho, block, grid, s)
              : launch_batched_rho<0, false>(a, rho, block, grid, s);
}

extern "C" {

int pp_mt_bp_decode_batched(const pc_code *const *codes, int32_t n_codes, const int32_t *d_code_id,
                            const int64_t *d_llr_off, const float *d_llr_pool, int64_t F,
                            const pc_bp_params *bp, const pc_pp_params *pp, uint8_t *d_bits_pool,
                            const int64_t *d_bits_off, int32_t *d_iters, uint8_t *d_ok, void *d_ws,
                            size_t ws_bytes, const pc_launch_cfg *cfg, void *stream) {
    return decode_batched_impl(codes, n_codes, d_code_id, d_llr_off, d_llr_pool, F, bp, pp, d_bits_pool,
                               d_bits_off, d_iters, d_ok, d_ws, ws_bytes, cfg, stream);
}

int pp_mt_bp_decode_batched_noalloc(const pc_code *const *codes, int32_t n_codes, const int32_t *d_code_id,
                                    const int64_t *d_llr_off, const float *d_llr_pool, int64_t F,
                                    const pc_bp_params *bp, const pc_pp_params *pp, uint8_t *d_bits_pool,
                                    const int64_t *d_bits_off, int32_t *d_iters, uint8_t *d_ok,
                                    const pc_launch_cfg *cfg, void *stream) {
    if (F > kNoAllocMaxFrames)
        return fail(PC_EINVAL, "pp_mt_bp_decode_batched_noalloc takes at most 1048576 frames per call");
    if (F <= 0 || !codes || n_codes < 1)
        return decode_batched_impl(codes, n_codes, d_code_id, d_llr_off, d_llr_pool, F, bp, pp, d_bits_pool,
                                   d_bits_off, d_iters, d_ok, nullptr, 0, cfg, stream);
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    for (int i = 0; i < n_codes; ++i)
        if (codes[i] && codes[i]->device != dev)
            return fail(PC_EINVAL, "the codes' device must be current (the scratch is per device)");
    void *ws = noalloc_scratch(dev);
    if (!ws) {
        const int rc = noalloc_scratch_init();
        if (rc != PC_OK) return rc;
        ws = noalloc_scratch(dev);
    }
    return decode_batched_impl(codes, n_codes, d_code_id, d_llr_off, d_llr_pool, F, bp, pp, d_bits_pool,
                               d_bits_off, d_iters, d_ok, ws, kNoAllocBytes, cfg, stream);
}

}  // extern "C"
