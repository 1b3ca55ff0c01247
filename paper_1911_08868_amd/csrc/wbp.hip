// wbp.hip -- weighted BP entry points: workspace sizing, validation, the
// forward and adjoint launches and the deterministic reduction of the
// per-workgroup weight-gradient partials.
#include <algorithm>
#include <cstring>

#include "wbp_inst.h"

namespace pbp {

int run_wbp_n4(const WbpLaunch &);
int run_wbp_n5(const WbpLaunch &);
int run_wbp_n6(const WbpLaunch &);
int run_wbp_n7(const WbpLaunch &);
int run_wbp_n8(const WbpLaunch &);
int run_wbp_n9(const WbpLaunch &);
int run_wbp_n10(const WbpLaunch &);
int run_wbp_n11(const WbpLaunch &);
int run_wbp_n12(const WbpLaunch &);

size_t wbp_big_scratch_floats(int n) {
    if (n == 11) return BigScratch<Plan<11, 0, 2>>::per_wg_floats > BigScratch<Plan<11, 5, 2>>::per_wg_floats
                            ? BigScratch<Plan<11, 0, 2>>::per_wg_floats : BigScratch<Plan<11, 5, 2>>::per_wg_floats;
    if (n == 12) return BigScratch<Plan<12, 0, 2>>::per_wg_floats > BigScratch<Plan<12, 5, 2>>::per_wg_floats
                            ? BigScratch<Plan<12, 0, 2>>::per_wg_floats : BigScratch<Plan<12, 5, 2>>::per_wg_floats;
    return 0;
}

int launch_wbp_n(int n, const WbpLaunch &L) {
    switch (n) {
        case 4: return run_wbp_n4(L);
        case 5: return run_wbp_n5(L);
        case 6: return run_wbp_n6(L);
        case 7: return run_wbp_n7(L);
        case 8: return run_wbp_n8(L);
        case 9: return run_wbp_n9(L);
        case 10: return run_wbp_n10(L);
        case 11: return run_wbp_n11(L);
        case 12: return run_wbp_n12(L);
        default: return fail(PC_ENOTSUP, "weighted BP is built for N = 16 .. 4096");
    }
}

// Deterministic two-level sum of the per-workgroup weight-gradient partials
// (rows of len floats): the first level sums chunks of kGradChunk consecutive
// rows, in row order, four columns per thread; the second sums the chunk
// totals in chunk order.  With one chunk the first level writes the result.
constexpr int64_t kGradChunk = 64;

__global__ void __launch_bounds__(256) k_grad_chunk_sum(const float4 *partial, int64_t groups, int64_t len4,
                                                        float4 *out) {
    const int64_t nchunks = (groups + kGradChunk - 1) / kGradChunk;
    for (int64_t c = blockIdx.y; c < nchunks; c += gridDim.y) {
        const int64_t g0 = c * kGradChunk;
        const int64_t g1 = g0 + kGradChunk < groups ? g0 + kGradChunk : groups;
        for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len4; i += (int64_t)gridDim.x * blockDim.x) {
            float4 s = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll 8
            for (int64_t g = g0; g < g1; ++g) {
                const float4 v = partial[g * len4 + i];
                s.x += v.x;
                s.y += v.y;
                s.z += v.z;
                s.w += v.w;
            }
            out[c * len4 + i] = s;
        }
    }
}

__global__ void __launch_bounds__(256) k_grad_reduce(const float *mid, int64_t nchunks, int64_t len, float *grad) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += (int64_t)gridDim.x * blockDim.x) {
        float s = 0.f;
        for (int64_t c = 0; c < nchunks; ++c) s += mid[c * len + i];
        grad[i] = s;
    }
}

__global__ void __launch_bounds__(256) k_grad_zero(float *grad, int64_t len) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += (int64_t)gridDim.x * blockDim.x)
        grad[i] = 0.f;
}

static unsigned clamp_grid(int64_t blocks) {
    return (unsigned)(blocks < 1 ? 1 : (blocks > 65535 ? 65535 : blocks));
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct WbpLayout {
    size_t ckpt_bytes = 0, partial_bytes = 0, mid_bytes = 0, scratch_bytes = 0, total = 0;
    int slots = 0, bslots = 0;
    int64_t groups = 0, nchunks = 0;
};

static WbpLayout wbp_layout(const pc_code *c, int64_t F, int T) {
    WbpLayout w;
    w.slots = wbp_slots(c->n);
    w.bslots = wbp_bwd_slots_n(c->n);
    const bool big = c->n >= kWbpBigLog;
    w.groups = big ? std::min<int64_t>(F, wbp_big_grid(c->n))
                   : std::min<int64_t>((F + w.bslots - 1) / w.bslots, wbp_small_grid(c->n));
    w.ckpt_bytes = align256((size_t)F * (size_t)(T > 1 ? T - 1 : 0) * (size_t)(c->n - 1) * c->N * sizeof(float));
    const size_t len = (size_t)T * c->n * 2 * (size_t)c->N;
    w.partial_bytes = align256((size_t)w.groups * len * sizeof(float));
    w.nchunks = (w.groups + kGradChunk - 1) / kGradChunk;
    w.mid_bytes = w.nchunks > 1 ? align256((size_t)w.nchunks * len * sizeof(float)) : 0;
    w.scratch_bytes = big ? align256((size_t)w.groups * wbp_big_scratch_floats(c->n) * sizeof(float)) : 0;
    w.total = w.ckpt_bytes + w.partial_bytes + w.mid_bytes + w.scratch_bytes;
    return w;
}

size_t wbp_ws_bytes(const pc_code *c, int64_t F, int T) { return wbp_layout(c, F, T).total; }

static int wbp_common(const pc_code *c, const float *d_llr, int64_t F, const float *d_w, int T,
                      const pc_pp_params *pp, void *d_ws, size_t ws_bytes, WbpLaunch &L,
                      WbpLayout &lay, bool need_ws = true) {
    if (!c) return fail(PC_EINVAL, "code is NULL");
    if (c->n < 4 || c->n > 12) return fail(PC_ENOTSUP, "weighted BP is built for N = 16 .. 4096");
    if (T < 1) return fail(PC_EINVAL, "T_unroll must be >= 1");
    if (F < 0) return fail(PC_EINVAL, "F < 0");
    if (F > 0 && (!d_llr || !d_w)) return fail(PC_EINVAL, "null buffer");
    lay = wbp_layout(c, F, T);
    const bool no_ws = !need_ws && !d_ws && ws_bytes == 0;
    if (F > 0 && !no_ws && (!d_ws || ws_bytes < lay.total)) return fail(PC_ENOMEM, "workspace too small");
    if (F > 0 && !no_ws && reinterpret_cast<uintptr_t>(d_ws) % 256)
        return fail(PC_EINVAL, "workspace must be 256-byte aligned");
    std::memset(&L.args, 0, sizeof(L.args));
    int8_t orders[kMaxPool * kMaxLog] = {0};
    int kp = 0, Q = 1, Tev = 1;
    const int n = c->n;
    if (pp && pp->noise_sigma != 0.f) return fail(PC_ENOTSUP, "weighted BP injects no noise");
    if (pp && pp->mode != PC_PP_NONE) {
        if (pp->mode != PC_PP_LASTK) return fail(PC_ENOTSUP, "weighted BP supports the fixed last-k schedule");
        if (pp->k < 2 || pp->k > n) return fail(PC_EINVAL, "k must satisfy 2 <= k <= n");
        if (pp->period_T < 1 || pp->pool_Q < 1 || pp->pool_Q > kMaxPool)
            return fail(PC_EINVAL, "period T >= 1 and pool Q in 1..8");
        Q = make_pool(n, pp->k, pp->pool_Q, pp->seed, orders);
        if (Q < 0) return Q;
        kp = Q > 1 ? pp->k : 0;
        Tev = pp->period_T;
        if (kp == n) return fail(PC_ENOTSUP, "weighted BP with full permutations is not built");
    } else {
        for (int s = 0; s < n; ++s) orders[s] = (int8_t)s;
    }
    WbpArgs &a = L.args;
    a.llr = d_llr;
    a.F = F;
    a.w = d_w;
    a.T = T;
    a.ckpt = no_ws ? nullptr : static_cast<float *>(d_ws);
    a.partial = no_ws ? nullptr : reinterpret_cast<float *>(static_cast<char *>(d_ws) + lay.ckpt_bytes);
    a.scratch = no_ws || !lay.scratch_bytes
                    ? nullptr
                    : reinterpret_cast<float *>(static_cast<char *>(d_ws) + lay.ckpt_bytes + lay.partial_bytes +
                                                lay.mid_bytes);
    a.meta = c->d.meta;
    a.Tev = Tev;
    a.Q = Q;
    for (int q = 0; q < Q; ++q)
        for (int s = 0; s < n; ++s) a.orders[q][s] = orders[q * n + s];
    L.kp = kp;
    L.slots = lay.slots;
    L.bslots = lay.bslots;
    // the forward takes one workgroup per `slots` frames; the adjoint one per
    // partial (a fixed grid whose workgroups walk the frames)
    L.grid = (int)((F + lay.slots - 1) / lay.slots);
    L.bgrid = (int)lay.groups;
    return PC_OK;
}

}  // namespace pbp

using namespace pbp;

extern "C" {

size_t wbp_workspace_bytes(const pc_code *code, int64_t F, int32_t T_unroll) {
    if (!code || F < 0 || T_unroll < 1) return 0;
    return wbp_ws_bytes(code, F, T_unroll);
}

int wbp_forward(const pc_code *code, const float *d_llr, int64_t F, const float *d_w,
                int32_t T_unroll, const pc_pp_params *pp, float *d_out_llr, void *d_ws,
                size_t ws_bytes, void *stream) {
    WbpLaunch L;
    WbpLayout lay;
    int rc = wbp_common(code, d_llr, F, d_w, T_unroll, pp, d_ws, ws_bytes, L, lay, false);
    if (rc) return rc;
    if (F == 0) return PC_OK;
    if (!d_out_llr) return fail(PC_EINVAL, "null output");
    L.args.out = d_out_llr;
    L.backward = false;
    L.stream = static_cast<hipStream_t>(stream);
    return launch_wbp_n(code->n, L);
}

int wbp_backward(const pc_code *code, const float *d_llr, int64_t F, const float *d_w,
                 int32_t T_unroll, const pc_pp_params *pp, const float *d_grad_out,
                 float *d_grad_w, void *d_ws, size_t ws_bytes, void *stream) {
    WbpLaunch L;
    WbpLayout lay;
    int rc = wbp_common(code, d_llr, F, d_w, T_unroll, pp, d_ws, ws_bytes, L, lay);
    if (rc) return rc;
    if (!d_grad_w) return fail(PC_EINVAL, "null gradient output");
    hipStream_t hs = static_cast<hipStream_t>(stream);
    const int64_t len = (int64_t)T_unroll * code->n * 2 * code->N;
    if (F == 0) {
        // a kernel, not a memset, so that the call can be captured in a graph
        hipLaunchKernelGGL(k_grad_zero, dim3(clamp_grid((len + 255) / 256)), dim3(256), 0, hs, d_grad_w, len);
        hipError_t e = hipGetLastError();
        return e == hipSuccess ? PC_OK : hip_fail(e, "gradient clear");
    }
    if (!d_grad_out) return fail(PC_EINVAL, "null output adjoint");
    L.args.gout = d_grad_out;
    L.backward = true;
    L.grid = L.bgrid;
    L.stream = hs;
    rc = launch_wbp_n(code->n, L);
    if (rc) return rc;
    const int64_t len4 = len / 4;  // len = T n 2 N, N >= 16
    float *mid = lay.nchunks > 1
                     ? reinterpret_cast<float *>(static_cast<char *>(d_ws) + lay.ckpt_bytes + lay.partial_bytes)
                     : d_grad_w;
    hipLaunchKernelGGL(k_grad_chunk_sum, dim3(clamp_grid((len4 + 255) / 256), clamp_grid(lay.nchunks)), dim3(256),
                       0, hs, reinterpret_cast<const float4 *>(L.args.partial), lay.groups, len4,
                       reinterpret_cast<float4 *>(mid));
    if (lay.nchunks > 1)
        hipLaunchKernelGGL(k_grad_reduce, dim3(clamp_grid((len + 255) / 256)), dim3(256), 0, hs, mid, lay.nchunks,
                           len, d_grad_w);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "gradient reduction launch");
    return PC_OK;
}

}  // extern "C"
