// alg1.hip -- Algorithm 1 (partially permuted BP with random subgraphs) on
// the GPU: one frame per workgroup, messages in LDS, a per-row stage order.
//
// Algorithm 1 permutes one subgraph at a time: at an event it draws a range
// rho_range in {2..P_range}, a level rho_level = min(U{1..P_level},
// n - rho_range + 1) and one of the N / 2^m connected blocks of stages 1..m
// of the current graph (m = rho_level + rho_range - 1), and gives stages
// rho_level..m of that block a new non-identity order of the bits they use;
// the nodes on the levels strictly between the permuted stages of the block
// are reset, and the next event follows Eq. 2 (iteration + max(N_min,
// floor(N_zero / D)), N_zero = 2^m (rho_range - 1)).  A draw is kept only if
// the component has 2^m rows and each of the stages uses one bit over it (so
// every graph still encodes x = u G_N); otherwise it is drawn again, at most
// 64 times.  Rows of different blocks then pair on different bits, so the
// relabelled, register-resident layout of k_decode does not apply: here every
// row carries its own order (4 bits per stage in registers) and every L and R
// level that a partner reads lives in LDS, (2n-2) N floats (the channel level
// and the prior are static per frame, so each row holds its partners' values
// of those in registers).  At N = 1024 that is 72 KiB (77 KiB with the
// control words and the syndrome columns), and two frames share a CU.
//
// One thread per row (up to 1024 rows).  At each stage a row computes its own
// output of its processing element (Sec. II-B): with j' the partner of row j,
// the top row needs f(L_{s-1}[j], L_{s-1}[j'] + R_s[j']) and the bottom row
// f(R_s[j'], L_{s-1}[j']) + L_{s-1}[j] (L sweep), so both read the same three
// values and select operands without branching; the R sweep is alike.  The
// check function is the clamp form of min-sum with an L operand as the bound,
// as in the fixed-schedule kernels.  Consecutive stages need a workgroup barrier
// only if some row of the reading stage pairs on a bit >= 6, i.e. with a row
// of another wave; a per-stage flag, recomputed after every event, says so,
// and the other stages are ordered by the wave's own in-order LDS accesses
// (in the original graph 6 of n stages pair inside a wave).  Overwrites of
// values other waves read are ordered by the barriers of the decision (L
// sweep reads, R levels) and by one barrier after the R sweep (its reads of
// L levels, rewritten by the next L sweep or an event's labels).  At an
// event the chosen block's first row publishes its order, which every row
// compares with its own.  The random draws come from a SplitMix64 stream per
// frame, started at seed + (frame + 1) * golden ratio, that every thread
// advances identically, so all control decisions are uniform.  The component
// labels of stages 1..m (the smallest row of each component) come from
// stage-ordered sweeps of pairwise minima, repeated until one changes
// nothing, and are kept for the event's later draws of the same m; blocks are
// ranked by their smallest row.
#include <climits>

#include "alg1_common.h"

namespace pbp {

template <int NLOG>
struct Alg1Lds {
    static constexpr int N = 1 << NLOG, n = NLOG;
    // partners read L levels 1..n-1 and R levels 1..n-1 from LDS; the channel
    // level and the prior level n are static per frame, so each row keeps its
    // partner's values of those in registers, and L level n is read only by
    // its own row
    static constexpr size_t msg_floats = (size_t)(2 * n - 2) * N;
    // + 352 control words + the rows' syndrome columns (read at every decision)
    static constexpr size_t bytes = msg_floats * 4 + 352 * 4 + (size_t)N * 4;
    static constexpr int threads = N >= 64 ? N : 64;  // one row per thread
};

// 8 waves per SIMD: two 1024-row frames per CU (the LDS of one is 77 KiB)
template <int NLOG, int CN>
__global__ void __launch_bounds__(Alg1Lds<NLOG>::threads, 8) k_alg1(Alg1Args a) {
    constexpr int N = 1 << NLOG, n = NLOG;
    const int tid = threadIdx.x, nt = blockDim.x;
    extern __shared__ __align__(16) float smem[];
    // L level l (1..n-1) at smem + (l-1) N, R level l (1..n-1) at smem + (n+l-2) N
    auto Lrow = [&](int l) -> float * { return smem + (size_t)(l - 1) * N; };
    auto Rrow = [&](int l) -> float * { return smem + (size_t)(n + l - 2) * N; };
    // component labels of stages 1..m (m = 2..n) at an event live in L level
    // m-1: the L levels are dead from the end of an R sweep until the next L
    // sweep rewrites them, so the labels of every m drawn at one event are
    // kept for its later attempts
    auto labs = [&](int m) -> int32_t * { return reinterpret_cast<int32_t *>(Lrow(m - 1)); };
    // misc: [0] frame, [3] root, [4..19] wave partials, [40 + s] stage s pairs
    // across waves, [64..95] wave partials of the decision hash (lo, hi),
    // [100..101] the root row's stage bits, [128..159] per-wave flags of the
    // label sweeps (two sets, by sweep parity), [160..175] per-wave member
    // counts and column flags of the block test, [192 + 16 (m-2) + w] wave w's
    // count of component roots for stages 1..m
    int32_t *const misc = reinterpret_cast<int32_t *>(smem + Alg1Lds<NLOG>::msg_floats);
    uint32_t *const synl = reinterpret_cast<uint32_t *>(misc + 352);
    const float alpha = a.alpha;
    const float inf = __builtin_huge_valf();
    auto Lv = [&](int l, int j) -> float & { return Lrow(l)[j]; };
    auto Rv = [&](int l, int j) -> float & { return Rrow(l)[j]; };

    const int wave = tid >> 6, nwaves = (nt + 63) >> 6, lane = tid & 63;
    // workgroup-wide or of a per-thread predicate with one barrier: each wave
    // publishes its ballot in misc[base + w] and every lane w reads wave w's.
    // The caller alternates base between calls whose flags could still be
    // read (the barrier of the next call orders those reads before reuse).
    auto wg_any = [&](bool v, int base) -> bool {
        const bool w = __ballot(v) != 0;
        if (lane == 0) misc[base + wave] = w ? 1 : 0;
        __syncthreads();
        const int f = lane < nwaves ? misc[base + lane] : 0;
        return __ballot(f != 0) != 0;
    };
    // sum of lanes 0..15 of v as a uniform value (called with every lane
    // active, so lane 0 holds the sum)
    auto sum16 = [&](int v) -> int {
        v += __shfl_xor(v, 1, 16);
        v += __shfl_xor(v, 2, 16);
        v += __shfl_xor(v, 4, 16);
        v += __shfl_xor(v, 8, 16);
        return __builtin_amdgcn_readlane(v, 0);
    };
    // (called once per iteration, from the decision: the previous reads of
    // misc[4 + w] are ordered before these writes by the barrier that ends
    // every R sweep or by the barrier at the top of the frame loop)
    auto wg_xor = [&](uint32_t v) -> uint32_t {
        v = lanes_xor<64>(v);
        if ((tid & 63) == 0) misc[4 + (tid >> 6)] = (int32_t)v;
        __syncthreads();
        // lane w of every wave reads wave w's partial: one read and one lane
        // reduction instead of a read per wave
        const uint32_t p = lane < nwaves ? (uint32_t)misc[4 + lane] : 0u;
        return lanes_xor<64>(p);
    };

    // the row's stage order: the bit that stage s pairs on, 4 bits per stage
    // (stage s at bit 4 (s-1)), held in registers
    uint64_t ordw = 0;
    auto obit = [&](uint64_t w, int s) -> int { return (int)((w >> (4 * (s - 1))) & 15u); };

    // stage s pairs some row with a row of another wave (bit >= 6); the
    // flags are gathered into a uniform mask (bit s-1) kept in a scalar
    // register until the next event
    uint32_t crossm = 0;
    auto update_cross = [&](bool row) {
        __syncthreads();
        if (tid < n) misc[41 + tid] = 0;
        __syncthreads();
        if (row)
            for (int s = 1; s <= n; ++s)
                if (obit(ordw, s) >= 6) misc[40 + s] = 1;
        __syncthreads();
        uint32_t c = 0;
        for (int s = 1; s <= n; ++s) c |= (misc[40 + s] != 0 ? 1u : 0u) << (s - 1);
        crossm = __builtin_amdgcn_readfirstlane(c);
    };
    // the thread's partner row at stage s, from the order in registers
    auto partner = [&](int j, int s) -> int { return j ^ (1 << obit(ordw, s)); };
    // between events the partner rows are cached, 10 bits per stage and three
    // stages per register; a row is the top one of its pair iff its partner
    // is the larger index.  The partner's channel LLR (stage 1) and prior
    // (stage n) are cached too.
    constexpr int kPk = (n + 2) / 3;
    uint32_t pk[kPk];
    sfor<0, kPk>([&](auto i) { pk[i] = 0u; });
    auto cpart = [&](int s) -> int { return (int)((pk[(s - 1) / 3] >> (10 * ((s - 1) % 3))) & 1023u); };
    float pch = 0.f, ppr = 0.f;
    // the channel level of row r after event e (e = 0: none yet): the received
    // LLR plus the event's noise, each product and sum rounded once
    auto channel = [&](const float *src, int64_t frame, int e, int r) -> float {
        if (e == 0) return src[r];
        const float z = a.noise_sigma * noise_gauss(a.noise_seed, frame, e, r);
        return src[r] + z;
    };
    auto load_pairs = [&](bool row, int j, const float *src, int64_t frame, int e) {
        sfor<0, kPk>([&](auto i) { pk[i] = 0u; });
        sfor<1, n + 1>([&](auto s) {
            const uint32_t p = row ? (uint32_t)partner(j, s) : 0u;
            pk[(s - 1) / 3] |= p << (10 * ((s - 1) % 3));
        });
        if (row) {
            pch = channel(src, frame, e, partner(j, 1));
            ppr = a.meta[partner(j, n)] == -2 ? inf : 0.f;
        }
    };
    auto stage_sync = [&](int s) {
        // the mask goes through an empty asm at every test, so that the
        // compiler does not precompute all 2n tests as lane masks and spill
        // them to VGPR lanes
        uint32_t cm = crossm;
        asm volatile("" : "+s"(cm));
        if ((cm >> (s - 1)) & 1u) {
            __syncthreads();
        } else {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
    };
    uint64_t ident = 0;
    for (int s = 1; s <= n; ++s) ident |= (uint64_t)(s - 1) << (4 * (s - 1));

    for (;;) {
        __syncthreads();
        if (tid == 0) misc[0] = (int32_t)atomicAdd(a.counter, 1u);
        __syncthreads();
        const int64_t frame = misc[0];
        if (frame >= a.F) break;

        // ---- initialise L and R (Alg. 1 initializeLandR) and the orders ----
        const float *src = a.llr + frame * N;
        const int j = tid;
        // the launch has N threads when N >= 64, so every thread owns a row
        const bool row = N >= 64 || j < N;
        // the thread's own row on every level, mirrored in registers
        float Lown[n + 1], Rown[n + 1];
        sfor<0, n + 1>([&](auto l) { Lown[l] = 0.f; Rown[l] = 0.f; });
        ordw = ident;
        if (row) {
            Lown[0] = src[j];
            Rown[n] = a.meta[j] == -2 ? inf : 0.f;
            sfor<1, n>([&](auto l) { Rv(l, j) = 0.f; });
            synl[j] = a.syn[j];  // read back by this thread only
        }
        uint64_t st = a.seed + (uint64_t)(frame + 1) * 0x9E3779B97F4A7C15ull;
        int next_reset = alg1_first_event(a, N, n);
        int ev = 0;  // events so far with noise injected (Sec. V reading)
        update_cross(row);
        load_pairs(row, j, src, frame, ev);
        const uint64_t hkey = a.hist ? decision_key(j) : 0ull;

        int it_done = a.max_iter;
        bool okv = false;
        for (int it = 1; it <= a.max_iter; ++it) {
            // ---- L sweep, stages 1..n ----
            sfor<1, n + 1>([&](auto sc) {
                constexpr int s = sc;
                stage_sync(s);  // level s-1 and R_s of the partner rows
                if (row) {
                    const int p = cpart(s);
                    const bool top = p > j;
                    const float A = Lown[s - 1];
                    const float B = s == 1 ? pch : Lrow(s - 1)[p];
                    const float C = s == n ? ppr : Rrow(s)[p];
                    // top: f(L[j], L[j'] + R[j']); bottom: f(L[j'], R[j']) + L[j]
                    const float c = alg1_check<CN>(top ? A : B, top ? B + C : C, alpha);
                    Lown[s] = top ? c : c + A;
                    if (s < n) Lv(s, j) = Lown[s];
                }
            });
            // ---- decision and CRC syndrome on level n+1 ----
            uint32_t syn = 0;
            const bool one = row && Lown[n] + Rown[n] < 0.f;
            if (one) syn = synl[j];
            if (a.hist) {
                // decision hash of this iteration (error classes, Sec. II-C);
                // the partials are read after wg_xor's barriers and rewritten
                // only after the next iteration's
                const uint64_t h = one ? hkey : 0ull;
                const uint32_t lo = lanes_xor<64>((uint32_t)h), hi = lanes_xor<64>((uint32_t)(h >> 32));
                if (lane == 0) {
                    misc[64 + 2 * wave] = (int32_t)lo;
                    misc[65 + 2 * wave] = (int32_t)hi;
                }
            }
            const bool pass = wg_xor(syn) == 0u;
            if (a.hist && tid == 0) {
                uint64_t h = 0;
                for (int w = 0; w < nwaves; ++w)
                    h ^= ((uint64_t)(uint32_t)misc[65 + 2 * w] << 32) | (uint32_t)misc[64 + 2 * w];
                a.hist[frame * a.H + (it - 1) % a.H] = h;
            }
            if (a.stop == PC_STOP_CRC && it >= a.it_min && pass) {
                it_done = it;
                okv = true;
                break;
            }
            if (it == a.max_iter) {
                okv = pass;
                break;
            }
            // ---- R sweep, stages n..2 (R on the channel level is never read) ----
            sfor<0, n - 1>([&](auto kc) {
                constexpr int s = n - kc;
                stage_sync(s);  // R_s and level s-1 of the partner rows
                if (row) {
                    const int p = cpart(s);
                    const bool top = p > j;
                    const float P = Rown[s];
                    const float Q = Lrow(s - 1)[p];
                    const float S = s == n ? ppr : Rrow(s)[p];
                    // top: f(L[j'] + R[j'], R[j]); bottom: f(L[j'], R[j']) + R[j]
                    const float c = alg1_check<CN>(top ? Q + S : Q, top ? P : S, alpha);
                    Rown[s - 1] = top ? c : c + P;
                    Rv(s - 1, j) = Rown[s - 1];
                }
            });
            // the R sweep read partners' L messages, which the next L sweep
            // (or an event's labels) overwrites; the decision's barriers order
            // the other hazards
            __syncthreads();
            // ---- partial permutation of one subgraph (Alg. 1 partialPermute) ----
            if (it == next_reset) {
                int n_zero = 0;
                uint32_t have = 0;  // the m whose labels this event has computed
                for (int attempt = 0; attempt < 64; ++attempt) {
                    const int rr = 2 + (int)draw_below(st, (uint32_t)(a.P_range - 1));
                    const int x = 1 + (int)draw_below(st, (uint32_t)a.P_level);
                    const int rl = x < n - rr + 1 ? x : n - rr + 1;
                    const int m = rl + rr - 1;
                    const int nblocks = N >> m;
                    const int blk = (int)draw_below(st, (uint32_t)nblocks);
                    // components of stages 1..m: smallest row index.  Sweeps over
                    // stages 1..m replace each row's label with the smaller of its
                    // own and its stage partner's, ordered like the decoding
                    // sweeps (a workgroup barrier only before a stage that pairs
                    // across waves).  Both rows of a pair end with the pair's
                    // minimum whichever order their accesses take.  Labels stay
                    // rows of the same component, at most the row itself; a sweep
                    // that changes nothing leaves them equal across every pair,
                    // so each component holds its smallest row.  On an unpermuted
                    // block one sweep reaches the minimum (a butterfly), the next
                    // confirms it.  The orders do not change between the attempts
                    // of an event, so labels already computed for this m are
                    // reused (each row reads back its own).
                    int32_t *const lab = labs(m);
                    int32_t *const rcnt = misc + 192 + 16 * (m - 2);
                    int lj = j;
                    const bool fresh = !((have >> m) & 1u);
                    if (!fresh) {
                        if (row) lj = lab[j];
                    } else {
                        have |= 1u << m;
                        if (row) lab[j] = j;
                        __syncthreads();
                        for (int sweep = 0;; ++sweep) {
                            bool c = false;
                            for (int s = 1; s <= m; ++s) {
                                if (s > 1) stage_sync(s);
                                if (row) {
                                    const int w = lab[partner(j, s)];
                                    if (w < lj) {
                                        lj = w;
                                        lab[j] = w;
                                        c = true;
                                    }
                                }
                            }
                            if (!wg_any(c, 128 + 16 * (sweep & 1))) break;
                        }
                    }
                    // components (their smallest rows) and the one of rank blk;
                    // the per-wave root counts are published with the labels
                    const bool is_root = row && lj == j;
                    const uint64_t rmask = __ballot(is_root);
                    if (fresh) {
                        if (lane == 0) rcnt[wave] = __popcll(rmask);
                        __syncthreads();
                    }
                    const int cnt = lane < nwaves ? rcnt[lane] : 0;
                    const int total = sum16(cnt), before = sum16(lane < wave ? cnt : 0);
                    if (total != nblocks) continue;
                    if (is_root && before + __popcll(rmask & ((1ull << lane) - 1)) == blk) {
                        misc[3] = j;
                        misc[100] = (int32_t)(uint32_t)ordw;
                        misc[101] = (int32_t)(uint32_t)(ordw >> 32);
                    }
                    __syncthreads();
                    const int root = misc[3];
                    const uint64_t rord = (uint64_t)(uint32_t)misc[100] | ((uint64_t)(uint32_t)misc[101] << 32);
                    // size of the block and one bit per permuted stage over it
                    const bool member = row && lj == root;
                    bool mixed = false;
                    if (member)
                        for (int s = rl; s <= m; ++s) mixed |= obit(ordw, s) != obit(rord, s);
                    // one exchange: each wave's member count and column flag
                    // (the previous attempt read these slots before the root
                    // barrier above)
                    {
                        const int mc = __popcll(__ballot(member));
                        const bool mx = __ballot(mixed) != 0;
                        if (lane == 0) misc[160 + wave] = mc | (mx ? 0x10000 : 0);
                    }
                    __syncthreads();
                    const int mv = lane < nwaves ? misc[160 + lane] : 0;
                    const int members = sum16(mv & 0xffff);
                    const bool bad = __ballot((mv >> 16) != 0) != 0;
                    if (bad || members != (1 << m)) continue;
                    // a new non-identity order of the bits of stages rl..m
                    int8_t bits[kMaxLog], cand[kMaxLog];
                    for (int i = 0; i < rr; ++i) bits[i] = (int8_t)obit(rord, rl + i);
                    bool same = true;
                    while (same) {
                        for (int i = 0; i < rr; ++i) cand[i] = bits[i];
                        for (int i = rr - 1; i >= 1; --i) {
                            const int jj = (int)draw_below(st, (uint32_t)(i + 1));
                            const int8_t tt = cand[i];
                            cand[i] = cand[jj];
                            cand[jj] = tt;
                        }
                        same = true;
                        for (int i = 0; i < rr; ++i) same &= cand[i] == bits[i];
                    }
                    if (member) {
                        for (int i = 0; i < rr; ++i) {
                            const int sh = 4 * (rl - 1 + i);
                            ordw = (ordw & ~(15ull << sh)) | ((uint64_t)(uint8_t)cand[i] << sh);
                        }
                        // levels strictly between the permuted stages (Sec. III);
                        // L levels are rewritten by the next L sweep before any
                        // read, so only the registers and the R levels in LDS
                        // are cleared
                        sfor<1, n>([&](auto l) {
                            if (l >= rl && l <= m - 1) {
                                Lown[l] = 0.f;
                                Rown[l] = 0.f;
                                Rv(l, j) = 0.f;
                            }
                        });
                    }
                    n_zero = (1 << m) * (rr - 1);
                    break;
                }
                int add = a.D > 0 ? n_zero / a.D : 0;
                if (add < a.N_min) add = a.N_min;
                next_reset = it + add;
                if (a.noise_sigma > 0.f) {
                    // fresh channel noise on the received LLRs, every event
                    ++ev;
                    if (row) Lown[0] = channel(src, frame, ev, j);
                }
                update_cross(row);
                load_pairs(row, j, src, frame, ev);
            }
        }

        // ---- outputs (Alg. 1 hardDecision) ----
        uint8_t *mo = a.msg + frame * a.K_msg;
        if (row) {
            const int mi = a.meta[j];
            const float v = Lown[n] + Rown[n];
            if (mi >= 0) mo[mi] = v < 0.f ? 1 : 0;
            if (a.soft) a.soft[frame * N + j] = Lown[n];
        }
        if (tid == 0) {
            if (a.iters) a.iters[frame] = it_done;
            if (a.ok) a.ok[frame] = okv ? 1 : 0;
        }
    }
}

template <int NLOG>
static int run_alg1_n(const Alg1Args &a, int cn, hipStream_t s) {
    constexpr size_t lds = Alg1Lds<NLOG>::bytes;
    static_assert(lds <= 160 * 1024, "Algorithm 1 frame exceeds LDS");
    const int threads = Alg1Lds<NLOG>::threads;
    auto kern = cn == 2 ? k_alg1<NLOG, 2> : cn == 1 ? k_alg1<NLOG, 1> : k_alg1<NLOG, 0>;
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, threads, lds);
    if (e != hipSuccess) return hip_fail(e, "occupancy query");
    if (per_cu < 1) per_cu = 1;
    int64_t grid = (int64_t)per_cu * device_cu_count();
    if (grid > a.F) grid = a.F;
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(threads), lds, s, a);
    e = hipGetLastError();
    return e == hipSuccess ? PC_OK : hip_fail(e, "Algorithm 1 launch");
}

int launch_alg1(const pc_code *c, const float *d_llr, int64_t F, const pc_bp_params &bp,
                const pc_pp_params &pp, uint8_t *d_msg, int32_t *d_iters, uint8_t *d_ok, float *d_soft,
                uint64_t *d_hist, int32_t H, hipStream_t s) {
    const bool orig = pp.mode == PC_PP_ALG1_ORIG;
    const int n = c->n;
    if (n < 4 || n > 10) return fail(PC_ENOTSUP, "Algorithm 1 on the GPU is built for N = 16 .. 1024");
    if (bp.stop == PC_STOP_G || (bp.stop == PC_STOP_NONE && c->crc_width == 0))
        return fail(PC_ENOTSUP, "Algorithm 1 on the GPU checks with the CRC (a code with a CRC, stop none or CRC)");
    if (pp.P_range < 2 || pp.P_range > n || pp.P_level < 1 || pp.P_level > n - 1 || pp.N_min < 1 || pp.D < 0)
        return fail(PC_EINVAL, "Algorithm 1 needs 2 <= P_range <= n, 1 <= P_level <= n-1, N_min >= 1, D >= 0");
    uint32_t *ctr = counter_block(c->device, s);
    if (!ctr) return PC_ENOMEM;
    hipLaunchKernelGGL(k_reset_queues, dim3(1), dim3(64), 0, s, ctr, 1);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "counter reset launch");
    Alg1Args a{};
    a.llr = d_llr;
    a.F = F;
    a.msg = d_msg;
    a.iters = d_iters;
    a.ok = d_ok;
    a.soft = d_soft;
    a.syn = c->d.syn;
    a.meta = c->d.meta;
    a.counter = ctr;
    a.K_msg = c->K_msg;
    a.max_iter = bp.max_iter;
    a.it_min = bp.it_min;
    a.stop = bp.stop;
    a.alpha = bp.alpha;
    a.P_range = pp.P_range;
    a.P_level = pp.P_level;
    a.D = pp.D;
    a.N_min = pp.N_min;
    a.first_reset = pp.first_reset;
    a.seed = pp.seed;
    a.hist = d_hist;
    a.H = H;
    a.noise_sigma = pp.noise_sigma;
    a.noise_seed = pp.seed;
    const int cn = bp.check == PC_CHECK_EXACT ? 2 : bp.alpha != 1.0f ? 1 : 0;
    if (orig) return run_alg1_orig(a, n, cn, s);
    switch (n) {
        case 4: return run_alg1_n<4>(a, cn, s);
        case 5: return run_alg1_n<5>(a, cn, s);
        case 6: return run_alg1_n<6>(a, cn, s);
        case 7: return run_alg1_n<7>(a, cn, s);
        case 8: return run_alg1_n<8>(a, cn, s);
        case 9: return run_alg1_n<9>(a, cn, s);
        default: return run_alg1_n<10>(a, cn, s);
    }
}

}  // namespace pbp
