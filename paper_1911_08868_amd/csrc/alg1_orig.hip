// alg1_orig.hip -- Algorithm 1 (Sec. III) under the reading in which each
// event permutes a subgraph of the ORIGINAL factor graph: one frame per
// workgroup, one processing element per thread and stage, messages in
// registers.
//
// At an event a frame draws rho_range in {2..P_range}, rho_level =
// min(U{1..P_level}, n - rho_range + 1) and one of the N / 2^m aligned blocks
// of 2^m rows (m = rho_level + rho_range - 1), then a new non-identity order
// c of the bits rho_level-1..m-1 that stages rho_level..m use in the original
// graph.  The block permuted at the previous event first goes back to the
// original order; the R messages on the inner levels of both blocks (levels
// rho_level..m-1) are reset, and N_zero of Eq. 2 counts the union of those
// nodes.  So the graph is the original one outside at most one block, and
// every graph is valid (each stage uses one bit over every component).
//
// Coordinates.  Inside the block, stage s (rho_level <= s <= m) pairs rows on
// bit c_s.  Relabelling the block's rows by rho (bit s-1 of rho(r) is bit c_s
// of r) turns every permuted stage into the original butterfly on bit s-1;
// stage s therefore works in "stage coordinates": rho for the block's stages,
// the row index elsewhere.  Only the two boundary levels rho_level-1 and m
// change coordinates between consecutive stages.
//
// Layout.  Thread t in [0, N/2) evaluates, at stage s, the processing element
// on positions insert0(t, s-1) (top) and that + 2^(s-1) (bottom) of the stage's
// coordinates, both of its outputs (Sec. II-B).  It keeps, per stage s, the
// stage's inputs L_{s-1} and R_s on its two positions in registers (R_n is the
// prior).  Between stages s and s+1 a row moves to the thread whose index
// differs in bit s-1, so the L sweep passes each output on by a butterfly on
// that thread bit, and the R sweep back by the same butterfly on bit s-2: one
// value crosses per thread, by DPP lane moves (bits 0..3), the gfx950 lane-row
// swaps v_permlane16_swap / v_permlane32_swap (bits 4, 5), or through LDS with
// a workgroup barrier (bits 6.., other waves).  At a boundary level of the
// block the two values go through LDS by row.  LDS holds two exchange buffers
// (alternated, so each exchange needs one barrier), the R levels while an
// event moves them to new coordinates, the channel LLRs and control words:
// 52.5 KiB at N = 1024, so three frames share a CU.  The launch bound asks
// for six waves per SIMD (three 8-wave frames per CU at N = 1024; at most 80
// VGPRs, a few spilled): the kernel's stages form one dependent chain per
// thread, and a third frame per CU hides more of its latency (measured 16%
// faster than two on Table I's 200-iteration set).
#include "alg1_common.h"

namespace pbp {

template <int NLOG>
struct Alg1OLds {
    static constexpr int N = 1 << NLOG, n = NLOG, NP = N / 2;
    static constexpr int threads = NP >= 64 ? NP : 64;
    // element bits (n-1), and the wave bits among them (above the 6 lane bits)
    static constexpr int EB = n - 1, W = EB > 6 ? EB - 6 : 0;
    // exchange buffers of N floats (two alternating ones for exchanges with a
    // workgroup barrier, one for exchanges within each wave), the R levels
    // 1..n-1 while an event moves them, the channel LLRs, control words
    static constexpr size_t xfloats = 3 * (size_t)N;
    // R levels 1..n-1 at an event, then the frame's channel LLRs
    static constexpr size_t evfloats = (size_t)n * N;
    // [0] frame, [4..19] wave partials of the syndrome, [32..47] wave flags
    // of the exchanges, [64..95] wave partials of the decision hash (lo, hi)
    static constexpr int misc_words = 128;
    static constexpr size_t bytes = (xfloats + evfloats + misc_words) * 4;
};

// t with a 0 inserted at bit b, and r with bit b removed
__device__ __forceinline__ int insert0(int t, int b) { return ((t >> b) << (b + 1)) | (t & ((1 << b) - 1)); }
__device__ __forceinline__ int remove_bit(int r, int b) { return ((r >> (b + 1)) << b) | (r & ((1 << b) - 1)); }

// Butterfly over lane bit K (K <= 5) of a pair held as (top, bottom): a lane
// with the bit clear keeps its top and takes its partner's top as bottom; a
// lane with the bit set takes its partner's bottom as top and keeps its
// bottom.
//  - bits 4 and 5: exactly the row swaps of v_permlane16_swap (odd 16-lane
//    rows of the first operand with even rows of the second) and
//    v_permlane32_swap (upper half of the first with lower half of the second);
//  - bits 2 and 3: DPP row shifts by 4 / 8 whose bank mask (4-lane groups)
//    writes only the lanes that take a value, the others keeping theirs;
//  - bits 0 and 1: one value crosses by a DPP quad permutation, with selects.
template <int K>
__device__ __forceinline__ void bfly_wave(float &top, float &bot, int lane) {
    if constexpr (K == 4 || K == 5) {
        const auto r = K == 4 ? __builtin_amdgcn_permlane16_swap(__float_as_uint(top), __float_as_uint(bot), false, false)
                              : __builtin_amdgcn_permlane32_swap(__float_as_uint(top), __float_as_uint(bot), false, false);
        top = __uint_as_float(r[0]);
        bot = __uint_as_float(r[1]);
    } else if constexpr (K == 2 || K == 3) {
        // row_shr:d (lane i reads i - d) into the banks with the bit set,
        // row_shl:d (lane i reads i + d) into the banks with it clear
        constexpr int shr = K == 2 ? 0x114 : 0x118, shl = K == 2 ? 0x104 : 0x108;
        constexpr int set = K == 2 ? 0xA : 0xC, clr = K == 2 ? 0x5 : 0x3;
        const int T = __float_as_int(top), B = __float_as_int(bot);
        top = __int_as_float(__builtin_amdgcn_update_dpp(T, B, shr, 0xF, set, false));
        bot = __int_as_float(__builtin_amdgcn_update_dpp(B, T, shl, 0xF, clr, false));
    } else {
        const bool b = (lane >> K) & 1;
        const int send = __float_as_int(b ? top : bot);
        const float recv = __int_as_float(__builtin_amdgcn_update_dpp(0, send, K == 0 ? 0xB1 : 0x4E, 0xF, 0xF, false));
        top = b ? recv : top;
        bot = b ? bot : recv;
    }
}

// Element (processing element index e in [0, N/2)) to thread.  With W wave
// bits (N >= 256) the stages split in two regions with a map each, so that
// every butterfly between stages of one region is a lane move, and the costly
// lane bits 0 and 1 (selects around a quad permutation) carry as few of them
// as possible: at stages 1..6, e's bits 0..4 sit on lane bits 1..5 and bit 5
// (moved only between stages 6 and 7) on lane bit 0; at stages 7..n, e's
// bits 0..2 sit on lane bits 0..2 (not moved there), its bits 6.. on the
// lane bits from 3 up, and its bits 3..5 above them.  The move from stage 6
// to 7 (and back) goes through LDS.  N <= 128 (one wave): e = t.
template <int W>
__device__ __forceinline__ int thread_of(int e, int s) {
    if constexpr (W == 0) {
        return e;
    } else if (s <= 6) {
        return ((e & 31) << 1) | ((e >> 5) & 1) | ((e >> 6) << 6);
    } else {
        return (e & 7) | (((e >> 6) & ((1 << W) - 1)) << 3) | (((e >> 3) & 7) << (3 + W));
    }
}

// Bank swizzle of the exchange slots: bits 7, 8, 9 of a slot index (the
// thread's bits 6, 7, 8) are xor-ed into bits 0, 1, 5, so that the
// transposition between stages 6 and 7 reads (and, backwards, writes) 64
// distinct banks per wave (32 at N = 256).  It keeps every slot within its
// 128-slot block (its wave's).
__device__ __forceinline__ int swz(int i) {
    return i ^ ((i >> 7) & 1) ^ (((i >> 8) & 1) << 1) ^ (((i >> 9) & 1) << 5);
}

template <int NLOG, int CN>
__global__ void __launch_bounds__(Alg1OLds<NLOG>::threads, 6) k_alg1o(Alg1Args a) {
    using Lay = Alg1OLds<NLOG>;
    constexpr int N = 1 << NLOG, n = NLOG, NP = N / 2, W = Lay::W;
    const int tid = threadIdx.x, nt = blockDim.x;
    extern __shared__ __align__(16) float smem[];
    float *const evr = smem + Lay::xfloats;  // R level l (1..n-1) at evr + (l-1) N
    float *const chan = evr + (size_t)(n - 1) * N;  // the frame's received LLRs
    int32_t *const misc = reinterpret_cast<int32_t *>(evr + Lay::evfloats);
    const float alpha = a.alpha;
    const float inf = __builtin_huge_valf();
    const int wave = tid >> 6, nwaves = (nt + 63) >> 6, lane = tid & 63;
    // the launch has N/2 threads when N >= 128, so every thread owns an element
    const bool pe = NP >= 64 || tid < NP;
    const int t = tid;
    // the thread's element at stages 1..6 and at stages 7..n
    const int eL = W > 0 ? (((t >> 1) & 31) | ((t & 1) << 5) | ((t >> 6) << 6)) : t;
    const int eH = W > 0 ? ((t & 7) | (((t >> 3) & ((1 << W) - 1)) << 6) | (((t >> (3 + W)) & 7) << 3)) : t;
    auto elem = [&](int s) -> int { return (W > 0 && s >= 7) ? eH : eL; };
    // the thread's two positions at stage s
    auto pos = [&](int s, int j) -> int { return insert0(elem(s), s - 1) + (j << (s - 1)); };

    // the permuted block (none: m = 0): stages rl..m (rr of them), rows
    // [blk << m, (blk + 1) << m), c_{rl+i} in 4-bit field i of cpk
    int rl = 0, m = 0, rr = 0, blk = -1;
    uint64_t cpk = 0;
    // position p of stage s's coordinates -> row, and back
    auto to_row = [&](int p, int s) -> int {
        if (m == 0 || s < rl || s > m || (p >> m) != blk) return p;
        int r = p & ~(((1 << rr) - 1) << (rl - 1));
        for (int i = 0; i < rr; ++i) r |= ((p >> (rl - 1 + i)) & 1) << (int)((cpk >> (4 * i)) & 15u);
        return r;
    };
    auto from_row = [&](int r, int s) -> int {
        if (m == 0 || s < rl || s > m || (r >> m) != blk) return r;
        int p = r & ~(((1 << rr) - 1) << (rl - 1));
        for (int i = 0; i < rr; ++i) p |= ((r >> (int)((cpk >> (4 * i)) & 15u)) & 1) << (rl - 1 + i);
        return p;
    };

    // messages: Li[s] = L_{s-1}, Ri[s] = R_s on the two positions of stage s
    float Li[n + 1][2], Ri[n + 1][2];
    // rows of the stage-n positions and their syndrome columns
    int rn0 = 0, rn1 = 0;
    uint32_t sy0 = 0u, sy1 = 0u;

    // Exchanges through LDS at a level b between stages b and b+1.  In the L
    // direction the stage-b thread stores its pair at its own slots 2 t,
    // 2 t + 1 and the stage-(b+1) thread loads the two slots that hold its
    // positions' rows; the R direction is the same move backwards (the
    // stage-(b+1) thread stores at those two slots, the stage-b thread loads
    // its own).  Three such levels: C = 6 (stage 6 <-> 7, when W > 0), A =
    // rl-1 and B = m (the block's boundaries, unless 0, n or C).  Per level
    // the two slots (bits 0..15 and 16..31), swizzled.
    uint32_t cS = 0u, aS = 0u, bS = 0u;
    // the thread's own pair: 2 t with the swizzle's upper bits, swapped when
    // it flips bit 0 (uniform over a wave)
    const int own = (W > 0 ? swz(2 * t) : 2 * t) & ~1;
    const bool own_swap = W > 0 && ((t >> 6) & 1) != 0;
    // L transitions after stage s through A or B (bit s), R transitions from
    // stage s through them (bit s), and which of A (bit 0) and B (bit 1) need a
    // workgroup barrier (an exchange within each wave needs none); uniform
    uint32_t lmask = 0u, rmask = 0u, abar = 0u;
    // A block of two stages (rho_range = 2) swaps bits rl-1 and rl, which in a
    // thread's pair is the butterfly on element bit rl-1 (element bit and slot
    // trade places).  Where that element bit sits on a lane bit, the block's
    // boundaries take that butterfly on the block's threads (fast: bit 0 A,
    // bit 1 B; lane bits kA, kB) in place of the exchange through LDS.
    uint32_t fast = 0u;
    int kA = 0, kB = 0;
    // alternating buffer of the exchanges with a barrier
    int xsel = 0;
    auto slot = [&](int b, int j) -> int {
        const int r = to_row(pos(b + 1, j), b + 1), q = from_row(r, b);
        const int i = 2 * thread_of<W>(remove_bit(q, b - 1), b) + ((q >> (b - 1)) & 1);
        return W > 0 ? swz(i) : i;
    };
    auto slots = [&](int b) -> uint32_t { return (uint32_t)slot(b, 0) | ((uint32_t)slot(b, 1) << 16); };
    // does the exchange of slots ss reach another wave (slot >> 7 is its wave)
    auto crosses = [&](uint32_t ss) -> bool {
        return (int)((ss & 0xFFFFu) >> 7) != wave || (int)(ss >> 23) != wave;
    };
    // The threads whose rows change coordinates at A: those with an element in
    // the block (the two stages share the thread map, and the butterfly there
    // pairs elements of one block); at B: the block's elements and their
    // butterfly partners, the elements of the sibling block, whose pairs at
    // stage m+1 hold one row of each.  Every other thread keeps its butterfly.
    auto in_a = [&](int e) -> bool { return (e >> (m - 1)) == blk; };
    auto in_b = [&](int e) -> bool { return (e >> m) == (blk >> 1); };
    // the lane bit that carries element bit k at stage s (6 and up: a wave bit)
    auto lane_bit = [&](int k, int s) -> int {
        if constexpr (W == 0) {
            return k;
        } else if (s <= 6) {
            return k <= 4 ? k + 1 : k == 5 ? 0 : 6;
        } else {
            return k <= 2 ? k : (k >= 6 && k < 6 + W) ? 3 + (k - 6) : 3 + W + (k - 3);
        }
    };
    // the butterfly on lane bit k (uniform), kept by the threads with sel; the
    // partner's value comes by ds_bpermute (one code path for every k)
    auto conv = [&](float &v0, float &v1, int k, bool sel) {
        const bool b = (lane >> k) & 1;
        const int recv = __builtin_amdgcn_ds_bpermute((lane ^ (1 << k)) << 2, __float_as_int(b ? v0 : v1));
        if (sel) {
            if (b)
                v0 = __int_as_float(recv);
            else
                v1 = __int_as_float(recv);
        }
    };
    // the exchange slots and masks for the current block (the C slots again
    // only if redo_c); the barrier needs are published as wave flags in
    // misc[32 + w] (read after the caller's next barrier)
    auto set_exchanges = [&](bool redo_c) {
        lmask = rmask = 0u;
        bool ca = false, cb = false;
        const bool hasA = m > 0 && rl >= 2 && !(W > 0 && rl - 1 == 6);
        const bool hasB = m > 0 && m < n && !(W > 0 && m == 6);
        fast = 0u;
        if (rr == 2) {
            kA = lane_bit(rl - 1, rl);
            kB = lane_bit(rl - 1, m);
            fast = (hasA && kA < 6 ? 1u : 0u) | (hasB && kB < 6 ? 2u : 0u);
        }
        if (hasA) {
            lmask |= 1u << (rl - 1);
            rmask |= 1u << rl;
        }
        if (hasB) {
            lmask |= 1u << m;
            rmask |= 1u << (m + 1);
        }
        if (pe) {
            if constexpr (W > 0)
                if (redo_c) cS = slots(6);
            if (hasA && !(fast & 1u) && in_a(elem(rl - 1))) {
                aS = slots(rl - 1);
                ca = crosses(aS);
            }
            if (hasB && !(fast & 2u) && in_b(elem(m))) {
                bS = slots(m);
                cb = crosses(bS);
            }
        }
        const uint32_t f = (__ballot(ca) != 0 ? 1u : 0u) | (__ballot(cb) != 0 ? 2u : 0u);
        if (lane == 0) misc[32 + wave] = (int32_t)f;
    };
    auto read_barrier_flags = [&]() {
        const uint32_t f = lane < nwaves ? (uint32_t)misc[32 + lane] : 0u;
        const uint64_t fa = __ballot((f & 1u) != 0), fb = __ballot((f & 2u) != 0);
        abar = (fa != 0 ? 1u : 0u) | (fb != 0 ? 2u : 0u);
    };
    // one exchange (backwards: the R direction): with a workgroup barrier
    // (alternating buffers) or within the waves (their own slots of the third
    // buffer)
    // (u0, u1): the pair the thread stores; only threads with `part` take part
    auto exchange = [&](float &v0, float &v1, float u0, float u1, uint32_t ss, bool barrier, bool back,
                        bool part) {
        float *const xb = smem + (size_t)(barrier ? xsel : 2) * N;
        if (barrier) xsel ^= 1;
        if (part) {
            if (back) {
                xb[ss & 0xFFFFu] = u0;
                xb[ss >> 16] = u1;
            } else {
                *reinterpret_cast<float2 *>(xb + own) = own_swap ? make_float2(u1, u0) : make_float2(u0, u1);
            }
        }
        if (barrier) {
            __syncthreads();
        } else {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
        if (part) {
            if (back) {
                const float2 v = *reinterpret_cast<const float2 *>(xb + own);
                v0 = own_swap ? v.y : v.x;
                v1 = own_swap ? v.x : v.y;
            } else {
                v0 = xb[ss & 0xFFFFu];
                v1 = xb[ss >> 16];
            }
        }
    };

    // the channel level of row r after event e (e = 0: none yet), from the
    // frame's LLRs in LDS
    auto channel = [&](int64_t frame, int e, int r) -> float {
        if (e == 0) return chan[r];
        const float z = a.noise_sigma * noise_gauss(a.noise_seed, frame, e, r);
        return chan[r] + z;
    };
    auto load_channel = [&](int64_t frame, int e) {
        if (!pe) return;
        Li[1][0] = channel(frame, e, to_row(pos(1, 0), 1));
        Li[1][1] = channel(frame, e, to_row(pos(1, 1), 1));
    };
    auto load_stage_n = [&]() {
        if (!pe) return;
        rn0 = to_row(pos(n, 0), n);
        rn1 = to_row(pos(n, 1), n);
        Ri[n][0] = a.meta[rn0] == -2 ? inf : 0.f;
        Ri[n][1] = a.meta[rn1] == -2 ? inf : 0.f;
        sy0 = a.syn[rn0];
        sy1 = a.syn[rn1];
    };
    // the decision: syndrome (and hash) partials of the wave
    auto publish = [&](uint32_t syn, uint64_t h) {
        const uint32_t v = lanes_xor<64>(syn);
        if (lane == 0) misc[4 + wave] = (int32_t)v;
        if (a.hist) {
            const uint32_t lo = lanes_xor<64>((uint32_t)h), hi = lanes_xor<64>((uint32_t)(h >> 32));
            if (lane == 0) {
                misc[64 + 2 * wave] = (int32_t)lo;
                misc[65 + 2 * wave] = (int32_t)hi;
            }
        }
    };
    // after a barrier that follows publish: the verdict, and the hash recorded
    auto gather = [&](int64_t frame, int it) -> bool {
        const uint32_t p = lane < nwaves ? (uint32_t)misc[4 + lane] : 0u;
        const bool pass = lanes_xor<64>(p) == 0u;
        if (a.hist && tid == 0) {
            uint64_t h = 0;
            for (int w = 0; w < nwaves; ++w)
                h ^= ((uint64_t)(uint32_t)misc[65 + 2 * w] << 32) | (uint32_t)misc[64 + 2 * w];
            a.hist[frame * a.H + (it - 1) % a.H] = h;
        }
        return pass;
    };

    for (;;) {
        __syncthreads();
        if (tid == 0) misc[0] = (int32_t)atomicAdd(a.counter, 1u);
        __syncthreads();
        const int64_t frame = misc[0];
        if (frame >= a.F) break;

        // ---- initialise L and R (Alg. 1 initializeLandR) ----
        const float *src = a.llr + frame * N;
        sfor<0, n + 1>([&](auto l) {
            Li[l][0] = Li[l][1] = 0.f;
            Ri[l][0] = Ri[l][1] = 0.f;
        });
        uint64_t st = a.seed + (uint64_t)(frame + 1) * 0x9E3779B97F4A7C15ull;
        int next_reset = alg1_first_event(a, N, n);
        int ev = 0;
        rl = m = rr = 0;
        blk = -1;
        cpk = 0;
        for (int r = tid; r < N; r += nt) chan[r] = src[r];
        load_stage_n();
        set_exchanges(true);  // no block: only C, which crosses waves by construction
        __syncthreads();      // the channel copy
        load_channel(frame, 0);
        abar = 0u;

        float ln0 = 0.f, ln1 = 0.f;  // L level n on the stage-n positions
        int it_done = a.max_iter;
        bool okv = false;
        for (int it = 1; it <= a.max_iter; ++it) {
            // ---- L sweep, stages 1..n ----
            sfor<1, n + 1>([&](auto sc) {
                constexpr int s = sc;
                const float a0 = Li[s][0], a1 = Li[s][1], r0 = Ri[s][0], r1 = Ri[s][1];
                // top: f(L[j], L[j'] + R[j']); bottom: f(L[j], R[j]) + L[j']
                float lt = alg1_check<CN>(a0, a1 + r1, alpha);
                float lb = alg1_check<CN>(a0, r0, alpha) + a1;
                if constexpr (s < n) {
                    if constexpr (W > 0 && s == 6) {
                        exchange(lt, lb, lt, lb, cS, true, false, pe);
                    } else {
                        // the butterfly in place; at a block boundary the
                        // threads whose rows change coordinates move the pair
                        // they had (the butterfly undone on copies: it is an
                        // involution) through LDS instead
                        constexpr int K = W == 0 ? s - 1 : s >= 7 ? s - 4 : s;
                        bfly_wave<K>(lt, lb, lane);
                        if (__builtin_expect((lmask >> s) & 1u, 0)) {
                            float u0 = lt, u1 = lb;
                            bfly_wave<K>(u0, u1, lane);
                            if (s == rl - 1) {
                                if (fast & 1u)  // into a two-stage block's coordinates
                                    conv(lt, lb, kA, in_a(elem(s)));
                                else
                                    exchange(lt, lb, u0, u1, aS, abar & 1u, false, pe && in_a(elem(s)));
                            } else if (fast & 2u) {
                                // out of a two-stage block: back to row order, then the butterfly
                                conv(u0, u1, kB, in_a(elem(s)));
                                lt = u0;
                                lb = u1;
                                bfly_wave<K>(lt, lb, lane);
                            } else {
                                exchange(lt, lb, u0, u1, bS, abar & 2u, false, pe && in_b(elem(s)));
                            }
                        }
                    }
                    Li[s + 1][0] = lt;
                    Li[s + 1][1] = lb;
                } else {
                    ln0 = lt;
                    ln1 = lb;
                }
            });
            // ---- decision and CRC syndrome on level n+1 ----
            const bool one0 = pe && ln0 + Ri[n][0] < 0.f, one1 = pe && ln1 + Ri[n][1] < 0.f;
            const uint32_t syn = (one0 ? sy0 : 0u) ^ (one1 ? sy1 : 0u);
            const uint64_t h = a.hist ? ((one0 ? decision_key(rn0) : 0ull) ^ (one1 ? decision_key(rn1) : 0ull)) : 0ull;
            const bool can_stop = a.stop == PC_STOP_CRC && it >= a.it_min;
            bool done = false;
            if constexpr (W == 0) {
                // one wave: the verdict at once
                const bool pass = lanes_xor<64>(syn) == 0u;
                if (a.hist && tid == 0) {
                    const uint64_t hh = ((uint64_t)lanes_xor<64>((uint32_t)(h >> 32)) << 32) |
                                        lanes_xor<64>((uint32_t)h);
                    a.hist[frame * a.H + (it - 1) % a.H] = hh;
                }
                if (can_stop && pass) {
                    it_done = it;
                    okv = true;
                    break;
                }
                if (it == a.max_iter) {
                    okv = pass;
                    break;
                }
            } else {
                publish(syn, h);
                if (it == a.max_iter) {
                    __syncthreads();
                    okv = gather(frame, it);
                    break;
                }
            }
            // ---- R sweep, stages n..2 (R on the channel level is never read);
            // with several waves the verdict is taken at its stage 7 -> 6
            // exchange, whose barrier follows every wave's partials ----
            sfor<0, n - 1>([&](auto kc) {
                constexpr int s = n - kc;
                float q0 = Li[s][0], q1 = Li[s][1];
                const float p0 = Ri[s][0], p1 = Ri[s][1];
                // hidden from the optimiser: otherwise it keeps the magnitude and
                // sign of the L sweep's bounds in registers for this use (two
                // more instructions and registers per stage)
                asm volatile("" : "+v"(q0), "+v"(q1));
                // top: f(L[j'] + R[j'], R[j]); bottom: f(L[j], R[j]) + R[j']
                float rt = alg1_check<CN>(q1 + p1, p0, alpha);
                float rb = alg1_check<CN>(q0, p0, alpha) + p1;
                if constexpr (W > 0 && s == 7) {
                    exchange(rt, rb, rt, rb, cS, true, true, pe);
                    if (gather(frame, it) && can_stop) done = true;
                } else {
                    constexpr int K = W == 0 ? s - 2 : s >= 8 ? s - 5 : s - 1;
                    bfly_wave<K>(rt, rb, lane);
                    if (__builtin_expect((rmask >> s) & 1u, 0)) {
                        float u0 = rt, u1 = rb;
                        bfly_wave<K>(u0, u1, lane);
                        if (s == rl) {
                            if (fast & 1u) {
                                // out of a two-stage block: back to row order, then the butterfly
                                conv(u0, u1, kA, in_a(elem(s)));
                                rt = u0;
                                rb = u1;
                                bfly_wave<K>(rt, rb, lane);
                            } else {
                                exchange(rt, rb, u0, u1, aS, abar & 1u, true, pe && in_a(elem(s)));
                            }
                        } else if (fast & 2u) {
                            conv(rt, rb, kB, in_a(elem(s)));  // into a two-stage block's coordinates
                        } else {
                            exchange(rt, rb, u0, u1, bS, abar & 2u, true, pe && in_b(elem(s)));
                        }
                    }
                }
                Ri[s - 1][0] = rt;
                Ri[s - 1][1] = rb;
            });
            if (done) {
                it_done = it;
                okv = true;
                break;
            }
            // ---- partial permutation of one subgraph (Alg. 1 partialPermute) ----
            if (it == next_reset) {
                const int nrr = 2 + (int)draw_below(st, (uint32_t)(a.P_range - 1));
                const int x = 1 + (int)draw_below(st, (uint32_t)a.P_level);
                const int nrl = x < n - nrr + 1 ? x : n - nrr + 1;
                const int nm = nrl + nrr - 1;
                const int nblk = (int)draw_below(st, (uint32_t)(N >> nm));
                int8_t cand[kMaxLog];
                bool same = true;
                while (same) {
                    for (int i = 0; i < nrr; ++i) cand[i] = (int8_t)(nrl - 1 + i);
                    for (int i = nrr - 1; i >= 1; --i) {
                        const int jj = (int)draw_below(st, (uint32_t)(i + 1));
                        const int8_t tt = cand[i];
                        cand[i] = cand[jj];
                        cand[jj] = tt;
                    }
                    same = true;
                    for (int i = 0; i < nrr; ++i) same &= cand[i] == nrl - 1 + i;
                }
                // N_zero: this block's inner nodes and the previous block's,
                // counted once where they overlap (aligned blocks nest or are
                // disjoint)
                int n_zero = (1 << nm) * (nrr - 1);
                if (m > 0) {
                    const int lo = rl > nrl ? rl : nrl, hi = (m < nm ? m : nm) - 1;
                    const bool nested = m <= nm ? (blk >> (nm - m)) == nblk : (nblk >> (m - nm)) == blk;
                    const int shared = nested && hi >= lo ? (1 << (m < nm ? m : nm)) * (hi - lo + 1) : 0;
                    n_zero += (1 << m) * (m - rl) - shared;
                }
                // the R levels whose coordinates change (those of the old and the
                // new block's stages), at their rows in the old coordinates, with
                // the inner levels of both blocks reset
                const uint32_t lv_old = m > 0 ? ((2u << m) - (1u << rl)) : 0u;
                const uint32_t lv = (lv_old | ((2u << nm) - (1u << nrl))) & ((1u << n) - 2u);
                const int orl = rl, om = m, oblk = blk;
                // only threads with an element in the old or the new block at
                // level l hold rows there whose coordinates change or that are
                // reset; the rows of a block move among its own threads
                auto moves = [&](int l) -> bool {
                    const int e = elem(l);
                    return (om > 0 && l >= orl && l <= om && (e >> (om - 1)) == oblk) ||
                           (l >= nrl && l <= nm && (e >> (nm - 1)) == nblk);
                };
                if (pe) {
                    sfor<1, n>([&](auto lc) {
                        constexpr int l = lc;
                        if (((lv >> l) & 1u) && moves(l)) {
                            sfor<0, 2>([&](auto j) {
                                const int r = to_row(pos(l, j), l);
                                const bool z = (om > 0 && l >= orl && l < om && (r >> om) == oblk) ||
                                               (l >= nrl && l < nm && (r >> nm) == nblk);
                                evr[(size_t)(l - 1) * N + r] = z ? 0.f : Ri[l][j];
                            });
                        }
                    });
                }
                rl = nrl;
                m = nm;
                rr = nrr;
                blk = nblk;
                cpk = 0;
                for (int i = 0; i < nrr; ++i) cpk |= (uint64_t)(uint8_t)cand[i] << (4 * i);
                int add = a.D > 0 ? n_zero / a.D : 0;
                if (add < a.N_min) add = a.N_min;
                next_reset = it + add;
                set_exchanges((orl <= 7 && om >= 6) || (rl <= 7 && m >= 6));
                __syncthreads();  // the rows above and the exchange flags
                read_barrier_flags();
                // the R levels back, in the new coordinates (the event area is
                // next written at the next event, after the decision's barriers)
                if (pe) {
                    sfor<1, n>([&](auto lc) {
                        constexpr int l = lc;
                        if (((lv >> l) & 1u) && moves(l)) {
                            Ri[l][0] = evr[(size_t)(l - 1) * N + to_row(pos(l, 0), l)];
                            Ri[l][1] = evr[(size_t)(l - 1) * N + to_row(pos(l, 1), l)];
                        }
                    });
                }
                // the channel level (fresh channel noise at every event), and the
                // stage-n tables if their coordinates changed
                if (a.noise_sigma > 0.f) ++ev;
                if (a.noise_sigma > 0.f || orl == 1 || rl == 1) load_channel(frame, ev);
                if (om == n || m == n) load_stage_n();
            }
        }

        // ---- outputs (Alg. 1 hardDecision) ----
        uint8_t *mo = a.msg + frame * a.K_msg;
        if (pe) {
            const int mi0 = a.meta[rn0], mi1 = a.meta[rn1];
            if (mi0 >= 0) mo[mi0] = ln0 + Ri[n][0] < 0.f ? 1 : 0;
            if (mi1 >= 0) mo[mi1] = ln1 + Ri[n][1] < 0.f ? 1 : 0;
            if (a.soft) {
                a.soft[frame * N + rn0] = ln0;
                a.soft[frame * N + rn1] = ln1;
            }
        }
        if (tid == 0) {
            if (a.iters) a.iters[frame] = it_done;
            if (a.ok) a.ok[frame] = okv ? 1 : 0;
        }
    }
}

template <int NLOG>
static int run_n(const Alg1Args &a, int cn, hipStream_t s) {
    constexpr size_t lds = Alg1OLds<NLOG>::bytes;
    static_assert(lds <= 160 * 1024, "Algorithm 1 frame exceeds LDS");
    const int threads = Alg1OLds<NLOG>::threads;
    auto kern = cn == 2 ? k_alg1o<NLOG, 2> : cn == 1 ? k_alg1o<NLOG, 1> : k_alg1o<NLOG, 0>;
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

int run_alg1_orig(const Alg1Args &a, int n, int cn, hipStream_t s) {
    switch (n) {
        case 4: return run_n<4>(a, cn, s);
        case 5: return run_n<5>(a, cn, s);
        case 6: return run_n<6>(a, cn, s);
        case 7: return run_n<7>(a, cn, s);
        case 8: return run_n<8>(a, cn, s);
        case 9: return run_n<9>(a, cn, s);
        default: return run_n<10>(a, cn, s);
    }
}

}  // namespace pbp
