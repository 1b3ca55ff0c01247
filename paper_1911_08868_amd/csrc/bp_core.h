// bp_core.h -- device building blocks of the belief-propagation kernels
// (gfx950, wave64): the stage-group plan, the thread -> row map, the
// processing element of Sec. II-B and the register-resident group passes.
//
// Layout of one frame on the GPU.  A frame of N = 2^n rows is decoded by
// TPS = N / 2^RHO threads; each thread owns 2^RHO rows of every level.  The n
// stages are cut into groups of at most RHO consecutive stages; inside a
// group all stage bits are register bits of the thread, so its processing
// elements run on registers with no data exchange.  Only the two messages of
// a group boundary level cross threads, through LDS, once per sweep.  The
// persistent R messages and the L messages of the current iteration stay in
// registers.
//
// Multi-trellis by relabelling.  BP on a graph whose stages 1..n use bits
// e_1..e_n equals BP on the original graph after the rows are relabelled by
// the bit permutation (relabelled bit s-1 = original bit e_s).  The permuted
// last-k stages therefore run in relabelled coordinates with the same
// register code as the original graph; only the accesses to the level below
// the permuted range, the prior and the decisions go through the row map,
// and the levels strictly inside the permuted range, which a permutation
// resets anyway (Sec. III), never need moving.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>
#include <utility>

namespace pbp {

template <int B, int E, class Fn>
__device__ __forceinline__ void sfor(Fn &&fn) {
    if constexpr (B < E) {
        fn(std::integral_constant<int, B>{});
        sfor<B + 1, E>(fn);
    }
}

// ---------------------------------------------------------------------------
// Compile-time plan: n = log2 N, KP permuted last stages (0 = none), RHO =
// log2 rows per thread per level.  Stages 1..n-KP (the unpermuted part) and
// n-KP+1..n (the permuted part) are each split into groups of at most RHO
// stages, so a group boundary sits at level n-KP (0-based level = number of
// stages below it).
template <int NLOG, int KP, int RHO>
struct Plan {
    static_assert(RHO >= 1 && RHO <= NLOG, "rows per thread exceed the frame");
    static_assert(KP == 0 || (KP >= 2 && KP <= NLOG), "permuted range");
    static constexpr int n = NLOG;
    static constexpr int N = 1 << NLOG;
    static constexpr int rho = RHO;
    static constexpr int ROWS = 1 << RHO;
    static constexpr int TPS = N / ROWS;
    static constexpr int NB = NLOG - KP;
    static constexpr int GB = (NB + RHO - 1) / RHO;
    static constexpr int GT = (KP + RHO - 1) / RHO;
    static constexpr int G = GB + GT;
    static constexpr int kp = KP;
    // first stage (0-based) of group g == its bottom level
    static constexpr int lo(int g) {
        if (g <= GB) {
            int s = 0;
            for (int i = 0; i < g; ++i) s += NB / GB + (i < NB % GB ? 1 : 0);
            return s;
        }
        int s = NB;
        for (int i = 0; i < g - GB; ++i) s += KP / GT + (i < KP % GT ? 1 : 0);
        return s;
    }
    static constexpr int size(int g) { return lo(g + 1) - lo(g); }
    static constexpr int RMAX = RHO;
    static constexpr int RI = RHO > 1 ? RHO - 1 : 1;  // interior-level array extent
    static constexpr int WPS = TPS >= 64 ? TPS / 64 : 1;  // waves per slot
};

// Padded layout of one boundary buffer in LDS: PAD words after every 2^SH
// rows break the power-of-two strides with which the thread -> row maps
// would otherwise hit the same banks (2- to 8-way conflicts).  A thread's
// base row and a register's offset occupy disjoint bits, so the padded
// address is a per-thread part plus a compile-time constant.  PAD is a
// multiple of 4, so the rows a thread owns contiguously stay 16-byte aligned.
template <class P>
struct LdsPad {
    static constexpr int SH = P::rho == 2 ? (P::n >= 8 ? 6 : 5) : (P::n >= 9 ? 6 : 5);
    static constexpr int PAD = P::n <= 5 ? 0 : (P::rho == 2 ? 12 : (P::n >= 9 ? 8 : 4));
    static constexpr int words = P::N + PAD * (P::N >> SH);
    __host__ __device__ static constexpr int at(int row) { return row + PAD * (row >> SH); }
};

// Thread -> row map of group g.  Register index i: its low r bits are the
// group's stage bits (positions lo..lo+r-1); the thread index t fills the
// remaining positions from the lowest up, and the high RHO-r bits of i fill
// what is left.  Consecutive threads therefore touch consecutive rows
// whenever lo > 0, and each thread's rows are contiguous when lo == 0.
template <class P, int g>
struct GMap {
    static constexpr int lo = P::lo(g);
    static constexpr int r = P::size(g);
    static constexpr int tbits = P::n - P::rho;
    static constexpr int off(int i) {
        int low = i & ((1 << r) - 1), high = i >> r;
        int o = low << lo;
        int c = 0, hb = 0;
        for (int p = 0; p < P::n; ++p) {
            if (p >= lo && p < lo + r) continue;
            if (c >= tbits) {
                if ((high >> hb) & 1) o |= 1 << p;
                ++hb;
            }
            ++c;
        }
        return o;
    }
    __device__ static __forceinline__ int base(int t) {
        if constexpr (tbits <= lo) {
            return t;
        } else {
            return (t & ((1 << lo) - 1)) | ((t >> lo) << (lo + r));
        }
    }
    // row position of thread-index bit k (k < tbits): the non-stage
    // positions in increasing order
    static constexpr int tpos(int k) { return k < lo ? k : k + r; }
    // the same rows in the padded LDS layout
    __device__ static __forceinline__ int pbase(int t) { return LdsPad<P>::at(base(t)); }
    static constexpr int poff(int i) { return LdsPad<P>::at(off(i)); }
};

// Is the exchange across the boundary between groups g and g+1 local to each
// wave?  Then no workgroup barrier is needed there: each wave reads only rows
// its own lanes wrote, and one wave's LDS accesses execute in order.  True
// when a frame fits in one wave, or when the wave-index bits of the thread
// index (bits 6.. of t) sit at the same row positions in both groups and, at
// the relabelled boundary, below the permuted range.
template <class P, int g>
constexpr bool wave_local_boundary(bool mapped_at_gb) {
    if constexpr (P::TPS <= 64) {
        return true;
    } else {
        constexpr int tb = P::n - P::rho;
        for (int k = 6; k < tb; ++k) {
            const int a = GMap<P, g>::tpos(k), b = GMap<P, g + 1>::tpos(k);
            if (a != b) return false;
            if (mapped_at_gb && g + 1 == P::GB && a >= P::n - P::kp) return false;
        }
        return true;
    }
}

// ---------------------------------------------------------------------------
// Check function of the processing element (Sec. II-B): min-sum
// sign(x) sign(y) min(|x|,|y|), optionally scaled.  The sign is the xor of the
// sign bits; the magnitude min(|x|,|y|) is exact; the only rounding is that
// of the scale.  Finite inputs and +inf priors never produce NaN.
// The magnitude uses IEEE-754-2019 minimum (v_minimum3_f32 on gfx950): on the
// non-negative, non-NaN magnitudes it equals fmin, and unlike fmin it needs no
// signalling-NaN quieting of its inputs.
template <bool SCALED>
__device__ __forceinline__ float cnode(float x, float y, float alpha) {
    float m = __builtin_elementwise_minimum(__builtin_fabsf(x), __builtin_fabsf(y));
    if constexpr (SCALED) m = alpha * m;
    uint32_t s = (__float_as_uint(x) ^ __float_as_uint(y)) & 0x80000000u;
    return __uint_as_float(__float_as_uint(m) | s);
}

// The same check function in clamp form, two instructions on gfx950: y
// clamped to [-|x|, |x|] (v_med3_f32 with abs/neg source modifiers) has the
// sign of y and the magnitude min(|x|,|y|); flipping its sign bit by that of
// x (v_bitop3_b32) gives sign(x) sign(y) min(|x|,|y|).  Every nonzero result
// equals cnode's bit for bit; a zero result (both inputs zero) may carry the
// other sign.  A zero's sign reaches no nonzero message (it only meets the
// check function, whose zero stays zero, and additions, where a nonzero
// addend wins) and no decision (-0 and +0 both decide 0), so decoding is
// unchanged.  The bound x should be the operand less likely to be zero.
//
// CN selects the check function: 0 min-sum, 1 scaled min-sum, 2 the exact
// boxplus below.
__device__ __forceinline__ float cnode_exact(float x, float y);

template <int CN>
__device__ __forceinline__ float cnode_clamp(float x, float y, float alpha) {
    if constexpr (CN == 2) {
        return cnode_exact(x, y);
    } else {
        const float ax = __builtin_fabsf(x);
        float t = __builtin_amdgcn_fmed3f(y, ax, -ax);
        if constexpr (CN == 1) t = alpha * t;
        return __uint_as_float(__float_as_uint(t) ^ (__float_as_uint(x) & 0x80000000u));
    }
}

// ln(1 + e^-d) for d >= 0 (or +inf), in base 2: log2(1 + 2^(-d log2 e)) on
// v_exp_f32 and v_log_f32; 1 + 2^(...) rounds to 1 once e^-d < 2^-24, where
// the true value is below 6e-8.
__device__ __forceinline__ float log2_1p_exp_neg(float d) {
    return __builtin_amdgcn_logf(1.0f + __builtin_amdgcn_exp2f(d * -1.44269504088896341f));
}

// Exact boxplus 2 atanh(tanh(x/2) tanh(y/2)) (Sec. II-B) as
// sgn(x) sgn(y) [min(|x|,|y|) + ln(1 + e^-(|x|+|y|)) - ln(1 + e^-||x|-|y||)],
// the same function without the saturation of the tanh form.  The difference
// of two infinite magnitudes (NaN) is replaced by the largest float through
// IEEE minNum (v_min_f32), whose correction term is 0, so +inf against +inf
// gives +inf as the limit does; +inf against a finite y gives y; a rounding
// that takes the magnitude below 0 gives 0.  The magnitude's minimum and the
// clamp use the IEEE-754-2019 minimum/maximum (no NaN reaches them); the last
// step is one fused multiply-add.
__device__ __forceinline__ float cnode_exact(float x, float y) {
    const float ax = __builtin_fabsf(x), ay = __builtin_fabsf(y);
    const float m = __builtin_elementwise_minimum(ax, ay);
    const float d = __builtin_fminf(__builtin_fabsf(ax - ay), 3.40282347e38f);
    const float l = log2_1p_exp_neg(ax + ay) - log2_1p_exp_neg(d);
    const float mag = __builtin_elementwise_maximum(__builtin_fmaf(l, 0.693147180559945309f, m), 0.f);
    return __uint_as_float(__float_as_uint(mag) ^ ((__float_as_uint(x) ^ __float_as_uint(y)) & 0x80000000u));
}

// ---------------------------------------------------------------------------
// Register state of one thread for one frame.
template <class P>
struct Regs {
    float Rint[P::G][P::RI][P::ROWS];  // R on interior levels of each group (persistent)
    float Lint[P::G][P::RI][P::ROWS];  // L on interior levels (current iteration)
    float Lbot[P::G][P::ROWS];         // L on each group's bottom level
    float Rtop[P::G][P::ROWS];         // R on each group's top level (g < G-1)
    float Ltop[P::ROWS];               // L on level n after the last L sweep
};

// L sweep over the stages of group g: input L on its bottom level (Lbot),
// R on its interior levels and top level; output L on its interior levels
// and on its top level (returned in `out`).  `rtop` is the R of the top
// level (the prior for the last group).
template <class P, int g, int CN>
__device__ __forceinline__ void group_L(Regs<P> &S, const float (&rtop)[P::ROWS],
                                        float (&out)[P::ROWS], float alpha) {
    constexpr int r = P::size(g);
    float cur[P::ROWS];
    sfor<0, P::ROWS>([&](auto i) { cur[i] = S.Lbot[g][i]; });
    sfor<0, r>([&](auto sl) {
        float nxt[P::ROWS];
        sfor<0, P::ROWS>([&](auto i) {
            constexpr int b = 1 << sl;
            if constexpr ((i & b) == 0) {
                constexpr int ip = i | b;
                float r1, r2;
                if constexpr (sl + 1 < r) {
                    r1 = S.Rint[g][sl][i];
                    r2 = S.Rint[g][sl][ip];
                } else {
                    r1 = rtop[i];
                    r2 = rtop[ip];
                }
                const float l1 = cur[i], l2 = cur[ip];
                nxt[i] = cnode_clamp<CN>(l1, l2 + r2, alpha);
                nxt[ip] = cnode_clamp<CN>(l1, r1, alpha) + l2;
            }
        });
        if constexpr (sl + 1 < r) {
            sfor<0, P::ROWS>([&](auto i) { S.Lint[g][sl][i] = nxt[i]; });
        }
        sfor<0, P::ROWS>([&](auto i) { cur[i] = nxt[i]; });
    });
    sfor<0, P::ROWS>([&](auto i) { out[i] = cur[i]; });
}

// R sweep over the stages of group g, top to bottom: input R on its top level
// (`rtop`), L on its interior and bottom levels; output R on its interior
// levels and on its bottom level (returned in `out`).
template <class P, int g, int CN>
__device__ __forceinline__ void group_R(Regs<P> &S, const float (&rtop)[P::ROWS],
                                        float (&out)[P::ROWS], float alpha) {
    constexpr int r = P::size(g);
    float cur[P::ROWS];
    sfor<0, P::ROWS>([&](auto i) { cur[i] = rtop[i]; });
    sfor<0, r>([&](auto k) {
        constexpr int sl = r - 1 - k;
        float nxt[P::ROWS];
        sfor<0, P::ROWS>([&](auto i) {
            constexpr int b = 1 << sl;
            if constexpr ((i & b) == 0) {
                constexpr int ip = i | b;
                float l1, l2;
                if constexpr (sl > 0) {
                    l1 = S.Lint[g][sl - 1][i];
                    l2 = S.Lint[g][sl - 1][ip];
                } else {
                    l1 = S.Lbot[g][i];
                    l2 = S.Lbot[g][ip];
                }
                const float r1 = cur[i], r2 = cur[ip];
                nxt[i] = cnode_clamp<CN>(l2 + r2, r1, alpha);
                nxt[ip] = cnode_clamp<CN>(l1, r1, alpha) + r2;
            }
        });
        if constexpr (sl > 0) {
            sfor<0, P::ROWS>([&](auto i) { S.Rint[g][sl - 1][i] = nxt[i]; });
        }
        sfor<0, P::ROWS>([&](auto i) { cur[i] = nxt[i]; });
    });
    sfor<0, P::ROWS>([&](auto i) { out[i] = cur[i]; });
}

// float at a byte offset from p (precomputed byte offsets save the scaling)
__device__ __forceinline__ float &byte_at(float *p, int byte_off) {
    return *reinterpret_cast<float *>(reinterpret_cast<char *>(p) + byte_off);
}
__device__ __forceinline__ float byte_at(const float *p, int byte_off) {
    return *reinterpret_cast<const float *>(reinterpret_cast<const char *>(p) + byte_off);
}

// Synchronisation at a group boundary: a workgroup barrier, or, where the
// exchange stays inside each wave, only a compiler barrier that keeps the
// LDS stores before the loads.
template <bool WAVE_LOCAL>
__device__ __forceinline__ void boundary_sync() {
    if constexpr (WAVE_LOCAL) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}

// relabelled row p -> original row for stage order e[0..n-1]: bit s of p is
// bit e[s] of the original row.  Only bits lowbits..n-1 can move.
__device__ __forceinline__ int relabel_to_row(int p, const int8_t *e, int n, int lowbits) {
    int j = p & ((1 << lowbits) - 1);
    for (int s = lowbits; s < n; ++s) j |= ((p >> s) & 1) << e[s];
    return j;
}

// xor-reduce over groups of W consecutive lanes (W a power of two <= 64,
// groups aligned to W); every lane of a group receives the result.  Within a
// 16-lane row the steps are DPP lane swaps (quad_perm, row_half_mirror,
// row_mirror); across rows the four row totals are read with readlane.
template <int CTRL>
__device__ __forceinline__ uint32_t swap_dpp(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)0, (int)v, CTRL, 0xF, 0xF, true);
}

template <int W>
__device__ __forceinline__ uint32_t lanes_xor(uint32_t v) {
    static_assert(W >= 1 && W <= 64 && (W & (W - 1)) == 0, "power-of-two lane group");
    if constexpr (W >= 2) v ^= swap_dpp<0xB1>(v);   // quad_perm [1,0,3,2]: lane ^ 1
    if constexpr (W >= 4) v ^= swap_dpp<0x4E>(v);   // quad_perm [2,3,0,1]: lane ^ 2
    if constexpr (W >= 8) v ^= swap_dpp<0x141>(v);  // row_half_mirror: the other quad of 8
    if constexpr (W >= 16) v ^= swap_dpp<0x140>(v); // row_mirror: the other half of 16
    if constexpr (W == 32) v ^= (uint32_t)__shfl_xor((int)v, 16, 64);
    if constexpr (W == 64) {
        v = (uint32_t)(__builtin_amdgcn_readlane((int)v, 0) ^ __builtin_amdgcn_readlane((int)v, 16) ^
                       __builtin_amdgcn_readlane((int)v, 32) ^ __builtin_amdgcn_readlane((int)v, 48));
    }
    return v;
}

// SplitMix64 (Steele, Lea, Flood 2014): add the golden-ratio increment, then
// two xor-shift-multiply rounds.
__device__ __forceinline__ uint64_t splitmix64_next(uint64_t &s) {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Noise of the noise-aided schedules: an Irwin-Hall approximation of N(0,1)
// for (frame, event e, row j): the twelve 16-bit fields k of three SplitMix64
// outputs from the state seed ^ frame 0x9E3779B97F4A7C15 ^ e 0xC2B2AE3D27D4EB4F
// ^ j 0x165667B19E3779F9, each read as (k + 1/2) / 2^16, summed, minus 6.
// The result is a multiple of 2^-16 in (-6, 6), exact in single precision.
__device__ __forceinline__ float noise_gauss(uint64_t seed, int64_t frame, int e, int j) {
    uint64_t s = seed ^ ((uint64_t)frame * 0x9E3779B97F4A7C15ull) ^
                 ((uint64_t)(uint32_t)e * 0xC2B2AE3D27D4EB4Full) ^
                 ((uint64_t)(uint32_t)j * 0x165667B19E3779F9ull);
    uint32_t sum = 6;
    for (int r = 0; r < 3; ++r) {
        const uint64_t o = splitmix64_next(s);
        sum += (uint32_t)(o & 0xFFFFu) + (uint32_t)((o >> 16) & 0xFFFFu) + (uint32_t)((o >> 32) & 0xFFFFu) +
               (uint32_t)(o >> 48);
    }
    return (float)sum * (1.0f / 65536.0f) - 6.0f;
}

// Zobrist key of row j for the decision history (error classes, Sec. II-C):
// the first SplitMix64 output from state j.  The hash of a decision vector
// is the xor of the keys of its ones.
__device__ __forceinline__ uint64_t decision_key(int j) {
    uint64_t s = (uint64_t)(uint32_t)j;
    return splitmix64_next(s);
}

}  // namespace pbp
