// wbp_kernel.h -- weighted (unrolled) BP: forward with message checkpoints and
// the hand-written adjoint (gfx950).
//
// Each check-node output of iteration t, stage s, sweep d (0 = L, 1 = R) is
// scaled by w[t][s-1][d][pos], pos the output's position in the drawing of the
// active trellis -- the row index the relabelled kernels already work in.
// Frozen priors are the finite 2^60 so that zero adjoints times huge messages
// stay zero.  There is no early stop; the output is o = L + R on level n+1
// after the last L sweep, so the last R sweep is never run.
//
// Layout and thread map are those of the decode kernels (bp_core.h); a
// workgroup holds S frames in lock step without refill (every frame runs T
// iterations).  The forward pass stores the R state entering each iteration
// t >= 1 (levels 1..n-1, (n-1) N floats per frame) in the thread's register
// order, so stores and loads are coalesced across threads.
//
// The adjoint walks the iterations backwards.  For iteration t it reloads the
// entering R state, recomputes the L sweep (keeping every L level) and the R
// sweep (keeping every R level), then runs the reverse of the R sweep over the
// groups bottom to top and the reverse of the L sweep top to bottom.  Adjoints
// of the two boundary messages cross groups through LDS like the messages.
// Min-sum derivative: for g = sgn(x) sgn(y) min(|x|,|y|), if |x| <= |y| then
// dg/dx = sgn(y), else dg/dy = sgn(x) (ties route to the first argument).
// Each reverse step stages the weight gradients of its group per frame in LDS;
// the next step (after the barrier that ends this one) sums them over the
// workgroup's frames in slot order and adds them into this workgroup's
// partial.  The adjoint's grid is fixed; each workgroup walks its batches of
// frames in order, the first storing the partial and the rest adding to it.
// A two-level reduction then sums the partials in workgroup order, so the
// result does not depend on scheduling or on the device.
#pragma once

#include "bp_core.h"

namespace pbp {

constexpr float kWbpPrior = 1152921504606846976.0f;  // 2^60
// block lengths from 2^kWbpBigLog on take the large-frame adjoint (k_wbp_bwd_big)
constexpr int kWbpBigLog = 11;

struct WbpArgs {
    const float *llr;
    int64_t F;
    const float *w;        // [T][n][2][N]
    int32_t T;
    float *out;            // [F][N] forward output
    const float *gout;     // [F][N] adjoint of the output
    float *ckpt;           // [F][T-1][(n-1) N]
    float *partial;        // [gridDim][T][n][2][N]
    float *scratch;        // large frames: per-workgroup arrays of the adjoint
    const int32_t *meta;   // per-row code table (frozen = -2)
    int32_t Tev, Q;
    int8_t orders[8][16];
};

// Min-sum check function in clamp form (two instructions), b the operand that
// bounds the other: equal to sgn(b) sgn(y) min(|b|,|y|) wherever that is
// nonzero.  A zero result (an input zero) may carry the other sign; no
// derivative below reads the sign of such a zero (a sign is read only from
// an operand of larger magnitude than another, or from an L message or a sum
// with one, which the channel's nonzero LLRs keep nonzero), so outputs and
// gradients are those of the sign-magnitude form.
__device__ __forceinline__ float ms0c(float b, float y) { return cnode_clamp<0>(b, y, 1.f); }
// d sgn(s) with sgn(s) = -1 when the sign bit of s is set (also for -0), else
// +1: the sign bit of d flipped by that of s, one v_bitop3_b32
__device__ __forceinline__ float xsign(float d, float s) {
    return __uint_as_float(__float_as_uint(d) ^ (__float_as_uint(s) & 0x80000000u));
}

// LDS per slot.  Forward: the L and R boundary ping-pong pairs (4N floats).
// Adjoint: the same two pairs, reused by the reverse sweeps for the adjoint
// handoffs (every phase ends at a barrier), plus a ping-pong pair of
// weight-gradient staging buffers of RHO N floats each, one per reverse step.
// The pool orders follow the slots.
// A frame of at most one wave (TPS <= 64) exchanges group boundaries only
// inside its wave: its kernels take no workgroup barrier per group step, and
// the adjoint stages a whole iteration's weight gradients per frame (2 n N
// floats) so that the sum over the workgroup's frames needs one barrier per
// iteration instead of one per step.
template <class P>
constexpr bool wbp_wave_frame() { return P::TPS <= 64; }

template <class P, bool BWD>
struct WbpLds {
    static constexpr size_t per_slot =
        (size_t)(BWD ? 4 + (wbp_wave_frame<P>() ? 2 * P::n : 2 * P::rho) : 4) * P::N * sizeof(float);
    // the forward keeps the pool orders in LDS after the slots; the adjoint
    // reads them from its arguments (at N = 256 its four slots take exactly
    // half of the LDS, so two workgroups share a CU)
    static constexpr size_t bytes(int S) { return (size_t)S * per_slot + (BWD ? 0 : 8 * 16); }
};

template <int NLOG, int RHO>
constexpr int wbp_launch_bound() {
    return ((1 << (NLOG - RHO)) > 256) ? (1 << (NLOG - RHO)) : 256;
}

// Frames per workgroup of the adjoint.  Every workgroup writes one
// weight-gradient partial of T n 2 N floats, so one-wave frames take 512
// threads: half as many partials to write and sum as with 256, at the same
// waves per CU (the LDS of one such workgroup fills the CU).  Longer frames
// take as many slots as the forward.
template <int NLOG, int RHO>
constexpr int wbp_bwd_slots() {
    constexpr int tps = 1 << (NLOG - RHO);
    return tps <= 64 ? 512 / tps : (tps >= 256 ? 1 : 256 / tps);
}
template <int NLOG, int RHO>
constexpr int wbp_bwd_launch_bound() {
    constexpr int w = (1 << (NLOG - RHO)) * wbp_bwd_slots<NLOG, RHO>();
    return w > 256 ? w : 256;
}

// Checkpoint layout of the persistent R state of one frame and iteration:
// one block per group, in group order; inside group g's block each thread's
// gsize(g) values (the interior levels, then the top level, in register
// order) are contiguous, so a thread moves its group with a few wide accesses
// and consecutive threads touch consecutive memory.
template <class P>
struct RState {
    static constexpr int NREG = (P::n - 1) * P::ROWS;  // values per thread
    static constexpr int gsize(int g) { return (P::size(g) - 1 + (g < P::G - 1 ? 1 : 0)) * P::ROWS; }
    static constexpr int gstart(int g) {
        int k = 0;
        for (int h = 0; h < g; ++h) k += gsize(h);
        return k;
    }
    // element j of group g of thread t, in floats from the frame-iteration base
    __device__ static __forceinline__ int64_t off(int g, int t, int j) {
        return (int64_t)gstart(g) * P::TPS + (int64_t)t * gsize(g) + j;
    }
    template <class Fn>
    __device__ static __forceinline__ void each(Regs<P> &st, int t, Fn &&fn) {
        sfor<0, P::G>([&](auto g) {
            sfor<0, P::size(g) - 1>([&](auto l) {
                sfor<0, P::ROWS>([&](auto i) { fn(st.Rint[g][l][i], off(g, t, l * P::ROWS + i)); });
            });
            if constexpr (g < P::G - 1)
                sfor<0, P::ROWS>([&](auto i) { fn(st.Rtop[g][i], off(g, t, (P::size(g) - 1) * P::ROWS + i)); });
        });
    }
};

// ---- forward passes with weights -------------------------------------------
// wg points at the weights of this iteration, offset by the thread's row base
// of group g; weight of stage-local sl, sweep d, register i:
// wg[((lo + sl) * 2 + d) * N + off(i)].  The group passes also take the
// group's weights already in registers, w[sl][i] (WgroupW, from wload), so
// that a kernel can load them a step ahead.
template <class P>
using WgroupW = float[P::RMAX][P::ROWS];

template <class P, int g>
__device__ __forceinline__ void wload(const float *wg, int d, WgroupW<P> &w) {
    sfor<0, P::size(g)>([&](auto sl) {
        sfor<0, P::ROWS>([&](auto i) { w[sl][i] = wg[((P::lo(g) + sl) * 2 + d) * P::N + GMap<P, g>::off(i)]; });
    });
}

template <class P, int g, int D, class WG>
__device__ __forceinline__ float wget(const WG &wg, int sl, int i) {
    if constexpr (std::is_pointer_v<WG>)
        return wg[((P::lo(g) + sl) * 2 + D) * P::N + GMap<P, g>::off(i)];
    else
        return wg[sl][i];
}
template <class P, int g, class WG>
__device__ __forceinline__ void wgroup_L(const float (&lbot)[P::ROWS], float (&lint)[P::RI][P::ROWS],
                                         const float (&rint)[P::RI][P::ROWS],
                                         const float (&rtop)[P::ROWS], float (&out)[P::ROWS],
                                         const WG &wg) {
    constexpr int r = P::size(g), lo = P::lo(g), N = P::N, ROWS = P::ROWS;
    float cur[ROWS];
    sfor<0, ROWS>([&](auto i) { cur[i] = lbot[i]; });
    sfor<0, r>([&](auto sl) {
        float wv[ROWS];
        sfor<0, ROWS>([&](auto i) { wv[i] = wget<P, g, 0>(wg, sl, i); });
        float nxt[ROWS];
        sfor<0, ROWS>([&](auto i) {
            constexpr int b = 1 << sl;
            if constexpr ((i & b) == 0) {
                constexpr int ip = i | b;
                float r1, r2;
                if constexpr (sl + 1 < r) { r1 = rint[sl][i]; r2 = rint[sl][ip]; }
                else { r1 = rtop[i]; r2 = rtop[ip]; }
                const float l1 = cur[i], l2 = cur[ip];
                nxt[i] = wv[i] * ms0c(l1, l2 + r2);
                nxt[ip] = wv[ip] * ms0c(l1, r1) + l2;
            }
        });
        if constexpr (sl + 1 < r) sfor<0, ROWS>([&](auto i) { lint[sl][i] = nxt[i]; });
        sfor<0, ROWS>([&](auto i) { cur[i] = nxt[i]; });
    });
    sfor<0, ROWS>([&](auto i) { out[i] = cur[i]; });
}

template <class P, int g, class WG>
__device__ __forceinline__ void wgroup_R(const float (&lbot)[P::ROWS], const float (&lint)[P::RI][P::ROWS],
                                         float (&rint)[P::RI][P::ROWS], const float (&rtop)[P::ROWS],
                                         float (&out)[P::ROWS], const WG &wg) {
    constexpr int r = P::size(g), lo = P::lo(g), N = P::N, ROWS = P::ROWS;
    float cur[ROWS];
    sfor<0, ROWS>([&](auto i) { cur[i] = rtop[i]; });
    sfor<0, r>([&](auto k) {
        constexpr int sl = r - 1 - k;
        float wv[ROWS];
        sfor<0, ROWS>([&](auto i) { wv[i] = wget<P, g, 1>(wg, sl, i); });
        float nxt[ROWS];
        sfor<0, ROWS>([&](auto i) {
            constexpr int b = 1 << sl;
            if constexpr ((i & b) == 0) {
                constexpr int ip = i | b;
                float l1, l2;
                if constexpr (sl > 0) { l1 = lint[sl - 1][i]; l2 = lint[sl - 1][ip]; }
                else { l1 = lbot[i]; l2 = lbot[ip]; }
                const float r1 = cur[i], r2 = cur[ip];
                nxt[i] = wv[i] * ms0c(l2 + r2, r1);
                nxt[ip] = wv[ip] * ms0c(l1, r1) + r2;
            }
        });
        if constexpr (sl > 0) sfor<0, ROWS>([&](auto i) { rint[sl - 1][i] = nxt[i]; });
        sfor<0, ROWS>([&](auto i) { cur[i] = nxt[i]; });
    });
    sfor<0, ROWS>([&](auto i) { out[i] = cur[i]; });
}

// ---- reverse passes ------------------------------------------------------
// Reverse of the weighted R pass of group g.  gbot: adjoint of the R message
// this group produces on its bottom level (ZBOT: known to be zero, the
// channel level's R, which nothing reads).  gstate: adjoint, from the next
// iteration, of the R messages it produces on its interior levels.  Writes
// the adjoints of the L messages it read into glint/glbot (every entry once),
// returns in gtop the adjoint of the R message it read on its top level, and
// stages the weight gradients of its stages (sweep 1) through
// gw(stage - lo, register, row offset, value).  The derivative routing is the
// min-sum rule of the forward's check function, written branch-free: a select
// per route and the sign flips as bit operations.
template <class P, int g, bool ZBOT, class WG, class Sink>
__device__ __forceinline__ void rev_group_R(const float (&lbot)[P::ROWS], const float (&lint)[P::RI][P::ROWS],
                                            const float (&rsw)[P::RI][P::ROWS], const float (&rtopsw)[P::ROWS],
                                            const float (&gbot)[P::ROWS], const float (&gstate)[P::RI][P::ROWS],
                                            float (&glint)[P::RI][P::ROWS], float (&glbot)[P::ROWS],
                                            float (&gtop)[P::ROWS], const WG &wg, Sink &&gw) {
    constexpr int r = P::size(g), lo = P::lo(g), N = P::N, ROWS = P::ROWS;
    float gacc[P::RI][ROWS];
    sfor<0, r - 1>([&](auto l) { sfor<0, ROWS>([&](auto i) { gacc[l][i] = gstate[l][i]; }); });
    sfor<0, r>([&](auto sl) {
        if constexpr (ZBOT && sl == 0) {
            // a zero adjoint: zero weight gradients, nothing flows on
            sfor<0, ROWS>([&](auto i) {
                gw(0, (int)i, GMap<P, g>::off(i), 0.f);
                glbot[i] = 0.f;
                if constexpr (r == 1) gtop[i] = 0.f;
            });
            return;
        }
        float go[ROWS];
        if constexpr (sl == 0) sfor<0, ROWS>([&](auto i) { go[i] = gbot[i]; });
        else sfor<0, ROWS>([&](auto i) { go[i] = gacc[sl - 1][i]; });
        float wv[ROWS];
        sfor<0, ROWS>([&](auto i) { wv[i] = wget<P, g, 1>(wg, sl, i); });
        sfor<0, ROWS>([&](auto i) {
            constexpr int b = 1 << sl;
            if constexpr ((i & b) == 0) {
                constexpr int ip = i | b;
                float r1, r2, l1, l2;
                if constexpr (sl + 1 < r) { r1 = rsw[sl][i]; r2 = rsw[sl][ip]; }
                else { r1 = rtopsw[i]; r2 = rtopsw[ip]; }
                if constexpr (sl > 0) { l1 = lint[sl - 1][i]; l2 = lint[sl - 1][ip]; }
                else { l1 = lbot[i]; l2 = lbot[ip]; }
                // outputs: R'1 = w1 ms(r1, l2 + r2), R'2 = w2 ms(r1, l1) + r2
                const float a = l2 + r2;
                gw(sl, (int)i, GMap<P, g>::off(i), go[i] * ms0c(a, r1));
                gw(sl, ip, GMap<P, g>::off(ip), go[ip] * ms0c(l1, r1));
                const float d1 = go[i] * wv[i], d2 = go[ip] * wv[ip];
                const bool c1 = __builtin_fabsf(r1) <= __builtin_fabsf(a);
                const bool c2 = __builtin_fabsf(r1) <= __builtin_fabsf(l1);
                const float ga = c1 ? 0.f : xsign(d1, r1);  // to l2 and r2
                const float gr1 = (c1 ? xsign(d1, a) : 0.f) + (c2 ? xsign(d2, l1) : 0.f);
                const float gl1 = c2 ? 0.f : xsign(d2, r1);
                const float gr2 = ga + go[ip];
                if constexpr (sl + 1 < r) { gacc[sl][i] += gr1; gacc[sl][ip] += gr2; }
                else { gtop[i] = gr1; gtop[ip] = gr2; }
                if constexpr (sl > 0) { glint[sl - 1][i] = gl1; glint[sl - 1][ip] = ga; }
                else { glbot[i] = gl1; glbot[ip] = ga; }
            }
        });
    });
}

// Reverse of the weighted L pass of group g.  gtop: adjoint of the L message
// it produced on its top level (ZTOP: known to be zero, the decision level's
// L before the last iteration); glint: adjoints (already holding the R-sweep
// contributions) of its interior L messages.  Adds to glbot, writes the
// adjoints of the entering R state it read into gsint/gstop (every entry
// once; gstop untouched when the top level is the prior), stages the weight
// gradients of its stages (sweep 0) through gw(stage - lo, register, row
// offset, value).
template <class P, int g, bool TOPPRIOR, bool ZTOP, class WG, class Sink>
__device__ __forceinline__ void rev_group_L(const float (&lbot)[P::ROWS], const float (&lint)[P::RI][P::ROWS],
                                            const float (&rint)[P::RI][P::ROWS], const float (&rtop)[P::ROWS],
                                            const float (&gtop)[P::ROWS], float (&glint)[P::RI][P::ROWS],
                                            float (&glbot)[P::ROWS], float (&gsint)[P::RI][P::ROWS],
                                            float (&gstop)[P::ROWS], const WG &wg, Sink &&gw) {
    constexpr int r = P::size(g), lo = P::lo(g), N = P::N, ROWS = P::ROWS;
    static_assert(!ZTOP || TOPPRIOR, "a zero top adjoint is the last group's");
    sfor<0, r>([&](auto k) {
        constexpr int sl = r - 1 - k;
        if constexpr (ZTOP && sl == r - 1) {
            // a zero adjoint on the prior-topped stage: zero weight gradients
            // and nothing flows on (its R side is the prior)
            sfor<0, ROWS>([&](auto i) { gw(sl, (int)i, GMap<P, g>::off(i), 0.f); });
            return;
        }
        float go[ROWS];
        if constexpr (sl == r - 1) sfor<0, ROWS>([&](auto i) { go[i] = gtop[i]; });
        else sfor<0, ROWS>([&](auto i) { go[i] = glint[sl][i]; });
        float wv[ROWS];
        sfor<0, ROWS>([&](auto i) { wv[i] = wget<P, g, 0>(wg, sl, i); });
        sfor<0, ROWS>([&](auto i) {
            constexpr int b = 1 << sl;
            if constexpr ((i & b) == 0) {
                constexpr int ip = i | b;
                float r1, r2, l1, l2;
                if constexpr (sl + 1 < r) { r1 = rint[sl][i]; r2 = rint[sl][ip]; }
                else { r1 = rtop[i]; r2 = rtop[ip]; }
                if constexpr (sl > 0) { l1 = lint[sl - 1][i]; l2 = lint[sl - 1][ip]; }
                else { l1 = lbot[i]; l2 = lbot[ip]; }
                // outputs: L'1 = w1 ms(l1, l2 + r2), L'2 = w2 ms(r1, l1) + l2
                const float a = l2 + r2;
                gw(sl, (int)i, GMap<P, g>::off(i), go[i] * ms0c(l1, a));
                gw(sl, ip, GMap<P, g>::off(ip), go[ip] * ms0c(l1, r1));
                const float d1 = go[i] * wv[i], d2 = go[ip] * wv[ip];
                const bool c1 = __builtin_fabsf(l1) <= __builtin_fabsf(a);
                const bool c2 = __builtin_fabsf(r1) <= __builtin_fabsf(l1);
                const float ga = c1 ? 0.f : xsign(d1, l1);  // to l2 and r2
                const float gl1 = (c1 ? xsign(d1, a) : 0.f) + (c2 ? 0.f : xsign(d2, r1));
                const float gr1 = c2 ? xsign(d2, l1) : 0.f;
                const float gl2 = ga + go[ip];
                if constexpr (sl > 0) { glint[sl - 1][i] += gl1; glint[sl - 1][ip] += gl2; }
                else { glbot[i] += gl1; glbot[ip] += gl2; }
                if constexpr (sl + 1 < r) { gsint[sl][i] = gr1; gsint[sl][ip] = ga; }
                else if constexpr (!TOPPRIOR) { gstop[i] = gr1; gstop[ip] = ga; }
            }
        });
    });
}

// ---------------------------------------------------------------------------
template <int NLOG, int KP, int RHO>
__global__ void __launch_bounds__((wbp_launch_bound<NLOG, RHO>())) k_wbp_fwd(WbpArgs a) {
    using P = Plan<NLOG, KP, RHO>;
    constexpr int N = P::N, ROWS = P::ROWS, TPS = P::TPS, G = P::G, n = NLOG, GB = P::GB;
    constexpr bool MAPPED = (KP > 0 && KP < NLOG);
    constexpr int LOWBITS = NLOG - KP;
    constexpr int NREG = RState<P>::NREG;
    constexpr bool WAVE = wbp_wave_frame<P>();
    const int tid = threadIdx.x, S = blockDim.x / TPS, slot = tid / TPS, t = tid & (TPS - 1);
    const int64_t frame = (int64_t)blockIdx.x * S + slot;
    const bool active = frame < a.F;
    extern __shared__ __align__(16) float smem[];
    float *const buf = smem + (size_t)slot * (WbpLds<P, false>::per_slot / sizeof(float));
    int8_t *const ords = reinterpret_cast<int8_t *>(smem + (size_t)S * (WbpLds<P, false>::per_slot / sizeof(float)));
    for (int i = tid; i < 8 * 16; i += blockDim.x) ords[i] = a.orders[i >> 4][i & 15];
    __syncthreads();

    Regs<P> st;
    int baddr[ROWS], toprow[ROWS];
    uint32_t frozen_bits = 0;
    int q = 0, next_ev = a.Tev;
    auto maps = [&](int qq) {
        const int8_t *e = ords + qq * 16;
        const int base = GMap<P, G - 1>::base(t);
        frozen_bits = 0;
        sfor<0, ROWS>([&](auto i) {
            const int p = base + GMap<P, G - 1>::off(i);
            const int j = (KP > 0) ? relabel_to_row(p, e, n, LOWBITS) : p;
            toprow[i] = j;
            frozen_bits |= (a.meta[j] == -2 ? 1u : 0u) << i;
        });
        if constexpr (MAPPED) {
            const int bb = GMap<P, GB>::base(t);
            sfor<0, ROWS>([&](auto i) { baddr[i] = relabel_to_row(bb + GMap<P, GB>::off(i), e, n, LOWBITS); });
        }
        const float *src = a.llr + frame * N;
        const int b0 = GMap<P, 0>::base(t);
        if constexpr (KP == NLOG) {
            sfor<0, ROWS>([&](auto i) { st.Lbot[0][i] = src[relabel_to_row(b0 + GMap<P, 0>::off(i), e, n, 0)]; });
        } else {
            sfor<0, ROWS>([&](auto i) { st.Lbot[0][i] = src[b0 + GMap<P, 0>::off(i)]; });
        }
    };
    sfor<0, G>([&](auto g) {
        sfor<0, P::RI>([&](auto l) { sfor<0, ROWS>([&](auto i) { st.Rint[g][l][i] = 0.f; }); });
        sfor<0, ROWS>([&](auto i) { st.Rtop[g][i] = 0.f; });
    });
    if (active) maps(0);

    // each group step's weights, loaded into registers before its pass
    // (loaded one step ahead, as the one-wave adjoint does, they gained
    // nothing here)
    WgroupW<P> wc;
    auto wown = [&](auto gc, const float *wtp, int d) {
        constexpr int g = decltype(gc)::value;
        wload<P, g>(wtp + GMap<P, g>::base(t), d, wc);
    };

    for (int it = 0; it < a.T; ++it) {
        if constexpr (KP > 0) {
            if (it == next_ev) {  // trellis event: the next order of the pool
                next_ev += a.Tev;
                q = q + 1 == a.Q ? 0 : q + 1;
                sfor<GB, G>([&](auto g) {
                    sfor<0, P::RI>([&](auto l) { sfor<0, ROWS>([&](auto i) { st.Rint[g][l][i] = 0.f; }); });
                    if constexpr (g < G - 1) sfor<0, ROWS>([&](auto i) { st.Rtop[g][i] = 0.f; });
                });
                if (active) maps(q);
            }
        }
        if (it > 0 && active && a.ckpt) {
            float *ck = a.ckpt + ((frame * (a.T - 1) + (it - 1)) * (int64_t)NREG) * TPS;
            if constexpr (NLOG >= kWbpBigLog) {
                // streaming writes: the large-frame adjoint cycles its scratch
                // through the caches, which the checkpoints would crowd out
                // (measured 3-5% faster at N = 4096; at N = 256 the adjoint
                // finds the last checkpoints still cached, and plain stores
                // measured 11% faster)
                RState<P>::each(st, t, [&](float &v, int64_t o) { __builtin_nontemporal_store(v, ck + o); });
            } else {
                RState<P>::each(st, t, [&](float &v, int64_t o) { ck[o] = v; });
            }
        }
        const float *wt = a.w + (int64_t)it * n * 2 * N;
        sfor<0, G - 1>([&](auto g) {
            if (active) {
                if constexpr (g > 0) {
                    const float *lb = buf + (g & 1) * N;
                    if constexpr (MAPPED && g == GB) sfor<0, ROWS>([&](auto i) { st.Lbot[g][i] = lb[baddr[i]]; });
                    else {
                        const int base = GMap<P, g>::base(t);
                        sfor<0, ROWS>([&](auto i) { st.Lbot[g][i] = lb[base + GMap<P, g>::off(i)]; });
                    }
                }
                float out[ROWS];
                const int base = GMap<P, g>::base(t);
                wown(g, wt, 0);
                wgroup_L<P, g>(st.Lbot[g], st.Lint[g], st.Rint[g], st.Rtop[g], out, wc);
                float *lt = buf + ((g + 1) & 1) * N;
                sfor<0, ROWS>([&](auto i) { lt[base + GMap<P, g>::off(i)] = out[i]; });
            }
            boundary_sync<WAVE>();
        });
        static_assert(G >= 2, "the step order below assumes two groups or more");
        float prior[ROWS];
        sfor<0, ROWS>([&](auto i) { prior[i] = ((frozen_bits >> i) & 1u) ? kWbpPrior : 0.f; });
        const int btop = GMap<P, G - 1>::base(t);
        if (active) {
            const float *lb = buf + ((G - 1) & 1) * N;
            if constexpr (MAPPED && G - 1 == GB) sfor<0, ROWS>([&](auto i) { st.Lbot[G - 1][i] = lb[baddr[i]]; });
            else sfor<0, ROWS>([&](auto i) { st.Lbot[G - 1][i] = lb[btop + GMap<P, G - 1>::off(i)]; });
            wown(std::integral_constant<int, G - 1>{}, wt, 0);
            wgroup_L<P, G - 1>(st.Lbot[G - 1], st.Lint[G - 1], st.Rint[G - 1], prior, st.Ltop, wc);
            if (it == a.T - 1)
                sfor<0, ROWS>([&](auto i) { a.out[frame * N + toprow[i]] = st.Ltop[i] + prior[i]; });
        }
        if (it < a.T - 1) {
            if (active) {
                float rb[ROWS];
                wown(std::integral_constant<int, G - 1>{}, wt, 1);
                wgroup_R<P, G - 1>(st.Lbot[G - 1], st.Lint[G - 1], st.Rint[G - 1], prior, rb, wc);
                float *rt = buf + 2 * N + ((G - 1) & 1) * N;
                if constexpr (MAPPED && G - 1 == GB) sfor<0, ROWS>([&](auto i) { rt[baddr[i]] = rb[i]; });
                else sfor<0, ROWS>([&](auto i) { rt[btop + GMap<P, G - 1>::off(i)] = rb[i]; });
            }
        }
        boundary_sync<WAVE>();
        if (it == a.T - 1) break;
        sfor<0, G - 1>([&](auto k) {
            constexpr int g = G - 2 - k;
            if (active) {
                const int base = GMap<P, g>::base(t);
                const float *rs = buf + 2 * N + ((g + 1) & 1) * N;
                sfor<0, ROWS>([&](auto i) { st.Rtop[g][i] = rs[base + GMap<P, g>::off(i)]; });
                float rb[ROWS];
                wown(std::integral_constant<int, g>{}, wt, 1);
                wgroup_R<P, g>(st.Lbot[g], st.Lint[g], st.Rint[g], st.Rtop[g], rb, wc);
                if constexpr (g > 0) {
                    float *rt = buf + 2 * N + (g & 1) * N;
                    if constexpr (MAPPED && g == GB) sfor<0, ROWS>([&](auto i) { rt[baddr[i]] = rb[i]; });
                    else sfor<0, ROWS>([&](auto i) { rt[base + GMap<P, g>::off(i)] = rb[i]; });
                }
            }
            boundary_sync<WAVE>();
        });
    }
}

template <int NLOG, int KP, int RHO>
__global__ void __launch_bounds__((wbp_bwd_launch_bound<NLOG, RHO>())) k_wbp_bwd(WbpArgs a) {
    using P = Plan<NLOG, KP, RHO>;
    constexpr int N = P::N, ROWS = P::ROWS, TPS = P::TPS, G = P::G, n = NLOG, GB = P::GB;
    constexpr bool MAPPED = (KP > 0 && KP < NLOG);
    constexpr int LOWBITS = NLOG - KP;
    constexpr int NREG = RState<P>::NREG;
    constexpr int RI = P::RI;
    constexpr bool WAVE = wbp_wave_frame<P>();
    const int tid = threadIdx.x, S = blockDim.x / TPS, slot = tid / TPS, t = tid & (TPS - 1);
    // batches of S consecutive frames; workgroup w takes batches w, w + grid,
    // ... in that order and adds each batch's gradients into its partial
    const int64_t nbatch = (a.F + S - 1) / S;
    constexpr size_t PS = WbpLds<P, true>::per_slot / sizeof(float);
    extern __shared__ __align__(16) float smem[];
    // [A0 A1 | B0 B1 | W]: L and R boundary pairs of the recomputed sweeps;
    // the reverse R sweep passes adjoints through A, the reverse L sweep
    // through B; W holds the weight gradients of one reverse step (W0 W1,
    // RHO N floats each) or, for a one-wave frame, of the whole iteration
    // ([n][2][N])
    float *const buf = smem + (size_t)slot * PS;
    const int8_t *const ords = &a.orders[0][0];

    Regs<P> st;                         // entering R state and this iteration's L messages
    float Rsw[G][RI][ROWS], Rtsw[G][ROWS];  // R messages of this iteration's R sweep
    float gsi[G][RI][ROWS], gst[G][ROWS];   // adjoint of the R state leaving the iteration
    float gli[G][RI][ROWS], glb[G][ROWS];   // adjoints of the L messages
    WgroupW<P> wc, wn;                      // weights of the current and the next group step
    sfor<0, P::RMAX>([&](auto l) { sfor<0, ROWS>([&](auto i) { wc[l][i] = 0.f; wn[l][i] = 0.f; }); });
    static_assert(G >= 2, "the step order below assumes two groups or more");
    int baddr[ROWS], toprow[ROWS];
    uint32_t frozen_bits = 0;
    auto order_at = [&](int it) { return (KP > 0 && a.Q > 1) ? (it / a.Tev) % a.Q : 0; };
    // flush: sum the weight gradients that one reverse step (group g, sweep
    // d) staged in W[par] over the batch's frames, in slot order, and add
    // them into this workgroup's partial of iteration it.  flush_all (one-wave
    // frames): the same for the whole iteration's staged gradients (the last
    // iteration's R weights get 0).  A batch whose slots all hold frames
    // sums its slots in a fixed unrolled order, four consecutive entries per
    // thread (16-byte LDS reads and global accesses); others take the general
    // loop.  Both add the slots in slot order.
    constexpr int SC = wbp_bwd_slots<NLOG, RHO>();
    // a full workgroup's flush of one iteration's partial (one-wave frames):
    // FV float4 entries, FPER per thread.  Without a permuted range each
    // thread loads their old values at the start of the iteration, to be
    // added at its end (it reads back only what it wrote); with one, the row
    // maps leave no registers to hold them, and the flush loads them itself
    constexpr int FV = n * 2 * N / 4, FB = SC * TPS, FPER = (FV + FB - 1) / FB;
    constexpr bool FPF = WAVE && KP == 0;
    float4 fold[FPER];
    auto fold_load = [&](int it) {
        const float *part = a.partial + ((int64_t)blockIdx.x * a.T + it) * (int64_t)n * 2 * N;
        sfor<0, FPER>([&](auto k) {
            const int i4 = tid + k * FB;
            if (FV % FB == 0 || i4 < FV) fold[k] = *reinterpret_cast<const float4 *>(part + 4 * i4);
        });
    };
    for (int64_t bt = blockIdx.x; bt < nbatch; bt += gridDim.x) {
        const bool first = bt == (int64_t)blockIdx.x;  // the partial's first batch stores
        const int64_t frame0 = bt * S, frame = frame0 + slot;
        const bool active = frame < a.F;
        const bool full = S == SC && frame0 + SC <= a.F;
        sfor<0, G>([&](auto g) {
            sfor<0, RI>([&](auto l) { sfor<0, ROWS>([&](auto i) { gsi[g][l][i] = 0.f; }); });
            sfor<0, ROWS>([&](auto i) { gst[g][i] = 0.f; });
        });
        // store into the partial (its first batch) or add to it
        auto put4 = [&](float *p, float4 v) {
            if (!first) {
                const float4 o = *reinterpret_cast<const float4 *>(p);
                v = make_float4(o.x + v.x, o.y + v.y, o.z + v.z, o.w + v.w);
            }
            *reinterpret_cast<float4 *>(p) = v;
        };
        auto put1 = [&](float *p, float v) { *p = first ? v : *p + v; };
        auto flush_all = [&](int it, bool lastit) {
            float *part = a.partial + ((int64_t)blockIdx.x * a.T + it) * (int64_t)n * 2 * N;
            if (full && !FPF) {
                for (int i4 = tid; i4 < n * 2 * N / 4; i4 += blockDim.x) {
                    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
                    if (!(lastit && (((4 * i4) / N) & 1))) {
                        sfor<0, SC>([&](auto sc) {
                            const float4 w = *reinterpret_cast<const float4 *>(smem + (size_t)sc * PS + 4 * N + 4 * i4);
                            v.x += w.x; v.y += w.y; v.z += w.z; v.w += w.w;
                        });
                    }
                    put4(part + 4 * i4, v);
                }
                return;
            }
            if constexpr (FPF) {
                if (full) {
                    sfor<0, FPER>([&](auto k) {
                        const int i4 = tid + k * FB;
                        if (FV % FB == 0 || i4 < FV) {
                            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
                            if (!(lastit && (((4 * i4) / N) & 1))) {
                                sfor<0, SC>([&](auto sc) {
                                    const float4 w = *reinterpret_cast<const float4 *>(smem + (size_t)sc * PS + 4 * N + 4 * i4);
                                    v.x += w.x; v.y += w.y; v.z += w.z; v.w += w.w;
                                });
                            }
                            if (!first) {
                                const float4 o = fold[k];
                                v = make_float4(o.x + v.x, o.y + v.y, o.z + v.z, o.w + v.w);
                            }
                            *reinterpret_cast<float4 *>(part + 4 * i4) = v;
                        }
                    });
                    return;
                }
            }
            for (int idx = tid; idx < n * 2 * N; idx += blockDim.x) {
                float v = 0.f;
                if (!(lastit && ((idx / N) & 1)))
                    for (int s = 0; s < S; ++s)
                        if (frame0 + s < a.F) v += smem[(size_t)s * PS + 4 * N + idx];
                put1(part + idx, v);
            }
        };
        auto flush = [&](auto gc, int d, int par, int it) {
            constexpr int g = decltype(gc)::value, r = P::size(g), lo = P::lo(g);
            float *part = a.partial + ((int64_t)blockIdx.x * a.T + it) * (int64_t)n * 2 * N + lo * 2 * N;
            const float *w0 = smem + 4 * N + par * RHO * N;
            if (full) {
                for (int i4 = tid; i4 < r * N / 4; i4 += blockDim.x) {
                    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
                    sfor<0, SC>([&](auto sc) {
                        const float4 w = *reinterpret_cast<const float4 *>(w0 + (size_t)sc * PS + 4 * i4);
                        v.x += w.x; v.y += w.y; v.z += w.z; v.w += w.w;
                    });
                    const int idx = 4 * i4;
                    put4(part + ((idx / N) * 2 + d) * N + (idx & (N - 1)), v);
                }
                return;
            }
            for (int idx = tid; idx < r * N; idx += blockDim.x) {
                float v = 0.f;
                for (int s = 0; s < S; ++s)
                    if (frame0 + s < a.F) v += w0[(size_t)s * PS + idx];
                put1(part + ((idx / N) * 2 + d) * N + (idx & (N - 1)), v);
            }
        };

        for (int it = a.T - 1; it >= 0; --it) {
            const int q = order_at(it);
            const float *wt = a.w + (int64_t)it * n * 2 * N;
            const bool lastit = (it == a.T - 1);
            if constexpr (FPF) {
                if (full && !first) fold_load(it);
            }
            if (active) {
                const int8_t *e = ords + q * 16;
                const int base = GMap<P, G - 1>::base(t);
                frozen_bits = 0;
                sfor<0, ROWS>([&](auto i) {
                    const int p = base + GMap<P, G - 1>::off(i);
                    const int j = (KP > 0) ? relabel_to_row(p, e, n, LOWBITS) : p;
                    toprow[i] = j;
                    frozen_bits |= (a.meta[j] == -2 ? 1u : 0u) << i;
                });
                if constexpr (MAPPED) {
                    const int bb = GMap<P, GB>::base(t);
                    sfor<0, ROWS>([&](auto i) { baddr[i] = relabel_to_row(bb + GMap<P, GB>::off(i), e, n, LOWBITS); });
                }
                const float *src = a.llr + frame * N;
                const int b0 = GMap<P, 0>::base(t);
                if constexpr (KP == NLOG) {
                    sfor<0, ROWS>([&](auto i) { st.Lbot[0][i] = src[relabel_to_row(b0 + GMap<P, 0>::off(i), e, n, 0)]; });
                } else {
                    sfor<0, ROWS>([&](auto i) { st.Lbot[0][i] = src[b0 + GMap<P, 0>::off(i)]; });
                }
                // entering R state
                if (it == 0) {
                    RState<P>::each(st, t, [&](float &v, int64_t) { v = 0.f; });
                } else {
                    const float *ck = a.ckpt + ((frame * (a.T - 1) + (it - 1)) * (int64_t)NREG) * TPS;
                    RState<P>::each(st, t, [&](float &v, int64_t o) { v = ck[o]; });
                }
                // a trellis switch after this iteration reset the inner levels of
                // the permuted range: nothing flows back through them
                if constexpr (KP > 0) {
                    if (!lastit && order_at(it + 1) != q) {
                        sfor<GB, G>([&](auto g) {
                            sfor<0, RI>([&](auto l) { sfor<0, ROWS>([&](auto i) { gsi[g][l][i] = 0.f; }); });
                            if constexpr (g < G - 1) sfor<0, ROWS>([&](auto i) { gst[g][i] = 0.f; });
                        });
                    }
                }
                // the reverse R sweep writes the L adjoints; without it (the last
                // iteration) they start at zero
                if (lastit) {
                    sfor<0, G>([&](auto g) {
                        sfor<0, RI>([&](auto l) { sfor<0, ROWS>([&](auto i) { gli[g][l][i] = 0.f; }); });
                        sfor<0, ROWS>([&](auto i) { glb[g][i] = 0.f; });
                    });
                }
            }
            // One-wave frames load each group step's weights one step ahead
            // (into wn, while the step before computes; wc holds the current
            // step's): steps that loaded their own waited on the L2, with two
            // waves per SIMD to hide it.  Longer frames, whose registers the
            // second set would cost occupancy, load each step's own (wown).
            constexpr bool WPF = WAVE;
            auto wnext = [&](auto gc, int d) {
                constexpr int g = decltype(gc)::value;
                if constexpr (WPF) wload<P, g>(wt + GMap<P, g>::base(t), d, wn);
            };
            auto wshift = [&]() {
                if constexpr (WPF)
                    sfor<0, P::RMAX>([&](auto l) { sfor<0, ROWS>([&](auto i) { wc[l][i] = wn[l][i]; }); });
            };
            auto wown = [&](auto gc, int d) {
                constexpr int g = decltype(gc)::value;
                if constexpr (!WPF) wload<P, g>(wt + GMap<P, g>::base(t), d, wc);
            };
            // ---- recompute the L sweep ----
            if constexpr (WPF) wload<P, 0>(wt + GMap<P, 0>::base(t), 0, wc);
            sfor<0, G - 1>([&](auto g) {
                wnext(std::integral_constant<int, g + 1>{}, 0);
                if (active) {
                    const int base = GMap<P, g>::base(t);
                    if constexpr (g > 0) {
                        const float *lb = buf + (g & 1) * N;
                        if constexpr (MAPPED && g == GB) sfor<0, ROWS>([&](auto i) { st.Lbot[g][i] = lb[baddr[i]]; });
                        else sfor<0, ROWS>([&](auto i) { st.Lbot[g][i] = lb[base + GMap<P, g>::off(i)]; });
                    }
                    float out[ROWS];
                    wown(g, 0);
                    wgroup_L<P, g>(st.Lbot[g], st.Lint[g], st.Rint[g], st.Rtop[g], out, wc);
                    float *lt = buf + ((g + 1) & 1) * N;
                    sfor<0, ROWS>([&](auto i) { lt[base + GMap<P, g>::off(i)] = out[i]; });
                }
                boundary_sync<WAVE>();
                wshift();
            });
            float prior[ROWS];
            sfor<0, ROWS>([&](auto i) { prior[i] = ((frozen_bits >> i) & 1u) ? kWbpPrior : 0.f; });
            // next: the R sweep's first step, or the reverse L sweep's (the same group)
            wnext(std::integral_constant<int, G - 1>{}, lastit ? 0 : 1);
            if (active) {
                const int base = GMap<P, G - 1>::base(t);
                if constexpr (G > 1) {
                    const float *lb = buf + ((G - 1) & 1) * N;
                    if constexpr (MAPPED && G - 1 == GB) sfor<0, ROWS>([&](auto i) { st.Lbot[G - 1][i] = lb[baddr[i]]; });
                    else sfor<0, ROWS>([&](auto i) { st.Lbot[G - 1][i] = lb[base + GMap<P, G - 1>::off(i)]; });
                }
                wown(std::integral_constant<int, G - 1>{}, 0);
                wgroup_L<P, G - 1>(st.Lbot[G - 1], st.Lint[G - 1], st.Rint[G - 1], prior, st.Ltop, wc);
            }
            wshift();
            // ---- recompute the R sweep, keeping every level ----
            if (!lastit) {
                wnext(std::integral_constant<int, G - 2>{}, 1);
                if (active) {
                    const int base = GMap<P, G - 1>::base(t);
                    sfor<0, ROWS>([&](auto i) { Rtsw[G - 1][i] = prior[i]; });
                    float rb[ROWS];
                    wown(std::integral_constant<int, G - 1>{}, 1);
                    wgroup_R<P, G - 1>(st.Lbot[G - 1], st.Lint[G - 1], Rsw[G - 1], prior, rb, wc);
                    if constexpr (G > 1) {
                        float *rt = buf + 2 * N + ((G - 1) & 1) * N;
                        if constexpr (MAPPED && G - 1 == GB) sfor<0, ROWS>([&](auto i) { rt[baddr[i]] = rb[i]; });
                        else sfor<0, ROWS>([&](auto i) { rt[base + GMap<P, G - 1>::off(i)] = rb[i]; });
                    }
                }
                wshift();
            }
            boundary_sync<WAVE>();
            if (!lastit) {
                sfor<0, G - 1>([&](auto k) {
                    constexpr int g = G - 2 - k;
                    // next: group g - 1; after group 0 the reverse R sweep starts on group 0
                    if constexpr (g > 0) wnext(std::integral_constant<int, g - 1>{}, 1);
                    if (active) {
                        const int base = GMap<P, g>::base(t);
                        const float *rs = buf + 2 * N + ((g + 1) & 1) * N;
                        sfor<0, ROWS>([&](auto i) { Rtsw[g][i] = rs[base + GMap<P, g>::off(i)]; });
                        float rb[ROWS];
                        wown(std::integral_constant<int, g>{}, 1);
                        wgroup_R<P, g>(st.Lbot[g], st.Lint[g], Rsw[g], Rtsw[g], rb, wc);
                        if constexpr (g > 0) {
                            float *rt = buf + 2 * N + (g & 1) * N;
                            if constexpr (MAPPED && g == GB) sfor<0, ROWS>([&](auto i) { rt[baddr[i]] = rb[i]; });
                            else sfor<0, ROWS>([&](auto i) { rt[base + GMap<P, g>::off(i)] = rb[i]; });
                        }
                    }
                    boundary_sync<WAVE>();
                    if constexpr (g > 0) wshift();
                });
                // ---- reverse of the R sweep: groups bottom to top ----
                sfor<0, G>([&](auto g) {
                    // next: group g + 1, or after the last the reverse L sweep's first
                    if constexpr (g + 1 < G) wnext(std::integral_constant<int, g + 1>{}, 1);
                    else wnext(std::integral_constant<int, G - 1>{}, 0);
                    if constexpr (g > 0 && !WAVE) flush(std::integral_constant<int, g - 1>{}, 1, (g - 1) & 1, it);
                    if (active) {
                        const int base = GMap<P, g>::base(t);
                        float gb[ROWS];
                        if constexpr (g == 0) {
                            sfor<0, ROWS>([&](auto i) { gb[i] = 0.f; });
                        } else {
                            const float *src = buf + (g & 1) * N;
                            if constexpr (MAPPED && g == GB) sfor<0, ROWS>([&](auto i) { gb[i] = src[baddr[i]]; });
                            else sfor<0, ROWS>([&](auto i) { gb[i] = src[base + GMap<P, g>::off(i)]; });
                        }
                        float gtop[ROWS];
                        // staged at [sl][row] of this step, or at [stage][1][row] for one-wave frames
                        float *const gws = WAVE ? buf + 4 * N + (P::lo(g) * 2 + 1) * N + base
                                                : buf + 4 * N + (g & 1) * RHO * N + base;
                        constexpr int SLS = WAVE ? 2 * N : N;
                        wown(g, 1);
                        rev_group_R<P, g, g == 0>(st.Lbot[g], st.Lint[g], Rsw[g], Rtsw[g], gb, gsi[g], gli[g], glb[g], gtop,
                                          wc, [&](int sl, int, int off, float v) { gws[sl * SLS + off] = v; });
                        if constexpr (g < G - 1) {
                            float *dst = buf + ((g + 1) & 1) * N;
                            sfor<0, ROWS>([&](auto i) { dst[base + GMap<P, g>::off(i)] = gtop[i] + gst[g][i]; });
                        }
                    }
                    boundary_sync<WAVE>();
                    wshift();
                });
            }
            // ---- reverse of the L sweep: groups top to bottom (it writes the new
            // state adjoint, every entry the reverse R sweep reads) ----
            const int step0 = lastit ? 0 : G;  // reverse steps already taken in this iteration
            sfor<0, G>([&](auto k) {
                constexpr int g = G - 1 - k;
                if constexpr (g > 0) wnext(std::integral_constant<int, g - 1>{}, 0);
                if constexpr (!WAVE) {
                    if constexpr (k == 0) {
                        if (!lastit) flush(std::integral_constant<int, G - 1>{}, 1, (G - 1) & 1, it);
                    } else {
                        flush(std::integral_constant<int, g + 1>{}, 0, (step0 + k - 1) & 1, it);
                    }
                }
                float *const gws = WAVE ? buf + 4 * N + (P::lo(g) * 2) * N : buf + 4 * N + ((step0 + k) & 1) * RHO * N;
                constexpr int SLS = WAVE ? 2 * N : N;
                if (active) {
                    const int base = GMap<P, g>::base(t);
                    float gt[ROWS];
                    auto sink = [&](int sl, int, int off, float v) { gws[sl * SLS + base + off] = v; };
                    wown(std::integral_constant<int, g>{}, 0);
                    if constexpr (g == G - 1) {
                        // the output adjoint enters at the last iteration only
                        if (lastit) {
                            sfor<0, ROWS>([&](auto i) { gt[i] = a.gout[frame * N + toprow[i]]; });
                            rev_group_L<P, g, true, false>(st.Lbot[g], st.Lint[g], st.Rint[g], prior, gt, gli[g], glb[g],
                                                           gsi[g], gst[g], wc, sink);
                        } else {
                            rev_group_L<P, g, true, true>(st.Lbot[g], st.Lint[g], st.Rint[g], prior, gt, gli[g], glb[g],
                                                          gsi[g], gst[g], wc, sink);
                        }
                    } else {
                        const float *src = buf + 2 * N + ((g + 1) & 1) * N;
                        sfor<0, ROWS>([&](auto i) { gt[i] = src[base + GMap<P, g>::off(i)]; });
                        rev_group_L<P, g, false, false>(st.Lbot[g], st.Lint[g], st.Rint[g], st.Rtop[g], gt, gli[g],
                                                        glb[g], gsi[g], gst[g], wc, sink);
                    }
                    if constexpr (g > 0) {
                        float *dst = buf + 2 * N + (g & 1) * N;
                        if constexpr (MAPPED && g == GB) sfor<0, ROWS>([&](auto i) { dst[baddr[i]] = glb[g][i]; });
                        else sfor<0, ROWS>([&](auto i) { dst[base + GMap<P, g>::off(i)] = glb[g][i]; });
                    }
                }
                boundary_sync<WAVE>();
                if constexpr (g > 0) wshift();
            });
            if constexpr (WAVE) {
                __syncthreads();
                flush_all(it, lastit);
            } else {
                flush(std::integral_constant<int, 0>{}, 0, (step0 + G - 1) & 1, it);
                if (lastit && first) {
                    // the last iteration runs no R sweep: its R weights get no gradient
                    float *part = a.partial + ((int64_t)blockIdx.x * a.T + it) * (int64_t)n * 2 * N;
                    for (int idx = tid; idx < n * N; idx += blockDim.x) part[((idx / N) * 2 + 1) * N + (idx & (N - 1))] = 0.f;
                }
            }
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------------------
// Large frames (N >= 2048, one frame of 512 or 1024 threads per workgroup).
// The adjoint's per-thread arrays (entering R state, L and R sweep messages,
// two adjoint sets) exceed the registers a thread of such a workgroup can
// hold, so this kernel keeps one group's arrays in registers at a time and
// streams the rest through a per-workgroup scratch in global memory, stored
// in the thread's register order: coalesced, and each thread reads back only
// what it wrote, so no barrier orders the scratch.  The four phases of an
// iteration (recompute L, recompute R, reverse R, reverse L) are those of
// k_wbp_bwd.  A persistent grid of fixed size walks the frames; each thread
// adds its own weight-gradient entries into its workgroup's partial in frame
// order (the workgroup's first frame stores), so the result does not depend
// on scheduling.
template <class P>
struct BigScratch {
    static constexpr int GE = (P::RI + 1) * P::ROWS;                  // floats per thread per group
    static constexpr size_t ASZ = (size_t)P::G * P::TPS * GE;         // floats per array
    static constexpr size_t per_wg_floats = 4 * ASZ;                  // [array][group][thread][GE]
};

// LDS of the large-frame adjoint: the four boundary buffers (4N floats) and,
// for its first LG groups, the L messages that three later phases read back
// (the one array read three times), as [group][value][thread] so that a
// wave's accesses fall on consecutive banks; the other groups' L messages
// stay in the scratch.  LG fills the workgroup's share of the LDS: all of it
// at N = 4096 (one workgroup per CU), half at N = 2048 (two per CU).
template <class P>
struct BigLds {
    static constexpr int GE = BigScratch<P>::GE;
    static constexpr size_t budget = (size_t)(P::N >= 4096 ? 160 : 80) * 1024;
    static constexpr size_t base_bytes = 4 * (size_t)P::N * sizeof(float);
    static constexpr int LG0 = (int)((budget - base_bytes) / ((size_t)GE * P::TPS * sizeof(float)));
    static constexpr int LG = LG0 < P::G ? LG0 : P::G;
    static constexpr size_t bytes = base_bytes + (size_t)LG * GE * P::TPS * sizeof(float);
};

template <int NLOG, int KP>
__global__ void __launch_bounds__(1 << (NLOG - 2)) k_wbp_bwd_big(WbpArgs a) {
    using P = Plan<NLOG, KP, 2>;
    constexpr int N = P::N, ROWS = P::ROWS, TPS = P::TPS, G = P::G, n = NLOG, GB = P::GB, RI = P::RI;
    constexpr bool MAPPED = (KP > 0 && KP < NLOG);
    constexpr int LOWBITS = NLOG - KP;
    constexpr int NREG = RState<P>::NREG;
    constexpr int GE = BigScratch<P>::GE;
    constexpr size_t ASZ = BigScratch<P>::ASZ;
    const int t = threadIdx.x;
    constexpr int LG = BigLds<P>::LG;
    extern __shared__ __align__(16) float smem[];
    float *const buf = smem;        // [A0 A1 | B0 B1]
    float *const lsl = smem + 4 * N;  // L messages of groups 0..LG-1
    const int8_t *const ords = &a.orders[0][0];

    float *const scr = a.scratch + (size_t)blockIdx.x * BigScratch<P>::per_wg_floats;
    // scratch arrays: L messages, R sweep messages, adjoint of the R state,
    // adjoint of the L messages; a thread's block of group g holds the
    // interior levels l < RI and, at l = RI, the bottom level (L and its
    // adjoint) or the top level (R sweep, adjoint of the R state)
    enum { LS = 0, RS = 1, GS = 2, GL = 3 };
    // The thread index is passed through an empty asm at every group step:
    // otherwise the compiler hoists every block address out of the frame
    // and iteration loops and runs out of registers.
    auto tid_here = [&]() {
        int tt = t;
        asm volatile("" : "+v"(tt));
        return tt;
    };
    auto blk = [&](int arr, int g, int tt) { return scr + arr * ASZ + ((size_t)g * TPS + tt) * GE; };
    auto order_at = [&](int it) { return (KP > 0 && a.Q > 1) ? (it / a.Tev) % a.Q : 0; };
    float *const part = a.partial + (size_t)blockIdx.x * a.T * n * 2 * N;

    for (int64_t frame = blockIdx.x; frame < a.F; frame += gridDim.x) {
        const bool first = frame == (int64_t)blockIdx.x;
        for (int it = a.T - 1; it >= 0; --it) {
            const int q = order_at(it);
            const bool lastit = (it == a.T - 1);
            const bool reset_next = KP > 0 && !lastit && order_at(it + 1) != q;
            const float *wt = a.w + (int64_t)it * n * 2 * N;
            float *const pt = part + (size_t)it * n * 2 * N;
            const float *ck = it > 0 ? a.ckpt + ((frame * (a.T - 1) + (it - 1)) * (int64_t)NREG) * TPS : nullptr;
            int baddr[ROWS], toprow[ROWS];
            float prior[ROWS];
            {
                const int8_t *e = ords + q * 16;
                const int base = GMap<P, G - 1>::base(t);
                sfor<0, ROWS>([&](auto i) {
                    const int p = base + GMap<P, G - 1>::off(i);
                    const int j = (KP > 0) ? relabel_to_row(p, e, n, LOWBITS) : p;
                    toprow[i] = j;
                    prior[i] = a.meta[j] == -2 ? kWbpPrior : 0.f;
                });
                if constexpr (MAPPED) {
                    const int bb = GMap<P, GB>::base(t);
                    sfor<0, ROWS>([&](auto i) { baddr[i] = relabel_to_row(bb + GMap<P, GB>::off(i), e, n, LOWBITS); });
                }
            }
            // The weight gradients of one reverse step (group g, sweep d) are
            // staged in registers and added into the partial together, and the
            // partial's entries are loaded at the start of the step beside its
            // other loads: one memory round trip per step, where adding each
            // gradient as it is made waited on a load per entry.
            struct GStep {
                float prev[P::RMAX][ROWS], val[P::RMAX][ROWS];
            };
            auto gstep_load = [&](auto gc, int d, int base, GStep &s) {
                constexpr int g = decltype(gc)::value, r = P::size(g), lo = P::lo(g);
                if (!first) {
                    sfor<0, r>([&](auto sl) {
                        sfor<0, ROWS>([&](auto i) { s.prev[sl][i] = pt[((lo + sl) * 2 + d) * N + base + GMap<P, g>::off(i)]; });
                    });
                } else {
                    sfor<0, r>([&](auto sl) { sfor<0, ROWS>([&](auto i) { s.prev[sl][i] = 0.f; }); });
                }
            };
            auto gstep_store = [&](auto gc, int d, int base, const GStep &s) {
                constexpr int g = decltype(gc)::value, r = P::size(g), lo = P::lo(g);
                sfor<0, r>([&](auto sl) {
                    sfor<0, ROWS>([&](auto i) {
                        float *p = pt + ((lo + sl) * 2 + d) * N + base + GMap<P, g>::off(i);
                        *p = first ? s.val[sl][i] : s.prev[sl][i] + s.val[sl][i];
                    });
                });
            };
            auto load_state = [&](auto gc, float (&rint)[RI][ROWS], float (&rtop)[ROWS]) {
                constexpr int g = decltype(gc)::value;
                if (ck) {
                    const float *b = ck + RState<P>::off(g, tid_here(), 0);
                    sfor<0, P::size(g) - 1>([&](auto l) { sfor<0, ROWS>([&](auto i) { rint[l][i] = b[l * ROWS + i]; }); });
                    if constexpr (g < G - 1)
                        sfor<0, ROWS>([&](auto i) { rtop[i] = b[(P::size(g) - 1) * ROWS + i]; });
                } else {
                    sfor<0, RI>([&](auto l) { sfor<0, ROWS>([&](auto i) { rint[l][i] = 0.f; }); });
                    if constexpr (g < G - 1) sfor<0, ROWS>([&](auto i) { rtop[i] = 0.f; });
                }
                if constexpr (g == G - 1) sfor<0, ROWS>([&](auto i) { rtop[i] = prior[i]; });
            };
            auto load2 = [&](int arr, auto gc, float (&x)[RI][ROWS], float (&y)[ROWS]) {
                constexpr int g = decltype(gc)::value;
                if constexpr (g < LG) {
                    if (arr == LS) {
                        const float *b = lsl + (size_t)g * GE * TPS + t;
                        sfor<0, P::size(g) - 1>([&](auto l) {
                            sfor<0, ROWS>([&](auto i) { x[l][i] = b[(l * ROWS + i) * TPS]; });
                        });
                        sfor<0, ROWS>([&](auto i) { y[i] = b[(RI * ROWS + i) * TPS]; });
                        return;
                    }
                }
                const float *b = blk(arr, g, tid_here());
                sfor<0, P::size(g) - 1>([&](auto l) { sfor<0, ROWS>([&](auto i) { x[l][i] = b[l * ROWS + i]; }); });
                sfor<0, ROWS>([&](auto i) { y[i] = b[RI * ROWS + i]; });
            };
            auto store2 = [&](int arr, auto gc, const float (&x)[RI][ROWS], const float (&y)[ROWS]) {
                constexpr int g = decltype(gc)::value;
                if constexpr (g < LG) {
                    if (arr == LS) {
                        float *b = lsl + (size_t)g * GE * TPS + t;
                        sfor<0, P::size(g) - 1>([&](auto l) {
                            sfor<0, ROWS>([&](auto i) { b[(l * ROWS + i) * TPS] = x[l][i]; });
                        });
                        sfor<0, ROWS>([&](auto i) { b[(RI * ROWS + i) * TPS] = y[i]; });
                        return;
                    }
                }
                float *b = blk(arr, g, tid_here());
                sfor<0, P::size(g) - 1>([&](auto l) { sfor<0, ROWS>([&](auto i) { b[l * ROWS + i] = x[l][i]; }); });
                sfor<0, ROWS>([&](auto i) { b[RI * ROWS + i] = y[i]; });
            };

            // Arrays that one phase's last group hands to the next phase's
            // first (the same group) stay in registers across the barrier:
            // the last group's L messages (recompute L -> recompute R), group
            // 0's R sweep messages (recompute R -> reverse R), the last group's
            // L adjoints (reverse R -> reverse L)
            float hl_lint[RI][ROWS], hl_lbot[ROWS];
            float h0_rsw[RI][ROWS], h0_rtop[ROWS];
            float hg_gli[RI][ROWS], hg_glb[ROWS];
            // ---- recompute the L sweep (groups 0..G-1) ----
            sfor<0, G>([&](auto g) {
                const int base = GMap<P, g>::base(t);
                float lbot[ROWS], lint[RI][ROWS], rint[RI][ROWS], rtop[ROWS], out[ROWS];
                if constexpr (g == 0) {
                    const float *src = a.llr + frame * N;
                    sfor<0, ROWS>([&](auto i) { lbot[i] = src[base + GMap<P, 0>::off(i)]; });
                } else {
                    const float *lb = buf + (g & 1) * N;
                    if constexpr (MAPPED && g == GB) sfor<0, ROWS>([&](auto i) { lbot[i] = lb[baddr[i]]; });
                    else sfor<0, ROWS>([&](auto i) { lbot[i] = lb[base + GMap<P, g>::off(i)]; });
                }
                load_state(g, rint, rtop);
                wgroup_L<P, g>(lbot, lint, rint, rtop, out, wt + base);
                store2(LS, g, lint, lbot);
                if constexpr (g == G - 1) {
                    sfor<0, RI>([&](auto l) { sfor<0, ROWS>([&](auto i) { hl_lint[l][i] = lint[l][i]; }); });
                    sfor<0, ROWS>([&](auto i) { hl_lbot[i] = lbot[i]; });
                }
                if constexpr (g < G - 1) {
                    float *lt = buf + ((g + 1) & 1) * N;
                    sfor<0, ROWS>([&](auto i) { lt[base + GMap<P, g>::off(i)] = out[i]; });
                }
                __syncthreads();
            });
            if (!lastit) {
                // ---- recompute the R sweep (groups G-1..0), keeping every level ----
                sfor<0, G>([&](auto k) {
                    constexpr int g = G - 1 - k;
                    const int base = GMap<P, g>::base(t);
                    float lbot[ROWS], lint[RI][ROWS], rsw[RI][ROWS], rtop[ROWS], rb[ROWS];
                    if constexpr (g == G - 1) {
                        sfor<0, RI>([&](auto l) { sfor<0, ROWS>([&](auto i) { lint[l][i] = hl_lint[l][i]; }); });
                        sfor<0, ROWS>([&](auto i) { lbot[i] = hl_lbot[i]; });
                    } else {
                        load2(LS, std::integral_constant<int, g>{}, lint, lbot);
                    }
                    if constexpr (g == G - 1) {
                        sfor<0, ROWS>([&](auto i) { rtop[i] = prior[i]; });
                    } else {
                        const float *rs = buf + 2 * N + ((g + 1) & 1) * N;
                        sfor<0, ROWS>([&](auto i) { rtop[i] = rs[base + GMap<P, g>::off(i)]; });
                    }
                    wgroup_R<P, g>(lbot, lint, rsw, rtop, rb, wt + base);
                    if constexpr (g == 0) {
                        sfor<0, RI>([&](auto l) { sfor<0, ROWS>([&](auto i) { h0_rsw[l][i] = rsw[l][i]; }); });
                        sfor<0, ROWS>([&](auto i) { h0_rtop[i] = rtop[i]; });
                    } else {
                        store2(RS, std::integral_constant<int, g>{}, rsw, rtop);
                    }
                    if constexpr (g > 0) {
                        float *rt = buf + 2 * N + (g & 1) * N;
                        if constexpr (MAPPED && g == GB) sfor<0, ROWS>([&](auto i) { rt[baddr[i]] = rb[i]; });
                        else sfor<0, ROWS>([&](auto i) { rt[base + GMap<P, g>::off(i)] = rb[i]; });
                    }
                    __syncthreads();
                });
                // ---- reverse of the R sweep (groups 0..G-1) ----
                sfor<0, G>([&](auto g) {
                    const int base = GMap<P, g>::base(t);
                    float lbot[ROWS], lint[RI][ROWS], rsw[RI][ROWS], rtsw[ROWS], gsi[RI][ROWS], gst[ROWS];
                    float gli[RI][ROWS], glb[ROWS], gb[ROWS], gtop[ROWS];
                    GStep gs;
                    gstep_load(g, 1, base, gs);
                    load2(LS, g, lint, lbot);
                    if constexpr (g == 0) {
                        sfor<0, RI>([&](auto l) { sfor<0, ROWS>([&](auto i) { rsw[l][i] = h0_rsw[l][i]; }); });
                        sfor<0, ROWS>([&](auto i) { rtsw[i] = h0_rtop[i]; });
                    } else {
                        load2(RS, g, rsw, rtsw);
                    }
                    // the adjoint of the R state leaving this iteration; a trellis
                    // switch after it reset the inner levels of the permuted range
                    load2(GS, g, gsi, gst);
                    if constexpr (KP > 0 && g >= GB) {
                        if (reset_next) {
                            sfor<0, RI>([&](auto l) { sfor<0, ROWS>([&](auto i) { gsi[l][i] = 0.f; }); });
                            sfor<0, ROWS>([&](auto i) { gst[i] = 0.f; });
                        }
                    }
                    if constexpr (g == 0) {
                        sfor<0, ROWS>([&](auto i) { gb[i] = 0.f; });
                    } else {
                        const float *src = buf + (g & 1) * N;
                        if constexpr (MAPPED && g == GB) sfor<0, ROWS>([&](auto i) { gb[i] = src[baddr[i]]; });
                        else sfor<0, ROWS>([&](auto i) { gb[i] = src[base + GMap<P, g>::off(i)]; });
                    }
                    sfor<0, RI>([&](auto l) { sfor<0, ROWS>([&](auto i) { gli[l][i] = 0.f; }); });
                    sfor<0, ROWS>([&](auto i) { glb[i] = 0.f; });
                    rev_group_R<P, g, g == 0>(lbot, lint, rsw, rtsw, gb, gsi, gli, glb, gtop, wt + base,
                                              [&](int sl, int i, int, float v) { gs.val[sl][i] = v; });
                    gstep_store(g, 1, base, gs);
                    if constexpr (g == G - 1) {
                        sfor<0, RI>([&](auto l) { sfor<0, ROWS>([&](auto i) { hg_gli[l][i] = gli[l][i]; }); });
                        sfor<0, ROWS>([&](auto i) { hg_glb[i] = glb[i]; });
                    } else {
                        store2(GL, g, gli, glb);
                    }
                    if constexpr (g < G - 1) {
                        float *dst = buf + ((g + 1) & 1) * N;
                        sfor<0, ROWS>([&](auto i) { dst[base + GMap<P, g>::off(i)] = gtop[i] + gst[i]; });
                    }
                    __syncthreads();
                });
            } else {
                // the last iteration runs no R sweep: its R weights get no gradient
                if (first) {
                    for (int idx = t; idx < n * N; idx += blockDim.x) pt[((idx / N) * 2 + 1) * N + (idx & (N - 1))] = 0.f;
                }
            }
            // ---- reverse of the L sweep (groups G-1..0) ----
            sfor<0, G>([&](auto k) {
                constexpr int g = G - 1 - k;
                const int base = GMap<P, g>::base(t);
                float lbot[ROWS], lint[RI][ROWS], rint[RI][ROWS], rtop[ROWS], gli[RI][ROWS], glb[ROWS];
                float gsi[RI][ROWS], gst[ROWS], gt[ROWS];
                GStep gs;
                gstep_load(std::integral_constant<int, g>{}, 0, base, gs);
                auto sink = [&](int sl, int i, int, float v) { gs.val[sl][i] = v; };
                load2(LS, std::integral_constant<int, g>{}, lint, lbot);
                load_state(std::integral_constant<int, g>{}, rint, rtop);
                if (lastit) {
                    sfor<0, RI>([&](auto l) { sfor<0, ROWS>([&](auto i) { gli[l][i] = 0.f; }); });
                    sfor<0, ROWS>([&](auto i) { glb[i] = 0.f; });
                } else if constexpr (g == G - 1) {
                    sfor<0, RI>([&](auto l) { sfor<0, ROWS>([&](auto i) { gli[l][i] = hg_gli[l][i]; }); });
                    sfor<0, ROWS>([&](auto i) { glb[i] = hg_glb[i]; });
                } else {
                    load2(GL, std::integral_constant<int, g>{}, gli, glb);
                }
                sfor<0, RI>([&](auto l) { sfor<0, ROWS>([&](auto i) { gsi[l][i] = 0.f; }); });
                sfor<0, ROWS>([&](auto i) { gst[i] = 0.f; });
                if constexpr (g == G - 1) {
                    // the output adjoint enters at the last iteration only
                    if (lastit) {
                        sfor<0, ROWS>([&](auto i) { gt[i] = a.gout[frame * N + toprow[i]]; });
                        rev_group_L<P, g, true, false>(lbot, lint, rint, rtop, gt, gli, glb, gsi, gst, wt + base,
                                                       sink);
                    } else {
                        rev_group_L<P, g, true, true>(lbot, lint, rint, rtop, gt, gli, glb, gsi, gst, wt + base,
                                                      sink);
                    }
                } else {
                    const float *src = buf + 2 * N + ((g + 1) & 1) * N;
                    sfor<0, ROWS>([&](auto i) { gt[i] = src[base + GMap<P, g>::off(i)]; });
                    rev_group_L<P, g, false, false>(lbot, lint, rint, rtop, gt, gli, glb, gsi, gst, wt + base,
                                                    sink);
                }
                gstep_store(std::integral_constant<int, g>{}, 0, base, gs);
                store2(GS, std::integral_constant<int, g>{}, gsi, gst);
                if constexpr (g > 0) {
                    float *dst = buf + 2 * N + (g & 1) * N;
                    if constexpr (MAPPED && g == GB) sfor<0, ROWS>([&](auto i) { dst[baddr[i]] = glb[i]; });
                    else sfor<0, ROWS>([&](auto i) { dst[base + GMap<P, g>::off(i)] = glb[i]; });
                }
                __syncthreads();
            });
        }
    }
}

}  // namespace pbp
