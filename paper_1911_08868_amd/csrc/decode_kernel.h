// decode_kernel.h -- persistent PP-MT-BP decoding kernel (gfx950).
//
// One workgroup holds `S` frame slots of TPS threads each.  All slots run the
// same sequence of group passes in lock step (workgroup barriers between
// passes); each slot is at its own iteration of its own frame.  A slot whose
// frame stops (CRC or G test, Sec. IV) or reaches N_it,max writes its outputs
// and takes the next frame from a device queue (one atomic per frame), so
// frames that stop early never leave their lanes idle while a long frame
// finishes.  The workgroup exits when the queue is empty and every slot is
// done.
//
// Per iteration (Algorithm 1, oneBPiteration): L passes of groups 0..G-2
// (channel side to u side), the last group's L pass, hard decision and CRC
// syndrome, the last group's R pass, then R passes of groups G-2..0.  A CRC
// stop is decided right after the decision, which does not depend on the R
// sweep, so a stopping frame skips the rest of the sweep.  Between
// iterations a frame that has not stopped switches trellis at multiples of T.
#pragma once

#include "bp_core.h"

namespace pbp {

struct DecodeArgs {
    const float *llr;
    int64_t F;
    uint8_t *msg;
    int32_t *iters;
    uint8_t *ok;
    float *soft;
    const uint32_t *syn;
    const int32_t *meta;
    uint32_t *counter;  // kQueues queue counters, 16 words apart
    int32_t K_msg, max_iter, it_min, stop;
    float alpha;
    int32_t T, Q;
    int8_t orders[8][16];
    uint64_t *hist;  // [F][H] decision hashes (trace kernels only)
    int32_t H;
    float noise_sigma;    // channel noise injected at every event (noise kernels only)
    uint64_t noise_seed;
};

template <class P>
struct DecodeLds {
    static constexpr int NW = (P::N + 31) / 32;
    // bytes of dynamic LDS for S slots
    static constexpr size_t bytes(int S) {
        return (size_t)S * 4 * LdsPad<P>::words * sizeof(float)  // L/R boundary ping-pong buffers
               + (size_t)S * sizeof(int)                // frame of each slot
               + (size_t)S * P::WPS * sizeof(uint32_t)  // syndrome partials
               + (size_t)S * P::WPS * 2 * sizeof(uint32_t)  // decision-hash partials
               + (size_t)S * 2 * NW * sizeof(uint32_t)  // G test words (u_hat, x_hat)
               + (size_t)S * sizeof(int)                // G test verdict
               + 8 * 16;                                // stage orders of the pool
    }
};

// launch bound: one frame's threads, at least 256
template <int NLOG, int RHO>
constexpr int decode_launch_bound() {
    return ((1 << (NLOG - RHO)) > 256) ? (1 << (NLOG - RHO)) : 256;
}
// waves per SIMD the register allocation must allow: 4 (<= 128 VGPRs) for
// two rows per thread, 2 for eight or for the decision-history kernels
template <int RHO, bool TRACE = false>
constexpr int decode_min_waves() {
    return RHO <= 2 && !TRACE ? 4 : 2;
}

// Iteration parameters shared by every frame source.
struct DecodeCtl {
    int32_t max_iter, it_min, stop;
    float alpha;
    int32_t T, Q;
    const int8_t *orders;  // [8][16], in global or kernel-argument memory
    float noise_sigma = 0.f;
    uint64_t noise_seed = 0;
};

// The lock-step slot loop.  Src supplies frames: pop() (slot leader only)
// returns the next frame or a value >= Src::F when the queue is empty;
// per frame it gives the LLR pointer, the code tables and the output sinks.
// With Src::kTrace the loop also hashes every iteration's decisions
// (decision_key) and hands the hash to Src::trace (slot leader only).  With
// Src::kNoise every event (after iterations T, 2T, ..., also where the graph
// stays) sets the channel level to the received LLRs plus
// noise_sigma * noise_gauss(frame, event, row).
// tid is the thread's index in the workgroup (threadIdx.x, or a copy the
// caller has hidden from the optimiser).
template <int NLOG, int KP, int RHO, int CN, bool GMODE, class Src>
__device__ __forceinline__ void decode_loop(Src &src, const DecodeCtl &a, float *smem, int S, const int tid) {
    using P = Plan<NLOG, KP, RHO>;
    constexpr int N = P::N, ROWS = P::ROWS, TPS = P::TPS, G = P::G, n = NLOG;
    constexpr int GB = P::GB;
    constexpr int NW = DecodeLds<P>::NW;
    constexpr int WPS = P::WPS;
    constexpr bool MAPPED_BOUNDARY = (KP > 0 && KP < NLOG);
    constexpr int LOWBITS = NLOG - KP;
    // A frame of at most one wave (TPS <= 64) exchanges nothing with other
    // waves: each wave then runs its slots on its own, with no workgroup
    // barrier in the loop (refill, syndrome and G test stay inside the wave)
    // and leaves when none of its slots has a frame.
    constexpr bool WSLOT = TPS <= 64;
    constexpr bool TRACE = Src::kTrace;
    constexpr bool NOISE = Src::kNoise;

    const int slot = tid / TPS;
    const int t = tid & (TPS - 1);
    const int F = (int)src.F;

    constexpr int NP = LdsPad<P>::words;  // padded length of one boundary buffer
    float *const buf = smem + (size_t)slot * 4 * NP;  // [L0 | L1 | R0 | R1]
    int *const frame_slot = reinterpret_cast<int *>(smem + (size_t)S * 4 * NP);
    uint32_t *const synpart = reinterpret_cast<uint32_t *>(frame_slot + S);
    uint32_t *const hpart = synpart + S * WPS;  // [slot][wave][lo, hi]
    uint32_t *const gwords = hpart + S * WPS * 2;
    int *const gflag = reinterpret_cast<int *>(gwords + S * 2 * NW);
    int8_t *const ords = reinterpret_cast<int8_t *>(gflag + S);

    // every workgroup size, also below 128 threads, copies the whole pool
    for (int i = tid; i < 8 * 16; i += blockDim.x) ords[i] = a.orders[i];
    if constexpr (GMODE) {
        for (int w = tid; w < S * 2 * NW; w += blockDim.x) gwords[w] = 0u;
    }
    if constexpr (WSLOT) __syncthreads();  // the orders and words before any wave starts

    Regs<P> st;
    uint32_t synv[ROWS];
    float prior[ROWS];  // R on level n+1 of this thread's rows: +inf frozen, 0 information
    // LDS addresses of the relabelled boundary rows in buffer 0 of this slot:
    // a 32-bit LDS pointer per row, so every access is one ds instruction
    // with the buffer's constant offset
    typedef __attribute__((address_space(3))) float lds_f32;
    lds_f32 *bptr[ROWS];
    uint64_t hkey[TRACE ? ROWS : 1];  // decision keys of this thread's rows
    uint64_t htotal = 0;               // the slot's decision hash (one-wave frames)
    uint32_t ubits = 0;
    uint32_t synv_total = 0;  // the slot's syndrome (one-wave frames)
    int it = 0, q = 0, next_ev = 0, ev = 0;
    int frame = 0;  // frame indices fit 31 bits (the host checks F)
    const uint32_t *tsyn = nullptr;
    const int32_t *tmeta = nullptr;
    bool active = false, need_new = true;
    const float alpha = a.alpha;
    const float inf = __builtin_huge_valf();

    // decision of register row i
    auto decide = [&](auto i) { return st.Ltop[i] < -prior[i]; };

    // --- per-frame (re)initialisation helpers ------------------------------
    auto load_top_info = [&](int qq) {
        const int8_t *e = ords + qq * 16;
        const int base = GMap<P, G - 1>::base(t);
        sfor<0, ROWS>([&](auto i) {
            int p = base + GMap<P, G - 1>::off(i);
            int j = (KP > 0) ? relabel_to_row(p, e, n, LOWBITS) : p;
            const int m = tmeta[j];
            synv[i] = tsyn[j];
            prior[i] = m == -2 ? inf : 0.f;
            if constexpr (TRACE) hkey[i] = decision_key(j);
        });
        if constexpr (MAPPED_BOUNDARY) {
            const int bb = GMap<P, GB>::base(t);
            sfor<0, ROWS>([&](auto i) {
                bptr[i] = (lds_f32 *)buf + LdsPad<P>::at(relabel_to_row(bb + GMap<P, GB>::off(i), e, n, LOWBITS));
            });
        }
    };
    auto load_channel = [&](int qq) {
        const float *lsrc = src.llr(frame);
        const int base = GMap<P, 0>::base(t);
        if constexpr (KP == NLOG) {
            const int8_t *e = ords + qq * 16;
            sfor<0, ROWS>([&](auto i) {
                st.Lbot[0][i] = lsrc[relabel_to_row(base + GMap<P, 0>::off(i), e, n, 0)];
            });
        } else {
            sfor<0, ROWS>([&](auto i) { st.Lbot[0][i] = lsrc[base + GMap<P, 0>::off(i)]; });
        }
    };
    auto start_frame = [&]() {
        it = 0;
        q = 0;
        next_ev = a.T;
        ev = 0;
        tsyn = src.syn(frame);
        tmeta = src.meta(frame);
        sfor<0, G>([&](auto g) {
            sfor<0, P::RI>([&](auto l) { sfor<0, ROWS>([&](auto i) { st.Rint[g][l][i] = 0.f; }); });
            sfor<0, ROWS>([&](auto i) { st.Rtop[g][i] = 0.f; });
        });
        load_channel(0);
        load_top_info(0);
    };
    // trellis switch (Sec. III): levels strictly inside the permuted range are
    // reset; in relabelled coordinates nothing else moves
    auto apply_event = [&]() {
        sfor<GB, G>([&](auto g) {
            sfor<0, P::RI>([&](auto l) { sfor<0, ROWS>([&](auto i) { st.Rint[g][l][i] = 0.f; }); });
            if constexpr (g < G - 1) sfor<0, ROWS>([&](auto i) { st.Rtop[g][i] = 0.f; });
        });
        if constexpr (KP == NLOG) load_channel(q);
        load_top_info(q);
    };
    // noise injection at event e: received LLR + sigma g, with the channel
    // row of each register row as load_channel reads it
    auto inject_noise = [&](int e) {
        const float *lsrc = src.llr(frame);
        const int base = GMap<P, 0>::base(t);
        const int8_t *eo = ords + q * 16;
        sfor<0, ROWS>([&](auto i) {
            const int p = base + GMap<P, 0>::off(i);
            const int j = (KP == NLOG) ? relabel_to_row(p, eo, n, 0) : p;
            const float g = noise_gauss(a.noise_seed, frame, e, j);
            const float z = a.noise_sigma * g;
            st.Lbot[0][i] = lsrc[j] + z;
        });
    };

    for (;;) {
        // ---- queue: refill finished slots --------------------------------
        if constexpr (WSLOT) {
            // the slot's leader pops; its lanes read the frame after a wave fence
            if (need_new) {
                if (t == 0) frame_slot[slot] = (int)src.pop();
                boundary_sync<true>();
                frame = frame_slot[slot];
                active = frame < F;
                need_new = false;
                if (active) start_frame();
            }
            if (__ballot(active) == 0ull) break;
        } else {
            // one frame per workgroup (S == 1): need_new is uniform, so the queue
            // round trip and its barrier happen only when the frame ends
            const bool refill = S > 1 || need_new;
            if (refill) {
                if (need_new && t == 0) frame_slot[slot] = (int)src.pop();
                __syncthreads();
            }
            if (need_new) {
                frame = frame_slot[slot];
                active = frame < F;
                need_new = false;
                if (active) start_frame();
            }
            if (refill) {
                bool any = false;
                for (int s = 0; s < S; ++s) any |= frame_slot[s] < F;
                if (!any) break;
            }
        }

        // ---- L sweep: groups 0..G-2 ---------------------------------------
        sfor<0, G - 1>([&](auto g) {
            if (active) {
                if constexpr (g > 0) {
                    const float *lb = buf + (g & 1) * NP;
                    if constexpr (MAPPED_BOUNDARY && g == GB) {
                        sfor<0, ROWS>([&](auto i) { st.Lbot[g][i] = bptr[i][(g & 1) * NP]; });
                    } else {
                        const int pb = GMap<P, g>::pbase(t);
                        sfor<0, ROWS>([&](auto i) { st.Lbot[g][i] = lb[pb + GMap<P, g>::poff(i)]; });
                    }
                }
                float out[ROWS];
                group_L<P, g, CN>(st, st.Rtop[g], out, alpha);
                float *lt = buf + ((g + 1) & 1) * NP;
                const int pb = GMap<P, g>::pbase(t);
                sfor<0, ROWS>([&](auto i) { lt[pb + GMap<P, g>::poff(i)] = out[i]; });
            }
            boundary_sync<wave_local_boundary<P, g>(MAPPED_BOUNDARY)>();
        });

        // ---- last group: L pass, decision, R pass ---------------------------
        if (active) {
            if constexpr (G > 1) {
                const float *lb = buf + ((G - 1) & 1) * NP;
                if constexpr (MAPPED_BOUNDARY && G - 1 == GB) {
                    sfor<0, ROWS>([&](auto i) { st.Lbot[G - 1][i] = bptr[i][((G - 1) & 1) * NP]; });
                } else {
                    const int pb = GMap<P, G - 1>::pbase(t);
                    sfor<0, ROWS>([&](auto i) { st.Lbot[G - 1][i] = lb[pb + GMap<P, G - 1>::poff(i)]; });
                }
            }
            group_L<P, G - 1, CN>(st, prior, st.Ltop, alpha);
            // hard decision (Sec. II-B): u = 1 iff L + R < 0 on level n+1,
            // R = +inf (frozen) or 0, i.e. iff L < -R (one compare: never for a
            // frozen row, and -0 decides 0); the CRC syndrome of the decided
            // rows accumulates their columns
            uint32_t syn = 0;
            sfor<0, ROWS>([&](auto i) { syn ^= decide(i) ? synv[i] : 0u; });
            uint64_t hh = 0;
            if constexpr (TRACE) sfor<0, ROWS>([&](auto i) { hh ^= decide(i) ? hkey[i] : 0ull; });
            if constexpr (GMODE) {
                ubits = 0;
                sfor<0, ROWS>([&](auto i) { ubits |= (decide(i) ? 1u : 0u) << i; });
            }
            float rb[ROWS];
            group_R<P, G - 1, CN>(st, prior, rb, alpha);
            if constexpr (G > 1) {
                float *rt = buf + 2 * NP + ((G - 1) & 1) * NP;
                if constexpr (MAPPED_BOUNDARY && G - 1 == GB) {
                    sfor<0, ROWS>([&](auto i) { bptr[i][2 * NP + ((G - 1) & 1) * NP] = rb[i]; });
                } else {
                    const int pb = GMap<P, G - 1>::pbase(t);
                    sfor<0, ROWS>([&](auto i) { rt[pb + GMap<P, G - 1>::poff(i)] = rb[i]; });
                }
            }
            if constexpr (TRACE) {
                const uint32_t lo = lanes_xor<(TPS < 64 ? TPS : 64)>((uint32_t)hh);
                const uint32_t hi = lanes_xor<(TPS < 64 ? TPS : 64)>((uint32_t)(hh >> 32));
                if constexpr (WSLOT) {
                    htotal = ((uint64_t)hi << 32) | lo;
                } else if ((t & 63) == 0) {
                    hpart[(slot * WPS + (t >> 6)) * 2] = lo;
                    hpart[(slot * WPS + (t >> 6)) * 2 + 1] = hi;
                }
            }
            if constexpr (!GMODE) {
                syn = lanes_xor<(TPS < 64 ? TPS : 64)>(syn);
                if constexpr (WSLOT) {
                    synv_total = syn;  // every lane of the slot holds the whole syndrome
                } else {
                    if ((t & 63) == 0) synpart[slot * WPS + (t >> 6)] = syn;
                }
            } else {
                uint32_t *U = gwords + slot * 2 * NW;
                const int base = GMap<P, G - 1>::base(t);
                sfor<0, ROWS>([&](auto i) {
                    if ((ubits >> i) & 1u) {
                        const int j = base + GMap<P, G - 1>::off(i);
                        atomicOr(&U[j >> 5], 1u << (j & 31));
                    }
                });
                if constexpr (G == 1) {
                    uint32_t *X = U + NW;
                    sfor<0, ROWS>([&](auto i) {
                        if (st.Lbot[0][i] + rb[i] < 0.f) {
                            const int j = base + GMap<P, 0>::off(i);
                            atomicOr(&X[j >> 5], 1u << (j & 31));
                        }
                    });
                }
            }
        }
        boundary_sync<WSLOT>();

        if constexpr (TRACE) {
            if (active) {
                uint64_t h = htotal;
                if constexpr (!WSLOT) {
                    h = 0;
                    for (int w = 0; w < WPS; ++w)
                        h ^= ((uint64_t)hpart[(slot * WPS + w) * 2 + 1] << 32) | hpart[(slot * WPS + w) * 2];
                }
                if (t == 0) src.trace(frame, it, h);
            }
        }

        bool finishing = false, pass = false;
        if constexpr (!GMODE) {
            if (active) {
                uint32_t s = synv_total;
                if constexpr (!WSLOT)
                    for (int w = 0; w < WPS; ++w) s ^= synpart[slot * WPS + w];
                pass = (s == 0u);
                finishing = (it + 1 == a.max_iter) || (a.stop == 2 && it + 1 >= a.it_min && pass);
            }
        }

        // ---- R sweep: groups G-2..0 ----------------------------------------
        sfor<0, G - 1>([&](auto k) {
            constexpr int g = G - 2 - k;
            if (active && !finishing) {
                const float *rsrc = buf + 2 * NP + ((g + 1) & 1) * NP;
                const int base = GMap<P, g>::base(t), pb = GMap<P, g>::pbase(t);
                sfor<0, ROWS>([&](auto i) { st.Rtop[g][i] = rsrc[pb + GMap<P, g>::poff(i)]; });
                float rb[ROWS];
                group_R<P, g, CN>(st, st.Rtop[g], rb, alpha);
                if constexpr (g > 0) {
                    float *rt = buf + 2 * NP + (g & 1) * NP;
                    if constexpr (MAPPED_BOUNDARY && g == GB) {
                        sfor<0, ROWS>([&](auto i) { bptr[i][2 * NP + (g & 1) * NP] = rb[i]; });
                    } else {
                        sfor<0, ROWS>([&](auto i) { rt[pb + GMap<P, g>::poff(i)] = rb[i]; });
                    }
                } else if constexpr (GMODE) {
                    uint32_t *X = gwords + slot * 2 * NW + NW;
                    sfor<0, ROWS>([&](auto i) {
                        if (st.Lbot[0][i] + rb[i] < 0.f) {
                            const int j = base + GMap<P, 0>::off(i);
                            atomicOr(&X[j >> 5], 1u << (j & 31));
                        }
                    });
                }
            }
            // the R messages written here are read by group g-1; after the
            // last step only the G test reads what every thread wrote (the
            // next LDS writes, at the first L boundary, are ordered behind
            // the cross-wave barriers of this iteration)
            if constexpr (g > 0) {
                boundary_sync<WSLOT || (!GMODE && wave_local_boundary<P, g - 1>(MAPPED_BOUNDARY))>();
            } else if constexpr (GMODE) {
                boundary_sync<WSLOT>();
            }
        });

        if constexpr (GMODE) {
            // G test (stopping criterion of the G-matrix kind): u_hat G_N == x_hat
            if (active && t == 0) {
                uint32_t *U = gwords + slot * 2 * NW, *X = U + NW;
                uint32_t w[NW];
                for (int i = 0; i < NW; ++i) w[i] = U[i];
                constexpr uint32_t M[5] = {0x55555555u, 0x33333333u, 0x0F0F0F0Fu, 0x00FF00FFu,
                                           0x0000FFFFu};
                for (int b = 0; b < n && b < 5; ++b)
                    for (int i = 0; i < NW; ++i) w[i] ^= (w[i] >> (1 << b)) & M[b];
                for (int b = 5; b < n; ++b)
                    for (int i = 0; i < NW; ++i)
                        if (!((i >> (b - 5)) & 1)) w[i] ^= w[i | (1 << (b - 5))];
                uint32_t diff = 0;
                const uint32_t last = (N >= 32) ? 0xFFFFFFFFu : ((1u << N) - 1u);
                for (int i = 0; i < NW; ++i) diff |= (w[i] ^ X[i]) & (i == NW - 1 ? last : 0xFFFFFFFFu);
                gflag[slot] = diff == 0u;
                for (int i = 0; i < 2 * NW; ++i) U[i] = 0u;
            }
            boundary_sync<WSLOT>();
            if (active) {
                pass = gflag[slot] != 0;
                finishing = (it + 1 == a.max_iter) || (a.stop == 1 && it + 1 >= a.it_min && pass);
            }
        }

        // ---- bookkeeping -----------------------------------------------------
        if (active) {
            if (finishing) {
                // message rows of this thread: original row -> message index
                uint8_t *mo = src.msg(frame);
                const int8_t *e = ords + q * 16;
                const int base = GMap<P, G - 1>::base(t);
                const bool soft = src.want_soft();
                sfor<0, ROWS>([&](auto i) {
                    const int p = base + GMap<P, G - 1>::off(i);
                    const int j = (KP > 0) ? relabel_to_row(p, e, n, LOWBITS) : p;
                    const int m = tmeta[j];
                    if (m >= 0) mo[m] = (uint8_t)(decide(i) ? 1 : 0);
                    if (soft) src.soft(frame, j, st.Ltop[i]);
                });
                if (t == 0) src.finish(frame, it + 1, pass);
                need_new = true;
            } else {
                it += 1;
                if constexpr (KP > 0 || NOISE) {
                    // trellis switch at iterations T, 2T, ...: pool entry (it/T) mod Q
                    if (it == next_ev) {
                        next_ev += a.T;
                        if constexpr (KP > 0) {
                            const int qn = q + 1 == a.Q ? 0 : q + 1;
                            if (qn != q) {
                                q = qn;
                                apply_event();
                            }
                        }
                        if constexpr (NOISE) inject_noise(++ev);
                    }
                }
            }
        }
    }
}


// ---------------------------------------------------------------------------
// Frames claimed from a queue counter in chunks of C consecutive queue
// entries: below N = 128 a frame finishes so fast that one atomic per frame
// caps the frame rate, so those lengths take C = 256 / N entries per claim;
// from N = 128 on every entry is its own chunk (larger chunks measured slower
// there: a longer tail and frames in flight spread further apart).  Each
// frame is decoded exactly once.
template <int N_>
struct ChunkClaim {
    static constexpr int C = N_ >= 128 ? 1 : 256 / N_;
    int64_t next = 0, end = 0;
    template <class Add>
    __device__ int64_t take(int64_t total, Add &&add) {
        if (next < end) return next++;
        const int64_t base = add(C);
        if (base >= total) return total;
        next = base + 1;
        end = base + C < total ? base + C : total;
        return base;
    }
};

// Frame source of a single-code launch.  Frames 0..F-1 are spread over QN
// interleaved queues, queue k holding frames k, k + QN, ..., each with its
// own counter on its own 64-byte line (a.counter + 16 k).  One counter
// serialises its atomics at about 1e8 per second (11.5 ns per frame): below
// N = 1024 a frame of a few tens of iterations takes less than that (about
// 0.14 ns per frame-iteration at N = 256 on the whole chip), so those lengths
// use kQueues queues; from N = 1024 on (1.6 ns per frame-iteration) one queue
// measured faster.  A slot starts at queue (workgroup + thread / 16) mod QN
// and moves to the next queue when one runs dry, so it leaves after at most
// QN failed claims.  With TR it records the decision hash of iteration it
// (0-based) of frame f at hist[f][it mod H]; NZ selects the noise-injecting
// schedule.
constexpr int kQueues = 8;  // counters the host clears per call
template <int N_, bool TR, bool NZ = false>
struct SingleSrc {
    static constexpr bool kTrace = TR;
    static constexpr bool kNoise = NZ;
    static constexpr int QN = N_ >= 1024 ? 1 : kQueues;
    const DecodeArgs &a;
    int64_t F;
    ChunkClaim<N_> claim;
    int q, left = QN;  // current queue; queues not yet found empty
    __device__ SingleSrc(const DecodeArgs &args)
        : a(args), F(args.F), q((int)((blockIdx.x + (threadIdx.x >> 4)) % QN)) {}
    __device__ int64_t pop() {
        if constexpr (QN == 1)
            return claim.take(F, [&](int b) { return (int64_t)atomicAdd(a.counter, (unsigned)b); });
        while (left > 0) {
            const int64_t nq = F > q ? (F - q + QN - 1) / QN : 0;  // frames of queue q
            const int64_t i = claim.take(nq, [&](int b) {
                return (int64_t)atomicAdd(a.counter + 16 * q, (unsigned)b);
            });
            if (i < nq) return q + (int64_t)QN * i;
            // queue q is empty (and stays so); its chunk is used up
            --left;
            q = (q + 1) % QN;
        }
        return F;
    }
    __device__ const float *llr(int64_t f) const { return a.llr + f * N_; }
    __device__ const uint32_t *syn(int64_t) const { return a.syn; }
    __device__ const int32_t *meta(int64_t) const { return a.meta; }
    __device__ uint8_t *msg(int64_t f) const { return a.msg + f * a.K_msg; }
    __device__ bool want_soft() const { return a.soft != nullptr; }
    __device__ void soft(int64_t f, int j, float v) const { a.soft[f * N_ + j] = v; }
    __device__ void finish(int64_t f, int iters, bool pass) const {
        if (a.iters) a.iters[f] = iters;
        if (a.ok) a.ok[f] = pass ? 1 : 0;
    }
    __device__ void trace(int64_t f, int it, uint64_t h) const {
        if constexpr (TR) a.hist[f * a.H + it % a.H] = h;
    }
};

template <int NLOG, int KP, int RHO, int CN, bool GMODE, bool TRACE, bool NOISE>
__global__ void __launch_bounds__((decode_launch_bound<NLOG, RHO>()), (decode_min_waves<RHO, TRACE || NOISE>()))
k_decode(DecodeArgs a) {
    extern __shared__ __align__(16) float smem[];
    constexpr int TPS = Plan<NLOG, KP, RHO>::TPS;
    const int S = blockDim.x / TPS;
    DecodeCtl c{a.max_iter, a.it_min, a.stop, a.alpha, a.T, a.Q, &a.orders[0][0], a.noise_sigma, a.noise_seed};
    SingleSrc<(1 << NLOG), TRACE, NOISE> src(a);
    decode_loop<NLOG, KP, RHO, CN, GMODE>(src, c, smem, S, (int)threadIdx.x);
}

}  // namespace pbp
