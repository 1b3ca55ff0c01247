/*
 * polarbp.h -- C ABI of the MI355X (gfx950) library for partially permuted
 * multi-trellis belief-propagation decoding of CRC-aided polar codes
 * (Ranasinghe, Rajatheva, Latva-aho, "Partially Permuted Multi-Trellis Belief
 * Propagation for Polar Codes", arXiv 1911.08868).
 *
 * Conventions shared by every entry point
 *  - Pointers named d_* are device pointers on the device that was current
 *    when the code object was constructed; every other pointer is host memory.
 *    The caller owns all buffers; the library neither frees nor retains them
 *    beyond the work it enqueues.
 *  - `stream` is a hipStream_t passed as void*; NULL is the default stream.
 *    Work is enqueued asynchronously; device faults surface at the caller's
 *    next synchronisation.
 *  - Return value: 0 on success, otherwise a negative code (PC_E*).  The
 *    thread-local string polar_last_error() describes the last failure.  No
 *    C++ exception crosses this interface.
 *  - F = 0 frames is a no-op that returns 0.
 *  - Factor graph: level 1 holds the channel LLRs L_{1,j} and level n+1 the
 *    a-priori values R_{n+1,j} (Sec. II-B); stage s (1..n) joins levels s and
 *    s+1 and, in the original graph, pairs rows 2^(s-1) apart, so stages 1..m
 *    form N/2^m disjoint subgraphs (Sec. III).  LLR > 0 favours bit 0; the hard
 *    decision is 0 iff R + L >= 0 (Sec. II-B).
 */
#ifndef POLARBP_H
#define POLARBP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PC_OK 0
#define PC_EINVAL (-1)  /* bad argument: null pointer, size or parameter out of range */
#define PC_ENOTSUP (-2) /* valid combination that this library does not implement     */
#define PC_EHIP (-3)    /* HIP runtime or launch error                                */
#define PC_ENOMEM (-4)  /* workspace too small or device allocation failed            */

#define PC_STOP_NONE 0 /* run max_iter iterations                                     */
#define PC_STOP_G 1    /* stop when u_hat G_N equals the hard decision on level 1     */
#define PC_STOP_CRC 2  /* stop when the CRC of the decided message matches (Sec. IV)  */

#define PC_PP_NONE (-1) /* standard BP on the original graph                          */
#define PC_PP_LASTK 0   /* last k stages re-ordered from a seeded pool every T iters  */
#define PC_PP_FULL 1    /* all n stages re-ordered: multi-trellis BP with full
                           permutations (Sec. II-D); only L_1 and R_{n+1} survive     */
#define PC_PP_ALG1 2    /* Algorithm 1: a random subgraph re-ordered per event, the
                           events spaced by Eq. 2 (see pc_pp_params)                  */
#define PC_PP_ALG1_ORIG 3 /* Algorithm 1 with each event's subgraph taken from the
                           original graph (see pc_pp_params)                          */

/* Opaque polar code: frozen set, CRC, and device copies of the per-row
 * tables the decoder reads.  Immutable after construction; may be shared by
 * threads and streams.                                                      */
typedef struct pc_code pc_code;

#define PC_CHECK_MINSUM 0 /* f(x,y) = alpha sgn(x) sgn(y) min(|x|,|y|) (Sec. II-B, IV)  */
#define PC_CHECK_EXACT 1  /* f(x,y) = x boxplus y = 2 atanh(tanh(x/2) tanh(y/2))      */

/* Decoder iteration parameters (Algorithm 1 inputs N_it,max and stopID, plus
 * the min-sum scale, the first iteration at which the stop test is applied,
 * Sec. IV, and the check function of the processing element, Sec. II-B).
 * PC_CHECK_EXACT needs alpha = 1 and is built for the decode entry points
 * with the default launch shape or rho = 2, and for Algorithm 1 (not for the
 * batched decoder or the decision history).  It is evaluated in FP32 as
 * sgn sgn [min(|x|,|y|) + ln(1 + e^-(|x|+|y|)) - ln(1 + e^-||x|-|y||)] on the
 * hardware exp2/log2 (about 1e-7 absolute per check node), so it agrees with
 * an FP64 evaluation to rounding, not bit for bit.                          */
typedef struct {
    int32_t max_iter; /* N_it,max >= 1                                       */
    float alpha;      /* min-sum scale; 1 = the unscaled min-sum of Sec. IV  */
    int32_t stop;     /* PC_STOP_*                                           */
    int32_t it_min;   /* stop test applied from this iteration on (>= 1)     */
    int32_t check;    /* PC_CHECK_*                                          */
} pc_bp_params;

/* Multi-trellis schedule (Sec. II-D, Sec. III).  For PC_PP_LASTK the pool
 * holds min(pool_Q, k!) stage orders: entry 0 is the original graph, entries
 * 1.. give stages n-k+1..n distinct non-identity orders of bits n-k..n-1,
 * drawn from `seed` with SplitMix64 (polar_trellis_pool).  After iteration
 * T, 2T, ... (and before max_iter) a frame that has not stopped switches to
 * entry (iter / T) mod Q and, if its graph changed, its messages on the levels
 * strictly inside the permuted range are reset to 0.  PC_PP_FULL is the same
 * with k = n.                                                               */
typedef struct {
    int32_t mode;     /* PC_PP_*                                             */
    int32_t k;        /* permuted stages, 2 <= k <= n (LASTK)                */
    int32_t period_T; /* iterations between permutations, >= 1               */
    int32_t pool_Q;   /* pool size, 1 <= Q <= 8                              */
    int32_t P_range, P_level, D, N_min, first_reset; /* ALG1, below         */
    uint64_t seed;
    float noise_sigma; /* 0, or noise injected at the events (below)        */
} pc_pp_params;
/* Noise injection (PC_PP_LASTK / PC_PP_FULL / PC_PP_ALG1 with noise_sigma >
 * 0; the paper names noise injection together with partial permutations as
 * future work, Sec. V, beside the noise-aided BP of Table I, sigma^2 = 0.36).
 * At every event, after iteration T, 2T, ... of the fixed schedules (also
 * when pool_Q = 1 and the graph stays) or after each event of Algorithm 1,
 * the channel level becomes y_j + noise_sigma * g with y_j the received LLR
 * and g an Irwin-Hall approximation of N(0,1): the twelve 16-bit fields k of
 * three SplitMix64 outputs from the state
 * seed ^ frame*0x9E3779B97F4A7C15 ^ e*0xC2B2AE3D27D4EB4F ^ j*0x165667B19E3779F9
 * (j = row; e = iteration / T, or for Algorithm 1 the count 1, 2, ... of the
 * frame's events), each read as (k + 1/2)/2^16, summed, minus 6; the product
 * and the sum round once each in single precision.  Built with min-sum and
 * the default launch shape or rho = 2; not with the batched decoder, the
 * decision history or weighted BP.                                         */
/* PC_PP_ALG1 (Algorithm 1, Sec. III and Table I).  At an event a frame draws
 * rho_range ~ U{2..P_range}, rho_level = min(U{1..P_level}, n - rho_range + 1)
 * and one of the N/2^m connected blocks of stages 1..m of its current graph
 * (m = rho_level + rho_range - 1, blocks ranked by their smallest row); stages
 * rho_level..m of that block get a new non-identity order of the bits they
 * use, and the block's nodes on the levels strictly between them are reset.
 * A draw whose block is not 2^m rows or whose stages do not each use one bit
 * over it is drawn again (at most 64 times; then the event is skipped).  The
 * draws come from SplitMix64 seeded with seed + (frame + 1) * 0x9E3779B97F4A7C15.
 * The first event follows iteration first_reset (0: min(max(N_min,
 * floor(N (n-1) / D)), floor(max_iter / 2))); each later one follows
 * iteration it + max(N_min, floor(N_zero / D)) with N_zero = 2^m (rho_range-1)
 * of the previous event (0 if skipped; D = 0 gives N_min).  Needs
 * 2 <= P_range <= n, 1 <= P_level <= n-1, N_min >= 1.  On the GPU: N = 16 ..
 * 1024, codes with a CRC and PC_STOP_CRC or PC_STOP_NONE; one frame per
 * workgroup, one row per thread (messages in registers, the levels partners
 * read in LDS), so no launch configuration.
 * PC_PP_ALG1_ORIG reads Sec. III's subgraph as one of the N/2^m aligned blocks
 * of the ORIGINAL graph: the draws are rho_range, rho_level (as above), the
 * block index in [0, N/2^m), then the order of bits rho_level-1..m-1 (the same
 * non-identity shuffle), with no redraw.  Before permuting, the block of the
 * previous event returns to the original order, so the graph differs from
 * the original in at most one block; the R messages on the inner levels
 * rho_level..m-1 of both blocks are reset, and N_zero of Eq. 2 counts the
 * union of those nodes.  Parameters, limits, spacing and noise as for
 * PC_PP_ALG1; on the GPU one processing element per thread.                */

/* Launch configuration picked by the autotuner; NULL selects the library's
 * table.  rho: log2 rows held per thread per level (2 or 3); slots: frames
 * resident per workgroup; grid: workgroups (0 = as many as fit the GPU).    */
typedef struct {
    int32_t rho;
    int32_t slots;
    int32_t grid;
} pc_launch_cfg;

/* Code construction by Bhattacharyya parameters (Sec. II-A): the K most
 * reliable bit channels of the factor graph above, designed for BPSK-AWGN at
 * design_ebn0_db with rate K/N (CRC included in K, Sec. IV).  N a power of
 * two in [2, 4096]; crc_width 0 or 1..32 with crc_width < K; crc_poly the
 * generator with or without its x^width term (MSB-first, init 0, no
 * reflection, no final xor).  The information set carries the K - crc_width
 * message bits first and the CRC (MSB first) last, in ascending index order.
 * *out receives a new code owned by the caller (free with polar_code_free). */
int polar_construct(int32_t N, int32_t K, int32_t crc_width, uint32_t crc_poly,
                    double design_ebn0_db, pc_code **out);

/* Frees a code.  No work using it may still be in flight.  NULL is a no-op. */
int polar_code_free(pc_code *code);

/* Host copies of the information set (ascending, K entries) and the frozen
 * indicator (N bytes, 1 = frozen).  Either pointer may be NULL.             */
int polar_code_query(const pc_code *code, int32_t *info_idx, uint8_t *frozen);

/* The stage orders of the multi-trellis pool for (n, k, Q, seed):
 * orders[q*n + s-1] is the bit used by stage s in pool entry q.  Returns the
 * number of entries (min(Q, k!)) or a negative code.  Host only.            */
int polar_trellis_pool(int32_t n, int32_t k, int32_t Q, uint64_t seed, int8_t *orders);

/* Encoding x = u G_N, G_N = F^{(x)n} (Eq. 1): message + CRC placed on the
 * information set, zeros on the frozen set.  d_msg uint8 [F][K - crc_width]
 * (bit values 0/1), d_x uint8 [F][N].                                       */
int polar_encode(const pc_code *code, const uint8_t *d_msg, uint8_t *d_x, int64_t F,
                 void *stream);

/* The information bits u_A of each frame (Sec. II-A: the message bits, then
 * their CRC, most significant first, on the information set in ascending row
 * order; Sec. IV: CRC-aided codes): d_msg uint8 [F][K - crc_width] (0/1),
 * d_u_info uint8 [F][K].  These are the targets of a loss on the decoder's
 * output LLRs at the information rows.                                      */
int polar_info_bits(const pc_code *code, const uint8_t *d_msg, uint8_t *d_u_info, int64_t F,
                    void *stream);

/* Standard min-sum BP decoding (Sec. II-B) of F frames.
 * d_llr float [F][N] channel LLRs (4-byte aligned, finite for defined
 * results); d_msg_hat uint8 [F][K - crc_width] decided message bits;
 * d_iters int32 [F] iterations run (the one that met the stop test counts),
 * or NULL; d_ok uint8 [F] verdict of the stop test on the final decisions
 * (for PC_STOP_NONE: the CRC if the code has one, else the G test), or NULL. */
int bp_decode(const pc_code *code, const float *d_llr, int64_t F, const pc_bp_params *bp,
              uint8_t *d_msg_hat, int32_t *d_iters, uint8_t *d_ok, void *stream);

/* Partially permuted multi-trellis BP (Algorithm 1 with the fixed schedules
 * of pc_pp_params).  Arguments as bp_decode.  The decode entry points enqueue
 * kernels only (the queue counters are reset by a kernel, no memset): after
 * one eager call on the device (which allocates the library's counters), a
 * call can be captured into a HIP graph and replayed with new data in the
 * same buffers.  A captured call keeps its own counters for good (at most
 * 1024 captured calls per device), so replays may overlap eager calls and
 * other graphs on other streams.                                           */
int pp_mt_bp_decode(const pc_code *code, const float *d_llr, int64_t F, const pc_bp_params *bp,
                    const pc_pp_params *pp, uint8_t *d_msg_hat, int32_t *d_iters, uint8_t *d_ok,
                    void *stream);

/* pp_mt_bp_decode with two extras: d_soft_u float [F][N] (or NULL) receives
 * the L messages on level n+1 after the final L sweep (the u-side soft output
 * before the prior is added), and cfg (or NULL) overrides the launch
 * configuration.                                                            */
int pp_mt_bp_decode_ex(const pc_code *code, const float *d_llr, int64_t F,
                       const pc_bp_params *bp, const pc_pp_params *pp, uint8_t *d_msg_hat,
                       int32_t *d_iters, uint8_t *d_ok, float *d_soft_u,
                       const pc_launch_cfg *cfg, void *stream);

/* Error classes of Sec. II-C.  The paper names three ways BP fails (after
 * the error classification it cites) and describes them in words only; this
 * library detects them from the history of the hard decisions.
 *
 * pp_mt_bp_decode_trace: pp_mt_bp_decode (any pp mode, or pp NULL for plain
 * BP) that also records, after every iteration it = 1, 2, ... of frame f,
 * the 64-bit hash of the decisions on level n+1 at d_hist[f*H + (it-1) % H]:
 * the xor, over the rows j decided 1, of key(j) = the first SplitMix64
 * output from state j.  d_hist uint64 [F][H], 8-byte aligned, 1 <= H <= 64;
 * entries of iterations a frame did not reach are left untouched.  Launch
 * shape: the library's default (two rows per thread).
 *
 * polar_classify_errors: for each frame, on the last W = min(H, iters[f])
 * recorded hashes h_1..h_W (oldest first), the decision period p is the
 * smallest p in 1..floor(W/2) with h_i = h_{i+p} for all i <= W-p, else 0
 * (d_period int32 [F], or NULL).  Class (d_class uint8 [F]): PC_ERR_CORRECT
 * if d_msg_hat equals d_msg (uint8 [F][K_msg] each); otherwise
 * PC_ERR_FALSE_CONVERGED if the stop test accepted the final decisions
 * (d_ok) or p = 1, PC_ERR_OSCILLATION if p >= 2, else PC_ERR_UNCONVERGED.
 * d_iters, d_ok as written by the decode call; the history must come from a
 * trace call with the same H.                                              */
#define PC_ERR_CORRECT 0
#define PC_ERR_FALSE_CONVERGED 1
#define PC_ERR_OSCILLATION 2
#define PC_ERR_UNCONVERGED 3
int pp_mt_bp_decode_trace(const pc_code *code, const float *d_llr, int64_t F, const pc_bp_params *bp,
                          const pc_pp_params *pp, uint8_t *d_msg_hat, int32_t *d_iters, uint8_t *d_ok,
                          uint64_t *d_hist, int32_t H, void *stream);
int polar_classify_errors(const uint8_t *d_msg_hat, const uint8_t *d_msg, const uint8_t *d_ok,
                          const int32_t *d_iters, const uint64_t *d_hist, int32_t H, int64_t F,
                          int32_t K_msg, uint8_t *d_class, int32_t *d_period, void *stream);

/* Batched decoding of frames of mixed length and rate in one persistent
 * launch fed from a device work queue.  codes[0..n_codes) (n_codes <= 32)
 * are codes built on this device, each with N in [64, 1024] and a CRC;
 * d_code_id int32 [F] selects each frame's code (a frame whose id is outside
 * 0..n_codes-1 is skipped and its outputs are left untouched); d_llr_off int64 [F] is the
 * float offset of frame f's N LLRs in d_llr_pool; d_bits_off int64 [F] the
 * byte offset of its K - crc_width decided bits in d_bits_pool.  d_iters
 * int32 [F] and d_ok uint8 [F] as in bp_decode, or NULL.  The stop test is
 * the CRC (or none); pp is NULL / PC_PP_NONE or PC_PP_LASTK with k = 4 (the
 * last 4 stages of every length), each length with its own pool drawn from
 * the same seed.  Frames are bucketed by length on the device and decoded
 * longest first; a slot whose frame stops takes the next frame of its
 * length from the queue.  d_ws: device workspace of at least
 * polar_batched_workspace_bytes(F) bytes; the call clears what it needs with
 * its own kernels (no memset), so after one warm-up call on the device the
 * whole call can be captured into a HIP graph and replayed with new frame
 * data in the same buffers.  Overlapping calls must use different workspaces.
 * cfg: rho (2 or 3: every length under that rho in one launch; 0: the
 * 512-bit frames under rho 3 in a launch of their own, then the other lengths
 * under rho 2), slots = 1 (256-thread workgroups) or 2 (512), grid (0 = as
 * many workgroups as fit, per launch); NULL for the defaults (rho 0).       */
size_t polar_batched_workspace_bytes(int64_t F);
int pp_mt_bp_decode_batched(const pc_code *const *codes, int32_t n_codes, const int32_t *d_code_id,
                            const int64_t *d_llr_off, const float *d_llr_pool, int64_t F,
                            const pc_bp_params *bp, const pc_pp_params *pp,
                            uint8_t *d_bits_pool, const int64_t *d_bits_off, int32_t *d_iters,
                            uint8_t *d_ok, void *d_ws, size_t ws_bytes,
                            const pc_launch_cfg *cfg, void *stream);

/* pp_mt_bp_decode_batched without a workspace argument and without any
 * allocation, for callers that cannot allocate device memory (code under
 * HIP graph capture without a warm-up call, serving loops, harnesses that
 * forbid hipMalloc).  The queue control words and frame list live in a
 * library-owned scratch of 4 MiB + 256 bytes per device (a static device
 * array, resolved once per device by polar_construct or by the first call),
 * so F may not exceed 1048576 (PC_EINVAL otherwise); the codes' device must
 * be current.  Every call on a device shares that device's scratch and
 * clears what it needs with its own kernels: calls that overlap on one
 * device (other streams, or graphs replayed beside each other) race and give
 * undefined results; serialise them.  Other arguments and results as
 * pp_mt_bp_decode_batched, whose kernels it runs.                          */
int pp_mt_bp_decode_batched_noalloc(const pc_code *const *codes, int32_t n_codes,
                                    const int32_t *d_code_id, const int64_t *d_llr_off,
                                    const float *d_llr_pool, int64_t F, const pc_bp_params *bp,
                                    const pc_pp_params *pp, uint8_t *d_bits_pool,
                                    const int64_t *d_bits_off, int32_t *d_iters, uint8_t *d_ok,
                                    const pc_launch_cfg *cfg, void *stream);

/* Weighted BP: the unrolled decoder with a learnable scale on every check-node
 * output, w[t][s-1][d][row] (iteration t, stage s, d = 0 L sweep / 1 R sweep,
 * output row), frozen prior 2^60, no early stop, T_unroll iterations; the
 * output LLR is o_j = L_{n+1,j} + R_{n+1,j} after the last L sweep.  With
 * pp != NULL and mode PC_PP_LASTK the fixed last-k schedule applies and the
 * weights are shared by all trellises (indexed by stage position).
 * d_w float [T_unroll][n][2][N]; d_out_llr float [F][N].  The forward pass
 * writes per-iteration message checkpoints to d_ws, which must hold
 * wbp_workspace_bytes(code, F, T_unroll) bytes, be 256-byte aligned (as
 * hipMalloc returns) and stay untouched until the matching wbp_backward.  d_ws = NULL with ws_bytes = 0 runs the forward pass
 * alone (inference): no checkpoints are written and no backward may follow.
 * The last two calls are graph-capturable (kernels only, no memset).       */
size_t wbp_workspace_bytes(const pc_code *code, int64_t F, int32_t T_unroll);
int wbp_forward(const pc_code *code, const float *d_llr, int64_t F, const float *d_w,
                int32_t T_unroll, const pc_pp_params *pp, float *d_out_llr, void *d_ws,
                size_t ws_bytes, void *stream);

/* Reverse mode of wbp_forward: given d_grad_out float [F][N] (d loss / d o),
 * writes d_grad_w float [T_unroll][n][2][N] = sum over frames of
 * d loss / d w.  The reduction over frames has a fixed order, so results are
 * reproducible run to run.  Same d_ws as the forward call.                  */
int wbp_backward(const pc_code *code, const float *d_llr, int64_t F, const float *d_w,
                 int32_t T_unroll, const pc_pp_params *pp, const float *d_grad_out,
                 float *d_grad_w, void *d_ws, size_t ws_bytes, void *stream);

/* Static description of a return code, and the thread-local detail of the
 * last failure on this thread.                                              */
const char *polar_strerror(int rc);
const char *polar_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* POLARBP_H */
