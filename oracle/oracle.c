/*
 * oracle.c -- plain, slow, obviously-correct CPU reference for partially
 * permuted multi-trellis belief-propagation (PP-MT-BP) decoding of polar codes
 * (Ranasinghe, Rajatheva, Latva-aho, arXiv 1911.08868).
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the
 * cpu_baseline leg of bench.py may load this library.  It shares no source,
 * header, table or helper with the GPU library; both are written from the
 * paper independently.
 *
 * Arithmetic.  Every floating-point value is held in a double.  In FP64 mode
 * each operation rounds once to double.  In FP32 mode every arithmetic result
 * is additionally rounded to float with rnd(); since 53 >= 2*24+2, an add or
 * multiply of two floats done in double and then rounded to float equals the
 * float operation exactly, so FP32 mode reproduces an IEEE single-precision
 * decoder bit for bit (no fused multiply-add anywhere; build with
 * -ffp-contract=off).
 *
 * Indexing.  The paper numbers factor-graph levels i = 1..n+1 with level 1
 * holding the channel LLRs L_{1,j} and level n+1 holding the a-priori values
 * R_{n+1,j} (Sec. II-B).  Here lev = i-1 runs 0..n.  Stage s = 1..n is the
 * column of N/2 processing elements between lev s-1 (channel side) and lev s
 * (u side).  In the original graph stage s pairs rows differing in bit s-1
 * (span 2^(s-1)), so stages 1..m form N/2^m disjoint blocks of 2^m rows, which
 * is the subgraph count of Sec. III.  A permuted graph assigns stage s the
 * bit order[s-1].
 *
 * Parity pins for every function live in tests/test_oracle_*.py.
 * Parity unpinned: or_decode's frame error rate against the paper's curves
 * (the figures are not available), and the FP32-vs-FP64 agreement beyond the
 * first iterations (min-selection flips are legitimate there).
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_ENOMEM (-4)

/* ------------------------------------------------------------------------ */
/* rounding helper: FP32 mode rounds every arithmetic result to float        */
static double rnd(int fp32, double x) { return fp32 ? (double)(float)x : x; }

static int ilog2_exact(int32_t N) {
    if (N < 2 || (N & (N - 1))) return -1;
    int n = 0;
    while ((1 << n) < N) n++;
    return n;
}

/* ------------------------------------------------------------------------ */
/* Code construction by Bhattacharyya parameters (Sec. II-A).
 *
 * The bit channels are those seen by successive cancellation on the same
 * factor graph the decoder uses.  With level 1 on the channel side and stage s
 * pairing rows 2^(s-1) apart, the stage next to u pairs rows N/2 apart, so the
 * last (u-side) combining step is on the most significant bit and the
 * successive-cancellation order of this graph is the bit-reversed index
 * order.  Bit channel i therefore follows from the channel parameter z0 by n
 * polarising steps, the step of the least significant bit first and that of
 * the most significant bit last: a bit equal to 0 takes the degraded channel
 * 2z - z^2, a bit equal to 1 the upgraded channel z^2 (exact on the binary
 * erasure channel, an upper bound otherwise).  For the binary-input AWGN
 * channel z0 = exp(-Es/N0) with Es/N0 = (K/N) * Eb/N0 (the rate counts CRC
 * bits, Sec. IV).  Values are kept as ln z so that nothing underflows at
 * N = 4096.  The K channels with the smallest z form the information set A
 * (ties go to the larger index); A is returned in ascending order.
 */
typedef struct {
    double lz;
    int32_t idx;
} lz_item;

static int cmp_lz(const void *a, const void *b) {
    const lz_item *x = (const lz_item *)a, *y = (const lz_item *)b;
    if (x->lz < y->lz) return -1;
    if (x->lz > y->lz) return 1;
    return (x->idx > y->idx) ? -1 : (x->idx < y->idx ? 1 : 0);
}
static int cmp_i32(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* ln z of every bit channel, starting from an arbitrary ln z0 */
int or_bhattacharyya(int32_t N, double lnz0, double *lnz) {
    int n = ilog2_exact(N);
    if (n < 0 || !lnz) return OR_EINVAL;
    for (int32_t i = 0; i < N; i++) {
        double lz = lnz0;
        for (int b = 0; b < n; b++) {
            if ((i >> b) & 1)
                lz = 2.0 * lz;                       /* z^2      */
            else
                lz = lz + log1p(-expm1(lz));         /* z(2 - z) */
        }
        lnz[i] = lz;
    }
    return OR_OK;
}

int or_construct(int32_t N, int32_t K, double design_ebn0_db, int32_t *info_idx,
                 uint8_t *frozen, double *lnz_out) {
    int n = ilog2_exact(N);
    if (n < 0 || K < 1 || K > N || !info_idx) return OR_EINVAL;
    double rate = (double)K / (double)N;
    double lnz0 = -rate * pow(10.0, design_ebn0_db / 10.0);
    lz_item *items = (lz_item *)malloc(sizeof(lz_item) * (size_t)N);
    double *lz = (double *)malloc(sizeof(double) * (size_t)N);
    if (!items || !lz) { free(items); free(lz); return OR_ENOMEM; }
    or_bhattacharyya(N, lnz0, lz);
    for (int32_t i = 0; i < N; i++) { items[i].lz = lz[i]; items[i].idx = i; }
    qsort(items, (size_t)N, sizeof(lz_item), cmp_lz);
    for (int32_t i = 0; i < K; i++) info_idx[i] = items[i].idx;
    qsort(info_idx, (size_t)K, sizeof(int32_t), cmp_i32);
    if (frozen) {
        for (int32_t i = 0; i < N; i++) frozen[i] = 1;
        for (int32_t i = 0; i < K; i++) frozen[info_idx[i]] = 0;
    }
    if (lnz_out) memcpy(lnz_out, lz, sizeof(double) * (size_t)N);
    free(items);
    free(lz);
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* CRC (Sec. I, Sec. IV: the decoders are CRC aided; the paper does not fix
 * the generator).  Bit-serial long division, most significant bit first,
 * register initialised to 0, no reflection, no final xor.  `poly` may carry
 * the x^width term or not; only its low `width` bits are used.             */
uint32_t or_crc_bits(const uint8_t *bits, int64_t nbits, int32_t width, uint32_t poly) {
    if (width <= 0 || width > 32) return 0;
    uint32_t mask = (width == 32) ? 0xFFFFFFFFu : ((1u << width) - 1u);
    uint32_t g = poly & mask;
    uint32_t reg = 0;
    for (int64_t i = 0; i < nbits; i++) {
        uint32_t top = (reg >> (width - 1)) & 1u;
        reg = (reg << 1) & mask;
        if (top ^ (uint32_t)(bits[i] & 1u)) reg ^= g;
    }
    return reg;
}

/* ------------------------------------------------------------------------ */
/* Polar transform x = u G_N, G_N = F^{(x)n}, F = [[1,0],[1,1]] (Eq. 1).
 * One XOR butterfly per bit position: v[j] ^= v[j + 2^b] for rows j whose bit
 * b is 0.  The n butterflies commute, so their order is immaterial.          */
void or_polar_transform(int32_t N, const uint8_t *u, uint8_t *x) {
    int n = ilog2_exact(N);
    memmove(x, u, (size_t)N);
    for (int b = 0; b < n; b++)
        for (int32_t j = 0; j < N; j++)
            if (!((j >> b) & 1)) x[j] ^= x[j | (1 << b)];
}

/* Place message + CRC on the information set (CRC bits last in A order,
 * most significant first), zeros on the frozen set, and encode.            */
int or_encode(int32_t N, int32_t K, const int32_t *info_idx, int32_t crc_width,
              uint32_t crc_poly, const uint8_t *msg, int64_t F, uint8_t *u_out,
              uint8_t *x_out) {
    if (ilog2_exact(N) < 0 || K < 1 || K > N || crc_width < 0 || crc_width >= K)
        return OR_EINVAL;
    int32_t km = K - crc_width;
    uint8_t *u = (uint8_t *)malloc((size_t)N);
    if (!u) return OR_ENOMEM;
    for (int64_t f = 0; f < F; f++) {
        const uint8_t *m = msg + f * km;
        memset(u, 0, (size_t)N);
        for (int32_t i = 0; i < km; i++) u[info_idx[i]] = m[i] & 1u;
        if (crc_width > 0) {
            uint32_t c = or_crc_bits(m, km, crc_width, crc_poly);
            for (int32_t t = 0; t < crc_width; t++)
                u[info_idx[km + t]] = (uint8_t)((c >> (crc_width - 1 - t)) & 1u);
        }
        if (u_out) memcpy(u_out + f * N, u, (size_t)N);
        if (x_out) or_polar_transform(N, u, x_out + f * N);
    }
    free(u);
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* SplitMix64 (Steele, Lea, Flood, OOPSLA 2014): add the golden-ratio
 * increment, then the two xor-shift-multiply mixing rounds.                 */
uint64_t or_splitmix64_next(uint64_t *state) {
    uint64_t z = (*state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* uniform integer in [0, m): high 32 bits scaled by m */
static uint32_t draw_below(uint64_t *st, uint32_t m) {
    uint64_t hi = or_splitmix64_next(st) >> 32;
    return (uint32_t)((hi * (uint64_t)m) >> 32);
}

static int64_t factorial_capped(int k, int64_t cap) {
    int64_t r = 1;
    for (int i = 2; i <= k; i++) {
        r *= i;
        if (r >= cap) return cap;
    }
    return r;
}

/* Pool of stage orders for the fixed multi-trellis modes.
 * Entry 0 is the original graph (stage s uses bit s-1).  Entries 1..Q-1 keep
 * stages 1..n-k and give the last k stages (n-k+1..n) a random,
 * non-identity order of the bits n-k..n-1, all entries distinct.  A
 * candidate is a Fisher-Yates shuffle of the identity, walking the position
 * from k-1 down to 1 and swapping it with a uniform position at or below it;
 * identity and repeats are drawn again.  k = n gives the full permutations of
 * multi-trellis BP with full permutations (Sec. II-D).  Returns the number of
 * entries written, min(Q, k!).                                              */
int or_trellis_pool(int32_t n, int32_t k, int32_t Q, uint64_t seed, int8_t *orders) {
    if (n < 1 || k < 0 || k > n || Q < 1 || !orders) return OR_EINVAL;
    int64_t qeff = factorial_capped(k, Q);
    if (qeff > Q) qeff = Q;
    uint64_t st = seed;
    for (int s = 0; s < n; s++) orders[s] = (int8_t)s;
    int8_t cand[64];
    for (int64_t q = 1; q < qeff; q++) {
        for (;;) {
            for (int i = 0; i < k; i++) cand[i] = (int8_t)(n - k + i);
            for (int i = k - 1; i >= 1; i--) {
                uint32_t j = draw_below(&st, (uint32_t)(i + 1));
                int8_t t = cand[i]; cand[i] = cand[j]; cand[j] = t;
            }
            int ident = 1;
            for (int i = 0; i < k; i++) if (cand[i] != n - k + i) ident = 0;
            if (ident) continue;
            int dup = 0;
            for (int64_t p = 1; p < q && !dup; p++) {
                int same = 1;
                for (int i = 0; i < k; i++)
                    if (orders[p * n + n - k + i] != cand[i]) { same = 0; break; }
                dup = same;
            }
            if (dup) continue;
            break;
        }
        for (int s = 0; s < n - k; s++) orders[q * n + s] = (int8_t)s;
        for (int i = 0; i < k; i++) orders[q * n + n - k + i] = cand[i];
    }
    return (int)qeff;
}

/* ------------------------------------------------------------------------ */
/* Check node functions (Sec. II-B).
 * Min-sum: sign(x) sign(y) min(|x|,|y|), optionally scaled by alpha; the sign
 * is the xor of the two sign bits (so signed zeros follow IEEE sign bits) and
 * the only rounding is that of the scale.
 * Exact boxplus: 2 atanh(tanh(x/2) tanh(y/2)), FP64 only, evaluated as
 * sgn(x) sgn(y) min(|x|,|y|) + ln(1 + e^-(|x|+|y|)) - ln(1 + e^-||x|-|y||),
 * the same function written so that it neither saturates nor loses digits
 * when both tanh factors round to 1 (for a <= b, both forms equal
 * ln((1 + e^(a+b)) / (e^a + e^b)) on the magnitudes).  A rounding that takes
 * the magnitude below 0 gives 0; infinite magnitudes enter as the limits
 * (inf against y gives y, inf against inf gives inf).                      */
static double minsum(double x, double y, double alpha, int fp32) {
    double m = fmin(fabs(x), fabs(y));
    if (alpha != 1.0) m = rnd(fp32, alpha * m);
    int neg = (signbit(x) != 0) != (signbit(y) != 0);
    return neg ? -m : m;
}

static double boxplus_exact(double x, double y) {
    double ax = fabs(x), ay = fabs(y);
    double m = fmin(ax, ay);
    double d = (ax == ay) ? 0.0 : fabs(ax - ay); /* inf - inf: equal magnitudes */
    double mag = m + log1p(exp(-(ax + ay))) - log1p(exp(-d));
    if (!(mag > 0.0)) mag = 0.0;
    int neg = (signbit(x) != 0) != (signbit(y) != 0);
    return neg ? -mag : mag;
}

/* ------------------------------------------------------------------------ */
/* Decoder parameters (Algorithm 1's inputs plus the fixed multi-trellis
 * schedules).  pp_mode: -1 plain BP; 0 fixed last-k partial permutation with
 * a pool of Q orders cycled every T iterations; 1 full permutation
 * (multi-trellis BP with full permutations; k is forced to n); 2 Algorithm 1
 * (random subgraph per event, Eq. 2 reset schedule).                        */
typedef struct {
    int32_t max_iter;
    double alpha;
    int32_t stop;      /* 0 none, 1 G-matrix, 2 CRC */
    int32_t it_min;    /* stop test only from this iteration on */
    int32_t pp_mode;
    int32_t k, T, Q;
    int32_t P_range, P_level, D, N_min, first_reset;
    uint64_t seed;
    int32_t fp32;
    int32_t exact_boxplus;
    float noise_sigma; /* > 0: noise injected at the trellis events (modes 0, 1, 2) */
} or_params;

typedef struct {
    int32_t N, n, K, crc_width;
    uint32_t crc_poly;
    const int32_t *info_idx;
    uint8_t *frozen; /* N */
} code_t;

/* hard decision (Sec. II-B): bit 0 iff R + L >= 0 */
static uint8_t hard(double l, double r, int fp32) { return rnd(fp32, l + r) < 0.0 ? 1 : 0; }

/* stop test on the current state: CRC of the message part of u_hat equals its
 * CRC part; or, for the G-matrix test, u_hat G_N equals the hard decision on
 * the channel level.                                                         */
static int check_crc(const code_t *c, const double *Lu, const double *Ru, int fp32,
                     uint8_t *scratch) {
    if (c->crc_width <= 0) return 0;
    int32_t km = c->K - c->crc_width;
    for (int32_t i = 0; i < c->K; i++) {
        int32_t j = c->info_idx[i];
        scratch[i] = hard(Lu[j], Ru[j], fp32);
    }
    uint32_t crc = or_crc_bits(scratch, km, c->crc_width, c->crc_poly);
    uint32_t got = 0;
    for (int32_t t = 0; t < c->crc_width; t++) got = (got << 1) | scratch[km + t];
    return crc == got;
}

static int check_g(const code_t *c, const double *Lu, const double *Ru, const double *L0,
                   const double *R0, int fp32, uint8_t *scratch) {
    int32_t N = c->N;
    uint8_t *u = scratch, *x = scratch + N;
    for (int32_t j = 0; j < N; j++) u[j] = hard(Lu[j], Ru[j], fp32);
    or_polar_transform(N, u, x);
    for (int32_t j = 0; j < N; j++)
        if (x[j] != hard(L0[j], R0[j], fp32)) return 0;
    return 1;
}

/* Noise injection at the trellis events.  The paper leaves "noise injection
 * along with partial permutations" to future work (Sec. V) and compares with
 * noise-aided BP at sigma^2 = 0.36 (Table I); the reading used here: at every
 * event of the fixed schedules (after iterations T, 2T, ...; also when the
 * pool has one entry and the graph stays) the channel level is set to
 * y_j + sigma g(frame, e, j), e = it / T, with fresh noise per event and the
 * received LLR y_j.  Algorithm 1 does the same at each of its events (Sec. III,
 * spaced by Eq. 2), after the partial permutation, with e = 1, 2, ... counting
 * the frame's events (an event whose draws all fail counts too).  g is an Irwin-Hall approximation of N(0,1): the sum of
 * the twelve 16-bit fields of three SplitMix64 outputs, each field k read as
 * the uniform (k + 1/2) / 2^16, minus 6.  The generator starts from the state
 * seed ^ frame * 0x9E3779B97F4A7C15 ^ e * 0xC2B2AE3D27D4EB4F
 * ^ j * 0x165667B19E3779F9.  Every g is a multiple of 2^-16 in (-6, 6), exact
 * in single precision.                                                     */
float or_noise_gauss(uint64_t seed, int64_t frame, int32_t e, int32_t j) {
    uint64_t st = seed ^ ((uint64_t)frame * 0x9E3779B97F4A7C15ull) ^
                  ((uint64_t)(uint32_t)e * 0xC2B2AE3D27D4EB4Full) ^
                  ((uint64_t)(uint32_t)j * 0x165667B19E3779F9ull);
    int64_t sum = 0;
    for (int i = 0; i < 3; i++) {
        uint64_t o = or_splitmix64_next(&st);
        for (int k = 0; k < 4; k++) sum += (int64_t)((o >> (16 * k)) & 0xFFFFu);
    }
    return (float)((double)(sum + 6) / 65536.0 - 6.0);
}

/* Decision history for the error classes of Sec. II-C.  After every
 * iteration the hard decisions on level n+1 are summarised by a 64-bit
 * Zobrist hash: the xor, over the rows j whose decision is 1, of key(j), the
 * first SplitMix64 output from state j.  Equal decision vectors give equal
 * hashes; two different ones collide with probability about 2^-64.        */
static uint64_t decision_key(int32_t j) {
    uint64_t st = (uint64_t)j;
    return or_splitmix64_next(&st);
}

static uint64_t decision_hash(const code_t *c, const double *Lu, const double *Ru, int fp32) {
    uint64_t h = 0;
    for (int32_t j = 0; j < c->N; j++)
        if (hard(Lu[j], Ru[j], fp32)) h ^= decision_key(j);
    return h;
}

/* One processing element (Sec. II-B, the four PE equations).  Top row j has
 * bit b = 0, bottom row jp = j | 2^b.  *_in,1 belong to the top row and
 * *_in,2 to the bottom row; L messages arrive from the channel side (lev s-1),
 * R messages from the u side (lev s).                                        */
typedef struct {
    double alpha;
    int fp32, exact;
} arith_t;

static double cn(const arith_t *a, double x, double y) {
    return a->exact ? boxplus_exact(x, y) : minsum(x, y, a->alpha, a->fp32);
}

/* L sweep at stage s (1..n) on bit b, restricted to rows [r0, r1) */
static void stage_L(const arith_t *a, int32_t N, double *L, double *R, int s, int b,
                    int32_t r0, int32_t r1) {
    double *Lin = L + (size_t)(s - 1) * N, *Lout = L + (size_t)s * N;
    const double *Rin = R + (size_t)s * N;
    for (int32_t j = r0; j < r1; j++) {
        if ((j >> b) & 1) continue;
        int32_t jp = j | (1 << b);
        double l1 = Lin[j], l2 = Lin[jp], r1v = Rin[j], r2v = Rin[jp];
        Lout[j] = cn(a, l1, rnd(a->fp32, l2 + r2v));
        Lout[jp] = rnd(a->fp32, cn(a, r1v, l1) + l2);
    }
}

/* R sweep at stage s on bit b */
static void stage_R(const arith_t *a, int32_t N, double *L, double *R, int s, int b,
                    int32_t r0, int32_t r1) {
    const double *Lin = L + (size_t)(s - 1) * N;
    const double *Rin = R + (size_t)s * N;
    double *Rout = R + (size_t)(s - 1) * N;
    for (int32_t j = r0; j < r1; j++) {
        if ((j >> b) & 1) continue;
        int32_t jp = j | (1 << b);
        double l1 = Lin[j], l2 = Lin[jp], r1v = Rin[j], r2v = Rin[jp];
        Rout[j] = cn(a, r1v, rnd(a->fp32, l2 + r2v));
        Rout[jp] = rnd(a->fp32, cn(a, r1v, l1) + r2v);
    }
}

/* Schedule of the current factor graph.  For the fixed modes every row block
 * shares one order; Algorithm 1 keeps a per-row order (row j's stage s uses
 * bit ord[j*n + s-1]) because it permutes one subgraph at a time.           */
typedef struct {
    int n;
    int8_t *ord; /* N*n */
} sched_t;

/* One BP iteration (Algorithm 1, oneBPiteration): the L sweep over stages 1..n
 * followed by the R sweep over stages n..1, each PE reading the freshest
 * messages.  The stage loop visits every row j once and applies the PE only
 * when j is the top row of its pair for that row's bit.                      */
static void one_iteration(const arith_t *a, int32_t N, const sched_t *sc, double *L,
                          double *R) {
    int n = sc->n;
    for (int s = 1; s <= n; s++) {
        double *Lin = L + (size_t)(s - 1) * N, *Lout = L + (size_t)s * N;
        const double *Rin = R + (size_t)s * N;
        for (int32_t j = 0; j < N; j++) {
            int b = sc->ord[(size_t)j * n + s - 1];
            if ((j >> b) & 1) continue;
            int32_t jp = j | (1 << b);
            double l1 = Lin[j], l2 = Lin[jp], r1v = Rin[j], r2v = Rin[jp];
            Lout[j] = cn(a, l1, rnd(a->fp32, l2 + r2v));
            Lout[jp] = rnd(a->fp32, cn(a, r1v, l1) + l2);
        }
    }
    for (int s = n; s >= 1; s--) {
        const double *Lin = L + (size_t)(s - 1) * N;
        const double *Rin = R + (size_t)s * N;
        double *Rout = R + (size_t)(s - 1) * N;
        for (int32_t j = 0; j < N; j++) {
            int b = sc->ord[(size_t)j * n + s - 1];
            if ((j >> b) & 1) continue;
            int32_t jp = j | (1 << b);
            double l1 = Lin[j], l2 = Lin[jp], r1v = Rin[j], r2v = Rin[jp];
            Rout[j] = cn(a, r1v, rnd(a->fp32, l2 + r2v));
            Rout[jp] = rnd(a->fp32, cn(a, r1v, l1) + r2v);
        }
    }
    (void)stage_L;
    (void)stage_R;
}

static void set_uniform_order(sched_t *sc, int32_t N, const int8_t *order) {
    for (int32_t j = 0; j < N; j++) memcpy(sc->ord + (size_t)j * sc->n, order, (size_t)sc->n);
}

/* zero L and R on levels lev_lo..lev_hi (inclusive) of rows [r0, r1) */
static void zero_levels(int32_t N, double *L, double *R, int lev_lo, int lev_hi, int32_t r0,
                        int32_t r1) {
    for (int lev = lev_lo; lev <= lev_hi; lev++)
        for (int32_t j = r0; j < r1; j++) {
            L[(size_t)lev * N + j] = 0.0;
            R[(size_t)lev * N + j] = 0.0;
        }
}

/* ------------------------------------------------------------------------ */
/* Algorithm 1 partial permutation on the current graph.
 *
 * rho_range is uniform on {2..P_range}; x uniform on {1..P_level};
 * rho_level = min(x, n - rho_range + 1); m = rho_level + rho_range - 1.  The
 * subgraph is one of the N/2^m connected blocks of stages 1..m, chosen
 * uniformly, and stages rho_level..m inside it receive a new order of the bits
 * they carry.  The reading taken for "a subgraph of the previous factor graph"
 * keeps the graph a valid representation of x = u G_N: in the current graph a
 * block is the connected component of stages 1..m containing a row, and a
 * draw is accepted only when each of the stages rho_level..m uses a single bit
 * across that component; otherwise the event is drawn again (at most 64
 * times, after which the event is skipped).  Nodes on the levels strictly
 * between the permuted stages (paper levels rho_level+1..m) of the block are
 * reset to 0.  N_zero = 2^m (rho_range - 1) and the next reset point follows
 * Eq. 2: iter + max(N_min, floor(N_zero / D)).                               */
/* label the connected components of stages 1..m of the current graph, in
 * the order of their smallest row; returns the number of components        */
static int32_t label_components(const sched_t *sc, int32_t N, int m, int32_t *label,
                                int32_t *queue) {
    int n = sc->n;
    for (int32_t j = 0; j < N; j++) label[j] = -1;
    int32_t nl = 0;
    for (int32_t r = 0; r < N; r++) {
        if (label[r] >= 0) continue;
        int32_t head = 0, tail = 0;
        queue[tail++] = r;
        label[r] = nl;
        while (head < tail) {
            int32_t j = queue[head++];
            for (int s = 1; s <= m; s++) {
                int32_t p = j ^ (1 << sc->ord[(size_t)j * n + s - 1]);
                if (label[p] < 0) { label[p] = nl; queue[tail++] = p; }
            }
        }
        nl++;
    }
    return nl;
}

/* draw (or NULL) receives the accepted draw: rho_range, x, m, the block and
 * the new bits of stages rho_level..m, for the pins of the draw distributions */
static int alg1_event(const sched_t *sc, int32_t N, double *L, double *R, uint64_t *st,
                      int32_t P_range, int32_t P_level, int32_t *n_zero, int32_t *label,
                      int32_t *queue, int32_t *draw) {
    int n = sc->n;
    for (int attempt = 0; attempt < 64; attempt++) {
        int rr = 2 + (int)draw_below(st, (uint32_t)(P_range - 1));
        int x = 1 + (int)draw_below(st, (uint32_t)P_level);
        int rl = x < (n - rr + 1) ? x : (n - rr + 1);
        int m = rl + rr - 1;
        int32_t nblocks = N >> m;
        int32_t blk = (int32_t)draw_below(st, (uint32_t)nblocks);
        int32_t nl = label_components(sc, N, m, label, queue);
        if (nl != nblocks) continue;
        int32_t cnt = 0;
        for (int32_t j = 0; j < N; j++) if (label[j] == blk) queue[cnt++] = j;
        if (cnt != (1 << m)) continue;
        /* each stage rl..m must carry one bit over the component */
        int8_t bits[64];
        int uniform = 1;
        for (int s = rl; s <= m && uniform; s++) {
            int b0 = sc->ord[(size_t)queue[0] * n + s - 1];
            for (int32_t t = 1; t < cnt; t++)
                if (sc->ord[(size_t)queue[t] * n + s - 1] != b0) { uniform = 0; break; }
            bits[s - rl] = (int8_t)b0;
        }
        if (!uniform) continue;
        /* new non-identity order of those bits */
        int8_t cand[64];
        int ident;
        do {
            for (int i = 0; i < rr; i++) cand[i] = bits[i];
            for (int i = rr - 1; i >= 1; i--) {
                uint32_t j = draw_below(st, (uint32_t)(i + 1));
                int8_t t = cand[i]; cand[i] = cand[j]; cand[j] = t;
            }
            ident = 1;
            for (int i = 0; i < rr; i++) if (cand[i] != bits[i]) ident = 0;
        } while (ident);
        for (int32_t t = 0; t < cnt; t++) {
            int32_t j = queue[t];
            for (int i = 0; i < rr; i++) sc->ord[(size_t)j * n + rl - 1 + i] = cand[i];
            for (int lev = rl; lev <= m - 1; lev++) {
                L[(size_t)lev * N + j] = 0.0;
                R[(size_t)lev * N + j] = 0.0;
            }
        }
        *n_zero = (1 << m) * (rr - 1);
        if (draw) {
            draw[0] = rr;
            draw[1] = x;
            draw[2] = m;
            draw[3] = blk;
            for (int i = 0; i < rr; i++) draw[4 + i] = cand[i];
        }
        return 1;
    }
    *n_zero = 0;
    if (draw) draw[0] = 0;
    return 0;
}

/* The alternative reading of "a subgraph of the previous factor graph is
 * permuted" (R2): every event permutes one block of the ORIGINAL graph.  The
 * draws are those of alg1_event (rho_range, x, the block among the N/2^m
 * contiguous blocks of 2^m rows, then a non-identity order of the bits of
 * stages rho_level..m, drawn from the original bits rho_level-1..m-1); the
 * block of the previous event first returns to the original order with its
 * inner levels reset, then the new block is re-ordered with its inner levels
 * reset.  Every graph is the original one with one block re-ordered, so it
 * stays a valid representation of u G_N and no draw is rejected.  N_zero is
 * the number of (level, row) nodes reset by the event, each counted once.
 * prev[0..2]: rho_level, m and first row of the block that is re-ordered now
 * (prev[1] = 0: none); updated.  mark: N ints of scratch.                    */
static int alg1_event_r2(const sched_t *sc, int32_t N, double *L, double *R, uint64_t *st,
                         int32_t P_range, int32_t P_level, int32_t *n_zero, int32_t *prev,
                         int32_t *mark) {
    int n = sc->n;
    int rr = 2 + (int)draw_below(st, (uint32_t)(P_range - 1));
    int x = 1 + (int)draw_below(st, (uint32_t)P_level);
    int rl = x < (n - rr + 1) ? x : (n - rr + 1);
    int m = rl + rr - 1;
    int32_t blk = (int32_t)draw_below(st, (uint32_t)(N >> m));
    int8_t cand[64];
    int ident;
    do {
        for (int i = 0; i < rr; i++) cand[i] = (int8_t)(rl - 1 + i);
        for (int i = rr - 1; i >= 1; i--) {
            uint32_t j = draw_below(st, (uint32_t)(i + 1));
            int8_t t = cand[i]; cand[i] = cand[j]; cand[j] = t;
        }
        ident = 1;
        for (int i = 0; i < rr; i++) if (cand[i] != rl - 1 + i) ident = 0;
    } while (ident);
    /* the nodes reset, as a bit mask of levels per row (n <= 30) */
    for (int32_t j = 0; j < N; j++) mark[j] = 0;
    if (prev[1] > 0) {
        int prl = prev[0], pm = prev[1];
        for (int32_t j = prev[2]; j < prev[2] + (1 << pm); j++) {
            for (int s = prl; s <= pm; s++) sc->ord[(size_t)j * n + s - 1] = (int8_t)(s - 1);
            for (int lev = prl; lev <= pm - 1; lev++) {
                L[(size_t)lev * N + j] = 0.0;
                R[(size_t)lev * N + j] = 0.0;
                mark[j] |= 1 << lev;
            }
        }
    }
    int32_t r0 = blk << m;
    for (int32_t j = r0; j < r0 + (1 << m); j++) {
        for (int i = 0; i < rr; i++) sc->ord[(size_t)j * n + rl - 1 + i] = cand[i];
        for (int lev = rl; lev <= m - 1; lev++) {
            L[(size_t)lev * N + j] = 0.0;
            R[(size_t)lev * N + j] = 0.0;
            mark[j] |= 1 << lev;
        }
    }
    int32_t nz = 0;
    for (int32_t j = 0; j < N; j++) nz += __builtin_popcount((unsigned)mark[j]);
    *n_zero = nz;
    prev[0] = rl;
    prev[1] = m;
    prev[2] = r0;
    return 1;
}

/* initializeIterationResetValue(N): the paper does not give it.  Reading:
 * the reset value a full permutation would get from Eq. 2 (N_zero = N(n-1)),
 * capped at half of N_it,max.                                                */
static int32_t alg1_first_reset(int32_t N, int n, const or_params *p) {
    if (p->first_reset > 0) return p->first_reset;
    int32_t full = p->D > 0 ? (N * (n - 1)) / p->D : 0;
    int32_t v = full > p->N_min ? full : p->N_min;
    int32_t half = p->max_iter / 2;
    return v < half ? v : half;
}

/* ------------------------------------------------------------------------ */
/* Decoding one frame (Algorithm 1 and its fixed-schedule special cases).   */
typedef struct {
    const code_t *c;
    const or_params *p;
    const int8_t *pool;
    int32_t pool_q;
    const float *llr;
    int64_t f0, f1;
    uint8_t *msg_hat;
    int32_t *iters;
    uint8_t *ok;
    double *soft_u;
    double *state;
    uint64_t *hist; /* [F][H] decision hashes, or NULL */
    int32_t H;
    int rc;
} job_t;

/* the channel level after the noise injection of event e */
static void inject_noise(const or_params *p, const float *y, int64_t f, int32_t e, int32_t N, double *L) {
    for (int32_t j = 0; j < N; j++) {
        double g = (double)or_noise_gauss(p->seed, f, e, j);
        L[j] = rnd(p->fp32, (double)y[j] + rnd(p->fp32, (double)p->noise_sigma * g));
    }
}

static void decode_frames(job_t *jb) {
    const code_t *c = jb->c;
    const or_params *p = jb->p;
    int32_t N = c->N, n = c->n;
    size_t lvl = (size_t)(n + 1) * N;
    double *L = (double *)malloc(sizeof(double) * lvl);
    double *R = (double *)malloc(sizeof(double) * lvl);
    uint8_t *scratch = (uint8_t *)malloc((size_t)(2 * N + c->K + 8));
    int8_t *ord = (int8_t *)malloc((size_t)N * n);
    int32_t *rows = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
    int32_t *mark = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
    if (!L || !R || !scratch || !ord || !rows || !mark) {
        jb->rc = OR_ENOMEM;
        goto out;
    }
    arith_t ar = {p->alpha, p->fp32, p->exact_boxplus};
    sched_t sc = {n, ord};
    int32_t km = c->K - c->crc_width;
    for (int64_t f = jb->f0; f < jb->f1; f++) {
        /* initializeLandR (Sec. II-B): channel LLRs on level 1, priors on level
         * n+1 (0 for information bits, +inf for frozen bits), 0 elsewhere.   */
        for (size_t t = 0; t < lvl; t++) { L[t] = 0.0; R[t] = 0.0; }
        for (int32_t j = 0; j < N; j++) L[j] = (double)jb->llr[f * N + j];
        for (int32_t j = 0; j < N; j++) R[(size_t)n * N + j] = c->frozen[j] ? INFINITY : 0.0;
        int32_t cur_q = 0;
        set_uniform_order(&sc, N, jb->pool);
        uint64_t st = p->seed + (uint64_t)(f + 1) * 0x9E3779B97F4A7C15ull;
        int32_t next_reset = (p->pp_mode == 2 || p->pp_mode == 3) ? alg1_first_reset(N, n, p) : 0;
        int32_t prev_blk[3] = {0, 0, 0};
        int32_t it_done = p->max_iter;
        int32_t events = 0;
        int okv = 0;
        for (int32_t it = 1; it <= p->max_iter; it++) {
            one_iteration(&ar, N, &sc, L, R);
            if (jb->hist)
                jb->hist[f * jb->H + (it - 1) % jb->H] =
                    decision_hash(c, L + (size_t)n * N, R + (size_t)n * N, p->fp32);
            if (p->stop != 0 && it >= p->it_min) {
                int pass = (p->stop == 2)
                               ? check_crc(c, L + (size_t)n * N, R + (size_t)n * N, p->fp32, scratch)
                               : check_g(c, L + (size_t)n * N, R + (size_t)n * N, L, R, p->fp32,
                                         scratch);
                if (pass) { it_done = it; okv = 1; break; }
            }
            if (it == p->max_iter) break;
            if ((p->pp_mode == 0 || p->pp_mode == 1) && it % p->T == 0) {
                int32_t q = (it / p->T) % jb->pool_q;
                if (jb->pool_q > 1 && q != cur_q) {
                    int kk = (p->pp_mode == 1) ? n : p->k;
                    set_uniform_order(&sc, N, jb->pool + (size_t)q * n);
                    /* the levels between the re-ordered stages lose meaning */
                    if (kk >= 2) zero_levels(N, L, R, n - kk + 1, n - 1, 0, N);
                    cur_q = q;
                }
                /* fresh channel noise on the received LLRs */
                if (p->noise_sigma > 0.0f) inject_noise(p, jb->llr + f * N, f, it / p->T, N, L);
            } else if ((p->pp_mode == 2 || p->pp_mode == 3) && it == next_reset) {
                int32_t nz = 0;
                if (p->pp_mode == 2)
                    alg1_event(&sc, N, L, R, &st, p->P_range, p->P_level, &nz, rows, mark, NULL);
                else
                    alg1_event_r2(&sc, N, L, R, &st, p->P_range, p->P_level, &nz, prev_blk, mark);
                int32_t add = p->D > 0 ? nz / p->D : 0;
                if (add < p->N_min) add = p->N_min;
                next_reset = it + add;
                events++;
                if (p->noise_sigma > 0.0f) inject_noise(p, jb->llr + f * N, f, events, N, L);
            }
        }
        if (p->stop == 0 || !okv) {
            /* final verdict of the configured test on the final state */
            if (p->stop == 1 || (p->stop == 0 && c->crc_width == 0))
                okv = check_g(c, L + (size_t)n * N, R + (size_t)n * N, L, R, p->fp32, scratch);
            else
                okv = check_crc(c, L + (size_t)n * N, R + (size_t)n * N, p->fp32, scratch);
        }
        /* hardDecision on the information set, message part only */
        for (int32_t i = 0; i < km; i++) {
            int32_t j = c->info_idx[i];
            jb->msg_hat[f * km + i] = hard(L[(size_t)n * N + j], R[(size_t)n * N + j], p->fp32);
        }
        if (jb->iters) jb->iters[f] = it_done;
        if (jb->ok) jb->ok[f] = (uint8_t)okv;
        if (jb->soft_u)
            for (int32_t j = 0; j < N; j++) jb->soft_u[f * N + j] = L[(size_t)n * N + j];
        if (jb->state) {
            memcpy(jb->state + (size_t)f * 2 * lvl, L, sizeof(double) * lvl);
            memcpy(jb->state + (size_t)f * 2 * lvl + lvl, R, sizeof(double) * lvl);
        }
    }
    jb->rc = OR_OK;
out:
    free(L); free(R); free(scratch); free(ord); free(rows); free(mark);
}

static void *decode_thread(void *arg) {
    decode_frames((job_t *)arg);
    return NULL;
}

/* Decode F frames.  llr: [F][N] float; msg_hat: [F][K - crc_width];
 * iters, ok: [F] or NULL; soft_u: [F][N] L messages at level n+1 after the
 * final L sweep, or NULL; state: [F][2][n+1][N] final L then R, or NULL;
 * hist: [F][H] decision hashes, the one after iteration it (1-based) at
 * (it - 1) mod H, or NULL (1 <= H <= 64).
 * The frames are split into contiguous chunks over nthreads threads.        */
static int decode_impl(int32_t N, int32_t K, const int32_t *info_idx, int32_t crc_width,
                       uint32_t crc_poly, const float *llr, int64_t F, const or_params *p,
                       uint8_t *msg_hat, int32_t *iters, uint8_t *ok, double *soft_u,
                       double *state, uint64_t *hist, int32_t H, int32_t nthreads) {
    int n = ilog2_exact(N);
    if (hist && (H < 1 || H > 64)) return OR_EINVAL;
    if (n < 0 || K < 1 || K > N || !info_idx || !p || !msg_hat || (F > 0 && !llr)) return OR_EINVAL;
    if (crc_width < 0 || crc_width >= K || p->max_iter < 1) return OR_EINVAL;
    if (p->stop == 2 && crc_width == 0) return OR_EINVAL;
    if (p->pp_mode == 0 && (p->k < 2 || p->k > n)) return OR_EINVAL;
    if ((p->pp_mode == 0 || p->pp_mode == 1) && (p->T < 1 || p->Q < 1)) return OR_EINVAL;
    if ((p->pp_mode == 2 || p->pp_mode == 3) &&
        (p->P_range < 2 || p->P_range > n || p->P_level < 1 || p->P_level > n - 1 || p->N_min < 1))
        return OR_EINVAL;
    if (p->exact_boxplus && p->fp32) return OR_EINVAL;
    if (!(p->noise_sigma >= 0.0f) || (p->noise_sigma > 0.0f && p->pp_mode != 0 && p->pp_mode != 1 &&
                                      p->pp_mode != 2 && p->pp_mode != 3))
        return OR_EINVAL;
    if (F == 0) return OR_OK;
    code_t c = {N, n, K, crc_width, crc_poly, info_idx, NULL};
    c.frozen = (uint8_t *)malloc((size_t)N);
    int8_t *pool = (int8_t *)malloc((size_t)(p->Q > 0 ? p->Q : 1) * n);
    if (!c.frozen || !pool) { free(c.frozen); free(pool); return OR_ENOMEM; }
    for (int32_t j = 0; j < N; j++) c.frozen[j] = 1;
    for (int32_t i = 0; i < K; i++) c.frozen[info_idx[i]] = 0;
    int32_t pool_q = 1;
    if (p->pp_mode == 0 || p->pp_mode == 1)
        pool_q = or_trellis_pool(n, p->pp_mode == 1 ? n : p->k, p->Q, p->seed, pool);
    else
        for (int s = 0; s < n; s++) pool[s] = (int8_t)s;
    if (nthreads < 1) nthreads = 1;
    if ((int64_t)nthreads > F) nthreads = (int32_t)F;
    job_t *jobs = (job_t *)calloc((size_t)nthreads, sizeof(job_t));
    pthread_t *th = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
    int rc = OR_OK;
    if (!jobs || !th) { rc = OR_ENOMEM; goto done; }
    for (int t = 0; t < nthreads; t++) {
        job_t *jb = &jobs[t];
        jb->c = &c; jb->p = p; jb->pool = pool; jb->pool_q = pool_q; jb->llr = llr;
        jb->f0 = F * t / nthreads; jb->f1 = F * (t + 1) / nthreads;
        jb->msg_hat = msg_hat; jb->iters = iters; jb->ok = ok; jb->soft_u = soft_u;
        jb->state = state;
        jb->hist = hist;
        jb->H = H;
    }
    if (nthreads == 1) {
        decode_frames(&jobs[0]);
    } else {
        for (int t = 0; t < nthreads; t++) pthread_create(&th[t], NULL, decode_thread, &jobs[t]);
        for (int t = 0; t < nthreads; t++) pthread_join(th[t], NULL);
    }
    for (int t = 0; t < nthreads; t++) if (jobs[t].rc != OR_OK) rc = jobs[t].rc;
done:
    free(jobs); free(th); free(c.frozen); free(pool);
    return rc;
}

int or_decode(int32_t N, int32_t K, const int32_t *info_idx, int32_t crc_width,
              uint32_t crc_poly, const float *llr, int64_t F, const or_params *p,
              uint8_t *msg_hat, int32_t *iters, uint8_t *ok, double *soft_u,
              double *state, int32_t nthreads) {
    return decode_impl(N, K, info_idx, crc_width, crc_poly, llr, F, p, msg_hat, iters, ok, soft_u,
                       state, NULL, 0, nthreads);
}

int or_decode_trace(int32_t N, int32_t K, const int32_t *info_idx, int32_t crc_width,
                    uint32_t crc_poly, const float *llr, int64_t F, const or_params *p,
                    uint8_t *msg_hat, int32_t *iters, uint8_t *ok, uint64_t *hist, int32_t H,
                    int32_t nthreads) {
    if (F > 0 && !hist) return OR_EINVAL;
    return decode_impl(N, K, info_idx, crc_width, crc_poly, llr, F, p, msg_hat, iters, ok, NULL,
                       NULL, hist, H, nthreads);
}

uint64_t or_decision_key(int32_t j) { return decision_key(j); }

/* Error classes of Sec. II-C for decoded frames, given the transmitted
 * messages.  The paper describes the three kinds of failure in words only:
 * a decoder that settles on a wrong word (false converged), one whose
 * decisions cycle between words (oscillation), and one that does neither
 * (unconverged).  Reading used here, on the last W = min(H, iters) decision
 * hashes h_1..h_W of a frame (oldest first):
 *   period p = the smallest p in 1..floor(W/2) with h_i = h_{i+p} for every
 *   i in 1..W-p, or 0 if there is none;
 *   class 0 (correct): the decided message equals the transmitted one;
 *   class 1 (false converged): wrong, and the stop test accepted the final
 *   decisions (ok) or they are stationary (p = 1);
 *   class 2 (oscillation): wrong, not accepted, p >= 2;
 *   class 3 (unconverged): wrong, not accepted, p = 0.
 * msg_hat, msg: [F][K_msg]; ok: [F]; iters: [F] (>= 1); hist: [F][H] as
 * written by or_decode_trace; cls: [F]; period: [F] or NULL.                 */
int or_classify(int64_t F, int32_t K_msg, const uint8_t *msg_hat, const uint8_t *msg,
                const uint8_t *ok, const int32_t *iters, const uint64_t *hist, int32_t H,
                uint8_t *cls, int32_t *period) {
    if (F < 0 || K_msg < 1 || H < 1 || H > 64) return OR_EINVAL;
    if (F > 0 && (!msg_hat || !msg || !ok || !iters || !hist || !cls)) return OR_EINVAL;
    for (int64_t f = 0; f < F; f++) {
        int wrong = 0;
        for (int32_t i = 0; i < K_msg; i++)
            if (msg_hat[f * K_msg + i] != msg[f * K_msg + i]) wrong = 1;
        int32_t it = iters[f];
        int32_t W = it < H ? it : H;
        uint64_t seq[64];
        for (int32_t i = 0; i < W; i++) seq[i] = hist[f * H + (it - W + i) % H];
        int32_t per = 0;
        for (int32_t p = 1; 2 * p <= W && per == 0; p++) {
            int match = 1;
            for (int32_t i = 0; i + p < W; i++)
                if (seq[i] != seq[i + p]) match = 0;
            if (match) per = p;
        }
        uint8_t k;
        if (!wrong) k = 0;
        else if (ok[f] || per == 1) k = 1;
        else if (per >= 2) k = 2;
        else k = 3;
        cls[f] = k;
        if (period) period[f] = per;
    }
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Weighted (unrolled) BP and its reverse-mode derivative.
 *
 * Each check-node output of the unrolled decoder is scaled by a learnable
 * weight w[t][s-1][d][pos]: t the iteration (0..T-1), s the stage position,
 * d = 0 for the L sweep and 1 for the R sweep, pos the position of the PE
 * output's row (j or jp).  Stages outside the permuted range keep their rows,
 * so pos = row there; inside the permuted range pos is the row's position in
 * the drawing of the active trellis (bit s-1 of pos is the bit stage s uses).
 * On the original graph pos is the row itself.  With all weights 1 this is plain min-sum BP.  Frozen
 * priors are the finite value 2^60 instead of +inf so that products with zero
 * derivatives stay zero.  No early stop.  The output LLR of row j is
 * o_j = L[n][j] + R[n][j] after the last L sweep.
 * Optional fixed last-k partial permutation (pool as above, cycled every
 * T_ev iterations, inner levels reset to 0); weights are indexed by stage
 * position, so one set of weights is shared by all trellises.
 *
 * min-sum derivative: for g = sgn(x)sgn(y)min(|x|,|y|), if |x| <= |y| then
 * g = sgn(y) x, else g = sgn(x) y (ties route to the first argument);
 * sgn(v) is -1 when v's sign bit is set.                                     */
#define WBP_FROZEN_PRIOR 1152921504606846976.0 /* 2^60 */

typedef struct {
    int32_t pp_mode; /* -1 none, 0 fixed last-k */
    int32_t k, T_ev, Q;
    uint64_t seed;
    int32_t fp32;
} or_wbp_params;

static double sgnb(double v) { return signbit(v) ? -1.0 : 1.0; }

/* position of row j in the drawing of the graph with stage order e: bit s-1
 * of the position is bit e[s-1] of j (the original graph draws row j at j) */
static int32_t drawn_pos(int32_t j, const int8_t *e, int n) {
    int32_t p = 0;
    for (int s = 0; s < n; s++) p |= ((j >> e[s]) & 1) << s;
    return p;
}

/* weight position of row j at stage s (1-based) under order e */
static int32_t weight_pos(int32_t j, const int8_t *e, int n, int s, int k_perm) {
    return (k_perm > 0 && s > n - k_perm) ? drawn_pos(j, e, n) : j;
}
static double ms0(double x, double y) {
    double m = fmin(fabs(x), fabs(y));
    return ((signbit(x) != 0) != (signbit(y) != 0)) ? -m : m;
}

typedef struct {
    int32_t N, n, T;
    const int8_t *pool;
    int32_t pool_q;
    const or_wbp_params *p;
    const uint8_t *frozen;
} wctx_t;

/* order index in force during iteration t, and whether an event after
 * iteration t re-orders the graph                                           */
static int32_t wbp_order_at(const wctx_t *w, int32_t t) {
    if (w->p->pp_mode != 0 || w->pool_q <= 1) return 0;
    return (t / w->p->T_ev) % w->pool_q;
}

/* forward pass of one frame; keeps every level of every iteration:
 * Ls[t] = L after iteration t's L sweep, Rs[t] = R at the entry of
 * iteration t (Rs[T] = after the last one).                                 */
static void wbp_forward_frame(const wctx_t *w, const float *llr, const double *wt, double *Ls,
                              double *Rs, double *Rsweep) {
    int32_t N = w->N, n = w->n, T = w->T;
    int fp32 = w->p->fp32;
    size_t lvl = (size_t)(n + 1) * N;
    double *R = Rs; /* Rs[0] */
    for (size_t i = 0; i < lvl; i++) R[i] = 0.0;
    for (int32_t j = 0; j < N; j++) R[(size_t)n * N + j] = w->frozen[j] ? WBP_FROZEN_PRIOR : 0.0;
    for (int32_t t = 0; t < T; t++) {
        double *L = Ls + (size_t)t * lvl;
        const double *Rin_state = Rs + (size_t)t * lvl;
        double *Rnext = Rs + (size_t)(t + 1) * lvl;
        double *Rw = Rsweep + (size_t)t * lvl; /* R values produced by this R sweep */
        const int8_t *ord = w->pool + (size_t)wbp_order_at(w, t) * n;
        const int kperm = (w->p->pp_mode == 0) ? w->p->k : 0;
        for (size_t i = 0; i < lvl; i++) L[i] = 0.0;
        for (int32_t j = 0; j < N; j++) L[j] = (double)llr[j];
        for (int s = 1; s <= n; s++) {
            int b = ord[s - 1];
            const double *wl = wt + (((size_t)t * n + (s - 1)) * 2 + 0) * N;
            for (int32_t j = 0; j < N; j++) {
                if ((j >> b) & 1) continue;
                int32_t jp = j | (1 << b);
                double l1 = L[(size_t)(s - 1) * N + j], l2 = L[(size_t)(s - 1) * N + jp];
                double r1 = Rin_state[(size_t)s * N + j], r2 = Rin_state[(size_t)s * N + jp];
                double a = rnd(fp32, l2 + r2);
                const int32_t pj = weight_pos(j, ord, n, s, kperm), pjp = weight_pos(jp, ord, n, s, kperm);
                L[(size_t)s * N + j] = rnd(fp32, wl[pj] * ms0(l1, a));
                L[(size_t)s * N + jp] = rnd(fp32, rnd(fp32, wl[pjp] * ms0(r1, l1)) + l2);
            }
        }
        /* R sweep: Rw level n is the prior; levels below are fresh */
        memcpy(Rw, Rin_state, sizeof(double) * lvl);
        for (int s = n; s >= 1; s--) {
            int b = ord[s - 1];
            const double *wr = wt + (((size_t)t * n + (s - 1)) * 2 + 1) * N;
            for (int32_t j = 0; j < N; j++) {
                if ((j >> b) & 1) continue;
                int32_t jp = j | (1 << b);
                double l1 = L[(size_t)(s - 1) * N + j], l2 = L[(size_t)(s - 1) * N + jp];
                double r1 = Rw[(size_t)s * N + j], r2 = Rw[(size_t)s * N + jp];
                double a = rnd(fp32, l2 + r2);
                const int32_t pj = weight_pos(j, ord, n, s, kperm), pjp = weight_pos(jp, ord, n, s, kperm);
                Rw[(size_t)(s - 1) * N + j] = rnd(fp32, wr[pj] * ms0(r1, a));
                Rw[(size_t)(s - 1) * N + jp] = rnd(fp32, rnd(fp32, wr[pjp] * ms0(r1, l1)) + r2);
            }
        }
        memcpy(Rnext, Rw, sizeof(double) * lvl);
        /* event after iteration t (not after the last one) */
        if (t + 1 < T && w->p->pp_mode == 0 && w->pool_q > 1 &&
            wbp_order_at(w, t + 1) != wbp_order_at(w, t)) {
            int kk = w->p->k;
            for (int lev = n - kk + 1; lev <= n - 1; lev++)
                for (int32_t j = 0; j < N; j++) Rnext[(size_t)lev * N + j] = 0.0;
        }
    }
}

int or_wbp_forward(int32_t N, int32_t K, const int32_t *info_idx, const float *llr, int64_t F,
                   const double *wt, int32_t T, const or_wbp_params *p, double *out) {
    int n = ilog2_exact(N);
    if (n < 0 || T < 1 || !p || !wt || !out || !info_idx || K < 1 || K > N) return OR_EINVAL;
    if (p->pp_mode == 0 && (p->k < 2 || p->k > n || p->T_ev < 1 || p->Q < 1)) return OR_EINVAL;
    size_t lvl = (size_t)(n + 1) * N;
    uint8_t *frozen = (uint8_t *)malloc((size_t)N);
    int8_t *pool = (int8_t *)malloc((size_t)(p->Q > 0 ? p->Q : 1) * n);
    double *Ls = (double *)malloc(sizeof(double) * lvl * T);
    double *Rs = (double *)malloc(sizeof(double) * lvl * (T + 1));
    double *Rw = (double *)malloc(sizeof(double) * lvl * T);
    if (!frozen || !pool || !Ls || !Rs || !Rw) {
        free(frozen); free(pool); free(Ls); free(Rs); free(Rw);
        return OR_ENOMEM;
    }
    for (int32_t j = 0; j < N; j++) frozen[j] = 1;
    for (int32_t i = 0; i < K; i++) frozen[info_idx[i]] = 0;
    int32_t pq = 1;
    if (p->pp_mode == 0) pq = or_trellis_pool(n, p->k, p->Q, p->seed, pool);
    else for (int s = 0; s < n; s++) pool[s] = (int8_t)s;
    wctx_t w = {N, n, T, pool, pq, p, frozen};
    for (int64_t f = 0; f < F; f++) {
        wbp_forward_frame(&w, llr + f * N, wt, Ls, Rs, Rw);
        const double *L = Ls + (size_t)(T - 1) * lvl;
        const double *R = Rs + (size_t)(T - 1) * lvl; /* level n prior, unchanged */
        for (int32_t j = 0; j < N; j++)
            out[f * N + j] = rnd(p->fp32, L[(size_t)n * N + j] + R[(size_t)n * N + j]);
    }
    free(frozen); free(pool); free(Ls); free(Rs); free(Rw);
    return OR_OK;
}

/* Reverse mode of one frame.  gout: d loss / d o of the frame's rows;
 * adds into grad_w [T][n][2][N]; grad_llr (or NULL): the frame's adjoint of
 * the channel LLRs.  The forward state Ls, Rs, Rsweep must hold the frame's
 * forward pass.
 *
 * absolute = 1 runs the same pass with every local derivative and every
 * upstream adjoint replaced by its magnitude: the min-sum routing is
 * unchanged, sgn() becomes 1, weights and forward messages enter as |w| and
 * |g|.  Each entry then holds the sum, over every path of the reverse
 * computation, of the magnitudes of the path's product of derivatives.  A
 * reverse pass that rounds each product and each sum once (with at most k
 * roundings on any path from the output to an entry) lies within
 * k u / (1 - k u) times that sum of the exact value, u the unit roundoff:
 * the bound the GPU adjoint is checked against.                            */
static double mg(int absolute, double v) { return absolute ? fabs(v) : v; }
static double sg(int absolute, double v) { return absolute ? 1.0 : sgnb(v); }

static void wbp_backward_frame(const wctx_t *w, const double *wt, const double *gout,
                               int absolute, const double *Ls, const double *Rs,
                               const double *Rw, double *gL, double *gR, double *gRs,
                               double *gRin, double *grad_w, double *grad_llr) {
    const int32_t N = w->N, n = w->n, T = w->T;
    const or_wbp_params *p = w->p;
    const size_t lvl = (size_t)(n + 1) * N;
    for (size_t i = 0; i < lvl; i++) gRs[i] = 0.0;
    for (int32_t t = T - 1; t >= 0; t--) {
        const double *L = Ls + (size_t)t * lvl;
        const double *Rin_state = Rs + (size_t)t * lvl;
        const double *Rsw = Rw + (size_t)t * lvl;
        const int8_t *ord = w->pool + (size_t)wbp_order_at(w, t) * n;
        const int kperm = (p->pp_mode == 0) ? p->k : 0;
        /* an event after iteration t reset the inner levels: nothing of
         * iteration t reaches iteration t+1 through them                 */
        if (t + 1 < T && p->pp_mode == 0 && w->pool_q > 1 &&
            wbp_order_at(w, t + 1) != wbp_order_at(w, t)) {
            for (int lev = n - p->k + 1; lev <= n - 1; lev++)
                for (int32_t j = 0; j < N; j++) gRs[(size_t)lev * N + j] = 0.0;
        }
        for (size_t i = 0; i < lvl; i++) { gL[i] = 0.0; gR[i] = 0.0; gRin[i] = 0.0; }
        /* R sweep outputs at levels 1..n-1 feed iteration t+1 */
        for (int lev = 1; lev <= n - 1; lev++)
            for (int32_t j = 0; j < N; j++) gR[(size_t)lev * N + j] = gRs[(size_t)lev * N + j];
        if (t == T - 1)
            for (int32_t j = 0; j < N; j++) gL[(size_t)n * N + j] = mg(absolute, gout[j]);
        /* reverse of the R sweep: stages 1..n */
        for (int s = 1; s <= n; s++) {
            int b = ord[s - 1];
            const double *wr = wt + (((size_t)t * n + (s - 1)) * 2 + 1) * N;
            double *gwr = grad_w + (((size_t)t * n + (s - 1)) * 2 + 1) * N;
            for (int32_t j = 0; j < N; j++) {
                if ((j >> b) & 1) continue;
                int32_t jp = j | (1 << b);
                double l1 = L[(size_t)(s - 1) * N + j], l2 = L[(size_t)(s - 1) * N + jp];
                double r1 = Rsw[(size_t)s * N + j], r2 = Rsw[(size_t)s * N + jp];
                double a = rnd(p->fp32, l2 + r2);
                double g1 = ms0(r1, a), g2 = ms0(r1, l1);
                double go1 = gR[(size_t)(s - 1) * N + j], go2 = gR[(size_t)(s - 1) * N + jp];
                const int32_t pj = weight_pos(j, ord, n, s, kperm), pjp = weight_pos(jp, ord, n, s, kperm);
                gwr[pj] += go1 * mg(absolute, g1);
                gwr[pjp] += go2 * mg(absolute, g2);
                double d1 = go1 * mg(absolute, wr[pj]), d2 = go2 * mg(absolute, wr[pjp]);
                double ga = 0.0;
                if (fabs(r1) <= fabs(a)) gR[(size_t)s * N + j] += d1 * sg(absolute, a);
                else ga += d1 * sg(absolute, r1);
                gL[(size_t)(s - 1) * N + jp] += ga;
                gR[(size_t)s * N + jp] += ga;
                if (fabs(r1) <= fabs(l1)) gR[(size_t)s * N + j] += d2 * sg(absolute, l1);
                else gL[(size_t)(s - 1) * N + j] += d2 * sg(absolute, r1);
                gR[(size_t)s * N + jp] += go2;
            }
        }
        /* reverse of the L sweep: stages n..1 */
        for (int s = n; s >= 1; s--) {
            int b = ord[s - 1];
            const double *wl = wt + (((size_t)t * n + (s - 1)) * 2 + 0) * N;
            double *gwl = grad_w + (((size_t)t * n + (s - 1)) * 2 + 0) * N;
            for (int32_t j = 0; j < N; j++) {
                if ((j >> b) & 1) continue;
                int32_t jp = j | (1 << b);
                double l1 = L[(size_t)(s - 1) * N + j], l2 = L[(size_t)(s - 1) * N + jp];
                double r1 = Rin_state[(size_t)s * N + j], r2 = Rin_state[(size_t)s * N + jp];
                double a = rnd(p->fp32, l2 + r2);
                double f1 = ms0(l1, a), f2 = ms0(r1, l1);
                double go1 = gL[(size_t)s * N + j], go2 = gL[(size_t)s * N + jp];
                const int32_t pj = weight_pos(j, ord, n, s, kperm), pjp = weight_pos(jp, ord, n, s, kperm);
                gwl[pj] += go1 * mg(absolute, f1);
                gwl[pjp] += go2 * mg(absolute, f2);
                double d1 = go1 * mg(absolute, wl[pj]), d2 = go2 * mg(absolute, wl[pjp]);
                double ga = 0.0;
                if (fabs(l1) <= fabs(a)) gL[(size_t)(s - 1) * N + j] += d1 * sg(absolute, a);
                else ga += d1 * sg(absolute, l1);
                gL[(size_t)(s - 1) * N + jp] += ga;
                gRin[(size_t)s * N + jp] += ga;
                if (fabs(r1) <= fabs(l1)) gRin[(size_t)s * N + j] += d2 * sg(absolute, l1);
                else gL[(size_t)(s - 1) * N + j] += d2 * sg(absolute, r1);
                gL[(size_t)(s - 1) * N + jp] += go2;
            }
        }
        /* adjoint of the R state entering iteration t (levels 1..n-1) */
        for (size_t i = 0; i < lvl; i++) gRs[i] = 0.0;
        for (int lev = 1; lev <= n - 1; lev++)
            for (int32_t j = 0; j < N; j++) gRs[(size_t)lev * N + j] = gRin[(size_t)lev * N + j];
        if (grad_llr) {
            if (t == T - 1)
                for (int32_t j = 0; j < N; j++) grad_llr[j] = 0.0;
            for (int32_t j = 0; j < N; j++) grad_llr[j] += gL[j];
        }
    }
}

/* reverse mode: grad_out [F][N] = d loss / d o; accumulates grad_w
 * [T][n][2][N] (summed over frames, in frame order, in double) and writes
 * grad_llr [F][N] if non-NULL.  grad_w_abs (or NULL) receives the same sums
 * taken over magnitudes (absolute = 1 above), the per-entry scale of the
 * rounding error of an FP32 adjoint.                                        */
int or_wbp_backward(int32_t N, int32_t K, const int32_t *info_idx, const float *llr, int64_t F,
                    const double *wt, int32_t T, const or_wbp_params *p, const double *grad_out,
                    double *grad_w, double *grad_llr, double *grad_w_abs) {
    int n = ilog2_exact(N);
    if (n < 0 || T < 1 || !p || !wt || !grad_out || !grad_w || !info_idx || K < 1 || K > N)
        return OR_EINVAL;
    if (p->pp_mode == 0 && (p->k < 2 || p->k > n || p->T_ev < 1 || p->Q < 1)) return OR_EINVAL;
    size_t lvl = (size_t)(n + 1) * N;
    uint8_t *frozen = (uint8_t *)malloc((size_t)N);
    int8_t *pool = (int8_t *)malloc((size_t)(p->Q > 0 ? p->Q : 1) * n);
    double *Ls = (double *)malloc(sizeof(double) * lvl * T);
    double *Rs = (double *)malloc(sizeof(double) * lvl * (T + 1));
    double *Rw = (double *)malloc(sizeof(double) * lvl * T);
    double *gL = (double *)malloc(sizeof(double) * lvl);
    double *gR = (double *)malloc(sizeof(double) * lvl);     /* adjoint of R sweep values */
    double *gRs = (double *)malloc(sizeof(double) * lvl);    /* adjoint of R state at exit */
    double *gRin = (double *)malloc(sizeof(double) * lvl);   /* adjoint of R state at entry */
    if (!frozen || !pool || !Ls || !Rs || !Rw || !gL || !gR || !gRs || !gRin) {
        free(frozen); free(pool); free(Ls); free(Rs); free(Rw);
        free(gL); free(gR); free(gRs); free(gRin);
        return OR_ENOMEM;
    }
    for (int32_t j = 0; j < N; j++) frozen[j] = 1;
    for (int32_t i = 0; i < K; i++) frozen[info_idx[i]] = 0;
    int32_t pq = 1;
    if (p->pp_mode == 0) pq = or_trellis_pool(n, p->k, p->Q, p->seed, pool);
    else for (int s = 0; s < n; s++) pool[s] = (int8_t)s;
    wctx_t w = {N, n, T, pool, pq, p, frozen};
    const size_t nw = (size_t)T * n * 2 * N;
    memset(grad_w, 0, sizeof(double) * nw);
    if (grad_w_abs) memset(grad_w_abs, 0, sizeof(double) * nw);
    for (int64_t f = 0; f < F; f++) {
        wbp_forward_frame(&w, llr + f * N, wt, Ls, Rs, Rw);
        wbp_backward_frame(&w, wt, grad_out + f * N, 0, Ls, Rs, Rw, gL, gR, gRs, gRin, grad_w,
                           grad_llr ? grad_llr + f * N : NULL);
        if (grad_w_abs)
            wbp_backward_frame(&w, wt, grad_out + f * N, 1, Ls, Rs, Rw, gL, gR, gRs, gRin,
                               grad_w_abs, NULL);
    }
    free(frozen); free(pool); free(Ls); free(Rs); free(Rw);
    free(gL); free(gR); free(gRs); free(gRin);
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Hooks used by the oracle's own pins.                                      */

/* Run n_iter plain BP iterations (no stop, no events) on a fixed graph whose
 * row j uses bit ord[j*n + s-1] at stage s.  Frozen rows get a +inf prior.
 * L_out, R_out: [n+1][N] final state (double).                              */
int or_bp_run(int32_t N, int32_t n_iter, const int8_t *ord, const float *llr,
              const uint8_t *frozen, double alpha, int32_t fp32, int32_t exact,
              double *L_out, double *R_out) {
    int n = ilog2_exact(N);
    if (n < 0 || n_iter < 0 || !ord || !llr || !frozen || !L_out || !R_out) return OR_EINVAL;
    size_t lvl = (size_t)(n + 1) * N;
    int8_t *o = (int8_t *)malloc((size_t)N * n);
    if (!o) return OR_ENOMEM;
    memcpy(o, ord, (size_t)N * n);
    sched_t sc = {n, o};
    arith_t ar = {alpha, fp32, exact};
    for (size_t t = 0; t < lvl; t++) { L_out[t] = 0.0; R_out[t] = 0.0; }
    for (int32_t j = 0; j < N; j++) L_out[j] = (double)llr[j];
    for (int32_t j = 0; j < N; j++) R_out[(size_t)n * N + j] = frozen[j] ? INFINITY : 0.0;
    for (int32_t it = 0; it < n_iter; it++) one_iteration(&ar, N, &sc, L_out, R_out);
    free(o);
    return OR_OK;
}

/* Continue n_iter plain BP iterations from a given state (in place). */
int or_bp_continue(int32_t N, int32_t n_iter, const int8_t *ord, double alpha, int32_t fp32,
                   int32_t exact, double *L, double *R) {
    int n = ilog2_exact(N);
    if (n < 0 || n_iter < 0 || !ord || !L || !R) return OR_EINVAL;
    int8_t *o = (int8_t *)malloc((size_t)N * n);
    if (!o) return OR_ENOMEM;
    memcpy(o, ord, (size_t)N * n);
    sched_t sc = {n, o};
    arith_t ar = {alpha, fp32, exact};
    for (int32_t it = 0; it < n_iter; it++) one_iteration(&ar, N, &sc, L, R);
    free(o);
    return OR_OK;
}

/* Encode through a (possibly permuted) graph: starting from u on the u side,
 * apply the XOR butterflies of stages n..1 with each row's own bit.          */
int or_graph_encode(int32_t N, const int8_t *ord, const uint8_t *u, uint8_t *x) {
    int n = ilog2_exact(N);
    if (n < 0) return OR_EINVAL;
    memmove(x, u, (size_t)N);
    for (int s = n; s >= 1; s--) {
        uint8_t *nx = (uint8_t *)malloc((size_t)N);
        if (!nx) return OR_ENOMEM;
        memcpy(nx, x, (size_t)N);
        for (int32_t j = 0; j < N; j++) {
            int b = ord[(size_t)j * n + s - 1];
            int32_t p = j ^ (1 << b);
            if ((int)ord[(size_t)p * n + s - 1] != b) { free(nx); return -2; } /* not a matching */
            if (!((j >> b) & 1)) nx[j] = x[j] ^ x[p];
        }
        memcpy(x, nx, (size_t)N);
        free(nx);
    }
    return OR_OK;
}

/* Apply n_events Algorithm-1 events to the original graph of length N.
 * ord_out: [n_events][N][n] schedule after each event; nzero_out,
 * reset_add_out: [n_events] N_zero and the Eq. 2 increment; zeroed_out:
 * [n_events] number of (level, row) nodes reset, counted on the state;
 * draw_out (or NULL): [n_events][4 + n] the accepted draw of each event.     */
int or_alg1_trace(int32_t N, int32_t P_range, int32_t P_level, int32_t D, int32_t N_min,
                  uint64_t seed, int32_t n_events, int8_t *ord_out, int32_t *nzero_out,
                  int32_t *reset_add_out, int32_t *zeroed_out, int32_t *draw_out) {
    int n = ilog2_exact(N);
    if (n < 0 || P_range < 2 || P_range > n || P_level < 1 || P_level > n - 1 || D < 1)
        return OR_EINVAL;
    size_t lvl = (size_t)(n + 1) * N;
    int8_t *o = (int8_t *)malloc((size_t)N * n);
    double *L = (double *)malloc(sizeof(double) * lvl);
    double *R = (double *)malloc(sizeof(double) * lvl);
    int32_t *lab = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
    int32_t *q = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
    if (!o || !L || !R || !lab || !q) { free(o); free(L); free(R); free(lab); free(q); return OR_ENOMEM; }
    sched_t sc = {n, o};
    for (int32_t j = 0; j < N; j++)
        for (int s = 0; s < n; s++) o[(size_t)j * n + s] = (int8_t)s;
    uint64_t st = seed;
    for (int32_t e = 0; e < n_events; e++) {
        for (size_t t = 0; t < lvl; t++) { L[t] = 1.0; R[t] = 1.0; }
        int32_t nz = 0;
        alg1_event(&sc, N, L, R, &st, P_range, P_level, &nz, lab, q,
                   draw_out ? draw_out + (size_t)e * (4 + n) : NULL);
        int32_t add = nz / D;
        if (add < N_min) add = N_min;
        int32_t z = 0;
        for (size_t t = 0; t < lvl; t++) z += (L[t] == 0.0);
        memcpy(ord_out + (size_t)e * N * n, o, (size_t)N * n);
        nzero_out[e] = nz;
        reset_add_out[e] = add;
        zeroed_out[e] = z;
    }
    free(o); free(L); free(R); free(lab); free(q);
    return OR_OK;
}

/* The R2 reading's events on the original graph of length N (as
 * or_alg1_trace): ord_out [n_events][N][n], nzero_out [n_events].           */
int or_alg1_trace_r2(int32_t N, int32_t P_range, int32_t P_level, uint64_t seed, int32_t n_events,
                     int8_t *ord_out, int32_t *nzero_out) {
    int n = ilog2_exact(N);
    if (n < 0 || n > 30 || P_range < 2 || P_range > n || P_level < 1 || P_level > n - 1) return OR_EINVAL;
    size_t lvl = (size_t)(n + 1) * N;
    int8_t *o = (int8_t *)malloc((size_t)N * n);
    double *L = (double *)malloc(sizeof(double) * lvl);
    double *R = (double *)malloc(sizeof(double) * lvl);
    int32_t *mk = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
    if (!o || !L || !R || !mk) { free(o); free(L); free(R); free(mk); return OR_ENOMEM; }
    sched_t sc = {n, o};
    for (int32_t j = 0; j < N; j++)
        for (int s = 0; s < n; s++) o[(size_t)j * n + s] = (int8_t)s;
    uint64_t st = seed;
    int32_t prev[3] = {0, 0, 0};
    for (int32_t e = 0; e < n_events; e++) {
        for (size_t t = 0; t < lvl; t++) { L[t] = 1.0; R[t] = 1.0; }
        int32_t nz = 0;
        alg1_event_r2(&sc, N, L, R, &st, P_range, P_level, &nz, prev, mk);
        memcpy(ord_out + (size_t)e * N * n, o, (size_t)N * n);
        nzero_out[e] = nz;
    }
    free(o); free(L); free(R); free(mk);
    return OR_OK;
}

/* sizes of the parameter structs, so the Python side can check its mirror */
int32_t or_sizeof_params(void) { return (int32_t)sizeof(or_params); }
int32_t or_sizeof_wbp_params(void) { return (int32_t)sizeof(or_wbp_params); }
