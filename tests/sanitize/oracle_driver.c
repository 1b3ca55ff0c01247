/*
 * oracle_driver.c -- runs every entry point of the CPU oracle once or more on
 * small synthetic inputs, for a host AddressSanitizer / UndefinedBehavior-
 * Sanitizer build (tests/test_sanitize.py).  The oracle's source is included
 * whole, so its static helpers run under the sanitizers too.  Inputs: random
 * messages, BPSK signs and Gaussian-like noise from a local xorshift
 * generator; the values are not checked here (the pins do that), only that
 * no access is out of bounds, no arithmetic is undefined and nothing leaks.
 */
#include "../../oracle/oracle.c"

#include <stdio.h>

static uint64_t xs = 0x9E3779B97F4A7C15ull;
static uint64_t xnext(void) {
    xs ^= xs << 13;
    xs ^= xs >> 7;
    xs ^= xs << 17;
    return xs;
}
static double unif(void) { return (double)(xnext() >> 11) / 9007199254740992.0; }

#define CHECK(x)                                                          \
    do {                                                                  \
        int rc_ = (x);                                                    \
        if (rc_ != OR_OK) {                                               \
            fprintf(stderr, "%s:%d: %s -> %d\n", __FILE__, __LINE__, #x, rc_); \
            return 1;                                                     \
        }                                                                 \
    } while (0)

static int run_code(int32_t N, int32_t K, int32_t cw, uint32_t poly, int64_t F) {
    int n = ilog2_exact(N);
    int32_t *info = (int32_t *)malloc(sizeof(int32_t) * K);
    uint8_t *frozen = (uint8_t *)malloc(N);
    double *lnz = (double *)malloc(sizeof(double) * N);
    int32_t km = K - cw;
    uint8_t *msg = (uint8_t *)malloc((size_t)F * km);
    uint8_t *u = (uint8_t *)malloc((size_t)F * N);
    uint8_t *x = (uint8_t *)malloc((size_t)F * N);
    float *llr = (float *)malloc(sizeof(float) * F * N);
    uint8_t *mh = (uint8_t *)malloc((size_t)F * km);
    int32_t *it = (int32_t *)malloc(sizeof(int32_t) * F);
    uint8_t *ok = (uint8_t *)malloc(F);
    double *soft = (double *)malloc(sizeof(double) * F * N);
    double *state = (double *)malloc(sizeof(double) * F * 2 * (n + 1) * N);
    const int32_t H = 16;
    uint64_t *hist = (uint64_t *)calloc((size_t)F * H, sizeof(uint64_t));
    uint8_t *cls = (uint8_t *)malloc(F);
    int32_t *per = (int32_t *)malloc(sizeof(int32_t) * F);
    CHECK(or_construct(N, K, 2.5, info, frozen, lnz));
    for (int64_t i = 0; i < F * km; i++) msg[i] = (uint8_t)(xnext() & 1);
    CHECK(or_encode(N, K, info, cw, poly, msg, F, u, x));
    for (int64_t i = 0; i < F * N; i++) {
        double g = 0.0;
        for (int r = 0; r < 12; r++) g += unif();
        llr[i] = (float)(2.0 * ((x[i] ? -1.0 : 1.0) + 0.8 * (g - 6.0)) / 0.64);
    }
    or_params base;
    memset(&base, 0, sizeof base);
    base.max_iter = 40;
    base.alpha = 1.0;
    base.stop = cw ? 2 : 1;
    base.it_min = 2;
    base.pp_mode = -1;
    base.seed = 11;
    base.fp32 = 1;
    for (int mode = -1; mode <= 3; mode++) {
        if (mode >= 2 && n < 3) continue;
        or_params p = base;
        p.pp_mode = mode;
        p.k = n >= 3 ? 3 : n;
        p.T = 3;
        p.Q = 8;
        p.P_range = n >= 3 ? 3 : 2;
        p.P_level = n - 1 < 2 ? n - 1 : 2;
        p.D = 8;
        p.N_min = 2;
        if (mode == 0 && p.k < 2) continue;
        CHECK(or_decode(N, K, info, cw, poly, llr, F, &p, mh, it, ok, soft, state, 2));
        CHECK(or_decode_trace(N, K, info, cw, poly, llr, F, &p, mh, it, ok, hist, H, 2));
        CHECK(or_classify(F, km, mh, msg, ok, it, hist, H, cls, per));
        p.fp32 = 0;
        p.exact_boxplus = 1;
        CHECK(or_decode(N, K, info, cw, poly, llr, F, &p, mh, it, ok, NULL, NULL, 1));
        p.exact_boxplus = 0;
        p.fp32 = 1;
        if (mode >= 0) {
            p.noise_sigma = 0.6f;
            CHECK(or_decode(N, K, info, cw, poly, llr, F, &p, mh, it, ok, NULL, NULL, 3));
        }
        p.alpha = 0.9375;
        p.stop = 0;
        CHECK(or_decode(N, K, info, cw, poly, llr, F, &p, mh, NULL, NULL, NULL, NULL, 1));
    }
    /* weighted BP: plain and last-k, gradients with magnitudes and LLR adjoint */
    if (n >= 3) {
        const int32_t T = 3;
        size_t nw = (size_t)T * n * 2 * N;
        double *w = (double *)malloc(sizeof(double) * nw);
        double *gw = (double *)malloc(sizeof(double) * nw);
        double *ga = (double *)malloc(sizeof(double) * nw);
        double *out = (double *)malloc(sizeof(double) * F * N);
        double *gout = (double *)malloc(sizeof(double) * F * N);
        double *gl = (double *)malloc(sizeof(double) * F * N);
        for (size_t i = 0; i < nw; i++) w[i] = 0.7 + 0.6 * unif();
        for (int64_t i = 0; i < F * N; i++) gout[i] = unif() - 0.5;
        for (int pm = -1; pm <= 0; pm++) {
            or_wbp_params wp = {pm, 3, 2, 4, 5, 1};
            CHECK(or_wbp_forward(N, K, info, llr, F, w, T, &wp, out));
            CHECK(or_wbp_backward(N, K, info, llr, F, w, T, &wp, gout, gw, gl, ga));
        }
        free(w); free(gw); free(ga); free(out); free(gout); free(gl);
    }
    /* plain BP hooks on one frame, with a per-row order table */
    int8_t *ord = (int8_t *)malloc((size_t)N * n);
    for (int32_t j = 0; j < N; j++)
        for (int s = 0; s < n; s++) ord[(size_t)j * n + s] = (int8_t)s;
    double *L = (double *)malloc(sizeof(double) * (n + 1) * N);
    double *R = (double *)malloc(sizeof(double) * (n + 1) * N);
    CHECK(or_bp_run(N, 5, ord, llr, frozen, 1.0, 1, 0, L, R));
    CHECK(or_bp_continue(N, 3, ord, 1.0, 0, 1, L, R));
    CHECK(or_graph_encode(N, ord, u, x));
    if (n >= 3) {
        const int32_t E = 6;
        int8_t *ords = (int8_t *)malloc((size_t)E * N * n);
        int32_t a[E], b[E], c[E];
        int32_t *dr = (int32_t *)malloc(sizeof(int32_t) * E * (4 + n));
        CHECK(or_alg1_trace(N, n, n - 1, 4, 2, 3, E, ords, a, b, c, dr));
        CHECK(or_alg1_trace_r2(N, n, n - 1, 5, E, ords, a));
        free(ords); free(dr);
    }
    for (int j = 0; j < 8; j++) (void)or_noise_gauss(7, j, j + 1, j * 3);
    (void)or_crc_bits(msg, km, 24, 0x1864CFB);
    free(ord); free(L); free(R);
    free(info); free(frozen); free(lnz); free(msg); free(u); free(x); free(llr); free(mh);
    free(it); free(ok); free(soft); free(state); free(hist); free(cls); free(per);
    return 0;
}

int main(void) {
    int8_t orders[8 * 12];
    for (int k = 0; k <= 12; k++)
        if (or_trellis_pool(12, k, 8, 99, orders) < 1) return 1;
    if (run_code(2, 1, 0, 0, 5)) return 1;
    if (run_code(8, 4, 0, 0, 9)) return 1;
    if (run_code(64, 32, 0, 0, 7)) return 1;
    if (run_code(128, 72, 8, 0x9B, 6)) return 1;
    if (run_code(256, 144, 16, 0x1021, 5)) return 1;
    if (run_code(1024, 536, 24, 0x1864CFB, 3)) return 1;
    puts("oracle sanitizer run ok");
    return 0;
}
