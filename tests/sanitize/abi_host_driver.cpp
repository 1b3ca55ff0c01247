// abi_host_driver.cpp -- runs the host logic of the C ABI (host.cpp: argument
// checks, the trellis pool, code construction up to its device upload, error
// strings) under host AddressSanitizer / UndefinedBehaviorSanitizer
// (tests/test_sanitize.py).  The kernel launchers of the other translation
// units are replaced by stubs that fail loudly, so nothing here touches a
// GPU; without one, device allocation fails and polar_construct returns
// PC_EHIP after construction, which is the path this exercises.
#include <cstdio>
#include <cstring>

#include "../../paper_1911_08868_amd/csrc/decode_inst.h"
#include "../../paper_1911_08868_amd/csrc/internal.h"

namespace pbp {
static int stub(const char *what) {
    std::fprintf(stderr, "stub launcher reached: %s\n", what);
    return PC_ENOTSUP;
}
int launch_decode_n(int, const DecodeLaunch &) { return stub("decode"); }
int launch_encode(const pc_code *, const uint8_t *, uint8_t *, uint8_t *, int64_t, hipStream_t) {
    return stub("encode");
}
int launch_alg1(const pc_code *, const float *, int64_t, const pc_bp_params &, const pc_pp_params &, uint8_t *,
                int32_t *, uint8_t *, float *, uint64_t *, int32_t, hipStream_t) {
    return stub("alg1");
}
int noalloc_scratch_init() { return PC_EHIP; }
int launch_classify(const uint8_t *, const uint8_t *, const uint8_t *, const int32_t *, const uint64_t *, int32_t,
                    int64_t, int32_t, uint8_t *, int32_t *, hipStream_t) {
    return stub("classify");
}
}  // namespace pbp

#define EXPECT(cond)                                                         \
    do {                                                                     \
        if (!(cond)) {                                                       \
            std::fprintf(stderr, "%s:%d: expected %s\n", __FILE__, __LINE__, #cond); \
            return 1;                                                        \
        }                                                                    \
    } while (0)

int main() {
    // the trellis pool for every (n, k, Q)
    int8_t orders[8 * 12];
    for (int n = 1; n <= 12; ++n)
        for (int k = 0; k <= n; ++k)
            for (int Q = 1; Q <= 8; ++Q) {
                const int q = polar_trellis_pool(n, k, Q, 1000u * n + 10u * k + Q, orders);
                EXPECT(q >= 1 && q <= Q);
            }
    EXPECT(polar_trellis_pool(13, 2, 8, 1, orders) == PC_EINVAL);
    EXPECT(polar_trellis_pool(10, 11, 8, 1, orders) == PC_EINVAL);
    EXPECT(polar_trellis_pool(10, 4, 9, 1, orders) == PC_EINVAL);
    EXPECT(polar_trellis_pool(10, 4, 8, 1, nullptr) == PC_EINVAL);
    // construction: invalid arguments, then every valid length up to the
    // device upload (no GPU here: PC_EHIP), CRC widths 0..32
    pc_code *c = nullptr;
    EXPECT(polar_construct(3, 2, 0, 0, 2.5, &c) == PC_EINVAL && !c);
    EXPECT(polar_construct(8192, 2, 0, 0, 2.5, &c) == PC_EINVAL);
    EXPECT(polar_construct(64, 65, 0, 0, 2.5, &c) == PC_EINVAL);
    EXPECT(polar_construct(64, 16, 16, 0x1021, 2.5, &c) == PC_EINVAL);
    EXPECT(polar_construct(64, 32, 33, 0, 2.5, &c) == PC_EINVAL);
    EXPECT(polar_construct(64, 32, 0, 0, 0.0 / 0.0, &c) == PC_EINVAL);
    EXPECT(polar_construct(64, 32, 0, 0, 2.5, nullptr) == PC_EINVAL);
    for (int N = 2; N <= 4096; N *= 2)
        for (int cw : {0, 1, 8, 16, 24, 32}) {
            if (cw >= N) continue;
            const int K = cw + 1 + (N - cw - 1) / 2;
            const int rc = polar_construct(N, K, cw, 0x1864CFBu, -1.0 / 0.0, &c);
            EXPECT(rc == PC_OK || rc == PC_EHIP);
            if (rc == PC_OK) polar_code_free(c);
            c = nullptr;
        }
    // entry points with a NULL code or bad sizes return before any launch
    pc_bp_params bp{200, 1.f, PC_STOP_CRC, 3, PC_CHECK_MINSUM};
    pc_pp_params pp{};
    EXPECT(bp_decode(nullptr, nullptr, 1, &bp, nullptr, nullptr, nullptr, nullptr) == PC_EINVAL);
    EXPECT(pp_mt_bp_decode(nullptr, nullptr, 1, &bp, &pp, nullptr, nullptr, nullptr, nullptr) == PC_EINVAL);
    EXPECT(polar_encode(nullptr, nullptr, nullptr, 1, nullptr) == PC_EINVAL);
    EXPECT(polar_info_bits(nullptr, nullptr, nullptr, 1, nullptr) == PC_EINVAL);
    EXPECT(pp_mt_bp_decode_trace(nullptr, nullptr, 1, &bp, &pp, nullptr, nullptr, nullptr, nullptr, 0, nullptr) ==
           PC_EINVAL);
    EXPECT(polar_classify_errors(nullptr, nullptr, nullptr, nullptr, nullptr, 8, 4, 4, nullptr, nullptr, nullptr) ==
           PC_EINVAL);
    EXPECT(polar_classify_errors(nullptr, nullptr, nullptr, nullptr, nullptr, 8, 0, 4, nullptr, nullptr, nullptr) ==
           PC_OK);
    for (int rc : {0, -1, -2, -3, -4, -99}) EXPECT(std::strlen(polar_strerror(rc)) > 0);
    EXPECT(std::strlen(polar_last_error()) > 0);
    std::puts("abi host sanitizer run ok");
    return 0;
}
