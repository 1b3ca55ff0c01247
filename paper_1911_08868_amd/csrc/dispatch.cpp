// dispatch.cpp -- routes a decode launch to the translation unit built for
// its block length and kernel family.
#include "decode_inst.h"

namespace pbp {
int run_decode_n1(const DecodeLaunch &);
int run_decode_n2(const DecodeLaunch &);
int run_decode_n3(const DecodeLaunch &);
int run_decode_n4(const DecodeLaunch &);
int run_decode_n5(const DecodeLaunch &);
int run_decode_n6(const DecodeLaunch &);
int run_decode_n7(const DecodeLaunch &);
int run_decode_n8(const DecodeLaunch &);
int run_decode_n9(const DecodeLaunch &);
int run_decode_n10(const DecodeLaunch &);
int run_decode_n11(const DecodeLaunch &);
int run_decode_n12(const DecodeLaunch &);
int run_decode_trace_n1(const DecodeLaunch &);
int run_decode_trace_n2(const DecodeLaunch &);
int run_decode_trace_n3(const DecodeLaunch &);
int run_decode_trace_n4(const DecodeLaunch &);
int run_decode_trace_n5(const DecodeLaunch &);
int run_decode_trace_n6(const DecodeLaunch &);
int run_decode_trace_n7(const DecodeLaunch &);
int run_decode_trace_n8(const DecodeLaunch &);
int run_decode_trace_n9(const DecodeLaunch &);
int run_decode_trace_n10(const DecodeLaunch &);
int run_decode_trace_n11(const DecodeLaunch &);
int run_decode_trace_n12(const DecodeLaunch &);
int run_decode_exact_n1(const DecodeLaunch &);
int run_decode_exact_n2(const DecodeLaunch &);
int run_decode_exact_n3(const DecodeLaunch &);
int run_decode_exact_n4(const DecodeLaunch &);
int run_decode_exact_n5(const DecodeLaunch &);
int run_decode_exact_n6(const DecodeLaunch &);
int run_decode_exact_n7(const DecodeLaunch &);
int run_decode_exact_n8(const DecodeLaunch &);
int run_decode_exact_n9(const DecodeLaunch &);
int run_decode_exact_n10(const DecodeLaunch &);
int run_decode_exact_n11(const DecodeLaunch &);
int run_decode_exact_n12(const DecodeLaunch &);
int run_decode_noise_n1(const DecodeLaunch &);
int run_decode_noise_n2(const DecodeLaunch &);
int run_decode_noise_n3(const DecodeLaunch &);
int run_decode_noise_n4(const DecodeLaunch &);
int run_decode_noise_n5(const DecodeLaunch &);
int run_decode_noise_n6(const DecodeLaunch &);
int run_decode_noise_n7(const DecodeLaunch &);
int run_decode_noise_n8(const DecodeLaunch &);
int run_decode_noise_n9(const DecodeLaunch &);
int run_decode_noise_n10(const DecodeLaunch &);
int run_decode_noise_n11(const DecodeLaunch &);
int run_decode_noise_n12(const DecodeLaunch &);

int launch_decode_n(int n, const DecodeLaunch &L) {
    switch (n) {
        case 1:
            return L.variant == 3 ? run_decode_noise_n1(L)
                 : L.variant == 2 ? run_decode_exact_n1(L)
                 : L.variant == 1 ? run_decode_trace_n1(L)
                                  : run_decode_n1(L);
        case 2:
            return L.variant == 3 ? run_decode_noise_n2(L)
                 : L.variant == 2 ? run_decode_exact_n2(L)
                 : L.variant == 1 ? run_decode_trace_n2(L)
                                  : run_decode_n2(L);
        case 3:
            return L.variant == 3 ? run_decode_noise_n3(L)
                 : L.variant == 2 ? run_decode_exact_n3(L)
                 : L.variant == 1 ? run_decode_trace_n3(L)
                                  : run_decode_n3(L);
        case 4:
            return L.variant == 3 ? run_decode_noise_n4(L)
                 : L.variant == 2 ? run_decode_exact_n4(L)
                 : L.variant == 1 ? run_decode_trace_n4(L)
                                  : run_decode_n4(L);
        case 5:
            return L.variant == 3 ? run_decode_noise_n5(L)
                 : L.variant == 2 ? run_decode_exact_n5(L)
                 : L.variant == 1 ? run_decode_trace_n5(L)
                                  : run_decode_n5(L);
        case 6:
            return L.variant == 3 ? run_decode_noise_n6(L)
                 : L.variant == 2 ? run_decode_exact_n6(L)
                 : L.variant == 1 ? run_decode_trace_n6(L)
                                  : run_decode_n6(L);
        case 7:
            return L.variant == 3 ? run_decode_noise_n7(L)
                 : L.variant == 2 ? run_decode_exact_n7(L)
                 : L.variant == 1 ? run_decode_trace_n7(L)
                                  : run_decode_n7(L);
        case 8:
            return L.variant == 3 ? run_decode_noise_n8(L)
                 : L.variant == 2 ? run_decode_exact_n8(L)
                 : L.variant == 1 ? run_decode_trace_n8(L)
                                  : run_decode_n8(L);
        case 9:
            return L.variant == 3 ? run_decode_noise_n9(L)
                 : L.variant == 2 ? run_decode_exact_n9(L)
                 : L.variant == 1 ? run_decode_trace_n9(L)
                                  : run_decode_n9(L);
        case 10:
            return L.variant == 3 ? run_decode_noise_n10(L)
                 : L.variant == 2 ? run_decode_exact_n10(L)
                 : L.variant == 1 ? run_decode_trace_n10(L)
                                  : run_decode_n10(L);
        case 11:
            return L.variant == 3 ? run_decode_noise_n11(L)
                 : L.variant == 2 ? run_decode_exact_n11(L)
                 : L.variant == 1 ? run_decode_trace_n11(L)
                                  : run_decode_n11(L);
        case 12:
            return L.variant == 3 ? run_decode_noise_n12(L)
                 : L.variant == 2 ? run_decode_exact_n12(L)
                 : L.variant == 1 ? run_decode_trace_n12(L)
                                  : run_decode_n12(L);
        default: return fail(PC_EINVAL, "block length out of range");
    }
}
}  // namespace pbp
