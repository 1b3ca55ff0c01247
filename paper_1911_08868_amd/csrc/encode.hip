// encode.hip -- polar encoder x = u G_N (Eq. 1) for batches of frames.
//
// One workgroup per frame at a time (grid-stride over frames).  The message
// bits go to their information rows, the CRC (linear, so the xor of the CRC
// of each set message bit) to the last crc_width information rows, and the
// n XOR butterflies v[j] ^= v[j + 2^b] (rows j with bit b = 0) run in LDS,
// one barrier per stage; pairs of a stage are disjoint, so each stage is a
// single parallel step.  With ua != NULL the kernel also writes u on the
// information rows, in ascending row order (the message, then its CRC); with
// x == NULL it stops there.
#include <algorithm>

#include "bp_core.h"
#include "internal.h"

namespace pbp {

__global__ void __launch_bounds__(256)
k_encode(const uint8_t *msg, uint8_t *x, uint8_t *ua, int64_t F, int N, int n, int K, int kmsg, int cw,
         const int32_t *info, const uint32_t *crc_bit) {
    extern __shared__ uint8_t u[];
    __shared__ uint32_t red[4];
    const int tid = threadIdx.x;
    for (int64_t f = blockIdx.x; f < F; f += gridDim.x) {
        for (int j = tid; j < N; j += blockDim.x) u[j] = 0;
        __syncthreads();
        uint32_t c = 0;
        const uint8_t *m = msg + f * kmsg;
        for (int i = tid; i < kmsg; i += blockDim.x) {
            const uint8_t b = m[i] & 1u;
            u[info[i]] = b;
            if (b && cw) c ^= crc_bit[i];
        }
        if (cw) {
            c = lanes_xor<64>(c);
            if ((tid & 63) == 0) red[tid >> 6] = c;
        }
        __syncthreads();
        if (cw) {
            const uint32_t crc = red[0] ^ red[1] ^ red[2] ^ red[3];
            for (int t = tid; t < cw; t += blockDim.x)
                u[info[kmsg + t]] = (uint8_t)((crc >> (cw - 1 - t)) & 1u);
        }
        if (ua) {
            __syncthreads();
            for (int i = tid; i < K; i += blockDim.x) ua[f * K + i] = u[info[i]];
        }
        if (!x) {
            __syncthreads();
            continue;
        }
        for (int b = 0; b < n; ++b) {
            __syncthreads();
            for (int p = tid; p < N / 2; p += blockDim.x) {
                const int j = ((p >> b) << (b + 1)) | (p & ((1 << b) - 1));
                u[j] ^= u[j | (1 << b)];
            }
        }
        __syncthreads();
        uint8_t *xo = x + f * N;
        for (int j = tid; j < N; j += blockDim.x) xo[j] = u[j];
        __syncthreads();
    }
}

int launch_encode(const pc_code *c, const uint8_t *d_msg, uint8_t *d_x, uint8_t *d_ua, int64_t F,
                  hipStream_t stream) {
    int64_t grid = std::min<int64_t>(F, (int64_t)device_cu_count() * 8);
    hipLaunchKernelGGL(k_encode, dim3((unsigned)grid), dim3(256), (size_t)c->N, stream, d_msg, d_x,
                       d_ua, F, c->N, c->n, c->K, c->K_msg, c->crc_width, c->d.info,
                       c->d.crc_of_msg_bit);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "encode launch");
    return PC_OK;
}

}  // namespace pbp
