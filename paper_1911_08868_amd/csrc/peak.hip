// peak.hip -- calibration kernels for the roofline constants of bench.py:
// the VALU issue rate of the decoder's own instruction mix and the LDS read
// bandwidth, measured on the device instead of taken from the data sheet.
// Built into its own library (libpbp_peak.so); the decoder never calls it.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

// Eight processing-element-like updates per half step, each the decoder's
// three VALU instructions: an add, the clamp v_med3_f32 by the magnitude of
// another chain's value and the sign v_bitop3_b32 of that value, all eight
// reading the previous half step's values (eight independent results).  Two
// half steps per loop trip alternate the two register sets, so a trip is 48
// VALU instructions (16 x 3) and nothing else on the vector unit; the values
// stay bounded and the result is stored, so nothing is folded or dropped.
template <int I>
__device__ __forceinline__ float pe_like(const float (&a)[8]) {
    const float x = a[(I + 1) & 7];
    const float y = a[I] + 0.25f * (float)(I + 1);
    const float ax = __builtin_fabsf(x);
    const float t = __builtin_amdgcn_fmed3f(y, ax, -ax);
    return __uint_as_float(__float_as_uint(t) ^ (__float_as_uint(x) & 0x80000000u));
}

__device__ __forceinline__ void half_step(const float (&a)[8], float (&b)[8]) {
    b[0] = pe_like<0>(a);
    b[1] = pe_like<1>(a);
    b[2] = pe_like<2>(a);
    b[3] = pe_like<3>(a);
    b[4] = pe_like<4>(a);
    b[5] = pe_like<5>(a);
    b[6] = pe_like<6>(a);
    b[7] = pe_like<7>(a);
}

// One instruction kind alone, eight independent chains, 8 x 8 instructions
// per loop trip: KIND 0 v_add_f32, 1 v_med3_f32 (bound by the next chain's
// magnitude), 2 v_bitop3_b32 (the next chain's sign bit xored in); the
// per-instruction issue rates behind the processing element's peak.
template <int KIND>
__global__ void __launch_bounds__(256) k_one(float *out, int steps, float seed) {
    float a[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) a[i] = seed + (float)(threadIdx.x + 3 * i) - 100.f;
    for (int s = 0; s < steps; ++s) {
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            float nx[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const float x = a[(i + 1) & 7];
                if constexpr (KIND == 0) nx[i] = a[i] + x;
                if constexpr (KIND == 1) nx[i] = __builtin_amdgcn_fmed3f(a[i], __builtin_fabsf(x), -__builtin_fabsf(x));
                if constexpr (KIND == 2) {
                    // written as one instruction: the compiler would otherwise
                    // solve the xor recurrence in closed form
                    float r;
                    asm volatile("v_xor_b32 %0, %1, %2" : "=v"(r) : "v"(a[i]), "v"(x));
                    nx[i] = r;
                }
            }
#pragma unroll
            for (int i = 0; i < 8; ++i) a[i] = nx[i];
        }
    }
    float r = 0.f;
#pragma unroll
    for (int i = 0; i < 8; ++i) r += a[i];
    out[blockIdx.x * blockDim.x + threadIdx.x] = r;
}

__global__ void __launch_bounds__(256) k_valu(float *out, int steps, float seed) {
    float a[8], b[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) a[i] = seed + (float)(threadIdx.x + 3 * i) - 100.f;
    for (int s = 0; s < steps; ++s) {
        half_step(a, b);
        half_step(b, a);
    }
    float r = 0.f;
#pragma unroll
    for (int i = 0; i < 8; ++i) r += a[i];
    out[blockIdx.x * blockDim.x + threadIdx.x] = r;
}

// LDS reads: every thread reads 16 consecutive bytes per access, consecutive
// lanes consecutive 16-byte chunks (no bank conflicts), eight accesses per
// loop trip within a 64 KiB array (base + u * 256 chunks, base < 2048 + 256),
// folding the words into xors so every load is used: 8 x 16 bytes per thread
// and trip.
__global__ void __launch_bounds__(1024) k_lds(uint32_t *out, int steps) {
    __shared__ uint4 buf[4096];  // 64 KiB
    for (int i = threadIdx.x; i < 4096; i += blockDim.x)
        buf[i] = make_uint4(i, i * 3u, i * 5u, i * 7u);
    __syncthreads();
    uint32_t x0 = 0, x1 = 0;
    // the base moves by a data-dependent multiple of 256 chunks per trip, so
    // no load can be hoisted; the eight accesses of a trip take constant
    // offsets from it
    const int lane_chunk = (int)threadIdx.x & 255;
    int base = lane_chunk;
    for (int s = 0; s < steps; ++s) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const uint4 v = buf[base + u * 256];
            x0 ^= v.x ^ v.y;
            x1 ^= v.z ^ v.w;
        }
        base = lane_chunk + 256 * (int)((x0 ^ (uint32_t)s) & 7u);
    }
    out[blockIdx.x * blockDim.x + threadIdx.x] = x0 ^ x1;
}

// The processing element with the decoder's own dependencies: ROWS values
// per thread, per stage ROWS/2 elements on the pairs (i, i | b) of register
// rows (b cycling over the thread's row bits as the decoder's stages do),
// each element's two outputs f(x_ip + r_ip, x_i) and f(x_i, r_i) + x_ip from
// the stage's inputs; 8 stages per loop trip, 6 VALU instructions per
// element.  Launched with dynamic LDS that caps the workgroups (one wave per
// SIMD each) per CU, it measures the mix's issue rate against independent
// chains per wave and waves per SIMD.
__device__ __forceinline__ float clamp_cn(float b, float y) {
    const float ab = __builtin_fabsf(b);
    const float t = __builtin_amdgcn_fmed3f(y, ab, -ab);
    return __uint_as_float(__float_as_uint(t) ^ (__float_as_uint(b) & 0x80000000u));
}

template <int ROWS>
__global__ void __launch_bounds__(256) k_pe_chain(float *out, int steps, float seed) {
    constexpr int LOG = ROWS == 2 ? 1 : ROWS == 4 ? 2 : 3;
    float v[ROWS], r[ROWS];
#pragma unroll
    for (int i = 0; i < ROWS; ++i) {
        v[i] = seed + (float)(threadIdx.x + 3 * i) - 100.f;
        r[i] = 0.5f * (float)(i + 1) - 1.3f;
    }
    for (int s = 0; s < steps; ++s) {
#pragma unroll
        for (int st = 0; st < 8; ++st) {
            const int b = 1 << (st % LOG);
            float nx[ROWS];
#pragma unroll
            for (int i = 0; i < ROWS; ++i) {
                if ((i & b) == 0) {
                    const int ip = i | b;
                    nx[i] = clamp_cn(v[ip] + r[ip], v[i]);
                    nx[ip] = clamp_cn(v[i], r[i]) + v[ip];
                }
            }
#pragma unroll
            for (int i = 0; i < ROWS; ++i) v[i] = nx[i];
        }
    }
    float acc = 0.f;
#pragma unroll
    for (int i = 0; i < ROWS; ++i) acc += v[i];
    out[blockIdx.x * blockDim.x + threadIdx.x] = acc;
}

}  // namespace

extern "C" {

// k_pe_chain<rows> (rows 2, 4 or 8) in workgroups of 256 threads with
// (160 KiB / waves_per_simd - 1 KiB) of dynamic LDS, so that at most
// waves_per_simd (1..8) workgroups share a CU; `blocks` workgroups, `steps`
// loop trips, d_out at least blocks * 256 floats.  Returns 0 or the HIP error.
int pbp_peak_launch_pe(int rows, int waves_per_simd, int blocks, int steps, void *d_out, void *stream) {
    if (waves_per_simd < 1 || waves_per_simd > 8) return (int)hipErrorInvalidValue;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int lds = (160 * 1024) / waves_per_simd - 1024;
    const void *k = rows == 2 ? (const void *)k_pe_chain<2> : rows == 4 ? (const void *)k_pe_chain<4>
                                                                        : (const void *)k_pe_chain<8>;
    hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return (int)e;
    float *o = static_cast<float *>(d_out);
    if (rows == 2)
        hipLaunchKernelGGL(k_pe_chain<2>, dim3(blocks), dim3(256), lds, s, o, steps, 0.5f);
    else if (rows == 4)
        hipLaunchKernelGGL(k_pe_chain<4>, dim3(blocks), dim3(256), lds, s, o, steps, 0.5f);
    else
        hipLaunchKernelGGL(k_pe_chain<8>, dim3(blocks), dim3(256), lds, s, o, steps, 0.5f);
    return (int)hipGetLastError();
}

// which = 0: k_valu (workgroups of 256 threads), 1: k_lds (workgroups of 1024
// threads, 16 waves, so that two workgroups keep 8 waves per SIMD reading
// LDS), 2..4: k_one<0..2> (256 threads, 64 instructions per trip); `blocks`
// workgroups, `steps` loop trips, d_out at least blocks * threads words.
// Returns 0 or the HIP error.
int pbp_peak_launch(int which, int blocks, int steps, void *d_out, void *stream) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (which == 0)
        hipLaunchKernelGGL(k_valu, dim3(blocks), dim3(256), 0, s, static_cast<float *>(d_out), steps, 0.5f);
    else if (which == 1)
        hipLaunchKernelGGL(k_lds, dim3(blocks), dim3(1024), 0, s, static_cast<uint32_t *>(d_out), steps);
    else if (which == 2)
        hipLaunchKernelGGL(k_one<0>, dim3(blocks), dim3(256), 0, s, static_cast<float *>(d_out), steps, 0.5f);
    else if (which == 3)
        hipLaunchKernelGGL(k_one<1>, dim3(blocks), dim3(256), 0, s, static_cast<float *>(d_out), steps, 0.5f);
    else
        hipLaunchKernelGGL(k_one<2>, dim3(blocks), dim3(256), 0, s, static_cast<float *>(d_out), steps, 0.5f);
    return (int)hipGetLastError();
}

}  // extern "C"
