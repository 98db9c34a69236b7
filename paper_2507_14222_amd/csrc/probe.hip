// Attainable-peak probes of the device (include/ig_probe.h): the rates that the
// contraction kernels and the memory-bound stages are measured against, beside
// the vendor's published peaks.  Measurement only; no step of the method.
//
//   k_probe_mfma_fp4  back-to-back v_mfma_scale_f32_32x32x64_f8f6f4 on fp4 (e2m1)
//                     register operands, four independent accumulator chains per
//                     wave, every SIMD filled: the fp4 matrix-core issue rate that
//                     the subset-test contractions use
//   k_probe_copy      16-byte vector loads and stores over a large buffer, grid
//                     stride: the HBM read + write bandwidth a streaming kernel gets
#include "common.h"
#include "kernels.h"

namespace ig {

typedef int v8i_p __attribute__((ext_vector_type(8)));
typedef float v16f_p __attribute__((ext_vector_type(16)));

constexpr int PR_NT = 256;   // threads per probe workgroup

__global__ __launch_bounds__(PR_NT) void k_probe_mfma_fp4(uint32_t iters, float *__restrict__ sink) {
    const uint32_t lane = threadIdx.x & 63;
    // arbitrary finite e2m1 nibbles (no NaN exists in e2m1): the rate does not
    // depend on the values
    const int x = (int)(0x2A2A2A2Au ^ (lane * 0x01010101u));
    const v8i_p a = {x, x ^ 0x11111111, x, x ^ 0x22222222, 0, 0, 0, 0};
    const v8i_p b = {x ^ 0x33333333, x, x ^ 0x44444444, x, 0, 0, 0, 0};
    v16f_p c0 = {0}, c1 = {0}, c2 = {0}, c3 = {0};
    for (uint32_t i = 0; i < iters; ++i) {
        c0 = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, c0, 4, 4, 0, 127, 0, 127);
        c1 = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(b, a, c1, 4, 4, 0, 127, 0, 127);
        c2 = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, a, c2, 4, 4, 0, 127, 0, 127);
        c3 = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(b, b, c3, 4, 4, 0, 127, 0, 127);
    }
    float s = 0.0f;
#pragma unroll
    for (int r = 0; r < 16; ++r) s += c0[r] + c1[r] + c2[r] + c3[r];
    // one value per workgroup keeps the chains live
    if (threadIdx.x == 0) sink[blockIdx.x] = s;
}

__global__ __launch_bounds__(PR_NT) void k_probe_copy(const uint4 *__restrict__ src, uint4 *__restrict__ dst,
                                                       size_t n) {
    const size_t stride = (size_t)gridDim.x * PR_NT;
    for (size_t i = (size_t)blockIdx.x * PR_NT + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

// Milliseconds of one launch made by `launch` between two events on stream s.
template <class F>
static float timed(hipStream_t s, F launch) {
    hipEvent_t e0, e1;
    IG_HIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        throw Error(IG_E_DEVICE, "hipEventCreate failed");
    }
    float ms = 0.0f;
    hipError_t err = hipEventRecord(e0, s);
    if (err == hipSuccess) {
        launch();
        err = hipGetLastError();
    }
    if (err == hipSuccess) err = hipEventRecord(e1, s);
    if (err == hipSuccess) err = hipEventSynchronize(e1);
    if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    IG_HIP(err);
    return ms;
}

double probe_mfma_fp4(uint32_t iters, hipStream_t s, float *ms_out) {
    IG_REQUIRE(iters >= 1 && iters <= (1u << 24), IG_E_INVAL, "iters must be in 1..2^24");
    const uint32_t blocks = device_cus() * 8;   // 8 workgroups of 4 waves per CU: 8 waves per SIMD
    Scratch<float> sink(blocks, s);
    const float ms = timed(s, [&] { k_probe_mfma_fp4<<<blocks, PR_NT, 0, s>>>(iters, sink.get()); });
    if (ms_out) *ms_out = ms;
    // four instructions per iteration per wave, 2 * 32 * 32 * 64 operations each
    const double ops = (double)blocks * (PR_NT / 64) * iters * 4.0 * 2.0 * 32 * 32 * 64;
    return ops / (ms * 1e-3);
}

double probe_copy(const void *src, void *dst, size_t bytes, hipStream_t s, float *ms_out) {
    IG_REQUIRE(src && dst, IG_E_INVAL, "src or dst is NULL");
    IG_REQUIRE(bytes >= 16 && bytes % 16 == 0, IG_E_INVAL, "bytes must be a positive multiple of 16");
    IG_REQUIRE(((uintptr_t)src | (uintptr_t)dst) % 16 == 0, IG_E_INVAL, "buffers must be 16-byte aligned");
    const size_t n = bytes / 16;
    const uint32_t blocks = device_cus() * 16;
    const float ms = timed(s, [&] {
        k_probe_copy<<<blocks, PR_NT, 0, s>>>(static_cast<const uint4 *>(src), static_cast<uint4 *>(dst), n);
    });
    if (ms_out) *ms_out = ms;
    return 2.0 * (double)bytes / (ms * 1e-3);   // read + write
}

}  // namespace ig
