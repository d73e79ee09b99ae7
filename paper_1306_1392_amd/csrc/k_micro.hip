// Measurement kernels for the roofline of the backprojector: VALU lane-op rate
// (independent FP32 FMA chains), the backprojector's own instruction mix without
// memory traffic, and LDS ds_read_b64 bandwidth in a conflict-free pattern.
#include "internal.hpp"

namespace pyhst {
namespace {

// 8 independent FMA chains per lane: 8 lane-ops per iteration.
__global__ __launch_bounds__(256) void valu_fma_kernel(float *out, int iters, float a, float b)
{
    float x[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) x[i] = (float)(threadIdx.x + i);
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int i = 0; i < 8; ++i) x[i] = fmaf(x[i], a, b);
    }
    float s = 0.0f;
#pragma unroll
    for (int i = 0; i < 8; ++i) s += x[i];
    if (s == 12345.678f) out[blockIdx.x * blockDim.x + threadIdx.x] = s;   // keeps the chains live
}

// The backprojector's per-update VALU sequence (add, trunc, fract, shift-add, add, fma),
// 8 independent updates per iteration, the LDS read replaced by register data.
__global__ __launch_bounds__(256) void valu_mix_kernel(float *out, int iters, float step)
{
    float t[8], acc[8];
    int sink = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        t[i] = 1.0f + 0.37f * (float)(threadIdx.x & 63) + (float)i;
        acc[i] = 0.0f;
    }
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const float tt = t[i] + step;
            const int k = (int)tt;
            const float f = __builtin_amdgcn_fractf(tt);
            const int addr = (k << 3) + it;
            sink ^= addr;
            acc[i] += tt;
            acc[i] = fmaf(f, tt, acc[i]);
            t[i] = tt - step;
        }
    }
    float s = (float)sink;
#pragma unroll
    for (int i = 0; i < 8; ++i) s += acc[i];
    if (s == 12345.678f) out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// ds_read_b64: each lane reads 8 consecutive window entries pattern (no bank conflicts).
__global__ __launch_bounds__(256) void lds_read_kernel(float *out, int iters)
{
    __shared__ float2 buf[4096];
    for (int i = threadIdx.x; i < 4096; i += 256) buf[i] = make_float2((float)i, 1.0f);
    __syncthreads();
    float acc = 0.0f;
    int idx = threadIdx.x & 63;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const float2 v = buf[(idx + 64 * u + (it & 7) * 512) & 4095];
            acc += v.x * v.y;
        }
    }
    if (acc == 12345.678f) out[blockIdx.x * blockDim.x + threadIdx.x] = acc;
}

}  // namespace
}  // namespace pyhst

using namespace pyhst;

extern "C" int pyhst_microbench(int32_t kind, int32_t blocks, int32_t iters, float *sink, hipStream_t st)
{
    if (blocks <= 0 || iters <= 0 || !sink) return fail(PYHST_EARG, "microbench: bad argument");
    switch (kind) {
    case 0: valu_fma_kernel<<<blocks, 256, 0, st>>>(sink, iters, 0.999f, 0.001f); break;
    case 1: valu_mix_kernel<<<blocks, 256, 0, st>>>(sink, iters, 0.25f); break;
    case 2: lds_read_kernel<<<blocks, 256, 0, st>>>(sink, iters); break;
    default: return fail(PYHST_EARG, "microbench: unknown kind");
    }
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? PYHST_OK : hip_fail(e, "microbench");
}
