// Measurement kernels for the roofline of the backprojector: VALU lane-op rate
// (independent FP32 FMA chains), the backprojector's own instruction mix without
// memory traffic, LDS ds_read_b64 and ds_read_b128 bandwidth in a conflict-free pattern,
// ds_read_b128 with consecutive lanes 1.25 entries apart (the projector's spread of reads
// along a line when a bin spans 1/|a| = 1.25 image positions), and ds_read_b128 with half
// of the lanes masked off.
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

// ds_read_b128, lane l reading entry idx(l) + 80 u + 256 (it mod 8), wrapped to the 2048-entry buffer:
// PAT 0: idx = l, every lane; PAT 1: idx = floor(1.25 l), every lane; PAT 2: idx = l, even lanes only;
// PAT 3: idx = l, lanes 0..31 only (the other lanes skip the loop, so the reads run with part of the
// wavefront masked off).
template <int PAT>
__global__ __launch_bounds__(256) void lds_read128_kernel(float *out, int iters)
{
    __shared__ float4 buf[2048];
    for (int i = threadIdx.x; i < 2048; i += 256) buf[i] = make_float4((float)i, 1.0f, 0.5f, 2.0f);
    __syncthreads();
    float acc = 0.0f;
    const int l = threadIdx.x & 63;
    const int idx = PAT == 1 ? (5 * l) >> 2 : l;
    const bool active = PAT == 2 ? (l & 1) == 0 : PAT == 3 ? l < 32 : true;
    if (active) {
        for (int it = 0; it < iters; ++it) {
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const float4 v = buf[(idx + 80 * u + (it & 7) * 256) & 2047];
                acc += v.x * v.y + v.z * v.w;
            }
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
    case 3: lds_read128_kernel<0><<<blocks, 256, 0, st>>>(sink, iters); break;
    case 4: lds_read128_kernel<1><<<blocks, 256, 0, st>>>(sink, iters); break;
    case 5: lds_read128_kernel<2><<<blocks, 256, 0, st>>>(sink, iters); break;
    case 6: lds_read128_kernel<3><<<blocks, 256, 0, st>>>(sink, iters); break;
    default: return fail(PYHST_EARG, "microbench: unknown kind");
    }
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? PYHST_OK : hip_fail(e, "microbench");
}
