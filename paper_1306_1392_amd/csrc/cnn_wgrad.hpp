// Weight gradient of a 3x3 convolution (zero padding 1, stride 1) as a direct MFMA kernel:
//   dW[n][tap cin + c] = sum over pixels p of dZ[p][n] X[p + (ty - 1, tx - 1)][c]
// the same sums as the implicit GEMM of cnn_gemm.hpp (Im2colT x PlainT), with every input pixel
// read once per 8 x 32-pixel output tile instead of once per tap.
//
// Workgroup = one block of 32 outputs n x 32 input channels c, and a contiguous range of output tiles
// (the split); each of its 4 wavefronts owns two rows of every tile and accumulates all nine taps,
// D_tap[n][c] (32 x 32, 16 accumulators per lane), over the split with
// v_mfma_f32_32x32x16_bf16: K = 16 consecutive pixels of one row, A = dZ[pixels][n] (n = lane % 32),
// B = X[pixels shifted by the tap][c] (c = lane % 32).  Both operands need eight consecutive pixels of
// one channel per lane, so a tile's dZ (8 x 32 pixels x 32 n) and input patch (10 rows x 32 pixels x 32 c,
// in three copies shifted by tx = 0, 1, 2 columns so that every read is 16-byte aligned) are staged in
// LDS channel-major: a thread loads 16-byte pixel vectors (8 channels each; ten consecutive pixels give
// all three copies of an 8-pixel group), transposes 8 x 8 blocks in registers (v_perm_b32) and writes
// 16-byte channel rows; a task's loads are issued together.  Channel strides of
// 264 and 328 elements (4 mod 32 dwords) put the 8 lanes of an LDS pass in 8 different bank groups.
// Each wavefront writes its nine 32 x 32 blocks as one split-K partial (4 partials per workgroup), in
// the partial layout of the GEMM path ([split][m = tap cin + c][n]); the partials are added in a fixed
// order afterwards, so the result does not depend on scheduling.
#pragma once

#include "cnn_conv.hpp"

namespace pyhst {
namespace cnn {

constexpr int WG_ZLD = 8 * CT_W + 8;    // dZ channel stride in LDS (elements): 256 pixels + 8
constexpr int WG_XLD = 10 * CT_W + 8;   // patch channel stride: 10 rows x 32 pixels + 8

// in[I0 + i], i = 0..7: 8 channels of pixel i (BF16 pairs per dword); store(j, v): v = 8 pixels of
// channel j, each row handed over as soon as it is formed
template <int I0, int NIN, class Store>
__device__ __forceinline__ void transpose8x8(const uint4 (&in)[NIN], Store store)
{
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        // channel j of pixels 2d (low half) and 2d + 1 (high half): v_perm_b32 takes bytes 0-3 from its
        // second operand and 4-7 from its first
        const uint32_t sel = (j & 1) ? 0x07060302u : 0x05040100u;
        uint32_t d[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint4 lo = in[I0 + 2 * q], hi = in[I0 + 2 * q + 1];
            const uint32_t wl = (j >> 1) == 0 ? lo.x : (j >> 1) == 1 ? lo.y : (j >> 1) == 2 ? lo.z : lo.w;
            const uint32_t wh = (j >> 1) == 0 ? hi.x : (j >> 1) == 1 ? hi.y : (j >> 1) == 2 ? hi.z : hi.w;
            d[q] = __builtin_amdgcn_perm(wh, wl, sel);
        }
        store(j, make_uint4(d[0], d[1], d[2], d[3]));
    }
}

// grid: (splits, N / 32 output blocks, cin / 32 input blocks); part: [4 splits][9 cin][N] floats per
// split index s (partials 4 s .. 4 s + 3); tiles: 8 x 32-pixel output tiles of the batch, tps per split.
// bpart (may be null): the bias gradient's partial sums [split][N], sum over the split's pixels of
// dZ[p][n], taken by the workgroups of input block 0 from the staged dZ (thread t: output n0 + t / 8,
// pixels 32 (t % 8) .. + 31 of every tile; the 8 partial sums meet in a fixed order by lane exchanges).
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
void wgrad3x3_kernel(Act x, Act dz, float *part, float *bpart, int cin, int N, int tiles, int tps)
{
    __shared__ uint4 sXv[3 * 32 * WG_XLD / 8];
    __shared__ uint4 sZv[32 * WG_ZLD / 8];
    bf16_t *sX = (bf16_t *)sXv, *sZ = (bf16_t *)sZv;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int col = lane & 31, half = lane >> 5;
    const int n0 = blockIdx.y * 32, c0 = blockIdx.z * 32;
    f32x16 acc[9];
#pragma unroll
    for (int k = 0; k < 9; ++k)
#pragma unroll
        for (int q = 0; q < 16; ++q) acc[k][q] = 0.0f;
    const bool bias = bpart != nullptr && blockIdx.z == 0;   // uniform over the workgroup
    float bacc = 0.0f;
    const int t_end = min(tiles, (int)(blockIdx.x + 1) * tps);
    for (int t = blockIdx.x * tps; t < t_end; ++t) {
        const ConvTile c = conv_tile<8>(x, t);
        __syncthreads();   // the previous tile's reads of sX and sZ are done
        // staging tasks, a task's loads issued together: threads 0..159 take the input patch task (patch
        // row r, column group g, channel group q): pixels x0 - 1 + 8 g + i, i = 0..9, give the three copies
        // tx (pixels 8 g + tx + 0..7 of the copy); dZ task d = (row y, column group g, output group q) goes
        // to thread 160 + d (d < 96), and d = 96 + t to thread t < 32 after its patch task
        uint4 in[10];
        if (tid < 160) {
            const int q = tid & 3, g = (tid >> 2) & 3, r = tid >> 4;
            const int yy = c.y0 - 1 + r;
            const bool rowin = (unsigned)yy < (unsigned)x.H;
            const bf16_t *src = x.p + ((int64_t)c.b * x.H + (rowin ? yy : 0)) * x.W * x.cs + x.co + c0 + 8 * q;
#pragma unroll
            for (int i = 0; i < 10; ++i) {
                const int xx = c.x0 - 1 + 8 * g + i;
                in[i] = rowin && (unsigned)xx < (unsigned)x.W ? ld8(src + (int64_t)xx * x.cs) : zero8();
            }
            bf16_t *dst = sX + (8 * q) * WG_XLD + r * CT_W + 8 * g;
            transpose8x8<0>(in, [&](int j, uint4 v) { *(uint4 *)&dst[j * WG_XLD] = v; });
            transpose8x8<1>(in, [&](int j, uint4 v) { *(uint4 *)&dst[(32 + j) * WG_XLD] = v; });
            transpose8x8<2>(in, [&](int j, uint4 v) { *(uint4 *)&dst[(64 + j) * WG_XLD] = v; });
        }
        auto stage_dz = [&](int d) {
            const int g = d & 3, q = (d >> 2) & 3, y = d >> 4;
            const int yy = c.y0 + y;
            const bool rowin = yy < x.H;
            const bf16_t *src = dz.p + ((int64_t)c.b * x.H + (rowin ? yy : 0)) * x.W * dz.cs + dz.co + n0 + 8 * q;
            uint4 in8[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int xx = c.x0 + 8 * g + i;
                in8[i] = rowin && xx < x.W ? ld8(src + (int64_t)xx * dz.cs) : zero8();
            }
            bf16_t *dst = sZ + (8 * q) * WG_ZLD + y * CT_W + 8 * g;
            transpose8x8<0>(in8, [&](int j, uint4 v) { *(uint4 *)&dst[j * WG_ZLD] = v; });
        };
        if (tid >= 160) stage_dz(tid - 160);
        else if (tid < 32) stage_dz(96 + tid);
        __syncthreads();
        if (bias) {
            const uint4 *row = (const uint4 *)&sZ[(tid >> 3) * WG_ZLD + 32 * (tid & 7)];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const uint4 u = row[v];
                const uint32_t w[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
                for (int e = 0; e < 4; ++e) bacc += bf16_lo(w[e]) + bf16_hi(w[e]);
            }
        }
        // wavefront w: output rows 2w, 2w + 1; K step kk = 16 pixels of one row
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
            const int y = 2 * wave + (kk >> 1), cofs = 16 * (kk & 1) + 8 * half;
            const bf16x8 a = *(const bf16x8 *)&sZ[col * WG_ZLD + y * CT_W + cofs];
#pragma unroll
            for (int ty = 0; ty < 3; ++ty)
#pragma unroll
                for (int tx = 0; tx < 3; ++tx) {
                    const bf16x8 b = *(const bf16x8 *)&sX[(tx * 32 + col) * WG_XLD + (y + ty) * CT_W + cofs];
                    acc[3 * ty + tx] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc[3 * ty + tx], 0, 0, 0);
                }
        }
    }
    if (bias) {
        bacc += __shfl_xor(bacc, 1, 64);
        bacc += __shfl_xor(bacc, 2, 64);
        bacc += __shfl_xor(bacc, 4, 64);
        if ((tid & 7) == 0) bpart[(int64_t)blockIdx.x * N + n0 + (tid >> 3)] = bacc;
    }
    // accumulator 4 g + q of tap k: D[n = 8 g + 4 half + q][c = col] -> part[m = k cin + c0 + col][n0 + n]
    const int M = 9 * cin;
    float *P = part + (int64_t)(4 * blockIdx.x + wave) * M * N;
#pragma unroll
    for (int k = 0; k < 9; ++k)
#pragma unroll
        for (int g = 0; g < 4; ++g)
            *(float4 *)&P[(int64_t)(k * cin + c0 + col) * N + n0 + 8 * g + 4 * half] =
                make_float4(acc[k][4 * g], acc[k][4 * g + 1], acc[k][4 * g + 2], acc[k][4 * g + 3]);
}

// splits (workgroups along the batch) for the direct weight gradient: about two workgroups per CU in
// all, within the partial buffer (4 partials of 9 cin x N floats and a bias partial of N per split);
// 0: not handled
inline int wgrad_splits(int cin, int N, int tiles, int cu_count, size_t part_floats)
{
    if (cin % 32 || N % 32) return 0;
    const int blocks = (N / 32) * (cin / 32);
    int s = std::max(1, (2 * cu_count + blocks - 1) / blocks);
    s = std::min(s, tiles);
    const size_t per = (size_t)4 * 9 * cin * N + N;   // weight partials and the bias partial
    while (s > 1 && (size_t)s * per > part_floats) --s;
    if ((size_t)s * per > part_floats) return 0;
    return s;
}

}  // namespace cnn
}  // namespace pyhst
