// MFMA BF16 implicit-GEMM building blocks of the learned sparse-angle corrector
// (an encoder-decoder CNN; not part of the paper, whose learned prior is a patch
// dictionary).  C[M][N] = sum_k A[m][k] B[k][n], A and B gathered on the fly from
// NHWC BF16 activations / weights, FP32 accumulation in v_mfma_f32_32x32x16_bf16.
//
// Lane layout of v_mfma_f32_32x32x16_bf16 (wave64): lane l holds A[l%32][8(l/32)..+7]
// and B[8(l/32)..+7][l%32]; accumulator register i holds
// C[8(i/4) + 4(l/32) + i%4][l%32].
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace pyhst {
namespace cnn {

typedef uint16_t bf16_t;
typedef __attribute__((__vector_size__(8 * sizeof(short)))) short bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

__device__ __host__ inline bf16_t f2bf(float f)
{
    uint32_t u;
    __builtin_memcpy(&u, &f, 4);
    if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;   // NaN
    u += 0x7fffu + ((u >> 16) & 1u);                       // round to nearest even
    return (bf16_t)(u >> 16);
}
__device__ __host__ inline float bf2f(bf16_t b)
{
    uint32_t u = (uint32_t)b << 16;
    float f;
    __builtin_memcpy(&f, &u, 4);
    return f;
}

constexpr int TM = 128, TK = 32, LDK = TK + 8;   // LDS row stride 80 B keeps 16 B alignment

// floor(n / d) for 0 <= n < 2^31 by multiply and shift: m = ceil(2^(32+l) / d), l = ceil(log2 d)
// (Granlund & Montgomery); exact in this range because n e / (d 2^(32+l)) < 1/d for e = m d - 2^(32+l) < d.
struct FastDiv {
    uint64_t m;
    uint32_t l, d;
};
inline FastDiv make_fastdiv(uint32_t d)
{
    uint32_t l = 0;
    while ((1ull << l) < d) ++l;
    const unsigned __int128 num = (unsigned __int128)1 << (32 + l);
    const uint64_t m = (uint64_t)((num + d - 1) / d);
    return FastDiv{m, l, d};
}
__device__ inline uint32_t fdiv(uint32_t n, const FastDiv &f)
{
    return (uint32_t)(((unsigned __int128)n * f.m) >> (32 + f.l));
}

template <int TN>
struct WaveGrid {
    static constexpr int WM = TN >= 128 ? 2 : 4;
    static constexpr int WN = 4 / WM;
};

// ---------------------------------------------------------------- operand loaders
// VK = true: load(row, k) returns the 8 elements [row][k..k+7] (vector along K).
// VK = false: loadv(row8, k) returns [row8..row8+7][k] (vector along M or N).
struct Act {          // NHWC activation view: channel stride cs, channel offset co
    const bf16_t *p;
    int B, H, W, cs, co;
};

__device__ inline uint4 ld8(const bf16_t *p) { return *(const uint4 *)p; }
__device__ inline uint4 zero8() { return make_uint4(0, 0, 0, 0); }

// A[m = pixel][k = (tap, c)] = X[pixel + (ty-1, tx-1)][c], zero outside the image
struct Im2colA {
    static constexpr bool VK = true;
    Act x;
    int C;
    __device__ uint4 load(int m, int k, int M, int kend) const
    {
        if (m >= M || k >= kend) return zero8();
        const int tap = k / C, c = k - tap * C;
        const int hw = x.H * x.W;
        const int b = m / hw, r = m - b * hw;
        const int y = r / x.W + tap / 3 - 1, xx = r % x.W + tap % 3 - 1;
        if ((unsigned)y >= (unsigned)x.H || (unsigned)xx >= (unsigned)x.W) return zero8();
        return ld8(x.p + ((int64_t)(b * x.H + y) * x.W + xx) * x.cs + x.co + c);
    }
};

// A[m = pixel][k] = X[pixel][k]
struct PlainA {
    static constexpr bool VK = true;
    Act x;
    __device__ uint4 load(int m, int k, int M, int kend) const
    {
        if (m >= M || k >= kend) return zero8();
        return ld8(x.p + (int64_t)m * x.cs + x.co + k);
    }
};

// A[m = low-res pixel (b,y,x)][k = (d, co)] = dY[(b, 2y+dy, 2x+dx)][co]  (dY at 2H x 2W)
struct UpGatherA {
    static constexpr bool VK = true;
    Act dy;     // high-resolution tensor
    int Cout;
    __device__ uint4 load(int m, int k, int M, int kend) const
    {
        if (m >= M || k >= kend) return zero8();
        const int d = k / Cout, co = k - d * Cout;
        const int h = dy.H >> 1, w = dy.W >> 1;
        const int b = m / (h * w), r = m - b * (h * w);
        const int y = 2 * (r / w) + (d >> 1), xx = 2 * (r % w) + (d & 1);
        return ld8(dy.p + ((int64_t)(b * dy.H + y) * dy.W + xx) * dy.cs + dy.co + co);
    }
};

// B[k][n] = Wt[n][k] (weights stored n-major, k contiguous)
struct WeightB {
    static constexpr bool VK = true;
    const bf16_t *w;
    int K;
    __device__ uint4 load(int n, int k, int N, int kend) const
    {
        if (n >= N || k >= kend) return zero8();
        return ld8(w + (int64_t)n * K + k);
    }
};

// A[m = (tap, c)][k = pixel] = X[pixel + off(tap)][c]   (weight gradient of a 3x3 conv)
struct Im2colT {
    static constexpr bool VK = false;
    Act x;
    int C;
    __device__ uint4 loadv(int m8, int k, int M, int kend) const
    {
        if (m8 >= M || k >= kend) return zero8();
        const int tap = m8 / C, c = m8 - tap * C;
        const int hw = x.H * x.W;
        const int b = k / hw, r = k - b * hw;
        const int y = r / x.W + tap / 3 - 1, xx = r % x.W + tap % 3 - 1;
        if ((unsigned)y >= (unsigned)x.H || (unsigned)xx >= (unsigned)x.W) return zero8();
        return ld8(x.p + ((int64_t)(b * x.H + y) * x.W + xx) * x.cs + x.co + c);
    }
};

// [row8..+7 = channels][k = pixel] of a plain NHWC tensor
struct PlainT {
    static constexpr bool VK = false;
    Act x;
    __device__ uint4 loadv(int n8, int k, int N, int kend) const
    {
        if (n8 >= N || k >= kend) return zero8();
        return ld8(x.p + (int64_t)k * x.cs + x.co + n8);
    }
};

// [n8 = (d, co)][k = low-res pixel] = dY[(b, 2y+dy, 2x+dx)][co]
struct UpGatherT {
    static constexpr bool VK = false;
    Act dy;
    int Cout;
    __device__ uint4 loadv(int n8, int k, int N, int kend) const
    {
        if (n8 >= N || k >= kend) return zero8();
        const int d = n8 / Cout, co = n8 - d * Cout;
        const int h = dy.H >> 1, w = dy.W >> 1;
        const int b = k / (h * w), r = k - b * (h * w);
        const int y = 2 * (r / w) + (d >> 1), xx = 2 * (r % w) + (d & 1);
        return ld8(dy.p + ((int64_t)(b * dy.H + y) * dy.W + xx) * dy.cs + dy.co + co);
    }
};

template <class L, int ROWS>
__device__ inline void stage(const L &ld, bf16_t *s, int row0, int k0, int R, int kend)
{
    constexpr int NV = ROWS * TK / 8;
    if constexpr (L::VK) {
        for (int idx = threadIdx.x; idx < NV; idx += 256) {
            const int r = idx >> 2, kq = (idx & 3) * 8;
            *(uint4 *)&s[r * LDK + kq] = ld.load(row0 + r, k0 + kq, R, kend);
        }
    } else {
        constexpr int R8 = ROWS / 8;
        for (int idx = threadIdx.x; idx < NV; idx += 256) {
            const int k = idx / R8, r8 = (idx - k * R8) * 8;
            const uint4 v = ld.loadv(row0 + r8, k0 + k, R, kend);
            const bf16_t *e = (const bf16_t *)&v;
#pragma unroll
            for (int j = 0; j < 8; ++j) s[(r8 + j) * LDK + k] = e[j];
        }
    }
}

// One workgroup: a TM x TN tile of C over the K range [kz * k_split, (kz+1) * k_split).
template <class AL, class BL, class EP, int TN>
__global__ __launch_bounds__(256) void gemm_kernel(AL A, BL B, EP E, int M, int N, int K, int k_split)
{
    constexpr int WMW = WaveGrid<TN>::WM, WNW = WaveGrid<TN>::WN;
    constexpr int WTM = TM / WMW, WTN = TN / WNW;
    constexpr int BM = WTM / 32, BN = WTN / 32;
    __shared__ __attribute__((aligned(16))) bf16_t sA[TM * LDK];
    __shared__ __attribute__((aligned(16))) bf16_t sB[TN * LDK];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave / WNW, wn = wave % WNW;
    const int m0 = blockIdx.x * TM, n0 = blockIdx.y * TN;
    const int kbeg = blockIdx.z * k_split;
    const int kend = min(K, kbeg + k_split);
    f32x16 acc[BM][BN];
#pragma unroll
    for (int i = 0; i < BM; ++i)
#pragma unroll
        for (int j = 0; j < BN; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;

    for (int k0 = kbeg; k0 < kend; k0 += TK) {
        stage<AL, TM>(A, sA, m0, k0, M, kend);
        stage<BL, TN>(B, sB, n0, k0, N, kend);
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < TK; kk += 16) {
            bf16x8 af[BM], bfr[BN];
#pragma unroll
            for (int i = 0; i < BM; ++i)
                af[i] = *(const bf16x8 *)&sA[(wm * WTM + i * 32 + (lane & 31)) * LDK + kk + 8 * (lane >> 5)];
#pragma unroll
            for (int j = 0; j < BN; ++j)
                bfr[j] = *(const bf16x8 *)&sB[(wn * WTN + j * 32 + (lane & 31)) * LDK + kk + 8 * (lane >> 5)];
#pragma unroll
            for (int i = 0; i < BM; ++i)
#pragma unroll
                for (int j = 0; j < BN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af[i], bfr[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < BM; ++i)
#pragma unroll
        for (int j = 0; j < BN; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int m = m0 + wm * WTM + i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                const int n = n0 + wn * WTN + j * 32 + (lane & 31);
                if (m < M && n < N) E(m, n, acc[i][j][r]);
            }
}

// ---------------------------------------------------------------- epilogues
struct StoreAct {     // y[m][n] = bf16(relu(v + bias[n]))
    bf16_t *y;
    int cs, co;
    const float *bias;
    int relu;
    __device__ void operator()(int m, int n, float v) const
    {
        v += bias[n];
        if (relu) v = fmaxf(v, 0.0f);
        y[(int64_t)m * cs + co + n] = f2bf(v);
    }
};

struct StoreUp {      // n = (d, co): y[(b, 2y+dy, 2x+dx)][co] = bf16(relu(v + bias[co]))
    bf16_t *y;
    int H2, W2, cs, co, Cout;
    const float *bias;
    __device__ void operator()(int m, int n, float v) const
    {
        const int d = n / Cout, c = n - d * Cout;
        const int h = H2 >> 1, w = W2 >> 1;
        const int b = m / (h * w), r = m - b * (h * w);
        const int yy = 2 * (r / w) + (d >> 1), xx = 2 * (r % w) + (d & 1);
        v = fmaxf(v + bias[c], 0.0f);
        y[((int64_t)(b * H2 + yy) * W2 + xx) * cs + co + c] = f2bf(v);
    }
};

struct StoreMasked {  // dx[m][n] = bf16(v) where act[m][n] > 0, else 0
    bf16_t *dx;
    int cs, co;
    const bf16_t *act;
    int acs, aco;
    __device__ void operator()(int m, int n, float v) const
    {
        const float a = bf2f(act[(int64_t)m * acs + aco + n]);
        dx[(int64_t)m * cs + co + n] = f2bf(a > 0.0f ? v : 0.0f);
    }
};

struct StorePartial { // part[kz][m][n] = v
    float *part;
    int M, N;
    __device__ void operator()(int m, int n, float v) const
    {
        part[((int64_t)blockIdx.z * M + m) * N + n] = v;
    }
};

template <class AL, class BL, class EP, int TN>
inline hipError_t run_gemm(const AL &a, const BL &b, const EP &e, int M, int N, int K, int splits, hipStream_t st)
{
    int k_split = (K + splits - 1) / splits;
    k_split = (k_split + TK - 1) / TK * TK;
    splits = (K + k_split - 1) / k_split;
    dim3 grid((M + TM - 1) / TM, (N + TN - 1) / TN, splits);
    gemm_kernel<AL, BL, EP, TN><<<grid, 256, 0, st>>>(a, b, e, M, N, K, k_split);
    return hipGetLastError();
}

}  // namespace cnn
}  // namespace pyhst
