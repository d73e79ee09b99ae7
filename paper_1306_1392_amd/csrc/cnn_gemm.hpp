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

constexpr int TM = 128, TK = 32;

// LDS tiles are [row][k] with k contiguous and no padding; the 16-byte chunk c of row r is stored at
// chunk swz(r, c).  With 32 banks and 8 lanes per 16-byte access, the XOR spreads over all banks the
// MFMA operand reads (8 consecutive rows, one chunk), the row-major staging writes (whole rows) and
// the transposed staging writes (rows 8 apart, one chunk); unswizzled, the last of these hit the same
// 4 banks from every lane of a group.
template <int KV>
__device__ inline int swz(int r, int c)
{
    return c ^ (((r >> 3) ^ (r / (8 / KV))) & (KV - 1));
}

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
    return (uint32_t)(((uint64_t)n * f.m) >> (32 + f.l));   // n < 2^31, m < 2^33: no overflow
}

template <int TN>
struct WaveGrid {
    static constexpr int WM = TN >= 128 ? 2 : 4;
    static constexpr int WN = 4 / WM;
};

// ---------------------------------------------------------------- operand loaders
// Each loader has a per-thread context prepared once per output tile (prep) and a
// load(ctx, k, kend) for every K tile.  VK = true: the context is a row m (or n)
// and load returns [row][k..k+7] (vector along K).  VK = false: the context is a
// group of 8 rows and load returns [row8..row8+7][k] (vector along M or N).
// Channel counts are powers of two (shifts); pixel indices are decoded with FastDiv.
struct Act {          // NHWC activation view: channel stride cs, channel offset co
    const bf16_t *p;
    int B, H, W, cs, co;
};

__device__ inline uint4 ld8(const bf16_t *p) { return *(const uint4 *)p; }
__device__ inline uint4 zero8() { return make_uint4(0, 0, 0, 0); }
__device__ inline int tap_row(int tap) { return (tap * 11) >> 5; }   // tap / 3 for tap in [0, 9)

inline int ilog2(int v)
{
    int l = 0;
    while ((1 << l) < v) ++l;
    return l;
}

// A[m = pixel][k = (tap, c)] = X[pixel + (ty-1, tx-1)][c], zero outside the image
struct Im2colA {
    static constexpr bool VK = true;
    Act x;
    int lgC;
    FastDiv fhw, fw;
    struct Ctx {
        int64_t base;
        int y, xx;
        bool ok;
    };
    __device__ Ctx prep(int m, int M) const
    {
        Ctx c;
        c.ok = m < M;
        const uint32_t mm = c.ok ? (uint32_t)m : 0u;
        const uint32_t b = fdiv(mm, fhw), r = mm - b * fhw.d;
        const uint32_t y = fdiv(r, fw);
        c.y = (int)y;
        c.xx = (int)(r - y * fw.d);
        c.base = (int64_t)mm * x.cs + x.co;
        return c;
    }
    __device__ uint4 load(const Ctx &c, int k, int kend) const
    {
        if (!c.ok || k >= kend) return zero8();
        const int tap = k >> lgC, ch = k & ((1 << lgC) - 1);
        const int ty = tap_row(tap), tx = tap - 3 * ty;
        if ((unsigned)(c.y + ty - 1) >= (unsigned)x.H || (unsigned)(c.xx + tx - 1) >= (unsigned)x.W) return zero8();
        return ld8(x.p + c.base + ((int64_t)(ty - 1) * x.W + (tx - 1)) * x.cs + ch);
    }
};
inline Im2colA im2col_a(Act x, int C) { return Im2colA{x, ilog2(C), make_fastdiv(x.H * x.W), make_fastdiv(x.W)}; }

// A[m = pixel][k] = X[pixel][k]
struct PlainA {
    static constexpr bool VK = true;
    Act x;
    struct Ctx {
        int64_t base;
        bool ok;
    };
    __device__ Ctx prep(int m, int M) const { return Ctx{(int64_t)(m < M ? m : 0) * x.cs + x.co, m < M}; }
    __device__ uint4 load(const Ctx &c, int k, int kend) const
    {
        return (c.ok && k < kend) ? ld8(x.p + c.base + k) : zero8();
    }
};

// A[m = low-res pixel (b,y,x)][k = (d, co)] = dY[(b, 2y+dy, 2x+dx)][co]  (dY at 2h x 2w)
struct UpGatherA {
    static constexpr bool VK = true;
    Act dy;     // high-resolution tensor
    int lgCout;
    FastDiv fhw, fw;   // low-resolution h*w and w
    struct Ctx {
        int64_t base;
        bool ok;
    };
    __device__ Ctx prep(int m, int M) const
    {
        Ctx c;
        c.ok = m < M;
        const uint32_t mm = c.ok ? (uint32_t)m : 0u;
        const uint32_t b = fdiv(mm, fhw), r = mm - b * fhw.d;
        const uint32_t y = fdiv(r, fw), xx = r - y * fw.d;
        c.base = ((int64_t)(b * dy.H + 2 * y) * dy.W + 2 * xx) * dy.cs + dy.co;
        return c;
    }
    __device__ uint4 load(const Ctx &c, int k, int kend) const
    {
        if (!c.ok || k >= kend) return zero8();
        const int d = k >> lgCout, co = k & ((1 << lgCout) - 1);
        return ld8(dy.p + c.base + ((int64_t)(d >> 1) * dy.W + (d & 1)) * dy.cs + co);
    }
};
inline UpGatherA upgather_a(Act dy, int Cout)
{
    return UpGatherA{dy, ilog2(Cout), make_fastdiv((dy.H >> 1) * (dy.W >> 1)), make_fastdiv(dy.W >> 1)};
}

// B[k][n] = Wt[n][k] (weights stored n-major, k contiguous)
struct WeightB {
    static constexpr bool VK = true;
    const bf16_t *w;
    int K;
    struct Ctx {
        int64_t base;
        bool ok;
    };
    __device__ Ctx prep(int n, int N) const { return Ctx{(int64_t)(n < N ? n : 0) * K, n < N}; }
    __device__ uint4 load(const Ctx &c, int k, int kend) const
    {
        return (c.ok && k < kend) ? ld8(w + c.base + k) : zero8();
    }
};

// A[m = (tap, c)][k = pixel] = X[pixel + off(tap)][c]   (weight gradient of a 3x3 conv)
struct Im2colT {
    static constexpr bool VK = false;
    Act x;
    int lgC;
    FastDiv fhw, fw;
    struct Ctx {
        int dy, dx, ch;
        bool ok;
    };
    __device__ Ctx prep(int m8, int M) const
    {
        Ctx c;
        c.ok = m8 < M;
        const int mm = c.ok ? m8 : 0;
        const int tap = mm >> lgC;
        c.ch = mm & ((1 << lgC) - 1);
        c.dy = tap_row(tap) - 1;
        c.dx = tap - 3 * (c.dy + 1) - 1;
        return c;
    }
    __device__ uint4 load(const Ctx &c, int k, int kend) const
    {
        if (!c.ok || k >= kend) return zero8();
        const uint32_t b = fdiv((uint32_t)k, fhw), r = (uint32_t)k - b * fhw.d;
        const uint32_t y0 = fdiv(r, fw);
        const int y = (int)y0 + c.dy, xx = (int)(r - y0 * fw.d) + c.dx;
        if ((unsigned)y >= (unsigned)x.H || (unsigned)xx >= (unsigned)x.W) return zero8();
        return ld8(x.p + ((int64_t)(b * x.H + y) * x.W + xx) * x.cs + x.co + c.ch);
    }
    // pixels k .. k+7: one division for the first, then the pixel walks along its row
    __device__ void load8(const Ctx &c, int k, int kend, uint4 *v) const
    {
        const uint32_t k0 = (uint32_t)min(k, kend);
        uint32_t b = fdiv(k0, fhw), r = k0 - b * fhw.d;
        uint32_t y = fdiv(r, fw), xx = r - y * fw.d;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int yy = (int)y + c.dy, xs = (int)xx + c.dx;
            const bool in = c.ok && k + i < kend && (unsigned)yy < (unsigned)x.H && (unsigned)xs < (unsigned)x.W;
            v[i] = in ? ld8(x.p + ((int64_t)(b * x.H + yy) * x.W + xs) * x.cs + x.co + c.ch) : zero8();
            if (++xx == (uint32_t)x.W) {
                xx = 0;
                if (++y == (uint32_t)x.H) {
                    y = 0;
                    ++b;
                }
            }
        }
    }
};
inline Im2colT im2col_t(Act x, int C) { return Im2colT{x, ilog2(C), make_fastdiv(x.H * x.W), make_fastdiv(x.W)}; }

// [row8..+7 = channels][k = pixel] of a plain NHWC tensor
struct PlainT {
    static constexpr bool VK = false;
    Act x;
    struct Ctx {
        int off;
        bool ok;
    };
    __device__ Ctx prep(int n8, int N) const { return Ctx{x.co + (n8 < N ? n8 : 0), n8 < N}; }
    __device__ uint4 load(const Ctx &c, int k, int kend) const
    {
        return (c.ok && k < kend) ? ld8(x.p + (int64_t)k * x.cs + c.off) : zero8();
    }
    __device__ void load8(const Ctx &c, int k, int kend, uint4 *v) const
    {
        const bf16_t *q = x.p + (int64_t)k * x.cs + c.off;
#pragma unroll
        for (int i = 0; i < 8; ++i) v[i] = (c.ok && k + i < kend) ? ld8(q + (int64_t)i * x.cs) : zero8();
    }
};

// [n8 = (d, co)][k = low-res pixel] = dY[(b, 2y+dy, 2x+dx)][co]
struct UpGatherT {
    static constexpr bool VK = false;
    Act dy;
    int lgCout;
    FastDiv fhw, fw;
    struct Ctx {
        int ddy, ddx, co;
        bool ok;
    };
    __device__ Ctx prep(int n8, int N) const
    {
        Ctx c;
        c.ok = n8 < N;
        const int nn = c.ok ? n8 : 0;
        const int d = nn >> lgCout;
        c.co = nn & ((1 << lgCout) - 1);
        c.ddy = d >> 1;
        c.ddx = d & 1;
        return c;
    }
    __device__ uint4 load(const Ctx &c, int k, int kend) const
    {
        if (!c.ok || k >= kend) return zero8();
        const uint32_t b = fdiv((uint32_t)k, fhw), r = (uint32_t)k - b * fhw.d;
        const uint32_t y = fdiv(r, fw), xx = r - y * fw.d;
        return ld8(dy.p + ((int64_t)(b * dy.H + 2 * y + c.ddy) * dy.W + 2 * xx + c.ddx) * dy.cs + dy.co + c.co);
    }
    __device__ void load8(const Ctx &c, int k, int kend, uint4 *v) const
    {
        const uint32_t k0 = (uint32_t)min(k, kend);
        const uint32_t h = fhw.d / fw.d, w = fw.d;
        uint32_t b = fdiv(k0, fhw), r = k0 - b * fhw.d;
        uint32_t y = fdiv(r, fw), xx = r - y * w;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            v[i] = (c.ok && k + i < kend)
                       ? ld8(dy.p + ((int64_t)(b * dy.H + 2 * y + c.ddy) * dy.W + 2 * xx + c.ddx) * dy.cs + dy.co + c.co)
                       : zero8();
            if (++xx == w) {
                xx = 0;
                if (++y == h) {
                    y = 0;
                    ++b;
                }
            }
        }
    }
};
inline UpGatherT upgather_t(Act dy, int Cout)
{
    return UpGatherT{dy, ilog2(Cout), make_fastdiv((dy.H >> 1) * (dy.W >> 1)), make_fastdiv(dy.W >> 1)};
}

// 8 x 8 transpose of 16-bit elements: out[q] element i = in[i] element q
__device__ inline void transpose8(const uint4 *in, uint4 *out)
{
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        uint32_t w[4];
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            const uint32_t a = ((const uint32_t *)&in[2 * d])[q >> 1], b = ((const uint32_t *)&in[2 * d + 1])[q >> 1];
            w[d] = (q & 1) ? ((a >> 16) | (b & 0xffff0000u)) : ((a & 0xffffu) | (b << 16));
        }
        out[q] = make_uint4(w[0], w[1], w[2], w[3]);
    }
}

// Register staging of one operand tile, stored in LDS as [row][k] (k contiguous, chunks swizzled).
//  VK loaders: SLOTS vectors of 8 consecutive k of one row per thread.
//  Other loaders (vectors run along the rows): each of the first ROWS/8 * TK/8 threads loads an
//  8-row x 8-k block as 8 vectors (one per k), transposes it in registers and stores 8 vectors.
template <class L, int ROWS, int TKv = TK, bool VK = L::VK>
struct Stager;

template <class L, int ROWS, int TKv>
struct Stager<L, ROWS, TKv, true> {
    static constexpr int KV = TKv / 8, LDKv = TKv;
    static constexpr int NV = ROWS * KV;
    static constexpr int SLOTS = (NV + 255) / 256;
    typename L::Ctx ctx[SLOTS];
    uint4 v[SLOTS];
    int row[SLOTS], kl[SLOTS];
    __device__ void prep(const L &ld, int row0, int R, int = 0)
    {
#pragma unroll
        for (int j = 0; j < SLOTS; ++j) {
            const int idx = threadIdx.x + 256 * j;
            row[j] = idx / KV;
            kl[j] = (idx % KV) * 8;
            ctx[j] = ld.prep(row0 + row[j], idx < NV ? R : 0);
        }
    }
    __device__ void load(const L &ld, int k0, int kend)
    {
#pragma unroll
        for (int j = 0; j < SLOTS; ++j) v[j] = ld.load(ctx[j], k0 + kl[j], kend);
    }
    __device__ void store(bf16_t *s) const
    {
#pragma unroll
        for (int j = 0; j < SLOTS; ++j)
            if (threadIdx.x + 256 * j < NV) *(uint4 *)&s[row[j] * LDKv + 8 * swz<KV>(row[j], kl[j] >> 3)] = v[j];
    }
};

template <class L, int ROWS, int TKv>
struct Stager<L, ROWS, TKv, false> {
    static constexpr int R8 = ROWS / 8, KV = TKv / 8, NBLK = R8 * KV, LDKv = TKv;
    static_assert(NBLK <= 256, "one 8x8 block per thread");
    typename L::Ctx ctx;
    uint4 v[8];
    int row, kl;
    bool act;
    // the first NBLK threads load (measured faster than spreading the blocks over all four waves)
    __device__ void prep(const L &ld, int row0, int R, int = 0)
    {
        act = threadIdx.x < NBLK;
        kl = (threadIdx.x / R8) * 8;
        row = (threadIdx.x % R8) * 8;
        ctx = ld.prep(row0 + row, act ? R : 0);
    }
    __device__ void load(const L &ld, int k0, int kend)
    {
        if (act) ld.load8(ctx, k0 + kl, kend, v);
    }
    __device__ void store(bf16_t *s) const
    {
        if (!act) return;
        uint4 o[8];
        transpose8(v, o);
#pragma unroll
        for (int q = 0; q < 8; ++q) *(uint4 *)&s[(row + q) * LDKv + 8 * swz<KV>(row + q, kl >> 3)] = o[q];
    }
};

// One workgroup: a TM x TN tile of C over the K range [kz * k_split, (kz+1) * k_split).
// The next K tile is fetched into registers while the current one is multiplied from
// LDS; two LDS buffers, one barrier per K tile.
// Row-major A loaders (forward and backward-data convolutions) fit 4 waves per SIMD with the
// accumulators in VGPRs; the transposed loaders of the weight gradients would spill there.
template <class AL, class BL, class EP, int TN, int TMv = TM, int TKv = TK>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(AL::VK ? 4 : 1)))
void gemm_kernel(AL A, BL B, EP E, int M, int N, int K, int k_split)
{
    constexpr int LDKv = TKv, KV = TKv / 8;
    constexpr int WMW = WaveGrid<TN>::WM, WNW = WaveGrid<TN>::WN;
    constexpr int WTM = TMv / WMW, WTN = TN / WNW;
    constexpr int BM = WTM / 32, BN = WTN / 32;
    __shared__ __attribute__((aligned(16))) bf16_t sA[2][TMv * LDKv];
    __shared__ __attribute__((aligned(16))) bf16_t sB[2][TN * LDKv];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave / WNW, wn = wave % WNW;
    const int m0 = blockIdx.x * TMv, n0 = blockIdx.y * TN;
    const int kbeg = blockIdx.z * k_split;
    const int kend = min(K, kbeg + k_split);
    f32x16 acc[BM][BN];
#pragma unroll
    for (int i = 0; i < BM; ++i)
#pragma unroll
        for (int j = 0; j < BN; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;

    Stager<AL, TMv, TKv> ga;
    Stager<BL, TN, TKv> gb;
    ga.prep(A, m0, M, 0);
    gb.prep(B, n0, N, 1);
    if (kbeg < kend) {
        ga.load(A, kbeg, kend);
        gb.load(B, kbeg, kend);
    }
    int buf = 0;
    for (int k0 = kbeg; k0 < kend; k0 += TKv, buf ^= 1) {
        ga.store(sA[buf]);
        gb.store(sB[buf]);
        __syncthreads();
        if (k0 + TKv < kend) {
            ga.load(A, k0 + TKv, kend);
            gb.load(B, k0 + TKv, kend);
        }
        const bf16_t *a = sA[buf], *bsm = sB[buf];
#pragma unroll
        for (int kk = 0; kk < TKv; kk += 16) {
            bf16x8 af[BM], bfr[BN];
#pragma unroll
            for (int i = 0; i < BM; ++i)
            {
                const int r = wm * WTM + i * 32 + (lane & 31);
                af[i] = *(const bf16x8 *)&a[r * LDKv + 8 * swz<KV>(r, (kk >> 3) + (lane >> 5))];
            }
#pragma unroll
            for (int j = 0; j < BN; ++j)
            {
                const int r = wn * WTN + j * 32 + (lane & 31);
                bfr[j] = *(const bf16x8 *)&bsm[r * LDKv + 8 * swz<KV>(r, (kk >> 3) + (lane >> 5))];
            }
#pragma unroll
            for (int i = 0; i < BM; ++i)
#pragma unroll
                for (int j = 0; j < BN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af[i], bfr[j], acc[i][j], 0, 0, 0);
        }
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
    int H2, W2, cs, co, lgCout;
    FastDiv fhw, fw;      // low-resolution h*w and w
    const float *bias;
    __device__ void operator()(int m, int n, float v) const
    {
        const int d = n >> lgCout, c = n & ((1 << lgCout) - 1);
        const uint32_t b = fdiv((uint32_t)m, fhw), r = (uint32_t)m - b * fhw.d;
        const uint32_t yl = fdiv(r, fw), xl = r - yl * fw.d;
        const int yy = 2 * (int)yl + (d >> 1), xx = 2 * (int)xl + (d & 1);
        v = fmaxf(v + bias[c], 0.0f);
        y[((int64_t)(b * H2 + yy) * W2 + xx) * cs + co + c] = f2bf(v);
    }
};
inline StoreUp store_up(bf16_t *y, int H2, int W2, int cs, int co, int Cout, const float *bias)
{
    return StoreUp{y, H2, W2, cs, co, ilog2(Cout), make_fastdiv((H2 >> 1) * (W2 >> 1)), make_fastdiv(W2 >> 1), bias};
}

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

template <class AL, class BL, class EP, int TN, int TMv = TM>
inline hipError_t run_gemm(const AL &a, const BL &b, const EP &e, int M, int N, int K, int splits, hipStream_t st)
{
    int k_split = (K + splits - 1) / splits;
    k_split = (k_split + TK - 1) / TK * TK;
    splits = (K + k_split - 1) / k_split;
    dim3 grid((M + TMv - 1) / TMv, (N + TN - 1) / TN, splits);
    gemm_kernel<AL, BL, EP, TN, TMv><<<grid, 256, 0, st>>>(a, b, e, M, N, K, k_split);
    return hipGetLastError();
}

}  // namespace cnn
}  // namespace pyhst
