// Direct 3x3 convolution (zero padding 1, stride 1) on the MFMA BF16 units, for the U-Net layers:
//   C[m = pixel][n] = sum_{tap, c} X[pixel + (ty - 1, tx - 1)][c] W[n][tap CIN + c]
// the same sums as the implicit GEMM of cnn_gemm.hpp (Im2colA x WeightB), with the input read
// once per output tile instead of once per tap.
//
// Output tile = CTH x CT_W = 4 or 8 x 32 pixels of one image (one 32-pixel MFMA block per tile row) x
// TN output channels.  The tile's input patch, (CTH + 2) x (CT_W + 2) pixels with zeros outside the
// image, and the weights of the TN outputs are staged in LDS; the MFMA K steps of the nine taps then
// read the patch at shifted positions.  The weights are the MFMA A operand and the patch the B
// operand, so each lane's accumulators hold four groups of four consecutive output channels of one
// pixel (8-byte stores, bias and ReLU on four values at a time).  Every LDS address of a step is a
// per-lane base plus a compile-time offset (the steps are unrolled).
// Two forms (run_conv3x3 picks): a persistent one that keeps its outputs' weights in LDS and streams
// the patches of many tiles (layers whose weights for TN outputs fit), and a general one that stages
// patch and weights per chunk of input channels, the next chunk loaded into registers meanwhile.
// K order: chunk, tap, channel within the chunk; with one chunk that is the GEMM's k = tap CIN + c.
//
// LDS layouts: patch pixel p = py (CT_W + 2) + px at 16-byte slots p CPP + chunk, CPP = CPX | 1 odd,
// so the 8 lanes of a pass (8 consecutive pixels, one chunk) fall in 8 distinct four-bank groups;
// weights of output n at slots n WS + tap CPX + chunk, WS = 1 mod 8 for the same reason.
#pragma once

#include <algorithm>
#include <type_traits>
#include <utility>

#include "cnn_gemm.hpp"

namespace pyhst {
namespace cnn {

constexpr int CT_W = 32, CT_PW = CT_W + 2;   // tile width; patch width

// wave layout of a CTH x 32-pixel, TN-channel tile: WM x WN wavefronts, each with BM row blocks (tile
// rows) and BN column blocks of 32 (8-row tiles: four wavefronts of two rows and every column, so an
// operand read from LDS serves BN or two MFMAs)
template <int TN, int CTH>
struct ConvGrid {
    static constexpr int WM = CTH >= 8 ? 4 : WaveGrid<TN>::WM, WN = 4 / WM;
    static constexpr int BM = CTH / WM, BN = TN / WN / 32, WTN = TN / WN;
    static constexpr int PIX = (CTH + 2) * CT_PW;   // patch pixels
    static_assert(CTH % WM == 0, "whole tile rows per wavefront");
};

// weight row stride in 16-byte slots: at least 9 CPX and 1 mod 8, so 8 consecutive output channels
// (the lanes of a pass of a B operand read) fall in 8 distinct four-bank groups
constexpr int conv_ws(int cpx)
{
    int s = 9 * cpx;
    while (s % 8 != 1) ++s;
    return s;
}

// Output tile t of an image batch: image b, first row y0, first column x0.
struct ConvTile {
    int b, y0, x0;
};
template <int CTH>
__device__ inline ConvTile conv_tile(const Act &x, int t)
{
    const int tiles_x = (x.W + CT_W - 1) / CT_W, tiles_y = (x.H + CTH - 1) / CTH;
    const int b = t / (tiles_x * tiles_y), r = t - b * tiles_x * tiles_y;
    return ConvTile{b, (r / tiles_x) * CTH, (r % tiles_x) * CT_W};
}

// ---- persistent form --------------------------------------------------------------------------
// Patch layout of the persistent form: pixel p at slots p CPP .. p CPP + CPX - 1, CPP = CPX | 1 (odd),
// so 8 consecutive pixels at one chunk fall in 8 distinct four-bank groups and every operand address
// is a per-lane base plus a compile-time offset.
__device__ inline uint32_t pack_bf16x2(float a, float b)   // round to nearest even (v_cvt_pk_bf16_f32)
{
    typedef float f2 __attribute__((ext_vector_type(2)));
    typedef __bf16 b2 __attribute__((ext_vector_type(2)));
    const b2 r = __builtin_convertvector((f2){a, b}, b2);
    uint32_t u;
    __builtin_memcpy(&u, &r, 4);
    return u;
}

// Epilogues.  pack4 turns the accumulators of four consecutive output channels n .. n + 3 of output
// pixel m into four BF16 values (ok: m and n are inside the output; an epilogue that reads memory reads
// only then); store8 writes eight consecutive channels n .. n + 7 of pixel m (16 bytes).  POOL: the
// epilogue also writes the 2x2 max pool of its output; HEAD: it applies the network's 1x1 head.
struct ConvStoreAct {    // y = bf16(relu(v + bias))
    static constexpr bool BIAS = true, POOL = false, HEAD = false;
    bf16_t *y;
    int cs, co;
    const float *bias;
    __device__ uint2 pack4(int, int, const float *v, const float4 &b, bool) const
    {
        return make_uint2(pack_bf16x2(fmaxf(v[0] + b.x, 0.0f), fmaxf(v[1] + b.y, 0.0f)),
                          pack_bf16x2(fmaxf(v[2] + b.z, 0.0f), fmaxf(v[3] + b.w, 0.0f)));
    }
    __device__ void store8(int m, int n, const uint4 &o) const { *(uint4 *)(y + (int64_t)m * cs + co + n) = o; }
};
// y as ConvStoreAct and its 2x2 max pool: pool[(b, yy / 2, xx / 2)][n] (channel stride pcs)
struct ConvStoreActPool : ConvStoreAct {
    static constexpr bool POOL = true;
    bf16_t *pool;
    int pcs;
};
// the head on the activation a = bf16(relu(v + bias)) of every channel (all in one workgroup):
// r = scale xin + (bh + sum_n wh[n] a[n]); out = r / scale (unscale) or r.  y (when not null) also
// receives a, for the backward pass.
struct ConvStoreHead : ConvStoreAct {
    static constexpr bool HEAD = true;
    const float *wh, *bh, *xin;
    float *out;
    float scale;
    int unscale;
};
struct ConvStoreMasked { // dx = bf16(v) where act > 0, else 0
    static constexpr bool BIAS = false, POOL = false, HEAD = false;
    bf16_t *dx;
    int cs, co;
    const bf16_t *act;
    int acs, aco;
    const float *bias;   // unused
    __device__ uint2 pack4(int m, int n, const float *v, const float4 &, bool ok) const
    {
        const uint2 a = ok ? *(const uint2 *)(act + (int64_t)m * acs + aco + n) : make_uint2(0u, 0u);
        float o[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint32_t h = ((q & 2) ? a.y : a.x) >> (16 * (q & 1));
            const uint32_t mag = h & 0x7fffu;
            o[q] = !(h & 0x8000u) && mag != 0 && mag <= 0x7f80u ? v[q] : 0.0f;   // act > 0 (BF16 bits)
        }
        return make_uint2(pack_bf16x2(o[0], o[1]), pack_bf16x2(o[2], o[3]));
    }
    __device__ void store8(int m, int n, const uint4 &o) const { *(uint4 *)(dx + (int64_t)m * cs + co + n) = o; }
};

// Lanes l and l + 32 (half-waves 0 and 1) hold channels 8 g + 4 half .. + 3 (a) and 8 (g + 1) + 4 half
// .. + 3 (b) of one pixel.  v_permlane32_swap exchanges lanes 32..63 of its first operand with lanes 0..31
// of its second, after which lane half h holds the eight channels 8 (g + h) .. + 7 (16 bytes).
__device__ __forceinline__ uint4 gather8(uint2 a, uint2 b)
{
    const auto x = __builtin_amdgcn_permlane32_swap(a.x, b.x, false, false);
    const auto y = __builtin_amdgcn_permlane32_swap(a.y, b.y, false, false);
    return make_uint4(x[0], y[0], x[1], y[1]);
}

// One MFMA K step S (16 K values) of the persistent form: weights as the A operand, the patch as the
// B operand, so accumulator register r holds output channel 8 (r / 4) + 4 (lane / 32) + r % 4 of
// pixel lane % 32.  la[i]: patch slot of this lane's pixel in row block i (plus its half of the step's
// channels when CIN >= 16); lw[j]: weight slot of its output channel in column block j (likewise).
template <int CIN, int TN, int CTH, int S>
__device__ __forceinline__ void pconv_step(const uint4 *sP, const uint4 *sW, const int *la, const int *lw, int half,
                                           f32x16 (&acc)[ConvGrid<TN, CTH>::BN][ConvGrid<TN, CTH>::BM])
{
    constexpr int CPX = CIN / 8, CPP = CPX | 1;
    constexpr int BM = ConvGrid<TN, CTH>::BM, BN = ConvGrid<TN, CTH>::BN;
    int oa, ow;
    bool live = true;
    if constexpr (CIN >= 16) {    // both halves of the step read one tap
        constexpr int tap = (16 * S) / CIN, c8 = ((16 * S) % CIN) / 8;
        oa = ((tap / 3) * CT_PW + tap % 3) * CPP + c8;
        ow = tap * CPX + c8;
    } else {                      // CIN == 8: the halves read taps 2S and 2S + 1
        constexpr int t0 = 2 * S, t1 = 2 * S + 1;
        oa = half ? ((t1 / 3) * CT_PW + t1 % 3) : ((t0 / 3) * CT_PW + t0 % 3);
        ow = half ? t1 : t0;
        live = !(half && t1 >= 9);
    }
    bf16x8 wf[BN], pf[BM];
#pragma unroll
    for (int j = 0; j < BN; ++j) {
        const uint4 v = live ? sW[lw[j] + ow] : zero8();
        wf[j] = *(const bf16x8 *)&v;
    }
#pragma unroll
    for (int i = 0; i < BM; ++i) {
        const uint4 v = live ? sP[la[i] + oa] : zero8();
        pf[i] = *(const bf16x8 *)&v;
    }
#pragma unroll
    for (int j = 0; j < BN; ++j)
#pragma unroll
        for (int i = 0; i < BM; ++i)
            acc[j][i] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wf[j], pf[i], acc[j][i], 0, 0, 0);
}

template <int CIN, int TN, int CTH, int... S>
__device__ __forceinline__ void pconv_steps(std::integer_sequence<int, S...>, const uint4 *sP, const uint4 *sW,
                                            const int *la, const int *lw, int half,
                                            f32x16 (&acc)[ConvGrid<TN, CTH>::BN][ConvGrid<TN, CTH>::BM])
{
    (pconv_step<CIN, TN, CTH, S>(sP, sW, la, lw, half, acc), ...);
}

// max of two packed pairs of BF16 values from a ReLU (compared as floats, so -0 and +0 tie)
__device__ __forceinline__ uint32_t max_bf16x2(uint32_t a, uint32_t b)
{
    const float lo = fmaxf(__uint_as_float(a << 16), __uint_as_float(b << 16));
    const float hi = fmaxf(__uint_as_float(a & 0xffff0000u), __uint_as_float(b & 0xffff0000u));
    return (__float_as_uint(lo) >> 16) | (__float_as_uint(hi) & 0xffff0000u);
}
// the value held by lane ^ 1 (DPP quad permutation 1, 0, 3, 2)
__device__ __forceinline__ uint32_t from_lane_xor1(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, false);
}
__device__ __forceinline__ float bf16_lo(uint32_t u) { return __uint_as_float(u << 16); }
__device__ __forceinline__ float bf16_hi(uint32_t u) { return __uint_as_float(u & 0xffff0000u); }

// Epilogue of one output tile, shared by both forms: accumulator register 4 g + q of column block j,
// row block i holds output channel 8 g + 4 (lane / 32) + q of the block, pixel lane % 32.  Groups g, g + 1
// are packed, exchanged between the half-waves (gather8) and stored as 16 bytes per lane; every lane
// takes part in the exchanges, and only the stores test the bounds (N is a multiple of 8).
// POOL: the two row blocks of a wavefront are the two rows of its pooling windows (the tile and the image
// start on even rows, H and W are even) and lanes col, col ^ 1 the two columns.  HEAD: the wavefront
// holds every channel of its pixels (one workgroup column, WN = 1), half of them in each half-wave.
template <class G_, class EP>
__device__ __forceinline__ void pconv_store(const Act &x, const ConvTile &c, int n0, int N, int wm, int wn, int col,
                                            int half, const EP &E, const float4 *sBias, const float4 *sHead,
                                            f32x16 (&acc)[G_::BN][G_::BM])
{
    constexpr int BM = G_::BM, BN = G_::BN, WTN = G_::WTN;
    const int xx = c.x0 + col;
    if constexpr (EP::POOL) {
        static_assert(BM % 2 == 0, "both rows of every pooling window in one wavefront");
#pragma unroll
        for (int ip = 0; ip < BM; ip += 2) {
        const int yy = c.y0 + wm * BM + ip;
        const bool in = yy < x.H && xx < x.W;   // alike for the lanes of a window (even W) and both half-waves
        const int m = (c.b * x.H + yy) * x.W + xx;
        const int64_t pm = ((int64_t)(c.b * (x.H >> 1) + (yy >> 1)) * (x.W >> 1) + (xx >> 1)) * E.pcs;
#pragma unroll
        for (int j = 0; j < BN; ++j)
#pragma unroll
            for (int g = 0; g < 4; g += 2) {
                const int nb = wn * WTN + j * 32 + 8 * g, nl0 = nb + 4 * half, nl1 = nl0 + 8;
                uint2 r[2][2];
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const int nl = h ? nl1 : nl0;
                        const float v[4] = {acc[j][ip + i][4 * (g + h)], acc[j][ip + i][4 * (g + h) + 1],
                                            acc[j][ip + i][4 * (g + h) + 2], acc[j][ip + i][4 * (g + h) + 3]};
                        r[i][h] = E.pack4(m + i * x.W, n0 + nl, v, sBias[nl >> 2], in && n0 + nl < N);
                    }
                uint2 pool[2];
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    uint32_t px = max_bf16x2(r[0][h].x, r[1][h].x), py = max_bf16x2(r[0][h].y, r[1][h].y);
                    px = max_bf16x2(px, from_lane_xor1(px));
                    py = max_bf16x2(py, from_lane_xor1(py));
                    pool[h] = make_uint2(px, py);
                }
                const uint4 o0 = gather8(r[0][0], r[0][1]), o1 = gather8(r[1][0], r[1][1]);
                const uint4 op = gather8(pool[0], pool[1]);
                const int nc = n0 + nb + 8 * half;
                if (in && nc < N) {
                    E.store8(m, nc, o0);
                    E.store8(m + x.W, nc, o1);
                    if (!(col & 1)) *(uint4 *)(E.pool + pm + nc) = op;
                }
            }
        }
        return;
    }
#pragma unroll
    for (int i = 0; i < BM; ++i) {
        const int yy = c.y0 + wm * BM + i;
        const bool in = yy < x.H && xx < x.W;   // alike in both half-waves (same pixel)
        const int m = in ? (c.b * x.H + yy) * x.W + xx : 0;
        float s = 0.0f;   // HEAD: this half-wave's share of the head's sum
#pragma unroll
        for (int j = 0; j < BN; ++j)
#pragma unroll
            for (int g = 0; g < 4; g += 2) {
                const int nb = wn * WTN + j * 32 + 8 * g;
                uint2 r[2];
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int nl = nb + 8 * h + 4 * half;
                    const float v[4] = {acc[j][i][4 * (g + h)], acc[j][i][4 * (g + h) + 1], acc[j][i][4 * (g + h) + 2],
                                        acc[j][i][4 * (g + h) + 3]};
                    const float4 bb = EP::BIAS ? sBias[nl >> 2] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                    r[h] = E.pack4(m, n0 + nl, v, bb, in && n0 + nl < N);
                    if constexpr (EP::HEAD) {
                        const float4 w = sHead[nl >> 2];   // zero beyond N
                        s = fmaf(bf16_lo(r[h].x), w.x, s);
                        s = fmaf(bf16_hi(r[h].x), w.y, s);
                        s = fmaf(bf16_lo(r[h].y), w.z, s);
                        s = fmaf(bf16_hi(r[h].y), w.w, s);
                    }
                }
                bool keep = true;
                if constexpr (EP::HEAD) keep = E.y != nullptr;
                if (keep) {
                    const uint4 o = gather8(r[0], r[1]);
                    const int nc = n0 + nb + 8 * half;
                    if (in && nc < N) E.store8(m, nc, o);
                }
            }
        if constexpr (EP::HEAD) {
            static_assert(G_::WN == 1, "every channel of a pixel in one wavefront");
            s += __shfl_xor(s, 32, 64);   // the other half-wave's channels (a + b = b + a: both halves agree)
            if (in && !half) {
                const float r = E.xin[m] * E.scale + (E.bh[0] + s);
                E.out[m] = E.unscale ? r / E.scale : r;
            }
        }
    }
}

// One MFMA K step S of the persistent form, whose weight operands wr[S][j] are held in registers: only
// the patch operands come from LDS (one read per MFMA when BM = 1).
template <int CIN, int TN, int CTH, int NSTEP, int S>
__device__ __forceinline__ void rconv_step(const uint4 *sP, const int *la, int half,
                                           const uint4 (&wr)[NSTEP][ConvGrid<TN, CTH>::BN],
                                           f32x16 (&acc)[ConvGrid<TN, CTH>::BN][ConvGrid<TN, CTH>::BM])
{
    constexpr int CPX = CIN / 8, CPP = CPX | 1;
    constexpr int BM = ConvGrid<TN, CTH>::BM, BN = ConvGrid<TN, CTH>::BN;
    int oa;
    bool live = true;
    if constexpr (CIN >= 16) {    // both halves of the step read one tap
        constexpr int tap = (16 * S) / CIN, c8 = ((16 * S) % CIN) / 8;
        oa = ((tap / 3) * CT_PW + tap % 3) * CPP + c8;
    } else {                      // CIN == 8: the halves read taps 2S and 2S + 1
        constexpr int t0 = 2 * S, t1 = 2 * S + 1;
        oa = half ? ((t1 / 3) * CT_PW + t1 % 3) : ((t0 / 3) * CT_PW + t0 % 3);
        live = !(half && t1 >= 9);
    }
    bf16x8 pf[BM];
#pragma unroll
    for (int i = 0; i < BM; ++i) {
        const uint4 v = live ? sP[la[i] + oa] : zero8();
        pf[i] = *(const bf16x8 *)&v;
    }
#pragma unroll
    for (int j = 0; j < BN; ++j) {
        const bf16x8 wf = *(const bf16x8 *)&wr[S][j];
#pragma unroll
        for (int i = 0; i < BM; ++i) acc[j][i] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wf, pf[i], acc[j][i], 0, 0, 0);
    }
}

template <int CIN, int TN, int CTH, int NSTEP, int... S>
__device__ __forceinline__ void rconv_steps(std::integer_sequence<int, S...>, const uint4 *sP, const int *la, int half,
                                            const uint4 (&wr)[NSTEP][ConvGrid<TN, CTH>::BN],
                                            f32x16 (&acc)[ConvGrid<TN, CTH>::BN][ConvGrid<TN, CTH>::BM])
{
    (rconv_step<CIN, TN, CTH, NSTEP, S>(sP, la, half, wr, acc), ...);
}

// Persistent form for layers whose weights for TN outputs fit in registers (TN x 9 x CIN <= 20480
// values: at most 144 VGPRs per lane): every lane loads the weight operands of its K steps and column
// blocks once, straight from memory, and the workgroup then walks output tiles blockIdx.x,
// blockIdx.x + gridDim.x, ...; the patches of the next two tiles are in flight in registers while the
// current one is summed from LDS.  One chunk, K steps in the GEMM's order k = tap CIN + c.
template <int CIN, int TN, int CTH, class EP>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
void conv3x3_persist_kernel(Act x, WeightB B, EP E, int N, int tiles)
{
    using G_ = ConvGrid<TN, CTH>;
    constexpr int CPX = CIN / 8, CPP = CPX | 1;
    constexpr int NPS = G_::PIX * CPX;            // patch vectors
    constexpr int NPV = (NPS + 255) / 256;        // patch vectors per thread
    constexpr int NSTEP = (9 * CIN + 15) / 16;
    constexpr int WNW = G_::WN, BM = G_::BM, BN = G_::BN, WTN = G_::WTN;
    static_assert(TN * 9 * CIN <= 20480, "weights of the workgroup's outputs fit in registers");
    __shared__ uint4 sP[G_::PIX * CPP];
    __shared__ float4 sBias[TN / 4];
    __shared__ float4 sHead[EP::HEAD ? TN / 4 : 1];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave / WNW, wn = wave % WNW;
    const int col = lane & 31, half = lane >> 5;
    const int n0 = blockIdx.y * TN;
    // A operand of step S, column block j: output n0 + wn WTN + 32 j + col, K values 16 S + 8 half .. + 7
    uint4 wr[NSTEP][BN];
#pragma unroll
    for (int S = 0; S < NSTEP; ++S)
#pragma unroll
        for (int j = 0; j < BN; ++j) {
            const int n = n0 + wn * WTN + 32 * j + col, k = 16 * S + 8 * half;
            wr[S][j] = n < N && k < 9 * CIN ? ld8(B.w + (int64_t)n * B.K + k) : zero8();
        }
    if (EP::BIAS && threadIdx.x < TN) ((float *)sBias)[threadIdx.x] = n0 + (int)threadIdx.x < N ? E.bias[n0 + threadIdx.x] : 0.0f;
    if constexpr (EP::HEAD)
        if (threadIdx.x < TN) ((float *)sHead)[threadIdx.x] = n0 + (int)threadIdx.x < N ? E.wh[n0 + threadIdx.x] : 0.0f;
    // this thread's patch vectors, the same for every tile: pixel (py, px), chunk c8, LDS slot
    int spos[NPV], sdst[NPV];
#pragma unroll
    for (int v = 0; v < NPV; ++v) {
        const int i = threadIdx.x + 256 * v;
        const int p = i / CPX, c8 = i - p * CPX, py = p / CT_PW, px = p - py * CT_PW;
        spos[v] = i < NPS ? (py << 16) | (px << 8) | c8 : -1;
        sdst[v] = p * CPP + c8;
    }
    // two patches in flight: the patch of tile t + 2 G (G = gridDim.x) is loaded into the registers
    // that held tile t's once those are in LDS, while tile t is summed
    uint4 pa[NPV], pb[NPV];
    auto load = [&](uint4 (&pv)[NPV], int t) {
        if (t >= tiles) return;
        const ConvTile c = conv_tile<CTH>(x, t);
        const bf16_t *img = x.p + (int64_t)c.b * x.H * x.W * x.cs + x.co;
#pragma unroll
        for (int v = 0; v < NPV; ++v) {
            const int yy = c.y0 - 1 + (spos[v] >> 16), xx = c.x0 - 1 + ((spos[v] >> 8) & 255);
            pv[v] = spos[v] >= 0 && (unsigned)yy < (unsigned)x.H && (unsigned)xx < (unsigned)x.W
                        ? ld8(img + (int64_t)(yy * x.W + xx) * x.cs + 8 * (spos[v] & 255))
                        : zero8();
        }
    };
    int la[BM];
#pragma unroll
    for (int i = 0; i < BM; ++i) la[i] = ((wm * BM + i) * CT_PW + col) * CPP + (CIN >= 16 ? half : 0);

    auto tile = [&](uint4 (&pv)[NPV], int t) {
        __syncthreads();   // the previous tile's reads of the patch are done (the biases are visible)
#pragma unroll
        for (int v = 0; v < NPV; ++v)
            if (spos[v] >= 0) sP[sdst[v]] = pv[v];
        __syncthreads();
        load(pv, t + 2 * (int)gridDim.x);   // in flight while this tile and the next are summed
        f32x16 acc[BN][BM];
#pragma unroll
        for (int j = 0; j < BN; ++j)
#pragma unroll
            for (int i = 0; i < BM; ++i)
#pragma unroll
                for (int q = 0; q < 16; ++q) acc[j][i][q] = 0.0f;
        rconv_steps<CIN, TN, CTH, NSTEP>(std::make_integer_sequence<int, NSTEP>{}, sP, la, half, wr, acc);
        pconv_store<G_>(x, conv_tile<CTH>(x, t), n0, N, wm, wn, col, half, E, sBias, sHead, acc);
    };
    const int G = gridDim.x;
    load(pa, blockIdx.x);
    load(pb, blockIdx.x + G);
    for (int t = blockIdx.x; t < tiles; t += 2 * G) {
        tile(pa, t);
        if (t + G < tiles) tile(pb, t + G);
    }
}

// The first two encoder convolutions of an inference pass in one persistent kernel.  Conv A (one real
// input channel; w0 [C][9]: its BF16 weights as FP32, b0: bias) is evaluated for every pixel of the patch
// that a tile of conv B needs, straight into the LDS patch, and is never stored: one MFMA per 32 patch
// pixels (weights of the C <= 32 channels x 9 taps padded to 16 as the A operand, the pixels' 3 x 3 input
// neighbourhoods as the B operand), bias, ReLU and BF16 rounding as in conv_first_kernel (the FP32 sums
// may round differently in the last place).  Conv B (C -> N <= 32 outputs, weights in registers, 8 x 32-
// pixel tiles) then runs as in the persistent form.  The next tile's 12 x 36 input pixels are in flight
// in registers while the current tile is summed.  xin: FP32 input [B][H][W] (x gives the batch geometry).
template <int C, class EP>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3)))
void conv_pair0_kernel(const float *xin, float scale, const float *w0, const float *b0, Act x, WeightB B, EP E, int N,
                       int tiles)
{
    constexpr int TN = 32, CTH = 8, CIN = C;
    using G_ = ConvGrid<TN, CTH>;
    constexpr int CPX = CIN / 8, CPP = CPX | 1;
    constexpr int NSTEP = (9 * CIN + 15) / 16;
    constexpr int WNW = G_::WN, BM = G_::BM, BN = G_::BN, WTN = G_::WTN;
    constexpr int IH = CTH + 4, IW = CT_W + 4, NIN = IH * IW, NINV = (NIN + 255) / 256;
    constexpr int NPB = (G_::PIX + 31) / 32;   // 32-pixel blocks of the patch
    static_assert(C % 8 == 0 && C <= 32, "conv A's channels in one MFMA block");
    __shared__ uint4 sP[G_::PIX * CPP];
    __shared__ unsigned short sIn[NIN];        // bf16(scale x), zero outside the image
    __shared__ float sBiasA[32];
    __shared__ float4 sBias[TN / 4];
    __shared__ float4 sHead[EP::HEAD ? TN / 4 : 1];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave / WNW, wn = wave % WNW;
    const int col = lane & 31, half = lane >> 5;
    const int n0 = blockIdx.y * TN;
    uint4 wr[NSTEP][BN];
#pragma unroll
    for (int S = 0; S < NSTEP; ++S)
#pragma unroll
        for (int j = 0; j < BN; ++j) {
            const int n = n0 + wn * WTN + 32 * j + col, k = 16 * S + 8 * half;
            wr[S][j] = n < N && k < 9 * CIN ? ld8(B.w + (int64_t)n * B.K + k) : zero8();
        }
    if (EP::BIAS && threadIdx.x < TN) ((float *)sBias)[threadIdx.x] = n0 + (int)threadIdx.x < N ? E.bias[n0 + threadIdx.x] : 0.0f;
    if constexpr (EP::HEAD)
        if (threadIdx.x < TN) ((float *)sHead)[threadIdx.x] = n0 + (int)threadIdx.x < N ? E.wh[n0 + threadIdx.x] : 0.0f;
    if (threadIdx.x < 32) sBiasA[threadIdx.x] = (int)threadIdx.x < C ? b0[threadIdx.x] : 0.0f;
    // conv A's A operand: channel col, taps 8 half .. 8 half + 7 (zero past tap 8 and channel C); the FP32
    // weights hold BF16 values, so their upper 16 bits are the BF16 encoding
    bf16x8 wa;
    {
        uint32_t u[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int t0 = 8 * half + 2 * q, t1 = t0 + 1;
            const uint32_t lo = col < C && t0 < 9 ? __float_as_uint(w0[9 * col + t0]) >> 16 : 0u;
            const uint32_t hi = col < C && t1 < 9 ? __float_as_uint(w0[9 * col + t1]) >> 16 : 0u;
            u[q] = lo | (hi << 16);
        }
        const uint4 v = make_uint4(u[0], u[1], u[2], u[3]);
        wa = *(const bf16x8 *)&v;
    }
    unsigned short pin[NINV];
    auto load = [&](int t) {
        if (t >= tiles) return;
        const ConvTile c = conv_tile<CTH>(x, t);
#pragma unroll
        for (int v = 0; v < NINV; ++v) {
            const int i = threadIdx.x + 256 * v, iy = i / IW, ix = i - iy * IW;
            const int yy = c.y0 - 2 + iy, xx = c.x0 - 2 + ix;
            pin[v] = i < NIN && (unsigned)yy < (unsigned)x.H && (unsigned)xx < (unsigned)x.W
                         ? (unsigned short)pack_bf16x2(xin[((int64_t)c.b * x.H + yy) * x.W + xx] * scale, 0.0f)
                         : (unsigned short)0;
        }
    };
    int la[BM];
#pragma unroll
    for (int i = 0; i < BM; ++i) la[i] = ((wm * BM + i) * CT_PW + col) * CPP + (CIN >= 16 ? half : 0);

    load(blockIdx.x);
    for (int t = blockIdx.x; t < tiles; t += gridDim.x) {
        const ConvTile c = conv_tile<CTH>(x, t);
        __syncthreads();   // the previous tile's reads of the input and the patch are done
#pragma unroll
        for (int v = 0; v < NINV; ++v) {
            const int i = threadIdx.x + 256 * v;
            if (i < NIN) sIn[i] = pin[v];
        }
        __syncthreads();
        load(t + (int)gridDim.x);   // in flight while this tile is computed
        // conv A: wavefront w takes patch blocks w, w + 4, ...; lane col is patch pixel 32 pb + col
        for (int pb = wave; pb < NPB; pb += 4) {   // uniform over the wavefront
            const int p = 32 * pb + col;
            const int pp = p < G_::PIX ? p : G_::PIX - 1;
            const int py = pp / CT_PW, px = pp - py * CT_PW;
            uint32_t u[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int t0 = 8 * half + 2 * q, t1 = t0 + 1;
                const uint32_t lo = t0 < 9 ? sIn[(py + t0 / 3) * IW + px + t0 % 3] : 0u;
                const uint32_t hi = t1 < 9 ? sIn[(py + t1 / 3) * IW + px + t1 % 3] : 0u;
                u[q] = lo | (hi << 16);
            }
            const uint4 bv = make_uint4(u[0], u[1], u[2], u[3]);
            f32x16 a = {};
            a = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wa, *(const bf16x8 *)&bv, a, 0, 0, 0);
            const int yy = c.y0 - 1 + py, xx = c.x0 - 1 + px;
            const bool live = p < G_::PIX && (unsigned)yy < (unsigned)x.H && (unsigned)xx < (unsigned)x.W;
#pragma unroll
            for (int g = 0; g < 4; g += 2) {
                uint2 r[2];
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int ch = 8 * (g + h) + 4 * half;   // accumulator 4 (g + h) + q: channel ch + q
                    r[h] = make_uint2(pack_bf16x2(fmaxf(a[4 * (g + h)] + sBiasA[ch], 0.0f),
                                                  fmaxf(a[4 * (g + h) + 1] + sBiasA[ch + 1], 0.0f)),
                                      pack_bf16x2(fmaxf(a[4 * (g + h) + 2] + sBiasA[ch + 2], 0.0f),
                                                  fmaxf(a[4 * (g + h) + 3] + sBiasA[ch + 3], 0.0f)));
                }
                const uint4 o = gather8(r[0], r[1]);   // lane half h: channels 8 (g + h) .. + 7
                const int grp = g + half;
                if (p < G_::PIX && grp < CPX) sP[p * CPP + grp] = live ? o : zero8();
            }
        }
        __syncthreads();
        f32x16 acc[BN][BM];
#pragma unroll
        for (int j = 0; j < BN; ++j)
#pragma unroll
            for (int i = 0; i < BM; ++i)
#pragma unroll
                for (int q = 0; q < 16; ++q) acc[j][i][q] = 0.0f;
        rconv_steps<CIN, TN, CTH, NSTEP>(std::make_integer_sequence<int, NSTEP>{}, sP, la, half, wr, acc);
        pconv_store<G_>(x, c, n0, N, wm, wn, col, half, E, sBias, sHead, acc);
    }
}

// conv_pair0_kernel for C = 8, 16 or 32 channels and N <= 32 outputs; false: not handled
template <class EP>
inline bool run_conv_pair0(const float *xin, float scale, const float *w0, const float *b0, const Act &x,
                           const WeightB &w, const EP &e, int C, int N, int cu_count, hipStream_t st, hipError_t &err)
{
    if (N > 32) return false;
    const int tiles = x.B * ((x.H + 7) / 8) * ((x.W + CT_W - 1) / CT_W);
    auto go = [&](auto kernel) {
        int per_cu = 0;
        err = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 256, 0);
        if (err != hipSuccess) return;
        const int wgs = std::min(tiles, std::max(1, per_cu) * cu_count);
        kernel<<<dim3(wgs, 1), 256, 0, st>>>(xin, scale, w0, b0, x, w, e, N, tiles);
        err = hipGetLastError();
    };
    switch (C) {
    case 8: go(conv_pair0_kernel<8, EP>); return true;
    case 16: go(conv_pair0_kernel<16, EP>); return true;
    case 32: go(conv_pair0_kernel<32, EP>); return true;
    default: return false;
    }
}

// One MFMA K step S of conv_upcat_kernel with the up half's weights in LDS (CU = 32): the skip half's
// weight operands are in registers (wr, tap by tap), the up half's at slots n WSU + tap CSX + chunk of sW.
template <int CU, int NR, int S>
__device__ __forceinline__ void upcat_step(const uint4 *sP, const uint4 *sW, int la, int lw, const uint4 (&wr)[NR],
                                           f32x16 &acc)
{
    constexpr int CIN = 2 * CU, CPP = (CIN / 8) | 1, CSX = CU / 8;
    constexpr int tap = (16 * S) / CIN, c8 = ((16 * S) % CIN) / 8;   // both halves read one tap (CIN >= 32)
    constexpr int oa = ((tap / 3) * CT_PW + tap % 3) * CPP + c8;
    uint4 w;
    if constexpr (c8 >= CSX) w = sW[lw + tap * CSX + c8 - CSX];
    else w = wr[tap * (CU / 16) + c8 / 2];
    const uint4 v = sP[la + oa];
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(*(const bf16x8 *)&w, *(const bf16x8 *)&v, acc, 0, 0, 0);
}
template <int CU, int NR, int... S>
__device__ __forceinline__ void upcat_steps(std::integer_sequence<int, S...>, const uint4 *sP, const uint4 *sW, int la,
                                            int lw, const uint4 (&wr)[NR], f32x16 &acc)
{
    (upcat_step<CU, NR, S>(sP, sW, la, lw, wr, acc), ...);
}

// Inference: the first convolution of a decoder level with the level's 2x2 up-sampling inside it, so the
// concatenation [skip | up(lo)] that the convolution reads is never stored.  The skip half of a tile's
// patch is loaded as in the persistent form; the up half is computed straight into the LDS patch from the
// low-resolution input lo: up[2 Y + dy][2 X + dx][co] = relu(ub[co] + sum_ci lo[Y][X][ci] U[(2 dy + dx) CU +
// co][ci]), zero outside the image.  The patch pixels of one sub-pixel parity d = (dy, dx) are 3 rows x 17
// columns of the tile's low-resolution footprint (4 x 18 pixels, staged in LDS); wavefront d sums them in
// two blocks of 32 MFMA columns with the parity's up weights (in LDS) as the A operand.  The convolution
// (CIN = 2 CU inputs, N <= 32 outputs, weights in registers, 4 x 32-pixel tiles) then runs as in the
// persistent form.  Both sums are those of up2x2_kernel and the persistent form, term for term in the
// same order with the same roundings, so the output equals the unfused pair's bit for bit.  The next
// tile's patch and footprint are in flight in registers while the current one is summed (two tiles in
// flight measured slower).
// xs: the skip activation (CU channels, the output geometry); uw: U as [(d, co)][ci] (CL inputs); ub: its
// bias.
template <int CU, int CL, class EP>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
void conv_upcat_kernel(Act xs, Act lo, const bf16_t *uw, const float *ub, WeightB B, EP E, int N, int tiles)
{
    constexpr int TN = 32, CTH = 4, CIN = 2 * CU;
    using G_ = ConvGrid<TN, CTH>;
    constexpr int CPX = CIN / 8, CPP = CPX | 1, CSX = CU / 8;
    constexpr int CLX = CL / 8, LPP = CLX | 1;                        // footprint and up-weight slot stride
    constexpr int FH = CTH / 2 + 2, FW = CT_W / 2 + 2;               // low-resolution footprint
    constexpr int PR = (CTH + 2) / 2, PC = CT_PW / 2, NE = PR * PC;  // patch pixels of one parity
    constexpr int NSS = G_::PIX * CSX;                               // skip vectors of the patch
    constexpr int NLS = FH * FW * CLX;                               // footprint vectors
    constexpr int NV = (NSS + NLS + 255) / 256;
    constexpr int NSTEP = (9 * CIN + 15) / 16;
    constexpr int WNW = G_::WN, BM = G_::BM, BN = G_::BN, WTN = G_::WTN;
    static_assert(CU % 8 == 0 && CU <= 32 && CL % 16 == 0, "whole MFMA blocks and K steps of the up-sampling");
    static_assert(TN * 9 * CIN <= 20480, "weights of the workgroup's outputs fit in registers");
    static_assert(NE <= 64, "two 32-column MFMA blocks per parity");
    static_assert(BM == 1 && BN == 1, "one 32 x 32 block per wavefront and tile");
    // CU = 32: the up half's conv weights in LDS (the registers hold the skip half's), else all in registers
    constexpr bool WL = CU == 32;
    constexpr int WSU = conv_ws(CSX), NR = WL ? 9 * (CU / 16) : NSTEP;
    __shared__ uint4 sP[G_::PIX * CPP];
    __shared__ uint4 sL[FH * FW * LPP];
    __shared__ uint4 sU[4 * CU * LPP];
    __shared__ uint4 sW[WL ? TN * WSU : 1];
    __shared__ float sBU[32];
    __shared__ float4 sBias[TN / 4];
    __shared__ float4 sHead[EP::HEAD ? TN / 4 : 1];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave / WNW, wn = wave % WNW;
    const int col = lane & 31, half = lane >> 5;
    const int n0 = blockIdx.y * TN;
    uint4 wr[NR][1];
    {
        const int n = n0 + col;
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            // register r: step S = r (all in registers) or tap r / (CU / 16), sub-step r % (CU / 16)
            const int S = WL ? (r / (CU / 16)) * (CIN / 16) + r % (CU / 16) : r;
            const int k = 16 * S + 8 * half;
            wr[r][0] = n < N && k < 9 * CIN ? ld8(B.w + (int64_t)n * B.K + k) : zero8();
        }
    }
    if constexpr (WL)
        for (int i = threadIdx.x; i < TN * 9 * CSX; i += 256) {
            const int n = i / (9 * CSX), r = i - n * (9 * CSX), tap = r / CSX, u8 = r - tap * CSX;
            sW[n * WSU + r] = n0 + n < N ? ld8(B.w + (int64_t)(n0 + n) * B.K + tap * CIN + CU + 8 * u8) : zero8();
        }
    for (int i = threadIdx.x; i < 4 * CU * CLX; i += 256) {
        const int r = i / CLX, c8 = i - r * CLX;
        sU[r * LPP + c8] = ld8(uw + (int64_t)r * CL + 8 * c8);
    }
    if (threadIdx.x < 32) sBU[threadIdx.x] = (int)threadIdx.x < CU ? ub[threadIdx.x] : 0.0f;
    if (EP::BIAS && threadIdx.x < TN) ((float *)sBias)[threadIdx.x] = n0 + (int)threadIdx.x < N ? E.bias[n0 + threadIdx.x] : 0.0f;
    if constexpr (EP::HEAD)
        if (threadIdx.x < TN) ((float *)sHead)[threadIdx.x] = n0 + (int)threadIdx.x < N ? E.wh[n0 + threadIdx.x] : 0.0f;
    // this thread's staged vectors, the same for every tile: index i < NSS a skip vector of the patch
    // (pixel (py, px), chunk c8), else footprint vector i - NSS (row fr, column fc, chunk c8); -1: none
    int spos[NV], sdst[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const int i = threadIdx.x + 256 * v;
        if (i < NSS) {
            const int p = i / CSX, c8 = i - p * CSX, py = p / CT_PW, px = p - py * CT_PW;
            spos[v] = (py << 16) | (px << 8) | c8;
            sdst[v] = p * CPP + c8;
        } else {
            const int k = i - NSS, f = k / CLX, c8 = k - f * CLX, fr = f / FW, fc = f - fr * FW;
            spos[v] = k < NLS ? (1 << 24) | (fr << 16) | (fc << 8) | c8 : -1;
            sdst[v] = f * LPP + c8;
        }
    }
    uint4 pv[NV];
    auto load = [&](int t) {
        if (t >= tiles) return;
        const ConvTile c = conv_tile<CTH>(xs, t);
        const bf16_t *img = xs.p + (int64_t)c.b * xs.H * xs.W * xs.cs + xs.co;
        const bf16_t *limg = lo.p + (int64_t)c.b * lo.H * lo.W * lo.cs + lo.co;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const int r = (spos[v] >> 16) & 255, q = (spos[v] >> 8) & 255, c8 = spos[v] & 255;
            const bool foot = spos[v] >> 24;
            const int yy = foot ? (c.y0 >> 1) - 1 + r : c.y0 - 1 + r, xx = foot ? (c.x0 >> 1) - 1 + q : c.x0 - 1 + q;
            const int h = foot ? lo.H : xs.H, w = foot ? lo.W : xs.W;
            const bf16_t *src = foot ? limg + (int64_t)(yy * lo.W + xx) * lo.cs : img + (int64_t)(yy * xs.W + xx) * xs.cs;
            pv[v] = spos[v] >= 0 && (unsigned)yy < (unsigned)h && (unsigned)xx < (unsigned)w ? ld8(src + 8 * c8) : zero8();
        }
    };
    int la[BM];
#pragma unroll
    for (int i = 0; i < BM; ++i) la[i] = ((wm * BM + i) * CT_PW + col) * CPP + (CIN >= 16 ? half : 0);
    // the up-sampling of wavefront d = (dy, dx): A operand rows (d CU + col) of U (zero past CU)
    const int dy = wave >> 1, dx = wave & 1;
    const int lu = (wave * CU + (col < CU ? col : 0)) * LPP + half;

    load(blockIdx.x);
    for (int t = blockIdx.x; t < tiles; t += gridDim.x) {
        const ConvTile c = conv_tile<CTH>(xs, t);
        __syncthreads();   // the previous tile's reads of the patch and the footprint are done
#pragma unroll
        for (int v = 0; v < NV; ++v)
            if (spos[v] >= 0) (spos[v] >> 24 ? sL : sP)[sdst[v]] = pv[v];
        __syncthreads();
        load(t + (int)gridDim.x);   // in flight while this tile is summed
        // up half of the patch: MFMA column e of block blk is parity pixel e = 32 blk + col (row e / PC,
        // column e % PC of the parity), i.e. patch pixel (2 (e / PC) + 1 - dy, 2 (e % PC) + 1 - dx) and
        // footprint pixel (e / PC + 1 - dy, e % PC + 1 - dx)
#pragma unroll
        for (int blk = 0; blk < 2; ++blk) {
            const int e = 32 * blk + col, ee = e < NE ? e : NE - 1;
            const int r3 = ee / PC, c17 = ee - r3 * PC;
            const int py = 2 * r3 + 1 - dy, px = 2 * c17 + 1 - dx;
            const int lb = ((r3 + 1 - dy) * FW + c17 + 1 - dx) * LPP + half;
            f32x16 a = {};
#pragma unroll
            for (int s = 0; s < CL / 16; ++s) {
                const uint4 wv = col < CU ? sU[lu + 2 * s] : zero8();
                const uint4 bv = sL[lb + 2 * s];
                a = __builtin_amdgcn_mfma_f32_32x32x16_bf16(*(const bf16x8 *)&wv, *(const bf16x8 *)&bv, a, 0, 0, 0);
            }
            const int yy = c.y0 - 1 + py, xx = c.x0 - 1 + px;
            const bool live = (unsigned)yy < (unsigned)xs.H && (unsigned)xx < (unsigned)xs.W;
#pragma unroll
            for (int g = 0; g < 4; g += 2) {
                uint2 r[2];
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int ch = 8 * (g + h) + 4 * half;   // accumulator 4 (g + h) + q: channel ch + q
                    r[h] = make_uint2(pack_bf16x2(fmaxf(a[4 * (g + h)] + sBU[ch], 0.0f),
                                                  fmaxf(a[4 * (g + h) + 1] + sBU[ch + 1], 0.0f)),
                                      pack_bf16x2(fmaxf(a[4 * (g + h) + 2] + sBU[ch + 2], 0.0f),
                                                  fmaxf(a[4 * (g + h) + 3] + sBU[ch + 3], 0.0f)));
                }
                const uint4 o = gather8(r[0], r[1]);   // lane half h: channels 8 (g + h) .. + 7
                const int grp = g + half;
                if (e < NE && grp < CSX) sP[(py * CT_PW + px) * CPP + CSX + grp] = live ? o : zero8();
            }
        }
        __syncthreads();
        f32x16 acc[BN][BM];
#pragma unroll
        for (int j = 0; j < BN; ++j)
#pragma unroll
            for (int i = 0; i < BM; ++i)
#pragma unroll
                for (int q = 0; q < 16; ++q) acc[j][i][q] = 0.0f;
        if constexpr (WL) {
            uint4 wk[NR];
#pragma unroll
            for (int r = 0; r < NR; ++r) wk[r] = wr[r][0];
            upcat_steps<CU, NR>(std::make_integer_sequence<int, NSTEP>{}, sP, sW, la[0], col * WSU + half, wk, acc[0][0]);
        } else {
            rconv_steps<CIN, TN, CTH, NSTEP>(std::make_integer_sequence<int, NSTEP>{}, sP, la, half, wr, acc);
        }
        pconv_store<G_>(xs, c, n0, N, wm, wn, col, half, E, sBias, sHead, acc);
    }
}

// conv_upcat_kernel for CU = 8, 16 or 32 skip and up channels, CL = 2 CU low-resolution channels and
// N <= 32 outputs, the output twice lo's size; false: not handled
template <class EP>
inline bool run_conv_upcat(const Act &xs, const Act &lo, const bf16_t *uw, const float *ub, const WeightB &w,
                           const EP &e, int CU, int CL, int N, int cu_count, hipStream_t st, hipError_t &err)
{
    if (N > 32 || CL != 2 * CU || xs.B != lo.B || xs.H != 2 * lo.H || xs.W != 2 * lo.W) return false;
    const int tiles = xs.B * ((xs.H + 3) / 4) * ((xs.W + CT_W - 1) / CT_W);
    auto go = [&](auto kernel) {
        int per_cu = 0;
        err = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 256, 0);
        if (err != hipSuccess) return;
        const int wgs = std::min(tiles, std::max(1, per_cu) * cu_count);
        kernel<<<dim3(wgs, 1), 256, 0, st>>>(xs, lo, uw, ub, w, e, N, tiles);
        err = hipGetLastError();
    };
    switch (CU) {
    case 8: go(conv_upcat_kernel<8, 16, EP>); return true;
    case 16: go(conv_upcat_kernel<16, 32, EP>); return true;
    case 32: go(conv_upcat_kernel<32, 64, EP>); return true;
    default: return false;
    }
}

// wave layout of the general form's CTH x 32-pixel, TN-channel tile: each wavefront owns one column
// block of 32 output channels (WN = min(4, TN / 32)) and CTH / WM consecutive tile rows (BM)
template <int TN, int CTH>
struct GenGrid {
    static constexpr int WN = TN >= 128 ? 4 : TN / 32, WM = 4 / WN;
    static constexpr int BM = CTH / WM, BN = 1, WTN = 32;
    static constexpr int PIX = (CTH + 2) * CT_PW;
    static_assert(TN <= 128 && TN % 32 == 0 && CTH % WM == 0, "whole column blocks and tile rows per wavefront");
};

// The K steps of one staged chunk (CC >= 16 channels) in the general form, ordered so that a patch row
// read from LDS serves every tap row that needs it: per 16-channel slice s and tap column tx the
// wavefront reads patch rows R = r0 .. r0 + BM + 1 (BM + 2 reads) and the weights of taps (ty, tx),
// ty = 0, 1, 2 (3 reads), then output row r0 + i takes W[ty] x P[i + ty] (3 BM MFMAs).  lp: this lane's
// patch slot of row r0, column col (plus its half of the slice); lw: its weight slot.
template <int CC, int BM, int SL, int TX>
__device__ __forceinline__ void gconv_taps(const uint4 *sP, const uint4 *sW, int lp, int lw, f32x16 (&acc)[1][BM])
{
    constexpr int CPX = CC / 8, CPP = CPX | 1;
    bf16x8 pf[BM + 2], wf[3];
#pragma unroll
    for (int R = 0; R < BM + 2; ++R) {
        const uint4 v = sP[lp + (R * CT_PW + TX) * CPP + 2 * SL];
        pf[R] = *(const bf16x8 *)&v;
    }
#pragma unroll
    for (int ty = 0; ty < 3; ++ty) {
        const uint4 v = sW[lw + (3 * ty + TX) * CPX + 2 * SL];
        wf[ty] = *(const bf16x8 *)&v;
    }
#pragma unroll
    for (int ty = 0; ty < 3; ++ty)
#pragma unroll
        for (int i = 0; i < BM; ++i) acc[0][i] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wf[ty], pf[i + ty], acc[0][i], 0, 0, 0);
}

template <int CC, int BM, int... Q>
__device__ __forceinline__ void gconv_chunk(std::integer_sequence<int, Q...>, const uint4 *sP, const uint4 *sW, int lp,
                                            int lw, f32x16 (&acc)[1][BM])
{
    (gconv_taps<CC, BM, Q / 3, Q % 3>(sP, sW, lp, lw, acc), ...);   // Q = 3 slice + tap column
}

// channels per chunk of the general form: the chunk's weights [TN][9][CC] take at most 36 KB, and patch
// plus weights about 70 KB (two workgroups per CU)
template <int CIN, int TN>
constexpr int conv_cc()
{
    constexpr int cap = TN >= 128 ? 16 : 32;
    return CIN < cap ? CIN : cap;
}

// General form (the layers whose weights do not fit the persistent form): one 8 x 32-pixel output
// tile per workgroup (a staged chunk of weights serves 256 pixels); per chunk of CC input channels the
// tile's patch and the chunk's weights for the TN outputs are staged in LDS (the layouts of the
// persistent form, for CC channels), the chunk's K steps run from LDS in the row-reusing order of
// gconv_taps, and the next chunk is meanwhile loaded into registers.  Two barriers per chunk.
// K order: chunk, 16-channel slice, tap column, tap row.
constexpr int CONV_GEN_CTH = 8;
template <int CIN, int TN, class EP>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
void conv3x3_kernel(Act x, WeightB B, EP E, int N)
{
    constexpr int CTH = CONV_GEN_CTH;
    using G_ = GenGrid<TN, CTH>;
    constexpr int CC = conv_cc<CIN, TN>(), CPX = CC / 8, CPP = CPX | 1, WS = conv_ws(CPX);
    constexpr int NCH = CIN / CC;
    constexpr int NPS = G_::PIX * CPX, NWS = TN * 9 * CPX;  // patch and weight vectors per chunk
    constexpr int NV = (NPS + NWS + 255) / 256;             // per thread
    constexpr int WNW = G_::WN, BM = G_::BM, BN = G_::BN, WTN = G_::WTN;
    static_assert(CIN % CC == 0 && CC % 16 == 0, "channels in chunks of 16-channel slices");
    __shared__ uint4 sP[G_::PIX * CPP];
    __shared__ uint4 sW[TN * WS];
    __shared__ float4 sBias[TN / 4];
    __shared__ float4 sHead[EP::HEAD ? TN / 4 : 1];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave / WNW, wn = wave % WNW;
    const int col = lane & 31, half = lane >> 5;
    const ConvTile c = conv_tile<CTH>(x, blockIdx.x);
    const int n0 = blockIdx.y * TN;
    if (EP::BIAS && threadIdx.x < TN) ((float *)sBias)[threadIdx.x] = n0 + (int)threadIdx.x < N ? E.bias[n0 + threadIdx.x] : 0.0f;
    if constexpr (EP::HEAD)
        if (threadIdx.x < TN) ((float *)sHead)[threadIdx.x] = n0 + (int)threadIdx.x < N ? E.wh[n0 + threadIdx.x] : 0.0f;

    // this thread's vectors of a chunk (the same for every chunk up to the channel offset ch CC):
    // source element offset (-1: zero) from the tile's image or from the weights, LDS slot
    const bf16_t *img = x.p + (int64_t)c.b * x.H * x.W * x.cs + x.co;
    int src[NV], dst[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const int i = threadIdx.x + 256 * v;
        if (i < NPS) {
            const int p = i / CPX, c8 = i - p * CPX, py = p / CT_PW, px = p - py * CT_PW;
            const int yy = c.y0 - 1 + py, xx = c.x0 - 1 + px;
            src[v] = (unsigned)yy < (unsigned)x.H && (unsigned)xx < (unsigned)x.W ? (yy * x.W + xx) * x.cs + 8 * c8 : -1;
            dst[v] = p * CPP + c8;
        } else {
            const int j = i - NPS, n = j / (9 * CPX), rr = j - n * (9 * CPX);
            const int tap = rr / CPX, c8 = rr - tap * CPX;
            src[v] = j < NWS && n0 + n < N ? (n0 + n) * B.K + tap * CIN + 8 * c8 : -1;
            dst[v] = j < NWS ? n * WS + tap * CPX + c8 : -1;
        }
    }
    uint4 rv[NV];
    auto load = [&](int ch) {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const bool patch = (int)threadIdx.x + 256 * v < NPS;
            rv[v] = src[v] >= 0 ? ld8((patch ? img : B.w) + src[v] + ch * CC) : zero8();
        }
    };
    auto store = [&]() {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const bool patch = (int)threadIdx.x + 256 * v < NPS;
            if (patch) sP[dst[v]] = rv[v];
            else if (dst[v] >= 0) sW[dst[v]] = rv[v];
        }
    };
    const int lp = (wm * BM * CT_PW + col) * CPP + half, lw = (wn * WTN + col) * WS + half;

    f32x16 acc[BN][BM];
#pragma unroll
    for (int j = 0; j < BN; ++j)
#pragma unroll
        for (int i = 0; i < BM; ++i)
#pragma unroll
            for (int q = 0; q < 16; ++q) acc[j][i][q] = 0.0f;
    load(0);
    store();
    __syncthreads();
    for (int ch = 0; ch < NCH; ++ch) {
        if (ch + 1 < NCH) load(ch + 1);   // in flight while this chunk is summed
        gconv_chunk<CC, BM>(std::make_integer_sequence<int, 3 * (CC / 16)>{}, sP, sW, lp, lw, acc);
        if (ch + 1 < NCH) {
            __syncthreads();   // every wave is done with this chunk
            store();
            __syncthreads();
        }
    }
    pconv_store<G_>(x, c, n0, N, wm, wn, col, half, E, sBias, sHead, acc);
}

// ---- transposed 2x2 convolution, stride 2 (the U-Net's up-sampling) ------------------------------
// out[(b, 2y + dy, 2x + dx)][co] = relu(bias[co] + sum_ci U[d][co][ci] X[(b, y, x)][ci]), d = 2 dy + dx:
// the GEMM M = input pixels, N = 4 cout (n = d cout + co), K = cin, in the persistent form of the
// convolutions (the workgroup's TN outputs' weights in LDS, input tiles of 4 x 32 pixels streamed with
// two in flight, weights as the A operand) with an epilogue that sends each lane's four consecutive
// channels (one d, four co) to their output pixel as one 8-byte store.

// weight row stride in 16-byte slots of the 1x1 form: at least CPX and 1 mod 8
constexpr int up_ws(int cpx)
{
    int s = cpx;
    while (s % 8 != 1) ++s;
    return s;
}

template <int CIN, int TN, int S>
__device__ __forceinline__ void up_step(const uint4 *sP, const uint4 *sW, const int *la, const int *lw,
                                        f32x16 (&acc)[ConvGrid<TN, 4>::BN][ConvGrid<TN, 4>::BM])
{
    constexpr int BM = ConvGrid<TN, 4>::BM, BN = ConvGrid<TN, 4>::BN;
    bf16x8 wf[BN], pf[BM];
#pragma unroll
    for (int j = 0; j < BN; ++j) {
        const uint4 v = sW[lw[j] + 2 * S];
        wf[j] = *(const bf16x8 *)&v;
    }
#pragma unroll
    for (int i = 0; i < BM; ++i) {
        const uint4 v = sP[la[i] + 2 * S];
        pf[i] = *(const bf16x8 *)&v;
    }
#pragma unroll
    for (int j = 0; j < BN; ++j)
#pragma unroll
        for (int i = 0; i < BM; ++i)
            acc[j][i] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wf[j], pf[i], acc[j][i], 0, 0, 0);
}

template <int CIN, int TN, int... S>
__device__ __forceinline__ void up_steps(std::integer_sequence<int, S...>, const uint4 *sP, const uint4 *sW,
                                         const int *la, const int *lw,
                                         f32x16 (&acc)[ConvGrid<TN, 4>::BN][ConvGrid<TN, 4>::BM])
{
    (up_step<CIN, TN, S>(sP, sW, la, lw, acc), ...);
}

// x: input (cin channels at x.co of stride x.cs); w: U as [(d, co)][ci]; y: output of 2 x.H x 2 x.W
// pixels, channels yco .. yco + cout - 1 of stride ycs; N = 4 cout, cout = 1 << lgc
template <int CIN, int TN>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
void up2x2_kernel(Act x, const bf16_t *w, const float *bias, int lgc, bf16_t *y, int ycs, int yco, int N, int tiles)
{
    constexpr int CTH = 4;
    using G_ = ConvGrid<TN, CTH>;
    constexpr int CPX = CIN / 8, CPP = CPX | 1, WS = up_ws(CPX);
    constexpr int NPS = CTH * CT_W * CPX;          // tile vectors (no halo)
    constexpr int NPV = (NPS + 255) / 256;
    constexpr int WNW = G_::WN, BM = G_::BM, BN = G_::BN, WTN = G_::WTN;
    static_assert(CIN % 16 == 0, "whole MFMA K steps");
    __shared__ uint4 sP[CTH * CT_W * CPP];
    __shared__ uint4 sW[TN * WS];
    __shared__ float4 sBias[TN / 4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave / WNW, wn = wave % WNW;
    const int col = lane & 31, half = lane >> 5;
    const int n0 = blockIdx.y * TN;
    const int cmask = (1 << lgc) - 1;
    for (int i = threadIdx.x; i < TN * CPX; i += 256) {
        const int n = i / CPX, c8 = i - n * CPX;
        sW[n * WS + c8] = n0 + n < N ? ld8(w + (int64_t)(n0 + n) * CIN + 8 * c8) : zero8();
    }
    if (threadIdx.x < TN) ((float *)sBias)[threadIdx.x] = n0 + (int)threadIdx.x < N ? bias[(n0 + threadIdx.x) & cmask] : 0.0f;
    int spos[NPV], sdst[NPV];
#pragma unroll
    for (int v = 0; v < NPV; ++v) {
        const int i = threadIdx.x + 256 * v;
        const int p = i / CPX, c8 = i - p * CPX, py = p / CT_W, px = p - py * CT_W;
        spos[v] = i < NPS ? (py << 16) | (px << 8) | c8 : -1;
        sdst[v] = p * CPP + c8;
    }
    uint4 pa[NPV], pb[NPV];
    auto load = [&](uint4 (&pv)[NPV], int t) {
        if (t >= tiles) return;
        const ConvTile c = conv_tile<CTH>(x, t);
        const bf16_t *img = x.p + (int64_t)c.b * x.H * x.W * x.cs + x.co;
#pragma unroll
        for (int v = 0; v < NPV; ++v) {
            const int yy = c.y0 + (spos[v] >> 16), xx = c.x0 + ((spos[v] >> 8) & 255);
            pv[v] = spos[v] >= 0 && yy < x.H && xx < x.W ? ld8(img + (int64_t)(yy * x.W + xx) * x.cs + 8 * (spos[v] & 255))
                                                         : zero8();
        }
    };
    int la[BM], lw[BN];
#pragma unroll
    for (int i = 0; i < BM; ++i) la[i] = ((wm * BM + i) * CT_W + col) * CPP + half;
#pragma unroll
    for (int j = 0; j < BN; ++j) lw[j] = (wn * WTN + j * 32 + col) * WS + half;
    const int H2 = 2 * x.H, W2 = 2 * x.W;

    auto tile = [&](uint4 (&pv)[NPV], int t) {
        __syncthreads();
#pragma unroll
        for (int v = 0; v < NPV; ++v)
            if (spos[v] >= 0) sP[sdst[v]] = pv[v];
        __syncthreads();
        load(pv, t + 2 * (int)gridDim.x);
        f32x16 acc[BN][BM];
#pragma unroll
        for (int j = 0; j < BN; ++j)
#pragma unroll
            for (int i = 0; i < BM; ++i)
#pragma unroll
                for (int q = 0; q < 16; ++q) acc[j][i][q] = 0.0f;
        up_steps<CIN, TN>(std::make_integer_sequence<int, CIN / 16>{}, sP, sW, la, lw, acc);
        const ConvTile c = conv_tile<CTH>(x, t);
        const int xx = c.x0 + col;
#pragma unroll
        for (int i = 0; i < BM; ++i) {
            const int yy = c.y0 + wm * BM + i;
            const bool in = yy < x.H && xx < x.W;
#pragma unroll
            for (int j = 0; j < BN; ++j)
#pragma unroll
                for (int g = 0; g < 4; g += 2) {
                    const int nb = wn * WTN + j * 32 + 8 * g;
                    uint2 r[2];
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const float4 bb = sBias[(nb + 8 * h + 4 * half) >> 2];
                        const float a0 = acc[j][i][4 * (g + h)], a1 = acc[j][i][4 * (g + h) + 1];
                        const float a2 = acc[j][i][4 * (g + h) + 2], a3 = acc[j][i][4 * (g + h) + 3];
                        r[h] = make_uint2(pack_bf16x2(fmaxf(a0 + bb.x, 0.0f), fmaxf(a1 + bb.y, 0.0f)),
                                          pack_bf16x2(fmaxf(a2 + bb.z, 0.0f), fmaxf(a3 + bb.w, 0.0f)));
                    }
                    const uint4 o = gather8(r[0], r[1]);
                    const int n = n0 + nb + 8 * half;   // eight channels of one sub-pixel d (cout >= 8)
                    if (!in || n >= N) continue;
                    const int d = n >> lgc, co = n & cmask;
                    const int m2 = (c.b * H2 + 2 * yy + (d >> 1)) * W2 + 2 * xx + (d & 1);
                    *(uint4 *)(y + (int64_t)m2 * ycs + yco + co) = o;
                }
        }
    };
    const int G = gridDim.x;
    load(pa, blockIdx.x);
    load(pb, blockIdx.x + G);
    for (int t = blockIdx.x; t < tiles; t += 2 * G) {
        tile(pa, t);
        if (t + G < tiles) tile(pb, t + G);
    }
}

// The up-sampling for inputs too wide for an LDS patch beside the weights (CIN = 256): wavefront w owns
// tile row w, so no patch operand is shared between wavefronts and each lane loads its pixel's B operands
// (channels 16 S + 8 half .. + 7 of every K step S) straight from memory, the next two tiles' in flight in
// registers; the weights of the TN = 128 outputs (four column blocks per wavefront) are staged in LDS once
// and the epilogue is up2x2_kernel's.  No barrier after the weights: the tiles share nothing in LDS.
template <int CIN>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
void up2x2_wide_kernel(Act x, const bf16_t *w, const float *bias, int lgc, bf16_t *y, int ycs, int yco, int N,
                       int tiles)
{
    constexpr int TN = 128, CTH = 4, BN = TN / 32, CPX = CIN / 8, WS = up_ws(CPX), NS = CIN / 16;
    static_assert(CIN % 16 == 0, "whole MFMA K steps");
    __shared__ uint4 sW[TN * WS];
    __shared__ float4 sBias[TN / 4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int col = lane & 31, half = lane >> 5;
    const int n0 = blockIdx.y * TN;
    const int cmask = (1 << lgc) - 1;
    for (int i = threadIdx.x; i < TN * CPX; i += 256) {
        const int n = i / CPX, c8 = i - n * CPX;
        sW[n * WS + c8] = n0 + n < N ? ld8(w + (int64_t)(n0 + n) * CIN + 8 * c8) : zero8();
    }
    if (threadIdx.x < TN) ((float *)sBias)[threadIdx.x] = n0 + (int)threadIdx.x < N ? bias[(n0 + threadIdx.x) & cmask] : 0.0f;
    __syncthreads();
    uint4 pa[NS], pb[NS];
    auto load = [&](uint4 (&pv)[NS], int t) {
        if (t >= tiles) return;
        const ConvTile c = conv_tile<CTH>(x, t);
        const int yy = c.y0 + wave, xx = c.x0 + col;
        const bool in = yy < x.H && xx < x.W;
        const bf16_t *src = x.p + ((int64_t)(c.b * x.H + (in ? yy : 0)) * x.W + (in ? xx : 0)) * x.cs + x.co + 8 * half;
#pragma unroll
        for (int S = 0; S < NS; ++S) pv[S] = in ? ld8(src + 16 * S) : zero8();
    };
    int lw[BN];
#pragma unroll
    for (int j = 0; j < BN; ++j) lw[j] = (j * 32 + col) * WS + half;
    const int H2 = 2 * x.H, W2 = 2 * x.W;

    auto tile = [&](uint4 (&pv)[NS], int t) {
        // a compiler memory barrier: the weight reads below stay in the loop (hoisted out of it, as loop
        // invariants, they would need 64 registers per K step)
        asm volatile("" ::: "memory");
        f32x16 acc[BN];
#pragma unroll
        for (int j = 0; j < BN; ++j)
#pragma unroll
            for (int q = 0; q < 16; ++q) acc[j][q] = 0.0f;
#pragma unroll
        for (int S = 0; S < NS; ++S)
#pragma unroll
            for (int j = 0; j < BN; ++j) {
                const uint4 wv = sW[lw[j] + 2 * S];
                acc[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(*(const bf16x8 *)&wv, *(const bf16x8 *)&pv[S], acc[j],
                                                                 0, 0, 0);
            }
        load(pv, t + 2 * (int)gridDim.x);   // in flight while the next tile is summed
        const ConvTile c = conv_tile<CTH>(x, t);
        const int yy = c.y0 + wave, xx = c.x0 + col;
        const bool in = yy < x.H && xx < x.W;
#pragma unroll
        for (int j = 0; j < BN; ++j)
#pragma unroll
            for (int g = 0; g < 4; g += 2) {
                const int nb = j * 32 + 8 * g;
                uint2 r[2];
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const float4 bb = sBias[(nb + 8 * h + 4 * half) >> 2];
                    const float a0 = acc[j][4 * (g + h)], a1 = acc[j][4 * (g + h) + 1];
                    const float a2 = acc[j][4 * (g + h) + 2], a3 = acc[j][4 * (g + h) + 3];
                    r[h] = make_uint2(pack_bf16x2(fmaxf(a0 + bb.x, 0.0f), fmaxf(a1 + bb.y, 0.0f)),
                                      pack_bf16x2(fmaxf(a2 + bb.z, 0.0f), fmaxf(a3 + bb.w, 0.0f)));
                }
                const uint4 o = gather8(r[0], r[1]);
                const int n = n0 + nb + 8 * half;   // eight channels of one sub-pixel d (cout >= 8)
                if (!in || n >= N) continue;
                const int d = n >> lgc, co = n & cmask;
                const int m2 = (c.b * H2 + 2 * yy + (d >> 1)) * W2 + 2 * xx + (d & 1);
                *(uint4 *)(y + (int64_t)m2 * ycs + yco + co) = o;
            }
    };
    const int G = gridDim.x;
    load(pa, blockIdx.x);
    load(pb, blockIdx.x + G);
    for (int t = blockIdx.x; t < tiles; t += 2 * G) {
        tile(pa, t);
        if (t + G < tiles) tile(pb, t + G);
    }
}

// the up-sampling by the kernel above for the channel counts it is built for; false: not handled
inline bool run_up2x2(const Act &x, const bf16_t *w, const float *bias, int cin, int cout, bf16_t *y, int ycs, int yco,
                      int cu_count, hipStream_t st, hipError_t &err)
{
    if (cout < 8 || (cout & (cout - 1))) return false;
    int lgc = 0;
    while ((1 << lgc) < cout) ++lgc;
    const int N = 4 * cout, tn = N >= 128 ? 128 : (N >= 64 ? 64 : 32);
    const int tiles = x.B * ((x.H + 3) / 4) * ((x.W + CT_W - 1) / CT_W);
    auto go = [&](auto kernel) {
        int per_cu = 0;
        err = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 256, 0);
        if (err != hipSuccess) return;
        const int wgs = std::min(tiles, std::max(1, per_cu) * cu_count);
        kernel<<<dim3(wgs, (N + tn - 1) / tn), 256, 0, st>>>(x, w, bias, lgc, y, ycs, yco, N, tiles);
        err = hipGetLastError();
    };
#define PYHST_UP_CASE(CI)                                              \
    case CI:                                                          \
        if (tn == 128) go(up2x2_kernel<CI, 128>);                     \
        else if (tn == 64) go(up2x2_kernel<CI, 64>);                  \
        else go(up2x2_kernel<CI, 32>);                                \
        return true;
    switch (cin) {
        PYHST_UP_CASE(16)
        PYHST_UP_CASE(32)
        PYHST_UP_CASE(64)
        PYHST_UP_CASE(128)
    case 256:
        if (tn != 128) return false;
        go(up2x2_wide_kernel<256>);
        return true;
    default: return false;
    }
#undef PYHST_UP_CASE
}

// the direct kernels' four-channel epilogue of a GEMM epilogue
inline ConvStoreAct conv_ep(const StoreAct &e) { return ConvStoreAct{e.y, e.cs, e.co, e.bias}; }
inline ConvStoreMasked conv_ep(const StoreMasked &e) { return ConvStoreMasked{e.dx, e.cs, e.co, e.act, e.acs, e.aco, nullptr}; }
inline const ConvStoreActPool &conv_ep(const ConvStoreActPool &e) { return e; }
inline const ConvStoreHead &conv_ep(const ConvStoreHead &e) { return e; }

// The persistent form where the weights of TN outputs fit in registers (TN x 9 x CIN <= 20480 values),
// with 8-row tiles (two row blocks per wavefront) where the registers allow, else 4-row tiles; every
// other layer takes the general form.
template <int CIN, int TN>
constexpr bool use_persist()
{
    return TN * 9 * CIN <= 20480;
}
// 8-row tiles where the registers of the 8-row form (weights, accumulators, two patches in flight, about
// 24 more) stay within 240 per lane, else 4-row tiles
template <int CIN, int TN>
constexpr int persist_cth()
{
    constexpr int nstep = (9 * CIN + 15) / 16, bm = ConvGrid<TN, 8>::BM, bn = ConvGrid<TN, 8>::BN;
    constexpr int npv = (ConvGrid<TN, 8>::PIX * (CIN / 8) + 255) / 256;
    return 4 * nstep * bn + 16 * bm * bn + 8 * npv + 24 <= 240 ? 8 : 4;
}

// row blocks per wavefront and wavefront columns of the kernel run_conv3x3 launches for CIN, TN
template <int CIN, int TN>
constexpr int conv_bm()
{
    if constexpr (use_persist<CIN, TN>()) return ConvGrid<TN, persist_cth<CIN, TN>()>::BM;
    else return GenGrid<TN, CONV_GEN_CTH>::BM;
}
template <int CIN, int TN>
constexpr int conv_wn()
{
    if constexpr (use_persist<CIN, TN>()) return ConvGrid<TN, persist_cth<CIN, TN>()>::WN;
    else return GenGrid<TN, CONV_GEN_CTH>::WN;
}

// hipErrorInvalidValue: the fused pool or head does not fit the launched kernel's wave layout
// (callers check conv_bm / conv_wn and the N tile first)
template <int CIN, int TN, class EP>
inline hipError_t run_conv3x3(const Act &x, const WeightB &w, const EP &e, int N, int cu_count, hipStream_t st)
{
    using CE = std::decay_t<decltype(conv_ep(e))>;
    if constexpr ((CE::POOL && conv_bm<CIN, TN>() % 2 != 0) || (CE::HEAD && conv_wn<CIN, TN>() != 1)) {
        return hipErrorInvalidValue;
    } else if constexpr (use_persist<CIN, TN>()) {
        constexpr int CTH = persist_cth<CIN, TN>();
        const int tiles = x.B * ((x.H + CTH - 1) / CTH) * ((x.W + CT_W - 1) / CT_W);
        int per_cu = 0;
        const hipError_t oc = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu,
                                                                           conv3x3_persist_kernel<CIN, TN, CTH, CE>, 256, 0);
        if (oc != hipSuccess) return oc;
        const int wgs = std::min(tiles, std::max(1, per_cu) * cu_count);
        conv3x3_persist_kernel<CIN, TN, CTH, CE><<<dim3(wgs, (N + TN - 1) / TN), 256, 0, st>>>(x, w, conv_ep(e), N,
                                                                                            tiles);
    } else {
        constexpr int CTH = CONV_GEN_CTH;
        const int tiles = x.B * ((x.H + CTH - 1) / CTH) * ((x.W + CT_W - 1) / CT_W);
        conv3x3_kernel<CIN, TN, CE><<<dim3(tiles, (N + TN - 1) / TN), 256, 0, st>>>(x, w, conv_ep(e), N);
    }
    return hipGetLastError();
}

}  // namespace cnn
}  // namespace pyhst
