// Learned sparse-angle corrector: a U-Net (encoder-decoder with skip
// connections) applied as x_hat = x + f(x) to FBP slices, trained and run with
// the MFMA BF16 implicit-GEMM kernels of cnn_gemm.hpp.  Not part of the paper
// (its learned prior is an overlapping-patch dictionary); it serves the same
// purpose: reconstruction quality from reduced data.
//
// Layout: activations NHWC BF16; master weights, gradients and Adam moments
// FP32 in one flat array.  Conv weights [co][tap][ci] (tap = 3 ty + tx),
// transposed-conv weights [d][co][ci] (d = 2 dy + dx), head [c] then bias.
// Every conv and transposed conv is followed by ReLU; the head is linear.
// Gradients of activations are BF16 and already multiplied by the ReLU mask of
// the activation they belong to; weight gradients are split-K partial sums
// reduced in a fixed order (deterministic).
#include <cmath>
#include <cstring>
#include <vector>

#include "cnn_conv.hpp"
#include "cnn_gemm.hpp"
#include "cnn_wgrad.hpp"
#include "internal.hpp"

using namespace pyhst;
using namespace pyhst::cnn;

namespace {

struct Conv {
    int cin, cout;          // cin as stored (first layer: 8, of which 1 is real)
    int64_t w, b;           // offsets in the flat parameter array
    bf16_t *wf, *wb;        // [co][tap][ci], [ci][8 - tap][co]
};
struct Up {
    int cin, cout;
    int64_t w, b;
    bf16_t *uf, *ub;        // [(d, co)][ci], [ci][(d, co)]
};
struct Buf {                // an activation and its gradient, same layout
    bf16_t *a, *g;
    int H, W, C;            // C = channel stride
};

int tn_for(int n) { return n >= 128 ? 128 : (n >= 64 ? 64 : 32); }

// K tile of the weight-gradient GEMMs (K = pixels, millions): deeper than the default to halve the
// barriers per MFMA
constexpr int TKW = 64;

}  // namespace

struct pyhst_unet {
    int B, H, W, base, L;
    int cu_count = 256;
    float scale = 1.0f;   // data scale: the network sees scale x and returns x + f(scale x) / scale
    int64_t n_params = 0;
    float *params = nullptr, *grads = nullptr, *m = nullptr, *v = nullptr;
    int *step = nullptr;
    std::vector<Conv> enc_a, enc_b, dec_a, dec_b;   // enc: levels 0..L-1 (L-1 = bottleneck); dec: 0..L-2
    std::vector<Up> up;                             // up[l]: level l+1 -> l
    int64_t head_w = 0, head_b = 0;
    Buf x8;
    float *w0 = nullptr;                            // first conv's weights, BF16-rounded, as FP32 [co][tap]
    std::vector<Buf> ea, cat, pool, da, db;         // ea[l]: enc conv a out; cat[l]: [enc b out | up out]
    Buf bott_b;                                     // bottleneck conv b out
    float *out = nullptr, *dout = nullptr;
    float *part = nullptr;                          // split-K partials / reduction partials
    size_t part_floats = 0;
    double *dpart = nullptr;
    void *block = nullptr;
};

namespace {

// ---------------------------------------------------------------- small kernels
unsigned blocks_for(int64_t n, int64_t cap = 16384)
{
    int64_t b = (n + 255) / 256;
    return (unsigned)std::max<int64_t>(1, std::min(b, cap));
}

#define GRID_LOOP(i, n) for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < (n); i += (int64_t)gridDim.x * blockDim.x)

// x8 = [scale x, 0, ..., 0] in BF16 (8 channels, only the first carries the image)
__global__ void input_pad_kernel(const float *x, int64_t npix, bf16_t *x8, float scale)
{
    GRID_LOOP(p, npix)
    {
        uint4 v = make_uint4(f2bf(x[p] * scale), 0, 0, 0);
        *(uint4 *)(x8 + p * 8) = v;
    }
}

// First encoder conv (one real input channel) straight from the FP32 input:
//   y[p][n] = bf16(relu(sum_tap w[n][tap] xs[p + tap] + bias[n])), xs = bf16(scale x), zero outside the image,
// with the BF16-rounded weights of the MFMA path (w0, kept as FP32; FP32 sums).  One thread per pixel and
// all C outputs: the weights are the same for every lane (scalar loads, scalar operands of the FMAs) and
// the nine inputs are loaded once per pixel.  The outputs (C channels per pixel, contiguous in y) go
// through LDS so that every store instruction writes 1 KB of consecutive memory.
template <int C>
__global__ __launch_bounds__(256) void conv_first_kernel(const float *x, FastDiv fw, FastDiv fh, int npix, float scale,
                                                         const float *__restrict__ w0, const float *__restrict__ bias,
                                                         bf16_t *y)
{
    constexpr int Q = C / 8;   // 16-byte pieces per pixel
    __shared__ uint4 sO[256 * Q];
    const int W = (int)fw.d, H = (int)fh.d;
    const int p0 = blockIdx.x * blockDim.x;   // one pixel per thread, no loop: the weights are loaded
    const int p = p0 + threadIdx.x;           // as they are used, not held
    if (p < npix) {
        const uint32_t row = fdiv((uint32_t)p, fw);
        const int xx = p - (int)(row * fw.d), yy = (int)(row - fdiv(row, fh) * fh.d);
        // the nine loads issue together: a neighbour outside the image reads the pixel itself instead
        // (always inside) and is then replaced by zero
        float v[9];
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            const int dy = t / 3 - 1, dx = t % 3 - 1;
            const int oy = (unsigned)(yy + dy) < (unsigned)H ? dy : 0, ox = (unsigned)(xx + dx) < (unsigned)W ? dx : 0;
            v[t] = x[(int64_t)p + oy * W + ox];
        }
        float xs[9];
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            const int dy = t / 3 - 1, dx = t % 3 - 1;
            const bool in = (unsigned)(yy + dy) < (unsigned)H && (unsigned)(xx + dx) < (unsigned)W;
            xs[t] = in ? bf16_lo(pack_bf16x2(v[t] * scale, 0.0f)) : 0.0f;
        }
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            uint32_t o[4];
#pragma unroll
            for (int k = 0; k < 8; k += 2) {
                const int n = 8 * q + k;
                float s0 = 0.0f, s1 = 0.0f;
#pragma unroll
                for (int t = 0; t < 9; ++t) {
                    s0 = fmaf(w0[9 * n + t], xs[t], s0);
                    s1 = fmaf(w0[9 * (n + 1) + t], xs[t], s1);
                }
                o[k / 2] = pack_bf16x2(fmaxf(s0 + bias[n], 0.0f), fmaxf(s1 + bias[n + 1], 0.0f));
            }
            // piece q of pixel t at slot t Q + (q ^ (t % Q)): the lanes of a write spread over the banks
            sO[threadIdx.x * Q + (q ^ (threadIdx.x & (Q - 1)))] = make_uint4(o[0], o[1], o[2], o[3]);
        }
    }
    __syncthreads();
    // piece i of the block's output (pixel p0 + i / Q, piece i % Q): thread threadIdx.x takes
    // i = threadIdx.x + 256 k, consecutive threads consecutive 16 bytes
#pragma unroll
    for (int k = 0; k < Q; ++k) {
        const int i = (int)threadIdx.x + 256 * k, t = i / Q, q = i % Q;
        if (p0 + t < npix) *(uint4 *)(y + ((int64_t)p0 * C + 8 * (int64_t)i)) = sO[t * Q + (q ^ (t & (Q - 1)))];
    }
}

// the first conv by conv_first_kernel for the channel counts it is built for; false: not handled
bool conv_first(const float *x, int n, int H, int W, float scale, const float *w0, const float *bias, int cout,
                bf16_t *y, int ycs, hipStream_t st)
{
    if (ycs != cout) return false;   // the kernel writes contiguous pixels
    const int npix = n * H * W;
    const dim3 grid((unsigned)((npix + 255) / 256));
    const FastDiv fw = make_fastdiv((uint32_t)W), fh = make_fastdiv((uint32_t)H);
    switch (cout) {
    case 8: conv_first_kernel<8><<<grid, 256, 0, st>>>(x, fw, fh, npix, scale, w0, bias, y); return true;
    case 16: conv_first_kernel<16><<<grid, 256, 0, st>>>(x, fw, fh, npix, scale, w0, bias, y); return true;
    case 32: conv_first_kernel<32><<<grid, 256, 0, st>>>(x, fw, fh, npix, scale, w0, bias, y); return true;
    case 64: conv_first_kernel<64><<<grid, 256, 0, st>>>(x, fw, fh, npix, scale, w0, bias, y); return true;
    default: return false;
    }
}

// 2x2 max pool: in [b][H][W] (C = 8 G channels at in.co, stride in.cs) -> out [b][H/2][W/2] (stride ocs);
// one thread per (output pixel, 8 channels): four 16-byte loads, one 16-byte store.  Pixel indices
// (below 2^31) in 32 bits, divided by multiply-shift.
struct PoolIdx {
    int lgG;          // G = 1 << lgG groups of 8 channels
    FastDiv fw, fhw;  // pooled width, pooled height x width
};
PoolIdx pool_idx(int H, int W, int C)
{
    int lg = 0;
    while ((8 << lg) < C) ++lg;
    return PoolIdx{lg, make_fastdiv((uint32_t)(W >> 1)), make_fastdiv((uint32_t)((H >> 1) * (W >> 1)))};
}
__device__ __forceinline__ int64_t pool_src(const Act &in, const PoolIdx &q, uint32_t p)
{
    const uint32_t b = fdiv(p, q.fhw), r = p - b * q.fhw.d, y = fdiv(r, q.fw), x = r - y * q.fw.d;
    return ((int64_t)(b * in.H + 2 * y) * in.W + 2 * x) * in.cs + in.co;
}

__global__ void pool_fwd_kernel(Act in, PoolIdx q, bf16_t *out, int ocs, int64_t n)
{
    GRID_LOOP(i, n)
    {
        const int g = (int)(i & ((1 << q.lgG) - 1));
        const uint32_t p = (uint32_t)(i >> q.lgG);
        const bf16_t *base = in.p + pool_src(in, q, p) + 8 * g;
        const int64_t row = (int64_t)in.W * in.cs;
        const uint4 q0 = *(const uint4 *)base, q1 = *(const uint4 *)(base + in.cs);
        const uint4 q2 = *(const uint4 *)(base + row), q3 = *(const uint4 *)(base + row + in.cs);
        const bf16_t *e0 = (const bf16_t *)&q0, *e1 = (const bf16_t *)&q1, *e2 = (const bf16_t *)&q2,
                     *e3 = (const bf16_t *)&q3;
        uint4 r;
        bf16_t *er = (bf16_t *)&r;
#pragma unroll
        for (int c = 0; c < 8; ++c)
            er[c] = f2bf(fmaxf(fmaxf(bf2f(e0[c]), bf2f(e1[c])), fmaxf(bf2f(e2[c]), bf2f(e3[c]))));
        *(uint4 *)(out + (int64_t)p * ocs + 8 * g) = r;
    }
}

// route the pooled gradient to the first maximum (row-major in the 2x2 window), adding to dE; one
// thread per (output pixel, 8 channels), which owns those channels of the window's four pixels in dE
// (read and written back as 16-byte vectors)
__global__ void pool_bwd_kernel(Act e, bf16_t *de, const bf16_t *dp, int pcs, PoolIdx q, int64_t n)
{
    GRID_LOOP(i, n)
    {
        const int gq = (int)(i & ((1 << q.lgG) - 1));
        const uint32_t p = (uint32_t)(i >> q.lgG);
        const uint4 gv = *(const uint4 *)(dp + (int64_t)p * pcs + 8 * gq);
        const bf16_t *ge = (const bf16_t *)&gv;
        const int64_t o0 = pool_src(e, q, p) + 8 * gq;
        const int64_t off[4] = {0, e.cs, (int64_t)e.W * e.cs, (int64_t)e.W * e.cs + e.cs};
        uint4 a[4], d[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            a[k] = *(const uint4 *)(e.p + o0 + off[k]);
            d[k] = *(const uint4 *)(de + o0 + off[k]);
        }
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const float g = bf2f(ge[c]);
            int arg = 0;
            float mx = bf2f(((const bf16_t *)&a[0])[c]);
#pragma unroll
            for (int k = 1; k < 4; ++k) {
                const float v = bf2f(((const bf16_t *)&a[k])[c]);
                if (v > mx) {
                    mx = v;
                    arg = k;
                }
            }
            if (mx > 0.0f && g != 0.0f) {
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    if (k == arg) {
                        bf16_t *t = (bf16_t *)&d[k] + c;
                        *t = f2bf(bf2f(*t) + g);
                    }
            }
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) *(uint4 *)(de + o0 + off[k]) = d[k];
    }
}

// out = v / scale (unscale) or v, with v = scale x + head(d): the residual output in the network's units
__global__ void head_fwd_kernel(const bf16_t *d, int C, const float *wh, const float *bh, const float *x, float *out,
                                int64_t npix, float scale, int unscale)
{
    GRID_LOOP(p, npix)
    {
        float s = 0.0f;
        for (int c0 = 0; c0 < C; c0 += 8) {
            const uint4 q = *(const uint4 *)(d + p * C + c0);
            const bf16_t *e = (const bf16_t *)&q;
#pragma unroll
            for (int c = 0; c < 8; ++c) s = fmaf(bf2f(e[c]), wh[c0 + c], s);
        }
        const float v = x[p] * scale + (bh[0] + s);
        out[p] = unscale ? v / scale : v;
    }
}

__device__ inline double block_sum_d(double v, double *sh)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += sh[i];
    return t;
}

// loss partials: sum (out - scale t)^2 per block; dout = 2 (out - scale t) / n
__global__ __launch_bounds__(256) void mse_kernel(const float *out, const float *t, float *dout, int64_t n,
                                                  double *partials, float scale)
{
    __shared__ double sh[4];
    double acc = 0.0;
    const float sc = 2.0f / (float)n;
    GRID_LOOP(p, n)
    {
        const float d = out[p] - t[p] * scale;
        acc += (double)d * d;
        dout[p] = sc * d;
    }
    const double s = block_sum_d(acc, sh);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void final_mean_kernel(const double *partials, int nb, int64_t n, float *loss)
{
    __shared__ double sh[4];
    double acc = 0.0;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) acc += partials[i];
    const double s = block_sum_d(acc, sh);
    if (threadIdx.x == 0 && loss) *loss = (float)(s / (double)n);
}

// dD[p][c] = bf16(dout[p] wh[c]) where D > 0 (C <= 256 threads per pixel chunk)
// one thread per (pixel, 8 channels)
__global__ void head_bwd_data_kernel(const bf16_t *d, int C, const float *wh, const float *dout, bf16_t *dd,
                                     int64_t n)
{
    const int G = C >> 3;
    GRID_LOOP(i, n)
    {
        const int g = (int)(i % G);
        const int64_t p = i / G;
        const uint4 q = *(const uint4 *)(d + p * C + 8 * g);
        const bf16_t *e = (const bf16_t *)&q;
        const float go = dout[p];
        uint4 r;
        bf16_t *er = (bf16_t *)&r;
#pragma unroll
        for (int c = 0; c < 8; ++c) er[c] = f2bf(bf2f(e[c]) > 0.0f ? go * wh[8 * g + c] : 0.0f);
        *(uint4 *)(dd + p * C + 8 * g) = r;
    }
}

// per-block partial sums over pixels of v[p][c] * (s ? s[p] : 1), channel c = threadIdx.x (< C)
// part[blk][c] = sum over this block's pixel chunk of v[p][co + c] (times s[p] when s is given).
// Thread t reads 8 channels (16 B) of one pixel per step: channel group t % G (G = C / 8), pixel
// lane t / G; the pixel lanes' sums are then added in a fixed order through LDS.  C is a power of
// two in [8, 2048]; cs and co are multiples of 8.
__global__ __launch_bounds__(256) void chan_partial_kernel(const bf16_t *v, int cs, int co, int C, const float *s,
                                                           int64_t npix, int64_t chunk, float *part)
{
    __shared__ float red[256 * 8];
    const int G = C >> 3;
    const int lanes = G >= 256 ? 1 : 256 / G;
    const int cg = threadIdx.x % G, pl = threadIdx.x / G;
    const int64_t p0 = blockIdx.x * chunk, p1 = min(npix, p0 + chunk);
    float acc[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) acc[q] = 0.0f;
    if (pl < lanes) {
        for (int64_t p = p0 + pl; p < p1; p += lanes) {
            const uint4 u = *(const uint4 *)(v + p * cs + co + 8 * cg);
            const bf16_t *e = (const bf16_t *)&u;
            const float w = s ? s[p] : 1.0f;
#pragma unroll
            for (int q = 0; q < 8; ++q) acc[q] = fmaf(bf2f(e[q]), w, acc[q]);
        }
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) red[threadIdx.x * 8 + q] = acc[q];
    __syncthreads();
    for (int c = threadIdx.x; c < C; c += blockDim.x) {
        const int g = c >> 3, q = c & 7;
        float t = 0.0f;
        for (int l = 0; l < lanes; ++l) t += red[(l * G + g) * 8 + q];
        part[(int64_t)blockIdx.x * C + c] = t;
    }
}

__global__ __launch_bounds__(256) void dout_partial_kernel(const float *d, int64_t npix, int64_t chunk, float *part)
{
    __shared__ double sh[4];
    const int64_t p0 = blockIdx.x * chunk, p1 = min(npix, p0 + chunk);
    double acc = 0.0;
    for (int64_t p = p0 + threadIdx.x; p < p1; p += blockDim.x) acc += d[p];
    const double s = block_sum_d(acc, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = (float)s;
}

// dst[c] = sum over nb blocks of part[blk][c] (one workgroup per channel, fixed order)
__global__ __launch_bounds__(256) void reduce_rows_kernel(const float *part, int nb, int C, float *dst)
{
    __shared__ double sh[4];
    const int c = blockIdx.x;
    double acc = 0.0;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) acc += part[(int64_t)i * C + c];
    const double t = block_sum_d(acc, sh);
    if (threadIdx.x == 0) dst[c] = (float)t;
}

// dst[n * M + m] = sum_s part[s][m][n].  A workgroup takes 64 consecutive outputs i = m N + n; its
// 4 wavefronts sum the splits s = w, w + 4, ... (consecutive lanes read consecutive n) and the 4
// partial sums are added in a fixed order.
// 64 outputs per workgroup, its 16 wavefronts take every 16th split (the weight-gradient GEMMs of the
// narrow layers have few outputs and many splits: the waves keep enough loads in flight); the 16
// partial sums are added in a fixed order
constexpr int RSK_WAVES = 16;
__global__ __launch_bounds__(64 * RSK_WAVES) void reduce_splitk_T_kernel(const float *part, int splits, int M, int N,
                                                                         float *dst)
{
    __shared__ double red[RSK_WAVES][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t i = (int64_t)blockIdx.x * 64 + lane, MN = (int64_t)M * N;
    double s = 0.0;
    if (i < MN)
        for (int k = w; k < splits; k += RSK_WAVES) s += part[(int64_t)k * MN + i];
    red[w][lane] = s;
    __syncthreads();
    if (w == 0 && i < MN) {
        double t = red[0][lane];
#pragma unroll
        for (int q = 1; q < RSK_WAVES; ++q) t += red[q][lane];
        const int m = (int)(i / N), n = (int)(i - (int64_t)m * N);
        dst[(int64_t)n * M + m] = (float)t;
    }
}

__global__ void adam_kernel(float *p, const float *g, float *m, float *v, int64_t n, const int *step, float lr,
                            float b1, float b2, float eps)
{
    const int t = *step + 1;
    const float c1 = 1.0f - powf(b1, (float)t), c2 = 1.0f - powf(b2, (float)t);
    GRID_LOOP(i, n)
    {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.0f - b1) * gi;
        const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    }
}

__global__ void step_inc_kernel(int *step) { *step += 1; }

// master W[co][tap][ci] -> wf (same layout) and wb[ci][8 - tap][co]
__global__ void cast_conv_kernel(const float *w, int cin, int cout, bf16_t *wf, bf16_t *wb)
{
    GRID_LOOP(i, (int64_t)cout * 9 * cin)
    {
        const int ci = (int)(i % cin), tap = (int)((i / cin) % 9), co = (int)(i / (9 * (int64_t)cin));
        const bf16_t b = f2bf(w[i]);
        wf[i] = b;
        wb[((int64_t)ci * 9 + (8 - tap)) * cout + co] = b;
    }
}

// first conv (cin 8, of which channel 0 is real): w0[co][tap] = bf16(W[co][tap][0]) as FP32
__global__ void cast_first_kernel(const float *w, int cout, float *w0)
{
    GRID_LOOP(i, (int64_t)cout * 9) w0[i] = bf2f(f2bf(w[i * 8]));
}

// master U[d][co][ci] -> uf (same layout) and ub[ci][(d, co)]
__global__ void cast_up_kernel(const float *u, int cin, int cout, bf16_t *uf, bf16_t *ub)
{
    GRID_LOOP(i, (int64_t)4 * cout * cin)
    {
        const int ci = (int)(i % cin);
        const int64_t dco = i / cin;
        const bf16_t b = f2bf(u[i]);
        uf[i] = b;
        ub[(int64_t)ci * 4 * cout + dco] = b;
    }
}

__global__ void fill_f32_kernel(float *p, int64_t n, float v)
{
    GRID_LOOP(i, n) p[i] = v;
}
__global__ void fill_i32_kernel(int *p, int v) { *p = v; }

// ---------------------------------------------------------------- layer drivers
Act act(const Buf &b, int n, int co = 0, bool grad = false) { return Act{grad ? b.g : b.a, n, b.H, b.W, b.C, co}; }

// 3x3 convolution of x (cin channels) with weights w [n][9 cin] by the direct kernel, for the channel
// counts it is built for; false: not handled (the caller runs the implicit GEMM)
template <int TN, class EP>
bool conv_direct(int cin, const Act &x, const WeightB &w, const EP &e, int n, int cu, hipStream_t st, hipError_t &err)
{
    switch (cin) {
    case 8: err = run_conv3x3<8, TN>(x, w, e, n, cu, st); return true;
    case 16: err = run_conv3x3<16, TN>(x, w, e, n, cu, st); return true;
    case 32: err = run_conv3x3<32, TN>(x, w, e, n, cu, st); return true;
    case 64: err = run_conv3x3<64, TN>(x, w, e, n, cu, st); return true;
    case 128: err = run_conv3x3<128, TN>(x, w, e, n, cu, st); return true;
    case 256: err = run_conv3x3<256, TN>(x, w, e, n, cu, st); return true;
    default: return false;
    }
}

// N tile of the direct kernels: the GEMM's
int direct_tn(int, int n) { return tn_for(n); }

template <int TN>
bool direct_layout(int cin, int &bm, int &wn)
{
    switch (cin) {
#define PYHST_LAYOUT_CASE(C)         \
    case C:                          \
        bm = conv_bm<C, TN>();       \
        wn = conv_wn<C, TN>();       \
        return true;
        PYHST_LAYOUT_CASE(8)
        PYHST_LAYOUT_CASE(16)
        PYHST_LAYOUT_CASE(32)
        PYHST_LAYOUT_CASE(64)
        PYHST_LAYOUT_CASE(128)
        PYHST_LAYOUT_CASE(256)
#undef PYHST_LAYOUT_CASE
    default: return false;
    }
}

// wave layout of the direct kernel for (cin, n): row blocks per wavefront, wavefront columns, N tile
bool direct_kernel_layout(int cin, int n, int &bm, int &wn, int &tn)
{
    tn = direct_tn(cin, n);
    switch (tn) {
    case 128: return direct_layout<128>(cin, bm, wn);
    case 64: return direct_layout<64>(cin, bm, wn);
    default: return direct_layout<32>(cin, bm, wn);
    }
}

// the 2x2 max pool fits the epilogue of the layer's direct kernel (a wavefront holds both rows of
// its windows: an even number of consecutive tile rows)
bool pool_fusable(const Conv &L)
{
    int bm = 0, wn = 0, tn = 0;
    return direct_kernel_layout(L.cin, L.cout, bm, wn, tn) && bm % 2 == 0;
}
// the head fits the epilogue (one workgroup column holds every output channel in one wavefront)
bool head_fusable(const Conv &L)
{
    int bm = 0, wn = 0, tn = 0;
    return direct_kernel_layout(L.cin, L.cout, bm, wn, tn) && wn == 1 && tn >= L.cout;
}

template <class EP>
bool conv_direct_tn(int cin, const Act &x, const WeightB &w, const EP &e, int n, int cu, hipStream_t st,
                    hipError_t &err)
{
    switch (direct_tn(cin, n)) {
    case 128: return conv_direct<128>(cin, x, w, e, n, cu, st, err);
    case 64: return conv_direct<64>(cin, x, w, e, n, cu, st, err);
    default: return conv_direct<32>(cin, x, w, e, n, cu, st, err);
    }
}

hipError_t conv_fwd(const pyhst_unet &net, const Conv &L, Act in, bf16_t *out, int ocs, int oco, hipStream_t st)
{
    const int M = in.B * in.H * in.W;
    StoreAct E{out, ocs, oco, net.params + L.b, 1};
    WeightB Bw{L.wf, 9 * L.cin};
    hipError_t err = hipSuccess;
    if (conv_direct_tn(L.cin, in, Bw, E, L.cout, net.cu_count, st, err)) return err;
    Im2colA A = im2col_a(in, L.cin);
    switch (tn_for(L.cout)) {
    case 128: return run_gemm<Im2colA, WeightB, StoreAct, 128>(A, Bw, E, M, L.cout, 9 * L.cin, 1, st);
    case 64: return run_gemm<Im2colA, WeightB, StoreAct, 64>(A, Bw, E, M, L.cout, 9 * L.cin, 1, st);
    default: return run_gemm<Im2colA, WeightB, StoreAct, 32>(A, Bw, E, M, L.cout, 9 * L.cin, 1, st);
    }
}

// conv + ReLU into out and its 2x2 max pool into pool, one kernel (pool_fusable(L))
hipError_t conv_fwd_pool(const pyhst_unet &net, const Conv &L, Act in, bf16_t *out, int ocs, bf16_t *pool, int pcs,
                         hipStream_t st)
{
    ConvStoreActPool E;
    E.y = out;
    E.cs = ocs;
    E.co = 0;
    E.bias = net.params + L.b;
    E.pool = pool;
    E.pcs = pcs;
    hipError_t err = hipSuccess;
    if (!conv_direct_tn(L.cin, in, WeightB{L.wf, 9 * L.cin}, E, L.cout, net.cu_count, st, err)) return hipErrorInvalidValue;
    return err;
}

// last decoder conv + ReLU with the head in its epilogue (head_fusable(L)): out = the network's output;
// act (may be null) receives the conv's activation
hipError_t conv_fwd_head(const pyhst_unet &net, const Conv &L, Act in, bf16_t *act_out, int acs, const float *x,
                         float *out, int unscale, hipStream_t st)
{
    ConvStoreHead E;
    E.y = act_out;
    E.cs = acs;
    E.co = 0;
    E.bias = net.params + L.b;
    E.wh = net.params + net.head_w;
    E.bh = net.params + net.head_b;
    E.xin = x;
    E.out = out;
    E.scale = net.scale;
    E.unscale = unscale;
    hipError_t err = hipSuccess;
    if (!conv_direct_tn(L.cin, in, WeightB{L.wf, 9 * L.cin}, E, L.cout, net.cu_count, st, err)) return hipErrorInvalidValue;
    return err;
}

hipError_t up_fwd(const pyhst_unet &net, const Up &L, Act in, bf16_t *out, int H2, int W2, int ocs, int oco,
                  hipStream_t st)
{
    hipError_t err = hipSuccess;
    if (H2 == 2 * in.H && W2 == 2 * in.W &&
        run_up2x2(in, L.uf, net.params + L.b, L.cin, L.cout, out, ocs, oco, net.cu_count, st, err))
        return err;
    const int M = in.B * in.H * in.W;
    PlainA A{in};
    WeightB Bw{L.uf, L.cin};
    StoreUp E = store_up(out, H2, W2, ocs, oco, L.cout, net.params + L.b);
    return run_gemm<PlainA, WeightB, StoreUp, 128>(A, Bw, E, M, 4 * L.cout, L.cin, 1, st);
}

// splits for a split-K weight gradient so that the grid has about 2048 workgroups
int splits_for(int M, int N, int TN, int K, size_t part_cap)
{
    const int tiles = ((M + TM - 1) / TM) * ((N + TN - 1) / TN);
    int s = std::max(1, 2048 / tiles);
    s = std::min(s, std::max(1, K / (4 * TK)));
    while (s > 1 && (size_t)s * M * N > part_cap) --s;
    int ks = (K + s - 1) / s;
    ks = (ks + TK - 1) / TK * TK;
    return (K + ks - 1) / ks;
}

hipError_t chan_sum(const pyhst_unet &net, Act g, int C, const float *scale, float *dst, hipStream_t st)
{
    const int64_t npix = (int64_t)g.B * g.H * g.W;
    const int nb = (int)std::min<int64_t>(1024, std::max<int64_t>(1, npix / 64));
    const int64_t chunk = (npix + nb - 1) / nb;
    chan_partial_kernel<<<nb, 256, 0, st>>>(g.p, g.cs, g.co, C, scale, npix, chunk, net.part);
    reduce_rows_kernel<<<C, 256, 0, st>>>(net.part, nb, C, dst);
    return hipGetLastError();
}

// dZ = gradient at this conv's (ReLU'd) output.  Writes dW, db; if dx != nullptr also dX (masked by X > 0).
hipError_t conv_bwd(const pyhst_unet &net, const Conv &L, Act x, Act dz, bf16_t *dx, int dxcs, int dxco,
                    hipStream_t st)
{
    const int npix = x.B * x.H * x.W;
    hipError_t e;
    // weight gradient: C[m = (tap, ci)][n = co] = sum_pix X[pix + off][ci] dZ[pix][co]
    const int wtiles = x.B * ((x.H + 7) / 8) * ((x.W + CT_W - 1) / CT_W);
    if (const int ws = wgrad_splits(L.cin, L.cout, wtiles, net.cu_count, net.part_floats)) {
        const int M = 9 * L.cin, N = L.cout;
        const int tps = (wtiles + ws - 1) / ws;
        float *bpart = net.part + (size_t)4 * ws * M * N;
        wgrad3x3_kernel<<<dim3(ws, N / 32, L.cin / 32), 256, 0, st>>>(x, dz, net.part, bpart, L.cin, N, wtiles, tps);
        reduce_splitk_T_kernel<<<(unsigned)(((int64_t)M * N + 63) / 64), 64 * RSK_WAVES, 0, st>>>(net.part, 4 * ws, M,
                                                                                                N, net.grads + L.w);
        reduce_rows_kernel<<<N, 256, 0, st>>>(bpart, ws, N, net.grads + L.b);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    } else {
        const int M = 9 * L.cin, N = L.cout, tn = tn_for(N);
        const int s = splits_for(M, N, tn, npix, net.part_floats);
        Im2colT A = im2col_t(x, L.cin);
        PlainT Bz{dz};
        StorePartial E{net.part, M, N};
        int ks = (npix + s - 1) / s;
        ks = (ks + TKW - 1) / TKW * TKW;
        const int sp = (npix + ks - 1) / ks;
        dim3 grid((M + TM - 1) / TM, (N + tn - 1) / tn, sp);
        if (tn == 128) gemm_kernel<Im2colT, PlainT, StorePartial, 128, TM, TKW><<<grid, 256, 0, st>>>(A, Bz, E, M, N, npix, ks);
        else if (tn == 64) gemm_kernel<Im2colT, PlainT, StorePartial, 64, TM, TKW><<<grid, 256, 0, st>>>(A, Bz, E, M, N, npix, ks);
        else gemm_kernel<Im2colT, PlainT, StorePartial, 32, TM, TKW><<<grid, 256, 0, st>>>(A, Bz, E, M, N, npix, ks);
        reduce_splitk_T_kernel<<<(unsigned)(((int64_t)M * N + 63) / 64), 64 * RSK_WAVES, 0, st>>>(net.part, sp, M, N, net.grads + L.w);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if ((e = chan_sum(net, dz, L.cout, nullptr, net.grads + L.b, st)) != hipSuccess) return e;
    }
    if (dx) {
        // dX[pix][ci] = sum_{tap', co} dZ[pix + off(tap')][co] Wb[ci][tap'][co], masked by X > 0
        const int M = npix, N = L.cin;
        StoreMasked E{dx, dxcs, dxco, x.p, x.cs, x.co};
        WeightB Bw{L.wb, 9 * L.cout};
        if (conv_direct_tn(L.cout, dz, Bw, E, N, net.cu_count, st, e)) return e;
        Im2colA A = im2col_a(dz, L.cout);
        switch (tn_for(N)) {
        case 128: e = run_gemm<Im2colA, WeightB, StoreMasked, 128>(A, Bw, E, M, N, 9 * L.cout, 1, st); break;
        case 64: e = run_gemm<Im2colA, WeightB, StoreMasked, 64>(A, Bw, E, M, N, 9 * L.cout, 1, st); break;
        default: e = run_gemm<Im2colA, WeightB, StoreMasked, 32>(A, Bw, E, M, N, 9 * L.cout, 1, st); break;
        }
    }
    return e;
}

// transposed conv backward.  x: low-res input, dy: high-res gradient (channels at its co), dx: input gradient
hipError_t up_bwd(const pyhst_unet &net, const Up &L, Act x, Act dy, bf16_t *dx, int dxcs, hipStream_t st)
{
    const int npix = x.B * x.H * x.W;
    hipError_t e;
    {
        const int M = L.cin, N = 4 * L.cout, tn = tn_for(N);
        const int s = splits_for(M, N, tn, npix, net.part_floats);
        PlainT A{x};
        UpGatherT Bz = upgather_t(dy, L.cout);
        StorePartial E{net.part, M, N};
        int ks = (npix + s - 1) / s;
        ks = (ks + TKW - 1) / TKW * TKW;
        const int sp = (npix + ks - 1) / ks;
        dim3 grid((M + TM - 1) / TM, (N + tn - 1) / tn, sp);
        if (tn == 128) gemm_kernel<PlainT, UpGatherT, StorePartial, 128, TM, TKW><<<grid, 256, 0, st>>>(A, Bz, E, M, N, npix, ks);
        else if (tn == 64) gemm_kernel<PlainT, UpGatherT, StorePartial, 64, TM, TKW><<<grid, 256, 0, st>>>(A, Bz, E, M, N, npix, ks);
        else gemm_kernel<PlainT, UpGatherT, StorePartial, 32, TM, TKW><<<grid, 256, 0, st>>>(A, Bz, E, M, N, npix, ks);
        reduce_splitk_T_kernel<<<(unsigned)(((int64_t)M * N + 63) / 64), 64 * RSK_WAVES, 0, st>>>(net.part, sp, M, N, net.grads + L.w);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if ((e = chan_sum(net, dy, L.cout, nullptr, net.grads + L.b, st)) != hipSuccess) return e;
    const int M = npix, N = L.cin;
    UpGatherA A = upgather_a(dy, L.cout);
    WeightB Bw{L.ub, 4 * L.cout};
    StoreMasked E{dx, dxcs, 0, x.p, x.cs, x.co};
    switch (tn_for(N)) {
    case 128: return run_gemm<UpGatherA, WeightB, StoreMasked, 128>(A, Bw, E, M, N, 4 * L.cout, 1, st);
    case 64: return run_gemm<UpGatherA, WeightB, StoreMasked, 64>(A, Bw, E, M, N, 4 * L.cout, 1, st);
    default: return run_gemm<UpGatherA, WeightB, StoreMasked, 32>(A, Bw, E, M, N, 4 * L.cout, 1, st);
    }
}

hipError_t cast_all(const pyhst_unet &net, hipStream_t st)
{
    auto cc = [&](const Conv &c) {
        cast_conv_kernel<<<blocks_for((int64_t)c.cout * 9 * c.cin), 256, 0, st>>>(net.params + c.w, c.cin, c.cout,
                                                                                  c.wf, c.wb);
    };
    for (auto &c : net.enc_a) cc(c);
    cast_first_kernel<<<1, 256, 0, st>>>(net.params + net.enc_a[0].w, net.enc_a[0].cout, net.w0);
    for (auto &c : net.enc_b) cc(c);
    for (auto &c : net.dec_a) cc(c);
    for (auto &c : net.dec_b) cc(c);
    for (auto &u : net.up)
        cast_up_kernel<<<blocks_for((int64_t)4 * u.cout * u.cin), 256, 0, st>>>(net.params + u.w, u.cin, u.cout,
                                                                                u.uf, u.ub);
    return hipGetLastError();
}

// unscale = 1: out in the caller's units; 0: in the network's (scaled) units.  keep: store every
// activation the backward pass reads (without it the last decoder conv's output, which only the fused
// head reads, is not written)
hipError_t forward(pyhst_unet &net, const float *in, int n, float *out, int unscale, bool keep, hipStream_t st)
{
    const int L = net.L;
    hipError_t e;
    const int64_t npix = (int64_t)n * net.H * net.W;
    const Conv &c0 = net.enc_a[0];
    // inference: the first conv runs inside the second's kernel (its activation is never stored), with
    // the level's pool in the epilogue
    bool pair0 = false;
    if (!keep && L > 1 && net.enc_b[0].cin == c0.cout) {
        ConvStoreActPool E;
        E.y = net.cat[0].a;
        E.cs = net.cat[0].C;
        E.co = 0;
        E.bias = net.params + net.enc_b[0].b;
        E.pool = net.pool[0].a;
        E.pcs = net.pool[0].C;
        hipError_t err = hipSuccess;
        pair0 = run_conv_pair0(in, net.scale, net.w0, net.params + c0.b, act(net.x8, n),
                               WeightB{net.enc_b[0].wf, 9 * net.enc_b[0].cin}, E, c0.cout, net.enc_b[0].cout,
                               net.cu_count, st, err);
        if (err != hipSuccess) return err;
    }
    const bool first = pair0 || conv_first(in, n, net.H, net.W, net.scale, net.w0, net.params + c0.b, c0.cout,
                                           net.ea[0].a, net.ea[0].C, st);
    if (keep || !first)   // the first conv's input as the backward pass reads it (8 channels, the first one real)
        input_pad_kernel<<<blocks_for(npix), 256, 0, st>>>(in, npix, net.x8.a, net.scale);
    Act cur = act(net.x8, n);
    for (int l = 0; l < L; ++l) {
        const bool bott = l == L - 1;
        if (l == 0 && pair0) {   // enc0a + enc0b + pool done
            cur = act(net.pool[0], n);
            continue;
        }
        if ((l > 0 || !first) && (e = conv_fwd(net, net.enc_a[l], cur, net.ea[l].a, net.ea[l].C, 0, st)) != hipSuccess)
            return e;
        Act a = act(net.ea[l], n);
        if (bott) {
            if ((e = conv_fwd(net, net.enc_b[l], a, net.bott_b.a, net.bott_b.C, 0, st)) != hipSuccess) return e;
        } else if (pool_fusable(net.enc_b[l])) {
            if ((e = conv_fwd_pool(net, net.enc_b[l], a, net.cat[l].a, net.cat[l].C, net.pool[l].a, net.pool[l].C,
                                   st)) != hipSuccess)
                return e;
            cur = act(net.pool[l], n);
        } else {
            if ((e = conv_fwd(net, net.enc_b[l], a, net.cat[l].a, net.cat[l].C, 0, st)) != hipSuccess) return e;
            const int c = net.enc_b[l].cout;
            const int64_t np = (int64_t)n * net.pool[l].H * net.pool[l].W * c;
            pool_fwd_kernel<<<blocks_for(np / 8), 256, 0, st>>>(act(net.cat[l], n), pool_idx(net.cat[l].H, net.cat[l].W, c),
                                                                net.pool[l].a, net.pool[l].C, np / 8);
            cur = act(net.pool[l], n);
        }
    }
    Act below = act(net.bott_b, n);
    for (int l = L - 2; l >= 0; --l) {
        const Up &u = net.up[l];
        const Conv &da = net.dec_a[l];
        // inference: the up-sampling inside the first decoder conv where that conv takes the persistent
        // form (the concatenation's up half is then never stored)
        bool fused = false;
        if (!keep && net.enc_b[l].cout == u.cout && da.cin == 2 * u.cout) {
            hipError_t err = hipSuccess;
            fused = run_conv_upcat(act(net.cat[l], n), below, u.uf, net.params + u.b, WeightB{da.wf, 9 * da.cin},
                                   ConvStoreAct{net.da[l].a, net.da[l].C, 0, net.params + da.b}, u.cout, u.cin,
                                   da.cout, net.cu_count, st, err);
            if (err != hipSuccess) return err;
        }
        if (!fused) {
            if ((e = up_fwd(net, u, below, net.cat[l].a, net.cat[l].H, net.cat[l].W, net.cat[l].C, u.cout, st)) !=
                hipSuccess)
                return e;
            if ((e = conv_fwd(net, da, act(net.cat[l], n), net.da[l].a, net.da[l].C, 0, st)) != hipSuccess) return e;
        }
        if (l == 0 && head_fusable(net.dec_b[0]))
            return conv_fwd_head(net, net.dec_b[0], act(net.da[0], n), keep ? net.db[0].a : nullptr, net.db[0].C, in,
                                 out, unscale, st);
        if ((e = conv_fwd(net, net.dec_b[l], act(net.da[l], n), net.db[l].a, net.db[l].C, 0, st)) != hipSuccess)
            return e;
        below = act(net.db[l], n);
    }
    head_fwd_kernel<<<blocks_for(npix), 256, 0, st>>>(net.db[0].a, net.db[0].C, net.params + net.head_w,
                                                      net.params + net.head_b, in, out, npix, net.scale, unscale);
    return hipGetLastError();
}

hipError_t backward(pyhst_unet &net, const float *in, const float *target, int n, float *loss, hipStream_t st)
{
    hipError_t e = forward(net, in, n, net.out, 0, true, st);
    if (e != hipSuccess) return e;
    const int L = net.L;
    const int64_t npix = (int64_t)n * net.H * net.W;
    const int nb = (int)blocks_for(npix, 1024);
    mse_kernel<<<nb, 256, 0, st>>>(net.out, target, net.dout, npix, net.dpart, net.scale);
    final_mean_kernel<<<1, 256, 0, st>>>(net.dpart, nb, npix, loss);
    // head
    {
        const int C = net.db[0].C;
        head_bwd_data_kernel<<<blocks_for(npix * C / 8), 256, 0, st>>>(net.db[0].a, C, net.params + net.head_w,
                                                                       net.dout, net.db[0].g, npix * C / 8);
        Act d0 = act(net.db[0], n);
        if ((e = chan_sum(net, d0, C, net.dout, net.grads + net.head_w, st)) != hipSuccess) return e;
        const int pb = (int)std::min<int64_t>(1024, std::max<int64_t>(1, npix / 256));
        const int64_t chunk = (npix + pb - 1) / pb;
        dout_partial_kernel<<<pb, 256, 0, st>>>(net.dout, npix, chunk, net.part);
        reduce_rows_kernel<<<1, 256, 0, st>>>(net.part, pb, 1, net.grads + net.head_b);
    }
    // decoder, top (level 0) to bottom
    for (int l = 0; l <= L - 2; ++l) {
        // dec b: input da[l], grad at output db[l].g
        if ((e = conv_bwd(net, net.dec_b[l], act(net.da[l], n), act(net.db[l], n, 0, true), net.da[l].g,
                          net.da[l].C, 0, st)) != hipSuccess)
            return e;
        // dec a: input cat[l] -> gradient into cat[l].g (both halves, masked)
        if ((e = conv_bwd(net, net.dec_a[l], act(net.cat[l], n), act(net.da[l], n, 0, true), net.cat[l].g,
                          net.cat[l].C, 0, st)) != hipSuccess)
            return e;
        // up[l]: input = level l+1 output (bott_b or db[l+1]); its gradient is in cat[l].g channels [c, 2c)
        const Up &u = net.up[l];
        Buf &below = (l + 1 == L - 1) ? net.bott_b : net.db[l + 1];
        if ((e = up_bwd(net, u, act(below, n), act(net.cat[l], n, u.cout, true), below.g, below.C, st)) !=
            hipSuccess)
            return e;
    }
    // bottleneck and encoder, bottom to top
    for (int l = L - 1; l >= 0; --l) {
        const bool bott = l == L - 1;
        Act a = act(net.ea[l], n);
        Act dz_b = bott ? act(net.bott_b, n, 0, true) : act(net.cat[l], n, 0, true);
        if ((e = conv_bwd(net, net.enc_b[l], a, dz_b, net.ea[l].g, net.ea[l].C, 0, st)) != hipSuccess) return e;
        Act in = l == 0 ? act(net.x8, n) : act(net.pool[l - 1], n);
        bf16_t *din = l == 0 ? nullptr : net.pool[l - 1].g;
        if ((e = conv_bwd(net, net.enc_a[l], in, act(net.ea[l], n, 0, true), din, l == 0 ? 0 : net.pool[l - 1].C, 0,
                          st)) != hipSuccess)
            return e;
        if (l > 0) {
            // pool of level l-1: add its gradient into the encoder output of level l-1 (cat[l-1] channels [0, c))
            const int c = net.enc_b[l - 1].cout;
            const int64_t np = (int64_t)n * net.pool[l - 1].H * net.pool[l - 1].W * c;
            pool_bwd_kernel<<<blocks_for(np / 8), 256, 0, st>>>(act(net.cat[l - 1], n), net.cat[l - 1].g,
                                                                net.pool[l - 1].g, net.pool[l - 1].C,
                                                                pool_idx(net.cat[l - 1].H, net.cat[l - 1].W, c), np / 8);
        }
    }
    return hipGetLastError();
}

}  // namespace

extern "C" {

int pyhst_unet_create(int32_t batch, int32_t height, int32_t width, int32_t base, int32_t levels, pyhst_unet **out)
{
    if (!out) return fail(PYHST_EARG, "unet_create: out is NULL");
    *out = nullptr;
    if (batch <= 0 || levels < 2 || levels > 6 || base < 8 || (base & (base - 1)) != 0)
        return fail(PYHST_EARG, "unet_create: need batch > 0, 2 <= levels <= 6, base a power of two >= 8");
    if ((int64_t)batch * height * width >= (1ll << 31))
        return fail(PYHST_EARG, "unet_create: batch x height x width must stay below 2^31");
    const int div = 1 << (levels - 1);
    if (height <= 0 || width <= 0 || height % div || width % div)
        return fail(PYHST_EARG, "unet_create: height and width must be divisible by 2^(levels-1)");
    auto *net = new pyhst_unet();
    {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
            net->cu_count = cus;
    }
    net->B = batch;
    net->H = height;
    net->W = width;
    net->base = base;
    net->L = levels;
    const int L = levels;
    int64_t np = 0;
    auto conv = [&](int cin, int cout) {
        Conv c{cin, cout, np, 0, nullptr, nullptr};
        np += (int64_t)cout * 9 * cin;
        c.b = np;
        np += cout;
        return c;
    };
    auto upl = [&](int cin, int cout) {
        Up u{cin, cout, np, 0, nullptr, nullptr};
        np += (int64_t)4 * cout * cin;
        u.b = np;
        np += cout;
        return u;
    };
    for (int l = 0; l < L; ++l) {
        const int c = base << l, cin = l == 0 ? 8 : (base << (l - 1));
        net->enc_a.push_back(conv(cin, c));
        net->enc_b.push_back(conv(c, c));
    }
    net->up.resize(L - 1);
    net->dec_a.resize(L - 1);
    net->dec_b.resize(L - 1);
    for (int l = L - 2; l >= 0; --l) {
        const int c = base << l;
        net->up[l] = upl(2 * c, c);
        net->dec_a[l] = conv(2 * c, c);
        net->dec_b[l] = conv(c, c);
    }
    net->head_w = np;
    np += base;
    net->head_b = np;
    np += 1;
    net->n_params = np;

    // memory plan
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = (off + bytes + 255) & ~(size_t)255;
        return o;
    };
    struct Pending {
        Buf *b;
        size_t oa, og;
    };
    std::vector<Pending> bufs;
    auto buf = [&](Buf &b, int H, int W, int C) {
        b.H = H;
        b.W = W;
        b.C = C;
        const size_t bytes = (size_t)batch * H * W * C * sizeof(bf16_t);
        bufs.push_back({&b, take(bytes), take(bytes)});
    };
    net->ea.resize(L);
    net->cat.resize(L - 1);
    net->pool.resize(L - 1);
    net->da.resize(L - 1);
    net->db.resize(L - 1);
    buf(net->x8, height, width, 8);
    for (int l = 0; l < L; ++l) {
        const int H = height >> l, W = width >> l, c = base << l;
        buf(net->ea[l], H, W, c);
        if (l < L - 1) {
            buf(net->cat[l], H, W, 2 * c);
            buf(net->pool[l], H >> 1, W >> 1, c);
            buf(net->da[l], H, W, c);
            buf(net->db[l], H, W, c);
        } else {
            buf(net->bott_b, H, W, c);
        }
    }
    const size_t o_params = take(4 * np), o_grads = take(4 * np), o_m = take(4 * np), o_v = take(4 * np);
    const size_t o_step = take(64);
    const size_t o_out = take((size_t)4 * batch * height * width), o_dout = take((size_t)4 * batch * height * width);
    // partial buffer: the largest split-K partial set, and reduction partials
    size_t part = 0;
    auto need = [&](int M, int N, int K) {
        const int tn = tn_for(N);
        const int tiles = ((M + TM - 1) / TM) * ((N + tn - 1) / tn);
        int s = std::max(1, 2048 / tiles);
        s = std::min(s, std::max(1, K / (4 * TK)));
        part = std::max(part, (size_t)s * M * N);
    };
    for (int l = 0; l < L; ++l) {
        const int npix = batch * (height >> l) * (width >> l);
        need(9 * net->enc_a[l].cin, net->enc_a[l].cout, npix);
        need(9 * net->enc_b[l].cin, net->enc_b[l].cout, npix);
        if (l < L - 1) {
            need(9 * net->dec_a[l].cin, net->dec_a[l].cout, npix);
            need(9 * net->dec_b[l].cin, net->dec_b[l].cout, npix);
            need(net->up[l].cin, 4 * net->up[l].cout, npix / 4);
        }
    }
    part = std::max<size_t>(part, (size_t)1024 * 512);
    net->part_floats = part;
    const size_t o_part = take(4 * part), o_dpart = take(8 * 4096);
    const size_t o_w0 = take((size_t)4 * 9 * base);
    std::vector<std::pair<bf16_t **, size_t>> wbufs;
    auto wb = [&](bf16_t **p, int64_t n) { wbufs.push_back({p, take(2 * n)}); };
    for (auto *vec : {&net->enc_a, &net->enc_b, &net->dec_a, &net->dec_b})
        for (auto &c : *vec) {
            wb(&c.wf, (int64_t)c.cout * 9 * c.cin);
            wb(&c.wb, (int64_t)c.cout * 9 * c.cin);
        }
    for (auto &u : net->up) {
        wb(&u.uf, (int64_t)4 * u.cout * u.cin);
        wb(&u.ub, (int64_t)4 * u.cout * u.cin);
    }
    hipError_t e = hipMalloc(&net->block, off);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        delete net;
        return fail(PYHST_ENOMEM, "unet_create: hipMalloc failed");
    }
    e = hipMemset(net->block, 0, off);
    if (e != hipSuccess) {
        (void)hipFree(net->block);
        delete net;
        return hip_fail(e, "unet_create: hipMemset");
    }
    unsigned char *b = (unsigned char *)net->block;
    for (auto &p : bufs) {
        p.b->a = (bf16_t *)(b + p.oa);
        p.b->g = (bf16_t *)(b + p.og);
    }
    for (auto &p : wbufs) *p.first = (bf16_t *)(b + p.second);
    net->params = (float *)(b + o_params);
    net->grads = (float *)(b + o_grads);
    net->m = (float *)(b + o_m);
    net->v = (float *)(b + o_v);
    net->step = (int *)(b + o_step);
    net->w0 = (float *)(b + o_w0);
    net->out = (float *)(b + o_out);
    net->dout = (float *)(b + o_dout);
    net->part = (float *)(b + o_part);
    net->dpart = (double *)(b + o_dpart);
    *out = net;
    return PYHST_OK;
}

int pyhst_unet_destroy(pyhst_unet *net)
{
    if (!net) return PYHST_OK;
    if (net->block) (void)hipFree(net->block);
    delete net;
    return PYHST_OK;
}

int pyhst_unet_set_scale(pyhst_unet *net, float scale)
{
    if (!net || !(scale > 0.0f) || !std::isfinite(scale)) return fail(PYHST_EARG, "unet_set_scale: bad argument");
    net->scale = scale;
    return PYHST_OK;
}

int pyhst_unet_get_scale(const pyhst_unet *net, float *scale)
{
    if (!net || !scale) return fail(PYHST_EARG, "unet_get_scale: NULL argument");
    *scale = net->scale;
    return PYHST_OK;
}

int pyhst_unet_num_params(const pyhst_unet *net, int64_t *n)
{
    if (!net || !n) return fail(PYHST_EARG, "unet_num_params: NULL argument");
    *n = net->n_params;
    return PYHST_OK;
}

int pyhst_unet_set_params(pyhst_unet *net, const float *params, hipStream_t st)
{
    if (!net || !params) return fail(PYHST_EARG, "unet_set_params: NULL argument");
    hipError_t e = hipMemcpyAsync(net->params, params, 4 * net->n_params, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return hip_fail(e, "unet_set_params");
    fill_f32_kernel<<<blocks_for(net->n_params), 256, 0, st>>>(net->m, net->n_params, 0.0f);
    fill_f32_kernel<<<blocks_for(net->n_params), 256, 0, st>>>(net->v, net->n_params, 0.0f);
    fill_i32_kernel<<<1, 1, 0, st>>>(net->step, 0);
    e = cast_all(*net, st);
    return e == hipSuccess ? PYHST_OK : hip_fail(e, "unet_set_params");
}

int pyhst_unet_get_params(const pyhst_unet *net, float *params, hipStream_t st)
{
    if (!net || !params) return fail(PYHST_EARG, "unet_get_params: NULL argument");
    hipError_t e = hipMemcpyAsync(params, net->params, 4 * net->n_params, hipMemcpyDeviceToDevice, st);
    return e == hipSuccess ? PYHST_OK : hip_fail(e, "unet_get_params");
}

int pyhst_unet_get_grads(const pyhst_unet *net, float *grads, hipStream_t st)
{
    if (!net || !grads) return fail(PYHST_EARG, "unet_get_grads: NULL argument");
    hipError_t e = hipMemcpyAsync(grads, net->grads, 4 * net->n_params, hipMemcpyDeviceToDevice, st);
    return e == hipSuccess ? PYHST_OK : hip_fail(e, "unet_get_grads");
}

int pyhst_unet_forward(pyhst_unet *net, const float *in, int32_t n, float *out, hipStream_t st)
{
    if (!net || !in || !out) return fail(PYHST_EARG, "unet_forward: NULL argument");
    if (n <= 0 || n > net->B) return fail(PYHST_EARG, "unet_forward: n must be in [1, batch]");
    hipError_t e = forward(*net, in, n, out, 1, false, st);
    return e == hipSuccess ? PYHST_OK : hip_fail(e, "unet_forward");
}

int pyhst_unet_backward(pyhst_unet *net, const float *in, const float *target, int32_t n, float *loss,
                        hipStream_t st)
{
    if (!net || !in || !target) return fail(PYHST_EARG, "unet_backward: NULL argument");
    if (n <= 0 || n > net->B) return fail(PYHST_EARG, "unet_backward: n must be in [1, batch]");
    hipError_t e = backward(*net, in, target, n, loss, st);
    return e == hipSuccess ? PYHST_OK : hip_fail(e, "unet_backward");
}

int pyhst_unet_adam(pyhst_unet *net, float lr, float beta1, float beta2, float eps, hipStream_t st)
{
    if (!net || !(lr >= 0.0f)) return fail(PYHST_EARG, "unet_adam: bad argument");
    adam_kernel<<<blocks_for(net->n_params), 256, 0, st>>>(net->params, net->grads, net->m, net->v, net->n_params,
                                                           net->step, lr, beta1, beta2, eps);
    step_inc_kernel<<<1, 1, 0, st>>>(net->step);
    hipError_t e = cast_all(*net, st);
    return e == hipSuccess ? PYHST_OK : hip_fail(e, "unet_adam");
}

int pyhst_unet_train_step(pyhst_unet *net, const float *in, const float *target, int32_t n, float lr, float *loss,
                          hipStream_t st)
{
    int rc = pyhst_unet_backward(net, in, target, n, loss, st);
    if (rc) return rc;
    return pyhst_unet_adam(net, lr, 0.9f, 0.999f, 1e-8f, st);
}

}  // extern "C"

// Copy an internal BF16 buffer (activation or its gradient) for inspection.
// kind: 0 input (8 channels), 1 encoder conv-a output, 2 concatenation
// [encoder conv-b output | upsampled], 3 pooled, 4 decoder conv-a output,
// 5 decoder conv-b output, 6 bottleneck conv-b output.  Elements:
// batch x H_l x W_l x channel stride of that buffer.
extern "C" int pyhst_unet_tensor(const pyhst_unet *net, int32_t kind, int32_t level, int32_t grad, uint16_t *dst,
                                 int64_t elems, hipStream_t st)
{
    if (!net || !dst) return fail(PYHST_EARG, "unet_tensor: NULL argument");
    const Buf *b = nullptr;
    const int L = net->L;
    auto in = [&](int lo, int hi) { return level >= lo && level < hi; };
    switch (kind) {
    case 0: b = &net->x8; break;
    case 1: if (in(0, L)) b = &net->ea[level]; break;
    case 2: if (in(0, L - 1)) b = &net->cat[level]; break;
    case 3: if (in(0, L - 1)) b = &net->pool[level]; break;
    case 4: if (in(0, L - 1)) b = &net->da[level]; break;
    case 5: if (in(0, L - 1)) b = &net->db[level]; break;
    case 6: b = &net->bott_b; break;
    default: break;
    }
    if (!b) return fail(PYHST_EARG, "unet_tensor: bad kind/level");
    const int64_t n = (int64_t)net->B * b->H * b->W * b->C;
    if (elems != n) return fail(PYHST_EARG, "unet_tensor: wrong element count");
    hipError_t e = hipMemcpyAsync(dst, grad ? b->g : b->a, 2 * n, hipMemcpyDeviceToDevice, st);
    return e == hipSuccess ? PYHST_OK : hip_fail(e, "unet_tensor");
}
