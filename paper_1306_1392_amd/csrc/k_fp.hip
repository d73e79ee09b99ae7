// Matched forward projection A = s^2 B^T (section 2.3: the projector used
// inside the iterations; eq. (1)), evaluated ray-driven as a gather so that
// every bin is summed by one lane in a fixed order (deterministic).
//
// The paper projects an image held in a texture, which interpolates the image
// along rays and is not the transpose of the pixel-driven backprojector.  Here
// bin j of projection k sums exactly the pixels whose hat weight
// hat(t_k(px) - j) is non-zero.  Along an image line of the dominant axis
// (rows when |cos| >= |sin|, else columns) t is linear in the position,
// t - j = a (i - u), a = s cos (or s sin), so the bin touches the positions
// i in (u - 1/|a|, u + 1/|a|): at most ceil(2/|a|) of them.
//
// Three kernels compute the same sums (up to FP32 rounding order):
//   fp_staged_kernel  one to four projections per workgroup staged in LDS, whenever the
//                     candidate count per line is fixed (pixels of at least half a bin);
//   fp_kernel         angle blocks, for smaller pixels on plans with enough blocks to fill
//                     the chip;
//   fp_lines_kernel   one projection per workgroup read from global memory, for smaller
//                     pixels on smaller plans.
//
// gfx950 layout of fp_kernel, the transpose of the backprojector's: workgroup = one
// angle block (up to FP_AMAX = 16 projections of similar direction, grouped by the
// plan so that their candidate positions share one segment) x 64 bins x one slice.
// The workgroup walks the image lines in blocks of 16; for each block it
// stages the shared segment of every line (fp_seg_len positions, zero outside
// the image) in LDS once, and every wavefront then serves its projections (m = w,
// w + 4, ...; lane = bin, one accumulator per projection) from LDS: a staged
// value is read up to ~2 x 16 times.  A wavefront's (up to 4) projections advance
// together line by line, so each line issues independent LDS reads for all of
// them; 16 rather than 32 projections per block keep that state within 128 VGPRs
// (4 wavefronts per SIMD).  Coordinates: per (lane, projection, line
// block) the crossing u of the block's first line is computed in FP64 and split
// into an integer base and an FP32 remainder; inside the block u advances by an
// FP32 slope, so every FP32 offset stays below FP_RB + 2 positions.
#include "internal.hpp"

namespace pyhst {

// segment length that holds one projection's 64 bins x FP_RB lines (65/|a| + FP_RB - 1 positions,
// |a| >= s / sqrt(2)) plus a drift allowance of 96 positions for the other members of a block
int fp_seg_len(double s_min)
{
    const int seg = (int)std::ceil(65.0 * 1.4142135623730951 / s_min + (FP_RB - 1) + 10.0 + 96.0);
    return (seg + 3) & ~3;
}

// candidates per line: ceil(2 sqrt 2 / s) <= 3 or <= 6, else counted at run time
int fp_nc_for(double s_min)
{
    const int need = (int)std::ceil(2.0 * 1.4142135623730951 / s_min - 1e-9);
    return need <= 3 ? 3 : (need <= 6 ? 6 : 0);
}

namespace {

constexpr int AW = FP_AMAX / 4;   // projections per wavefront

// Bin chunk (64 bins) of workgroup column i of n.  The hardware deals consecutive workgroups
// round-robin to the 8 XCDs, so column i runs on XCD i % 8 (n is a multiple of 8 whenever the remap
// applies, whatever the other grid dimensions).  Each XCD gets whole pairs (c, n - 1 - c) of chunks at
// the same distance from the detector centre: over all projections the bins of such a pair see one
// annulus of the image, so an XCD's projector sweep touches that annulus rather than the whole image
// and leaves the rest of its L2 (the backprojector's sinogram in the iterative solvers) in place.
__device__ __forceinline__ int fp_chunk(int i, int n)
{
    if (n & 15) return i;
    const int x = i & 7, k = i >> 3;            // XCD; k-th column of this XCD
    const int pair = x * (n >> 4) + (k >> 1);   // n / 16 consecutive pairs per XCD
    return (k & 1) ? n - 1 - pair : pair;
}

// The NC candidates of one line: weights hat(d), hat(d + a), ... with d the signed offset t - j of the
// first one.  With 2/3 <= |a| <= 1 (UNIT: pixel size in [0.943, 1], three candidates) the first candidate
// lies in (u - 1/|a|, u - 1/|a| + 1], so |d| < 1 and |d + a| <= 1: only the third weight can be
// clamped to zero, and the other two skip the max (they differ from the clamped form only by FP32
// rounding at the hat's end points, where the weight is zero to within an ulp).
// Since 1 - |d| never exceeds 1, max(0, 1 - |d|) is its clamp to [0, 1], which the subtraction applies
// as an output modifier (no separate max).
template <int NC, bool UNIT>
__device__ __forceinline__ float hat_line(const float *row, float d, float af, float acc)
{
#pragma unroll
    for (int n = 0; n < NC; ++n, d += af) {
        const float w = (UNIT && n < 2) ? 1.0f - fabsf(d) : __builtin_amdgcn_fmed3f(1.0f - fabsf(d), 0.0f, 1.0f);
        acc = fmaf(w, row[n], acc);
    }
    return acc;
}

// First candidate of one line from v = u - 1/|a| (u: the bin's crossing, in positions from the staged
// base): the candidates are floor(v) + 1, + 2, ..., and the first one's offset is
// t - j = a (floor(v) + 1 - u) = a - sign(a) - a fract(v) = fma(-a, fract(v), c0), c0 = a - sign(a).
struct FirstCand {
    int idx;   // floor(v) + 1
    float d;   // t - j at idx
};
__device__ __forceinline__ FirstCand first_cand(float v, float af, float c0)
{
    int fl;   // floor(v) converted in one instruction (|v| stays below a few hundred positions)
    asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(fl) : "v"(v));
    return {fl + 1, fmaf(-af, __builtin_amdgcn_fractf(v), c0)};
}

// One block of lines for the first MINE projection slots of a wavefront (NC > 0).  The slots advance
// together line by line, so every line issues MINE independent groups of LDS reads and the wavefront
// has that many accumulation chains in flight instead of one.
template <int NC, bool UNIT, int MINE>
__device__ __forceinline__ void fp_block_lines(const float *stage, int seg_len, int nl, int l0, int seg0,
                                               const double *u_first, const double *slope, const float *af,
                                               const float *rhof, const float *slopef, const float *c0f,
                                               float *acc)
{
    float remv[MINE];
    int boff[MINE];
#pragma unroll
    for (int i = 0; i < MINE; ++i) {
        const double ub = fma((double)l0, slope[i], u_first[i]);
        const double ubase = floor(ub);
        remv[i] = (float)(ub - ubase - (double)rhof[i]);   // u - 1/|a| at the block's first line
        boff[i] = (int)ubase - seg0;
    }
    float rf = 0.0f;
    for (int r = 0; r < nl; ++r, rf += 1.0f) {
        const float *line = stage + r * seg_len;
#pragma unroll
        for (int i = 0; i < MINE; ++i) {
            const FirstCand fc = first_cand(fmaf(rf, slopef[i], remv[i]), af[i], c0f[i]);
            acc[i] = hat_line<NC, UNIT>(line + boff[i] + fc.idx, fc.d, af[i], acc[i]);
        }
    }
}

// NC > 0: a fixed number of candidates per line (the surplus ones get zero weight), so the reads of
// a line are independent and issue together; NC == 0: the exact count, ceil(2/|a|), at run time.
// Epilogue of every projector kernel for the value v = alpha (A x)[o]:
//   MODE 0: out[o] = v
//   MODE 1: Chambolle-Pock dual step p = (p + sigma (v - y)) / (1 + sigma)
//   MODE 2: residual p = v - y (gradient step of ISTA/FISTA)
//   MODE 3: one projection's residual row per slice, p[row_o] = v - y
// In modes 1 and 2 a non-null cp.ax is updated to ax_a v + ax_b ax: the projection of the
// primal iterate, carried by linearity from the projection of the extrapolated point, for
// the energy of eq. (3) without a projector call of its own.
template <int MODE>
__device__ __forceinline__ void fp_store(const CpDual &cp, float *out, int64_t o, float v, int64_t row_o)
{
    if (MODE == 0) {
        out[o] = v;
    } else if (MODE == 3) {
        cp.p[row_o] = v - cp.y[o];
    } else {
        if (MODE == 1) cp.p[o] = (cp.p[o] + cp.sigma * (v - cp.y[o])) / (1.0f + cp.sigma);
        else cp.p[o] = v - cp.y[o];
        if (cp.ax) cp.ax[o] = cp.ax_a * v + cp.ax_b * cp.ax[o];
    }
}

template <int MODE, int NC, bool UNIT>
__global__ __launch_bounds__(256) void fp_kernel(Tables T, const float *__restrict__ img, float *__restrict__ out,
                                                 float alpha, CpDual cp, int k_single, int seg_len)
{
    extern __shared__ float stage[];   // [FP_RB][seg_len]
    __shared__ double s_lo[4];
    const int slice = blockIdx.z;
    const SliceDev sd = T.slc[slice];
    const GeoDev &g = T.geo[sd.g];
    const int nb = g.nb, nx = g.nx, ny = g.ny;
    int start = 0, count = 1;
    if (MODE != 3) {
        if ((int)blockIdx.y >= g.fp_nblk) return;            // whole workgroup
        const int2 bk = T.fp_blk[g.fp_blk_off + blockIdx.y];
        start = bk.x;
        count = bk.y;
    }
    const int chunk = fp_chunk(blockIdx.x, gridDim.x);
    if (chunk * 64 >= nb) return;                            // whole workgroup
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform
    const int j = chunk * 64 + lane;
    const double s = g.s;
    const double cx = 0.5 * (nx - 1), cy = 0.5 * (ny - 1);
    const int k_first = MODE == 3 ? k_single : T.fp_ang[start];
    const bool rows = fabs(T.cosd[g.ang_off + k_first]) >= fabs(T.sind[g.ang_off + k_first]);   // same for the block
    const int n_lines = rows ? ny : nx;

    // this lane's projections: u = U0 + j / a + slope * line, candidates within rho of u
    double u_first[AW], slope[AW];
    float af[AW], rhof[AW], slopef[AW], c0f[AW];
    int ncand[AW], kk[AW];
    int mine = 0;
#pragma unroll
    for (int i = 0; i < AW; ++i) {
        const int m = wv + 4 * i;
        const bool on = m < count;
        const int k = MODE == 3 ? k_single : T.fp_ang[start + (on ? m : 0)];
        const double c = T.cosd[g.ang_off + k], sn = T.sind[g.ang_off + k];
        const double a = rows ? s * c : s * sn, bb = rows ? s * sn : s * c;
        const double ci = rows ? cx : cy, cl = rows ? cy : cx;
        const double t0 = g.axis + T.shiftd[g.ang_off + k];
        const double rho = 1.0 / fabs(a);
        kk[i] = k;
        slope[i] = -bb / a;
        u_first[i] = ((double)j - t0 + a * ci + bb * cl) / a;
        af[i] = (float)a;
        c0f[i] = af[i] - copysignf(1.0f, af[i]);
        rhof[i] = (float)rho;
        slopef[i] = (float)slope[i];
        ncand[i] = on ? (int)ceil(2.0 * rho) : 0;
        mine += on ? 1 : 0;
    }

    float acc[AW];
#pragma unroll
    for (int i = 0; i < AW; ++i) acc[i] = 0.0f;
    const float *im = img + sd.img_off;
    for (int l0 = 0; l0 < n_lines; l0 += FP_RB) {
        // segment start: lowest candidate over the block's projections, 64 bins and FP_RB lines
        double lo = 1e300;
#pragma unroll
        for (int i = 0; i < AW; ++i) {
            if (i >= mine) break;
            const double ub = fma((double)l0, slope[i], u_first[i]);
            lo = fmin(lo, fmin(ub, ub + (FP_RB - 1) * slope[i]) - (double)rhof[i]);
        }
        for (int off = 32; off > 0; off >>= 1) lo = fmin(lo, __shfl_xor(lo, off, 64));
        __syncthreads();   // the previous block's reads are done
        if (lane == 0) s_lo[wv] = lo;
        __syncthreads();
        const int seg0 = (int)floor(fmin(fmin(s_lo[0], s_lo[1]), fmin(s_lo[2], s_lo[3]))) - 1;
        if (rows) {
            for (int r = 0; r < FP_RB; ++r) {
                const int line = l0 + r;
                const float *src = im + (int64_t)line * nx;
                for (int p = threadIdx.x; p < seg_len; p += 256) {
                    const int pos = seg0 + p;
                    stage[r * seg_len + p] = (line < ny && (unsigned)pos < (unsigned)nx) ? src[pos] : 0.0f;
                }
            }
        } else {
            // columns: 16 threads read 16 neighbouring columns of one row (64 B), 16 rows per step
            const int r = threadIdx.x & 15;
            const int line = l0 + r;
            for (int p = threadIdx.x >> 4; p < seg_len; p += 16) {
                const int pos = seg0 + p;
                stage[r * seg_len + p] = (line < nx && (unsigned)pos < (unsigned)ny) ? im[(int64_t)pos * nx + line] : 0.0f;
            }
        }
        __syncthreads();
        const int nl = min(FP_RB, n_lines - l0);
        if constexpr (NC > 0) {
#define FP_LINES_CASE(M)                                                                                  \
    case M:                                                                                               \
        fp_block_lines<NC, UNIT, M>(stage, seg_len, nl, l0, seg0, u_first, slope, af, rhof, slopef, c0f, acc); \
        break;
            switch (mine) {   // uniform over the wavefront
                FP_LINES_CASE(8)
                FP_LINES_CASE(7)
                FP_LINES_CASE(6)
                FP_LINES_CASE(5)
                FP_LINES_CASE(4)
                FP_LINES_CASE(3)
                FP_LINES_CASE(2)
                FP_LINES_CASE(1)
                default: break;
            }
#undef FP_LINES_CASE
        } else {
#pragma unroll
            for (int i = 0; i < AW; ++i) {
                if (i >= mine) break;
                const double ub = fma((double)l0, slope[i], u_first[i]);
                const double ubase = floor(ub);
                const float remv = (float)(ub - ubase - (double)rhof[i]);   // u - 1/|a| at the block's first line
                const float *base = stage + ((int)ubase - seg0);
                for (int r = 0; r < nl; ++r) {
                    const FirstCand fc = first_cand(fmaf((float)r, slopef[i], remv), af[i], c0f[i]);
                    const float *row = base + r * seg_len + fc.idx;
                    float d = fc.d;
                    for (int n = 0; n < ncand[i]; ++n, d += af[i]) acc[i] = fmaf(fmaxf(0.0f, 1.0f - fabsf(d)), row[n], acc[i]);
                }
            }
        }
    }
    if (j >= nb) return;
    const float sc = alpha * (float)(s * s);   // A = s^2 B^T
#pragma unroll
    for (int i = 0; i < AW; ++i) {
        if (i >= mine) break;
        const int64_t o = sd.sino_off + (int64_t)kk[i] * nb + j;
        fp_store<MODE>(cp, out, o, sc * acc[i], (int64_t)slice * nb + j);
    }
}

// Smaller plans with pixels below half a bin (or when forced): one projection per workgroup, its 4
// wavefronts take every fourth image line and add their partial sums in a fixed order through LDS.
// The crossing position is anchored in FP64 every 8 lines of a wavefront (FP32 offsets below 30
// positions in between); the candidates are read from global memory (L2).
template <int MODE, int NC>
__global__ __launch_bounds__(256) void fp_lines_kernel(Tables T, const float *__restrict__ img,
                                                       float *__restrict__ out, float alpha, CpDual cp, int k0)
{
    __shared__ float part[3][64];
    const int slice = blockIdx.z;
    const SliceDev sd = T.slc[slice];
    const GeoDev &g = T.geo[sd.g];
    const int K = g.K, nb = g.nb, nx = g.nx, ny = g.ny;
    const int k = k0 + blockIdx.y;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int chunk = fp_chunk(blockIdx.x, gridDim.x);
    const int j = chunk * 64 + lane;
    if (k >= K || chunk * 64 >= nb) return;        // uniform over the workgroup

    const double c = T.cosd[g.ang_off + k], sn = T.sind[g.ang_off + k];
    const double s = g.s;
    const double cx = 0.5 * (nx - 1), cy = 0.5 * (ny - 1);
    const double t0 = g.axis + T.shiftd[g.ang_off + k];
    const bool rows = fabs(c) >= fabs(sn);
    const double a = rows ? s * c : s * sn, bb = rows ? s * sn : s * c;
    const double ci = rows ? cx : cy, cl = rows ? cy : cx;
    const int n_lines = rows ? ny : nx, n_pos = rows ? nx : ny;
    const int64_t step_line = rows ? nx : 1, step_pos = rows ? 1 : nx;
    const double rho = 1.0 / fabs(a);
    const int ncand = (int)ceil(2.0 * rho);
    const double slope = -bb / a;
    const double u_first = ((double)j - t0 + a * ci + bb * cl) / a;
    const float af = (float)a, rhof = (float)rho, slopef = (float)slope;
    const float *im = img + sd.img_off;
    float acc = 0.0f;
    // this wavefront's lines wv, wv + 4, ...: an FP64 anchor every 8 of them, FP32 offsets in between
    for (int la = wv; la < n_lines; la += 32) {
        const double ub = fma((double)la, slope, u_first);
        const double ubase = floor(ub);
        const float rem = (float)(ub - ubase);
        const int ib = (int)ubase;
#pragma unroll
        for (int m = 0; m < 8; ++m) {                             // unrolled: the 8 lines' loads overlap
            const int l = la + 4 * m;
            if (l >= n_lines) break;
            const float u = fmaf((float)(4 * m), slopef, rem);   // crossing relative to ubase
            const float fl = floorf(u - rhof);                      // first candidate = fl + 1
            const int i0 = (int)fl + 1;
            float d = fmaf(af, fl - u, af);                         // t - j at the first candidate
            const float *line = im + (int64_t)l * step_line;
            const int nc = NC > 0 ? NC : ncand;
#pragma unroll
            for (int n = 0; n < (NC > 0 ? NC : 8); ++n, d += af) {
                if (NC == 0 && n >= nc) break;
                const int q = ib + i0 + n;
                const float w = fmaxf(0.0f, 1.0f - fabsf(d));
                const float v = (unsigned)q < (unsigned)n_pos ? line[(int64_t)q * step_pos] : 0.0f;
                acc = fmaf(w, v, acc);
            }
        }
    }
    if (wv > 0) part[wv - 1][lane] = acc;
    __syncthreads();
    if (wv > 0 || j >= nb) return;
    acc = ((acc + part[0][lane]) + part[1][lane]) + part[2][lane];
    const int64_t o = sd.sino_off + (int64_t)k * nb + j;
    fp_store<MODE>(cp, out, o, alpha * (float)(s * s) * acc, (int64_t)slice * nb + j);
}

// Pixel size >= 0.5 (NC > 0): one to FP_SGRP = 4 projections per workgroup, staged through LDS.
// The plan groups neighbouring projections (similar direction) whose candidates share the staged
// segment; a staged value then serves all of them.  The workgroup walks the image lines in blocks of FP_RB;
// the 64 bins of one projection touch, over a block, a segment of at most 63/|a| + (FP_RB - 1)|slope|
// + 1/|a| + NC + 3 positions of every line (< FpStaged<NC>::SEG; the plan checks the group's union),
// which 256 threads stage with 16-wide contiguous reads along the image rows in both walking
// directions (so a column-walking projection reads rows of 16 neighbouring columns rather than 64
// separate rows).  The next block is loaded into registers while the current one is summed from the
// other LDS buffer: one barrier per block.  Each wavefront serves one projection of the group on every
// (4 / group size)-th line of a block (fp_staged_body_wp).
template <int NC> struct FpStaged {
    static constexpr int SEG = NC == 3 ? FP_SSEG3 : FP_SSEG6;   // positions staged per line
    static constexpr int LD = SEG + 17;               // LDS row stride: 17 mod 32 spreads the banks
    static constexpr int PER = SEG / 16;              // staged values per thread and block
};

// One projection of a staged group, for this lane's bin j of the workgroup's chunk j0..j0+63.
struct StagedProj {
    double u_first, slope, rho, blk_lo;   // crossing at line 0, per line, 1/|a|; lowest first candidate
    float af, slopef, c0;                 // a, slope, a - sign(a) in FP32
    float aa, c1, c2;                     // |a|, 2|a| - 1, 2 - 3|a| (closed-form weights of three candidates)
    int k;
};

// One line of a staged projection from v = u - 1/|a| (u: the bin's crossing, in positions from the
// line's staged base).  The candidates are floor(v) + 1 + n, n = 0, 1, 2, at offsets
// t - j = d_n = +-(|a| (1 + n - f) - 1), f = fract(v) (the sign is that of a, and only |d_n| enters).
// With 2/3 <= |a| <= 1 (UNIT) the three hat weights 1 - |d_n| are, without any case:
//   w0 = |a| (1 - f)                 (d_0 in (-1, 0])
//   w1 = 1 - | |a| (2 - f) - 1 |     (|d_1| <= 1)
//   w2 = max(0, 2 - 3 |a| + |a| f)   (d_2 > 0)
// one FMA each, plus the absolute difference of w1 and the clamp of w2 as output modifiers.
template <int NC, bool UNIT>
__device__ __forceinline__ float staged_line(const float *line, float v, const StagedProj &q, float acc)
{
    int fl;   // floor(v) converted in one instruction (|v| stays below a few hundred positions)
    asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(fl) : "v"(v));
    const float f = __builtin_amdgcn_fractf(v);
    const float *row = line + fl + 1;
    if (NC == 3 && UNIT) {
        acc = fmaf(fmaf(-q.aa, f, q.aa), row[0], acc);
        acc = fmaf(1.0f - fabsf(fmaf(-q.aa, f, q.c1)), row[1], acc);
        return fmaf(__builtin_amdgcn_fmed3f(fmaf(q.aa, f, q.c2), 0.0f, 1.0f), row[2], acc);
    }
    return hat_line<NC, UNIT>(row, fmaf(-q.af, f, q.c0), q.af, acc);
}

__device__ __forceinline__ StagedProj staged_proj(const Tables &T, const GeoDev &g, int k, int j, int j0,
                                                  bool &rows)
{
    const double c = T.cosd[g.ang_off + k], sn = T.sind[g.ang_off + k];
    const double s = g.s;
    const double cx = 0.5 * (g.nx - 1), cy = 0.5 * (g.ny - 1);
    const double t0 = g.axis + T.shiftd[g.ang_off + k];
    rows = fabs(c) >= fabs(sn);
    const double a = rows ? s * c : s * sn, bb = rows ? s * sn : s * c;
    const double ci = rows ? cx : cy, cl = rows ? cy : cx;
    StagedProj q;
    q.k = k;
    q.rho = 1.0 / fabs(a);
    q.slope = -bb / a;
    const double u_c = -t0 + a * ci + bb * cl;
    q.u_first = ((double)j + u_c) / a;
    // lowest first candidate of the chunk's 64 bins over a block's FP_RB lines, relative to its first line
    q.blk_lo = fmin(((double)j0 + u_c) / a, ((double)(j0 + 63) + u_c) / a) + fmin(0.0, (FP_RB - 1) * q.slope) -
               q.rho;
    q.af = (float)a;
    q.slopef = (float)q.slope;
    q.c0 = q.af - copysignf(1.0f, q.af);
    q.aa = fabsf(q.af);
    q.c1 = 2.0f * q.aa - 1.0f;
    q.c2 = 2.0f - 3.0f * q.aa;
    return q;
}

// Groups of one, two or four projections: 4 / P wavefronts per projection, wavefront w serving projection
// w / (4 / P) on lines w % (4 / P), + 4 / P, ... of every block (16, 8 or 4 lines).  The crossing is
// anchored in FP64 once per (lane, block) for the wavefront's one projection (a quarter of the anchors
// of every wavefront serving every projection); partial sums of a projection's wavefronts are added in a
// fixed order through LDS.  A group of n = 3 runs as P = 4 with pr[3] = pr[0]: the last wavefront repeats
// the first projection and stores nothing.
template <int MODE, int NC, bool UNIT, int P>
__device__ __forceinline__ void fp_staged_body_wp(const Tables &T, const SliceDev &sd, const GeoDev &g,
                                                  const StagedProj *pr, int n, bool rows, int j, const float *img,
                                                  float *out, float alpha, const CpDual &cp, int slice,
                                                  float (*stage)[FP_RB * FpStaged<NC>::LD], float (*part)[3][64])
{
    using F = FpStaged<NC>;
    static_assert(P == 1 || P == 2 || P == 4, "whole wavefronts per projection");
    constexpr int WPP = 4 / P, LPW = FP_RB / WPP;   // wavefronts per projection, lines per wavefront and block
    const int nb = g.nb, nx = g.nx, ny = g.ny;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int pw = wv / WPP, ph = wv % WPP;          // this wavefront's projection and line phase
    const int n_lines = rows ? ny : nx, n_pos = rows ? nx : ny;
    const float *im = img + sd.img_off;
    const int sr = rows ? tid >> 4 : tid & 15;
    const int sp = rows ? tid & 15 : tid >> 4;
    const int step_line = rows ? nx : 1, step_pos = rows ? 1 : nx;
    const int n_blk = (n_lines + FP_RB - 1) / FP_RB;
    StagedProj q = pr[0];
#pragma unroll
    for (int m = 1; m < P; ++m)
        if (pw == m) q = pr[m];   // wave-uniform

    float v[F::PER];
    auto load = [&](int b, int &seg0) {
        const int l0 = b * FP_RB;
        double lo = fma((double)l0, pr[0].slope, pr[0].blk_lo);
#pragma unroll
        for (int m = 1; m < P; ++m) lo = fmin(lo, fma((double)l0, pr[m].slope, pr[m].blk_lo));
        seg0 = (int)floor(lo) - 2;
        const int line = l0 + sr;
        if (line < n_lines && seg0 >= 0 && seg0 + F::SEG <= n_pos) {
            const float *src = im + (line * step_line + (seg0 + sp) * step_pos);
            const int d16 = 16 * step_pos;
#pragma unroll
            for (int i = 0; i < F::PER; ++i) v[i] = src[i * d16];
        } else {
#pragma unroll
            for (int i = 0; i < F::PER; ++i) {
                const int pos = seg0 + sp + 16 * i;
                v[i] = (line < n_lines && (unsigned)pos < (unsigned)n_pos) ? im[line * step_line + pos * step_pos] : 0.0f;
            }
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int i = 0; i < F::PER; ++i) stage[buf][sr * F::LD + sp + 16 * i] = v[i];
    };

    float acc[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    int seg_cur, seg_next = 0;
    load(0, seg_cur);
    store(0);
    __syncthreads();
    for (int b = 0; b < n_blk; ++b) {
        const bool more = b + 1 < n_blk;
        if (more) load(b + 1, seg_next);
        const int l0 = b * FP_RB;
        const double ub = fma((double)l0, q.slope, q.u_first);
        const double ubase = floor(ub);
        const float remv = (float)(ub - ubase - q.rho);            // u - 1/|a| at the block's first line
        const float *base = stage[b & 1] + ((int)ubase - seg_cur) + ph * F::LD;
        if (l0 + FP_RB <= n_lines) {
#pragma unroll
            for (int k = 0; k < LPW; ++k)
                acc[k & 3] = staged_line<NC, UNIT>(base + k * WPP * F::LD, fmaf((float)(ph + WPP * k), q.slopef, remv), q,
                                                   acc[k & 3]);
        } else {
#pragma unroll
            for (int k = 0; k < LPW; ++k)   // no break: the loop stays unrolled and acc in registers
                if (l0 + ph + WPP * k < n_lines)                      // uniform
                    acc[k & 3] = staged_line<NC, UNIT>(base + k * WPP * F::LD, fmaf((float)(ph + WPP * k), q.slopef, remv),
                                                       q, acc[k & 3]);
        }
        if (more) {
            store((b + 1) & 1);
            seg_cur = seg_next;
        }
        __syncthreads();
    }
    float tot = (acc[0] + acc[1]) + (acc[2] + acc[3]);
    if constexpr (WPP > 1) {
        if (ph > 0) part[pw][ph - 1][lane] = tot;
        __syncthreads();
        if (ph > 0) return;
#pragma unroll
        for (int m = 1; m < WPP; ++m) tot += part[pw][m - 1][lane];
    }
    if (j >= nb || pw >= n) return;
    const int64_t o = sd.sino_off + (int64_t)q.k * nb + j;
    fp_store<MODE>(cp, out, o, alpha * (float)(g.s * g.s) * tot, (int64_t)slice * nb + j);
}

// grid: (bin chunks, staged groups of the geometry with the most, slices); MODE 3: one projection k0.
// GMAX: the largest group the plan formed, 2 or 4 (the 4-wide build needs more VGPRs, so plans with
// groups of at most two keep the occupancy of the 2-wide one).
template <int MODE, int NC, bool UNIT, int GMAX>
__global__ __launch_bounds__(256) void fp_staged_kernel(Tables T, const float *__restrict__ img,
                                                        float *__restrict__ out, float alpha, CpDual cp, int k0)
{
    __shared__ float stage[2][FP_RB * FpStaged<NC>::LD];
    __shared__ float part[FP_SGRP][3][64];
    const int slice = blockIdx.z;
    const SliceDev sd = T.slc[slice];
    const GeoDev &g = T.geo[sd.g];
    const int j0 = fp_chunk(blockIdx.x, gridDim.x) * 64;
    int kk[FP_SGRP] = {k0, -1, -1, -1};
    if (MODE != 3) {
        if ((int)blockIdx.y >= g.fp_npair) return;   // uniform over the workgroup
        const int4 grp = T.fp_pair[g.fp_pair_off + blockIdx.y];
        kk[0] = grp.x;
        kk[1] = grp.y;
        kk[2] = grp.z;
        kk[3] = grp.w;
    } else if (k0 >= g.K) {
        return;
    }
    if (j0 >= g.nb) return;                          // uniform over the workgroup
    const int j = j0 + (int)(threadIdx.x & 63);
    const int n = kk[1] < 0 ? 1 : (kk[2] < 0 ? 2 : (kk[3] < 0 ? 3 : 4));   // members (the plan fills in order)
    bool rows, rows_m;
    StagedProj pr[FP_SGRP];
    pr[0] = staged_proj(T, g, kk[0], j, j0, rows);
#pragma unroll
    for (int m = 1; m < FP_SGRP; ++m) {
        // same walking axis (the plan groups only such); members past n repeat the first
        if (m < n) pr[m] = staged_proj(T, g, kk[m], j, j0, rows_m);
        else pr[m] = pr[0];
    }
    if (GMAX > 2 && n >= 3) {   // uniform over the workgroup
        fp_staged_body_wp<MODE, NC, UNIT, 4>(T, sd, g, pr, n, rows, j, img, out, alpha, cp, slice, stage, part);
    } else if (n == 2) {
        fp_staged_body_wp<MODE, NC, UNIT, 2>(T, sd, g, pr, n, rows, j, img, out, alpha, cp, slice, stage, part);
    } else {
        fp_staged_body_wp<MODE, NC, UNIT, 1>(T, sd, g, pr, n, rows, j, img, out, alpha, cp, slice, stage, part);
    }
}

// SP = 2 or 4 slices of a uniform plan per workgroup (slices SP z .. SP z + SP - 1; three candidates with
// 2/3 <= |a| <= 1): the staged segment holds the SP slices' values of a position side by side, so
// one 8- or 16-byte LDS read serves them all, and a line's position, floor, fraction, address and three
// hat weights are computed once for them (with two slices about 7.5 instead of 12 VALU instructions per
// line and slice).  Each slice's sums are staged_line's, term for term in the same order, so every value
// equals fp_staged_body_wp's.  Groups of three run as groups of four whose last wavefront repeats the
// first projection and stores nothing.
template <int SP> struct SliceVec;
template <> struct SliceVec<2> { using T = float2; };
template <> struct SliceVec<4> { using T = float4; };

template <int SP>
__device__ __forceinline__ void staged_line_sp(const float *line, float v, const StagedProj &q, float (&acc)[SP])
{
    using V = typename SliceVec<SP>::T;
    int fl;
    asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(fl) : "v"(v));
    const float f = __builtin_amdgcn_fractf(v);
    const float *row = line + SP * (fl + 1);
    const float w[3] = {fmaf(-q.aa, f, q.aa), 1.0f - fabsf(fmaf(-q.aa, f, q.c1)),
                        __builtin_amdgcn_fmed3f(fmaf(q.aa, f, q.c2), 0.0f, 1.0f)};
    V r[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) r[c] = *(const V *)(row + SP * c);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const float *rv = (const float *)&r[c];
#pragma unroll
        for (int t = 0; t < SP; ++t) acc[t] = fmaf(w[c], rv[t], acc[t]);
    }
}

struct SegBound {   // slope and lowest first candidate of each member of a staged group
    double s0, b0, s1, b1, s2, b2, s3, b3;
};

// One LDS buffer (the segment is SP times the one-slice kernel's): the next block waits in registers
// while the current one is summed, then two barriers around its store; the partial sums of the last
// step reuse the buffer.  The group's segment bound needs only each member's slope and lowest candidate
// (the same for every lane), the sums only the wavefront's own projection q.  ns: slices present (the
// last workgroup of a plan whose slice count SP does not divide holds fewer).
template <int MODE, int SP, int P>
__device__ __forceinline__ void fp_staged_sp_body(const Tables &T, int slice0, int ns, const GeoDev &g,
                                                  const StagedProj &q, const SegBound &sb, int n, bool rows, int j,
                                                  const float *img, float *out, float alpha, const CpDual &cp,
                                                  float *stage)
{
    using F = FpStaged<3>;
    using V = typename SliceVec<SP>::T;
    static_assert(P == 1 || P == 2 || P == 4, "whole wavefronts per projection");
    static_assert(FP_SGRP * 3 * 64 <= FP_RB * F::LD, "partial sums fit the staging buffer");
    constexpr int WPP = 4 / P, LPW = FP_RB / WPP;
    const int nb = g.nb, nx = g.nx, ny = g.ny;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int pw = wv / WPP, ph = wv % WPP;
    const int n_lines = rows ? ny : nx, n_pos = rows ? nx : ny;
    const float *im[SP];
#pragma unroll
    for (int t = 0; t < SP; ++t) im[t] = img + T.slc[slice0 + (t < ns ? t : 0)].img_off;
    const int sr = rows ? tid >> 4 : tid & 15;
    const int sp = rows ? tid & 15 : tid >> 4;
    const int step_line = rows ? nx : 1, step_pos = rows ? 1 : nx;
    const int n_blk = (n_lines + FP_RB - 1) / FP_RB;

    float vv[SP][F::PER];
    auto load = [&](int b, int &seg0) {
        const int l0 = b * FP_RB;
        double lo = fma((double)l0, sb.s0, sb.b0);
        if (P > 1) lo = fmin(lo, fma((double)l0, sb.s1, sb.b1));
        if (P > 2) lo = fmin(fmin(lo, fma((double)l0, sb.s2, sb.b2)), fma((double)l0, sb.s3, sb.b3));
        seg0 = (int)floor(lo) - 2;
        const int line = l0 + sr;
        if (line < n_lines && seg0 >= 0 && seg0 + F::SEG <= n_pos) {
            const int off = line * step_line + (seg0 + sp) * step_pos;
            const int d16 = 16 * step_pos;
#pragma unroll
            for (int i = 0; i < F::PER; ++i)
#pragma unroll
                for (int t = 0; t < SP; ++t) vv[t][i] = t < ns ? im[t][off + i * d16] : 0.0f;
        } else {
#pragma unroll
            for (int i = 0; i < F::PER; ++i) {
                const int pos = seg0 + sp + 16 * i;
                const bool in = line < n_lines && (unsigned)pos < (unsigned)n_pos;
                const int off = in ? line * step_line + pos * step_pos : 0;
#pragma unroll
                for (int t = 0; t < SP; ++t) vv[t][i] = in && t < ns ? im[t][off] : 0.0f;
            }
        }
    };
    auto store = [&]() {
#pragma unroll
        for (int i = 0; i < F::PER; ++i) {
            V o;
            float *ov = (float *)&o;
#pragma unroll
            for (int t = 0; t < SP; ++t) ov[t] = vv[t][i];
            *(V *)&stage[SP * (sr * F::LD + sp + 16 * i)] = o;
        }
    };

    float acc[4][SP];
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int t = 0; t < SP; ++t) acc[k][t] = 0.0f;
    int seg_cur, seg_next = 0;
    load(0, seg_cur);
    store();
    __syncthreads();
    for (int b = 0; b < n_blk; ++b) {
        const bool more = b + 1 < n_blk;
        if (more) load(b + 1, seg_next);
        const int l0 = b * FP_RB;
        const double ub = fma((double)l0, q.slope, q.u_first);
        const double ubase = floor(ub);
        const float remv = (float)(ub - ubase - q.rho);
        const float *base = stage + SP * (((int)ubase - seg_cur) + ph * F::LD);
        if (l0 + FP_RB <= n_lines) {
#pragma unroll
            for (int k = 0; k < LPW; ++k)
                staged_line_sp<SP>(base + SP * k * WPP * F::LD, fmaf((float)(ph + WPP * k), q.slopef, remv), q, acc[k & 3]);
        } else {
#pragma unroll
            for (int k = 0; k < LPW; ++k)   // no break: the loop stays unrolled and acc in registers
                if (l0 + ph + WPP * k < n_lines)                      // uniform
                    staged_line_sp<SP>(base + SP * k * WPP * F::LD, fmaf((float)(ph + WPP * k), q.slopef, remv), q,
                                       acc[k & 3]);
        }
        __syncthreads();   // every read of this block is done
        if (more) {
            store();
            seg_cur = seg_next;
            __syncthreads();
        }
    }
    float tot[SP];
#pragma unroll
    for (int t = 0; t < SP; ++t) tot[t] = (acc[0][t] + acc[1][t]) + (acc[2][t] + acc[3][t]);
    if constexpr (WPP > 1) {
        float *part = stage;   // [FP_SGRP][3][64][SP], free after the last block's barrier
        if (ph > 0) {
            V o;
            float *ov = (float *)&o;
#pragma unroll
            for (int t = 0; t < SP; ++t) ov[t] = tot[t];
            *(V *)&part[SP * ((pw * 3 + ph - 1) * 64 + lane)] = o;
        }
        __syncthreads();
        if (ph > 0) return;
#pragma unroll
        for (int m = 1; m < WPP; ++m) {
            const V o = *(const V *)&part[SP * ((pw * 3 + m - 1) * 64 + lane)];
            const float *ov = (const float *)&o;
#pragma unroll
            for (int t = 0; t < SP; ++t) tot[t] += ov[t];
        }
    }
    if (j >= nb || pw >= n) return;
    const float sc = alpha * (float)(g.s * g.s);
#pragma unroll
    for (int t = 0; t < SP; ++t)
        if (t < ns)
            fp_store<MODE>(cp, out, T.slc[slice0 + t].sino_off + (int64_t)q.k * nb + j, sc * tot[t],
                           (int64_t)(slice0 + t) * nb + j);
}

// grid: (bin chunks, staged groups, slice groups of SP); GMAX as in fp_staged_kernel
template <int MODE, int SP, int GMAX>
__global__ __launch_bounds__(256) void fp_staged_sp_kernel(Tables T, const float *__restrict__ img,
                                                           float *__restrict__ out, float alpha, CpDual cp,
                                                           int n_slices)
{
    __shared__ __attribute__((aligned(16))) float stage[SP * FP_RB * FpStaged<3>::LD];
    const int s0 = SP * (int)blockIdx.z;
    const int ns = min(SP, n_slices - s0);
    const GeoDev &g = T.geo[T.slc[s0].g];
    const int j0 = fp_chunk(blockIdx.x, gridDim.x) * 64;
    if ((int)blockIdx.y >= g.fp_npair) return;       // uniform over the workgroup
    const int4 grp = T.fp_pair[g.fp_pair_off + blockIdx.y];
    if (j0 >= g.nb) return;                          // uniform over the workgroup
    const int j = j0 + (int)(threadIdx.x & 63);
    const int n = grp.y < 0 ? 1 : (grp.z < 0 ? 2 : (grp.w < 0 ? 3 : 4));   // members (the plan fills in order)
    const int k1 = n > 1 ? grp.y : grp.x, k2 = n > 2 ? grp.z : grp.x, k3 = n > 3 ? grp.w : grp.x;
    // this wavefront's projection (wave-uniform; members past n repeat the first) and every member's
    // segment bound (scalars: no per-lane array)
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int P = (GMAX > 2 && n >= 3) ? 4 : (n == 2 ? 2 : 1);
    const int pw = wv / (4 / P);
    int kq = grp.x;
    if (pw == 1) kq = k1;
    if (pw == 2) kq = k2;
    if (pw == 3) kq = k3;
    bool rows, rows_m;
    const StagedProj q = staged_proj(T, g, kq, j, j0, rows);
    SegBound sb;
    {
        StagedProj e = staged_proj(T, g, grp.x, j, j0, rows_m);   // same walking axis for every member
        sb.s0 = e.slope;
        sb.b0 = e.blk_lo;
        e = staged_proj(T, g, k1, j, j0, rows_m);
        sb.s1 = e.slope;
        sb.b1 = e.blk_lo;
        e = staged_proj(T, g, k2, j, j0, rows_m);
        sb.s2 = e.slope;
        sb.b2 = e.blk_lo;
        e = staged_proj(T, g, k3, j, j0, rows_m);
        sb.s3 = e.slope;
        sb.b3 = e.blk_lo;
    }
    if (P == 4) {   // uniform over the workgroup
        fp_staged_sp_body<MODE, SP, 4>(T, s0, ns, g, q, sb, n, rows, j, img, out, alpha, cp, stage);
    } else if (P == 2) {
        fp_staged_sp_body<MODE, SP, 2>(T, s0, ns, g, q, sb, n, rows, j, img, out, alpha, cp, stage);
    } else {
        fp_staged_sp_body<MODE, SP, 1>(T, s0, ns, g, q, sb, n, rows, j, img, out, alpha, cp, stage);
    }
}

int fp_nc(const pyhst_plan &p)
{
    double s_min = 1e300;
    for (const auto &g : p.gd) s_min = std::min(s_min, g.s);
    return fp_nc_for(s_min);
}

// three candidates and no pixel wider than a bin: |a| in [2/3, 1] for every projection
bool fp_unit(const pyhst_plan &p)
{
    double s_max = 0.0;
    for (const auto &g : p.gd) s_max = std::max(s_max, g.s);
    return fp_nc(p) == 3 && s_max <= 1.0;
}

template <int MODE, int NC, bool UNIT>
hipError_t launch_fp_nc(const pyhst_plan &p, dim3 grid, const float *img, float *sino, float alpha,
                        const CpDual &cp, int k_single, hipStream_t st)
{
    int kind = p.fp_kernel;
    if (kind == PYHST_FP_AUTO) {
        // a fixed candidate count: the staged kernel (one to four projections per workgroup), faster
        // than the angle blocks at every measured size; otherwise angle blocks when they give enough
        // workgroups to fill the chip, else one projection per workgroup read from global memory
        const int64_t wgs = (int64_t)grid.x * grid.y * grid.z;
        kind = (NC > 0 || MODE == 3 || wgs < 8 * (int64_t)p.cu_count) ? PYHST_FP_STAGED : PYHST_FP_BLOCKS;
    }
    if (kind == PYHST_FP_STAGED && NC == 0) kind = PYHST_FP_LINES;
    const dim3 g2(grid.x, MODE == 3 ? 1u : (unsigned)p.max_K, grid.z);
    if (kind == PYHST_FP_STAGED) {
        const dim3 gs(grid.x, MODE == 3 ? 1u : (unsigned)p.fp_max_pairs, grid.z);
        if constexpr (NC == 3 && UNIT && MODE != 3) {
            // automatic choice on a uniform plan of several slices: four slices per workgroup, or two,
            // when that still gives at least eight workgroups per CU
            const int64_t per4 = (int64_t)gs.x * gs.y * ((gs.z + 3) / 4), per2 = (int64_t)gs.x * gs.y * ((gs.z + 1) / 2);
            const int64_t enough = 8 * (int64_t)p.cu_count;
            if (p.fp_kernel == PYHST_FP_AUTO && p.uniform && p.n_slices >= 2 && per2 >= enough) {
                const bool four = p.n_slices >= 4 && per4 >= enough;
                const dim3 gp(gs.x, gs.y, four ? (gs.z + 3) / 4 : (gs.z + 1) / 2);
                if (four) {
                    if (p.fp_max_grp > 2)
                        fp_staged_sp_kernel<MODE, 4, 4><<<gp, 256, 0, st>>>(p.t, img, sino, alpha, cp, p.n_slices);
                    else
                        fp_staged_sp_kernel<MODE, 4, 2><<<gp, 256, 0, st>>>(p.t, img, sino, alpha, cp, p.n_slices);
                } else if (p.fp_max_grp > 2) {
                    fp_staged_sp_kernel<MODE, 2, 4><<<gp, 256, 0, st>>>(p.t, img, sino, alpha, cp, p.n_slices);
                } else {
                    fp_staged_sp_kernel<MODE, 2, 2><<<gp, 256, 0, st>>>(p.t, img, sino, alpha, cp, p.n_slices);
                }
                return hipGetLastError();
            }
        }
        if constexpr (NC > 0) {
            if (MODE != 3 && p.fp_max_grp > 2)
                fp_staged_kernel<MODE, NC, UNIT, 4><<<gs, 256, 0, st>>>(p.t, img, sino, alpha, cp, 0);
            else
                fp_staged_kernel<MODE, NC, UNIT, 2><<<gs, 256, 0, st>>>(p.t, img, sino, alpha, cp, MODE == 3 ? k_single : 0);
        }
        return hipGetLastError();
    }
    if (kind == PYHST_FP_LINES) {
        fp_lines_kernel<MODE, NC><<<g2, 256, 0, st>>>(p.t, img, sino, alpha, cp, MODE == 3 ? k_single : 0);
        return hipGetLastError();
    }
    const int seg = p.fp_seg;
    const size_t lds = (size_t)FP_RB * seg * sizeof(float);
    if (lds > 65536) {
        if (lds > 160 * 1024) return hipErrorInvalidValue;
        hipError_t e = hipFuncSetAttribute((const void *)fp_kernel<MODE, NC, UNIT>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    fp_kernel<MODE, NC, UNIT><<<grid, 256, lds, st>>>(p.t, img, sino, alpha, cp, k_single, seg);
    return hipGetLastError();
}

template <int MODE>
hipError_t launch_fp(const pyhst_plan &p, dim3 grid, const float *img, float *sino, float alpha, const CpDual &cp,
                     int k_single, hipStream_t st)
{
    switch (fp_nc(p)) {
    case 3:
        if (fp_unit(p)) return launch_fp_nc<MODE, 3, true>(p, grid, img, sino, alpha, cp, k_single, st);
        return launch_fp_nc<MODE, 3, false>(p, grid, img, sino, alpha, cp, k_single, st);
    case 6: return launch_fp_nc<MODE, 6, false>(p, grid, img, sino, alpha, cp, k_single, st);
    default: return launch_fp_nc<MODE, 0, false>(p, grid, img, sino, alpha, cp, k_single, st);
    }
}

}  // namespace

hipError_t launch_forward(const pyhst_plan &p, const float *img, float *sino, float alpha, const CpDual *cp,
                          hipStream_t st)
{
    int maxnb = 0;
    for (const auto &g : p.gd) maxnb = std::max(maxnb, g.nb);
    dim3 grid((maxnb + 63) / 64, (unsigned)p.fp_max_blocks, p.n_slices);
    if (cp && cp->residual) return launch_fp<2>(p, grid, img, nullptr, alpha, *cp, 0, st);
    if (cp) return launch_fp<1>(p, grid, img, nullptr, alpha, *cp, 0, st);
    CpDual none{};
    return launch_fp<0>(p, grid, img, sino, alpha, none, 0, st);
}

// row[s][j] = (A img_s)[k][j] - y_s[k][j] for one projection k of a uniform plan
hipError_t launch_forward_row(const pyhst_plan &p, const float *img, const float *y, int k, float *row,
                              hipStream_t st)
{
    const GeoDev &g = p.gd[0];
    dim3 grid((g.nb + 63) / 64, 1, p.n_slices);
    CpDual r{row, y, 0.0f, 1};
    return launch_fp<3>(p, grid, img, nullptr, 1.0f, r, k, st);
}

}  // namespace pyhst
