// Matched forward projection A = s^2 B^T (section 2.3: the projector used
// inside the iterations; eq. (1)), evaluated ray-driven as a gather so that
// every bin is summed by one lane in a fixed order (deterministic).
//
// The paper projects an image held in a texture, which interpolates the image
// along rays and is not the transpose of the pixel-driven backprojector.  Here
// bin j of projection k sums exactly the pixels whose hat weight
// hat(t_k(px) - j) is non-zero.  Along an image line of the dominant axis
// (rows when |cos| >= |sin|, else columns) t is linear in the position,
// t - j = a (i - u_j), a = s cos (or s sin), so the bin touches the positions
// i in (u_j - 1/|a|, u_j + 1/|a|): at most ceil(2/|a|) of them.
//
// gfx950 layout.  Workgroup = 4 wavefronts = 4 projections x 64 bins of one
// slice; lane = bin.  A wavefront walks the lines of its projection in blocks
// of RB: for each block it stages the covering segment of every line (SEG
// positions, zero outside the image) in LDS with coalesced loads, then every
// lane reads its 2-3 candidates per line from LDS.  Coordinates: per (lane,
// line block) the crossing u of the block's first line is computed in FP64 and
// split into an integer base and an FP32 remainder; inside the block u advances
// by an FP32 slope, so every FP32 quantity stays below RB + 2 (ulp < 2e-6).
// Per candidate: offset, |.|, max, LDS read, FMA.
#include "internal.hpp"

namespace pyhst {

namespace {

constexpr int RB = 16;   // lines per staged block

// segment length (positions) that covers 64 bins x RB lines of one projection for pixel size s:
// 63/|a| + (RB - 1) |slope| + 2/|a| + 4 with |a| >= s / sqrt(2) and |slope| <= 1
inline int fp_seg(double s)
{
    const double ainv = 1.4142135623730951 / s;
    int seg = (int)std::ceil(65.0 * ainv + (RB - 1) + 4.0);
    return (seg + 3) & ~3;
}

template <int MODE>
__global__ __launch_bounds__(256) void fp_kernel(Tables T, const float *__restrict__ img, float *__restrict__ out,
                                                 float alpha, CpDual cp, int k0, int seg_len)
{
    extern __shared__ float stage[];   // [4 waves][RB][seg_len]
    const int slice = blockIdx.z;
    const SliceDev sd = T.slc[slice];
    const GeoDev &g = T.geo[sd.g];
    const int K = g.K, nb = g.nb, nx = g.nx, ny = g.ny;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int k = k0 + blockIdx.y * 4 + wv;
    const int j = blockIdx.x * 64 + lane;
    // MODE 3 projects the single projection k0 (wavefront 0 only)
    const bool wave_on = k < K && (MODE != 3 || wv == 0) && blockIdx.x * 64 < nb;
    float *seg = stage + wv * RB * seg_len;
    const float *im = img + sd.img_off;

    // projection geometry (wave-uniform); t = s (x c + y sn) + axis + shift
    const int kk = wave_on ? k : 0;
    const double c = T.cosd[g.ang_off + kk], sn = T.sind[g.ang_off + kk];
    const double s = g.s;
    const double cx = 0.5 * (nx - 1), cy = 0.5 * (ny - 1);
    const double t0 = g.axis + T.shiftd[g.ang_off + kk];
    const bool rows = fabs(c) >= fabs(sn);
    // along a line: t - j = a (i - u), u(line) = (j - t0 + a ci + bb cl - bb line) / a, where a and ci
    // belong to the axis walked along the line and bb and cl to the other one
    const double a = rows ? s * c : s * sn;
    const double bb = rows ? s * sn : s * c;
    const double ci = rows ? cx : cy, cl = rows ? cy : cx;
    const int n_lines = rows ? ny : nx;
    const double rho = 1.0 / fabs(a);
    const int ncand = (int)ceil(2.0 * rho);
    const double slope = -bb / a;                          // du per line
    const double u_first = ((double)j - t0 + a * ci + bb * cl) / a;   // u at line 0
    const float af = (float)a, rhof = (float)rho, slopef = (float)slope;
    const int lines_max = max(nx, ny);

    float acc = 0.0f;
    for (int l0 = 0; l0 < lines_max; l0 += RB) {
        const bool blk_on = wave_on && l0 < n_lines;
        // lane's crossing at the block's first line: FP64, split into base + remainder
        const double ub = fma((double)l0, slope, u_first);
        const double ubase = floor(ub);
        const float rem = (float)(ub - ubase);
        // segment start: lowest candidate over the wave's 64 bins and RB lines
        double lo = fmin(ub, ub + (RB - 1) * slope) - rho;
        for (int off = 32; off > 0; off >>= 1) lo = fmin(lo, __shfl_xor(lo, off, 64));
        const int seg0 = (int)floor(lo) - 1;
        __syncthreads();   // the previous block's reads are done
        if (blk_on) {
            if (rows) {
                for (int r = 0; r < RB; ++r) {
                    const int line = l0 + r;
                    const float *src = im + (int64_t)line * nx;
                    for (int p = lane; p < seg_len; p += 64) {
                        const int pos = seg0 + p;
                        seg[r * seg_len + p] = (line < ny && (unsigned)pos < (unsigned)nx) ? src[pos] : 0.0f;
                    }
                }
            } else {
                // columns: 16 lanes read 16 neighbouring columns of one row (64 B), 4 rows per step
                const int r = lane & 15;
                const int line = l0 + r;
                for (int p = lane >> 4; p < seg_len; p += 4) {
                    const int pos = seg0 + p;
                    seg[r * seg_len + p] =
                        (line < nx && (unsigned)pos < (unsigned)ny) ? im[(int64_t)pos * nx + line] : 0.0f;
                }
            }
        }
        __syncthreads();
        if (blk_on) {
            const int rel = (int)ubase - seg0;                 // base position inside the segment
            const int nl = min(RB, n_lines - l0);
            for (int r = 0; r < nl; ++r) {
                const float u = rem + (float)r * slopef;       // crossing relative to ubase
                const int i0 = (int)floorf(u - rhof) + 1;
                const float *row = seg + r * seg_len + rel;
                for (int n = 0; n < ncand; ++n) {
                    const int i = i0 + n;
                    const float w = fmaxf(0.0f, 1.0f - fabsf(af * ((float)i - u)));
                    acc = fmaf(w, row[i], acc);
                }
            }
        }
    }
    if (!wave_on || j >= nb) return;
    const int64_t o = sd.sino_off + (int64_t)k * nb + j;
    const float v = alpha * (float)(s * s) * acc;   // A = s^2 B^T
    if (MODE == 0) {
        out[o] = v;
    } else if (MODE == 1) {
        cp.p[o] = (cp.p[o] + cp.sigma * (v - cp.y[o])) / (1.0f + cp.sigma);
    } else if (MODE == 2) {
        cp.p[o] = v - cp.y[o];   // residual A x - y of the gradient step of ISTA/FISTA
    } else {
        cp.p[(int64_t)slice * nb + j] = v - cp.y[o];   // one projection's residual row per slice
    }
}

int plan_seg(const pyhst_plan &p)
{
    double smin = 1e300;
    for (const auto &g : p.gd) smin = std::min(smin, g.s);
    return fp_seg(smin);
}

template <int MODE>
hipError_t launch_fp(const pyhst_plan &p, dim3 grid, const float *img, float *sino, float alpha, const CpDual &cp,
                     int k0, hipStream_t st)
{
    const int seg = plan_seg(p);
    const size_t lds = (size_t)4 * RB * seg * sizeof(float);
    if (lds > 65536) {
        if (lds > 160 * 1024) return hipErrorInvalidValue;
        hipError_t e = hipFuncSetAttribute((const void *)fp_kernel<MODE>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)lds);
        if (e != hipSuccess) return e;
    }
    fp_kernel<MODE><<<grid, 256, lds, st>>>(p.t, img, sino, alpha, cp, k0, seg);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_forward(const pyhst_plan &p, const float *img, float *sino, float alpha, const CpDual *cp,
                          hipStream_t st)
{
    int maxnb = 0;
    for (const auto &g : p.gd) maxnb = std::max(maxnb, g.nb);
    dim3 grid((maxnb + 63) / 64, (unsigned)((p.max_K + 3) / 4), p.n_slices);
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
