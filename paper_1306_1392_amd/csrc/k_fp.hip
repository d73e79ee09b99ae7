// Matched forward projection A = s^2 B^T, evaluated ray-driven as a gather
// (section 2.3: the projector used inside the iterations; eq. (1)).
//
// The paper projects an image held in a texture, which interpolates the image
// along rays and is not the transpose of the pixel-driven backprojector.
// Here every detector bin j of projection k sums exactly the pixels whose hat
// weight hat(t_k(px) - j) is non-zero: walking the dominant image axis
// (rows when |cos| >= |sin|, else columns), at most ceil(2 / (s |cos|)) pixels
// per line can touch the bin.  Their positions are anchored in FP64 per line
// (t reaches ~2000 bins, where FP32 would lose 2e-4 bin); the weights are FP32.
//
// Launch: workgroup = one projection x 64 bins; its 4 wavefronts take every
// fourth image line and their partial sums are added in a fixed order (LDS),
// so one slice already gives nb/64 x K workgroups and the result is deterministic.
#include "internal.hpp"

namespace pyhst {

namespace {

template <int MODE>
__global__ __launch_bounds__(256) void fp_kernel(Tables T, const float *__restrict__ img, float *__restrict__ out,
                                                 float alpha, CpDual cp, int k0)
{
    __shared__ float part[3][64];
    const int slice = blockIdx.z;
    const SliceDev sd = T.slc[slice];
    const GeoDev &g = T.geo[sd.g];
    const int K = g.K, nb = g.nb, nx = g.nx, ny = g.ny;
    const int k = blockIdx.y + k0;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int j = blockIdx.x * 64 + lane;
    if (k >= K || blockIdx.x * 64 >= nb) return;   // uniform over the workgroup

    const double c = T.cosd[g.ang_off + k], sn = T.sind[g.ang_off + k];
    const double s = g.s;
    const double off = g.axis + T.shiftd[g.ang_off + k] - (double)j;   // t - j = s (x c + y sn) + off
    const double cx = 0.5 * (nx - 1), cy = 0.5 * (ny - 1);
    const float *im = img + sd.img_off;
    float acc = 0.0f;

    if (fabs(c) >= fabs(sn)) {
        // walk rows (the 4 wavefronts take rows wv, wv + 4, ...): along a row
        // t - j = s c (ix - cx) + B(iy), B(iy) = off + s sn (iy - cy)
        const double sc = s * c;
        const double rho = 1.0 / fabs(sc);
        const int ncand = (int)ceil(2.0 * rho);
        const double du = -(s * sn) / sc;                 // change of the crossing position per row
        const double u0 = cx - (off - s * sn * cy) / sc;  // crossing ix (real) of row 0
        const float scf = (float)sc;
        for (int iy = wv; iy < ny; iy += 4) {
            const double u = fma((double)iy, du, u0);
            const double fl = floor(u - rho);
            const int i0 = (int)fl + 1;
            float d = (float)((fl + 1.0) - u) * scf;      // t - j at pixel i0
            const float *rowp = im + (int64_t)iy * nx;
            for (int n = 0; n < ncand; ++n, d += scf) {
                const int ix = i0 + n;
                const float w = fmaxf(0.0f, 1.0f - fabsf(d));
                if ((unsigned)ix < (unsigned)nx) acc = fmaf(w, rowp[ix], acc);
            }
        }
    } else {
        // walk columns: along a column, t - j = s sn (iy - cy) + C(ix), C(ix) = off + s c (ix - cx)
        const double ss = s * sn;
        const double rho = 1.0 / fabs(ss);
        const int ncand = (int)ceil(2.0 * rho);
        const double dv = -(s * c) / ss;
        const double v0 = cy - (off - s * c * cx) / ss;
        const float ssf = (float)ss;
        for (int ix = wv; ix < nx; ix += 4) {
            const double v = fma((double)ix, dv, v0);
            const double fl = floor(v - rho);
            const int i0 = (int)fl + 1;
            float d = (float)((fl + 1.0) - v) * ssf;
            for (int n = 0; n < ncand; ++n, d += ssf) {
                const int iy = i0 + n;
                const float w = fmaxf(0.0f, 1.0f - fabsf(d));
                if ((unsigned)iy < (unsigned)ny) acc = fmaf(w, im[(int64_t)iy * nx + ix], acc);
            }
        }
    }
    // fixed-order reduction of the four partial sums
    if (wv > 0) part[wv - 1][lane] = acc;
    __syncthreads();
    if (wv > 0 || j >= nb) return;
    acc = ((acc + part[0][lane]) + part[1][lane]) + part[2][lane];
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

}  // namespace

hipError_t launch_forward(const pyhst_plan &p, const float *img, float *sino, float alpha, const CpDual *cp,
                          hipStream_t st)
{
    int maxnb = 0;
    for (const auto &g : p.gd) maxnb = std::max(maxnb, g.nb);
    dim3 grid((maxnb + 63) / 64, (unsigned)p.max_K, p.n_slices);
    if (cp && cp->residual) {
        fp_kernel<2><<<grid, 256, 0, st>>>(p.t, img, nullptr, alpha, *cp, 0);
    } else if (cp) {
        fp_kernel<1><<<grid, 256, 0, st>>>(p.t, img, nullptr, alpha, *cp, 0);
    } else {
        CpDual none{};
        fp_kernel<0><<<grid, 256, 0, st>>>(p.t, img, sino, alpha, none, 0);
    }
    return hipGetLastError();
}

// row[s][j] = (A img_s)[k][j] - y_s[k][j] for one projection k of a uniform plan
hipError_t launch_forward_row(const pyhst_plan &p, const float *img, const float *y, int k, float *row,
                              hipStream_t st)
{
    const GeoDev &g = p.gd[0];
    dim3 grid((g.nb + 63) / 64, 1, p.n_slices);
    CpDual r{row, y, 0.0f, 1};
    fp_kernel<3><<<grid, 256, 0, st>>>(p.t, img, nullptr, 1.0f, r, k);
    return hipGetLastError();
}

}  // namespace pyhst
