// Total-variation operators (eq. (2), discretised as in Chambolle (2004):
// forward differences with a zero last difference, div = -grad^T), the ROF
// proximal map, the Chambolle-Pock dual TV step, the energy of eq. (3) and the
// power iteration for |[A; grad]|.  Memory-bound stencils on 2-D tiles: the
// ROF prox takes two dual steps per launch through LDS, the other stencils
// read their neighbours from L1/L2.  Reductions are deterministic:
// per-workgroup FP64 partials, then one workgroup sums them in a fixed order.
#include <cmath>

#include "internal.hpp"

namespace pyhst {

namespace {

__device__ inline float grad_x(const float *x, int64_t o, int ix, int nx) { return ix + 1 < nx ? x[o + 1] - x[o] : 0.0f; }
__device__ inline float grad_y(const float *x, int64_t o, int iy, int ny, int nx)
{
    return iy + 1 < ny ? x[o + nx] - x[o] : 0.0f;
}
__device__ inline float divergence(const float *q1, const float *q2, int64_t o, int ix, int iy, int nx, int ny)
{
    float a, b;
    if (nx == 1) a = 0.0f;
    else if (ix == 0) a = q1[o];
    else if (ix == nx - 1) a = -q1[o - 1];
    else a = q1[o] - q1[o - 1];
    if (ny == 1) b = 0.0f;
    else if (iy == 0) b = q2[o];
    else if (iy == ny - 1) b = -q2[o - nx];
    else b = q2[o] - q2[o - nx];
    return a + b;
}

// 2-D launch over images: workgroup = 64 x 8 pixels of one slice (256 threads, two rows each), so that
// no thread divides a 64-bit index; grid (ceil(nx / 64), ceil(ny / 8), slices).
constexpr int TTX = 64, TTY = 8;

// One fused inner step of the ROF dual projection:  q = (p + tau grad v) / (1 + tau |grad v|) with
// v = div p - g / lambda (p read, q written: ping-pong).  The workgroup evaluates v once per pixel of its
// tile plus the row below and the column to the right into LDS, then takes the forward differences
// from there.  ZERO: p = 0 (the first step), which is neither read nor needs clearing.
template <bool ZERO>
__global__ __launch_bounds__(256) void prox_step_kernel(int ny, int nx, const float *__restrict__ p1,
                                                        const float *__restrict__ p2, const float *__restrict__ g,
                                                        float inv_lambda, float tau, float *__restrict__ q1,
                                                        float *__restrict__ q2)
{
    __shared__ float v[TTY + 1][TTX + 1];
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int x0 = blockIdx.x * TTX, y0 = blockIdx.y * TTY;
    const int64_t base = (int64_t)blockIdx.z * ny * nx;
    auto v_at = [&](int x, int y) {
        const int64_t o = base + (int64_t)y * nx + x;
        const float d = ZERO ? 0.0f : divergence(p1, p2, o, x, y, nx, ny);
        return d - g[o] * inv_lambda;
    };
#pragma unroll
    for (int r = ty; r < TTY; r += 4)
        if (x0 + tx < nx && y0 + r < ny) v[r][tx] = v_at(x0 + tx, y0 + r);
    if (ty == 0) {
        if (x0 + tx < nx && y0 + TTY < ny) v[TTY][tx] = v_at(x0 + tx, y0 + TTY);
    } else if (ty == 1 && tx < TTY) {
        if (x0 + TTX < nx && y0 + tx < ny) v[tx][TTX] = v_at(x0 + TTX, y0 + tx);
    }
    __syncthreads();
#pragma unroll
    for (int r = ty; r < TTY; r += 4) {
        const int x = x0 + tx, y = y0 + r;
        if (x >= nx || y >= ny) continue;
        const float v0 = v[r][tx];
        const float a = x + 1 < nx ? v[r][tx + 1] - v0 : 0.0f;
        const float b = y + 1 < ny ? v[r + 1][tx] - v0 : 0.0f;
        const float im = 1.0f / (1.0f + tau * sqrtf(a * a + b * b));   // one division for both components
        const int64_t o = base + (int64_t)y * nx + x;
        q1[o] = ((ZERO ? 0.0f : p1[o]) + tau * a) * im;
        q2[o] = ((ZERO ? 0.0f : p2[o]) + tau * b) * im;
    }
}

// Two fused inner steps (p -> p' -> q) on a 64 x 16 tile.  q on the tile needs p' on the tile grown
// by one pixel on every side, which needs p on the tile grown by two; the workgroup stages p and g on
// that region in LDS, updates p to p' in place where it is needed, and writes only q: the dual field
// crosses HBM once per two steps.  Same operations in the same order as two single steps.
constexpr int FTX = 64, FTY = 16;
constexpr int FRX = FTX + 4, FRY = FTY + 4;   // staged region: x0 - 2 .. x0 + 65, y0 - 2 .. y0 + 17

template <bool ZERO>
__global__ __launch_bounds__(256) void prox_step2_kernel(int ny, int nx, const float *__restrict__ p1,
                                                         const float *__restrict__ p2, const float *__restrict__ g,
                                                         float inv_lambda, float tau, float *__restrict__ q1,
                                                         float *__restrict__ q2)
{
    __shared__ float s1[FRY][FRX], s2[FRY][FRX], sg[FRY][FRX], sv[FRY][FRX];
    const int tid = threadIdx.x;
    const int x0 = blockIdx.x * FTX - 2, y0 = blockIdx.y * FTY - 2;   // image coordinates of region (0, 0)
    const int64_t base = (int64_t)blockIdx.z * ny * nx;
    auto inside = [&](int x, int y) { return (unsigned)x < (unsigned)nx && (unsigned)y < (unsigned)ny; };
    for (int i = tid; i < FRX * FRY; i += 256) {
        const int ry = i / FRX, rx = i - ry * FRX;
        const int x = x0 + rx, y = y0 + ry;
        const bool in = inside(x, y);
        const int64_t o = base + (int64_t)y * nx + x;
        s1[ry][rx] = (!ZERO && in) ? p1[o] : 0.0f;
        s2[ry][rx] = (!ZERO && in) ? p2[o] : 0.0f;
        sg[ry][rx] = in ? g[o] : 0.0f;
    }
    __syncthreads();
    // v = div p - g / lambda at an image point whose region coordinates are (rx, ry)
    auto v_at = [&](int rx, int ry, int x, int y) {
        float a, b;
        if (nx == 1) a = 0.0f;
        else if (x == 0) a = s1[ry][rx];
        else if (x == nx - 1) a = -s1[ry][rx - 1];
        else a = s1[ry][rx] - s1[ry][rx - 1];
        if (ny == 1) b = 0.0f;
        else if (y == 0) b = s2[ry][rx];
        else if (y == ny - 1) b = -s2[ry - 1][rx];
        else b = s2[ry][rx] - s2[ry - 1][rx];
        return (a + b) - sg[ry][rx] * inv_lambda;
    };
    // Region coordinates: the tile is [2, FRX - 2) x [2, FRY - 2).  q there needs v' on [2, FRX - 1) x
    // [2, FRY - 1), which needs p' on [1, FRX - 1) x [1, FRY - 1), which needs v on [1, FRX) x [1, FRY),
    // which needs p and g on the whole region.
    // first step: v on [1, FRX) x [1, FRY)
    for (int i = tid; i < (FRX - 1) * (FRY - 1); i += 256) {
        const int ry = 1 + i / (FRX - 1), rx = 1 + i % (FRX - 1);
        const int x = x0 + rx, y = y0 + ry;
        if (inside(x, y)) sv[ry][rx] = v_at(rx, ry, x, y);
    }
    __syncthreads();
    // p' on [1, FRX - 1) x [1, FRY - 1), held in registers until every read of p is done
    constexpr int NP = (FRX - 2) * (FRY - 2);   // 1188 <= 5 * 256
    float n1[5], n2[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        const int i = tid + 256 * k;
        n1[k] = 0.0f;
        n2[k] = 0.0f;
        if (i >= NP) continue;
        const int ry = 1 + i / (FRX - 2), rx = 1 + i % (FRX - 2);
        const int x = x0 + rx, y = y0 + ry;
        if (!inside(x, y)) continue;
        const float v0 = sv[ry][rx];
        const float a = x + 1 < nx ? sv[ry][rx + 1] - v0 : 0.0f;
        const float b = y + 1 < ny ? sv[ry + 1][rx] - v0 : 0.0f;
        const float im = 1.0f / (1.0f + tau * sqrtf(a * a + b * b));
        n1[k] = (s1[ry][rx] + tau * a) * im;
        n2[k] = (s2[ry][rx] + tau * b) * im;
    }
    __syncthreads();   // every read of p is done
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        const int i = tid + 256 * k;
        if (i >= NP) continue;
        const int ry = 1 + i / (FRX - 2), rx = 1 + i % (FRX - 2);
        s1[ry][rx] = n1[k];
        s2[ry][rx] = n2[k];
    }
    __syncthreads();
    // second step: v' on [2, FRX - 1) x [2, FRY - 1), q on the tile [2, FRX - 2) x [2, FRY - 2)
    for (int i = tid; i < (FRX - 3) * (FRY - 3); i += 256) {
        const int ry = 2 + i / (FRX - 3), rx = 2 + i % (FRX - 3);
        const int x = x0 + rx, y = y0 + ry;
        if (inside(x, y)) sv[ry][rx] = v_at(rx, ry, x, y);
    }
    __syncthreads();
    for (int i = tid; i < FTX * FTY; i += 256) {
        const int ry = 2 + i / FTX, rx = 2 + i % FTX;
        const int x = x0 + rx, y = y0 + ry;
        if (!inside(x, y)) continue;
        const float v0 = sv[ry][rx];
        const float a = x + 1 < nx ? sv[ry][rx + 1] - v0 : 0.0f;
        const float b = y + 1 < ny ? sv[ry + 1][rx] - v0 : 0.0f;
        const float im = 1.0f / (1.0f + tau * sqrtf(a * a + b * b));
        const int64_t o = base + (int64_t)y * nx + x;
        q1[o] = (s1[ry][rx] + tau * a) * im;
        q2[o] = (s2[ry][rx] + tau * b) * im;
    }
}

// u = g - lambda div p
__global__ __launch_bounds__(256) void prox_final_kernel(int ny, int nx, const float *__restrict__ p1,
                                                         const float *__restrict__ p2, const float *g, float lambda,
                                                         float *u)
{
    const int x = blockIdx.x * TTX + (threadIdx.x & 63);
    if (x >= nx) return;
    const int64_t base = (int64_t)blockIdx.z * ny * nx;
#pragma unroll
    for (int r = threadIdx.x >> 6; r < TTY; r += 4) {
        const int y = blockIdx.y * TTY + r;
        if (y >= ny) break;
        const int64_t o = base + (int64_t)y * nx + x;
        u[o] = g[o] - lambda * divergence(p1, p2, o, x, y, nx, ny);
    }
}

__global__ void fill_kernel(float *buf, int64_t n, float v)
{
    for (int64_t o = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; o < n; o += (int64_t)gridDim.x * blockDim.x)
        buf[o] = v;
}

__global__ void copy_kernel(float *dst, const float *src, int64_t n)
{
    for (int64_t o = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; o < n; o += (int64_t)gridDim.x * blockDim.x)
        dst[o] = src[o];
}

// y = a x + b y
__global__ void axpby_kernel(float *y, const float *x, int64_t n, float a, float b)
{
    for (int64_t o = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; o < n; o += (int64_t)gridDim.x * blockDim.x)
        y[o] = a * x[o] + b * y[o];
}

// dst = src where src > thr, else 0 (the strongly absorbing part of a first reconstruction)
__global__ void threshold_kernel(float *__restrict__ dst, const float *__restrict__ src, int64_t n, float thr)
{
    for (int64_t o = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; o < n; o += (int64_t)gridDim.x * blockDim.x) {
        const float v = src[o];
        dst[o] = v > thr ? v : 0.0f;
    }
}

// FISTA extrapolation: z = xn + m (xn - xo)
__global__ void momentum_kernel(float *__restrict__ z, const float *__restrict__ xn, const float *__restrict__ xo,
                                int64_t n, float m)
{
    for (int64_t o = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; o < n; o += (int64_t)gridDim.x * blockDim.x) {
        const float a = xn[o];
        z[o] = fmaf(m, a - xo[o], a);
    }
}

// Chambolle-Pock dual TV step: q <- pi_lambda(q + sigma grad xbar)
__global__ __launch_bounds__(256) void cp_q_kernel(int ny, int nx, const float *__restrict__ xb,
                                                   float *__restrict__ q1, float *__restrict__ q2, float sigma,
                                                   float lambda)
{
    const int ix = blockIdx.x * TTX + (threadIdx.x & 63);
    if (ix >= nx) return;
    const int64_t base = (int64_t)blockIdx.z * ny * nx;
#pragma unroll
    for (int r = threadIdx.x >> 6; r < TTY; r += 4) {
        const int iy = blockIdx.y * TTY + r;
        if (iy >= ny) break;
        const int64_t o = base + (int64_t)iy * nx + ix;
        float a = q1[o] + sigma * grad_x(xb, o, ix, nx);
        float b = q2[o] + sigma * grad_y(xb, o, iy, ny, nx);
        if (lambda > 0.0f) {
            const float d = fmaxf(1.0f, sqrtf(a * a + b * b) / lambda);
            const float id = 1.0f / d;
            a *= id;
            b *= id;
        } else {
            a = 0.0f;
            b = 0.0f;
        }
        q1[o] = a;
        q2[o] = b;
    }
}

// out -= c div(grad x)  (so that out = A^T A x + c grad^T grad x)
__global__ __launch_bounds__(256) void sub_divgrad_kernel(int ny, int nx, const float *__restrict__ x,
                                                          float *__restrict__ out, float c)
{
    const int ix = blockIdx.x * TTX + (threadIdx.x & 63);
    if (ix >= nx) return;
    const int64_t base = (int64_t)blockIdx.z * ny * nx;
#pragma unroll
    for (int r = threadIdx.x >> 6; r < TTY; r += 4) {
        const int iy = blockIdx.y * TTY + r;
        if (iy >= ny) break;
        const int64_t o = base + (int64_t)iy * nx + ix;
        // div(grad x) at o, from the forward differences around o
        float a, b;
        const float gx = grad_x(x, o, ix, nx), gy = grad_y(x, o, iy, ny, nx);
        const float gxl = ix > 0 ? grad_x(x, o - 1, ix - 1, nx) : 0.0f;
        const float gyu = iy > 0 ? grad_y(x, o - nx, iy - 1, ny, nx) : 0.0f;
        if (nx == 1) a = 0.0f;
        else if (ix == 0) a = gx;
        else if (ix == nx - 1) a = -gxl;
        else a = gx - gxl;
        if (ny == 1) b = 0.0f;
        else if (iy == 0) b = gy;
        else if (iy == ny - 1) b = -gyu;
        else b = gy - gyu;
        out[o] -= c * (a + b);
    }
}

__device__ inline double block_sum(double v, double *sh)
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

// partials[b] = sum over this block's share of 0.5 (ax - y)^2 + lambda |grad x|
__global__ __launch_bounds__(256) void energy_partial_kernel(int64_t n_s, const float *__restrict__ ax,
                                                             const float *__restrict__ y, int64_t n_i, int ny, int nx,
                                                             const float *__restrict__ x, float lambda,
                                                             double *__restrict__ partials)
{
    __shared__ double sh[4];
    double acc = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t o = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; o < n_s; o += stride) {
        const double d = (double)ax[o] - (double)y[o];
        acc += 0.5 * d * d;
    }
    for (int64_t o = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; o < n_i; o += stride) {
        const int64_t pix = o % ((int64_t)ny * nx);
        const int iy = (int)(pix / nx), ix = (int)(pix - (int64_t)iy * nx);
        const double a = grad_x(x, o, ix, nx), b = grad_y(x, o, iy, ny, nx);
        acc += (double)lambda * sqrt(a * a + b * b);
    }
    const double t = block_sum(acc, sh);
    if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

// partials[b] = sum of squares of v
__global__ __launch_bounds__(256) void sumsq_partial_kernel(int64_t n, const float *__restrict__ v,
                                                            double *__restrict__ partials)
{
    __shared__ double sh[4];
    double acc = 0.0;
    for (int64_t o = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; o < n; o += (int64_t)gridDim.x * blockDim.x)
        acc += (double)v[o] * (double)v[o];
    const double t = block_sum(acc, sh);
    if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

__global__ __launch_bounds__(256) void final_sum_kernel(const double *__restrict__ partials, int n,
                                                        float *out_f, double *out_d)
{
    __shared__ double sh[4];
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) acc += partials[i];
    const double t = block_sum(acc, sh);
    if (threadIdx.x == 0) {
        if (out_f) *out_f = (float)t;
        if (out_d) *out_d = t;
    }
}

__global__ void scale_inv_sqrt_kernel(float *x, int64_t n, const double *sumsq)
{
    const float inv = (float)(1.0 / sqrt(*sumsq));
    for (int64_t o = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; o < n; o += (int64_t)gridDim.x * blockDim.x)
        x[o] *= inv;
}

dim3 grid_img(int S, int ny, int nx)
{
    return dim3((unsigned)((nx + TTX - 1) / TTX), (unsigned)((ny + TTY - 1) / TTY), (unsigned)S);
}

unsigned grid_for(int64_t n)
{
    int64_t b = (n + 255) / 256;
    if (b > 8192) b = 8192;
    if (b < 1) b = 1;
    return (unsigned)b;
}

}  // namespace

int energy_partials(const pyhst_plan &) { return 1024; }

hipError_t launch_fill(float *buf, int64_t n, float v, hipStream_t st)
{
    fill_kernel<<<grid_for(n), 256, 0, st>>>(buf, n, v);
    return hipGetLastError();
}

hipError_t launch_momentum(float *z, const float *xn, const float *xo, int64_t n, float m, hipStream_t st)
{
    momentum_kernel<<<grid_for(n), 256, 0, st>>>(z, xn, xo, n, m);
    return hipGetLastError();
}

hipError_t launch_threshold(float *dst, const float *src, int64_t n, float thr, hipStream_t st)
{
    threshold_kernel<<<grid_for(n), 256, 0, st>>>(dst, src, n, thr);
    return hipGetLastError();
}

hipError_t launch_copy(float *dst, const float *src, int64_t n, hipStream_t st)
{
    copy_kernel<<<grid_for(n), 256, 0, st>>>(dst, src, n);
    return hipGetLastError();
}

hipError_t launch_axpby(float *y, const float *x, int64_t n, float a, float b, hipStream_t st)
{
    axpby_kernel<<<grid_for(n), 256, 0, st>>>(y, x, n, a, b);
    return hipGetLastError();
}

hipError_t launch_tv_prox(int S, int ny, int nx, const float *in, float *out, float lambda, int n_inner,
                          float *work, hipStream_t st)
{
    const int64_t n = (int64_t)S * ny * nx;
    if (!(lambda > 0.0f) || n_inner <= 0) {
        if (out != in) copy_kernel<<<grid_for(n), 256, 0, st>>>(out, in, n);
        return hipGetLastError();
    }
    float *p1 = work, *p2 = work + n, *q1 = work + 2 * n, *q2 = work + 3 * n;
    const dim3 gi = grid_img(S, ny, nx);
    const dim3 g2((unsigned)((nx + FTX - 1) / FTX), (unsigned)((ny + FTY - 1) / FTY), (unsigned)S);
    const float il = 1.0f / lambda;
    for (int it = 0; it < n_inner;) {
        if (n_inner - it >= 2) {   // two steps per launch
            if (it == 0) prox_step2_kernel<true><<<g2, 256, 0, st>>>(ny, nx, p1, p2, in, il, 0.125f, q1, q2);
            else prox_step2_kernel<false><<<g2, 256, 0, st>>>(ny, nx, p1, p2, in, il, 0.125f, q1, q2);
            it += 2;
        } else {
            if (it == 0) prox_step_kernel<true><<<gi, 256, 0, st>>>(ny, nx, p1, p2, in, il, 0.125f, q1, q2);
            else prox_step_kernel<false><<<gi, 256, 0, st>>>(ny, nx, p1, p2, in, il, 0.125f, q1, q2);
            it += 1;
        }
        std::swap(p1, q1);
        std::swap(p2, q2);
    }
    prox_final_kernel<<<gi, 256, 0, st>>>(ny, nx, p1, p2, in, lambda, out);
    return hipGetLastError();
}

hipError_t launch_cp_dual_q(const pyhst_plan &p, const float *xbar, float *q1, float *q2, float sigma, float lambda,
                            hipStream_t st)
{
    const GeoDev &g = p.gd[0];
    cp_q_kernel<<<grid_img(p.n_slices, g.ny, g.nx), 256, 0, st>>>(g.ny, g.nx, xbar, q1, q2, sigma, lambda);
    return hipGetLastError();
}

hipError_t launch_cp_energy(const pyhst_plan &p, const float *ax, const float *y, const float *x, float lambda,
                            double *partials, int n_part, float *energy_dev, hipStream_t st)
{
    const GeoDev &g = p.gd[0];
    const int64_t ns = (int64_t)p.n_slices * g.K * g.nb, ni = (int64_t)p.n_slices * g.ny * g.nx;
    energy_partial_kernel<<<n_part, 256, 0, st>>>(ns, ax, y, ni, g.ny, g.nx, x, lambda, partials);
    final_sum_kernel<<<1, 256, 0, st>>>(partials, n_part, energy_dev, nullptr);
    return hipGetLastError();
}

// out = K^T K x = A^T A x - mu^2 div grad x (grad_scale = mu^2 > 0) or A^T A x (grad_scale = 0);
// then norm_dev = |out|^2
hipError_t launch_power_step(const pyhst_plan &p, const float *x, float *out, float *tmp_sino, double *partials,
                             int n_part, double *norm_dev, float grad_scale, hipStream_t st)
{
    const GeoDev &g = p.gd[0];
    const float s2 = (float)(g.s * g.s);
    hipError_t e = launch_forward(p, x, tmp_sino, 1.0f, nullptr, st);
    if (e != hipSuccess) return e;
    e = launch_backproject(p, tmp_sino, 0, out, s2, 0.0f, nullptr, st);
    if (e != hipSuccess) return e;
    const int64_t n = (int64_t)p.n_slices * g.ny * g.nx;
    if (grad_scale > 0.0f)
        sub_divgrad_kernel<<<grid_img(p.n_slices, g.ny, g.nx), 256, 0, st>>>(g.ny, g.nx, x, out, grad_scale);
    sumsq_partial_kernel<<<n_part, 256, 0, st>>>(n, out, partials);
    final_sum_kernel<<<1, 256, 0, st>>>(partials, n_part, nullptr, norm_dev);
    return hipGetLastError();
}

hipError_t launch_scale_by_inv(float *x, int64_t n, const double *norm_dev, hipStream_t st)
{
    scale_inv_sqrt_kernel<<<grid_for(n), 256, 0, st>>>(x, n, norm_dev);
    return hipGetLastError();
}

}  // namespace pyhst

namespace pyhst {
namespace {

// rel[s] = |ax_s - y_s| / |y_s| over the sinogram of slice s (one workgroup per slice)
__global__ __launch_bounds__(256) void residual_kernel(Tables T, const float *__restrict__ ax,
                                                       const float *__restrict__ y, float *__restrict__ rel)
{
    __shared__ double sh[4];
    const SliceDev sd = T.slc[blockIdx.x];
    const GeoDev &g = T.geo[sd.g];
    const int64_t n = (int64_t)g.K * g.nb;
    double num = 0.0, den = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        const double a = ax[sd.sino_off + i], b = y[sd.sino_off + i];
        num += (a - b) * (a - b);
        den += b * b;
    }
    const double tn = block_sum(num, sh);
    const double td = block_sum(den, sh);
    if (threadIdx.x == 0) rel[blockIdx.x] = (float)(td > 0.0 ? sqrt(tn / td) : 0.0);
}

// err[s] = weight sum_j row[s][j]^2 (+ err[s] when accumulating; one workgroup per slice)
__global__ __launch_bounds__(256) void rowsq_kernel(const float *__restrict__ row, int nb, float *__restrict__ err,
                                                    float weight, int accumulate)
{
    __shared__ double sh[4];
    const float *r = row + (int64_t)blockIdx.x * nb;
    double acc = 0.0;
    for (int j = threadIdx.x; j < nb; j += blockDim.x) acc += (double)r[j] * (double)r[j];
    const double t = block_sum(acc, sh);
    if (threadIdx.x == 0) err[blockIdx.x] = (float)((double)weight * t + (accumulate ? (double)err[blockIdx.x] : 0.0));
}

// e[s] = cos(xb_s - x0_s, xb_s) (one workgroup per slice, FP64 sums)
__global__ __launch_bounds__(256) void decoherence_kernel(Tables T, const float *__restrict__ xb,
                                                          const float *__restrict__ x0, float *__restrict__ e)
{
    __shared__ double sh[4];
    const SliceDev sd = T.slc[blockIdx.x];
    const GeoDev &g = T.geo[sd.g];
    const int64_t n = (int64_t)g.ny * g.nx;
    double da = 0.0, dd = 0.0, aa = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        const double a = xb[sd.img_off + i], d = a - (double)x0[sd.img_off + i];
        da += d * a;
        dd += d * d;
        aa += a * a;
    }
    const double t_da = block_sum(da, sh);
    const double t_dd = block_sum(dd, sh);
    const double t_aa = block_sum(aa, sh);
    if (threadIdx.x == 0) e[blockIdx.x] = (float)(t_dd > 0.0 && t_aa > 0.0 ? t_da / sqrt(t_dd * t_aa) : 0.0);
}

}  // namespace
}  // namespace pyhst

extern "C" int pyhst_cv_error(const pyhst_plan *p, const float *x, const float *y, int32_t k, float *row, float *err,
                              float weight, int32_t accumulate, hipStream_t st)
{
    using namespace pyhst;
    if (!p || !x || !y || !row || !err) return fail(PYHST_EARG, "cv_error: NULL argument");
    if (!std::isfinite(weight)) return fail(PYHST_EARG, "cv_error: weight must be finite");
    if (!p->uniform) return fail(PYHST_EARG, "cv_error: needs a uniform plan");
    if (k < 0 || k >= p->gd[0].K) return fail(PYHST_EARG, "cv_error: projection index out of range");
    hipError_t e = launch_forward_row(*p, x, y, k, row, st);
    if (e == hipSuccess) {
        rowsq_kernel<<<p->n_slices, 256, 0, st>>>(row, p->gd[0].nb, err, weight, accumulate ? 1 : 0);
        e = hipGetLastError();
    }
    return e == hipSuccess ? PYHST_OK : hip_fail(e, "cv_error");
}

extern "C" int pyhst_decoherence(const pyhst_plan *p, const float *x_beta, const float *x_zero, float *e_out,
                                 hipStream_t st)
{
    using namespace pyhst;
    if (!p || !x_beta || !x_zero || !e_out) return fail(PYHST_EARG, "decoherence: NULL argument");
    decoherence_kernel<<<p->n_slices, 256, 0, st>>>(p->t, x_beta, x_zero, e_out);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? PYHST_OK : hip_fail(e, "decoherence");
}

extern "C" int pyhst_slice_residual(const pyhst_plan *p, const float *ax, const float *y, float *rel,
                                    hipStream_t st)
{
    using namespace pyhst;
    if (!p || !ax || !y || !rel) return fail(PYHST_EARG, "slice_residual: NULL argument");
    residual_kernel<<<p->n_slices, 256, 0, st>>>(p->t, ax, y, rel);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? PYHST_OK : hip_fail(e, "slice_residual");
}
