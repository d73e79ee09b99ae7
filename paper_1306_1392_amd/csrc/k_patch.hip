// Overlapping-patch dictionary prior (section 3.2, eqs. (4)-(9)) solved by
// ISTA / FISTA on the patch coefficients W, for a batch of slices.
//
// Patches: m x m, top-left corners on a grid of step `stride` per axis (the
// last corner moved to n - m); patch p = row-corner index * n_cx + column-corner
// index.  The core of a pixel is its L1-nearest patch centre (lowest index on
// ties); with a separable corner grid that is the pair of per-axis nearest
// corners, tabulated by a small kernel at the start of every call.
//
// One gradient evaluation at coefficients Z (eq. (9)):
//   X = Z D                      (GEMM, [S*N_p][n_atoms] x [n_atoms][m*m])
//   x_i = X_core(i)(i - r)       (assemble kernel)
//   R = Pi^T (Pi x - y)          (projector residual + backprojector, or x - y when Pi = I)
//   R_i += rho sum_{p covering i} (x_i - X_p(i - r_p))
//   G = core_patches(R) + rho (X - patches(x))
//   grad = 2 G D^T               (GEMM with D^T)
// The GEMMs run on the FP32 matrix cores (v_mfma_f32_32x32x2f32) when N <= 128 and N, K are
// multiples of 32 (the dictionary shapes in practice), else on an FP32 register-tiled kernel (LDS
// tiles of 64 x 64 x 16, 4 x 4 outputs per thread).  Both sum in a fixed order.
#include <cmath>
#include <cstring>
#include <vector>

#include "internal.hpp"

namespace pyhst {
namespace {

constexpr int GT = 64, GK = 16;

// C[M][N] = alpha * A[M][K] B[K][N]   (row-major, leading dimensions K, N, N)
__global__ __launch_bounds__(256) void sgemm_kernel(const float *__restrict__ A, const float *__restrict__ B,
                                                    float *__restrict__ C, int M, int N, int K, float alpha)
{
    __shared__ float sA[GK][GT + 4];
    __shared__ float sB[GK][GT + 4];
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int m0 = blockIdx.x * GT, n0 = blockIdx.y * GT;
    float acc[4][4] = {};
    for (int k0 = 0; k0 < K; k0 += GK) {
        // A tile: 64 rows x 16 k; B tile: 16 k x 64 columns; 4 elements per thread each
        for (int e = threadIdx.x; e < GT * GK; e += 256) {
            const int r = e / GK, kk = e % GK;
            const int gm = m0 + r, gk = k0 + kk;
            sA[kk][r] = (gm < M && gk < K) ? A[(int64_t)gm * K + gk] : 0.0f;
            const int kb = e / GT, c = e % GT;
            const int gkb = k0 + kb, gn = n0 + c;
            sB[kb][c] = (gkb < K && gn < N) ? B[(int64_t)gkb * N + gn] : 0.0f;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < GK; ++kk) {
            float a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = sA[kk][ty * 4 + i];
#pragma unroll
            for (int j = 0; j < 4; ++j) b[j] = sB[kk][tx * 4 + j];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = fmaf(a[i], b[j], acc[i][j]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int gm = m0 + ty * 4 + i;
        if (gm >= M) continue;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int gn = n0 + tx * 4 + j;
            if (gn < N) C[(int64_t)gm * N + gn] = alpha * acc[i][j];
        }
    }
}

struct PatchGeo {
    const int *cy, *cx;          // corners per axis
    const int *core_y, *core_x;  // per pixel row / column: index of the nearest corner (its core)
    const int *first_y, *last_y; // per pixel row: range of corner indices whose patch covers the row
    const int *first_x, *last_x;
    int ny, nx, m, ncy, ncx, np;
};

__device__ inline int64_t pix_of(int64_t i, int ny, int nx, int &s, int &iy, int &ix)
{
    const int64_t per = (int64_t)ny * nx;
    s = (int)(i / per);
    const int64_t r = i - (int64_t)s * per;
    iy = (int)(r / nx);
    ix = (int)(r - (int64_t)iy * nx);
    return r;
}

// x[s][i] = X[s][core(i)][i - r_core]
__global__ void assemble_kernel(PatchGeo g, const float *__restrict__ X, float *__restrict__ x, int S)
{
    const int64_t n = (int64_t)S * g.ny * g.nx;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        int s, iy, ix;
        pix_of(i, g.ny, g.nx, s, iy, ix);
        const int a = g.core_y[iy], b = g.core_x[ix];
        const int p = a * g.ncx + b;
        const int ly = iy - g.cy[a], lx = ix - g.cx[b];
        x[i] = X[((int64_t)s * g.np + p) * g.m * g.m + ly * g.m + lx];
    }
}

// R[s][i] += rho * sum over patches p covering i of (x_i - X_p(i - r_p))
__global__ void similarity_kernel(PatchGeo g, const float *__restrict__ X, const float *__restrict__ x,
                                  float *__restrict__ R, float rho, int S)
{
    const int64_t n = (int64_t)S * g.ny * g.nx;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        int s, iy, ix;
        pix_of(i, g.ny, g.nx, s, iy, ix);
        const float xi = x[i];
        float acc = 0.0f;
        for (int a = g.first_y[iy]; a <= g.last_y[iy]; ++a)
            for (int b = g.first_x[ix]; b <= g.last_x[ix]; ++b) {
                const int p = a * g.ncx + b;
                acc += xi - X[((int64_t)s * g.np + p) * g.m * g.m + (iy - g.cy[a]) * g.m + (ix - g.cx[b])];
            }
        R[i] += rho * acc;
    }
}

// G[s][p][l] = (core(i) == p ? R_i : 0) + rho (X[s][p][l] - x_i),  i = r_p + l
__global__ void patch_grad_kernel(PatchGeo g, const float *__restrict__ X, const float *__restrict__ x,
                                  const float *__restrict__ R, float rho, float *__restrict__ G, int S)
{
    const int mm = g.m * g.m;
    const int64_t n = (int64_t)S * g.np * mm;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t sp = e / mm;
        const int l = (int)(e - sp * mm);
        const int s = (int)(sp / g.np), p = (int)(sp - (int64_t)s * g.np);
        const int a = p / g.ncx, b = p - a * g.ncx;
        const int iy = g.cy[a] + l / g.m, ix = g.cx[b] + l % g.m;
        const int64_t i = ((int64_t)s * g.ny + iy) * g.nx + ix;
        const bool core = g.core_y[iy] == a && g.core_x[ix] == b;
        G[e] = (core ? R[i] : 0.0f) + rho * (X[e] - x[i]);
    }
}

// W_new = soft(Z - grad / L, beta / L);  FISTA: Z = W_new + mom (W_new - W_old);  ISTA: Z = W_new
__global__ void shrink_kernel(const float *__restrict__ grad, float *__restrict__ Z, float *__restrict__ W,
                              int64_t n, float invL, float thr, float mom, int fast)
{
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const float v = Z[e] - grad[e] * invL;
        const float wn = copysignf(fmaxf(fabsf(v) - thr, 0.0f), v);
        const float wo = W[e];
        W[e] = wn;
        Z[e] = fast ? fmaf(mom, wn - wo, wn) : wn;
    }
}

// r = x - y (identity projector)
__global__ void diff_kernel(const float *__restrict__ x, const float *__restrict__ y, float *__restrict__ r, int64_t n)
{
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        r[e] = y ? x[e] - y[e] : x[e];
}

// partials: sum of a^2 over one buffer, rho * sum (patches(x) - X)^2 and beta * sum |W| (FP64)
__global__ __launch_bounds__(256) void patch_energy_kernel(PatchGeo g, const float *__restrict__ r, int64_t nr,
                                                           const float *__restrict__ X, const float *__restrict__ x,
                                                           const float *__restrict__ W, int64_t nw, float rho,
                                                           float beta, int S, double *__restrict__ partials)
{
    __shared__ double sh[4];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    double acc = 0.0;
    for (int64_t e = t0; e < nr; e += stride) acc += (double)r[e] * r[e];
    const int mm = g.m * g.m;
    const int64_t nx_ = (int64_t)S * g.np * mm;
    for (int64_t e = t0; e < nx_; e += stride) {
        const int64_t sp = e / mm;
        const int l = (int)(e - sp * mm);
        const int s = (int)(sp / g.np), p = (int)(sp - (int64_t)s * g.np);
        const int a = p / g.ncx, b = p - a * g.ncx;
        const int iy = g.cy[a] + l / g.m, ix = g.cx[b] + l % g.m;
        const double d = (double)x[((int64_t)s * g.ny + iy) * g.nx + ix] - (double)X[e];
        acc += rho * d * d;
    }
    for (int64_t e = t0; e < nw; e += stride) acc += beta * fabs((double)W[e]);
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) sh[w] = acc;
    __syncthreads();
    if (threadIdx.x == 0) partials[blockIdx.x] = ((sh[0] + sh[1]) + sh[2]) + sh[3];
}

__global__ void patch_final_kernel(const double *__restrict__ partials, int n, float *out)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double t = 0.0;
        for (int i = 0; i < n; ++i) t += partials[i];
        *out = (float)t;
    }
}

// <a, b> and <a, a> partial sums for the power iteration
__global__ __launch_bounds__(256) void dot2_kernel(const float *__restrict__ a, const float *__restrict__ b, int64_t n,
                                                   double *__restrict__ partials)
{
    __shared__ double sh[2][4];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    double ab = 0.0, aa = 0.0;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += stride) {
        ab += (double)a[e] * b[e];
        aa += (double)a[e] * a[e];
    }
    for (int off = 32; off > 0; off >>= 1) {
        ab += __shfl_xor(ab, off, 64);
        aa += __shfl_xor(aa, off, 64);
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) {
        sh[0][w] = ab;
        sh[1][w] = aa;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = ((sh[0][0] + sh[0][1]) + sh[0][2]) + sh[0][3];
        partials[2 * blockIdx.x + 1] = ((sh[1][0] + sh[1][1]) + sh[1][2]) + sh[1][3];
    }
}

// v <- hv / |hv| with |hv| from the partials; lam_out = <hv, v_old> (v_old unit)
__global__ void power_norm_kernel(const double *__restrict__ partials, int nblk, double *__restrict__ res)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double ab = 0.0, aa = 0.0;
        for (int i = 0; i < nblk; ++i) {
            ab += partials[2 * i];
            aa += partials[2 * i + 1];
        }
        res[0] = ab;
        res[1] = aa;
    }
}

__global__ void scale_by_norm_kernel(float *__restrict__ dst, const float *__restrict__ src, int64_t n,
                                     const double *__restrict__ res)
{
    const float inv = (float)(1.0 / sqrt(res[1]));
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        dst[e] = src[e] * inv;
}

unsigned grid_n(int64_t n)
{
    int64_t b = (n + 255) / 256;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(b, 8192));
}

typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

// C[M][N] = alpha * A[M][K] B[K][N] on the matrix cores, N = 32 NB, K a multiple of 32.  Workgroup =
// 128 rows (a wavefront per 32 rows, all N columns: NB accumulator blocks of 32 x 32).  K runs in
// chunks of 32 staged in LDS; A rows padded to 34 floats and B rows to a stride of 32 mod 64 floats
// keep the fragment reads of both lane halves on distinct banks.  Lane layout of the instruction:
// lane l holds A[l % 32][l / 32] and B[l / 32][l % 32]; accumulator register i holds
// C[8 (i / 4) + 4 (l / 32) + i % 4][l % 32].
template <int NB>
__global__ __launch_bounds__(256) void mfma_sgemm_kernel(const float *__restrict__ A, const float *__restrict__ B,
                                                         float *__restrict__ C, int64_t M, int K, float alpha)
{
    constexpr int N = 32 * NB, LDA = 34, LDB = N + ((96 - N % 64) % 64);
    __shared__ float sA[128 * LDA];
    __shared__ float sB[32 * LDB];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int64_t m0 = (int64_t)blockIdx.x * 128;
    f32x16 acc[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int i = 0; i < 16; ++i) acc[nb][i] = 0.0f;
    for (int k0 = 0; k0 < K; k0 += 32) {
        // A chunk: 128 rows x 32 floats, 8 threads per row (16 B each)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = tid + 256 * q, r = e >> 3, c = (e & 7) * 4;
            float4 v = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            if (m0 + r < M) v = *(const float4 *)(A + (m0 + r) * K + k0 + c);
            float *d = sA + r * LDA + c;
            d[0] = v.x; d[1] = v.y; d[2] = v.z; d[3] = v.w;
        }
        // B chunk: 32 rows x N floats
        for (int e = tid; e < 8 * N; e += 256) {
            const int r = e / (N / 4), c = (e % (N / 4)) * 4;
            const float4 v = *(const float4 *)(B + (int64_t)(k0 + r) * N + c);
            float *d = sB + r * LDB + c;
            d[0] = v.x; d[1] = v.y; d[2] = v.z; d[3] = v.w;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < 32; kk += 2) {
            const float a = sA[(wv * 32 + (lane & 31)) * LDA + kk + (lane >> 5)];
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                const float b = sB[(kk + (lane >> 5)) * LDB + nb * 32 + (lane & 31)];
                acc[nb] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc[nb], 0, 0, 0);
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int64_t m = m0 + wv * 32 + 8 * (i >> 2) + 4 * (lane >> 5) + (i & 3);
            if (m < M) C[m * N + nb * 32 + (lane & 31)] = alpha * acc[nb][i];
        }
}

hipError_t sgemm(const float *A, const float *B, float *C, int64_t M, int N, int K, float alpha, hipStream_t st)
{
    // the matrix-core kernel reads A and B with 16-byte loads: rows of K and N floats from 16-byte
    // aligned bases
    const bool aligned = (((uintptr_t)A | (uintptr_t)B) & 15) == 0;
    if (aligned && K % 32 == 0 && N % 32 == 0 && N <= 128 && M > 0) {
        const unsigned grid = (unsigned)((M + 127) / 128);
        switch (N / 32) {
        case 1: mfma_sgemm_kernel<1><<<grid, 256, 0, st>>>(A, B, C, M, K, alpha); break;
        case 2: mfma_sgemm_kernel<2><<<grid, 256, 0, st>>>(A, B, C, M, K, alpha); break;
        case 3: mfma_sgemm_kernel<3><<<grid, 256, 0, st>>>(A, B, C, M, K, alpha); break;
        default: mfma_sgemm_kernel<4><<<grid, 256, 0, st>>>(A, B, C, M, K, alpha); break;
        }
        return hipGetLastError();
    }
    dim3 grid((unsigned)((M + GT - 1) / GT), (unsigned)((N + GT - 1) / GT));
    sgemm_kernel<<<grid, 256, 0, st>>>(A, B, C, (int)M, N, K, alpha);
    return hipGetLastError();
}

// Per-axis patch tables on the device (so that a call enqueues them instead of copying host
// memory): corners c_a = min(a stride, n - m) for a < nc; for every pixel i the core corner
// (the nearest centre c_a + (m - 1)/2, lowest index on ties) and the first / last corner whose
// patch covers i.  One thread per pixel; ties and distances in exact integer arithmetic
// (|2 i - 2 c_a - (m - 1)| orders the centre distances).
__global__ void axis_tables_kernel(int n, int m, int stride, int nc, int *__restrict__ corner, int *__restrict__ core,
                                   int *__restrict__ first, int *__restrict__ last)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nc) corner[i] = min(i * stride, n - m);
    if (i >= n) return;
    int best = 0x7fffffff, bi = 0, f = -1, l = -1;
    for (int a = 0; a < nc; ++a) {
        const int c = min(a * stride, n - m);
        const int d = abs(2 * (i - c) - (m - 1));
        if (d < best) {
            best = d;
            bi = a;
        }
        if (c <= i && i < c + m) {
            if (f < 0) f = a;
            l = a;
        }
    }
    core[i] = bi;
    first[i] = f;
    last[i] = l;
}

// DT[l][k] = D[k][l]  (D [na][mm])
__global__ void transpose_kernel(const float *__restrict__ D, int na, int mm, float *__restrict__ DT)
{
    const int64_t n = (int64_t)na * mm;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const int k = (int)(e / mm), l = (int)(e - (int64_t)k * mm);
        DT[(int64_t)l * na + k] = D[e];
    }
}

// start vector of the power iteration: a hash of the index mapped to [-0.5, 0.5)
__global__ void seed_kernel(float *__restrict__ z, int64_t n)
{
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        uint32_t h = (uint32_t)e * 0x9e3779b9u + 0x7f4a7c15u;
        h ^= h >> 16;
        h *= 0x21f0aaadu;
        h ^= h >> 15;
        h *= 0x735a2d97u;
        h ^= h >> 15;
        z[e] = (float)((h >> 8) * (1.0 / 16777216.0) - 0.5);
    }
}

int n_corners(int n, int m, int stride) { return (n - m) / stride + 1 + ((n - m) % stride ? 1 : 0); }

struct PatchLayout {
    size_t tables, X, x, r, R, G, grad, Z, dt, partials, res, total;
};

}  // namespace
}  // namespace pyhst

using namespace pyhst;

namespace pyhst {
namespace {

// Everything one patch call needs: sizes, the work layout, the device tables and the gradient of
// eq. (9).  Construction only checks arguments and computes the layout.
struct PatchCall {
    const pyhst_plan &p;
    pyhst_patch_args &a;
    int rc = PYHST_OK;
    int S = 0, ny = 0, nx = 0, m = 0, na = 0, ncy = 0, ncx = 0, np = 0, mm = 0;
    int64_t ni = 0, nw = 0, nX = 0, ns = 0;
    static constexpr int nblk = 1024;
    PatchLayout L{};
    PatchGeo g{};
    float *X = nullptr, *x = nullptr, *r = nullptr, *R = nullptr, *G = nullptr, *grad = nullptr, *Z = nullptr,
          *DT = nullptr;
    double *partials = nullptr, *res = nullptr;
    float s2 = 1.0f;

    PatchCall(const pyhst_plan &plan, pyhst_patch_args &args, const char *who) : p(plan), a(args)
    {
        if (!p.uniform) {
            rc = fail(PYHST_EARG, std::string(who) + ": needs a uniform plan");
            return;
        }
        const GeoDev &geo = p.gd[0];
        S = p.n_slices;
        ny = geo.ny;
        nx = geo.nx;
        m = a.m;
        na = a.n_atoms;
        const int st_ = a.stride;
        if (m < 1 || m > ny || m > nx || st_ < 1 || st_ > m || na < 1 || a.n_iter < 0 || !(a.rho >= 0.0f) ||
            !(a.beta >= 0.0f)) {
            rc = fail(PYHST_EARG, std::string(who) + ": bad patch size, stride, atoms, iterations, rho or beta");
            return;
        }
        ncy = n_corners(ny, m, st_);
        ncx = n_corners(nx, m, st_);
        np = ncy * ncx;
        mm = m * m;
        ni = (int64_t)S * ny * nx;
        nw = (int64_t)S * np * na;
        nX = (int64_t)S * np * mm;
        ns = a.identity ? ni : (int64_t)p.sino_elems;
        s2 = (float)(geo.s * geo.s);
        size_t o = 0;
        auto take = [&](size_t bytes) {
            size_t r0 = o;
            o = (o + bytes + 255) & ~(size_t)255;
            return r0;
        };
        L.tables = take((size_t)4 * (ncy + ncx + 3 * (size_t)(ny + nx)));
        L.X = take((size_t)nX * 4);
        L.x = take((size_t)ni * 4);
        L.r = take((size_t)ns * 4);
        L.R = take((size_t)ni * 4);
        L.G = take((size_t)nX * 4);
        L.grad = take((size_t)nw * 4);
        L.Z = take((size_t)nw * 4);
        L.dt = take((size_t)na * mm * 4);
        L.partials = take(sizeof(double) * 2 * nblk);
        L.res = take(sizeof(double) * 2);
        L.total = o;
    }

    // bind the work buffer and enqueue the tables and D^T
    int bind(hipStream_t st, const char *who)
    {
        if (!a.dict) return fail(PYHST_EARG, std::string(who) + ": NULL dict");
        if (!a.work || a.work_bytes < L.total) {
            set_error(std::string(who) + ": work buffer too small");
            return PYHST_ENOMEM;
        }
        unsigned char *w = (unsigned char *)a.work;
        int *t = (int *)(w + L.tables);
        int *cy = t, *cx = cy + ncy, *core_y = cx + ncx, *core_x = core_y + ny, *first_y = core_x + nx,
            *last_y = first_y + ny, *first_x = last_y + ny, *last_x = first_x + nx;
        axis_tables_kernel<<<(ny + 255) / 256, 256, 0, st>>>(ny, m, a.stride, ncy, cy, core_y, first_y, last_y);
        axis_tables_kernel<<<(nx + 255) / 256, 256, 0, st>>>(nx, m, a.stride, ncx, cx, core_x, first_x, last_x);
        DT = (float *)(w + L.dt);
        transpose_kernel<<<grid_n((int64_t)na * mm), 256, 0, st>>>(a.dict, na, mm, DT);
        g = PatchGeo{cy, cx, core_y, core_x, first_y, last_y, first_x, last_x, ny, nx, m, ncy, ncx, np};
        X = (float *)(w + L.X);
        x = (float *)(w + L.x);
        r = (float *)(w + L.r);
        R = (float *)(w + L.R);
        G = (float *)(w + L.G);
        grad = (float *)(w + L.grad);
        Z = (float *)(w + L.Z);
        partials = (double *)(w + L.partials);
        res = (double *)(w + L.res);
        hipError_t e = hipGetLastError();
        return e == hipSuccess ? PYHST_OK : hip_fail(e, who);
    }

    // gradient of eq. (9) at coefficients C into grad (data term dropped when with_y is false)
    hipError_t gradient(const float *C, bool with_y, hipStream_t st)
    {
        hipError_t er = sgemm(C, a.dict, X, (int64_t)S * np, mm, na, 1.0f, st);
        if (er != hipSuccess) return er;
        assemble_kernel<<<grid_n(ni), 256, 0, st>>>(g, X, x, S);
        if (a.identity) {
            diff_kernel<<<grid_n(ni), 256, 0, st>>>(x, with_y ? a.y : nullptr, R, ni);
        } else {
            if (with_y) {
                CpDual rd{r, a.y, 0.0f, 1};
                er = launch_forward(p, x, nullptr, 1.0f, &rd, st);
            } else {
                er = launch_forward(p, x, r, 1.0f, nullptr, st);
            }
            if (er == hipSuccess) er = launch_backproject(p, r, 0, R, s2, 0.0f, nullptr, st);
            if (er != hipSuccess) return er;
        }
        similarity_kernel<<<grid_n(ni), 256, 0, st>>>(g, X, x, R, a.rho, S);
        patch_grad_kernel<<<grid_n(nX), 256, 0, st>>>(g, X, x, R, a.rho, G, S);
        return sgemm(G, DT, grad, (int64_t)S * np, na, mm, 2.0f, st);
    }
};

}  // namespace
}  // namespace pyhst

using namespace pyhst;

extern "C" int pyhst_patch_fista(const pyhst_plan *pc, pyhst_patch_args *a, hipStream_t st)
{
    if (!pc || !a) return fail(PYHST_EARG, "patch_fista: NULL argument");
    PatchCall c(*pc, *a, "patch_fista");
    if (c.rc) return c.rc;
    if (!a->w) {
        a->work_bytes = c.L.total;
        a->n_patches = c.np;
        return PYHST_OK;
    }
    if (!a->y || !a->out) return fail(PYHST_EARG, "patch_fista: NULL y or out");
    if (!(a->lipschitz > 0.0) || !std::isfinite(a->lipschitz))
        return fail(PYHST_EARG, "patch_fista: lipschitz must be > 0 (see pyhst_patch_lipschitz)");
    int rc = c.bind(st, "patch_fista");
    if (rc) return rc;
    const double Lf = a->lipschitz;
    float *W = a->w;
    hipError_t e = launch_fill(W, c.nw, 0.0f, st);
    if (e == hipSuccess) e = launch_fill(c.Z, c.nw, 0.0f, st);
    if (e != hipSuccess) return hip_fail(e, "patch_fista: clear");
    double t = 1.0;
    for (int it = 0; it < a->n_iter; ++it) {
        e = c.gradient(c.Z, true, st);
        if (e != hipSuccess) return hip_fail(e, "patch_fista: gradient");
        double tn = 0.5 * (1.0 + std::sqrt(1.0 + 4.0 * t * t));
        const float mom = (float)((t - 1.0) / tn);
        shrink_kernel<<<grid_n(c.nw), 256, 0, st>>>(c.grad, c.Z, W, c.nw, (float)(1.0 / Lf), (float)(a->beta / Lf),
                                                     mom, a->fast);
        t = tn;
        if (a->energy) {
            e = sgemm(W, a->dict, c.X, (int64_t)c.S * c.np, c.mm, c.na, 1.0f, st);
            if (e != hipSuccess) return hip_fail(e, "patch_fista: energy");
            assemble_kernel<<<grid_n(c.ni), 256, 0, st>>>(c.g, c.X, c.x, c.S);
            if (a->identity) {
                diff_kernel<<<grid_n(c.ni), 256, 0, st>>>(c.x, a->y, c.r, c.ni);
            } else {
                CpDual rd{c.r, a->y, 0.0f, 1};
                e = launch_forward(*pc, c.x, nullptr, 1.0f, &rd, st);
                if (e != hipSuccess) return hip_fail(e, "patch_fista: energy");
            }
            patch_energy_kernel<<<c.nblk, 256, 0, st>>>(c.g, c.r, c.ns, c.X, c.x, W, c.nw, a->rho, a->beta, c.S,
                                                         c.partials);
            patch_final_kernel<<<1, 64, 0, st>>>(c.partials, c.nblk, a->energy + it);
        }
    }
    // final image from the final coefficients
    e = sgemm(W, a->dict, c.X, (int64_t)c.S * c.np, c.mm, c.na, 1.0f, st);
    if (e != hipSuccess) return hip_fail(e, "patch_fista: image");
    assemble_kernel<<<grid_n(c.ni), 256, 0, st>>>(c.g, c.X, a->out, c.S);
    e = hipGetLastError();
    return e == hipSuccess ? PYHST_OK : hip_fail(e, "patch_fista: image");
}

extern "C" int pyhst_patch_lipschitz(const pyhst_plan *pc, pyhst_patch_args *a, hipStream_t st)
{
    if (!pc || !a) return fail(PYHST_EARG, "patch_lipschitz: NULL argument");
    PatchCall c(*pc, *a, "patch_lipschitz");
    if (c.rc) return c.rc;
    int rc = c.bind(st, "patch_lipschitz");
    if (rc) return rc;
    // power iteration on the (linear) gradient map with y = 0; Z holds the iterate
    seed_kernel<<<grid_n(c.nw), 256, 0, st>>>(c.Z, c.nw);
    hipError_t e = hipGetLastError();
    for (int it = 0; it < 60 && e == hipSuccess; ++it) {
        dot2_kernel<<<c.nblk, 256, 0, st>>>(c.Z, c.Z, c.nw, c.partials);
        power_norm_kernel<<<1, 64, 0, st>>>(c.partials, c.nblk, c.res);
        scale_by_norm_kernel<<<grid_n(c.nw), 256, 0, st>>>(c.Z, c.Z, c.nw, c.res);
        e = c.gradient(c.Z, false, st);
        if (e != hipSuccess) break;
        dot2_kernel<<<c.nblk, 256, 0, st>>>(c.grad, c.Z, c.nw, c.partials);
        power_norm_kernel<<<1, 64, 0, st>>>(c.partials, c.nblk, c.res);
        e = hipMemcpyAsync(c.Z, c.grad, (size_t)c.nw * 4, hipMemcpyDeviceToDevice, st);
    }
    double hr[2] = {0.0, 0.0};
    if (e == hipSuccess) e = hipMemcpyAsync(hr, c.res, sizeof(hr), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "patch_lipschitz");
    if (!(hr[0] > 0.0) || !std::isfinite(hr[0])) return fail(PYHST_ENUM, "patch_lipschitz: estimate failed");
    a->lipschitz = 1.02 * hr[0];
    a->n_patches = c.np;
    return PYHST_OK;
}
