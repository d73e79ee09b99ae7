// Dark/flat normalisation with -log (section 2.3) and the ramp filter of FBP.
//
// The filter is a linear convolution with the Ram-Lak kernel on [0, L), done
// as a zero-padded FFT of length P >= 2L - 1 in LDS (the circular result then
// equals the linear one on [0, L)).  The kernel is real and even, so its
// spectrum is real and two real rows share one complex FFT (row a in the real
// part, row b in the imaginary part).  Forward: decimation in frequency,
// natural in, bit-reversed out; the spectrum is stored bit-reversed with 1/P
// folded in; inverse: decimation in time, bit-reversed in, natural out.  Two
// radix-2 stages are fused per LDS pass (radix-4 data movement).
//
// For raw input the normalisation is fused into the load: uint16 radiograph
// rows are read in acquisition order [K][R][nb] and the filtered rows are
// written in sinogram order [R][K][L], so the -log sinogram never goes to HBM.
#include "internal.hpp"

namespace pyhst {

struct FlatInfo {
    double pos[32];
    int n;
};

namespace {

__device__ inline float2 operator+(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ inline float2 operator-(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ inline float2 cmul(float2 a, float2 w) { return make_float2(a.x * w.x - a.y * w.y, a.x * w.y + a.y * w.x); }
__device__ inline float2 cmulc(float2 a, float2 w) { return make_float2(a.x * w.x + a.y * w.y, a.y * w.x - a.x * w.y); }

__device__ inline void flat_interp(const FlatInfo &fi, int k, int &i0, int &i1, float &a)
{
    i0 = i1 = 0;
    double al = 0.0;
    if (fi.n > 1) {
        if (k <= fi.pos[0]) {
            i0 = i1 = 0;
        } else if (k >= fi.pos[fi.n - 1]) {
            i0 = i1 = fi.n - 1;
        } else {
            int i = 0;
            while (i + 1 < fi.n && !(k < fi.pos[i + 1])) ++i;
            i0 = i;
            i1 = i + 1;
            al = ((double)k - fi.pos[i0]) / (fi.pos[i1] - fi.pos[i0]);
        }
    }
    a = (float)al;
}

__device__ inline float norm_value(float I, float d, float f0, float f1, float a, float eps)
{
    const float f = (1.0f - a) * f0 + a * f1;
    const float den = f - d;
    if (!(den > 0.0f)) return 0.0f;
    float ratio = (I - d) / den;
    if (!(ratio >= eps)) ratio = eps;
    return -logf(ratio);
}

__global__ __launch_bounds__(256) void normalize_kernel(const uint16_t *__restrict__ raw,
                                                        const float *__restrict__ flats, FlatInfo fi,
                                                        const float *__restrict__ dark, float eps, int K, int R,
                                                        int nb, float *__restrict__ out)
{
    const int row = blockIdx.x;          // raw row order: k * R + r
    const int k = row / R, r = row - k * R;
    int i0, i1;
    float a;
    flat_interp(fi, k, i0, i1, a);
    const uint16_t *src = raw + (int64_t)row * nb;
    const float *f0 = flats + ((int64_t)i0 * R + r) * nb;
    const float *f1 = flats + ((int64_t)i1 * R + r) * nb;
    const float *dk = dark + (int64_t)r * nb;
    float *dst = out + ((int64_t)r * K + k) * nb;
    for (int j = threadIdx.x; j < nb; j += blockDim.x)
        dst[j] = norm_value((float)src[j], dk[j], f0[j], f1[j], a, eps);
}

// Hot-spot removal on the flat-field-corrected transmission (section 2.3): a pixel whose 3x3
// neighbours' median (up to 8 neighbours of the same radiograph, mean of the middle two for an
// even count) is below it by more than thr takes that median; then -log as above.  One thread per
// pixel; the 9 transmissions are recomputed per thread (neighbours come from L1/L2).  The input
// rows are R_in = h0 + R + (halo after): output row r reads input row h0 + r, and the halo rows
// serve only as neighbours, so a volume reconstructed in chunks of rows gives the same result as
// in one piece.
__device__ inline float transmission(const uint16_t *raw, const float *f0, const float *f1, const float *dk, float a,
                                     int64_t o, bool &dead)
{
    const float d = dk[o];
    const float den = ((1.0f - a) * f0[o] + a * f1[o]) - d;
    dead = !(den > 0.0f);
    return dead ? 1.0f : ((float)raw[o] - d) / den;
}

__device__ inline void cswap(float &a, float &b)
{
    const float lo = fminf(a, b), hi = fmaxf(a, b);
    a = lo;
    b = hi;
}

__global__ __launch_bounds__(256) void normalize_hotspot_kernel(const uint16_t *__restrict__ raw,
                                                                const float *__restrict__ flats, FlatInfo fi,
                                                                const float *__restrict__ dark, float eps, float thr,
                                                                int K, int R, int R_in, int h0, int nb,
                                                                float *__restrict__ out)
{
    const int row = blockIdx.x;          // output row order: k * R + r
    const int k = row / R, r = row - k * R;
    const int ri = r + h0;               // its input row
    int i0, i1;
    float a;
    flat_interp(fi, k, i0, i1, a);
    const uint16_t *img = raw + (int64_t)k * R_in * nb;      // radiograph k, [R_in][nb]
    const float *f0 = flats + (int64_t)i0 * R_in * nb, *f1 = flats + (int64_t)i1 * R_in * nb;
    float *dst = out + ((int64_t)r * K + k) * nb;
    for (int j = threadIdx.x; j < nb; j += blockDim.x) {
        bool dead;
        float t = transmission(img, f0, f1, dark, a, (int64_t)ri * nb + j, dead);
        if (dead) {
            dst[j] = 0.0f;
            continue;
        }
        float v[8];
        int n = 0;
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            const int dr = q / 3 - 1, dj = q % 3 - 1;
            if (q == 4) continue;
            const int rr = ri + dr, jj = j + dj;
            const bool in = rr >= 0 && rr < R_in && jj >= 0 && jj < nb;
            bool dd;
            const float tv = in ? transmission(img, f0, f1, dark, a, (int64_t)rr * nb + jj, dd) : INFINITY;
            v[q < 4 ? q : q - 1] = tv;
            n += in ? 1 : 0;
        }
        // sorting network for 8 values (absent neighbours are +inf and sort last)
        cswap(v[0], v[1]); cswap(v[2], v[3]); cswap(v[4], v[5]); cswap(v[6], v[7]);
        cswap(v[0], v[2]); cswap(v[1], v[3]); cswap(v[4], v[6]); cswap(v[5], v[7]);
        cswap(v[1], v[2]); cswap(v[5], v[6]); cswap(v[0], v[4]); cswap(v[3], v[7]);
        cswap(v[1], v[5]); cswap(v[2], v[6]);
        cswap(v[1], v[4]); cswap(v[3], v[6]);
        cswap(v[2], v[4]); cswap(v[3], v[5]);
        cswap(v[3], v[4]);
        float lo = v[0], hi = v[0];
#pragma unroll
        for (int q = 1; q < 8; ++q) {
            if (q == (n - 1) / 2) lo = v[q];
            if (q == n / 2) hi = v[q];
        }
        if (n > 0) {
            const float med = (n & 1) ? hi : 0.5f * (lo + hi);
            if (t - med > thr) t = med;
        }
        if (!(t >= eps)) t = eps;
        dst[j] = -logf(t);
    }
}

// Ring filter (section 2.3).  m[s][j] = mean_k (p - obj)[s][k][j] (FP64); one thread per bin.
__global__ __launch_bounds__(256) void ring_mean_kernel(const float *__restrict__ p, const float *__restrict__ obj,
                                                        int K, int L, double *__restrict__ m)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x, s = blockIdx.y;
    if (j >= L) return;
    const int64_t base = (int64_t)s * K * L + j;
    double acc = 0.0;
    for (int k = 0; k < K; ++k) acc += (double)p[base + (int64_t)k * L] - (obj ? (double)obj[base + (int64_t)k * L] : 0.0);
    m[(int64_t)s * L + j] = acc / K;
}

// hp[s][j] = m[j] - mean of m over the bins j-w..j+w that exist
__global__ __launch_bounds__(256) void ring_highpass_kernel(const double *__restrict__ m, int L, int w,
                                                            double *__restrict__ hp)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x, s = blockIdx.y;
    if (j >= L) return;
    const double *ms = m + (int64_t)s * L;
    const int lo = max(0, j - w), hi = min(L - 1, j + w);
    double acc = 0.0;
    for (int i = lo; i <= hi; ++i) acc += ms[i];
    hp[(int64_t)s * L + j] = ms[j] - acc / (hi - lo + 1);
}

// p[s][k][j] -= hp[s][j]
__global__ __launch_bounds__(256) void ring_subtract_kernel(float *__restrict__ p, const double *__restrict__ hp,
                                                            int K, int L)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x, k = blockIdx.y, s = blockIdx.z;
    if (j >= L) return;
    p[((int64_t)s * K + k) * L + j] -= (float)hp[(int64_t)s * L + j];
}

__device__ inline float2 times_mi(float2 a) { return make_float2(a.y, -a.x); }   // a * (-i)

// One table load per radix-4 butterfly: of its three twiddles w^i, w^(i + h/2), w^(2i) (w a root of
// unity of order 2h), the second is the first times -i exactly and the third is its square.
__device__ void fft_forward(float2 *z, int P, int lg, const float2 *__restrict__ tw, int lgmax)
{
    int h = P >> 1, lh = lg - 1;
    while (h >= 2) {
        const int h2 = h >> 1;
        for (int t = threadIdx.x; t < (P >> 2); t += blockDim.x) {
            const int gq = t >> (lh - 1), i = t & (h2 - 1);
            const int b0 = (gq << (lh + 1)) + i;
            const float2 e0 = z[b0], e1 = z[b0 + h2], e2 = z[b0 + h], e3 = z[b0 + h + h2];
            const float2 w0 = tw[i << (lgmax - lh - 1)];
            const float2 w1 = times_mi(w0);
            const float2 w2 = cmul(w0, w0);
            const float2 s0 = e0 + e2, d0 = cmul(e0 - e2, w0);
            const float2 s1 = e1 + e3, d1 = cmul(e1 - e3, w1);
            z[b0] = s0 + s1;
            z[b0 + h2] = cmul(s0 - s1, w2);
            z[b0 + h] = d0 + d1;
            z[b0 + h + h2] = cmul(d0 - d1, w2);
        }
        __syncthreads();
        h >>= 2;
        lh -= 2;
    }
    if (h == 1) {
        for (int t = threadIdx.x; t < (P >> 1); t += blockDim.x) {
            const float2 a = z[2 * t], b = z[2 * t + 1];
            z[2 * t] = a + b;
            z[2 * t + 1] = a - b;
        }
        __syncthreads();
    }
}

__device__ void fft_inverse(float2 *z, int P, int lg, const float2 *__restrict__ tw, int lgmax)
{
    int h = 1, lh = 0;
    if (lg & 1) {
        for (int t = threadIdx.x; t < (P >> 1); t += blockDim.x) {
            const float2 a = z[2 * t], b = z[2 * t + 1];
            z[2 * t] = a + b;
            z[2 * t + 1] = a - b;
        }
        __syncthreads();
        h = 2;
        lh = 1;
    }
    while (h < P) {
        for (int t = threadIdx.x; t < (P >> 2); t += blockDim.x) {
            const int gq = t >> lh, i = t & (h - 1);
            const int b0 = (gq << (lh + 2)) + i;
            const float2 e0 = z[b0], e1 = z[b0 + h], e2 = z[b0 + 2 * h], e3 = z[b0 + 3 * h];
            const float2 u = tw[i << (lgmax - lh - 2)];   // u^i of order 4h: w = u^2, u^(i + h) = -i u^i
            const float2 w = cmul(u, u);
            const float2 b1 = cmulc(e1, w), b3 = cmulc(e3, w);
            const float2 s0 = e0 + b1, d0 = e0 - b1, s1 = e2 + b3, d1 = e2 - b3;
            const float2 t1 = cmulc(s1, u);
            const float2 t2 = cmulc(d1, times_mi(u));
            z[b0] = s0 + t1;
            z[b0 + 2 * h] = s0 - t1;
            z[b0 + h] = d0 + t2;
            z[b0 + 3 * h] = d0 - t2;
        }
        __syncthreads();
        h <<= 2;
        lh += 2;
    }
}

template <bool RAW>
__global__ __launch_bounds__(256) void filter_kernel(Tables T, const float *__restrict__ sino,
                                                     const uint16_t *__restrict__ raw,
                                                     const float *__restrict__ flats, FlatInfo fi,
                                                     const float *__restrict__ dark, float eps, int R,
                                                     float *__restrict__ out)
{
    extern __shared__ float2 z[];
    const int2 pr = T.pairs[blockIdx.x];
    const SliceDev sd = T.slc[pr.x];
    const GeoDev &g = T.geo[sd.g];
    const int K = g.K, nb = g.nb, Lf = g.Lf, pad = g.fpad, P = g.P, lg = g.log2P;
    const int ka = pr.y, kb = pr.y + 1;
    const bool hasb = kb < K;
    const float *hw = T.haw + g.hw_off;

    int a0 = 0, a1 = 0, b0 = 0, b1 = 0;
    float aa = 0.0f, ab = 0.0f;
    if (RAW) {
        flat_interp(fi, ka, a0, a1, aa);
        flat_interp(fi, hasb ? kb : ka, b0, b1, ab);
    }
    const int r = pr.x;   // raw input: uniform plan, slice index = detector row
    const bool half = g.half != 0;
    const bool same_flats = a0 == b0 && a1 == b1;   // both rows between the same two flats (uniform)
    for (int n = threadIdx.x; n < P; n += blockDim.x) {
        float va = 0.0f, vb = 0.0f;
        const int jj = n - pad;
        if (n < Lf && jj >= 0 && jj < nb) {
            const float w = half ? hw[n] : 1.0f;
            if (RAW) {
                const float d = dark[(int64_t)r * nb + jj];
                const float Ia = (float)raw[((int64_t)ka * R + r) * nb + jj];
                const float fa0 = flats[((int64_t)a0 * R + r) * nb + jj], fa1 = flats[((int64_t)a1 * R + r) * nb + jj];
                va = norm_value(Ia, d, fa0, fa1, aa, eps);
                if (hasb) {
                    const float Ib = (float)raw[((int64_t)kb * R + r) * nb + jj];
                    const float fb0 = same_flats ? fa0 : flats[((int64_t)b0 * R + r) * nb + jj];
                    const float fb1 = same_flats ? fa1 : flats[((int64_t)b1 * R + r) * nb + jj];
                    vb = norm_value(Ib, d, fb0, fb1, ab, eps);
                }
            } else {
                va = sino[sd.sino_off + (int64_t)ka * nb + jj];
                vb = hasb ? sino[sd.sino_off + (int64_t)kb * nb + jj] : 0.0f;
            }
            va *= w;
            vb *= w;
        }
        z[n] = make_float2(va, vb);
    }
    __syncthreads();
    fft_forward(z, P, lg, T.twid, T.log2Pmax);
    const float *H = T.spec + g.spec_off;
    for (int n = threadIdx.x; n < P; n += blockDim.x) {
        const float h = H[n];
        const float2 v = z[n];
        z[n] = make_float2(v.x * h, v.y * h);
    }
    __syncthreads();
    fft_inverse(z, P, lg, T.twid, T.log2Pmax);
    const float wa = T.wang[g.ang_off + ka];
    const float wb = hasb ? T.wang[g.ang_off + kb] : 0.0f;
    float *oa = out + sd.filt_off + (int64_t)ka * Lf;
    for (int n = threadIdx.x; n < Lf; n += blockDim.x) {
        const float2 v = z[n];
        oa[n] = wa * v.x;
        if (hasb) oa[Lf + n] = wb * v.y;
    }
}

// P = 4096 = 16^3 (2048-bin rows): the same filter with the FFT in registers.  Each of the 256 threads
// holds 16 points and every pass is a 16-point DFT in registers (two radix-4 stages with constant
// twiddles) followed by one twiddle multiply; the three passes of each direction exchange data
// through LDS twice (instead of six radix-4 passes through LDS).  The twiddles are products of
// eight values of the plan's table (half circle) per thread, loaded once: the kernel is bound by
// the latency of its global loads, not by arithmetic.
//   forward, thread a:        x[a + 256 m] over m -> Y1[a][k1] = w^(a k1) DFT16_m(..)[k1]
//   forward, thread (k1, c):  Y1[c + 16 d][k1] over d -> Y2[k1][c][b1] = w^(16 c b1) DFT16_d(..)[b1]
//   forward, thread (k1, b1): Y2[k1][c][b1] over c -> X[k1 + 16 b1 + 256 b2] = DFT16_c(..)[b2]
// with w = exp(-2 pi i / 4096); the inverse runs the same passes backwards with conjugate twiddles.
// LDS: Y1 at k1 * 256 + a, Y2 at k1 * 272 + b1 * 17 + c (the pad spreads the stride-17 reads over
// the banks).  Inside a 16-point DFT, input m sits at register m and output k at register
// rev4(k) = (k >> 2) | ((k & 3) << 2).
namespace f16 {

__device__ __forceinline__ float2 mul_mi(float2 a) { return make_float2(a.y, -a.x); }   // a * (-i)

// 4-point DFT in place, exp(-+2 pi i / 4) per step (INV: inverse, +)
template <bool INV>
__device__ __forceinline__ void dft4(float2 &x0, float2 &x1, float2 &x2, float2 &x3)
{
    const float2 s02 = x0 + x2, d02 = x0 - x2, s13 = x1 + x3, d13 = x1 - x3;
    const float2 r = mul_mi(d13);   // -i (x1 - x3)
    x0 = s02 + s13;
    x2 = s02 - s13;
    x1 = INV ? d02 - r : d02 + r;
    x3 = INV ? d02 + r : d02 - r;
}

constexpr int rev4(int k) { return (k >> 2) | ((k & 3) << 2); }

// 16-point DFT of v[0..15] (input m at register m); output k at register rev4(k)
template <bool INV>
__device__ __forceinline__ void dft16(float2 (&v)[16])
{
    // cos / sin of 2 pi e / 16, e = 0..9
    constexpr float C[10] = {1.0f, 0.92387953251128674f, 0.70710678118654752f, 0.38268343236508977f, 0.0f,
                             -0.38268343236508977f, -0.70710678118654752f, -0.92387953251128674f, -1.0f,
                             -0.92387953251128674f};
    constexpr float S[10] = {0.0f, 0.38268343236508977f, 0.70710678118654752f, 0.92387953251128674f, 1.0f,
                             0.92387953251128674f, 0.70710678118654752f, 0.38268343236508977f, 0.0f,
                             -0.38268343236508977f};
#pragma unroll
    for (int q = 0; q < 4; ++q) dft4<INV>(v[q], v[q + 4], v[q + 8], v[q + 12]);   // over p, m = q + 4 p
    // v[q + 4 r] *= exp(-+2 pi i q r / 16)
#pragma unroll
    for (int q = 1; q < 4; ++q)
#pragma unroll
        for (int r = 1; r < 4; ++r) {
            const float c = C[q * r], sn = INV ? S[q * r] : -S[q * r];
            const float2 a = v[q + 4 * r];
            v[q + 4 * r] = make_float2(a.x * c - a.y * sn, a.x * sn + a.y * c);
        }
#pragma unroll
    for (int r = 0; r < 4; ++r) dft4<INV>(v[4 * r], v[4 * r + 1], v[4 * r + 2], v[4 * r + 3]);   // over q
    // now X[r + 4 s] sits at register 4 r + s = rev4(r + 4 s)
}

// exp(-2 pi i e / 4096) for 0 <= e < 4096 from the table exp(-2 pi i m / Pmax), m < Pmax / 2
__device__ __forceinline__ float2 w4096(const float2 *__restrict__ tw, int e, int sh)
{
    const float2 t = tw[(e & 2047) << sh];
    return (e & 2048) ? make_float2(-t.x, -t.y) : t;
}

__device__ __forceinline__ float2 twiddle(float2 a, float2 w, bool conj)
{
    return conj ? cmulc(a, w) : cmul(a, w);
}

// w^k, 0 <= k < 16, from the bases w, w^2, w^4, w^8 (table values): a product of at most four of
// them, so each twiddle stays within a few FP32 roundings of the table (k is a constant once unrolled)
__device__ __forceinline__ float2 wpow(const float2 (&b)[4], int k)
{
    float2 r = make_float2(1.0f, 0.0f);
    bool first = true;
#pragma unroll
    for (int i = 0; i < 4; ++i)
        if ((k >> i) & 1) {
            r = first ? b[i] : cmul(r, b[i]);
            first = false;
        }
    return r;
}

}  // namespace f16

template <bool RAW>
__global__ __launch_bounds__(256) void filter4096_kernel(Tables T, const float *__restrict__ sino,
                                                         const uint16_t *__restrict__ raw,
                                                         const float *__restrict__ flats, FlatInfo fi,
                                                         const float *__restrict__ dark, float eps, int R,
                                                         float *__restrict__ out)
{
    using namespace f16;
    __shared__ float2 z[16 * 272];
    const int2 pr = T.pairs[blockIdx.x];
    const SliceDev sd = T.slc[pr.x];
    const GeoDev &g = T.geo[sd.g];
    const int K = g.K, nb = g.nb, Lf = g.Lf, pad = g.fpad;
    const int ka = pr.y, kb = pr.y + 1;
    const bool hasb = kb < K;
    const float *hw = T.haw + g.hw_off;
    const float2 *tw = T.twid;
    const int sh = T.log2Pmax - 12;
    const int t = threadIdx.x;

    int a0 = 0, a1 = 0, b0 = 0, b1 = 0;
    float aa = 0.0f, ab = 0.0f;
    if (RAW) {
        flat_interp(fi, ka, a0, a1, aa);
        flat_interp(fi, hasb ? kb : ka, b0, b1, ab);
    }
    const int r = pr.x;   // raw input: uniform plan, slice index = detector row
    const bool half = g.half != 0;
    const bool same_flats = a0 == b0 && a1 == b1;   // both rows between the same two flats (uniform)
    float2 v[16];
#pragma unroll
    for (int m = 0; m < 16; ++m) {
        const int n = t + 256 * m;
        float va = 0.0f, vb = 0.0f;
        const int jj = n - pad;
        if (n < Lf && jj >= 0 && jj < nb) {
            const float w = half ? hw[n] : 1.0f;
            if (RAW) {
                const float d = dark[(int64_t)r * nb + jj];
                const float Ia = (float)raw[((int64_t)ka * R + r) * nb + jj];
                const float fa0 = flats[((int64_t)a0 * R + r) * nb + jj], fa1 = flats[((int64_t)a1 * R + r) * nb + jj];
                va = norm_value(Ia, d, fa0, fa1, aa, eps);
                if (hasb) {
                    const float Ib = (float)raw[((int64_t)kb * R + r) * nb + jj];
                    const float fb0 = same_flats ? fa0 : flats[((int64_t)b0 * R + r) * nb + jj];
                    const float fb1 = same_flats ? fa1 : flats[((int64_t)b1 * R + r) * nb + jj];
                    vb = norm_value(Ib, d, fb0, fb1, ab, eps);
                }
            } else {
                va = sino[sd.sino_off + (int64_t)ka * nb + jj];
                vb = hasb ? sino[sd.sino_off + (int64_t)kb * nb + jj] : 0.0f;
            }
            va *= w;
            vb *= w;
        }
        v[m] = make_float2(va, vb);
    }

    // twiddle bases: w^(t k1) and w^(16 c b1) are products of these (w = exp(-2 pi i / 4096))
    const int hi = t >> 4, lo = t & 15;
    float2 b1w[4], b2w[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        b1w[i] = w4096(tw, t << i, sh);
        b2w[i] = w4096(tw, (16 * lo) << i, sh);
    }
    // forward pass 1 (thread a = t)
    dft16<false>(v);
#pragma unroll
    for (int k1 = 0; k1 < 16; ++k1) z[k1 * 256 + t] = twiddle(v[rev4(k1)], wpow(b1w, k1), false);
    __syncthreads();
    // forward pass 2 (thread (k1, c))
#pragma unroll
    for (int d = 0; d < 16; ++d) v[d] = z[hi * 256 + lo + 16 * d];
    dft16<false>(v);
    __syncthreads();   // every pass-2 read is done before the exchange is overwritten
#pragma unroll
    for (int b = 0; b < 16; ++b) z[hi * 272 + b * 17 + lo] = twiddle(v[rev4(b)], wpow(b2w, b), false);
    __syncthreads();
    // forward pass 3 (thread (k1, b1)), spectrum (bit-reversed table, 1/P folded), inverse pass 3
#pragma unroll
    for (int c = 0; c < 16; ++c) v[c] = z[hi * 272 + lo * 17 + c];
    dft16<false>(v);
    const float *H = T.spec + g.spec_off;
#pragma unroll
    for (int b2 = 0; b2 < 16; ++b2) {
        const int k = hi + 16 * lo + 256 * b2;
        const float h = H[__brev((unsigned)k) >> 20];
        const float2 x = v[rev4(b2)];
        v[rev4(b2)] = make_float2(x.x * h, x.y * h);
    }
    {
        float2 u[16];
#pragma unroll
        for (int b2 = 0; b2 < 16; ++b2) u[b2] = v[rev4(b2)];
        dft16<true>(u);
        __syncthreads();   // every pass-3 read is done
#pragma unroll
        for (int c = 0; c < 16; ++c) z[hi * 272 + lo * 17 + c] = u[rev4(c)];
    }
    __syncthreads();
    // inverse pass 2 (thread (k1, c))
#pragma unroll
    for (int b = 0; b < 16; ++b) v[b] = twiddle(z[hi * 272 + b * 17 + lo], wpow(b2w, b), true);
    dft16<true>(v);
    __syncthreads();
#pragma unroll
    for (int d = 0; d < 16; ++d) z[hi * 256 + lo + 16 * d] = v[rev4(d)];
    __syncthreads();
    // inverse pass 1 (thread a = t)
#pragma unroll
    for (int k1 = 0; k1 < 16; ++k1) v[k1] = twiddle(z[k1 * 256 + t], wpow(b1w, k1), true);
    dft16<true>(v);
    const float wa = T.wang[g.ang_off + ka];
    const float wb = hasb ? T.wang[g.ang_off + kb] : 0.0f;
    float *oa = out + sd.filt_off + (int64_t)ka * Lf;
#pragma unroll
    for (int m = 0; m < 16; ++m) {
        const int n = t + 256 * m;
        if (n < Lf) {
            const float2 x = v[rev4(m)];
            oa[n] = wa * x.x;
            if (hasb) oa[Lf + n] = wb * x.y;
        }
    }
}

FlatInfo make_flats(const double *pos, int n)
{
    FlatInfo fi{};
    fi.n = n;
    for (int i = 0; i < n && i < 32; ++i) fi.pos[i] = pos[i];
    return fi;
}

}  // namespace

hipError_t launch_normalize_hotspot(const pyhst_plan &p, const uint16_t *raw, const float *flats,
                                    const double *flat_pos, int n_flats, const float *dark, float eps, float thr,
                                    int halo_lo, int halo_hi, float *sino, hipStream_t st)
{
    const GeoDev &g = p.gd[0];
    const int R = p.n_slices;
    normalize_hotspot_kernel<<<(unsigned)((int64_t)g.K * R), 256, 0, st>>>(
        raw, flats, make_flats(flat_pos, n_flats), dark, eps, thr, g.K, R, halo_lo + R + halo_hi, halo_lo, g.nb,
        sino);
    return hipGetLastError();
}

hipError_t launch_ring_filter(const pyhst_plan &p, float *sino, const float *obj, int width, double *work,
                              hipStream_t st)
{
    const GeoDev &g = p.gd[0];
    const int S = p.n_slices, K = g.K, L = g.nb;
    double *m = work, *hp = work + (int64_t)S * L;
    dim3 g2((L + 255) / 256, S);
    ring_mean_kernel<<<g2, 256, 0, st>>>(sino, obj, K, L, m);
    ring_highpass_kernel<<<g2, 256, 0, st>>>(m, L, width, hp);
    ring_subtract_kernel<<<dim3((L + 255) / 256, K, S), 256, 0, st>>>(sino, hp, K, L);
    return hipGetLastError();
}

hipError_t launch_normalize(const pyhst_plan &p, const uint16_t *raw, const float *flats, const double *flat_pos,
                            int n_flats, const float *dark, float eps, float *sino, hipStream_t st)
{
    const GeoDev &g = p.gd[0];
    const int R = p.n_slices;
    normalize_kernel<<<(unsigned)((int64_t)g.K * R), 256, 0, st>>>(raw, flats, make_flats(flat_pos, n_flats), dark,
                                                                   eps, g.K, R, g.nb, sino);
    return hipGetLastError();
}

hipError_t launch_filter(const pyhst_plan &p, const float *sino, const uint16_t *raw, const float *flats,
                         const double *flat_pos, int n_flats, const float *dark, float eps, float *filt,
                         hipStream_t st)
{
    int Pmax = 0;
    for (const auto &g : p.gd) Pmax = std::max(Pmax, g.P);
    const size_t lds = (size_t)Pmax * sizeof(float2);
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute((const void *)filter_kernel<true>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e == hipSuccess)
            e = hipFuncSetAttribute((const void *)filter_kernel<false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)lds);
        if (e != hipSuccess) return e;
    }
    bool all4096 = true;
    for (const auto &g : p.gd) all4096 = all4096 && g.P == 4096;
    if (all4096) {
        // 2048-bin rows: the register FFT (the twiddle table covers Pmax >= 4096)
        if (raw) {
            filter4096_kernel<true><<<(unsigned)p.n_pairs, 256, 0, st>>>(p.t, nullptr, raw, flats,
                                                                        make_flats(flat_pos, n_flats), dark, eps,
                                                                        p.n_slices, filt);
        } else {
            FlatInfo none{};
            filter4096_kernel<false><<<(unsigned)p.n_pairs, 256, 0, st>>>(p.t, sino, nullptr, nullptr, none, nullptr,
                                                                         0.0f, p.n_slices, filt);
        }
        return hipGetLastError();
    }
    if (raw) {
        filter_kernel<true><<<(unsigned)p.n_pairs, 256, lds, st>>>(p.t, nullptr, raw, flats,
                                                                   make_flats(flat_pos, n_flats), dark, eps,
                                                                   p.n_slices, filt);
    } else {
        FlatInfo none{};
        filter_kernel<false><<<(unsigned)p.n_pairs, 256, lds, st>>>(p.t, sino, nullptr, nullptr, none, nullptr, 0.0f,
                                                                    p.n_slices, filt);
    }
    return hipGetLastError();
}

}  // namespace pyhst
