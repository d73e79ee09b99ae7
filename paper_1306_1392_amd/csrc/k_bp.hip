// Pixel-driven backprojection with linear detector interpolation (section 2.3:
// the reconstructed slice is cut into tiles, one workgroup per tile).
//
// gfx950 design.  The paper reads the sinogram through a texture with hardware
// interpolation; here a block of AB projections' detector windows is staged in
// LDS as (q[j], q[j+1] - q[j]) pairs and interpolated in FP32 registers:
//   per update: t = t0 + off (1), i = trunc(t) (1), f = fract(t) (1),
//   LDS address (1), ds_read_b64, acc += q (1), acc = fma(f, dq, acc) (1).
// Coordinates: per (tile, projection) the tile-origin coordinate is computed in
// FP64 and split into an integer window base and an FP32 remainder, so every
// FP32 coordinate stays below ~100 bins (ulp < 8e-6 bin).  Lanes of a wave own
// one 8x8 pixel block per register slot, so one ds_read_b64 of a wave touches
// at most ~13 consecutive window entries (no bank conflicts).  The per-block
// coordinate offsets are wave-uniform and come from a scalar table (the
// pipelined loop stages them in LDS with each block's other parameters).  The
// bound is the LDS read port: 8 B per update against 128 B/clk/CU for 8-byte
// reads.  On uniform plans of several slices bp2_kernel serves two slices per
// workgroup with 16-byte reads, which the LDS delivers at about twice the rate
// (136 against 78 TB/s measured on the whole chip), and shares the coordinate
// arithmetic between them: 4 VALU lane-ops and 8 LDS bytes per update.
#include "internal.hpp"

namespace pyhst {

namespace {

constexpr int AB = 32;   // projections staged per LDS block

// Window length bound of the pipelined angle loop: the widest window of a tile at pixel size <= 1,
// floor(sqrt((TW-1)^2 + (TH-1)^2)) + 4 rounded up to even (the plan's bp_w for that tile).  Plans
// whose windows are longer (pixels larger than a bin) take the plain loop.
constexpr int pipe_wmax(int c)
{
    int r = 0;
    const int d2 = (tile_w(c) - 1) * (tile_w(c) - 1) + (tile_h(c) - 1) * (tile_h(c) - 1);
    while ((r + 1) * (r + 1) <= d2) ++r;
    return (r + 4) + ((r + 4) & 1);
}
// window elements each thread carries in registers from one block to the next
constexpr int pipe_elems(int c) { return (TILE_AG[c] * AB * pipe_wmax(c) + 256 * TILE_AG[c] - 1) / (256 * TILE_AG[c]); }

// The per-projection table is read through the constant address space so that
// the wave-uniform loads become scalar loads into SGPRs.
typedef __attribute__((address_space(4))) const float cfloat;

// PIPE: the windows of the next block of projections are loaded into registers while the current
// block is summed (two LDS window buffers of wstride entries, three parameter slots, one barrier per
// block), so the L2 / HBM latency of the staging loads overlaps the sums; the parameters of the block
// after that (cos, sin, shift, table entries) are in flight in registers at the same time.  It pays where a launch has
// few workgroups per CU (a single slice in the iterative solvers, after a projector whose sweep of the
// image has evicted the sinogram from every L2): the 32 x 32 tiles; the larger tiles, chosen when there
// are at least four workgroups per CU, keep the plain loop (their accumulators leave few registers).
template <int CFG, int MODE, bool PIPE>
__global__ __launch_bounds__(256 * TILE_AG[CFG]) void bp_kernel(Tables T, const float *__restrict__ sino,
                                                                int filtered, float *__restrict__ img, float alpha,
                                                                float beta, int64_t n_items, int *counter,
                                                                int xcd_remap, CpPrimal cp, int wstride)
{
    constexpr int BX = TILE_BX[CFG], BY = TILE_BY[CFG];
    constexpr int TW = 8 * BX, TH = 32 * BY;
    constexpr int PX = BX * BY;
    constexpr int AG = TILE_AG[CFG];        // angle groups; a staged block holds AG x AB projections
    constexpr int NT = 256 * AG;            // threads per workgroup
    constexpr int ABLK = AG * AB;           // projections per staged block
    constexpr int NSLOT = PIPE ? 3 : 1;
    constexpr int NTAB = 2 + 8 * (BY - 1) + BX;   // table entries a tile reads per projection
    static_assert(!PIPE || ABLK * NTAB <= NT, "one thread per staged table entry of a block");
    extern __shared__ float2 win[];   // [PIPE ? 2 : 1][wstride]: [AG AB][W] per buffer
    __shared__ int s_jb[NSLOT][ABLK];
    __shared__ float s_r[NSLOT][ABLK];
    __shared__ float s_tab[PIPE ? NSLOT : 1][PIPE ? ABLK * NTAB : 1];
    __shared__ int64_t s_item;

    const int tid = threadIdx.x;
    const int lane = tid & 63, wv = (tid >> 6) & 3;
    const int ag = AG > 1 ? tid >> 8 : 0;   // this thread's angle group
    const int lx = lane & 7, ly = lane >> 3;
    const float flx = (float)lx, fly = (float)(ly + 8 * BY * wv);

    for (int64_t round = 0;; ++round) {
        int64_t item;
        if (counter) {   // persistent: take the next item of the cost-sorted list
            if (tid == 0) s_item = atomicAdd(counter, 1);
            __syncthreads();
            item = s_item;
            __syncthreads();
        } else {
            if (round > 0) break;
            // Workgroups are dealt round-robin to the 8 XCDs.  For a uniform batch give each
            // XCD a contiguous range of the work list (whole slices) so a slice's sinogram is
            // fetched into one XCD's L2 rather than into all eight.  (Uneven batches keep the
            // cost-sorted order, which round-robin spreads evenly over the XCDs.)
            item = blockIdx.x;
            if (xcd_remap) {
                const int64_t b = blockIdx.x, q = n_items >> 3, r = n_items & 7;
                const int64_t x = b & 7;
                item = x * q + min(x, r) + (b >> 3);
            }
        }
        if (item >= n_items) break;

        const int2 wi = T.items[CFG][item];
        const SliceDev sd = T.slc[wi.x];
        const GeoDev &g = T.geo[sd.g];
        const int nx = g.nx, ny = g.ny, K = g.K;
        const int L = filtered ? g.Lf : g.nb;
        const double axis = filtered ? g.axis_f : g.axis;
        const float *rows = sino + (filtered ? sd.filt_off : sd.sino_off);
        const int W = g.bp_w[CFG];
        const float invW = 1.0f / (float)W;
        const int ntx = g.ntx[CFG];
        const int tx = wi.y % ntx, ty = wi.y / ntx;
        const int ix0 = tx * TW, iy0 = ty * TH;
        const double x0 = ix0 - 0.5 * (nx - 1), y0 = iy0 - 0.5 * (ny - 1);
        const double s = g.s;
        const double *cosd = T.cosd + g.ang_off, *sind = T.sind + g.ang_off, *shd = T.shiftd + g.ang_off;
        // the table offset taken as wave-uniform (readfirstlane): the per-projection addresses of the scalar
        // table loads are then formed in SGPRs, not in VGPRs read back every projection
        const cfloat *tab = (const cfloat *)(T.bpt + (int64_t)__builtin_amdgcn_readfirstlane(g.ang_off) * BPT);

        float acc[PX];
#pragma unroll
        for (int p = 0; p < PX; ++p) acc[p] = 0.0f;

        // window base and FP32 remainder of the tile origin for projections kb .. kb + ABLK - 1
        auto params = [&](int kb, int slot) {
            const int na = min(ABLK, K - kb);
            if (tid < na) {
                const int k = kb + tid;
                const double c = cosd[k], sn = sind[k];
                const double torg = axis + shd[k] + s * (x0 * c + y0 * sn);
                const double tmin = torg + s * ((TW - 1) * fmin(c, 0.0) + (TH - 1) * fmin(sn, 0.0));
                const int jb = (int)floor(tmin) - 1;
                s_jb[slot][tid] = jb;
                s_r[slot][tid] = (float)(torg - (double)jb);
            }
        };
        // angle group ag sums projections [ag AB, ag AB + AB) of the staged block
        // tl: the block's table entries staged in LDS (pipelined loop), else null (scalar loads of tab)
        auto sum_block = [&](const float2 *wb, const float *sr, const float *tl, int kb, int na) {
            const int a_end = AG > 1 ? min(na, (ag + 1) * AB) : na;
            for (int a = ag * AB; a < a_end; ++a) {
                const cfloat *tg = tab + (int64_t)(kb + a) * BPT;
                const float *tt = tl + a * NTAB;
                auto tk = [&](int c) { return PIPE ? tt[c] : tg[c]; };
                const float t0 = fmaf(fly, tk(1), fmaf(flx, tk(0), sr[a]));
                const float2 *wa = wb + a * W;
#pragma unroll
                for (int by = 0; by < BY; ++by) {
#pragma unroll
                    for (int bx = 0; bx < BX; ++bx) {
                        const float t = t0 + tk(2 + 8 * by + bx);
                        const int i = (int)t;
                        const float f = __builtin_amdgcn_fractf(t);
                        const float2 v = wa[i];
                        float &A = acc[by * BX + bx];
                        A += v.x;
                        A = fmaf(f, v.y, A);
                    }
                }
            }
        };

        if constexpr (!PIPE) {
            for (int kb = 0; kb < K; kb += ABLK) {
                const int na = min(ABLK, K - kb);
                params(kb, 0);
                __syncthreads();
                const int tot = na * W;
                for (int e = tid; e < tot; e += NT) {
                    const int a = (int)(((float)e + 0.5f) * invW);
                    const int j = s_jb[0][a] + (e - a * W);
                    const float *row = rows + (int64_t)(kb + a) * L;
                    const float q0 = ((unsigned)j < (unsigned)L) ? row[j] : 0.0f;
                    const float q1 = ((unsigned)(j + 1) < (unsigned)L) ? row[j + 1] : 0.0f;
                    win[e] = make_float2(q0, q1 - q0);
                }
                __syncthreads();
                sum_block(win, s_r[0], nullptr, kb, na);
                __syncthreads();
            }
        } else {
            // W <= pipe_wmax(CFG) (checked by the host), so a block's na W <= ABLK W entries take at most
            // E per thread
            constexpr int E = pipe_elems(CFG);
            float q0r[E], q1r[E];
            const int nblk = (K + ABLK - 1) / ABLK;
            auto gload = [&](int b, int slot) {
                const int kb = b * ABLK, tot = min(ABLK, K - kb) * W;
#pragma unroll
                for (int i = 0; i < E; ++i) {
                    const int e = tid + i * NT;
                    q0r[i] = 0.0f;
                    q1r[i] = 0.0f;
                    if (e < tot) {
                        const int a = (int)(((float)e + 0.5f) * invW);
                        const int j = s_jb[slot][a] + (e - a * W);
                        const float *row = rows + (int64_t)(kb + a) * L;
                        if ((unsigned)j < (unsigned)L) q0r[i] = row[j];
                        if ((unsigned)(j + 1) < (unsigned)L) q1r[i] = row[j + 1];
                    }
                }
            };
            auto lstore = [&](int b, float2 *wb) {
                const int tot = min(ABLK, K - b * ABLK) * W;
#pragma unroll
                for (int i = 0; i < E; ++i) {
                    const int e = tid + i * NT;
                    if (e < tot) wb[e] = make_float2(q0r[i], q1r[i] - q0r[i]);
                }
            };
            // a block's parameters (the projections' cos, sin and shift; NTAB table entries each) are
            // loaded into registers two blocks ahead and stored into their slot after the current block's
            // sums, so their L2 / memory latency overlaps two blocks of work
            double pc = 0.0, ps = 0.0, ph = 0.0;
            float pt = 0.0f;
            auto pload = [&](int kb) {
                const int na = min(ABLK, K - kb);
                if (tid < na) {
                    pc = cosd[kb + tid];
                    ps = sind[kb + tid];
                    ph = shd[kb + tid];
                }
                if (tid < na * NTAB) {
                    const int a = tid / NTAB;
                    pt = T.bpt[(int64_t)(g.ang_off + kb + a) * BPT + (tid - a * NTAB)];
                }
            };
            auto pstore = [&](int kb, int slot) {
                const int na = min(ABLK, K - kb);
                if (tid < na) {
                    const double torg = axis + ph + s * (x0 * pc + y0 * ps);
                    const double tmin = torg + s * ((TW - 1) * fmin(pc, 0.0) + (TH - 1) * fmin(ps, 0.0));
                    const int jb = (int)floor(tmin) - 1;
                    s_jb[slot][tid] = jb;
                    s_r[slot][tid] = (float)(torg - (double)jb);
                }
                if (tid < na * NTAB) s_tab[slot][tid] = pt;
            };
            pload(0);
            pstore(0, 0);
            if (nblk > 1) {
                pload(ABLK);
                pstore(ABLK, 1);
            }
            __syncthreads();
            gload(0, 0);
            lstore(0, win);
            __syncthreads();
            for (int b = 0; b < nblk; ++b) {
                if (b + 1 < nblk) gload(b + 1, (b + 1) % 3);
                if (b + 2 < nblk) pload((b + 2) * ABLK);
                const int kb = b * ABLK;
                sum_block(win + (b & 1) * wstride, s_r[b % 3], s_tab[b % 3], kb, min(ABLK, K - kb));
                // buffer (b + 1) & 1 was last read while summing block b - 1, and slot (b + 2) % 3 while
                // summing block b - 1 too, both before the barrier that ended it
                if (b + 1 < nblk) lstore(b + 1, win + ((b + 1) & 1) * wstride);
                if (b + 2 < nblk) pstore((b + 2) * ABLK, (b + 2) % 3);
                __syncthreads();
            }
        }

        if constexpr (AG > 1) {
            // add the groups' partial sums in a fixed order (group 0 + 1 + 2 + 3), through the window
            // buffer, which the last barrier of the projection loop has freed
            float *red = (float *)win;   // [AG - 1][PX][256]
            if (ag > 0) {
#pragma unroll
                for (int q = 0; q < PX; ++q) red[((ag - 1) * PX + q) * 256 + (tid & 255)] = acc[q];
            }
            __syncthreads();
            if (ag == 0) {
#pragma unroll
                for (int h = 0; h < AG - 1; ++h)
#pragma unroll
                    for (int q = 0; q < PX; ++q) acc[q] += red[(h * PX + q) * 256 + tid];
            }
            __syncthreads();   // the buffer is staged again by the next work item
            if (ag > 0) continue;
        }

        // epilogue
        const int64_t ioff = sd.img_off;
#pragma unroll
        for (int by = 0; by < BY; ++by) {
#pragma unroll
            for (int bx = 0; bx < BX; ++bx) {
                const int ix = ix0 + 8 * bx + lx;
                const int iy = iy0 + 8 * BY * wv + 8 * by + ly;
                if (ix < nx && iy < ny) {
                    const int64_t o = ioff + (int64_t)iy * nx + ix;
                    const float v = alpha * acc[by * BX + bx];
                    if (MODE == 0) {
                        img[o] = (beta != 0.0f) ? fmaf(beta, img[o], v) : v;
                    } else {
                        // Chambolle-Pock primal step: x+ = x - tau (A^T p - div q)
                        float dq1, dq2;
                        if (nx == 1) dq1 = 0.0f;
                        else if (ix == 0) dq1 = cp.q1[o];
                        else if (ix == nx - 1) dq1 = -cp.q1[o - 1];
                        else dq1 = cp.q1[o] - cp.q1[o - 1];
                        if (ny == 1) dq2 = 0.0f;
                        else if (iy == 0) dq2 = cp.q2[o];
                        else if (iy == ny - 1) dq2 = -cp.q2[o - nx];
                        else dq2 = cp.q2[o] - cp.q2[o - nx];
                        const float xo = cp.x[o];
                        const float xn = xo - cp.tau * (v - (dq1 + dq2));
                        cp.x[o] = xn;
                        cp.xbar[o] = 2.0f * xn - xo;
                    }
                }
            }
        }
    }
}

// Two slices of a uniform plan per workgroup (slices 2z and 2z + 1, one angle group, the plain loop):
// the staged window holds both slices' (q[j], q[j+1] - q[j]) pairs of a bin side by side, so one
// 16-byte LDS read (which the LDS serves at twice the bytes per clock of an 8-byte one) feeds the
// two slices' updates of a pixel, and the coordinate, truncation, fraction and address are computed
// once for both: 4 + 2 x 2 VALU lane-ops per two updates.  Each slice's sum takes bp_kernel's
// operations in bp_kernel's order, so the images equal bp_kernel's with the same tile bit for bit.
// Work item z n_tiles + tile; an odd last slice runs as a pair with itself and stores once.
// projections staged per LDS block of the two-slice kernel: 16 keep a 64 x 64 tile's block at 24 KB, so
// its 92 VGPRs, not the LDS, set the occupancy (five workgroups per CU; 32 projections, 48 KB, allow three
// and measured 56 instead of 41 ms on 64 x 2048^2 x 1800)
constexpr int AB2 = 16;

template <int CFG>
__global__ __launch_bounds__(256) void bp2_kernel(Tables T, const float *__restrict__ sino, int filtered,
                                                  float *__restrict__ img, float alpha, float beta,
                                                  int n_slices, int n_tiles, int64_t n_items)
{
    constexpr int BX = TILE_BX[CFG], BY = TILE_BY[CFG];
    constexpr int TW = 8 * BX, TH = 32 * BY;
    constexpr int PX = BX * BY;
    static_assert(TILE_AG[CFG] == 1, "one angle group");
    extern __shared__ float4 win4[];   // [AB2][W]
    __shared__ int s_jb[AB2];
    __shared__ float s_r[AB2];

    const int tid = threadIdx.x;
    const int lane = tid & 63, wv = tid >> 6;
    const int lx = lane & 7, ly = lane >> 3;
    const float flx = (float)lx, fly = (float)(ly + 8 * BY * wv);

    // workgroups are dealt round-robin to the 8 XCDs: give each XCD a contiguous range of the work list
    const int64_t b = blockIdx.x, qn = n_items >> 3, rn = n_items & 7, xc = b & 7;
    const int64_t item = xc * qn + min(xc, rn) + (b >> 3);
    if (item >= n_items) return;
    const int z = (int)(item / n_tiles), tile = (int)(item - (int64_t)z * n_tiles);
    const int sl0 = 2 * z;
    const bool two = sl0 + 1 < n_slices;
    const SliceDev sd0 = T.slc[sl0], sd1 = T.slc[two ? sl0 + 1 : sl0];
    const GeoDev &g = T.geo[sd0.g];
    const int nx = g.nx, ny = g.ny, K = g.K;
    const int L = filtered ? g.Lf : g.nb;
    const double axis = filtered ? g.axis_f : g.axis;
    const float *rows0 = sino + (filtered ? sd0.filt_off : sd0.sino_off);
    const float *rows1 = sino + (filtered ? sd1.filt_off : sd1.sino_off);
    const int W = g.bp_w[CFG];
    const float invW = 1.0f / (float)W;
    const int ntx = g.ntx[CFG];
    const int tx = tile % ntx, ty = tile / ntx;
    const int ix0 = tx * TW, iy0 = ty * TH;
    const double x0 = ix0 - 0.5 * (nx - 1), y0 = iy0 - 0.5 * (ny - 1);
    const double s = g.s;
    const double *cosd = T.cosd + g.ang_off, *sind = T.sind + g.ang_off, *shd = T.shiftd + g.ang_off;
    const cfloat *tab = (const cfloat *)(T.bpt + (int64_t)__builtin_amdgcn_readfirstlane(g.ang_off) * BPT);

    float acc0[PX], acc1[PX];
#pragma unroll
    for (int p = 0; p < PX; ++p) {
        acc0[p] = 0.0f;
        acc1[p] = 0.0f;
    }
    for (int kb = 0; kb < K; kb += AB2) {
        const int na = min(AB2, K - kb);
        if (tid < na) {
            const int k = kb + tid;
            const double c = cosd[k], sn = sind[k];
            const double torg = axis + shd[k] + s * (x0 * c + y0 * sn);
            const double tmin = torg + s * ((TW - 1) * fmin(c, 0.0) + (TH - 1) * fmin(sn, 0.0));
            const int jb = (int)floor(tmin) - 1;
            s_jb[tid] = jb;
            s_r[tid] = (float)(torg - (double)jb);
        }
        __syncthreads();
        const int tot = na * W;
        for (int e = tid; e < tot; e += 256) {
            const int a = (int)(((float)e + 0.5f) * invW);
            const int j = s_jb[a] + (e - a * W);
            const int64_t ro = (int64_t)(kb + a) * L;
            const bool in0 = (unsigned)j < (unsigned)L, in1 = (unsigned)(j + 1) < (unsigned)L;
            const float a0 = in0 ? rows0[ro + j] : 0.0f, a1 = in1 ? rows0[ro + j + 1] : 0.0f;
            const float b0 = in0 ? rows1[ro + j] : 0.0f, b1 = in1 ? rows1[ro + j + 1] : 0.0f;
            win4[e] = make_float4(a0, a1 - a0, b0, b1 - b0);
        }
        __syncthreads();
        for (int a = 0; a < na; ++a) {
            const cfloat *tg = tab + (int64_t)(kb + a) * BPT;
            const float t0 = fmaf(fly, tg[1], fmaf(flx, tg[0], s_r[a]));
            const float4 *wa = win4 + a * W;
#pragma unroll
            for (int by = 0; by < BY; ++by) {
#pragma unroll
                for (int bx = 0; bx < BX; ++bx) {
                    const float t = t0 + tg[2 + 8 * by + bx];
                    const int i = (int)t;
                    const float f = __builtin_amdgcn_fractf(t);
                    const float4 v = wa[i];
                    float &A = acc0[by * BX + bx];
                    A += v.x;
                    A = fmaf(f, v.y, A);
                    float &B = acc1[by * BX + bx];
                    B += v.z;
                    B = fmaf(f, v.w, B);
                }
            }
        }
        __syncthreads();
    }

#pragma unroll
    for (int by = 0; by < BY; ++by) {
#pragma unroll
        for (int bx = 0; bx < BX; ++bx) {
            const int ix = ix0 + 8 * bx + lx;
            const int iy = iy0 + 8 * BY * wv + 8 * by + ly;
            if (ix < nx && iy < ny) {
                const int64_t pix = (int64_t)iy * nx + ix;
                const int64_t o0 = sd0.img_off + pix;
                const float v0 = alpha * acc0[by * BX + bx];
                img[o0] = (beta != 0.0f) ? fmaf(beta, img[o0], v0) : v0;
                if (two) {
                    const int64_t o1 = sd1.img_off + pix;
                    const float v1 = alpha * acc1[by * BX + bx];
                    img[o1] = (beta != 0.0f) ? fmaf(beta, img[o1], v1) : v1;
                }
            }
        }
    }
}

__global__ void zero_counter(int *c) { *c = 0; }

template <int CFG, int MODE, bool PIPE>
hipError_t launch_kernel(const pyhst_plan &p, const float *sino, int filtered, float *img, float alpha, float beta,
                         const CpPrimal &cp, int wmax, hipStream_t st)
{
    constexpr int AG = TILE_AG[CFG];
    const int wstride = AG * AB * wmax;   // float2 entries per window buffer
    size_t lds = (size_t)(PIPE ? 2 : 1) * wstride * sizeof(float2);
    if (AG > 1) lds = std::max(lds, (size_t)(AG - 1) * TILE_BX[CFG] * TILE_BY[CFG] * 256 * sizeof(float));
    const int64_t n = p.n_items[CFG];
    if (lds > 65536) {
        if (lds > 160 * 1024) return hipErrorInvalidValue;
        hipError_t e = hipFuncSetAttribute((const void *)bp_kernel<CFG, MODE, PIPE>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    int *counter = p.persistent ? stream_counter(p, st) : nullptr;
    if (counter) {
        zero_counter<<<1, 1, 0, st>>>(counter);
        int per_cu = 0;
        hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, bp_kernel<CFG, MODE, PIPE>, 256 * AG, lds);
        if (e != hipSuccess) return e;
        if (per_cu < 1) per_cu = 1;
        int64_t grid = (int64_t)per_cu * p.cu_count;
        if (grid > n) grid = n;
        bp_kernel<CFG, MODE, PIPE><<<(unsigned)grid, 256 * AG, lds, st>>>(p.t, sino, filtered, img, alpha, beta, n,
                                                                          counter, 0, cp, wstride);
    } else {
        bp_kernel<CFG, MODE, PIPE><<<(unsigned)n, 256 * AG, lds, st>>>(p.t, sino, filtered, img, alpha, beta, n,
                                                                       nullptr, p.uniform ? 1 : 0, cp, wstride);
    }
    return hipGetLastError();
}

template <int CFG>
hipError_t launch_bp2(const pyhst_plan &p, const float *sino, int filtered, float *img, float alpha, float beta,
                      int wmax, hipStream_t st)
{
    const size_t lds = (size_t)AB2 * wmax * sizeof(float4);
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute((const void *)bp2_kernel<CFG>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)lds);
        if (e != hipSuccess) return e;
    }
    // a uniform plan lists every slice's tiles, slice by slice
    const int n_tiles = (int)(p.n_items[CFG] / p.n_slices);
    const int64_t n = (int64_t)((p.n_slices + 1) / 2) * n_tiles;
    bp2_kernel<CFG><<<(unsigned)n, 256, lds, st>>>(p.t, sino, filtered, img, alpha, beta, p.n_slices, n_tiles, n);
    return hipGetLastError();
}

template <int CFG, int MODE>
hipError_t launch_cfg(const pyhst_plan &p, const float *sino, int filtered, float *img, float alpha, float beta,
                      const CpPrimal &cp, hipStream_t st)
{
    int wmax = 0;
    for (const auto &g : p.gd) wmax = std::max(wmax, g.bp_w[CFG]);
    if (p.n_items[CFG] == 0) return hipSuccess;
    if constexpr (MODE == 0 && TILE_AG[CFG] == 1) {
        // (windows of large pixels that would not fit the LDS twice over keep one slice)
        if (two_slice_bp(p) && (size_t)AB2 * wmax * sizeof(float4) <= 160 * 1024)
            return launch_bp2<CFG>(p, sino, filtered, img, alpha, beta, wmax, st);
    }
    if constexpr (CFG == 3 || CFG == 5) {   // the tiles chosen when a launch has few workgroups per CU
        if (wmax <= pipe_wmax(CFG))
            return launch_kernel<CFG, MODE, true>(p, sino, filtered, img, alpha, beta, cp, wmax, st);
    }
    return launch_kernel<CFG, MODE, false>(p, sino, filtered, img, alpha, beta, cp, wmax, st);
}

template <int MODE>
hipError_t launch_mode(const pyhst_plan &p, int cfg, const float *sino, int filtered, float *img, float alpha,
                       float beta, const CpPrimal &cp, hipStream_t st)
{
    switch (cfg) {
    case 0: return launch_cfg<0, MODE>(p, sino, filtered, img, alpha, beta, cp, st);
    case 1: return launch_cfg<1, MODE>(p, sino, filtered, img, alpha, beta, cp, st);
    case 2: return launch_cfg<2, MODE>(p, sino, filtered, img, alpha, beta, cp, st);
    case 3: return launch_cfg<3, MODE>(p, sino, filtered, img, alpha, beta, cp, st);
    case 5: return launch_cfg<5, MODE>(p, sino, filtered, img, alpha, beta, cp, st);
    default: return launch_cfg<4, MODE>(p, sino, filtered, img, alpha, beta, cp, st);
    }
}

}  // namespace

hipError_t launch_backproject(const pyhst_plan &p, const float *sino, int filtered, float *img, float alpha,
                              float beta, const CpPrimal *cp, hipStream_t st)
{
    const int cfg = choose_tile(p);
    if (cp) return launch_mode<1>(p, cfg, sino, filtered, img, alpha, 0.0f, *cp, st);
    CpPrimal none{};
    return launch_mode<0>(p, cfg, sino, filtered, img, alpha, beta, none, st);
}

}  // namespace pyhst
