// Host side of the library: geometry validation, the immutable plan (FP64
// angle tables, quadrature and half-acquisition weights, filter spectra, work
// lists) and the C-ABI entry points.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <memory>
#include <numeric>

#include "internal.hpp"

namespace pyhst {

static thread_local std::string g_err;

void set_error(const std::string &msg) { g_err = msg; }
int fail(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}
int hip_fail(hipError_t e, const char *where)
{
    g_err = std::string(where) + ": " + hipGetErrorString(e);
    return PYHST_EHIP;
}

bool two_slice_bp(const pyhst_plan &p)
{
    return p.uniform && p.n_slices >= 2 && !p.persistent && p.bp_slices != 1;
}

int choose_tile(const pyhst_plan &p)
{
    if (p.bp_tile >= 0 && p.bp_tile < N_TILE_CFG) return p.bp_tile;
    // the largest tile that still gives 4 workgroups per CU (a single 1024^2 slice measures 32 us with
    // 32x32 tiles against 43 us with 64x32 ones, which give only 2)
    const int64_t want = 4LL * p.cu_count;
    if (two_slice_bp(p)) {
        // two slices per workgroup: 64 x 64 tiles (64 x 2048^2 x 1800: 41.0 ms, against 41.5 with 64 x 128
        // and 44.2 with 64 x 32), while their pairs still give 4 workgroups per CU
        if (p.n_items[0] >= 2 * want) return 0;
        if (p.n_items[1] >= 2 * want) return 1;
        if (p.n_items[3] >= 2 * want) return 3;
    }
    if (p.n_items[4] >= want) return 4;
    if (p.n_items[0] >= want) return 0;
    if (p.n_items[1] >= want) return 1;
    // too few 32x32 tiles for 2 workgroups per CU (a single 256^2 slice has 64): split the projections
    // of each tile over 4 angle groups instead
    if (p.n_items[3] < 2LL * p.cu_count) return 5;
    return 3;
}

namespace {

constexpr double PI = 3.14159265358979323846;

// In-place radix-2 FFT in double precision (host, plan creation only).
void fft_host(std::vector<std::complex<double>> &a)
{
    const size_t n = a.size();
    for (size_t i = 1, j = 0; i < n; ++i) {
        size_t bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) std::swap(a[i], a[j]);
    }
    for (size_t len = 2; len <= n; len <<= 1) {
        const double ang = -2.0 * PI / (double)len;
        for (size_t i = 0; i < n; i += len)
            for (size_t k = 0; k < len / 2; ++k) {
                const std::complex<double> w(std::cos(ang * (double)k), std::sin(ang * (double)k));
                const std::complex<double> u = a[i + k], v = a[i + k + len / 2] * w;
                a[i + k] = u + v;
                a[i + k + len / 2] = u - v;
            }
    }
}

unsigned bitrev(unsigned x, int bits)
{
    unsigned r = 0;
    for (int i = 0; i < bits; ++i) r |= ((x >> i) & 1u) << (bits - 1 - i);
    return r;
}

// Spectrum of the Ram-Lak kernel restricted to lags |n| < L, as a length-P
// circular kernel; real because the kernel is even.  Bit-reversed, / P.
std::vector<float> ramp_spectrum(int L, int P, int log2P)
{
    std::vector<std::complex<double>> h(P, 0.0);
    for (int n = -(L - 1); n <= L - 1; ++n) {
        double v;
        if (n == 0) v = 0.25;
        else if (n % 2 == 0) v = 0.0;
        else v = -1.0 / (PI * PI * (double)n * (double)n);
        h[(n + P) % P] += v;
    }
    fft_host(h);
    std::vector<float> out(P);
    for (int i = 0; i < P; ++i) out[i] = (float)(h[bitrev((unsigned)i, log2P)].real() / (double)P);
    return out;
}

int setup_geom(const pyhst_geom &in, GeoHost &h)
{
    if (in.n_x <= 0 || in.n_y <= 0 || in.n_det <= 0 || in.n_angles <= 0)
        return fail(PYHST_EARG, "geometry: sizes must be positive");
    if ((int64_t)in.n_x * in.n_y >= (int64_t)1 << 31)
        return fail(PYHST_EARG, "geometry: n_x * n_y must stay below 2^31 pixels per slice");
    if (!in.angles) return fail(PYHST_EARG, "geometry: angles is NULL");
    if (in.scan < PYHST_SCAN_180 || in.scan > PYHST_SCAN_360_HALF) return fail(PYHST_EARG, "geometry: bad scan type");
    if (!std::isfinite(in.axis_pos) || in.axis_pos < 0.0 || in.axis_pos > in.n_det - 1)
        return fail(PYHST_EARG, "geometry: rotation axis outside the detector");
    h.g = in;
    const int K = in.n_angles;
    h.ang.assign(in.angles, in.angles + K);
    h.shift.assign(K, 0.0);
    if (in.axis_shift) h.shift.assign(in.axis_shift, in.axis_shift + K);
    for (int k = 0; k < K; ++k)
        if (!std::isfinite(h.ang[k]) || !std::isfinite(h.shift[k]))
            return fail(PYHST_EARG, "geometry: non-finite angle or axis shift");
    h.s = in.pixel_size > 0.0 ? in.pixel_size : 1.0;
    h.g.angles = nullptr;
    h.g.axis_shift = nullptr;

    // angular coverage (section 2.1): a scan period of 180 degrees, 360 for 360 degree scans
    const double period = in.scan == PYHST_SCAN_180 ? PI : 2.0 * PI;
    std::vector<int> ord(K);
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return h.ang[a] < h.ang[b]; });
    const double span = h.ang[ord[K - 1]] - h.ang[ord[0]];
    const double mean_gap = K > 1 ? span / (K - 1) : 0.0;
    if (K < 2 || span + 1.5 * mean_gap < period * (1.0 - 1e-9))
        return fail(PYHST_EGEOM, "geometry: projections do not cover the scan period (180 or 360 degrees)");

    // quadrature weights: mid-point rule, circular over the scan period
    h.w.assign(K, 0.0);
    const double factor = in.scan == PYHST_SCAN_360 ? 0.5 : 1.0;
    for (int i = 0; i < K; ++i) {
        const double cur = h.ang[ord[i]];
        const double prev = i == 0 ? h.ang[ord[K - 1]] - period : h.ang[ord[i - 1]];
        const double next = i == K - 1 ? h.ang[ord[0]] + period : h.ang[ord[i + 1]];
        h.w[ord[i]] = factor * 0.5 * (std::max(0.0, cur - prev) + std::max(0.0, next - cur));
    }

    // filtered-row layout; half acquisition extends rows to a symmetric span
    const int nb = in.n_det;
    const double c = in.axis_pos;
    if (in.scan == PYHST_SCAN_360_HALF) {
        const bool right = c >= 0.5 * (nb - 1);
        const double delta = right ? (nb - 1 - c) : c;
        if (delta > 0.25 * nb)
            return fail(PYHST_EGEOM, "half acquisition: the axis must lie in the outer quarter of the detector");
        const double df = in.ha_overlap > 0.0 ? in.ha_overlap : delta;
        if (in.ha_overlap > delta) return fail(PYHST_EARG, "half acquisition: overlap exceeds the axis-edge distance");
        double sgn;
        if (right) {
            h.fpad = 0;
            h.Lf = (int)std::floor(2.0 * c) + 1;
            h.axis_f = c;
            sgn = 1.0;
        } else {
            h.fpad = (int)std::ceil(nb - 1 - 2.0 * c);
            h.Lf = nb + h.fpad;
            h.axis_f = c + h.fpad;
            sgn = -1.0;
        }
        h.haw.assign(h.Lf, 0.0);
        for (int j = 0; j < h.Lf; ++j) {
            const double u = sgn * ((double)j - h.axis_f);
            double w;
            if (df > 0.0) {
                if (u <= -df) w = 1.0;
                else if (u >= df) w = 0.0;
                else w = 0.5 * (1.0 - std::sin(PI * u / (2.0 * df)));
            } else {
                w = u < 0.0 ? 1.0 : (u == 0.0 ? 0.5 : 0.0);
            }
            h.haw[j] = w;
        }
    } else {
        h.fpad = 0;
        h.Lf = nb;
        h.axis_f = c;
        h.haw.assign(nb, 1.0);
    }
    int P = 4, lg = 2;
    while (P < 2 * h.Lf - 1) {
        P <<= 1;
        ++lg;
    }
    if (P > 16384) return fail(PYHST_EARG, "filter: rows longer than 8192 bins are not supported");
    h.P = P;
    h.log2P = lg;
    return PYHST_OK;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

int *stream_counter(const pyhst_plan &p, hipStream_t st)
{
    std::lock_guard<std::mutex> lk(p.counter_mu);
    auto it = p.counter_slot.find(st);
    if (it == p.counter_slot.end()) {
        if (p.counter_slot.size() >= (size_t)PYHST_MAX_STREAMS) return nullptr;
        const int slot = (int)p.counter_slot.size();
        it = p.counter_slot.emplace(st, slot).first;
    }
    return p.t.counter + it->second;
}
}  // namespace pyhst

using namespace pyhst;

extern "C" {

const char *pyhst_last_error(void) { return g_err.c_str(); }

const char *pyhst_strerror(int code)
{
    switch (code) {
    case PYHST_OK: return "ok";
    case PYHST_EARG: return "invalid argument";
    case PYHST_EGEOM: return "invalid geometry";
    case PYHST_ENOMEM: return "out of memory";
    case PYHST_EHIP: return "HIP runtime error";
    case PYHST_ENUM: return "non-finite energy";
    default: return "unknown error";
    }
}

namespace pyhst {
namespace {

// Forward-projection angle blocks of one geometry.  Along the dominant image axis of
// projection k (rows when |cos| >= |sin|), bin j crosses line l at position
// u = U0_k + j / a_k + slope_k l, and touches the positions within 1/|a_k| of it.  Projections are
// sorted by (walking axis, sign of a, slope) and grouped greedily; a block is kept while the union
// of its members' candidate positions for any 64-bin chunk and FP_RB-line block fits in `seg`
// positions.  The union's extent is a convex function of the chunk and block starts (a maximum of
// linear functions minus a minimum of linear functions), so the four corners of that domain bound it.
struct FpAng {
    int k;
    int rows, sgn;
    double a, slope, U0, rho;
};

std::vector<FpAng> fp_sorted(const GeoHost &h, const GeoDev &d)
{
    const double cx = 0.5 * (d.nx - 1), cy = 0.5 * (d.ny - 1);
    std::vector<FpAng> v(d.K);
    for (int k = 0; k < d.K; ++k) {
        const double c = std::cos(h.ang[k]), sn = std::sin(h.ang[k]);
        const bool rows = std::fabs(c) >= std::fabs(sn);
        const double a = rows ? h.s * c : h.s * sn, bb = rows ? h.s * sn : h.s * c;
        const double ci = rows ? cx : cy, cl = rows ? cy : cx;
        const double t0 = h.g.axis_pos + h.shift[k];
        v[k] = FpAng{k, rows ? 1 : 0, a > 0 ? 1 : 0, a, -bb / a, (-t0 + a * ci + bb * cl) / a, 1.0 / std::fabs(a)};
    }
    std::stable_sort(v.begin(), v.end(), [](const FpAng &x, const FpAng &y) {
        if (x.rows != y.rows) return x.rows > y.rows;
        if (x.sgn != y.sgn) return x.sgn > y.sgn;
        return x.slope < y.slope;
    });
    return v;
}

void build_fp_blocks(const GeoHost &h, const GeoDev &d, int seg, std::vector<int> &members,
                     std::vector<int2> &blocks)
{
    const std::vector<FpAng> v = fp_sorted(h, d);
    const int nchunk = (d.nb + 63) / 64;
    const double jc[2] = {0.0, 64.0 * (nchunk - 1)};
    auto extent = [&](const FpAng &x, double j0, double l0, double &lo, double &hi) {
        // positions touched by bins j0..j0+63 on lines l0..l0+RB-1 (u linear in j and l)
        double mn = 1e300, mx = -1e300;
        for (int cj = 0; cj < 2; ++cj)
            for (int cl = 0; cl < 2; ++cl) {
                const double u = x.U0 + (j0 + 63.0 * cj) / x.a + x.slope * (l0 + (FP_RB - 1) * cl);
                mn = std::min(mn, u);
                mx = std::max(mx, u);
            }
        lo = mn - x.rho;
        hi = mx + x.rho;
    };
    size_t i = 0;
    while (i < v.size()) {
        size_t e = i + 1;
        const int nl = v[i].rows ? d.ny : d.nx;
        const double lc[2] = {0.0, (double)(((nl - 1) / FP_RB) * FP_RB)};
        while (e < v.size() && e - i < (size_t)FP_AMAX && v[e].rows == v[i].rows) {
            bool ok = true;
            for (int a = 0; a < 2 && ok; ++a)
                for (int b = 0; b < 2 && ok; ++b) {
                    double lo = 1e300, hi = -1e300;
                    for (size_t m = i; m <= e; ++m) {
                        double l1, h1;
                        extent(v[m], jc[a], lc[b], l1, h1);
                        lo = std::min(lo, l1);
                        hi = std::max(hi, h1);
                    }
                    ok = (hi - lo) + 6.0 <= (double)seg;   // floor slack and up to 2 zero-weight reads
                }
            if (!ok) break;
            ++e;
        }
        blocks.push_back(make_int2((int)members.size(), (int)(e - i)));
        for (size_t m = i; m < e; ++m) members.push_back(v[m].k);
        i = e;
    }
}

// Groups of the staged projector: neighbours in the sorted order are grouped greedily (up to
// FP_SGRP) while, for every 64-bin chunk and FP_RB-line block, the first candidates of all members
// (u - 1/|a| over the chunk's bins and the block's lines) span at most sseg - nc - 5 positions.  The
// staged kernel starts the segment 2 positions below the lowest first candidate and reads nc - 1
// positions past the highest, so this keeps every read inside the sseg staged positions with a
// margin of 2 for FP32 rounding.  Corners bound the span as in build_fp_blocks.
void build_fp_groups(const GeoHost &h, const GeoDev &d, int nc, int cap, std::vector<int4> &groups)
{
    const std::vector<FpAng> v = fp_sorted(h, d);
    const int sseg = nc == 3 ? FP_SSEG3 : FP_SSEG6;
    const int nchunk = (d.nb + 63) / 64;
    const double jc[2] = {0.0, 64.0 * (nchunk - 1)};
    auto fits = [&](size_t i, size_t e) {   // members v[i..e]
        for (size_t m = i + 1; m <= e; ++m)
            if (v[m].rows != v[i].rows) return false;
        const int nl = v[i].rows ? d.ny : d.nx;
        const double lc[2] = {0.0, (double)(((nl - 1) / FP_RB) * FP_RB)};
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) {
                double lo = 1e300, hi = -1e300;
                for (size_t m = i; m <= e; ++m)
                    for (int cj = 0; cj < 2; ++cj)
                        for (int cl = 0; cl < 2; ++cl) {
                            const double w = v[m].U0 + (jc[a] + 63.0 * cj) / v[m].a +
                                             v[m].slope * (lc[b] + (FP_RB - 1) * cl) - v[m].rho;
                            lo = std::min(lo, w);
                            hi = std::max(hi, w);
                        }
                if ((hi - lo) + nc + 5 > sseg) return false;
            }
        return true;
    };
    size_t i = 0;
    while (i < v.size()) {
        size_t e = i;   // last member
        while (e + 1 < v.size() && e + 1 - i < (size_t)cap && fits(i, e + 1)) ++e;
        int k[FP_SGRP] = {-1, -1, -1, -1};
        for (size_t m = i; m <= e; ++m) k[m - i] = v[m].k;
        groups.push_back(make_int4(k[0], k[1], k[2], k[3]));
        i = e + 1;
    }
}

}  // namespace
}  // namespace pyhst

int pyhst_plan_create(const pyhst_geom *g, int32_t n_geom, const int32_t *slice_geom, int32_t n_slices,
                      pyhst_plan **out)
{
    if (!out) return fail(PYHST_EARG, "plan_create: out is NULL");
    *out = nullptr;
    if (!g || n_geom <= 0 || n_slices <= 0) return fail(PYHST_EARG, "plan_create: need geometries and slices");
    if (n_slices > PYHST_MAX_SLICES)
        return fail(PYHST_EARG, "plan_create: at most 65535 slices per plan (split larger stacks)");
    try {
        auto *p = new pyhst_plan();
        std::unique_ptr<pyhst_plan> guard(p);
        std::vector<int> sg(n_slices, 0);
        for (int i = 0; i < n_slices; ++i) {
            sg[i] = slice_geom ? slice_geom[i] : 0;
            if (sg[i] < 0 || sg[i] >= n_geom) return fail(PYHST_EARG, "plan_create: slice_geom out of range");
        }
        p->uniform = std::all_of(sg.begin(), sg.end(), [&](int v) { return v == sg[0]; });
        // A uniform plan keeps only the geometry its slices use, as geometry 0: every path that
        // assumes one geometry reads gd[0].
        const pyhst_geom *gsrc = g;
        if (p->uniform) {
            gsrc = g + sg[0];
            n_geom = 1;
            std::fill(sg.begin(), sg.end(), 0);
        }
        p->n_geom = n_geom;
        p->n_slices = n_slices;
        p->gh.resize(n_geom);
        for (int i = 0; i < n_geom; ++i) {
            int rc = setup_geom(gsrc[i], p->gh[i]);
            if (rc) return rc;
        }
        if (const char *f = std::getenv("PYHST_FAKE_OOM"); f && f[0] == '1')
            return fail(PYHST_ENOMEM, "plan_create: allocation failure injected by PYHST_FAKE_OOM");

        hipError_t e = hipGetDevice(&p->device);
        if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device) == hipSuccess && cus > 0)
            p->cu_count = cus;

        // per-geometry device descriptors and table offsets
        int64_t nang = 0, nhw = 0, nspec = 0;
        int Pmax = 4, lgmax = 2;
        p->gd.resize(n_geom);
        std::map<std::pair<int, int>, int64_t> spec_cache;
        std::vector<std::vector<float>> spectra;
        for (int i = 0; i < n_geom; ++i) {
            const GeoHost &h = p->gh[i];
            GeoDev &d = p->gd[i];
            d.nx = h.g.n_x;
            d.ny = h.g.n_y;
            d.nb = h.g.n_det;
            d.K = h.g.n_angles;
            d.Lf = h.Lf;
            d.fpad = h.fpad;
            d.P = h.P;
            d.log2P = h.log2P;
            d.s = h.s;
            d.axis = h.g.axis_pos;
            d.axis_f = h.axis_f;
            d.ang_off = nang;
            nang += d.K;
            d.hw_off = nhw;
            d.half = h.g.scan == PYHST_SCAN_360_HALF ? 1 : 0;
            nhw += h.Lf;
            auto key = std::make_pair(h.Lf, h.P);
            auto it = spec_cache.find(key);
            if (it == spec_cache.end()) {
                spectra.push_back(ramp_spectrum(h.Lf, h.P, h.log2P));
                spec_cache[key] = nspec;
                d.spec_off = nspec;
                nspec += h.P;
            } else {
                d.spec_off = it->second;
            }
            if (h.P > Pmax) {
                Pmax = h.P;
                lgmax = h.log2P;
            }
            for (int c = 0; c < N_TILE_CFG; ++c) {
                double range = 0.0;
                for (int k = 0; k < d.K; ++k)
                    range = std::max(range, h.s * ((tile_w(c) - 1) * std::fabs(std::cos(h.ang[k])) +
                                                   (tile_h(c) - 1) * std::fabs(std::sin(h.ang[k]))));
                int W = (int)std::floor(range) + 4;
                W += W & 1;
                d.bp_w[c] = W;
                d.ntx[c] = (d.nx + tile_w(c) - 1) / tile_w(c);
            }
            p->max_K = std::max<int64_t>(p->max_K, d.K);
        }

        // forward-projection angle blocks (segment length from the smallest pixel size)
        double s_min = 1e300;
        for (const auto &h : p->gh) s_min = std::min(s_min, h.s);
        p->fp_seg = fp_seg_len(s_min);
        std::vector<int> fp_members;
        std::vector<int2> fp_blocks;
        for (int i = 0; i < n_geom; ++i) {
            GeoDev &d = p->gd[i];
            d.fp_blk_off = (int)fp_blocks.size();
            std::vector<int> mem;
            std::vector<int2> blk;
            build_fp_blocks(p->gh[i], d, p->fp_seg, mem, blk);
            for (auto &b : blk) fp_blocks.push_back(make_int2(b.x + (int)fp_members.size(), b.y));
            fp_members.insert(fp_members.end(), mem.begin(), mem.end());
            d.fp_nblk = (int)blk.size();
            p->fp_max_blocks = std::max(p->fp_max_blocks, d.fp_nblk);
        }
        // staged-projector groups (the staged kernel needs a fixed candidate count): up to FP_SGRP
        // projections per group, or up to two when bigger groups would leave fewer than 16 workgroups
        // per compute unit (few slices and angles: then occupancy and balance matter more than reuse)
        const int nc = fp_nc_for(s_min);
        std::vector<int4> fp_pairs;
        for (int cap : {FP_SGRP, 2}) {
            fp_pairs.clear();
            p->fp_max_pairs = 0;
            for (int i = 0; i < n_geom; ++i) {
                GeoDev &d = p->gd[i];
                d.fp_pair_off = (int)fp_pairs.size();
                if (nc > 0) build_fp_groups(p->gh[i], d, nc, cap, fp_pairs);
                d.fp_npair = (int)fp_pairs.size() - d.fp_pair_off;
                p->fp_max_pairs = std::max(p->fp_max_pairs, d.fp_npair);
            }
            int64_t wgs = 0;
            for (int i = 0; i < n_slices; ++i) {
                const GeoDev &d = p->gd[sg[i]];
                wgs += (int64_t)((d.nb + 63) / 64) * d.fp_npair;
            }
            if (wgs >= 16LL * p->cu_count) break;
        }
        for (const int4 &q : fp_pairs)
            p->fp_max_grp = std::max(p->fp_max_grp, q.w >= 0 ? 4 : (q.z >= 0 ? 3 : (q.y >= 0 ? 2 : 1)));
        if (fp_pairs.empty()) fp_pairs.push_back(make_int4(0, -1, -1, -1));   // keeps the table non-empty

        // slices: packed offsets
        p->sd.resize(n_slices);
        int64_t so = 0, fo = 0, io = 0;
        for (int i = 0; i < n_slices; ++i) {
            const GeoDev &d = p->gd[sg[i]];
            SliceDev &s = p->sd[i];
            s.g = sg[i];
            s.sino_off = so;
            s.filt_off = fo;
            s.img_off = io;
            so += (int64_t)d.K * d.nb;
            fo += (int64_t)d.K * d.Lf;
            io += (int64_t)d.nx * d.ny;
        }
        p->sino_elems = so;
        p->filt_elems = fo;
        p->img_elems = io;

        // work lists: filter row pairs; backprojection (slice, tile), costliest slices first
        std::vector<int2> pairs;
        for (int i = 0; i < n_slices; ++i)
            for (int k = 0; k < p->gd[sg[i]].K; k += 2) pairs.push_back(make_int2(i, k));
        p->n_pairs = (int)pairs.size();
        std::vector<int> sorder(n_slices);
        std::iota(sorder.begin(), sorder.end(), 0);
        std::stable_sort(sorder.begin(), sorder.end(), [&](int a, int b) {
            const GeoDev &A = p->gd[sg[a]], &B = p->gd[sg[b]];
            return (int64_t)A.K * A.nx * A.ny > (int64_t)B.K * B.nx * B.ny;
        });
        std::vector<int2> items[N_TILE_CFG];
        for (int c = 0; c < N_TILE_CFG; ++c) {
            for (int i : sorder) {
                const GeoDev &d = p->gd[sg[i]];
                const int nt = d.ntx[c] * ((d.ny + tile_h(c) - 1) / tile_h(c));
                for (int t = 0; t < nt; ++t) items[c].push_back(make_int2(i, t));
            }
            p->n_items[c] = (int64_t)items[c].size();
        }

        // one device block for every table
        size_t off = 0;
        auto take = [&](size_t bytes) {
            size_t o = off;
            off = align256(off + bytes);
            return o;
        };
        const size_t o_geo = take(sizeof(GeoDev) * n_geom);
        const size_t o_slc = take(sizeof(SliceDev) * n_slices);
        const size_t o_cos = take(sizeof(double) * nang), o_sin = take(sizeof(double) * nang),
                     o_sh = take(sizeof(double) * nang);
        const size_t o_bpt = take(sizeof(float) * nang * BPT);
        const size_t o_w = take(sizeof(float) * nang);
        const size_t o_hw = take(sizeof(float) * nhw);
        const size_t o_spec = take(sizeof(float) * nspec);
        const size_t o_tw = take(sizeof(float2) * (Pmax / 2));
        const size_t o_pairs = take(sizeof(int2) * pairs.size());
        size_t o_items[N_TILE_CFG];
        for (int c = 0; c < N_TILE_CFG; ++c) o_items[c] = take(sizeof(int2) * items[c].size());
        const size_t o_cnt = take(sizeof(int) * PYHST_MAX_STREAMS);
        const size_t o_fpa = take(sizeof(int) * fp_members.size());
        const size_t o_fpb = take(sizeof(int2) * fp_blocks.size());
        const size_t o_fpp = take(sizeof(int4) * fp_pairs.size());
        const size_t total = off;

        std::vector<unsigned char> hbuf(total, 0);
        auto put = [&](size_t o, const void *src, size_t bytes) {
            if (bytes) std::memcpy(hbuf.data() + o, src, bytes);
        };
        put(o_geo, p->gd.data(), sizeof(GeoDev) * n_geom);
        put(o_slc, p->sd.data(), sizeof(SliceDev) * n_slices);
        std::vector<double> cs(nang), sn(nang), sh(nang);
        std::vector<float> bpt(nang * BPT, 0.0f), wv(nang), hw(nhw), spec(nspec);
        for (int i = 0; i < n_geom; ++i) {
            const GeoHost &h = p->gh[i];
            const GeoDev &d = p->gd[i];
            for (int k = 0; k < d.K; ++k) {
                const int64_t a = d.ang_off + k;
                const double c = std::cos(h.ang[k]), s = std::sin(h.ang[k]);
                cs[a] = c;
                sn[a] = s;
                sh[a] = h.shift[k];
                wv[a] = (float)h.w[k];
                float *t = &bpt[a * BPT];
                t[0] = (float)(h.s * c);
                t[1] = (float)(h.s * s);
                for (int by = 0; by < 4; ++by)
                    for (int bx = 0; bx < 8; ++bx) t[2 + 8 * by + bx] = (float)(8.0 * h.s * (bx * c + by * s));
            }
            for (int j = 0; j < h.Lf; ++j) hw[d.hw_off + j] = (float)h.haw[j];
        }
        {
            int64_t o = 0;
            for (auto &v : spectra) {
                std::copy(v.begin(), v.end(), spec.begin() + o);
                o += (int64_t)v.size();
            }
        }
        std::vector<float2> tw(Pmax / 2);
        for (int m = 0; m < Pmax / 2; ++m) {
            const double a = -2.0 * PI * (double)m / (double)Pmax;
            tw[m] = make_float2((float)std::cos(a), (float)std::sin(a));
        }
        put(o_cos, cs.data(), sizeof(double) * nang);
        put(o_sin, sn.data(), sizeof(double) * nang);
        put(o_sh, sh.data(), sizeof(double) * nang);
        put(o_bpt, bpt.data(), sizeof(float) * bpt.size());
        put(o_w, wv.data(), sizeof(float) * nang);
        put(o_hw, hw.data(), sizeof(float) * nhw);
        put(o_spec, spec.data(), sizeof(float) * nspec);
        put(o_tw, tw.data(), sizeof(float2) * tw.size());
        put(o_pairs, pairs.data(), sizeof(int2) * pairs.size());
        for (int c = 0; c < N_TILE_CFG; ++c) put(o_items[c], items[c].data(), sizeof(int2) * items[c].size());
        put(o_fpa, fp_members.data(), sizeof(int) * fp_members.size());
        put(o_fpb, fp_blocks.data(), sizeof(int2) * fp_blocks.size());
        put(o_fpp, fp_pairs.data(), sizeof(int4) * fp_pairs.size());

        e = hipMalloc(&p->dev_block, total);
        if (e != hipSuccess) {
            p->dev_block = nullptr;
            (void)hipGetLastError();
            return fail(PYHST_ENOMEM, std::string("plan_create: hipMalloc: ") + hipGetErrorString(e));
        }
        e = hipMemcpy(p->dev_block, hbuf.data(), total, hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            (void)hipFree(p->dev_block);
            p->dev_block = nullptr;
            return hip_fail(e, "plan_create: hipMemcpy");
        }
        unsigned char *b = (unsigned char *)p->dev_block;
        Tables &t = p->t;
        t.geo = (const GeoDev *)(b + o_geo);
        t.slc = (const SliceDev *)(b + o_slc);
        t.cosd = (const double *)(b + o_cos);
        t.sind = (const double *)(b + o_sin);
        t.shiftd = (const double *)(b + o_sh);
        t.bpt = (const float *)(b + o_bpt);
        t.wang = (const float *)(b + o_w);
        t.haw = (const float *)(b + o_hw);
        t.spec = (const float *)(b + o_spec);
        t.twid = (const float2 *)(b + o_tw);
        t.pairs = (const int2 *)(b + o_pairs);
        for (int c = 0; c < N_TILE_CFG; ++c) t.items[c] = (const int2 *)(b + o_items[c]);
        t.counter = (int *)(b + o_cnt);
        t.fp_ang = (const int *)(b + o_fpa);
        t.fp_blk = (const int2 *)(b + o_fpb);
        t.fp_pair = (const int4 *)(b + o_fpp);
        t.Pmax = Pmax;
        t.log2Pmax = lgmax;
        *out = guard.release();
        return PYHST_OK;
    } catch (const std::bad_alloc &) {
        return fail(PYHST_ENOMEM, "plan_create: host allocation failed");
    } catch (...) {
        return fail(PYHST_EARG, "plan_create: unexpected failure");
    }
}

int pyhst_plan_destroy(pyhst_plan *plan)
{
    if (!plan) return PYHST_OK;
    for (auto &kv : plan->graphs) (void)hipGraphExecDestroy(kv.second);
    if (plan->dev_block) (void)hipFree(plan->dev_block);
    delete plan;
    return PYHST_OK;
}

int pyhst_plan_slice_info(const pyhst_plan *p, int32_t slice, pyhst_slice_info *out)
{
    if (!p || !out || slice < 0 || slice >= p->n_slices) return fail(PYHST_EARG, "slice_info: bad argument");
    const SliceDev &s = p->sd[slice];
    const GeoDev &g = p->gd[s.g];
    out->n_x = g.nx;
    out->n_y = g.ny;
    out->n_det = g.nb;
    out->n_angles = g.K;
    out->filt_len = g.Lf;
    out->filt_pad = g.fpad;
    out->filt_axis = g.axis_f;
    out->sino_offset = s.sino_off;
    out->filt_offset = s.filt_off;
    out->img_offset = s.img_off;
    return PYHST_OK;
}

int pyhst_plan_sizes(const pyhst_plan *p, int64_t *sino_elems, int64_t *filt_elems, int64_t *img_elems)
{
    if (!p) return fail(PYHST_EARG, "plan_sizes: plan is NULL");
    if (sino_elems) *sino_elems = p->sino_elems;
    if (filt_elems) *filt_elems = p->filt_elems;
    if (img_elems) *img_elems = p->img_elems;
    return PYHST_OK;
}

int pyhst_plan_set_tiles(pyhst_plan *p, int32_t bp_tile, int32_t persistent)
{
    if (!p || bp_tile < -1 || bp_tile >= N_TILE_CFG) return fail(PYHST_EARG, "set_tiles: bad argument");
    std::lock_guard<std::mutex> lk(p->mu);
    p->bp_tile = bp_tile;
    p->persistent = persistent ? 1 : 0;
    for (auto &kv : p->graphs) (void)hipGraphExecDestroy(kv.second);
    p->graphs.clear();
    return PYHST_OK;
}

int pyhst_plan_set_fp_kernel(pyhst_plan *p, int32_t kind)
{
    if (!p || kind < PYHST_FP_AUTO || kind > PYHST_FP_LINES) return fail(PYHST_EARG, "set_fp_kernel: bad argument");
    std::lock_guard<std::mutex> lk(p->mu);
    p->fp_kernel = kind;
    for (auto &kv : p->graphs) (void)hipGraphExecDestroy(kv.second);
    p->graphs.clear();
    return PYHST_OK;
}

int pyhst_plan_set_bp_slices(pyhst_plan *p, int32_t per_workgroup)
{
    if (!p || per_workgroup < 0 || per_workgroup > 2) return fail(PYHST_EARG, "set_bp_slices: bad argument");
    std::lock_guard<std::mutex> lk(p->mu);
    p->bp_slices = per_workgroup;
    for (auto &kv : p->graphs) (void)hipGraphExecDestroy(kv.second);
    p->graphs.clear();
    return PYHST_OK;
}

int pyhst_plan_get_fp_kernel(const pyhst_plan *p, int32_t *kind)
{
    if (!p || !kind) return fail(PYHST_EARG, "get_fp_kernel: NULL argument");
    *kind = p->fp_kernel;
    return PYHST_OK;
}

int pyhst_plan_get_tiles(const pyhst_plan *p, int32_t *bp_tile, int32_t *persistent)
{
    if (!p) return fail(PYHST_EARG, "get_tiles: plan is NULL");
    if (bp_tile) *bp_tile = choose_tile(*p);
    if (persistent) *persistent = p->persistent;
    return PYHST_OK;
}

int pyhst_normalize(const pyhst_plan *p, const uint16_t *raw, const float *flats, const double *flat_pos,
                    int32_t n_flats, const float *dark, float eps, float *sino, hipStream_t st)
{
    if (!p || !raw || !flats || !flat_pos || !dark || !sino) return fail(PYHST_EARG, "normalize: NULL argument");
    if (!p->uniform) return fail(PYHST_EARG, "normalize: raw radiographs need a uniform plan");
    if (n_flats < 1 || n_flats > 32) return fail(PYHST_EARG, "normalize: n_flats must be in [1, 32]");
    for (int i = 1; i < n_flats; ++i)
        if (!(flat_pos[i] > flat_pos[i - 1])) return fail(PYHST_EARG, "normalize: flat positions must increase");
    hipError_t e = launch_normalize(*p, raw, flats, flat_pos, n_flats, dark, eps, sino, st);
    return e == hipSuccess ? PYHST_OK : hip_fail(e, "normalize");
}

int pyhst_normalize_hotspot(const pyhst_plan *p, const uint16_t *raw, const float *flats, const double *flat_pos,
                            int32_t n_flats, const float *dark, float eps, float threshold, int32_t halo_lo,
                            int32_t halo_hi, float *sino, hipStream_t st)
{
    if (!p || !raw || !flats || !flat_pos || !dark || !sino) return fail(PYHST_EARG, "normalize_hotspot: NULL argument");
    if (!p->uniform) return fail(PYHST_EARG, "normalize_hotspot: raw radiographs need a uniform plan");
    if (n_flats < 1 || n_flats > 32) return fail(PYHST_EARG, "normalize_hotspot: n_flats must be in [1, 32]");
    for (int i = 1; i < n_flats; ++i)
        if (!(flat_pos[i] > flat_pos[i - 1]))
            return fail(PYHST_EARG, "normalize_hotspot: flat positions must increase");
    if (!(threshold >= 0.0f)) return fail(PYHST_EARG, "normalize_hotspot: threshold must be >= 0");
    if (halo_lo < 0 || halo_lo > 1 || halo_hi < 0 || halo_hi > 1)
        return fail(PYHST_EARG, "normalize_hotspot: halo rows must be 0 or 1 on each side");
    hipError_t e = launch_normalize_hotspot(*p, raw, flats, flat_pos, n_flats, dark, eps, threshold, halo_lo, halo_hi,
                                            sino, st);
    return e == hipSuccess ? PYHST_OK : hip_fail(e, "normalize_hotspot");
}

int pyhst_ring_filter(const pyhst_plan *p, float *sino, int32_t width, const float *obj, double *work,
                      size_t work_doubles, hipStream_t st)
{
    if (!p || !sino) return fail(PYHST_EARG, "ring_filter: NULL argument");
    if (!p->uniform) return fail(PYHST_EARG, "ring_filter: needs a uniform plan");
    if (width < 0) return fail(PYHST_EARG, "ring_filter: width must be >= 0");
    if (!work || work_doubles < 2 * (size_t)p->n_slices * p->gd[0].nb)
        return fail(PYHST_EARG, "ring_filter: work needs 2 * n_slices * n_det doubles");
    hipError_t e = launch_ring_filter(*p, sino, obj, width, work, st);
    return e == hipSuccess ? PYHST_OK : hip_fail(e, "ring_filter");
}

int fbp_filter(const pyhst_plan *p, const float *sino, float *filt, hipStream_t st)
{
    if (!p || !sino || !filt) return fail(PYHST_EARG, "fbp_filter: NULL argument");
    if (sino == filt && p->filt_elems != p->sino_elems)
        return fail(PYHST_EARG, "fbp_filter: in place needs unextended rows");
    hipError_t e = launch_filter(*p, sino, nullptr, nullptr, nullptr, 0, nullptr, 0.0f, filt, st);
    return e == hipSuccess ? PYHST_OK : hip_fail(e, "fbp_filter");
}

int backproject(const pyhst_plan *p, const float *sino, int32_t filtered_layout, float *img, float alpha, float beta,
                hipStream_t st)
{
    if (!p || !sino || !img) return fail(PYHST_EARG, "backproject: NULL argument");
    if (filtered_layout != 0 && filtered_layout != 1) return fail(PYHST_EARG, "backproject: layout must be 0 or 1");
    hipError_t e = launch_backproject(*p, sino, filtered_layout, img, alpha, beta, nullptr, st);
    return e == hipSuccess ? PYHST_OK : hip_fail(e, "backproject");
}

int forward_project(const pyhst_plan *p, const float *img, float *sino, float alpha, hipStream_t st)
{
    if (!p || !img || !sino) return fail(PYHST_EARG, "forward_project: NULL argument");
    if (!std::isfinite(alpha)) return fail(PYHST_EARG, "forward_project: alpha must be finite");
    hipError_t e = launch_forward(*p, img, sino, alpha, nullptr, st);
    return e == hipSuccess ? PYHST_OK : hip_fail(e, "forward_project");
}

int tv_prox(int32_t n_slices, int32_t n_y, int32_t n_x, const float *in, float *out, float lambda, int32_t n_inner,
            float *work, size_t work_floats, hipStream_t st)
{
    if (n_slices <= 0 || n_y <= 0 || n_x <= 0 || !in || !out) return fail(PYHST_EARG, "tv_prox: bad argument");
    if (n_slices > PYHST_MAX_SLICES || n_y > 8 * 65535)
        return fail(PYHST_EARG, "tv_prox: at most 65535 slices of at most 524280 rows");
    if (!std::isfinite(lambda) || lambda < 0.0f || n_inner < 0) return fail(PYHST_EARG, "tv_prox: bad lambda/n_inner");
    const size_t need = 4 * (size_t)n_slices * n_y * n_x;
    if (lambda > 0.0f && n_inner > 0 && (!work || work_floats < need))
        return fail(PYHST_EARG, "tv_prox: work must hold 4*n_slices*n_y*n_x floats");
    hipError_t e = launch_tv_prox(n_slices, n_y, n_x, in, out, lambda, n_inner, work, st);
    return e == hipSuccess ? PYHST_OK : hip_fail(e, "tv_prox");
}

}  // extern "C"

// Backprojector autotuner: time every tile shape, with and without the
// persistent work queue, on the caller's buffers, keep the fastest.
extern "C" int pyhst_plan_autotune(pyhst_plan *p, const float *filt, float *img, int32_t reps, float *best_ms,
                                   hipStream_t st)
{
    if (!p || !filt || !img || reps <= 0) return fail(PYHST_EARG, "autotune: bad argument");
    hipEvent_t e0, e1;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e != hipSuccess) return hip_fail(e, "autotune: event");
    float best = 1e30f;
    int bt = 0, bp = 0;
    const int keep_tile = p->bp_tile, keep_pers = p->persistent;
    for (int pers = 0; pers < 2 && e == hipSuccess; ++pers) {
        for (int t = 0; t < N_TILE_CFG && e == hipSuccess; ++t) {
            p->bp_tile = t;
            p->persistent = pers;
            e = launch_backproject(*p, filt, 1, img, 1.0f, 0.0f, nullptr, st);   // warm-up
            if (e == hipSuccess) e = hipEventRecord(e0, st);
            for (int r = 0; r < reps && e == hipSuccess; ++r)
                e = launch_backproject(*p, filt, 1, img, 1.0f, 0.0f, nullptr, st);
            if (e == hipSuccess) e = hipEventRecord(e1, st);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e == hipSuccess && ms / reps < best) {
                best = ms / reps;
                bt = t;
                bp = pers;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) {
        p->bp_tile = keep_tile;
        p->persistent = keep_pers;
        return hip_fail(e, "autotune");
    }
    {
        std::lock_guard<std::mutex> lk(p->mu);
        p->bp_tile = bt;
        p->persistent = bp;
        for (auto &kv : p->graphs) (void)hipGraphExecDestroy(kv.second);
        p->graphs.clear();
    }
    if (best_ms) *best_ms = best;
    return PYHST_OK;
}
