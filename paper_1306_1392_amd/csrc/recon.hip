// reconstruct_slices: the whole path for a batch of slices.
//   FBP        : (normalise + weight + ramp filter) -> backprojection      (section 2.3)
//   TV_CP      : eq. (3) by Chambolle-Pock with K = [A; grad]              (section 3.1)
//   ISTA/FISTA : eq. (3) by gradient step + TV proximal map, the solvers section 3.1 names
// Each is a plain launch sequence on one stream, so the sequence can be
// captured into a HIP graph (use_graph) and replayed without host work.
#include <cmath>
#include <cstring>

#include "internal.hpp"

using namespace pyhst;

namespace {

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct CpLayout {
    size_t y, xbar, q1, q2, p, ax, partials, total;
};

// Optional preprocessing of section 2.3 (hot spots, rings): the data go through a work copy y.
struct PreLayout {
    bool on;
    size_t y, ring, obj, img, filt, total;
};

PreLayout pre_layout(const pyhst_plan &p, const pyhst_recon_args &a)
{
    PreLayout L{};
    L.on = a.hot_spot != 0 || a.ring_width > 0;
    if (!L.on) return L;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t r = o;
        o = align256(o + bytes);
        return r;
    };
    L.y = take((size_t)p.sino_elems * 4);
    if (a.ring_width > 0) L.ring = take((size_t)2 * p.n_slices * p.gd[0].nb * 8);
    if (a.ring_width > 0 && a.ring_object) {
        L.obj = take((size_t)p.sino_elems * 4);
        L.img = take((size_t)p.img_elems * 4);
        L.filt = take((size_t)p.filt_elems * 4);
    }
    L.total = o;
    return L;
}

CpLayout cp_layout(const pyhst_plan &p, const pyhst_recon_args &a, size_t base, bool need_y)
{
    CpLayout L{};
    size_t o = base;
    auto take = [&](size_t bytes) {
        size_t r = o;
        o = align256(o + bytes);
        return r;
    };
    const size_t ni = (size_t)p.img_elems, ns = (size_t)p.sino_elems;
    L.y = need_y ? take(ns * 4) : (size_t)-1;
    L.xbar = take(ni * 4);
    L.q1 = take(ni * 4);
    L.q2 = take(ni * 4);
    L.p = take(ns * 4);
    L.ax = a.energy ? take(ns * 4) : (size_t)-1;
    L.partials = take(sizeof(double) * 1024);
    L.total = o;
    return L;
}

struct FiLayout {
    size_t y, r, ax, z, xb, prox, partials, total;
};

FiLayout fista_layout(const pyhst_plan &p, const pyhst_recon_args &a, size_t base, bool need_y)
{
    FiLayout L{};
    size_t o = base;
    auto take = [&](size_t bytes) {
        size_t r = o;
        o = align256(o + bytes);
        return r;
    };
    const size_t ni = (size_t)p.img_elems, ns = (size_t)p.sino_elems;
    L.y = need_y ? take(ns * 4) : (size_t)-1;
    L.r = take(ns * 4);
    L.ax = a.energy ? take(ns * 4) : (size_t)-1;
    L.z = take(ni * 4);
    L.xb = take(ni * 4);
    L.prox = take(4 * ni * 4);
    L.partials = take(sizeof(double) * 1024);
    L.total = o;
    return L;
}

// scratch of pyhst_opnorm: two images, one sinogram, reduction partials and the norm
struct NormLayout {
    size_t x, y, tmp, partials, norm, total;
};

NormLayout norm_layout(const pyhst_plan &p)
{
    NormLayout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t r = o;
        o = align256(o + bytes);
        return r;
    };
    L.x = take((size_t)p.img_elems * 4);
    L.y = take((size_t)p.img_elems * 4);
    L.tmp = take((size_t)p.sino_elems * 4);
    L.partials = take(sizeof(double) * 1024);
    L.norm = take(sizeof(double) * 2);
    L.total = o;
    return L;
}

size_t fbp_work(const pyhst_plan &p, size_t base) { return base + align256((size_t)p.filt_elems * 4); }

// y = normalised (hot-spot filtered) data or a copy of sino, then the ring filter (with the
// thresholded object removed from its average when asked).
int enqueue_pre(const pyhst_plan &p, const pyhst_recon_args &a, const PreLayout &L, hipStream_t st)
{
    unsigned char *w = (unsigned char *)a.work;
    float *y = (float *)(w + L.y);
    hipError_t e;
    if (a.raw) {
        e = a.hot_spot ? launch_normalize_hotspot(p, a.raw, a.flats, a.flat_pos, a.n_flats, a.dark, a.eps,
                                                  a.hot_threshold, a.hot_halo_lo, a.hot_halo_hi, y, st)
                       : launch_normalize(p, a.raw, a.flats, a.flat_pos, a.n_flats, a.dark, a.eps, y, st);
    } else {
        e = launch_copy(y, a.sino, p.sino_elems, st);
    }
    if (e != hipSuccess) return hip_fail(e, "reconstruct_slices: preprocessing");
    if (a.ring_width > 0) {
        const float *obj = nullptr;
        if (a.ring_object) {
            float *filt = (float *)(w + L.filt), *img = (float *)(w + L.img), *ob = (float *)(w + L.obj);
            e = launch_filter(p, y, nullptr, nullptr, nullptr, 0, nullptr, 0.0f, filt, st);
            if (e == hipSuccess) e = launch_backproject(p, filt, 1, img, 1.0f, 0.0f, nullptr, st);
            if (e == hipSuccess) e = launch_threshold(img, img, p.img_elems, a.ring_threshold, st);
            if (e == hipSuccess) e = launch_forward(p, img, ob, 1.0f, nullptr, st);
            if (e != hipSuccess) return hip_fail(e, "reconstruct_slices: ring object");
            obj = ob;
        }
        e = launch_ring_filter(p, y, obj, a.ring_width, (double *)(w + L.ring), st);
        if (e != hipSuccess) return hip_fail(e, "reconstruct_slices: ring filter");
    }
    return PYHST_OK;
}

int enqueue_fbp(const pyhst_plan &p, const pyhst_recon_args &a, const PreLayout &PL, hipStream_t st)
{
    float *filt = (float *)((unsigned char *)a.work + PL.total);
    hipError_t e;
    if (PL.on) {
        int rc = enqueue_pre(p, a, PL, st);
        if (rc) return rc;
        e = launch_filter(p, (const float *)((unsigned char *)a.work + PL.y), nullptr, nullptr, nullptr, 0, nullptr,
                          0.0f, filt, st);
    } else {
        e = launch_filter(p, a.raw ? nullptr : a.sino, a.raw, a.flats, a.flat_pos, a.n_flats, a.dark, a.eps, filt,
                          st);
    }
    if (e != hipSuccess) return hip_fail(e, "reconstruct_slices: filter");
    e = launch_backproject(p, filt, 1, a.out, 1.0f, 0.0f, nullptr, st);
    if (e != hipSuccess) return hip_fail(e, "reconstruct_slices: backproject");
    return PYHST_OK;
}

// Chambolle-Pock for eq. (3) with K = [A; mu grad] (mu = 1: the plain operator), tau = sigma = 1/|K|.
// The dual field of the gradient block is kept as q~ = mu q, so its step is sigma mu^2 with the bound
// lambda and the primal step reads div q~ (the same iterates as the textbook form with q in
// [-lambda/mu, lambda/mu]).  With energy, A x_k is carried by linearity,
//   A x_k = (A xbar_k + A x_{k-1}) / 2   (xbar_k = 2 x_k - x_{k-1}),
// in the projector's epilogue, and E(x_k) is summed right after it; the last iterate gets one
// direct projection.
int enqueue_cp(const pyhst_plan &p, const pyhst_recon_args &a, const PreLayout &PL, const CpLayout &L,
               hipStream_t st)
{
    unsigned char *w = (unsigned char *)a.work;
    const float *y = PL.on ? (const float *)(w + PL.y) : a.raw ? (const float *)(w + L.y) : a.sino;
    float *x = a.out, *xbar = (float *)(w + L.xbar), *q1 = (float *)(w + L.q1), *q2 = (float *)(w + L.q2);
    float *pd = (float *)(w + L.p);
    float *ax = a.energy ? (float *)(w + L.ax) : nullptr;
    double *partials = (double *)(w + L.partials);
    const int64_t ni = p.img_elems, ns = p.sino_elems;
    const float s2 = (float)(p.gd[0].s * p.gd[0].s);
    const double mu = a.tv_mu > 0.0 ? a.tv_mu : 1.0;
    const float tau = (float)(1.0 / a.op_norm), sigma = (float)(1.0 / a.op_norm);
    const float sigma_q = (float)(mu * mu / a.op_norm);
    hipError_t e;
    if (PL.on) {
        int rc = enqueue_pre(p, a, PL, st);
        if (rc) return rc;
    } else if (a.raw) {
        e = launch_normalize(p, a.raw, a.flats, a.flat_pos, a.n_flats, a.dark, a.eps, (float *)(w + L.y), st);
        if (e != hipSuccess) return hip_fail(e, "reconstruct_slices: normalize");
    }
    for (float *b : {x, xbar, q1, q2}) {
        e = launch_fill(b, ni, 0.0f, st);
        if (e != hipSuccess) return hip_fail(e, "reconstruct_slices: fill");
    }
    e = launch_fill(pd, ns, 0.0f, st);
    if (e == hipSuccess && ax) e = launch_fill(ax, ns, 0.0f, st);
    if (e != hipSuccess) return hip_fail(e, "reconstruct_slices: fill");
    const int npart = energy_partials(p);
    for (int it = 0; it < a.n_iter; ++it) {
        CpDual dual{pd, y, sigma, 0, ax, 0.5f, 0.5f};
        e = launch_forward(p, xbar, nullptr, 1.0f, &dual, st);
        if (e != hipSuccess) return hip_fail(e, "reconstruct_slices: projector");
        if (ax && it > 0) {   // ax = A x_it, x = x_it: energy of iteration it - 1
            e = launch_cp_energy(p, ax, y, x, a.lambda, partials, npart, a.energy + it - 1, st);
            if (e != hipSuccess) return hip_fail(e, "reconstruct_slices: energy");
        }
        e = launch_cp_dual_q(p, xbar, q1, q2, sigma_q, a.lambda, st);
        if (e != hipSuccess) return hip_fail(e, "reconstruct_slices: tv dual");
        CpPrimal prim{x, xbar, q1, q2, tau};
        e = launch_backproject(p, pd, 0, nullptr, s2, 0.0f, &prim, st);
        if (e != hipSuccess) return hip_fail(e, "reconstruct_slices: backprojector");
    }
    if (ax && a.n_iter > 0) {
        e = launch_forward(p, x, ax, 1.0f, nullptr, st);
        if (e == hipSuccess) e = launch_cp_energy(p, ax, y, x, a.lambda, partials, npart, a.energy + a.n_iter - 1, st);
        if (e != hipSuccess) return hip_fail(e, "reconstruct_slices: energy");
    }
    return PYHST_OK;
}

// ISTA / FISTA (Beck & Teboulle 2009) with step 1/La, La = op_norm^2:
//   r = A z - y                       (projector, residual epilogue)
//   z <- z - (s^2/La) B r             (backprojector accumulating into z: the gradient step, in place)
//   x_k = prox_{(lambda/La) TV}(z)    (tv_prox, n_inner dual iterations from zero)
//   ISTA: z is x itself; FISTA: z = x_k + m_k (x_k - x_{k-1}) with the t_k sequence
// The iterates alternate between out and one work buffer; the last one is copied to out if needed.
// With energy, the projector's epilogue also carries A x_{k} = (A z + m A x_{k-1}) / (1 + m)
// (ISTA: A x_k = A z), and E(x_k) is summed right after it; the last iterate gets one direct
// projection.
int enqueue_fista(const pyhst_plan &p, const pyhst_recon_args &a, const PreLayout &PL, const FiLayout &L,
                  hipStream_t st)
{
    unsigned char *w = (unsigned char *)a.work;
    const bool fast = a.method == PYHST_FISTA;
    const float *y = PL.on ? (const float *)(w + PL.y) : a.raw ? (const float *)(w + L.y) : a.sino;
    float *r = (float *)(w + L.r), *z = (float *)(w + L.z);
    float *ax = a.energy ? (float *)(w + L.ax) : nullptr;
    float *xa = a.out, *xb = (float *)(w + L.xb), *prox = (float *)(w + L.prox);
    double *partials = (double *)(w + L.partials);
    const GeoDev &g = p.gd[0];
    const int64_t ni = p.img_elems, ns = p.sino_elems;
    const double La = a.op_norm * a.op_norm;
    const float s2 = (float)(g.s * g.s);
    const float step = (float)(-(double)s2 / La);
    const float plam = (float)((double)a.lambda / La);
    hipError_t e;
    if (PL.on) {
        int rc = enqueue_pre(p, a, PL, st);
        if (rc) return rc;
    } else if (a.raw) {
        e = launch_normalize(p, a.raw, a.flats, a.flat_pos, a.n_flats, a.dark, a.eps, (float *)(w + L.y), st);
        if (e != hipSuccess) return hip_fail(e, "reconstruct_slices: normalize");
    }
    e = launch_fill(xa, ni, 0.0f, st);
    if (e == hipSuccess && fast) e = launch_fill(z, ni, 0.0f, st);
    if (e == hipSuccess && ax) e = launch_fill(ax, ns, 0.0f, st);
    if (e != hipSuccess) return hip_fail(e, "reconstruct_slices: fill");
    const int npart = energy_partials(p);
    double t = 1.0, m = 0.0;   // m: momentum that made the current z
    for (int it = 0; it < a.n_iter; ++it) {
        float *zin = fast ? z : xa;
        CpDual res{r, y, 0.0f, 1, ax, (float)(1.0 / (1.0 + m)), (float)(m / (1.0 + m))};
        e = launch_forward(p, zin, nullptr, 1.0f, &res, st);
        if (e != hipSuccess) return hip_fail(e, "reconstruct_slices: projector");
        if (ax && it > 0) {   // ax = A x_it and xa = x_it: energy of iteration it - 1
            e = launch_cp_energy(p, ax, y, xa, a.lambda, partials, npart, a.energy + it - 1, st);
            if (e != hipSuccess) return hip_fail(e, "reconstruct_slices: energy");
        }
        e = launch_backproject(p, r, 0, zin, step, 1.0f, nullptr, st);
        if (e != hipSuccess) return hip_fail(e, "reconstruct_slices: backprojector");
        float *dst = fast ? xb : xa;
        e = launch_tv_prox(p.n_slices, g.ny, g.nx, zin, dst, plam, a.n_inner, prox, st);
        if (e != hipSuccess) return hip_fail(e, "reconstruct_slices: tv prox");
        if (fast) {
            const double tn = 0.5 * (1.0 + std::sqrt(1.0 + 4.0 * t * t));
            m = (double)(float)((t - 1.0) / tn);
            e = launch_momentum(z, xb, xa, ni, (float)m, st);
            if (e != hipSuccess) return hip_fail(e, "reconstruct_slices: momentum");
            t = tn;
            std::swap(xa, xb);   // xa = x_k
        }
    }
    if (ax && a.n_iter > 0) {
        e = launch_forward(p, xa, ax, 1.0f, nullptr, st);
        if (e == hipSuccess) e = launch_cp_energy(p, ax, y, xa, a.lambda, partials, npart, a.energy + a.n_iter - 1, st);
        if (e != hipSuccess) return hip_fail(e, "reconstruct_slices: energy");
    }
    if (xa != a.out) {
        e = launch_copy(a.out, xa, ni, st);
        if (e != hipSuccess) return hip_fail(e, "reconstruct_slices: copy");
    }
    return PYHST_OK;
}

// |[A; mu grad]| (with_grad) or |A| by power iteration on K^T K or A^T A (synchronises the stream once).
int estimate_opnorm(const pyhst_plan &p, const NormLayout &L, unsigned char *w, int with_grad, double mu,
                    hipStream_t st, double *out)
{
    const int64_t ni = p.img_elems;
    float *x = (float *)(w + L.x), *y = (float *)(w + L.y), *tmp = (float *)(w + L.tmp);
    double *partials = (double *)(w + L.partials), *nrm = (double *)(w + L.norm);
    // constant start: the leading eigenvector of K^T K (dominated by A^T A) is smooth and positive
    hipError_t e = launch_fill(x, ni, 1.0f, st);
    double sq = 0.0;
    for (int it = 0; it < 50 && e == hipSuccess; ++it) {
        e = launch_power_step(p, x, y, tmp, partials, energy_partials(p), nrm, with_grad ? (float)(mu * mu) : 0.0f,
                              st);
        if (e == hipSuccess) e = launch_scale_by_inv(y, ni, nrm, st);
        std::swap(x, y);
    }
    if (e != hipSuccess) return hip_fail(e, "opnorm: power iteration");
    e = hipMemcpyAsync(&sq, nrm, sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "opnorm: power iteration");
    if (!(sq > 0.0) || !std::isfinite(sq)) return fail(PYHST_ENUM, "opnorm: operator norm estimate failed");
    *out = 1.02 * std::sqrt(std::sqrt(sq));   // |K^T K x| -> |K|^2; 2 % margin keeps tau sigma |K|^2 < 1
    return PYHST_OK;
}

}  // namespace

extern "C" int pyhst_opnorm(const pyhst_plan *p, int32_t with_grad, double mu, void *work, size_t *work_bytes,
                            double *norm, hipStream_t st)
{
    if (!p || !work_bytes) return fail(PYHST_EARG, "opnorm: NULL argument");
    if (!p->uniform) return fail(PYHST_EARG, "opnorm: needs a uniform plan");
    const NormLayout L = norm_layout(*p);
    if (!work) {
        *work_bytes = L.total;
        return PYHST_OK;
    }
    if (!norm) return fail(PYHST_EARG, "opnorm: NULL norm");
    if (!std::isfinite(mu)) return fail(PYHST_EARG, "opnorm: mu must be finite");
    if (*work_bytes < L.total) {
        set_error("opnorm: work buffer too small");
        return PYHST_ENOMEM;
    }
    return estimate_opnorm(*p, L, (unsigned char *)work, with_grad ? 1 : 0, mu > 0.0 ? mu : 1.0, st, norm);
}

extern "C" int reconstruct_slices(const pyhst_plan *pc, pyhst_recon_args *a, hipStream_t st)
{
    if (!pc || !a) return fail(PYHST_EARG, "reconstruct_slices: NULL argument");
    const pyhst_plan &p = *pc;
    if (a->method != PYHST_FBP && a->method != PYHST_TV_CP && a->method != PYHST_ISTA && a->method != PYHST_FISTA)
        return fail(PYHST_EARG, "reconstruct_slices: bad method");
    if (!a->raw && !a->sino) return fail(PYHST_EARG, "reconstruct_slices: need raw or sino");
    const bool cp = a->method == PYHST_TV_CP;
    const bool fi = a->method == PYHST_ISTA || a->method == PYHST_FISTA;
    const bool iterative = cp || fi;
    if (iterative) {
        if (!p.uniform) return fail(PYHST_EARG, "reconstruct_slices: TV needs a uniform plan");
        if (a->n_iter < 0 || !(a->lambda >= 0.0f)) return fail(PYHST_EARG, "reconstruct_slices: bad n_iter/lambda");
        if (fi && a->n_inner < 0) return fail(PYHST_EARG, "reconstruct_slices: bad n_inner");
        if (!std::isfinite(a->tv_mu)) return fail(PYHST_EARG, "reconstruct_slices: tv_mu must be finite");
    }
    if (a->ring_width < 0) return fail(PYHST_EARG, "reconstruct_slices: ring_width must be >= 0");
    if (a->hot_spot && !a->raw) return fail(PYHST_EARG, "reconstruct_slices: the hot-spot filter needs raw input");
    if (a->hot_spot && !(a->hot_threshold >= 0.0f))
        return fail(PYHST_EARG, "reconstruct_slices: hot_threshold must be >= 0");
    if (a->hot_halo_lo < 0 || a->hot_halo_lo > 1 || a->hot_halo_hi < 0 || a->hot_halo_hi > 1 ||
        ((a->hot_halo_lo || a->hot_halo_hi) && !a->hot_spot))
        return fail(PYHST_EARG, "reconstruct_slices: halo rows (0 or 1 per side) need the hot-spot filter");
    const PreLayout PL = pre_layout(p, *a);
    if (PL.on && !p.uniform) return fail(PYHST_EARG, "reconstruct_slices: preprocessing needs a uniform plan");
    CpLayout L{};
    FiLayout F{};
    size_t need;
    if (cp) {
        L = cp_layout(p, *a, PL.total, a->raw && !PL.on);
        need = L.total;
    } else if (fi) {
        F = fista_layout(p, *a, PL.total, a->raw && !PL.on);
        need = F.total;
    } else {
        need = fbp_work(p, PL.total);
    }
    if (!a->out) {
        a->work_bytes = need;
        return PYHST_OK;
    }
    if (a->raw) {
        if (!p.uniform) return fail(PYHST_EARG, "reconstruct_slices: raw radiographs need a uniform plan");
        if (!a->flats || !a->flat_pos || !a->dark || a->n_flats < 1 || a->n_flats > 32)
            return fail(PYHST_EARG, "reconstruct_slices: raw input needs 1..32 flats, positions and a dark");
        for (int i = 1; i < a->n_flats; ++i)
            if (!(a->flat_pos[i] > a->flat_pos[i - 1]))
                return fail(PYHST_EARG, "reconstruct_slices: flat positions must increase");
    }
    if (iterative && !(a->op_norm > 0.0 && std::isfinite(a->op_norm)))
        return fail(PYHST_EARG, "reconstruct_slices: iterative methods need op_norm > 0 (see pyhst_opnorm)");
    if (!a->work || a->work_bytes < need) {
        set_error("reconstruct_slices: work buffer too small");
        return PYHST_ENOMEM;
    }

    // graphs are captured on the caller's stream; the legacy null stream cannot be captured
    const bool graphable = a->use_graph && st != nullptr;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (graphable) {
        hipError_t e = hipStreamIsCapturing(st, &cs);
        if (e != hipSuccess) return hip_fail(e, "reconstruct_slices: hipStreamIsCapturing");
    }
    auto enqueue = [&]() {
        return cp ? enqueue_cp(p, *a, PL, L, st) : fi ? enqueue_fista(p, *a, PL, F, st) : enqueue_fbp(p, *a, PL, st);
    };

    if (graphable && cs == hipStreamCaptureStatusNone) {
        std::vector<uint64_t> key = {(uint64_t)a->method, (uint64_t)(uintptr_t)a->raw, (uint64_t)(uintptr_t)a->sino,
                                     (uint64_t)(uintptr_t)a->flats, (uint64_t)(uintptr_t)a->dark,
                                     (uint64_t)(uintptr_t)a->out, (uint64_t)(uintptr_t)a->work,
                                     (uint64_t)(uintptr_t)a->energy,
                                     (uint64_t)a->n_flats, (uint64_t)a->n_iter, (uint64_t)(uintptr_t)st,
                                     (uint64_t)(fi ? a->n_inner : 0), (uint64_t)a->hot_spot,
                                     (uint64_t)a->ring_width, (uint64_t)a->ring_object,
                                     (uint64_t)a->hot_halo_lo, (uint64_t)a->hot_halo_hi};
        for (float f : {a->hot_threshold, a->ring_threshold, a->lambda, a->eps}) {
            uint32_t fb;
            std::memcpy(&fb, &f, 4);
            key.push_back(fb);
        }
        for (double d : {iterative ? a->op_norm : 0.0, cp ? a->tv_mu : 0.0}) {
            uint64_t db;
            std::memcpy(&db, &d, 8);
            key.push_back(db);
        }
        if (a->raw)
            for (int i = 0; i < a->n_flats; ++i) {
                uint64_t fb;
                std::memcpy(&fb, &a->flat_pos[i], 8);
                key.push_back(fb);
            }
        std::unique_lock<std::mutex> lk(p.mu);
        auto it = p.graphs.find(key);
        if (it == p.graphs.end() && p.graphs.size() >= (size_t)PYHST_MAX_GRAPHS) {
            // bounded cache: a further distinct call runs as plain launches (cached graphs may still be
            // in flight on other streams, so none is destroyed here)
            lk.unlock();
            return enqueue();
        }
        if (it == p.graphs.end()) {
            hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess) return hip_fail(e, "reconstruct_slices: begin capture");
            int rc = enqueue();
            hipGraph_t graph = nullptr;
            e = hipStreamEndCapture(st, &graph);
            if (rc) {
                if (graph) (void)hipGraphDestroy(graph);
                return rc;
            }
            if (e != hipSuccess) return hip_fail(e, "reconstruct_slices: end capture");
            hipGraphExec_t exec = nullptr;
            e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (e != hipSuccess) return hip_fail(e, "reconstruct_slices: instantiate");
            it = p.graphs.emplace(key, exec).first;
        }
        hipError_t e = hipGraphLaunch(it->second, st);
        return e == hipSuccess ? PYHST_OK : hip_fail(e, "reconstruct_slices: graph launch");
    }
    return enqueue();
}

// ---- allocation-free variant ----------------------------------------------------------------
// Scratch of reconstruct_slices_static: one copy per device in the code object.  In host code the
// name is only a stand-in; the device address of each device's copy comes from hipGetSymbolAddress
// (first call on that device, with it current) and only that address reaches kernels.
static __device__ __align__(256) unsigned char scratch[PYHST_STATIC_SCRATCH_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[MAX_DEVICES] = {};

int device_scratch(int dev, void **out)
{
    if (dev < 0 || dev >= MAX_DEVICES) return fail(PYHST_EARG, "reconstruct_slices_static: device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "reconstruct_slices_static: hipGetSymbolAddress");
        if (!ptr) return fail(PYHST_EHIP, "reconstruct_slices_static: no device address for the scratch array");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return PYHST_OK;
}
}  // namespace

extern "C" int reconstruct_slices_static(const pyhst_plan *pc, pyhst_recon_args *a, hipStream_t st)
{
    if (!pc || !a) return fail(PYHST_EARG, "reconstruct_slices_static: NULL argument");
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "reconstruct_slices_static: hipGetDevice");
    if (dev != pc->device) return fail(PYHST_EARG, "reconstruct_slices_static: the plan's device must be current");
    pyhst_recon_args q = *a;
    q.out = nullptr;   // size query: validates the method and fills work_bytes, enqueues nothing
    q.work = nullptr;
    q.work_bytes = 0;
    int rc = reconstruct_slices(pc, &q, st);
    if (rc) return rc;
    a->work_bytes = q.work_bytes;
    if (q.work_bytes > (size_t)PYHST_STATIC_SCRATCH_BYTES)
        return fail(PYHST_ENOMEM, "reconstruct_slices_static: the call needs " + std::to_string(q.work_bytes) +
                                      " bytes of scratch, more than the static " +
                                      std::to_string((size_t)PYHST_STATIC_SCRATCH_BYTES) +
                                      " bytes; use reconstruct_slices with a work buffer");
    if (!a->out) return PYHST_OK;
    void *ptr = nullptr;
    rc = device_scratch(dev, &ptr);
    if (rc) return rc;
    q = *a;
    q.work = ptr;
    q.work_bytes = (size_t)PYHST_STATIC_SCRATCH_BYTES;
    q.use_graph = 0;
    return reconstruct_slices(pc, &q, st);
}
