// Internal declarations shared by the host plan code and the kernel
// translation units of the gfx950 reconstruction library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "pyhst.h"

namespace pyhst {

// Backprojector tile configurations.  A workgroup is 4 wavefronts per angle
// group; each lane owns one pixel of every 8x8 block its wave covers; a wave
// covers BX x BY blocks, the 4 waves are stacked in y.  Tile = (8 BX) x (32 BY)
// pixels.  With AG > 1 angle groups (workgroup = 256 AG threads) each group sums
// its share of the projections and the shares are added in a fixed order: for
// slices too small to fill the chip with tiles alone.
constexpr int N_TILE_CFG = 6;
constexpr int TILE_BX[N_TILE_CFG] = {8, 8, 4, 4, 8, 4};
constexpr int TILE_BY[N_TILE_CFG] = {2, 1, 2, 1, 4, 1};
constexpr int TILE_AG[N_TILE_CFG] = {1, 1, 1, 1, 1, 4};
inline constexpr int tile_w(int c) { return 8 * TILE_BX[c]; }
inline constexpr int tile_h(int c) { return 32 * TILE_BY[c]; }

// Floats per projection in the backprojection scalar table:
// [0] s cos, [1] s sin, [2 + 8 by + bx] = 8 s (bx cos + by sin), bx < 8, by < 4.
constexpr int BPT = 36;

// One slice geometry, as the kernels read it (device memory, read-only).
struct GeoDev {
    int32_t nx, ny, nb, K;
    int32_t Lf, fpad;         // filtered-row layout: length, zero bins prepended
    int32_t P, log2P;         // FFT length of the ramp filter (P >= 2 Lf - 1)
    double s;                 // pixel size in bins
    double axis, axis_f;      // axis position: detector layout, filtered layout
    int64_t ang_off;          // first projection of this geometry in the per-angle tables
    int64_t hw_off;           // first element of its half-acquisition weights [Lf]
    int64_t spec_off;         // first element of its filter spectrum [P] (bit-reversed order, 1/P folded)
    int32_t bp_w[N_TILE_CFG]; // LDS window length (bins) per tile configuration
    int32_t ntx[N_TILE_CFG];  // tiles along x per tile configuration
    int32_t fp_blk_off;       // first forward-projection angle block of this geometry
    int32_t fp_nblk;          // its number of angle blocks
    int32_t fp_pair_off;      // first staged-projector group (one to FP_SGRP projections) of this geometry
    int32_t fp_npair;         // its number of staged-projector groups
    int32_t half, pad2;       // 1: 360-degree half acquisition (weights other than 1 in the filter load)
};

// Forward projection: projections of one geometry grouped into blocks of at most FP_AMAX
// whose staged line segments share one LDS segment of FP_SEG positions (see k_fp.hip).
constexpr int FP_RB = 16, FP_AMAX = 16;
int fp_seg_len(double s_min);
// Staged projector (one workgroup per group of one to FP_SGRP projections and 64 bins): positions
// staged per line for 3 and for 6 candidates per line.
constexpr int FP_SSEG3 = 128, FP_SSEG6 = 224, FP_SGRP = 4;
// candidates per line for the smallest pixel size s_min: 3, 6, or 0 (counted at run time)
int fp_nc_for(double s_min);

struct SliceDev {
    int32_t g, pad;
    int64_t sino_off, filt_off, img_off;
};

struct Tables {
    const GeoDev *geo;
    const SliceDev *slc;
    const double *cosd, *sind, *shiftd;  // [sum K]
    const float *bpt;                    // [sum K][BPT]
    const float *wang;                   // [sum K] quadrature weights
    const float *haw;                    // half-acquisition weights
    const float *spec;                   // filter spectra
    const float2 *twid;                  // exp(-2 pi i m / Pmax), m < Pmax/2
    const int2 *pairs;                   // filter work: (slice, first projection of a row pair)
    const int2 *items[N_TILE_CFG];       // backprojection work: (slice, tile), costliest first
    int *counter;                        // persistent work counters [PYHST_MAX_STREAMS]
    const int *fp_ang;                   // forward-projection block members: projection index within its geometry
    const int2 *fp_blk;                  // forward-projection blocks: (first member, count)
    const int4 *fp_pair;                 // staged-projector groups: up to FP_SGRP projections, -1 for none
    int32_t Pmax, log2Pmax;
};

struct GeoHost {
    pyhst_geom g;
    std::vector<double> ang, shift;
    double s;
    int Lf, fpad;
    double axis_f;
    int P, log2P;
    std::vector<double> w;      // angle weights
    std::vector<double> haw;    // [Lf]
};

}  // namespace pyhst

struct pyhst_plan {
    int device = 0;
    int n_geom = 0, n_slices = 0;
    bool uniform = true;
    std::vector<pyhst::GeoHost> gh;
    std::vector<pyhst::GeoDev> gd;
    std::vector<pyhst::SliceDev> sd;
    int64_t sino_elems = 0, filt_elems = 0, img_elems = 0;
    int64_t max_K = 0;
    int n_pairs = 0;
    int fp_seg = 0, fp_max_blocks = 0, fp_max_pairs = 0, fp_max_grp = 1;
    int64_t n_items[pyhst::N_TILE_CFG] = {};
    int bp_tile = -1, persistent = 0;
    int bp_slices = 0;   // slices per backprojector workgroup: 0 automatic, 1, 2
    int fp_kernel = PYHST_FP_AUTO;
    void *dev_block = nullptr;
    pyhst::Tables t{};
    int cu_count = 256;
    // caches filled by const entry points (guarded by mu)
    mutable std::mutex mu;
    mutable std::map<std::vector<uint64_t>, hipGraphExec_t> graphs;
    // persistent-work counter of each stream, under its own lock: a graph capture runs with mu held and
    // takes a counter slot inside it
    mutable std::mutex counter_mu;
    mutable std::map<hipStream_t, int> counter_slot;
};

namespace pyhst {

// thread-local error message
void set_error(const std::string &msg);
int fail(int code, const std::string &msg);
int hip_fail(hipError_t e, const char *where);

int choose_tile(const pyhst_plan &p);
// whether plain backprojections (no fused primal step) of this plan run two slices per workgroup
bool two_slice_bp(const pyhst_plan &p);
// persistent-work counter of `st` on this plan (nullptr once every slot is taken)
int *stream_counter(const pyhst_plan &p, hipStream_t st);

// CP epilogues
struct CpPrimal {   // x+ = x - tau (alpha B p - div q); xbar = 2 x+ - x
    float *x, *xbar;
    const float *q1, *q2;
    float tau;
};
struct CpDual {     // p = (p + sigma (alpha A xbar - y)) / (1 + sigma);  residual != 0: p = alpha A xbar - y
    float *p;
    const float *y;
    float sigma;
    int residual;
    float *ax;      // optional: ax = ax_a (alpha A xbar) + ax_b ax
    float ax_a, ax_b;
};

// launchers (return hipGetLastError())
hipError_t launch_normalize(const pyhst_plan &p, const uint16_t *raw, const float *flats, const double *flat_pos,
                            int n_flats, const float *dark, float eps, float *sino, hipStream_t st);
hipError_t launch_normalize_hotspot(const pyhst_plan &p, const uint16_t *raw, const float *flats,
                                    const double *flat_pos, int n_flats, const float *dark, float eps, float thr,
                                    int halo_lo, int halo_hi, float *sino, hipStream_t st);
hipError_t launch_ring_filter(const pyhst_plan &p, float *sino, const float *obj, int width, double *work,
                              hipStream_t st);
hipError_t launch_threshold(float *dst, const float *src, int64_t n, float thr, hipStream_t st);
hipError_t launch_filter(const pyhst_plan &p, const float *sino, const uint16_t *raw, const float *flats,
                         const double *flat_pos, int n_flats, const float *dark, float eps, float *filt,
                         hipStream_t st);
hipError_t launch_backproject(const pyhst_plan &p, const float *sino, int filtered, float *img, float alpha,
                              float beta, const CpPrimal *cp, hipStream_t st);
hipError_t launch_forward(const pyhst_plan &p, const float *img, float *sino, float alpha, const CpDual *cp,
                          hipStream_t st);
hipError_t launch_forward_row(const pyhst_plan &p, const float *img, const float *y, int k, float *row,
                              hipStream_t st);

// TV / CP helpers (k_tv.hip); images are packed by the plan's img offsets when a plan is given,
// otherwise a plain [S][ny][nx] stack.
hipError_t launch_tv_prox(int S, int ny, int nx, const float *in, float *out, float lambda, int n_inner,
                          float *work, hipStream_t st);
hipError_t launch_cp_dual_q(const pyhst_plan &p, const float *xbar, float *q1, float *q2, float sigma,
                            float lambda, hipStream_t st);
hipError_t launch_fill(float *buf, int64_t n, float v, hipStream_t st);
hipError_t launch_cp_energy(const pyhst_plan &p, const float *ax, const float *y, const float *x, float lambda,
                            double *partials, int n_part, float *energy_dev, hipStream_t st);
int energy_partials(const pyhst_plan &p);
hipError_t launch_axpby(float *y, const float *x, int64_t n, float a, float b, hipStream_t st);
hipError_t launch_power_step(const pyhst_plan &p, const float *x, float *out, float *tmp_sino,
                             double *partials, int n_part, double *norm_dev, float grad_scale, hipStream_t st);
hipError_t launch_momentum(float *z, const float *xn, const float *xo, int64_t n, float m, hipStream_t st);
hipError_t launch_copy(float *dst, const float *src, int64_t n, hipStream_t st);
hipError_t launch_scale_by_inv(float *x, int64_t n, const double *norm_dev, hipStream_t st);

}  // namespace pyhst
