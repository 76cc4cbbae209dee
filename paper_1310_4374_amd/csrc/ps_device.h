// Device-side descriptors shared by the kernels and the host orchestration.
#pragma once
#include <cstdint>

namespace ps {

constexpr int kTile = 256;         // sources staged per LDS tile
constexpr int kGroup = 32;         // sources per near/far decision
// A source is "far" for a target block of radius rT (about its centre c) when it
// lies farther than kFarFactor * rT from c, and a group is far when all of its
// sources are (both pair kernels).  A far
// pair is then more than (kFarFactor - 1) rT apart, and the sum of the two
// points' distances from c is at most (kFarFactor + 1)/(kFarFactor - 1) times
// their separation.  That ratio (5 at 1.5) bounds the one-float coordinate
// error relative to the separation, and its square the cancellation in the
// expanded r^2 = |t|^2 + |s|^2 - 2 t.s, in units of the rounding.
constexpr double kFarFactor = 1.5;
// The plane's -log r turns a relative error of r^2 into an absolute error of the
// term (the log of the expanded r^2 carries it unscaled), so its FP32 kernels take
// far groups only beyond 3 rT: ratio 2, cancellation at most 4 roundings.  At the
// particle counts the plane is used with, blocks are small against the near
// radius and the share of near groups barely moves.
constexpr double kFarFactorPlane = 3.0;
template <int KERN>
constexpr double far_factor() { return KERN == 2 ? kFarFactorPlane : kFarFactor; }
// -ln(2)/2: the plane's potential term -log(r) = kLog2Half log2(r^2)
constexpr double kLog2Half = -0.34657359027997265471;
// Waves per workgroup of the FP32 check-point sums (k_chk_f32): they share one
// block of 64 targets and split each staged source tile between them.
constexpr int kChkWaves = 4;
constexpr int kChunk = 1024;       // particles per chunk in the per-particle kernels
// Lanes per target in the far-field/combine kernel: 8 when a shape has at most
// kFarWideMax targets in all (spreading each target's work wider shortens a
// small solve), else 4 (fewer lanes read the split partials of large ones).
constexpr int64_t kFarWideMax = 65536;
// Box mean by corners (k_mean_corners): one wave per kMeanWave particles keeps,
// per (x, y) image column, a bit mask of the particle's near images along z in
// LDS; a system qualifies when it has at most kMeanCols columns and kMeanZ
// images per column (else the per-entry kernel k_mean serves it).
constexpr int kMeanWave = 64;
constexpr int kMeanCols = 64;
constexpr int kMeanZ = 31;
// The corner columns of a chunk are split over up to (x range + 1) waves so
// that a launch reaches about kMeanTargetWaves waves; a launch that would
// still have fewer than kMeanMinWaves takes the per-entry kernel (a handful of
// long waves is slower than many short lanes).
constexpr int64_t kMeanTargetWaves = 4096;
constexpr int64_t kMeanMinWaves = 2048;

// One periodic system (a box with its particles).  Offsets index packed arrays.
struct SysDev {
    double box[3], half[3], inv_cell[3];
    double R0, inv_R0, thr, V0;
    int g[3], gbits;
    int p, P, L, nimg;
    int mean_mode, basis;        // basis: 0 spherical harmonics, 1 RBF centres
    int M, dim;                  // RBF: number of centres (P = M + 1); dim: 3, or 2 (the plane: every z is 0,
                                 // basis 1, Re w^n, Im w^n, P = 2p - 1, box mean over the rectangle)
    int64_t cen_off;             // RBF: centres in the packed SoA arrays
    int64_t n_off, n;            // particles in the packed input / sorted arrays
    int64_t cell_off, ncell;     // cell counters (ncell + 1 entries)
    int64_t near_off, near_cap;  // near list
    int64_t img_off;             // images, 3 doubles each
    int64_t chk_off;             // 2L check targets (first L: y_l, then y~_l)
    int64_t pinv_off;            // (P-1) x L
    int64_t coef_off;            // P coefficients; coef[0] holds C1
    int64_t bm_off;              // P box means R_t^(0)
    int64_t rec_off;             // recurrence tables: a[P], b[P], c[p]
    int64_t inv_off;             // inverse near map: nimg x n (entry index or -1)
    int64_t nitem_begin, nitem_end;  // near-build items of this system
    int64_t f_off;               // L right-hand-side values
    int64_t witem_off, witem_n;  // this system's workgroups in the near-size-weighted item table
    int mr[3], mcorner;          // box mean by corners: image ranges |i_k| <= mr[k]; 1 if used
    int64_t imap_off;            // dense image map over the ranges (image index or -1)
    int64_t mitem_off, mitem_n;  // this system's workgroups of the corner box mean
    int periodic;                // periodic axes: 7 (x, y, z), 3 (x, y: a slab) or 1 (x: a wire)
    int Lf;                      // rows of the fit: L periodicity rows, then ndec decay rows (slab, wire)
    int ndec, m2;                // decay rows; points per decay surface (slab: two planes, top first;
                                 // wire: one cylinder, x-major)
    int64_t dec_off;             // decay-surface points in the packed SoA arrays (nsurf m2 per system)
    int64_t dw_off;              // their quadrature weights (m2, shared by the surfaces)
    int64_t drow_off;            // decay rows, 5 doubles each (slab: kx, ky, |k|, s, trig;
                                 // wire: k, m, beta, trig in x, trig in theta)
    int kernel, nsurf;           // kernel: 0 Coulomb 1/r; 1 screened exp(-kappa r)/r (no neutrality, no C1);
                                 // 2 the plane's -log r;
                                 // nsurf: decay surfaces (2 slab, 1 wire, 0 otherwise)
    double kappa;                // screening constant (screened kernel)
};

// A pair-sum job: every target of a set against every source of another.
struct PJob {
    const double* tx;
    const double* ty;
    const double* tz;
    int64_t nt;
    const double* sx;
    const double* sy;
    const double* sz;
    const double* sq;
    const int64_t* ns_dev;  // device source count (or null)
    int64_t ns_host;        // host source count when ns_dev is null
    double* tblk;           // 4 doubles per target block: centre xyz, radius
    double* part;           // partial sums [nsplit][ncomp][nt]
    int nsplit, ncomp, bt, pad;
    double kappa;           // screened kernel: exp(-kappa r)/r (0 for the Coulomb kernel)
};

struct PItem { int job, tb, split, pad; };           // one workgroup of a pair sum
struct TItem { int job, tb; };                       // one target block
struct CItem { int sys, count; int64_t start; };     // a chunk of a system's particles
struct MItem { int sys, count; int64_t start; int ax0, ax1; };  // corner box mean: a chunk, corner columns ax0..ax1
struct NItem { int sys, img; int64_t start; int count, pad; };  // near-build item

}  // namespace ps
