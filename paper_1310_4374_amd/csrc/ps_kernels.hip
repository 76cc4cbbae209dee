// HIP kernels (gfx950) of the periodized Coulomb sum, algorithm "get" (Sec. 2.3).
//
// Data layout in HBM: structure-of-arrays FP64 for positions, charges, the near
// list and all outputs; partial sums of the pair kernels as [split][component][target].
// Every kernel takes its work from small descriptor tables (SysDev, PJob, items),
// so one launch serves one box or a batch of boxes.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "ps_device.h"
#include "ps_kernels.h"

namespace ps {

// ----------------------------------------------------------------------------
// deterministic reductions (fixed order for a given launch shape)
// ----------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_min(double v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ double wave_max(double v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ int64_t wave_sum_i64(int64_t v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Block-wide reductions; the result is valid in every thread.  `sh` needs
// blockDim/64 entries.  All threads of the block must call them.
template <int OP>
__device__ double block_reduce(double v, double* sh)
{
    v = OP == 0 ? wave_sum(v) : (OP == 1 ? wave_min(v) : wave_max(v));
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[w] = v;
    __syncthreads();
    double r = sh[0];
    for (int i = 1; i < nw; ++i) r = OP == 0 ? r + sh[i] : (OP == 1 ? fmin(r, sh[i]) : fmax(r, sh[i]));
    return r;
}

// Block-wide int64 sum, valid in every thread (same contract as block_reduce).
__device__ int64_t block_sum_i64(int64_t v, int64_t* sh)
{
    v = wave_sum_i64(v);
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[w] = v;
    __syncthreads();
    int64_t r = 0;
    for (int i = 0; i < nw; ++i) r += sh[i];
    return r;
}

// Exclusive block scan of one int64 per thread (blockDim <= 1024); returns the
// exclusive prefix, and the block total in *total.
__device__ int64_t block_exclusive_scan(int64_t v, int64_t* sh, int64_t* total)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    int64_t x = v;
    for (int o = 1; o < 64; o <<= 1) {
        const int64_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    __syncthreads();
    if (lane == 63) sh[w] = x;
    __syncthreads();
    int64_t base = 0, tot = 0;
    for (int i = 0; i < nw; ++i) {
        if (i < w) base += sh[i];
        tot += sh[i];
    }
    *total = tot;
    return base + x - v;
}

// ----------------------------------------------------------------------------
// utilities
// ----------------------------------------------------------------------------
__global__ void k_fill_i32(int* p, int64_t n, int v)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

// Neutrality (eq. (1)) and box membership of every particle: partial sums of
// q and |q| per workgroup (grid: blocks x systems), then a per-system check.
__global__ __launch_bounds__(256) void k_validate(const SysDev* __restrict__ sys, const double* __restrict__ X,
                                                  const double* __restrict__ Y, const double* __restrict__ Z,
                                                  const double* __restrict__ Q, int* status, double* __restrict__ part)
{
    __shared__ double sh[4];
    const SysDev& S = sys[blockIdx.y];
    double sq = 0.0, sa = 0.0, bad = 0.0;
    for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < S.n; i += (int64_t)gridDim.x * 256) {
        const int64_t k = S.n_off + i;
        const double q = Q[k];
        sq += q;
        sa += fabs(q);
        const double x = X[k], y = Y[k], z = Z[k];
        const bool in = x >= -S.half[0] && x < S.half[0] && y >= -S.half[1] && y < S.half[1] && z >= -S.half[2] &&
                        z < S.half[2] && q == q;
        if (!in) bad = 1.0;
    }
    sq = block_reduce<0>(sq, sh);
    sa = block_reduce<0>(sa, sh);
    bad = block_reduce<2>(bad, sh);
    if (threadIdx.x == 0) {
        double* o = part + 2 * ((int64_t)blockIdx.y * gridDim.x + blockIdx.x);
        o[0] = sq;
        o[1] = sa;
        if (bad > 0.0) atomicOr(status, 2);
    }
}

// One wave per system: lane-strided partial sums, then a butterfly (fixed order).
// The screened kernel's lattice sum converges for any net charge.
__global__ __launch_bounds__(64) void k_validate_final(const SysDev* __restrict__ sys, const double* __restrict__ part,
                                                       int nblk, int* status)
{
    double sq = 0.0, sa = 0.0;
    const double* o = part + 2 * (int64_t)blockIdx.x * nblk;
    for (int b = threadIdx.x; b < nblk; b += 64) {
        sq += o[2 * b];
        sa += o[2 * b + 1];
    }
    sq = wave_sum(sq);
    sa = wave_sum(sa);
    if (threadIdx.x == 0 && sys[blockIdx.x].kernel != 1 && !(fabs(sq) <= 1e-12 * sa)) atomicOr(status, 1);
}

// ----------------------------------------------------------------------------
// spatial ordering: counting sort of particles by the Hilbert index of their
// cell, with each cell's entries put back in index order (deterministic result)
// ----------------------------------------------------------------------------
// Hilbert index of cell c on the 2^b grid of n axes (3, or 2 in the plane):
// Skilling's transform of the axes to the transposed index ("Programming the
// Hilbert curve", 2004), then its bits interleaved from the top.  Consecutive
// indices are face-adjacent cells, so BT consecutive particles stay compact;
// the Morton order jumps across the box at its octant boundaries, which left a
// few target blocks 4-5 times wider than the rest (measured on 1e5 uniform
// particles in 256-target blocks: largest block radius 0.70 against 0.18, and
// the sum of the radii cubed, which sets the near-form work, 3.3 against 1.1).
__device__ __forceinline__ uint32_t hilbert_key(uint32_t c[3], int n, int b)
{
    if (b == 0) return 0u;
    const uint32_t M = 1u << (b - 1);
    for (uint32_t Q = M; Q > 1u; Q >>= 1) {
        const uint32_t P = Q - 1u;
        for (int i = 0; i < n; ++i) {
            if (c[i] & Q) {
                c[0] ^= P;
            } else {
                const uint32_t t = (c[0] ^ c[i]) & P;
                c[0] ^= t;
                c[i] ^= t;
            }
        }
    }
    for (int i = 1; i < n; ++i) c[i] ^= c[i - 1];
    uint32_t t = 0u;
    for (uint32_t Q = M; Q > 1u; Q >>= 1)
        if (c[n - 1] & Q) t ^= Q - 1u;
    for (int i = 0; i < n; ++i) c[i] ^= t;
    uint32_t key = 0u;
    for (int bit = b - 1; bit >= 0; --bit)
        for (int i = 0; i < n; ++i) key = (key << 1) | ((c[i] >> bit) & 1u);
    return key;
}

__global__ __launch_bounds__(256) void k_cell_keys(const SysDev* __restrict__ sys, const CItem* __restrict__ items,
                                                   const double* __restrict__ X, const double* __restrict__ Y,
                                                   const double* __restrict__ Z, int* __restrict__ keys,
                                                   int* __restrict__ slots, int* __restrict__ cnt)
{
    const CItem it = items[blockIdx.x];
    const SysDev& S = sys[it.sys];
    for (int k = threadIdx.x; k < it.count; k += 256) {
        const int64_t g = S.n_off + it.start + k;
        const double v[3] = {X[g], Y[g], Z[g]};
        uint32_t c[3];
        for (int d = 0; d < 3; ++d) {
            double u = floor((v[d] + S.half[d]) * S.inv_cell[d]);
            u = fmin(fmax(u, 0.0), (double)(S.g[d] - 1));  // also maps NaN to 0
            c[d] = (uint32_t)u;
        }
        const int key = (int)hilbert_key(c, S.dim == 2 ? 2 : 3, S.gbits);
        keys[g] = key;
        slots[g] = atomicAdd(&cnt[S.cell_off + key], 1);
    }
}

// Exclusive scan of each system's ncell+1 counters in three phases: block
// totals over contiguous chunks, a scan of those totals, and the chunk rescan.
__device__ __forceinline__ void scan_chunk(int64_t len, int nblk, int b, int64_t* lo, int64_t* hi)
{
    const int64_t per = (len + nblk - 1) / nblk;
    *lo = (int64_t)b * per < len ? (int64_t)b * per : len;
    *hi = *lo + per < len ? *lo + per : len;
}

__global__ __launch_bounds__(256) void k_scan_totals(const SysDev* __restrict__ sys, const int* __restrict__ cnt,
                                                     int64_t* __restrict__ btot)
{
    __shared__ double sh[4];
    const SysDev& S = sys[blockIdx.y];
    int64_t lo, hi;
    scan_chunk(S.ncell + 1, gridDim.x, blockIdx.x, &lo, &hi);
    double acc = 0.0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += 256) acc += (double)cnt[S.cell_off + i];
    acc = block_reduce<0>(acc, sh);
    if (threadIdx.x == 0) btot[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = (int64_t)acc;
}

__global__ __launch_bounds__(256) void k_scan_chunks(const SysDev* __restrict__ sys, const int* __restrict__ cnt,
                                                     const int64_t* __restrict__ btot, int* __restrict__ start)
{
    __shared__ int64_t sh[4];
    const SysDev& S = sys[blockIdx.y];
    int64_t base = 0;
    for (int b = threadIdx.x; b < (int)blockIdx.x; b += 256) base += btot[(int64_t)blockIdx.y * gridDim.x + b];
    base = block_sum_i64(base, sh);
    int64_t lo, hi;
    scan_chunk(S.ncell + 1, gridDim.x, blockIdx.x, &lo, &hi);
    for (int64_t c0 = lo; c0 < hi; c0 += 256) {
        const int64_t i = c0 + threadIdx.x;
        const int64_t v = i < hi ? cnt[S.cell_off + i] : 0;
        int64_t tot;
        const int64_t ex = block_exclusive_scan(v, sh, &tot);
        if (i < hi) start[S.cell_off + i] = (int)(base + ex);
        base += tot;
    }
}

__global__ __launch_bounds__(256) void k_cell_scatter(const SysDev* __restrict__ sys, const CItem* __restrict__ items,
                                                      const int* __restrict__ keys, const int* __restrict__ slots,
                                                      const int* __restrict__ start, int* __restrict__ perm)
{
    const CItem it = items[blockIdx.x];
    const SysDev& S = sys[it.sys];
    for (int k = threadIdx.x; k < it.count; k += 256) {
        const int64_t i = it.start + k;
        const int64_t g = S.n_off + i;
        const int64_t pos = (int64_t)start[S.cell_off + keys[g]] + slots[g];
        perm[S.n_off + pos] = (int)i;
    }
}

// Put each cell's particles in increasing index order (insertion sort; cells are small).
__global__ __launch_bounds__(256) void k_cell_fixup(const SysDev* __restrict__ sys, const int* __restrict__ start,
                                                    int* __restrict__ perm)
{
    const SysDev& S = sys[blockIdx.y];
    const int64_t c = blockIdx.x * 256ll + threadIdx.x;
    if (c >= S.ncell) return;
    const int64_t b = start[S.cell_off + c], e = start[S.cell_off + c + 1];
    int* p = perm + S.n_off;
    for (int64_t i = b + 1; i < e; ++i) {
        const int v = p[i];
        int64_t j = i - 1;
        while (j >= b && p[j] > v) {
            p[j + 1] = p[j];
            --j;
        }
        p[j + 1] = v;
    }
}

__global__ __launch_bounds__(256) void k_gather(const SysDev* __restrict__ sys, const CItem* __restrict__ items,
                                                const int* __restrict__ perm, const double* __restrict__ X,
                                                const double* __restrict__ Y, const double* __restrict__ Z,
                                                const double* __restrict__ Q, double* __restrict__ sx,
                                                double* __restrict__ sy, double* __restrict__ sz,
                                                double* __restrict__ sq)
{
    const CItem it = items[blockIdx.x];
    const SysDev& S = sys[it.sys];
    for (int k = threadIdx.x; k < it.count; k += 256) {
        const int64_t j = S.n_off + it.start + k;
        const int64_t o = S.n_off + perm[j];
        sx[j] = X[o];
        sy[j] = Y[o];
        sz[j] = Z[o];
        sq[j] = Q[o];
    }
}

// ----------------------------------------------------------------------------
// near set (algorithm "get", steps 1-2): x_j + p with |x_j + p| <= R_b
// ----------------------------------------------------------------------------
// The membership test is evaluated exactly as ((X*X + Y*Y) + Z*Z) <= R_b^2 (1 + 1e-12)
// with X = x + p_x, without fused multiply-add, so that ties on the sphere are
// decided the same way by any FP64 implementation of the rule.
struct BallTest {
    double X, Y, Z;
    bool in;
};
__device__ __forceinline__ BallTest in_ball(double x, double y, double z, double px, double py, double pz, double thr)
{
#pragma clang fp contract(off)
    BallTest b;
    b.X = x + px;
    b.Y = y + py;
    b.Z = z + pz;
    const double s = b.X * b.X + b.Y * b.Y;
    b.in = s + b.Z * b.Z <= thr;
    return b;
}

__global__ __launch_bounds__(256) void k_near_count(const SysDev* __restrict__ sys, const NItem* __restrict__ items,
                                                    const double* __restrict__ img, const double* __restrict__ sx,
                                                    const double* __restrict__ sy, const double* __restrict__ sz,
                                                    int* __restrict__ ncount)
{
    __shared__ double sh[4];
    const NItem it = items[blockIdx.x];
    const SysDev& S = sys[it.sys];
    const double* pv = img + (S.img_off + it.img) * 3;
    const double px = pv[0], py = pv[1], pz = pv[2];
    double c = 0.0;
    for (int e = 0; e < 4; ++e) {
        const int k = threadIdx.x * 4 + e;
        if (k < it.count) {
            const int64_t g = S.n_off + it.start + k;
            if (in_ball(sx[g], sy[g], sz[g], px, py, pz, S.thr).in) c += 1.0;
        }
    }
    c = block_reduce<0>(c, sh);
    if (threadIdx.x == 0) ncount[blockIdx.x] = (int)c;
}

// Per system: exclusive scan of the item counts -> item offsets and N_b.
__global__ __launch_bounds__(1024) void k_near_scan(const SysDev* __restrict__ sys, const int* __restrict__ ncount,
                                                    int64_t* __restrict__ ioff, int64_t* __restrict__ nnear)
{
    __shared__ int64_t sh[16];
    const SysDev& S = sys[blockIdx.x];
    const int64_t len = S.nitem_end - S.nitem_begin;
    const int64_t seg = (len + 1023) / 1024;
    const int64_t b = threadIdx.x * seg, e = b + seg < len ? b + seg : len;
    int64_t loc = 0;
    for (int64_t i = b; i < e; ++i) loc += ncount[S.nitem_begin + i];
    int64_t tot;
    int64_t run = block_exclusive_scan(loc, sh, &tot);
    for (int64_t i = b; i < e; ++i) {
        ioff[S.nitem_begin + i] = run;
        run += ncount[S.nitem_begin + i];
    }
    if (threadIdx.x == 0) nnear[blockIdx.x] = tot;
}

__global__ __launch_bounds__(256) void k_near_write(const SysDev* __restrict__ sys, const NItem* __restrict__ items,
                                                    const int64_t* __restrict__ ioff, const double* __restrict__ img,
                                                    const double* __restrict__ sx, const double* __restrict__ sy,
                                                    const double* __restrict__ sz, const double* __restrict__ sq,
                                                    double* __restrict__ nx, double* __restrict__ ny,
                                                    double* __restrict__ nz, double* __restrict__ nq,
                                                    int* __restrict__ nbase, int* __restrict__ inv)
{
    __shared__ int64_t sh[4];
    const NItem it = items[blockIdx.x];
    const SysDev& S = sys[it.sys];
    const double* pv = img + (S.img_off + it.img) * 3;
    const double px = pv[0], py = pv[1], pz = pv[2];
    bool f[4];
    double X[4], Y[4], Z[4];
    int64_t cnt = 0;
    for (int e = 0; e < 4; ++e) {
        const int k = threadIdx.x * 4 + e;
        f[e] = false;
        if (k < it.count) {
            const int64_t g = S.n_off + it.start + k;
            const BallTest b = in_ball(sx[g], sy[g], sz[g], px, py, pz, S.thr);
            f[e] = b.in;
            X[e] = b.X;
            Y[e] = b.Y;
            Z[e] = b.Z;
        }
        cnt += f[e] ? 1 : 0;
    }
    int64_t tot;
    int64_t pos = block_exclusive_scan(cnt, sh, &tot) + ioff[blockIdx.x];
    for (int e = 0; e < 4; ++e) {
        const int k = threadIdx.x * 4 + e;
        if (k >= it.count) continue;
        const int64_t j = it.start + k;
        int* iv = inv + S.inv_off + (int64_t)it.img * S.n;
        if (f[e]) {
            const int64_t o = S.near_off + pos;
            nx[o] = X[e];
            ny[o] = Y[e];
            nz[o] = Z[e];
            nq[o] = sq[S.n_off + j];
            nbase[o] = (int)j;
            iv[j] = (int)pos;
            ++pos;
        } else {
            iv[j] = -1;
        }
    }
}

// ----------------------------------------------------------------------------
// centre and radius of each target block
// ----------------------------------------------------------------------------
// Centre and radius of one target block (all threads of the workgroup call it).
__device__ void target_block(const PJob* __restrict__ jobs, const TItem it)
{
    __shared__ double sh[4];
    const PJob& J = jobs[it.job];
    const int64_t i = (int64_t)it.tb * J.bt + threadIdx.x;
    const bool v = (int)threadIdx.x < J.bt && i < J.nt;
    const double x = v ? J.tx[i] : 0.0, y = v ? J.ty[i] : 0.0, z = v ? J.tz[i] : 0.0;
    const double lx = block_reduce<1>(v ? x : 1e300, sh), ly = block_reduce<1>(v ? y : 1e300, sh),
                 lz = block_reduce<1>(v ? z : 1e300, sh);
    const double hx = block_reduce<2>(v ? x : -1e300, sh), hy = block_reduce<2>(v ? y : -1e300, sh),
                 hz = block_reduce<2>(v ? z : -1e300, sh);
    const double cx = 0.5 * (lx + hx), cy = 0.5 * (ly + hy), cz = 0.5 * (lz + hz);
    const double d = v ? sqrt((x - cx) * (x - cx) + (y - cy) * (y - cy) + (z - cz) * (z - cz)) : 0.0;
    const double r = block_reduce<2>(d, sh);
    if (threadIdx.x == 0) {
        double* o = J.tblk + (int64_t)it.tb * 4;
        o[0] = cx;
        o[1] = cy;
        o[2] = cz;
        o[3] = r * (1.0 + 1e-12);
    }
}

__global__ __launch_bounds__(256) void k_tblock(const PJob* __restrict__ jobs, const TItem* __restrict__ items)
{
    target_block(jobs, items[blockIdx.x]);
}

// ----------------------------------------------------------------------------
// pair sums (the free-space finite sum of eq. (r2) over the near set)
// ----------------------------------------------------------------------------
// A workgroup owns BT consecutive targets (one per lane) and one split of the
// source tiles.  Sources are staged kTile at a time in LDS and read as
// broadcasts.  A group of kGroup sources of a tile whose sources all lie
// farther than kFarFactor x (target-block radius) from the block centre is
// "far": it cannot hold a source coinciding with a target, so its loop has no
// K(0) = 0 test; other groups are "near" and apply K(0) = 0.
// Accumulation (FP32 kernel): the potential of every 8 pairs is summed as a
// balanced FP32 tree, four such sums are added in FP32 and the result goes to
// an FP64 accumulator; the field runs in FP32 chains flushed to FP64 every 32
// pairs.  (A serial FP32 sum over a whole tile would add an error growing like
// sqrt(tile) times the per-pair rounding.)  The FP64 kernel accumulates every
// pair in FP64.  Splits are combined later in a fixed order.
struct SourceSplit {
    int64_t ns, t0, t1;
};
__device__ __forceinline__ SourceSplit split_range(const PJob& J, int split)
{
    SourceSplit s;
    s.ns = J.ns_dev ? *J.ns_dev : J.ns_host;
    const int64_t ntiles = (s.ns + kTile - 1) / kTile;
    const int64_t per = (ntiles + J.nsplit - 1) / J.nsplit;
    s.t0 = (int64_t)split * per;
    s.t1 = s.t0 + per < ntiles ? s.t0 + per : ntiles;
    return s;
}

// FP32 pair arithmetic on coordinates relative to the target-block centre.
// LDS holds, per source, A = (-2 s_hi, q) and B = (s_lo, |s_hi|^2), where
// s_hi + s_lo is the FP64 relative position split into two floats.
// Near groups: d = (t_hi - s_hi) + (t_lo - s_lo), so close pairs keep their
// full FP64-derived separation, and K(0) = 0 is applied; the field adds
// 2 w_j d_j (w_j = q_j / r_j^3) to the accumulators.
// Far groups: one-float coordinates and the expanded form
// r^2 = |t|^2 + |s|^2 - 2 t.s (an add and three FMAs instead of three
// differences, a product and two FMAs); the field adds w_j (-2 s_j) and,
// apart, w_j, whose FP64 sum over the split is multiplied by t once at the end:
// the field is t sum_j w_j + (1/2) (accumulators).  Far pairs are at least
// (kFarFactor - 1) x (block radius) apart, so the cancellation in the expanded
// r^2 stays a bounded multiple of the FP32 rounding.
// KERN = 1, the screened kernel exp(-kappa r)/r: with ri = 1/r, r = r^2 ri and
// e = 2^(r nk2) (nk2 = -kappa log2(e)), the potential term is q ri e and the
// field weight q e (1 + kappa r)/r^3 = (q ri e) ri (ri + kappa).  A masked pair
// (ri = 0) gives r = 0, e = 1 and zero terms; padding sources give e = 0.
// KERN = 2, the plane's -log r (every z is 0): the potential accumulates
// q log2(r^2), scaled by -ln(2)/2 once at the end, and the field weight is
// q / r^2; a masked pair gives zero terms, padding (r^2 = 2^120) finite ones
// times q = 0.  Its far groups start at far_factor<2>() block radii (ps_device.h).
// KERN = 3, the biharmonic r.  Rounding each term q r at FP32 precision would
// not do: the terms grow with r (and the field terms q (t - s)/r do not decay),
// and summed over a near set of 1e6 sources the rounding reaches 1e-5 of the
// result.  So a source farther than kFarFactor
// block radii from the block centre c (every source of a far group, and such
// sources inside near groups; the flag sC.w, the same for the whole block, so
// the branch is uniform) is taken relative to c: with u = s - c, rho = |u|,
// r = rho sqrt(1 + delta) and delta = (|h|^2 - 2 h.u)/rho^2, it contributes
// q rho + q rho g, g = sqrt(1 + delta) - 1.  The block adds sum q rho over
// those sources once, in FP64 (k_p2p_f32), and the pair only q rho g, which is
// of the size of q |h|.  With y = rsq(1 + delta) and s = (1 + delta) y,
// g = s - 1 is refined by one Newton step on (1 + g)^2 = 1 + delta, which
// gives g to a few roundings of itself rather than of 1.  Likewise the field
// term -q (h - u)/r = q u/rho - q y (h + g u)/rho (1/y = 1 + g): the block adds
// sum q u/rho once, in FP64, and the pair the rest, of the size of q |h|/rho.
// sC holds (1/rho^2, q rho, -q/rho, 1) per such source.  The other sources of near groups take the potential term
// q r = q r^2 ri and the field weight -q ri (E = -grad(q r) = -q (t - s)/r); a
// masked pair (ri = 0) and padding (q = 0) give zero terms.
template <bool NEAR, bool FIELD, int KERN>
__device__ __forceinline__ void group32_f32(const float4* __restrict__ sA, const float4* __restrict__ sB,
                                            const float4* __restrict__ sC, float hx, float hy, float hz, float lx,
                                            float ly, float lz, float tt, float kap, float nk2, double& aP,
                                            double& aW, double& aX, double& aY, double& aZ)
{
    float fX = 0.f, fY = 0.f, fZ = 0.f, fW = 0.f;
    float p32 = 0.f;
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        float qv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const float4 s = sA[g * 8 + u];
            if constexpr (KERN == 3) {
                const float4 c = sC[g * 8 + u];
                if (!NEAR || c.w != 0.f) {
                    const float dl =
                        __builtin_fmaf(hz, s.z, __builtin_fmaf(hy, s.y, __builtin_fmaf(hx, s.x, tt))) * c.x;
                    const float op = 1.f + dl;
                    const float y = __builtin_amdgcn_rsqf(op);
                    const float sq = op * y, hy2 = 0.5f * y;
                    const float res = __builtin_fmaf(sq, sq, -1.f) - dl;
                    const float gg = __builtin_fmaf(-res, hy2, sq - 1.f);
                    qv[u] = c.y * gg;
                    if (FIELD) {  // -q y (h + g u)/rho: a term of the size of q |h|/rho, so y's own rounding is enough
                        const float w = c.z * y;
                        const float hg = -0.5f * gg;  // h + g u = h - (g/2) A
                        fX = __builtin_fmaf(w, __builtin_fmaf(hg, s.x, hx), fX);
                        fY = __builtin_fmaf(w, __builtin_fmaf(hg, s.y, hy), fY);
                        fZ = __builtin_fmaf(w, __builtin_fmaf(hg, s.z, hz), fZ);
                    }
                    continue;
                }
            }
            float dx = 0.f, dy = 0.f, dz = 0.f, r2;
            if (NEAR) {
                const float4 l = sB[g * 8 + u];
                dx = __builtin_fmaf(0.5f, s.x, hx) + (lx - l.x);
                dy = __builtin_fmaf(0.5f, s.y, hy) + (ly - l.y);
                r2 = dx * dx;
                r2 = __builtin_fmaf(dy, dy, r2);
                if constexpr (KERN != 2) {  // the plane: every z is 0
                    dz = __builtin_fmaf(0.5f, s.z, hz) + (lz - l.z);
                    r2 = __builtin_fmaf(dz, dz, r2);
                }
            } else {
                r2 = tt + sB[g * 8 + u].w;
                r2 = __builtin_fmaf(hx, s.x, r2);
                r2 = __builtin_fmaf(hy, s.y, r2);
                if constexpr (KERN != 2) r2 = __builtin_fmaf(hz, s.z, r2);
            }
            float ri = __builtin_amdgcn_rsqf(r2);
            if (NEAR) ri = r2 > 0.f ? ri : 0.f;  // K(0) = 0
            float qr3;
            if constexpr (KERN == 2) {
                float lg = __builtin_amdgcn_logf(r2);
                float inv = __builtin_amdgcn_rcpf(r2);
                if (NEAR) {
                    lg = r2 > 0.f ? lg : 0.f;  // K(0) = 0
                    inv = r2 > 0.f ? inv : 0.f;
                }
                qv[u] = s.w * lg;
                if (FIELD) qr3 = s.w * inv;
            } else if constexpr (KERN == 1) {
                const float e = __builtin_amdgcn_exp2f((r2 * ri) * nk2);
                qv[u] = (s.w * ri) * e;
                if (FIELD) qr3 = qv[u] * (ri * (ri + kap));
            } else if constexpr (KERN == 3) {
                qv[u] = s.w * (r2 * ri);
                if (FIELD) qr3 = -(s.w * ri);
            } else {
                qv[u] = s.w * ri;
                if (FIELD) qr3 = qv[u] * (ri * ri);
            }
            if (FIELD) {
                if (NEAR) {
                    fX = __builtin_fmaf(qr3, dx, fX);
                    fY = __builtin_fmaf(qr3, dy, fY);
                    if constexpr (KERN != 2) fZ = __builtin_fmaf(qr3, dz, fZ);
                } else {
                    fW += qr3;
                    fX = __builtin_fmaf(qr3, s.x, fX);
                    fY = __builtin_fmaf(qr3, s.y, fY);
                    if constexpr (KERN != 2) fZ = __builtin_fmaf(qr3, s.z, fZ);
                }
            }
        }
        p32 += ((qv[0] + qv[1]) + (qv[2] + qv[3])) + ((qv[4] + qv[5]) + (qv[6] + qv[7]));
    }
    aP += (double)p32;
    if (FIELD) {
        if (NEAR || KERN == 3) {  // fX, fY, fZ hold the field itself
            aX += 2.0 * (double)fX;
            aY += 2.0 * (double)fY;
            aZ += 2.0 * (double)fZ;
        } else {
            aW += (double)fW;
            aX += (double)fX;
            aY += (double)fY;
            aZ += (double)fZ;
        }
    }
}

// Near/far decisions of a staged tile's kTile/kGroup groups.  While staging,
// each thread tests its own source: far when its FP64 distance from the target
// block's centre exceeds kFarFactor x (block radius).  A group is far when all
// of its sources are (then every pair of the group is at least
// (kFarFactor - 1) x radius apart, the bound both pair forms rely on); a
// coincident source is never far.  The 64 sources a wave stages in one step
// are two whole groups: one ballot gives both groups' bits, which lane 0
// writes to LDS.  After the barrier every wave reads the tile's mask back, so
// the group branch is wave-uniform.
__device__ __forceinline__ void store_far_bits(uint32_t* far_bits, int first, bool far)
{
    const uint64_t m = __ballot(far);
    if ((threadIdx.x & 63) == 0) {
        far_bits[(first >> 5)] = (uint32_t)m == 0xffffffffu;
        far_bits[(first >> 5) + 1] = (uint32_t)(m >> 32) == 0xffffffffu;
    }
}
__device__ __forceinline__ uint32_t load_far_mask(const uint32_t* far_bits)
{
    uint32_t m = 0;
#pragma unroll
    for (int g = 0; g < kTile / kGroup; ++g) m |= far_bits[g] << g;
    return __builtin_amdgcn_readfirstlane(m);
}

// Occupancy hint for the register allocator: six waves per SIMD (at most 80
// VGPRs) for 256- and 128-wide workgroups (79 VGPRs; 80 and one spilled
// register outside the loops); 64-wide workgroups stage four sources per thread
// and are held to four (92 VGPRs; their LDS allows five).
template <int BT>
constexpr int p2p_waves_hint() { return BT >= 128 ? 6 : 4; }

template <int BT, bool FIELD, int KERN>
__global__ __launch_bounds__(BT) __attribute__((amdgpu_waves_per_eu(p2p_waves_hint<BT>()))) void k_p2p_f32(
    const PJob* __restrict__ jobs, const PItem* __restrict__ items)
{
    constexpr int PF = kTile / BT;  // sources each thread stages per tile
    __shared__ float4 sA[kTile];
    __shared__ float4 sB[kTile];
    __shared__ float4 sC[KERN == 3 ? kTile : 1];  // the biharmonic far form: (1/rho^2, q rho, -q/rho)
    __shared__ double sRed[4][BT / 64];
    __shared__ uint32_t sFar[kTile / kGroup];
    const PItem it = items[blockIdx.x];
    const PJob& J = jobs[it.job];
    const SourceSplit sp = split_range(J, it.split);
    const int64_t i = (int64_t)it.tb * BT + threadIdx.x;
    const bool active = i < J.nt;
    const double* tb = J.tblk + (int64_t)it.tb * 4;
    const double cx = tb[0], cy = tb[1], cz = tb[2], rT = tb[3];
    const double far2 = far_factor<KERN>() * far_factor<KERN>() * rT * rT;
    double rx = 0.0, ry = 0.0, rz = 0.0;
    if (active) {
        rx = J.tx[i] - cx;
        ry = J.ty[i] - cy;
        rz = J.tz[i] - cz;
    }
    const float hx = (float)rx, hy = (float)ry, hz = (float)rz;
    const float lx = (float)(rx - (double)hx), ly = (float)(ry - (double)hy), lz = (float)(rz - (double)hz);
    const float tt = __builtin_fmaf(hz, hz, __builtin_fmaf(hy, hy, hx * hx));
    const float kap = (float)J.kappa, nk2 = (float)(-J.kappa * 1.4426950408889634);
    const double* __restrict__ SX = J.sx;
    const double* __restrict__ SY = J.sy;
    const double* __restrict__ SZ = J.sz;
    const double* __restrict__ SQ = J.sq;
    // staging: all of a thread's loads of a tile are issued before any is used
    double px[PF], py[PF], pz[PF], pq[PF];
    // the biharmonic form: sums of q rho and q u/rho over the staged sources that take it (FP64)
    double cq = 0.0, cvx = 0.0, cvy = 0.0, cvz = 0.0;
    auto fetch = [&](int64_t t) {
#pragma unroll
        for (int u = 0; u < PF; ++u) {
            const int64_t j = t * kTile + u * BT + threadIdx.x;
            const bool v = j < sp.ns;
            px[u] = v ? SX[j] : 0.0;
            py[u] = v ? SY[j] : 0.0;
            pz[u] = v ? SZ[j] : 0.0;
            pq[u] = v ? SQ[j] : 0.0;
        }
    };
    auto stage = [&](int64_t t) {
#pragma unroll
        for (int u = 0; u < PF; ++u) {
            const int k = u * BT + threadIdx.x;
            // padding: a source of charge 0 at (2^60, 0, 0) from the centre, which
            // coincides with no target and keeps r^2 finite in FP32
            float4 a = make_float4(-0x1p61f, 0.f, 0.f, 0.f), b = make_float4(0.f, 0.f, 0.f, 0x1p120f);
            float4 c = make_float4(0x1p-120f, 0.f, 0.f, 0.f);
            bool far = true;
            if (t * kTile + k < sp.ns) {
                const double ux = px[u] - cx, uy = py[u] - cy, uz = pz[u] - cz;
                const double u2 = ux * ux + uy * uy + uz * uz;
                far = u2 > far2;
                const float ax = (float)ux, ay = (float)uy, az = (float)uz;
                a = make_float4(-2.f * ax, -2.f * ay, -2.f * az, (float)pq[u]);
                b = make_float4((float)(ux - (double)ax), (float)(uy - (double)ay), (float)(uz - (double)az),
                                __builtin_fmaf(az, az, __builtin_fmaf(ay, ay, ax * ax)));
                if constexpr (KERN == 3) {
                    if (far) {  // rho > 0
                        const double rho = sqrt(u2), qr = pq[u] * rho, qo = pq[u] / rho;
                        c = make_float4((float)(1.0 / u2), (float)qr, (float)(-qo), 1.f);
                        cq += qr;
                        cvx = __builtin_fma(qo, ux, cvx);
                        cvy = __builtin_fma(qo, uy, cvy);
                        cvz = __builtin_fma(qo, uz, cvz);
                    }
                }
            }
            sA[k] = a;
            sB[k] = b;
            if constexpr (KERN == 3) sC[k] = c;
            store_far_bits(sFar, k & ~63, far);
        }
    };
    double aP = 0.0, aW = 0.0, aX = 0.0, aY = 0.0, aZ = 0.0;
    for (int64_t t = sp.t0; t < sp.t1; ++t) {
        __syncthreads();
        fetch(t);
        stage(t);
        __syncthreads();
        const uint32_t farm = load_far_mask(sFar);
        const float4* A = sA;
        const float4* B = sB;
#pragma unroll 1
        for (int gq = 0; gq < kTile / kGroup; ++gq) {
            if ((farm >> gq) & 1)
                group32_f32<false, FIELD, KERN>(A + gq * kGroup, B + gq * kGroup, sC + (KERN == 3 ? gq * kGroup : 0),
                                                hx, hy, hz, lx, ly, lz, tt, kap, nk2, aP, aW, aX, aY, aZ);
            else
                group32_f32<true, FIELD, KERN>(A + gq * kGroup, B + gq * kGroup, sC + (KERN == 3 ? gq * kGroup : 0),
                                               hx, hy, hz, lx, ly, lz, tt, kap, nk2, aP, aW, aX, aY, aZ);
        }
    }
    if constexpr (KERN == 3) {  // every target of the block gets the sums of q rho and q u/rho, in fixed order
        cq = wave_sum(cq);
        cvx = wave_sum(cvx);
        cvy = wave_sum(cvy);
        cvz = wave_sum(cvz);
        if ((threadIdx.x & 63) == 0) {
            sRed[0][threadIdx.x >> 6] = cq;
            sRed[1][threadIdx.x >> 6] = cvx;
            sRed[2][threadIdx.x >> 6] = cvy;
            sRed[3][threadIdx.x >> 6] = cvz;
        }
        __syncthreads();
        for (int w = 0; w < BT / 64; ++w) {
            aP += sRed[0][w];
            aX += 2.0 * sRed[1][w];  // the field is read as 0.5 aX + h aW
            aY += 2.0 * sRed[2][w];
            aZ += 2.0 * sRed[3][w];
        }
    }
    if (active) {
        double* P_ = J.part + (int64_t)it.split * J.ncomp * J.nt;
        P_[i] = KERN == 2 ? kLog2Half * aP : aP;
        if (FIELD) {
            P_[J.nt + i] = __builtin_fma((double)hx, aW, 0.5 * aX);
            P_[2 * J.nt + i] = __builtin_fma((double)hy, aW, 0.5 * aY);
            P_[3 * J.nt + i] = __builtin_fma((double)hz, aW, 0.5 * aZ);
        }
    }
}

// FP64 pair kernel.  The reciprocal square root is the hardware estimate y0
// (relative error ~5e-8) refined by one Newton step and kept doubled,
// u = y0 (3 - r2 y0^2) = 2/r to rounding: with the halved charge (q/2) u = q/r,
// and (q/r) u^2 = 4 q/r^3, whose factor 4 is removed once at the end.  Far
// groups (beyond kFarFactor times the block radius) work relative to the block
// centre c: r^2 = |h|^2 + |s|^2 - 2 h.s and the field h sum w - sum w s
// (w = 4 q/r^3), with the cancellation bounded as for the FP32 kernel.  Near
// groups take differences of the absolute coordinates, exact for close pairs,
// and apply K(0) = 0.  LDS per source: F = (-(x - c), |x - c|^2) for far groups
// and N = (x, q/2) for near groups (which read the halved charge for both).
// KERN = 1 (screened): r = r^2 u / 2, e = exp(-kappa r), the potential term
// (q/2) u e = q e/r and the weight (q e/r) u (u + 2 kappa) = 4 q e (1 + kappa r)/r^3.
// KERN = 2 (the plane's -log r): the potential term -(q/2) log(r^2) and the
// weight 2 (q/2) u^2 = 4 q / r^2.  The logarithm is log_pos below.
// KERN = 3 (the biharmonic r): the potential term (q/2) u r^2 = q r and the
// weight -4 (q/2) u = 4 (-q/r).
// log(x) for x > 0: x = m 2^e with m in [sqrt(1/2), sqrt(2)), and
// log m = 2 atanh(s) = 2 (s + s^3/3 + ... + s^21/21), s = (m - 1)/(m + 1), |s| < 0.172,
// whose first omitted term is below 2^-55 of the sum; e ln 2 with ln 2 split in
// two parts.  Within 3 ulp of the C library's logarithm (checked on 1e7 points
// over e^-30 .. e^30).  x = 0 gives a finite value (the callers discard it).
__device__ __forceinline__ double log_pos(double x)
{
    int e;
    double m = frexp(x, &e);
    if (m < 0.70710678118654752440) {
        m *= 2.0;
        e -= 1;
    }
    const double s = (m - 1.0) / (m + 1.0), s2 = s * s;
    double p = 1.0 / 21.0;
    p = __builtin_fma(p, s2, 1.0 / 19.0);
    p = __builtin_fma(p, s2, 1.0 / 17.0);
    p = __builtin_fma(p, s2, 1.0 / 15.0);
    p = __builtin_fma(p, s2, 1.0 / 13.0);
    p = __builtin_fma(p, s2, 1.0 / 11.0);
    p = __builtin_fma(p, s2, 1.0 / 9.0);
    p = __builtin_fma(p, s2, 1.0 / 7.0);
    p = __builtin_fma(p, s2, 1.0 / 5.0);
    p = __builtin_fma(p, s2, 1.0 / 3.0);
    p = __builtin_fma(p, s2, 1.0);
    const double de = static_cast<double>(e);
    return __builtin_fma(de, 6.93147180369123816490e-01, __builtin_fma(de, 1.90821492927058770002e-10, 2.0 * s * p));
}

template <bool NEAR, bool FIELD, int KERN>
__device__ __forceinline__ void group32_f64(const double4* __restrict__ sF, const double4* __restrict__ sN, double tx,
                                            double ty, double tz, double h2x, double h2y, double h2z, double tt,
                                            double kap, double& aP, double& aW, double& aX, double& aY, double& aZ)
{
#pragma unroll 2  // 90 VGPRs: five waves per SIMD hide the FP64 latency (unroll 8: 129, three waves, 5% slower)
    for (int k = 0; k < kGroup; ++k) {
        const double4 n = sN[k];
        double r2, dx, dy, dz;
        if (NEAR) {
            dx = tx - n.x;
            dy = ty - n.y;
            dz = KERN == 2 ? 0.0 : tz - n.z;  // the plane: every z is 0
            r2 = KERN == 2 ? __builtin_fma(dy, dy, dx * dx) : __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx));
        } else {
            const double4 f = sF[k];
            dx = f.x;  // -(x - c): the far field accumulates w times these
            dy = f.y;
            dz = KERN == 2 ? 0.0 : f.z;
            r2 = KERN == 2 ? __builtin_fma(h2x, f.x, __builtin_fma(h2y, f.y, tt + f.w))
                           : __builtin_fma(h2x, f.x, __builtin_fma(h2y, f.y, __builtin_fma(h2z, f.z, tt + f.w)));
        }
        const double y0 = __builtin_amdgcn_rsq(r2);
        double u = y0 * __builtin_fma(-(r2 * y0), y0, 3.0);  // 2/r
        if (NEAR) u = r2 > 0.0 ? u : 0.0;                     // K(0) = 0
        double qr, w;
        if constexpr (KERN == 2) {
            const bool live = !NEAR || r2 > 0.0;              // K(0) = 0
            qr = live ? -n.w * log_pos(r2) : 0.0;
            if (FIELD) w = 2.0 * n.w * (u * u);               // 4 q / r^2 (u = 0 for a masked pair)
        } else if constexpr (KERN == 1) {
            qr = (n.w * u) * exp(-kap * (0.5 * (r2 * u)));        // q e/r
            if (FIELD) w = qr * (u * (u + 2.0 * kap));            // 4 q e (1 + kappa r)/r^3
        } else if constexpr (KERN == 3) {
            qr = (n.w * u) * r2;                                  // q r
            if (FIELD) w = -4.0 * (n.w * u);                      // 4 (-q/r)
        } else {
            qr = n.w * u;                                         // q/r
            if (FIELD) w = qr * (u * u);                          // 4 q/r^3
        }
        aP += qr;
        if (FIELD) {
            if (!NEAR) aW += w;
            aX = __builtin_fma(w, dx, aX);
            aY = __builtin_fma(w, dy, aY);
            aZ = __builtin_fma(w, dz, aZ);
        }
    }
}

template <int BT, bool FIELD, int KERN>
__global__ __launch_bounds__(BT) void k_p2p_f64(const PJob* __restrict__ jobs, const PItem* __restrict__ items)
{
    __shared__ double4 sF[kTile];
    __shared__ double4 sN[kTile];
    __shared__ uint32_t sFar[kTile / kGroup];
    const PItem it = items[blockIdx.x];
    const PJob& J = jobs[it.job];
    const SourceSplit sp = split_range(J, it.split);
    const int64_t i = (int64_t)it.tb * BT + threadIdx.x;
    const bool active = i < J.nt;
    const double* tb = J.tblk + (int64_t)it.tb * 4;
    const double cx = tb[0], cy = tb[1], cz = tb[2], rT = tb[3];
    const double far2 = kFarFactor * kFarFactor * rT * rT;
    double tx = cx, ty = cy, tz = cz;
    if (active) {
        tx = J.tx[i];
        ty = J.ty[i];
        tz = J.tz[i];
    }
    const double hx = tx - cx, hy = ty - cy, hz = tz - cz;
    const double tt = __builtin_fma(hz, hz, __builtin_fma(hy, hy, hx * hx));
    const double h2x = 2.0 * hx, h2y = 2.0 * hy, h2z = 2.0 * hz;
    double aP = 0.0, aW = 0.0, aX = 0.0, aY = 0.0, aZ = 0.0;
    for (int64_t t = sp.t0; t < sp.t1; ++t) {
        __syncthreads();
        for (int k = threadIdx.x; k < kTile; k += BT) {
            const int64_t j = t * kTile + k;
            // padding: charge 0 at 2^500 from the centre, coincides with no target
            double4 f = make_double4(-0x1p500, 0.0, 0.0, 0x1p1000);
            double4 n = make_double4(cx + 0x1p500, cy, cz, 0.0);
            bool far = true;
            if (j < sp.ns) {
                const double x = J.sx[j], y = J.sy[j], z = J.sz[j];
                const double ux = x - cx, uy = y - cy, uz = z - cz;
                far = ux * ux + uy * uy + uz * uz > far2;
                f = make_double4(-ux, -uy, -uz, __builtin_fma(uz, uz, __builtin_fma(uy, uy, ux * ux)));
                n = make_double4(x, y, z, 0.5 * J.sq[j]);
            }
            sF[k] = f;
            sN[k] = n;
            store_far_bits(sFar, k & ~63, far);
        }
        __syncthreads();
        const uint32_t farm = load_far_mask(sFar);
#pragma unroll 1
        for (int gq = 0; gq < kTile / kGroup; ++gq) {
            if ((farm >> gq) & 1)
                group32_f64<false, FIELD, KERN>(sF + gq * kGroup, sN + gq * kGroup, tx, ty, tz, h2x, h2y, h2z, tt,
                                                J.kappa, aP, aW, aX, aY, aZ);
            else
                group32_f64<true, FIELD, KERN>(sF + gq * kGroup, sN + gq * kGroup, tx, ty, tz, h2x, h2y, h2z, tt,
                                               J.kappa, aP, aW, aX, aY, aZ);
        }
    }
    if (active) {
        double* P_ = J.part + (int64_t)it.split * J.ncomp * J.nt;
        P_[i] = aP;
        if (FIELD) {
            P_[J.nt + i] = 0.25 * __builtin_fma(hx, aW, aX);
            P_[2 * J.nt + i] = 0.25 * __builtin_fma(hy, aW, aY);
            P_[3 * J.nt + i] = 0.25 * __builtin_fma(hz, aW, aZ);
        }
    }
}

// ----------------------------------------------------------------------------
// check-point sums in FP32 (step 3 at Y_c1 and Y_c2: potential only)
// ----------------------------------------------------------------------------
// The 2L check targets are few and the near set is large, so each target block
// meets every source tile, and the blocks are kept small (64 targets, compact
// by the order the plan gives the check targets) to keep the share of near
// source groups low.  A workgroup of WS waves owns one such block (one target
// per lane, the same in every wave): the waves stage each tile together
// (kTile / (64 WS) sources per thread) and split every group of kGroup
// sources, kGroup / WS to a wave, so the near/far decision stays per group and
// the waves' work stays balanced; the per-target sums of the waves are added
// in a fixed order at the end.  The global loads of the next tile are issued
// before the current one is summed.  Far groups read |s_hi|^2 from an array of
// its own, four sources per LDS read.  The pair arithmetic is group32_f32's
// potential form, and so is the accumulation: a balanced FP32 tree per 8 pairs,
// four trees added in FP32, then an FP64 accumulator.
template <bool NEAR, int KERN>
__device__ __forceinline__ float pot8_f32(const float4* __restrict__ sA, const float4* __restrict__ sB,
                                          const float* __restrict__ sW, float hx, float hy, float hz, float lx,
                                          float ly, float lz, float tt, float nk2)
{
    float qv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const float4 s = sA[u];
        float r2;
        if (NEAR) {
            const float4 l = sB[u];
            const float dx = __builtin_fmaf(0.5f, s.x, hx) + (lx - l.x);
            const float dy = __builtin_fmaf(0.5f, s.y, hy) + (ly - l.y);
            r2 = dx * dx;
            r2 = __builtin_fmaf(dy, dy, r2);
            if constexpr (KERN != 2) {  // the plane: every z is 0
                const float dz = __builtin_fmaf(0.5f, s.z, hz) + (lz - l.z);
                r2 = __builtin_fmaf(dz, dz, r2);
            }
        } else {
            r2 = tt + sW[u];
            r2 = __builtin_fmaf(hx, s.x, r2);
            r2 = __builtin_fmaf(hy, s.y, r2);
            if constexpr (KERN != 2) r2 = __builtin_fmaf(hz, s.z, r2);
        }
        float ri = __builtin_amdgcn_rsqf(r2);
        if (NEAR) ri = r2 > 0.f ? ri : 0.f;  // K(0) = 0
        if constexpr (KERN == 2) {
            const float lg = __builtin_amdgcn_logf(r2);  // the plane, as in group32_f32
            qv[u] = s.w * (NEAR ? (r2 > 0.f ? lg : 0.f) : lg);
        } else if constexpr (KERN == 1)
            qv[u] = (s.w * ri) * __builtin_amdgcn_exp2f((r2 * ri) * nk2);  // screened, as in group32_f32
        else
            qv[u] = s.w * ri;
    }
    return ((qv[0] + qv[1]) + (qv[2] + qv[3])) + ((qv[4] + qv[5]) + (qv[6] + qv[7]));
}

// A load through the global address space: the source arrays of a job are
// device memory, but a pointer read from a job descriptor is generic, and a
// generic (flat) load also counts against the LDS counter, so every LDS wait
// would wait for it as well.
__device__ __forceinline__ double load_global(const double* p, int64_t j)
{
    return ((const __attribute__((address_space(1))) double*)p)[j];
}

template <int WS, int KERN>
__global__ __launch_bounds__(64 * WS) void k_chk_f32(const PJob* __restrict__ jobs, const PItem* __restrict__ items)
{
    constexpr int NT = 64 * WS;     // threads of the workgroup
    constexpr int PF = kTile / NT;  // sources each thread stages per tile
    constexpr int SPW = kGroup / WS;  // sources of each group a wave takes
    static_assert(SPW % 8 == 0 && PF >= 1, "WS must be 1, 2 or 4");
    __shared__ float4 sA[kTile];
    __shared__ float4 sB[kTile];
    __shared__ float sW[kTile];  // |s_hi|^2 again, contiguous: far groups read it four sources at a time
    __shared__ uint32_t sFar[kTile / kGroup];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const PItem it = items[blockIdx.x];
    const PJob& J = jobs[it.job];
    const SourceSplit sp = split_range(J, it.split);
    const int64_t i = (int64_t)it.tb * 64 + lane;
    const bool active = i < J.nt;
    const double* tb = J.tblk + (int64_t)it.tb * 4;
    const double cx = tb[0], cy = tb[1], cz = tb[2], rT = tb[3];
    const double far2 = far_factor<KERN>() * far_factor<KERN>() * rT * rT;
    double rx = 0.0, ry = 0.0, rz = 0.0;
    if (active) {
        rx = J.tx[i] - cx;
        ry = J.ty[i] - cy;
        rz = J.tz[i] - cz;
    }
    const float hx = (float)rx, hy = (float)ry, hz = (float)rz;
    const float lx = (float)(rx - (double)hx), ly = (float)(ry - (double)hy), lz = (float)(rz - (double)hz);
    const float tt = __builtin_fmaf(hz, hz, __builtin_fmaf(hy, hy, hx * hx));
    const float nk2 = (float)(-J.kappa * 1.4426950408889634);
    const double* __restrict__ SX = J.sx;
    const double* __restrict__ SY = J.sy;
    const double* __restrict__ SZ = J.sz;
    const double* __restrict__ SQ = J.sq;
    double px[PF], py[PF], pz[PF], pq[PF];
    auto fetch = [&](int64_t t) {
#pragma unroll
        for (int u = 0; u < PF; ++u) {
            const int64_t j = t * kTile + u * NT + threadIdx.x;
            const bool v = j < sp.ns;
            px[u] = v ? load_global(SX, j) : 0.0;
            py[u] = v ? load_global(SY, j) : 0.0;
            pz[u] = v ? load_global(SZ, j) : 0.0;
            pq[u] = v ? load_global(SQ, j) : 0.0;
        }
    };
    auto stage = [&](int64_t t) {
#pragma unroll
        for (int u = 0; u < PF; ++u) {
            const int k = u * NT + threadIdx.x;
            // padding as in k_p2p_f32: charge 0, far from every target
            float4 a = make_float4(-0x1p61f, 0.f, 0.f, 0.f), b = make_float4(0.f, 0.f, 0.f, 0x1p120f);
            bool far = true;
            if (t * kTile + k < sp.ns) {
                const double ux = px[u] - cx, uy = py[u] - cy, uz = pz[u] - cz;
                far = ux * ux + uy * uy + uz * uz > far2;
                const float ax = (float)ux, ay = (float)uy, az = (float)uz;
                a = make_float4(-2.f * ax, -2.f * ay, -2.f * az, (float)pq[u]);
                b = make_float4((float)(ux - (double)ax), (float)(uy - (double)ay), (float)(uz - (double)az),
                                __builtin_fmaf(az, az, __builtin_fmaf(ay, ay, ax * ax)));
            }
            sA[k] = a;
            sB[k] = b;
            sW[k] = b.w;
            store_far_bits(sFar, k & ~63, far);
        }
    };
    double aP = 0.0;
    // the loads of tile t + 1 are in flight while tile t is summed
    if (sp.t0 < sp.t1) fetch(sp.t0);
    for (int64_t t = sp.t0; t < sp.t1; ++t) {
        __syncthreads();
        stage(t);
        __syncthreads();
        if (t + 1 < sp.t1) fetch(t + 1);
        const uint32_t farm = load_far_mask(sFar);
        // WS groups per FP64 flush: four trees of 8 pairs each
#pragma unroll 1
        for (int g0 = 0; g0 < kTile / kGroup; g0 += WS) {
            float p32 = 0.f;
#pragma unroll
            for (int g = g0; g < g0 + WS; ++g) {
                const int o = g * kGroup + w * SPW;
#pragma unroll
                for (int c = 0; c < SPW; c += 8)
                    p32 += ((farm >> g) & 1)
                               ? pot8_f32<false, KERN>(sA + o + c, sB + o + c, sW + o + c, hx, hy, hz, lx, ly, lz, tt,
                                                       nk2)
                               : pot8_f32<true, KERN>(sA + o + c, sB + o + c, sW + o + c, hx, hy, hz, lx, ly, lz, tt,
                                                      nk2);
            }
            aP += (double)p32;
        }
    }
    if (WS > 1) {
        __syncthreads();
        double* red = reinterpret_cast<double*>(sA);  // (WS - 1) x 64 doubles
        if (w > 0) red[(w - 1) * 64 + lane] = aP;
        __syncthreads();
        if (w == 0)
            for (int k = 1; k < WS; ++k) aP += red[(k - 1) * 64 + lane];
    }
    if (w == 0 && active) J.part[(int64_t)it.split * J.nt + i] = KERN == 2 ? kLog2Half * aP : aP;
}

// ----------------------------------------------------------------------------
// least-squares solve (steps 4-5): f = phi_near(Y_c2) - phi_near(Y_c1), C = A^+ f
// ----------------------------------------------------------------------------
// f_l = phi_near(y~_l) - phi_near(y_l) from the split partials (the check job
// holds the targets in its own order; slot maps a check target to its place):
// 64 check points per workgroup, 16 lane groups over the splits, combined in
// fixed order.  The biharmonic kernel's check job also carries the field E:
// its gradient rows f[L + k L + l] = R0 (E_k(y_l) - E_k(y~_l)), the periodicity
// of d phi_near / du_k (u = y/R0, d/du = -R0 E).
__global__ __launch_bounds__(1024) void k_rhs(const SysDev* __restrict__ sys, const PJob* __restrict__ cjobs,
                                              const int* __restrict__ slot, double* __restrict__ fout)
{
    __shared__ double sa[16][64], sb[16][64];
    const SysDev& S = sys[blockIdx.y];
    const PJob& J = cjobs[blockIdx.y];
    const int g = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int l = blockIdx.x * 64 + lane;
    const int ncomp = S.kernel == 3 ? 4 : 1;  // uniform over the workgroup
    for (int c = 0; c < ncomp; ++c) {
        double a = 0.0, b = 0.0;
        if (l < S.L) {
            const int ia = slot[S.chk_off + l], ib = slot[S.chk_off + S.L + l];
            for (int s = g; s < J.nsplit; s += 16) {
                const double* P_ = J.part + ((int64_t)s * J.ncomp + c) * J.nt;
                a += P_[ia];
                b += P_[ib];
            }
        }
        if (c > 0) __syncthreads();  // the previous component's reads are done
        sa[g][lane] = a;
        sb[g][lane] = b;
        __syncthreads();
        if (g == 0 && l < S.L) {
            double A = 0.0, B = 0.0;
            for (int k = 0; k < 16; ++k) {
                A += sa[k][lane];
                B += sb[k][lane];
            }
            fout[S.f_off + (int64_t)c * S.L + l] = c == 0 ? B - A : S.R0 * (A - B);
        }
    }
}

// Near sums at the decay-surface points, reduced once over the source splits
// (in split order) so that the rows below read two or three values per point
// instead of re-reading every split for every row:
//   dfield[0][i] = phi_near, dfield[1][i] = the normal field (slab: E_z; wire:
//   E_rho = E_y cos(theta) + E_z sin(theta)), dfield[2][i] = theta (wire).
__global__ __launch_bounds__(256) void k_decay_fields(const SysDev* __restrict__ sys, const PJob* __restrict__ djobs,
                                                      const double* __restrict__ dpts, int64_t dec_tot,
                                                      double* __restrict__ dfield)
{
    const SysDev& S = sys[blockIdx.y];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (S.ndec == 0 || i >= (int64_t)S.nsurf * S.m2) return;
    const PJob& J = djobs[blockIdx.y];
    double phi = 0.0, ey = 0.0, ez = 0.0;
    for (int sp = 0; sp < J.nsplit; ++sp) {
        const double* P_ = J.part + (int64_t)sp * 4 * J.nt;
        phi += P_[i];
        ey += P_[2 * J.nt + i];
        ez += P_[3 * J.nt + i];
    }
    double en = ez, th = 0.0;
    if (S.periodic == 1) {
        th = atan2(dpts[2 * dec_tot + S.dec_off + i], dpts[dec_tot + S.dec_off + i]);
        double st, ct;
        sincos(th, &st, &ct);
        en = ey * ct + ez * st;
    }
    dfield[S.dec_off + i] = phi;
    dfield[dec_tot + S.dec_off + i] = en;
    dfield[2 * dec_tot + S.dec_off + i] = th;
}

// Decay rows (fewer than three periodic axes), from the reduced near sums at the
// decay-surface points (potential and field E = -grad phi):
//   slab: f[L + r] = <(E_z - s|k| phi_near) trig(k.rho)> over decay plane s,
//         i.e. -<(d phi_near/dz + s|k| phi_near) trig(k.rho)>;
//   wire: f[L + r] = <(E_rho + beta phi_near) trig(k x) trig(m theta)> over the
//         cylinder, i.e. -<(d phi_near/drho - beta phi_near) trig(k x) trig(m theta)>.
// One workgroup per (row, system); fixed-order reduction.
__global__ __launch_bounds__(256) void k_decay_rhs(const SysDev* __restrict__ sys, const double* __restrict__ dpts,
                                                   int64_t dec_tot, const double* __restrict__ dfield,
                                                   const double* __restrict__ dw, const double* __restrict__ drows,
                                                   double* __restrict__ fout)
{
    __shared__ double sh[4];
    const SysDev& S = sys[blockIdx.y];
    const int r = blockIdx.x;
    if (r >= S.ndec) return;  // uniform over the workgroup
    const double* row = drows + S.drow_off + (int64_t)r * 5;
    const double* px = dpts + S.dec_off;
    const double* fphi = dfield + S.dec_off;
    const double* fn = dfield + dec_tot + S.dec_off;
    double acc = 0.0;
    if (S.periodic == 1) {
        const double k = row[0], mm = row[1], beta = row[2];
        const bool sin_x = row[3] != 0.0, sin_t = row[4] != 0.0;
        const double* fth = dfield + 2 * dec_tot + S.dec_off;
        for (int i = threadIdx.x; i < S.m2; i += 256) {
            const double tx = sin_x ? sin(k * px[i]) : cos(k * px[i]);
            const double tt = sin_t ? sin(mm * fth[i]) : cos(mm * fth[i]);
            acc = __builtin_fma(dw[S.dw_off + i] * (tx * tt), fn[i] + beta * fphi[i], acc);
        }
    } else {
        const double kx = row[0], ky = row[1], kk = row[2], sg = row[3];
        const bool use_sin = row[4] != 0.0;
        const int plane = sg > 0.0 ? 0 : 1;
        const double* py = dpts + dec_tot + S.dec_off;
        for (int k = threadIdx.x; k < S.m2; k += 256) {
            const int64_t i = (int64_t)plane * S.m2 + k;
            const double ph = kx * px[i] + ky * py[i];
            const double tr = use_sin ? sin(ph) : cos(ph);
            acc = __builtin_fma(dw[S.dw_off + k] * tr, fn[i] - sg * kk * fphi[i], acc);
        }
    }
    acc = block_reduce<0>(acc, sh);
    if (threadIdx.x == 0) fout[S.f_off + S.L + r] = acc;
}

__global__ __launch_bounds__(256) void k_gemv(const SysDev* __restrict__ sys, const double* __restrict__ pinv,
                                              const double* __restrict__ f, double* __restrict__ coef)
{
    const SysDev& S = sys[blockIdx.y];
    const int lane = threadIdx.x & 63;
    const int r = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (r >= S.P - 1) return;
    const double* row = pinv + S.pinv_off + (int64_t)r * S.Lf;
    const double* fs = f + S.f_off;
    double acc = 0.0;
    for (int l = lane; l < S.Lf; l += 64) acc = __builtin_fma(row[l], fs[l], acc);
    acc = wave_sum(acc);
    if (lane == 0) coef[S.coef_off + 1 + r] = acc;
}

// ----------------------------------------------------------------------------
// zero-mean constant (step 6, eqs. (pfx3)-(pfx4))
// ----------------------------------------------------------------------------
// Phi0(x) = (1/V0) int_box dV/|y - x| by the closed-form potential of a uniform
// rectangular prism: the alternating sum over the eight corners of
// F(a,b,c) = ab ln(c+r) + bc ln(a+r) + ca ln(b+r)
//            - a^2/2 atan(bc/(ar)) - b^2/2 atan(ca/(br)) - c^2/2 atan(ab/(cr)),
// (a,b,c) = corner - x.  Each term is taken as zero where its prefactor
// vanishes (its limit), and c + r is formed as (a^2+b^2)/(r-c) when c < 0.
__device__ __forceinline__ double log_c_plus_r(double c, double r, double s)
{
    return log(c >= 0.0 ? c + r : s / (r - c));
}

__device__ double prism_corner(double a, double b, double c)
{
    const double a2 = a * a, b2 = b * b, c2 = c * c;
    const double r = sqrt(a2 + b2 + c2);
    if (r == 0.0) return 0.0;
    double F = 0.0;
    if (a * b != 0.0) F += a * b * log_c_plus_r(c, r, a2 + b2);
    if (b * c != 0.0) F += b * c * log_c_plus_r(a, r, b2 + c2);
    if (c * a != 0.0) F += c * a * log_c_plus_r(b, r, c2 + a2);
    if (a != 0.0) F -= 0.5 * a2 * atan(b * c / (a * r));
    if (b != 0.0) F -= 0.5 * b2 * atan(c * a / (b * r));
    if (c != 0.0) F -= 0.5 * c2 * atan(a * b / (c * r));
    return F;
}

// The biharmonic kernel's box mean Psi0(x) = (1/V0) int_box |y - x| dV takes the
// corner primitive G with d^3 G/(da db dc) = r = sqrt(a^2 + b^2 + c^2):
// G = abc r/4 + [ab (a^2 + b^2) ln(c + r) + bc (b^2 + c^2) ln(a + r)
//     + ca (c^2 + a^2) ln(b + r)]/6 - [a^4 atan(bc/(ar)) + b^4 atan(ca/(br))
//     + c^4 atan(ab/(cr))]/12
// (r = (1/4) div(r x) turns the volume integral into face integrals of r (x.n),
// each of which has a closed form), with the same limits as prism_corner.
__device__ double dist_corner(double a, double b, double c)
{
    const double a2 = a * a, b2 = b * b, c2 = c * c;
    const double r = sqrt(a2 + b2 + c2);
    if (r == 0.0) return 0.0;
    double F = 0.25 * a * b * c * r;
    double L = 0.0;
    if (a * b != 0.0) L += a * b * (a2 + b2) * log_c_plus_r(c, r, a2 + b2);
    if (b * c != 0.0) L += b * c * (b2 + c2) * log_c_plus_r(a, r, b2 + c2);
    if (c * a != 0.0) L += c * a * (c2 + a2) * log_c_plus_r(b, r, c2 + a2);
    double T = 0.0;
    if (a != 0.0) T += a2 * a2 * atan(b * c / (a * r));
    if (b != 0.0) T += b2 * b2 * atan(c * a / (b * r));
    if (c != 0.0) T += c2 * c2 * atan(a * b / (c * r));
    return F + L / 6.0 - T / 12.0;
}

// The plane's rectangle primitive F with d^2F/du dv = log(u^2 + v^2):
// F = u v (log(u^2 + v^2) - 3) + u^2 atan(v/u) + v^2 atan(u/v), a term taken as
// zero where its prefactor vanishes.
__device__ double rect_corner(double u, double v)
{
    const double r2 = u * u + v * v;
    if (r2 == 0.0) return 0.0;
    double F = u * v * (log(r2) - 3.0);
    if (u != 0.0) F += u * u * atan(v / u);
    if (v != 0.0) F += v * v * atan(u / v);
    return F;
}

// Corner k (bit 0: +x side, bit 1: +y, bit 2: +z) of Phi0(x): its signed term over V0.
// In the plane (V0 is the rectangle's area) the four corners k < 4 give
// Phi0 = -(1/(2 V0)) sum_k s_k F(corner_k - x), the potential of a uniform rectangle.
__device__ double box_mean_corner(const SysDev& S, int k, double x, double y, double z)
{
    if (S.dim == 2) {
        if (k >= 4) return 0.0;
        const double sx = (k & 1) ? 1.0 : -1.0, sy = (k & 2) ? 1.0 : -1.0;
        return -0.5 * sx * sy * rect_corner(sx * S.half[0] - x, sy * S.half[1] - y) / S.V0;
    }
    const double sx = (k & 1) ? 1.0 : -1.0, sy = (k & 2) ? 1.0 : -1.0, sz = (k & 4) ? 1.0 : -1.0;
    const double a = sx * S.half[0] - x, b = sy * S.half[1] - y, c = sz * S.half[2] - z;
    return sx * sy * sz * (S.kernel == 3 ? dist_corner(a, b, c) : prism_corner(a, b, c)) / S.V0;
}

// One workgroup per item of the near-size-weighted table (see k_bounds);
// part[item] receives the workgroup's share of sum_e q_e Phi0(x_e).
__global__ __launch_bounds__(256) void k_mean(const SysDev* __restrict__ sys, const CItem* __restrict__ witems,
                                              const int64_t* __restrict__ nnear, const double* __restrict__ nx,
                                              const double* __restrict__ ny, const double* __restrict__ nz,
                                              const double* __restrict__ nq, double* __restrict__ part)
{
    __shared__ double sh[4];
    const CItem it = witems[blockIdx.x];
    const SysDev& S = sys[it.sys];
    const int64_t nb = S.mcorner ? 0 : nnear[it.sys];  // k_mean_corners serves the system
    // one lane per (near source, corner): q_e times corner k of Phi0(x_e)
    double acc = 0.0;
    for (int64_t u = it.start * 256 + threadIdx.x; u < 8 * nb; u += (int64_t)it.count * 256) {
        const int64_t o = S.near_off + (u >> 3);
        acc += nq[o] * box_mean_corner(S, static_cast<int>(u & 7), nx[o], ny[o], nz[o]);
    }
    acc = block_reduce<0>(acc, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

// The same sum regrouped by corner points.  Corner a (per axis) of the image
// boxes sits at G_a = (1/2 - a) d: it is the upper corner (sign +) of box a and
// the lower corner (sign -) of box a - 1.  So sum_{p in P_j} Phi0(x_j + p) V0 =
// sum_a W_a F(G_a - x_j), where W_a adds the signs of corner a over the boxes
// of P_j (particle j's near images) that share it.  W_a is zero wherever P_j's
// indicator has no mixed difference across the corner, which removes about four
// in five of the 8 |P_j| corner terms.  One wave per kMeanWave particles of a
// system.  P_j is kept as one bit mask over the z images per (x, y) image
// column (bit w: box (u, v, w - mr[2]) holds x_j + p within the ball, by the
// same test as the near list).  The nonzero (particle, corner, W) go to a
// queue in LDS, and the log/atan corner term is evaluated kMeanWave queue
// entries at a time, so that every lane does one.  A workgroup takes the
// corner columns ax0..ax1 (along x) of its chunk.
// Queue entry: lane (6 bits) | corner column ax << 6 | ay << 13 | corner t along z << 20 | (W + 8) << 25;
// ax, ay and t count from the lowest corner (a = -mr).
__device__ __forceinline__ double mean_corner_term(const SysDev& S, unsigned e, const double4* sp)
{
    const int lane = e & 63, ax = (e >> 6) & 127, ay = (e >> 13) & 127, t = (e >> 20) & 31;
    const int W = static_cast<int>((e >> 25) & 31) - 8;
    const double4 P = sp[lane];
    const double gx = (0.5 - (ax - S.mr[0])) * S.box[0];
    const double gy = (0.5 - (ay - S.mr[1])) * S.box[1];
    const double gz = (0.5 - (t - S.mr[2])) * S.box[2];
    return P.w * W * (S.kernel == 3 ? dist_corner(gx - P.x, gy - P.y, gz - P.z) : prism_corner(gx - P.x, gy - P.y, gz - P.z));
}

__device__ __forceinline__ int mask_step(unsigned m, int t)  // bit t minus bit t - 1
{
    return static_cast<int>((m >> t) & 1u) - static_cast<int>(((m << 1) >> t) & 1u);
}

__global__ __launch_bounds__(kMeanWave) void k_mean_corners(const SysDev* __restrict__ sys,
                                                            const MItem* __restrict__ mitems,
                                                            const int* __restrict__ imap,
                                                            const double* __restrict__ img,
                                                            const double* __restrict__ sx,
                                                            const double* __restrict__ sy,
                                                            const double* __restrict__ sz,
                                                            const double* __restrict__ sq, double* __restrict__ mpart)
{
    extern __shared__ unsigned smask[];  // [columns][kMeanWave]
    __shared__ double4 sp[kMeanWave];
    __shared__ unsigned sque[2 * kMeanWave];
    const MItem it = mitems[blockIdx.x];
    const SysDev& S = sys[it.sys];
    const int lane = threadIdx.x;
    const bool act = lane < it.count;
    double x = 0.0, y = 0.0, z = 0.0, q = 0.0;
    if (act) {
        const int64_t g = S.n_off + it.start + lane;
        x = sx[g];
        y = sy[g];
        z = sz[g];
        q = sq[g];
    }
    sp[lane] = make_double4(x, y, z, q);
    const int nx = 2 * S.mr[0] + 1, ny = 2 * S.mr[1] + 1, nz = 2 * S.mr[2] + 1;
    const int* map = imap + S.imap_off;
    // the columns next to corner columns ax0..ax1
    const int c0 = (it.ax0 > 0 ? it.ax0 - 1 : 0) * ny, c1 = (it.ax1 < nx ? it.ax1 + 1 : nx) * ny;
    for (int c = c0; c < c1; ++c) {
        unsigned m = 0u;
        for (int w = 0; w < nz; ++w) {
            const int idx = map[c * nz + w];
            if (idx >= 0 && act) {
                const double* pv = img + (S.img_off + idx) * 3;
                if (in_ball(x, y, z, pv[0], pv[1], pv[2], S.thr).in) m |= 1u << w;
            }
        }
        smask[c * kMeanWave + lane] = m;
    }
    __syncthreads();
    const uint64_t below = (uint64_t(1) << lane) - 1;
    int cnt = 0;  // queued entries (wave-uniform)
    double acc = 0.0;
    for (int ax = it.ax0; ax <= it.ax1; ++ax)
        for (int ay = 0; ay <= ny; ++ay) {
            // the four columns sharing corner column (ax, ay), with their x-y signs
            const unsigned m00 = (ax < nx && ay < ny) ? smask[(ax * ny + ay) * kMeanWave + lane] : 0u;
            const unsigned m10 = (ax > 0 && ay < ny) ? smask[((ax - 1) * ny + ay) * kMeanWave + lane] : 0u;
            const unsigned m01 = (ax < nx && ay > 0) ? smask[(ax * ny + ay - 1) * kMeanWave + lane] : 0u;
            const unsigned m11 = (ax > 0 && ay > 0) ? smask[((ax - 1) * ny + ay - 1) * kMeanWave + lane] : 0u;
            const unsigned edge = (m00 ^ (m00 << 1)) | (m10 ^ (m10 << 1)) | (m01 ^ (m01 << 1)) | (m11 ^ (m11 << 1));
            for (int t = 0; t <= nz; ++t) {
                if (!__ballot((edge >> t) & 1u)) continue;
                const int W = mask_step(m00, t) - mask_step(m10, t) - mask_step(m01, t) + mask_step(m11, t);
                const uint64_t b = __ballot(W != 0);
                if (W != 0)
                    sque[cnt + __popcll(b & below)] = static_cast<unsigned>(lane) | (static_cast<unsigned>(ax) << 6) |
                                                      (static_cast<unsigned>(ay) << 13) |
                                                      (static_cast<unsigned>(t) << 20) |
                                                      (static_cast<unsigned>(W + 8) << 25);
                cnt += __popcll(b);
                if (cnt >= kMeanWave) {
                    __syncthreads();
                    acc += mean_corner_term(S, sque[cnt - kMeanWave + lane], sp);
                    cnt -= kMeanWave;
                    __syncthreads();
                }
            }
        }
    __syncthreads();
    if (lane < cnt) acc += mean_corner_term(S, sque[lane], sp);
    acc = wave_sum(acc);
    if (lane == 0) mpart[blockIdx.x] = acc / S.V0;
}

__global__ __launch_bounds__(256) void k_c1(const SysDev* __restrict__ sys, const double* __restrict__ part,
                                            const double* __restrict__ mpart, const double* __restrict__ bm,
                                            double* __restrict__ coef)
{
    __shared__ double sh[4];
    const SysDev& S = sys[blockIdx.x];
    double sm = 0.0, d = 0.0;
    if (S.mcorner)
        for (int64_t b = threadIdx.x; b < S.mitem_n; b += 256) sm += mpart[S.mitem_off + b];
    else
        for (int64_t b = threadIdx.x; b < S.witem_n; b += 256) sm += part[S.witem_off + b];
    for (int t = 1 + threadIdx.x; t < S.P; t += 256) d += coef[S.coef_off + t] * bm[S.bm_off + t];
    sm = block_reduce<0>(sm, sh);
    d = block_reduce<0>(d, sh);
    if (threadIdx.x == 0) coef[S.coef_off] = S.mean_mode == 0 ? -sm - d : 0.0;
}

// ----------------------------------------------------------------------------
// far field (step 7) and combination (step 8)
// ----------------------------------------------------------------------------
// phi_far = sum_{t>=2} C_t R^_t(u), u = y/R0, with the renormalized recurrence
// (coefficients a, b, c in LDS) differentiated in forward mode: every value is
// carried with its gradient, which gives grad phi_far without separate
// gradient coefficients.  The orders m are shared among the FL lanes of a
// target: in round r lane g takes m = r FL + g (r even) or r FL + FL - 1 - g
// (r odd), which keeps the loop lengths of the
// lanes of one round close and each lane's orders increasing, so that the
// sectoral values (m, +-m) are carried forward from the lane's previous order.
// The biharmonic basis adds |u|^2 R^_t for degrees below p2 = p - 2 with the
// coefficients C2[t] (C2 = C + p^2; p2 = 0 otherwise): their sum Q rides on the
// same recurrence, and phi = P + |u|^2 Q, grad = grad P + |u|^2 grad Q + 2 u Q.
template <int FL>
__device__ void far_field_lane(int p, int p2, int g, const double* __restrict__ C, const double* __restrict__ C2,
                               const double* __restrict__ A, const double* __restrict__ B,
                               const double* __restrict__ Cd, double x, double y, double z, double& phi, double& gx,
                               double& gy, double& gz)
{
    const double r2 = x * x + y * y + z * z;
    double dA = 1.0, dAx = 0.0, dAy = 0.0, dAz = 0.0;
    double dB = 0.0, dBx = 0.0, dBy = 0.0, dBz = 0.0;
    double P0 = 0.0, X0 = 0.0, Y0 = 0.0, Z0 = 0.0;
    double Q0 = 0.0, QX = 0.0, QY = 0.0, QZ = 0.0;
    int mc = 0;
    for (int r = 0; r * FL < p; ++r) {
        const int m = r * FL + ((r & 1) ? FL - 1 - g : g);
        if (m >= p) continue;
        while (mc < m) {
            const double c = Cd[++mc];
            const double nA = -c * (x * dA + y * dB);
            const double nAx = -c * (dA + x * dAx + y * dBx);
            const double nAy = -c * (x * dAy + dB + y * dBy);
            const double nAz = -c * (x * dAz + y * dBz);
            const double nB = c * (y * dA - x * dB);
            const double nBx = c * (y * dAx - dB - x * dBx);
            const double nBy = c * (dA + y * dAy - x * dBy);
            const double nBz = c * (y * dAz - x * dBz);
            dA = nA; dAx = nAx; dAy = nAy; dAz = nAz;
            dB = nB; dBx = nBx; dBy = nBy; dBz = nBz;
        }
        for (int s = 0; s < (m ? 2 : 1); ++s) {
            const int mm = s ? -m : m;
            double v1 = s ? dB : dA, v1x = s ? dBx : dAx, v1y = s ? dBy : dAy, v1z = s ? dBz : dAz;
            double v2 = 0.0, v2x = 0.0, v2y = 0.0, v2z = 0.0;
            const int t0 = m * m + m + mm;
            if (t0 > 0) {
                const double ct = C[t0];
                P0 = __builtin_fma(ct, v1, P0);
                X0 = __builtin_fma(ct, v1x, X0);
                Y0 = __builtin_fma(ct, v1y, Y0);
                Z0 = __builtin_fma(ct, v1z, Z0);
            }
            if (m < p2) {
                const double c2 = C2[t0];
                Q0 = __builtin_fma(c2, v1, Q0);
                QX = __builtin_fma(c2, v1x, QX);
                QY = __builtin_fma(c2, v1y, QY);
                QZ = __builtin_fma(c2, v1z, QZ);
            }
            for (int n = m + 1; n < p; ++n) {
                const int t = n * n + n + mm;
                const double a = A[t], b = B[t];
                const double v = -a * z * v1 - b * r2 * v2;
                const double vx = -a * z * v1x - b * (2.0 * x * v2 + r2 * v2x);
                const double vy = -a * z * v1y - b * (2.0 * y * v2 + r2 * v2y);
                const double vz = -a * (v1 + z * v1z) - b * (2.0 * z * v2 + r2 * v2z);
                const double ct = C[t];
                P0 = __builtin_fma(ct, v, P0);
                X0 = __builtin_fma(ct, vx, X0);
                Y0 = __builtin_fma(ct, vy, Y0);
                Z0 = __builtin_fma(ct, vz, Z0);
                if (n < p2) {
                    const double c2 = C2[t];
                    Q0 = __builtin_fma(c2, v, Q0);
                    QX = __builtin_fma(c2, vx, QX);
                    QY = __builtin_fma(c2, vy, QY);
                    QZ = __builtin_fma(c2, vz, QZ);
                }
                v2 = v1; v2x = v1x; v2y = v1y; v2z = v1z;
                v1 = v; v1x = vx; v1y = vy; v1z = vz;
            }
        }
    }
    phi = __builtin_fma(r2, Q0, P0);
    gx = __builtin_fma(r2, QX, __builtin_fma(2.0 * x, Q0, X0));
    gy = __builtin_fma(r2, QY, __builtin_fma(2.0 * y, Q0, Y0));
    gz = __builtin_fma(r2, QZ, __builtin_fma(2.0 * z, Q0, Z0));
}

// The plane's far field at the scaled point w = x + iy, lane g of FL: with
// c_n = C[2n-1] - i C[2n], sum_t C_t R_t = Re S and its gradient (Re D, -Im D),
// S = sum_n c_n w^n, D = sum_n n c_n w^(n-1) (Cauchy-Riemann), n = 1..p-1.  Lane
// g takes n = g + 1, g + 1 + FL, ...: it forms w^g by repeated products, then
// steps by w^FL.
template <int FL>
__device__ __forceinline__ void far_field_plane_lane(int p, int g, const double* C, double x, double y, double& phi,
                                                     double& gx, double& gy)
{
    double pr = 1.0, pi = 0.0;  // w^(n-1) for the lane's first n = g + 1
    for (int k = 0; k < g; ++k) {
        const double a = pr * x - pi * y, b = pr * y + pi * x;
        pr = a;
        pi = b;
    }
    double sr = 1.0, si = 0.0;  // w^FL
    for (int k = 0; k < FL; ++k) {
        const double a = sr * x - si * y, b = sr * y + si * x;
        sr = a;
        si = b;
    }
    double Sr = 0.0, Dr = 0.0, Di = 0.0;
    for (int n = g + 1; n < p; n += FL) {
        const double cr = C[2 * n - 1], ci = -C[2 * n];
        const double wr = pr * x - pi * y, wi = pr * y + pi * x;  // w^n
        Sr += cr * wr - ci * wi;
        Dr += n * (cr * pr - ci * pi);
        Di += n * (cr * pi + ci * pr);
        const double a = pr * sr - pi * si, b = pr * si + pi * sr;
        pr = a;
        pi = b;
    }
    phi = Sr;
    gx = Dr;
    gy = -Di;
}

// Sum over the FL adjacent lanes of one target (butterfly: the same
// value in each of them, in a fixed order).
template <int FL>
__device__ __forceinline__ double far_lanes_sum(double v)
{
    for (int o = 1; o < FL; o <<= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// One workgroup per chunk of 256 / FL targets of a system, FL lanes per
// target (8 where the shape has few targets, so that each target's work is
// spread wider; 4 otherwise): fixed-order sum of the pair partials (lane g takes the splits
// s = g mod FL), far field and constant, store (to the original particle
// order when perm is given; `osort` keeps a copy in sorted order: phi, ex, ey,
// ez).  Spherical basis: the far field is evaluated here from the coefficients.
// RBF basis: it was summed by the far pair job (fjobs), whose partials hold
// sum_t C_t K(y - x_t) and its field.
template <int FL>
__global__ __launch_bounds__(256) void k_far_combine(const SysDev* __restrict__ sys, const CItem* __restrict__ items,
                                                     const PJob* __restrict__ pjobs, const PJob* __restrict__ fjobs,
                                                     const double* __restrict__ coef, const double* __restrict__ rec,
                                                     const int* __restrict__ perm, double* __restrict__ phi,
                                                     double* __restrict__ ex, double* __restrict__ ey,
                                                     double* __restrict__ ez, double* __restrict__ osort)
{
    static_assert(FL >= 1 && FL <= 64 && (FL & (FL - 1)) == 0, "far-combine lane layout");
    extern __shared__ double lds[];
    const CItem it = items[blockIdx.x];
    const SysDev& S = sys[it.sys];
    const PJob& J = pjobs[it.sys];
    const int P = S.P, p = S.p;
    const bool rbf = S.basis == 1;
    const bool plane = S.dim == 2;
    double* C = lds;
    double* A = lds + P;
    double* B = lds + 2 * P;
    double* Cd = lds + 3 * P;
    if (plane) {
        for (int t = threadIdx.x; t < P; t += 256) C[t] = coef[S.coef_off + t];
    } else if (!rbf) {
        for (int t = threadIdx.x; t < P; t += 256) {
            C[t] = coef[S.coef_off + t];
            A[t] = rec[S.rec_off + t];
            B[t] = rec[S.rec_off + P + t];
        }
        for (int t = threadIdx.x; t < p; t += 256) Cd[t] = rec[S.rec_off + 2 * P + t];
    }
    __syncthreads();
    const int k = threadIdx.x / FL, g = threadIdx.x % FL;
    const bool act = k < it.count;  // every lane stays for the shuffles below
    const int64_t i = it.start + (act ? k : 0);
    double ph = 0.0, fx = 0.0, fy = 0.0, fz = 0.0;
    if (act) {
#pragma unroll 8
        for (int s = g; s < J.nsplit; s += FL) {
            const double* P_ = J.part + (int64_t)s * 4 * J.nt;
            ph += P_[i];
            fx += P_[J.nt + i];
            fy += P_[2 * J.nt + i];
            fz += P_[3 * J.nt + i];
        }
        if (rbf) {
            if (g == 0) {
                const PJob& F = fjobs[it.sys];
                ph += F.part[i] + coef[S.coef_off];
                fx += F.part[F.nt + i];
                fy += F.part[2 * F.nt + i];
                fz += F.part[3 * F.nt + i];
            }
        } else if (plane) {
            double pf, gx, gy;
            far_field_plane_lane<FL>(p, g, C, J.tx[i] * S.inv_R0, J.ty[i] * S.inv_R0, pf, gx, gy);
            ph += pf + (g == 0 ? C[0] : 0.0);
            fx -= gx * S.inv_R0;
            fy -= gy * S.inv_R0;
        } else {
            double pf, gx, gy, gz;
            far_field_lane<FL>(p, S.kernel == 3 ? p - 2 : 0, g, C, C + p * p, A, B, Cd, J.tx[i] * S.inv_R0,
                               J.ty[i] * S.inv_R0, J.tz[i] * S.inv_R0, pf, gx, gy, gz);
            ph += pf + (g == 0 ? C[0] : 0.0);
            fx -= gx * S.inv_R0;
            fy -= gy * S.inv_R0;
            fz -= gz * S.inv_R0;
        }
    }
    ph = far_lanes_sum<FL>(ph);
    fx = far_lanes_sum<FL>(fx);
    fy = far_lanes_sum<FL>(fy);
    fz = far_lanes_sum<FL>(fz);
    if (!act || g != 0) return;
    const int64_t o = perm ? S.n_off + perm[S.n_off + i] : S.n_off + i;
    if (phi) phi[o] = ph;
    if (ex) ex[o] = fx;
    if (ey) ey[o] = fy;
    if (ez) ez[o] = fz;
    if (osort) {
        const int64_t gi = S.n_off + i;
        osort[4 * gi + 0] = ph;
        osort[4 * gi + 1] = fx;
        osort[4 * gi + 2] = fy;
        osort[4 * gi + 3] = fz;
    }
}

// ----------------------------------------------------------------------------
// host launchers
// ----------------------------------------------------------------------------
#define PS_LAUNCH(...) hipLaunchKernelGGL(__VA_ARGS__)

void launch_fill_i32(int* p, int64_t n, int v, hipStream_t st)
{
    if (n <= 0) return;
    int64_t g = (n + 255) / 256;
    if (g > 4096) g = 4096;
    PS_LAUNCH(k_fill_i32, dim3((unsigned)g), dim3(256), 0, st, p, n, v);
}
void launch_validate(int nsys, int nblk, const SysDev* sys, const double* X, const double* Y, const double* Z,
                     const double* Q, int* status, double* part, hipStream_t st)
{
    PS_LAUNCH(k_validate, dim3(nblk, nsys), dim3(256), 0, st, sys, X, Y, Z, Q, status, part);
    PS_LAUNCH(k_validate_final, dim3(nsys), dim3(64), 0, st, sys, part, nblk, status);
}
void launch_sort(int nsys, int64_t ncitems, int64_t max_ncell, const SysDev* sys, const CItem* citems, const double* X,
                 const double* Y, const double* Z, const double* Q, int* keys, int* slots, int* cnt, int* start,
                 int64_t ncnt_total, int scan_blocks, int64_t* scan_tot, int* perm, double* sx, double* sy, double* sz,
                 double* sq, hipStream_t st)
{
    launch_fill_i32(cnt, ncnt_total, 0, st);
    PS_LAUNCH(k_cell_keys, dim3((unsigned)ncitems), dim3(256), 0, st, sys, citems, X, Y, Z, keys, slots, cnt);
    PS_LAUNCH(k_scan_totals, dim3(scan_blocks, nsys), dim3(256), 0, st, sys, cnt, scan_tot);
    PS_LAUNCH(k_scan_chunks, dim3(scan_blocks, nsys), dim3(256), 0, st, sys, cnt, scan_tot, start);
    PS_LAUNCH(k_cell_scatter, dim3((unsigned)ncitems), dim3(256), 0, st, sys, citems, keys, slots, start, perm);
    PS_LAUNCH(k_cell_fixup, dim3((unsigned)((max_ncell + 255) / 256), nsys), dim3(256), 0, st, sys, start, perm);
    PS_LAUNCH(k_gather, dim3((unsigned)ncitems), dim3(256), 0, st, sys, citems, perm, X, Y, Z, Q, sx, sy, sz, sq);
}
void launch_near(int nsys, int64_t nnitems, const SysDev* sys, const NItem* nitems, const double* img,
                 const double* sx, const double* sy, const double* sz, const double* sq, int* ncount, int64_t* ioff,
                 int64_t* nnear, double* nx, double* ny, double* nz, double* nq, int* nbase, int* inv, hipStream_t st)
{
    PS_LAUNCH(k_near_count, dim3((unsigned)nnitems), dim3(256), 0, st, sys, nitems, img, sx, sy, sz, ncount);
    PS_LAUNCH(k_near_scan, dim3(nsys), dim3(1024), 0, st, sys, ncount, ioff, nnear);
    PS_LAUNCH(k_near_write, dim3((unsigned)nnitems), dim3(256), 0, st, sys, nitems, ioff, img, sx, sy, sz, sq, nx, ny,
              nz, nq, nbase, inv);
}
void launch_tblock(int64_t nitems, const PJob* jobs, const TItem* items, hipStream_t st)
{
    if (nitems <= 0) return;
    PS_LAUNCH(k_tblock, dim3((unsigned)nitems), dim3(256), 0, st, jobs, items);
}
void launch_p2p(int prec, int bt, bool field, int kern, int64_t nitems, const PJob* jobs, const PItem* items,
                hipStream_t st)
{
    if (nitems <= 0) return;
    const dim3 g((unsigned)nitems);
#define P2P_CASE(BT, K)                                                                                    \
    if (bt == BT && kern == K) {                                                                           \
        if (prec == 1) {                                                                                   \
            if (field) PS_LAUNCH((k_p2p_f32<BT, true, K>), g, dim3(BT), 0, st, jobs, items);               \
            else PS_LAUNCH((k_p2p_f32<BT, false, K>), g, dim3(BT), 0, st, jobs, items);                    \
        } else {                                                                                           \
            if (field) PS_LAUNCH((k_p2p_f64<BT, true, K>), g, dim3(BT), 0, st, jobs, items);               \
            else PS_LAUNCH((k_p2p_f64<BT, false, K>), g, dim3(BT), 0, st, jobs, items);                    \
        }                                                                                                  \
        return;                                                                                            \
    }
    P2P_CASE(64, 0)
    P2P_CASE(128, 0)
    P2P_CASE(256, 0)
    P2P_CASE(64, 1)
    P2P_CASE(128, 1)
    P2P_CASE(256, 1)
    P2P_CASE(64, 2)
    P2P_CASE(128, 2)
    P2P_CASE(256, 2)
    P2P_CASE(64, 3)
    P2P_CASE(128, 3)
    P2P_CASE(256, 3)
#undef P2P_CASE
}
void launch_chk_f32(int kern, int64_t nitems, const PJob* jobs, const PItem* items, hipStream_t st)
{
    if (nitems <= 0) return;
    if (kern == 1)
        PS_LAUNCH((k_chk_f32<kChkWaves, 1>), dim3((unsigned)nitems), dim3(64 * kChkWaves), 0, st, jobs, items);
    else if (kern == 2)
        PS_LAUNCH((k_chk_f32<kChkWaves, 2>), dim3((unsigned)nitems), dim3(64 * kChkWaves), 0, st, jobs, items);
    else
        PS_LAUNCH((k_chk_f32<kChkWaves, 0>), dim3((unsigned)nitems), dim3(64 * kChkWaves), 0, st, jobs, items);
}
void launch_decay_rhs(int nsys, int maxdec, int64_t maxpts, const SysDev* sys, const PJob* djobs, const double* dpts,
                      int64_t dec_tot, double* dfield, const double* dw, const double* drows, double* f, hipStream_t st)
{
    if (maxdec <= 0) return;
    PS_LAUNCH(k_decay_fields, dim3(static_cast<unsigned>((maxpts + 255) / 256), nsys), dim3(256), 0, st, sys, djobs,
              dpts, dec_tot, dfield);
    PS_LAUNCH(k_decay_rhs, dim3(maxdec, nsys), dim3(256), 0, st, sys, dpts, dec_tot, dfield, dw, drows, f);
}
void launch_solve(int nsys, int maxL, int maxP, const SysDev* sys, const PJob* cjobs, const int* slot,
                  const double* pinv, double* coef, double* f, hipStream_t st)
{
    PS_LAUNCH(k_rhs, dim3((maxL + 63) / 64, nsys), dim3(1024), 0, st, sys, cjobs, slot, f);
    PS_LAUNCH(k_gemv, dim3((maxP - 1 + 3) / 4, nsys), dim3(256), 0, st, sys, pinv, f, coef);
}
void launch_mean(int nsys, int64_t nwitems, const SysDev* sys, const CItem* witems, const int64_t* nnear,
                 const double* nx, const double* ny, const double* nz, const double* nq, double* part,
                 int64_t nmitems, int mcols, const MItem* mitems, const int* imap, const double* img,
                 const double* sx, const double* sy, const double* sz, const double* sq, double* mpart,
                 const double* bm, double* coef, hipStream_t st)
{
    if (nwitems > 0) PS_LAUNCH(k_mean, dim3((unsigned)nwitems), dim3(256), 0, st, sys, witems, nnear, nx, ny, nz, nq, part);
    if (nmitems > 0)
        PS_LAUNCH(k_mean_corners, dim3((unsigned)nmitems), dim3(kMeanWave), sizeof(unsigned) * kMeanWave * mcols, st,
                  sys, mitems, imap, img, sx, sy, sz, sq, mpart);
    PS_LAUNCH(k_c1, dim3(nsys), dim3(256), 0, st, sys, part, mpart, bm, coef);
}
void launch_far(int lanes, int64_t nitems, int maxP, int maxp, const SysDev* sys, const CItem* items,
                const PJob* pjobs, const PJob* fjobs, const double* coef, const double* rec, const int* perm,
                double* phi, double* ex, double* ey, double* ez, double* osort, hipStream_t st)
{
    if (nitems <= 0) return;
    const size_t lds = (3 * maxP + maxp) * sizeof(double);
    if (lanes == 8)
        PS_LAUNCH(k_far_combine<8>, dim3((unsigned)nitems), dim3(256), lds, st, sys, items, pjobs, fjobs, coef, rec,
                  perm, phi, ex, ey, ez, osort);
    else
        PS_LAUNCH(k_far_combine<4>, dim3((unsigned)nitems), dim3(256), lds, st, sys, items, pjobs, fjobs, coef, rec,
                  perm, phi, ex, ey, ez, osort);
}

}  // namespace ps

// ----------------------------------------------------------------------------
// energy and its gradient (adjoint of the discrete method)
// ----------------------------------------------------------------------------
namespace ps {

// E = (1/2) sum_i q_i phi_i over a system's particles (sorted order).
__global__ __launch_bounds__(256) void k_energy(const SysDev* __restrict__ sys, const double* __restrict__ sq,
                                                const double* __restrict__ osort, double* __restrict__ energy)
{
    __shared__ double sh[4];
    const SysDev& S = sys[blockIdx.x];
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < S.n; i += 256) acc += sq[S.n_off + i] * osort[4 * (S.n_off + i)];
    acc = block_reduce<0>(acc, sh);
    if (threadIdx.x == 0) energy[blockIdx.x] = 0.5 * acc;
}

// Partial moments u_t = sum_k q_k R^_t(x_k / R0), t >= 1, over a slice of the
// particles: one wave per workgroup evaluates the basis recurrence for 64
// particles at a time and reduces every term across its lanes; part[block][t].
// The biharmonic basis adds |u|^2 R^_t for degrees below p - 2 at t + p^2.
// (One wave keeps the LDS at (3P + p) doubles, under 40 KB for p <= 40.)
__global__ __launch_bounds__(64) void k_moment(const SysDev* __restrict__ sys, const double* __restrict__ sx,
                                               const double* __restrict__ sy, const double* __restrict__ sz,
                                               const double* __restrict__ sq, const double* __restrict__ rec,
                                               double* __restrict__ part)
{
    extern __shared__ double lds[];
    const SysDev& S = sys[0];
    const int P = S.P, p = S.p, p2 = S.kernel == 3 ? p - 2 : 0;
    double* A = lds;
    double* B = lds + P;
    double* Cd = lds + 2 * P;
    double* acc = lds + 2 * P + p;  // [P]
    for (int t = threadIdx.x; t < P; t += 64) {
        A[t] = rec[S.rec_off + t];
        B[t] = rec[S.rec_off + P + t];
        acc[t] = 0.0;
    }
    for (int t = threadIdx.x; t < p; t += 64) Cd[t] = rec[S.rec_off + 2 * P + t];
    __syncthreads();
    const int lane = threadIdx.x & 63;
    for (int64_t base = (int64_t)blockIdx.x * 64; base < S.n; base += (int64_t)gridDim.x * 64) {
        const int64_t i = base + lane;
        const bool v = i < S.n;
        const double x = v ? sx[S.n_off + i] * S.inv_R0 : 0.0, y = v ? sy[S.n_off + i] * S.inv_R0 : 0.0,
                     z = v ? sz[S.n_off + i] * S.inv_R0 : 0.0, q = v ? sq[S.n_off + i] : 0.0;
        const double r2 = x * x + y * y + z * z, qr2 = q * r2;
        double dA = 1.0, dB = 0.0;
        for (int m = 0; m < p; ++m) {
            if (m > 0) {
                const double c = Cd[m];
                const double nA = -c * (x * dA + y * dB);
                const double nB = c * (y * dA - x * dB);
                dA = nA;
                dB = nB;
            }
            for (int s = 0; s < (m ? 2 : 1); ++s) {
                const int mm = s ? -m : m;
                double v1 = s ? dB : dA, v2 = 0.0;
                const int t0 = m * m + m + mm;
                if (t0 > 0) {
                    const double r = wave_sum(q * v1);
                    if (lane == 0) acc[t0] += r;
                }
                if (m < p2) {
                    const double r = wave_sum(qr2 * v1);
                    if (lane == 0) acc[p * p + t0] += r;
                }
                for (int n = m + 1; n < p; ++n) {
                    const int t = n * n + n + mm;
                    const double vv = -A[t] * z * v1 - B[t] * r2 * v2;
                    const double r = wave_sum(q * vv);
                    if (lane == 0) acc[t] += r;
                    if (n < p2) {
                        const double r3 = wave_sum(qr2 * vv);
                        if (lane == 0) acc[p * p + t] += r3;
                    }
                    v2 = v1;
                    v1 = vv;
                }
            }
        }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < P; t += 64) part[(int64_t)blockIdx.x * P + t] = acc[t];
}

// The plane's moments u_t = sum_k q_k R_t(x_k / R0): R_{2n-1} = Re w^n,
// R_{2n} = Im w^n (w = (x + iy)/R0), reduced across the wave per term;
// part[block][t] as k_moment.
__global__ __launch_bounds__(64) void k_moment2d(const SysDev* __restrict__ sys, const double* __restrict__ sx,
                                                 const double* __restrict__ sy, const double* __restrict__ sq,
                                                 double* __restrict__ part)
{
    extern __shared__ double acc[];  // [P]
    const SysDev& S = sys[0];
    const int P = S.P, p = S.p;
    for (int t = threadIdx.x; t < P; t += 64) acc[t] = 0.0;
    __syncthreads();
    const int lane = threadIdx.x & 63;
    for (int64_t base = (int64_t)blockIdx.x * 64; base < S.n; base += (int64_t)gridDim.x * 64) {
        const int64_t i = base + lane;
        const bool v = i < S.n;
        const double x = v ? sx[S.n_off + i] * S.inv_R0 : 0.0, y = v ? sy[S.n_off + i] * S.inv_R0 : 0.0;
        const double q = v ? sq[S.n_off + i] : 0.0;
        double wr = 1.0, wi = 0.0;
        for (int n = 1; n < p; ++n) {
            const double a = wr * x - wi * y, b = wr * y + wi * x;
            wr = a;
            wi = b;
            const double sr = wave_sum(q * wr), si = wave_sum(q * wi);
            if (lane == 0) {
                acc[2 * n - 1] += sr;
                acc[2 * n] += si;
            }
        }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < P; t += 64) part[(int64_t)blockIdx.x * P + t] = acc[t];
}

// u = sum of the moment partials; w = (A^+)^T u; adjoint sources: the sorted
// particles, then +w_l at the partners y~_l, then -w_l at the check points y_l.
// (the moment partials hold u_t at part[b * stride + t - toff] for t >= 1)
// The decay rows' weights w_r (rows L..Lf-1) go to wdec.
__global__ __launch_bounds__(256) void k_adj_weights(const SysDev* __restrict__ sys, const double* __restrict__ part,
                                                     int nblk, int stride, int toff, const double* __restrict__ pinv,
                                                     const double* __restrict__ chk, int64_t chk_tot,
                                                     double* __restrict__ ax, double* __restrict__ ay,
                                                     double* __restrict__ az, double* __restrict__ aq,
                                                     double* __restrict__ wdec)
{
    extern __shared__ double u[];
    const SysDev& S = sys[0];
    const int P = S.P, L = S.L;
    for (int t = threadIdx.x; t < P; t += 256) {
        double s = 0.0;
        if (t >= 1)
            for (int b = 0; b < nblk; ++b) s += part[(int64_t)b * stride + t - toff];
        u[t] = s;
    }
    __syncthreads();
    for (int l = threadIdx.x; l < L; l += 256) {
        double w = 0.0;
        for (int t = 1; t < P; ++t) w = __builtin_fma(pinv[S.pinv_off + (int64_t)(t - 1) * S.Lf + l], u[t], w);
        const int64_t o1 = S.n + l, o2 = S.n + L + l;
        const double* cx = chk + S.chk_off;
        const double* cy = chk + chk_tot + S.chk_off;
        const double* cz = chk + 2 * chk_tot + S.chk_off;
        ax[o1] = cx[L + l];
        ay[o1] = cy[L + l];
        az[o1] = cz[L + l];
        aq[o1] = w;
        ax[o2] = cx[l];
        ay[o2] = cy[l];
        az[o2] = cz[l];
        aq[o2] = -w;
    }
    for (int l = S.L + threadIdx.x; l < S.Lf; l += 256) {
        double w = 0.0;
        for (int t = 1; t < P; ++t) w = __builtin_fma(pinv[S.pinv_off + (int64_t)(t - 1) * S.Lf + l], u[t], w);
        wdec[l - S.L] = w;
    }
}

// Adjoint sources of the decay rows (slab, wire): with the row weights w_r,
// a_i = sum_r w_r W_ri and b_i = sum_r w_r c_r W_ri at decay point i, where
// W_ri is row r's quadrature weight times its trigonometric factor at the point
// (as in k_decay_rhs) and c_r = -s|k| (slab plane s) or beta (wire).  One
// thread per point, rows in order.
__global__ __launch_bounds__(256) void k_adj_decay_src(const SysDev* __restrict__ sys, const double* __restrict__ dpts,
                                                       int64_t dec_tot, const double* __restrict__ dw,
                                                       const double* __restrict__ drows,
                                                       const double* __restrict__ wdec, double* __restrict__ ad,
                                                       double* __restrict__ bd)
{
    const SysDev& S = sys[0];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= (int64_t)S.nsurf * S.m2) return;
    const double x = dpts[S.dec_off + i], y = dpts[dec_tot + S.dec_off + i], z = dpts[2 * dec_tot + S.dec_off + i];
    double a = 0.0, b = 0.0;
    if (S.periodic == 1) {
        const double th = atan2(z, y), wi = dw[S.dw_off + i];
        for (int r = 0; r < S.ndec; ++r) {
            const double* row = drows + S.drow_off + (int64_t)r * 5;
            const double tx = row[3] != 0.0 ? sin(row[0] * x) : cos(row[0] * x);
            const double tt = row[4] != 0.0 ? sin(row[1] * th) : cos(row[1] * th);
            const double W = wdec[r] * (wi * (tx * tt));
            a += W;
            b = __builtin_fma(W, row[2], b);
        }
    } else {
        const int plane = static_cast<int>(i / S.m2);
        const double wi = dw[S.dw_off + i % S.m2];
        for (int r = 0; r < S.ndec; ++r) {
            const double* row = drows + S.drow_off + (int64_t)r * 5;
            if ((row[3] > 0.0 ? 0 : 1) != plane) continue;
            const double ph = row[0] * x + row[1] * y;
            const double W = wdec[r] * (wi * (row[4] != 0.0 ? sin(ph) : cos(ph)));
            a += W;
            b = __builtin_fma(W, -row[3] * row[2], b);
        }
    }
    ad[i] = a;
    bd[i] = b;
}

// The decay points' part of psi at the near entries: a charge b_i and a dipole
// -a_i n_i at each decay point y_i (n_i = +z on a slab's planes, the outward
// radial direction on the wire's cylinder):
//   psi(z) = sum_i b_i / r + a_i n_i . (y_i - z) / r^3,  r = |z - y_i|,
// written as psi and the field -grad psi into dpart[4][stride], the layout of a
// split of the adjoint pair sum.  The decay points stay R0/10 from every near
// entry.  FP64; one thread per near entry, decay points staged in LDS.
__global__ __launch_bounds__(256) void k_adj_decay(const SysDev* __restrict__ sys, const double* __restrict__ nx,
                                                   const double* __restrict__ ny, const double* __restrict__ nz,
                                                   int64_t nb, const double* __restrict__ dpts, int64_t dec_tot,
                                                   const double* __restrict__ ad, const double* __restrict__ bd,
                                                   double* __restrict__ dpart)
{
    __shared__ double sy[256][8];  // y, n, a, b
    const SysDev& S = sys[0];
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const bool act = e < nb;
    const double zx = act ? nx[S.near_off + e] : 0.0, zy = act ? ny[S.near_off + e] : 0.0,
                 zz = act ? nz[S.near_off + e] : 0.0;
    const int64_t npts = (int64_t)S.nsurf * S.m2;
    double ps = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
    for (int64_t t0 = 0; t0 < npts; t0 += 256) {
        __syncthreads();
        const int64_t j = t0 + threadIdx.x;
        if (j < npts) {
            const double x = dpts[S.dec_off + j], y = dpts[dec_tot + S.dec_off + j], z = dpts[2 * dec_tot + S.dec_off + j];
            double nxv = 0.0, nyv = 0.0, nzv = 1.0;
            if (S.periodic == 1) {
                const double rho = sqrt(y * y + z * z);
                nyv = y / rho;
                nzv = z / rho;
            }
            sy[threadIdx.x][0] = x;
            sy[threadIdx.x][1] = y;
            sy[threadIdx.x][2] = z;
            sy[threadIdx.x][3] = nxv;
            sy[threadIdx.x][4] = nyv;
            sy[threadIdx.x][5] = nzv;
            sy[threadIdx.x][6] = ad[j];
            sy[threadIdx.x][7] = bd[j];
        }
        __syncthreads();
        const int cnt = npts - t0 < 256 ? static_cast<int>(npts - t0) : 256;
        for (int k = 0; k < cnt; ++k) {
            const double dx = zx - sy[k][0], dy = zy - sy[k][1], dz = zz - sy[k][2];
            const double r2 = __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx));
            const double ri = 1.0 / sqrt(r2), ri3 = ri * ri * ri;
            const double nd = __builtin_fma(sy[k][5], dz, __builtin_fma(sy[k][4], dy, sy[k][3] * dx));  // n . (z - y)
            const double a = sy[k][6], b = sy[k][7];
            ps += b * ri - a * nd * ri3;
            // grad psi = -b d / r^3 - a (n / r^3 - 3 (n . d) d / r^5)
            const double c = 3.0 * a * nd * ri3 / r2 - b * ri3;
            gx += c * dx - a * sy[k][3] * ri3;
            gy += c * dy - a * sy[k][4] * ri3;
            gz += c * dz - a * sy[k][5] * ri3;
        }
    }
    if (act) {
        dpart[e] = ps;
        dpart[nb + e] = -gx;
        dpart[2 * nb + e] = -gy;
        dpart[3 * nb + e] = -gz;
    }
}

// The biharmonic fit's gradient rows in the adjoint: with their weights
// w[k L + l] (k = x, y, z), a dipole D_l = R0 (w[l], w[L + l], w[2L + l]) at each
// partner y~_l and -D_l at each check point y_l, for K = r:
//   psi(z) = sum_l D_l . [(y~_l - z)/|y~_l - z| - (y_l - z)/|y_l - z|],
//   grad psi = sum_l +-[-D_l/r + (D_l . (y - z)) (y - z)/r^3],
// at every near entry z (FP64, 256 check targets staged in LDS at a time);
// dpart receives psi and -grad psi as k_adj_decay's.
__global__ __launch_bounds__(256) void k_adj_dip(const SysDev* __restrict__ sys, const double* __restrict__ nx,
                                                 const double* __restrict__ ny, const double* __restrict__ nz,
                                                 int64_t nb, const double* __restrict__ chk, int64_t chk_tot,
                                                 const double* __restrict__ wg, double* __restrict__ dpart)
{
    __shared__ double sy[256][6];  // y, sign x D
    const SysDev& S = sys[0];
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const bool act = e < nb;
    const double zx = act ? nx[S.near_off + e] : 0.0, zy = act ? ny[S.near_off + e] : 0.0,
                 zz = act ? nz[S.near_off + e] : 0.0;
    const int L = S.L, npts = 2 * L;
    double ps = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
    for (int t0 = 0; t0 < npts; t0 += 256) {
        __syncthreads();
        const int j = t0 + threadIdx.x;
        if (j < npts) {  // check target j: y_l for j < L (sign -), y~_l after (sign +)
            const int l = j < L ? j : j - L;
            const double sg = j < L ? -S.R0 : S.R0;
            sy[threadIdx.x][0] = chk[S.chk_off + j];
            sy[threadIdx.x][1] = chk[chk_tot + S.chk_off + j];
            sy[threadIdx.x][2] = chk[2 * chk_tot + S.chk_off + j];
            sy[threadIdx.x][3] = sg * wg[l];
            sy[threadIdx.x][4] = sg * wg[L + l];
            sy[threadIdx.x][5] = sg * wg[2 * L + l];
        }
        __syncthreads();
        const int cnt = npts - t0 < 256 ? npts - t0 : 256;
        for (int k = 0; k < cnt; ++k) {
            const double dx = sy[k][0] - zx, dy = sy[k][1] - zy, dz = sy[k][2] - zz;  // y - z
            const double r2 = __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx));
            const double ri = r2 > 0.0 ? 1.0 / sqrt(r2) : 0.0;  // a coincident point adds nothing, as K(0) = 0
            const double dd = __builtin_fma(sy[k][5], dz, __builtin_fma(sy[k][4], dy, sy[k][3] * dx)) * ri;
            ps += dd;
            const double c = dd * ri * ri;
            gx += __builtin_fma(c, dx, -sy[k][3] * ri);
            gy += __builtin_fma(c, dy, -sy[k][4] * ri);
            gz += __builtin_fma(c, dz, -sy[k][5] * ri);
        }
    }
    if (act) {
        dpart[e] = ps;
        dpart[nb + e] = -gx;
        dpart[2 * nb + e] = -gy;
        dpart[3 * nb + e] = -gz;
    }
}

__global__ void k_copy4(int64_t n, const double* __restrict__ a, const double* __restrict__ b,
                        const double* __restrict__ c, const double* __restrict__ d, double* __restrict__ A,
                        double* __restrict__ B, double* __restrict__ C, double* __restrict__ D)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        A[i] = a[i];
        B[i] = b[i];
        C[i] = c[i];
        D[i] = d[i];
    }
}

// Gather psi and grad psi from every near image of each particle (inverse map,
// image order) and form the unprojected gradients in sorted order:
// dq[i] = (phi_i + sum psi)/2,  dx[k][i] = q_i/2 (grad phi_i + sum grad psi).
// The pair kernel returned the field of psi, i.e. -grad psi.
// dpart (may be null): psi and its field from the decay points, [4][dstride].
__global__ __launch_bounds__(256) void k_adj_gather(const SysDev* __restrict__ sys, const PJob* __restrict__ ajob,
                                                    const int* __restrict__ inv, const double* __restrict__ sq,
                                                    const double* __restrict__ osort, int exact,
                                                    const double* __restrict__ dpart, int64_t dstride,
                                                    double* __restrict__ dq, double* __restrict__ dx)
{
    const SysDev& S = sys[0];
    const int64_t i = blockIdx.x * 256ll + threadIdx.x;
    if (i >= S.n) return;
    const double* o = osort + 4 * (S.n_off + i);
    const double q = sq[S.n_off + i];
    if (!exact) {
        dq[i] = o[0];
        dx[i] = -q * o[1];
        dx[S.n + i] = -q * o[2];
        dx[2 * S.n + i] = -q * o[3];
        return;
    }
    const PJob& J = ajob[0];
    double ps = 0.0, fx = 0.0, fy = 0.0, fz = 0.0;
    for (int m = 0; m < S.nimg; ++m) {
        const int e = inv[S.inv_off + (int64_t)m * S.n + i];
        if (e < 0) continue;
        for (int s = 0; s < J.nsplit; ++s) {
            const double* P_ = J.part + (int64_t)s * 4 * J.nt;
            ps += P_[e];
            fx += P_[J.nt + e];
            fy += P_[2 * J.nt + e];
            fz += P_[3 * J.nt + e];
        }
        if (dpart) {
            ps += dpart[e];
            fx += dpart[dstride + e];
            fy += dpart[2 * dstride + e];
            fz += dpart[3 * dstride + e];
        }
    }
    dq[i] = 0.5 * (o[0] + ps);
    dx[i] = 0.5 * q * (-o[1] - fx);
    dx[S.n + i] = 0.5 * q * (-o[2] - fy);
    dx[2 * S.n + i] = 0.5 * q * (-o[3] - fz);
}

// Remove the mean of dq (neutral charges; not for the screened kernel, whose
// energy is defined for any charges), scale by gE and store in the original
// particle order.
__global__ __launch_bounds__(1024) void k_adj_finish(const SysDev* __restrict__ sys, const int* __restrict__ perm,
                                                     const double* __restrict__ dq, const double* __restrict__ dx,
                                                     const double* __restrict__ gE, double* __restrict__ oq,
                                                     double* __restrict__ ox, double* __restrict__ oy,
                                                     double* __restrict__ oz)
{
    __shared__ double sh[16];
    const SysDev& S = sys[0];
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < S.n; i += 1024) acc += dq[i];
    acc = block_reduce<0>(acc, sh);
    const double mean = S.kernel != 1 ? acc / (double)S.n : 0.0;
    const double g = gE[0];
    for (int64_t i = threadIdx.x; i < S.n; i += 1024) {
        const int64_t o = perm[S.n_off + i];
        if (oq) oq[o] = g * (dq[i] - mean);
        if (ox) ox[o] = g * dx[i];
        if (oy) oy[o] = g * dx[S.n + i];
        if (oz) oz[o] = g * dx[2 * S.n + i];
    }
}

void launch_energy(int nsys, const SysDev* sys, const double* sq, const double* osort, double* energy, hipStream_t st)
{
    PS_LAUNCH(k_energy, dim3(nsys), dim3(256), 0, st, sys, sq, osort, energy);
}
void launch_moments(int P, int p, const SysDev* sys, const double* sx, const double* sy, const double* sz,
                    const double* sq, const double* rec, double* mom_part, int mom_blocks, hipStream_t st)
{
    PS_LAUNCH(k_moment, dim3(mom_blocks), dim3(64), (3 * P + p) * sizeof(double), st, sys, sx, sy, sz, sq, rec,
              mom_part);
}
void launch_moments2d(int P, const SysDev* sys, const double* sx, const double* sy, const double* sq, double* mom_part,
                      int mom_blocks, hipStream_t st)
{
    PS_LAUNCH(k_moment2d, dim3(mom_blocks), dim3(64), P * sizeof(double), st, sys, sx, sy, sq, mom_part);
}
void launch_adjoint_sources(int P, int L, int64_t n, const SysDev* sys, const double* sx, const double* sy,
                            const double* sz, const double* sq, const double* mom_part, int mom_blocks, int stride,
                            int toff, const double* pinv, const double* chk, int64_t chk_tot, double* ax, double* ay,
                            double* az, double* aq, double* wdec, hipStream_t st)
{
    PS_LAUNCH(k_copy4, dim3((unsigned)std::min<int64_t>(1024, (n + 255) / 256)), dim3(256), 0, st, n, sx, sy, sz, sq,
              ax, ay, az, aq);
    PS_LAUNCH(k_adj_weights, dim3(1), dim3(256), P * sizeof(double), st, sys, mom_part, mom_blocks, stride, toff, pinv,
              chk, chk_tot, ax, ay, az, aq, wdec);
}
void launch_adjoint_decay(int64_t npts, int64_t nb, const SysDev* sys, const double* dpts, int64_t dec_tot,
                          const double* dw, const double* drows, const double* wdec, double* ad, double* bd,
                          const double* nx, const double* ny, const double* nz, double* dpart, hipStream_t st)
{
    if (npts <= 0 || nb <= 0) return;
    PS_LAUNCH(k_adj_decay_src, dim3((unsigned)((npts + 255) / 256)), dim3(256), 0, st, sys, dpts, dec_tot, dw, drows,
              wdec, ad, bd);
    PS_LAUNCH(k_adj_decay, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, st, sys, nx, ny, nz, nb, dpts, dec_tot, ad,
              bd, dpart);
}
void launch_adjoint_dipoles(int64_t nb, const SysDev* sys, const double* nx, const double* ny, const double* nz,
                            const double* chk, int64_t chk_tot, const double* wg, double* dpart, hipStream_t st)
{
    if (nb <= 0) return;
    PS_LAUNCH(k_adj_dip, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, st, sys, nx, ny, nz, nb, chk, chk_tot, wg,
              dpart);
}
void launch_adjoint_finish(int64_t n, const SysDev* sys, const PJob* ajob, const int* inv, const double* sq,
                           const double* osort, int exact, const double* dpart, int64_t dstride, double* dq, double* dx,
                           const int* perm, const double* gE, double* oq, double* ox, double* oy, double* oz,
                           hipStream_t st)
{
    PS_LAUNCH(k_adj_gather, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, sys, ajob, inv, sq, osort, exact,
              dpart, dstride, dq, dx);
    PS_LAUNCH(k_adj_finish, dim3(1), dim3(1024), 0, st, sys, perm, dq, dx, gE, oq, ox, oy, oz);
}

}  // namespace ps

namespace ps {
// Resident workgroups per compute unit of the pair kernels (occupancy query).
int p2p_blocks_per_cu(int prec, int bt)
{
    int nb = 0;
    hipError_t e = hipErrorInvalidValue;
#define OCC(BT)                                                                                               \
    if (bt == BT)                                                                                             \
        e = prec == 1 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_p2p_f32<BT, true, 0>, BT, 0) \
                      : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_p2p_f64<BT, true, 0>, BT, 0);
    OCC(64)
    OCC(128)
    OCC(256)
#undef OCC
    return e == hipSuccess && nb > 0 ? nb : 1;
}
}  // namespace ps
