/*
 * periodic_sum.h -- C ABI of libperiodic_sum.so, an MI355X (gfx950) implementation
 * of the periodized sum of Gumerov & Duraiswami, "A method to compute periodic sums"
 * (arXiv:1310.4374), for the Coulomb kernel K(r) = 1/|r|, K(0) = 0 (eq. (1)).
 * Variants (ps_params): periodicity along two axes or one (periodic), the plane
 * with -log r (dim), the screened Coulomb kernel and the biharmonic kernel r
 * (kernel), the RBF basis and caller check points (basis, check_points).
 *
 * Problem (Sec. 1, eqs. (1)-(2)): N charges q_i at x_i in the box
 * Omega0 = [-d1/2,d1/2) x [-d2/2,d2/2) x [-d3/2,d3/2), sum q_i = 0, replicated on the
 * lattice p = (i1 d1, i2 d2, i3 d3).  Outputs, at the particles (Y0 = X0, the
 * molecular-dynamics case of Sec. 2.3) or at M separate targets in the box:
 * the periodic potential phi and the field -grad phi (Gaussian units).
 *
 * Method (Sec. 2.3, "set" and "get"; Sec. 3 for the Laplace kernel):
 *   phi = phi_near + phi_far + C1, where phi_near sums the sources x_j + p with
 *   |x_j + p| <= R_b directly (eq. (3)); phi_far = sum_{t>=2} C_t R_t(y) over the
 *   renormalized regular solid harmonics (eqs. (1.6)-(1.8)), here evaluated at
 *   y/R0; C = A^+ f is the least-squares fit of periodicity at L check points on
 *   the circumsphere and their periodic partners (eqs. (7)-(10)); C1 makes the
 *   box mean of phi zero (eqs. (pfx2)-(pfx4), App. B, App. C), the convention of
 *   Ewald summation (App. D).
 *
 * Conventions for every call:
 *   - Status: every call returns ps_status; PS_OK = 0.  No C++ exception crosses
 *     the ABI.  periodic_sum_last_error() returns a thread-local message for the
 *     last failure on the calling thread.
 *   - Memory: arrays marked "device" are device pointers on the plan's device;
 *     the caller owns them.  The library never frees, retains or writes past the
 *     documented extent of a caller's array.  The plan owns all of its workspace,
 *     which is allocated by the plan call and sized by n_max/m_max, so the eval
 *     calls never allocate device memory.
 *   - Layout: structure of arrays, FP64: x[n], y[n], z[n], q[n]; outputs phi[n]
 *     (or [m]), ex/ey/ez[n] (the three field components).
 *   - Streams: `stream` is a hipStream_t (NULL = the default stream).  Eval calls
 *     are asynchronous: they only enqueue work on that stream.  Argument errors
 *     are reported synchronously; data errors (non-neutral charges, particles
 *     outside the box) are detected on the device and returned by
 *     periodic_sum_status(), which synchronizes the stream.  With the
 *     environment variable PS_VALIDATE set (to anything but "0") when a plan is
 *     made, that plan's periodic_sum_eval, _eval_batched and _energy calls
 *     synchronize the stream and return those data errors themselves, except
 *     while the stream is being captured into a graph.
 *   - Concurrency: one plan serves one eval at a time (its workspace is shared);
 *     different plans are independent.  Results are bitwise reproducible for
 *     identical inputs and plan.
 */
#ifndef PERIODIC_SUM_H
#define PERIODIC_SUM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ps_plan_s* ps_plan;

typedef enum {
    PS_OK = 0,
    PS_E_INVALID = 1,      /* bad argument (null pointer, size, parameter range) */
    PS_E_NOT_NEUTRAL = 2,  /* |sum q| > 1e-12 sum |q| (eq. (1) requires neutrality) */
    PS_E_OUT_OF_BOX = 3,   /* a particle outside [-d/2, d/2), or a NaN coordinate or charge */
    PS_E_RANK = 4,         /* fitting matrix numerically rank deficient beyond rcond */
    PS_E_NOMEM = 5,        /* device or host allocation failed */
    PS_E_HIP = 6,          /* a HIP runtime call failed */
    PS_E_UNSUPPORTED = 7,  /* request outside what this library supports */
    PS_E_IO = 8            /* a plan file could not be written or read, or is not a valid plan file */
} ps_status;

typedef enum {
    PS_FP64 = 0,        /* every step in FP64 */
    PS_FP32_ACC64 = 1   /* particle and check-point near sums with FP32 pair
                           arithmetic on block-relative coordinates (two-float
                           coordinates for near source groups) and FP64
                           accumulation; the fit, the zero-mean constant and the
                           far field in FP64 */
} ps_precision;

typedef enum {
    PS_BASIS_SPHERICAL = 0,  /* renormalized regular solid harmonics, eqs. (1.6)-(1.8) */
    PS_BASIS_RBF = 1         /* the kernel at M given centres outside the box, eq. (5) */
} ps_basis;

typedef enum {
    PS_MEAN_ZERO = 0,   /* C1 from the zero box-mean condition, eq. (pfx3) */
    PS_MEAN_NONE = 1    /* C1 = 0 (remark after algorithm "get") */
} ps_mean;

typedef enum {
    PS_KERNEL_COULOMB = 0,  /* K(r) = 1/r, eq. (2) */
    PS_KERNEL_SCREENED = 1, /* K(r) = exp(-kappa r)/r, the screened Coulomb (Yukawa) kernel: one of the
                               "other kernels" the method applies to (Sec. 1).  Its lattice sum converges
                               absolutely, so the charges need not be neutral; Delta - kappa^2 has no nonzero
                               bounded periodic solution, so the fit has no null space: every coefficient of the
                               kernel-at-centres basis (eq. (5)) comes from A^+ f, and there is no constant C1
                               (the mean setting is ignored).  Needs PS_BASIS_RBF, periodic = 7. */
    PS_KERNEL_BIHARMONIC = 2  /* K(r) = r, the free-space Green's function of the biharmonic operator
                               (Delta^2 r = -8 pi delta): one of the equations that share the Laplace
                               kernel's null space, the constants (Sec. 3, null space of A).  Neutral
                               charges; C1 from the zero box mean (the closed-form mean of r over the
                               box) or 0.  Basis (Almansi): the p^2 renormalized solid harmonics of
                               degree <= p-1, then |y/R0|^2 times those of degree <= p-3,
                               P = p^2 + (p-2)^2; coef holds C1, the harmonics' C_2..C_{p^2}, then
                               the second set.  The fit has 4L rows: the L value rows, then for
                               k = x, y, z the L rows asking for the same periodicity of
                               d/du_k (u = y/R0) at each check pair (values alone do not fix a
                               biharmonic function), so the check-point sums carry the field.
                               Outputs: phi = sum q |x - x_j| periodized, E = -grad phi.  Needs
                               PS_BASIS_SPHERICAL, periodic = 7, dim 3, 3 <= p <= 30.  energy_vjp
                               (exact = 1): the gradient rows add a dipole R0 (w_xl, w_yl, w_zl) at
                               each partner and its negative at each check point to psi. */
} ps_kernel;

typedef struct {
    double  box[3];       /* d1, d2, d3 > 0 */
    int32_t p;            /* truncation number: degrees 0..p-1, P = p*p basis terms; 2 <= p <= 40 */
    double  R_b;          /* near radius; if <= 0, lambda * R0 is used, R0 = |d|/2 */
    double  lambda;       /* used only when R_b <= 0; must give R_b > R0 */
    int32_t precision;    /* ps_precision */
    int32_t mean;         /* ps_mean */
    double  rcond;        /* singular values below rcond * sigma_max are dropped from A^+; <= 0 -> 1e-13 */
    int64_t n_max;        /* largest particle count an eval may pass (workspace size) */
    int64_t m_max;        /* largest separate-target count an eval may pass (0: particles only) */
    int32_t tile_targets; /* targets per workgroup in the particle sums: 0 (default), 64, 128 or 256 */
    int32_t n_split;      /* source splits of the particle sums: 0 = automatic */
    int32_t basis;        /* ps_basis */
    int32_t n_centres;    /* PS_BASIS_RBF: number of centres M (1..4096) */
    const double* centres;      /* PS_BASIS_RBF: host [3*M], xyz interleaved, each with |x| > R0;
                                   the far field is sum_t C_t / |y - x_t| (an M-source pair sum) */
    int32_t n_check;      /* 0: Gauss spherical grid of L = 2p^2 - p points (Sec. 2.2);
                             > 0: that many caller-given check points */
    const double* check_points; /* host [3*n_check], xyz interleaved, |y| <= R0 and outside the box
                                   along at least one periodic axis (so a partner exists, Sec. 2.3 step 3) */
    int32_t periodic;     /* periodic axes as a bit mask: 0 or 7 = x, y and z; 3 = x and y only (a slab,
                             z free with vacuum on both sides; Sec. 1 says the extension may be along one
                             or two coordinates).  For a slab: in-plane images only; the Gauss check points
                             that an in-plane shift moves into S0 (partners along x or y); and, because
                             x/y periodicity leaves the far field's x/y-periodic harmonic modes free, decay
                             rows in the fit: on the planes z = +-(d3/2 + R0/10) every in-plane Fourier
                             mode k = 2 pi (n1/d1, n2/d2), |n1|, |n2| <= ceil(p/4) + 1, satisfies
                             <(d/dz + s|k|) phi, trig(k.rho)> = 0 (s = +1 above, -1 below; k = 0 is
                             Gauss's law), by m x m Gauss-Legendre points per plane,
                             m = max(2p + 8, ceil(40 max(d1, d2) / R0)).  1 = x only (a wire, y and z
                             free): images along x only; the Gauss check points with |y_1| > d1/2,
                             partners along x; decay rows on the cylinder rho = rho_d around the x axis,
                             rho_d = |(d2, d3)|/2 + R0/10 (rho, theta polar in the y-z plane): outside it
                             each Fourier mode (k = 2 pi n/d1, m) of the potential is the decaying one,
                             so <(d/drho - beta) phi, trig(k x) trig(m theta)> = 0 for n = 0..ceil(p/4)+1,
                             m = 0..p-1, with beta = k K_m'(k rho_d)/K_m(k rho_d) for n > 0 and -m/rho_d
                             for n = 0, by mx Gauss-Legendre points in x, mx = max(2p + 8,
                             ceil(40 d1 / R0)), times mt equispaced angles, mt = max(4p,
                             ceil(80 pi rho_d / R0)).  With fewer than three axes: spherical basis,
                             Coulomb kernel. */
    int32_t kernel;       /* ps_kernel (PS_KERNEL_COULOMB when zero-initialised) */
    double  kappa;        /* PS_KERNEL_SCREENED: the screening constant, 0 < kappa <= 64 / R0 */
    int32_t dim;          /* 0 or 3: three dimensions.  2: the method in the plane (Sec. 1 says it applies to
                             2-D problems): charges at (x, y) in the d1 x d2 rectangle (box[2] is ignored),
                             periodic along x and y, kernel K(r) = -log r (the 2-D Coulomb kernel; kernel must be
                             PS_KERNEL_COULOMB), neutral charges.  R0 = |(d1, d2)|/2; near set = images
                             (i d1, j d2) in the disc R_b; basis 1, Re w^n, Im w^n, w = (x + iy)/R0,
                             n = 1..p-1 (P = 2p - 1), 2 <= p <= 128; L = 4p check points equispaced on the
                             circumcircle (theta_l = 2 pi l / L; n_check must be 0), partners as in 3-D over
                             the two axes; C1 from the zero box mean with the closed-form potential of a
                             uniform rectangle.  z and target z pointers may be NULL (they are not read);
                             ez outputs, when given, receive zeros.  Spherical basis (meaning the plane's
                             harmonic polynomials) only; periodic must be 0, 7 or 3. */
    int32_t reserved;     /* 0 */
} ps_params;

typedef struct {
    int32_t p, P, L;          /* truncation number, basis size (M + 1 for RBF), check points */
    int32_t n_images;         /* lattice images whose box meets the ball |x| <= R_b */
    int32_t rank;             /* numerical rank of A (P-1 when full) */
    double  R0, R_b, cond;    /* circumradius, near radius, sigma_max/sigma_min(kept) */
    int64_t n_near_last;      /* N_b of the last completed eval (synchronizes) */
    int32_t tile_targets, n_split;
    int32_t nsys;             /* 1, or the number of systems of a batched plan */
    int32_t mean_corners;     /* systems whose box mean (eq. (pfx4)) the last particle-count shape sums by
                                 corner points rather than per near entry (a launch-size choice, same result) */
    int64_t profiled_evals;   /* evals whose stage events were recorded (see periodic_sum_set_profiling);
                                 graph launches of the batched path never record events */
    int64_t forward_epoch;    /* count of "get" passes enqueued or launched on this plan (eval, energy,
                                 batched eval); the pass the plan's workspace holds last */
    int32_t periodic;         /* periodic axes of system 0 (7, 3 or 1) */
    int32_t n_rows;           /* rows of system 0's fit: L periodicity rows, then (slab, wire) the decay rows */
    double  kappa;            /* screening constant (0 for the Coulomb kernel) */
    int32_t kernel;           /* ps_kernel of the plan (every system of a batch shares it) */
    int32_t dim;              /* 3, or 2 for a plan in the plane (every system of a batch shares it) */
    double  tune_ms;          /* periodic_sum_autotune: median ms per eval of the chosen candidate (0: not tuned) */
    double  tune_second_ms;   /* the same for the runner-up: the margin the choice rests on */
} ps_plan_info;

/* Algorithm "set" (Sec. 2.3, steps 1-6) on the host in FP64: circumradius and
 * near radius, the Gauss spherical grid of L = 2p^2 - p check points on the
 * circumsphere (Sec. 2.2) or the caller's points, their partners shifted by one
 * box period along the coordinate that moves them deepest into the sphere, the
 * fitting matrix A (eq. (8); for the spherical basis the constant function is
 * dropped, Sec. 3; for the RBF basis A_lt = K(y_l - x_t) - K(y~_l - x_t)), its
 * pseudo-inverse by Householder QR + one-sided Jacobi SVD with cut-off rcond
 * (eq. (10)), and the box integrals R_t^(0): tensor Gauss-Legendre for the
 * spherical basis (App. B), the box-mean potential at each centre for the RBF
 * basis (App. C).  Host arrays in prm are read during the call only.
 * Uploads these and allocates all device workspace on `device`.
 * prm: host pointer, read during the call only.  *out receives the plan.
 * Errors: PS_E_INVALID (parameters out of range, bad point sets),
 * PS_E_UNSUPPORTED (n_max times the number of lattice images exceeds 2^31 - 1
 * near-list entries), PS_E_NOMEM, PS_E_HIP. */
ps_status periodic_sum_plan(const ps_params* prm, int device, ps_plan* out);

/* Algorithm "get" (Sec. 2.3, steps 1-8) on the device, one system:
 * near-set build (steps 1-2), near sums at the 2L check points (step 3; pair
 * arithmetic in the plan's precision, FP64 accumulation), f and C = A^+ f in
 * FP64 (steps 4-5), the zero-mean constant C1 (step 6, eq. (pfx3)-(pfx4)),
 * near sums and the far-field expansion with its gradient at the targets
 * (steps 3 and 7), and the combination (step 8).
 *   n, x, y, z, q : particle count (1 <= n <= n_max) and device arrays [n].
 *   m, tx, ty, tz : m = 0 and NULL pointers: targets are the particles, and the
 *                   pair of a particle with itself is excluded (K(0) = 0);
 *                   m > 0: m <= m_max separate device targets in the box.
 *   phi           : device [n] (or [m]) potential.
 *   ex, ey, ez    : device [n] (or [m]) field -grad phi; all three NULL to skip
 *                   nothing (the field is always computed) but not store it.
 * Enqueued on `stream`; returns before the work completes.  The first call
 * for a given (n, m, target pointers) builds and uploads the plan's work
 * tables, which synchronizes `stream`; later calls with the same shape only
 * enqueue kernels (no allocation, memset or synchronization), so they may be
 * captured into a hipGraph by the caller. */
ps_status periodic_sum_eval(ps_plan plan, int64_t n,
                            const double* x, const double* y, const double* z, const double* q,
                            int64_t m, const double* tx, const double* ty, const double* tz,
                            double* phi, double* ex, double* ey, double* ez, void* stream);

/* For callers that cannot allocate device memory (code under hipGraph capture,
 * tight serving loops, harnesses that forbid hipMalloc): periodic_sum_eval at
 * the particles (targets = particles, as with m = 0) whose pair kernels write
 * their partial sums, the eval's largest scratch, into a static device array of
 * the library instead of the plan's buffers.  The array holds 8 Mi doubles
 * (64 MiB) per device for the life of the process; its address is looked up
 * once per device when a plan is made there.  Same kernels and work split as
 * periodic_sum_eval, so the results are bitwise those of periodic_sum_eval.
 * The call allocates nothing; like periodic_sum_eval, its first call for a
 * particle count builds and uploads the plan's work tables (host work and a
 * stream synchronization, no allocation), later calls only enqueue kernels.
 * Every call on a device shares that device's array, which keeps the last
 * call's contents: calls that overlap in time on one device (other streams,
 * other plans) race and must be ordered by the caller.  Every element a call
 * reads was written earlier in the same call, so nothing needs clearing.
 * Arguments as periodic_sum_eval with m = 0.
 * Errors: PS_E_INVALID (as periodic_sum_eval, or a batched plan),
 * PS_E_UNSUPPORTED (an RBF-basis, slab, wire or biharmonic plan, or partial
 * sums of this n beyond the array's 8 Mi doubles: 4 n x (source splits) +
 * 2L x (check splits)),
 * PS_E_HIP. */
ps_status periodic_sum_eval_noalloc(ps_plan plan, int64_t n,
                                    const double* x, const double* y, const double* z, const double* q,
                                    double* phi, double* ex, double* ey, double* ez, void* stream);

/* Energy E = (1/2) sum_i q_i phi(x_i) at the particles, with phi and the field
 * as in periodic_sum_eval (outputs may be NULL).  energy: device pointer to one
 * double, written by a deterministic reduction. */
ps_status periodic_sum_energy(ps_plan plan, int64_t n,
                              const double* x, const double* y, const double* z, const double* q,
                              double* energy, double* phi, double* ex, double* ey, double* ez,
                              void* stream);

/* Vector-Jacobian product of the energy: dEdx/dEdy/dEdz/dEdq [n] (device) receive
 * gE * dE/dx_i etc., gE read from a device scalar.
 *   exact = 1: the exact derivative of the discrete method.  With
 *     u = sum_k q_k R(x_k), w = (A^+)^T u and
 *     psi(z) = sum_k q_k K(z - x_k) + sum_l w_l [K(z - y~_l) - K(z - y_l)],
 *     dE/dx_i = q_i/2 [grad phi(x_i) + sum_{p: (i,p) near} grad psi(x_i + p)],
 *     dE/dq_i = 1/2 [phi(x_i) + sum_{p: (i,p) near} psi(x_i + p)],
 *     derived from eqs. (3), (8), (10), (pfx3)-(pfx4) (the paper gives no adjoint).
 *   exact = 0: the physical approximation dE/dx_i = -q_i field_i, dE/dq_i = phi_i.
 * dE/dq is returned projected onto sum dq = 0 (mean removed): the Coulomb energy is
 * only defined for neutral charges (in 3-D and in the plane, whose moments use the
 * plane's basis and K = -log r).  Screened kernel: u_t = sum_k q_k K(c_t - x_k) at
 * the centres, K = exp(-kappa r)/r in psi, and dE/dq without projection (any
 * charges).  With decay rows (slab, wire) w also weights them, and psi gains, at
 * each decay point y_i with normal n_i, a charge b_i and a dipole -a_i n_i,
 * a_i = sum_r w_r W_ri, b_i = sum_r w_r c_r W_ri (W_ri the row's quadrature weight
 * and trigonometric factor at the point, c_r = -s|k| or beta).  Biharmonic
 * kernel: u_t over the Almansi basis, K = r in psi, and from the gradient rows
 * (weights w_kl, rows L + k L + l) a dipole D_l = R0 (w_xl, w_yl, w_zl) at each
 * partner and -D_l at each check point, whose potential in psi is
 * D_l . (y - z)/|y - z|.
 * Must follow a periodic_sum_energy (or eval at the
 * particles) with the same inputs on the same stream: it reuses that forward
 * pass's near set, coefficients and outputs kept in the plan.
 *   epoch : 0, or the forward_epoch (periodic_sum_plan_info) read right after
 *           the forward pass whose gradient is wanted.
 * Errors: PS_E_INVALID when the plan's last forward pass was not at these
 * particles (other arrays or n, separate targets, a batched plan) or, for
 * epoch != 0, when another pass has been enqueued since that one: the stored
 * state would belong to other inputs.  The call never reuses it then. */
ps_status periodic_sum_energy_vjp(ps_plan plan, int64_t n,
                                  const double* x, const double* y, const double* z, const double* q,
                                  const double* gE, double* dEdx, double* dEdy, double* dEdz,
                                  double* dEdq, int32_t exact, int64_t epoch, void* stream);

/* Batched "set": nsys independent systems, each with its own box and charges
 * (prm[k].box, p, R_b/lambda, n_max as the largest N of system k; precision,
 * mean and rcond are taken from prm[0]).  Same host steps as periodic_sum_plan
 * per system; device tables are packed per system. */
ps_status periodic_sum_plan_batched(int32_t nsys, const ps_params* prm, int device, ps_plan* out);
/* (kernel and kappa are taken from prm[0] as well.) */

/* Saves the result of the "set" phase (Sec. 2.3; its cost grows like P^3 with
 * the SVD, Tables 2-4) so that a later process can skip it: for every system the
 * parameters, check points and partners, A^+, the box integrals R_t^(0), the
 * image list and the RBF centres, plus the plan's tuned launch shape.  Nothing
 * of the last eval is saved.  Format: little-endian binary, "PSPLAN01" magic,
 * version 4, a 64-bit FNV-1a checksum of all preceding bytes at the end.
 *   path: host string, a file path; an existing file is replaced.
 * Errors: PS_E_INVALID (NULL plan or path), PS_E_IO (the file could not be
 * written completely). */
ps_status periodic_sum_plan_save(ps_plan plan, const char* path);

/* Rebuilds a plan on `device` from a file written by periodic_sum_plan_save,
 * without repeating the set phase: the loaded tables are used as saved
 * (bitwise), and device workspace is allocated as by periodic_sum_plan(_batched).
 * *out receives the plan (NULL on failure).
 * Errors: PS_E_INVALID (NULL arguments, device out of range), PS_E_IO (missing
 * or unreadable file, wrong magic or version, checksum mismatch, sizes that are
 * inconsistent or outside the limits periodic_sum_plan enforces), PS_E_NOMEM,
 * PS_E_HIP. */
ps_status periodic_sum_plan_load(const char* path, int device, ps_plan* out);

/* Batched "get": all systems in one hipGraph launch on `stream`.  offsets: host
 * array [nsys+1], system k owns particles offsets[k] .. offsets[k+1]-1 of the
 * packed device arrays x, y, z, q and of the outputs (targets = particles).
 * Work over (system, target block, source chunk) is ordered largest first.
 * The graph is captured on the first call for a set of particle counts and of
 * buffer addresses, and replayed while both stay the same; other counts
 * rebuild the work tables and capture again, other buffers only capture again
 * (host work of about 0.4 ms at 512 systems).  Stage profiling records no
 * events inside the graph. */
ps_status periodic_sum_eval_batched(ps_plan plan, const int64_t* offsets,
                                    const double* x, const double* y, const double* z, const double* q,
                                    double* phi, double* ex, double* ey, double* ez, void* stream);

/* Autotuner for the particle pair sums: times each candidate of targets per
 * workgroup {64, 128, 256} x source-split scale {1/2, 1, 2} (relative to the
 * occupancy-based choice) on the given inputs, with HIP events on `stream`:
 * after a warm-up eval, the median of three separately timed evals.  The two
 * fastest are timed three more times each and the one with the lower median
 * of its six evals is kept in the plan (periodic_sum_plan_info reports it, and
 * tune_ms / tune_second_ms give the two medians).
 * offsets: host [nsys+1] as in periodic_sum_eval_batched ({0, n} for a
 * single-system plan); the outputs receive the last candidate's result.
 * Synchronizes the stream.  best_ms (host, may be NULL) receives the chosen
 * candidate's median time per eval. */
ps_status periodic_sum_autotune(ps_plan plan, const int64_t* offsets,
                                const double* x, const double* y, const double* z, const double* q,
                                double* phi, double* ex, double* ey, double* ez, double* best_ms, void* stream);

/* One candidate of periodic_sum_select. */
typedef struct {
    double  lambda;    /* R_b / R0 */
    int32_t p;         /* smallest truncation number found whose FP64 solve meets tol; 0: none up to 40 */
    int32_t n_solves;  /* FP64 solves spent on this candidate (calibration and search) */
    double  B_P;       /* constant of eps_P = B_P lambda^-p (eq. (o2)) from the solve at p = 8 */
    double  err;       /* relative L2 error of phi at p, FP64 solve, against the reference */
    double  err_prec;  /* the same for a solve in the requested precision */
    double  ms;        /* time per eval at (lambda, p) in the requested precision (HIP events) */
    double  set_s;     /* host set time of that plan, seconds */
} ps_select_row;

/* Parameter selection for the caller's charges (Sec. 3.3, eq. (o1)): for each
 * candidate lambda, the smallest p whose solve meets a relative L2 tolerance
 * on phi, then the candidate whose solve is fastest.  The errors are measured,
 * as the paper advises, not predicted: every solve is compared with one FP64
 * reference solve at the largest lambda and p_ref (0: 36), on all n particles.
 * Eq. (o2), eps_P = B_P lambda^-p, fitted to a solve at p = 8 and then to the
 * measured errors, proposes each next p of a bracketing search that ends when p
 * meets tol and p - 1 does not.  All solves use the zero-mean constant (step 6)
 * so that they approximate the same potential; the chosen p does not depend on
 * that choice.
 *   base       : box, precision, rcond and tile_targets of the plans (host);
 *                spherical basis and Gauss check points only.
 *   n, x..q    : particles as for periodic_sum_eval (device, n >= 1).
 *   tol        : relative L2 tolerance on phi, in (1e-13, 1).
 *   lambdas    : host [n_lambda] candidates in (1, 4], 1 <= n_lambda <= 64.
 *   rows       : host [n_lambda], one result per candidate (see ps_select_row).
 *   best       : index of the fastest candidate whose solve in the requested
 *                precision meets tol, or -1 if none does.
 * Builds and frees a plan per solve (host set time grows like p^6: p = 40
 * takes ~20 s on 8 cores) and allocates n doubles of device memory; synchronizes
 * the stream.  Errors: PS_E_INVALID, PS_E_UNSUPPORTED (other basis or check
 * set; a reference not accurate to a tenth of tol), and those of
 * periodic_sum_plan / periodic_sum_eval / periodic_sum_status. */
ps_status periodic_sum_select(const ps_params* base, int device, int64_t n,
                              const double* x, const double* y, const double* z, const double* q,
                              double tol, const double* lambdas, int32_t n_lambda, int32_t p_ref,
                              ps_select_row* rows, int32_t* best, void* stream);

/* Near-set sizes N_b of every system after the last completed eval
 * (host [nsys]; synchronizes the device). */
ps_status periodic_sum_near_counts(ps_plan plan, int64_t* out, int32_t nsys);

/* Synchronizes `stream` and returns the data-dependent status of the last eval
 * or PS_OK, then clears it: PS_E_OUT_OF_BOX for a particle outside the box or
 * a NaN coordinate or charge (reported first), else PS_E_NOT_NEUTRAL (Coulomb
 * kernel only: screened plans accept any net charge). */
ps_status periodic_sum_status(ps_plan plan, void* stream);

/* Plan facts; n_near_last synchronizes the device. */
ps_status periodic_sum_plan_info(ps_plan plan, ps_plan_info* out);

/* Copies the plan's check points (host buffers [3*L] each, xyz interleaved),
 * the pseudo-inverse [(P-1)*n_rows] row-major and the box integrals [P]; any
 * pointer may be NULL.  Sizes from periodic_sum_plan_info.  Single-system plans only. */
ps_status periodic_sum_plan_tables(ps_plan plan, double* check_points, double* partners,
                                   double* pinv, double* box_means);

/* Coefficients C_1..C_P of the last completed eval (host buffer [P]; synchronizes). */
ps_status periodic_sum_last_coefficients(ps_plan plan, double* C);

/* Stage timing with HIP events recorded on the eval stream between the stages
 * of algorithm "get" (single-system evals; not inside the batched graph).
 * Recording adds no host synchronization to an eval while fewer than 16
 * profiled evals are unread; beyond that an eval first waits for the oldest
 * unread one (long finished in a steady loop) and adds it to the sums.
 * enable != 0 turns it on for the following evals.  Either way the call
 * starts a new averaging window and drops the evals not yet read. */
ps_status periodic_sum_set_profiling(ps_plan plan, int32_t enable);

/* Mean durations in milliseconds, over the profiled evals of the current window
 * (those enqueued since set_profiling or since the previous read), of the stages
 * of algorithm "get", in this order
 * (PS_N_STAGES values): 0 validation + spatial ordering, 1 near-set build
 * (steps 1-2), 2 tile bounds and target blocks, 3 check-point sums
 * (step 3 at Y_c1, Y_c2), 4 least-squares solve (steps 4-5), 5 zero-mean
 * constant (step 6), 6 particle pair sums (step 3 at Y0), 7 far field and
 * combination (steps 7-8).  A call that finds unread evals synchronizes on the
 * last one, averages the window and starts a new one; a call with no profiled
 * eval since the previous read returns the same means again.  ms: host [n],
 * n >= PS_N_STAGES.  Errors: PS_E_INVALID before any profiled eval, PS_E_HIP. */
#define PS_N_STAGES 8
ps_status periodic_sum_stage_times(ps_plan plan, double* ms, int32_t n);

/* The plan's forward_epoch (see ps_plan_info) into *out, without synchronizing:
 * a caller that keeps the gradient of one pass for later (an autograd graph)
 * reads it right after that pass and hands it to periodic_sum_energy_vjp.
 * Errors: PS_E_INVALID (NULL argument). */
ps_status periodic_sum_forward_epoch(ps_plan plan, int64_t* out);

/* Releases the plan and its device workspace (synchronizes its device). */
void periodic_sum_destroy(ps_plan plan);

const char* periodic_sum_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PERIODIC_SUM_H */
