/*
 * FP64 direct sums for the oracle of the periodic Coulomb sum.
 *
 * TEST INFRASTRUCTURE ONLY: this file belongs to the CPU oracle.  Only the
 * test-suite, the smoke check and the benchmark's CPU-baseline leg may load it.
 *
 * Kernel K(r) = 1/|r| (and, below, exp(-kappa r)/r, -log r in 2-D and r),
 * with K(0) = 0 (paper Sec. 1, eq. (1)): a pair whose
 * squared distance is exactly zero contributes nothing.  Every sum is a plain
 * loop over all sources with Neumaier-compensated accumulation; OpenMP splits
 * the targets only, so each target's sum has a fixed order.
 */
#include <math.h>
#include <stddef.h>

typedef struct { double s, c; } acc_t;

static inline void acc_add(acc_t* a, double v)
{
    double t = a->s + v;
    if (fabs(a->s) >= fabs(v)) a->c += (a->s - t) + v;
    else                        a->c += (v - t) + a->s;
    a->s = t;
}
static inline double acc_get(const acc_t* a) { return a->s + a->c; }

/* phi(y) = sum_j q_j K(y - x_j)   and   grad phi(y) = -sum_j q_j (y - x_j)/|y - x_j|^3
 * (free-space finite sum, eq. (r2)); gx may be NULL for potential only. */
void orc_direct(long nt, const double* tx, const double* ty, const double* tz,
                long ns, const double* sx, const double* sy, const double* sz, const double* sq,
                double* phi, double* gx, double* gy, double* gz)
{
    #pragma omp parallel for schedule(dynamic, 16)
    for (long i = 0; i < nt; ++i) {
        acc_t p = {0, 0}, ax = {0, 0}, ay = {0, 0}, az = {0, 0};
        const double yx = tx[i], yy = ty[i], yz = tz[i];
        for (long j = 0; j < ns; ++j) {
            double dx = yx - sx[j], dy = yy - sy[j], dz = yz - sz[j];
            double r2 = dx * dx + dy * dy + dz * dz;
            if (r2 == 0.0) continue;
            double r = sqrt(r2);
            double k = sq[j] / r;
            acc_add(&p, k);
            if (gx) {
                double k3 = k / r2;
                acc_add(&ax, -k3 * dx);
                acc_add(&ay, -k3 * dy);
                acc_add(&az, -k3 * dz);
            }
        }
        phi[i] = acc_get(&p);
        if (gx) { gx[i] = acc_get(&ax); gy[i] = acc_get(&ay); gz[i] = acc_get(&az); }
    }
}

/* Same sum with every source shifted by each lattice vector p in a list:
 * phi(y) = sum_p sum_j q_j K(y - x_j - p).  Used for brute-force image sums. */
void orc_direct_images(long nt, const double* tx, const double* ty, const double* tz,
                       long ns, const double* sx, const double* sy, const double* sz, const double* sq,
                       long nimg, const double* px, const double* py, const double* pz,
                       double* phi, double* gx, double* gy, double* gz)
{
    #pragma omp parallel for schedule(dynamic, 1)
    for (long i = 0; i < nt; ++i) {
        acc_t p = {0, 0}, ax = {0, 0}, ay = {0, 0}, az = {0, 0};
        for (long m = 0; m < nimg; ++m) {
            const double yx = tx[i] - px[m], yy = ty[i] - py[m], yz = tz[i] - pz[m];
            for (long j = 0; j < ns; ++j) {
                double dx = yx - sx[j], dy = yy - sy[j], dz = yz - sz[j];
                double r2 = dx * dx + dy * dy + dz * dz;
                if (r2 == 0.0) continue;
                double r = sqrt(r2);
                double k = sq[j] / r;
                acc_add(&p, k);
                double k3 = k / r2;
                acc_add(&ax, -k3 * dx);
                acc_add(&ay, -k3 * dy);
                acc_add(&az, -k3 * dz);
            }
        }
        phi[i] = acc_get(&p);
        if (gx) { gx[i] = acc_get(&ax); gy[i] = acc_get(&ay); gz[i] = acc_get(&az); }
    }
}

/* Real-space part of the Ewald split (paper App. D, eqs. (e1)-(e3)):
 * phi1(y) = sum_p sum_j q_j erfc(xi r)/r over images p in a list, r = |y - x_j - p|,
 * skipping r = 0 (its K1(0) self value is added by the caller).
 * The field part returns grad phi1 = -sum q (y-x) [erfc(xi r)/r + 2 xi/sqrt(pi) e^{-xi^2 r^2}]/r^2.
 * Pairs beyond rcut are skipped (their terms are below erfc(xi rcut)). */
void orc_ewald_real(long nt, const double* tx, const double* ty, const double* tz,
                    long ns, const double* sx, const double* sy, const double* sz, const double* sq,
                    long nimg, const double* px, const double* py, const double* pz,
                    double xi, double rcut,
                    double* phi, double* gx, double* gy, double* gz)
{
    const double two_over_sqrtpi = 1.12837916709551257390;
    const double rc2 = rcut * rcut;
    #pragma omp parallel for schedule(dynamic, 1)
    for (long i = 0; i < nt; ++i) {
        acc_t p = {0, 0}, ax = {0, 0}, ay = {0, 0}, az = {0, 0};
        for (long m = 0; m < nimg; ++m) {
            const double yx = tx[i] - px[m], yy = ty[i] - py[m], yz = tz[i] - pz[m];
            for (long j = 0; j < ns; ++j) {
                double dx = yx - sx[j], dy = yy - sy[j], dz = yz - sz[j];
                double r2 = dx * dx + dy * dy + dz * dz;
                if (r2 == 0.0 || r2 > rc2) continue;
                double r = sqrt(r2);
                double e = erfc(xi * r) / r;
                acc_add(&p, sq[j] * e);
                if (gx) {
                    double g = sq[j] * (e + two_over_sqrtpi * xi * exp(-xi * xi * r2)) / r2;
                    acc_add(&ax, -g * dx);
                    acc_add(&ay, -g * dy);
                    acc_add(&az, -g * dz);
                }
            }
        }
        phi[i] = acc_get(&p);
        if (gx) { gx[i] = acc_get(&ax); gy[i] = acc_get(&ay); gz[i] = acc_get(&az); }
    }
}

/* Reciprocal-space part of the Ewald split for a list of wave vectors k != 0
 * with weights w_k = (4 pi / V) exp(-k^2/(4 xi^2)) / k^2 (paper App. D, eq. (e4)-(e5),
 * written as an explicit Fourier sum instead of a gridded FFT):
 * phi2(y) = sum_k w_k sum_j q_j cos(k.(y - x_j)),
 * grad phi2(y) = -sum_k w_k k sum_j q_j sin(k.(y - x_j)).
 * The structure factors S_k = sum_j q_j e^{i k.x_j} are passed in (re, im). */
void orc_ewald_recip(long nt, const double* tx, const double* ty, const double* tz,
                     long nk, const double* kx, const double* ky, const double* kz, const double* w,
                     const double* sre, const double* sim,
                     double* phi, double* gx, double* gy, double* gz)
{
    #pragma omp parallel for schedule(static)
    for (long i = 0; i < nt; ++i) {
        acc_t p = {0, 0}, ax = {0, 0}, ay = {0, 0}, az = {0, 0};
        for (long k = 0; k < nk; ++k) {
            double a = kx[k] * tx[i] + ky[k] * ty[i] + kz[k] * tz[i];
            double c = cos(a), s = sin(a);
            /* Re[S_k e^{-i k.y}] = sre c + sim s ; Im part gives the sine sum */
            double re = sre[k] * c + sim[k] * s;
            double im = sim[k] * c - sre[k] * s;   /* = -sum_j q_j sin(k.(y-x_j)) */
            acc_add(&p, w[k] * re);
            if (gx) {
                acc_add(&ax, w[k] * kx[k] * im);
                acc_add(&ay, w[k] * ky[k] * im);
                acc_add(&az, w[k] * kz[k] * im);
            }
        }
        phi[i] = acc_get(&p);
        if (gx) { gx[i] = acc_get(&ax); gy[i] = acc_get(&ay); gz[i] = acc_get(&az); }
    }
}

/* ------------------------------------------------------------------------ */
/* Screened Coulomb kernel K(r) = exp(-kappa r)/r (the Green's function of    */
/* the modified Helmholtz operator, up to 4 pi), K(0) = 0.                    */
/* grad_y K(y - x) = -(1 + kappa r) exp(-kappa r) (y - x) / r^3.              */

/* phi(y) = sum_m sum_j q_j K(y - x_j - p_m) over a list of shifts p_m (one zero
 * shift gives the free-space finite sum of eq. (r2)); gx may be NULL. */
void orc_direct_screened(long nt, const double* tx, const double* ty, const double* tz,
                         long ns, const double* sx, const double* sy, const double* sz, const double* sq,
                         long nimg, const double* px, const double* py, const double* pz, double kappa,
                         double* phi, double* gx, double* gy, double* gz)
{
    #pragma omp parallel for schedule(dynamic, 1)
    for (long i = 0; i < nt; ++i) {
        acc_t p = {0, 0}, ax = {0, 0}, ay = {0, 0}, az = {0, 0};
        for (long m = 0; m < nimg; ++m) {
            const double yx = tx[i] - px[m], yy = ty[i] - py[m], yz = tz[i] - pz[m];
            for (long j = 0; j < ns; ++j) {
                double dx = yx - sx[j], dy = yy - sy[j], dz = yz - sz[j];
                double r2 = dx * dx + dy * dy + dz * dz;
                if (r2 == 0.0) continue;
                double r = sqrt(r2);
                double k = sq[j] * exp(-kappa * r) / r;
                acc_add(&p, k);
                if (gx) {
                    double g = k * (1.0 + kappa * r) / r2;
                    acc_add(&ax, -g * dx);
                    acc_add(&ay, -g * dy);
                    acc_add(&az, -g * dz);
                }
            }
        }
        phi[i] = acc_get(&p);
        if (gx) { gx[i] = acc_get(&ax); gy[i] = acc_get(&ay); gz[i] = acc_get(&az); }
    }
}

/* Real-space part of an Ewald split of the screened kernel.  With
 * K(r) = (2/sqrt(pi)) int_0^inf exp(-r^2 t^2 - kappa^2/(4 t^2)) dt, the part
 * t > alpha is
 *   K1(r) = [exp(kappa r) erfc(alpha r + b) + exp(-kappa r) erfc(alpha r - b)] / (2 r),  b = kappa/(2 alpha),
 * and dK1/dr = [kappa (A - B) - (4 alpha/sqrt(pi)) exp(-alpha^2 r^2 - b^2)]/(2 r) - K1/r with A, B the
 * two products above.  Pairs beyond rcut and r = 0 are skipped. */
void orc_ewald_screened_real(long nt, const double* tx, const double* ty, const double* tz,
                             long ns, const double* sx, const double* sy, const double* sz, const double* sq,
                             long nimg, const double* px, const double* py, const double* pz,
                             double kappa, double alpha, double rcut,
                             double* phi, double* gx, double* gy, double* gz)
{
    const double four_over_sqrtpi = 2.25675833419102514780;
    const double rc2 = rcut * rcut, b = kappa / (2.0 * alpha);
    #pragma omp parallel for schedule(dynamic, 1)
    for (long i = 0; i < nt; ++i) {
        acc_t p = {0, 0}, ax = {0, 0}, ay = {0, 0}, az = {0, 0};
        for (long m = 0; m < nimg; ++m) {
            const double yx = tx[i] - px[m], yy = ty[i] - py[m], yz = tz[i] - pz[m];
            for (long j = 0; j < ns; ++j) {
                double dx = yx - sx[j], dy = yy - sy[j], dz = yz - sz[j];
                double r2 = dx * dx + dy * dy + dz * dz;
                if (r2 == 0.0 || r2 > rc2) continue;
                double r = sqrt(r2);
                double A = exp(kappa * r) * erfc(alpha * r + b);
                double B = exp(-kappa * r) * erfc(alpha * r - b);
                double k1 = (A + B) / (2.0 * r);
                acc_add(&p, sq[j] * k1);
                if (gx) {
                    double dk = (kappa * (A - B) - four_over_sqrtpi * alpha * exp(-alpha * alpha * r2 - b * b)) / (2.0 * r)
                                - k1 / r;
                    double g = sq[j] * dk / r;   /* grad_y = dK1/dr (y - x)/r */
                    acc_add(&ax, g * dx);
                    acc_add(&ay, g * dy);
                    acc_add(&az, g * dz);
                }
            }
        }
        phi[i] = acc_get(&p);
        if (gx) { gx[i] = acc_get(&ax); gy[i] = acc_get(&ay); gz[i] = acc_get(&az); }
    }
}

/* ------------------------------------------------------------------------ */
/* Two dimensions: K(r) = -log r (the Green's function of the 2-D Laplacian, */
/* up to 2 pi), K(0) = 0.  grad_y K(y - x) = -(y - x) / r^2.                 */

/* phi(y) = sum_m sum_j q_j K(y - x_j - p_m) over a list of 2-D shifts p_m (one
 * zero shift gives the free-space finite sum), and grad phi; gx may be NULL. */
void orc_direct_log2d(long nt, const double* tx, const double* ty,
                      long ns, const double* sx, const double* sy, const double* sq,
                      long nimg, const double* px, const double* py,
                      double* phi, double* gx, double* gy)
{
    #pragma omp parallel for schedule(dynamic, 1)
    for (long i = 0; i < nt; ++i) {
        acc_t p = {0, 0}, ax = {0, 0}, ay = {0, 0};
        for (long m = 0; m < nimg; ++m) {
            const double yx = tx[i] - px[m], yy = ty[i] - py[m];
            for (long j = 0; j < ns; ++j) {
                double dx = yx - sx[j], dy = yy - sy[j];
                double r2 = dx * dx + dy * dy;
                if (r2 == 0.0) continue;
                acc_add(&p, -0.5 * sq[j] * log(r2));
                if (gx) {
                    double g = sq[j] / r2;
                    acc_add(&ax, -g * dx);
                    acc_add(&ay, -g * dy);
                }
            }
        }
        phi[i] = acc_get(&p);
        if (gx) { gx[i] = acc_get(&ax); gy[i] = acc_get(&ay); }
    }
}

/* ------------------------------------------------------------------------ */
/* The biharmonic kernel K(r) = r (Delta^2 r = -8 pi delta in 3-D), K(0) = 0. */
/* grad_y K(y - x) = (y - x) / r.                                             */

/* phi(y) = sum_m sum_j q_j |y - x_j - p_m| over a list of shifts p_m (one zero
 * shift gives the free-space finite sum), and grad phi; gx may be NULL. */
void orc_direct_dist(long nt, const double* tx, const double* ty, const double* tz,
                     long ns, const double* sx, const double* sy, const double* sz, const double* sq,
                     long nimg, const double* px, const double* py, const double* pz,
                     double* phi, double* gx, double* gy, double* gz)
{
    #pragma omp parallel for schedule(dynamic, 1)
    for (long i = 0; i < nt; ++i) {
        acc_t p = {0, 0}, ax = {0, 0}, ay = {0, 0}, az = {0, 0};
        for (long m = 0; m < nimg; ++m) {
            const double yx = tx[i] - px[m], yy = ty[i] - py[m], yz = tz[i] - pz[m];
            for (long j = 0; j < ns; ++j) {
                double dx = yx - sx[j], dy = yy - sy[j], dz = yz - sz[j];
                double r2 = dx * dx + dy * dy + dz * dz;
                if (r2 == 0.0) continue;
                double r = sqrt(r2);
                acc_add(&p, sq[j] * r);
                if (gx) {
                    double g = sq[j] / r;
                    acc_add(&ax, g * dx);
                    acc_add(&ay, g * dy);
                    acc_add(&az, g * dz);
                }
            }
        }
        phi[i] = acc_get(&p);
        if (gx) { gx[i] = acc_get(&ax); gy[i] = acc_get(&ay); gz[i] = acc_get(&az); }
    }
}

/* Real-space part of an Ewald split of K(r) = r.  With m = r * g_alpha (the
 * kernel smoothed by the normalized Gaussian exp(-alpha^2 r^2)), the remainder
 * r - m = S(r) - 1/(2 alpha^2 r), where
 *   S(r) = r erfc(alpha r) + erfc(alpha r)/(2 alpha^2 r) - exp(-alpha^2 r^2)/(alpha sqrt(pi))
 * decays like a Gaussian and
 *   dS/dr = erfc(alpha r) (1 - 1/(2 alpha^2 r^2)) - exp(-alpha^2 r^2)/(alpha sqrt(pi) r).
 * This routine sums S over images within rcut (r = 0 skipped). */
void orc_ewald_bih_real(long nt, const double* tx, const double* ty, const double* tz,
                        long ns, const double* sx, const double* sy, const double* sz, const double* sq,
                        long nimg, const double* px, const double* py, const double* pz,
                        double alpha, double rcut,
                        double* phi, double* gx, double* gy, double* gz)
{
    const double inv_sqrtpi = 0.56418958354775628695;
    const double rc2 = rcut * rcut, h = 1.0 / (2.0 * alpha * alpha), ea = inv_sqrtpi / alpha;
    #pragma omp parallel for schedule(dynamic, 1)
    for (long i = 0; i < nt; ++i) {
        acc_t p = {0, 0}, ax = {0, 0}, ay = {0, 0}, az = {0, 0};
        for (long m = 0; m < nimg; ++m) {
            const double yx = tx[i] - px[m], yy = ty[i] - py[m], yz = tz[i] - pz[m];
            for (long j = 0; j < ns; ++j) {
                double dx = yx - sx[j], dy = yy - sy[j], dz = yz - sz[j];
                double r2 = dx * dx + dy * dy + dz * dz;
                if (r2 == 0.0 || r2 > rc2) continue;
                double r = sqrt(r2);
                double ec = erfc(alpha * r), ex = exp(-alpha * alpha * r2);
                acc_add(&p, sq[j] * (r * ec + h * ec / r - ea * ex));
                if (gx) {
                    double ds = ec * (1.0 - h / r2) - ea * ex / r;
                    double g = sq[j] * ds / r;   /* grad_y = dS/dr (y - x)/r */
                    acc_add(&ax, g * dx);
                    acc_add(&ay, g * dy);
                    acc_add(&az, g * dz);
                }
            }
        }
        phi[i] = acc_get(&p);
        if (gx) { gx[i] = acc_get(&ax); gy[i] = acc_get(&ay); gz[i] = acc_get(&az); }
    }
}
