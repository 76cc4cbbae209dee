// Host FP64 "set" phase (Sec. 2.3, algorithm "set", steps 1-6; Sec. 3; App. B).
#include "ps_setup.h"

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>

namespace ps {

void Recurrence::build(int p_)
{
    p = p_;
    a.assign(p * p, 0.0);
    b.assign(p * p, 0.0);
    c.assign(p, 0.0);
    for (int m = 1; m < p; ++m) c[m] = std::sqrt((2.0 * m - 1.0) / (2.0 * m));
    for (int n = 1; n < p; ++n)
        for (int m = -n + 1; m <= n - 1; ++m) {
            const double am = std::abs(m);
            const double lo = n - am, hi = n + am;
            const int t = n * n + n + m;
            a[t] = (2.0 * n - 1.0) / std::sqrt(lo * hi);
            b[t] = (n - am >= 2) ? std::sqrt((lo - 1.0) * (hi - 1.0) / (lo * hi)) : 0.0;
        }
}

void Recurrence::eval(double x, double y, double z, double* out) const
{
    const double r2 = x * x + y * y + z * z;
    double dA = 1.0, dB = 0.0;  // R^_m^{m}, R^_m^{-m} on the diagonal
    for (int m = 0; m < p; ++m) {
        if (m > 0) {
            const double nA = -c[m] * (x * dA + y * dB);
            const double nB = c[m] * (y * dA - x * dB);
            dA = nA;
            dB = nB;
        }
        for (int s = 0; s < (m ? 2 : 1); ++s) {
            const int mm = s ? -m : m;
            double prev2 = 0.0, prev1 = s ? dB : dA;
            out[m * m + m + mm] = prev1;
            for (int n = m + 1; n < p; ++n) {
                const int t = n * n + n + mm;
                const double v = -a[t] * z * prev1 - b[t] * r2 * prev2;
                out[t] = v;
                prev2 = prev1;
                prev1 = v;
            }
        }
    }
}

void Recurrence::eval_dz(double x, double y, double z, double* out, double* dout) const
{
    const double r2 = x * x + y * y + z * z;
    double dA = 1.0, dB = 0.0;
    for (int m = 0; m < p; ++m) {
        if (m > 0) {
            const double nA = -c[m] * (x * dA + y * dB);
            const double nB = c[m] * (y * dA - x * dB);
            dA = nA;
            dB = nB;
        }
        for (int s = 0; s < (m ? 2 : 1); ++s) {
            const int mm = s ? -m : m;
            double prev2 = 0.0, prev1 = s ? dB : dA, dprev2 = 0.0, dprev1 = 0.0;
            out[m * m + m + mm] = prev1;
            dout[m * m + m + mm] = 0.0;
            for (int n = m + 1; n < p; ++n) {
                const int t = n * n + n + mm;
                const double v = -a[t] * z * prev1 - b[t] * r2 * prev2;
                const double dv = -a[t] * (prev1 + z * dprev1) - b[t] * (2.0 * z * prev2 + r2 * dprev2);
                out[t] = v;
                dout[t] = dv;
                prev2 = prev1;
                prev1 = v;
                dprev2 = dprev1;
                dprev1 = dv;
            }
        }
    }
}

void Recurrence::eval_dir(double x, double y, double z, double u, double v, double w, double* out, double* dout) const
{
    const double r2 = x * x + y * y + z * z;
    const double dr2 = 2.0 * (x * u + y * v + z * w);
    double dA = 1.0, dB = 0.0, gA = 0.0, gB = 0.0;   // diagonal R^_m^{+-m} and their derivatives
    for (int m = 0; m < p; ++m) {
        if (m > 0) {
            const double nA = -c[m] * (x * dA + y * dB);
            const double nB = c[m] * (y * dA - x * dB);
            const double ngA = -c[m] * (u * dA + x * gA + v * dB + y * gB);
            const double ngB = c[m] * (v * dA + y * gA - u * dB - x * gB);
            dA = nA;
            dB = nB;
            gA = ngA;
            gB = ngB;
        }
        for (int s = 0; s < (m ? 2 : 1); ++s) {
            const int mm = s ? -m : m;
            double prev2 = 0.0, prev1 = s ? dB : dA, dprev2 = 0.0, dprev1 = s ? gB : gA;
            out[m * m + m + mm] = prev1;
            dout[m * m + m + mm] = dprev1;
            for (int n = m + 1; n < p; ++n) {
                const int t = n * n + n + mm;
                const double val = -a[t] * z * prev1 - b[t] * r2 * prev2;
                const double dv = -a[t] * (w * prev1 + z * dprev1) - b[t] * (dr2 * prev2 + r2 * dprev2);
                out[t] = val;
                dout[t] = dv;
                prev2 = prev1;
                prev1 = val;
                dprev2 = dprev1;
                dprev1 = dv;
            }
        }
    }
}

void basis2d(int p, double x, double y, double* out)
{
    out[0] = 1.0;
    double re = 1.0, im = 0.0;   // w^(n-1)
    for (int n = 1; n < p; ++n) {
        const double r2 = re * x - im * y, i2 = re * y + im * x;
        re = r2;
        im = i2;
        out[2 * n - 1] = re;
        out[2 * n] = im;
    }
}

// Nodes and weights of n-point Gauss-Legendre quadrature on [-1, 1], ascending:
// Newton's method on P_n evaluated by the three-term recurrence.
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w)
{
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 0; i < (n + 1) / 2; ++i) {
        double zr = std::cos(M_PI * (i + 0.75) / (n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = zr;
            for (int k = 2; k <= n; ++k) {
                const double p2 = ((2.0 * k - 1.0) * zr * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            if (n == 1) { p1 = zr; p0 = 1.0; }
            dp = n * (zr * p1 - p0) / (zr * zr - 1.0);
            const double dz = p1 / dp;
            zr -= dz;
            if (std::fabs(dz) <= 1e-17 && it > 2) break;
        }
        // final derivative at the converged node
        double p0 = 1.0, p1 = zr;
        for (int k = 2; k <= n; ++k) {
            const double p2 = ((2.0 * k - 1.0) * zr * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        dp = (n == 1) ? 1.0 : n * (zr * p1 - p0) / (zr * zr - 1.0);
        if ((n & 1) && i == (n - 1) / 2) zr = 0.0;
        const double wt = 2.0 / ((1.0 - zr * zr) * dp * dp);
        x[i] = -zr;
        x[n - 1 - i] = zr;
        w[i] = wt;
        w[n - 1 - i] = wt;
    }
}

namespace {

// Corner term of the prism potential: F(a,b,c) = ab ln(c+r) + bc ln(a+r) + ca ln(b+r)
// - a^2/2 atan(bc/(ar)) - b^2/2 atan(ca/(br)) - c^2/2 atan(ab/(cr)), with each
// term zero where its prefactor vanishes and c + r formed stably for c < 0.
double log_c_plus_r(double c, double r, double s) { return std::log(c >= 0.0 ? c + r : s / (r - c)); }

double prism_corner(double a, double b, double c)
{
    const double a2 = a * a, b2 = b * b, c2 = c * c;
    const double r = std::sqrt(a2 + b2 + c2);
    if (r == 0.0) return 0.0;
    double F = 0.0;
    if (a * b != 0.0) F += a * b * log_c_plus_r(c, r, a2 + b2);
    if (b * c != 0.0) F += b * c * log_c_plus_r(a, r, b2 + c2);
    if (c * a != 0.0) F += c * a * log_c_plus_r(b, r, c2 + a2);
    if (a != 0.0) F -= 0.5 * a2 * std::atan(b * c / (a * r));
    if (b != 0.0) F -= 0.5 * b2 * std::atan(c * a / (b * r));
    if (c != 0.0) F -= 0.5 * c2 * std::atan(a * b / (c * r));
    return F;
}

}  // namespace

double box_mean_potential(const double box[3], double x, double y, double z)
{
    double tot = 0.0;
    for (int k = 0; k < 8; ++k) {
        const double sx = (k & 1) ? 1.0 : -1.0, sy = (k & 2) ? 1.0 : -1.0, sz = (k & 4) ? 1.0 : -1.0;
        tot += sx * sy * sz * prism_corner(sx * 0.5 * box[0] - x, sy * 0.5 * box[1] - y, sz * 0.5 * box[2] - z);
    }
    return tot / (box[0] * box[1] * box[2]);
}

namespace {

// Pseudo-inverse of the L x n matrix A (column-major) by Householder QR
// followed by a one-sided (Hestenes) Jacobi SVD of the n x n factor R:
// A = Q R, R = U S V^T, A^+ = V S^+ U^T Q^T with singular values below
// rcond * s_max dropped.  Returns A^+ row-major (n x L).  The Jacobi sweeps
// visit the column pairs in round-robin order: each step rotates n/2 disjoint
// pairs, which run in parallel; the result does not depend on the thread count.
void pseudo_inverse(int L, int n, std::vector<double> A, double rcond, std::vector<double>& pinv,
                    int& rank, double& cond)
{
    std::vector<double> vs(static_cast<size_t>(L) * n, 0.0), beta(n, 0.0);
    for (int k = 0; k < n; ++k) {
        double* col = &A[static_cast<size_t>(k) * L];
        double nrm = 0.0;
        for (int i = k; i < L; ++i) nrm += col[i] * col[i];
        nrm = std::sqrt(nrm);
        double* v = &vs[static_cast<size_t>(k) * L];
        if (nrm == 0.0) { beta[k] = 0.0; continue; }
        const double alpha = col[k] >= 0 ? -nrm : nrm;
        for (int i = k; i < L; ++i) v[i] = col[i];
        v[k] -= alpha;
        double vv = 0.0;
        for (int i = k; i < L; ++i) vv += v[i] * v[i];
        beta[k] = vv > 0 ? 2.0 / vv : 0.0;
        const double bk = beta[k];
#pragma omp parallel for schedule(static) if (n - k > 64)
        for (int j = k; j < n; ++j) {
            double* cj = &A[static_cast<size_t>(j) * L];
            double sum = 0.0;
            for (int i = k; i < L; ++i) sum += v[i] * cj[i];
            sum *= bk;
            for (int i = k; i < L; ++i) cj[i] -= sum * v[i];
        }
    }
    // R (n x n, column-major) and V = I
    std::vector<double> R(static_cast<size_t>(n) * n, 0.0), V(static_cast<size_t>(n) * n, 0.0);
    for (int j = 0; j < n; ++j) {
        for (int i = 0; i <= j; ++i) R[static_cast<size_t>(j) * n + i] = A[static_cast<size_t>(j) * L + i];
        V[static_cast<size_t>(j) * n + j] = 1.0;
    }
    // round-robin pairing over m = n rounded up to even; index n (if present) is a dummy
    const int m = n + (n & 1);
    std::vector<int> pos(m);
    for (int i = 0; i < m; ++i) pos[i] = i;
    for (int sweep = 0; sweep < 80; ++sweep) {
        double off = 0.0;
        for (int step = 0; step < m - 1; ++step) {
#pragma omp parallel for schedule(static) reduction(max : off) if (n > 64)
            for (int h = 0; h < m / 2; ++h) {
                int i = pos[h], j = pos[m - 1 - h];
                if (i >= n || j >= n) continue;
                if (i > j) std::swap(i, j);
                double* ci = &R[static_cast<size_t>(i) * n];
                double* cj = &R[static_cast<size_t>(j) * n];
                double al = 0, be = 0, ga = 0;
                for (int k = 0; k < n; ++k) {
                    al += ci[k] * ci[k];
                    be += cj[k] * cj[k];
                    ga += ci[k] * cj[k];
                }
                if (ga == 0.0) continue;
                const double o = std::fabs(ga) / std::sqrt(al * be);
                off = std::max(off, o);
                if (o < 1e-15) continue;
                const double zeta = (be - al) / (2.0 * ga);
                const double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
                const double c = 1.0 / std::sqrt(1.0 + t * t), sn = c * t;
                for (int k = 0; k < n; ++k) {
                    const double xi = ci[k], xj = cj[k];
                    ci[k] = c * xi - sn * xj;
                    cj[k] = sn * xi + c * xj;
                }
                double* vi = &V[static_cast<size_t>(i) * n];
                double* vj = &V[static_cast<size_t>(j) * n];
                for (int k = 0; k < n; ++k) {
                    const double xi = vi[k], xj = vj[k];
                    vi[k] = c * xi - sn * xj;
                    vj[k] = sn * xi + c * xj;
                }
            }
            // rotate positions 1 .. m-1 (position 0 stays)
            const int last = pos[m - 1];
            for (int q = m - 1; q > 1; --q) pos[q] = pos[q - 1];
            if (m > 1) pos[1] = last;
        }
        if (off < 1e-15) break;
    }
    std::vector<double> sig(n);
    double smax = 0.0;
    for (int j = 0; j < n; ++j) {
        double sum = 0.0;
        for (int k = 0; k < n; ++k) sum += R[static_cast<size_t>(j) * n + k] * R[static_cast<size_t>(j) * n + k];
        sig[j] = std::sqrt(sum);
        smax = std::max(smax, sig[j]);
    }
    rank = 0;
    double smin = smax;
    std::vector<double> inv2(n, 0.0);
    for (int j = 0; j < n; ++j)
        if (sig[j] > rcond * smax) {
            ++rank;
            smin = std::min(smin, sig[j]);
            inv2[j] = 1.0 / (sig[j] * sig[j]);
        }
    cond = smax / smin;
    // B = R^+ = V S^-2 (R V)^T  (columns of R now hold R V = U S); M = [B^T; 0] (L x n)
    std::vector<double> M(static_cast<size_t>(L) * n, 0.0);  // column-major
#pragma omp parallel for schedule(static) if (n > 64)
    for (int a = 0; a < n; ++a)        // row a of B
        for (int r = 0; r < n; ++r) {  // column r of B
            double sum = 0.0;
            for (int j = 0; j < n; ++j)
                if (inv2[j] != 0.0) sum += V[static_cast<size_t>(j) * n + a] * inv2[j] * R[static_cast<size_t>(j) * n + r];
            M[static_cast<size_t>(a) * L + r] = sum;  // M[r][a] = B[a][r]
        }
    // A^+T = H_0 H_1 ... H_{n-1} M
    for (int k = n - 1; k >= 0; --k) {
        if (beta[k] == 0.0) continue;
        const double* v = &vs[static_cast<size_t>(k) * L];
        const double bk = beta[k];
#pragma omp parallel for schedule(static) if (n > 64)
        for (int j = 0; j < n; ++j) {
            double* cj = &M[static_cast<size_t>(j) * L];
            double sum = 0.0;
            for (int i = k; i < L; ++i) sum += v[i] * cj[i];
            sum *= bk;
            for (int i = k; i < L; ++i) cj[i] -= sum * v[i];
        }
    }
    pinv.assign(static_cast<size_t>(n) * L, 0.0);
    for (int a = 0; a < n; ++a)
        for (int l = 0; l < L; ++l) pinv[static_cast<size_t>(a) * L + l] = M[static_cast<size_t>(a) * L + l];
}

}  // namespace

namespace {

// exp(z) K_nu(z) for nu = 0, 1 and z > 0, from K_nu(z) = int_0^inf exp(-z cosh t) cosh(nu t) dt
// by the trapezoidal rule (exponentially convergent for this analytic, even
// integrand; the step shrinks as 1/sqrt(z) where the integrand narrows).
void scaled_bessel_k01(double z, double& k0, double& k1)
{
    const double h = std::min(0.1, 0.4 / std::sqrt(z));
    double s0 = 0.5, s1 = 0.5;   // the t = 0 terms, half weight
    for (int i = 1; i < 100000; ++i) {
        const double t = i * h, sh = std::sinh(0.5 * t);
        const double e = std::exp(-2.0 * z * sh * sh);   // exp(-z (cosh t - 1))
        s0 += e;
        s1 += e * std::cosh(t);
        if (e * std::cosh(t) < 1e-20 * s0 && t > 1.0) break;
    }
    k0 = h * s0;
    k1 = h * s1;
}

// beta_m = k K_m'(k rho) / K_m(k rho), m = 0..p-1, for k > 0: the ratio
// u_m = K_{m+1}/K_m grows by the (stable, upward) recurrence
// u_m = 1/u_{m-1} + 2m/z, and K_m' = -K_{m-1} - (m/z) K_m, K_0' = -K_1.
void decay_betas(double k, double rho, int p, std::vector<double>& beta)
{
    const double z = k * rho;
    double k0, k1;
    scaled_bessel_k01(z, k0, k1);
    beta.assign(p, 0.0);
    double u = k1 / k0;   // K_1 / K_0
    beta[0] = -k * u;
    for (int m = 1; m < p; ++m) {
        beta[m] = k * (-1.0 / u - m / z);
        u = 1.0 / u + 2.0 * m / z;
    }
}

}  // namespace

void SystemSetup::build_decay()
{
    dec_pts.clear();
    dec_w.clear();
    dec_rows.clear();
    n_dec = nk = m = mx = mt = nsurf = npts = 0;
    zd = rho_d = 0.0;
    if (periodic == 7 || dim == 2) return;   // the plane's torus has no free direction
    const double h = R0 / 10.0;
    nk = (p + 3) / 4 + 1;
    if (periodic == 1) {
        // wire: the cylinder rho = rho_d over one period, mx Gauss-Legendre points
        // in x times mt equispaced angles; rows over n = 0..nk, m = 0..p-1
        rho_d = std::hypot(0.5 * box[1], 0.5 * box[2]) + h;
        mx = std::max(2 * p + 8, static_cast<int>(std::ceil(4.0 * box[0] / h)));
        mt = std::max(4 * p, static_cast<int>(std::ceil(8.0 * M_PI * rho_d / h)));
        nsurf = 1;
        npts = mx * mt;
        std::vector<double> g, w;
        gauss_legendre(mx, g, w);
        dec_w.resize(static_cast<size_t>(npts));
        dec_pts.resize(static_cast<size_t>(npts) * 3);
        for (int i = 0; i < mx; ++i)
            for (int j = 0; j < mt; ++j) {
                const size_t k = static_cast<size_t>(i) * mt + j;
                const double th = 2.0 * M_PI * j / mt;
                dec_w[k] = w[i] / 2.0 * (1.0 / mt);
                dec_pts[k * 3 + 0] = 0.5 * box[0] * g[i];
                dec_pts[k * 3 + 1] = rho_d * std::cos(th);
                dec_pts[k * 3 + 2] = rho_d * std::sin(th);
            }
        std::vector<double> beta;
        for (int n = 0; n <= nk; ++n) {
            const double k = 2.0 * M_PI * n / box[0];
            if (n > 0) decay_betas(k, rho_d, p, beta);
            for (int mm = 0; mm < p; ++mm) {
                const double b = n > 0 ? beta[mm] : -mm / rho_d;
                for (int tx = 0; tx < (n == 0 ? 1 : 2); ++tx)
                    for (int tt = 0; tt < (mm == 0 ? 1 : 2); ++tt)
                        dec_rows.insert(dec_rows.end(),
                                        {k, static_cast<double>(mm), b, static_cast<double>(tx), static_cast<double>(tt)});
            }
        }
        n_dec = static_cast<int>(dec_rows.size() / 5);
        return;
    }
    zd = 0.5 * box[2] + h;
    m = std::max(2 * p + 8, static_cast<int>(std::ceil(4.0 * std::max(box[0], box[1]) / h)));
    nsurf = 2;
    npts = m * m;
    std::vector<double> g, w;
    gauss_legendre(m, g, w);
    dec_w.resize(static_cast<size_t>(m) * m);
    dec_pts.resize(static_cast<size_t>(2) * m * m * 3);
    for (int pl = 0; pl < 2; ++pl)
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j) {
                const size_t k = static_cast<size_t>(i) * m + j;
                dec_w[k] = 0.25 * w[i] * w[j];
                double* q = &dec_pts[(static_cast<size_t>(pl) * m * m + k) * 3];
                q[0] = 0.5 * box[0] * g[i];
                q[1] = 0.5 * box[1] * g[j];
                q[2] = pl == 0 ? zd : -zd;
            }
    for (int pl = 0; pl < 2; ++pl)
        for (int n1 = 0; n1 <= nk; ++n1)
            for (int n2 = -nk; n2 <= nk; ++n2) {
                if (n1 == 0 && n2 < 0) continue;   // one of each +-k pair
                const double kx = 2.0 * M_PI * n1 / box[0], ky = 2.0 * M_PI * n2 / box[1];
                const double kk = std::sqrt(kx * kx + ky * ky);
                for (int trig = 0; trig < (n1 == 0 && n2 == 0 ? 1 : 2); ++trig)
                    dec_rows.insert(dec_rows.end(), {kx, ky, kk, pl == 0 ? 1.0 : -1.0, static_cast<double>(trig)});
            }
    n_dec = static_cast<int>(dec_rows.size() / 5);
}

void bih_eval(const Recurrence& rec, double x, double y, double z, double* out, int dir, double* dout)
{
    const int p = rec.p, n1 = p * p, n2 = (p - 2) * (p - 2);
    const double s2 = x * x + y * y + z * z;
    if (dir < 0) {
        rec.eval(x, y, z, out);
        for (int t = 0; t < n2; ++t) out[n1 + t] = s2 * out[t];
        return;
    }
    const double u[3] = {x, y, z};
    rec.eval_dir(x, y, z, dir == 0 ? 1.0 : 0.0, dir == 1 ? 1.0 : 0.0, dir == 2 ? 1.0 : 0.0, out, dout);
    for (int t = 0; t < n2; ++t) {
        out[n1 + t] = s2 * out[t];
        dout[n1 + t] = __builtin_fma(s2, dout[t], 2.0 * u[dir] * out[t]);
    }
}

std::string SystemSetup::build(const double bx[3], int p_, double Rb, double lambda, double rcond, int basis_,
                               int n_centres, const double* cen, int n_check, const double* chk, int periodic_,
                               int kernel_, double kappa_, int dim_)
{
    basis = basis_;
    if (dim_ != 3 && dim_ != 2) return "dim must be 3 or 2";
    dim = dim_;
    if (dim == 2) {
        if (basis_ != 0) return "the plane has only its harmonic-polynomial basis";
        if (periodic_ != 3) return "in the plane both axes are periodic";
        if (kernel_ != 0) return "the plane takes the Coulomb kernel only (-log r)";
        if (n_check != 0) return "the plane uses its own check points (n_check must be 0)";
        if (p_ < 2 || p_ > 128) return "p must be in [2, 128] in the plane";
    }
    if (periodic_ != 7 && periodic_ != 3 && periodic_ != 1) return "periodic axes must be 7 (x, y, z), 3 (x, y) or 1 (x)";
    if (periodic_ != 7 && basis_ != 0) return "the RBF basis needs three periodic axes";
    if (kernel_ != 0 && kernel_ != 1 && kernel_ != 2) return "kernel must be 0 (Coulomb), 1 (screened) or 2 (biharmonic)";
    if (kernel_ == 1 && (basis_ != 1 || periodic_ != 7))
        return "the screened kernel needs the RBF basis and three periodic axes";
    if (kernel_ == 2 && (basis_ != 0 || periodic_ != 7 || dim_ != 3))
        return "the biharmonic kernel needs the spherical basis, three periodic axes and three dimensions";
    if (kernel_ == 2 && (p_ < 3 || p_ > 30)) return "the biharmonic kernel needs 3 <= p <= 30";
    kernel = kernel_;
    kappa = kernel_ == 1 ? kappa_ : 0.0;
    periodic = periodic_;
    const int nper = periodic == 7 ? 3 : (periodic == 3 ? 2 : 1);   // axes a partner may be shifted along
    for (int k = 0; k < dim; ++k) {
        if (!(bx[k] > 0.0) || !std::isfinite(bx[k])) return "box lengths must be positive and finite";
        box[k] = bx[k];
    }
    if (dim == 2) box[2] = 1.0;   // every z is 0: the slab of unit height holds them
    if (dim == 3 && (p_ < 2 || p_ > 40)) return "p must be in [2, 40]";
    p = p_;
    P = dim == 2 ? 2 * p - 1 : (kernel == 2 ? p * p + (p - 2) * (p - 2) : p * p);
    V0 = box[0] * box[1] * box[2];
    R0 = dim == 2 ? 0.5 * std::sqrt(box[0] * box[0] + box[1] * box[1])
                  : 0.5 * std::sqrt(box[0] * box[0] + box[1] * box[1] + box[2] * box[2]);   // step 1
    R_b = Rb > 0 ? Rb : lambda * R0;
    if (!(R_b > R0) || !std::isfinite(R_b)) return "the near radius must exceed the circumradius (lambda > 1)";
    if (kernel == 1 && !(kappa > 0.0 && kappa * R0 <= 64.0)) return "kappa must lie in (0, 64 / R0]";
    thr = R_b * R_b * (1.0 + 1e-12);
    if (rcond <= 0) rcond = 1e-13;

    // lattice images whose box [i d - d/2, i d + d/2] comes within R_b of the centre
    images.clear();
    images.insert(images.end(), {0, 0, 0});
    int K[3];
    for (int k = 0; k < 3; ++k) K[k] = k < nper ? static_cast<int>(std::floor(R_b / box[k] + 0.5)) : 0;
    for (int i = -K[0]; i <= K[0]; ++i)
        for (int j = -K[1]; j <= K[1]; ++j)
            for (int l = -K[2]; l <= K[2]; ++l) {
                if (i == 0 && j == 0 && l == 0) continue;
                const int ii[3] = {i, j, l};
                double dmin2 = 0.0;
                for (int k = 0; k < 3; ++k) {
                    const double g = std::max(0.0, std::abs(ii[k]) * box[k] - 0.5 * box[k]);
                    dmin2 += g * g;
                }
                if (dmin2 <= thr * (1.0 + 1e-9)) images.insert(images.end(), {i, j, l});
            }

    // step 2: Gauss spherical grid on the circumsphere, L = p (2p - 1), or the caller's points
    if (n_check > 0) {
        if (!chk) return "check_points is NULL";
        L = n_check;
        yc.assign(chk, chk + static_cast<size_t>(L) * 3);
        for (int l = 0; l < L; ++l) {
            const double* y = &yc[static_cast<size_t>(l) * 3];
            const double r2 = y[0] * y[0] + y[1] * y[1] + y[2] * y[2];
            bool outside = false;
            for (int k = 0; k < nper; ++k) outside = outside || std::fabs(y[k]) > 0.5 * box[k];
            if (!(r2 <= R0 * R0 * (1.0 + 1e-9)) || !outside)
                return "a check point is outside S0 or inside the box along every periodic axis";
        }
    } else if (dim == 2) {
        // L = 4p points equispaced on the circumcircle (the trapezoidal rule plays
        // the part of the Gauss grid); each lies outside the box along x or y
        L = 4 * p;
        yc.assign(static_cast<size_t>(L) * 3, 0.0);
        for (int l = 0; l < L; ++l) {
            const double th = 2.0 * M_PI * l / L;
            yc[static_cast<size_t>(l) * 3 + 0] = R0 * std::cos(th);
            yc[static_cast<size_t>(l) * 3 + 1] = R0 * std::sin(th);
        }
    } else {
        std::vector<double> mu, wq;
        gauss_legendre(p, mu, wq);
        const int nphi = 2 * p - 1;
        L = p * nphi;
        yc.assign(static_cast<size_t>(L) * 3, 0.0);
        for (int a = 0; a < p; ++a) {
            const double st = std::sqrt(1.0 - mu[a] * mu[a]);
            for (int bph = 0; bph < nphi; ++bph) {
                const double ph = 2.0 * M_PI * bph / nphi;
                double* y = &yc[(static_cast<size_t>(a) * nphi + bph) * 3];
                y[0] = R0 * st * std::cos(ph);
                y[1] = R0 * st * std::sin(ph);
                y[2] = R0 * mu[a];
            }
        }
        if (periodic != 7) {   // keep the points that a shift along a periodic axis moves into S0
            std::vector<double> kept;
            for (int l = 0; l < L; ++l) {
                const double* y = &yc[static_cast<size_t>(l) * 3];
                bool outside = false;
                for (int k = 0; k < nper; ++k) outside = outside || std::fabs(y[k]) > 0.5 * box[k];
                if (outside) kept.insert(kept.end(), y, y + 3);
            }
            yc.swap(kept);
            L = static_cast<int>(yc.size() / 3);
        }
    }
    yt.assign(static_cast<size_t>(L) * 3, 0.0);
    // step 3: partner = one coordinate shifted by its period, the coordinate that
    // brings the point deepest into S0 (largest d_k (2|y_k| - d_k)), towards the centre
    for (int l = 0; l < L; ++l) {
        const double* y = &yc[static_cast<size_t>(l) * 3];
        int kb = 0;
        double best = -1e300;
        for (int k = 0; k < nper; ++k) {
            const double g = box[k] * (2.0 * std::fabs(y[k]) - box[k]);
            if (g > best) { best = g; kb = k; }
        }
        double* t = &yt[static_cast<size_t>(l) * 3];
        for (int k = 0; k < 3; ++k) t[k] = y[k];
        t[kb] = y[kb] - (y[kb] > 0 ? 1.0 : (y[kb] < 0 ? -1.0 : 0.0)) * box[kb];
    }
    // step 4: A_lt = R_t(y_l) - R_t(y~_l) for the basis functions t = 2..P (column-major L x (P-1))
    rec.build(p);
    if (basis == 1) {
        if (n_centres < 1 || n_centres > 4096 || !cen) return "RBF basis needs 1..4096 centres";
        centres.assign(cen, cen + static_cast<size_t>(n_centres) * 3);
        for (int t = 0; t < n_centres; ++t) {
            const double* c = &centres[static_cast<size_t>(t) * 3];
            if (!(c[0] * c[0] + c[1] * c[1] + c[2] * c[2] > R0 * R0 * (1.0 + 1e-9))) return "an RBF centre lies inside S0";
        }
        P = n_centres + 1;
    }
    const int n = P - 1;
    build_decay();
    const int Lf = rows();
    if (Lf < n) return "fewer fit rows than basis functions: raise the number of check points";
    std::vector<double> A(static_cast<size_t>(Lf) * n), r1(std::max(P, p * p)), r2(std::max(P, p * p));
    for (int l = 0; l < L; ++l) {
        const double* y = &yc[static_cast<size_t>(l) * 3];
        const double* t = &yt[static_cast<size_t>(l) * 3];
        if (basis == 1) {
            for (int j = 0; j < n; ++j) {
                const double* c = &centres[static_cast<size_t>(j) * 3];
                const double a0 = y[0] - c[0], a1 = y[1] - c[1], a2 = y[2] - c[2];
                const double b0 = t[0] - c[0], b1 = t[1] - c[1], b2 = t[2] - c[2];
                const double ra = std::sqrt(a0 * a0 + a1 * a1 + a2 * a2), rb = std::sqrt(b0 * b0 + b1 * b1 + b2 * b2);
                A[static_cast<size_t>(j) * Lf + l] =
                    kernel == 1 ? std::exp(-kappa * ra) / ra - std::exp(-kappa * rb) / rb : 1.0 / ra - 1.0 / rb;
            }
        } else if (dim == 2) {
            basis2d(p, y[0] / R0, y[1] / R0, r1.data());
            basis2d(p, t[0] / R0, t[1] / R0, r2.data());
            for (int j = 0; j < n; ++j) A[static_cast<size_t>(j) * Lf + l] = r1[j + 1] - r2[j + 1];
        } else if (kernel == 2) {
            // value row l, then gradient rows L + k L + l: d/du_k B_t(u_l) - d/du_k B_t(u~_l)
            std::vector<double> d1(P), d2(P);
            for (int k = 0; k < 3; ++k) {
                bih_eval(rec, y[0] / R0, y[1] / R0, y[2] / R0, r1.data(), k, d1.data());
                bih_eval(rec, t[0] / R0, t[1] / R0, t[2] / R0, r2.data(), k, d2.data());
                for (int j = 0; j < n; ++j) A[static_cast<size_t>(j) * Lf + L + k * L + l] = d1[j + 1] - d2[j + 1];
            }
            for (int j = 0; j < n; ++j) A[static_cast<size_t>(j) * Lf + l] = r1[j + 1] - r2[j + 1];
        } else {
            rec.eval(y[0] / R0, y[1] / R0, y[2] / R0, r1.data());
            rec.eval(t[0] / R0, t[1] / R0, t[2] / R0, r2.data());
            for (int j = 0; j < n; ++j) A[static_cast<size_t>(j) * Lf + l] = r1[j + 1] - r2[j + 1];
        }
    }
    if (n_dec > 0 && periodic == 1) {
        // wire decay rows: <(dR_t/drho - beta R_t) trig(k x) trig(m theta)> over the
        // cylinder, R_t at y/R0.  Separable: first, per x node i and angular
        // harmonic (m, trig), the angular means G_V = <trig(m theta) R_t>_theta and
        // G_D = <trig(m theta) dR_t/drho>_theta; then each row is a sum over i.
        const int nh = 2 * p - 1;   // angular harmonics: cos(0), then cos(m .), sin(m .) for m >= 1
        std::vector<double> GV(static_cast<size_t>(mx) * nh * P, 0.0), GD(GV.size(), 0.0);
#pragma omp parallel
        {
            std::vector<double> V(P), D(P);
#pragma omp for schedule(dynamic, 1)
            for (int i = 0; i < mx; ++i) {
                double* gv = &GV[static_cast<size_t>(i) * nh * P];
                double* gd = &GD[static_cast<size_t>(i) * nh * P];
                for (int j = 0; j < mt; ++j) {
                    const double* q = &dec_pts[(static_cast<size_t>(i) * mt + j) * 3];
                    const double th = 2.0 * M_PI * j / mt;
                    rec.eval_dir(q[0] / R0, q[1] / R0, q[2] / R0, 0.0, std::cos(th), std::sin(th), V.data(), D.data());
                    for (int hh = 0; hh < nh; ++hh) {
                        const int mm = (hh + 1) / 2;
                        const double c = (hh == 0 || (hh & 1) ? std::cos(mm * th) : std::sin(mm * th)) / mt;
                        double* a = gv + static_cast<size_t>(hh) * P;
                        double* d = gd + static_cast<size_t>(hh) * P;
                        for (int t = 1; t < P; ++t) {
                            a[t] += c * V[t];
                            d[t] += c * (D[t] / R0);
                        }
                    }
                }
            }
        }
        std::vector<double> gq, wq;
        gauss_legendre(mx, gq, wq);
#pragma omp parallel for schedule(dynamic, 1)
        for (int r = 0; r < n_dec; ++r) {
            const double* row = &dec_rows[static_cast<size_t>(r) * 5];
            const int mm = static_cast<int>(row[1]);
            const int hh = mm == 0 ? 0 : 2 * mm - 1 + static_cast<int>(row[4]);
            std::vector<double> acc(n, 0.0);
            for (int i = 0; i < mx; ++i) {
                const double x = dec_pts[static_cast<size_t>(i) * mt * 3];
                const double wt = wq[i] / 2.0 * (row[3] == 0.0 ? std::cos(row[0] * x) : std::sin(row[0] * x));
                const double* gv = &GV[(static_cast<size_t>(i) * nh + hh) * P];
                const double* gd = &GD[(static_cast<size_t>(i) * nh + hh) * P];
                for (int j = 0; j < n; ++j) acc[j] += wt * (gd[j + 1] - row[2] * gv[j + 1]);
            }
            for (int j = 0; j < n; ++j) A[static_cast<size_t>(j) * Lf + L + r] = acc[j];
        }
    } else if (n_dec > 0) {
        // decay rows: <(dR_t/dz + s|k| R_t) trig(k.rho)> over a plane, R_t at y/R0
        const int m2 = m * m;
        std::vector<double> V(static_cast<size_t>(2) * m2 * P), D(static_cast<size_t>(2) * m2 * P);
#pragma omp parallel for schedule(static)
        for (int k = 0; k < 2 * m2; ++k) {
            const double* q = &dec_pts[static_cast<size_t>(k) * 3];
            rec.eval_dz(q[0] / R0, q[1] / R0, q[2] / R0, &V[static_cast<size_t>(k) * P], &D[static_cast<size_t>(k) * P]);
        }
#pragma omp parallel for schedule(dynamic, 1)
        for (int r = 0; r < n_dec; ++r) {
            const double* row = &dec_rows[static_cast<size_t>(r) * 5];
            const int pl = row[3] > 0 ? 0 : 1;
            std::vector<double> acc(n, 0.0);
            for (int k = 0; k < m2; ++k) {
                const double* q = &dec_pts[(static_cast<size_t>(pl) * m2 + k) * 3];
                const double ph = row[0] * q[0] + row[1] * q[1];
                const double wt = dec_w[k] * (row[4] == 0.0 ? std::cos(ph) : std::sin(ph));
                const double* v = &V[(static_cast<size_t>(pl) * m2 + k) * P];
                const double* d = &D[(static_cast<size_t>(pl) * m2 + k) * P];
                const double sk = row[3] * row[2];
                for (int j = 0; j < n; ++j) acc[j] += wt * (d[j + 1] / R0 + sk * v[j + 1]);
            }
            for (int j = 0; j < n; ++j) A[static_cast<size_t>(j) * Lf + L + r] = acc[j];
        }
    }
    // step 5: decomposition -> pseudo-inverse
    pseudo_inverse(Lf, n, std::move(A), rcond, pinv, rank, cond);
    if (rank < 1) return "fitting matrix has numerical rank zero";
    // step 6: box integrals of the basis: the box-mean potential at each RBF centre
    // (App. C), or tensor Gauss-Legendre with N_q = floor((p-1)/2) + 1 nodes (App. B)
    if (basis == 1) {
        box_means.assign(P, 0.0);
        if (kernel == 1) return std::string();   // no constant to fix: nothing uses the box integrals
        box_means[0] = 1.0;
        for (int t = 1; t < P; ++t) {
            const double* c = &centres[static_cast<size_t>(t - 1) * 3];
            box_means[t] = box_mean_potential(box, c[0], c[1], c[2]);
        }
        return std::string();
    }
    const int nq = (p - 1) / 2 + 1;
    std::vector<double> xg, wg;
    gauss_legendre(nq, xg, wg);
    box_means.assign(P, 0.0);
    if (dim == 2) {   // over the rectangle
        for (int i = 0; i < nq; ++i)
            for (int j = 0; j < nq; ++j) {
                basis2d(p, 0.5 * box[0] * xg[i] / R0, 0.5 * box[1] * xg[j] / R0, r1.data());
                const double w = wg[i] * wg[j] / 4.0;
                for (int t = 0; t < P; ++t) box_means[t] += w * r1[t];
            }
        return std::string();
    }
    for (int i = 0; i < nq; ++i)
        for (int j = 0; j < nq; ++j)
            for (int k = 0; k < nq; ++k) {
                const double u[3] = {0.5 * box[0] * xg[i] / R0, 0.5 * box[1] * xg[j] / R0, 0.5 * box[2] * xg[k] / R0};
                if (kernel == 2) bih_eval(rec, u[0], u[1], u[2], r1.data());
                else rec.eval(u[0], u[1], u[2], r1.data());
                const double w = wg[i] * wg[j] * wg[k] / 8.0;
                for (int t = 0; t < P; ++t) box_means[t] += w * r1[t];
            }
    return std::string();
}

// ---------------------------------------------------------------------------
// serialization of the set data
// ---------------------------------------------------------------------------
namespace {
template <typename T>
void put(std::vector<unsigned char>& out, const T& v)
{
    const unsigned char* b = reinterpret_cast<const unsigned char*>(&v);
    out.insert(out.end(), b, b + sizeof(T));
}
template <typename T>
void put_vec(std::vector<unsigned char>& out, const std::vector<T>& v)
{
    const unsigned char* b = reinterpret_cast<const unsigned char*>(v.data());
    out.insert(out.end(), b, b + sizeof(T) * v.size());
}
template <typename T>
bool get(const unsigned char* data, size_t size, size_t& pos, T& v)
{
    if (size - pos < sizeof(T) || pos > size) return false;
    std::memcpy(&v, data + pos, sizeof(T));
    pos += sizeof(T);
    return true;
}
template <typename T>
bool get_vec(const unsigned char* data, size_t size, size_t& pos, std::vector<T>& v, size_t n)
{
    if (pos > size || (size - pos) / sizeof(T) < n) return false;
    v.resize(n);
    if (n) std::memcpy(v.data(), data + pos, sizeof(T) * n);
    pos += sizeof(T) * n;
    return true;
}
}  // namespace

uint64_t fnv1a64(const unsigned char* data, size_t n)
{
    uint64_t h = 0xcbf29ce484222325ull;
    for (size_t i = 0; i < n; ++i) {
        h ^= data[i];
        h *= 0x100000001b3ull;
    }
    return h;
}

void SystemSetup::serialize(std::vector<unsigned char>& out) const
{
    for (int k = 0; k < 3; ++k) put(out, box[k]);
    put(out, static_cast<int32_t>(basis));
    put(out, R0);
    put(out, R_b);
    put(out, thr);
    put(out, V0);
    put(out, static_cast<int32_t>(p));
    put(out, static_cast<int32_t>(P));
    put(out, static_cast<int32_t>(L));
    put(out, static_cast<int32_t>(rank));
    put(out, cond);
    put(out, static_cast<int32_t>(images.size() / 3));
    put(out, static_cast<int32_t>(centres.size() / 3));
    put(out, static_cast<int32_t>(periodic));
    put(out, static_cast<int32_t>(kernel));
    put(out, kappa);
    put(out, static_cast<int32_t>(dim));
    put_vec(out, yc);
    put_vec(out, yt);
    put_vec(out, pinv);
    put_vec(out, box_means);
    put_vec(out, images);
    put_vec(out, centres);
}

std::string SystemSetup::deserialize(const unsigned char* data, size_t size, size_t& pos)
{
    int32_t b = 0, p_ = 0, P_ = 0, L_ = 0, rank_ = 0, nimg = 0, M = 0, per = 0, ker = 0, dm = 0;
    double kap = 0.0;
    bool ok = true;
    for (int k = 0; k < 3; ++k) ok = ok && get(data, size, pos, box[k]);
    ok = ok && get(data, size, pos, b) && get(data, size, pos, R0) && get(data, size, pos, R_b) &&
         get(data, size, pos, thr) && get(data, size, pos, V0) && get(data, size, pos, p_) &&
         get(data, size, pos, P_) && get(data, size, pos, L_) && get(data, size, pos, rank_) &&
         get(data, size, pos, cond) && get(data, size, pos, nimg) && get(data, size, pos, M) &&
         get(data, size, pos, per) && get(data, size, pos, ker) && get(data, size, pos, kap) &&
         get(data, size, pos, dm);
    if (!ok) return "truncated system record";
    if (per != 7 && per != 3 && per != 1) return "bad periodic axes";
    if (per != 7 && b != 0) return "the RBF basis needs three periodic axes";
    if (ker != 0 && ker != 1 && ker != 2) return "bad kernel";
    if (ker == 1 && (b != 1 || per != 7 || !(kap > 0.0) || !std::isfinite(kap))) return "bad screened-kernel record";
    if (ker == 2 && (b != 0 || per != 7 || dm != 3 || p_ < 3 || p_ > 30)) return "bad biharmonic-kernel record";
    for (int k = 0; k < 3; ++k)
        if (!(box[k] > 0.0) || !std::isfinite(box[k])) return "bad box lengths";
    if (b != 0 && b != 1) return "bad basis";
    if (dm != 3 && dm != 2) return "bad dimension";
    if (dm == 2 && (b != 0 || per != 3 || ker != 0 || box[2] != 1.0)) return "bad record of a plane system";
    if (p_ < 2 || p_ > (dm == 2 ? 128 : 40)) return "p out of range";
    if (b == 0 && (P_ != (dm == 2 ? 2 * p_ - 1 : (ker == 2 ? p_ * p_ + (p_ - 2) * (p_ - 2) : p_ * p_)) || M != 0))
        return "basis size does not match p";
    if (b == 1 && (M < 1 || M > 4096 || P_ != M + 1)) return "bad RBF centre count";
    if (L_ < 1 || L_ > (1 << 20)) return "bad check-point count";
    if (rank_ < 1 || rank_ > P_ - 1) return "bad rank";
    if (nimg < 1 || nimg > (1 << 20)) return "bad image count";
    if (!(R0 > 0.0) || !(R_b > R0) || !std::isfinite(R_b) || !(thr > 0.0) || !(V0 > 0.0)) return "bad geometry";
    basis = b;
    p = p_;
    P = P_;
    L = L_;
    rank = rank_;
    periodic = per;
    dim = dm;
    kernel = ker;
    kappa = ker == 1 ? kap : 0.0;
    if (kernel == 1 && !(kappa * R0 <= 64.0)) return "kappa out of range";
    build_decay();
    if (rows() < P - 1) return "bad check-point count";
    const size_t l3 = static_cast<size_t>(L) * 3;
    ok = get_vec(data, size, pos, yc, l3) && get_vec(data, size, pos, yt, l3) &&
         get_vec(data, size, pos, pinv, static_cast<size_t>(P - 1) * rows()) && get_vec(data, size, pos, box_means, P) &&
         get_vec(data, size, pos, images, static_cast<size_t>(nimg) * 3) &&
         get_vec(data, size, pos, centres, static_cast<size_t>(M) * 3);
    if (!ok) return "truncated system arrays";
    if (images[0] != 0 || images[1] != 0 || images[2] != 0) return "the first image must be the box itself";
    for (int v : images)
        if (v < -(1 << 16) || v > (1 << 16)) return "image index out of range";
    {
        std::vector<std::array<int, 3>> sorted(nimg);
        for (int i = 0; i < nimg; ++i) sorted[i] = {images[3 * i], images[3 * i + 1], images[3 * i + 2]};
        std::sort(sorted.begin(), sorted.end());
        if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end()) return "repeated image";
    }
    for (double v : pinv)
        if (!std::isfinite(v)) return "non-finite pseudo-inverse entry";
    rec.build(p);
    return std::string();
}

}  // namespace ps
