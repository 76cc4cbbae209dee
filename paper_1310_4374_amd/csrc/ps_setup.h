// Host-side FP64 "set" phase of the periodized sum (Sec. 2.3, algorithm "set").
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace ps {

// Coefficients of the renormalized solid-harmonic recurrence, obtained by
// folding the scale factors sqrt((n-|m|)!(n+|m|)!) of eq. (1.7) into the
// Cartesian recurrence of eq. (1.6):
//   R^_m^{+m} = -c_m (x R^_{m-1}^{m-1} + y R^_{m-1}^{-(m-1)}),
//   R^_m^{-m} =  c_m (y R^_{m-1}^{m-1} - x R^_{m-1}^{-(m-1)}),   c_m = sqrt((2m-1)/(2m)),
//   R^_n^m    = -a_nm z R^_{n-1}^m - b_nm r^2 R^_{n-2}^m          (n > |m|),
//   a_nm = (2n-1)/sqrt((n-|m|)(n+|m|)),  b_nm = sqrt((n-|m|-1)(n+|m|-1)/((n-|m|)(n+|m|))),
// with R^_0^0 = 1 and R^_0^{-0} = 0.  Index t = n^2 + n + m (eq. (1.8), 0-based).
struct Recurrence {
    int p = 0;
    std::vector<double> a, b;  // [p*p], indexed by t
    std::vector<double> c;     // [p], c[0] unused
    void build(int p_);
    // R^_t at (x, y, z) for t < p*p.
    void eval(double x, double y, double z, double* out) const;
    // R^_t and dR^_t/dz (forward-mode differentiation of the same recurrence;
    // the diagonal terms do not depend on z).
    void eval_dz(double x, double y, double z, double* out, double* dout) const;
    // R^_t and its derivative along the direction (u, v, w) (forward mode).
    void eval_dir(double x, double y, double z, double u, double v, double w, double* out, double* dout) const;
};

void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w);

// The plane's harmonic polynomials at the scaled point (x, y): out[0] = 1,
// out[2n-1] = Re w^n, out[2n] = Im w^n, w = x + iy, n = 1..p-1.
void basis2d(int p, double x, double y, double* out);

// The biharmonic basis at the scaled point u = (x, y, z): the p^2 harmonics R^_t,
// then |u|^2 R^_t for t < (p-2)^2.  With dir in 0..2 also d/du_dir of each (dout).
void bih_eval(const Recurrence& rec, double x, double y, double z, double* out, int dir = -1, double* dout = nullptr);

// Mean of 1/|y - x| over the box [-d/2, d/2]^3 (divided by its volume): the
// closed-form potential of a uniform rectangular prism, summed over corners.
double box_mean_potential(const double box[3], double x, double y, double z);

struct SystemSetup {
    double box[3] = {0, 0, 0};
    int basis = 0;                     // 0 spherical, 1 RBF
    std::vector<double> centres;       // RBF: [M*3]
    double R0 = 0, R_b = 0, thr = 0, V0 = 0;
    int p = 0, P = 0, L = 0;
    int rank = 0;
    double cond = 0;
    std::vector<double> yc, yt;        // [L*3] check points and partners
    std::vector<double> pinv;          // (P-1) x rows(), row-major: C_{t+1} = sum_l pinv[t*rows()+l] f_l
    std::vector<double> box_means;     // [P]: R_t^(0), App. B
    std::vector<int> images;           // [nimg*3] lattice integers, (0,0,0) first
    Recurrence rec;
    // Periodic axes: 7 (x, y and z), 3 (x and y: a slab, z free) or 1 (x only: a
    // wire, y and z free).  With fewer than three axes the fit has n_dec decay
    // rows after the L periodicity rows, which fix the far field's modes that
    // periodicity alone leaves free:
    //   slab: on the planes z = +-zd (zd = d3/2 + R0/10) the in-plane Fourier
    //     modes of the potential decay away from the charges,
    //     <(d/dz + s|k|) phi, trig(k.rho)> = 0;
    //   wire: on the cylinder rho = rho_d (rho_d = |(d2, d3)|/2 + R0/10) each
    //     Fourier mode in (x, theta) is the decaying one,
    //     <(d/drho - beta_{k,m}) phi, trig(k x) trig(m theta)> = 0,
    //     beta = |k| K_m'(|k| rho_d) / K_m(|k| rho_d) (k != 0), -m / rho_d (k = 0).
    int periodic = 7;
    int n_dec = 0, nk = 0;             // decay rows; wave numbers 2 pi n / d, |n| <= nk
    int m = 0;                         // slab: m x m Gauss points per plane
    int mx = 0, mt = 0;                // wire: Gauss points along x, equispaced angles
    int nsurf = 0, npts = 0;           // decay surfaces (2 planes, 1 cylinder), points per surface
    double zd = 0, rho_d = 0;
    std::vector<double> dec_pts;       // [nsurf * npts * 3]: slab top plane then bottom; wire x-major, theta minor
    std::vector<double> dec_w;         // [npts] quadrature weights (sum 1), shared by the surfaces
    std::vector<double> dec_rows;      // [n_dec * 5]: slab kx, ky, |k|, s (+1 top, -1 bottom), trig (0 cos, 1 sin);
                                       // wire k, m, beta, trig in x, trig in theta
    // rows of the fit (columns of pinv): L periodicity rows of the potential, then
    // the decay rows (slab, wire) or the 3L gradient rows (biharmonic kernel)
    int rows() const { return L + (kernel == 2 ? 3 * L : n_dec); }
    // Kernel: 0 Coulomb 1/r; 1 screened exp(-kappa r)/r (RBF basis, three periodic
    // axes; no constant basis function to fix: box_means stay zero); 2 the
    // biharmonic r (spherical basis extended by |u|^2 times the harmonics of
    // degree <= p-3, P = p^2 + (p-2)^2; after the L value rows, rows L + k L + l
    // ask for the same periodicity of d/du_k at check pair l, u = y/R0).
    int kernel = 0;
    double kappa = 0;
    // Dimension: 3, or 2 for the method in the plane (kernel -log r, x and y
    // periodic; the basis 1, Re w^n, Im w^n with w = (x + iy)/R0, P = 2p - 1;
    // L = 4p check points equispaced on the circumcircle; box[2] is held at 1 and
    // every z at 0, so the 3-D near set, ordering and pair sums apply unchanged).
    int dim = 3;
    // Returns an empty string on success, or the reason for failure.
    std::string build(const double box[3], int p, double R_b, double lambda, double rcond, int basis = 0,
                      int n_centres = 0, const double* centres = nullptr, int n_check = 0,
                      const double* check_points = nullptr, int periodic = 7, int kernel = 0, double kappa = 0,
                      int dim = 3);
    // The decay surfaces and rows (a function of the periodic axes, box, p and R0 alone).
    void build_decay();
    // Binary form of the set data (little-endian scalars and arrays; the
    // recurrence coefficients and the decay tables are rebuilt on reading).
    void serialize(std::vector<unsigned char>& out) const;
    // Reads what serialize wrote, advancing pos; checks every size against the
    // bounds build() enforces.  Returns an empty string on success.
    std::string deserialize(const unsigned char* data, size_t size, size_t& pos);
};

// 64-bit FNV-1a hash of a byte range (file integrity check).
uint64_t fnv1a64(const unsigned char* data, size_t n);

}  // namespace ps
