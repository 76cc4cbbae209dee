"""FP64 CPU oracle for the periodized Coulomb sum of Gumerov & Duraiswami
("A method to compute periodic sums").

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call, link
or execute anything in this package; only the test-suite, the smoke check and
the benchmark's CPU-baseline leg use it.  It shares no code with the HIP library.

Parts:
  * ``method``  -- the method's "set" and "get" algorithms (Sec. 2.3), for the
    Laplace kernel with the renormalized solid-harmonic basis (Sec. 3.1,
    eqs. (1.6)-(1.8)), Gauss spherical check points (Sec. 2.2), SVD
    pseudo-inverse (eq. (10)), box integrals (App. B) and the zero-mean
    constant via the face/edge reduction of App. C;
  * ``ewald``   -- an independent classical Ewald sum (App. D);
  * ``adjoint`` -- the exact gradient of the method's energy with respect to
    positions and charges (derived from eqs. (3), (8), (10), (pfx3)-(pfx4));
  * ``slab``    -- the method with the periodic extension along x and y only
    (Sec. 1, closing paragraph), with the reading that completes it: decay
    rows on planes above and below the box fix the far field's x/y-periodic
    harmonic modes that periodicity alone leaves free;
  * ``ewald2d`` -- an independent Ewald sum for charges periodic in x and y;
  * ``screened`` -- the method for the screened Coulomb kernel exp(-kappa r)/r
    (the paper's "other kernels", Sec. 1) with the kernel-at-centres basis of
    eq. (5), and an independent Ewald-type split of its periodic sum;
  * ``wire``    -- the method with the periodic extension along x only (Sec. 1,
    closing paragraph), completed by decay rows on a cylinder around the
    box that fix the far field's Fourier modes (K_m Bessel and rho^-m
    decay), and a brute-force row sum with Richardson extrapolation;
  * ``twod``    -- the method in two dimensions (Sec. 1: it applies to 2-D problems)
    for K = -log r: harmonic-polynomial basis, check points on the
    circumcircle, the uniform-rectangle box mean; an independent 2-D Ewald
    split, the Jacobi theta-function closed form and brute-force squares;
  * ``biharmonic`` -- the method for K = r (the biharmonic equation, whose
    null space Sec. 3 names as the Laplace kernel's): the Almansi basis
    (harmonics and |u|^2 times harmonics), value and gradient periodicity
    rows, the closed-form box mean of r; and an independent Ewald-type split;
  * ``pairs.c`` -- FP64 compensated direct sums (eq. (r2)), OpenMP over targets.

Pins (tests/test_oracle_*.py): the basis against an independent assembly from
associated Legendre functions (eq. (1.1)-(1.4.1)), harmonicity and finite
differences; the Gauss grid counts L = 2p^2 - p against the N+2L columns of
Tables 2-3; near-set sizes against A_gf lambda^3 N (eq. (o2.1), Table 5); box
integrals against closed forms; Phi0 against the textbook prism potential,
quadrature and its Laplacian; Ewald against its splitting-parameter
independence and the NaCl Madelung constant (eq. (st1)); the method against
the Madelung constant, Table 1's Gauss-grid errors, Ewald, periodicity and
translation invariance; the adjoint against central finite differences; the
slab Ewald sum against brute-force square-shell lattice sums (extrapolated), its
splitting parameter and Gauss's law; the slab method against that Ewald sum
(thin, thick and elongated cells, a dipolar cell), x/y periodicity and in-plane
translation invariance; the screened direct sums against the modified Helmholtz
equation, finite differences and the Coulomb limit; the screened split against
its splitting parameter and brute-force lattice sums; the screened method
against that split, periodicity and translation invariance; the wire row sum
against its K_0 Fourier series (Poisson summation along x), the exact
potential against the decay rows, the periodicity rows' exact null space
(rho^m e^{i m theta}), and the wire method against the row sum (thin and long
cells, charges next to the cylinder, a transverse dipole), x periodicity and
translation invariance along x; the 2-D basis against closed forms, harmonicity
and differences, the rectangle potential against quadrature and its Laplacian,
the 2-D Ewald split against its parameter, the theta-function closed form and
brute-force squares of images, and the 2-D method against Ewald (other cells,
a strong dipole, targets on particles), periodicity and translation invariance;
the biharmonic corner primitive against its third derivative and quadrature,
its box mean's Laplacian against twice Phi0, the Almansi basis against the far
expansion of r, the biharmonic split against its parameter, periodicity and
Delta phi = 2 phi_Coulomb, and the biharmonic method against that split (to
1e-12), its convergence in p and translation invariance, and its exact energy
gradient against central differences.
"""
