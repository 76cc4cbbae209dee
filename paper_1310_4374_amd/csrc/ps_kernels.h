// Host launchers of the HIP kernels (ps_kernels.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "ps_device.h"

namespace ps {

void launch_fill_i32(int* p, int64_t n, int v, hipStream_t st);
void launch_validate(int nsys, int nblk, const SysDev* sys, const double* X, const double* Y, const double* Z,
                     const double* Q, int* status, double* part, hipStream_t st);
void launch_sort(int nsys, int64_t ncitems, int64_t max_ncell, const SysDev* sys, const CItem* citems, const double* X,
                 const double* Y, const double* Z, const double* Q, int* keys, int* slots, int* cnt, int* start,
                 int64_t ncnt_total, int scan_blocks, int64_t* scan_tot, int* perm, double* sx, double* sy, double* sz,
                 double* sq, hipStream_t st);
void launch_near(int nsys, int64_t nnitems, const SysDev* sys, const NItem* nitems, const double* img,
                 const double* sx, const double* sy, const double* sz, const double* sq, int* ncount, int64_t* ioff,
                 int64_t* nnear, double* nx, double* ny, double* nz, double* nq, int* nbase, int* inv, hipStream_t st);
void launch_tblock(int64_t nitems, const PJob* jobs, const TItem* items, hipStream_t st);
// kern: 0 Coulomb 1/r, 1 screened exp(-kappa r)/r (kappa from each job)
void launch_p2p(int prec, int bt, bool field, int kern, int64_t nitems, const PJob* jobs, const PItem* items,
                hipStream_t st);
// FP32 check-point sums (potential only); every job has 64-target blocks and ncomp = 1.
void launch_chk_f32(int kern, int64_t nitems, const PJob* jobs, const PItem* items, hipStream_t st);
// dfield: 3 x dec_tot scratch for the decay-surface near sums reduced over splits
void launch_decay_rhs(int nsys, int maxdec, int64_t maxpts, const SysDev* sys, const PJob* djobs, const double* dpts,
                      int64_t dec_tot, double* dfield, const double* dw, const double* drows, double* f, hipStream_t st);
// slot[chk_off + k]: position of check target k of a system in its check job
void launch_solve(int nsys, int maxL, int maxP, const SysDev* sys, const PJob* cjobs, const int* slot,
                  const double* pinv, double* coef, double* f, hipStream_t st);
void launch_mean(int nsys, int64_t nwitems, const SysDev* sys, const CItem* witems, const int64_t* nnear,
                 const double* nx, const double* ny, const double* nz, const double* nq, double* part,
                 int64_t nmitems, int mcols, const MItem* mitems, const int* imap, const double* img,
                 const double* sx, const double* sy, const double* sz, const double* sq, double* mpart,
                 const double* bm, double* coef, hipStream_t st);
void launch_far(int lanes, int64_t nitems, int maxP, int maxp, const SysDev* sys, const CItem* items,
                const PJob* pjobs, const PJob* fjobs, const double* coef, const double* rec, const int* perm,
                double* phi, double* ex, double* ey, double* ez, double* osort, hipStream_t st);

}  // namespace ps

namespace ps {
void launch_energy(int nsys, const SysDev* sys, const double* sq, const double* osort, double* energy, hipStream_t st);
// the plane's moments (basis 1, Re w^n, Im w^n)
void launch_moments2d(int P, const SysDev* sys, const double* sx, const double* sy, const double* sq, double* mom_part,
                      int mom_blocks, hipStream_t st);
void launch_moments(int P, int p, const SysDev* sys, const double* sx, const double* sy, const double* sz,
                    const double* sq, const double* rec, double* mom_part, int mom_blocks, hipStream_t st);
void launch_adjoint_sources(int P, int L, int64_t n, const SysDev* sys, const double* sx, const double* sy,
                            const double* sz, const double* sq, const double* mom_part, int mom_blocks, int stride,
                            int toff, const double* pinv, const double* chk, int64_t chk_tot, double* ax, double* ay,
                            double* az, double* aq, double* wdec, hipStream_t st);
// the decay rows' adjoint sources (slab, wire) and their psi at the nb near entries
// The biharmonic fit's gradient rows in the adjoint: dipoles at the check
// points and partners (weights wg = the rows' w, 3L), psi and -grad psi at the
// nb near entries into dpart (4 x nb).
void launch_adjoint_dipoles(int64_t nb, const SysDev* sys, const double* nx, const double* ny, const double* nz,
                            const double* chk, int64_t chk_tot, const double* wg, double* dpart, hipStream_t st);
void launch_adjoint_decay(int64_t npts, int64_t nb, const SysDev* sys, const double* dpts, int64_t dec_tot,
                          const double* dw, const double* drows, const double* wdec, double* ad, double* bd,
                          const double* nx, const double* ny, const double* nz, double* dpart, hipStream_t st);
void launch_adjoint_finish(int64_t n, const SysDev* sys, const PJob* ajob, const int* inv, const double* sq,
                           const double* osort, int exact, const double* dpart, int64_t dstride, double* dq, double* dx,
                           const int* perm, const double* gE, double* oq, double* ox, double* oy, double* oz,
                           hipStream_t st);
}  // namespace ps
namespace ps {
int p2p_blocks_per_cu(int prec, int bt);
}
