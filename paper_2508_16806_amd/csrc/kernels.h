// kernels.h -- host-side launch wrappers of the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "pdhg_internal.h"

namespace pdhg {

template <typename T>
void launch_primal(const Dev &d, int j, int avg, uint8_t *mask, hipStream_t s);
template <typename T>
void launch_dual(const Dev &d, int j, int avg, uint8_t *mask, hipStream_t s);
template <typename T>
void launch_primal_ad(const Dev &d, hipStream_t s);
template <typename T>
void launch_dual_ad(const Dev &d, hipStream_t s);
void launch_step_ad(const Dev &d, hipStream_t s);
template <typename T>
void launch_commit_ad(const Dev &d, hipStream_t s);
template <typename T>
void launch_kx_ad(const Dev &d, int all, hipStream_t s);
template <typename T>
void launch_infeas(const Dev &d, const void *xp, const void *yp, hipStream_t s);
template <typename T>
void launch_save_prev(const Dev &d, hipStream_t s);
template <typename T>
void launch_check(const Dev &d, int avg, hipStream_t s);
void launch_check64(const Dev &d, const double *xs, const double *ys, hipStream_t s);
void launch_control(const Dev &d, const CtlParams &P, int iters_done, hipStream_t s);
// active lists of the running instances; budget > 0 admits waiting instances
// (first = 1: instances beyond the budget start waiting)
void launch_active(const Dev &d, hipStream_t s, int64_t budget = 0, int first = 0);
template <typename T>
void launch_restart(const Dev &d, hipStream_t s);

void launch_fill(double *p, int64_t n, double v, hipStream_t s);
void launch_rowmax(const OpDev &op, int remap, bool row_first, const double *rowfac,
                   const double *colfac, double *out, hipStream_t s);
void launch_ruiz_update(double *fac, const double *mx, int64_t n, hipStream_t s);
void launch_scale_vals(const OpDev &op, double *v64, float *v32, bool row_first,
                       const double *rowfac, const double *colfac, hipStream_t s);
template <typename T>
void launch_scale_data(const Dev &d, hipStream_t s);
void launch_spmv64(const OpDev &op, int remap, const double *v, double *out, double *partials,
                   const int32_t *list, const int32_t *cnt, hipStream_t s);
void launch_inst_sum(const Dev &d, int onK, const double *partials, double *out, hipStream_t s);
void launch_normalize(double *v, const int32_t *inst_of, int64_t n, const double *nrm2, hipStream_t s);
void launch_power_test(const Dev &d, const double *w2, int it, double tol, int final_pass, hipStream_t s);
void launch_inst_nrm2(const Dev &d, int primal, const double *v, double *out, hipStream_t s);
template <typename T>
void launch_init_point(const Dev &d, hipStream_t s);
template <typename T>
void launch_epoch_start(const Dev &d, hipStream_t s);
template <typename T>
void launch_point_to64(const Dev &d, int which, double *xo, double *yo, hipStream_t s);
void launch_unscale_x(const Dev &d, int64_t off, int64_t n, const double *xs, double *out, hipStream_t s);
void launch_unscale_y(const Dev &d, int64_t off, int64_t m, const double *ys, double *out, hipStream_t s);
void launch_lambda(const Dev &d, const double *ys, double *lam, hipStream_t s);
void launch_permute_out(const int32_t *perm, int64_t off, int64_t n, const double *src, double *out,
                        hipStream_t s);
void launch_scale_in(const Dev &d, int64_t xoff, int64_t n, int64_t yoff, int64_t m, const double *xin,
                     const double *yin, double *xs, double *ys, hipStream_t s);
template <typename T>
void launch_set_point(const Dev &d, int64_t xoff, int64_t n, int64_t yoff, int64_t m, int64_t m1,
                      const double *xs, const double *ys, hipStream_t s);
void launch_kkt_final(const Dev &d, int inst, double *out9, hipStream_t s);

template <typename T>
void launch_fish_step(const Dev &d, const FishDev &f, int lj, double tau, double sigma, int64_t m1, hipStream_t s);
template <typename T>
void launch_fish_init(const Dev &d, const FishDev &f, int lp, double sc, hipStream_t s);
template <typename T>
int launch_fish_gap_rank(const Dev &d, const FishDev &f, int lj, int round, int repop, int half, int64_t wpos,
                         hipStream_t s);
template <typename T>
void launch_fish_gather(const Dev &d, const FishDev &f, int lnext, int half, hipStream_t s);
template <typename T>
void launch_fish_out(const Dev &d, const FishDev &f, hipStream_t s);

void launch_adj_init(const Dev &d, const AdjBufs &a, const double *gx, const double *gy, hipStream_t s);
void launch_adj_w(const Dev &d, const AdjBufs &a, const uint8_t *mask_y, hipStream_t s);
template <typename T>
void launch_rev_primal(const Dev &d, const AdjBufs &a, const uint8_t *mask_x, hipStream_t s);
template <typename T>
void launch_rev_dual(const Dev &d, const AdjBufs &a, hipStream_t s);
void launch_adj_out(const Dev &d, const AdjBufs &a, double *gc, double *gq, double *gl, double *gu,
                    double *gx0, double *gy0, hipStream_t s);
void launch_set_raw(const Dev &d, const double *c, const double *q, const double *l, const double *u,
                    hipStream_t s);

// the fixed workspace of pdhg_setup_noalloc (noalloc.hip)
hipError_t noalloc_claim(int dev, const void *owner, void **ptr, int *busy);
void noalloc_release(int dev, const void *owner);

}  // namespace pdhg
