// kernels.hip -- gfx950 kernels of the PDHG hot path and its setup.
//
// Iteration (Algorithm 1 in the sign-consistent form of Appendices C/D,
// theta = 1), all in the scaled variables of Section 2.4.1:
//   primal sweep over rows j of K~^T:  g = (K~^T y)_j,
//       x+_j = clip(x_j - tau (c~_j - g), l~_j, u~_j),  xbar_j = 2 x+_j - x_j,
//       running epoch average kept as the mean offset from the epoch start x0:
//       xavg_j += ((x+_j - x0_j) - xavg_j) / (t + 1), average = x0 + xavg
//   dual sweep over rows i of K~:      r = (K~ xbar)_i,
//       y+_i = proj_Y(y_i + sigma (q~_i - r)) (clip at 0 for ">=" rows), yavg
// Check every N iterations: FP64 residual sums of the current iterate and of
// the epoch average (Section 2.3.2 on the original LP, the omega-weighted
// metric of Section 2.4.2 on the scaled one) as per-workgroup partials;
// control: candidate choice, termination, the three restart criteria and the
// primal-weight update (Algorithm 4), one workgroup per instance.
#include <hip/hip_runtime.h>
#include <math.h>

#include "../../include/pdhg.h"
#include "kernels.h"
#include "sweep.h"

namespace pdhg {

// ---------------------------------------------------------------------------
// hot path: fused SpMV + update sweeps
// ---------------------------------------------------------------------------

// The solve-time sweeps run a bounded grid that walks the compacted list of
// logical blocks of instances still running (see k_act_fill), so finished
// instances of a batch cost nothing.  Each logical block computes exactly what
// it would in a full launch.
//
// Column slices (op.slices = S > 1, opts.col_slices / col_slices_t): rows of
// sliced segments keep their entries grouped by slice of the gathered vector
// and are swept in S launches, so each launch gathers from one slice of it,
// which stays in the L2 of each XCD.  SL selects the launch's role:
//   SL = 0  whole rows, one launch (no slices);
//   SL = 1  pass `pass` < S-1: the sliced rows only, their FP64 partial
//           product over slice `pass` into op.part (pass 0 writes it, later
//           passes add theirs);
//   SL = 2  pass S-1: the sliced rows add their last slice to the partial,
//           the rows of unsliced segments are swept whole, and every row is
//           updated as with SL = 0.
// The partial store and the update stores are in different launches, so no
// launch chooses between two store targets for one row.

// One partial pass over the rows of a sliced block (SL = 1).
template <int L, int R, typename T>
__device__ __forceinline__ void slice_partial(const OpDev &op, const Seg &s, int bi, const T *__restrict__ g,
                                              double *red, int pass)
{
    using RS = RowSweep<L, 1, T, T, R, false, true, true>;
    const typename RS::Pos ps = RS::locate(s, bi);
    double acc[R][1];
    RS::dot(op, ps, g, nullptr, nullptr, red, acc, op.sb, op.slices, pass);
    if (ps.leader) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (r >= ps.nvalid) break;
            const int64_t i = ps.row0 + r;
            op.part[i] = pass > 0 ? op.part[i] + acc[r][0] : acc[r][0];
        }
    }
}

// MASK: also record the clip region of x (0 interior, 1 at l, 2 at u) for the
// adjoint replay (whole rows only).
template <typename T, int AVG, int MASK, int RM, int SL>
__global__ __launch_bounds__(WG) void k_primal(Dev d, int j_in_chunk, uint8_t *__restrict__ mask, int pass)
{
    __shared__ double red[8];
    const OpDev &op = d.Kt;
    T *__restrict__ x = (T *)d.x;
    T *__restrict__ xb = (T *)d.xbar;
    T *__restrict__ xa = (T *)d.xavg;
    const T *__restrict__ x0 = (const T *)d.x0;
    const T *__restrict__ c = (const T *)d.c;
    const T *__restrict__ l = (const T *)d.l;
    const T *__restrict__ u = (const T *)d.u;
    const T *__restrict__ y = (const T *)d.y;
    const int cnt = d.act_cnt[1];
    const bool full = cnt == op.nblk;  // every block active: the list is the identity
    for_each_item_split(cnt, d.remap, d.act_split + 9, j_in_chunk & 1, [&](int it) {
        const int lb = full ? it : d.actT[it];
        const Seg s = block_seg(op, lb);
        if (SL == 1 && !s.sliced) return;
        const InstState *st = d.st + s.inst;
        const double tau = st->tau;
        const double w = AVG ? 1.0 / (double)(st->t_inner + j_in_chunk + 1) : 0.0;
        const int bi = lb - s.blk0;
        dispatch_lanes<RM>(s.lanes_log2, [&](auto tag, auto rtag) {
            constexpr int L = decltype(tag)::value, R = decltype(rtag)::value;
            if constexpr (SL == 1) {
                slice_partial<L, R>(op, s, bi, y, red, pass);
                return;
            }
            using RS = RowSweep<L, 1, T, T, R, false, true, SL == 2>;
            const typename RS::Pos ps = RS::locate(s, bi);
            // the update's operands are loaded before the dot products so their
            // latency overlaps the streaming of the rows (unconditional loads
            // from clamped rows: no branch forces a wait)
            T r_x[R], r_c[R], r_l[R], r_u[R], r_a[R], r_0[R];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int64_t jj = r < ps.nvalid ? ps.row0 + r : ps.blk_row0;
                r_x[r] = x[jj];
                r_c[r] = c[jj];
                r_l[r] = l[jj];
                r_u[r] = u[jj];
                r_a[r] = AVG ? xa[jj] : T(0);
                r_0[r] = AVG ? x0[jj] : T(0);
            }
            double acc[R][1];
            // SL = 2: rows of unsliced segments as one slice, the whole row
            RS::dot(op, ps, y, nullptr, nullptr, red, acc, op.sb, s.sliced ? op.slices : 1, s.sliced ? pass : 0);
            if (ps.leader) {
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    if (r >= ps.nvalid) break;
                    const int64_t j = ps.row0 + r;
                    const double g = (SL == 2 && s.sliced) ? op.part[j] + acc[r][0] : acc[r][0];
                    const double xo = (double)r_x[r], cj = (double)r_c[r], lo = (double)r_l[r];
                    const double hi = (double)r_u[r], xav = (double)r_a[r];
                    const double v = xo - tau * (cj - g);
                    const double xn = v < lo ? lo : (v > hi ? hi : v);
                    const T xnT = (T)xn;
                    x[j] = xnT;
                    xb[j] = (T)(2.0 * (double)xnT - xo);
                    if (AVG) xa[j] = (T)(xav + (((double)xnT - (double)r_0[r]) - xav) * w);
                    if (MASK) mask[j] = (uint8_t)(v <= lo ? 1 : (v >= hi ? 2 : 0));
                }
            }
        });
    });
}

template <typename T, int AVG, int MASK, int RM, int SL>
__global__ __launch_bounds__(WG) void k_dual(Dev d, int j_in_chunk, uint8_t *__restrict__ mask, int pass)
{
    __shared__ double red[8];
    const OpDev &op = d.K;
    T *__restrict__ y = (T *)d.y;
    T *__restrict__ ya = (T *)d.yavg;
    const T *__restrict__ y0 = (const T *)d.y0;
    const T *__restrict__ q = (const T *)d.q;
    const T *__restrict__ xb = (const T *)d.xbar;
    const int cnt = d.act_cnt[0];
    const bool full = cnt == op.nblk;
    for_each_item_split(cnt, d.remap, d.act_split, j_in_chunk & 1, [&](int it) {
        const int lb = full ? it : d.actK[it];
        const Seg s = block_seg(op, lb);
        if (SL == 1 && !s.sliced) return;
        const InstState *st = d.st + s.inst;
        const double sigma = st->sigma;
        const double w = AVG ? 1.0 / (double)(st->t_inner + j_in_chunk + 1) : 0.0;
        const bool ineq = s.ineq != 0;
        const int bi = lb - s.blk0;
        dispatch_lanes<RM>(s.lanes_log2, [&](auto tag, auto rtag) {
            constexpr int L = decltype(tag)::value, R = decltype(rtag)::value;
            if constexpr (SL == 1) {
                slice_partial<L, R>(op, s, bi, xb, red, pass);
                return;
            }
            using RS = RowSweep<L, 1, T, T, R, false, true, SL == 2>;
            const typename RS::Pos ps = RS::locate(s, bi);
            T r_y[R], r_q[R], r_a[R], r_0[R];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int64_t ii = r < ps.nvalid ? ps.row0 + r : ps.blk_row0;
                r_y[r] = y[ii];
                r_q[r] = q[ii];
                r_a[r] = AVG ? ya[ii] : T(0);
                r_0[r] = AVG ? y0[ii] : T(0);
            }
            double acc[R][1];
            RS::dot(op, ps, xb, nullptr, nullptr, red, acc, op.sb, s.sliced ? op.slices : 1, s.sliced ? pass : 0);
            if (ps.leader) {
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    if (r >= ps.nvalid) break;
                    const int64_t i = ps.row0 + r;
                    const double a = (SL == 2 && s.sliced) ? op.part[i] + acc[r][0] : acc[r][0];
                    const double yo = (double)r_y[r], qi = (double)r_q[r], yav = (double)r_a[r];
                    const double wv = yo + sigma * (qi - a);
                    const double yn = (ineq && wv < 0.0) ? 0.0 : wv;
                    const T ynT = (T)yn;
                    y[i] = ynT;
                    if (AVG) ya[i] = (T)(yav + (((double)ynT - (double)r_0[r]) - yav) * w);
                    if (MASK) mask[i] = (uint8_t)((!ineq || wv > 0.0) ? 1 : 0);
                }
            }
        });
    });
}

// ---------------------------------------------------------------------------
// adaptive step size (Section 2.4.4, Algorithm 5)
//
// One attempt = k_primal_ad, k_dual_ad, k_step_ad.  The sweeps read the
// instance's current buffer `par` and write the candidate into the other one:
//   x' = clip(x - (eta/omega)(c~ - K~^T y)),  a = K~ x' (FP64 sums),
//   K~ xbar = 2a - K~ x  (K~ x is cached per buffer: kx0 / kx1),
//   y' = proj_Y(y + eta omega (q~ - K~ xbar)),  K~ (x' - x) = a - K~ x,
// together with the step-weighted averages of the candidate,
//   zavg' = zavg + (z' - zavg) eta / (eta_sum + eta),
// and per-block FP64 sums of ||x'-x||^2, ||y'-y||^2 and (y'-y)'K~(x'-x).  The
// step kernel reduces them per instance, forms etabar and eta' and accepts the
// candidate (flips `par`) when eta <= etabar; a rejected candidate is simply
// overwritten by the next attempt.  Before each check k_commit_ad moves every
// instance's current buffer to buffer 0, so the check, the restart and the
// solution readers see the usual layout.
// ---------------------------------------------------------------------------

template <typename T, int RM>
__global__ __launch_bounds__(WG) void k_primal_ad(Dev d)
{
    __shared__ double red[8];
    __shared__ double lds[4];
    const OpDev &op = d.Kt;
    const T *__restrict__ c = (const T *)d.c;
    const T *__restrict__ l = (const T *)d.l;
    const T *__restrict__ u = (const T *)d.u;
    const int cnt = d.act_cnt[1];
    const bool full = cnt == op.nblk;
    for_each_item_split(cnt, d.remap, d.act_split + 9, 0, [&](int it) {
        const int lb = full ? it : d.actT[it];
        const Seg s = block_seg(op, lb);
        const InstState *st = d.st + s.inst;
        // the state is uniform per block: keep it (and the pointers the buffer
        // flag selects) in scalar registers
        const int par = uniform_i(st->par);
        const double eta = uniform_d(st->eta_try), esum = uniform_d(st->eta_sum);
        const double tau = uniform_d(eta / uniform_d(st->omega));
        const bool first = !(esum > 0.0);
        const double wa = uniform_d(eta / (esum + eta));
        const T *__restrict__ x = (const T *)(par ? d.xbar : d.x);
        T *__restrict__ xn = (T *)(par ? d.x : d.xbar);
        const T *__restrict__ xa = (const T *)(par ? d.xavg1 : d.xavg);
        T *__restrict__ xan = (T *)(par ? d.xavg : d.xavg1);
        const T *__restrict__ x0 = (const T *)d.x0;
        const T *__restrict__ y = (const T *)(par ? d.y1 : d.y);
        const int bi = lb - s.blk0;
        double part[1] = {0.0};
        dispatch_lanes<RM>(s.lanes_log2, [&](auto tag, auto rtag) {
            constexpr int L = decltype(tag)::value, R = decltype(rtag)::value;
            using RS = RowSweep<L, 1, T, T, R>;
            const typename RS::Pos ps = RS::locate(s, bi);
            // rows are < 2^29: 32-bit offsets from the scalar bases
            T r_x[R], r_c[R], r_l[R], r_u[R], r_a[R], r_0[R];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const uint32_t jj = (uint32_t)(r < ps.nvalid ? ps.row0 + r : ps.blk_row0);
                r_x[r] = ldo(x, jj);
                r_c[r] = ldo(c, jj);
                r_l[r] = ldo(l, jj);
                r_u[r] = ldo(u, jj);
                r_a[r] = ldo(xa, jj);
                r_0[r] = ldo(x0, jj);
            }
            double acc[R][1];
            RS::dot(op, ps, y, nullptr, nullptr, red, acc);
            if (ps.leader) {
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    if (r >= ps.nvalid) break;
                    const uint32_t j = (uint32_t)(ps.row0 + r);
                    const double xo = (double)r_x[r], cj = (double)r_c[r], lo = (double)r_l[r];
                    const double hi = (double)r_u[r], xav = (double)r_a[r];
                    const double v = xo - tau * (cj - acc[r][0]);
                    const double xv = v < lo ? lo : (v > hi ? hi : v);
                    const T xnT = (T)xv;
                    sto(xn, j, xnT);
                    const double off = (double)xnT - (double)r_0[r];
                    sto(xan, j, (T)(first ? off : xav + (off - xav) * wa));
                    const double dx = (double)xnT - xo;
                    part[0] += dx * dx;
                }
            }
        });
        block_sum<1>(part, lds);
        if (threadIdx.x == 0) d.adp[2 * (size_t)d.K.nblk + lb] = part[0];
    });
}

// SL: the column-slice role of the launch, as for k_dual (the partial passes
// write the sliced rows' FP64 partials of K~ x'; the last pass completes
// them and does everything else, the per-block sums included).
template <typename T, int RM, int SL>
__global__ __launch_bounds__(WG) void k_dual_ad(Dev d, int pass)
{
    __shared__ double red[8];
    __shared__ double lds[8];
    const OpDev &op = d.K;
    const T *__restrict__ q = (const T *)d.q;
    const int cnt = d.act_cnt[0];
    const bool full = cnt == op.nblk;
    for_each_item_split(cnt, d.remap, d.act_split, 0, [&](int it) {
        const int lb = full ? it : d.actK[it];
        const Seg s = block_seg(op, lb);
        if (SL == 1 && !s.sliced) return;
        const InstState *st = d.st + s.inst;
        const int par = uniform_i(st->par);
        const double eta = uniform_d(st->eta_try), esum = uniform_d(st->eta_sum);
        const double sigma = uniform_d(eta * uniform_d(st->omega));
        const bool first = !(esum > 0.0);
        const double wa = uniform_d(eta / (esum + eta));
        const T *__restrict__ xc = (const T *)(par ? d.x : d.xbar);  // candidate x'
        const T *__restrict__ y = (const T *)(par ? d.y1 : d.y);
        T *__restrict__ yn = (T *)(par ? d.y : d.y1);
        const T *__restrict__ ya = (const T *)(par ? d.yavg1 : d.yavg);
        T *__restrict__ yan = (T *)(par ? d.yavg : d.yavg1);
        const T *__restrict__ y0 = (const T *)d.y0;
        const double *__restrict__ kx = par ? d.kx1 : d.kx0;
        double *__restrict__ kxn = par ? d.kx0 : d.kx1;
        const bool ineq = s.ineq != 0;
        const int bi = lb - s.blk0;
        if constexpr (SL == 1) {
            dispatch_lanes<RM>(s.lanes_log2, [&](auto tag, auto rtag) {
                slice_partial<decltype(tag)::value, decltype(rtag)::value>(op, s, bi, xc, red, pass);
            });
            return;
        }
        double part[2] = {0.0, 0.0};
        dispatch_lanes<RM>(s.lanes_log2, [&](auto tag, auto rtag) {
            constexpr int L = decltype(tag)::value, R = decltype(rtag)::value;
            using RS = RowSweep<L, 1, T, T, R, false, true, SL == 2>;
            const typename RS::Pos ps = RS::locate(s, bi);
            T r_y[R], r_q[R], r_a[R], r_0[R];
            double r_k[R];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const uint32_t ii = (uint32_t)(r < ps.nvalid ? ps.row0 + r : ps.blk_row0);
                r_y[r] = ldo(y, ii);
                r_q[r] = ldo(q, ii);
                r_a[r] = ldo(ya, ii);
                r_0[r] = ldo(y0, ii);
                r_k[r] = ldo(kx, ii);
            }
            double acc[R][1];
            RS::dot(op, ps, xc, nullptr, nullptr, red, acc, op.sb, s.sliced ? op.slices : 1, s.sliced ? pass : 0);
            if (ps.leader) {
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    if (r >= ps.nvalid) break;
                    const uint32_t i = (uint32_t)(ps.row0 + r);
                    const double a = (SL == 2 && s.sliced) ? op.part[i] + acc[r][0] : acc[r][0];
                    const double kxo = r_k[r];
                    const double yo = (double)r_y[r], qi = (double)r_q[r], yav = (double)r_a[r];
                    const double wv = yo + sigma * (qi - (2.0 * a - kxo));
                    const double yv = (ineq && wv < 0.0) ? 0.0 : wv;
                    const T ynT = (T)yv;
                    sto(yn, i, ynT);
                    sto(kxn, i, a);
                    const double off = (double)ynT - (double)r_0[r];
                    sto(yan, i, (T)(first ? off : yav + (off - yav) * wa));
                    const double dy = (double)ynT - yo;
                    part[0] += dy * dy;
                    part[1] += dy * (a - kxo);
                }
            }
        });
        block_sum<2>(part, lds);
        if (threadIdx.x == 0) {
            d.adp[2 * (size_t)lb] = part[0];
            d.adp[2 * (size_t)lb + 1] = part[1];
        }
    });
}

// One 1024-lane workgroup per instance: the accept / reject decision of the
// attempt.  The per-block sums are read 8 per lane in flight (the kernel is
// bound by the latency of these loads), then reduced in a fixed order.
// k counts the attempts of the solve including this one.
constexpr int STEP_WG = 1024;
constexpr int STEP_U = 8;

__global__ __launch_bounds__(STEP_WG) void k_step_ad(Dev d)
{
    __shared__ double lds[3 * (STEP_WG / 64)];
    const int b = blockIdx.x;
    InstState &st = d.st[b];
    if (st.done) return;
    const InstInfo in = d.info[b];
    const int nT = in.blkT1 - in.blkT0, nK = in.blkK1 - in.blkK0;
    const double *pT = d.adp + 2 * (size_t)d.K.nblk + in.blkT0;
    const double *pK = d.adp + 2 * (size_t)in.blkK0;
    const int tid = threadIdx.x;
    double v[3] = {0.0, 0.0, 0.0};
    for (int r0 = tid; r0 < nT; r0 += STEP_U * STEP_WG) {
        double a[STEP_U];
#pragma unroll
        for (int k = 0; k < STEP_U; ++k) {
            const int r = r0 + k * STEP_WG;
            a[k] = r < nT ? pT[r] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < STEP_U; ++k) v[0] += a[k];
    }
    for (int r0 = tid; r0 < nK; r0 += STEP_U * STEP_WG) {
        double a[STEP_U], c[STEP_U];
#pragma unroll
        for (int k = 0; k < STEP_U; ++k) {
            const int r = r0 + k * STEP_WG;
            a[k] = r < nK ? pK[2 * r] : 0.0;
            c[k] = r < nK ? pK[2 * r + 1] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < STEP_U; ++k) {
            v[1] += a[k];
            v[2] += c[k];
        }
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) v[k] = group_reduce<64, false>(v[k]);
    const int wave = tid >> 6;
    if ((tid & 63) == 0) {
#pragma unroll
        for (int k = 0; k < 3; ++k) lds[k * (STEP_WG / 64) + wave] = v[k];
    }
    __syncthreads();
    if (tid != 0) return;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        double t = 0.0;
        for (int w = 0; w < STEP_WG / 64; ++w) t += lds[k * (STEP_WG / 64) + w];
        v[k] = t;
    }
    const double w = st.omega, eta = st.eta_try;
    const long long k = st.k_att + 1;
    const double den = fabs(2.0 * v[2]);
    const double etabar = den > 0.0 ? (w * v[0] + v[1] / w) / den : INFINITY;
    const double kk = (double)k + 1.0;
    const double shrink = (1.0 - pow(kk, -0.3)) * etabar;
    const double grow = (1.0 + pow(kk, -0.6)) * eta;
    st.k_att = k;
    st.prev_ok = eta <= etabar;
    if (eta <= etabar) {
        st.par ^= 1;
        st.eta_sum += eta;
        st.n_acc += 1;
    }
    st.eta_try = shrink < grow ? shrink : grow;
}

// Before a check: every running instance's current iterate, its average and
// K~ x move to buffer 0 (the iterates are swapped, so buffer 1 then holds the
// iterate before the last accepted step).  An epoch without an accepted step
// has no average: the average is set to the iterate.  (k_control then resets
// par.)
template <typename T>
__global__ __launch_bounds__(WG) void k_commit_ad(Dev d)
{
    const int nT = d.act_cnt[1], nK = d.act_cnt[0];
    const bool fullK = nK == d.K.nblk, fullT = nT == d.Kt.nblk;
    for_each_item(nT + nK, d.remap, [&](int it) {
        const bool onT = it < nT;
        const int lb = onT ? (fullT ? it : d.actT[it]) : (fullK ? it - nT : d.actK[it - nT]);
        const OpDev &op = onT ? d.Kt : d.K;
        const Seg s = block_seg(op, lb);
        const InstState &st = d.st[s.inst];
        const bool flip = st.par != 0, noavg = !(st.eta_sum > 0.0);
        if (!flip && !noavg) return;
        T *z0 = (T *)(onT ? d.x : d.y);
        const T *z1 = (const T *)(onT ? d.xbar : d.y1);
        T *za0 = (T *)(onT ? d.xavg : d.yavg);
        const T *za1 = (const T *)(onT ? d.xavg1 : d.yavg1);
        const T *ze = (const T *)(onT ? d.x0 : d.y0);  // epoch start
        const int64_t r1 = s.row0 + s.nrows;
        T *z1w = (T *)z1;
        for (int64_t r = s.row0 + threadIdx.x; r < r1; r += WG) {
            const T v = flip ? z1[r] : z0[r];
            if (flip) {
                // swap: buffer 1 keeps the iterate before the last accepted step
                z1w[r] = z0[r];
                z0[r] = v;
            }
            // averages are offsets from the epoch start
            za0[r] = noavg ? (T)((double)v - (double)ze[r]) : za1[r];
            if (!onT && flip) d.kx0[r] = d.kx1[r];
        }
    });
}

// kx0 = K~ x (buffer 0) with the sweep's own values and summation, for every
// running instance (all = 1: solve start) or those that just restarted.
template <typename T, int RM>
__global__ __launch_bounds__(WG) void k_kx_ad(Dev d, int all)
{
    __shared__ double red[8];
    const OpDev &op = d.K;
    const T *__restrict__ x = (const T *)d.x;
    const int cnt = d.act_cnt[0];
    const bool full = cnt == op.nblk;
    for_each_item(cnt, d.remap, [&](int it) {
        const int lb = full ? it : d.actK[it];
        const Seg s = block_seg(op, lb);
        if (!all && !d.st[s.inst].restart) return;
        const int bi = lb - s.blk0;
        dispatch_lanes<RM>(s.lanes_log2, [&](auto tag, auto rtag) {
            constexpr int L = decltype(tag)::value, R = decltype(rtag)::value;
            using RS = RowSweep<L, 1, T, T, R>;
            const typename RS::Pos ps = RS::locate(s, bi);
            double acc[R][1];
            RS::dot(op, ps, x, nullptr, nullptr, red, acc);
            if (ps.leader) {
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    if (r >= ps.nvalid) break;
                    d.kx0[ps.row0 + r] = acc[r][0];
                }
            }
        });
    });
}

// ---------------------------------------------------------------------------
// check: per-workgroup FP64 partial sums for NC candidates
//   K rows i   : s0 += e^2 (e = q~ - K~x, clipped at 0 on ">=" rows),
//                s1 += (e / rho_i)^2, s2 += q~_i y_i, s3 += (y_i - y0_i)^2
//   K^T rows j : d = c~_j - (K~^T y)_j, lambda = proj_Lambda(d), rd = d - lambda,
//                s4 += rd^2, s5 += (rd / kap_j)^2, s6 += c~_j x_j,
//                s7 += l~_j lambda^+ + u~_j lambda^-, s8 += (x_j - x0_j)^2
// Scaled residual e relates to the original one by e = rho_i (q - Kx)_i, and
// rd = kap_j (c - K^T y - lambda)_j; objective terms are scale invariant.
// ---------------------------------------------------------------------------

__device__ __forceinline__ double proj_lambda(double v, double l, double u)
{
    const bool lf = isfinite(l), uf = isfinite(u);
    if (!lf && !uf) return 0.0;
    if (!lf) return v < 0.0 ? v : 0.0;
    if (!uf) return v > 0.0 ? v : 0.0;
    return v;
}

// The solve-time check with K in column slices (K.slices = S > 1): passes
// 0 .. S-2 of the products K~ x of its NC candidates over the sliced rows of
// K, into FP64 partials (candidate a at K.part + a M); k_check<..., true>
// adds the last slice.
template <typename V, int NC, int RM>
__global__ __launch_bounds__(WG) void k_check_part(Dev d, const V *__restrict__ xa0, const V *__restrict__ xa1,
                                                   int pass)
{
    __shared__ double red[NC * 4];
    const OpDev &op = d.K;
    const int nK = d.act_cnt[0];
    const bool fullK = nK == op.nblk;
    for_each_item(nK, d.remap, [&](int it) {
        const int lb = fullK ? it : d.actK[it];
        const Seg s = block_seg(op, lb);
        if (!s.sliced) return;
        const int bi = lb - s.blk0;
        dispatch_lanes<RM>(s.lanes_log2, [&](auto tag, auto rtag) {
            constexpr int L = decltype(tag)::value, R = decltype(rtag)::value;
            using RS = RowSweep<L, NC, double, V, R, false, true, true>;
            const typename RS::Pos ps = RS::locate(s, bi);
            double acc[R][NC];
            RS::dot(op, ps, xa0, xa1, nullptr, red, acc, op.sb, op.slices, pass);
            if (ps.leader) {
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    if (r >= ps.nvalid) break;
                    const int64_t i = ps.row0 + r;
#pragma unroll
                    for (int a = 0; a < NC; ++a) {
                        double *pa = op.part + (size_t)a * d.M;
                        pa[i] = pass > 0 ? pa[i] + acc[r][a] : acc[r][a];
                    }
                }
            }
        });
    });
}

// use_list: walk the active lists (solve); otherwise every block (caller KKT).
// SLC: K's sliced rows add their last slice to k_check_part's partials.
template <typename V, int NC, int RM, bool SLC = false>
__global__ __launch_bounds__(WG) void k_check(Dev d, const V *__restrict__ xa0, const V *__restrict__ xa1,
                                              const V *__restrict__ ya0, const V *__restrict__ ya1,
                                              const V *__restrict__ xs, const V *__restrict__ ys,
                                              int use_list)
{
    __shared__ double red[NCAND * NSUM * 4];
    const int nK = use_list ? d.act_cnt[0] : d.K.nblk;
    const int nT = use_list ? d.act_cnt[1] : d.Kt.nblk;
    const bool fullK = nK == d.K.nblk, fullT = nT == d.Kt.nblk;
    for_each_item(nK + nT, d.remap, [&](int it) {
        const bool onK = it < nK;
        const int lb = onK ? (fullK ? it : d.actK[it]) : (fullT ? it - nK : d.actT[it - nK]);
        const int lbc = onK ? lb : d.K.nblk + lb;
        const OpDev &op = onK ? d.K : d.Kt;
        const Seg s = block_seg(op, lb);
        const int bi = lb - s.blk0;
        const bool ineq = s.ineq != 0;
        double *out = d.partials + (size_t)lbc * NPART;
        // each operator keeps only its own sums live (4 per candidate on K,
        // 5 on K^T): half the registers of one 18-sum set, twice the waves
        if (onK) {
            double sum[NC * 4];
#pragma unroll
            for (int k = 0; k < NC * 4; ++k) sum[k] = 0.0;
            dispatch_lanes<RM>(s.lanes_log2, [&](auto tag, auto rtag) {
                constexpr int L = decltype(tag)::value, R = decltype(rtag)::value;
                auto row_terms = [&](int64_t r, const double *acc) {
                    const double qi = d.q64[r], rh = d.rho[r];
#pragma unroll
                    for (int a = 0; a < NC; ++a) {
                        double e = qi - acc[a];
                        if (ineq && e < 0.0) e = 0.0;
                        const double eu = e / rh;
                        const double ya = (double)(a == 0 ? ya0 : ya1)[r];
                        const double dy = ya - (double)ys[r];
                        sum[a * 4 + 0] += e * e;
                        sum[a * 4 + 1] += eu * eu;
                        sum[a * 4 + 2] += qi * ya;
                        sum[a * 4 + 3] += dy * dy;
                    }
                };
                if (SLC && s.sliced) {
                    using RS = RowSweep<L, NC, double, V, R, false, true, true>;
                    const typename RS::Pos ps = RS::locate(s, bi);
                    double acc[R][NC];
                    RS::dot(op, ps, xa0, xa1, nullptr, red, acc, op.sb, op.slices, op.slices - 1);
                    if (ps.leader) {
#pragma unroll
                        for (int r = 0; r < R; ++r) {
                            if (r >= ps.nvalid) break;
                            const int64_t i = ps.row0 + r;
                            double tot[NC];
#pragma unroll
                            for (int a = 0; a < NC; ++a) tot[a] = op.part[(size_t)a * d.M + i] + acc[r][a];
                            row_terms(i, tot);
                        }
                    }
                } else {
                    sweep_rows<L, NC, double, V, R>(op, s, bi, xa0, xa1, nullptr, red, row_terms);
                }
            });
            block_sum<NC * 4>(sum, red);
            if (threadIdx.x == 0) {
#pragma unroll
                for (int k = 0; k < NCAND * NSUM; ++k) {
                    const int a = k / NSUM, j = k % NSUM;
                    out[k] = (a < NC && j < 4) ? sum[a * 4 + j] : 0.0;
                }
            }
        } else {
            double sum[NC * 5];
#pragma unroll
            for (int k = 0; k < NC * 5; ++k) sum[k] = 0.0;
            dispatch_lanes<RM>(s.lanes_log2, [&](auto tag, auto rtag) {
                constexpr int L = decltype(tag)::value, R = decltype(rtag)::value;
                sweep_rows<L, NC, double, V, R>(op, s, bi, ya0, ya1, nullptr, red, [&](int64_t r, const double *acc) {
                    const double cj = d.c64[r], lj = d.l64[r], uj = d.u64[r], kj = d.kap[r];
#pragma unroll
                    for (int a = 0; a < NC; ++a) {
                        const double dd = cj - acc[a];
                        const double lam = proj_lambda(dd, lj, uj);
                        const double rd = dd - lam;
                        const double rdu = rd / kj;
                        const double xv = (double)(a == 0 ? xa0 : xa1)[r];
                        const double dx = xv - (double)xs[r];
                        sum[a * 5 + 0] += rd * rd;
                        sum[a * 5 + 1] += rdu * rdu;
                        sum[a * 5 + 2] += cj * xv;
                        sum[a * 5 + 3] += lam > 0.0 ? lj * lam : (lam < 0.0 ? uj * lam : 0.0);
                        sum[a * 5 + 4] += dx * dx;
                    }
                });
            });
            block_sum<NC * 5>(sum, red);
            if (threadIdx.x == 0) {
#pragma unroll
                for (int k = 0; k < NCAND * NSUM; ++k) {
                    const int a = k / NSUM, j = k % NSUM;
                    out[k] = (a < NC && j >= 4) ? sum[a * 5 + (j - 4)] : 0.0;
                }
            }
        }
        __syncthreads();
    });
}

// ---------------------------------------------------------------------------
// infeasibility detection (Section 2.4.5, Algorithm 6): per-block terms of
// the tests on the last step's difference, in ORIGINAL variables
// (x = kap x~, y = rho y~, (K x)_i = (K~ x~)_i / rho_i,
// (c - K^T y)_j = (c~ - K~^T y~)_j / kap_j), FP64 matrix:
//   K rows i   : kd = (K dx)_i, dy_i
//                s0 += kd^2 ("=" rows), s1 = max(-kd) (">=" rows),
//                s2 = max(-dy_i) (">=" rows), s3 += q_i dy_i
//   K^T rows j : dx_j, dlambda_j = lambda_j(y) - lambda_j(yp) with
//                lambda = proj_Lambda(c - K^T y), r = (K^T dy)_j + dlambda_j,
//                s4 += c_j dx_j, s5 = max violation of dx_j in V_j,
//                s6 += r^2, s7 += l_j dlambda^+ + u_j dlambda^- (-inf when an
//                infinite bound meets a nonzero multiplier)
// (x, y) is the current iterate, (xp, yp) the one before the last step.
// ---------------------------------------------------------------------------
template <typename V, int RM>
__global__ __launch_bounds__(WG) void k_infeas(Dev d, const V *__restrict__ xp, const V *__restrict__ yp)
{
    __shared__ double red[2 * 4];
    __shared__ double lds[NINF * 4];
    const V *__restrict__ x = (const V *)d.x;
    const V *__restrict__ y = (const V *)d.y;
    const int nK = d.act_cnt[0], nT = d.act_cnt[1];
    const bool fullK = nK == d.K.nblk, fullT = nT == d.Kt.nblk;
    for_each_item(nK + nT, d.remap, [&](int it) {
        const bool onK = it < nK;
        const int lb = onK ? (fullK ? it : d.actK[it]) : (fullT ? it - nK : d.actT[it - nK]);
        const int lbc = onK ? lb : d.K.nblk + lb;
        const OpDev &op = onK ? d.K : d.Kt;
        const Seg s = block_seg(op, lb);
        double f[NINF];
#pragma unroll
        for (int k = 0; k < NINF; ++k) f[k] = (k == 1 || k == 2 || k == 5) ? -INFINITY : 0.0;
        const int bi = lb - s.blk0;
        const bool ineq = s.ineq != 0;
        dispatch_lanes<RM>(s.lanes_log2, [&](auto tag, auto rtag) {
            constexpr int L = decltype(tag)::value, R = decltype(rtag)::value;
            if (onK) {
                sweep_rows<L, 2, double, V, R>(op, s, bi, x, xp, nullptr, red, [&](int64_t r, const double *acc) {
                    const double rh = d.rho[r];
                    const double kd = (acc[0] - acc[1]) / rh;
                    const double dy = rh * ((double)y[r] - (double)yp[r]);
                    if (ineq) {
                        f[1] = fmax(f[1], -kd);
                        f[2] = fmax(f[2], -dy);
                    } else {
                        f[0] += kd * kd;
                    }
                    f[3] += d.qraw[r] * dy;
                });
            } else {
                sweep_rows<L, 2, double, V, R>(op, s, bi, y, yp, nullptr, red, [&](int64_t r, const double *acc) {
                    const double cj = d.c64[r], kj = d.kap[r];
                    const double ls = d.l64[r], us = d.u64[r];
                    const double dl = (proj_lambda(cj - acc[0], ls, us) - proj_lambda(cj - acc[1], ls, us)) / kj;
                    const double res = (acc[0] - acc[1]) / kj + dl;
                    const double dx = kj * ((double)x[r] - (double)xp[r]);
                    const double lo = d.lraw[r], hi = d.uraw[r];
                    const bool lf = isfinite(lo), uf = isfinite(hi);
                    f[4] += d.craw[r] * dx;
                    const double v = (lf && uf) ? fabs(dx) : (lf ? -dx : (uf ? dx : 0.0));
                    f[5] = fmax(f[5], v);
                    f[6] += res * res;
                    if (dl > 0.0) f[7] += lf ? lo * dl : -INFINITY;
                    else if (dl < 0.0) f[7] += uf ? hi * dl : -INFINITY;
                });
            }
        });
#pragma unroll
        for (int k = 0; k < NINF; ++k)
            f[k] = (k == 1 || k == 2 || k == 5) ? group_reduce<64, true>(f[k]) : group_reduce<64, false>(f[k]);
        const int tid = threadIdx.x, wave = tid >> 6;
        __syncthreads();
        if ((tid & 63) == 0) {
#pragma unroll
            for (int k = 0; k < NINF; ++k) lds[k * 4 + wave] = f[k];
        }
        __syncthreads();
        if (tid == 0) {
            double *out = d.partials + (size_t)lbc * NPART + NCAND * NSUM;
#pragma unroll
            for (int k = 0; k < NINF; ++k) {
                const double *q = lds + k * 4;
                out[k] = (k == 1 || k == 2 || k == 5) ? fmax(fmax(q[0], q[1]), fmax(q[2], q[3]))
                                                      : (q[0] + q[1]) + (q[2] + q[3]);
            }
        }
    });
}

// Fixed steps: the iterate before the last step of a check period, saved to
// (xavg1, y1) for the infeasibility tests.  Walks the running instances' rows.
template <typename T>
__global__ __launch_bounds__(WG) void k_save_prev(Dev d)
{
    const int nT = d.act_cnt[1], nK = d.act_cnt[0];
    const bool fullK = nK == d.K.nblk, fullT = nT == d.Kt.nblk;
    for_each_item(nT + nK, d.remap, [&](int it) {
        const bool onT = it < nT;
        const int lb = onT ? (fullT ? it : d.actT[it]) : (fullK ? it - nT : d.actK[it - nT]);
        const Seg s = block_seg(onT ? d.Kt : d.K, lb);
        const T *src = (const T *)(onT ? d.x : d.y);
        T *dst = (T *)(onT ? d.xavg1 : d.y1);
        const int64_t r1 = s.row0 + s.nrows;
        for (int64_t r = s.row0 + threadIdx.x; r < r1; r += WG) dst[r] = src[r];
    });
}

// Block-wide reduction of the NPART per-thread partials (sums, and maxima in
// the part_is_max slots), fixed order; result valid in thread 0.
__device__ __forceinline__ void block_reduce_part(double (&v)[NPART], double *lds)
{
#pragma unroll
    for (int k = 0; k < NPART; ++k)
        v[k] = part_is_max(k) ? group_reduce<64, true>(v[k]) : group_reduce<64, false>(v[k]);
    const int tid = threadIdx.x, wave = tid >> 6;
    __syncthreads();
    if ((tid & 63) == 0) {
#pragma unroll
        for (int k = 0; k < NPART; ++k) lds[k * 4 + wave] = v[k];
    }
    __syncthreads();
    if (tid == 0) {
#pragma unroll
        for (int k = 0; k < NPART; ++k) {
            const double *r = lds + k * 4;
            v[k] = part_is_max(k) ? fmax(fmax(r[0], r[1]), fmax(r[2], r[3])) : (r[0] + r[1]) + (r[2] + r[3]);
        }
    }
}

__device__ __forceinline__ void part_init(double (&v)[NPART])
{
#pragma unroll
    for (int k = 0; k < NPART; ++k) v[k] = part_is_max(k) ? -INFINITY : 0.0;
}

__device__ __forceinline__ void part_acc(double (&v)[NPART], const double *p)
{
#pragma unroll
    for (int k = 0; k < NPART; ++k) v[k] = part_is_max(k) ? fmax(v[k], p[k]) : v[k] + p[k];
}

// Second level of the check reduction: block t reduces up to L2CH consecutive
// first-level rows of its instance (K blocks first, then K^T blocks), in a
// fixed order, so the totals of one instance do not depend on the batch.
__global__ __launch_bounds__(WG) void k_reduce_l2(Dev d, int skip_done)
{
    __shared__ double lds[NPART * 4];
    const int t = blockIdx.x;
    const int b = d.l2_inst[t];
    if (skip_done && d.st[b].done) return;
    const InstInfo in = d.info[b];
    const int nK = in.blkK1 - in.blkK0, nT = in.blkT1 - in.blkT0;
    const int r0 = (t - in.l2off) * L2CH;
    const int r1 = min(r0 + L2CH, nK + nT);
    double v[NPART];
    part_init(v);
    for (int r = r0 + (int)threadIdx.x; r < r1; r += WG) {
        const int lbc = r < nK ? in.blkK0 + r : d.K.nblk + in.blkT0 + (r - nK);
        part_acc(v, d.partials + (size_t)lbc * NPART);
    }
    block_reduce_part(v, lds);
    if (threadIdx.x == 0) {
        double *o = d.partials2 + (size_t)t * NPART;
#pragma unroll
        for (int k = 0; k < NPART; ++k) o[k] = v[k];
    }
}

// Reduces the instance's second-level rows (fixed order) into tot[NPART].
__device__ void reduce_instance(const Dev &d, const InstInfo &in, double *tot)
{
    __shared__ double lds[NPART * 4];
    double v[NPART];
    part_init(v);
    for (int t = threadIdx.x; t < in.l2cnt; t += WG) part_acc(v, d.partials2 + (size_t)(in.l2off + t) * NPART);
    block_reduce_part(v, lds);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NPART; ++k) tot[k] = v[k];
    }
}

struct Metrics {
    double kkt[9];   // original-LP terms (pdhg_kkt_out order)
    double kw_parts[3];  // scaled pres^2, scaled dres^2, gap^2
};

__device__ void metrics_from_sums(const double *s, const InstInfo &in, Metrics &m)
{
    const double pres = sqrt(s[1]), dres = sqrt(s[5]);
    const double pobj = s[6], dobj = s[2] + s[7];
    const double gap = fabs(dobj - pobj);
    m.kkt[0] = pres;
    m.kkt[1] = dres;
    m.kkt[2] = pobj;
    m.kkt[3] = dobj;
    m.kkt[4] = gap;
    m.kkt[5] = pres / (1.0 + in.qnorm);
    m.kkt[6] = dres / (1.0 + in.cnorm);
    m.kkt[7] = gap / (1.0 + fabs(dobj) + fabs(pobj));
    m.kkt[8] = fmax(m.kkt[7], fmax(m.kkt[5], m.kkt[6]));
    m.kw_parts[0] = s[0];
    m.kw_parts[1] = s[4];
    m.kw_parts[2] = gap * gap;
}

// KKT error in the omega-weighted form of Section 2.4.2.
__device__ __forceinline__ double kkt_omega(const Metrics &m, double w)
{
    return sqrt(w * w * m.kw_parts[0] + m.kw_parts[1] / (w * w) + m.kw_parts[2]);
}

// The inputs of one check's restart decision, as they were before it.
struct CheckIn {
    long long t_inner;
    double kkt0, kkt_prev, omega;
};

// Record of one check in the instance's ring (when the handle keeps one).
__device__ void trace_put(const Dev &d, int b, InstState &st, int cand, double kwc, const Metrics *mt, int nc,
                          const CtlParams &P, const CheckIn &ci, double dx = 0.0, double dy = 0.0)
{
    if (d.trace_cap <= 0) return;
    pdhg_trace_rec r;
    r.iter = st.k_total;
    r.restarted = st.restart;
    r.cand_avg = cand;
    r.kkt_cand = kwc;
    r.omega = st.omega;
    r.rel_kkt_cur = mt[0].kkt[8];
    r.rel_kkt_avg = nc > 1 ? mt[1].kkt[8] : INFINITY;
    r.eta_next = P.adaptive ? st.eta_try : st.eta;
    r.accepted = P.adaptive ? st.n_acc : st.k_total;
    r.t_inner = ci.t_inner;
    r.kkt0 = ci.kkt0;
    r.kkt_prev = ci.kkt_prev;
    r.omega_before = ci.omega;
    r.delta_x = dx;
    r.delta_y = dy;
    r.kkt0_next = st.kkt0;
    r.cand_pres = sqrt(mt[cand].kw_parts[0]);
    r.cand_dres = sqrt(mt[cand].kw_parts[1]);
    r.cand_gap = sqrt(mt[cand].kw_parts[2]);
    d.trace[(size_t)b * d.trace_cap + (size_t)(st.ntrace % d.trace_cap)] = r;
    st.ntrace += 1;
}

// One workgroup per instance.  iters_done: iterations since the last check
// (0 for the check of the starting point).
__global__ __launch_bounds__(WG) void k_control(Dev d, CtlParams P, int iters_done)
{
    __shared__ double tot[NPART];
    const int b = blockIdx.x;
    InstState &st = d.st[b];
    if (st.done) return;
    const InstInfo in = d.info[b];
    reduce_instance(d, in, tot);
    if (threadIdx.x != 0) return;
    if (P.adaptive) st.par = 0;  // k_commit_ad moved the current iterate to buffer 0

    st.k_total += iters_done;
    st.t_inner += iters_done;
    const int nc = P.use_restarts ? 2 : 1;
    Metrics mt[2];
    bool finite = true;
    for (int a = 0; a < nc; ++a) {
        metrics_from_sums(tot + a * NSUM, in, mt[a]);
        for (int k = 0; k < NSUM; ++k) finite = finite && isfinite(tot[a * NSUM + k]);
    }
    const double omega = st.omega;
    const double kw0 = kkt_omega(mt[0], omega);
    const CheckIn ci = {st.t_inner, st.kkt0, st.kkt_prev, omega};
    st.restart = 0;
    if (!finite) {
        st.done = 1;
        st.status = PDHG_NUMERICAL_ERROR;
        st.sol_avg = 0;
        for (int k = 0; k < 9; ++k) st.kkt[k] = mt[0].kkt[k];
        if (iters_done > 0) trace_put(d, b, st, 0, kw0, mt, nc, P, ci);
        d.hdone[b] = 1;
        return;
    }
    if (iters_done == 0) {
        // starting point: termination test and the first epoch's reference value
        st.kkt0 = kw0;
        st.kkt_prev = INFINITY;
        st.cand_avg = 0;
        for (int k = 0; k < 9; ++k) st.kkt[k] = mt[0].kkt[k];
        if (mt[0].kkt[8] <= P.eps) {
            st.done = 1;
            st.status = PDHG_OPTIMAL;
            st.sol_avg = 0;
            d.hdone[b] = 1;
        }
        return;
    }
    const double kw1 = nc > 1 ? kkt_omega(mt[1], omega) : INFINITY;
    // restart candidate: the iterate when strictly better, else the average
    const int cand = (nc > 1 && !(kw0 < kw1)) ? 1 : 0;
    const double kwc = cand ? kw1 : kw0;
    st.cand_avg = cand;
    int stop = 0, sol = cand;
    if (mt[cand].kkt[8] <= P.eps) {
        stop = PDHG_OPTIMAL + 1;
    } else if (nc > 1 && mt[1 - cand].kkt[8] <= P.eps) {
        stop = PDHG_OPTIMAL + 1;
        sol = 1 - cand;
    } else if (P.detect && (!P.adaptive || st.prev_ok)) {
        // Algorithm 6 on the last step's difference; each test relative to
        // the ray's objective improvement (dual test first)
        const double *f = tot + NCAND * NSUM;
        const double tol = P.infeas_tol, sd = -f[4], sp = f[3] + f[7];
        if (sd > 0.0 && sqrt(f[0]) <= tol * sd && f[1] <= tol * sd && f[5] <= tol * sd) {
            stop = PDHG_DUAL_INFEASIBLE + 1;
            sol = 0;
        } else if (sp > 0.0 && sqrt(f[6]) <= tol * sp && f[2] <= tol * sp) {
            stop = PDHG_PRIMAL_INFEASIBLE + 1;
            sol = 0;
        }
    }
    if (!stop && st.k_total >= P.max_iters) stop = PDHG_ITERATION_LIMIT + 1;
    if (stop) {
        st.done = 1;
        st.status = stop - 1;
        st.sol_avg = sol;
        for (int k = 0; k < 9; ++k) st.kkt[k] = mt[sol].kkt[k];
        trace_put(d, b, st, cand, kwc, mt, nc, P, ci);
        d.hdone[b] = 1;
        return;
    }
    for (int k = 0; k < 9; ++k) st.kkt[k] = mt[cand].kkt[k];
    st.sol_avg = cand;
    if (!P.use_restarts) {
        trace_put(d, b, st, cand, kwc, mt, nc, P, ci);
        return;
    }
    const bool suff = kwc <= P.beta_suff * st.kkt0;
    const bool nec = kwc <= P.beta_nec * st.kkt0 && kwc > st.kkt_prev;
    const bool art = (double)st.t_inner > P.beta_art * (double)st.k_total;
    if (suff || nec || art) {
        const double dx = sqrt(tot[cand * NSUM + 8]), dy = sqrt(tot[cand * NSUM + 3]);
        double w = omega;
        if (P.use_pw && dx > P.eps_zero && dy > P.eps_zero) w = exp(0.5 * log(dy / dx) + 0.5 * log(omega));
        st.omega = w;
        st.tau = st.eta / w;
        st.sigma = st.eta * w;
        st.kkt0 = kkt_omega(mt[cand], w);
        st.kkt_prev = INFINITY;
        st.t_inner = 0;
        st.eta_sum = 0.0;
        st.restart = 1;
        st.nrestarts += 1;
        trace_put(d, b, st, cand, kwc, mt, nc, P, ci, dx, dy);
        return;
    }
    st.kkt_prev = kwc;
    trace_put(d, b, st, cand, kwc, mt, nc, P, ci);
}

// The average point of the running instances, x0 + xavg rounded to T, into
// (xam, yam): what the check evaluates and a restart copies.  Walks K^T blocks
// then K blocks of the running instances.
template <typename T>
__global__ __launch_bounds__(WG) void k_avg_point(Dev d)
{
    const int nT = d.act_cnt[1], nK = d.act_cnt[0];
    const bool fullK = nK == d.K.nblk, fullT = nT == d.Kt.nblk;
    for_each_item(nT + nK, d.remap, [&](int it) {
        const bool onT = it < nT;
        const int lb = onT ? (fullT ? it : d.actT[it]) : (fullK ? it - nT : d.actK[it - nT]);
        const Seg s = block_seg(onT ? d.Kt : d.K, lb);
        const int64_t r1 = s.row0 + s.nrows;
        const T *za = (const T *)(onT ? d.xavg : d.yavg);
        const T *z0 = (const T *)(onT ? d.x0 : d.y0);
        T *zm = (T *)(onT ? d.xam : d.yam);
        for (int64_t r = s.row0 + threadIdx.x; r < r1; r += WG) zm[r] = (T)((double)z0[r] + (double)za[r]);
    });
}

// On restart: z <- candidate, epoch start <- z.  Walks K^T blocks then K blocks
// of the running instances.
template <typename T>
__global__ __launch_bounds__(WG) void k_restart(Dev d)
{
    const int nT = d.act_cnt[1], nK = d.act_cnt[0];
    const bool fullK = nK == d.K.nblk, fullT = nT == d.Kt.nblk;
    for_each_item(nT + nK, d.remap, [&](int it) {
        const bool onT = it < nT;
        const int lb = onT ? (fullT ? it : d.actT[it]) : (fullK ? it - nT : d.actK[it - nT]);
        const OpDev &op = onT ? d.Kt : d.K;
        const Seg s = block_seg(op, lb);
        const InstState &st = d.st[s.inst];
        if (!st.restart) return;
        const int64_t r0 = s.row0;  // one logical block = rows [row0, row0 + nrows)
        const int64_t r1 = s.row0 + s.nrows;
        T *z = (T *)(onT ? d.x : d.y);
        const T *za = (const T *)(onT ? d.xam : d.yam);  // the average the check evaluated
        T *z0 = (T *)(onT ? d.x0 : d.y0);
        for (int64_t r = r0 + threadIdx.x; r < r1; r += WG) {
            const T v = st.cand_avg ? za[r] : z[r];
            z[r] = v;
            z0[r] = v;
        }
    });
}

// Active lists, rebuilt after every check by one workgroup of ACT_T threads
// walking the batch in chunks of ACT_T instances (block-wide scans in LDS).
constexpr int ACT_T = 1024;

// inclusive sum over the ACT_T entries of each of the NQ rows of s
template <int NQ>
__device__ void act_scan_lds(int64_t (*s)[ACT_T])
{
    const int t = threadIdx.x;
    for (int off = 1; off < ACT_T; off <<= 1) {
        int64_t a[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) a[q] = t >= off ? s[q][t - off] : 0;
        __syncthreads();
#pragma unroll
        for (int q = 0; q < NQ; ++q) s[q][t] += a[q];
        __syncthreads();
    }
}

// Admission of waiting instances under the byte budget (first = 1 at the
// start of a solve: instances beyond the budget start waiting).  Walking the
// admission order, a candidate (running at the first call, waiting later)
// is admitted while the running bytes plus the candidates' bytes before it
// plus its own stay within the budget, and always when nothing runs and no
// candidate precedes it: every instance needs some bytes, so the candidates
// admitted are a prefix of the order, as a one-by-one walk that stops at
// the first candidate that does not fit gives.
__global__ __launch_bounds__(ACT_T) void k_act_admit(Dev d, int64_t budget, int first)
{
    __shared__ int64_t s[1][ACT_T];
    const int t = threadIdx.x, B = d.batch;
    int64_t lv = 0;
    if (!first)
        for (int b = t; b < B; b += ACT_T)
            if (d.st[b].done == 0) lv += d.info[b].sweep_bytes;
    s[0][t] = lv;
    __syncthreads();
    act_scan_lds<1>(s);
    const int64_t live = s[0][ACT_T - 1];
    __syncthreads();
    int64_t carry = 0;
    for (int k0 = 0; k0 < B; k0 += ACT_T) {
        const int k = k0 + t;
        int b = -1;
        bool cand = false;
        int64_t need = 0;
        if (k < B) {
            b = d.adm_order[k];
            const int dn = d.st[b].done;
            cand = first ? dn == 0 : dn == 2;
            need = cand ? d.info[b].sweep_bytes : 0;
        }
        s[0][t] = need;
        __syncthreads();
        act_scan_lds<1>(s);
        const int64_t before = carry + s[0][t] - need;  // candidates' bytes ahead of this one
        if (cand) d.st[b].done = ((live == 0 && before == 0) || live + before + need <= budget) ? 0 : 2;
        carry += s[0][ACT_T - 1];
        __syncthreads();
    }
}

// ... then exclusive scans over the running instances' block counts and
// costs in instance order ...
__global__ __launch_bounds__(ACT_T) void k_act_scan(Dev d)
{
    __shared__ int64_t s[4][ACT_T];
    const int t = threadIdx.x, B = d.batch;
    int64_t carry[4] = {0, 0, 0, 0};
    for (int b0 = 0; b0 < B; b0 += ACT_T) {
        const int b = b0 + t;
        int64_t v[4] = {0, 0, 0, 0};
        if (b < B && d.st[b].done == 0) {
            const InstInfo &in = d.info[b];
            v[0] = in.blkK1 - in.blkK0;
            v[1] = in.blkT1 - in.blkT0;
            v[2] = d.bcumK[in.blkK1] - d.bcumK[in.blkK0];
            v[3] = d.bcumT[in.blkT1] - d.bcumT[in.blkT0];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) s[q][t] = v[q];
        __syncthreads();
        act_scan_lds<4>(s);
        if (b < B) {
            d.act_off[2 * b] = (int32_t)(carry[0] + s[0][t] - v[0]);
            d.act_off[2 * b + 1] = (int32_t)(carry[1] + s[1][t] - v[1]);
            d.act_coff[2 * b] = carry[2] + s[2][t] - v[2];
            d.act_coff[2 * b + 1] = carry[3] + s[3][t] - v[3];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) carry[q] += s[q][ACT_T - 1];
        __syncthreads();
    }
    if (t == 0) {
        d.act_cnt[0] = (int32_t)carry[0];
        d.act_cnt[1] = (int32_t)carry[1];
        d.act_coff[2 * B] = carry[2];
        d.act_coff[2 * B + 1] = carry[3];
    }
}

// XCD boundaries of the sweeps' active lists: thread (op, x) finds the list
// position where the running cost reaches x/8 of the total: the instance by
// bisection of the running-cost prefix (it rises only at running instances),
// then the block by bisection of the blocks' cost prefix sums.
__global__ void k_act_split(Dev d)
{
    const int t = threadIdx.x;
    if (t >= 16) return;
    const int op = t >> 3, x = t & 7;
    int32_t *sp = d.act_split + op * 9;
    const int cnt = d.act_cnt[op];
    if (x == 0) {
        sp[0] = 0;
        sp[8] = cnt;
        return;
    }
    const int64_t *cum = op == 0 ? d.bcumK : d.bcumT;
    const int B = d.batch;
    const int64_t total = d.act_coff[2 * B + op];
    const int64_t target = total * x / 8;
    // first instance whose running cost through itself exceeds the target
    int lo = 0, hi = B;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (d.act_coff[2 * (mid + 1) + op] > target) hi = mid;
        else lo = mid + 1;
    }
    int pos = cnt;
    if (lo < B) {
        const int b = lo;
        const InstInfo &in = d.info[b];
        const int b0 = op == 0 ? in.blkK0 : in.blkT0, b1 = op == 0 ? in.blkK1 : in.blkT1;
        const int64_t c0 = d.act_coff[2 * b + op];
        // largest k in [b0, b1) with cum[k] - cum[b0] <= target - c0
        int l2 = b0, h2 = b1 - 1;
        while (l2 < h2) {
            const int mid = (l2 + h2 + 1) >> 1;
            if (cum[mid] - cum[b0] <= target - c0) l2 = mid;
            else h2 = mid - 1;
        }
        pos = d.act_off[2 * b + op] + (l2 - b0);
    }
    sp[x] = pos;
}

// ... then every logical block of a running instance writes itself into place
// (instance order, block order: the lists are deterministic).
__global__ void k_act_fill(Dev d)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < d.K.nblk) {
        const int b = block_seg(d.K, t).inst;
        if (!d.st[b].done) d.actK[d.act_off[2 * b] + (t - d.info[b].blkK0)] = t;
    }
    if (t < d.Kt.nblk) {
        const int b = block_seg(d.Kt, t).inst;
        if (!d.st[b].done) d.actT[d.act_off[2 * b + 1] + (t - d.info[b].blkT0)] = t;
    }
}

// ---------------------------------------------------------------------------
// setup and service kernels (not on the per-iteration path)
// ---------------------------------------------------------------------------

__global__ void k_fill(double *p, int64_t n, double v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// max over each row of |(rowfac * a) * colfac|  (Ruiz norm of the scaled matrix).
// For K: rowfac = rho, colfac = kap; for K^T the same products are formed as
// (colfac * a) * rowfac so both operators see (rho_i * K_ij) * kap_j.
template <bool ROW_FIRST>
__global__ __launch_bounds__(WG) void k_rowmax(OpDev op, int remap, const double *rowfac,
                                               const double *colfac, double *out)
{
    __shared__ double red[8];
    const int lb = logical_block(remap);
    const Seg s = block_seg(op, lb);
    const int bi = lb - s.blk0;
    dispatch_lanes<4>(s.lanes_log2, [&](auto tag, auto rtag) {
        constexpr int L = decltype(tag)::value, R = decltype(rtag)::value;
        sweep_rows<L, 1, double, double, R, true, ROW_FIRST>(op, s, bi, colfac, nullptr, rowfac, red,
                                                              [&](int64_t r, const double *acc) { out[r] = acc[0]; });
    });
}

__global__ void k_ruiz_update(double *fac, const double *mx, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && mx[i] > 0.0) fac[i] = fac[i] / sqrt(mx[i]);
}

// scaled values (rho_i * K_ij) * kap_j in FP64 (and FP32 when v32 != null)
template <bool ROW_FIRST>
__global__ void k_scale_vals(int64_t nrows, const int64_t *rp, const int32_t *ci, double *v64,
                             float *v32, const double *rowfac, const double *colfac)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrows) return;
    const double rf = rowfac[r];
    for (int64_t p = rp[r]; p < rp[r + 1]; ++p) {
        const double cf = colfac[ci[p]];
        const double v = ROW_FIRST ? (rf * v64[p]) * cf : (cf * v64[p]) * rf;
        v64[p] = v;
        if (v32) v32[p] = (float)v;
    }
}

// c~ = kap c, l~ = l / kap, u~ = u / kap  (FP64 and iterate-type copies)
template <typename T>
__global__ void k_scale_primal(Dev d)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= d.N) return;
    const double k = d.kap[j];
    const double c = k * d.craw[j], l = d.lraw[j] / k, u = d.uraw[j] / k;
    d.c64[j] = c;
    d.l64[j] = l;
    d.u64[j] = u;
    ((T *)d.c)[j] = (T)c;
    ((T *)d.l)[j] = (T)l;
    ((T *)d.u)[j] = (T)u;
}

template <typename T>
__global__ void k_scale_dual(Dev d)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= d.M) return;
    const double q = d.rho[i] * d.qraw[i];
    d.q64[i] = q;
    ((T *)d.q)[i] = (T)q;
}

// out = K v (FP64), per-workgroup partial of sum(out^2) in partials[lb]
// out = op v (FP64) over the blocks of `list` (list[0 .. *cnt); every block
// when list is NULL), with each block's sum of squares in partials[block]
__global__ __launch_bounds__(WG) void k_spmv64(OpDev op, int remap, const double *v, double *out,
                                               double *partials, const int32_t *list, const int32_t *cntp)
{
    __shared__ double red[8];
    const int cnt = list ? *cntp : op.nblk;
    for_each_item(cnt, remap, [&](int it) {
        const int lb = list ? list[it] : it;
        const Seg s = block_seg(op, lb);
        const int bi = lb - s.blk0;
        double sq[1] = {0.0};
        dispatch_lanes<4>(s.lanes_log2, [&](auto tag, auto rtag) {
            constexpr int L = decltype(tag)::value, R = decltype(rtag)::value;
            sweep_rows<L, 1, double, double, R>(op, s, bi, v, nullptr, nullptr, red, [&](int64_t r, const double *acc) {
                out[r] = acc[0];
                sq[0] += acc[0] * acc[0];
            });
        });
        block_sum<1>(sq, red);
        if (threadIdx.x == 0 && partials) partials[lb] = sq[0];
        __syncthreads();
    });
}

// per-instance sum of partials[blk0 .. blk1) (ranges from InstInfo), fixed order
__global__ __launch_bounds__(WG) void k_inst_sum(const InstInfo *info, int onK, const double *partials,
                                                 double *out)
{
    __shared__ double lds[4];
    const InstInfo in = info[blockIdx.x];
    const int b0 = onK ? in.blkK0 : in.blkT0, b1 = onK ? in.blkK1 : in.blkT1;
    double v[1] = {0.0};
    for (int t = b0 + threadIdx.x; t < b1; t += WG) v[0] += partials[t];
    block_sum<1>(v, lds);
    if (threadIdx.x == 0) out[blockIdx.x] = v[0];
}

// The stopping test of the power iteration (Algorithm 2) for every instance
// still iterating (one lane each): est = ||K b|| from w2 = ||K b||^2; stop
// when two successive estimates differ by at most tol * est.  The state keeps
// est in knorm, the previous estimate in kkt_prev (negative before the first)
// and the pass in power_iters; a stopped instance is marked done, so the next
// active-list rebuild drops it from the sweeps.  final_pass: the pass limit
// was reached, every instance still iterating takes this estimate.
__global__ void k_power_test(Dev d, const double *w2, int it, double tol, int final_pass)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= d.batch) return;
    InstState &st = d.st[b];
    if (st.done) return;
    const double est = sqrt(w2[b]);
    st.knorm = est;
    st.power_iters = it;
    if (final_pass) return;
    if (st.kkt_prev >= 0.0 && fabs(est - st.kkt_prev) <= tol * est) st.done = 1;
    st.kkt_prev = est;
}

// v_i /= sqrt(nrm2[inst(i)])  (skips zero norms)
__global__ void k_normalize(double *v, const int32_t *inst_of, int64_t n, const double *nrm2)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double s = nrm2[inst_of[i]];
    if (s > 0.0) v[i] = v[i] / sqrt(s);
}

// per-instance sum of squares of a vector over [off, off + len)
__global__ __launch_bounds__(WG) void k_inst_nrm2(const InstInfo *info, int primal, const double *v,
                                                  double *out)
{
    __shared__ double lds[4];
    const InstInfo in = info[blockIdx.x];
    const int64_t off = primal ? in.xoff : in.yoff;
    const int64_t len = primal ? in.n : in.m;
    double s[1] = {0.0};
    for (int64_t t = threadIdx.x; t < len; t += WG) {
        const double a = v[off + t];
        s[0] += a * a;
    }
    block_sum<1>(s, lds);
    if (threadIdx.x == 0) out[blockIdx.x] = s[0];
}

// x = proj_X(0), y = 0 (and the epoch start / averages)
template <typename T>
__global__ void k_init_point(Dev d)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < d.N) {
        const double l = d.l64[i], u = d.u64[i];
        const T v = (T)(0.0 < l ? l : (0.0 > u ? u : 0.0));
        ((T *)d.x)[i] = v;
        ((T *)d.x0)[i] = v;
        ((T *)d.xavg)[i] = (T)0;  // offset from the epoch start
        ((T *)d.xbar)[i] = v;
    }
    if (i < d.M) {
        ((T *)d.y)[i] = (T)0;
        ((T *)d.y0)[i] = (T)0;
        ((T *)d.yavg)[i] = (T)0;
    }
}

// epoch start <- current iterate (start of a solve)
template <typename T>
__global__ void k_epoch_start(Dev d)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < d.N) {
        ((T *)d.x0)[i] = ((T *)d.x)[i];
        ((T *)d.xavg)[i] = (T)0;
    }
    if (i < d.M) {
        ((T *)d.y0)[i] = ((T *)d.y)[i];
        ((T *)d.yavg)[i] = (T)0;
    }
}

// FP64 copies of a point (which: 0 current, 1 average) in scaled variables;
// the average is x0 + xavg rounded to T, as the check evaluates it
template <typename T>
__global__ void k_point_to64(Dev d, int which, double *xo, double *yo)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < d.N)
        xo[i] = which ? (double)(T)((double)((const T *)d.x0)[i] + (double)((const T *)d.xavg)[i])
                      : (double)((const T *)d.x)[i];
    if (i < d.M)
        yo[i] = which ? (double)(T)((double)((const T *)d.y0)[i] + (double)((const T *)d.yavg)[i])
                      : (double)((const T *)d.y)[i];
}

// original-variable outputs of one instance: x (clipped to [l, u]), y
__global__ void k_unscale_x(Dev d, int64_t off, int64_t n, const double *xs, double *out)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int64_t j = off + t;
    double v = d.kap[j] * xs[j];
    const double l = d.lraw[j], u = d.uraw[j];
    v = v < l ? l : (v > u ? u : v);
    out[d.col_orig[j]] = v;
}

__global__ void k_unscale_y(Dev d, int64_t off, int64_t m, const double *ys, double *out)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= m) return;
    const int64_t i = off + t;
    out[d.row_orig[i]] = d.rho[i] * ys[i];
}

// lambda = proj_Lambda(c - K^T y) in original variables, from scaled y (FP64)
__global__ __launch_bounds__(WG) void k_lambda(Dev d, const double *ys, double *lam_s)
{
    __shared__ double red[8];
    const int lb = logical_block(d.remap);
    const OpDev &op = d.Kt;
    const Seg s = block_seg(op, lb);
    const int bi = lb - s.blk0;
    dispatch_lanes<4>(s.lanes_log2, [&](auto tag, auto rtag) {
        constexpr int L = decltype(tag)::value, R = decltype(rtag)::value;
        sweep_rows<L, 1, double, double, R>(op, s, bi, ys, nullptr, nullptr, red, [&](int64_t j, const double *acc) {
            const double dd = d.c64[j] - acc[0];
            lam_s[j] = proj_lambda(dd, d.l64[j], d.u64[j]) / d.kap[j];
        });
    });
}

__global__ void k_permute_out(const int32_t *perm, int64_t off, int64_t n, const double *src,
                              double *out)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) out[perm[off + t]] = src[off + t];
}

// caller point (original variables, caller order) -> scaled FP64 internal
__global__ void k_scale_in_x(Dev d, int64_t off, int64_t n, const double *in, double *xs)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int64_t j = off + t;
    xs[j] = in[d.col_orig[j]] / d.kap[j];
}

__global__ void k_scale_in_y(Dev d, int64_t off, int64_t m, const double *in, double *ys)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= m) return;
    const int64_t i = off + t;
    ys[i] = in[d.row_orig[i]] / d.rho[i];
}

// current iterate <- scaled FP64 point, projected onto X and Y
template <typename T>
__global__ void k_set_point(Dev d, int64_t xoff, int64_t n, int64_t yoff, int64_t m, int64_t m1,
                            const double *xs, const double *ys)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) {
        const int64_t j = xoff + t;
        double v = xs[j];
        const double l = d.l64[j], u = d.u64[j];
        v = v < l ? l : (v > u ? u : v);
        ((T *)d.x)[j] = (T)v;
        ((T *)d.x0)[j] = (T)v;
        ((T *)d.xavg)[j] = (T)0;
    }
    if (t < m) {
        const int64_t i = yoff + t;
        double v = ys[i];
        if (t < m1 && v < 0.0) v = 0.0;
        ((T *)d.y)[i] = (T)v;
        ((T *)d.y0)[i] = (T)v;
        ((T *)d.yavg)[i] = (T)0;
    }
}

// KKT terms of a single candidate for one instance from the check partials
__global__ __launch_bounds__(WG) void k_kkt_final(Dev d, int inst, double *out9)
{
    __shared__ double tot[NPART];
    const InstInfo in = d.info[inst];
    reduce_instance(d, in, tot);
    if (threadIdx.x != 0) return;
    Metrics m;
    metrics_from_sums(tot, in, m);
    for (int k = 0; k < 9; ++k) out9[k] = m.kkt[k];
}


// ---------------------------------------------------------------------------
// adjoint of fixed-step PDHG (reverse mode, scaled variables)
//   forward step:  v = x - tau (c - K^T y), x+ = clip(v, l, u), xbar = 2x+ - x,
//                  w = y + sigma (q - K xbar), y+ = proj_Y(w)
//   reverse step, given ax = dL/dx+, ay = dL/dy+:
//     aw = [row is "=" or w > 0] ay,          aq += sigma aw
//     axb = -sigma K^T aw,  g = ax + 2 axb
//     av = g where l < v < u (else g goes to al or au),  ac -= tau av
//     ax <- av - axb,       ay <- aw + tau K av
// ---------------------------------------------------------------------------

// ax = kap * gx, ay = rho * gy (caller layout -> internal), accumulators = 0
__global__ void k_adj_init(Dev d, AdjBufs a, const double *gx, const double *gy)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < d.N) {
        const InstInfo &in = d.info[d.inst_of_col[t]];
        a.ax[t] = d.kap[t] * gx[in.xoff + d.col_orig[t]];
        a.ac[t] = 0.0;
        a.al[t] = 0.0;
        a.au[t] = 0.0;
    }
    if (t < d.M) {
        const InstInfo &in = d.info[d.inst_of_row[t]];
        a.ay[t] = d.rho[t] * gy[in.yoff + d.row_orig[t]];
        a.aq[t] = 0.0;
    }
}

// aw = mask_y * ay ; aq += sigma * aw
__global__ void k_adj_w(Dev d, AdjBufs a, const uint8_t *__restrict__ mask_y)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= d.M) return;
    const double sigma = d.st[d.inst_of_row[i]].sigma;
    const double w = mask_y[i] ? a.ay[i] : 0.0;
    a.aw[i] = w;
    a.aq[i] += sigma * w;
}

template <typename T, int RM>
__global__ __launch_bounds__(WG) void k_rev_primal(Dev d, AdjBufs a, const uint8_t *__restrict__ mask_x)
{
    __shared__ double red[8];
    const int lb = logical_block(d.remap);
    const OpDev &op = d.Kt;
    const Seg s = block_seg(op, lb);
    const InstState *st = d.st + s.inst;
    const double tau = st->tau, sigma = st->sigma;
    const int bi = lb - s.blk0;
    dispatch_lanes<RM>(s.lanes_log2, [&](auto tag, auto rtag) {
        constexpr int L = decltype(tag)::value, R = decltype(rtag)::value;
        sweep_rows<L, 1, T, double, R>(op, s, bi, a.aw, nullptr, nullptr, red, [&](int64_t j, const double *acc) {
            const double axb = -sigma * acc[0];
            const double g = a.ax[j] + 2.0 * axb;
            const uint8_t code = mask_x[j];
            double av = 0.0;
            if (code == 1)
                a.al[j] += g;
            else if (code == 2)
                a.au[j] += g;
            else
                av = g;
            a.av[j] = av;
            a.ac[j] -= tau * av;
            a.ax[j] = av - axb;
        });
    });
}

template <typename T, int RM>
__global__ __launch_bounds__(WG) void k_rev_dual(Dev d, AdjBufs a)
{
    __shared__ double red[8];
    const int lb = logical_block(d.remap);
    const OpDev &op = d.K;
    const Seg s = block_seg(op, lb);
    const double tau = d.st[s.inst].tau;
    const int bi = lb - s.blk0;
    dispatch_lanes<RM>(s.lanes_log2, [&](auto tag, auto rtag) {
        constexpr int L = decltype(tag)::value, R = decltype(rtag)::value;
        sweep_rows<L, 1, T, double, R>(op, s, bi, a.av, nullptr, nullptr, red,
                                       [&](int64_t i, const double *acc) { a.ay[i] = a.aw[i] + tau * acc[0]; });
    });
}

// gradients in the caller's variables and layout (concatenated over the batch)
__global__ void k_adj_out(Dev d, AdjBufs a, double *gc, double *gq, double *gl, double *gu, double *gx0,
                          double *gy0)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < d.N) {
        const InstInfo &in = d.info[d.inst_of_col[t]];
        const int64_t o = in.xoff + d.col_orig[t];
        const double k = d.kap[t];
        if (gc) gc[o] = k * a.ac[t];
        if (gl) gl[o] = a.al[t] / k;
        if (gu) gu[o] = a.au[t] / k;
        if (gx0) gx0[o] = a.ax[t] / k;
    }
    if (t < d.M) {
        const InstInfo &in = d.info[d.inst_of_row[t]];
        const int64_t o = in.yoff + d.row_orig[t];
        const double r = d.rho[t];
        if (gq) gq[o] = r * a.aq[t];
        if (gy0) gy0[o] = a.ay[t] / r;
    }
}

// caller-layout FP64 data of all instances -> raw internal copies
__global__ void k_set_raw(Dev d, const double *c, const double *q, const double *l, const double *u)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < d.N) {
        const InstInfo &in = d.info[d.inst_of_col[t]];
        const int64_t o = in.xoff + d.col_orig[t];
        if (c) d.craw[t] = c[o];
        if (l) d.lraw[t] = l[o];
        if (u) d.uraw[t] = u[o];
    }
    if (t < d.M && q) {
        const InstInfo &in = d.info[d.inst_of_row[t]];
        d.qraw[t] = q[in.yoff + d.row_orig[t]];
    }
}

// ---------------------------------------------------------------------------
// launch wrappers
// ---------------------------------------------------------------------------

static inline unsigned nblk_elem(int64_t n) { return (unsigned)((n + WG - 1) / WG); }

#define LAUNCH(kern, grid, ...)                                                  \
    do {                                                                        \
        if ((grid) > 0) hipLaunchKernelGGL(kern, dim3(grid), dim3(WG), 0, s, __VA_ARGS__); \
    } while (0)

static inline unsigned sweep_grid(const Dev &d, int64_t nitems)
{
    const int64_t g = nitems < d.grid_cap ? nitems : d.grid_cap;
    return (unsigned)(g > 0 ? g : 0);
}

// kernel variant for the largest rows-per-group of the operator(s)
#define RM_SWITCH(rmax, BODY)                 \
    do {                                      \
        if ((rmax) >= 4) {                    \
            constexpr int RMV = 4;            \
            BODY;                             \
        } else if ((rmax) >= 2) {             \
            constexpr int RMV = 2;            \
            BODY;                             \
        } else {                              \
            constexpr int RMV = 1;            \
            BODY;                             \
        }                                     \
    } while (0)

template <typename T>
void launch_primal(const Dev &d, int j, int avg, uint8_t *mask, hipStream_t s)
{
    const unsigned g = sweep_grid(d, d.Kt.nblk);
    if (d.Kt.slices > 1 && !mask) {
        // column-sliced sweep: S launches (the recorded steps sweep whole rows)
        const int last = d.Kt.slices - 1;
        RM_SWITCH(d.Kt.rmax, {
            for (int pass = 0; pass < last; ++pass) LAUNCH((k_primal<T, 0, 0, RMV, 1>), g, d, j, nullptr, pass);
            if (avg) {
                LAUNCH((k_primal<T, 1, 0, RMV, 2>), g, d, j, nullptr, last);
            } else {
                LAUNCH((k_primal<T, 0, 0, RMV, 2>), g, d, j, nullptr, last);
            }
        });
        return;
    }
    RM_SWITCH(d.Kt.rmax, {
        if (mask) {
            LAUNCH((k_primal<T, 0, 1, RMV, 0>), g, d, j, mask, 0);
        } else if (avg) {
            LAUNCH((k_primal<T, 1, 0, RMV, 0>), g, d, j, mask, 0);
        } else {
            LAUNCH((k_primal<T, 0, 0, RMV, 0>), g, d, j, mask, 0);
        }
    });
}

template <typename T>
void launch_dual(const Dev &d, int j, int avg, uint8_t *mask, hipStream_t s)
{
    const unsigned g = sweep_grid(d, d.K.nblk);
    if (d.K.slices > 1 && !mask) {
        const int last = d.K.slices - 1;
        RM_SWITCH(d.K.rmax, {
            for (int pass = 0; pass < last; ++pass) LAUNCH((k_dual<T, 0, 0, RMV, 1>), g, d, j, nullptr, pass);
            if (avg) {
                LAUNCH((k_dual<T, 1, 0, RMV, 2>), g, d, j, nullptr, last);
            } else {
                LAUNCH((k_dual<T, 0, 0, RMV, 2>), g, d, j, nullptr, last);
            }
        });
        return;
    }
    RM_SWITCH(d.K.rmax, {
        if (mask) {
            LAUNCH((k_dual<T, 0, 1, RMV, 0>), g, d, j, mask, 0);
        } else if (avg) {
            LAUNCH((k_dual<T, 1, 0, RMV, 0>), g, d, j, mask, 0);
        } else {
            LAUNCH((k_dual<T, 0, 0, RMV, 0>), g, d, j, mask, 0);
        }
    });
}

template <typename T>
void launch_primal_ad(const Dev &d, hipStream_t s)
{
    const unsigned g = sweep_grid(d, d.Kt.nblk);
    RM_SWITCH(d.Kt.rmax, { LAUNCH((k_primal_ad<T, RMV>), g, d); });
}

template <typename T>
void launch_dual_ad(const Dev &d, hipStream_t s)
{
    const unsigned g = sweep_grid(d, d.K.nblk);
    if (d.K.slices > 1) {
        const int last = d.K.slices - 1;
        RM_SWITCH(d.K.rmax, {
            for (int pass = 0; pass < last; ++pass) LAUNCH((k_dual_ad<T, RMV, 1>), g, d, pass);
            LAUNCH((k_dual_ad<T, RMV, 2>), g, d, last);
        });
        return;
    }
    RM_SWITCH(d.K.rmax, { LAUNCH((k_dual_ad<T, RMV, 0>), g, d, 0); });
}

void launch_step_ad(const Dev &d, hipStream_t s)
{
    if (d.batch > 0) hipLaunchKernelGGL(k_step_ad, dim3(d.batch), dim3(STEP_WG), 0, s, d);
}

template <typename T>
void launch_commit_ad(const Dev &d, hipStream_t s)
{
    LAUNCH(k_commit_ad<T>, sweep_grid(d, d.K.nblk + d.Kt.nblk), d);
}

template <typename T>
void launch_kx_ad(const Dev &d, int all, hipStream_t s)
{
    const unsigned g = sweep_grid(d, d.K.nblk);
    RM_SWITCH(d.K.rmax, { LAUNCH((k_kx_ad<T, RMV>), g, d, all); });
}

template <typename T>
void launch_infeas(const Dev &d, const void *xp, const void *yp, hipStream_t s)
{
    const unsigned g = sweep_grid(d, d.K.nblk + d.Kt.nblk);
    const int rm = d.K.rmax > d.Kt.rmax ? d.K.rmax : d.Kt.rmax;
    RM_SWITCH(rm, { LAUNCH((k_infeas<T, RMV>), g, d, (const T *)xp, (const T *)yp); });
}

template <typename T>
void launch_save_prev(const Dev &d, hipStream_t s)
{
    LAUNCH(k_save_prev<T>, sweep_grid(d, d.K.nblk + d.Kt.nblk), d);
}

template <typename T>
void launch_check(const Dev &d, int avg, hipStream_t s)
{
    const unsigned g = sweep_grid(d, d.K.nblk + d.Kt.nblk);
    const T *x = (const T *)d.x, *xa = (const T *)d.xam, *x0 = (const T *)d.x0;
    const T *y = (const T *)d.y, *ya = (const T *)d.yam, *y0 = (const T *)d.y0;
    const int rm = d.K.rmax > d.Kt.rmax ? d.K.rmax : d.Kt.rmax;
    if (avg) LAUNCH(k_avg_point<T>, sweep_grid(d, d.K.nblk + d.Kt.nblk), d);
    if (d.K.slices > 1) {
        // K's sliced rows in S passes, as the sweeps take them
        const unsigned gk = sweep_grid(d, d.K.nblk);
        RM_SWITCH(rm, {
            for (int pass = 0; pass + 1 < d.K.slices; ++pass) {
                if (avg) {
                    LAUNCH((k_check_part<T, 2, RMV>), gk, d, x, xa, pass);
                } else {
                    LAUNCH((k_check_part<T, 1, RMV>), gk, d, x, x, pass);
                }
            }
            if (avg) {
                LAUNCH((k_check<T, 2, RMV, true>), g, d, x, xa, y, ya, x0, y0, 1);
            } else {
                LAUNCH((k_check<T, 1, RMV, true>), g, d, x, x, y, y, x0, y0, 1);
            }
        });
        return;
    }
    RM_SWITCH(rm, {
        if (avg) {
            LAUNCH((k_check<T, 2, RMV>), g, d, x, xa, y, ya, x0, y0, 1);
        } else {
            LAUNCH((k_check<T, 1, RMV>), g, d, x, x, y, y, x0, y0, 1);
        }
    });
}

void launch_check64(const Dev &d, const double *xs, const double *ys, hipStream_t s)
{
    const unsigned g = sweep_grid(d, d.K.nblk + d.Kt.nblk);
    const int rm = d.K.rmax > d.Kt.rmax ? d.K.rmax : d.Kt.rmax;
    RM_SWITCH(rm, { LAUNCH((k_check<double, 1, RMV>), g, d, xs, xs, ys, ys, xs, ys, 0); });
}

void launch_active(const Dev &d, hipStream_t s, int64_t budget, int first)
{
    if (budget > 0) hipLaunchKernelGGL(k_act_admit, dim3(1), dim3(ACT_T), 0, s, d, budget, first);
    hipLaunchKernelGGL(k_act_scan, dim3(1), dim3(ACT_T), 0, s, d);
    const int64_t n = d.K.nblk > d.Kt.nblk ? d.K.nblk : d.Kt.nblk;
    LAUNCH(k_act_fill, nblk_elem(n), d);
    hipLaunchKernelGGL(k_act_split, dim3(1), dim3(64), 0, s, d);
}

void launch_control(const Dev &d, const CtlParams &P, int iters_done, hipStream_t s)
{
    LAUNCH(k_reduce_l2, (unsigned)d.nl2, d, 1);
    LAUNCH(k_control, (unsigned)d.batch, d, P, iters_done);
}

template <typename T>
void launch_restart(const Dev &d, hipStream_t s)
{
    LAUNCH(k_restart<T>, sweep_grid(d, d.K.nblk + d.Kt.nblk), d);
}

void launch_fill(double *p, int64_t n, double v, hipStream_t s) { LAUNCH(k_fill, nblk_elem(n), p, n, v); }

void launch_rowmax(const OpDev &op, int remap, bool row_first, const double *rowfac,
                   const double *colfac, double *out, hipStream_t s)
{
    if (row_first) {
        LAUNCH(k_rowmax<true>, (unsigned)op.nblk, op, remap, rowfac, colfac, out);
    } else {
        LAUNCH(k_rowmax<false>, (unsigned)op.nblk, op, remap, rowfac, colfac, out);
    }
}

void launch_ruiz_update(double *fac, const double *mx, int64_t n, hipStream_t s)
{
    LAUNCH(k_ruiz_update, nblk_elem(n), fac, mx, n);
}

void launch_scale_vals(const OpDev &op, double *v64, float *v32, bool row_first,
                       const double *rowfac, const double *colfac, hipStream_t s)
{
    if (row_first) {
        LAUNCH(k_scale_vals<true>, nblk_elem(op.nrows), op.nrows, op.rp, op.ci, v64, v32, rowfac, colfac);
    } else {
        LAUNCH(k_scale_vals<false>, nblk_elem(op.nrows), op.nrows, op.rp, op.ci, v64, v32, rowfac, colfac);
    }
}

template <typename T>
void launch_scale_data(const Dev &d, hipStream_t s)
{
    LAUNCH(k_scale_primal<T>, nblk_elem(d.N), d);
    LAUNCH(k_scale_dual<T>, nblk_elem(d.M), d);
}

void launch_spmv64(const OpDev &op, int remap, const double *v, double *out, double *partials,
                   const int32_t *list, const int32_t *cnt, hipStream_t s)
{
    const unsigned g = (unsigned)(op.nblk < 65536 ? op.nblk : 65536);
    if (g == 0) return;
    LAUNCH(k_spmv64, g, op, remap, v, out, partials, list, cnt);
}

void launch_inst_sum(const Dev &d, int onK, const double *partials, double *out, hipStream_t s)
{
    LAUNCH(k_inst_sum, (unsigned)d.batch, d.info, onK, partials, out);
}

void launch_power_test(const Dev &d, const double *w2, int it, double tol, int final_pass, hipStream_t s)
{
    LAUNCH(k_power_test, (unsigned)((d.batch + WG - 1) / WG), d, w2, it, tol, final_pass);
}

void launch_normalize(double *v, const int32_t *inst_of, int64_t n, const double *nrm2, hipStream_t s)
{
    LAUNCH(k_normalize, nblk_elem(n), v, inst_of, n, nrm2);
}

void launch_inst_nrm2(const Dev &d, int primal, const double *v, double *out, hipStream_t s)
{
    LAUNCH(k_inst_nrm2, (unsigned)d.batch, d.info, primal, v, out);
}

template <typename T>
void launch_init_point(const Dev &d, hipStream_t s)
{
    LAUNCH(k_init_point<T>, nblk_elem(d.N > d.M ? d.N : d.M), d);
}

template <typename T>
void launch_epoch_start(const Dev &d, hipStream_t s)
{
    LAUNCH(k_epoch_start<T>, nblk_elem(d.N > d.M ? d.N : d.M), d);
}

template <typename T>
void launch_point_to64(const Dev &d, int which, double *xo, double *yo, hipStream_t s)
{
    LAUNCH(k_point_to64<T>, nblk_elem(d.N > d.M ? d.N : d.M), d, which, xo, yo);
}

void launch_unscale_x(const Dev &d, int64_t off, int64_t n, const double *xs, double *out, hipStream_t s)
{
    LAUNCH(k_unscale_x, nblk_elem(n), d, off, n, xs, out);
}

void launch_unscale_y(const Dev &d, int64_t off, int64_t m, const double *ys, double *out, hipStream_t s)
{
    LAUNCH(k_unscale_y, nblk_elem(m), d, off, m, ys, out);
}

void launch_lambda(const Dev &d, const double *ys, double *lam, hipStream_t s)
{
    LAUNCH(k_lambda, (unsigned)d.Kt.nblk, d, ys, lam);
}

void launch_permute_out(const int32_t *perm, int64_t off, int64_t n, const double *src, double *out,
                        hipStream_t s)
{
    LAUNCH(k_permute_out, nblk_elem(n), perm, off, n, src, out);
}

void launch_scale_in(const Dev &d, int64_t xoff, int64_t n, int64_t yoff, int64_t m, const double *xin,
                     const double *yin, double *xs, double *ys, hipStream_t s)
{
    if (xin) LAUNCH(k_scale_in_x, nblk_elem(n), d, xoff, n, xin, xs);
    if (yin) LAUNCH(k_scale_in_y, nblk_elem(m), d, yoff, m, yin, ys);
}

template <typename T>
void launch_set_point(const Dev &d, int64_t xoff, int64_t n, int64_t yoff, int64_t m, int64_t m1,
                      const double *xs, const double *ys, hipStream_t s)
{
    LAUNCH(k_set_point<T>, nblk_elem(n > m ? n : m), d, xoff, n, yoff, m, m1, xs, ys);
}

void launch_kkt_final(const Dev &d, int inst, double *out9, hipStream_t s)
{
    LAUNCH(k_reduce_l2, (unsigned)d.nl2, d, 0);
    hipLaunchKernelGGL(k_kkt_final, dim3(1), dim3(WG), 0, s, d, inst, out9);
}

void launch_adj_init(const Dev &d, const AdjBufs &a, const double *gx, const double *gy, hipStream_t s)
{
    LAUNCH(k_adj_init, nblk_elem(d.N > d.M ? d.N : d.M), d, a, gx, gy);
}

void launch_adj_w(const Dev &d, const AdjBufs &a, const uint8_t *mask_y, hipStream_t s)
{
    LAUNCH(k_adj_w, nblk_elem(d.M), d, a, mask_y);
}

template <typename T>
void launch_rev_primal(const Dev &d, const AdjBufs &a, const uint8_t *mask_x, hipStream_t s)
{
    RM_SWITCH(d.Kt.rmax, { LAUNCH((k_rev_primal<T, RMV>), (unsigned)d.Kt.nblk, d, a, mask_x); });
}

template <typename T>
void launch_rev_dual(const Dev &d, const AdjBufs &a, hipStream_t s)
{
    RM_SWITCH(d.K.rmax, { LAUNCH((k_rev_dual<T, RMV>), (unsigned)d.K.nblk, d, a); });
}

void launch_adj_out(const Dev &d, const AdjBufs &a, double *gc, double *gq, double *gl, double *gu,
                    double *gx0, double *gy0, hipStream_t s)
{
    LAUNCH(k_adj_out, nblk_elem(d.N > d.M ? d.N : d.M), d, a, gc, gq, gl, gu, gx0, gy0);
}

void launch_set_raw(const Dev &d, const double *c, const double *q, const double *l, const double *u,
                    hipStream_t s)
{
    LAUNCH(k_set_raw, nblk_elem(d.N > d.M ? d.N : d.M), d, c, q, l, u);
}

#define INST(T)                                                                              \
    template void launch_primal<T>(const Dev &, int, int, uint8_t *, hipStream_t);           \
    template void launch_dual<T>(const Dev &, int, int, uint8_t *, hipStream_t);             \
    template void launch_primal_ad<T>(const Dev &, hipStream_t);                             \
    template void launch_dual_ad<T>(const Dev &, hipStream_t);                               \
    template void launch_commit_ad<T>(const Dev &, hipStream_t);                             \
    template void launch_kx_ad<T>(const Dev &, int, hipStream_t);                            \
    template void launch_infeas<T>(const Dev &, const void *, const void *, hipStream_t);    \
    template void launch_save_prev<T>(const Dev &, hipStream_t);                             \
    template void launch_check<T>(const Dev &, int, hipStream_t);                            \
    template void launch_restart<T>(const Dev &, hipStream_t);                               \
    template void launch_scale_data<T>(const Dev &, hipStream_t);                            \
    template void launch_init_point<T>(const Dev &, hipStream_t);                            \
    template void launch_epoch_start<T>(const Dev &, hipStream_t);                           \
    template void launch_point_to64<T>(const Dev &, int, double *, double *, hipStream_t);   \
    template void launch_set_point<T>(const Dev &, int64_t, int64_t, int64_t, int64_t, int64_t, \
                                      const double *, const double *, hipStream_t);                 \
    template void launch_rev_primal<T>(const Dev &, const AdjBufs &, const uint8_t *, hipStream_t); \
    template void launch_rev_dual<T>(const Dev &, const AdjBufs &, hipStream_t);
INST(float)
INST(double)

}  // namespace pdhg
