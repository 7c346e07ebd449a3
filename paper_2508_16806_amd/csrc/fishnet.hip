// fishnet.hip -- gfx950 kernels of fishnet casting (Section 2.5, Algorithm 7).
//
// Up to PS candidate points run fixed-step PDHG together on the scaled LP.
// The points are interleaved (entry r of point q at [r * PS + q]), and a row
// of K~ (or K~^T) is handled by a group of j lanes, lane q for point q, where
// j is the number of live points (a power of two <= 64).  Every lane of the
// group loads the same matrix entry (one transaction for the group) and
// gathers point q's entry of the column, so a gather moves j contiguous
// values: the multi-point sweep reads the matrix once for all points.  Rows
// longer than FISH_CHUNK entries are cut into chunks (their partial sums are
// added by a combine pass in chunk order), and the tasks run longest first,
// so no lane group walks a long dependent chain.
//
// One round: k primal/dual steps on the live points, the duality gap of each
// point (grid-stride partials, reduced in a fixed order), a one-workgroup
// ranking that keeps the better half (ties by index) and, in odd rounds that
// start with more than two points, builds the repopulation weights, then a
// gather pass that writes the next round's points: the kept ones (best first)
// followed by the new convex combinations.
#include <hip/hip_runtime.h>
#include <math.h>

#include "../../include/pdhg.h"
#include "kernels.h"
#include "sweep.h"

namespace pdhg {

// sum over entries [b, e) of a row for the lane's point:
// acc = sum_p v_p * G[c_p * PS + q], in entry order (4 loads in flight)
template <typename MV, typename GV>
__device__ __forceinline__ double fish_dot(const OpDev &op, const MV *__restrict__ va, int64_t b, int64_t e,
                                           const GV *__restrict__ G, int PS, int q)
{
    const int32_t *__restrict__ ci = op.ci;
    double acc = 0.0;
    int64_t p = b;
    for (; p + 4 <= e; p += 4) {
        const int32_t c0 = ci[p], c1 = ci[p + 1], c2 = ci[p + 2], c3 = ci[p + 3];
        const double v0 = (double)va[p], v1 = (double)va[p + 1], v2 = (double)va[p + 2], v3 = (double)va[p + 3];
        const double g0 = (double)G[(int64_t)c0 * PS + q], g1 = (double)G[(int64_t)c1 * PS + q];
        const double g2 = (double)G[(int64_t)c2 * PS + q], g3 = (double)G[(int64_t)c3 * PS + q];
        acc += v0 * g0;
        acc += v1 * g1;
        acc += v2 * g2;
        acc += v3 * g3;
    }
    for (; p < e; ++p) acc += (double)va[p] * (double)G[(int64_t)ci[p] * PS + q];
    return acc;
}

template <typename MV, typename GV>
__device__ __forceinline__ double fish_row_dot(const OpDev &op, const MV *__restrict__ va, int64_t row,
                                               const GV *__restrict__ G, int PS, int q)
{
    return fish_dot(op, va, op.rp[row], op.rp[row + 1], G, PS, q);
}

// x+ = clip(x - tau (c~ - g), l~, u~), xbar = 2 x+ - x
template <typename T>
__device__ __forceinline__ void fish_primal_epi(const Dev &d, const FishDev &f, int64_t row, int q, double g,
                                                double tau)
{
    T *X = (T *)f.X;
    const int64_t at = row * f.PS + q;
    const double xo = (double)X[at];
    const double v = xo - tau * ((double)((const T *)d.c)[row] - g);
    const double lo = (double)((const T *)d.l)[row], hi = (double)((const T *)d.u)[row];
    const T xn = (T)(v < lo ? lo : (v > hi ? hi : v));
    X[at] = xn;
    ((T *)f.XB)[at] = (T)(2.0 * (double)xn - xo);
}

// INIT = 0: y+ = proj_Y(y + sigma (q~ - r)); INIT = 1: y = r
template <typename T, int INIT>
__device__ __forceinline__ void fish_dual_epi(const Dev &d, const FishDev &f, int64_t row, int q, double r,
                                              double sigma, int64_t m1)
{
    T *Y = (T *)f.Y;
    const int64_t at = row * f.PS + q;
    if (INIT) {
        Y[at] = (T)r;
        return;
    }
    const double w = (double)Y[at] + sigma * ((double)((const T *)d.q)[row] - r);
    Y[at] = (T)((row < m1 && w < 0.0) ? 0.0 : w);
}

// One lane group (j lanes, one per live point) per task, tasks longest first.
// A task that covers its whole row applies the update; a chunk of a split
// row stores its partial sum for the combine pass.
template <typename T>
__global__ __launch_bounds__(WG) void k_fish_primal(Dev d, FishDev f, int lj, double tau)
{
    const int tid = threadIdx.x, q = tid & ((1 << lj) - 1);
    const int64_t g = (int64_t)blockIdx.x * (WG >> lj) + (tid >> lj);
    if (g >= f.ntaskT) return;
    const int4 t = f.taskT[g];
    const double acc = fish_dot(d.Kt, op_vals<T>(d.Kt), t.y, t.z, (const T *)f.Y, f.PS, q);
    if (t.w < 0)
        fish_primal_epi<T>(d, f, t.x, q, acc, tau);
    else
        f.cpart[(int64_t)t.w * f.PS + q] = acc;
}

template <typename T, int INIT>
__global__ __launch_bounds__(WG) void k_fish_dual(Dev d, FishDev f, int lj, double sigma, int64_t m1)
{
    const int tid = threadIdx.x, q = tid & ((1 << lj) - 1);
    const int64_t g = (int64_t)blockIdx.x * (WG >> lj) + (tid >> lj);
    if (g >= f.ntaskK) return;
    const int4 t = f.taskK[g];
    const double acc = fish_dot(d.K, op_vals<T>(d.K), t.y, t.z, (const T *)(INIT ? f.X : f.XB), f.PS, q);
    if (t.w < 0)
        fish_dual_epi<T, INIT>(d, f, t.x, q, acc, sigma, m1);
    else
        f.cpart[(int64_t)t.w * f.PS + q] = acc;
}

// Combine passes: the chunk partials of each split row, in chunk order.
template <typename T>
__global__ __launch_bounds__(WG) void k_fish_combine_primal(Dev d, FishDev f, int lj, double tau)
{
    const int tid = threadIdx.x, q = tid & ((1 << lj) - 1);
    const int64_t g = (int64_t)blockIdx.x * (WG >> lj) + (tid >> lj);
    if (g >= f.nsplitT) return;
    const int4 sp = f.splitT[g];
    double acc = 0.0;
    for (int c = 0; c < sp.z; ++c) acc += f.cpart[(int64_t)(sp.y + c) * f.PS + q];
    fish_primal_epi<T>(d, f, sp.x, q, acc, tau);
}

template <typename T, int INIT>
__global__ __launch_bounds__(WG) void k_fish_combine_dual(Dev d, FishDev f, int lj, double sigma, int64_t m1)
{
    const int tid = threadIdx.x, q = tid & ((1 << lj) - 1);
    const int64_t g = (int64_t)blockIdx.x * (WG >> lj) + (tid >> lj);
    if (g >= f.nsplitK) return;
    const int4 sp = f.splitK[g];
    double acc = 0.0;
    for (int c = 0; c < sp.z; ++c) acc += f.cpart[(int64_t)(sp.y + c) * f.PS + q];
    fish_dual_epi<T, INIT>(d, f, sp.x, q, acc, sigma, m1);
}

// Per-workgroup partials of dobj - pobj for every live point (scaled data,
// FP64 matrix): K~^T rows add l~ lambda^+ + u~ lambda^- - c~ x with
// lambda = proj_Lambda(c~ - K~^T y); K rows add q~ y.  Row groups are
// visited grid-stride, so each workgroup's sum has a fixed order.
template <typename T>
__global__ __launch_bounds__(WG) void k_fish_gap(Dev d, FishDev f, int lj, int64_t gT, int64_t gK)
{
    __shared__ double lds[4 * 64];
    const int j = 1 << lj;
    const int tid = threadIdx.x, q = tid & (j - 1), rl = tid >> lj, rpw = WG >> lj;
    const int PS = f.PS;
    const T *X = (const T *)f.X;
    const T *Y = (const T *)f.Y;
    double v = 0.0;
    for (int64_t it = blockIdx.x; it < gT + gK; it += gridDim.x) {
        if (it < gT) {
            const int64_t g = it * rpw + rl;
            if (g < d.Kt.nrows) {
                const int64_t row = f.rowT[g];
                const double a = fish_row_dot(d.Kt, d.Kt.v64, row, Y, PS, q);
                const double cj = d.c64[row], lo = d.l64[row], hi = d.u64[row];
                const bool lf = isfinite(lo), uf = isfinite(hi);
                const double dd = cj - a;
                // proj_Lambda: {0} free, R^- upper only, R^+ lower only, R boxed
                const double lam = (!lf && !uf) ? 0.0 : (!lf ? fmin(dd, 0.0) : (!uf ? fmax(dd, 0.0) : dd));
                const double t = lam > 0.0 ? lo * lam : (lam < 0.0 ? hi * lam : 0.0);
                v += t - cj * (double)X[row * PS + q];
            }
        } else {
            const int64_t g = (it - gT) * rpw + rl;
            if (g < d.K.nrows) {
                const int64_t row = f.rowK[g];
                v += d.q64[row] * (double)Y[row * PS + q];
            }
        }
    }
    // lanes of one point: across the rows of a wavefront, then the four wavefronts
    for (int off = 32; off >= j; off >>= 1) v += __shfl_xor(v, off);
    const int wave = tid >> 6, lane = tid & 63;
    if (lane < j) lds[wave * 64 + lane] = v;
    __syncthreads();
    if (tid < j) f.part[(size_t)blockIdx.x * PS + tid] = (lds[tid] + lds[64 + tid]) + (lds[128 + tid] + lds[192 + tid]);
}

// One workgroup: gaps of the live points, the kept half (stable order by
// gap, then index), the round's record, and in repopulating rounds the
// weights w_as = |g_as| / sum_s |g_as| (equal weights for an all-zero row).
__global__ __launch_bounds__(WG) void k_fish_rank(FishDev f, int lj, int nparts, int round, int repop, int half,
                                                  int64_t wpos)
{
    __shared__ double lds[WG];
    __shared__ double gap[64];
    __shared__ int idx[64];
    const int j = 1 << lj;
    const int tid = threadIdx.x, q = tid & (j - 1), sl = tid >> lj, nsl = WG >> lj;
    const int PS = f.PS;
    double v = 0.0;
    for (int b = sl; b < nparts; b += nsl) v += f.part[(size_t)b * PS + q];
    lds[tid] = v;
    __syncthreads();
    if (tid < j) {
        double t = 0.0;
        for (int s = 0; s < nsl; ++s) t += lds[s * j + tid];
        gap[tid] = fabs(t);
        idx[tid] = tid;
    }
    __syncthreads();
    if (tid == 0) {
        for (int a = 1; a < j; ++a) {
            const int t = idx[a];
            int b = a - 1;
            while (b >= 0 && (gap[idx[b]] > gap[t] || (gap[idx[b]] == gap[t] && idx[b] > t))) {
                idx[b + 1] = idx[b];
                --b;
            }
            idx[b + 1] = t;
        }
        if (round < f.nrec) {
            for (int r = 0; r < PS; ++r) {
                f.rec_gaps[(size_t)round * PS + r] = r < j ? gap[r] : 0.0;
                f.rec_keep[(size_t)round * PS + r] = r < half ? idx[r] : -1;
            }
        }
        for (int r = 0; r < half; ++r) f.keep[r] = idx[r];
    }
    if (repop && tid < half) {
        const double *w = f.wstage + wpos + (int64_t)tid * half;
        double tot = 0.0;
        for (int s = 0; s < half; ++s) tot += fabs(w[s]);
        for (int s = 0; s < half; ++s)
            f.wmat[tid * (PS / 2) + s] = tot > 0.0 ? fabs(w[s]) / tot : 1.0 / half;
    }
}

// Next round's points: column t < half is kept point keep[t]; column
// half + a is sum_s w_as * (kept point s), accumulated in FP64.
template <typename T>
__global__ void k_fish_gather(FishDev f, int lnext, int half, int64_t N, int64_t M)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t row = t >> lnext;
    const int col = (int)(t & ((1 << lnext) - 1));
    if (row >= N + M) return;
    const bool onX = row < N;
    const int64_t r = onX ? row : row - N;
    const int PS = f.PS;
    const T *src = (const T *)(onX ? f.X : f.Y) + r * PS;
    T *dst = (T *)(onX ? f.X2 : f.Y2) + r * PS;
    if (col < half) {
        dst[col] = src[f.keep[col]];
        return;
    }
    const double *w = f.wmat + (col - half) * (PS / 2);
    double v = 0.0;
    for (int s = 0; s < half; ++s) v += w[s] * (double)src[f.keep[s]];
    dst[col] = (T)v;
}

// X^0 = sc * G (G in the caller's column order, point-major)
template <typename T>
__global__ void k_fish_init(Dev d, FishDev f, int lp, double sc)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t r = t >> lp;
    const int q = (int)(t & ((1 << lp) - 1));
    if (r >= d.N) return;
    ((T *)f.X)[r * f.PS + q] = (T)(sc * f.gstage[(int64_t)q * d.N + d.col_orig[r]]);
}

// the last point to FP64 scratch vectors (the caller then installs it)
template <typename T>
__global__ void k_fish_out(Dev d, FishDev f)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < d.N) d.vecN64[t] = (double)((const T *)f.X)[t * f.PS];
    if (t < d.M) d.vecM64[t] = (double)((const T *)f.Y)[t * f.PS];
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

static inline unsigned fish_groups(int64_t rows, int lj)
{
    const int64_t rpw = WG >> lj;
    return (unsigned)((rows + rpw - 1) / rpw);
}

template <typename T>
void launch_fish_step(const Dev &d, const FishDev &f, int lj, double tau, double sigma, int64_t m1, hipStream_t s)
{
    const unsigned tT = fish_groups(f.ntaskT, lj), cT = fish_groups(f.nsplitT, lj);
    const unsigned tK = fish_groups(f.ntaskK, lj), cK = fish_groups(f.nsplitK, lj);
    if (tT) hipLaunchKernelGGL(k_fish_primal<T>, dim3(tT), dim3(WG), 0, s, d, f, lj, tau);
    if (cT) hipLaunchKernelGGL(k_fish_combine_primal<T>, dim3(cT), dim3(WG), 0, s, d, f, lj, tau);
    if (tK) hipLaunchKernelGGL((k_fish_dual<T, 0>), dim3(tK), dim3(WG), 0, s, d, f, lj, sigma, m1);
    if (cK) hipLaunchKernelGGL((k_fish_combine_dual<T, 0>), dim3(cK), dim3(WG), 0, s, d, f, lj, sigma, m1);
}

template <typename T>
void launch_fish_init(const Dev &d, const FishDev &f, int lp, double sc, hipStream_t s)
{
    const int64_t tot = d.N << lp;
    if (tot > 0) hipLaunchKernelGGL(k_fish_init<T>, dim3((unsigned)((tot + WG - 1) / WG)), dim3(WG), 0, s, d, f, lp, sc);
    const unsigned tK = fish_groups(f.ntaskK, lp), cK = fish_groups(f.nsplitK, lp);
    if (tK) hipLaunchKernelGGL((k_fish_dual<T, 1>), dim3(tK), dim3(WG), 0, s, d, f, lp, 0.0, (int64_t)0);
    if (cK) hipLaunchKernelGGL((k_fish_combine_dual<T, 1>), dim3(cK), dim3(WG), 0, s, d, f, lp, 0.0, (int64_t)0);
}

template <typename T>
int launch_fish_gap_rank(const Dev &d, const FishDev &f, int lj, int round, int repop, int half, int64_t wpos,
                         hipStream_t s)
{
    const int64_t gT = fish_groups(d.Kt.nrows, lj), gK = fish_groups(d.K.nrows, lj);
    const int64_t items = gT + gK;
    const int grid = (int)(items < FISH_GRID ? (items > 0 ? items : 1) : FISH_GRID);
    hipLaunchKernelGGL(k_fish_gap<T>, dim3(grid), dim3(WG), 0, s, d, f, lj, gT, gK);
    hipLaunchKernelGGL(k_fish_rank, dim3(1), dim3(WG), 0, s, f, lj, grid, round, repop, half, wpos);
    return grid;
}

template <typename T>
void launch_fish_gather(const Dev &d, const FishDev &f, int lnext, int half, hipStream_t s)
{
    const int64_t tot = (d.N + d.M) << lnext;
    if (tot > 0)
        hipLaunchKernelGGL(k_fish_gather<T>, dim3((unsigned)((tot + WG - 1) / WG)), dim3(WG), 0, s, f, lnext, half,
                           d.N, d.M);
}

template <typename T>
void launch_fish_out(const Dev &d, const FishDev &f, hipStream_t s)
{
    const int64_t n = d.N > d.M ? d.N : d.M;
    if (n > 0) hipLaunchKernelGGL(k_fish_out<T>, dim3((unsigned)((n + WG - 1) / WG)), dim3(WG), 0, s, d, f);
}

#define FISH_INST(T)                                                                                       \
    template void launch_fish_step<T>(const Dev &, const FishDev &, int, double, double, int64_t, hipStream_t); \
    template void launch_fish_init<T>(const Dev &, const FishDev &, int, double, hipStream_t);           \
    template int launch_fish_gap_rank<T>(const Dev &, const FishDev &, int, int, int, int, int64_t, hipStream_t); \
    template void launch_fish_gather<T>(const Dev &, const FishDev &, int, int, hipStream_t);            \
    template void launch_fish_out<T>(const Dev &, const FishDev &, hipStream_t);
FISH_INST(float)
FISH_INST(double)

}  // namespace pdhg
