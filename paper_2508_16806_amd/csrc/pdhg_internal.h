// pdhg_internal.h -- device data layout shared by the host library and the
// gfx950 kernels.  Not part of the public ABI.
//
// Layout in HBM (one workspace, carved by the host):
//
//  * Two sparse operators in row-binned CSR:
//      K   rows = dual variables (all instances, internal row order),
//          columns index the concatenated primal vectors;
//      K^T rows = primal variables, columns index the dual vectors.
//    Inside an instance, rows are grouped into segments of similar length
//    (">=" rows of K before "=" rows, so y_1..m1 >= 0 is a contiguous range);
//    a segment is swept by lane groups of L = 1..64 lanes per row, or by a
//    whole 256-lane workgroup per row for long rows.  Entries keep the caller's
//    order inside a row of K; a row of K^T lists its entries by increasing
//    internal row of K.
//    Values exist in FP64 (check, setup) and, in FP32 mode, in FP32 (sweeps).
//  * Vectors are concatenated over the batch in internal order; every
//    instance owns a contiguous range of the primal and of the dual vectors.
//  * Logical workgroup b of a sweep belongs to segment blk_seg[b]; the blocks
//    of one instance are contiguous, so per-instance reductions read a fixed
//    contiguous range of per-block partial sums (deterministic, no atomics).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/pdhg.h"

namespace pdhg {

constexpr int WG = 256;   // workgroup size of every sweep (4 wave64)
constexpr int NBIN = 8;   // row-length bins
constexpr int NSUM = 9;   // partial sums per candidate in the check
constexpr int NCAND = 2;  // candidates: current iterate, epoch average
constexpr int L2CH = 512; // first-level partial rows summed by one second-level block
// Infeasibility detection adds NINF per-block terms after the check's sums:
// sums, except slots 1, 2 and 5, which are maxima.
constexpr int NINF = 8;
constexpr int NPART = NCAND * NSUM + NINF;  // stride of the per-block partials
__host__ __device__ constexpr bool part_is_max(int k)
{
    return k == NCAND * NSUM + 1 || k == NCAND * NSUM + 2 || k == NCAND * NSUM + 5;
}

struct Seg {
    int64_t row0;       // first row (global internal index)
    int32_t nrows;
    int32_t blk0;       // first logical block of the sweep
    int32_t nblk;
    int32_t lanes_log2; // log2 of lanes per row: 0..6, or 8 (whole workgroup)
    int32_t inst;
    int32_t ineq;       // rows of this segment are ">=" rows (dual operator only)
    int32_t sliced;     // rows swept in column slices (opts.col_slices / col_slices_t)
};

struct OpDev {
    int64_t nrows;
    const int64_t *rp;   // nrows + 1 (global entry offsets)
    const int32_t *ci;   // global column index into the gathered vector
    const float *v32;    // scaled values, FP32 (FP32 mode)
    const double *v64;   // scaled values, FP64 (after setup)
    const Seg *seg;
    const int32_t *blk_seg;
    const int4 *bdesc;   // per logical block: {first row, rows, instance, lanes_log2 | ineq << 8 | sliced << 9}
    int32_t nseg;
    int32_t nblk;
    int32_t rmax;        // largest rows per lane group in any block (1, 2, 4)
    // column slices (S > 1): for every row, the offsets from its first entry
    // where slices 1 .. S-1 begin (nrows x (S - 1); rows of unsliced segments
    // hold zeros), and the FP64 partial products of the sliced rows (nrows;
    // 2 nrows for K, whose solve-time check keeps one set per candidate)
    int32_t slices;
    const int32_t *sb;
    double *part;
};

// Immutable per-instance facts.
struct InstInfo {
    int64_t xoff, yoff;  // offsets into the primal / dual vectors
    int32_t n, m, m1;
    int32_t blkK0, blkK1;  // logical block range of K-sweeps
    int32_t blkT0, blkT1;  // logical block range of K^T-sweeps
    int32_t l2off, l2cnt;  // second-level partial rows of this instance
    double cnorm, qnorm;   // ||c||_2 and ||q||_2 of the ORIGINAL LP
    double cnorm_s, qnorm_s;  // of the scaled LP
    int64_t sweep_bytes;   // bytes one iteration's two sweeps read and write
};

// Solver state per instance, read by every sweep, written by the control kernel.
struct InstState {
    double tau, sigma, omega, eta, omega0, knorm;
    double kkt0;       // restart metric at the start of the epoch
    double kkt_prev;   // restart metric of the previous candidate (inf at epoch start)
    long long k_total; // iterations of this solve
    long long t_inner; // iterations of the current restart epoch
    int32_t done;      // 1: stopped, 2: waiting for admission; sweeps skip both
    int32_t status;    // PDHG_OPTIMAL / ..._ITERATION_LIMIT / ..._NUMERICAL_ERROR
    int32_t restart;   // the last check decided a restart
    int32_t cand_avg;  // the last check's candidate is the average
    int32_t sol_avg;   // the returned point is the average
    int32_t nrestarts;
    int32_t power_iters;
    int32_t par;       // adaptive steps: buffer (0 or 1) holding the current iterate
    double kkt[9];     // pres, dres, pobj, dobj, gap, rel_pres, rel_dres, rel_gap, rel_kkt
    // adaptive step size (Algorithm 5)
    double eta_try;    // step the next attempt tries
    double eta_sum;    // sum of the accepted steps of the current epoch (average weights)
    long long k_att;   // attempts of this solve
    long long n_acc;   // accepted steps of this solve
    int32_t prev_ok;   // the last attempt was accepted: buffer 1 holds the iterate before it
    int32_t pad2;
    long long ntrace;  // check records written by this solve
};

struct CtlParams {
    double eps, beta_suff, beta_nec, beta_art, eps_zero;
    long long max_iters;
    int32_t check_every;
    int32_t use_restarts, use_pw;
    int32_t batch;
    int32_t adaptive;  // adaptive step size: the check follows a commit to buffer 0
    int32_t detect;    // infeasibility detection (Algorithm 6)
    double infeas_tol;
};

// Device pointers and sizes of one handle (passed by value to kernels).
struct Dev {
    int32_t batch;
    int32_t remap;       // XCD-contiguous workgroup numbering
    int64_t N, M;        // total primal / dual length
    OpDev K, Kt;
    // primal vectors (length N).  With adaptive steps the iterate and its
    // average are double-buffered per instance: buffer 0 = (x, xavg), buffer 1
    // = (xbar, xavg1); likewise (y, yavg, kx0) / (y1, yavg1, kx1) for the dual.
    // The epoch averages are kept as means of offsets from the epoch start:
    // xavg holds mean_t (x_t - x0), so the average is x0 + xavg (its FP32
    // rounding error scales with the distance from x0, not with |x|).  xam /
    // yam receive the average point (x0 + xavg rounded to T) before a check.
    void *x, *xbar, *xavg, *x0;   // iterate type T
    void *xavg1;
    void *xam, *yam;              // the average point of the last check, type T
    void *c, *l, *u;              // scaled data, type T
    double *c64, *l64, *u64;      // scaled data, FP64
    double *kap;                  // column factors (x = kap * x~)
    double *craw, *lraw, *uraw;   // original data, internal order
    int32_t *col_orig;            // internal column -> caller column (per instance)
    int32_t *inst_of_col;
    // dual vectors (length M)
    void *y, *yavg, *y0, *q;      // type T
    void *y1, *yavg1;
    double *kx0, *kx1;            // K~ x of the buffer's iterate (sweep precision, FP64 sums)
    double *q64, *rho, *qraw;
    int32_t *row_orig;            // internal row -> caller row (per instance)
    int32_t *inst_of_row;
    // per instance
    const InstInfo *info;
    InstState *st;
    int32_t *hdone;               // host-mapped copy of done flags
    // scratch
    double *partials;             // (K.nblk + Kt.nblk) * NPART
    double *partials2;            // nl2 * NPART (second level)
    double *adp;                  // adaptive step: 2 per K block, then 1 per K^T block
    const int32_t *l2_inst;       // instance of each second-level row
    int32_t nl2;
    int32_t *actK, *actT;         // logical blocks of running instances (K, K^T sweeps)
    int32_t *act_cnt;             // [2]: lengths of actK, actT
    int32_t *act_off;             // [2 * batch]: list offsets per instance
    // XCD split of the sweeps' active lists by cost: bcum = prefix sums of the
    // blocks' cost (entries + 4 per row) in block order, act_coff the list
    // cost before each instance, act_split 2 x 9 list positions (K, then K^T)
    const int64_t *bcumK, *bcumT;
    int64_t *act_coff;            // [2 * batch + 2]: per instance, then the totals
    int32_t *act_split;
    int32_t *adm_order;           // [batch]: admission order (decreasing sweep bytes)
    int32_t grid_cap;             // workgroups of a solve-time sweep launch
    pdhg_trace_rec *trace;        // batch x trace_cap check records (ring per instance)
    int32_t trace_cap;
    double *vecN64, *vecN64b;     // FP64 scratch vectors (N)
    double *vecM64, *vecM64b;     // FP64 scratch vectors (M)
    double *inst_scratch;         // batch * 16
};

// Fishnet casting (Algorithm 7): up to PS candidate points, interleaved
// (entry r of point q at [r * PS + q]) so that one gather of a matrix entry
// serves every point with a contiguous load.
struct FishDev {
    int32_t PS;                 // point capacity (stride), a power of two <= 64
    int32_t nrec;               // rounds the record arrays hold
    void *X, *XB, *Y;           // current points (type T): N x PS, N x PS, M x PS
    void *X2, *Y2;              // next round's points
    const int32_t *rowK, *rowT; // rows of K / K^T by decreasing length
    // sweep tasks: {row, first entry, end entry, partial slot or -1}; rows
    // longer than FISH_CHUNK entries are split into chunks whose partial sums
    // a combine pass adds ({row, first slot, chunks, 0} per split row)
    const int4 *taskK, *taskT;
    const int4 *splitK, *splitT;
    int64_t ntaskK, ntaskT, nsplitK, nsplitT;
    double *cpart;              // chunk partials, slots x PS
    double *part;               // per-workgroup gap partials, FISH_GRID x PS
    double *wmat;               // repopulation weights, (PS/2) x (PS/2)
    int32_t *keep;              // kept point indices of the current round (PS)
    double *gstage;             // caller's normal draws, PS x N (FP64)
    double *wstage;             // caller's repopulation draws (PS * PS)
    double *rec_gaps;           // nrec x PS
    int32_t *rec_keep;          // nrec x PS
};
constexpr int FISH_GRID = 512;  // workgroups of the gap pass
constexpr int FISH_CHUNK = 256; // longest row a lane group sums in one pass

// FP64 adjoint vectors of the unrolled-step backward pass.
struct AdjBufs {
    double *ax, *av, *ac, *al, *au;  // length N
    double *ay, *aw, *aq;            // length M
};

}  // namespace pdhg
