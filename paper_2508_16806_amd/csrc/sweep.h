// sweep.h -- the row-binned CSR sweep every gfx950 kernel of the library is
// built on.  One workgroup = 256 lanes = 4 wave64.  A workgroup processes
// rows of one segment; each row is handled by a group of L lanes (L = 1..64
// inside a wavefront, or the whole workgroup for long rows).  Lanes of a group
// stride over the row's entries, multiply the stored value by the gathered
// vector entry and accumulate in FP64; the group then reduces its lanes with
// cross-lane shuffles (and LDS across wavefronts for the whole-workgroup
// case).  The group's first lane receives the row's dot product(s) and runs
// the caller's epilogue.
#pragma once
#include <hip/hip_runtime.h>

#include "pdhg_internal.h"

namespace pdhg {

// Logical workgroup index.  The hardware hands consecutive workgroup ids to
// the 8 XCDs round-robin; with `remap` the logical numbering gives each XCD a
// contiguous run of blocks (so neighbouring rows share one XCD's L2).
__device__ __forceinline__ int logical_block(int remap)
{
    const int b = blockIdx.x;
    if (!remap) return b;
    const int nb = gridDim.x;
    const int xcd = b & 7, q = nb >> 3, r = nb & 7;
    return xcd * q + (xcd < r ? xcd : r) + (b >> 3);
}

// A value the caller knows to be the same in every lane (read from per-
// instance state at a uniform address), moved to scalar registers so it costs
// no vector registers.
__device__ __forceinline__ int uniform_i(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ double uniform_d(double v)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)b);
    const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(b >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Work items [0, cnt) of a bounded grid.  With `remap`, XCD x (the hardware
// places workgroup b on XCD b mod 8) takes the contiguous item range
// [x * ceil(cnt/8), (x + 1) * ceil(cnt/8)) and its workgroups stride through
// it, so neighbouring rows share one XCD's L2.  The loop is uniform across a
// workgroup (f may use __syncthreads).
template <typename F>
__device__ __forceinline__ void for_each_item(int cnt, int remap, F &&f)
{
    const int G = gridDim.x, b = blockIdx.x;
    if (!remap || G < 8) {
        for (int it = b; it < cnt; it += G) f(it);
        return;
    }
    const int xcd = b & 7, loc = b >> 3;
    const int nloc = (G - xcd + 7) >> 3;
    const int per = (cnt + 7) >> 3;
    const int i0 = xcd * per;
    const int i1 = min(cnt, i0 + per);
    for (int it = i0 + loc; it < i1; it += nloc) f(it);
}

// As for_each_item, but with `remap` XCD x takes the item range
// [split[x], split[x + 1]) (ranges of equal cost, computed by k_act_split).
// With `rev` the walk runs backwards: the two sweeps of an iteration alternate
// direction between iterations, and each then starts on the part of its matrix
// that the other sweep's pass has not yet pushed out of the last-level cache.
// Without `remap` item i becomes item cnt - 1 - i; with it, each XCD walks its
// own range from its end, so it keeps its share of the cost.
template <typename F>
__device__ __forceinline__ void for_each_item_split(int cnt, int remap, const int32_t *split, int rev, F &&f)
{
    const int G = gridDim.x, b = blockIdx.x;
    if (!remap || G < 8) {
        const int last = rev ? cnt - 1 : 0, sgn = rev ? -1 : 1;
        for (int it = b; it < cnt; it += G) f(last + sgn * it);
        return;
    }
    const int xcd = b & 7, loc = b >> 3;
    const int nloc = (G - xcd + 7) >> 3;
    const int i0 = split[xcd], i1 = min(cnt, split[xcd + 1]);
    if (rev) {
        for (int it = i1 - 1 - loc; it >= i0; it -= nloc) f(it);
    } else {
        for (int it = i0 + loc; it < i1; it += nloc) f(it);
    }
}

// The rows of logical block lb as a one-block segment (one 16-byte load):
// rows [row0, row0 + nrows) of one instance and one length bin.
__device__ __forceinline__ Seg block_seg(const OpDev &op, int lb)
{
    const int4 v = op.bdesc[lb];
    Seg s;
    s.row0 = v.x;
    s.nrows = v.y;
    s.blk0 = lb;
    s.nblk = 1;
    s.inst = v.z;
    s.lanes_log2 = v.w & 0xff;  // lanes (bits 0-3) and rows per group (bits 4-5)
    s.ineq = (v.w >> 8) & 1;
    s.sliced = (v.w >> 9) & 1;
    return s;
}

template <typename V>
__device__ __forceinline__ const V *op_vals(const OpDev &op);
template <>
__device__ __forceinline__ const float *op_vals<float>(const OpDev &op) { return op.v32; }
template <>
__device__ __forceinline__ const double *op_vals<double>(const OpDev &op) { return op.v64; }

template <typename V>
__device__ __forceinline__ double ld(const V *p, int64_t i) { return (double)p[i]; }

// Load with a 32-bit byte offset from a workgroup-uniform base: the compiler
// emits the scalar-base + 32-bit-offset global load (one VGPR per address).
template <typename V>
__device__ __forceinline__ V ldo(const V *base, uint32_t idx)
{
    return *(const V *)((const char *)base + idx * (uint32_t)sizeof(V));
}

// Store with a 32-bit byte offset from a workgroup-uniform base (as ldo).
template <typename V>
__device__ __forceinline__ void sto(V *base, uint32_t idx, V v)
{
    *(V *)((char *)base + idx * (uint32_t)sizeof(V)) = v;
}

// Sum (or max when MAXABS) of a value across the L lanes of a group.
template <int L, bool MAXABS>
__device__ __forceinline__ double group_reduce(double v)
{
#pragma unroll
    for (int off = L / 2; off > 0; off >>= 1) {
        const double o = __shfl_xor(v, off);
        v = MAXABS ? fmax(v, o) : v + o;
    }
    return v;
}

// Per-row dot products of one workgroup's rows.  NR gathered vectors (1 or 2).
// A group of L lanes handles R consecutive rows (R = 1 for whole-workgroup
// rows); their loads are interleaved so one chain of memory latencies moves
// R rows.  MAXABS: instead of a dot product, the max over the row of
// |(a * v) * b| with the factor vectors (Ruiz pass).  SLICE: only the entries
// of column slice `pass` of each row (its entries are grouped by slice; sb
// holds where slices 1 .. S-1 begin, relative to the row's first entry).
template <int L, int NR, typename MV, typename GV, int R = 1, bool MAXABS = false, bool FAC_ROW_FIRST = true,
          bool SLICE = false>
struct RowSweep {
    static constexpr int G = (L >= WG) ? 1 : WG / L;
    static constexpr int U = (L >= WG) ? 4 : (R >= 4 ? 1 : (R == 2 ? 2 : 4));

    // Position of this lane: the first of its group's R rows, how many of them
    // exist, and whether this lane leads the group (receives the products).
    struct Pos {
        int64_t row0;
        int64_t blk_row0;  // first row of the workgroup (uniform)
        int lane;
        int nvalid;
        bool leader;
    };

    __device__ __forceinline__ static Pos locate(const Seg &s, int bi)
    {
        const int tid = threadIdx.x;
        const int grp = (L >= WG) ? 0 : tid / L;
        const int lane = (L >= WG) ? tid : (tid & (L - 1));
        const int64_t first = (int64_t)bi * G * R;
        const int64_t rloc = first + (int64_t)grp * R;
        int64_t nv = s.nrows - rloc;
        nv = nv < 0 ? 0 : (nv > R ? R : nv);
        return {s.row0 + rloc, s.row0 + first, lane, (int)nv, nv > 0 && lane == 0};
    }

    // Dot products of the group's rows with the gathered vector(s); valid in
    // the leader lane.  Every lane of the workgroup must call it.
    __device__ __forceinline__ static void dot(const OpDev &op, const Pos &ps,
                                               const GV *__restrict__ g0, const GV *__restrict__ g1,
                                               const double *__restrict__ rowfac, double *red_lds,
                                               double (&acc)[R][NR], const int32_t *__restrict__ sb = nullptr,
                                               int S = 1, int pass = 0)
    {
        const int tid = threadIdx.x;
        const int lane = ps.lane;
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int k = 0; k < NR; ++k) acc[r][k] = 0.0;
        if (ps.nvalid > 0) {
            if constexpr (MAXABS) {
                const MV *__restrict__ va = op_vals<MV>(op);
                const int32_t *__restrict__ ci = op.ci;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    if (r >= ps.nvalid) break;
                    const int64_t row = ps.row0 + r;
                    const int64_t b = op.rp[row], e = op.rp[row + 1];
                    const double rf = rowfac[row];
                    for (int64_t p = b + lane; p < e; p += L) {
                        const double cf = ld(g0, ci[p]);
                        const double a = ld(va, p);
                        const double t = FAC_ROW_FIRST ? (rf * a) * cf : (cf * a) * rf;
                        acc[r][0] = fmax(acc[r][0], fabs(t));
                    }
                }
            } else {
                // Entries are addressed relative to the workgroup's first entry
                // (a uniform base) with 32-bit offsets.  Each round issues, per
                // row, U column and U value loads and then the U independent
                // gathers, with no branches: a slot past its row's end reloads
                // the workgroup's first entry (in range: the loop only runs when
                // the group's rows hold entries) and contributes zero.
                const int64_t base = op.rp[ps.blk_row0];
                const int32_t *__restrict__ cib = op.ci + base;
                const MV *__restrict__ vab = op_vals<MV>(op) + base;
                uint32_t ob[R], oe[R];
                uint32_t maxlen = 0;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int64_t row = ps.row0 + (r < ps.nvalid ? r : ps.nvalid - 1);
                    int64_t b = op.rp[row], e = op.rp[row + 1];
                    if constexpr (SLICE) {
                        const int32_t *rs = sb + (size_t)row * (S - 1);
                        const int64_t b0 = b;
                        if (pass > 0) b = b0 + rs[pass - 1];
                        if (pass < S - 1) e = b0 + rs[pass];
                    }
                    ob[r] = (uint32_t)(b - base);
                    oe[r] = r < ps.nvalid ? (uint32_t)(e - base) : ob[r];
                    maxlen = max(maxlen, oe[r] - ob[r]);
                }
                for (uint32_t off = lane; off < maxlen; off += U * L) {
                    uint32_t c[R][U];
                    MV raw[R][U];
#pragma unroll
                    for (int r = 0; r < R; ++r)
#pragma unroll
                        for (int k = 0; k < U; ++k) {
                            const uint32_t p = ob[r] + off + (uint32_t)(k * L);
                            const uint32_t q = p < oe[r] ? p : 0u;
                            c[r][k] = (uint32_t)ldo(cib, q);
                            raw[r][k] = ldo(vab, q);
                        }
                    double g[R][U];
#pragma unroll
                    for (int r = 0; r < R; ++r)
#pragma unroll
                        for (int k = 0; k < U; ++k) g[r][k] = (double)ldo(g0, c[r][k]);
#pragma unroll
                    for (int r = 0; r < R; ++r)
#pragma unroll
                        for (int k = 0; k < U; ++k) {
                            const double a = (ob[r] + off + (uint32_t)(k * L) < oe[r]) ? (double)raw[r][k] : 0.0;
                            acc[r][0] += a * g[r][k];
                        }
                    if constexpr (NR > 1) {
#pragma unroll
                        for (int r = 0; r < R; ++r)
#pragma unroll
                            for (int k = 0; k < U; ++k) g[r][k] = (double)ldo(g1, c[r][k]);
#pragma unroll
                        for (int r = 0; r < R; ++r)
#pragma unroll
                            for (int k = 0; k < U; ++k) {
                                const double a =
                                    (ob[r] + off + (uint32_t)(k * L) < oe[r]) ? (double)raw[r][k] : 0.0;
                                acc[r][1] += a * g[r][k];
                            }
                    }
                }
            }
        }
        if constexpr (L >= WG) {
            // wavefront reduce, then the four wavefront totals in LDS, fixed order
#pragma unroll
            for (int k = 0; k < NR; ++k) acc[0][k] = group_reduce<64, MAXABS>(acc[0][k]);
            const int wave = tid >> 6;
            if ((tid & 63) == 0) {
#pragma unroll
                for (int k = 0; k < NR; ++k) red_lds[k * 4 + wave] = acc[0][k];
            }
            __syncthreads();
            if (tid == 0) {
#pragma unroll
                for (int k = 0; k < NR; ++k) {
                    const double *rr = red_lds + k * 4;
                    acc[0][k] = MAXABS ? fmax(fmax(rr[0], rr[1]), fmax(rr[2], rr[3]))
                                       : (rr[0] + rr[1]) + (rr[2] + rr[3]);
                }
            }
            __syncthreads();
        } else {
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int k = 0; k < NR; ++k) acc[r][k] = group_reduce<L, MAXABS>(acc[r][k]);
        }
    }
};

// locate + dot, then f(row, products) for each of the group's rows, in the
// leader lane.
template <int L, int NR, typename MV, typename GV, int R, bool MAXABS = false, bool FRF = true, typename F>
__device__ __forceinline__ void sweep_rows(const OpDev &op, const Seg &s, int bi, const GV *g0, const GV *g1,
                                           const double *rowfac, double *red, F &&f)
{
    using RS = RowSweep<L, NR, MV, GV, R, MAXABS, FRF>;
    const typename RS::Pos ps = RS::locate(s, bi);
    double acc[R][NR];
    RS::dot(op, ps, g0, g1, rowfac, red, acc);
    if (ps.leader) {
#pragma unroll
        for (int r = 0; r < R; ++r)
            if (r < ps.nvalid) f(ps.row0 + r, acc[r]);
    }
}

// Dispatch on the block's lanes per row and rows per group (uniform across
// the workgroup).  f is called as f(LaneTag<L>{}, LaneTag<R>{}).
template <int L>
struct LaneTag {
    static constexpr int value = L;
};

// RM: the largest rows-per-group the launch supports (the host picks the
// kernel variant from the operator's bins, so kernels over R = 1 layouts keep
// the register footprint of the single-row path).
template <int RM = 1, typename F>
__device__ __forceinline__ void dispatch_lanes(int code, F &&f)
{
    const int lanes_log2 = code & 15, rows_log2 = (code >> 4) & 3;
    switch (lanes_log2) {
#define PDHG_LR(LL, LV)                                                   \
    case LL:                                                            \
        if constexpr (RM >= 4) {                                        \
            if (rows_log2 == 2) {                                       \
                f(LaneTag<LV>{}, LaneTag<4>{});                         \
                break;                                                  \
            }                                                           \
        }                                                               \
        if constexpr (RM >= 2) {                                        \
            if (rows_log2 >= 1) {                                       \
                f(LaneTag<LV>{}, LaneTag<(RM >= 2 ? 2 : 1)>{});         \
                break;                                                  \
            }                                                           \
        }                                                               \
        f(LaneTag<LV>{}, LaneTag<1>{});                                 \
        break;
        PDHG_LR(0, 1)
        PDHG_LR(1, 2)
        PDHG_LR(2, 4)
        PDHG_LR(3, 8)
        PDHG_LR(4, 16)
#undef PDHG_LR
        case 5: f(LaneTag<32>{}, LaneTag<1>{}); break;
        case 6: f(LaneTag<64>{}, LaneTag<1>{}); break;
        default: f(LaneTag<WG>{}, LaneTag<1>{}); break;
    }
}

// Rows of one logical block of a segment with this lanes / rows code.
__host__ __device__ __forceinline__ int block_rows(int code)
{
    const int lanes_log2 = code & 15, rows_log2 = (code >> 4) & 3;
    return (lanes_log2 >= 8 ? 1 : (WG >> lanes_log2)) << rows_log2;
}

// Block-wide sum of NV per-thread values, fixed reduction order; result valid
// in thread 0.  lds must hold NV * 4 doubles.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double *lds)
{
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = group_reduce<64, false>(v[k]);
    const int tid = threadIdx.x, wave = tid >> 6;
    __syncthreads();
    if ((tid & 63) == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) lds[k * 4 + wave] = v[k];
    }
    __syncthreads();
    if (tid == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            const double *r = lds + k * 4;
            v[k] = (r[0] + r[1]) + (r[2] + r[3]);
        }
    }
}

}  // namespace pdhg
