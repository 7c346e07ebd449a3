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
    s.lanes_log2 = v.w & 0xff;
    s.ineq = v.w >> 8;
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
// MAXABS: instead of a dot product, max over the row of |(a * v) * b| where
// the products use the factor vectors (Ruiz pass).
template <int L, int NR, typename MV, typename GV, bool MAXABS = false, bool FAC_ROW_FIRST = true>
struct RowSweep {
    static constexpr int G = (L >= WG) ? 1 : WG / L;

    // Position of this lane: the row its group handles, whether that row
    // exists, and whether this lane leads the group (receives the dot product).
    struct Pos {
        int64_t row;
        int64_t blk_row0;  // first row of the workgroup (uniform)
        int lane;
        bool valid;
        bool leader;
    };

    __device__ __forceinline__ static Pos locate(const Seg &s, int bi)
    {
        const int tid = threadIdx.x;
        const int grp = (L >= WG) ? 0 : tid / L;
        const int lane = (L >= WG) ? tid : (tid & (L - 1));
        const int64_t rloc = (int64_t)bi * G + grp;
        const bool valid = rloc < s.nrows;
        return {s.row0 + rloc, s.row0 + (int64_t)bi * G, lane, valid, valid && lane == 0};
    }

    // Dot product(s) of the row at p with the gathered vector(s); the result
    // is valid in the leader lane.  Every lane of the workgroup must call it.
    __device__ __forceinline__ static void dot(const OpDev &op, const Pos &ps,
                                               const GV *__restrict__ g0, const GV *__restrict__ g1,
                                               const double *__restrict__ rowfac, double *red_lds,
                                               double (&acc)[NR])
    {
        const int tid = threadIdx.x;
        const int lane = ps.lane;
        const int64_t row = ps.row;
#pragma unroll
        for (int k = 0; k < NR; ++k) acc[k] = 0.0;
        if (ps.valid) {
            const int64_t b = op.rp[row], e = op.rp[row + 1];
            if constexpr (MAXABS) {
                const MV *__restrict__ va = op_vals<MV>(op);
                const int32_t *__restrict__ ci = op.ci;
                const double rf = rowfac[row];
                for (int64_t p = b + lane; p < e; p += L) {
                    const double cf = ld(g0, ci[p]);
                    const double a = ld(va, p);
                    const double t = FAC_ROW_FIRST ? (rf * a) * cf : (cf * a) * rf;
                    acc[0] = fmax(acc[0], fabs(t));
                }
            } else {
                // Entries are addressed relative to the workgroup's first entry
                // (a uniform base) with 32-bit offsets.  U-deep unroll with
                // clamped offsets: every lane issues U column and U value
                // loads, then U independent gathers, with no branches (a slot
                // past the row end reloads the lane's first entry, which is in
                // range, and contributes zero).
                constexpr int U = 4;
                const int64_t base = op.rp[ps.blk_row0];
                const int32_t *__restrict__ cib = op.ci + base;
                const MV *__restrict__ vab = op_vals<MV>(op) + base;
                const uint32_t ob = (uint32_t)(b - base), oe = (uint32_t)(e - base);
                for (uint32_t p0 = ob + lane; p0 < oe; p0 += U * L) {
                    uint32_t c[U];
                    MV raw[U];
#pragma unroll
                    for (int k = 0; k < U; ++k) {
                        const uint32_t p = p0 + (uint32_t)(k * L);
                        const uint32_t q = p < oe ? p : p0;
                        c[k] = (uint32_t)ldo(cib, q);
                        raw[k] = ldo(vab, q);
                    }
                    double a[U];
#pragma unroll
                    for (int k = 0; k < U; ++k) a[k] = (p0 + (uint32_t)(k * L) < oe) ? (double)raw[k] : 0.0;
                    double g[U];
#pragma unroll
                    for (int k = 0; k < U; ++k) g[k] = (double)ldo(g0, c[k]);
#pragma unroll
                    for (int k = 0; k < U; ++k) acc[0] += a[k] * g[k];
                    if constexpr (NR > 1) {
#pragma unroll
                        for (int k = 0; k < U; ++k) g[k] = (double)ldo(g1, c[k]);
#pragma unroll
                        for (int k = 0; k < U; ++k) acc[1] += a[k] * g[k];
                    }
                }
            }
        }
        if constexpr (L >= WG) {
            // wavefront reduce, then the four wavefront totals in LDS, fixed order
#pragma unroll
            for (int k = 0; k < NR; ++k) acc[k] = group_reduce<64, MAXABS>(acc[k]);
            const int wave = tid >> 6;
            if ((tid & 63) == 0) {
#pragma unroll
                for (int k = 0; k < NR; ++k) red_lds[k * 4 + wave] = acc[k];
            }
            __syncthreads();
            if (tid == 0) {
#pragma unroll
                for (int k = 0; k < NR; ++k) {
                    const double *r = red_lds + k * 4;
                    acc[k] = MAXABS ? fmax(fmax(r[0], r[1]), fmax(r[2], r[3]))
                                    : (r[0] + r[1]) + (r[2] + r[3]);
                }
            }
            __syncthreads();
        } else {
#pragma unroll
            for (int k = 0; k < NR; ++k) acc[k] = group_reduce<L, MAXABS>(acc[k]);
        }
    }

    // locate + dot; returns whether this lane leads a valid row.
    __device__ __forceinline__ static bool run(const OpDev &op, const Seg &s, int bi,
                                               const GV *__restrict__ g0, const GV *__restrict__ g1,
                                               const double *__restrict__ rowfac,
                                               double *red_lds, int64_t &row, double (&acc)[NR])
    {
        const Pos ps = locate(s, bi);
        row = ps.row;
        dot(op, ps, g0, g1, rowfac, red_lds, acc);
        return ps.leader;
    }
};

// Dispatch on the segment's lanes-per-row (uniform across the workgroup).
// F is called as f(std::integral_constant<int, L>{}).
template <int L>
struct LaneTag {
    static constexpr int value = L;
};

template <typename F>
__device__ __forceinline__ void dispatch_lanes(int lanes_log2, F &&f)
{
    switch (lanes_log2) {
        case 0: f(LaneTag<1>{}); break;
        case 1: f(LaneTag<2>{}); break;
        case 2: f(LaneTag<4>{}); break;
        case 3: f(LaneTag<8>{}); break;
        case 4: f(LaneTag<16>{}); break;
        case 5: f(LaneTag<32>{}); break;
        case 6: f(LaneTag<64>{}); break;
        default: f(LaneTag<WG>{}); break;
    }
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
