// capi.cpp -- the extern "C" surface of libpdhg (declared in include/pdhg.h):
// validation, layout planning (row reordering, row-length bins, CSR of K and
// K^T), workspace carving, setup on the GPU (Ruiz scaling, power iteration,
// step sizes), the restarted solve loop and the service calls.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include <stdlib.h>
#include <sys/mman.h>

#include "../../include/pdhg.h"
#include "kernels.h"
#include "pdhg_internal.h"

using namespace pdhg;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------

static thread_local std::string g_err;
static thread_local int g_err_code = PDHG_OK;

static int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    g_err_code = code;
    return code;
}

#define HIPCHK(call)                                                                        \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail(PDHG_ERR_HIP, "%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), \
                        __FILE__, __LINE__);                                                \
    } while (0)

extern "C" const char *pdhg_last_error(void) { return g_err.c_str(); }

extern "C" int pdhg_last_error_code(void) { return g_err_code; }

extern "C" void pdhg_default_opts(pdhg_opts *o)
{
    std::memset(o, 0, sizeof(*o));
    o->precision = PDHG_PREC_F32;
    o->ruiz_iters = 10;
    o->use_restarts = 1;
    o->use_pw_update = 1;
    o->check_every = 64;
    o->power_max_iters = 1000;
    o->max_iters = 1000000;
    o->eps = 1e-4;
    o->time_limit = 0.0;
    o->step_size = 0.0;
    o->step_frac = 0.9;
    o->primal_weight = 0.0;
    o->power_tol = 1e-6;
    o->beta_suff = 0.2;
    o->beta_nec = 0.8;
    o->beta_art = 0.36;
    o->eps_zero = 1e-6;
    o->unroll_capacity = 0;
    o->unroll_checkpoint = 50;
    o->use_graph = 1;
    o->xcd_remap = 1;
    o->max_grid = 8192;
    o->adaptive_step = 0;
    o->detect_infeas = 0;
    o->infeas_tol = 1e-4;
    o->fishnet_points = 0;
    o->batch_resident_bytes = 192000000;
    o->trace_capacity = 0;
    o->col_slices = 0;
    o->col_slices_t = 0;
}

// ---------------------------------------------------------------------------
// host view of one input LP (downloaded when it lives on the device)
// ---------------------------------------------------------------------------

struct HostLP {
    int64_t n = 0, m = 0, nnz = 0, m1 = 0;
    const int64_t *rp = nullptr;
    const int32_t *ci = nullptr;
    const double *v = nullptr, *c = nullptr, *rhs = nullptr, *l = nullptr, *u = nullptr;
    const uint8_t *rt = nullptr;
    std::vector<int64_t> rp_s;
    std::vector<int32_t> ci_s;
    std::vector<double> v_s, c_s, rhs_s, l_s, u_s;
    std::vector<uint8_t> rt_s;
};

template <typename X>
static int fetch(const X *src, size_t cnt, int mem, std::vector<X> &store, const X *&view)
{
    if (cnt == 0) {
        view = nullptr;
        return PDHG_OK;
    }
    if (!src) return fail(PDHG_ERR_INVALID_ARG, "NULL input array");
    if (mem == PDHG_MEM_HOST) {
        view = src;
        return PDHG_OK;
    }
    store.resize(cnt);
    HIPCHK(hipMemcpy(store.data(), src, cnt * sizeof(X), hipMemcpyDeviceToHost));
    view = store.data();
    return PDHG_OK;
}

// pattern_only: only row_ptr / col / row_type (for sizing)
static int load_lp(const pdhg_lp &in, HostLP &h, bool pattern_only)
{
    if (in.n < 1 || in.m < 0 || in.nnz < 0)
        return fail(PDHG_ERR_SHAPE, "need n >= 1, m >= 0, nnz >= 0 (got n=%lld m=%lld nnz=%lld)",
                    (long long)in.n, (long long)in.m, (long long)in.nnz);
    if (in.mem != PDHG_MEM_HOST && in.mem != PDHG_MEM_DEVICE)
        return fail(PDHG_ERR_INVALID_ARG, "mem must be PDHG_MEM_HOST or PDHG_MEM_DEVICE");
    if (in.n >= INT32_MAX || in.m >= INT32_MAX) return fail(PDHG_ERR_SHAPE, "n and m must be < 2^31");
    h.n = in.n;
    h.m = in.m;
    h.nnz = in.nnz;
    int rc;
    if (!in.row_ptr) return fail(PDHG_ERR_INVALID_ARG, "row_ptr is NULL");
    if ((rc = fetch(in.row_ptr, (size_t)in.m + 1, in.mem, h.rp_s, h.rp))) return rc;
    if ((rc = fetch(in.col, (size_t)in.nnz, in.mem, h.ci_s, h.ci))) return rc;
    if (in.row_type && (rc = fetch(in.row_type, (size_t)in.m, in.mem, h.rt_s, h.rt))) return rc;
    if (!in.row_type) h.rt = nullptr;
    if (h.rp[0] != 0 || h.rp[in.m] != in.nnz)
        return fail(PDHG_ERR_SHAPE, "row_ptr[0] must be 0 and row_ptr[m] must equal nnz");
    for (int64_t i = 0; i < in.m; ++i)
        if (h.rp[i + 1] < h.rp[i]) return fail(PDHG_ERR_SHAPE, "row_ptr not monotone at row %lld", (long long)i);
    for (int64_t k = 0; k < in.nnz; ++k)
        if (h.ci[k] < 0 || h.ci[k] >= in.n)
            return fail(PDHG_ERR_SHAPE, "column index %d out of range at entry %lld", h.ci[k], (long long)k);
    h.m1 = 0;
    for (int64_t i = 0; i < in.m; ++i) {
        const uint8_t t = h.rt ? h.rt[i] : (uint8_t)PDHG_ROW_EQ;
        if (t != PDHG_ROW_GE && t != PDHG_ROW_EQ) return fail(PDHG_ERR_INVALID_ARG, "bad row_type at row %lld", (long long)i);
        h.m1 += (t == PDHG_ROW_GE);
    }
    if (pattern_only) return PDHG_OK;
    if ((rc = fetch(in.val, (size_t)in.nnz, in.mem, h.v_s, h.v))) return rc;
    if ((rc = fetch(in.c, (size_t)in.n, in.mem, h.c_s, h.c))) return rc;
    if ((rc = fetch(in.rhs, (size_t)in.m, in.mem, h.rhs_s, h.rhs))) return rc;
    if ((rc = fetch(in.l, (size_t)in.n, in.mem, h.l_s, h.l))) return rc;
    if ((rc = fetch(in.u, (size_t)in.n, in.mem, h.u_s, h.u))) return rc;
    for (int64_t k = 0; k < in.nnz; ++k)
        if (!std::isfinite(h.v[k])) return fail(PDHG_ERR_NONFINITE, "matrix value %lld is not finite", (long long)k);
    for (int64_t j = 0; j < in.n; ++j) {
        if (!std::isfinite(h.c[j])) return fail(PDHG_ERR_NONFINITE, "c[%lld] is not finite", (long long)j);
        if (std::isnan(h.l[j]) || std::isnan(h.u[j])) return fail(PDHG_ERR_NONFINITE, "bound %lld is NaN", (long long)j);
        if (h.l[j] > h.u[j] || h.l[j] == INFINITY || h.u[j] == -INFINITY)
            return fail(PDHG_ERR_BOUNDS, "inconsistent bounds at variable %lld", (long long)j);
    }
    for (int64_t i = 0; i < in.m; ++i)
        if (!std::isfinite(h.rhs[i])) return fail(PDHG_ERR_NONFINITE, "rhs[%lld] is not finite", (long long)i);
    return PDHG_OK;
}

// ---------------------------------------------------------------------------
// layout planning
// ---------------------------------------------------------------------------

struct SegH {
    int64_t row0;  // local row within the instance's internal order
    int32_t nrows, lanes_log2, ineq;
    int32_t sliced = 0;  // rows swept in column slices (dual operator)
};

// rows of K (of K^T) swept in column slices: at least SLICE_MIN (SLICE_MIN_T)
// entries per slice on average
constexpr int64_t SLICE_MIN = 16, SLICE_MIN_T = 16;
static bool row_sliced(int64_t len, int S) { return S > 1 && len >= SLICE_MIN * S; }
static bool row_sliced_t(int64_t len, int S) { return S > 1 && len >= SLICE_MIN_T * S; }

struct InstPlan {
    int64_t n, m, m1, nnz;
    std::vector<int32_t> row_order;  // internal row -> caller row
    std::vector<int32_t> col_order;  // internal col -> caller col
    std::vector<SegH> segK, segT;
};

struct Bins {
    int32_t max_len[NBIN];
    int32_t code[NBIN];  // lanes_log2 | rows_log2 << 4
};

// lim: row-length limits; rows: rows per lane group (1, 2, 4; only for bins
// of at most 16 lanes)
static Bins make_bins(const int32_t *lim, const int32_t *rows)
{
    static const int32_t def_len[NBIN] = {4, 8, 16, 32, 64, 128, 512, INT32_MAX};
    static const int32_t lanes[NBIN] = {0, 1, 2, 3, 4, 5, 6, 8};
    Bins b;
    for (int k = 0; k < NBIN; ++k) {
        b.max_len[k] = (lim && lim[k] > 0) ? lim[k] : def_len[k];
        if (k > 0 && b.max_len[k] < b.max_len[k - 1]) b.max_len[k] = b.max_len[k - 1];
        int rl = 0;
        if (rows && k <= 4) rl = rows[k] >= 4 ? 2 : (rows[k] >= 2 ? 1 : 0);
        b.code[k] = lanes[k] | (rl << 4);
    }
    b.max_len[NBIN - 1] = INT32_MAX;
    return b;
}

static int bin_of(const Bins &b, int64_t len)
{
    for (int k = 0; k < NBIN; ++k)
        if (len <= b.max_len[k]) return k;
    return NBIN - 1;
}

// rows per logical block of a segment with this lanes / rows code
static int seg_group(int code)
{
    const int lanes_log2 = code & 15, rows_log2 = (code >> 4) & 3;
    return (lanes_log2 >= 8 ? 1 : (WG >> lanes_log2)) << rows_log2;
}

static void plan_instance(const HostLP &h, const Bins &bins, const Bins &tbins, int S, int St, InstPlan &p)
{
    p.n = h.n;
    p.m = h.m;
    p.m1 = h.m1;
    p.nnz = h.nnz;
    // rows: ">=" group then "=" group, each split into whole rows and rows
    // swept in S column slices (binned by their per-slice length), each
    // ordered by bin, stable
    std::vector<std::vector<int32_t>> buck(4 * NBIN);
    for (int64_t i = 0; i < h.m; ++i) {
        const int eq = h.rt ? (h.rt[i] == PDHG_ROW_EQ) : 1;
        const int64_t len = h.rp[i + 1] - h.rp[i];
        const int sl = row_sliced(len, S) ? 1 : 0;
        const int64_t blen = sl ? (len + S - 1) / S : len;
        buck[(2 * eq + sl) * NBIN + bin_of(bins, blen)].push_back((int32_t)i);
    }
    p.row_order.clear();
    p.row_order.reserve(h.m);
    p.segK.clear();
    for (int g = 0; g < 4; ++g)
        for (int b = 0; b < NBIN; ++b) {
            auto &v = buck[g * NBIN + b];
            if (v.empty()) continue;
            SegH sh{(int64_t)p.row_order.size(), (int32_t)v.size(), bins.code[b], g < 2};
            sh.sliced = g & 1;
            p.segK.push_back(sh);
            p.row_order.insert(p.row_order.end(), v.begin(), v.end());
        }
    // columns: whole rows of K^T, then rows swept in St slices (binned by
    // their per-slice count), each ordered by bin of their entry count, stable
    std::vector<int64_t> cnt(h.n, 0);
    for (int64_t k = 0; k < h.nnz; ++k) cnt[h.ci[k]]++;
    std::vector<std::vector<int32_t>> cb(2 * NBIN);
    for (int64_t j = 0; j < h.n; ++j) {
        const int sl = row_sliced_t(cnt[j], St) ? 1 : 0;
        cb[sl * NBIN + bin_of(tbins, sl ? (cnt[j] + St - 1) / St : cnt[j])].push_back((int32_t)j);
    }
    p.col_order.clear();
    p.col_order.reserve(h.n);
    p.segT.clear();
    for (int g = 0; g < 2; ++g)
        for (int b = 0; b < NBIN; ++b) {
            auto &v = cb[g * NBIN + b];
            if (v.empty()) continue;
            SegH sh{(int64_t)p.col_order.size(), (int32_t)v.size(), tbins.code[b], 0};
            sh.sliced = g;
            p.segT.push_back(sh);
            p.col_order.insert(p.col_order.end(), v.begin(), v.end());
        }
}

// ---------------------------------------------------------------------------
// workspace carving
// ---------------------------------------------------------------------------

struct Carve {
    size_t off = 0;
    char *base = nullptr;
    template <typename X>
    X *take(size_t cnt)
    {
        off = (off + 255) & ~(size_t)255;
        X *p = base ? (X *)(base + off) : nullptr;
        off += cnt * sizeof(X);
        return p;
    }
};

struct Sizes {
    int64_t N = 0, M = 0, NNZ = 0;
    int64_t nsegK = 0, nsegT = 0, nblkK = 0, nblkT = 0, nl2 = 0;
    int32_t batch = 0;
};

struct Buffers {
    // operators
    int64_t *Krp, *Ktrp;
    int32_t *Kci, *Ktci, *Kbs, *Ktbs;
    double *Kv64, *Ktv64;
    float *Kv32, *Ktv32;
    Seg *Kseg, *Ktseg;
    int4 *Kbd, *Ktbd;
    // record / adjoint
    void *ckx, *cky;
    uint8_t *maskx, *masky;
    double *ax, *ay, *aw, *av, *axb, *ac, *al, *au, *aq;
    double *vecN64c;
    int32_t *l2inst;
    int64_t *bcumK, *bcumT;  // block cost prefix sums
    int32_t *Ksb, *Ktsb;     // column-slice starts of every row of K / K^T (col_slices(_t) > 1)
    double *Kpart, *Ktpart;  // FP64 partial products of the sliced rows
};

struct pdhg_handle {
    int32_t batch = 0;
    int32_t prec = PDHG_PREC_F32;
    pdhg_opts opts{};
    Sizes sz;
    Dev d{};
    Buffers buf{};
    std::vector<InstInfo> info;
    std::vector<InstState> st0;  // per-instance parameters after setup
    std::vector<InstPlan> plan;
    std::vector<int32_t> sol_avg;  // returned point of the last solve
    std::vector<double> knorm;
    int32_t *hdone_host = nullptr;
    size_t ws_bytes = 0;
    double setup_seconds = 0;
    double setup_phase[5] = {0, 0, 0, 0, 0};  // plan, host images, copies, device, power iteration
    hipGraphExec_t graph = nullptr;
    hipStream_t cap_stream = nullptr;
    FishDev fish{};          // fishnet buffers (opts.fishnet_points > 0)
    bool fish_rows = false;  // fish.rowK / rowT hold the rows by decreasing length
    int32_t noalloc_dev = -1;         // device whose fixed workspace holds this handle (pdhg_setup_noalloc)
    void *noalloc_owner = nullptr;    // its claim on that workspace
    int64_t rec_steps = 0;  // steps recorded by the last recording pdhg_iterate
    int rec_valid = 0;      // the tape matches the handle's data (cleared by pdhg_set_data)
    int64_t rec_gen = 0;    // bumped by every recording pdhg_iterate and by pdhg_set_data
    std::vector<InstState> rec_st;  // step parameters of the recorded steps
};

static size_t elem_size(int prec) { return prec == PDHG_PREC_F64 ? sizeof(double) : sizeof(float); }

static int ilog2(int v)
{
    int r = 0;
    while ((1 << (r + 1)) <= v) ++r;
    return r;
}

static void carve(Carve &cv, const Sizes &sz, int prec, const pdhg_opts &o, Dev &d, Buffers &b,
                  InstInfo **info, InstState **st, FishDev *fish)
{
    const size_t es = elem_size(prec);
    const int64_t N = sz.N, M = sz.M, NNZ = sz.NNZ;
    b.Krp = cv.take<int64_t>(M + 1);
    b.Kci = cv.take<int32_t>(NNZ);
    b.Kv64 = cv.take<double>(NNZ);
    b.Kv32 = prec == PDHG_PREC_F32 ? cv.take<float>(NNZ) : nullptr;
    b.Kseg = cv.take<Seg>(sz.nsegK);
    b.Kbs = cv.take<int32_t>(sz.nblkK);
    b.Kbd = cv.take<int4>(sz.nblkK);
    b.Ktrp = cv.take<int64_t>(N + 1);
    b.Ktci = cv.take<int32_t>(NNZ);
    b.Ktv64 = cv.take<double>(NNZ);
    b.Ktv32 = prec == PDHG_PREC_F32 ? cv.take<float>(NNZ) : nullptr;
    b.Ktseg = cv.take<Seg>(sz.nsegT);
    b.Ktbs = cv.take<int32_t>(sz.nblkT);
    b.Ktbd = cv.take<int4>(sz.nblkT);
    d.x = cv.take<char>(N * es);
    d.xbar = cv.take<char>(N * es);
    d.xavg = cv.take<char>(N * es);
    d.x0 = cv.take<char>(N * es);
    d.c = cv.take<char>(N * es);
    d.l = cv.take<char>(N * es);
    d.u = cv.take<char>(N * es);
    d.c64 = cv.take<double>(N);
    d.l64 = cv.take<double>(N);
    d.u64 = cv.take<double>(N);
    d.kap = cv.take<double>(N);
    d.craw = cv.take<double>(N);
    d.lraw = cv.take<double>(N);
    d.uraw = cv.take<double>(N);
    d.col_orig = cv.take<int32_t>(N);
    d.inst_of_col = cv.take<int32_t>(N);
    d.y = cv.take<char>(M * es);
    d.yavg = cv.take<char>(M * es);
    d.y0 = cv.take<char>(M * es);
    d.q = cv.take<char>(M * es);
    d.q64 = cv.take<double>(M);
    d.rho = cv.take<double>(M);
    d.qraw = cv.take<double>(M);
    d.row_orig = cv.take<int32_t>(M);
    d.inst_of_row = cv.take<int32_t>(M);
    *info = cv.take<InstInfo>(sz.batch);
    *st = cv.take<InstState>(sz.batch);
    d.partials = cv.take<double>((size_t)(sz.nblkK + sz.nblkT) * NPART + 1);
    d.partials2 = cv.take<double>((size_t)sz.nl2 * NPART + 1);
    d.adp = cv.take<double>(2 * (size_t)sz.nblkK + sz.nblkT + 1);
    // second buffers of the adaptive step size
    d.xavg1 = cv.take<char>(N * es);
    d.y1 = cv.take<char>(M * es);
    d.yavg1 = cv.take<char>(M * es);
    d.kx0 = cv.take<double>(M);
    d.kx1 = cv.take<double>(M);
    d.xam = cv.take<char>(N * es);
    d.yam = cv.take<char>(M * es);
    const int S = o.col_slices > 1 ? o.col_slices : 1, St = o.col_slices_t > 1 ? o.col_slices_t : 1;
    b.Ksb = S > 1 ? cv.take<int32_t>((size_t)M * (S - 1)) : nullptr;
    // the sweeps' partials (M), and the solve-time check's for its two
    // candidates (2 M, the first M shared: the check runs between chunks)
    b.Kpart = S > 1 ? cv.take<double>(2 * (size_t)M) : nullptr;
    b.Ktsb = St > 1 ? cv.take<int32_t>((size_t)N * (St - 1)) : nullptr;
    b.Ktpart = St > 1 ? cv.take<double>(N) : nullptr;
    d.actK = cv.take<int32_t>(sz.nblkK + 1);
    d.actT = cv.take<int32_t>(sz.nblkT + 1);
    d.act_cnt = cv.take<int32_t>(2);
    d.act_off = cv.take<int32_t>(2 * (size_t)sz.batch);
    d.act_coff = cv.take<int64_t>(2 * (size_t)sz.batch + 2);
    d.act_split = cv.take<int32_t>(18);
    d.adm_order = cv.take<int32_t>(sz.batch);
    d.trace_cap = o.trace_capacity;
    d.trace = o.trace_capacity > 0 ? cv.take<pdhg_trace_rec>((size_t)sz.batch * o.trace_capacity) : nullptr;
    b.bcumK = cv.take<int64_t>(sz.nblkK + 1);
    b.bcumT = cv.take<int64_t>(sz.nblkT + 1);
    b.l2inst = cv.take<int32_t>(sz.nl2 + 1);
    d.vecN64 = cv.take<double>(N);
    d.vecN64b = cv.take<double>(N);
    b.vecN64c = cv.take<double>(N);
    d.vecM64 = cv.take<double>(M);
    d.vecM64b = cv.take<double>(M);
    d.inst_scratch = cv.take<double>((size_t)sz.batch * 16 + 16);
    // fishnet casting: PS interleaved points
    if (o.fishnet_points > 0) {
        const int64_t PS = o.fishnet_points;
        fish->PS = (int32_t)PS;
        fish->nrec = 2 * ilog2((int)PS);
        fish->X = cv.take<char>(N * PS * es);
        fish->XB = cv.take<char>(N * PS * es);
        fish->X2 = cv.take<char>(N * PS * es);
        fish->Y = cv.take<char>(M * PS * es);
        fish->Y2 = cv.take<char>(M * PS * es);
        fish->rowK = cv.take<int32_t>(M + 1);
        fish->rowT = cv.take<int32_t>(N + 1);
        const int64_t chunks = NNZ / FISH_CHUNK + 1;
        fish->taskK = cv.take<int4>(M + chunks + 1);
        fish->taskT = cv.take<int4>(N + chunks + 1);
        fish->splitK = cv.take<int4>(std::min<int64_t>(M, chunks) + 1);
        fish->splitT = cv.take<int4>(std::min<int64_t>(N, chunks) + 1);
        fish->cpart = cv.take<double>((2 * chunks + 2) * PS);
        fish->part = cv.take<double>((size_t)FISH_GRID * PS);
        fish->wmat = cv.take<double>((size_t)(PS / 2) * (PS / 2) + 1);
        fish->keep = cv.take<int32_t>(PS);
        fish->gstage = cv.take<double>(N * PS + 1);
        fish->wstage = cv.take<double>(PS * PS);
        fish->rec_gaps = cv.take<double>((size_t)fish->nrec * PS);
        fish->rec_keep = cv.take<int32_t>((size_t)fish->nrec * PS);
    }
    // adjoint of unrolled steps
    if (o.unroll_capacity > 0) {
        const int64_t C = std::max(1, o.unroll_checkpoint);
        const int64_t nck = (o.unroll_capacity + C - 1) / C + 1;
        b.ckx = cv.take<char>(nck * N * es);
        b.cky = cv.take<char>(nck * M * es);
        b.maskx = cv.take<uint8_t>(C * N);
        b.masky = cv.take<uint8_t>(C * M);
        b.ax = cv.take<double>(N);
        b.av = cv.take<double>(N);
        b.axb = cv.take<double>(N);
        b.ac = cv.take<double>(N);
        b.al = cv.take<double>(N);
        b.au = cv.take<double>(N);
        b.ay = cv.take<double>(M);
        b.aw = cv.take<double>(M);
        b.aq = cv.take<double>(M);
    }
}

static int check_opts(const pdhg_opts *o)
{
    if (o->precision != PDHG_PREC_F32 && o->precision != PDHG_PREC_F64)
        return fail(PDHG_ERR_INVALID_ARG, "precision must be PDHG_PREC_F32 or PDHG_PREC_F64");
    if (o->check_every < 1 || o->check_every > 4096) return fail(PDHG_ERR_INVALID_ARG, "check_every must be in 1..4096");
    if (o->ruiz_iters < 0 || o->power_max_iters < 1) return fail(PDHG_ERR_INVALID_ARG, "bad ruiz/power iteration count");
    if (!(o->eps > 0.0)) return fail(PDHG_ERR_INVALID_ARG, "eps must be > 0");
    if (o->max_iters < 1) return fail(PDHG_ERR_INVALID_ARG, "max_iters must be >= 1");
    if (o->unroll_capacity < 0 || (o->unroll_capacity > 0 && o->unroll_checkpoint < 1))
        return fail(PDHG_ERR_INVALID_ARG, "bad unroll capacity / checkpoint");
    if (!(o->step_frac > 0.0) && !(o->step_size > 0.0)) return fail(PDHG_ERR_INVALID_ARG, "step_frac must be > 0");
    if (o->adaptive_step != 0 && o->adaptive_step != 1) return fail(PDHG_ERR_INVALID_ARG, "adaptive_step must be 0 or 1");
    if (o->detect_infeas != 0 && o->detect_infeas != 1) return fail(PDHG_ERR_INVALID_ARG, "detect_infeas must be 0 or 1");
    if (o->detect_infeas && !(o->infeas_tol > 0.0)) return fail(PDHG_ERR_INVALID_ARG, "infeas_tol must be > 0");
    if (o->fishnet_points != 0 &&
        (o->fishnet_points < 2 || o->fishnet_points > 64 || (o->fishnet_points & (o->fishnet_points - 1))))
        return fail(PDHG_ERR_INVALID_ARG, "fishnet_points must be 0 or a power of two in 2..64");
    if (o->batch_resident_bytes < 0) return fail(PDHG_ERR_INVALID_ARG, "batch_resident_bytes must be >= 0");
    for (int k = 0; k < NBIN; ++k) {
        const int32_t rd = o->bin_rows_dual[k], rp = o->bin_rows_primal[k];
        const bool ok = k <= 4 ? (rd == 0 || rd == 1 || rd == 2 || rd == 4) && (rp == 0 || rp == 1 || rp == 2 || rp == 4)
                               : (rd == 0 || rd == 1) && (rp == 0 || rp == 1);
        if (!ok)
            return fail(PDHG_ERR_INVALID_ARG, "bin_rows[%d] must be %s", k, k <= 4 ? "0, 1, 2 or 4" : "0 or 1");
        if (o->bin_len_dual[k] < 0 || o->bin_len_primal[k] < 0)
            return fail(PDHG_ERR_INVALID_ARG, "bin_len[%d] must be >= 0", k);
    }
    if (o->col_slices < 0 || o->col_slices > 16 || o->col_slices_t < 0 || o->col_slices_t > 16)
        return fail(PDHG_ERR_INVALID_ARG, "col_slices and col_slices_t must be in 0..16");
    if (o->trace_capacity < 0 || o->trace_capacity > (1 << 20))
        return fail(PDHG_ERR_INVALID_ARG, "trace_capacity must be in 0..2^20");
    return PDHG_OK;
}

// Host vectors whose elements are all written before use: no zero fill (the
// matrix images run to hundreds of MB, and the fill would be a full pass).
// Large ones sit on 2 MB-aligned memory marked for transparent huge pages, so
// the first touch faults in 2 MB steps rather than 4 KB ones.
template <typename T>
struct NoInitAlloc : std::allocator<T> {
    template <typename U>
    struct rebind {
        using other = NoInitAlloc<U>;
    };
    NoInitAlloc() = default;
    template <typename U>
    NoInitAlloc(const NoInitAlloc<U> &) noexcept
    {
    }
    static constexpr size_t HUGE_MIN = (size_t)8 << 20, HUGE_ALIGN = (size_t)2 << 20;
    T *allocate(size_t n)
    {
        const size_t bytes = n * sizeof(T);
        if (bytes < HUGE_MIN) return std::allocator<T>::allocate(n);
        void *p = nullptr;
        if (posix_memalign(&p, HUGE_ALIGN, (bytes + HUGE_ALIGN - 1) & ~(HUGE_ALIGN - 1)) != 0 || !p)
            throw std::bad_alloc();
        (void)madvise(p, (bytes + HUGE_ALIGN - 1) & ~(HUGE_ALIGN - 1), MADV_HUGEPAGE);
        return (T *)p;
    }
    void deallocate(T *p, size_t n)
    {
        if (n * sizeof(T) < HUGE_MIN) {
            std::allocator<T>::deallocate(p, n);
            return;
        }
        free(p);
    }
    template <typename U>
    void construct(U *) noexcept
    {
    }
    template <typename U, typename... A>
    void construct(U *p, A &&...a)
    {
        ::new ((void *)p) U(std::forward<A>(a)...);
    }
};
template <typename T>
using hvec = std::vector<T, NoInitAlloc<T>>;

// Host threads for setup work: the machine's, at most 16.
static int host_threads()
{
    const unsigned hc = std::thread::hardware_concurrency();
    return (int)std::max(1u, std::min(16u, hc ? hc : 1u));
}

// f(t, begin, end) on T contiguous ranges of [0, n) (T = 1 below `grain`
// items per thread), each on its own thread; returns when all are done.  f
// must not throw (it runs on threads of its own).
template <typename F>
static void parallel_ranges(int64_t n, int64_t grain, int T, F &&f)
{
    T = (int)std::max<int64_t>(1, std::min<int64_t>(T, n / std::max<int64_t>(1, grain)));
    if (T <= 1) {
        f(0, (int64_t)0, n);
        return;
    }
    std::vector<std::thread> th;
    th.reserve(T);
    for (int t = 0; t < T; ++t) {
        try {
            th.emplace_back(f, t, n * t / T, n * (t + 1) / T);
        } catch (...) {
            f(t, n * t / T, n * (t + 1) / T);  // no thread to spare: run the range here
        }
    }
    for (auto &x : th) x.join();
}

// f(i) for every i in [0, n) on up to T threads, items handed out in order
// as threads become free.  f must not throw.
template <typename F>
static void parallel_items(int64_t n, int T, F &&f)
{
    std::atomic<int64_t> next{0};
    parallel_ranges(std::min<int64_t>(T, n), 1, T, [&](int, int64_t, int64_t) {
        for (;;) {
            const int64_t i = next.fetch_add(1);
            if (i >= n) break;
            f(i);
        }
    });
}

static int plan_all(const pdhg_lp *lp, int32_t batch, const pdhg_opts *o, std::vector<HostLP> &hosts,
                    std::vector<InstPlan> &plans, Sizes &sz, bool pattern_only)
{
    if (!lp || batch < 1) return fail(PDHG_ERR_INVALID_ARG, "need lp != NULL and batch >= 1");
    int rc = check_opts(o);
    if (rc) return rc;
    hosts.resize(batch);
    plans.resize(batch);
    const Bins bins = make_bins(o->bin_len_dual, o->bin_rows_dual);
    const Bins tbins = make_bins(o->bin_len_primal, o->bin_rows_primal);
    sz = Sizes{};
    sz.batch = batch;
    // validation and binning of each instance: on host threads, one
    // instance at a time each, when every instance is in host memory
    // (device inputs are copied with the caller's current device)
    bool all_host = true;
    for (int b = 0; b < batch; ++b) all_host = all_host && lp[b].mem == PDHG_MEM_HOST;
    std::vector<int> rcs(batch, PDHG_OK);
    std::vector<std::string> msgs(batch);
    auto plan_one = [&](int64_t b) {
        try {
            rcs[b] = load_lp(lp[b], hosts[b], pattern_only);
            if (rcs[b]) {
                msgs[b] = g_err;  // the message is per thread
                return;
            }
            plan_instance(hosts[b], bins, tbins, o->col_slices, o->col_slices_t, plans[b]);
        } catch (...) {
            rcs[b] = PDHG_ERR_NOMEM;
            msgs[b] = "host memory exhausted";
        }
    };
    if (all_host && batch > 1)
        parallel_items(batch, host_threads(), plan_one);
    else
        for (int b = 0; b < batch; ++b) plan_one(b);
    for (int b = 0; b < batch; ++b)
        if (rcs[b]) return batch > 1 ? fail(rcs[b], "instance %d: %s", b, msgs[b].c_str()) : fail(rcs[b], "%s", msgs[b].c_str());
    for (int b = 0; b < batch; ++b) {
        sz.N += hosts[b].n;
        sz.M += hosts[b].m;
        sz.NNZ += hosts[b].nnz;
        int64_t pb = 0;
        for (auto &s : plans[b].segK) pb += (s.nrows + seg_group(s.lanes_log2) - 1) / seg_group(s.lanes_log2);
        sz.nblkK += pb;
        int64_t pt = 0;
        for (auto &s : plans[b].segT) pt += (s.nrows + seg_group(s.lanes_log2) - 1) / seg_group(s.lanes_log2);
        sz.nblkT += pt;
        sz.nl2 += (pb + pt + L2CH - 1) / L2CH;
        sz.nsegK += plans[b].segK.size();
        sz.nsegT += plans[b].segT.size();
    }
    // sweeps address the gathered vectors with 32-bit byte offsets
    if (sz.N >= (int64_t(1) << 29) || sz.M >= (int64_t(1) << 29))
        return fail(PDHG_ERR_SHAPE, "total n and m over the batch must be < 2^29");
    if (sz.nblkK + sz.nblkT >= INT32_MAX) return fail(PDHG_ERR_SHAPE, "too many workgroups");
    return PDHG_OK;
}

static size_t workspace_bytes_impl(const pdhg_lp *lp, int32_t batch, const pdhg_opts *o)
{
    pdhg_opts def;
    if (!o) {
        pdhg_default_opts(&def);
        o = &def;
    }
    std::vector<HostLP> hosts;
    std::vector<InstPlan> plans;
    Sizes sz;
    if (plan_all(lp, batch, o, hosts, plans, sz, false)) return 0;
    Carve cv;
    Dev d{};
    Buffers b{};
    InstInfo *info;
    InstState *st;
    FishDev fish{};
    carve(cv, sz, o->precision, *o, d, b, &info, &st, &fish);
    return (cv.off + 255) & ~(size_t)255;
}

extern "C" size_t pdhg_workspace_bytes(const pdhg_lp *lp, int32_t batch, const pdhg_opts *o)
{
    try {
        return workspace_bytes_impl(lp, batch, o);
    } catch (...) {
        fail(PDHG_ERR_NOMEM, "sizing: host memory exhausted");
        return 0;
    }
}

// ---------------------------------------------------------------------------
// setup
// ---------------------------------------------------------------------------

template <typename X>
static int h2d(X *dst, const X *src, size_t cnt, hipStream_t s)
{
    if (cnt) HIPCHK(hipMemcpyAsync(dst, src, cnt * sizeof(X), hipMemcpyHostToDevice, s));
    return PDHG_OK;
}

// builds the host images of both operators and all vectors, then uploads
static int upload(pdhg_handle *h, std::vector<HostLP> &hosts, hipStream_t s)
{
    const auto t_up = std::chrono::steady_clock::now();
    const Sizes &sz = h->sz;
    Buffers &b = h->buf;
    Dev &d = h->d;
    hvec<int64_t> Krp(sz.M + 1), Ktrp(sz.N + 1);
    hvec<int32_t> Kci(sz.NNZ), Ktci(sz.NNZ);
    std::vector<int32_t> Kbs(sz.nblkK), Ktbs(sz.nblkT);
    std::vector<int4> Kbd(sz.nblkK), Ktbd(sz.nblkT);
    hvec<double> Kv(sz.NNZ), Ktv(sz.NNZ);
    const int S = h->opts.col_slices > 1 ? h->opts.col_slices : 1;
    const int St = h->opts.col_slices_t > 1 ? h->opts.col_slices_t : 1;
    hvec<int32_t> Ksb(S > 1 ? (size_t)sz.M * (S - 1) : 0), Ktsb(St > 1 ? (size_t)sz.N * (St - 1) : 0);
    const int HT = host_threads();
    std::vector<Seg> Kseg, Ktseg;
    std::vector<int32_t> l2inst;
    std::vector<double> craw(sz.N), lraw(sz.N), uraw(sz.N), qraw(sz.M);
    std::vector<int32_t> col_orig(sz.N), row_orig(sz.M), inst_col(sz.N), inst_row(sz.M);
    h->info.assign(h->batch, InstInfo{});
    // offsets of every instance in the concatenated vectors and operators
    std::vector<int64_t> xo(h->batch + 1, 0), yo(h->batch + 1, 0), zo(h->batch + 1, 0);
    for (int bi = 0; bi < h->batch; ++bi) {
        xo[bi + 1] = xo[bi] + h->plan[bi].n;
        yo[bi + 1] = yo[bi] + h->plan[bi].m;
        zo[bi + 1] = zo[bi] + h->plan[bi].nnz;
    }
    // the row pointers at instance boundaries, written here: an instance's
    // build writes only the pointers strictly inside its range
    for (int bi = 0; bi <= h->batch; ++bi) {
        Krp[yo[bi]] = zo[bi];
        Ktrp[xo[bi]] = zo[bi];
    }
    // each instance's part of the images depends on no other instance: one
    // instance uses every thread; a batch gives each thread whole instances,
    // largest first
    auto build_inst = [&](int bi, int HT) {
        const HostLP &lp = hosts[bi];
        const InstPlan &p = h->plan[bi];
        InstInfo &in = h->info[bi];
        const int64_t xoff = xo[bi], yoff = yo[bi], nzoff = zo[bi];
        in.xoff = xoff;
        in.yoff = yoff;
        in.n = (int32_t)p.n;
        in.m = (int32_t)p.m;
        in.m1 = (int32_t)p.m1;
        std::vector<int32_t> col_new(p.n);
        for (int64_t j = 0; j < p.n; ++j) col_new[p.col_order[j]] = (int32_t)j;
        // K rows in internal order, global column index: row pointers by a
        // scan, then the entries on HT threads over ranges of rows
        {
            int64_t acc = nzoff;
            for (int64_t i = 0; i + 1 < p.m; ++i) {
                const int32_t r = p.row_order[i];
                acc += lp.rp[r + 1] - lp.rp[r];
                Krp[yoff + i + 1] = acc;
            }
        }
        const int64_t pos = zo[bi + 1];
        // a row swept in S column slices lists its entries slice by slice
        // (internal columns [s W, (s + 1) W), W = ceil(n / S); caller order
        // within a slice) and records where slices 1 .. S-1 begin
        const int64_t W = S > 1 ? std::max<int64_t>(1, (p.n + S - 1) / S) : 1;
        parallel_ranges(p.m, 4096, HT, [&](int, int64_t i0, int64_t i1) {
            std::vector<int64_t> cnt(S + 1);
            for (int64_t i = i0; i < i1; ++i) {
                const int32_t r = p.row_order[i];
                int64_t q = Krp[yoff + i];
                const int64_t len = lp.rp[r + 1] - lp.rp[r];
                if (row_sliced(len, S)) {
                    std::fill(cnt.begin(), cnt.end(), 0);
                    for (int64_t k = lp.rp[r]; k < lp.rp[r + 1]; ++k) cnt[1 + col_new[lp.ci[k]] / W]++;
                    for (int t = 1; t <= S; ++t) cnt[t] += cnt[t - 1];
                    for (int t = 1; t < S; ++t) Ksb[(size_t)(yoff + i) * (S - 1) + (t - 1)] = (int32_t)cnt[t];
                    for (int64_t k = lp.rp[r]; k < lp.rp[r + 1]; ++k) {
                        const int64_t dst = q + cnt[col_new[lp.ci[k]] / W]++;
                        Kci[dst] = (int32_t)(xoff + col_new[lp.ci[k]]);
                        Kv[dst] = lp.v[k];
                    }
                } else {
                    for (int t = 1; t < S; ++t) Ksb[(size_t)(yoff + i) * (S - 1) + (t - 1)] = 0;
                    for (int64_t k = lp.rp[r]; k < lp.rp[r + 1]; ++k, ++q) {
                        Kci[q] = (int32_t)(xoff + col_new[lp.ci[k]]);
                        Kv[q] = lp.v[k];
                    }
                }
                row_orig[yoff + i] = r;
                inst_row[yoff + i] = bi;
                qraw[yoff + i] = lp.rhs[r];
            }
        });
        // K^T by a stable counting sort over the internal rows of K.  Column
        // counts: per-thread histograms over ranges of rows, summed.  Entries:
        // thread t owns a range of columns holding about 1/T of the entries,
        // scans K in row order and places only its own columns' entries, so
        // every column lists its rows in increasing order and no two threads
        // write the same cache lines.
        {
            const int64_t nzi = pos - nzoff;
            int TT = (int)std::max<int64_t>(1, std::min<int64_t>(HT, nzi / (1 << 18)));
            while (TT > 1 && (int64_t)TT * (p.n + 1) > ((int64_t)1 << 26)) --TT;  // <= 512 MB of counters
            std::vector<int64_t> hist((size_t)TT * p.n, 0);
            parallel_ranges(TT, 1, TT, [&](int, int64_t t0, int64_t t1) {
                for (int64_t t = t0; t < t1; ++t) {
                    int64_t *hc = hist.data() + (size_t)t * p.n;
                    const int64_t r0 = p.m * t / TT, r1 = p.m * (t + 1) / TT;
                    for (int64_t k = Krp[yoff + r0]; k < Krp[yoff + r1]; ++k) hc[Kci[k] - xoff]++;
                }
            });
            int64_t acc = nzoff;
            for (int64_t j = 0; j + 1 < p.n; ++j) {
                for (int t = 0; t < TT; ++t) acc += hist[(size_t)t * p.n + j];
                Ktrp[xoff + j + 1] = acc;
            }
            std::vector<int64_t>().swap(hist);
            std::vector<int64_t> ccut(TT + 1, p.n);
            ccut[0] = 0;
            for (int t = 1, j = 0; t < TT; ++t) {
                const int64_t target = nzoff + nzi * t / TT;
                while (j < p.n && Ktrp[xoff + j] < target) ++j;
                ccut[t] = j;
            }
            std::vector<int64_t> nx(Ktrp.begin() + xoff, Ktrp.begin() + xoff + p.n);  // next slot per column
            parallel_ranges(TT, 1, TT, [&](int, int64_t t0, int64_t t1) {
                for (int64_t t = t0; t < t1; ++t) {
                    const int64_t c0 = ccut[t], c1 = ccut[t + 1];
                    if (c1 <= c0) continue;
                    for (int64_t i = 0; i < p.m; ++i)
                        for (int64_t k = Krp[yoff + i]; k < Krp[yoff + i + 1]; ++k) {
                            const int64_t j = Kci[k] - xoff;
                            if (j < c0 || j >= c1) continue;
                            const int64_t dst = nx[j]++;
                            Ktci[dst] = (int32_t)(yoff + i);
                            Ktv[dst] = Kv[k];
                        }
                }
            });
        }
        // slices of the rows of K^T swept in St passes: every column lists its
        // rows in increasing order, so slice t (rows [t Wt, (t + 1) Wt) of the
        // instance) is a contiguous run; record where runs 1 .. St-1 begin
        if (St > 1) {
            const int64_t Wt = std::max<int64_t>(1, (p.m + St - 1) / St);
            parallel_ranges(p.n, 4096, HT, [&](int, int64_t j0, int64_t j1) {
                for (int64_t j = j0; j < j1; ++j) {
                    int32_t *sb = Ktsb.data() + (size_t)(xoff + j) * (St - 1);
                    const int64_t b = Ktrp[xoff + j], e = Ktrp[xoff + j + 1];
                    if (!row_sliced_t(e - b, St)) {
                        for (int t = 1; t < St; ++t) sb[t - 1] = 0;
                        continue;
                    }
                    int64_t k = b;
                    for (int t = 1; t < St; ++t) {
                        const int64_t lim = yoff + t * Wt;
                        while (k < e && Ktci[k] < lim) ++k;
                        sb[t - 1] = (int32_t)(k - b);
                    }
                }
            });
        }
        for (int64_t j = 0; j < p.n; ++j) {
            const int32_t cj = p.col_order[j];
            col_orig[xoff + j] = cj;
            inst_col[xoff + j] = bi;
            craw[xoff + j] = lp.c[cj];
            lraw[xoff + j] = lp.l[cj];
            uraw[xoff + j] = lp.u[cj];
        }
        double cn = 0, qn = 0;
        for (int64_t j = 0; j < p.n; ++j) cn += lp.c[j] * lp.c[j];
        for (int64_t i = 0; i < p.m; ++i) qn += lp.rhs[i] * lp.rhs[i];
        in.cnorm = std::sqrt(cn);
        in.qnorm = std::sqrt(qn);
        {
            // one iteration's two sweeps: values + columns of K~ and K~^T, row
            // pointers, and the swept and gathered vectors
            const int64_t es = (int64_t)elem_size(h->prec), nz = pos - nzoff;
            in.sweep_bytes = 2 * (es + 4) * nz + 8 * (p.n + p.m + 2) + es * (9 * p.n + 6 * p.m);
        }
    };
    if (h->batch == 1) {
        build_inst(0, HT);
    } else {
        std::vector<int32_t> order(h->batch);
        for (int bi = 0; bi < h->batch; ++bi) order[bi] = bi;
        std::stable_sort(order.begin(), order.end(),
                         [&](int32_t u, int32_t v) { return h->plan[u].nnz > h->plan[v].nnz; });
        std::atomic<bool> oom{false};
        parallel_items(h->batch, HT, [&](int64_t k) {
            try {
                build_inst(order[k], 1);
            } catch (...) {
                oom = true;
            }
        });
        if (oom) throw std::bad_alloc();
    }
    // segments and block maps, in instance order
    int32_t blkK = 0, blkT = 0;
    for (int bi = 0; bi < h->batch; ++bi) {
        const InstPlan &p = h->plan[bi];
        InstInfo &in = h->info[bi];
        const int64_t xoff = xo[bi], yoff = yo[bi];
        // segments and block maps (instance-major, so an instance's blocks are contiguous)
        // block numbering: segments of long rows first (the dispatcher starts
        // the expensive workgroups early and short-row workgroups fill the
        // tail); the rows keep their internal order
        auto by_lanes = [](const std::vector<SegH> &v) {
            std::vector<int> o(v.size());
            for (size_t k = 0; k < v.size(); ++k) o[k] = (int)k;
            std::stable_sort(o.begin(), o.end(),
                             [&](int a, int b) { return (v[a].lanes_log2 & 15) > (v[b].lanes_log2 & 15); });
            return o;
        };
        in.blkK0 = blkK;
        for (int si : by_lanes(p.segK)) {
            const SegH &sh = p.segK[si];
            Seg sg{};
            sg.row0 = yoff + sh.row0;
            sg.nrows = sh.nrows;
            sg.blk0 = blkK;
            sg.nblk = (sh.nrows + seg_group(sh.lanes_log2) - 1) / seg_group(sh.lanes_log2);
            sg.lanes_log2 = sh.lanes_log2;
            sg.inst = bi;
            sg.ineq = sh.ineq;
            sg.sliced = sh.sliced;
            for (int t = 0; t < sg.nblk; ++t) {
                Kbs[blkK + t] = (int32_t)Kseg.size();
                const int G = seg_group(sg.lanes_log2);
                const int64_t r0 = sg.row0 + (int64_t)t * G;
                const int nr = (int)std::min<int64_t>(G, sg.row0 + sg.nrows - r0);
                Kbd[blkK + t] = make_int4((int)r0, nr, bi, sg.lanes_log2 | (sg.ineq << 8) | (sg.sliced << 9));
            }
            blkK += sg.nblk;
            Kseg.push_back(sg);
        }
        in.blkK1 = blkK;
        in.blkT0 = blkT;
        for (int si : by_lanes(p.segT)) {
            const SegH &sh = p.segT[si];
            Seg sg{};
            sg.row0 = xoff + sh.row0;
            sg.nrows = sh.nrows;
            sg.blk0 = blkT;
            sg.nblk = (sh.nrows + seg_group(sh.lanes_log2) - 1) / seg_group(sh.lanes_log2);
            sg.lanes_log2 = sh.lanes_log2;
            sg.inst = bi;
            sg.ineq = 0;
            for (int t = 0; t < sg.nblk; ++t) {
                Ktbs[blkT + t] = (int32_t)Ktseg.size();
                const int G = seg_group(sg.lanes_log2);
                const int64_t r0 = sg.row0 + (int64_t)t * G;
                const int nr = (int)std::min<int64_t>(G, sg.row0 + sg.nrows - r0);
                Ktbd[blkT + t] = make_int4((int)r0, nr, bi, sg.lanes_log2 | (sg.sliced << 9));
            }
            blkT += sg.nblk;
            Ktseg.push_back(sg);
        }
        in.blkT1 = blkT;
        in.l2off = (int32_t)l2inst.size();
        in.l2cnt = (int32_t)((in.blkK1 - in.blkK0 + in.blkT1 - in.blkT0 + L2CH - 1) / L2CH);
        for (int t = 0; t < in.l2cnt; ++t) l2inst.push_back(bi);
    }
    // no row long enough to slice: one whole-row pass
    auto any_sliced = [](const std::vector<Seg> &v) {
        return std::any_of(v.begin(), v.end(), [](const Seg &g) { return g.sliced != 0; });
    };
    if (!any_sliced(Kseg)) d.K.slices = 1;
    if (!any_sliced(Ktseg)) d.Kt.slices = 1;
    // block costs for the XCD split of the sweeps: entries + 4 per row
    std::vector<int64_t> cumK(sz.nblkK + 1, 0), cumT(sz.nblkT + 1, 0);
    for (int64_t t = 0; t < sz.nblkK; ++t)
        cumK[t + 1] = cumK[t] + (Krp[Kbd[t].x + Kbd[t].y] - Krp[Kbd[t].x]) + 4 * (int64_t)Kbd[t].y;
    for (int64_t t = 0; t < sz.nblkT; ++t)
        cumT[t + 1] = cumT[t] + (Ktrp[Ktbd[t].x + Ktbd[t].y] - Ktrp[Ktbd[t].x]) + 4 * (int64_t)Ktbd[t].y;
    // admission order of a batch: decreasing sweep bytes, ties by index
    std::vector<int32_t> adm(h->batch);
    for (int bi = 0; bi < h->batch; ++bi) adm[bi] = bi;
    std::stable_sort(adm.begin(), adm.end(),
                     [&](int32_t a, int32_t c) { return h->info[a].sweep_bytes > h->info[c].sweep_bytes; });
    const auto t_copy = std::chrono::steady_clock::now();
    h->setup_phase[1] = std::chrono::duration<double>(t_copy - t_up).count();
    int rc;
    if ((rc = h2d(b.bcumK, cumK.data(), cumK.size(), s)) || (rc = h2d(b.bcumT, cumT.data(), cumT.size(), s)) ||
        (rc = h2d(d.adm_order, adm.data(), adm.size(), s)))
        return rc;
    if ((rc = h2d(b.Krp, Krp.data(), Krp.size(), s)) || (rc = h2d(b.Kci, Kci.data(), Kci.size(), s)) ||
        (rc = h2d(b.Kv64, Kv.data(), Kv.size(), s)) || (rc = h2d(b.Kseg, Kseg.data(), Kseg.size(), s)) ||
        (rc = h2d(b.Kbs, Kbs.data(), Kbs.size(), s)) || (rc = h2d(b.Ktrp, Ktrp.data(), Ktrp.size(), s)) ||
        (rc = h2d(b.Kbd, Kbd.data(), Kbd.size(), s)) || (rc = h2d(b.Ktbd, Ktbd.data(), Ktbd.size(), s)) ||
        (rc = h2d(b.Ktci, Ktci.data(), Ktci.size(), s)) || (rc = h2d(b.Ktv64, Ktv.data(), Ktv.size(), s)) ||
        (rc = h2d(b.Ktseg, Ktseg.data(), Ktseg.size(), s)) || (rc = h2d(b.Ktbs, Ktbs.data(), Ktbs.size(), s)) ||
        (rc = h2d(d.craw, craw.data(), craw.size(), s)) || (rc = h2d(d.lraw, lraw.data(), lraw.size(), s)) ||
        (rc = h2d(d.uraw, uraw.data(), uraw.size(), s)) || (rc = h2d(d.qraw, qraw.data(), qraw.size(), s)) ||
        (rc = h2d(d.col_orig, col_orig.data(), col_orig.size(), s)) ||
        (rc = h2d(d.row_orig, row_orig.data(), row_orig.size(), s)) ||
        (rc = h2d(d.inst_of_col, inst_col.data(), inst_col.size(), s)) ||
        (rc = h2d(d.inst_of_row, inst_row.data(), inst_row.size(), s)) ||
        (rc = h2d((InstInfo *)d.info, h->info.data(), h->info.size(), s)) ||
        (rc = h2d(b.l2inst, l2inst.data(), l2inst.size(), s)) ||
        (S > 1 && (rc = h2d(b.Ksb, Ksb.data(), Ksb.size(), s))) ||
        (St > 1 && (rc = h2d(b.Ktsb, Ktsb.data(), Ktsb.size(), s))))
        return rc;
    // the host images die with this scope: wait for the copies
    HIPCHK(hipStreamSynchronize(s));
    h->setup_phase[2] = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_copy).count();
    return PDHG_OK;
}

template <typename T>
static int device_setup(pdhg_handle *h, hipStream_t s)
{
    Dev &d = h->d;
    const pdhg_opts &o = h->opts;
    const int B = h->batch;
    // Ruiz scaling (Algorithm 3): both norms from the same scaled matrix, then
    // rho /= sqrt(row norm), kap /= sqrt(col norm); values rescaled once at the end
    launch_fill(d.rho, d.M, 1.0, s);
    launch_fill(d.kap, d.N, 1.0, s);
    for (int it = 0; it < o.ruiz_iters; ++it) {
        launch_rowmax(d.K, d.remap, true, d.rho, d.kap, d.vecM64, s);
        launch_rowmax(d.Kt, d.remap, false, d.kap, d.rho, d.vecN64, s);
        launch_ruiz_update(d.rho, d.vecM64, d.M, s);
        launch_ruiz_update(d.kap, d.vecN64, d.N, s);
    }
    launch_scale_vals(d.K, h->buf.Kv64, h->buf.Kv32, true, d.rho, d.kap, s);
    launch_scale_vals(d.Kt, h->buf.Ktv64, h->buf.Ktv32, false, d.kap, d.rho, s);
    launch_scale_data<T>(d, s);
    HIPCHK(hipGetLastError());
    // norms of the scaled cost and right-hand side (primal weight, Section 2.4.3)
    std::vector<double> cn2(B), qn2(B);
    double *sc = d.inst_scratch;
    launch_inst_nrm2(d, 1, d.c64, sc, s);
    launch_inst_nrm2(d, 0, d.q64, sc + B, s);
    HIPCHK(hipMemcpyAsync(cn2.data(), sc, B * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(qn2.data(), sc + B, B * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    // power iteration (Algorithm 2) on every instance at once.  Each pass's
    // stopping test runs on the device (k_power_test), so the host does not
    // wait on the passes; it reads the states back every POLL passes to stop
    // enqueuing once every instance has stopped (later passes sweep nothing).
    const auto t_pow = std::chrono::steady_clock::now();
    std::vector<double> est(B, 0.0);
    std::vector<int> its(B, 0);
    double *bv = d.vecN64, *wv = d.vecM64, *bt = d.vecN64b;
    double *pk = d.partials, *pt = d.partials + h->sz.nblkK + 1;
    launch_fill(bv, d.N, 1.0, s);
    std::vector<InstState> pst(B, InstState{});
    for (auto &x : pst) x.kkt_prev = -1.0;  // no previous estimate
    HIPCHK(hipMemcpyAsync(d.st, pst.data(), B * sizeof(InstState), hipMemcpyHostToDevice, s));
    launch_active(d, s);
    const int32_t *lK = d.actK, *lT = d.actT, *cK = d.act_cnt, *cT = d.act_cnt + 1;
    const int POLL = 16;
    auto remaining = [&](int *left) -> int {
        HIPCHK(hipMemcpyAsync(pst.data(), d.st, B * sizeof(InstState), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        *left = 0;
        for (int b = 0; b < B; ++b) *left += pst[b].done ? 0 : 1;
        return PDHG_OK;
    };
    int left = B;
    for (int it = 0; it < o.power_max_iters; ++it) {
        launch_spmv64(d.K, d.remap, bv, wv, pk, lK, cK, s);
        if (it > 0) {
            launch_inst_sum(d, 1, pk, sc, s);
            launch_power_test(d, sc, it, o.power_tol, 0, s);
            launch_active(d, s);
            if (it % POLL == 0) {
                if (remaining(&left)) return PDHG_ERR_HIP;
                if (left == 0) break;
            }
        }
        launch_spmv64(d.Kt, d.remap, wv, bt, pt, lT, cT, s);
        launch_inst_sum(d, 0, pt, sc + B, s);
        launch_normalize(bt, d.inst_of_col, d.N, sc + B, s);
        std::swap(bv, bt);
    }
    if (remaining(&left)) return PDHG_ERR_HIP;
    if (left > 0) {
        // the pass limit: every instance still iterating takes ||K b|| of its last b
        launch_spmv64(d.K, d.remap, bv, wv, pk, lK, cK, s);
        launch_inst_sum(d, 1, pk, sc, s);
        launch_power_test(d, sc, o.power_max_iters, o.power_tol, 1, s);
        if (remaining(&left)) return PDHG_ERR_HIP;
    }
    for (int b = 0; b < B; ++b) {
        est[b] = pst[b].knorm;
        its[b] = pst[b].power_iters;
    }
    // the handle's lists hold every instance again
    pst.assign(B, InstState{});
    HIPCHK(hipMemcpyAsync(d.st, pst.data(), B * sizeof(InstState), hipMemcpyHostToDevice, s));
    launch_active(d, s);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s));
    h->setup_phase[4] = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_pow).count();
    // step size and primal weight (Sections 2.3.1, 2.4.3)
    h->st0.assign(B, InstState{});
    h->knorm = est;
    for (int b = 0; b < B; ++b) {
        InstState &st = h->st0[b];
        const double kn = est[b];
        const double eta = o.step_size > 0.0 ? o.step_size : (kn > 0.0 ? o.step_frac / kn : 1.0);
        const double cn = std::sqrt(cn2[b]), qn = std::sqrt(qn2[b]);
        h->info[b].cnorm_s = cn;
        h->info[b].qnorm_s = qn;
        double omega;
        if (o.primal_weight > 0.0)
            omega = o.primal_weight;
        else if (cn > o.eps_zero && qn > o.eps_zero)
            omega = cn / qn;
        else
            omega = 1.0;
        st.eta = eta;
        st.omega0 = omega;
        st.omega = omega;
        st.tau = eta / omega;
        st.sigma = eta * omega;
        st.knorm = kn;
        st.kkt0 = INFINITY;
        st.kkt_prev = INFINITY;
        st.power_iters = its[b];
        st.eta_try = eta;
    }
    HIPCHK(hipMemcpyAsync(d.st, h->st0.data(), B * sizeof(InstState), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync((InstInfo *)d.info, h->info.data(), B * sizeof(InstInfo), hipMemcpyHostToDevice, s));
    launch_init_point<T>(d, s);
    // the adaptive step's second buffers start defined (they are overwritten
    // before they are read)
    const size_t es = sizeof(T);
    HIPCHK(hipMemsetAsync(d.xbar, 0, d.N * es, s));
    HIPCHK(hipMemsetAsync(d.xavg1, 0, d.N * es, s));
    HIPCHK(hipMemsetAsync(d.y1, 0, d.M * es, s));
    HIPCHK(hipMemsetAsync(d.yavg1, 0, d.M * es, s));
    HIPCHK(hipMemsetAsync(d.kx0, 0, d.M * sizeof(double), s));
    HIPCHK(hipMemsetAsync(d.kx1, 0, d.M * sizeof(double), s));
    HIPCHK(hipMemsetAsync(d.partials, 0, (size_t)(d.K.nblk + d.Kt.nblk) * NPART * sizeof(double), s));
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s));
    return PDHG_OK;
}

// dev_done: NULL keeps the done flags in mapped pinned host memory (polled
// without a copy); otherwise they live at dev_done in device memory and the
// solve loop copies them out (pdhg_setup_noalloc)
static int setup_impl(const pdhg_lp *lp, int32_t batch, const pdhg_opts *o, void *ws, size_t ws_bytes,
                      hipStream_t stream, pdhg_handle **out, int32_t *dev_done = nullptr)
{
    auto t0 = std::chrono::steady_clock::now();
    if (!out) return fail(PDHG_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    pdhg_opts def;
    if (!o) {
        pdhg_default_opts(&def);
        o = &def;
    }
    if (!ws) return fail(PDHG_ERR_INVALID_ARG, "workspace is NULL");
    if (((uintptr_t)ws & 255) != 0) return fail(PDHG_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    std::vector<HostLP> hosts;
    auto *h = new pdhg_handle();
    int rc = plan_all(lp, batch, o, hosts, h->plan, h->sz, false);
    if (rc) {
        delete h;
        return rc;
    }
    h->setup_phase[0] = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    h->batch = batch;
    h->prec = o->precision;
    h->opts = *o;
    Carve cv;
    cv.base = (char *)ws;
    InstInfo *info;
    InstState *st;
    carve(cv, h->sz, h->prec, *o, h->d, h->buf, &info, &st, &h->fish);
    if (cv.off > ws_bytes) {
        delete h;
        return fail(PDHG_ERR_NOMEM, "workspace too small: need %zu bytes, got %zu", cv.off, ws_bytes);
    }
    h->ws_bytes = cv.off;
    Dev &d = h->d;
    d.batch = batch;
    d.remap = o->xcd_remap ? 1 : 0;
    d.N = h->sz.N;
    d.M = h->sz.M;
    d.info = info;
    d.st = st;
    d.l2_inst = h->buf.l2inst;
    d.bcumK = h->buf.bcumK;
    d.bcumT = h->buf.bcumT;
    d.nl2 = (int32_t)h->sz.nl2;
    d.grid_cap = o->max_grid > 0 ? o->max_grid : 8192;
    Buffers &b = h->buf;
    int rmK = 1, rmT = 1;
    for (const InstPlan &p : h->plan) {
        for (const SegH &sg : p.segK) rmK = std::max(rmK, 1 << ((sg.lanes_log2 >> 4) & 3));
        for (const SegH &sg : p.segT) rmT = std::max(rmT, 1 << ((sg.lanes_log2 >> 4) & 3));
    }
    d.K = OpDev{h->sz.M, b.Krp, b.Kci, b.Kv32, b.Kv64, b.Kseg, b.Kbs, b.Kbd, (int32_t)h->sz.nsegK,
                (int32_t)h->sz.nblkK, rmK};
    d.Kt = OpDev{h->sz.N, b.Ktrp, b.Ktci, b.Ktv32, b.Ktv64, b.Ktseg, b.Ktbs, b.Ktbd, (int32_t)h->sz.nsegT,
                 (int32_t)h->sz.nblkT, rmT};
    d.K.slices = o->col_slices > 1 ? o->col_slices : 1;
    d.K.sb = b.Ksb;
    d.K.part = b.Kpart;
    d.Kt.slices = o->col_slices_t > 1 ? o->col_slices_t : 1;
    d.Kt.sb = b.Ktsb;
    d.Kt.part = b.Ktpart;
    if (dev_done) {
        d.hdone = dev_done;
    } else {
        if (hipHostMalloc((void **)&h->hdone_host, sizeof(int32_t) * batch,
                          hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess) {
            delete h;
            return fail(PDHG_ERR_HIP, "hipHostMalloc failed");
        }
        std::memset(h->hdone_host, 0, sizeof(int32_t) * batch);
        if (hipHostGetDevicePointer((void **)&d.hdone, h->hdone_host, 0) != hipSuccess) {
            (void)hipHostFree(h->hdone_host);
            delete h;
            return fail(PDHG_ERR_HIP, "hipHostGetDevicePointer failed");
        }
    }
    rc = upload(h, hosts, stream);
    hosts.clear();
    auto t_dev = std::chrono::steady_clock::now();
    if (!rc) rc = h->prec == PDHG_PREC_F32 ? device_setup<float>(h, stream) : device_setup<double>(h, stream);
    h->setup_phase[3] = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_dev).count();
    if (rc) {
        std::string m = g_err;
        pdhg_destroy(h);
        return fail(rc, "%s", m.c_str());
    }
    h->sol_avg.assign(batch, 0);
    h->setup_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    *out = h;
    return PDHG_OK;
}

// host allocations of setup may fail: report that instead of letting the
// exception cross the C ABI
extern "C" int pdhg_setup(const pdhg_lp *lp, int32_t batch, const pdhg_opts *o, void *ws, size_t ws_bytes,
                          hipStream_t stream, pdhg_handle **out)
{
    try {
        return setup_impl(lp, batch, o, ws, ws_bytes, stream, out);
    } catch (const std::bad_alloc &) {
        return fail(PDHG_ERR_NOMEM, "setup: host memory exhausted");
    } catch (...) {
        return fail(PDHG_ERR_INVALID_ARG, "setup: unexpected host error");
    }
}

extern "C" int pdhg_setup_noalloc(const pdhg_lp *lp, int32_t batch, const pdhg_opts *o, hipStream_t stream,
                                  pdhg_handle **out)
{
    if (!out) return fail(PDHG_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    if (stream) {
        int sdev = -1;
        HIPCHK(hipStreamGetDevice(stream, &sdev));
        if (sdev != dev) return fail(PDHG_ERR_INVALID_ARG, "stream belongs to device %d, current device is %d", sdev, dev);
    }
    pdhg_opts def;
    if (!o) {
        pdhg_default_opts(&def);
        o = &def;
    }
    const size_t need = pdhg_workspace_bytes(lp, batch, o);
    if (need == 0) return g_err_code;  // the sizing call's own error
    // the done flags follow the workspace in the same array
    const size_t flags_off = (need + 255) & ~(size_t)255;
    const size_t total = flags_off + sizeof(int32_t) * (size_t)batch;
    if (total > (size_t)PDHG_NOALLOC_MAX_BYTES)
        return fail(PDHG_ERR_NOMEM, "pdhg_setup_noalloc: the LP needs %zu bytes, the fixed workspace holds %zu "
                    "(use pdhg_setup with a caller workspace)", total, (size_t)PDHG_NOALLOC_MAX_BYTES);
    int8_t *owner = nullptr;
    try {
        // the claim's token lives as long as the handle (pdhg_destroy releases it)
        owner = new int8_t;
        void *ptr = nullptr;
        int busy = 0;
        const hipError_t e = noalloc_claim(dev, owner, &ptr, &busy);
        if (e != hipSuccess) {
            delete owner;
            if (busy)
                return fail(PDHG_ERR_STATE, "a handle from pdhg_setup_noalloc is still live on device %d "
                            "(pdhg_destroy it first)", dev);
            return fail(PDHG_ERR_HIP, "locating the fixed workspace on device %d: %s", dev, hipGetErrorString(e));
        }
        pdhg_handle *h = nullptr;
        const int rc = setup_impl(lp, batch, o, ptr, need, stream, &h, (int32_t *)((char *)ptr + flags_off));
        if (rc) {
            noalloc_release(dev, owner);
            delete owner;
            return rc;
        }
        h->noalloc_dev = dev;
        h->noalloc_owner = owner;
        *out = h;
        return PDHG_OK;
    } catch (const std::bad_alloc &) {
        if (owner) {
            noalloc_release(dev, owner);
            delete owner;
        }
        return fail(PDHG_ERR_NOMEM, "setup: host memory exhausted");
    } catch (...) {
        if (owner) {
            noalloc_release(dev, owner);
            delete owner;
        }
        return fail(PDHG_ERR_INVALID_ARG, "setup: unexpected host error");
    }
}

extern "C" void pdhg_destroy(pdhg_handle *h)
{
    if (!h) return;
    if (h->graph) (void)hipGraphExecDestroy(h->graph);
    if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
    if (h->hdone_host) (void)hipHostFree(h->hdone_host);
    if (h->noalloc_owner) {
        noalloc_release(h->noalloc_dev, h->noalloc_owner);
        delete (int8_t *)h->noalloc_owner;
    }
    delete h;
}

// ---------------------------------------------------------------------------
// solve
// ---------------------------------------------------------------------------

// admission budget of pdhg_solve (batches only)
static int64_t admission_budget(const pdhg_handle *h)
{
    return h->batch > 1 ? h->opts.batch_resident_bytes : 0;
}

static CtlParams ctl_params(const pdhg_handle *h)
{
    const pdhg_opts &o = h->opts;
    CtlParams P{};
    P.eps = o.eps;
    P.beta_suff = o.beta_suff;
    P.beta_nec = o.beta_nec;
    P.beta_art = o.beta_art;
    P.eps_zero = o.eps_zero;
    P.max_iters = o.max_iters;
    P.check_every = o.check_every;
    P.use_restarts = o.use_restarts;
    P.use_pw = o.use_pw_update;
    P.batch = h->batch;
    P.adaptive = o.adaptive_step;
    P.detect = o.detect_infeas;
    P.infeas_tol = o.infeas_tol;
    return P;
}

// one chunk: check_every iterations, the check, the control decision, restart
template <typename T>
static void enqueue_chunk(const pdhg_handle *h, hipStream_t s)
{
    const Dev &d = h->d;
    const int avg = h->opts.use_restarts;
    const int detect = h->opts.detect_infeas;
    if (h->opts.adaptive_step) {
        // Algorithm 5: check_every attempts, then the current buffers move to 0
        for (int j = 0; j < h->opts.check_every; ++j) {
            launch_primal_ad<T>(d, s);
            launch_dual_ad<T>(d, s);
            launch_step_ad(d, s);
        }
        launch_commit_ad<T>(d, s);
    } else {
        for (int j = 0; j < h->opts.check_every; ++j) {
            if (detect && j == h->opts.check_every - 1) launch_save_prev<T>(d, s);
            launch_primal<T>(d, j, avg, nullptr, s);
            launch_dual<T>(d, j, avg, nullptr, s);
        }
    }
    launch_check<T>(d, avg, s);
    // Algorithm 6 on the difference of the last step: the iterate before it is
    // in (xavg1, y1) with fixed steps, in buffer 1 (xbar, y1) with adaptive ones
    if (detect) launch_infeas<T>(d, h->opts.adaptive_step ? d.xbar : d.xavg1, d.y1, s);
    launch_control(d, ctl_params(h), h->opts.check_every, s);
    if (avg) {
        launch_restart<T>(d, s);
        if (h->opts.adaptive_step) launch_kx_ad<T>(d, 0, s);  // K~x of the restarted iterates
    }
    launch_active(d, s, admission_budget(h), 0);
}

template <typename T>
static int build_graph(pdhg_handle *h)
{
    if (h->graph) return PDHG_OK;
    if (!h->cap_stream) HIPCHK(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
    hipGraph_t g;
    HIPCHK(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
    enqueue_chunk<T>(h, h->cap_stream);
    HIPCHK(hipStreamEndCapture(h->cap_stream, &g));
    hipError_t e = hipGraphInstantiate(&h->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        h->graph = nullptr;
        return fail(PDHG_ERR_HIP, "hipGraphInstantiate failed: %s", hipGetErrorString(e));
    }
    return PDHG_OK;
}

template <typename T>
static int solve_impl(pdhg_handle *h, pdhg_result *res, hipStream_t s)
{
    auto t0 = std::chrono::steady_clock::now();
    const int B = h->batch;
    const Dev &d = h->d;
    if (h->opts.use_graph) {
        int rc = build_graph<T>(h);
        if (rc) return rc;
    }
    // fresh solve state from the current iterate
    std::vector<InstState> st = h->st0;
    for (auto &x : st) {
        x.k_total = 0;
        x.t_inner = 0;
        x.done = 0;
        x.status = PDHG_ITERATION_LIMIT;
        x.nrestarts = 0;
        x.kkt0 = INFINITY;
        x.kkt_prev = INFINITY;
        x.par = 0;
        x.eta_try = x.eta;
        x.eta_sum = 0.0;
        x.k_att = 0;
        x.n_acc = 0;
        x.prev_ok = 0;
        x.ntrace = 0;
    }
    if (h->hdone_host)
        std::memset(h->hdone_host, 0, sizeof(int32_t) * B);
    else
        HIPCHK(hipMemsetAsync(d.hdone, 0, sizeof(int32_t) * B, s));
    HIPCHK(hipMemcpyAsync(d.st, st.data(), B * sizeof(InstState), hipMemcpyHostToDevice, s));
    launch_active(d, s);
    launch_epoch_start<T>(d, s);
    launch_check<T>(d, 0, s);
    launch_control(d, ctl_params(h), 0, s);
    launch_active(d, s);
    if (h->opts.adaptive_step) launch_kx_ad<T>(d, 1, s);
    // every instance has had its starting-point check: those beyond the
    // admission budget wait from here on
    const int64_t budget = admission_budget(h);
    if (budget > 0) launch_active(d, s, budget, 1);
    HIPCHK(hipGetLastError());

    const int DEPTH = 4;
    hipEvent_t ev[DEPTH];
    for (int k = 0; k < DEPTH; ++k) HIPCHK(hipEventCreateWithFlags(&ev[k], hipEventDisableTiming));
    HIPCHK(hipEventRecord(ev[0], s));
    HIPCHK(hipEventSynchronize(ev[0]));
    std::vector<int32_t> flags(h->hdone_host ? 0 : B);
    auto all_done = [&]() {
        const int32_t *f = (const int32_t *)h->hdone_host;
        if (!f) {
            // device-resident flags: copy them out (waits for the chunks in flight)
            if (hipMemcpyAsync(flags.data(), d.hdone, sizeof(int32_t) * B, hipMemcpyDeviceToHost, s) != hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess)
                return false;
            f = flags.data();
        }
        for (int b = 0; b < B; ++b)
            if (!((volatile const int32_t *)f)[b]) return false;
        return true;
    };
    const double tl = h->opts.time_limit;
    bool timed_out = false;
    int rc = PDHG_OK;
    // no instance can run past max_iters, so never enqueue more chunks than
    // that (times the batch when instances are admitted one after another)
    const int64_t max_chunks = (h->opts.max_iters + h->opts.check_every - 1) / h->opts.check_every *
                               (budget > 0 ? B : 1);
    if (!all_done()) {
        for (int64_t chunk = 0; chunk < max_chunks; ++chunk) {
            if (h->opts.use_graph) {
                if (hipGraphLaunch(h->graph, s) != hipSuccess) {
                    rc = fail(PDHG_ERR_HIP, "hipGraphLaunch failed");
                    break;
                }
            } else {
                enqueue_chunk<T>(h, s);
            }
            if (hipEventRecord(ev[chunk % DEPTH], s) != hipSuccess) {
                rc = fail(PDHG_ERR_HIP, "hipEventRecord failed");
                break;
            }
            if (chunk >= DEPTH - 1) {
                if (hipEventSynchronize(ev[(chunk - (DEPTH - 1)) % DEPTH]) != hipSuccess) {
                    rc = fail(PDHG_ERR_HIP, "solve: %s", hipGetErrorString(hipGetLastError()));
                    break;
                }
                if (all_done()) break;
                if (tl > 0.0 &&
                    std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count() > tl) {
                    timed_out = true;
                    break;
                }
            }
        }
    }
    hipError_t se = hipStreamSynchronize(s);
    for (int k = 0; k < DEPTH; ++k) (void)hipEventDestroy(ev[k]);
    if (rc) return rc;
    if (se != hipSuccess) return fail(PDHG_ERR_HIP, "solve: %s", hipGetErrorString(se));
    HIPCHK(hipMemcpy(st.data(), d.st, B * sizeof(InstState), hipMemcpyDeviceToHost));
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    for (int b = 0; b < B; ++b) {
        const InstState &x = st[b];
        pdhg_result &r = res[b];
        std::memset(&r, 0, sizeof r);
        r.status = x.done == 1 ? x.status : (timed_out ? PDHG_TIME_LIMIT : PDHG_ITERATION_LIMIT);
        r.from_avg = x.sol_avg;
        r.iters = x.k_total;
        r.restarts = x.nrestarts;
        r.power_iters = x.power_iters;
        r.knorm = x.knorm;
        r.eta = x.eta;
        r.omega0 = x.omega0;
        r.omega = x.omega;
        r.tau = x.tau;
        r.sigma = x.sigma;
        std::memcpy(&r.kkt, x.kkt, sizeof(double) * 9);
        r.seconds = secs;
        r.accepted = h->opts.adaptive_step ? x.n_acc : x.k_total;
        r.eta_next = h->opts.adaptive_step ? x.eta_try : x.eta;
        h->sol_avg[b] = x.sol_avg;
    }
    // keep tau / sigma / omega of the end of the solve for later fixed-step calls
    for (int b = 0; b < B; ++b) {
        h->st0[b].omega = st[b].omega;
        h->st0[b].tau = st[b].tau;
        h->st0[b].sigma = st[b].sigma;
    }
    return PDHG_OK;
}

extern "C" int pdhg_solve(pdhg_handle *h, pdhg_result *res, hipStream_t stream)
{
    if (!h || !res) return fail(PDHG_ERR_INVALID_ARG, "NULL handle or result");
    return h->prec == PDHG_PREC_F32 ? solve_impl<float>(h, res, stream) : solve_impl<double>(h, res, stream);
}

// ---------------------------------------------------------------------------
// fixed-step iterations
// ---------------------------------------------------------------------------

template <typename T>
static int iterate_impl(pdhg_handle *h, int64_t k, int32_t record, hipStream_t s)
{
    Dev d = h->d;
    // recorded steps sweep whole rows, as the adjoint's replay of them does
    if (record) d.K.slices = d.Kt.slices = 1;
    // fixed steps use the handle's tau / sigma and ignore done flags
    std::vector<InstState> st = h->st0;
    for (auto &x : st) x.done = 0;
    if (record) {
        if (h->opts.unroll_capacity <= 0)
            return fail(PDHG_ERR_STATE, "recording needs opts.unroll_capacity > 0 at setup");
        if (k > h->opts.unroll_capacity)
            return fail(PDHG_ERR_INVALID_ARG, "k = %lld exceeds unroll_capacity = %d", (long long)k,
                        h->opts.unroll_capacity);
    }
    HIPCHK(hipMemcpyAsync(d.st, st.data(), h->batch * sizeof(InstState), hipMemcpyHostToDevice, s));
    launch_active(d, s);
    const int64_t C = std::max(1, h->opts.unroll_checkpoint);
    const size_t es = elem_size(h->prec);
    for (int64_t t = 0; t < k; ++t) {
        if (record && t % C == 0) {
            const int64_t slot = t / C;
            HIPCHK(hipMemcpyAsync((char *)h->buf.ckx + slot * d.N * es, d.x, d.N * es, hipMemcpyDeviceToDevice, s));
            HIPCHK(hipMemcpyAsync((char *)h->buf.cky + slot * d.M * es, d.y, d.M * es, hipMemcpyDeviceToDevice, s));
        }
        launch_primal<T>(d, 0, 0, nullptr, s);
        launch_dual<T>(d, 0, 0, nullptr, s);
    }
    HIPCHK(hipGetLastError());
    if (record) {
        h->rec_steps = k;
        h->rec_valid = 1;
        h->rec_gen += 1;
        h->rec_st = st;
    }
    return PDHG_OK;
}

template <typename T>
static int backward_impl(pdhg_handle *h, const double *gx, const double *gy, double *gc, double *grhs,
                         double *gl, double *gu, double *gx0, double *gy0, int32_t mem, hipStream_t s)
{
    if (!h->rec_valid)
        return fail(PDHG_ERR_STATE, "no recorded pdhg_iterate to differentiate (none since setup or the last "
                                    "pdhg_set_data)");
    Dev d = h->d;
    Buffers &b = h->buf;
    AdjBufs a{b.ax, b.av, b.ac, b.al, b.au, b.ay, b.aw, b.aq};
    const int64_t K = h->rec_steps, C = std::max(1, h->opts.unroll_checkpoint);
    const int64_t nseg = (K + C - 1) / C;
    const size_t es = elem_size(h->prec);
    const int64_t N = d.N, M = d.M;
    const double *gxd = gx, *gyd = gy;
    if (mem == PDHG_MEM_HOST) {
        HIPCHK(hipMemcpyAsync(d.vecN64b, gx, N * sizeof(double), hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(d.vecM64b, gy, M * sizeof(double), hipMemcpyHostToDevice, s));
        gxd = d.vecN64b;
        gyd = d.vecM64b;
    }
    HIPCHK(hipMemcpyAsync(d.st, h->rec_st.data(), h->batch * sizeof(InstState), hipMemcpyHostToDevice, s));
    launch_active(d, s);
    // keep the live iterate: the replay runs in the iterate buffers
    char *bx = (char *)b.ckx + nseg * N * es, *by = (char *)b.cky + nseg * M * es;
    HIPCHK(hipMemcpyAsync(bx, d.x, N * es, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(by, d.y, M * es, hipMemcpyDeviceToDevice, s));
    launch_adj_init(d, a, gxd, gyd, s);
    for (int64_t sg = nseg - 1; sg >= 0; --sg) {
        const int64_t len = std::min(C, K - sg * C);
        HIPCHK(hipMemcpyAsync(d.x, (char *)b.ckx + sg * N * es, N * es, hipMemcpyDeviceToDevice, s));
        HIPCHK(hipMemcpyAsync(d.y, (char *)b.cky + sg * M * es, M * es, hipMemcpyDeviceToDevice, s));
        for (int64_t t = 0; t < len; ++t) {
            launch_primal<T>(d, 0, 0, b.maskx + t * N, s);
            launch_dual<T>(d, 0, 0, b.masky + t * M, s);
        }
        for (int64_t t = len - 1; t >= 0; --t) {
            launch_adj_w(d, a, b.masky + t * M, s);
            launch_rev_primal<T>(d, a, b.maskx + t * N, s);
            launch_rev_dual<T>(d, a, s);
        }
    }
    HIPCHK(hipMemcpyAsync(d.x, bx, N * es, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(d.y, by, M * es, hipMemcpyDeviceToDevice, s));
    if (mem == PDHG_MEM_HOST) {
        double *o[6] = {d.vecN64, d.vecN64b, b.vecN64c, b.axb, d.vecM64, d.vecM64b};
        launch_adj_out(d, a, gc ? o[0] : nullptr, grhs ? o[4] : nullptr, gl ? o[1] : nullptr,
                       gu ? o[2] : nullptr, gx0 ? o[3] : nullptr, gy0 ? o[5] : nullptr, s);
        double *dst[6] = {gc, gl, gu, gx0, grhs, gy0};
        const double *src[6] = {o[0], o[1], o[2], o[3], o[4], o[5]};
        const int64_t cnt[6] = {N, N, N, N, M, M};
        for (int q = 0; q < 6; ++q)
            if (dst[q] && cnt[q])
                HIPCHK(hipMemcpyAsync(dst[q], src[q], cnt[q] * sizeof(double), hipMemcpyDeviceToHost, s));
    } else {
        launch_adj_out(d, a, gc, grhs, gl, gu, gx0, gy0, s);
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s));
    return PDHG_OK;
}

extern "C" int pdhg_iterate(pdhg_handle *h, int64_t k, int32_t record, hipStream_t stream)
{
    if (!h || k < 0) return fail(PDHG_ERR_INVALID_ARG, "bad handle or step count");
    return h->prec == PDHG_PREC_F32 ? iterate_impl<float>(h, k, record, stream)
                                    : iterate_impl<double>(h, k, record, stream);
}

// ---------------------------------------------------------------------------
// solution read-out, warm start, KKT of a caller point
// ---------------------------------------------------------------------------

static int out_copy(double *dst, const double *dev_src, size_t cnt, int mem, hipStream_t s)
{
    if (!dst || cnt == 0) return PDHG_OK;
    HIPCHK(hipMemcpyAsync(dst, dev_src, cnt * sizeof(double),
                          mem == PDHG_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, s));
    return PDHG_OK;
}

extern "C" int pdhg_get_solution(pdhg_handle *h, int32_t inst, int32_t which, double *x, double *y,
                                 double *lambda, int32_t mem, hipStream_t s)
{
    if (!h || inst < 0 || inst >= h->batch) return fail(PDHG_ERR_INVALID_ARG, "bad handle or instance");
    if (which < PDHG_SOL_RESULT || which > PDHG_SOL_AVERAGE) return fail(PDHG_ERR_INVALID_ARG, "bad 'which'");
    if (mem != PDHG_MEM_HOST && mem != PDHG_MEM_DEVICE) return fail(PDHG_ERR_INVALID_ARG, "bad mem");
    const Dev &d = h->d;
    const InstInfo &in = h->info[inst];
    const int avg = which == PDHG_SOL_AVERAGE || (which == PDHG_SOL_RESULT && h->sol_avg[inst]);
    if (h->prec == PDHG_PREC_F32)
        launch_point_to64<float>(d, avg, d.vecN64, d.vecM64, s);
    else
        launch_point_to64<double>(d, avg, d.vecN64, d.vecM64, s);
    int rc;
    if (x) {
        launch_unscale_x(d, in.xoff, in.n, d.vecN64, d.vecN64b, s);
        if ((rc = out_copy(x, d.vecN64b, in.n, mem, s))) return rc;
    }
    if (y) {
        launch_unscale_y(d, in.yoff, in.m, d.vecM64, d.vecM64b, s);
        if ((rc = out_copy(y, d.vecM64b, in.m, mem, s))) return rc;
    }
    if (lambda) {
        launch_lambda(d, d.vecM64, h->buf.vecN64c, s);
        launch_permute_out(d.col_orig, in.xoff, in.n, h->buf.vecN64c, d.vecN64b, s);
        if ((rc = out_copy(lambda, d.vecN64b, in.n, mem, s))) return rc;
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s));
    return PDHG_OK;
}

// stages a caller vector on the device (FP64); returns the device pointer
static int stage_in(const double *src, size_t cnt, int mem, double *scratch, const double **dev, hipStream_t s)
{
    if (mem == PDHG_MEM_DEVICE) {
        *dev = src;
        return PDHG_OK;
    }
    if (cnt) HIPCHK(hipMemcpyAsync(scratch, src, cnt * sizeof(double), hipMemcpyHostToDevice, s));
    *dev = scratch;
    return PDHG_OK;
}

static int scale_caller_point(pdhg_handle *h, int32_t inst, const double *x, const double *y, int32_t mem,
                              hipStream_t s)
{
    const Dev &d = h->d;
    const InstInfo &in = h->info[inst];
    const double *xd = nullptr, *yd = nullptr;
    int rc;
    if ((rc = stage_in(x, in.n, mem, d.vecN64b, &xd, s))) return rc;
    if ((rc = stage_in(y, in.m, mem, d.vecM64b, &yd, s))) return rc;
    launch_scale_in(d, in.xoff, in.n, in.yoff, in.m, xd, yd, d.vecN64, d.vecM64, s);
    HIPCHK(hipGetLastError());
    return PDHG_OK;
}

extern "C" int pdhg_set_state(pdhg_handle *h, int32_t inst, const double *x, const double *y, int32_t mem,
                              hipStream_t s)
{
    if (!h || inst < 0 || inst >= h->batch || !x || !y) return fail(PDHG_ERR_INVALID_ARG, "bad arguments");
    int rc = scale_caller_point(h, inst, x, y, mem, s);
    if (rc) return rc;
    const InstInfo &in = h->info[inst];
    if (h->prec == PDHG_PREC_F32)
        launch_set_point<float>(h->d, in.xoff, in.n, in.yoff, in.m, in.m1, h->d.vecN64, h->d.vecM64, s);
    else
        launch_set_point<double>(h->d, in.xoff, in.n, in.yoff, in.m, in.m1, h->d.vecN64, h->d.vecM64, s);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s));
    return PDHG_OK;
}

// ---------------------------------------------------------------------------
// fishnet casting (Section 2.5, Algorithm 7)
// ---------------------------------------------------------------------------

// Once per handle: the rows of each operator by decreasing length (stable)
// for the gap pass, and the sweep tasks: whole rows, or FISH_CHUNK-entry
// chunks of longer rows (with one partial slot each), longest first.
static int fish_build_tables(pdhg_handle *h, hipStream_t s)
{
    const Dev &d = h->d;
    FishDev &f = h->fish;
    for (int op = 0; op < 2; ++op) {
        const OpDev &o = op == 0 ? d.K : d.Kt;
        std::vector<int64_t> rp(o.nrows + 1);
        HIPCHK(hipMemcpyAsync(rp.data(), o.rp, rp.size() * sizeof(int64_t), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (rp[o.nrows] >= INT32_MAX) return fail(PDHG_ERR_SHAPE, "fishnet casting needs fewer than 2^31 nonzeros");
        std::vector<int32_t> ord(o.nrows);
        for (int64_t r = 0; r < o.nrows; ++r) ord[r] = (int32_t)r;
        std::stable_sort(ord.begin(), ord.end(),
                         [&](int32_t a, int32_t b) { return rp[a + 1] - rp[a] > rp[b + 1] - rp[b]; });
        std::vector<int4> tasks, splits;
        int32_t slot = 0;
        for (int64_t r = 0; r < o.nrows; ++r) {
            const int32_t b = (int32_t)rp[r], e = (int32_t)rp[r + 1];
            if (e - b <= FISH_CHUNK) {
                tasks.push_back(make_int4((int32_t)r, b, e, -1));
                continue;
            }
            const int32_t nch = (e - b + FISH_CHUNK - 1) / FISH_CHUNK;
            splits.push_back(make_int4((int32_t)r, slot, nch, 0));
            for (int32_t c = 0; c < nch; ++c)
                tasks.push_back(make_int4((int32_t)r, b + c * FISH_CHUNK, std::min(e, b + (c + 1) * FISH_CHUNK), slot + c));
            slot += nch;
        }
        std::stable_sort(tasks.begin(), tasks.end(), [](const int4 &a, const int4 &b) { return a.z - a.y > b.z - b.y; });
        std::stable_sort(splits.begin(), splits.end(), [](const int4 &a, const int4 &b) { return a.z > b.z; });
        int32_t *rows = (int32_t *)(op == 0 ? f.rowK : f.rowT);
        int4 *tk = (int4 *)(op == 0 ? f.taskK : f.taskT);
        int4 *sp = (int4 *)(op == 0 ? f.splitK : f.splitT);
        if (o.nrows) HIPCHK(hipMemcpyAsync(rows, ord.data(), ord.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
        if (!tasks.empty()) HIPCHK(hipMemcpyAsync(tk, tasks.data(), tasks.size() * sizeof(int4), hipMemcpyHostToDevice, s));
        if (!splits.empty()) HIPCHK(hipMemcpyAsync(sp, splits.data(), splits.size() * sizeof(int4), hipMemcpyHostToDevice, s));
        HIPCHK(hipStreamSynchronize(s));
        if (op == 0) {
            f.ntaskK = (int64_t)tasks.size();
            f.nsplitK = (int64_t)splits.size();
        } else {
            f.ntaskT = (int64_t)tasks.size();
            f.nsplitT = (int64_t)splits.size();
        }
    }
    h->fish_rows = true;
    return PDHG_OK;
}

// rounds of Algorithm 7 for P points and the repopulation draws they consume
static void fish_plan(int P, int *rounds, int64_t *draws)
{
    int j = P, r = 0;
    int64_t need = 0;
    while (j > 1) {
        const int half = j / 2;
        const bool rep = (r & 1) && j > 2;
        if (rep) need += (int64_t)half * half;
        j = rep ? 2 * half : half;
        ++r;
    }
    *rounds = r;
    *draws = need;
}

template <typename T>
static int fishnet_impl(pdhg_handle *h, int P, int32_t k, const double *G, const double *wraw, int mem,
                        double *gaps, int32_t *keep, hipStream_t s)
{
    Dev &d = h->d;
    if (!h->fish_rows) {
        int rc = fish_build_tables(h, s);
        if (rc) return rc;
    }
    FishDev f = h->fish;
    int rounds;
    int64_t need;
    fish_plan(P, &rounds, &need);
    const size_t ng = (size_t)P * d.N;
    if (mem == PDHG_MEM_HOST) {
        for (size_t t = 0; t < ng; ++t)
            if (!std::isfinite(G[t])) return fail(PDHG_ERR_NONFINITE, "fishnet draws: G[%zu] is not finite", t);
        for (int64_t t = 0; t < need; ++t)
            if (!std::isfinite(wraw[t])) return fail(PDHG_ERR_NONFINITE, "fishnet draws: wraw[%lld] is not finite",
                                                     (long long)t);
    }
    const hipMemcpyKind kind = mem == PDHG_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    if (ng) HIPCHK(hipMemcpyAsync(f.gstage, G, ng * sizeof(double), kind, s));
    if (need) HIPCHK(hipMemcpyAsync(f.wstage, wraw, need * sizeof(double), kind, s));
    const InstState &st = h->st0[0];
    const InstInfo &in = h->info[0];
    const double sc = d.N > 0 ? st.knorm / std::sqrt((double)d.N) : 0.0;
    launch_fish_init<T>(d, f, ilog2(P), sc, s);
    int j = P, round = 0;
    int64_t wpos = 0;
    while (j > 1) {
        const int lj = ilog2(j);
        for (int t = 0; t < k; ++t) launch_fish_step<T>(d, f, lj, st.tau, st.sigma, in.m1, s);
        const int half = j / 2;
        const int rep = (round & 1) && j > 2;
        const int next = rep ? 2 * half : half;
        launch_fish_gap_rank<T>(d, f, lj, round, rep, half, wpos, s);
        launch_fish_gather<T>(d, f, ilog2(next), half, s);
        std::swap(f.X, f.X2);
        std::swap(f.Y, f.Y2);
        if (rep) wpos += (int64_t)half * half;
        j = next;
        ++round;
    }
    launch_fish_out<T>(d, f, s);
    launch_set_point<T>(d, 0, d.N, 0, d.M, in.m1, d.vecN64, d.vecM64, s);
    HIPCHK(hipGetLastError());
    // the record, repacked to P columns
    std::vector<double> rg((size_t)f.nrec * f.PS);
    std::vector<int32_t> rk((size_t)f.nrec * f.PS);
    HIPCHK(hipMemcpyAsync(rg.data(), f.rec_gaps, rg.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(rk.data(), f.rec_keep, rk.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    std::vector<double> og((size_t)rounds * P);
    std::vector<int32_t> ok((size_t)rounds * P);
    for (int r = 0; r < rounds; ++r)
        for (int q = 0; q < P; ++q) {
            og[(size_t)r * P + q] = rg[(size_t)r * f.PS + q];
            ok[(size_t)r * P + q] = rk[(size_t)r * f.PS + q];
        }
    const hipMemcpyKind back = mem == PDHG_MEM_HOST ? hipMemcpyHostToHost : hipMemcpyHostToDevice;
    if (gaps) HIPCHK(hipMemcpy(gaps, og.data(), og.size() * sizeof(double), back));
    if (keep) HIPCHK(hipMemcpy(keep, ok.data(), ok.size() * sizeof(int32_t), back));
    return PDHG_OK;
}

extern "C" int pdhg_fishnet_rounds(int32_t npoints, int32_t *rounds, int64_t *draws)
{
    if (npoints < 2 || npoints > 64 || (npoints & (npoints - 1)) || !rounds || !draws)
        return fail(PDHG_ERR_INVALID_ARG, "npoints must be a power of two in 2..64");
    int r;
    int64_t n;
    fish_plan(npoints, &r, &n);
    *rounds = r;
    *draws = n;
    return PDHG_OK;
}

extern "C" int pdhg_fishnet(pdhg_handle *h, int32_t npoints, int32_t k, const double *G, const double *wraw,
                            int64_t nw, int32_t mem, double *gaps, int32_t *keep, hipStream_t s)
{
    if (!h || !G) return fail(PDHG_ERR_INVALID_ARG, "NULL handle or draws");
    if (h->batch != 1) return fail(PDHG_ERR_STATE, "fishnet casting runs on a handle of one LP");
    if (h->opts.fishnet_points <= 0)
        return fail(PDHG_ERR_STATE, "fishnet casting needs opts.fishnet_points > 0 at setup");
    if (npoints < 2 || npoints > h->opts.fishnet_points || (npoints & (npoints - 1)))
        return fail(PDHG_ERR_INVALID_ARG, "npoints must be a power of two in 2..%d", h->opts.fishnet_points);
    if (k < 1) return fail(PDHG_ERR_INVALID_ARG, "k must be >= 1");
    if (mem != PDHG_MEM_HOST && mem != PDHG_MEM_DEVICE) return fail(PDHG_ERR_INVALID_ARG, "bad mem");
    int rounds;
    int64_t need;
    fish_plan(npoints, &rounds, &need);
    if (need > 0 && (!wraw || nw < need))
        return fail(PDHG_ERR_INVALID_ARG, "%d points need %lld repopulation draws, got %lld", npoints,
                    (long long)need, (long long)(wraw ? nw : 0));
    return h->prec == PDHG_PREC_F32 ? fishnet_impl<float>(h, npoints, k, G, wraw, mem, gaps, keep, s)
                                    : fishnet_impl<double>(h, npoints, k, G, wraw, mem, gaps, keep, s);
}

extern "C" int pdhg_kkt(pdhg_handle *h, int32_t inst, const double *x, const double *y, int32_t mem,
                        pdhg_kkt_out *out, hipStream_t s)
{
    if (!h || inst < 0 || inst >= h->batch || !x || !y || !out) return fail(PDHG_ERR_INVALID_ARG, "bad arguments");
    const Dev &d = h->d;
    // other instances' entries of the scratch vectors are never read for `inst`
    int rc = scale_caller_point(h, inst, x, y, mem, s);
    if (rc) return rc;
    launch_check64(d, d.vecN64, d.vecM64, s);
    launch_kkt_final(d, inst, d.inst_scratch, s);
    double v[9];
    HIPCHK(hipMemcpyAsync(v, d.inst_scratch, sizeof v, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    out->pres = v[0];
    out->dres = v[1];
    out->pobj = v[2];
    out->dobj = v[3];
    out->gap = v[4];
    out->rel_pres = v[5];
    out->rel_dres = v[6];
    out->rel_gap = v[7];
    out->rel_kkt = v[8];
    return PDHG_OK;
}

extern "C" int pdhg_backward(pdhg_handle *h, const double *gx, const double *gy, double *gc, double *grhs,
                             double *gl, double *gu, double *gx0, double *gy0, int32_t mem, hipStream_t s)
{
    if (!h || !gx || !gy) return fail(PDHG_ERR_INVALID_ARG, "NULL handle or input gradient");
    if (mem != PDHG_MEM_HOST && mem != PDHG_MEM_DEVICE) return fail(PDHG_ERR_INVALID_ARG, "bad mem");
    return h->prec == PDHG_PREC_F32 ? backward_impl<float>(h, gx, gy, gc, grhs, gl, gu, gx0, gy0, mem, s)
                                    : backward_impl<double>(h, gx, gy, gc, grhs, gl, gu, gx0, gy0, mem, s);
}

extern "C" int pdhg_set_data(pdhg_handle *h, const double *c, const double *rhs, const double *l,
                             const double *u, int32_t mem, hipStream_t s)
{
    if (!h) return fail(PDHG_ERR_INVALID_ARG, "NULL handle");
    if (mem != PDHG_MEM_HOST && mem != PDHG_MEM_DEVICE) return fail(PDHG_ERR_INVALID_ARG, "bad mem");
    Dev &d = h->d;
    const int64_t N = d.N, M = d.M;
    if (mem == PDHG_MEM_HOST) {
        for (int64_t j = 0; c && j < N; ++j)
            if (!std::isfinite(c[j])) return fail(PDHG_ERR_NONFINITE, "c[%lld] is not finite", (long long)j);
        for (int64_t i = 0; rhs && i < M; ++i)
            if (!std::isfinite(rhs[i])) return fail(PDHG_ERR_NONFINITE, "rhs[%lld] is not finite", (long long)i);
        std::vector<double> lh(N), uh(N);
        if (l || u) {
            HIPCHK(hipMemcpy(lh.data(), d.lraw, N * sizeof(double), hipMemcpyDeviceToHost));
            HIPCHK(hipMemcpy(uh.data(), d.uraw, N * sizeof(double), hipMemcpyDeviceToHost));
        }
        // bounds are checked per variable in the caller's layout
        for (int bi = 0; (l || u) && bi < h->batch; ++bi) {
            const InstInfo &in = h->info[bi];
            const InstPlan &p = h->plan[bi];
            for (int64_t j = 0; j < in.n; ++j) {
                const int64_t o = in.xoff + p.col_order[j];
                const double lo = l ? l[o] : lh[in.xoff + j], hi = u ? u[o] : uh[in.xoff + j];
                if (std::isnan(lo) || std::isnan(hi)) return fail(PDHG_ERR_NONFINITE, "bound %lld is NaN", (long long)o);
                if (lo > hi || lo == INFINITY || hi == -INFINITY)
                    return fail(PDHG_ERR_BOUNDS, "inconsistent bounds at variable %lld", (long long)o);
            }
        }
    }
    const double *cd = c, *qd = rhs, *ld = l, *ud = u;
    // the recorded tape belongs to the old data: pdhg_backward refuses it from here on
    h->rec_valid = 0;
    h->rec_gen += 1;
    if (mem == PDHG_MEM_HOST) {
        double *st[4] = {d.vecN64, d.vecM64, d.vecN64b, h->buf.vecN64c};
        const double *src[4] = {c, rhs, l, u};
        const int64_t cnt[4] = {N, M, N, N};
        const double **dd[4] = {&cd, &qd, &ld, &ud};
        for (int q = 0; q < 4; ++q)
            if (src[q]) {
                if (cnt[q]) HIPCHK(hipMemcpyAsync(st[q], src[q], cnt[q] * sizeof(double), hipMemcpyHostToDevice, s));
                *dd[q] = st[q];
            }
    }
    launch_set_raw(d, cd, qd, ld, ud, s);
    if (h->prec == PDHG_PREC_F32)
        launch_scale_data<float>(d, s);
    else
        launch_scale_data<double>(d, s);
    // relative KKT terms use the norms of the original c and q
    const int B = h->batch;
    std::vector<double> n2(2 * B);
    launch_inst_nrm2(d, 1, d.craw, d.inst_scratch, s);
    launch_inst_nrm2(d, 0, d.qraw, d.inst_scratch + B, s);
    HIPCHK(hipMemcpyAsync(n2.data(), d.inst_scratch, 2 * B * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (int bi = 0; bi < B; ++bi) {
        h->info[bi].cnorm = std::sqrt(n2[bi]);
        h->info[bi].qnorm = std::sqrt(n2[B + bi]);
    }
    HIPCHK(hipMemcpyAsync((InstInfo *)d.info, h->info.data(), B * sizeof(InstInfo), hipMemcpyHostToDevice, s));
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s));
    return PDHG_OK;
}

template <typename T>
static int time_impl(pdhg_handle *h, int32_t reps, pdhg_kernel_times *out, hipStream_t s)
{
    const Dev &d = h->d;
    const int avg = h->opts.use_restarts;
    std::vector<InstState> st = h->st0;
    for (auto &x : st) x.done = 0;
    HIPCHK(hipMemcpyAsync(d.st, st.data(), h->batch * sizeof(InstState), hipMemcpyHostToDevice, s));
    launch_active(d, s);
    // an event between every two launches, created up front
    const int NE = 3 * reps + 1;
    std::vector<hipEvent_t> ev(NE, nullptr);
    int rc = PDHG_OK;
    for (int k = 0; k < NE && !rc; ++k)
        if (hipEventCreate(&ev[k]) != hipSuccess) rc = fail(PDHG_ERR_HIP, "hipEventCreate failed");
    auto gap = [&](int k0, int k1) -> double {
        float t = 0.f;
        if (hipEventElapsedTime(&t, ev[k0], ev[k1]) != hipSuccess && !rc)
            rc = fail(PDHG_ERR_HIP, "hipEventElapsedTime failed");
        return (double)t;
    };
    double ms[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    const CtlParams P = ctl_params(h);
    // Times a sequence of `nk` kernels launched in turn, `reps` times, into
    // out[0..nk).  An event after every launch separates the kernels but adds
    // its own packet to each interval, so the same sequence also runs with
    // events at its two ends only, and the excess of the separated total over
    // that total is taken out evenly from the intervals.
    auto time_seq = [&](int nk, auto &&launch, double *out) {
        if (rc) return;
        for (int k = 0; k < nk; ++k) launch(k, 0); // untimed, warms the caches
        (void)hipEventRecord(ev[0], s);
        for (int r = 0; r < reps; ++r)
            for (int k = 0; k < nk; ++k) launch(k, r);
        (void)hipEventRecord(ev[1], s);
        (void)hipEventSynchronize(ev[1]);
        const double whole = gap(0, 1);
        (void)hipEventRecord(ev[0], s);
        for (int r = 0; r < reps; ++r)
            for (int k = 0; k < nk; ++k) {
                launch(k, r);
                (void)hipEventRecord(ev[nk * r + k + 1], s);
            }
        (void)hipEventSynchronize(ev[nk * reps]);
        double sep = 0;
        for (int k = 0; k < nk; ++k) out[k] = 0;
        for (int r = 0; r < reps; ++r)
            for (int k = 0; k < nk; ++k) {
                const double t = gap(nk * r + k, nk * r + k + 1);
                out[k] += t;
                sep += t;
            }
        const double excess = sep > whole ? (sep - whole) / ((double)nk * reps) : 0.0;
        // a kernel shorter than the event packet itself would come out at or
        // below zero: it then gets its share of the unseparated total instead
        const double share = sep > 0.0 ? whole / sep : 1.0;
        for (int k = 0; k < nk; ++k) out[k] = std::max(out[k] / reps - excess, out[k] / reps * share);
    };
    // the two sweeps alternate as in the iteration (each one finds the caches
    // as the other leaves them)
    time_seq(2, [&](int k, int r) {
        if (k == 0) launch_primal<T>(d, r, avg, nullptr, s);
        else launch_dual<T>(d, r, avg, nullptr, s);
    }, ms);
    // once-per-chunk kernels, back to back, each on the path a check takes
    // when it restarts: the control kernel runs a whole check decision (a
    // check interval done, no stop: eps 0, no iteration limit, and the long
    // inner loop rule always met, so every launch restarts and updates omega),
    // the restart kernel copies every running instance's candidate
    CtlParams Pr = P;
    Pr.eps = 0.0;
    Pr.max_iters = LLONG_MAX;
    Pr.beta_art = 0.0;
    Pr.detect = 0;
    std::vector<InstState> sr = st;
    for (auto &x : sr) {
        x.kkt0 = x.kkt0 < INFINITY ? x.kkt0 : 1.0;
        x.restart = 1;
        x.cand_avg = 1;
    }
    for (int phase = 2; phase < 5 && !rc; ++phase) {
        if (phase == 4 && !avg) continue;
        if (phase >= 3 &&
            hipMemcpyAsync(d.st, sr.data(), h->batch * sizeof(InstState), hipMemcpyHostToDevice, s) != hipSuccess)
            rc = fail(PDHG_ERR_HIP, "state upload failed");
        (void)hipEventRecord(ev[0], s);
        for (int r = 0; r < reps; ++r) {
            switch (phase) {
                case 2: launch_check<T>(d, avg, s); break;
                case 3: launch_control(d, Pr, h->opts.check_every, s); break;
                default: launch_restart<T>(d, s); break;
            }
        }
        (void)hipEventRecord(ev[1], s);
        (void)hipEventSynchronize(ev[1]);
        ms[phase] = gap(0, 1) / reps;
        if (phase >= 3) {
            // restore the state the timed launches changed
            if (hipMemcpyAsync(d.st, st.data(), h->batch * sizeof(InstState), hipMemcpyHostToDevice, s) != hipSuccess)
                rc = fail(PDHG_ERR_HIP, "state restore failed");
            launch_active(d, s);
        }
    }
    // adaptive attempts: the primal sweep, the dual sweep and the step
    // decision in turn, as the solve runs them
    if (!rc) launch_kx_ad<T>(d, 1, s);
    time_seq(3, [&](int k, int) {
        if (k == 0) launch_primal_ad<T>(d, s);
        else if (k == 1) launch_dual_ad<T>(d, s);
        else launch_step_ad(d, s);
    }, ms + 5);
    if (!rc) {
        // the step kernel flips buffers: restore the state
        if (hipMemcpyAsync(d.st, st.data(), h->batch * sizeof(InstState), hipMemcpyHostToDevice, s) != hipSuccess)
            rc = fail(PDHG_ERR_HIP, "state restore failed");
        launch_active(d, s);
    }
    for (auto &e : ev)
        if (e) (void)hipEventDestroy(e);
    if (rc) return rc;
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s));
    out->ms_primal = ms[0];
    out->ms_dual = ms[1];
    out->ms_check = ms[2];
    out->ms_control = ms[3];
    out->ms_restart = ms[4];
    out->ms_primal_ad = ms[5];
    out->ms_dual_ad = ms[6];
    out->ms_step_ad = ms[7];
    out->reps = reps;
    return PDHG_OK;
}

extern "C" int pdhg_time_kernels(pdhg_handle *h, int32_t reps, pdhg_kernel_times *out, hipStream_t s)
{
    if (!h || !out || reps < 1 || reps > 10000) return fail(PDHG_ERR_INVALID_ARG, "bad arguments (1 <= reps <= 10000)");
    return h->prec == PDHG_PREC_F32 ? time_impl<float>(h, reps, out, s) : time_impl<double>(h, reps, out, s);
}

// ---------------------------------------------------------------------------
// autotuner of the launch layout
// ---------------------------------------------------------------------------

namespace {

void tune_limits(int f, int w, int32_t *lim)
{
    for (int k = 0; k < 6; ++k) lim[k] = f << k;
    lim[6] = std::max(w, 64 * f);
    lim[7] = 0;
}

// the candidate grid, in the order it is timed (stage 0: bins, 1: rows per
// group, 2: launch shape); later stages start from the best of earlier ones
std::vector<pdhg_opts> tune_stage(const pdhg_opts &base, int stage, const pdhg_opts &bp, const pdhg_opts &bd,
                                  std::vector<int> *tag)
{
    std::vector<pdhg_opts> out;
    if (stage == 0) {
        for (int f : {2, 4, 8, 16})
            for (int w : {512, 2048}) {
                if (w < 64 * f) continue;
                pdhg_opts o = base;
                tune_limits(f, w, o.bin_len_primal);
                tune_limits(f, w, o.bin_len_dual);
                out.push_back(o);
                if (tag) tag->push_back(f * 100000 + w);
            }
    } else if (stage == 1) {
        for (int r : {1, 2, 4}) {
            pdhg_opts o = base;
            std::memcpy(o.bin_len_primal, bp.bin_len_primal, sizeof o.bin_len_primal);
            std::memcpy(o.bin_len_dual, bd.bin_len_dual, sizeof o.bin_len_dual);
            for (int k = 0; k < 8; ++k) o.bin_rows_primal[k] = o.bin_rows_dual[k] = k < 5 ? r : 1;
            out.push_back(o);
            if (tag) tag->push_back(r);
        }
    } else if (stage == 3) {
        // column slices of both sweeps on the chosen layout (bp): none, then
        // S in {2, 4, 8} with every stage-0 limit set for the dual sweep
        // (sliced rows are binned by their per-slice length); the primal
        // sweep keeps its limits
        pdhg_opts o = bp;
        o.col_slices = o.col_slices_t = 0;
        out.push_back(o);
        if (tag) tag->push_back(0);
        for (int S : {2, 4, 8})
            for (int f : {2, 4, 8, 16})
                for (int w : {512, 2048}) {
                    if (w < 64 * f) continue;
                    o = bp;
                    o.col_slices = o.col_slices_t = S;
                    tune_limits(f, w, o.bin_len_dual);
                    out.push_back(o);
                    if (tag) tag->push_back(S * 10000000 + f * 100000 + w);
                }
    } else {
        for (int remap : {0, 1})
            for (int grid : {4096, 8192, 16384, 65536}) {
                pdhg_opts o = base;
                std::memcpy(o.bin_len_primal, bp.bin_len_primal, sizeof o.bin_len_primal);
                std::memcpy(o.bin_len_dual, bd.bin_len_dual, sizeof o.bin_len_dual);
                std::memcpy(o.bin_rows_primal, bp.bin_rows_primal, sizeof o.bin_rows_primal);
                std::memcpy(o.bin_rows_dual, bd.bin_rows_dual, sizeof o.bin_rows_dual);
                o.xcd_remap = remap;
                o.max_grid = grid;
                out.push_back(o);
                if (tag) tag->push_back(remap * 100000 + grid);
            }
    }
    return out;
}

int tune_time(const pdhg_lp *lp, int32_t batch, const pdhg_opts &o, void *ws, size_t ws_bytes, int32_t reps,
              hipStream_t s, pdhg_kernel_times *kt)
{
    pdhg_handle *h = nullptr;
    int rc = pdhg_setup(lp, batch, &o, ws, ws_bytes, s, &h);
    if (rc) return rc;
    pdhg_kernel_times warm;
    rc = pdhg_time_kernels(h, 3, &warm, s);
    if (!rc) rc = pdhg_time_kernels(h, reps, kt, s);
    pdhg_destroy(h);
    return rc;
}

std::string jnum(double v)
{
    char buf[32];
    std::snprintf(buf, sizeof buf, "%.9g", v);
    return buf;
}

void json_ints(std::string &js, const char *key, const int32_t *v)
{
    js += "\"";
    js += key;
    js += "\": [";
    for (int k = 0; k < 8; ++k) js += (k ? ", " : "") + std::to_string(v[k]);
    js += "]";
}

}  // namespace

static int autotune_impl(const pdhg_lp *lp, int32_t batch, const pdhg_opts *base, void *ws, size_t ws_bytes,
                         size_t *ws_needed, int32_t reps, hipStream_t s, pdhg_opts *best, const char *out_json)
{
    if (!lp || !base || !best || batch < 1 || reps < 1)
        return fail(PDHG_ERR_INVALID_ARG, "need lp, base, best != NULL, batch >= 1 and reps >= 1");
    // workspace: every candidate pairs one of the stage-0 limit sets per
    // operator with rows per group >= 1, so the largest workspace has at most
    // the most blocks and segments any limit set gives with one row per group
    // (and with every column-slice count of the last stage, whose sliced rows
    // form segments and blocks of their own)
    const int slice_cand[] = {std::max(base->col_slices, base->col_slices_t), 0, 2, 4, 8};
    Sizes bound{};
    {
        std::vector<int> t0;
        for (pdhg_opts o : tune_stage(*base, 0, *base, *base, &t0))
            for (int S : slice_cand) {
                for (int k = 0; k < 8; ++k) o.bin_rows_primal[k] = o.bin_rows_dual[k] = 1;
                o.col_slices = o.col_slices_t = S;
                std::vector<HostLP> hosts;
                std::vector<InstPlan> plans;
                Sizes sz;
                const int rc = plan_all(lp, batch, &o, hosts, plans, sz, true);
                if (rc) {
                    if (ws_needed) *ws_needed = 0;
                    return rc;
                }
                bound.N = sz.N, bound.M = sz.M, bound.NNZ = sz.NNZ, bound.batch = sz.batch;
                bound.nsegK = std::max(bound.nsegK, sz.nsegK);
                bound.nsegT = std::max(bound.nsegT, sz.nsegT);
                bound.nblkK = std::max(bound.nblkK, sz.nblkK);
                bound.nblkT = std::max(bound.nblkT, sz.nblkT);
            }
        // second-level rows: sum over instances of ceil((K + K^T blocks) / L2CH)
        bound.nl2 = (bound.nblkK + bound.nblkT + L2CH - 1) / L2CH + batch;
    }
    size_t need = 0;
    for (int S : slice_cand) {
        Carve cv;
        Dev d{};
        Buffers b{};
        InstInfo *info;
        InstState *st;
        FishDev fish{};
        pdhg_opts o = *base;
        o.col_slices = o.col_slices_t = S;
        carve(cv, bound, base->precision, o, d, b, &info, &st, &fish);
        need = std::max(need, (cv.off + 255) & ~(size_t)255);
    }
    if (ws_needed) *ws_needed = need;
    if (!ws || ws_bytes < need)
        return fail(PDHG_ERR_NOMEM, "autotune needs a workspace of %zu bytes", need);
    pdhg_opts bp = *base, bd = *base;
    double best_p = INFINITY, best_d = INFINITY;
    std::vector<int> tag;
    std::string js = "{\"trials\": [";
    int nt = 0;
    for (const pdhg_opts &o : tune_stage(*base, 0, bp, bd, &tag)) {
        pdhg_kernel_times kt;
        const int rc = tune_time(lp, batch, o, ws, ws_bytes, reps, s, &kt);
        if (rc) return rc;
        if (kt.ms_primal < best_p) best_p = kt.ms_primal, bp = o;
        if (kt.ms_dual < best_d) best_d = kt.ms_dual, bd = o;
        const int t = tag[nt];
        js += std::string(nt++ ? ", " : "") + "{\"f\": " + std::to_string(t / 100000) + ", \"w\": " +
              std::to_string(t % 100000) + ", \"ms_primal\": " + jnum(kt.ms_primal) +
              ", \"ms_dual\": " + jnum(kt.ms_dual) + "}";
    }
    js += "], \"rows_trials\": [";
    tag.clear();
    best_p = best_d = INFINITY;
    int32_t rows_p[8], rows_d[8];
    std::memcpy(rows_p, base->bin_rows_primal, sizeof rows_p);
    std::memcpy(rows_d, base->bin_rows_dual, sizeof rows_d);
    nt = 0;
    for (const pdhg_opts &o : tune_stage(*base, 1, bp, bd, &tag)) {
        pdhg_kernel_times kt;
        const int rc = tune_time(lp, batch, o, ws, ws_bytes, reps, s, &kt);
        if (rc) return rc;
        if (kt.ms_primal < best_p) best_p = kt.ms_primal, std::memcpy(rows_p, o.bin_rows_primal, sizeof rows_p);
        if (kt.ms_dual < best_d) best_d = kt.ms_dual, std::memcpy(rows_d, o.bin_rows_dual, sizeof rows_d);
        const int t = tag[nt];
        js += std::string(nt++ ? ", " : "") + "{\"rows\": " + std::to_string(t) + ", \"ms_primal\": " +
              jnum(kt.ms_primal) + ", \"ms_dual\": " + jnum(kt.ms_dual) + "}";
    }
    std::memcpy(bp.bin_rows_primal, rows_p, sizeof rows_p);
    std::memcpy(bd.bin_rows_dual, rows_d, sizeof rows_d);
    js += "], \"shapes\": [";
    tag.clear();
    double best_it = INFINITY;
    pdhg_opts shape = *base;
    pdhg_kernel_times best_kt{};
    nt = 0;
    for (const pdhg_opts &o : tune_stage(*base, 2, bp, bd, &tag)) {
        pdhg_kernel_times kt;
        const int rc = tune_time(lp, batch, o, ws, ws_bytes, reps, s, &kt);
        if (rc) return rc;
        const double it = kt.ms_primal + kt.ms_dual + kt.ms_check / std::max(1, base->check_every);
        if (it < best_it) best_it = it, shape = o, best_kt = kt;
        const int t = tag[nt];
        js += std::string(nt++ ? ", " : "") + "{\"xcd_remap\": " + std::to_string(t / 100000) +
              ", \"max_grid\": " + std::to_string(t % 100000) + ", \"ms_primal\": " +
              jnum(kt.ms_primal) + ", \"ms_dual\": " + jnum(kt.ms_dual) +
              ", \"ms_check\": " + jnum(kt.ms_check) + ", \"ms_iter\": " + jnum(it) + "}";
    }
    js += "], \"slice_trials\": [";
    tag.clear();
    nt = 0;
    {
        // slices are kept only when they beat the unsliced sweep by 2%
        double t0p = 0, t0d = 0, bsp = INFINITY, bsd = INFINITY;
        pdhg_opts dual = shape;
        int sp = 0;
        for (const pdhg_opts &o : tune_stage(*base, 3, shape, shape, &tag)) {
            pdhg_kernel_times kt;
            const int rc = tune_time(lp, batch, o, ws, ws_bytes, reps, s, &kt);
            if (rc) return rc;
            const int t = tag[nt];
            if (t == 0) {
                t0p = kt.ms_primal, t0d = kt.ms_dual;
            } else {
                if (kt.ms_primal < bsp) bsp = kt.ms_primal, sp = o.col_slices_t;
                if (kt.ms_dual < bsd) bsd = kt.ms_dual, dual = o;
            }
            js += std::string(nt ? ", " : "") + "{\"col_slices\": " + std::to_string(t / 10000000) +
                  ", \"f\": " + std::to_string(t / 100000 % 100) + ", \"w\": " + std::to_string(t % 100000) +
                  ", \"ms_primal\": " + jnum(kt.ms_primal) + ", \"ms_dual\": " + jnum(kt.ms_dual) + "}";
            ++nt;
        }
        best_kt.ms_primal = t0p, best_kt.ms_dual = t0d;
        shape.col_slices = shape.col_slices_t = 0;
        if (bsd <= 0.98 * t0d) {
            shape.col_slices = dual.col_slices;
            std::memcpy(shape.bin_len_dual, dual.bin_len_dual, sizeof shape.bin_len_dual);
            best_kt.ms_dual = bsd;
        }
        if (bsp <= 0.98 * t0p) shape.col_slices_t = sp, best_kt.ms_primal = bsp;
    }
    *best = shape;
    js += "], ";
    json_ints(js, "bin_len_primal", shape.bin_len_primal);
    js += ", ";
    json_ints(js, "bin_len_dual", shape.bin_len_dual);
    js += ", ";
    json_ints(js, "bin_rows_primal", shape.bin_rows_primal);
    js += ", ";
    json_ints(js, "bin_rows_dual", shape.bin_rows_dual);
    js += ", \"xcd_remap\": " + std::to_string(shape.xcd_remap) + ", \"max_grid\": " + std::to_string(shape.max_grid) +
          ", \"col_slices\": " + std::to_string(shape.col_slices) +
          ", \"col_slices_t\": " + std::to_string(shape.col_slices_t) +
          ", \"ms_primal\": " + jnum(best_kt.ms_primal) + ", \"ms_dual\": " + jnum(best_kt.ms_dual) +
          ", \"precision\": \"" + (base->precision == PDHG_PREC_F64 ? "f64" : "f32") + "\"}\n";
    if (out_json) {
        FILE *fp = std::fopen(out_json, "w");
        if (!fp) return fail(PDHG_ERR_INVALID_ARG, "cannot write %s", out_json);
        std::fputs(js.c_str(), fp);
        std::fclose(fp);
    }
    return PDHG_OK;
}

extern "C" int pdhg_autotune(const pdhg_lp *lp, int32_t batch, const pdhg_opts *base, void *ws, size_t ws_bytes,
                             size_t *ws_needed, int32_t reps, hipStream_t s, pdhg_opts *best, const char *out_json)
{
    try {
        return autotune_impl(lp, batch, base, ws, ws_bytes, ws_needed, reps, s, best, out_json);
    } catch (...) {
        return fail(PDHG_ERR_NOMEM, "autotune: host memory exhausted");
    }
}

extern "C" int pdhg_set_opts(pdhg_handle *h, const pdhg_opts *o)
{
    if (!h || !o) return fail(PDHG_ERR_INVALID_ARG, "NULL argument");
    pdhg_opts t = h->opts;
    t.use_restarts = o->use_restarts;
    t.use_pw_update = o->use_pw_update;
    t.check_every = o->check_every;
    t.max_iters = o->max_iters;
    t.eps = o->eps;
    t.time_limit = o->time_limit;
    t.beta_suff = o->beta_suff;
    t.beta_nec = o->beta_nec;
    t.beta_art = o->beta_art;
    t.eps_zero = o->eps_zero;
    t.use_graph = o->use_graph;
    t.adaptive_step = o->adaptive_step;
    t.detect_infeas = o->detect_infeas;
    t.infeas_tol = o->infeas_tol;
    t.batch_resident_bytes = o->batch_resident_bytes;
    int rc = check_opts(&t);
    if (rc) return rc;
    const bool regraph = t.use_restarts != h->opts.use_restarts || t.check_every != h->opts.check_every ||
                         t.use_pw_update != h->opts.use_pw_update || t.eps != h->opts.eps ||
                         t.max_iters != h->opts.max_iters || t.beta_suff != h->opts.beta_suff ||
                         t.beta_nec != h->opts.beta_nec || t.beta_art != h->opts.beta_art ||
                         t.eps_zero != h->opts.eps_zero || t.adaptive_step != h->opts.adaptive_step ||
                         t.detect_infeas != h->opts.detect_infeas || t.infeas_tol != h->opts.infeas_tol ||
                         t.batch_resident_bytes != h->opts.batch_resident_bytes;
    if (regraph && h->graph) {
        (void)hipGraphExecDestroy(h->graph);
        h->graph = nullptr;
    }
    h->opts = t;
    return PDHG_OK;
}

extern "C" int pdhg_get_trace(pdhg_handle *h, int32_t inst, pdhg_trace_rec *out, int32_t cap, int64_t *total,
                              hipStream_t s)
{
    if (!h || inst < 0 || inst >= h->batch) return fail(PDHG_ERR_INVALID_ARG, "bad handle or instance");
    if (h->d.trace_cap <= 0) return fail(PDHG_ERR_STATE, "the handle keeps no trace (opts.trace_capacity = 0)");
    if (cap < 0 || (cap > 0 && !out)) return fail(PDHG_ERR_INVALID_ARG, "need cap >= 0 and out != NULL");
    InstState st;
    HIPCHK(hipMemcpyAsync(&st, h->d.st + inst, sizeof st, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (total) *total = st.ntrace;
    const int64_t R = h->d.trace_cap;
    const int64_t keep = std::min<int64_t>(std::min<int64_t>(st.ntrace, R), cap);
    if (keep <= 0) return PDHG_OK;
    std::vector<pdhg_trace_rec> ring((size_t)R);
    HIPCHK(hipMemcpyAsync(ring.data(), h->d.trace + (size_t)inst * R, R * sizeof(pdhg_trace_rec),
                          hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (int64_t k = 0; k < keep; ++k) out[k] = ring[(size_t)((st.ntrace - keep + k) % R)];
    return PDHG_OK;
}

extern "C" int pdhg_get_scaling(pdhg_handle *h, int32_t inst, double *rho, double *kappa, int32_t mem,
                                hipStream_t s)
{
    if (!h || inst < 0 || inst >= h->batch) return fail(PDHG_ERR_INVALID_ARG, "bad handle or instance");
    const Dev &d = h->d;
    const InstInfo &in = h->info[inst];
    int rc;
    if (kappa) {
        launch_permute_out(d.col_orig, in.xoff, in.n, d.kap, d.vecN64b, s);
        if ((rc = out_copy(kappa, d.vecN64b, in.n, mem, s))) return rc;
    }
    if (rho) {
        launch_permute_out(d.row_orig, in.yoff, in.m, d.rho, d.vecM64b, s);
        if ((rc = out_copy(rho, d.vecM64b, in.m, mem, s))) return rc;
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s));
    return PDHG_OK;
}

extern "C" int pdhg_get_info(const pdhg_handle *h, pdhg_info *info)
{
    if (!h || !info) return fail(PDHG_ERR_INVALID_ARG, "NULL argument");
    std::memset(info, 0, sizeof *info);
    for (int b = 0; b < h->batch; ++b) {
        info->n += h->plan[b].n;
        info->m += h->plan[b].m;
        info->m_ineq += h->plan[b].m1;
        info->nnz += h->plan[b].nnz;
    }
    const InstState &st = h->st0[0];
    info->knorm = st.knorm;
    info->eta = st.eta;
    info->omega = st.omega;
    info->tau = st.tau;
    info->sigma = st.sigma;
    info->setup_seconds = h->setup_seconds;
    info->precision = h->prec;
    info->batch = h->batch;
    info->workspace_bytes = (int64_t)h->ws_bytes;
    info->nseg_primal = (int32_t)h->sz.nsegT;
    info->nseg_dual = (int32_t)h->sz.nsegK;
    info->nblk_primal = h->sz.nblkT;
    info->nblk_dual = h->sz.nblkK;
    info->setup_plan_seconds = h->setup_phase[0];
    info->setup_host_seconds = h->setup_phase[1];
    info->setup_copy_seconds = h->setup_phase[2];
    info->setup_device_seconds = h->setup_phase[3];
    info->setup_power_seconds = h->setup_phase[4];
    for (int b = 0; b < h->batch; ++b) info->power_iters_max = std::max(info->power_iters_max, h->st0[b].power_iters);
    info->record_generation = h->rec_gen;
    info->record_valid = h->rec_valid;
    return PDHG_OK;
}
