/* Host-only paths of the C-ABI under AddressSanitizer and UBSan: option and
 * input validation, sizing of single LPs and batches (row binning, block
 * plans), the autotuner's workspace bound and the fishnet round counts.
 * Nothing here touches a GPU.  Built and run by tests/test_host_sanitizers.py
 * against an instrumented build of the host library code; exits 0 when every
 * expectation holds (the sanitizers abort on the first memory error). */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "pdhg.h"

static int fails = 0;
#define EXPECT(c)                                                              \
    do {                                                                       \
        if (!(c)) {                                                            \
            fprintf(stderr, "FAILED line %d: %s (%s)\n", __LINE__, #c, pdhg_last_error()); \
            ++fails;                                                           \
        }                                                                      \
    } while (0)

/* a small LP in CSR: m rows, n columns, row i holds `len(i)` entries */
typedef struct {
    int64_t n, m, nnz;
    int64_t *rp;
    int32_t *ci;
    double *v, *c, *rhs, *l, *u;
    uint8_t *rt;
} lp_buf;

static unsigned rng_state = 12345u;
static unsigned rnd(void)
{
    rng_state = rng_state * 1664525u + 1013904223u;
    return rng_state >> 8;
}

static lp_buf make_lp(int64_t m, int64_t n, int maxlen)
{
    lp_buf b;
    b.m = m;
    b.n = n;
    b.rp = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m + 1));
    b.rp[0] = 0;
    for (int64_t i = 0; i < m; ++i) {
        /* heavy-tailed lengths: mostly short rows, a few long ones */
        int64_t len = 1 + (int64_t)(rnd() % 4);
        if (rnd() % 17 == 0) len = 1 + (int64_t)(rnd() % (unsigned)maxlen);
        if (len > n) len = n;
        if (rnd() % 29 == 0) len = 0; /* empty rows */
        b.rp[i + 1] = b.rp[i] + len;
    }
    b.nnz = b.rp[m];
    b.ci = (int32_t *)malloc(sizeof(int32_t) * (size_t)(b.nnz ? b.nnz : 1));
    b.v = (double *)malloc(sizeof(double) * (size_t)(b.nnz ? b.nnz : 1));
    for (int64_t k = 0; k < b.nnz; ++k) {
        b.ci[k] = (int32_t)(rnd() % (unsigned)n);
        b.v[k] = (double)((int)(rnd() % 2001) - 1000) / 250.0;
    }
    b.c = (double *)malloc(sizeof(double) * (size_t)n);
    b.l = (double *)malloc(sizeof(double) * (size_t)n);
    b.u = (double *)malloc(sizeof(double) * (size_t)n);
    for (int64_t j = 0; j < n; ++j) {
        b.c[j] = (double)(rnd() % 100) / 10.0;
        b.l[j] = (rnd() % 5 == 0) ? -INFINITY : 0.0;
        b.u[j] = (rnd() % 4 == 0) ? INFINITY : 1.0 + (double)(rnd() % 9);
    }
    b.rhs = (double *)malloc(sizeof(double) * (size_t)(m ? m : 1));
    b.rt = (uint8_t *)malloc((size_t)(m ? m : 1));
    for (int64_t i = 0; i < m; ++i) {
        b.rhs[i] = (double)(rnd() % 50) / 7.0;
        b.rt[i] = (rnd() % 2) ? PDHG_ROW_GE : PDHG_ROW_EQ;
    }
    return b;
}

static void free_lp(lp_buf *b)
{
    free(b->rp);
    free(b->ci);
    free(b->v);
    free(b->c);
    free(b->l);
    free(b->u);
    free(b->rhs);
    free(b->rt);
}

static pdhg_lp desc(const lp_buf *b)
{
    pdhg_lp d;
    d.n = b->n;
    d.m = b->m;
    d.nnz = b->nnz;
    d.row_ptr = b->rp;
    d.col = b->ci;
    d.val = b->v;
    d.c = b->c;
    d.rhs = b->rhs;
    d.l = b->l;
    d.u = b->u;
    d.row_type = b->rt;
    d.mem = PDHG_MEM_HOST;
    return d;
}

int main(void)
{
    pdhg_opts o;
    pdhg_default_opts(&o);

    /* valid single LPs of several shapes, every precision, with the extra
     * workspace users (unroll record, fishnet points, trace ring) */
    const int64_t shapes[][3] = {{1, 1, 1}, {0, 5, 1}, {40, 90, 12}, {700, 1500, 300}, {3000, 2000, 2500}};
    for (int s = 0; s < 5; ++s) {
        lp_buf b = make_lp(shapes[s][0], shapes[s][1], (int)shapes[s][2]);
        pdhg_lp d = desc(&b);
        for (int prec = 0; prec < 2; ++prec) {
            pdhg_opts t = o;
            t.precision = prec;
            EXPECT(pdhg_workspace_bytes(&d, 1, &t) > 0);
            t.unroll_capacity = 20;
            t.unroll_checkpoint = 3;
            t.fishnet_points = 16;
            t.trace_capacity = 100;
            EXPECT(pdhg_workspace_bytes(&d, 1, &t) > 0);
        }
        free_lp(&b);
    }

    /* a batch with many bins in use, custom bins and rows per group */
    {
        lp_buf bs[8];
        pdhg_lp ds[8];
        for (int i = 0; i < 8; ++i) {
            bs[i] = make_lp(200 + 97 * i, 300 + 51 * i, 600);
            ds[i] = desc(&bs[i]);
        }
        EXPECT(pdhg_workspace_bytes(ds, 8, &o) > 0);
        pdhg_opts t = o;
        const int32_t lim[8] = {2, 4, 8, 16, 32, 64, 128, 0};
        const int32_t rows[8] = {4, 4, 2, 2, 1, 1, 1, 1};
        memcpy(t.bin_len_dual, lim, sizeof lim);
        memcpy(t.bin_len_primal, lim, sizeof lim);
        memcpy(t.bin_rows_dual, rows, sizeof rows);
        memcpy(t.bin_rows_primal, rows, sizeof rows);
        EXPECT(pdhg_workspace_bytes(ds, 8, &t) > 0);
        /* the autotuner's workspace bound, without a workspace */
        size_t need = 0;
        pdhg_opts best;
        EXPECT(pdhg_autotune(ds, 8, &o, NULL, 0, &need, 1, 0, &best, NULL) == PDHG_ERR_NOMEM);
        EXPECT(need >= pdhg_workspace_bytes(ds, 8, &o));
        /* one bad instance in the batch */
        bs[5].ci[0] = (int32_t)bs[5].n;
        EXPECT(pdhg_workspace_bytes(ds, 8, &o) == 0);
        EXPECT(strstr(pdhg_last_error(), "5") != NULL);
        bs[5].ci[0] = 0;
        for (int i = 0; i < 8; ++i) free_lp(&bs[i]);
    }

    /* rejected inputs */
    {
        lp_buf b = make_lp(50, 80, 20);
        pdhg_lp d = desc(&b);
        EXPECT(pdhg_workspace_bytes(&d, 1, &o) > 0);
        int64_t keep = b.rp[10];
        b.rp[10] = b.rp[11] + 1; /* not monotone */
        EXPECT(pdhg_workspace_bytes(&d, 1, &o) == 0);
        b.rp[10] = keep;
        b.ci[b.nnz - 1] = -1;
        EXPECT(pdhg_workspace_bytes(&d, 1, &o) == 0);
        b.ci[b.nnz - 1] = 0;
        b.v[3] = NAN;
        EXPECT(pdhg_workspace_bytes(&d, 1, &o) == 0);
        b.v[3] = 1.0;
        b.c[2] = INFINITY;
        EXPECT(pdhg_workspace_bytes(&d, 1, &o) == 0);
        b.c[2] = 1.0;
        b.l[4] = 5.0;
        b.u[4] = 4.0;
        EXPECT(pdhg_workspace_bytes(&d, 1, &o) == 0);
        b.u[4] = 6.0;
        b.rt[7] = 9;
        EXPECT(pdhg_workspace_bytes(&d, 1, &o) == 0);
        b.rt[7] = PDHG_ROW_EQ;
        d.mem = 7;
        EXPECT(pdhg_workspace_bytes(&d, 1, &o) == 0);
        d.mem = PDHG_MEM_HOST;
        d.nnz = b.nnz + 1; /* row_ptr[m] != nnz */
        EXPECT(pdhg_workspace_bytes(&d, 1, &o) == 0);
        d.nnz = b.nnz;
        d.row_ptr = NULL;
        EXPECT(pdhg_workspace_bytes(&d, 1, &o) == 0);
        d.row_ptr = b.rp;
        EXPECT(pdhg_workspace_bytes(&d, 0, &o) == 0);
        EXPECT(pdhg_workspace_bytes(NULL, 1, &o) == 0);
        pdhg_opts t = o;
        t.check_every = 0;
        EXPECT(pdhg_workspace_bytes(&d, 1, &t) == 0);
        t = o;
        t.fishnet_points = 12;
        EXPECT(pdhg_workspace_bytes(&d, 1, &t) == 0);
        t = o;
        t.trace_capacity = -3;
        EXPECT(pdhg_workspace_bytes(&d, 1, &t) == 0);
        t = o;
        t.bin_rows_dual[0] = 3;
        EXPECT(pdhg_workspace_bytes(&d, 1, &t) == 0);
        t = o;
        t.bin_rows_primal[6] = 2;
        EXPECT(pdhg_workspace_bytes(&d, 1, &t) == 0);
        t = o;
        t.bin_len_dual[2] = -5;
        EXPECT(pdhg_workspace_bytes(&d, 1, &t) == 0);
        EXPECT(pdhg_workspace_bytes(&d, 1, &o) > 0);
        free_lp(&b);
    }

    /* fishnet round counts */
    for (int p = 2; p <= 64; p *= 2) {
        int32_t rounds = 0;
        int64_t draws = -1;
        EXPECT(pdhg_fishnet_rounds(p, &rounds, &draws) == PDHG_OK);
        EXPECT(rounds > 0 && draws >= 0);
    }
    {
        int32_t rounds;
        int64_t draws;
        EXPECT(pdhg_fishnet_rounds(3, &rounds, &draws) != PDHG_OK);
        EXPECT(pdhg_fishnet_rounds(128, &rounds, &draws) != PDHG_OK);
    }

    if (fails) {
        fprintf(stderr, "%d expectation(s) failed\n", fails);
        return 1;
    }
    printf("host paths ok\n");
    return 0;
}
