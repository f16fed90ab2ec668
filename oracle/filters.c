/*
 * Oracle MSV and SSV filters: plain scalar C, one residue row and one model
 * node at a time.  TEST INFRASTRUCTURE ONLY: the GPU library's results are
 * compared with this file's.  It shares no code, header or table with
 * the library, and nothing in the library may call it.
 *
 * What is computed (paper Sec. 2.1 for the models, Alg. 2 and Alg. 7 for the
 * per-cell operations; the special-state updates and the quantized tables are
 * the HMMER3 MSV model's, which the paper uses without restating):
 *
 *  MSV (Alg. 2), unsigned 8-bit saturating, one row i per residue x_i:
 *    v      = max(gamma, scB)          vmaxu4   (gamma = M[k-1] of row i-1)
 *    v      = v + dbias, capped 255    vaddus4
 *    v      = v - sigma, floored 0     vsubus4  (sigma = cost_k(x_i))
 *    scE    = max(scE, v)              vmaxu4
 *   After the row (special states, Alg. 2 "update special states"):
 *    overflow if scE >= 255 - dbias (the biased sum would have capped at 255)
 *    scJ    = max(scJ, scE - tec floored 0)
 *    scB    = max(base, scJ) - (tjb + tbm), floored 0
 *   Node 1's predecessor in the row above is -inf (0).  Score = scJ, or
 *   255 with the overflow flag.
 *
 *  SSV (Alg. 7), signed 8-bit saturating, -inf = -128 (0x80):
 *    v      = clamp(gamma + sc_k(x_i), -128, 127)
 *    scE    = max(scE, v)
 *   overflow if scE reaches 127.  Score = scE (never reset), or 127 with
 *   the overflow flag.
 *
 * Tables are residue-major: cost[x * M + k], sc[x * M + k], x in 0..31.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <stdatomic.h>

static int imax(int a, int b) { return a > b ? a : b; }
static int imin(int a, int b) { return a < b ? a : b; }

/* One sequence through the MSV filter.  m_row is caller scratch of M ints. */
static void msv_one(const uint8_t *cost, int M, int dbias, int base, int tec,
                    int tjbm, const uint8_t *x, int64_t L, int *m_row,
                    uint8_t *score, uint8_t *flag)
{
    int scJ = 0;
    int scB = imax(0, base - tjbm);
    int overflow = 0;
    for (int k = 0; k < M; k++) m_row[k] = 0;           /* -inf */
    for (int64_t i = 0; i < L; i++) {
        const uint8_t *sigma_row = cost + (size_t)x[i] * (size_t)M;
        int scE = 0;
        int gamma = 0;                                   /* M_0 of row i-1 = -inf */
        for (int k = 0; k < M; k++) {
            int old = m_row[k];
            int v = imax(gamma, scB);
            v = imin(255, v + dbias);
            v = imax(0, v - (int)sigma_row[k]);
            m_row[k] = v;
            scE = imax(scE, v);
            gamma = old;
        }
        if (scE >= 255 - dbias) { overflow = 1; break; }
        scJ = imax(scJ, imax(0, scE - tec));
        scB = imax(0, imax(base, scJ) - tjbm);
    }
    *score = overflow ? 255 : (uint8_t)scJ;
    *flag = (uint8_t)overflow;
}

/* One sequence through the SSV filter.  d_row is caller scratch of M ints. */
static void ssv_one(const int8_t *sc, int M, const uint8_t *x, int64_t L,
                    int *d_row, int8_t *score, uint8_t *flag)
{
    int scE = -128;
    int overflow = 0;
    for (int k = 0; k < M; k++) d_row[k] = -128;         /* -inf */
    for (int64_t i = 0; i < L; i++) {
        const int8_t *sc_row = sc + (size_t)x[i] * (size_t)M;
        int gamma = -128;
        for (int k = 0; k < M; k++) {
            int old = d_row[k];
            int v = gamma + (int)sc_row[k];
            v = imax(-128, imin(127, v));
            d_row[k] = v;
            scE = imax(scE, v);
            gamma = old;
        }
        if (scE == 127) { overflow = 1; break; }
    }
    *score = overflow ? 127 : (int8_t)scE;
    *flag = (uint8_t)overflow;
}

/* ---- exported single-sequence entry points --------------------------- */

void oracle_msv_seq(const uint8_t *cost, int M, int dbias, int base, int tec,
                    int tjbm, const uint8_t *x, int64_t L,
                    uint8_t *score, uint8_t *flag)
{
    int *row = (int *)malloc(sizeof(int) * (size_t)(M > 0 ? M : 1));
    msv_one(cost, M, dbias, base, tec, tjbm, x, L, row, score, flag);
    free(row);
}

void oracle_ssv_seq(const int8_t *sc, int M, const uint8_t *x, int64_t L,
                    int8_t *score, uint8_t *flag)
{
    int *row = (int *)malloc(sizeof(int) * (size_t)(M > 0 ? M : 1));
    ssv_one(sc, M, x, L, row, score, flag);
    free(row);
}

/* ---- multithreaded batch over a list of sequences ------------------- */

typedef struct {
    int is_msv;
    const uint8_t *cost; const int8_t *sc; int M, dbias, base, tec, tbm;
    const uint8_t *res; const int64_t *offsets; const int32_t *tjb;
    const int64_t *order; int64_t n;
    uint8_t *score; uint8_t *flag;
    atomic_llong next;
} batch_t;

static void *batch_worker(void *arg)
{
    batch_t *b = (batch_t *)arg;
    int *row = (int *)malloc(sizeof(int) * (size_t)(b->M > 0 ? b->M : 1));
    for (;;) {
        long long t = atomic_fetch_add(&b->next, 1);
        if (t >= b->n) break;
        int64_t s = b->order ? b->order[t] : t;
        const uint8_t *x = b->res + b->offsets[s];
        int64_t L = b->offsets[s + 1] - b->offsets[s];
        if (b->is_msv)
            msv_one(b->cost, b->M, b->dbias, b->base, b->tec, b->tjb[s] + b->tbm,
                    x, L, row, &b->score[s], &b->flag[s]);
        else
            ssv_one(b->sc, b->M, x, L, row, (int8_t *)&b->score[s], &b->flag[s]);
    }
    free(row);
    return NULL;
}

/* Score sequences order[0..n) (or 0..n when order is NULL).  Results are
 * written at the sequence's own index.  Returns 0, or -1 on thread failure. */
int oracle_batch(int is_msv, const uint8_t *cost, const int8_t *sc, int M,
                 int dbias, int base, int tec, int tbm,
                 const uint8_t *res, const int64_t *offsets, const int32_t *tjb,
                 const int64_t *order, int64_t n, int nthreads,
                 uint8_t *score, uint8_t *flag)
{
    batch_t b;
    memset(&b, 0, sizeof b);
    b.is_msv = is_msv; b.cost = cost; b.sc = sc; b.M = M; b.dbias = dbias;
    b.base = base; b.tec = tec; b.tbm = tbm; b.res = res; b.offsets = offsets;
    b.tjb = tjb; b.order = order; b.n = n; b.score = score; b.flag = flag;
    atomic_init(&b.next, 0);
    if (nthreads < 1) nthreads = 1;
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)nthreads);
    int started = 0, rc = 0;
    for (int t = 0; t < nthreads; t++) {
        if (pthread_create(&th[t], NULL, batch_worker, &b) != 0) { rc = -1; break; }
        started++;
    }
    if (started == 0) batch_worker(&b);
    for (int t = 0; t < started; t++) pthread_join(th[t], NULL);
    free(th);
    return rc;
}
