/*
 * Oracle P7Viterbi filter: plain scalar C, one residue row and one model
 * node at a time.  TEST INFRASTRUCTURE ONLY: the GPU library's results are
 * compared with it; it shares no code, header or table with the library.
 *
 * What is computed (paper Sec. 2.1, Eq. 1 for the match, insert and delete
 * cells; the special states N, B, E, C, J of the Plan-7 model around them),
 * in int16 saturating arithmetic (every sum clamped to [-32768, 32767];
 * -32768 is -inf), for residues x_1..x_L and nodes j = 1..M:
 *
 *   M[i][j] = msc_j(x_i) + max( M[i-1][j-1] + tMM_{j-1},
 *                               I[i-1][j-1] + tIM_{j-1},
 *                               D[i-1][j-1] + tDM_{j-1},
 *                               B[i-1]      + tBM )
 *   I[i][j] =              max( M[i-1][j]   + tMI_j,
 *                               I[i-1][j]   + tII_j )      (insert score 0)
 *   D[i][j] =              max( M[i][j-1]   + tMD_{j-1},
 *                               D[i][j-1]   + tDD_{j-1} )
 *   (terms with node 0 are -inf), then the special states of row i:
 *   E[i] = max_j M[i][j]                         (local exit, score 0)
 *   J[i] = max( J[i-1] + tJJ, E[i] + tEJ )
 *   C[i] = max( C[i-1] + tCC, E[i] + tEC )
 *   N[i] = N[i-1] + tNN
 *   B[i] = max( N[i] + tNB, J[i] + tJB )
 * Row 0: N = 0, B = N + tNB, every other value -inf.  Each "+" above is a
 * saturating int16 add, each max a plain max.  If some E[i] reaches 32767
 * the score has saturated: the result is (32767, overflow flag 1).
 * Otherwise the score is C[L] + tCT with flag 0.
 *
 * Tables: msc[x * M + j - 1] (x in 0..31), trans[t * M + j - 1] with t in
 * the order MM, MI, MD, IM, II, DM, DD (transitions out of node j).
 */
#include <stdint.h>
#include <stdlib.h>
#include <pthread.h>
#include <stdatomic.h>

enum { P7_NEG = -32768, P7_POS = 32767 };

static int sat(int v) { return v < P7_NEG ? P7_NEG : (v > P7_POS ? P7_POS : v); }
static int mx(int a, int b) { return a > b ? a : b; }

typedef struct {
    int NN, JJ, CC, NB, JB, CT, EJ, EC;
} p7_len;

/* One sequence.  rows: caller scratch of 6 * M ints. */
static void p7_one(const int16_t *msc, const int16_t *trans, int M, int tbm,
                   const p7_len *t, const uint8_t *x, int64_t L, int *rows,
                   int16_t *score, uint8_t *flag)
{
    const int16_t *tMM = trans, *tMI = trans + M, *tMD = trans + 2 * M,
                  *tIM = trans + 3 * M, *tII = trans + 4 * M, *tDM = trans + 5 * M,
                  *tDD = trans + 6 * M;
    int *pM = rows, *pI = rows + M, *pD = rows + 2 * M;     /* row i-1 */
    int *cM = rows + 3 * M, *cI = rows + 4 * M, *cD = rows + 5 * M;   /* row i */
    for (int j = 0; j < M; j++) pM[j] = pI[j] = pD[j] = P7_NEG;
    int xN = 0, xB = sat(xN + t->NB), xJ = P7_NEG, xC = P7_NEG;
    int overflow = 0;
    for (int64_t i = 0; i < L; i++) {
        const int16_t *e = msc + (size_t)x[i] * (size_t)M;
        const int b = sat(xB + tbm);
        int xE = P7_NEG;
        for (int j = 0; j < M; j++) {            /* node j + 1 */
            int m = b;
            if (j > 0) {
                m = mx(m, sat(pM[j - 1] + tMM[j - 1]));
                m = mx(m, sat(pI[j - 1] + tIM[j - 1]));
                m = mx(m, sat(pD[j - 1] + tDM[j - 1]));
            }
            cM[j] = sat(m + e[j]);
            cI[j] = mx(sat(pM[j] + tMI[j]), sat(pI[j] + tII[j]));
            cD[j] = j > 0 ? mx(sat(cM[j - 1] + tMD[j - 1]), sat(cD[j - 1] + tDD[j - 1]))
                          : P7_NEG;
            xE = mx(xE, cM[j]);
        }
        if (xE >= P7_POS) { overflow = 1; break; }
        xJ = mx(sat(xJ + t->JJ), sat(xE + t->EJ));
        xC = mx(sat(xC + t->CC), sat(xE + t->EC));
        xN = sat(xN + t->NN);
        xB = mx(sat(xN + t->NB), sat(xJ + t->JB));
        int *s;
        s = pM; pM = cM; cM = s;
        s = pI; pI = cI; cI = s;
        s = pD; pD = cD; cD = s;
    }
    *score = (int16_t)(overflow ? P7_POS : sat(xC + t->CT));
    *flag = (uint8_t)overflow;
}

void oracle_p7_seq(const int16_t *msc, const int16_t *trans, int M, int tbm,
                   const int *lenmodel, const uint8_t *x, int64_t L,
                   int16_t *score, uint8_t *flag)
{
    p7_len t = {lenmodel[0], lenmodel[1], lenmodel[2], lenmodel[3],
                lenmodel[4], lenmodel[5], lenmodel[6], lenmodel[7]};
    int *rows = (int *)malloc(sizeof(int) * 6 * (size_t)(M > 0 ? M : 1));
    p7_one(msc, trans, M, tbm, &t, x, L, rows, score, flag);
    free(rows);
}

/* Many sequences on a pool of threads.  lenmodels: [n][8] per sequence
 * (the length model of its own length), order: the sequences to score. */
typedef struct {
    const int16_t *msc, *trans;
    int M, tbm;
    const int *lenmodels;
    const uint8_t *res;
    const int64_t *offsets, *order;
    int64_t n;
    _Atomic int64_t next;
    int16_t *score;
    uint8_t *flag;
} p7_job;

static void *p7_worker(void *arg)
{
    p7_job *j = (p7_job *)arg;
    int *rows = (int *)malloc(sizeof(int) * 6 * (size_t)(j->M > 0 ? j->M : 1));
    if (!rows) return NULL;
    for (;;) {
        int64_t t = atomic_fetch_add(&j->next, 1);
        if (t >= j->n) break;
        int64_t s = j->order[t];
        const int *lm = j->lenmodels + 8 * s;
        p7_len len = {lm[0], lm[1], lm[2], lm[3], lm[4], lm[5], lm[6], lm[7]};
        p7_one(j->msc, j->trans, j->M, j->tbm, &len, j->res + j->offsets[s],
               j->offsets[s + 1] - j->offsets[s], rows, j->score + s, j->flag + s);
    }
    free(rows);
    return NULL;
}

int oracle_p7_batch(const int16_t *msc, const int16_t *trans, int M, int tbm,
                    const int *lenmodels, const uint8_t *res, const int64_t *offsets,
                    const int64_t *order, int64_t n, int nthreads,
                    int16_t *score, uint8_t *flag)
{
    p7_job job = {msc, trans, M, tbm, lenmodels, res, offsets, order, n, 0, score, flag};
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    pthread_t th[256];
    int started = 0;
    for (int i = 0; i < nthreads; i++)
        if (pthread_create(&th[i], NULL, p7_worker, &job) == 0) started++;
    if (started == 0) return -1;
    for (int i = 0; i < started; i++) pthread_join(th[i], NULL);
    return 0;
}
