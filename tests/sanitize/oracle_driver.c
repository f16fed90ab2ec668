/* Runs the oracle's C filters (MSV, SSV, P7Viterbi; single sequences and
 * the threaded batch entry points) on random tables and sequences,
 * including empty sequences, every code 0..31 and one-node profiles.  Built
 * with AddressSanitizer and UndefinedBehaviorSanitizer by
 * tests/test_sanitizers.py: any out-of-bounds access, use after free, leak
 * or undefined operation ends the run with a report and a non-zero status.
 * The values computed are not checked here (the oracle's pins do that). */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

void oracle_msv_seq(const uint8_t *cost, int M, int dbias, int base, int tec, int tjbm,
                    const uint8_t *x, int64_t L, uint8_t *score, uint8_t *flag);
void oracle_ssv_seq(const int8_t *sc, int M, const uint8_t *x, int64_t L, int8_t *score,
                    uint8_t *flag);
int oracle_batch(int is_msv, const uint8_t *cost, const int8_t *sc, int M, int dbias, int base,
                 int tec, int tbm, const uint8_t *res, const int64_t *offsets,
                 const int32_t *tjb, const int64_t *order, int64_t n, int nthreads,
                 uint8_t *score, uint8_t *flag);
void oracle_p7_seq(const int16_t *msc, const int16_t *trans, int M, int tbm,
                   const int *lenmodel, const uint8_t *x, int64_t L, int16_t *score,
                   uint8_t *flag);
int oracle_p7_batch(const int16_t *msc, const int16_t *trans, int M, int tbm,
                    const int *lenmodels, const uint8_t *res, const int64_t *offsets,
                    const int64_t *order, int64_t n, int nthreads, int16_t *score,
                    uint8_t *flag);

static uint64_t state = 88172645463325252ull;
static uint32_t rnd(void) {           /* xorshift64 */
    state ^= state << 13;
    state ^= state >> 7;
    state ^= state << 17;
    return (uint32_t)(state >> 16);
}

int main(void) {
    const int Ms[] = {1, 2, 17, 100, 400};
    for (size_t mi = 0; mi < sizeof(Ms) / sizeof(Ms[0]); ++mi) {
        const int M = Ms[mi];
        uint8_t *cost = malloc(32 * (size_t)M);
        int8_t *sc = malloc(32 * (size_t)M);
        int16_t *msc = malloc(sizeof(int16_t) * 32 * (size_t)M);
        int16_t *tr = malloc(sizeof(int16_t) * 7 * (size_t)M);
        for (int i = 0; i < 32 * M; ++i) {
            cost[i] = (uint8_t)(rnd() % 256);
            sc[i] = (int8_t)((int)(rnd() % 256) - 128);
            msc[i] = (rnd() % 20 == 0) ? (int16_t)-32768 : (int16_t)((int)(rnd() % 700) - 500);
        }
        for (int i = 0; i < 7 * M; ++i)
            tr[i] = (rnd() % 15 == 0) ? (int16_t)-32768 : (int16_t)(-(int)(rnd() % 300));
        const int n = 40;
        int64_t off[41];
        off[0] = 0;
        for (int s = 0; s < n; ++s) off[s + 1] = off[s] + (s % 7 == 0 ? 0 : (int64_t)(rnd() % 600));
        uint8_t *res = malloc((size_t)(off[n] > 0 ? off[n] : 1));
        for (int64_t i = 0; i < off[n]; ++i) res[i] = (uint8_t)(rnd() % 32);
        int32_t tjb[40];
        int lm[40 * 8];
        int64_t order[40];
        for (int s = 0; s < n; ++s) {
            tjb[s] = (int32_t)(rnd() % 40);
            for (int k = 0; k < 8; ++k) lm[8 * s + k] = -(int)(rnd() % 100);
            order[s] = n - 1 - s;
        }
        uint8_t score[40], flag[40];
        int8_t ss;
        int16_t ps[40];
        for (int s = 0; s < n; ++s) {
            const int64_t L = off[s + 1] - off[s];
            oracle_msv_seq(cost, M, (int)(rnd() % 65), 190, 3, (int)(rnd() % 60), res + off[s], L,
                           &score[s], &flag[s]);
            oracle_ssv_seq(sc, M, res + off[s], L, &ss, &flag[s]);
            oracle_p7_seq(msc, tr, M, -(int)(rnd() % 400), lm + 8 * s, res + off[s], L, &ps[s],
                          &flag[s]);
        }
        for (int is_msv = 0; is_msv < 2; ++is_msv) {
            if (oracle_batch(is_msv, cost, sc, M, 20, 190, 3, 10, res, off, tjb, order, n, 3,
                             score, flag) != 0)
                return 2;
            if (oracle_batch(is_msv, cost, sc, M, 20, 190, 3, 10, res, off, tjb, NULL, n, 2,
                             score, flag) != 0)
                return 2;
        }
        if (oracle_p7_batch(msc, tr, M, -300, lm, res, off, order, n, 3, ps, flag) != 0) return 3;
        free(cost);
        free(sc);
        free(msc);
        free(tr);
        free(res);
    }
    puts("oracle driver done");
    return 0;
}
