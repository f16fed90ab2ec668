/*
 * hmsv: MSV and SSV profile-HMM filters for AMD Instinct MI355X (gfx950).
 *
 * C ABI.  Plain pointers and sizes only.  "host" pointers are ordinary CPU
 * memory; "device" pointers are gfx950 global memory (for instance the data
 * pointer of a torch tensor on a ROCm device).  All calls that take a stream
 * are asynchronous on that stream; their outputs are valid once the stream
 * has completed the call.  No call throws; every call returns an hmsv_status
 * (0 = success, negative = error), and hmsv_strerror() names it.
 *
 * What is computed: the multiple-segment (MSV) and single-segment (SSV)
 * ungapped Viterbi filters of HMMER3's pipeline (paper Sec. 2.1), scoring
 * one quantized profile against every sequence of a packed database with
 * 8-bit saturating arithmetic: unsigned with an offset ("dbias") for MSV
 * (Alg. 2), signed with -inf = -128 for SSV (Alg. 7).  Results are the raw
 * 8-bit filter scores and overflow flags, one per database sequence, in the
 * caller's original sequence order.  The pipeline's next stage runs here
 * too: the gapped P7Viterbi filter (Eq. 1, 16-bit saturating) on the whole
 * database or, after a device-side selection of the filters' survivors,
 * on those only (hmsv_select, hmsv_p7_score_selected).
 */
#ifndef HMSV_H
#define HMSV_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
typedef int hmsv_status;
#define HMSV_OK            0
#define HMSV_EINVAL       -1   /* bad argument (null pointer, size, code range) */
#define HMSV_EUNSUPPORTED -2   /* valid but beyond the library's limits */
#define HMSV_ENOMEM       -3   /* device or host allocation failed */
#define HMSV_EDEVICE      -4   /* a HIP runtime call failed */
#define HMSV_ENOKERNEL    -5   /* no kernel instantiated for the requested plan */

const char *hmsv_strerror(hmsv_status s);

/* ---- model constants (MSV model of paper Sec. 2.1, Fig. 1) ------------- */
#define HMSV_K        20    /* scoring amino acids, codes 0..19 (ACDEFGHIKLMNPQRSTVWY) */
#define HMSV_KP       32    /* table rows per node (Alg. 4's 32-entry table) */
/* Residue codes: 0..19 the amino acids ACDEFGHIKLMNPQRSTVWY; 21..26 the
 * degenerate codes B = {D, N}, J = {I, L}, Z = {E, Q}, U = {C}, O = {K},
 * X = any of the twenty; 20 and 27..31 are non-scoring (-inf).  The paper's
 * table has 32 entries per node but does not say how ambiguous residues
 * score: here a degenerate code scores the background-weighted mean of its
 * members' log2 odds ratios (the expected score of a residue drawn from the
 * background restricted to the set). */
#define HMSV_DEGEN_FIRST 21
#define HMSV_DEGEN_LAST  26
#define HMSV_BASE    190    /* N/J level of the MSV special states */
#define HMSV_TEC       3    /* E->J and E->C cost, -round(3 log2 1/2) */
#define HMSV_MAX_M  3839    /* longest profile: its LDS table (21 rows x 3840 fp16) fits 160 KiB;
                               a database with degenerate codes needs 27 rows (M up to 2559
                               with 64-lane groups; HMSV_EUNSUPPORTED beyond) */
#define HMSV_MAX_BIAS 64    /* dbias bound under which the kernels may omit the 255 cap */

/* Uniform local-entry cost of a length-M profile: -round(3 log2(2/(M(M+1)))),
 * rounding half away from zero.  M >= 1.  Returns -1 for M < 1. */
int32_t hmsv_tbm(int32_t M);

/* Length-model move cost for a target of length L: -round(3 log2(3/(L+3))).
 * L >= 0.  Returns -1 for L < 0. */
int32_t hmsv_tjb(int64_t L);

/* ---- scores in nats (host) ---------------------------------------------
 * Raw 8-bit scores as log-odds in nats, for ranking and thresholds (not
 * bit-exact; P-values need a calibration the paper does not give).  The
 * filters count in third-bits (s = 3 / ln 2 units per nat) and their raw
 * scores still carry the length-model and entry costs (paper Sec. 2.1
 * defers these units to HMMER3):
 *   MSV: (raw - tjb(L) - base) / s - 3
 *   SSV: (raw + 128 - tbm(M) - 2 tjb(L) - tec) / s - 3
 * where the final 3 nats stand for the N/C/J length loops.  A sequence
 * with flags[i] = 1 (saturated) gets +infinity.
 * score: host, n raw scores (uint8_t for MSV, int8_t for SSV); flags,
 * lengths (residues per sequence, >= 0) and nats: host, n entries.  Fails
 * with HMSV_EINVAL on a null pointer, n < 0, M < 1 or a negative length. */
hmsv_status hmsv_score_nats(int32_t is_msv, int32_t M, const void *score, const uint8_t *flags,
                            const int64_t *lengths, int64_t n, double *nats);

/* P-values of scores in nats under a Gumbel null (paper Alg. 2 records a
 * P-value at each sequence end; the location mu and scale lambda of the
 * null distribution are a calibration the paper does not give, so the
 * caller supplies them): P(S >= x) = 1 - exp(-exp(-lambda (x - mu))),
 * computed without cancellation for large x; +infinity (overflow) gives 0.
 * nats, p: host arrays of n entries.  Fails with HMSV_EINVAL on a null
 * pointer, n < 0 or lambda <= 0. */
hmsv_status hmsv_gumbel_pvalue(const double *nats, int64_t n, double mu, double lambda,
                               double *p);

/* ---- quantization (host) ----------------------------------------------
 * Turns per-node match emission probabilities into the 8-bit tables of the
 * MSV (Alg. 2 sigma/dbias) and SSV (Alg. 7) kernels:
 *   r_k(x)    = round(3 log2(emis[k][x] / bg[x])) for x < 20 (-inf if emis = 0)
 *   r_k(D)    = round(3 m), m = sum_x bg[x] log2(emis[k][x] / bg[x]) / sum_x bg[x]
 *               over the members x of degenerate code D (21..26), summed in
 *               ascending code order (-inf if a member's emis = 0)
 *   dbias     = max_{k,x<20} r_k(x)
 *   cost[x][k]= min(255, dbias - r_k(x)) for x < 20 and x in 21..26 (255
 *               for -inf), 255 for x = 20 and x >= 27
 *   sc[x][k]  = max(-128, dbias - cost[x][k])
 * emis: host, [M][20] float64, row k = node k+1, columns in code order.
 * bg:   host, [20] float64 background frequencies, all > 0.
 * cost: host, [32][M] uint8 out (residue-major).  sc: host, [32][M] int8 out.
 * dbias: host, out.  Fails with HMSV_EINVAL on null pointers, M out of
 * [1, HMSV_MAX_M], non-finite or negative probabilities, or bg <= 0. */
hmsv_status hmsv_quantize(const double *emis, const double *bg, int32_t M,
                          uint8_t *cost, int8_t *sc, int32_t *dbias);

/* ---- profile ------------------------------------------------------------
 * A quantized profile whose tables live in caller-owned device memory.
 * cost (MSV) and sc (SSV) are [32][M] residue-major, as hmsv_quantize writes
 * them.  Rows 0..19 and 21..26 are read (21..26 only for databases that
 * hold degenerate codes); codes 20 and 27..31 (and the kernels' padding
 * rows) always score as -inf, i.e. cost 255 and sc -128, whatever the
 * caller's rows 20 and 27..31 hold (hmsv_quantize writes exactly those
 * values there).  The library only reads the tables.  Either table may be NULL if
 * that filter is not used.  Preconditions checked on the host:
 * 1 <= M <= HMSV_MAX_M and 0 <= dbias <= HMSV_MAX_BIAS.  MSV reads only
 * cost (and dbias), SSV only sc. */
typedef struct {
    int32_t M;
    int32_t dbias;
    const uint8_t *cost;   /* device */
    const int8_t *sc;      /* device */
} hmsv_profile;

/* ---- packed database ----------------------------------------------------
 * Opaque, device-resident copy of a sequence database, in the layout the
 * kernels stream (sequences ordered longest first, each padded to a whole
 * number of 4-residue words, with its length-model cost tjb(L) alongside).
 * It owns its device memory until hmsv_db_destroy.  This replaces the
 * paper's warp-based sequence blocks (Sec. 3.2, Alg. 1): sequences are
 * handed to lane groups dynamically instead of being pre-packed per warp.
 *
 * res:     host, concatenated residue codes (uint8, each < 32).
 * offsets: host, [nseq+1] int64, sequence i = res[offsets[i] .. offsets[i+1]).
 * Synchronous.  Fails with HMSV_EINVAL on null pointers, decreasing offsets
 * or codes >= 32; HMSV_EUNSUPPORTED if the packed size reaches 2^32 bytes,
 * a sequence is longer than 2^24 - 4 residues, or nseq >= 2^31. */
/* The paper's warp-based sequence blocks (Sec. 3.2, Alg. 1), as an
 * alternative layout to compare against hmsv_db_create's (which hands
 * sequences to lane groups dynamically): nblocks blocks (the paper: one per
 * resident warp) of width columns (the paper: 128 sequences side by side).
 * Sequences are placed longest first (ties in input order), each taking
 * its residues plus one ending residue; the first nblocks x width seed the
 * columns in order; every later one goes to the first column, sweeping
 * down from where the previous one went, whose fill plus its own stays
 * within the tallest column so far, or, when the sweep passes column 0,
 * onto the last column (the sweep then restarts at the top).  A block's
 * height is its tallest column; padding fills the other columns to it.
 * lengths: host [nseq].  container: host [nseq] out, the column of each
 * sequence in input order (may be NULL: then the ending statistics are
 * -1).  heights: host [nblocks] out (may be NULL).  Host only, allocates
 * host memory. */
typedef struct {
    int64_t real;          /* residues */
    int64_t ending;        /* ending residues (one per sequence) */
    int64_t padding;       /* padding residues */
    int64_t max_height;    /* tallest block */
    double mean_height;    /* block heights: mean and standard deviation */
    double sd_height;
    double mean_ending;    /* ending residues per block: mean and sd */
    double sd_ending;
    double prr;            /* padding / real (Table 2's PRR) */
    double efficiency;     /* mean height / max height: busy share of a grid
                              whose blocks all start together */
} hmsv_alg1_stats;
hmsv_status hmsv_alg1_pack(const int64_t *lengths, int64_t nseq, int32_t nblocks, int32_t width,
                           int32_t *container, int64_t *heights, hmsv_alg1_stats *stats);

/* Protein FASTA text (host memory, n bytes) -> residue codes and offsets
 * for hmsv_db_create.  A record starts at a '>' and its header is the rest
 * of that line; the lines up to the next '>' are its sequence.  Sequence
 * letters map case-insensitively to ACDEFGHIKLMNPQRSTVWY = 0..19 and the
 * degenerate B J Z U O X = 21..26; whitespace, digits, '*' (stop) and the
 * gap symbols '-' '.' are skipped.  Any other byte, or a residue before the
 * first header, is HMSV_EINVAL with its byte offset in *err_at (if
 * err_at is not NULL; -1 otherwise).
 * Two calls: first with res, offsets and names NULL, which sets *nres and
 * *nseq; then with caller buffers res [*nres] uint8, offsets [*nseq + 1]
 * int64 and names [*nseq][2] int64 (each header's byte offset in text and
 * its length, without the '>' and a trailing '\r'), *nres and *nseq
 * holding those counts (HMSV_EINVAL if the text does not match them).
 * res may stay NULL in the second call to get offsets and names only. */
hmsv_status hmsv_fasta_parse(const char *text, int64_t n, uint8_t *res, int64_t *offsets,
                             int64_t *names, int64_t *nres, int64_t *nseq, int64_t *err_at);

typedef struct hmsv_db hmsv_db;
hmsv_status hmsv_db_create(const uint8_t *res, const int64_t *offsets, int64_t nseq,
                           hmsv_db **out);
void hmsv_db_destroy(hmsv_db *db);
int64_t hmsv_db_nseq(const hmsv_db *db);
int64_t hmsv_db_residues(const hmsv_db *db);     /* real residues (no padding) */
int64_t hmsv_db_padded_rows(const hmsv_db *db);  /* rows the kernels run */
/* Table rows the database's scoring calls put in LDS: 27 if it holds a
 * degenerate code (21..26), else 21 (-1 for NULL).  hmsv_db_create keeps
 * codes 0..19 and 21..26 and stores every other code as 20. */
int32_t hmsv_db_table_rows(const hmsv_db *db);

/* ---- launch plan --------------------------------------------------------
 * How one filter call maps onto the GPU.  A lane group of G lanes (a power
 * of two, 1..64) aligns one sequence; each lane holds Q packed pairs of
 * cells, so the group covers 2*G*Q - 1 >= M nodes (one cell is a fixed
 * -inf node).  64/G sequences share a wavefront (the paper's
 * multi-sequence alignment, Sec. 3.1 tier 4).  waves_per_block (1..8, or
 * 1..16 for G >= 32) wavefronts share one LDS copy of the profile;
 * blocks = 0 picks a persistent grid of the resident maximum. */
typedef struct {
    int32_t G;
    int32_t Q;
    int32_t waves_per_block;
    int32_t blocks;
} hmsv_plan;

/* The library's default plan for a filter ("msv" = 1, "ssv" = 0) and M: the
 * autotuned plan (paper Sec. 3.4 chooses its kernel per model length).  A
 * table of the plans measured fastest on MI355X (gfx950, 256 CUs) per
 * filter and profile-length bin is compiled in; the bin nearest to M in
 * log distance (ties to the smaller bin) whose group width G holds the
 * profile in Q <= 32 registers per lane gives G and waves_per_block, and
 * Q = ceil((M + 1) / 2G).  Lengths no tuned width can hold fall back to the
 * narrowest group that can.  Host only; no device is queried.  Fails with
 * HMSV_EINVAL on a null plan or M < 1, HMSV_EUNSUPPORTED for
 * M > HMSV_MAX_M. */
hmsv_status hmsv_default_plan(int32_t is_msv, int32_t M, hmsv_plan *plan);

/* Bytes of LDS a plan's kernels hold per workgroup (the profile's image in
 * the kernel's layout, the same for both filters), or 0 if G is not a power
 * of two in 1..64 or Q < 1.  Plans above 160 KiB are rejected by the
 * scoring calls (HMSV_EUNSUPPORTED); a scheduler can add the figures of
 * kernels it wants to co-reside on one CU.  This is the 21-row image; on a
 * database that holds degenerate codes it has 27 rows (x 27 / 21). */
size_t hmsv_plan_lds_bytes(int32_t G, int32_t Q);

/* The plan a call with plan = NULL uses on this database: hmsv_default_plan,
 * or, when the database holds degenerate codes and that plan's 27-row image
 * does not fit the LDS, the narrowest lane group whose image does (LDS
 * bytes are then hmsv_plan_lds_bytes x 27 / 21).  HMSV_EUNSUPPORTED if none
 * does (or, for MSV, if the exact pass's 64-lane image does not). */
hmsv_status hmsv_db_default_plan(const hmsv_db *db, int32_t is_msv, int32_t M, hmsv_plan *plan);

/* Device workspace needed by a scoring call on a database of nseq
 * sequences (bytes; pass the database's full sequence count, also for
 * range calls): the work-queue counters, the MSV per-residue best scores,
 * the profile converted to the kernel's LDS layout, the records of split
 * sequences' segments (at most 131072 segments of 65536 sequences per
 * call; about 8.7 MB), and 16 bytes per sequence for the MSV rescoring
 * windows. */
size_t hmsv_workspace_bytes(int64_t nseq);

/* ---- scoring -----------------------------------------------------------
 * MSV (paper Alg. 2): score[i] = raw 8-bit MSV score of sequence i (the
 * final scJ), flags[i] = 1 if the biased score saturated (then score = 255).
 * SSV (paper Alg. 7): score[i] = best single-segment score in signed 8-bit
 * (-128 = no positive segment), flags[i] = 1 on saturation (score = 127).
 * score, flags: device, [nseq] each, written for every sequence (NULL
 * allowed when the database or range holds no sequence).
 * workspace: device, hmsv_workspace_bytes(nseq) bytes, 256-byte aligned,
 * caller-owned; its content need not be initialised; calls that share a
 * workspace must be ordered on one stream.  plan: NULL for the default.  The call allocates nothing.
 * Fails with HMSV_EINVAL on null pointers or a profile outside its
 * preconditions, HMSV_ENOKERNEL if the plan was not instantiated,
 * HMSV_EDEVICE if the launch fails.
 *
 * A launch takes at least as long as one lane group needs for its longest
 * sequence.  Sequences much longer than the launch's mean work per lane
 * group (total rows / lane groups) are therefore cut into segments of about
 * that many rows, scored in parallel and combined: each segment starts
 * M - 1 rows (rounded up to 16) before its own rows, so all of its own
 * cells are exact (a cell depends only on the M rows above it along its
 * diagonal), and the sequence's maximum is the maximum over its segments.
 * MSV runs every sequence with scB fixed first (exact unless the J state
 * opens, Alg. 2); a second launch on the same stream rescores, with
 * Alg. 2's special states after every row, only a window of each sequence
 * whose running max passed base + tec: from M - 1 rows (rounded up to 16)
 * before the first step of 8 or 16 rows in which a cell passed that level
 * to the end of the last such step (scB can move only there).  Scores are
 * the same either way. */
hmsv_status hmsv_msv_score(const hmsv_profile *prof, const hmsv_db *db,
                           uint8_t *score, uint8_t *flags, void *workspace,
                           const hmsv_plan *plan, hipStream_t stream);
hmsv_status hmsv_ssv_score(const hmsv_profile *prof, const hmsv_db *db,
                           int8_t *score, uint8_t *flags, void *workspace,
                           const hmsv_plan *plan, hipStream_t stream);

/* ---- MSV scoring without allocation ---------------------------------------
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  As
 * hmsv_msv_score, but the workspace is the library's own device array of
 * hmsv_workspace_bytes(HMSV_NOALLOC_MAX_SEQ) bytes (about 25 MB), one per
 * GPU, held until the process ends.  The call allocates nothing: no
 * hipMalloc, no host heap.  Every call on a GPU shares that GPU's array,
 * so calls that overlap on one GPU (different streams, or different host
 * threads) race and must be ordered by the caller; each call initialises
 * what it reads.  Fails with HMSV_EUNSUPPORTED if the database has more
 * than HMSV_NOALLOC_MAX_SEQ sequences, otherwise as hmsv_msv_score. */
#define HMSV_NOALLOC_MAX_SEQ 1048576
hmsv_status hmsv_msv_score_noalloc(const hmsv_profile *prof, const hmsv_db *db,
                                   uint8_t *score, uint8_t *flags, const hmsv_plan *plan,
                                   hipStream_t stream);

/* ---- partial scoring (serving) -------------------------------------------
 * As hmsv_msv_score / hmsv_ssv_score, but only for the sequences at
 * positions [first, first + count) of the database's processing order
 * (longest first, see hmsv_db_order); results land at their original
 * indices and other entries of score/flags are left untouched.  Lets a
 * server split one search into chunks and interleave the chunks of
 * several searches.  Fails with HMSV_EINVAL if the range is outside
 * [0, nseq]. */
hmsv_status hmsv_msv_score_range(const hmsv_profile *prof, const hmsv_db *db, int64_t first,
                                 int64_t count, uint8_t *score, uint8_t *flags,
                                 void *workspace, const hmsv_plan *plan, hipStream_t stream);
hmsv_status hmsv_ssv_score_range(const hmsv_profile *prof, const hmsv_db *db, int64_t first,
                                 int64_t count, int8_t *score, uint8_t *flags,
                                 void *workspace, const hmsv_plan *plan, hipStream_t stream);

/* How a scoring call with this filter, profile length, plan (NULL: the
 * default) and range (first = 0, count = -1: the whole database) splits its
 * longest sequences: *nsplit sequences into *nsegs segments of *seg_rows
 * rows each (the last segment of a sequence may be shorter).  For
 * diagnostics and tests; persistent-grid plans need the device the call
 * would run on.  Fails as the scoring calls do on a bad plan or range. */
hmsv_status hmsv_split_info(const hmsv_db *db, int64_t first, int64_t count, int32_t is_msv,
                            int32_t M, const hmsv_plan *plan, int32_t *nsplit,
                            int32_t *nsegs, int32_t *seg_rows);

/* Processing order of a packed database: ids[t] = original index of the
 * t-th sequence (longest first; ties keep the original order).
 * ids: host, [nseq] int64 out. */
hmsv_status hmsv_db_order(const hmsv_db *db, int64_t *ids);

/* ---- batched launches ---------------------------------------------------
 * Many queries (profiles of any length, MSV or SSV) against one database in
 * a single graph launch.  hmsv_batch_create captures, for every query, the
 * prep and filter kernels of its plan into one hipGraph whose queries are
 * spread over `branches` independent branches (longest profiles first,
 * balanced by M), so their persistent kernels can overlap on the device;
 * hmsv_batch_launch replays the whole batch with one hipGraphLaunch.
 * Every query's results are identical to its plain hmsv_*_score call with
 * the same plan.
 * Each query owns its outputs and workspace (device, caller-owned, distinct
 * per query); score is uint8 for MSV, int8 for SSV.  plan.G == 0 selects
 * the library's default (autotuned) plan.  The batch keeps pointers, not copies, of
 * the device buffers; the profile struct is copied.  branches: 1..16.
 * Fails with HMSV_EINVAL on bad arguments (including a workspace shared by
 * two queries), the errors of hmsv_*_score for a query, HMSV_EDEVICE if
 * capture or instantiation fails. */
typedef struct {
    int32_t is_msv;
    hmsv_profile prof;
    void *score;        /* device, [nseq] */
    uint8_t *flags;     /* device, [nseq] */
    void *workspace;    /* device, hmsv_workspace_bytes(nseq) */
    hmsv_plan plan;     /* plan.G == 0: default */
} hmsv_query;

typedef struct hmsv_batch hmsv_batch;
hmsv_status hmsv_batch_create(const hmsv_query *queries, int32_t nq, const hmsv_db *db,
                              int32_t branches, hmsv_batch **out);
hmsv_status hmsv_batch_launch(hmsv_batch *batch, hipStream_t stream);
void hmsv_batch_destroy(hmsv_batch *batch);

/* ---- P7Viterbi: the gapped Plan-7 Viterbi filter ------------------------
 * The pipeline's next stage (paper Sec. 2.1, Eq. 1): match, insert and
 * delete cells per node with the Plan-7 special states N, B, E, C, J
 * around them, in int16 saturating arithmetic (scores in 1/32 bit,
 * HMSV_P7_UNITS per bit; -32768 is -inf).  Per row i and node j:
 *   M[i][j] = msc_j(x_i) + max(M[i-1][j-1] + tMM, I[i-1][j-1] + tIM,
 *                              D[i-1][j-1] + tDM, B[i-1] + tbm)
 *   I[i][j] = max(M[i-1][j] + tMI, I[i-1][j] + tII)      (insert score 0)
 *   D[i][j] = max(M[i][j-1] + tMD, D[i][j-1] + tDD)
 * (transitions out of the node before j, or of j for tMI, tII), then
 * E = max_j M[i][j] (local exit), J = max(J + loop, E - 32),
 * C = max(C + loop, E - 32), N = N + loop, B = max(N + move, J + move),
 * with loop = round(32 log2(L/(L+3))), move = round(32 log2(3/(L+3))) for a
 * target of L residues (the MSV model's length model); row 0 has N = 0,
 * B = move, all else -inf.  Score = C[L] + move, or 32767 with flags = 1
 * once a row's E saturates at 32767. */
#define HMSV_P7_UNITS 32
#define HMSV_P7_MAX_M 2815  /* 64-lane groups of 22 registers: 28 table rows fill 160 KiB
                               (34 rows with degenerate codes: M up to 2047) */

/* Emissions [M][20] (as hmsv_quantize), transitions [M][7] float64
 * probabilities out of each node in the order M->M, M->I, M->D, I->M,
 * I->I, D->M, D->D, background [20] -> msc [32][M] int16 =
 * round(32 log2(emis / bg)) (-32768 for zero emissions and codes 20, 27..31;
 * degenerate codes 21..26 score round(32 m) with m as in hmsv_quantize),
 * trans_out [7][M] int16 = round(32 log2 p) (-32768 for p = 0, and for
 * every transition of node M, which has no successor and no insert state),
 * tbm = round(32 log2(2 / (M (M + 1)))), all rounded half away from zero
 * in float64.  Host memory.  Fails with HMSV_EINVAL on null pointers, M
 * outside [1, HMSV_P7_MAX_M], negative or non-finite probabilities, or
 * bg <= 0. */
hmsv_status hmsv_p7_quantize(const double *emis, const double *trans, const double *bg,
                             int32_t M, int16_t *msc, int16_t *trans_out, int32_t *tbm);

/* The length model of a target of L residues: loop = round(32 log2(L /
 * (L + 3))) (N->N, J->J, C->C; -32768 for L = 0), move = round(32 log2(3 /
 * (L + 3))) (N->B, J->B, C->T).  hmsv_db_create stores it per record.
 * HMSV_EINVAL on null pointers or L < 0. */
hmsv_status hmsv_p7_length_model(int64_t L, int32_t *loop, int32_t *move);

/* A quantized P7 profile; tables in caller-owned device memory as
 * hmsv_p7_quantize writes them. */
typedef struct {
    int32_t M;
    int32_t tbm;
    const int16_t *msc;     /* device, [32][M] */
    const int16_t *trans;   /* device, [7][M] */
} hmsv_p7_profile;

/* LDS bytes per workgroup of a P7 plan's kernel (0 for an invalid shape). */
size_t hmsv_p7_lds_bytes(int32_t G, int32_t Q);

/* Default P7 plan for M: the measured plan of the nearest profile-length
 * bin (group width and waves per block, with the fewest registers per lane
 * that hold the profile: at most 16, 22 for 64-lane groups), or the
 * narrowest group that holds it; persistent grid. */
hmsv_status hmsv_p7_default_plan(int32_t M, hmsv_plan *plan);

/* Scores every sequence of the database: score[i] int16, flags[i] = 1 on
 * saturation (score 32767), both device arrays of nseq entries in the
 * caller's original order.  workspace: hmsv_workspace_bytes(nseq) bytes,
 * 256-byte aligned (calls sharing it must be ordered on one stream).  plan:
 * NULL for the default (plans take 1..8 waves per block, 1..16 for
 * 64-lane groups of at most 18 registers or of 20).  Lane groups take
 * the records (longest first) from a queue in the workspace as they finish
 * one; each sequence runs exactly its L rows.  score and flags may be
 * NULL for a database without sequences.
 * Asynchronous on the stream; allocates nothing.  Fails with HMSV_EINVAL on
 * null pointers or a bad plan, HMSV_EUNSUPPORTED for M > HMSV_P7_MAX_M,
 * HMSV_ENOKERNEL if the plan was not instantiated, HMSV_EDEVICE if the
 * launch fails. */
hmsv_status hmsv_p7_score(const hmsv_p7_profile *prof, const hmsv_db *db, int16_t *score,
                          uint8_t *flags, void *workspace, const hmsv_plan *plan,
                          hipStream_t stream);

/* ---- Pipeline stages on the device (Sec. 2.1) --------------------------
 * The MSV/SSV stage passes on to P7Viterbi only the sequences whose filter
 * score reaches a threshold (a few percent of a database).  hmsv_select
 * finds them on the device and hmsv_p7_score_selected scores just those, so
 * the stages chain on one stream with no host round trip.
 *
 * hmsv_select: score = a filter call's score array (device, nseq entries in
 * the original order; uint8 for is_msv = 1, int8 for is_msv = 0), flags its
 * overflow flags (an overflowed sequence always passes).  Writes to
 * positions (device, int32, capacity nseq) the processing-order positions
 * p (hmsv_db_order maps p to the original id) of the sequences with flag
 * set or score >= threshold, in increasing p (so longest first), and their
 * number to *count (device int32).  Deterministic.  workspace:
 * hmsv_workspace_bytes(nseq) bytes, 256-byte aligned; it uses the part
 * that P7 calls leave alone, so the same workspace may serve the P7 call
 * that follows on the stream.  Asynchronous; allocates nothing.  score
 * and flags may be NULL for a database without sequences (*count = 0).
 * HMSV_EINVAL on null pointers, is_msv not 0/1 or a misaligned workspace,
 * HMSV_EDEVICE if a launch fails. */
hmsv_status hmsv_select(const hmsv_db *db, const void *score, const uint8_t *flags,
                        int32_t is_msv, int32_t threshold, int32_t *positions, int32_t *count,
                        void *workspace, hipStream_t stream);

/* hmsv_p7_score restricted to the records at positions[0 .. *count)
 * (device; processing-order positions in 0..nseq-1, each at most once, in
 * any order, though longest first balances best: what hmsv_select writes;
 * a count above nseq is taken as nseq, one below 0 as 0).  score and flags are written at those records'
 * original ids only; every other entry keeps its value.  The other
 * arguments and errors are hmsv_p7_score's (the launch grid is sized for the
 * whole database; lane groups left without a record exit at once), except
 * that plan = NULL picks 64-lane groups (the fewest registers per lane
 * that hold the profile): a selection of a few percent of a database is
 * bound by the time of its longest records, which those groups run
 * fastest.  A selection of a large share of the database runs at higher
 * throughput on the hmsv_p7_default_plan plan. */
hmsv_status hmsv_p7_score_selected(const hmsv_p7_profile *prof, const hmsv_db *db,
                                   const int32_t *positions, const int32_t *count,
                                   int16_t *score, uint8_t *flags, void *workspace,
                                   const hmsv_plan *plan, hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* HMSV_H */
