// Host side of libhmsv: quantization, database packing, plan selection and
// kernel dispatch.  The C ABI is declared in include/hmsv.h.
#include "hmsv.h"
#include "hmsv_internal.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <numeric>
#include <vector>

using namespace hmsv;

namespace hmsv {
int register_kernels(const KernelEntry *entries, int n);
}

struct hmsv_batch {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int nq = 0;
};

struct hmsv_db {
    int64_t nseq = 0;
    int64_t residues = 0;
    int64_t rows = 0;
    uint8_t *d_res = nullptr;
    SeqRec *d_seqs = nullptr;
    uint32_t *d_p7len = nullptr;   // per record: P7 length model, loop | move << 16
    uint32_t pad_off = 0;
    int32_t table_rows = kRows;    // table rows its scoring calls need (kDegenRows
                                   // if it holds degenerate codes 21..26)
    int device = 0;
    std::vector<int64_t> order;   // processing order -> original index
    std::vector<int64_t> cum_rows; // rows run by records [0, t), t = 0..nseq
};

namespace {

// Round half away from zero of a finite double.
double rhaz(double v) {
    double t = std::trunc(v);
    if (std::fabs(v - t) >= 0.5) t += (v > 0 ? 1.0 : -1.0);
    return t;
}

// Third-bit cost of a probability p in (0, 1]: -round(3 log2 p).
int32_t third_bit_cost(double p) { return (int32_t)(-rhaz(3.0 * std::log2(p))); }

// P7Viterbi score of a probability (or odds ratio) p: round(32 log2 p),
// clamped to int16; -32768 (-inf) for p = 0.
// Degenerate residue codes and their member residues (codes of
// ACDEFGHIKLMNPQRSTVWY, ascending): B = {D, N}, J = {I, L}, Z = {E, Q},
// U = {C}, O = {K}, X = any.  A degenerate code scores the
// background-weighted mean of its members' log2 odds ratios.
struct Degenerate {
    int code;
    int n;
    int member[HMSV_K];
};
constexpr Degenerate kDegenerate[] = {
    {21, 2, {2, 11}},
    {22, 2, {7, 9}},
    {23, 2, {3, 13}},
    {24, 1, {1}},
    {25, 1, {8}},
    {26, 20, {0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 15, 16, 17, 18, 19}},
};

// sum_x bg(x) log2(e(x) / bg(x)) / sum_x bg(x) over the members (summed in
// ascending code order, one rounding per operation); false if a member's
// emission is 0 (the score is then -inf).
bool degenerate_mean(const double *e, const double *bg, const Degenerate &d, double *mean) {
    double num = 0.0, den = 0.0;
    for (int t = 0; t < d.n; ++t) {
        const int x = d.member[t];
        const double ratio = e[x] / bg[x];
        if (!(ratio > 0.0)) return false;
        const double term = bg[x] * std::log2(ratio);
        num = num + term;
        den = den + bg[x];
    }
    *mean = num / den;
    return true;
}

// Packed code of an input code: residues and degenerate codes stay, every
// other code (20, 27..31) becomes the non-scoring code 20.
uint8_t keep_code(uint8_t c) {
    return c < HMSV_K || (c >= 21 && c <= 26) ? c : kInvalidCode;
}

constexpr int kP7Units = 32;
int32_t p7_score(double p) {
    if (!(p > 0.0)) return -32768;
    double v = rhaz((double)kP7Units * std::log2(p));
    return (int32_t)std::max(-32768.0, std::min(32767.0, v));
}

// The P7Viterbi length model of a target of L residues: N/J/C loops and
// N->B, J->B, C->T moves, packed as two int16.
uint32_t p7_lenmodel(int64_t L) {
    const int32_t loop = L > 0 ? p7_score((double)L / ((double)L + 3.0)) : -32768;
    const int32_t move = p7_score(3.0 / ((double)L + 3.0));
    return (uint32_t)(uint16_t)(int16_t)loop | ((uint32_t)(uint16_t)(int16_t)move << 16);
}

struct Registry {
    std::vector<KernelEntry> entries;
    ExactLaunchFn exact[kMaxExactQ + 1] = {};
    std::vector<P7KernelEntry> p7;
    const P7KernelEntry *find_p7(int G, int Q) const {
        for (const auto &e : p7)
            if (e.G == G && e.Q == Q) return &e;
        return nullptr;
    }
    const KernelEntry *find(int is_msv, int G, int Q) const {
        for (const auto &e : entries)
            if (e.is_msv == is_msv && e.G == G && e.Q == Q) return &e;
        return nullptr;
    }
};

Registry &registry() {
    static Registry r;
    return r;
}

// Launch plans the autotuner measured fastest on MI355X (gfx950, 256 CUs)
// per filter and profile-length bin, compiled in from tuned_plans.json.
struct TunedPlan { int is_msv; int bin; int G; int waves_per_block; };
const TunedPlan kTuned[] = {
#include "tuned_plans.inc"
};
constexpr int kNumTuned = (int)(sizeof(kTuned) / sizeof(kTuned[0]));


// Persistent-grid size per (kernel, waves_per_block), measured once per
// device.  A fixed table (no allocation on the scoring path); when it is
// full the figure is measured again at each call.
struct OccEntry { const KernelEntry *e; int wpb; int rows; int dev; int blocks; };
constexpr int kOccCap = 4096;
std::mutex g_occ_mu;
OccEntry g_occ[kOccCap];
int g_nocc = 0;

// Compute units of the current device (fixed table, no allocation).
int device_cus() {
    static std::mutex mu;
    static int cus[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) return 0;
    if (dev < 64) {
        std::lock_guard<std::mutex> lk(mu);
        if (cus[dev] > 0) return cus[dev];
    }
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    if (dev < 64) {
        std::lock_guard<std::mutex> lk(mu);
        cus[dev] = n;
    }
    return n;
}

int resident_blocks(const KernelEntry *e, int wpb, int rows) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    {
        std::lock_guard<std::mutex> lk(g_occ_mu);
        for (int i = 0; i < g_nocc; ++i)
            if (g_occ[i].e == e && g_occ[i].wpb == wpb && g_occ[i].rows == rows &&
                g_occ[i].dev == dev)
                return g_occ[i].blocks;
    }
    int per_cu = e->occupancy(wpb, rows);
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    int blocks = per_cu * cus;
    std::lock_guard<std::mutex> lk(g_occ_mu);
    if (g_nocc < kOccCap) g_occ[g_nocc++] = OccEntry{e, wpb, rows, dev, blocks};
    return blocks;
}

hmsv_status check_profile(const hmsv_profile *p, int is_msv) {
    if (!p) return HMSV_EINVAL;
    if (p->M < 1) return HMSV_EINVAL;
    if (p->M > HMSV_MAX_M) return HMSV_EUNSUPPORTED;
    if (p->dbias < 0 || p->dbias > HMSV_MAX_BIAS) return HMSV_EINVAL;
    if (is_msv && !p->cost) return HMSV_EINVAL;
    if (!is_msv && !p->sc) return HMSV_EINVAL;
    return HMSV_OK;
}

hmsv_status check_plan(const hmsv_plan *pl, int M, int rows = kRows) {
    if (pl->G < 1 || pl->G > 64 || (64 % pl->G) != 0) return HMSV_EINVAL;
    if (pl->Q < 1) return HMSV_EINVAL;
    if (plan_nodes(pl->G, pl->Q) < M) return HMSV_EINVAL;
    if (pl->waves_per_block < 1 || pl->waves_per_block > (pl->G >= 32 ? 16 : 8))
        return HMSV_EINVAL;
    if (pl->blocks < 0) return HMSV_EINVAL;
    if (lds_bytes(pl->G, pl->Q, rows) > (size_t)kLdsBytes) return HMSV_EUNSUPPORTED;
    return HMSV_OK;
}

// The plan of a call on a database whose images need `rows` table rows:
// the caller's, or the default; if the default's image does not fit the
// LDS with the degenerate rows, the narrowest lane group whose image does.
// MSV also needs the exact pass's image (64-lane groups) to fit.
hmsv_status resolve_plan(int is_msv, int M, int rows, const hmsv_plan *in, hmsv_plan *out) {
    if (is_msv && lds_bytes(kExactG, exact_q(M), rows) > (size_t)kLdsBytes)
        return HMSV_EUNSUPPORTED;
    if (in) {
        *out = *in;
        return check_plan(out, M, rows);
    }
    hmsv_status st = hmsv_default_plan(is_msv, M, out);
    if (st != HMSV_OK) return st;
    if (lds_bytes(out->G, out->Q, rows) <= (size_t)kLdsBytes) return check_plan(out, M, rows);
    for (int G : {1, 2, 4, 8, 16, 32, 64}) {
        const int Q = (M + 1 + 2 * G - 1) / (2 * G);
        if (Q > 32 || lds_bytes(G, Q, rows) > (size_t)kLdsBytes) continue;
        if (!registry().find(is_msv ? 1 : 0, G, Q)) continue;
        out->G = G;
        out->Q = Q;
        out->waves_per_block = lds_bytes(G, Q, rows) > 48 * 1024 ? 8 : 4;
        out->blocks = 0;
        return check_plan(out, M, rows);
    }
    return HMSV_EUNSUPPORTED;
}

// Blocks of a call's launch: the plan's, or a persistent grid of the
// resident maximum with no more wavefronts than there are lane groups'
// worth of sequences.  0 on a device error.
int grid_blocks(const KernelEntry *e, const hmsv_plan &plan, int64_t count, int rows) {
    int blocks = plan.blocks;
    if (blocks == 0) {
        blocks = resident_blocks(e, plan.waves_per_block, rows);
        if (blocks <= 0) return 0;
        int64_t groups_per_block = (int64_t)plan.waves_per_block * (64 / plan.G);
        int64_t need = (count + groups_per_block - 1) / groups_per_block;
        if (need < blocks) blocks = (int)need;
    }
    return blocks;
}

// Which sequences of a call's range [first, first + count) to split, for
// ngroups lane groups and profile length M.  A launch ends no earlier than
// its longest sequence, which one lane group runs at the speed of a
// wavefront sharing its SIMD; sequences well above the mean work per group
// (total rows / ngroups) are therefore cut into segments of about that
// many rows.  Segments carry M - 1 warm-up rows (rounded up to 16), so
// segments are at least four times that long, and their number is capped.
void plan_split(const hmsv_db *db, int64_t first, int64_t count, int64_t ngroups, int M,
                KArgs &a) {
    a.nsplit = 0;
    a.nsegs = 0;
    a.nbins = 0;
    a.warm = ((M - 1) + 15) & ~15;
    a.seg_rows = 0;
    const int64_t *cum = db->cum_rows.data() + first;
    const int64_t total = cum[count] - cum[0];
    if (ngroups <= 0 || count < 2) return;
    int64_t T = std::max<int64_t>({total / ngroups, 4 * (int64_t)a.warm, 256});
    T = (T + 15) & ~(int64_t)15;
    for (; T < (int64_t)kRowsLimit; T *= 2) {
        // split the sequences above 1.5 T (they come first: longest first)
        const int64_t thr = T + T / 2;
        int64_t ns = 0, segs = 0, bins = 0, prev_v = -1;
        bool fits = true;
        while (ns < count && cum[ns + 1] - cum[ns] > thr) {
            int64_t v = (cum[ns + 1] - cum[ns] + T - 1) / T;
            if (v != prev_v) {
                if (bins == kMaxBins) { fits = false; break; }
                a.bin_t[bins] = (int32_t)ns;
                a.bin_p[bins] = (int32_t)segs;
                a.bin_v[bins] = (int32_t)v;
                ++bins;
                prev_v = v;
            }
            segs += v;
            ++ns;
            if (ns > kMaxSplit || segs > kMaxSegs) { fits = false; break; }
        }
        if (!fits) continue;
        a.nsplit = (int32_t)ns;
        a.nsegs = (int32_t)segs;
        a.nbins = (int32_t)bins;
        a.seg_rows = (int32_t)T;
        return;
    }
}

hmsv_status score_common(int is_msv, const hmsv_profile *prof, const hmsv_db *db,
                         int64_t first, int64_t count,
                         uint8_t *score, uint8_t *flags, void *workspace,
                         const hmsv_plan *plan_in, hipStream_t stream) {
    hmsv_status st = check_profile(prof, is_msv);
    if (st != HMSV_OK) return st;
    if (!db || !workspace) return HMSV_EINVAL;
    if (plan_in) {
        // the plan's shape first, without the database
        st = check_plan(plan_in, prof->M);
        if (st != HMSV_OK) return st;
    }
    hmsv_plan plan;
    st = resolve_plan(is_msv, prof->M, db->table_rows, plan_in, &plan);
    if (st != HMSV_OK) return st;
    const KernelEntry *e = registry().find(is_msv, plan.G, plan.Q);
    if (!e) return HMSV_ENOKERNEL;
    if (count == -1 && first == 0) count = db->nseq;      // whole database
    if (first < 0 || count < 0 || first > db->nseq || count > db->nseq - first) return HMSV_EINVAL;
    if (count == 0) return HMSV_OK;          // nothing to write (outputs may be NULL)
    if (!score || !flags) return HMSV_EINVAL;

    KArgs a{};
    a.cost = prof->cost;
    a.sc = prof->sc;
    a.M = prof->M;
    a.dbias = prof->dbias;
    a.tbm = hmsv_tbm(prof->M);
    a.res = db->d_res;
    a.seqs = db->d_seqs + first;
    a.nseq = (int32_t)count;
    a.pad_off = db->pad_off;
    a.score = score;
    a.flag = flags;
    a.counter = (uint32_t *)workspace;
    a.image = (uint32_t *)((char *)workspace + kWsCounterBytes);
    a.best = (int32_t *)((char *)workspace + 64);
    a.segs = (SeqRec *)((char *)workspace + kWsSegOff);
    a.slots = (uint32_t *)((char *)workspace + kWsSlotOff);
    a.segx = (uint32_t *)((char *)workspace + kWsSegxOff);
    a.ximage = (uint32_t *)((char *)workspace + kWsXImageOff);
    a.win = (uint4 *)((char *)workspace + kWsWinOff);
    a.qx = exact_q(prof->M);
    a.rows = db->table_rows;
    if (((uintptr_t)workspace & 255u) != 0) return HMSV_EINVAL;

    const int blocks = grid_blocks(e, plan, count, db->table_rows);
    if (blocks <= 0) return HMSV_EDEVICE;
    plan_split(db, first, count, (int64_t)blocks * plan.waves_per_block * (64 / plan.G),
               prof->M, a);
    // MSV: a second kernel rescores the windows the first one stored
    ExactLaunchFn xf = nullptr;
    int cus = 0;
    if (is_msv) {
        xf = a.qx >= 1 && a.qx <= kMaxExactQ ? registry().exact[a.qx] : nullptr;
        if (!xf) return HMSV_ENOKERNEL;
        cus = device_cus();
        if (cus <= 0) return HMSV_EDEVICE;
    }
    if (e->launch(a, plan.waves_per_block, blocks, stream) != hipSuccess) return HMSV_EDEVICE;
    if (xf && xf(a, cus, stream) != hipSuccess) return HMSV_EDEVICE;
    return HMSV_OK;
}

// ---- MSV scoring without allocation ---------------------------------------
// The workspace of hmsv_msv_score_noalloc: a file-scope device array, one
// copy per GPU, held until the process ends.  Host code never passes the
// array's name to a kernel (on the host it only stands in for the symbol);
// it uses the device address hipGetSymbolAddress returns, looked up once
// per device on the entry point's first call there.
constexpr int64_t kNoAllocMaxSeq = (int64_t)1 << 20;
constexpr size_t kScratchBytes = ws_bytes(kNoAllocMaxSeq);
static __device__ __align__(256) uint8_t scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch[kMaxDevices] = {};

hmsv_status scratch_ptr(void **out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return HMSV_EDEVICE;
    if (dev < 0 || dev >= kMaxDevices) return HMSV_EUNSUPPORTED;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return HMSV_EDEVICE;
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return HMSV_OK;
}

}  // namespace

namespace hmsv {
int register_kernels(const KernelEntry *entries, int n) {
    registry().entries.insert(registry().entries.end(), entries, entries + n);
    return n;
}

int register_p7_kernels(const P7KernelEntry *entries, int n) {
    registry().p7.insert(registry().p7.end(), entries, entries + n);
    return n;
}

int register_exact(int qx, ExactLaunchFn fn) {
    if (qx >= 1 && qx <= kMaxExactQ) registry().exact[qx] = fn;
    return qx;
}

}  // namespace hmsv

extern "C" {

const char *hmsv_strerror(hmsv_status s) {
    switch (s) {
        case HMSV_OK: return "success";
        case HMSV_EINVAL: return "invalid argument";
        case HMSV_EUNSUPPORTED: return "unsupported size";
        case HMSV_ENOMEM: return "out of memory";
        case HMSV_EDEVICE: return "HIP runtime error";
        case HMSV_ENOKERNEL: return "no kernel instantiated for this plan";
        default: return "unknown status";
    }
}

int32_t hmsv_tbm(int32_t M) {
    if (M < 1) return -1;
    double m = (double)M;
    return third_bit_cost(2.0 / (m * (m + 1.0)));
}

int32_t hmsv_tjb(int64_t L) {
    if (L < 0) return -1;
    return third_bit_cost(3.0 / ((double)L + 3.0));
}

hmsv_status hmsv_score_nats(int32_t is_msv, int32_t M, const void *score, const uint8_t *flags,
                            const int64_t *lengths, int64_t n, double *nats) {
    if (n < 0 || M < 1) return HMSV_EINVAL;
    if (n > 0 && (!score || !flags || !lengths || !nats)) return HMSV_EINVAL;
    const double units_per_nat = 3.0 / std::log(2.0);
    const int32_t tbm = hmsv_tbm(M);
    for (int64_t i = 0; i < n; ++i) {
        if (lengths[i] < 0) return HMSV_EINVAL;
        if (flags[i]) {
            nats[i] = HUGE_VAL;
            continue;
        }
        const int32_t tjb = hmsv_tjb(lengths[i]);
        const double u = is_msv
            ? (double)((const uint8_t *)score)[i] - tjb - HMSV_BASE
            : (double)((const int8_t *)score)[i] + 128.0 - tbm - 2.0 * tjb - HMSV_TEC;
        nats[i] = u / units_per_nat - 3.0;
    }
    return HMSV_OK;
}

hmsv_status hmsv_gumbel_pvalue(const double *nats, int64_t n, double mu, double lambda,
                               double *p) {
    if (n < 0 || !(lambda > 0.0)) return HMSV_EINVAL;
    if (n > 0 && (!nats || !p)) return HMSV_EINVAL;
    for (int64_t i = 0; i < n; ++i) {
        const double y = -lambda * (nats[i] - mu);
        // 1 - exp(-e^y) = -expm1(-e^y); e^y underflows to 0 for large scores
        p[i] = -std::expm1(-std::exp(y));
    }
    return HMSV_OK;
}

hmsv_status hmsv_quantize(const double *emis, const double *bg, int32_t M, uint8_t *cost,
                          int8_t *sc, int32_t *dbias) {
    if (!emis || !bg || !cost || !sc || !dbias) return HMSV_EINVAL;
    if (M < 1 || M > HMSV_MAX_M) return HMSV_EINVAL;
    for (int x = 0; x < HMSV_K; ++x)
        if (!(bg[x] > 0.0) || !std::isfinite(bg[x])) return HMSV_EINVAL;
    const int64_t kNegInf = INT64_MIN / 4;
    std::vector<int64_t> r((size_t)M * HMSV_K);
    int64_t best = kNegInf;
    for (int k = 0; k < M; ++k) {
        for (int x = 0; x < HMSV_K; ++x) {
            double e = emis[(size_t)k * HMSV_K + x];
            if (!(e >= 0.0) || !std::isfinite(e)) return HMSV_EINVAL;
            int64_t v = kNegInf;
            if (e > 0.0) v = (int64_t)rhaz(3.0 * std::log2(e / bg[x]));
            r[(size_t)k * HMSV_K + x] = v;
            best = std::max(best, v);
        }
    }
    if (best == kNegInf) return HMSV_EINVAL;
    for (int x = 0; x < HMSV_KP; ++x) {
        for (int k = 0; k < M; ++k) {
            int64_t c = 255;
            if (x < HMSV_K) c = std::min<int64_t>(255, best - r[(size_t)k * HMSV_K + x]);
            cost[(size_t)x * M + k] = (uint8_t)c;
            sc[(size_t)x * M + k] = (int8_t)std::max<int64_t>(-128, best - c);
        }
    }
    for (const Degenerate &d : kDegenerate) {
        for (int k = 0; k < M; ++k) {
            double mean = 0.0;
            int64_t c = 255;
            if (degenerate_mean(emis + (size_t)k * HMSV_K, bg, d, &mean))
                c = std::min<int64_t>(255, best - (int64_t)rhaz(3.0 * mean));
            cost[(size_t)d.code * M + k] = (uint8_t)c;
            sc[(size_t)d.code * M + k] = (int8_t)std::max<int64_t>(-128, best - c);
        }
    }
    *dbias = (int32_t)best;
    return HMSV_OK;
}

// ---- the paper's warp-based sequence blocks (Sec. 3.2, Alg. 1) ---------------

hmsv_status hmsv_alg1_pack(const int64_t *lengths, int64_t nseq, int32_t nblocks, int32_t width,
                           int32_t *container, int64_t *heights, hmsv_alg1_stats *stats) {
    if (nseq < 0 || (nseq > 0 && !lengths) || nblocks < 1 || width < 1 || !stats)
        return HMSV_EINVAL;
    const int64_t lines = (int64_t)nblocks * width;
    if (lines > ((int64_t)1 << 31)) return HMSV_EUNSUPPORTED;
    for (int64_t i = 0; i < nseq; ++i)
        if (lengths[i] < 0) return HMSV_EINVAL;
    // longest first, ties in input order
    std::vector<int64_t> order((size_t)nseq);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int64_t a, int64_t b) { return lengths[a] > lengths[b]; });
    // each sequence fills its residues plus one ending residue
    std::vector<int64_t> fill((size_t)lines, 0);
    const int64_t seeds = std::min(lines, nseq);
    int64_t max_len = 0;
    for (int64_t x = 0; x < seeds; ++x) {
        const int64_t sq = order[(size_t)x];
        if (container) container[sq] = (int32_t)x;
        fill[(size_t)x] = lengths[sq] + 1;
        max_len = std::max(max_len, fill[(size_t)x]);
    }
    // the rest: a pointer sweeps the containers downward (continuing from
    // the last placement) to the first whose fill stays within the longest
    // container; below container 0 the sequence goes onto the last one and
    // the sweep starts over
    int64_t ptr = lines;
    for (int64_t y = seeds; y < nseq; ++y) {
        const int64_t sq = order[(size_t)y];
        const int64_t need = lengths[sq] + 1;
        int64_t target;
        for (;;) {
            --ptr;
            if (ptr < 0) {
                ptr = lines;
                target = lines - 1;
                break;
            }
            if (need + fill[(size_t)ptr] <= max_len) {
                target = ptr;
                break;
            }
        }
        if (container) container[sq] = (int32_t)target;
        fill[(size_t)target] += need;
        max_len = std::max(max_len, fill[(size_t)target]);
    }
    int64_t padding = 0, real = 0, max_h = 0;
    double sum_h = 0.0, sum_h2 = 0.0, sum_e = 0.0, sum_e2 = 0.0;
    std::vector<int64_t> per_block_end((size_t)nblocks, 0);
    for (int64_t i = 0; i < nseq; ++i) real += lengths[i];
    if (container)
        for (int64_t i = 0; i < nseq; ++i) per_block_end[(size_t)(container[i] / width)] += 1;
    for (int32_t b = 0; b < nblocks; ++b) {
        int64_t h = 0, tot = 0;
        for (int32_t c = 0; c < width; ++c) {
            const int64_t f = fill[(size_t)b * width + c];
            h = std::max(h, f);
            tot += f;
        }
        if (heights) heights[b] = h;
        padding += (int64_t)width * h - tot;
        max_h = std::max(max_h, h);
        sum_h += (double)h;
        sum_h2 += (double)h * (double)h;
        const double e = (double)per_block_end[(size_t)b];
        sum_e += e;
        sum_e2 += e * e;
    }
    const double nb = (double)nblocks;
    stats->real = real;
    stats->ending = nseq;
    stats->padding = padding;
    stats->max_height = max_h;
    stats->mean_height = sum_h / nb;
    stats->sd_height = std::sqrt(std::max(0.0, sum_h2 / nb - (sum_h / nb) * (sum_h / nb)));
    stats->mean_ending = container ? sum_e / nb : -1.0;
    stats->sd_ending = container
        ? std::sqrt(std::max(0.0, sum_e2 / nb - (sum_e / nb) * (sum_e / nb))) : -1.0;
    stats->prr = real > 0 ? (double)padding / (double)real : 0.0;
    stats->efficiency = max_h > 0 ? stats->mean_height / (double)max_h : 1.0;
    return HMSV_OK;
}

// ---- FASTA ------------------------------------------------------------------

namespace {
// Residue code of a sequence byte: 0..31, -1 to skip (whitespace, digits,
// stop and gap symbols), -2 if invalid.
int fasta_code(unsigned char c) {
    static const char kAlpha[] = "ACDEFGHIKLMNPQRSTVWY";
    if (c >= 'a' && c <= 'z') c = (unsigned char)(c - 'a' + 'A');
    for (int i = 0; i < HMSV_K; ++i)
        if (kAlpha[i] == (char)c) return i;
    switch (c) {
    case 'B': return 21;
    case 'J': return 22;
    case 'Z': return 23;
    case 'U': return 24;
    case 'O': return 25;
    case 'X': return 26;
    case ' ': case '\t': case '\r': case '\n': case '\v': case '\f':
    case '*': case '-': case '.':
        return -1;
    default:
        return (c >= '0' && c <= '9') ? -1 : -2;
    }
}
}  // namespace

hmsv_status hmsv_fasta_parse(const char *text, int64_t n, uint8_t *res, int64_t *offsets,
                             int64_t *names, int64_t *nres, int64_t *nseq, int64_t *err_at) {
    if ((!text && n > 0) || n < 0 || !nres || !nseq) return HMSV_EINVAL;
    const bool fill = res || offsets || names;
    if (fill && (!offsets || !names)) return HMSV_EINVAL;
    const int64_t cap_res = fill ? *nres : 0, cap_seq = fill ? *nseq : 0;
    int64_t r = 0, s = 0;
    if (err_at) *err_at = -1;
    int64_t i = 0;
    while (i < n) {
        const unsigned char c = (unsigned char)text[i];
        if (c == '>') {
            // header: the rest of the line
            int64_t e = i + 1;
            while (e < n && text[e] != '\n') ++e;
            int64_t hl = e - (i + 1);
            if (hl > 0 && text[i + hl] == '\r') --hl;
            if (fill) {
                if (s >= cap_seq) return HMSV_EINVAL;
                offsets[s] = r;
                names[2 * s] = i + 1;
                names[2 * s + 1] = hl;
            }
            ++s;
            i = e < n ? e + 1 : e;
            continue;
        }
        const int code = fasta_code(c);
        if (code == -2 || (code >= 0 && s == 0)) {
            if (err_at) *err_at = i;
            return HMSV_EINVAL;
        }
        if (code >= 0) {
            if (fill) {
                if (r >= cap_res) return HMSV_EINVAL;
                if (res) res[r] = (uint8_t)code;
            }
            ++r;
        }
        ++i;
    }
    if (fill) {
        if (s != cap_seq || r != cap_res) return HMSV_EINVAL;
        offsets[s] = r;
    }
    *nres = r;
    *nseq = s;
    return HMSV_OK;
}

hmsv_status hmsv_db_create(const uint8_t *res, const int64_t *offsets, int64_t nseq,
                           hmsv_db **out) {
    if (!out || !offsets || nseq < 0) return HMSV_EINVAL;
    *out = nullptr;
    if (nseq > 0 && !res && offsets[nseq] > offsets[0]) return HMSV_EINVAL;
    if (nseq >= ((int64_t)1 << 31)) return HMSV_EUNSUPPORTED;
    std::vector<int64_t> len((size_t)nseq);
    int64_t residues = 0;
    for (int64_t i = 0; i < nseq; ++i) {
        len[i] = offsets[i + 1] - offsets[i];
        if (len[i] < 0) return HMSV_EINVAL;
        residues += len[i];
    }
    bool degenerate = false;
    for (int64_t i = 0; i < nseq; ++i) {
        const uint8_t *p = res + offsets[i];
        for (int64_t t = 0; t < len[i]; ++t) {
            if (p[t] >= HMSV_KP) return HMSV_EINVAL;
            degenerate = degenerate || (p[t] >= 21 && p[t] <= 26);
        }
    }
    // Longest first: the dynamic queue then ends with short sequences.
    std::vector<int64_t> order((size_t)nseq);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int64_t a, int64_t b) { return len[a] > len[b]; });
    std::vector<SeqRec> recs((size_t)nseq);
    std::vector<uint32_t> p7len((size_t)std::max<int64_t>(1, nseq), 0u);
    uint64_t total = 0, rows = 0;
    std::vector<int64_t> cum_rows((size_t)nseq + 1, 0);
    for (int64_t t = 0; t < nseq; ++t) {
        int64_t i = order[t];
        uint64_t r = (uint64_t)std::max<int64_t>(4, (len[i] + 3) & ~(int64_t)3);
        if (r >= kRowsLimit) return HMSV_EUNSUPPORTED;
        recs[t].off = (uint32_t)total;
        recs[t].rt = (uint32_t)r | ((uint32_t)hmsv_tjb(len[i]) << 24);
        recs[t].id = (uint32_t)i;
        p7len[t] = p7_lenmodel(len[i]);

        // 16-byte aligned; the rows rounded up to 16, then 16 bytes of code 20
        // (narrow lane groups run 16 rows per step and read past the end)
        total += ((r + 15) & ~(uint64_t)15) + 16;
        rows += r;
        cum_rows[(size_t)t + 1] = (int64_t)rows;
        if (total >= ((uint64_t)1 << 32) - 64) return HMSV_EUNSUPPORTED;
    }
    const uint32_t pad_off = (uint32_t)total;
    const size_t bytes = (size_t)total + 64;
    std::vector<uint8_t> packed(bytes, kInvalidCode);
    for (int64_t t = 0; t < nseq; ++t) {
        int64_t i = order[t];
        const uint8_t *p = res + offsets[i];
        uint8_t *d = packed.data() + recs[t].off;
        for (int64_t k = 0; k < len[i]; ++k) d[k] = keep_code(p[k]);
        recs[t].len = (uint32_t)len[i];
        std::memcpy(recs[t].first16, d, 4 * sizeof(uint32_t));
    }
    hmsv_db *db = new (std::nothrow) hmsv_db;
    if (!db) return HMSV_ENOMEM;
    db->nseq = nseq;
    db->residues = residues;
    db->rows = (int64_t)rows;
    db->pad_off = pad_off;
    db->table_rows = degenerate ? kDegenRows : kRows;
    try {
        db->order = order;
        db->cum_rows = cum_rows;
    } catch (...) {
        delete db;
        return HMSV_ENOMEM;
    }
    if (hipGetDevice(&db->device) != hipSuccess) { delete db; return HMSV_EDEVICE; }
    if (hipMalloc(&db->d_res, bytes) != hipSuccess) { delete db; return HMSV_ENOMEM; }
    if (hipMalloc(&db->d_seqs, sizeof(SeqRec) * (size_t)std::max<int64_t>(1, nseq)) != hipSuccess) {
        hipFree(db->d_res);
        delete db;
        return HMSV_ENOMEM;
    }
    if (hipMalloc(&db->d_p7len, sizeof(uint32_t) * p7len.size()) != hipSuccess) {
        hmsv_db_destroy(db);
        return HMSV_ENOMEM;
    }
    if (hipMemcpy(db->d_res, packed.data(), bytes, hipMemcpyHostToDevice) != hipSuccess ||
        (nseq > 0 && hipMemcpy(db->d_seqs, recs.data(), sizeof(SeqRec) * (size_t)nseq,
                               hipMemcpyHostToDevice) != hipSuccess) ||
        hipMemcpy(db->d_p7len, p7len.data(), sizeof(uint32_t) * p7len.size(),
                  hipMemcpyHostToDevice) != hipSuccess) {
        hmsv_db_destroy(db);
        return HMSV_EDEVICE;
    }
    *out = db;
    return HMSV_OK;
}

void hmsv_db_destroy(hmsv_db *db) {
    if (!db) return;
    if (db->d_res) hipFree(db->d_res);
    if (db->d_seqs) hipFree(db->d_seqs);
    if (db->d_p7len) hipFree(db->d_p7len);
    delete db;
}

int64_t hmsv_db_nseq(const hmsv_db *db) { return db ? db->nseq : -1; }
int64_t hmsv_db_residues(const hmsv_db *db) { return db ? db->residues : -1; }
int64_t hmsv_db_padded_rows(const hmsv_db *db) { return db ? db->rows : -1; }
int32_t hmsv_db_table_rows(const hmsv_db *db) { return db ? db->table_rows : -1; }

hmsv_status hmsv_db_default_plan(const hmsv_db *db, int32_t is_msv, int32_t M, hmsv_plan *plan) {
    if (!db || !plan || M < 1) return HMSV_EINVAL;
    if (M > HMSV_MAX_M) return HMSV_EUNSUPPORTED;
    return resolve_plan(is_msv ? 1 : 0, M, db->table_rows, nullptr, plan);
}

hmsv_status hmsv_default_plan(int32_t is_msv, int32_t M, hmsv_plan *plan) {
    if (!plan) return HMSV_EINVAL;
    if (M < 1) return HMSV_EINVAL;
    if (M > HMSV_MAX_M) return HMSV_EUNSUPPORTED;
    // The autotuned plan (paper Sec. 3.4 picks its kernel per model length
    // the same way): among the tuned M-bins of this filter, nearest to M in
    // log distance first (ties to the smaller bin), the first whose group
    // width still holds the profile within Q <= 32 registers and the LDS.
    int idx[kNumTuned];
    int n = 0;
    for (int i = 0; i < kNumTuned; ++i)
        if (kTuned[i].is_msv == (is_msv ? 1 : 0)) idx[n++] = i;
    auto dist = [M](int b) { return std::fabs(std::log((double)b) - std::log((double)M)); };
    auto before = [&](int a, int b) {
        double da = dist(kTuned[a].bin), db = dist(kTuned[b].bin);
        if (da != db) return da < db;
        return kTuned[a].bin < kTuned[b].bin;
    };
    // insertion sort of the few bins (stable, and allocates nothing)
    for (int t = 1; t < n; ++t)
        for (int u = t; u > 0 && before(idx[u], idx[u - 1]); --u) std::swap(idx[u], idx[u - 1]);
    for (int t = 0; t < n; ++t) {
        const TunedPlan &tp = kTuned[idx[t]];
        int G = tp.G;
        int Q = (M + 1 + 2 * G - 1) / (2 * G);
        if (Q > 32 || lds_bytes(G, Q) > (size_t)kLdsBytes) continue;
        if (!registry().find(is_msv ? 1 : 0, G, Q)) continue;
        plan->G = G;
        plan->Q = Q;
        plan->waves_per_block = tp.waves_per_block;
        plan->blocks = 0;
        return HMSV_OK;
    }
    // Untuned fallback: the narrowest lane group whose registers (Q <= 32
    // per lane) still hold the profile.
    for (int G : {1, 2, 4, 8, 16, 32, 64}) {
        int Q = (M + 1 + 2 * G - 1) / (2 * G);
        if (Q > 32 || lds_bytes(G, Q) > (size_t)kLdsBytes) continue;
        if (!registry().find(is_msv ? 1 : 0, G, Q)) continue;
        plan->G = G;
        plan->Q = Q;
        // large tables allow one block per CU: fill it with wavefronts
        plan->waves_per_block = lds_bytes(G, Q) > 48 * 1024 ? 8 : 4;
        plan->blocks = 0;
        return HMSV_OK;
    }
    return HMSV_ENOKERNEL;
}

size_t hmsv_plan_lds_bytes(int32_t G, int32_t Q) {
    if (G < 1 || G > 64 || (64 % G) != 0 || Q < 1) return 0;
    return lds_bytes(G, Q);
}

size_t hmsv_workspace_bytes(int64_t nseq) {
    return ws_bytes(nseq);
}

hmsv_status hmsv_msv_score(const hmsv_profile *prof, const hmsv_db *db, uint8_t *score,
                           uint8_t *flags, void *workspace, const hmsv_plan *plan,
                           hipStream_t stream) {
    return score_common(1, prof, db, 0, -1, score, flags, workspace, plan, stream);
}

hmsv_status hmsv_msv_score_noalloc(const hmsv_profile *prof, const hmsv_db *db,
                                   uint8_t *score, uint8_t *flags, const hmsv_plan *plan,
                                   hipStream_t stream) {
    if (!db) return HMSV_EINVAL;
    if (db->nseq > kNoAllocMaxSeq) return HMSV_EUNSUPPORTED;
    void *ws = nullptr;
    hmsv_status st = scratch_ptr(&ws);
    if (st != HMSV_OK) return st;
    return score_common(1, prof, db, 0, -1, score, flags, ws, plan, stream);
}

hmsv_status hmsv_ssv_score(const hmsv_profile *prof, const hmsv_db *db, int8_t *score,
                           uint8_t *flags, void *workspace, const hmsv_plan *plan,
                           hipStream_t stream) {
    return score_common(0, prof, db, 0, -1, (uint8_t *)score, flags, workspace, plan, stream);
}

hmsv_status hmsv_msv_score_range(const hmsv_profile *prof, const hmsv_db *db, int64_t first,
                                 int64_t count, uint8_t *score, uint8_t *flags,
                                 void *workspace, const hmsv_plan *plan, hipStream_t stream) {
    if (count < 0) return HMSV_EINVAL;
    return score_common(1, prof, db, first, count, score, flags, workspace, plan, stream);
}

hmsv_status hmsv_ssv_score_range(const hmsv_profile *prof, const hmsv_db *db, int64_t first,
                                 int64_t count, int8_t *score, uint8_t *flags,
                                 void *workspace, const hmsv_plan *plan, hipStream_t stream) {
    if (count < 0) return HMSV_EINVAL;
    return score_common(0, prof, db, first, count, (uint8_t *)score, flags, workspace, plan,
                        stream);
}

hmsv_status hmsv_split_info(const hmsv_db *db, int64_t first, int64_t count, int32_t is_msv,
                            int32_t M, const hmsv_plan *plan_in, int32_t *nsplit,
                            int32_t *nsegs, int32_t *seg_rows) {
    if (!db || !nsplit || !nsegs || !seg_rows) return HMSV_EINVAL;
    if (M < 1) return HMSV_EINVAL;
    if (M > HMSV_MAX_M) return HMSV_EUNSUPPORTED;
    hmsv_plan plan;
    hmsv_status st = resolve_plan(is_msv ? 1 : 0, M, db->table_rows, plan_in, &plan);
    if (st != HMSV_OK) return st;
    const KernelEntry *e = registry().find(is_msv ? 1 : 0, plan.G, plan.Q);
    if (!e) return HMSV_ENOKERNEL;
    if (count == -1 && first == 0) count = db->nseq;
    if (first < 0 || count < 0 || first > db->nseq || count > db->nseq - first) return HMSV_EINVAL;
    *nsplit = *nsegs = *seg_rows = 0;
    if (count == 0) return HMSV_OK;
    const int blocks = grid_blocks(e, plan, count, db->table_rows);
    if (blocks <= 0) return HMSV_EDEVICE;
    KArgs a{};
    plan_split(db, first, count, (int64_t)blocks * plan.waves_per_block * (64 / plan.G), M, a);
    *nsplit = a.nsplit;
    *nsegs = a.nsegs;
    *seg_rows = a.seg_rows;
    return HMSV_OK;
}

// ---- P7Viterbi -------------------------------------------------------------

hmsv_status hmsv_p7_quantize(const double *emis, const double *trans, const double *bg,
                             int32_t M, int16_t *msc, int16_t *trans_out, int32_t *tbm) {
    if (!emis || !trans || !bg || !msc || !trans_out || !tbm) return HMSV_EINVAL;
    if (M < 1 || M > HMSV_P7_MAX_M) return HMSV_EINVAL;
    for (int x = 0; x < HMSV_K; ++x)
        if (!(bg[x] > 0.0) || !std::isfinite(bg[x])) return HMSV_EINVAL;
    for (int64_t i = 0; i < (int64_t)M * HMSV_K; ++i)
        if (!(emis[i] >= 0.0) || !std::isfinite(emis[i])) return HMSV_EINVAL;
    for (int64_t i = 0; i < (int64_t)M * 7; ++i)
        if (!(trans[i] >= 0.0) || !std::isfinite(trans[i])) return HMSV_EINVAL;
    for (int x = 0; x < HMSV_KP; ++x)
        for (int k = 0; k < M; ++k)
            msc[(size_t)x * M + k] = (int16_t)(x < HMSV_K
                ? p7_score(emis[(size_t)k * HMSV_K + x] / bg[x]) : -32768);
    for (const Degenerate &d : kDegenerate) {
        for (int k = 0; k < M; ++k) {
            double mean = 0.0;
            int32_t v = -32768;
            if (degenerate_mean(emis + (size_t)k * HMSV_K, bg, d, &mean))
                v = (int32_t)std::max(-32768.0, std::min(32767.0, rhaz((double)kP7Units * mean)));
            msc[(size_t)d.code * M + k] = (int16_t)v;
        }
    }
    for (int t = 0; t < 7; ++t)
        for (int k = 0; k < M; ++k)
            trans_out[(size_t)t * M + k] = (int16_t)p7_score(trans[(size_t)k * 7 + t]);
    // node M has no successor and no insert state
    for (int t = 0; t < 7; ++t) trans_out[(size_t)t * M + M - 1] = (int16_t)-32768;
    *tbm = p7_score(2.0 / ((double)M * ((double)M + 1.0)));
    return HMSV_OK;
}

hmsv_status hmsv_p7_length_model(int64_t L, int32_t *loop, int32_t *move) {
    if (!loop || !move || L < 0) return HMSV_EINVAL;
    const uint32_t v = p7_lenmodel(L);
    *loop = (int32_t)(int16_t)(v & 0xffffu);
    *move = (int32_t)(int16_t)(v >> 16);
    return HMSV_OK;
}

size_t hmsv_p7_lds_bytes(int32_t G, int32_t Q) {
    if (G < 1 || G > 64 || (64 % G) != 0 || Q < 1) return 0;
    return p7_lds_bytes(G, Q);
}

// P7Viterbi plans measured on MI355X (the 500,000-sequence lognormal
// database, every (G, waves per block) with the fewest registers per lane):
// profile length bin, group width, waves per block.
struct P7Tuned {
    int bin, G, wpb;
};
constexpr P7Tuned kP7Tuned[] = {
    {30, 8, 4},     {64, 8, 4},     {100, 8, 8},    {200, 8, 4},    {400, 16, 4},
    {700, 32, 8},   {1000, 32, 8},  {1100, 64, 16}, {1500, 64, 16}, {2047, 64, 16},
    {2200, 64, 16}, {2400, 64, 16}, {2815, 64, 8},
};

// Largest block (in wavefronts) of a P7 plan: 16 for the 64-lane kernels
// that fit a 1024-thread block's 128 VGPRs without spilling, else 8.
int p7_max_waves(int G, int Q) { return (G == 64 && (Q <= 18 || Q == 20)) ? 16 : 8; }

hmsv_status hmsv_p7_default_plan(int32_t M, hmsv_plan *plan) {
    if (!plan || M < 1) return HMSV_EINVAL;
    if (M > HMSV_P7_MAX_M) return HMSV_EUNSUPPORTED;
    auto fits = [&](int G, int Q) {
        return Q <= (G == 64 ? 22 : 16) && p7_lds_bytes(G, Q) <= (size_t)kLdsBytes &&
               registry().find_p7(G, Q) != nullptr;
    };
    // the tuned bin nearest to M in log distance (ties to the smaller bin)
    constexpr int nt = (int)(sizeof(kP7Tuned) / sizeof(kP7Tuned[0]));
    int best = -1;
    double bd = 0.0;
    for (int i = 0; i < nt; ++i) {
        const double d = std::fabs(std::log((double)kP7Tuned[i].bin) - std::log((double)M));
        if (best < 0 || d < bd) {
            best = i;
            bd = d;
        }
    }
    // its group width if that holds the profile, else the narrowest that does
    const int G0 = kP7Tuned[best].G;
    int Q0 = (M + 1 + 2 * G0 - 1) / (2 * G0);
    // 64 lanes of 19 registers run as 20 (one more slot per register): the
    // 20-register kernel fits blocks of 16 wavefronts, the 19 one does not
    // (measured at M = 2400: 4.05 against 3.25 TCUPS)
    if (G0 == 64 && Q0 == 19 && kP7Tuned[best].wpb > 8) Q0 = 20;
    if (fits(G0, Q0)) {
        plan->G = G0;
        plan->Q = Q0;
        plan->waves_per_block = std::min(kP7Tuned[best].wpb, p7_max_waves(G0, Q0));
        plan->blocks = 0;
        return HMSV_OK;
    }
    for (int G : {4, 8, 16, 32, 64}) {
        const int Q = (M + 1 + 2 * G - 1) / (2 * G);
        if (!fits(G, Q)) continue;
        plan->G = G;
        plan->Q = Q;
        plan->waves_per_block = 8;
        plan->blocks = 0;
        return HMSV_OK;
    }
    return HMSV_ENOKERNEL;
}

namespace {

hmsv_status p7_common(const hmsv_p7_profile *prof, const hmsv_db *db, const int32_t *sel,
                      const int32_t *nsel, int16_t *score, uint8_t *flags, void *workspace,
                      const hmsv_plan *plan_in, hipStream_t stream) {
    if (!prof || !db || !workspace || !prof->msc || !prof->trans) return HMSV_EINVAL;
    if (prof->M < 1) return HMSV_EINVAL;
    if (prof->M > HMSV_P7_MAX_M) return HMSV_EUNSUPPORTED;
    if (((uintptr_t)workspace & 255u) != 0) return HMSV_EINVAL;
    hmsv_plan plan;
    const int Q64 = (prof->M + 1 + 127) / 128;
    if (plan_in) {
        plan = *plan_in;
    } else if (sel && registry().find_p7(64, Q64) &&
               p7_lds_bytes(64, Q64, db->table_rows) <= (size_t)kLdsBytes) {
        // A selection holds few records, mostly started at once: the call
        // lasts as long as its longest record, and a 64-lane group (the
        // fewest registers per lane) runs one fastest.
        plan.G = 64;
        plan.Q = Q64;
        plan.waves_per_block = p7_max_waves(64, Q64);
        plan.blocks = 0;
    } else {
        hmsv_status st = hmsv_p7_default_plan(prof->M, &plan);
        if (st != HMSV_OK) return st;
        // with the degenerate rows the image may no longer fit: the
        // narrowest group that still holds it
        for (int G : {4, 8, 16, 32, 64}) {
            if (p7_lds_bytes(plan.G, plan.Q, db->table_rows) <= (size_t)kLdsBytes) break;
            const int Q = (prof->M + 1 + 2 * G - 1) / (2 * G);
            if (Q > (G == 64 ? 22 : 16) || !registry().find_p7(G, Q)) continue;
            plan.G = G;
            plan.Q = Q;
        }
    }
    if (plan.G < 1 || plan.G > 64 || (64 % plan.G) != 0 || plan.Q < 1 ||
        plan_nodes(plan.G, plan.Q) < prof->M || plan.blocks < 0 ||
        plan.waves_per_block < 1 || plan.waves_per_block > p7_max_waves(plan.G, plan.Q))
        return HMSV_EINVAL;
    const P7KernelEntry *e = registry().find_p7(plan.G, plan.Q);
    if (!e) return HMSV_ENOKERNEL;
    if (p7_lds_bytes(plan.G, plan.Q, db->table_rows) > (size_t)kLdsBytes) return HMSV_EUNSUPPORTED;
    if (db->nseq == 0) return HMSV_OK;       // nothing to write (outputs may be NULL)
    if (!score || !flags) return HMSV_EINVAL;
    int blocks = plan.blocks;
    if (blocks == 0) {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            return HMSV_EDEVICE;
        const int per_cu = e->occupancy(plan.waves_per_block, db->table_rows);
        if (per_cu <= 0) return HMSV_EDEVICE;
        blocks = per_cu * cus;
        const int64_t groups_per_block = (int64_t)plan.waves_per_block * (64 / plan.G);
        const int64_t need = (db->nseq + groups_per_block - 1) / groups_per_block;
        if (need < blocks) blocks = (int)need;
    }
    P7Args a{};
    a.msc = prof->msc;
    a.trans = prof->trans;
    a.M = prof->M;
    a.tbm = prof->tbm;
    a.res = db->d_res;
    a.seqs = db->d_seqs;
    a.lenmodel = db->d_p7len;
    a.nseq = (int32_t)db->nseq;
    a.pad_off = db->pad_off;
    a.score = score;
    a.flag = flags;
    a.image = (uint32_t *)((char *)workspace + kWsP7ImageOff);
    a.queue = (uint32_t *)((char *)workspace + kWsP7QueueOff);
    a.aux = (int32_t *)workspace;
    a.rows = db->table_rows;
    a.sel = sel;
    a.nsel = nsel;
    if (e->launch(a, plan.waves_per_block, blocks, stream) != hipSuccess) return HMSV_EDEVICE;
    return HMSV_OK;
}

}  // namespace

hmsv_status hmsv_p7_score(const hmsv_p7_profile *prof, const hmsv_db *db, int16_t *score,
                          uint8_t *flags, void *workspace, const hmsv_plan *plan_in,
                          hipStream_t stream) {
    return p7_common(prof, db, nullptr, nullptr, score, flags, workspace, plan_in, stream);
}

hmsv_status hmsv_p7_score_selected(const hmsv_p7_profile *prof, const hmsv_db *db,
                                   const int32_t *positions, const int32_t *count,
                                   int16_t *score, uint8_t *flags, void *workspace,
                                   const hmsv_plan *plan_in, hipStream_t stream) {
    if (!positions || !count) return HMSV_EINVAL;
    return p7_common(prof, db, positions, count, score, flags, workspace, plan_in, stream);
}

hmsv_status hmsv_select(const hmsv_db *db, const void *score, const uint8_t *flags,
                        int32_t is_msv, int32_t threshold, int32_t *positions, int32_t *count,
                        void *workspace, hipStream_t stream) {
    if (!db || !positions || !count || !workspace) return HMSV_EINVAL;
    if (is_msv != 0 && is_msv != 1) return HMSV_EINVAL;
    if (((uintptr_t)workspace & 255u) != 0) return HMSV_EINVAL;
    if (db->nseq > 0 && (!score || !flags)) return HMSV_EINVAL;   // NULL only when empty
    if (db->nseq > (int64_t)INT32_MAX) return HMSV_EUNSUPPORTED;
    // the per-block counts sit in the window area, which P7 calls leave alone
    static_assert(kWsP7ImageOff + 160 * 1024 <= kWsWinOff, "selection scratch apart from P7");
    int32_t *scratch = (int32_t *)((char *)workspace + kWsWinOff);
    if (select_scratch_bytes(db->nseq) > ws_bytes(db->nseq) - kWsWinOff) return HMSV_EINVAL;
    if (launch_select(db->d_seqs, db->nseq, score, flags, is_msv, threshold, positions, count,
                      scratch, stream) != hipSuccess)
        return HMSV_EDEVICE;
    return HMSV_OK;
}

hmsv_status hmsv_db_order(const hmsv_db *db, int64_t *ids) {
    if (!db || (!ids && db->nseq > 0)) return HMSV_EINVAL;
    if (db->nseq > 0) std::memcpy(ids, db->order.data(), sizeof(int64_t) * (size_t)db->nseq);
    return HMSV_OK;
}

hmsv_status hmsv_batch_create(const hmsv_query *queries, int32_t nq, const hmsv_db *db,
                              int32_t branches, hmsv_batch **out) {
    if (!out || !queries || !db || nq < 1 || branches < 1 || branches > 16) return HMSV_EINVAL;
    *out = nullptr;
    // validate everything before any capture starts
    std::vector<hmsv_plan> plans((size_t)nq);
    for (int i = 0; i < nq; ++i) {
        const hmsv_query &q = queries[i];
        hmsv_status st = check_profile(&q.prof, q.is_msv ? 1 : 0);
        if (st != HMSV_OK) return st;
        if (!q.score || !q.flags || !q.workspace) return HMSV_EINVAL;
        if (((uintptr_t)q.workspace & 255u) != 0) return HMSV_EINVAL;
        for (int k = 0; k < i; ++k)
            if (queries[k].workspace == q.workspace) return HMSV_EINVAL;
        st = resolve_plan(q.is_msv ? 1 : 0, q.prof.M, db->table_rows,
                          q.plan.G == 0 ? nullptr : &q.plan, &plans[i]);
        if (st != HMSV_OK) return st;
        if (!registry().find(q.is_msv ? 1 : 0, plans[i].G, plans[i].Q)) return HMSV_ENOKERNEL;
    }
    // longest profiles first, each onto the branch with the least work so far
    std::vector<int> order((size_t)nq);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return queries[a].prof.M > queries[b].prof.M; });
    std::vector<int64_t> load((size_t)branches, 0);
    std::vector<int> branch_of((size_t)nq);
    for (int i : order) {
        int b = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        branch_of[i] = b;
        load[b] += queries[i].prof.M;
    }
    std::vector<hipStream_t> st((size_t)branches, nullptr);
    std::vector<hipEvent_t> ev((size_t)branches + 1, nullptr);
    hmsv_status rc = HMSV_OK;
    hipGraph_t graph = nullptr;
    bool capturing = false;
    for (int b = 0; b < branches && rc == HMSV_OK; ++b)
        if (hipStreamCreateWithFlags(&st[b], hipStreamNonBlocking) != hipSuccess) rc = HMSV_EDEVICE;
    for (auto &e : ev)
        if (rc == HMSV_OK && hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess)
            rc = HMSV_EDEVICE;
    if (rc == HMSV_OK) {
        if (hipStreamBeginCapture(st[0], hipStreamCaptureModeRelaxed) != hipSuccess) rc = HMSV_EDEVICE;
        else capturing = true;
    }
    if (rc == HMSV_OK) {
        // fork: every branch starts after the capture origin
        if (hipEventRecord(ev[branches], st[0]) != hipSuccess) rc = HMSV_EDEVICE;
        for (int b = 1; b < branches && rc == HMSV_OK; ++b)
            if (hipStreamWaitEvent(st[b], ev[branches], 0) != hipSuccess) rc = HMSV_EDEVICE;
    }
    for (int i : order) {
        if (rc != HMSV_OK) break;
        const hmsv_query &q = queries[i];
        rc = score_common(q.is_msv ? 1 : 0, &q.prof, db, 0, db->nseq, (uint8_t *)q.score,
                          q.flags, q.workspace, &plans[i], st[branch_of[i]]);
    }
    if (rc == HMSV_OK) {
        // join every branch back into the origin stream
        for (int b = 1; b < branches && rc == HMSV_OK; ++b) {
            if (hipEventRecord(ev[b], st[b]) != hipSuccess ||
                hipStreamWaitEvent(st[0], ev[b], 0) != hipSuccess)
                rc = HMSV_EDEVICE;
        }
    }
    if (capturing) {
        if (hipStreamEndCapture(st[0], &graph) != hipSuccess && rc == HMSV_OK) rc = HMSV_EDEVICE;
    }
    hmsv_batch *bt = nullptr;
    if (rc == HMSV_OK) {
        bt = new (std::nothrow) hmsv_batch;
        if (!bt) rc = HMSV_ENOMEM;
    }
    if (rc == HMSV_OK) {
        bt->graph = graph;
        bt->nq = nq;
        if (hipGraphInstantiate(&bt->exec, graph, nullptr, nullptr, 0) != hipSuccess) {
            rc = HMSV_EDEVICE;
            bt->graph = nullptr;
            delete bt;
            bt = nullptr;
        } else {
            graph = nullptr;
        }
    }
    if (graph) hipGraphDestroy(graph);
    for (auto e : ev)
        if (e) hipEventDestroy(e);
    for (auto s2 : st)
        if (s2) hipStreamDestroy(s2);
    if (rc == HMSV_OK) *out = bt;
    return rc;
}

hmsv_status hmsv_batch_launch(hmsv_batch *batch, hipStream_t stream) {
    if (!batch || !batch->exec) return HMSV_EINVAL;
    return hipGraphLaunch(batch->exec, stream) == hipSuccess ? HMSV_OK : HMSV_EDEVICE;
}

void hmsv_batch_destroy(hmsv_batch *batch) {
    if (!batch) return;
    if (batch->exec) hipGraphExecDestroy(batch->exec);
    if (batch->graph) hipGraphDestroy(batch->graph);
    delete batch;
}

}  // extern "C"
