// MSV / SSV filter kernel for gfx950.
//
// Mapping (compare paper Sec. 3.1, tiers 3-5):
//  * A lane group of G lanes aligns one sequence at a time; 64/G groups share
//    a wavefront (the paper's S-lane multi-sequence alignment, tier 4).
//  * Each lane holds Q 32-bit registers of two 16-bit cells (the K40 packs
//    four 8-bit cells per register with SIMD video instructions, tier 5;
//    gfx950 has packed 16-bit VALU instead).  The group's 2*G*Q cell slots
//    are striped: register q, element e (lane e/2, half e%2) is slot
//    q + Q*e, so only register Q-1 crosses lanes when the row moves one node
//    to the right (Alg. 5's reorder becomes one DPP move and one v_alignbit
//    per row).  Slot 0 of every group is a dummy node scored -inf, so node 1
//    always sees -inf as its upper-left neighbour without masking the
//    value shifted in from the neighbouring group; real node k is slot k.
//  * Cells hold u/1024 in fp16.  For SSV u = d + 128; for MSV u is the
//    8-bit cell value v relative to scB: u = max(v, scB) - scB.  Every value
//    is a multiple of 2^-10 below 1, so fp16 adds and maxima are exact, the
//    clamp modifier's floor at 0.0 is the floor of the 8-bit arithmetic, and
//    its cap at 1.0 is never reached before the overflow row.  With scB
//    fixed, Alg. 2's cell update max(0, max(v, scB) + dbias - cost) is
//    exactly max(u + dbias - cost, 0) on the relative value, so both filters
//    update a cell with one clamped add:
//      MSV  u = clamp(gamma + (dbias - cost)/1024)   (Alg. 2 cell update)
//      SSV  u = clamp(gamma + sc/1024)               (Alg. 7 cell update)
//    and scE = max(scE, u, u') takes two cells per v_pk_maximum3_f16 (a
//    running max, never reset per row).  The 255 (MSV) / 127 (SSV) caps are
//    not applied; overflow is flagged from the running max instead, which is
//    exact because no cap can fire before the first overflow row.
//  * Per-node scores of the 21 table rows live in LDS as fp16 pairs, laid
//    out [row][chunk][copy][lane][W] so each lane reads W consecutive dwords
//    and the groups served by one LDS read pass (256 bytes) use disjoint
//    banks: no bank conflicts between groups reading different rows.
//  * Sequences are handed out longest first from a global counter as groups
//    finish (replaces the pre-packed warp blocks of Alg. 1).
//  * MSV special states: scB fixed for every sequence first, then an exact
//    rescoring of short windows of the few sequences where the J state may
//    open, in a second launch (see filter_kernel).  When scB rises by
//    d, every relative cell becomes max(u - d, 0); the running max of
//    earlier scB values is kept as an integer.  A sequence whose cells never
//    rise above scB has running max
//    max(0, scB + max over its residues of max_k (dbias - cost_k)), computed
//    at its end from a per-residue table.
#pragma once
#include <utility>
#include <type_traits>
#include "hmsv_internal.h"

namespace hmsv {

typedef _Float16 h2 __attribute__((ext_vector_type(2)));
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

constexpr uint32_t kMinus2 = 0xC000u;        // fp16 -2.0: score of dummy/padding slots
constexpr int kBase = 190;
constexpr int kTec = 3;

// The lane's view of the profile's LDS image (lds_layout in
// hmsv_internal.h describes the image).
template <int G, int Q, int ROWS = kRows>
struct Layout {
    static constexpr LdsLayout D = lds_layout(G, Q, ROWS);
    static constexpr int W = 4;                       // dwords per chunk read
    static constexpr int NF = D.NF;
    static constexpr int R = D.R;
    static constexpr bool T2 = (R & 2) != 0;
    static constexpr bool T1 = (R & 1) != 0;
    static constexpr int CW = D.CW;
    static constexpr int OFF2 = D.OFF2;
    static constexpr int OFF1 = D.OFF1;
    static constexpr int RS = D.RS;
    static constexpr int Q2 = NF * W;                 // first register of the 2-dword tail
    static constexpr int Q1 = NF * W + (T2 ? 2 : 0);  // register of the 1-dword tail
    static constexpr int copies(int w) { return lds_copies(G, w); }
    __device__ static int lane_off(int lane, int w) {
        return ((lane / G) % copies(w)) * G * w + (lane % G) * w;
    }
};

__device__ __forceinline__ h2 as_h2(uint32_t v) { return __builtin_bit_cast(h2, v); }
__device__ __forceinline__ uint32_t as_u32(h2 v) { return __builtin_bit_cast(uint32_t, v); }

__device__ __forceinline__ uint32_t add_clamp(uint32_t a, uint32_t b) {
    const h2 z = {(_Float16)0.0f, (_Float16)0.0f};
    const h2 one = {(_Float16)1.0f, (_Float16)1.0f};
    h2 s = as_h2(a) + as_h2(b);
    return as_u32(__builtin_elementwise_min(__builtin_elementwise_max(s, z), one));
}

__device__ __forceinline__ uint32_t hmax(uint32_t a, uint32_t b) {
    return as_u32(__builtin_elementwise_maximum(as_h2(a), as_h2(b)));
}

__device__ __forceinline__ uint32_t hmax3(uint32_t a, uint32_t b, uint32_t c) {
    return as_u32(__builtin_elementwise_maximum(__builtin_elementwise_maximum(as_h2(a), as_h2(b)),
                                                as_h2(c)));
}

// fp16 bit patterns of non-negative values order like the values, so an
// integer max over patterns is the max over values.
__device__ __forceinline__ int lane_max_bits(uint32_t v) {
    int lo = (int)(v & 0xffffu);
    int hi = (int)(v >> 16);
    return lo > hi ? lo : hi;
}

template <int G>
__device__ __forceinline__ int group_max(int m) {
    // within 16 lanes by DPP (quad swaps, then the half-row and row mirrors),
    // beyond by lane shuffles; every lane of the group ends with the maximum
    auto dmax = [](int v, auto ctrl) {
        int t = __builtin_amdgcn_update_dpp(0, v, decltype(ctrl)::value, 0xf, 0xf, true);
        return v > t ? v : t;
    };
    if constexpr (G >= 2) m = dmax(m, std::integral_constant<int, 0xB1>{});   // lane ^ 1
    if constexpr (G >= 4) m = dmax(m, std::integral_constant<int, 0x4E>{});   // lane ^ 2
    if constexpr (G >= 8) m = dmax(m, std::integral_constant<int, 0x141>{});  // 7 - lane in 8
    if constexpr (G >= 16) m = dmax(m, std::integral_constant<int, 0x140>{}); // 15 - lane in 16
#pragma unroll
    for (int o = 16; o < G; o <<= 1) {
        int t = __shfl_xor(m, o);
        m = m > t ? m : t;
    }
    return m;
}

// fp16 pattern -> integer filter value u (exact: u/1024 is representable).
__device__ __forceinline__ int bits_to_units(int bits) {
    _Float16 h = __builtin_bit_cast(_Float16, (unsigned short)bits);
    return (int)((float)h * 1024.0f);
}

__device__ __forceinline__ uint32_t units_splat(int u) {
    _Float16 h = (_Float16)((float)u * (1.0f / 1024.0f));
    uint32_t b = (uint32_t)__builtin_bit_cast(unsigned short, h);
    return b | (b << 16);
}

// Row above shifted one node to the right, for register 0: element e takes
// element e-1 of register Q-1.  Element 0 of a group receives the previous
// group's last element (or 0 in lane 0); it is the dummy slot, so any value
// is fine there.
__device__ __forceinline__ uint32_t shift_in(uint32_t last) {
    uint32_t nb = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)last, 0x138, 0xf, 0xf, true);
    return __builtin_amdgcn_alignbit(last, nb, 16);
}

// Score (filter units) added at node k (0-based) for table row x: MSV
// dbias - cost, SSV sc.  Row kInvalidCode (every code 20..31, and the
// padding rows) scores -inf whatever the caller's table holds there: cost
// 255, sc -128.
template <bool MSV>
__device__ __forceinline__ int node_score(const KArgs &a, int x, int k) {
    if (x == kInvalidCode) return MSV ? a.dbias - 255 : -128;
    return MSV ? a.dbias - (int)a.cost[x * a.M + k] : (int)a.sc[x * a.M + k];
}

// fp16 pattern of the score added at slot s (node s, slot 0 = dummy) for
// table row x.
template <bool MSV>
__device__ __forceinline__ uint32_t slot_bits(const KArgs &a, int x, int s) {
    if (s < 1 || s > a.M) return kMinus2;
    int v = node_score<MSV>(a, x, s - 1);
    _Float16 h = (_Float16)((float)v * (1.0f / 1024.0f));
    return (uint32_t)__builtin_bit_cast(unsigned short, h);
}

template <int G, int Q, bool MSV>
struct Lane {
    using Lay = Layout<G, Q>;
    static constexpr int W = Lay::W;
    static constexpr int RS = Lay::RS;
    uint32_t R[Q];
    uint32_t xE;

    __device__ __forceinline__ void reset() {
#pragma unroll
        for (int q = 0; q < Q; ++q) R[q] = 0u;
        xE = 0u;
    }

    // MSV: scB rose by d units; every relative cell becomes max(u - d, 0).
    __device__ __forceinline__ void lower(int d) {
        const uint32_t m = units_splat(-d);
#pragma unroll
        for (int q = 0; q < Q; ++q) R[q] = add_clamp(R[q], m);
    }

    // Score pairs of row x for this lane.  TW/T2/T1: the lane's base in the
    // LDS image for full chunks and the two tails.
    __device__ __forceinline__ void load_row(const uint32_t *TW, const uint32_t *T2,
                                             const uint32_t *T1, uint32_t x,
                                             uint32_t (&c)[Q]) {
        // byte offset of row x: one multiply of the residue byte, no shift
        const uint32_t rb = x * (uint32_t)(RS * 4);
        auto at = [rb](const uint32_t *base) {
            return (const uint32_t *)((const char *)base + rb);
        };
#pragma unroll
        for (int ch = 0; ch < Lay::NF; ++ch) {
            const uint32_t *p = at(TW) + ch * Lay::CW;
            uint4 v = *(const uint4 *)p;
            if (ch * 4 + 0 < Q) c[ch * 4 + 0] = v.x;
            if (ch * 4 + 1 < Q) c[ch * 4 + 1] = v.y;
            if (ch * 4 + 2 < Q) c[ch * 4 + 2] = v.z;
            if (ch * 4 + 3 < Q) c[ch * 4 + 3] = v.w;
        }
        if constexpr (Lay::T2) {
            uint2 v = *(const uint2 *)at(T2);
            c[Lay::Q2] = v.x;
            c[Lay::Q2 + 1] = v.y;
        }
        if constexpr (Lay::T1) c[Lay::Q1] = *at(T1);
    }

    // One residue row of Alg. 2 (MSV) / Alg. 7 (SSV): shift, fetch, cell update.
    __device__ __forceinline__ void row(const uint32_t *const (&T)[3], uint32_t x) {
        uint32_t c[Q];
        load_row(T[0], T[1], T[2], x, c);
        update(c);
    }

    // The cell update of one row, given the row's scores.
    __device__ __forceinline__ void update(const uint32_t (&c)[Q]) {
        uint32_t gam = shift_in(R[Q - 1]);
        uint32_t prev_v = 0;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            uint32_t old = R[q];
            uint32_t v = add_clamp(gam, c[q]);
            R[q] = v;
            if (q & 1) xE = hmax3(xE, prev_v, v);
            else prev_v = v;
            gam = old;
        }
        if (Q & 1) xE = hmax(xE, prev_v);
    }
};

// Kernel modes.  MSV runs as two launches: filter_kernel in mode kMSV
// scores every sequence with scB fixed and settles all but the few whose
// running max passes base + tec (where the J state may open); for those it
// stores a short window of rows, and exact_kernel rescores each window in
// exact mode.  Keeping the exact-mode
// code out of the kernel that does almost all of the work keeps its
// register count at SSV's.
enum Mode : int {
    kSSV = 0,      // SSV (Alg. 7)
    kMSV = 1,      // MSV (Alg. 2) with scB fixed
};

// Counters in the workspace.
constexpr int kCtrMain = 0;      // next sequence of the range

// Flag value that marks a sequence whose score the exact pass still owes.
constexpr uint8_t kFlagPending = 2;

// MSV: "no loud step" (the offset of a lane's first loud step before it has
// one).
constexpr uint32_t kNoStep = 0xffffffffu;

// MSV: the end of a sequence's first pass (one lane per sequence): its
// score and flag, or, if the J state may have opened (a maximum above
// base + tec without overflow), its rescoring window for the exact pass:
// `warm` rows before the first loud step (not before the sequence's start)
// to the end of the last one, never past send; the whole sequence if no
// step was loud.  K: words of four residues per step of the filter kernel.
template <int K>
__device__ __forceinline__ void msv_settle(const KArgs &a, uint32_t sid, int mx,
                                           uint32_t wfirst, uint32_t wlast, uint32_t sstart,
                                           uint32_t send, uint32_t tjb) {
    const bool of = mx >= 255 - a.dbias;
    const bool loud = !of && mx > kBase + kTec;
    if (!loud) {
        const int v = mx - kTec;
        a.score[sid] = of ? 255 : (uint8_t)(v < 0 ? 0 : v);
        a.flag[sid] = of ? 1 : 0;
        return;
    }
    const uint32_t w = (uint32_t)a.warm;
    const bool known = wfirst != kNoStep && wfirst < send;
    const uint32_t ws = known && wfirst >= sstart + w ? (wfirst - w) & ~15u : sstart;
    uint32_t we = known ? wlast + 4u * K : send;
    we = we < send ? we : send;
    a.win[sid] = make_uint4(ws, (we - ws) | (tjb << 24), sid, 0u);
    a.flag[sid] = kFlagPending;
}

// Sequence ends a wavefront collects before it leaves the row loop to
// record scores and hand out sequences (see filter_kernel).
template <int G>
constexpr int kExitGroups = G == 1 ? 8 : G == 2 ? 4 : G == 4 ? 2 : 1;

// Lanes with at most this many registers read each row's scores one row
// ahead (a second set of Q registers).
constexpr int kPipeQ = 17;

// Residue words (four residues each) per load and lane: 16 or 8 residues.
template <int G>
constexpr int kWordsPerLoad = G <= 8 ? 4 : 2;

// One filter launch.  Every lane group pulls sequences (longest first)
// from the call's range and runs their rows in steps of 4K residues.
//
// kMSV runs a sequence with scB fixed at sat0(base - tjb - tbm).  Cells
// relative to scB then follow the SSV-like recurrence u = max(0, u + dbias
// - cost), and this result is exact when the running max stays at or below
// base + tec (the J state never opens) or reaches the overflow threshold
// (cells only grow with scB).  Otherwise the sequence is loud: the group
// stores a window of its rows for exact_kernel (indexed by the sequence's
// original index, flag set to kFlagPending).  A step is loud if a cell in it
// passed the level; rescoring in exact mode from `warm` (>= M - 1) rows
// before the first loud step to the end of the last one gives the exact
// score, because
//  * before the first loud row scB never moved, so fresh cells started
//    `warm` rows earlier are exact from that step on, and the rows skipped
//    or warmed up stay at or below base + tec;
//  * once scB has risen, relative cells follow the same recurrence and are
//    only lowered at each rise, so they never exceed their fixed-scB
//    values; after the last loud step no cell passes tjb + tbm + tec above
//    scB, which is what a rise (or a first overflow) needs, so scJ, scB
//    and the running max keep their values to the end.
template <int G, int Q, int MODE, int THREADS>
__global__ void __launch_bounds__(THREADS)
filter_kernel(KArgs a) {
    constexpr bool MSV = MODE == kMSV;
    extern __shared__ uint32_t lds[];
    using L = Lane<G, Q, MSV>;
    constexpr int W = L::W;
    constexpr int RS = L::RS;
    static_assert(RS % 4 == 0, "rows must stay 16-byte aligned");

    // Stage the profile image (built by prep_kernel) into LDS.
    {
        const uint4 *src = (const uint4 *)a.image;
        uint4 *dst = (uint4 *)lds;
        const int n16 = a.rows * (RS / 4);
        for (int i = threadIdx.x; i < n16; i += blockDim.x) dst[i] = src[i];
    }
    __syncthreads();

    const int lane = threadIdx.x & 63;
    const int j = lane % G;
    const bool gstart = (j == 0);
    using Lay = typename L::Lay;
    const uint32_t *T[3] = {lds + Lay::lane_off(lane, W),
                            lds + Lay::OFF2 + Lay::lane_off(lane, 2),
                            lds + Lay::OFF1 + Lay::lane_off(lane, 1)};
    const int dbias = a.dbias;

    // Records: the range's, with its split sequences (records [0, nsplit))
    // replaced by their segments (nv = nsegs + nseq - nsplit records, the
    // segments first).
    const uint4 *recs = (const uint4 *)a.seqs;
    const uint4 *segs = (const uint4 *)a.segs;
    const int nsegs = a.nsegs;
    const int nsplit = a.nsplit;
    const int nv = nsegs + a.nseq - nsplit;       // ranges are never empty
    const int ngroups = (int)(gridDim.x * (blockDim.x / G));
    const int gid = (int)(blockIdx.x * (blockDim.x / G) + threadIdx.x / G);

    L st;
    uint32_t off = a.pad_off;
    uint32_t id = 0;
    uint32_t seq_off = 0;
    uint32_t seq_end = 0xffffffffu;   // offset just past the sequence's rows
    int tjbm = 0;
    int xb = 0;                  // MSV: scB (integer filter units)
    uint32_t lvl = 0xffffffffu;  // MSV: level (two u16 halves)
    // MSV: running max over earlier steps (st.xE holds the current step's),
    // and the offsets of this lane's first and last loud steps
    uint32_t xrun = 0u;
    uint32_t first_loud = kNoStep, last_loud = 0u;
    bool active = false;
    bool need = false;           // group wants a sequence
    // Residues come in words of four, K words per load (16 residues for
    // groups of up to 8 lanes, 8 for wider ones): each group streams its own
    // sequence, and a load issued 4K rows before its first use hides the
    // memory latency of the first touch of each line.  Sequences then run
    // in whole 4K-row steps (the extra rows are non-scoring padding, which
    // cannot change a score).
    constexpr int K = kWordsPerLoad<G>;
    uint32_t wv[K];              // next 4K residues of the group's sequence
#pragma unroll
    for (int k = 0; k < K; ++k) wv[k] = 0u;

    // Sequence pipeline (group-uniform).  While a group runs a sequence, the
    // record of its next one (A, with A's first sixteen residues stored in the
    // record) is loaded and the queue position after that (qc) is claimed.
    // At a switch: run A, load the record at qc as the new A, claim a new
    // qc.  The record load and the claim's atomic issued at a switch are
    // first used at a later one, so neither stalls the switch.  At every
    // switch of the wavefront all lanes reload A (groups that keep theirs
    // reload the same record), so the load is unconditional and its result
    // lands in place without a wait.  A claim's atomic result stays in the
    // lane that issued it (pend_b, in lane pend_first) until the next switch
    // of the wavefront resolves it.
    //
    // Queue positions map to records so that the grid's N groups start on
    // the N longest sequences and each holds two of the shortest as A and
    // qc: positions [0, N) are records [0, N), positions [N, 3N) the last
    // 2N records (shortest first from the end), positions from 3N (claimed
    // dynamically) the records in between, longest first.  No group thus
    // queues a long sequence behind its first one.  Ranges with fewer than
    // 3N records use positions as record numbers (so a group whose number is
    // at least the record count never gets one).
    const bool tail = nv >= 3 * ngroups;
    constexpr int kNone = 0x7fffffff;             // position past the range
    auto record_of = [&](int p) -> int {          // queue position -> record
        if (p >= nv) return kNone;
        if (!tail || p < ngroups) return p;
        if (p < 3 * ngroups) return nv - 1 - (p - ngroups);
        return p - 2 * ngroups;
    };
    auto fetch = [&](int r, uint4 &h, uint4 &f) {
        r = r < nv ? r : nv - 1;
        const uint4 *p = r < nsegs ? segs + 2 * r : recs + 2 * (r - nsegs + nsplit);
        h = p[0];
        if constexpr (K > 1) f = p[1];
    };
    // the residue words at offset o
    auto load_words = [&](uint32_t o, uint32_t (&d)[K]) {
        if constexpr (K == 4) {
            uint4 v = *(const uint4 *)(a.res + o);
            d[0] = v.x; d[1] = v.y; d[2] = v.z; d[3] = v.w;
        } else if constexpr (K == 2) {
            uint2 v = *(const uint2 *)(a.res + o);
            d[0] = v.x; d[1] = v.y;
        } else {
            d[0] = *(const uint32_t *)(a.res + o);
        }
    };
    uint4 ra;                    // record A: off, rows | tjb << 24, id, length
    uint4 ra16;                  // record A's first sixteen residues (K > 1)
    int qa, qc;                  // records of A and of the claimed position (kNone: none)
    uint32_t pend_b = 0;
    int pend_first = -1;         // wave-uniform
    auto start_record = [&](const uint4 &r, const uint4 &r16, bool valid) {
        active = valid;
        uint32_t rows = r.y & kRowsMask;
        if constexpr (K > 1) rows = (rows + 4u * K - 1u) & ~(4u * K - 1u);
        seq_off = valid ? r.x : a.pad_off;
        seq_end = valid ? r.x + rows : a.pad_off;
        id = r.z;
        tjbm = (int)(r.y >> 24) + a.tbm;
        static_assert(K == 4 || K == 2, "residues come 16 or 8 per load");
        if constexpr (K == 4) {
            wv[0] = r16.x; wv[1] = r16.y; wv[2] = r16.z; wv[3] = r16.w;
        } else {
            wv[0] = r16.x; wv[1] = r16.y;
        }
    };

    // MSV running max with scB fixed: max over the lane group of its cells'
    // running max, plus scB; -1 while no cell rose above scB.  Called by
    // whole wavefronts.
    auto run_max = [&]() -> int {
        int m = bits_to_units(group_max<G>(lane_max_bits(hmax(st.xE, xrun))));
        return m > 0 ? m + xb : -1;
    };
    // The level: the largest relative cell value at which the running max
    // neither passes base + tec nor reaches 255 - dbias, as an fp16 pattern
    // in both halves; and whether any cell of this lane's step passed it
    // (saturating u16 subtract).
    auto above_level = [&]() -> bool {
        return (uint32_t)__builtin_bit_cast(
                   uint32_t, __builtin_elementwise_sub_sat(__builtin_bit_cast(u16x2, st.xE),
                                                           __builtin_bit_cast(u16x2, lvl))) != 0u;
    };
    const int lim0 = kBase + kTec < 254 - dbias ? kBase + kTec : 254 - dbias;
    auto start_sequence = [&]() {
        off = seq_off;
        xb = kBase - tjbm;
        xb = xb < 0 ? 0 : xb;
        st.reset();
        xrun = 0u;
        first_loud = kNoStep;
        last_loud = 0u;
        if constexpr (MSV) {
            const int rel = lim0 - xb;
            lvl = units_splat(rel < 0 ? 0 : rel);
        }
    };

    {
        int q0 = record_of(gid);
        uint4 r0, r016 = {0u, 0u, 0u, 0u};
        fetch(q0, r0, r016);
        qa = record_of(ngroups + gid);
        fetch(qa, ra, ra16);
        qc = record_of(2 * ngroups + gid);
        start_record(r0, r016, q0 != kNone);
        start_sequence();
    }

    for (;;) {
        // ---- hand sequences to groups that need one (uniform) ----------
        if (__any(need)) {
            // resolve the previous claim (its atomic has long returned); a
            // group with a pending claim holds -1 - its rank in qc
            if (pend_first >= 0) {
                int b = __builtin_amdgcn_readlane((int)pend_b, pend_first);
                if (qc < 0) qc = record_of(3 * ngroups + b - 1 - qc);
            }
            if (need) {
                start_record(ra, ra16, qa != kNone);
                qa = qc;
                start_sequence();
            }
            fetch(qa, ra, ra16);
            // new claims for the groups that just switched
            unsigned long long m = __ballot(need && gstart);
            int first = __ffsll((long long)m) - 1;
            if (lane == first) pend_b = atomicAdd(a.counter + kCtrMain, (uint32_t)__popcll(m));
            pend_first = first;
            // the group's rank: claiming groups below its first lane
            int rank = __popcll(m & ((1ull << (lane - j)) - 1ull));
            if (need) qc = -1 - rank;
            need = false;
        }
        if (!__any(active)) break;

        // ---- rows, four residues at a time --------------------------------
        // A group that reaches its end parks: its offset moves to the
        // non-scoring residues after the database, so its cells fall to zero
        // and its running max is kept.  The rows
        // continue until kExitGroups<G> groups of the wavefront have ended
        // (all of them if fewer are active), so narrow groups pay for the
        // switch code once per several sequence ends.
        const int n_act = __popcll(__ballot(active && gstart));
        const int e_min = n_act < kExitGroups<G> ? n_act : kExitGroups<G>;
        const uint32_t step = active ? 4u * K : 0u;
        bool ended = false;
        // Short rows are latency bound when a wavefront runs alone (the
        // last, longest sequences of a launch): their scores are read one
        // row ahead, into two alternating register sets.
        constexpr bool PIPE = Q <= kPipeQ;
        uint32_t ca[PIPE ? Q : 1], cb[PIPE ? Q : 1];
        auto xrow = [&](int r) -> uint32_t { return (wv[r / 4] >> (8 * (r % 4))) & 0xffu; };
        if constexpr (PIPE) st.load_row(T[0], T[1], T[2], xrow(0), ca);
        do {
            uint32_t offn = off + step;
            if constexpr (kExitGroups<G> > 1) offn = offn < seq_end ? offn : a.pad_off;
            uint32_t wn[K];
            load_words(offn, wn);                                    // next 4K residues
            // one residue row
            auto one_row = [&](auto r_c) {
                constexpr int r = decltype(r_c)::value;
                if constexpr (PIPE) {
                    uint32_t (&cur)[PIPE ? Q : 1] = (r & 1) ? cb : ca;
                    uint32_t (&nxt)[PIPE ? Q : 1] = (r & 1) ? ca : cb;
                    if constexpr (r + 1 < 4 * K) {
                        st.load_row(T[0], T[1], T[2], xrow(r + 1), nxt);
                    } else {
                        // first row of the next step: its residues must be in
#pragma unroll
                        for (int k = 0; k < K; ++k) asm volatile("" : "+v"(wn[k]));
                        st.load_row(T[0], T[1], T[2], wn[0] & 0xffu, nxt);
                    }
                    st.update(cur);
                } else {
                    st.row(T, xrow(r));
                }
            };
            [&]<int... R>(std::integer_sequence<int, R...>) {
                (one_row(std::integral_constant<int, R>{}), ...);
            }(std::make_integer_sequence<int, 4 * K>{});
            // Consume the next words only here, so their load stays issued
            // before the rows and its latency hides behind them.
#pragma unroll
            for (int k = 0; k < K; ++k) asm volatile("" : "+v"(wn[k]));
            if constexpr (MSV) {
                // the step's maximum joins the running max; note the step if
                // a cell in it passed the level (parked groups, past their
                // sequence, note nothing)
                const bool loud = above_level() && off < seq_end;
                xrun = hmax(xrun, st.xE);
                st.xE = 0u;
                if (loud) {
                    first_loud = first_loud == kNoStep ? off : first_loud;
                    last_loud = off;
                }
            }
            off = offn;
            ended = active && off == (kExitGroups<G> > 1 ? a.pad_off : seq_end);
#pragma unroll
            for (int k = 0; k < K; ++k) wv[k] = wn[k];
        } while (__popcll(__ballot(ended && gstart)) < e_min);

        // ---- finished sequences: record scores (Alg. 2 end-residue branch) -----
        if constexpr (MODE == kSSV) {
            int mx = bits_to_units(group_max<G>(lane_max_bits(st.xE)));
            // A split sequence's maximum is the maximum over its segments
            // (every cell of the sequence lies in some segment's own rows,
            // and a warm-up row's cells never exceed the true ones): SSV
            // segments store theirs for combine_kernel.
            if (ended && gstart) {
                if (id & kSegBit) {
                    a.segx[4 * (id & ~kSegBit)] = (uint32_t)mx;
                } else {
                    bool of = mx >= 255;
                    a.score[id] = of ? (uint8_t)127 : (uint8_t)(int8_t)(mx - 128);
                    a.flag[id] = of ? 1 : 0;
                }
            }
            need = ended;
        } else {
            // scB and tjb + tbm follow from the level (lim - scB, lim >= scB
            // since scB <= base), so neither stays in a register over the rows
            xb = lim0 - bits_to_units((int)(lvl & 0xffffu));
            tjbm = kBase - xb;
            int mx = run_max();
            // never above scB: max(0, scB + best score of its residues)
            int bst = -(1 << 30);
            if (ended && mx < 0) {
                for (uint32_t p = seq_off + j; p < seq_end; p += G) {
                    int v = a.best[a.res[p]];
                    bst = v > bst ? v : bst;
                }
            }
            bst = group_max<G>(bst);
            if (mx < 0) {
                int v = xb + bst;
                mx = v > 0 ? v : 0;
            }
            // the group's first and last loud steps (unsigned min by a signed
            // max of the flipped complement, unsigned max by a signed max of
            // the flipped value); called by whole wavefronts
            const uint32_t gfirst =
                ~((uint32_t)group_max<G>((int)(~first_loud ^ 0x80000000u)) ^ 0x80000000u);
            const uint32_t glast =
                (uint32_t)group_max<G>((int)(last_loud ^ 0x80000000u)) ^ 0x80000000u;
            // A segment stores its maximum and loud steps for
            // combine_msv_kernel, which settles its sequence after this
            // kernel; a whole sequence settles here.
            if (ended && gstart) {
                if (id & kSegBit) {
                    uint32_t *x = a.segx + 4 * (id & ~kSegBit);
                    x[0] = (uint32_t)mx;
                    x[2] = gfirst;
                    x[3] = glast;
                } else {
                    msv_settle<K>(a, id, mx, gfirst, glast, seq_off, seq_end,
                                  (uint32_t)(tjbm - a.tbm));
                }
            }
            need = ended;
        }
    }
}

// Segment record p of the call (one thread each) and, from each split
// sequence's first segment, the sequence's slot.
__device__ __forceinline__ void build_segment(const KArgs &a, int p) {
    // its bin: the last with bin_p <= p (unrolled, so the kernel argument
    // arrays are read at constant offsets); within a bin every split
    // sequence has bv segments, so p names sequence t and segment s
    int bt = 0, bp = 0, bv = 1;
#pragma unroll
    for (int b = 0; b < kMaxBins; ++b) {
        if (b < a.nbins && a.bin_p[b] <= p) {
            bt = a.bin_t[b];
            bp = a.bin_p[b];
            bv = a.bin_v[b];
        }
    }
    const int k = (p - bp) / bv;
    const int t = bt + k;
    const int s = (p - bp) - k * bv;
    const SeqRec &r = a.seqs[t];
    const uint32_t rows = r.rt & kRowsMask;
    const uint32_t T = (uint32_t)a.seg_rows;
    const uint32_t beg = (uint32_t)s * T;
    const uint32_t end = beg + T < rows ? beg + T : rows;
    const uint32_t st = s == 0 ? 0u : beg - (uint32_t)a.warm;
    const uint32_t off = r.off + st;
    const uint4 w = *(const uint4 *)(a.res + off);
    uint4 *d = (uint4 *)(a.segs + p);
    d[0] = make_uint4(off, (end - st) | (r.rt & ~kRowsMask), kSegBit | (uint32_t)p, w.x);
    d[1] = w;
    a.segx[4 * p + 1] = (uint32_t)t;
    if (s == 0) {
        uint4 *sl = (uint4 *)(a.slots + kSlotWords * t);
        sl[0] = make_uint4((uint32_t)bv, 0u, r.id, (uint32_t)t);
        sl[1] = make_uint4(0xffffffffu, (uint32_t)p, 0u, 0u);
    }
}

// SSV: score and flag of each split sequence from its segments' maxima
// (one thread each).
static __global__ void __launch_bounds__(256) combine_kernel(KArgs a) {
    const int t = (int)(blockIdx.x * 256 + threadIdx.x);
    if (t >= a.nsplit) return;
    const uint32_t *sl = a.slots + kSlotWords * t;
    const uint32_t v = sl[0], id = sl[2], p = sl[5];
    uint32_t m = 0;
    for (uint32_t k = 0; k < v; ++k) {
        uint32_t x = a.segx[4 * (p + k)];
        m = x > m ? x : m;
    }
    bool of = m >= 255;
    a.score[id] = of ? (uint8_t)127 : (uint8_t)(int8_t)((int)m - 128);
    a.flag[id] = of ? 1 : 0;
}

// MSV: settle each split sequence from its segments (one thread each): the
// maximum over them (every cell of the sequence lies in some segment's own
// rows, and warm-up cells never exceed the true ones) and the earliest and
// latest loud steps; then score and flag, or a rescoring window, as for a
// whole sequence.  Runs between the filter kernel and the exact pass.
template <int K>
__global__ void __launch_bounds__(256) combine_msv_kernel(KArgs a) {
    const int t = (int)(blockIdx.x * 256 + threadIdx.x);
    if (t >= a.nsplit) return;
    const uint32_t *sl = a.slots + kSlotWords * t;
    const uint32_t v = sl[0], sid = sl[2], rec = sl[3], p = sl[5];
    int mx = 0;
    uint32_t wfirst = kNoStep, wlast = 0u;
    for (uint32_t k = 0; k < v; ++k) {
        const uint4 x = *(const uint4 *)(a.segx + 4 * (p + k));
        mx = (int)x.x > mx ? (int)x.x : mx;
        wfirst = x.z < wfirst ? x.z : wfirst;
        wlast = x.w > wlast ? x.w : wlast;
    }
    const SeqRec &r = a.seqs[rec];
    const uint32_t send = r.off + (((r.rt & kRowsMask) + 4u * K - 1u) & ~(4u * K - 1u));
    msv_settle<K>(a, sid, mx, wfirst, wlast, r.off, send, r.rt >> 24);
}

// One dword of a profile's LDS image for a lane group of G lanes with Q
// registers, laid out as D = lds_layout(G, Q) describes: for table row x,
// register q and lane j, the dword holds slots (q + 2jQ, q + (2j+1)Q) as two
// fp16 scores, in every copy of q's chunk.
template <bool MSV>
__device__ __forceinline__ uint32_t image_dword(const KArgs &a, const LdsLayout &D, int G, int Q,
                                                int idx) {
    const int x = idx / D.RS;
    int rem = idx - x * D.RS;
    int w, q0;
    if (rem < D.OFF2) {
        const int ch = rem / D.CW;
        rem -= ch * D.CW;
        w = 4;
        q0 = ch * 4;
    } else if (rem < D.OFF1) {
        rem -= D.OFF2;
        w = 2;
        q0 = D.NF * 4;
    } else {
        rem -= D.OFF1;
        w = 1;
        q0 = D.NF * 4 + ((D.R & 2) ? 2 : 0);
    }
    rem %= G * w;                                  // same data in every copy
    const int jj = rem / w;
    const int qq = q0 + (rem - jj * w);
    const int s0 = qq + Q * (2 * jj);
    return qq >= Q ? 0u                            // padding of a partial chunk
                   : slot_bits<MSV>(a, x, s0) | (slot_bits<MSV>(a, x, s0 + Q) << 16);
}

// Per call: the filter kernel's LDS image of the profile and, for MSV, the
// exact pass's image (Layout<64, qx>); threads 0..3 reset the counters.
// For MSV, a.rows more blocks compute best[x] = max_k (dbias - cost_k(x)).
// The last blocks build the records and slots of split sequences.
template <int G, int Q, bool MSV>
__global__ void __launch_bounds__(256) prep_kernel(KArgs a, int image_blocks, int ximage_blocks) {
    constexpr LdsLayout D = lds_layout(G, Q);
    const int best_block0 = image_blocks + ximage_blocks;
    const int seg_block0 = best_block0 + (MSV ? a.rows : 0);
    const int b = (int)blockIdx.x;
    if (b >= seg_block0) {
        const int p = (b - seg_block0) * 256 + (int)threadIdx.x;
        if (p < a.nsegs) build_segment(a, p);
        return;
    }
    if (b >= best_block0) {
        // MSV: best[x] = max_k (dbias - cost_k(x)) for each table row x
        __shared__ int red[256];
        int x = b - best_block0;
        int m = -(1 << 30);
        for (int k = threadIdx.x; k < a.M; k += blockDim.x) {
            int v = node_score<true>(a, x, k);
            m = v > m ? v : m;
        }
        red[threadIdx.x] = m;
        __syncthreads();
        for (int h = 128; h > 0; h >>= 1) {
            if ((int)threadIdx.x < h && red[threadIdx.x + h] > red[threadIdx.x])
                red[threadIdx.x] = red[threadIdx.x + h];
            __syncthreads();
        }
        if (threadIdx.x == 0) a.best[x] = red[0];
        return;
    }
    if (b >= image_blocks) {
        // MSV: the exact pass's image
        const LdsLayout X = lds_layout(kExactG, a.qx);
        const int idx = (b - image_blocks) * 256 + (int)threadIdx.x;
        if (idx < a.rows * X.RS) a.ximage[idx] = image_dword<true>(a, X, kExactG, a.qx, idx);
        return;
    }
    const int idx = b * 256 + (int)threadIdx.x;
    if (idx < 4) a.counter[idx] = 0u;
    if (idx < a.rows * D.RS) a.image[idx] = image_dword<MSV>(a, D, G, Q, idx);
}

// MSV exact pass over the windows the filter kernel stored (Alg. 2 with
// its special states after every row).  Wavefront w of nw owns records
// w, w + nw, w + 2 nw, ... of the call (interleaved: records run longest
// first, and long sequences have more and longer windows) and rescores
// those whose flag the filter kernel left at kFlagPending, one window at a
// time, as a single 64-lane
// group holding QX registers of two cells per lane: the rows of a window
// depend on each other, and with few registers per lane a row is a few
// instructions.  A window {start offset, rows | tjb << 24, original id}
// starts with fresh cells and scB at sat0(base - tjb - tbm).
//
// Rows run in steps of 16 with scB fixed; since scE is a running maximum,
// one saturating u16 subtract of it against the level at the end of a step
// tells whether any cell in the step passed the value at which scB would
// change or the score overflows (invariant I4 of the kernel algebra).  Only
// then is the step replayed from a copy of its starting cells with that
// check after every row, and the special-state update (group max, new scJ
// and scB, cells lowered by the rise of scB: u becomes max(u - d, 0)) run
// where it fires.
constexpr int kExactAhead = 3;

template <int QX, int THREADS>
__global__ void __launch_bounds__(THREADS) exact_kernel(KArgs a) {
    constexpr int G = kExactG;
    using L = Lane<G, QX, true>;
    using Lay = typename L::Lay;
    constexpr int RS = Lay::RS;
    const int lane = threadIdx.x & 63;
    const uint32_t waves = blockDim.x / 64;
    const uint32_t nw = gridDim.x * waves;
    const uint32_t w = blockIdx.x * waves + threadIdx.x / 64;
    const uint32_t count = (uint32_t)a.nseq;
    // this wavefront's records: w + (b * 64 + lane) * nw for batches b
    const uint32_t nb = (count + 64u * nw - 1u) / (64u * nw);
    auto pending = [&](uint32_t b, uint32_t &id) -> bool {
        const uint32_t t = w + (b * 64u + (uint32_t)lane) * nw;
        id = t < count ? a.seqs[t].id : 0u;
        return t < count && a.flag[id] == kFlagPending;
    };
    bool mine = false;
    for (uint32_t b = 0; b < nb; ++b) {
        uint32_t id;
        mine = mine || __any(pending(b, id));
    }
    if (!__syncthreads_or(mine)) return;          // no window in this block
    extern __shared__ uint32_t lds[];
    {
        const uint4 *src = (const uint4 *)a.ximage;
        uint4 *dst = (uint4 *)lds;
        const int n16 = a.rows * (RS / 4);
        for (int i = threadIdx.x; i < n16; i += blockDim.x) dst[i] = src[i];
    }
    __syncthreads();
    if (!mine) return;
    const uint32_t *T[3] = {lds + Lay::lane_off(lane, 4),
                            lds + Lay::OFF2 + Lay::lane_off(lane, 2),
                            lds + Lay::OFF1 + Lay::lane_off(lane, 1)};
    const int dbias = a.dbias;
    const int top = 254 - dbias;
    L st;
    for (uint32_t b = 0; b < nb; ++b) {
        uint32_t myid;
        unsigned long long todo = __ballot(pending(b, myid));
        while (todo) {
            const int k = __ffsll((long long)todo) - 1;
            todo &= todo - 1ull;
            const uint32_t sid = (uint32_t)__builtin_amdgcn_readlane((int)myid, k);
            const uint4 r = a.win[sid];
            // the window in whole 16-row steps: rows after its last loud step
            // (the sequence's own, then its non-scoring padding) change nothing
            const uint32_t ws = r.x, rows = ((r.y & kRowsMask) + 15u) & ~15u;
            const int tjbm = (int)(r.y >> 24) + a.tbm;
            int xb = kBase - tjbm;
            xb = xb < 0 ? 0 : xb;
            int cm = -1;              // exact running max of earlier scB epochs
            int built = 0;            // running max scB was last computed from
            bool ovf = false;
            uint32_t lvl = 0u;
            // the level: the largest relative cell value at which the running
            // max neither passes max(base + tec, built) nor reaches 255 - dbias
            auto set_level = [&]() {
                int lim = built > kBase + kTec ? built : kBase + kTec;
                lim = lim < top ? lim : top;
                int rel = lim - xb;
                rel = rel < 0 ? 0 : rel;
                lvl = ovf ? 0xffffffffu : units_splat(rel);
            };
            auto above_level = [&]() -> bool {
                return (uint32_t)__builtin_bit_cast(
                           uint32_t, __builtin_elementwise_sub_sat(
                                         __builtin_bit_cast(u16x2, st.xE),
                                         __builtin_bit_cast(u16x2, lvl))) != 0u;
            };
            // running max = max(cm, current epoch's max + scB); -1 while the
            // current epoch never rose above scB
            auto epoch_max = [&]() -> int {
                int m = bits_to_units(group_max<G>(lane_max_bits(st.xE)));
                return m > 0 ? m + xb : -1;
            };
            set_level();
            st.reset();
            // The window's residues come 1024 at a time, 16 per lane (windows
            // start 16-byte aligned; sequences are stored in whole 16-residue
            // steps); each step takes its 16 from one lane into scalar
            // registers.  Scores are read
            // kExactAhead rows ahead (the LDS latency is what bounds a row).
            uint4 blk = make_uint4(0u, 0u, 0u, 0u);
            uint32_t cbuf[kExactAhead + 1][QX];
            for (uint32_t s = 0; s < rows; s += 16) {
                if ((s & 1023u) == 0u) {
                    const uint32_t o = s + 16u * (uint32_t)lane;
                    blk = o < rows ? *(const uint4 *)(a.res + ws + o) : make_uint4(0u, 0u, 0u, 0u);
                }
                const int src = (int)((s & 1023u) >> 4);
                uint4 wv;
                wv.x = (uint32_t)__builtin_amdgcn_readlane((int)blk.x, src);
                wv.y = (uint32_t)__builtin_amdgcn_readlane((int)blk.y, src);
                wv.z = (uint32_t)__builtin_amdgcn_readlane((int)blk.z, src);
                wv.w = (uint32_t)__builtin_amdgcn_readlane((int)blk.w, src);
                auto xrow = [&](int k2) -> uint32_t {
                    const uint32_t word = k2 < 4 ? wv.x : k2 < 8 ? wv.y : k2 < 12 ? wv.z : wv.w;
                    return (word >> (8 * (k2 % 4))) & 0xffu;
                };
                // the step's rows; CHECK: the special states after each row
                // the step's 16 rows; CHECK: the special states after each
                auto step = [&](auto check_c) {
                    constexpr int N = 16;
#pragma unroll
                    for (int k2 = 0; k2 < kExactAhead; ++k2)
                        st.load_row(T[0], T[1], T[2], xrow(k2), cbuf[k2]);
                    auto one_row = [&](auto k_c) {
                        constexpr int k2 = decltype(k_c)::value;
                        constexpr int ahead = k2 + kExactAhead;
                        if constexpr (ahead < N)
                            st.load_row(T[0], T[1], T[2], xrow(ahead),
                                        cbuf[ahead % (kExactAhead + 1)]);
                        st.update(cbuf[k2 % (kExactAhead + 1)]);
                        if constexpr (decltype(check_c)::value) {
                            if (__any(above_level())) {
                                int e2 = epoch_max();
                                int m2 = cm > e2 ? cm : e2;
                                int lim = built > kBase + kTec ? built : kBase + kTec;
                                if (!ovf && (m2 > lim || m2 >= 255 - dbias)) {
                                    if (m2 >= 255 - dbias) ovf = true;
                                    int j2 = m2 - kTec > kBase ? m2 - kTec : kBase;
                                    int xbn = j2 - tjbm;
                                    xbn = xbn < 0 ? 0 : (xbn > 255 ? 255 : xbn);
                                    if (xbn > xb) {          // new scB epoch
                                        st.lower(xbn - xb);
                                        st.xE = 0u;
                                        cm = m2;
                                        xb = xbn;
                                    }
                                    built = m2;
                                    set_level();
                                }
                            }
                        }
                    };
                    [&]<int... R>(std::integer_sequence<int, R...>) {
                        (one_row(std::integral_constant<int, R>{}), ...);
                    }(std::make_integer_sequence<int, N>{});
                };
                // with scB fixed; replayed from its starting cells, row by row
                // with the special states, if a cell passed the level
                uint32_t save[QX];
#pragma unroll
                for (int q = 0; q < QX; ++q) save[q] = st.R[q];
                const uint32_t save_xe = st.xE;
                step(std::false_type{});
                if (__any(above_level())) {
#pragma unroll
                    for (int q = 0; q < QX; ++q) st.R[q] = save[q];
                    st.xE = save_xe;
                    step(std::true_type{});
                }
            }
            int em = epoch_max();
            int mx = cm > em ? cm : em;
            if (lane == 0) {
                const bool of = ovf || mx >= 255 - dbias;
                const int v = mx - kTec;
                a.score[sid] = of ? 255 : (uint8_t)(v < 0 ? 0 : v);
                a.flag[sid] = of ? 1 : 0;
            }
        }
    }
}

// Block sizes: up to 8 wavefronts, or up to 16 for groups of 32 and 64 lanes
// (their large LDS tables allow one block per CU, so a 16-wavefront block is
// the only way to four wavefronts per SIMD).  Each size is its own kernel:
// the compiler budgets registers for the block size it is told.
template <int G>
constexpr int kMaxWaves = G >= 32 ? 16 : 8;

template <int G, int Q, int MODE, int THREADS>
hipError_t launch_filter_kernel(const KArgs &a, int wpb, int blocks, hipStream_t s) {
    size_t lds = lds_bytes(G, Q, a.rows);
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void *)filter_kernel<G, Q, MODE, THREADS>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((filter_kernel<G, Q, MODE, THREADS>), dim3(blocks), dim3(wpb * 64), lds,
                       s, a);
    return hipGetLastError();
}

template <int G, int Q, int MODE>
hipError_t launch_filter_mode(const KArgs &a, int wpb, int blocks, hipStream_t s) {
    if constexpr (kMaxWaves<G> > 8) {
        if (wpb > 8) return launch_filter_kernel<G, Q, MODE, 1024>(a, wpb, blocks, s);
    }
    return launch_filter_kernel<G, Q, MODE, 512>(a, wpb, blocks, s);
}

// prep (LDS images, counters, MSV best scores, split-sequence records),
// then the filter kernel: SSV (and the combination of split sequences), or
// MSV with scB fixed (the host launches the exact pass next).
template <int G, int Q, bool MSV>
hipError_t launch_filter(const KArgs &a, int wpb, int blocks, hipStream_t s) {
    if (a.rows != kRows && a.rows != kDegenRows) return hipErrorInvalidValue;
    const int n = a.rows * Layout<G, Q>::RS;
    const int nb = (n + 255) / 256;
    if (wpb < 1 || wpb > kMaxWaves<G>) return hipErrorInvalidValue;
    const int xb = MSV ? (a.rows * lds_layout(kExactG, a.qx).RS + 255) / 256 : 0;
    const int seg_blocks = (a.nsegs + 255) / 256;
    hipLaunchKernelGGL((prep_kernel<G, Q, MSV>), dim3(nb + xb + (MSV ? a.rows : 0) + seg_blocks),
                       dim3(256), 0, s, a, nb, xb);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if constexpr (MSV) {
        e = launch_filter_mode<G, Q, kMSV>(a, wpb, blocks, s);
        if (e != hipSuccess || a.nsplit == 0) return e;
        hipLaunchKernelGGL(combine_msv_kernel<kWordsPerLoad<G>>, dim3((a.nsplit + 255) / 256),
                           dim3(256), 0, s, a);
        return hipGetLastError();
    }
    e = launch_filter_mode<G, Q, kSSV>(a, wpb, blocks, s);
    if (e != hipSuccess || a.nsplit == 0) return e;
    hipLaunchKernelGGL(combine_kernel, dim3((a.nsplit + 255) / 256), dim3(256), 0, s, a);
    return hipGetLastError();
}

template <int G, int Q, int MODE, int THREADS>
int occupancy_kernel(int wpb, int rows) {
    int nb = 0;
    size_t lds = lds_bytes(G, Q, rows);
    if (hipFuncSetAttribute((const void *)filter_kernel<G, Q, MODE, THREADS>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
        return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, filter_kernel<G, Q, MODE, THREADS>,
                                                     wpb * 64, lds) != hipSuccess)
        return 0;
    return nb;
}

template <int G, int Q, bool MSV>
int occupancy_filter(int wpb, int rows) {
    constexpr int MODE = MSV ? kMSV : kSSV;
    if (wpb < 1 || wpb > kMaxWaves<G>) return 0;
    if constexpr (kMaxWaves<G> > 8) {
        if (wpb > 8) return occupancy_kernel<G, Q, MODE, 1024>(wpb, rows);
    }
    return occupancy_kernel<G, Q, MODE, 512>(wpb, rows);
}

// The exact pass: blocks of four wavefronts, as many as fit on the device
// at once (blocks without a window leave after their scan).
constexpr int kExactThreads = 256;

template <int QX>
hipError_t launch_exact(const KArgs &a, int cus, hipStream_t s) {
    const size_t lds = lds_bytes(kExactG, QX, a.rows);
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void *)exact_kernel<QX, kExactThreads>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    int per_cu = (int)((size_t)kLdsBytes / lds);
    per_cu = per_cu < 1 ? 1 : (per_cu > 8 ? 8 : per_cu);
    hipLaunchKernelGGL((exact_kernel<QX, kExactThreads>), dim3(cus * per_cu),
                       dim3(kExactThreads), lds, s, a);
    return hipGetLastError();
}

}  // namespace hmsv
