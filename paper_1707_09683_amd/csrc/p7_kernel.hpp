// P7Viterbi (gapped Plan-7 Viterbi) filter kernel for gfx950.
//
// What it computes (paper Sec. 2.1, Eq. 1, with the Plan-7 special states
// N, B, E, C, J of the DP matrix's flanks), in int16 saturating arithmetic
// with -32768 as -inf, for residues x_1..x_L and nodes j = 1..M:
//   M[i][j] = msc_j(x_i) + max(M[i-1][j-1] + tMM, I[i-1][j-1] + tIM,
//                              D[i-1][j-1] + tDM, B[i-1] + tBM)
//   I[i][j] = max(M[i-1][j] + tMI, I[i-1][j] + tII)        (insert score 0)
//   D[i][j] = max(M[i][j-1] + tMD, D[i][j-1] + tDD)
// then per row E = max_j M, J = max(J + tJJ, E + tEJ), C = max(C + tCC,
// E + tEC), N = N + tNN, B = max(N + tNB, J + tJB); score = C[L] + tCT, or
// 32767 with the overflow flag once a row's E saturates.
//
// Mapping (as the MSV/SSV kernel): a lane group of G lanes aligns one
// sequence; each lane holds Q registers of two int16 cells for each of M,
// I and D, striped (register q, element e = lane e/2, half e%2, is slot
// q + Q e; slot 0 is a dummy node whose emissions and transitions are -inf,
// so every value it holds reaches a real node only through a -inf
// transition).  Packed saturating adds (v_pk_add_i16 clamp) and maxima
// (v_pk_max_i16) update two cells per instruction.
//
// Per row: M and I in place, registers in descending order; D within each
// element in ascending order, its first slot taking the previous element's
// last M (M->D); then the D->D chains across elements are completed
// Farrar-style ("lazy F"): each element takes the last D of the element
// before it (one DPP shift) and carries it along its slots, max-ing it in,
// while some element's last D rises to a value that can still raise a
// cell of the next row (max and a saturating add of a fixed score commute,
// so every such value is the sequential chain's; values below that bound
// change no M, no E and no score).  Scores come from LDS: 21 rows of match
// emissions by residue (27 with the degenerate codes) and 7 rows of
// transitions, in the MSV image's conflict-free layout.  The special
// states, packed int16, are updated once per row from the group's maximum.
//
// Lane groups take records (longest first) from queues as they finish one;
// the next record is loaded, and the one after it claimed, while the
// current one runs.  A sequence runs exactly L rows: the rows of the last
// 16-residue step past L leave the special states untouched.
#pragma once
#include <utility>
#include "filter_kernel.hpp"

namespace hmsv {

typedef short s16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ s16x2 as_s16x2(uint32_t v) { return __builtin_bit_cast(s16x2, v); }
__device__ __forceinline__ uint32_t s16_bits(s16x2 v) { return __builtin_bit_cast(uint32_t, v); }
__device__ __forceinline__ s16x2 adds(s16x2 a, s16x2 b) { return __builtin_elementwise_add_sat(a, b); }
__device__ __forceinline__ s16x2 smax(s16x2 a, s16x2 b) { return __builtin_elementwise_max(a, b); }
__device__ __forceinline__ s16x2 splat16(int v) { return s16x2{(short)v, (short)v}; }

constexpr int kP7Neg = -32768;
constexpr int kP7Pos = 32767;
constexpr int kP7Half = -32;          // E->J and E->C: 32 log2(1/2)
__device__ __forceinline__ int sat16(int v) { return v < kP7Neg ? kP7Neg : (v > kP7Pos ? kP7Pos : v); }

// Score of table row r (emissions by residue below a.rows, transitions
// from there) at slot s (node s; slot 0 is the dummy).
__device__ __forceinline__ int p7_slot_score(const P7Args &a, int r, int s) {
    const int M = a.M;
    if (r < a.rows) {
        if (s < 1 || s > M || r == kInvalidCode) return kP7Neg;
        return a.msc[r * M + s - 1];
    }
    // transitions: MMp, IMp, DMp, MDp, DDp come from node s - 1; MI, II
    // from node s (their table rows: MM 0, MI 1, MD 2, IM 3, II 4, DM 5, DD 6)
    const int t = r - a.rows;
    const int from = (t == kP7MI || t == kP7II) ? s : s - 1;
    if (from < 1 || from > M) return kP7Neg;
    const int row = t == kP7MMp ? 0 : t == kP7IMp ? 3 : t == kP7DMp ? 5 : t == kP7MI ? 1
                  : t == kP7II ? 4 : t == kP7MDp ? 2 : 6;
    return a.trans[row * M + from - 1];
}

// The LDS image (a.rows + 7 rows of the lds_layout(G, Q, kP7Rows) shape),
// one dword per thread.
template <int G, int Q>
__global__ void __launch_bounds__(256) p7_prep_kernel(P7Args a, int image_blocks) {
    constexpr LdsLayout D = lds_layout(G, Q, kP7Rows);
    if ((int)blockIdx.x == image_blocks) {
        // the last block: max over nodes of D->M into aux[0]
        __shared__ int red[256];
        int m = kP7Neg;
        for (int k = threadIdx.x; k < a.M; k += 256) {
            const int v = a.trans[5 * a.M + k];
            m = v > m ? v : m;
        }
        red[threadIdx.x] = m;
        __syncthreads();
        for (int h = 128; h > 0; h >>= 1) {
            if ((int)threadIdx.x < h && red[threadIdx.x + h] > red[threadIdx.x])
                red[threadIdx.x] = red[threadIdx.x + h];
            __syncthreads();
        }
        if (threadIdx.x == 0) a.aux[0] = red[0];
        if (threadIdx.x < kP7Parts) a.queue[threadIdx.x * 32] = 0u;   // the record queues
        return;
    }
    const int idx = (int)(blockIdx.x * 256 + threadIdx.x);
    if (idx >= (a.rows + 7) * D.RS) return;
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
    rem %= G * w;
    const int jj = rem / w;
    const int qq = q0 + (rem - jj * w);
    const int s0 = qq + Q * (2 * jj);
    uint32_t v = 0u;
    if (qq < Q) {
        const uint32_t lo = (uint16_t)(short)p7_slot_score(a, x, s0);
        const uint32_t hi = (uint16_t)(short)p7_slot_score(a, x, s0 + Q);
        v = lo | (hi << 16);
    }
    a.image[idx] = v;
}

template <int G, int Q, int THREADS>
__global__ void __launch_bounds__(THREADS) p7_kernel(P7Args a) {
    using Lay = Layout<G, Q, kP7Rows>;
    constexpr int RS = Lay::RS;
    extern __shared__ uint32_t lds[];
    {
        const uint4 *src = (const uint4 *)a.image;
        uint4 *dst = (uint4 *)lds;
        const int n16 = (a.rows + 7) * (RS / 4);
        for (int i = threadIdx.x; i < n16; i += blockDim.x) dst[i] = src[i];
    }
    __syncthreads();
    const int maxdm = a.aux[0];       // max over nodes of D->M (prep kernel)

    const int lane = threadIdx.x & 63;
    const int j = lane % G;
    const bool gstart = j == 0;
    const uint32_t *T[3] = {lds + Lay::lane_off(lane, 4),
                            lds + Lay::OFF2 + Lay::lane_off(lane, 2),
                            lds + Lay::OFF1 + Lay::lane_off(lane, 1)};
    // Dwords of table row r for this lane: chunk ch of 4 (registers
    // 4ch..4ch+3), the 2-dword tail (registers Q2, Q2+1), the 1-dword tail
    // (register Q1).
    auto chunk = [&](uint32_t r, int ch) -> uint4 {
        return *(const uint4 *)((const char *)T[0] + r * (uint32_t)(RS * 4) + ch * Lay::CW * 4);
    };
    auto tail2 = [&](uint32_t r) -> uint2 {
        return *(const uint2 *)((const char *)T[1] + r * (uint32_t)(RS * 4));
    };
    auto tail1 = [&](uint32_t r) -> uint32_t {
        return *(const uint32_t *)((const char *)T[2] + r * (uint32_t)(RS * 4));
    };
    auto comp = [](const uint4 &v, int u) -> uint32_t {
        return u == 0 ? v.x : u == 1 ? v.y : u == 2 ? v.z : v.w;
    };
    const uint32_t rT = (uint32_t)a.rows;    // first transition row

    // Records: the whole database (processing positions 0..nseq-1), or the
    // positions a selection pass left in sel[0 .. *nsel) (a device count,
    // known only here; never more than the database holds).
    const int32_t *sel = a.sel;
    const int nseq = sel ? min(*a.nsel, a.nseq) : a.nseq;
    // Records come from queues (counters the prep kernel zeroed), longest
    // first: a lane group claims a record as it starts one, so a group that
    // drew a long sequence draws fewer others.  Blocks are spread over up to
    // kP7Parts queues, each on its own 128-byte line: queue p hands out
    // records p, p + P, p + 2P, ... (each longest first), so one counter's
    // atomics come from a fraction of the grid.  A claim is taken (its value
    // broadcast from the group's first lane) only at the group's next
    // switch, by when it has returned: `issue` for the groups that claim,
    // `take` by the whole wavefront.
    const int nparts = (int)(gridDim.x < (unsigned)kP7Parts ? gridDim.x : (unsigned)kP7Parts);
    const int part = (int)(blockIdx.x % (unsigned)nparts);
    uint32_t *ctr = a.queue + part * 32;
    uint32_t craw = 0u;
    auto issue = [&](bool want) {    // called by the whole wavefront
        // one atomic per wavefront (by lane 0) for all of its claiming
        // groups, each group's claim its rank among them
        const bool w = want && gstart;
        const unsigned long long m = __ballot(w);
        if (m == 0ull) return;
        uint32_t base = 0u;
        if (lane == 0) base = atomicAdd(ctr, (uint32_t)__popcll(m));
        base = (uint32_t)__builtin_amdgcn_readfirstlane((int)base);
        const uint32_t rank = __builtin_amdgcn_mbcnt_hi(
            (uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
        if (w) craw = base + rank;
    };
    auto take = [&]() -> int {    // a processing position, or -1: none left
        int k = (int)craw;
        if constexpr (G > 1) k = __shfl(k, lane - j);
        const long long r = (long long)part + (long long)nparts * (long long)k;
        if (r >= (long long)nseq) return -1;
        return sel ? sel[r] : (int)r;
    };

    s16x2 Mr[Q], Ir[Q], Dr[Q];
    issue(true);
    int t = take();
    uint4 rec = make_uint4(0u, 0u, 0u, 0u), rec16 = rec;
    uint32_t lm = 0u;
    if (t >= 0) {
        rec = *(const uint4 *)(a.seqs + t);
        rec16 = *((const uint4 *)(a.seqs + t) + 1);
        lm = a.lenmodel[t];
    }
    // the next record, claimed and loaded while the current one runs
    issue(true);
    int tn = take();
    uint4 nrec = rec, nrec16 = rec16;
    uint32_t nlm = lm;
    auto prefetch = [&]() {
        if (tn >= 0) {
            nrec = *(const uint4 *)(a.seqs + tn);
            nrec16 = *((const uint4 *)(a.seqs + tn) + 1);
            nlm = a.lenmodel[tn];
        }
    };

    bool active = false;
    uint32_t off = a.pad_off, seq_off = a.pad_off, id = 0;
    int len = 0, done = 0;       // residues of the sequence, rows run so far
    int loop = 0, move = 0;      // length model: N/J/C loops, N/J->B and C->T
    // special states, packed: JC = (J, C), NN = (N, N), B in Bv's low half
    s16x2 JC = splat16(kP7Neg), NN = splat16(0), Bv = splat16(0);
    s16x2 loop2 = splat16(0), move2 = splat16(0);
    const s16x2 tbm2 = splat16(a.tbm), half2 = splat16(kP7Half);
    bool ovf = false;
    uint4 wv = make_uint4(0u, 0u, 0u, 0u);   // this step's 16 residues
    const s16x2 neg = splat16(kP7Neg);
    auto start = [&]() {
        active = t >= 0;
        seq_off = active ? rec.x : a.pad_off;
        off = seq_off;
        id = rec.z;
        len = active ? (int)rec.w : 0;
        done = 0;
        loop = (int)(short)(lm & 0xffffu);
        move = (int)(short)(lm >> 16);
        loop2 = splat16(loop);
        move2 = splat16(move);
        NN = splat16(0);
        Bv = adds(NN, move2);
        JC = splat16(kP7Neg);
        ovf = false;
        wv = active ? rec16 : make_uint4(0x14141414u, 0x14141414u, 0x14141414u, 0x14141414u);
#pragma unroll
        for (int q = 0; q < Q; ++q) Mr[q] = Ir[q] = Dr[q] = neg;
    };
    start();
    prefetch();
    issue(true);                 // the record after that, taken at the switch

    for (;;) {
        if (!__any(active)) break;
        bool ended = false;
        do {
            // residues of the next step (the database stores every sequence
            // in whole 16-residue steps plus 16 more bytes)
            const uint4 wn = *(const uint4 *)(a.res + off + 16u);
            // The floor under the B->M score of the rows after this step's
            // rows (B >= N + move, and N only falls: the loop score is <= 0,
            // so N after the step's last row bounds every row of the step).
            // A D value d can raise a cell of the next row only through
            // D->M, to at most d + maxdm, while every such cell is at least
            // that floor: D values below thr cannot change any M, hence no E
            // and no score (D feeds nothing else).  A lower bound than the
            // row's own is still a bound, so one per step serves its rows.
            int thr_step;
            {
                const int nEnd = sat16((int)NN.x + 16 * loop);
                const int t1 = sat16(sat16(nEnd + move) + a.tbm) - maxdm - 1;
                thr_step = active ? (t1 > kP7Pos ? kP7Pos : (t1 < kP7Neg ? kP7Neg : t1)) : kP7Pos;
            }
            const s16x2 thr1 = splat16(thr_step);
#pragma unroll 1
            for (int r = 0; r < 16; ++r) {
                const uint32_t word = r < 4 ? wv.x : r < 8 ? wv.y : r < 12 ? wv.z : wv.w;
                const uint32_t x = __builtin_amdgcn_ubfe(word, 8u * (uint32_t)(r & 3), 8u);
                const bool live = active && done + r < len;
                const s16x2 bc = adds(__builtin_shufflevector(Bv, Bv, 0, 0), tbm2);
                // ---- M and I, registers in descending order ----------------
                // (in place: slot q's new M reads the old M, I and D of slot
                // q - 1, not yet overwritten; its new I reads its own old M
                // and I, updated first).  Slot 0 of each element reads the
                // previous element's last slot, shifted in before the pass.
                const s16x2 sM = as_s16x2(shift_in(s16_bits(Mr[Q - 1])));
                const s16x2 sI = as_s16x2(shift_in(s16_bits(Ir[Q - 1])));
                const s16x2 sD = as_s16x2(shift_in(s16_bits(Dr[Q - 1])));
                s16x2 xe = neg;
                auto mi_cell = [&](int q, uint32_t e, uint32_t mm, uint32_t im, uint32_t dm,
                                   uint32_t mi, uint32_t ii) {
                    const s16x2 gM = q > 0 ? Mr[q - 1] : sM;
                    const s16x2 gI = q > 0 ? Ir[q - 1] : sI;
                    const s16x2 gD = q > 0 ? Dr[q - 1] : sD;
                    // (pinned here: left to itself the compiler sinks the I
                    // update to the row's end and keeps copies of the old M)
                    s16x2 nI = smax(adds(Mr[q], as_s16x2(mi)), adds(Ir[q], as_s16x2(ii)));
                    asm volatile("" : "+v"(nI));
                    Ir[q] = nI;
                    const s16x2 c = smax(smax(adds(gM, as_s16x2(mm)), adds(gI, as_s16x2(im))),
                                         smax(adds(gD, as_s16x2(dm)), bc));
                    Mr[q] = adds(c, as_s16x2(e));
                    xe = smax(xe, Mr[q]);
                };
                if constexpr (Lay::T1) {
                    mi_cell(Lay::Q1, tail1(x), tail1(rT + kP7MMp), tail1(rT + kP7IMp),
                            tail1(rT + kP7DMp), tail1(rT + kP7MI), tail1(rT + kP7II));
                }
                if constexpr (Lay::T2) {
                    const uint2 ve = tail2(x), vmm = tail2(rT + kP7MMp), vim = tail2(rT + kP7IMp),
                                vdm = tail2(rT + kP7DMp), vmi = tail2(rT + kP7MI),
                                vii = tail2(rT + kP7II);
                    mi_cell(Lay::Q2 + 1, ve.y, vmm.y, vim.y, vdm.y, vmi.y, vii.y);
                    mi_cell(Lay::Q2, ve.x, vmm.x, vim.x, vdm.x, vmi.x, vii.x);
                }
#pragma unroll
                for (int ch = Lay::NF - 1; ch >= 0; --ch) {
                    // one chunk's 24 score dwords at a time: keeps the
                    // scheduler from hoisting every chunk's loads at once
                    __builtin_amdgcn_sched_barrier(0);
                    const uint4 ve = chunk(x, ch), vmm = chunk(rT + kP7MMp, ch),
                                vim = chunk(rT + kP7IMp, ch), vdm = chunk(rT + kP7DMp, ch),
                                vmi = chunk(rT + kP7MI, ch), vii = chunk(rT + kP7II, ch);
#pragma unroll
                    for (int u = 3; u >= 0; --u) {
                        if (ch * 4 + u < Q)
                            mi_cell(ch * 4 + u, comp(ve, u), comp(vmm, u), comp(vim, u),
                                    comp(vdm, u), comp(vmi, u), comp(vii, u));
                    }
                }
                // ---- D within each element, ascending ----------------------
                // (from the new M; slot 0 takes the previous element's last M
                // through M->D here, its last D below)
                const s16x2 sMn = as_s16x2(shift_in(s16_bits(Mr[Q - 1])));
                uint32_t dd0 = 0u;
                auto d_cell = [&](int q, uint32_t md, uint32_t dd) {
                    if (q == 0) {
                        Dr[0] = adds(sMn, as_s16x2(md));
                        dd0 = dd;
                    } else {
                        Dr[q] = smax(adds(Mr[q - 1], as_s16x2(md)), adds(Dr[q - 1], as_s16x2(dd)));
                    }
                };
#pragma unroll
                for (int ch = 0; ch < Lay::NF; ++ch) {
                    const uint4 vmd = chunk(rT + kP7MDp, ch), vdd = chunk(rT + kP7DDp, ch);
#pragma unroll
                    for (int u = 0; u < 4; ++u)
                        if (ch * 4 + u < Q) d_cell(ch * 4 + u, comp(vmd, u), comp(vdd, u));
                }
                if constexpr (Lay::T2) {
                    const uint2 vmd = tail2(rT + kP7MDp), vdd = tail2(rT + kP7DDp);
                    d_cell(Lay::Q2, vmd.x, vdd.x);
                    d_cell(Lay::Q2 + 1, vmd.y, vdd.y);
                }
                if constexpr (Lay::T1) d_cell(Lay::Q1, tail1(rT + kP7MDp), tail1(rT + kP7DDp));
                // ---- D chains across elements, where they matter ----------
                // Each element's first slot takes the previous element's last
                // D (through D->D), carried along its slots; passes repeat
                // while some element's last D rose to a value that matters
                // (at least thr).  Values that do not matter may stay below
                // the sequential chain's.
                s16x2 in0 = adds(as_s16x2(shift_in(s16_bits(Dr[Q - 1]))), as_s16x2(dd0));
                s16x2 lim = smax(Dr[0], thr1);
                bool more = __any(s16_bits(smax(in0, lim)) != s16_bits(lim));
                while (more) {
                    const s16x2 last = Dr[Q - 1];
                    Dr[0] = smax(Dr[0], in0);
                    auto link = [&](int q, uint32_t dd) {
                        if (q > 0) Dr[q] = smax(Dr[q], adds(Dr[q - 1], as_s16x2(dd)));
                    };
#pragma unroll
                    for (int ch = 0; ch < Lay::NF; ++ch) {
                        const uint4 vdd = chunk(rT + kP7DDp, ch);
#pragma unroll
                        for (int u = 0; u < 4; ++u)
                            if (ch * 4 + u < Q) link(ch * 4 + u, comp(vdd, u));
                    }
                    if constexpr (Lay::T2) {
                        const uint2 vdd = tail2(rT + kP7DDp);
                        link(Lay::Q2, vdd.x);
                        link(Lay::Q2 + 1, vdd.y);
                    }
                    if constexpr (Lay::T1) link(Lay::Q1, tail1(rT + kP7DDp));
                    lim = smax(last, thr1);
                    more = __any(s16_bits(smax(Dr[Q - 1], lim)) != s16_bits(lim));
                    in0 = adds(as_s16x2(shift_in(s16_bits(Dr[Q - 1]))), as_s16x2(dd0));
                }
                // ---- special states (Plan-7 N, B, E, C, J) ----------------
                const int eh = (int)xe.x > (int)xe.y ? (int)xe.x : (int)xe.y;
                const int E = group_max<G>(eh);
                if (live) {
                    if (E >= kP7Pos) ovf = true;
                    // J = max(J + loop, E - 32), C = max(C + loop, E - 32)
                    JC = smax(adds(JC, loop2), adds(splat16(E), half2));
                    NN = adds(NN, loop2);
                    // B = max(N + move, J + move) = max(N, J) + move
                    // (saturation is monotone): the low halves
                    Bv = adds(smax(NN, JC), move2);
                }
            }
            done += 16;
            // groups without a sequence stay on the padding (>= 64 bytes of
            // code 20 at pad_off)
            if (active) off += 16u;
            wv = wn;
            ended = active && done >= len;
        } while (!__any(ended));

        // ---- finished sequences: score, then the next record ---------------
        if (ended && gstart) {
            a.score[id] = ovf ? (int16_t)kP7Pos : (int16_t)sat16((int)JC.y + move);
            a.flag[id] = ovf ? 1 : 0;
        }
        const int claimed = take();
        if (ended) {
            t = tn;
            tn = claimed;
            rec = nrec;
            rec16 = nrec16;
            lm = nlm;
            start();
            prefetch();
        }
        issue(ended);
    }
}

// Blocks of up to 8 wavefronts (512 threads), or 16 for 64-lane groups
// whose kernel fits the 128 VGPRs of a 1024-thread block without spilling
// (Q <= 18 and Q = 20; the compiler spills 20-40 bytes per lane at Q = 19,
// 21 and 22): their LDS image allows one block per CU, so 16 wavefronts per
// block is the way to 4 per SIMD.
template <int G, int Q>
constexpr int kP7MaxWaves = (G == 64 && (Q <= 18 || Q == 20)) ? 16 : 8;

template <int G, int Q, int THREADS>
hipError_t launch_p7_kernel(const P7Args &a, int wpb, int blocks, hipStream_t s) {
    const size_t lds = p7_lds_bytes(G, Q, a.rows);
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void *)p7_kernel<G, Q, THREADS>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((p7_kernel<G, Q, THREADS>), dim3(blocks), dim3(wpb * 64), lds, s, a);
    return hipGetLastError();
}

// The LDS image, then the filter kernel.
template <int G, int Q>
hipError_t launch_p7(const P7Args &a, int wpb, int blocks, hipStream_t s) {
    if (a.rows != kRows && a.rows != kDegenRows) return hipErrorInvalidValue;
    const int n = (a.rows + 7) * lds_layout(G, Q, kP7Rows).RS;
    if (wpb < 1 || wpb > kP7MaxWaves<G, Q>) return hipErrorInvalidValue;
    hipLaunchKernelGGL((p7_prep_kernel<G, Q>), dim3((n + 255) / 256 + 1), dim3(256), 0, s, a,
                       (n + 255) / 256);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if constexpr (kP7MaxWaves<G, Q> > 8) {
        if (wpb > 8) return launch_p7_kernel<G, Q, 1024>(a, wpb, blocks, s);
    }
    return launch_p7_kernel<G, Q, 512>(a, wpb, blocks, s);
}

template <int G, int Q, int THREADS>
int occupancy_p7_kernel(int wpb, int rows) {
    int nb = 0;
    const size_t lds = p7_lds_bytes(G, Q, rows);
    if (hipFuncSetAttribute((const void *)p7_kernel<G, Q, THREADS>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
        return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, p7_kernel<G, Q, THREADS>, wpb * 64,
                                                     lds) != hipSuccess)
        return 0;
    return nb;
}

// Resident blocks of wpb wavefronts per CU (0 on error or an unsupported
// block size).
template <int G, int Q>
int occupancy_p7(int wpb, int rows) {
    if (wpb < 1 || wpb > kP7MaxWaves<G, Q>) return 0;
    if constexpr (kP7MaxWaves<G, Q> > 8) {
        if (wpb > 8) return occupancy_p7_kernel<G, Q, 1024>(wpb, rows);
    }
    return occupancy_p7_kernel<G, Q, 512>(wpb, rows);
}

}  // namespace hmsv
