// MSV / SSV filter kernel for gfx950.
//
// Mapping (compare paper Sec. 3.1, tiers 3-5):
//  * A lane group of G lanes aligns one sequence at a time; 64/G groups share
//    a wavefront (the paper's S-lane multi-sequence alignment, tier 4).
//  * Each lane holds Q 32-bit registers, each two 16-bit cells (tier 5 uses
//    4x8-bit SIMD video ops on the K40; gfx950 has packed 16-bit saturating
//    VALU ops instead).  The group's 2*G*Q cells are striped: register q,
//    element e (lane e/2, half e%2) is node q + Q*e, so only register Q-1
//    crosses lanes when the row moves one node to the right (Alg. 5's
//    reorder becomes one DPP move plus one v_alignbit per row).
//  * Cells are kept as signed 16-bit "offset" values so that the floor of
//    the 8-bit arithmetic is the i16 saturation point -32768:
//      MSV  v  - 32768, per-cell add  dbias - cost   (Alg. 2 lines 17-19
//           fused into one saturating add; the 255 cap never fires before
//           the overflow row, and overflow is flagged from the running max)
//      SSV  d  - 32640, per-cell add  sc             (Alg. 7)
//    so -inf is 0x8000 for both, and a cell update is
//      MSV  v = adds(max(gamma, scB), s)     SSV  v = adds(gamma, s)
//    followed by scE = max(scE, v) (running max, never reset per row).
//  * Per-node scores of the 21 table rows live in LDS, laid out
//    [row][q][lane-in-group] so the G lanes of a group read consecutive
//    dwords.
//  * Sequences are handed out longest first from a global counter as
//    groups finish (replaces the pre-packed warp blocks of Alg. 1).
//  * MSV special states: scB only changes when the running max exceeds
//    max(base + tec, the max it was last computed from), so rows run in
//    tiles with scB fixed; at the tile end the group max is checked and, if
//    it moved (or overflowed), the tile is replayed from a register
//    checkpoint with the per-row special-state update (Alg. 2 lines 24-25).
#pragma once
#include "hmsv_internal.h"

namespace hmsv {

typedef short s16x2 __attribute__((ext_vector_type(2)));

constexpr uint32_t kNeg2 = 0x80008000u;       // two cells at -inf
constexpr uint32_t kInvalid4 = 0x14141414u;   // four non-scoring residues
constexpr int kBase = 190;
constexpr int kTec = 3;

__device__ __forceinline__ uint32_t pk_max(uint32_t a, uint32_t b) {
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(
        __builtin_bit_cast(s16x2, a), __builtin_bit_cast(s16x2, b)));
}

__device__ __forceinline__ uint32_t pk_adds(uint32_t a, uint32_t b) {
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_add_sat(
        __builtin_bit_cast(s16x2, a), __builtin_bit_cast(s16x2, b)));
}

__device__ __forceinline__ int lane_max(uint32_t v) {
    int lo = (int)(short)(v & 0xffffu);
    int hi = (int)(short)(v >> 16);
    return lo > hi ? lo : hi;
}

template <int G>
__device__ __forceinline__ int group_max(int m) {
#pragma unroll
    for (int o = 1; o < G; o <<= 1) {
        int t = __shfl_xor(m, o);
        m = m > t ? m : t;
    }
    return m;
}

// Cells of the previous row shifted one node to the right, for register 0:
// element e takes element e-1 of register Q-1; element 0 of each group
// takes -inf (node 1 has no upper-left neighbour).
template <int G>
__device__ __forceinline__ uint32_t shift_in(uint32_t last, bool gstart) {
    uint32_t nb;
    if constexpr (G == 64) {
        nb = (uint32_t)__builtin_amdgcn_update_dpp((int)kNeg2, (int)last, 0x138, 0xf, 0xf, false);
    } else if constexpr (G == 16) {
        nb = (uint32_t)__builtin_amdgcn_update_dpp((int)kNeg2, (int)last, 0x111, 0xf, 0xf, false);
    } else if constexpr (G == 32) {
        nb = (uint32_t)__builtin_amdgcn_update_dpp((int)kNeg2, (int)last, 0x138, 0xf, 0xf, false);
        nb = gstart ? kNeg2 : nb;
    } else {
        nb = (uint32_t)__builtin_amdgcn_update_dpp((int)kNeg2, (int)last, 0x111, 0xf, 0xf, false);
        nb = gstart ? kNeg2 : nb;
    }
    return __builtin_amdgcn_alignbit(last, nb, 16);
}

__device__ __forceinline__ uint32_t splat16(int v) {
    uint32_t u = (uint32_t)(v & 0xffff);
    return u | (u << 16);
}

template <bool MSV>
__device__ __forceinline__ int table_value(const KArgs &a, int x, int k) {
    if (k >= a.M) return -32768;                    // padding node: -inf
    if (MSV) return a.dbias - (int)a.cost[x * a.M + k];
    return (int)a.sc[x * a.M + k];
}

template <int G, int Q, bool MSV>
struct Lane {
    uint32_t R[Q];
    uint32_t xE;
    uint32_t xB;

    __device__ __forceinline__ void reset(uint32_t xb) {
#pragma unroll
        for (int q = 0; q < Q; ++q) R[q] = kNeg2;
        xE = kNeg2;
        xB = xb;
    }

    // One residue row: Alg. 2 lines 13-23 (MSV) / Alg. 7 lines 12-20 (SSV).
    __device__ __forceinline__ void row(const uint32_t *T, uint32_t x, bool gstart) {
        const uint32_t *t = T + x * (uint32_t)(Q * G);
        uint32_t c[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) c[q] = t[q * G];
        uint32_t gam = shift_in<G>(R[Q - 1], gstart);
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            uint32_t old = R[q];
            uint32_t v = MSV ? pk_adds(pk_max(gam, xB), c[q]) : pk_adds(gam, c[q]);
            R[q] = v;
            xE = pk_max(xE, v);
            gam = old;
        }
    }
};

template <int G, int Q, bool MSV>
__global__ void __launch_bounds__(512)
filter_kernel(KArgs a) {
    extern __shared__ uint32_t lds[];
    constexpr int QG = Q * G;

    // Stage the profile: lds[(x*Q + q)*G + j] = cells (q + 2jQ, q + (2j+1)Q).
    for (int idx = threadIdx.x; idx < kRows * QG; idx += blockDim.x) {
        int jj = idx % G;
        int qq = (idx / G) % Q;
        int x = idx / QG;
        int k0 = qq + Q * (2 * jj);
        uint32_t lo = (uint32_t)table_value<MSV>(a, x, k0) & 0xffffu;
        uint32_t hi = (uint32_t)table_value<MSV>(a, x, k0 + Q) & 0xffffu;
        lds[idx] = lo | (hi << 16);
    }
    __syncthreads();

    const int lane = threadIdx.x & 63;
    const int j = lane % G;
    const bool gstart = (j == 0);
    const uint32_t *T = lds + j;
    const int dbias = a.dbias;

    Lane<G, Q, MSV> st;
    uint32_t off = a.pad_off;
    int rows_left = 0x7fffffff;
    uint32_t id = 0;
    int tjbm = 0;
    int built = -(1 << 30);
    bool ovf = false;
    bool active = false;
    bool need = true;   // group wants a sequence

    for (;;) {
        // ---- hand sequences to groups that need one (uniform) ----------
        if (__any(need)) {
            unsigned long long m = __ballot(need && gstart);
            int cnt = __popcll(m);
            int first = __ffsll((long long)m) - 1;
            uint32_t b = 0;
            if (lane == first) b = atomicAdd(a.counter, (uint32_t)cnt);
            b = (uint32_t)__shfl((int)b, first);
            int rank = __popcll(m & ((1ull << lane) - 1ull));
            int s = (int)b + rank;
            s = __shfl(s, lane - j);
            if (need) {
                if (s < a.nseq) {
                    SeqRec r = a.seqs[s];
                    off = r.off;
                    rows_left = (int)r.rows;
                    id = r.id;
                    tjbm = (int)r.tjb + a.tbm;
                    active = true;
                } else {
                    off = a.pad_off;
                    rows_left = 0x7fffffff;
                    active = false;
                }
                int xb0 = kBase - tjbm;
                xb0 = xb0 < 0 ? 0 : xb0;
                st.reset(splat16(xb0 - 32768));
                built = -(1 << 30);
                ovf = false;
                need = false;
            }
        }
        if (!__any(active)) break;

        // ---- one tile of rows ------------------------------------------
        uint32_t ckR[MSV ? Q : 1];
        uint32_t ckE = st.xE;
        const uint32_t ck_off = off;
        if constexpr (MSV) {
#pragma unroll
            for (int q = 0; q < Q; ++q) ckR[q] = st.R[q];
        }
        const uint32_t step = active ? 4u : 0u;
        int nb = 0;
        bool ended = false;
        uint32_t w = *(const uint32_t *)(a.res + off);
        do {
            uint32_t wn = *(const uint32_t *)(a.res + off + step);   // prefetch
            st.row(T, w & 0xffu, gstart);
            st.row(T, (w >> 8) & 0xffu, gstart);
            st.row(T, (w >> 16) & 0xffu, gstart);
            st.row(T, w >> 24, gstart);
            off += step;
            rows_left -= (int)step;
            ++nb;
            ended = active && rows_left == 0;
            w = wn;
        } while (nb < a.tile_blocks && !__any(ended));

        if constexpr (MSV) {
            // ---- special states: did scB move in this tile? -------------
            int mx = group_max<G>(lane_max(st.xE)) + 32768;
            int lim = built > kBase + kTec ? built : kBase + kTec;
            bool trig = active && !ovf && (mx > lim || mx >= 255 - dbias);
            if (__any(trig)) {
#pragma unroll
                for (int q = 0; q < Q; ++q) st.R[q] = ckR[q];
                st.xE = ckE;
                uint32_t o = ck_off;
                for (int b = 0; b < nb; ++b) {
                    uint32_t ww = *(const uint32_t *)(a.res + o);
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        st.row(T, (ww >> (8 * r)) & 0xffu, gstart);
                        int m2 = group_max<G>(lane_max(st.xE)) + 32768;
                        if (m2 >= 255 - dbias) ovf = true;
                        int j2 = m2 - kTec > kBase ? m2 - kTec : kBase;
                        int xb = j2 - tjbm;
                        xb = xb < 0 ? 0 : (xb > 255 ? 255 : xb);
                        st.xB = splat16(xb - 32768);
                        built = m2;
                    }
                    o += step;
                }
            }
        }

        // ---- finished sequences: record scores (Alg. 2 lines 27-31) -----
        if (__any(ended)) {
            int mx = group_max<G>(lane_max(st.xE));
            if (ended && gstart) {
                uint8_t sc, fl;
                if constexpr (MSV) {
                    int cm = mx + 32768;
                    bool of = ovf || cm >= 255 - dbias;
                    int v = cm - kTec;
                    sc = of ? 255 : (uint8_t)(v < 0 ? 0 : v);
                    fl = of ? 1 : 0;
                } else {
                    int cm = mx + 32640;
                    bool of = cm >= 127;
                    sc = of ? (uint8_t)127 : (uint8_t)(int8_t)cm;
                    fl = of ? 1 : 0;
                }
                a.score[id] = sc;
                a.flag[id] = fl;
            }
            need = ended;
        }
    }
}

template <int G, int Q, bool MSV>
hipError_t launch_filter(const KArgs &a, int wpb, int blocks, hipStream_t s) {
    size_t lds = lds_bytes(G, Q);
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void *)filter_kernel<G, Q, MSV>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((filter_kernel<G, Q, MSV>), dim3(blocks), dim3(wpb * 64), lds, s, a);
    return hipGetLastError();
}

template <int G, int Q, bool MSV>
int occupancy_filter(int wpb) {
    int nb = 0;
    size_t lds = lds_bytes(G, Q);
    if (hipFuncSetAttribute((const void *)filter_kernel<G, Q, MSV>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
        return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, filter_kernel<G, Q, MSV>, wpb * 64, lds)
        != hipSuccess)
        return 0;
    return nb;
}

}  // namespace hmsv

