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
//  * Cells hold u/1024 in fp16, where u is the 8-bit filter value (MSV v,
//    SSV d + 128).  Every value is a multiple of 2^-10 below 1, so fp16 adds
//    and maxima are exact, the clamp modifier's floor at 0.0 is the 8-bit
//    floor (-inf), and its cap at 1.0 is never reached before the overflow
//    row.  A cell update is then
//      MSV  v = clamp(max(gamma, scB) + (dbias - cost)/1024)   (Alg. 2 cell update)
//      SSV  v = clamp(gamma + sc/1024)                          (Alg. 7 cell update)
//    and scE = max(scE, v, v') takes two cells per v_pk_maximum3_f16
//    (a running max, never reset per row).  The 255 (MSV) / 127 (SSV) caps
//    are not applied; overflow is flagged from the running max instead,
//    which is exact because no cap can fire before the first overflow row.
//  * Per-node scores of the 21 table rows live in LDS as fp16 pairs, laid
//    out [row][chunk][lane][W] so each lane reads W consecutive dwords and
//    every LDS read pass (128 bytes) is served by one group's contiguous
//    block: no bank conflicts between groups reading different rows.
//  * Sequences are handed out longest first from a global counter as groups
//    finish (replaces the pre-packed warp blocks of Alg. 1).
//  * MSV special states: scB only changes when the running max exceeds
//    max(base + tec, the max it was last computed from), so rows run in
//    tiles with scB fixed; at the tile end the group max is checked and, if
//    it moved (or overflowed), the tile is replayed from a register
//    checkpoint with the per-row special-state update of Alg. 2.
#pragma once
#include "hmsv_internal.h"

namespace hmsv {

typedef _Float16 h2 __attribute__((ext_vector_type(2)));

constexpr uint32_t kMinus2 = 0xC000u;        // fp16 -2.0: score of dummy/padding slots
constexpr int kBase = 190;
constexpr int kTec = 3;

// Width in dwords of one lane's LDS read: 32 lanes x 4 bytes per pass, so a
// group of G lanes fills a pass with W = 32 / G dwords each (1 to 4).
template <int G>
constexpr int read_width() { return G >= 32 ? 1 : (G >= 16 ? 2 : 4); }

template <int G, int Q>
constexpr int padded_q() { return (Q + read_width<G>() - 1) / read_width<G>() * read_width<G>(); }

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
#pragma unroll
    for (int o = 1; o < G; o <<= 1) {
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

// fp16 pattern of the score added at slot s (node s, slot 0 = dummy) for
// table row x.
template <bool MSV>
__device__ __forceinline__ uint32_t slot_bits(const KArgs &a, int x, int s) {
    if (s < 1 || s > a.M) return kMinus2;
    int k = s - 1;
    int v = MSV ? a.dbias - (int)a.cost[x * a.M + k] : (int)a.sc[x * a.M + k];
    _Float16 h = (_Float16)((float)v * (1.0f / 1024.0f));
    return (uint32_t)__builtin_bit_cast(unsigned short, h);
}

template <int G, int Q, bool MSV>
struct Lane {
    static constexpr int W = read_width<G>();
    static constexpr int RS = padded_q<G, Q>() * G;     // dwords per table row
    uint32_t R[Q];
    uint32_t xE;
    uint32_t xB;

    __device__ __forceinline__ void reset(uint32_t xb) {
#pragma unroll
        for (int q = 0; q < Q; ++q) R[q] = 0u;
        xE = 0u;
        xB = xb;
    }

    // Score pairs of row x for this lane (T = lds + j*W).
    __device__ __forceinline__ void load_row(const uint32_t *T, uint32_t x, uint32_t (&c)[Q]) {
        const uint32_t *t = T + x * (uint32_t)RS;
#pragma unroll
        for (int ch = 0; ch * W < Q; ++ch) {
            const uint32_t *p = t + ch * G * W;
            if (ch * W + W <= Q) {
                if constexpr (W == 4) {
                    uint4 v = *(const uint4 *)p;
                    c[ch * 4 + 0] = v.x; c[ch * 4 + 1] = v.y;
                    c[ch * 4 + 2] = v.z; c[ch * 4 + 3] = v.w;
                } else if constexpr (W == 2) {
                    uint2 v = *(const uint2 *)p;
                    c[ch * 2 + 0] = v.x; c[ch * 2 + 1] = v.y;
                } else {
                    c[ch] = p[0];
                }
            } else {
                const int r = Q - ch * W;      // 1..W-1 dwords left
                if (r >= 2) {
                    uint2 v = *(const uint2 *)p;
                    c[ch * W + 0] = v.x; c[ch * W + 1] = v.y;
                    if (r == 3) c[ch * W + 2] = p[2];
                } else {
                    c[ch * W] = p[0];
                }
            }
        }
    }

    // One residue row of Alg. 2 (MSV) / Alg. 7 (SSV): shift, fetch, cell update.
    __device__ __forceinline__ void row(const uint32_t *T, uint32_t x) {
        uint32_t c[Q];
        load_row(T, x, c);
        uint32_t gam = shift_in(R[Q - 1]);
        uint32_t prev_v = 0;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            uint32_t old = R[q];
            uint32_t v = MSV ? add_clamp(hmax(gam, xB), c[q]) : add_clamp(gam, c[q]);
            R[q] = v;
            if (q & 1) xE = hmax3(xE, prev_v, v);
            else prev_v = v;
            gam = old;
        }
        if (Q & 1) xE = hmax(xE, prev_v);
    }
};

template <int G, int Q, bool MSV>
__global__ void __launch_bounds__(512)
filter_kernel(KArgs a) {
    extern __shared__ uint32_t lds[];
    using L = Lane<G, Q, MSV>;
    constexpr int W = L::W;
    constexpr int RS = L::RS;

    // Stage the profile image (built by prep_kernel) into LDS.
    {
        const uint4 *src = (const uint4 *)a.image;
        uint4 *dst = (uint4 *)lds;
        constexpr int n16 = kRows * RS / 4;
        for (int i = threadIdx.x; i < n16; i += blockDim.x) dst[i] = src[i];
    }
    __syncthreads();

    const int lane = threadIdx.x & 63;
    const int j = lane % G;
    const bool gstart = (j == 0);
    const uint32_t *T = lds + j * W;
    const int dbias = a.dbias;

    L st;
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
                st.reset(units_splat(xb0));
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
            uint32_t wn = *(const uint32_t *)(a.res + off + step);   // next 4 residues
            st.row(T, w & 0xffu);
            st.row(T, (w >> 8) & 0xffu);
            st.row(T, (w >> 16) & 0xffu);
            st.row(T, w >> 24);
            // Consume the next word only here, so its load stays issued before
            // the four rows and its latency hides behind them.
            asm volatile("" : "+v"(wn));
            off += step;
            rows_left -= (int)step;
            ++nb;
            ended = active && rows_left == 0;
            w = wn;
        } while (nb < a.tile_blocks && !__any(ended));

        if constexpr (MSV) {
            // ---- special states: did scB move in this tile? -------------
            int mx = bits_to_units(group_max<G>(lane_max_bits(st.xE)));
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
                        st.row(T, (ww >> (8 * r)) & 0xffu);
                        int m2 = bits_to_units(group_max<G>(lane_max_bits(st.xE)));
                        if (m2 >= 255 - dbias) ovf = true;
                        int j2 = m2 - kTec > kBase ? m2 - kTec : kBase;
                        int xb = j2 - tjbm;
                        xb = xb < 0 ? 0 : (xb > 255 ? 255 : xb);
                        st.xB = units_splat(xb);
                        built = m2;
                    }
                    o += step;
                }
            }
        }

        // ---- finished sequences: record scores (Alg. 2 end-residue branch) -----
        if (__any(ended)) {
            int mx = bits_to_units(group_max<G>(lane_max_bits(st.xE)));
            if (ended && gstart) {
                uint8_t sc, fl;
                if constexpr (MSV) {
                    bool of = ovf || mx >= 255 - dbias;
                    int v = mx - kTec;
                    sc = of ? 255 : (uint8_t)(v < 0 ? 0 : v);
                    fl = of ? 1 : 0;
                } else {
                    bool of = mx >= 255;
                    sc = of ? (uint8_t)127 : (uint8_t)(int8_t)(mx - 128);
                    fl = of ? 1 : 0;
                }
                a.score[id] = sc;
                a.flag[id] = fl;
            }
            need = ended;
        }
    }
}

// LDS image of the profile: dword (x, q, j) at x*RS + (q/W)*G*W + j*W + q%W
// holds slots (q + 2jQ, q + (2j+1)Q) as two fp16 scores.  Thread 0 also
// resets the work-queue counter.
template <int G, int Q, bool MSV>
__global__ void __launch_bounds__(256) prep_kernel(KArgs a) {
    constexpr int W = read_width<G>();
    constexpr int RS = padded_q<G, Q>() * G;
    int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx == 0) {
        a.counter[0] = 0u;
        a.counter[1] = 0u;
    }
    if (idx >= kRows * RS) return;
    int x = idx / RS;
    int rem = idx - x * RS;
    int ch = rem / (G * W);
    int r2 = rem - ch * G * W;
    int jj = r2 / W;
    int qq = ch * W + (r2 - jj * W);
    uint32_t v = (kMinus2 << 16) | kMinus2;
    if (qq < Q) {
        int s0 = qq + Q * (2 * jj);
        v = slot_bits<MSV>(a, x, s0) | (slot_bits<MSV>(a, x, s0 + Q) << 16);
    }
    a.image[idx] = v;
}

template <int G, int Q, bool MSV>
hipError_t launch_filter(const KArgs &a, int wpb, int blocks, hipStream_t s) {
    constexpr int n = kRows * padded_q<G, Q>() * G;
    hipLaunchKernelGGL((prep_kernel<G, Q, MSV>), dim3((n + 255) / 256), dim3(256), 0, s, a);
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
