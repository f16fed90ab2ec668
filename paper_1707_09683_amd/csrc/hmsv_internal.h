// Internal declarations shared by the host side of the library and the
// kernel translation units.  Not part of the public ABI.
#pragma once
#include <stdint.h>
#include <stddef.h>
#include <hip/hip_runtime.h>

namespace hmsv {

// Table rows staged in LDS: the 20 amino acids plus one non-scoring row.
// The database packer maps every code 20..31 to 20.
constexpr int kRows = 21;
// With the degenerate residue codes 21..26 (B, J, Z, U, O, X) the images
// hold rows 0..26; a database without them needs only the first 21.
constexpr int kDegenRows = 27;
constexpr uint8_t kInvalidCode = 20;
constexpr int kLdsBytes = 160 * 1024;

// One database sequence in processing order (longest first).
struct SeqRec {
    uint32_t off;       // byte offset of its first residue (16-byte aligned)
    uint32_t rt;        // rows | tjb << 24: rows to run (length rounded up to a
                        // multiple of 4, at least 4, below kRowsLimit) and the
                        // length-model cost tjb(L) of its true length (< 256)
    uint32_t id;        // index in the caller's original order; for a
                        // segment of a split sequence, kSegBit | its
                        // index among the call's segments
    uint32_t len;       // its length in residues (database records; a
                        // segment's record holds its first four residues)
    uint32_t first16[4];  // its first sixteen residues
};
static_assert(sizeof(SeqRec) == 32, "records are two 16-byte loads");
constexpr uint32_t kRowsMask = 0xffffffu;
constexpr uint32_t kRowsLimit = 0xffffffu;    // rows must stay below
constexpr uint32_t kSegBit = 0x80000000u;     // record is a segment (ids stay below 2^31)

// Split sequences.  A call may cut its longest sequences into segments of
// seg_rows rows, each preceded by `warm` rows of the sequence (warm >= M - 1)
// so that every cell of the segment's own rows is exact: a cell depends only
// on the M rows above it along its diagonal.  Segment records live in the
// workspace, with four words per segment {its maximum, its split sequence,
// MSV: offset of its first loud step, MSV: offset of its last loud step}
// (a loud step holds a cell above the level where scB would rise), and
// each split sequence has a slot of kSlotWords words: {segments, -,
// original id, record, -, first segment, -, -}.  The segments store their
// results and a small kernel combines them after the filter kernel (for
// MSV it also decides whether the sequence needs an exact rescoring).
constexpr int kMaxSegs = 1 << 17;     // segment records per call
constexpr int kMaxSplit = 1 << 16;    // split sequences per call
constexpr int kMaxBins = 32;          // distinct segment counts per call
constexpr int kSlotWords = 8;

struct KArgs {
    const uint8_t *cost;   // [32][M] MSV costs (device)
    const int8_t *sc;      // [32][M] SSV scores (device)
    int32_t M;
    int32_t dbias;
    int32_t tbm;
    const uint8_t *res;    // packed residues
    const SeqRec *seqs;    // already offset to the first record of the range
    int32_t nseq;          // records in the range
    uint32_t pad_off;      // offset of >= 16 non-scoring residues
    uint8_t *score;
    uint8_t *flag;
    uint32_t *counter;     // work-queue head, zeroed by the prep kernel
    uint32_t *image;       // LDS image of the profile (workspace), 16-byte aligned
    int32_t *best;         // MSV: per table row, max over nodes of dbias - cost (workspace)
    int32_t rows;          // table rows of the LDS images: kRows or kDegenRows
    // split sequences: records [0, nsplit) of the range are replaced by
    // nsegs segment records (workspace), processed first
    SeqRec *segs;          // [kMaxSegs] segment records (workspace)
    uint32_t *slots;       // [kMaxSplit][kSlotWords] per split sequence (workspace)
    uint32_t *segx;        // [kMaxSegs][4] per segment (workspace), 16-byte aligned
    // MSV exact pass: windows {start, rows | tjb << 24, original id, -} of
    // the sequences it rescores, by original index
    uint4 *win;            // [database nseq] (workspace)
    uint32_t *ximage;      // its LDS image of the profile (workspace)
    int32_t qx;            // its registers per lane (64-lane groups)
    int32_t nsplit;
    int32_t nsegs;
    int32_t seg_rows;      // rows per segment (multiple of 16)
    int32_t warm;          // rows before a segment (multiple of 16, >= M - 1)
    // Split sequence t has v = ceil(rows / seg_rows) segments, which take
    // records p .. p + v - 1.  Records are longest first, so v only falls
    // with t: bin b covers t >= bin_t[b] with v = bin_v[b] and
    // p = bin_p[b] + (t - bin_t[b]) * v.
    int32_t nbins;
    int32_t bin_t[kMaxBins];
    int32_t bin_p[kMaxBins];
    int32_t bin_v[kMaxBins];
};

// Workspace layout: queue counters (bytes 0..63), the MSV per-residue best
// scores (bytes 64..147), the profile's LDS image from byte 256, then the
// segment records, the split-sequence slots, the MSV exact pass's LDS
// image and a 16-byte window record per sequence of the database (by
// original index).
constexpr size_t kWsCounterBytes = 256;
constexpr size_t kWsSegOff = kWsCounterBytes + 160 * 1024;
constexpr size_t kWsSlotOff = kWsSegOff + (size_t)kMaxSegs * sizeof(SeqRec);
constexpr size_t kWsSegxOff = kWsSlotOff + (size_t)kMaxSplit * kSlotWords * 4;
constexpr size_t kWsXImageOff = kWsSegxOff + (size_t)kMaxSegs * 16;
static_assert(kWsSegxOff % 16 == 0, "segment words are read as uint4");
constexpr size_t kWsWinOff = kWsXImageOff + 160 * 1024;
constexpr size_t ws_bytes(int64_t nseq) { return kWsWinOff + 16 * (size_t)(nseq > 1 ? nseq : 1); }

typedef hipError_t (*LaunchFn)(const KArgs &, int waves_per_block, int blocks,
                               hipStream_t);
typedef hipError_t (*ExactLaunchFn)(const KArgs &, int cus, hipStream_t);
typedef int (*OccupancyFn)(int waves_per_block, int rows);

struct KernelEntry {
    int is_msv;
    int G;
    int Q;
    LaunchFn launch;
    OccupancyFn occupancy;
};

// P7Viterbi's LDS image rows: 21 (or 27, with the degenerate codes) of
// match emissions (residue rows, row 20 = -inf), then 7 of transitions (see
// P7Args).  The chunk layout is chosen for kP7Rows rows.
constexpr int kP7EmisRows = kRows;
constexpr int kP7Rows = kRows + 7;

// The profile's LDS image: kRows table rows of RS dwords.  A lane reads its
// Q score pairs in chunks of 4 dwords (ds_read_b128), then a 2-dword and/or
// a 1-dword tail; a partial last chunk is instead read whole (its unused
// dwords are padding) when the padded table still fits, so one LDS address
// per row serves every read.  gfx950's LDS serves 256 bytes (64 banks) per
// pass, so a read of w dwords per lane is served 64/w lanes at a time: the
// groups of G lanes that share a pass read different table rows, and to
// keep them on disjoint banks a chunk of width w is stored
// copies(w) = max(1, 64/(G w)) times side by side, group g reading copy
// g % copies(w).  A group of 16 or more lanes fills a pass by itself.
// Dwords of the row: NF chunk regions of CW, then the tails at OFF2, OFF1.
struct LdsLayout {
    int NF;      // 4-dword chunks (the last one partial if WIDE)
    int R;       // tail dwords after them (0..3)
    bool WIDE;   // partial last chunk read whole
    int CW;      // dwords of one chunk region (all copies)
    int OFF2;    // the 2-dword tail region
    int OFF1;    // the 1-dword tail region
    int RS;      // dwords per table row
};

constexpr int lds_copies(int G, int w) { return 64 / (G * w) > 1 ? 64 / (G * w) : 1; }

constexpr LdsLayout lds_layout(int G, int Q, int rows = kRows) {
    LdsLayout L{};
    L.CW = lds_copies(G, 4) * G * 4;
    int nf = Q / 4, r = Q % 4;
    L.WIDE = r != 0 && (size_t)rows * (size_t)(nf + 1) * (size_t)L.CW * 4 <= kLdsBytes;
    L.NF = L.WIDE ? nf + 1 : nf;
    L.R = L.WIDE ? 0 : r;
    L.OFF2 = L.NF * L.CW;
    L.OFF1 = L.OFF2 + ((L.R & 2) ? lds_copies(G, 2) * G * 2 : 0);
    L.RS = L.OFF1 + ((L.R & 1) ? lds_copies(G, 1) * G : 0);
    return L;
}

// LDS bytes of an image of `rows` table rows (the chunk layout is the one
// chosen for kRows, or kP7Rows, rows).
inline size_t lds_bytes(int G, int Q, int rows = kRows) {
    return (size_t)rows * lds_layout(G, Q).RS * 4;
}
inline size_t p7_lds_bytes(int G, int Q, int rows = kRows) {
    return (size_t)(rows + 7) * lds_layout(G, Q, kP7Rows).RS * 4;
}

// A group of G lanes with Q registers covers nodes 1..2GQ-1 (slot 0 is a
// dummy -inf node).
inline int64_t plan_nodes(int G, int Q) { return (int64_t)2 * G * Q - 1; }

// ---- P7Viterbi (gapped Plan-7 Viterbi) -------------------------------------
// The transition rows of the LDS image, each laid out as the MSV/SSV image
// (lds_layout with kP7Rows rows): slot s holds the transition used by node
// s's cells, so the ones into node s from node s-1 are stored shifted by
// one slot.
enum P7TransRow : int { kP7MMp = 0, kP7IMp, kP7DMp, kP7MI, kP7II, kP7MDp, kP7DDp };

struct P7Args {
    const int16_t *msc;    // [32][M] match emission scores (device)
    const int16_t *trans;  // [7][M] MM, MI, MD, IM, II, DM, DD out of each node (device)
    int32_t M;
    int32_t tbm;           // B->M_k
    const uint8_t *res;    // packed residues
    const SeqRec *seqs;    // records in processing order
    const uint32_t *lenmodel;  // per record: loop (low 16 bits) | move << 16 (int16 each)
    int32_t nseq;
    uint32_t pad_off;
    int16_t *score;
    uint8_t *flag;
    uint32_t *image;       // the LDS image (workspace)
    int32_t *aux;          // workspace word: max over nodes of D->M (prep kernel)
    uint32_t *queue;       // kP7Parts record queues, 128 bytes apart (zeroed by the
                           // prep kernel)
    int32_t rows;          // emission rows (kRows or kDegenRows); the 7
                           // transition rows follow them
    const int32_t *sel;    // NULL: records 0..nseq-1; else the processing-order
    const int32_t *nsel;   // positions sel[0 .. *nsel) (device), longest first
};

// Survivor selection (select.hip): positions (processing order) of the
// records whose score reaches thr or whose flag is set, into pos[0 ..
// *count); scratch: select_scratch_bytes(nseq) bytes of device memory.
size_t select_scratch_bytes(int64_t nseq);
hipError_t launch_select(const SeqRec *seqs, int64_t nseq, const void *score,
                         const uint8_t *flags, int is_msv, int32_t thr, int32_t *pos,
                         int32_t *count, int32_t *scratch, hipStream_t s);

constexpr int kMaxP7G = 64;
constexpr int kP7Parts = 16;                 // record queues of a P7 call
// P7 calls' workspace: aux word at 0, the queues from kWsCounterBytes, the
// LDS image after them (P7 uses none of the MSV/SSV regions).
constexpr size_t kWsP7QueueOff = kWsCounterBytes;
constexpr size_t kWsP7ImageOff = kWsP7QueueOff + (size_t)kP7Parts * 128;
static_assert(kWsP7ImageOff + 160 * 1024 <= kWsWinOff, "P7 image within the workspace");
typedef hipError_t (*P7LaunchFn)(const P7Args &, int waves_per_block, int blocks, hipStream_t);
struct P7KernelEntry {
    int G;
    int Q;
    P7LaunchFn launch;
    OccupancyFn occupancy;
};
int register_p7_kernels(const P7KernelEntry *entries, int n);

// Each kernel translation unit registers its instantiations at load time.
int register_kernels(const KernelEntry *entries, int n);

// The MSV exact pass runs one window per wavefront as a single 64-lane
// group with the fewest registers that hold the profile: one kernel per
// register count qx = 1..kMaxExactQ.
constexpr int kExactG = 64;
constexpr int kMaxExactQ = 30;
inline int exact_q(int M) { return (M + 1 + 2 * kExactG - 1) / (2 * kExactG); }
int register_exact(int qx, ExactLaunchFn fn);


}  // namespace hmsv
