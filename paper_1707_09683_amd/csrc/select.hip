// Survivor selection between pipeline stages: the processing-order
// positions of the sequences whose filter score reaches a threshold (or
// that overflowed), longest first, compacted on the device so that the
// next stage (P7Viterbi) runs on them without a host round trip.
//
// Three launches over blocks of 1024 positions: count the survivors of each
// block, scan the counts (one block), write each block's survivors at its
// offset in position order.
#include "hmsv_internal.h"

namespace hmsv {
namespace {

constexpr int kSelBlock = 1024;

__device__ __forceinline__ bool survives(const SeqRec *seqs, int64_t p, int64_t nseq,
                                         const void *score, const uint8_t *flags, int is_msv,
                                         int32_t thr) {
    if (p >= nseq) return false;
    const uint32_t id = seqs[p].id;
    const int s = is_msv ? (int)((const uint8_t *)score)[id] : (int)((const int8_t *)score)[id];
    return flags[id] != 0 || s >= thr;
}

__global__ void __launch_bounds__(kSelBlock)
select_count_kernel(const SeqRec *seqs, int64_t nseq, const void *score, const uint8_t *flags,
                    int is_msv, int32_t thr, int32_t *counts) {
    const int64_t p = (int64_t)blockIdx.x * kSelBlock + threadIdx.x;
    const int n = __syncthreads_count(survives(seqs, p, nseq, score, flags, is_msv, thr));
    if (threadIdx.x == 0) counts[blockIdx.x] = n;
}

// Exclusive scan of nb block counts into offsets (in place), total into
// *count.  One block of 1024 threads, in chunks of 1024 with a carry.
__global__ void __launch_bounds__(kSelBlock)
select_scan_kernel(int32_t *counts, int32_t nb, int32_t *count) {
    __shared__ int32_t buf[kSelBlock];
    __shared__ int32_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int32_t base = 0; base < nb; base += kSelBlock) {
        const int32_t i = base + (int32_t)threadIdx.x;
        const int32_t v = i < nb ? counts[i] : 0;
        buf[threadIdx.x] = v;
        __syncthreads();
        // Hillis-Steele inclusive scan within the chunk
        for (int o = 1; o < kSelBlock; o <<= 1) {
            const int32_t add = (int)threadIdx.x >= o ? buf[threadIdx.x - o] : 0;
            __syncthreads();
            buf[threadIdx.x] += add;
            __syncthreads();
        }
        if (i < nb) counts[i] = carry + buf[threadIdx.x] - v;
        __syncthreads();
        if (threadIdx.x == kSelBlock - 1) carry += buf[kSelBlock - 1];
        __syncthreads();
    }
    if (threadIdx.x == 0) *count = carry;
}

__global__ void __launch_bounds__(kSelBlock)
select_write_kernel(const SeqRec *seqs, int64_t nseq, const void *score, const uint8_t *flags,
                    int is_msv, int32_t thr, const int32_t *offsets, int32_t *pos) {
    __shared__ int32_t wave_base[kSelBlock / 64];
    const int64_t p = (int64_t)blockIdx.x * kSelBlock + threadIdx.x;
    const bool s = survives(seqs, p, nseq, score, flags, is_msv, thr);
    const unsigned long long m = __ballot(s);
    const int lane = (int)(threadIdx.x & 63), wave = (int)(threadIdx.x >> 6);
    if (lane == 0) wave_base[wave] = __popcll(m);
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t acc = 0;
        for (int w = 0; w < kSelBlock / 64; ++w) {
            const int32_t c = wave_base[w];
            wave_base[w] = acc;
            acc += c;
        }
    }
    __syncthreads();
    if (s) {
        const int rank = __popcll(m & ((1ull << lane) - 1ull));
        pos[offsets[blockIdx.x] + wave_base[wave] + rank] = (int32_t)p;
    }
}

}  // namespace

size_t select_scratch_bytes(int64_t nseq) {
    return sizeof(int32_t) * (size_t)((nseq + kSelBlock - 1) / kSelBlock + 1);
}

hipError_t launch_select(const SeqRec *seqs, int64_t nseq, const void *score,
                         const uint8_t *flags, int is_msv, int32_t thr, int32_t *pos,
                         int32_t *count, int32_t *scratch, hipStream_t s) {
    const int64_t nb = (nseq + kSelBlock - 1) / kSelBlock;
    if (nb == 0) {
        hipLaunchKernelGGL(select_scan_kernel, dim3(1), dim3(kSelBlock), 0, s, scratch, 0, count);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(select_count_kernel, dim3((unsigned)nb), dim3(kSelBlock), 0, s, seqs, nseq,
                       score, flags, is_msv, thr, scratch);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(select_scan_kernel, dim3(1), dim3(kSelBlock), 0, s, scratch, (int32_t)nb,
                       count);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(select_write_kernel, dim3((unsigned)nb), dim3(kSelBlock), 0, s, seqs, nseq,
                       score, flags, is_msv, thr, scratch, pos);
    return hipGetLastError();
}

}  // namespace hmsv
