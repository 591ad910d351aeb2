// Stable device-wide LSD radix sort of (uint32 key, uint64 value) pairs,
// 8-bit digits.  Each pass:
//   upsweep    per tile of kTile keys, a 256-bin LDS histogram of the digit,
//              stored digit-major: counts[d * ntiles + tile];
//   scan       exclusive scan of counts -> first output slot of (d, tile);
//   downsweep  per tile, sub-tiles of 256 elements in order: every wave
//              ranks its lanes among equal digits with 8 ballots, waves are
//              ordered through LDS counters, and each element goes to
//              slot(d, tile) + running count of d in the tile.
// Ranks follow input order inside a tile and tiles follow input order, so
// every pass is stable and the whole sort is an LSD sort.
#include "common.hpp"

namespace dibella {

constexpr int kSortBlock = 256;
constexpr int kSortItems = 16;
constexpr int kTile = kSortBlock * kSortItems;

__global__ __launch_bounds__(kSortBlock) void k_rs_upsweep(const uint32_t* __restrict__ keys, int64_t n, int shift,
                                                           int64_t ntiles, int32_t* __restrict__ counts) {
    __shared__ int32_t hist[256];
    hist[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kTile;
    for (int q = 0; q < kSortItems; ++q) {
        const int64_t e = base + (int64_t)q * kSortBlock + threadIdx.x;
        if (e < n) atomicAdd(&hist[(keys[e] >> shift) & 255u], 1);
    }
    __syncthreads();
    counts[(int64_t)threadIdx.x * ntiles + blockIdx.x] = hist[threadIdx.x];
}

__global__ __launch_bounds__(kSortBlock) void k_rs_downsweep(const uint32_t* __restrict__ kin,
                                                             const uint64_t* __restrict__ vin, int64_t n, int shift,
                                                             int64_t ntiles, const int64_t* __restrict__ offsets,
                                                             uint32_t* __restrict__ kout, uint64_t* __restrict__ vout) {
    constexpr int W = kSortBlock / kWave;
    __shared__ int64_t run[256];
    __shared__ int32_t wcnt[W][256];
    __shared__ int64_t wpre[W][256];
    const int tid = threadIdx.x, w = wave_id();
    run[tid] = offsets[(int64_t)tid * ntiles + blockIdx.x];
    for (int q = 0; q < W; ++q) wcnt[q][tid] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kTile;
    // all loads of the tile are issued before any ranking work
    uint32_t keyr[kSortItems];
    uint64_t valr[kSortItems];
#pragma unroll
    for (int sub = 0; sub < kSortItems; ++sub) {
        const int64_t e = base + (int64_t)sub * kSortBlock + tid;
        keyr[sub] = e < n ? kin[e] : 0u;
        valr[sub] = e < n ? vin[e] : 0ull;
    }
#pragma unroll
    for (int sub = 0; sub < kSortItems; ++sub) {
        const int64_t e = base + (int64_t)sub * kSortBlock + tid;
        const bool valid = e < n;
        const uint32_t key = keyr[sub];
        const uint64_t val = valr[sub];
        const int d = (int)((key >> shift) & 255u);
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1;
            const uint64_t bal = __ballot(valid && bit);
            peers &= bit ? bal : ~bal;
        }
        const int rank = __popcll(peers & lanemask_lt());
        if (valid && rank == 0) wcnt[w][d] = __popcll(peers);
        __syncthreads();
        {
            int64_t acc = run[tid];
            for (int q = 0; q < W; ++q) {
                wpre[q][tid] = acc;
                acc += wcnt[q][tid];
                wcnt[q][tid] = 0;
            }
            run[tid] = acc;
        }
        __syncthreads();
        if (valid) {
            const int64_t pos = wpre[w][d] + rank;
            kout[pos] = key;
            vout[pos] = val;
        }
    }
}

int64_t radix_sort_workspace_words(int64_t n) {
    if (n <= 0) return 0;
    const int64_t ntiles = ceil_div(n, kTile);
    return 256 * ntiles;
}

// Sorts (ka, va) by the low `bits` bits of the keys using (kb, vb) as the
// other buffer.  *in_b = 1 if the result ended in (kb, vb).
int radix_sort_pairs(uint32_t* ka, uint64_t* va, uint32_t* kb, uint64_t* vb, int64_t n, int bits, int* in_b,
                     Arena& ar) {
    *in_b = 0;
    if (n <= 1 || bits <= 0) return DIBELLA_OK;
    hipStream_t st = ar.stream();
    const int64_t ntiles = ceil_div(n, kTile);
    int32_t* counts;
    int64_t* offsets;
    DB_TRY(ar.work_n(256 * ntiles, &counts));
    DB_TRY(ar.work_n(256 * ntiles + 1, &offsets));
    int64_t* scan_tiles;
    DB_TRY(ar.work_n(scan_workspace_elems(256 * ntiles), &scan_tiles));
    const int passes = (bits + 7) / 8;
    uint32_t *kin = ka, *kout = kb;
    uint64_t *vin = va, *vout = vb;
    for (int p = 0; p < passes; ++p) {
        int tok = -1;
        DB_TRY(timing_begin(kPhSortUp, st, &tok));
        hipLaunchKernelGGL(k_rs_upsweep, dim3((unsigned)ntiles), dim3(kSortBlock), 0, st, kin, n, 8 * p, ntiles,
                           counts);
        DB_HIP(hipGetLastError());
        DB_TRY(timing_end(tok, st));
        DB_TRY(scan_exclusive_ws(counts, offsets, 256 * ntiles, nullptr, scan_tiles, st));
        DB_TRY(timing_begin(kPhSortDown, st, &tok));
        hipLaunchKernelGGL(k_rs_downsweep, dim3((unsigned)ntiles), dim3(kSortBlock), 0, st, kin, vin, n, 8 * p,
                           ntiles, offsets, kout, vout);
        DB_HIP(hipGetLastError());
        DB_TRY(timing_end(tok, st));
        uint32_t* tk = kin; kin = kout; kout = tk;
        uint64_t* tv = vin; vin = vout; vout = tv;
    }
    *in_b = (passes & 1) ? 1 : 0;
    return DIBELLA_OK;
}

}  // namespace dibella
