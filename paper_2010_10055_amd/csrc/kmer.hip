// A from the reads (Sec. IV-C; Alg. diBELLA 2D, KmerCounter and GenerateA):
// every window of k bases of every read is a k-mer, counted under its
// canonical form (the smaller 2-bit code of the k-mer and of its reverse
// complement; bases A0 C1 G2 T3, the first base most significant); k-mers
// whose count over all windows lies in [lo, hi] are reliable and are A's
// columns in the order of their first occurrence (the first read holding
// the k-mer, then its smallest position there: the k-mers of one read get
// consecutive columns, so that the rows of A^T one read's walk visits lie
// side by side); A_ic is the smallest position of k-mer c in read i, or
// (position << 1) | strand (1: the read holds the canonical k-mer reverse
// complemented).
//
// On the device, with no hashing: every window's canonical code is sorted
// (stable LSD radix sort, 8-bit digits, keys and window numbers), so equal
// k-mers form runs in window order; a run's length is its frequency (read
// from its first element, at most hi + 1 steps) and its first element is
// the k-mer's first occurrence.  A reliable run marks its first window in a
// bitmap over the windows; a column is the number of marked windows before
// the run's first one (a popcount prefix), so columns follow first
// occurrence.  The first element of each read within a reliable run
// (stable order: the read's smallest position) becomes an entry
// (read, column, value), placed in column order by a scan of the columns'
// entry counts.  A second stable radix sort by read turns the entries into
// A's rows with their columns in order.  Two host synchronisations: the
// window count (to size the sort) and the reliable k-mers and entries (to
// size A).
#include "common.hpp"

#include <cstring>
#include <utility>

namespace dibella {

enum : int32_t {
    kKmBadOffsets = 1,
    kKmBadBase = 2,
};

// ---------------------------------------------------------------------------
// Stable device-wide LSD radix sort of (key, value) pairs, 8-bit digits.
// Per pass: an upsweep histogram per tile of kTile keys (digit-major
// counts[d * ntiles + tile]), an exclusive scan over them, and a downsweep
// in which every wave ranks its lanes among equal digits of its 64
// elements with 8 ballots, the counts of the tile's 64 groups of 64 are
// scanned per digit in LDS (one thread per digit), each element's slot in
// the tile (its digit's first slot, plus the digit's elements in the groups
// before its own, plus its rank) places it in LDS in digit order, and the
// tile is written out from there so that each digit's run of the tile
// lands in consecutive places: ranks follow input order inside a tile and
// tiles follow input order, so every pass is stable.
// ---------------------------------------------------------------------------
constexpr int kSortBlock = 256;
constexpr int kSortItems = 16;
constexpr int kTile = kSortBlock * kSortItems;

template <class K>
__global__ __launch_bounds__(kSortBlock) void k_km_upsweep(const K* __restrict__ keys, int64_t n, K kmask, int shift,
                                                           int64_t ntiles, int32_t* __restrict__ counts) {
    __shared__ int32_t hist[256];
    hist[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kTile;
    for (int q = 0; q < kSortItems; ++q) {
        const int64_t e = base + (int64_t)q * kSortBlock + threadIdx.x;
        if (e < n) atomicAdd(&hist[(uint32_t)((keys[e] & kmask) >> shift) & 255u], 1);
    }
    __syncthreads();
    counts[(int64_t)threadIdx.x * ntiles + blockIdx.x] = hist[threadIdx.x];
}

template <class K, class V>
__global__ __launch_bounds__(kSortBlock) void k_km_downsweep(const K* __restrict__ kin, const V* __restrict__ vin,
                                                             int64_t n, K kmask, int shift, int64_t ntiles,
                                                             const int64_t* __restrict__ offsets,
                                                             K* __restrict__ kout, V* __restrict__ vout) {
    constexpr int W = kSortBlock / kWave;
    constexpr int G = kSortItems * W;   // (sub-tile, wave) groups of 64 elements, in element order
    constexpr size_t kCnt = sizeof(uint16_t) * G * 256;
    constexpr size_t kStage = (sizeof(K) + sizeof(V)) * kTile;
    // cnt[g][d] (elements of digit d in group g, then the digit's elements
    // in the groups before g; a digit's column is scanned by one thread)
    // and, once every element knows its slot, the tile in digit order
    __shared__ __align__(16) unsigned char smem[kCnt > kStage ? kCnt : kStage];
    __shared__ int64_t run[256];
    __shared__ int32_t tstart[256];
    __shared__ int32_t s_tmp[kSortBlock / kWave + 1];
    uint16_t(*cnt)[256] = reinterpret_cast<uint16_t(*)[256]>(smem);
    K* skey = reinterpret_cast<K*>(smem);
    V* sval = reinterpret_cast<V*>(smem + sizeof(K) * kTile);
    const int tid = threadIdx.x, w = wave_id();
    run[tid] = offsets[(int64_t)tid * ntiles + blockIdx.x];
    for (int g = 0; g < G; ++g) cnt[g][tid] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kTile;
    const int tn = (int)min<int64_t>(kTile, n - base);   // elements of this tile
    K keyr[kSortItems];
    V valr[kSortItems];
#pragma unroll
    for (int sub = 0; sub < kSortItems; ++sub) {
        const int64_t e = min(base + (int64_t)sub * kSortBlock + tid, n - 1);   // clamped: no branch per load
        keyr[sub] = kin[e];
        valr[sub] = vin[e];
    }
    // rank of each element among the equal digits of its wave and sub-tile
    // (8 ballots); the group's count per digit goes to LDS from its first lane
    uint32_t slot[kSortItems];   // first rank << 8 | digit, then the slot in the tile
#pragma unroll
    for (int sub = 0; sub < kSortItems; ++sub) {
        const bool valid = sub * kSortBlock + tid < tn;
        const int d = (int)((uint32_t)((keyr[sub] & kmask) >> shift) & 255u);
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1;
            const uint64_t bal = __ballot(valid && bit);
            peers &= bit ? bal : ~bal;
        }
        const int rank = __popcll(peers & lanemask_lt());
        if (valid && rank == 0) cnt[sub * W + w][d] = (uint16_t)__popcll(peers);
        slot[sub] = ((uint32_t)rank << 8) | (uint32_t)d;
    }
    __syncthreads();
    // digit tid: its count in each group becomes its elements before it;
    // the digits' totals give their first slots in the tile
    int32_t total = 0;
    for (int g = 0; g < G; ++g) {
        const int32_t c = cnt[g][tid];
        cnt[g][tid] = (uint16_t)total;
        total += c;
    }
    int32_t all;
    const int32_t first = block_exclusive_sum<kSortBlock>(total, s_tmp, &all);
    tstart[tid] = first;
    __syncthreads();
#pragma unroll
    for (int sub = 0; sub < kSortItems; ++sub) {
        const int d = (int)(slot[sub] & 255u);
        slot[sub] = (uint32_t)(tstart[d] + cnt[sub * W + w][d]) + (slot[sub] >> 8);
    }
    __syncthreads();   // cnt is overwritten by the staged tile from here on
#pragma unroll
    for (int sub = 0; sub < kSortItems; ++sub) {
        if (sub * kSortBlock + tid < tn) {
            skey[slot[sub]] = keyr[sub];
            sval[slot[sub]] = valr[sub];
        }
    }
    __syncthreads();
    // the tile in digit order: consecutive slots of a digit go to
    // consecutive places of its output run
    for (int q = tid; q < tn; q += kSortBlock) {
        const K key = skey[q];
        const int d = (int)((uint32_t)((key & kmask) >> shift) & 255u);
        const int64_t pos = run[d] + (q - tstart[d]);
        kout[pos] = key;
        vout[pos] = sval[q];
    }
}

// Sorts (ka, va) by the low `bits` bits of the keys (bits above them are
// carried along, not sorted by) with (kb, vb) as the other buffer; *in_b = 1
// if the result ended in (kb, vb).
template <class K, class V>
static int radix_sort(K* ka, V* va, K* kb, V* vb, int64_t n, int bits, int* in_b, Arena& ar) {
    *in_b = 0;
    if (n <= 1 || bits <= 0) return DIBELLA_OK;
    hipStream_t st = ar.stream();
    const int64_t ntiles = ceil_div(n, kTile);
    int32_t* counts;
    int64_t* offsets;
    int64_t* scan_ws;
    DB_TRY(ar.work_n(256 * ntiles, &counts));
    DB_TRY(ar.work_n(256 * ntiles + 1, &offsets));
    DB_TRY(ar.work_n(scan_workspace_elems(256 * ntiles), &scan_ws));
    const int passes = (bits + 7) / 8;
    const K kmask = bits >= (int)(8 * sizeof(K)) ? ~K(0) : (K(1) << bits) - 1;
    K *kin = ka, *kout = kb;
    V *vin = va, *vout = vb;
    int tok = -1;
    DB_TRY(timing_begin(kPhKmerSort, st, &tok));
    for (int p = 0; p < passes; ++p) {
        hipLaunchKernelGGL(k_km_upsweep<K>, dim3((unsigned)ntiles), dim3(kSortBlock), 0, st, kin, n, kmask, 8 * p,
                           ntiles, counts);
        DB_HIP(hipGetLastError());
        DB_TRY(scan_exclusive_ws(counts, offsets, 256 * ntiles, nullptr, scan_ws, st));
        hipLaunchKernelGGL((k_km_downsweep<K, V>), dim3((unsigned)ntiles), dim3(kSortBlock), 0, st, kin, vin, n,
                           kmask, 8 * p, ntiles, offsets, kout, vout);
        DB_HIP(hipGetLastError());
        std::swap(kin, kout);
        std::swap(vin, vout);
    }
    DB_TRY(timing_end(tok, st));
    *in_b = (passes & 1) ? 1 : 0;
    return DIBELLA_OK;
}

// ---------------------------------------------------------------------------
// Windows
// ---------------------------------------------------------------------------
// Windows per read (and the check of the read offsets).
__global__ void k_km_count(const int64_t* __restrict__ off, int64_t n, int64_t nbases, int32_t k,
                           int64_t* __restrict__ wc, int32_t* __restrict__ flags) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t lo = off[i], hi = off[i + 1];
        const bool bad = (i == 0 && lo != 0) || (i == n - 1 && hi != nbases) || lo < 0 || hi < lo || hi > nbases;
        const int64_t L = bad ? 0 : hi - lo;
        wc[i] = L >= k ? L - k + 1 : 0;
        if (bad) atomicOr(flags, kKmBadOffsets);
    }
}

// A window's sort key: its canonical code in the low 2k bits and its strand
// in bit 63 (the sort reads only the low 2k bits, so the strand rides along).
constexpr int kStrandBit = 63;

// Every window of read i at woff[i] + p: key (canonical code, strand) and
// its number.  One wave per read, in chunks of 64 * kWinPer windows: the
// chunk's bases are staged in LDS with coalesced loads, each lane rolls the
// codes of kWinPer consecutive windows (one new base per window), the keys
// are staged in LDS and written out coalesced.
constexpr int kWinPer = 8;
constexpr int kWinChunk = kWave * kWinPer;
// LDS written by some lanes of a wave and read by others: order the
// accesses of the wave (its waves never wait for each other here, so a
// workgroup barrier is not an option).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
template <int WPB>
__global__ __launch_bounds__(WPB* kWave) void k_km_windows(const uint8_t* __restrict__ bases,
                                                           const int64_t* __restrict__ off,
                                                           const int64_t* __restrict__ woff, int64_t n, int32_t k,
                                                           uint64_t* __restrict__ keys, uint32_t* __restrict__ wid,
                                                           int32_t* __restrict__ flags) {
    __shared__ uint8_t s_base[WPB][kWinChunk + 32];
    __shared__ uint64_t s_key[WPB][kWinChunk];
    const int lane = lane_id(), wv = wave_id();
    const uint64_t mask = (k == 32) ? ~0ull : ((1ull << (2 * k)) - 1);
    int32_t bad = 0;
    for (int64_t i = (int64_t)blockIdx.x * WPB + __builtin_amdgcn_readfirstlane(wv); i < n;
         i += (int64_t)gridDim.x * WPB) {
        const int64_t lo = off[i], base = woff[i], nw = woff[i + 1] - base;
        for (int64_t p0 = 0; p0 < nw; p0 += kWinChunk) {
            const int cw = (int)min<int64_t>(kWinChunk, nw - p0);   // windows of this chunk
            const int cb = cw + k - 1;                              // their bases
            // all the chunk's base loads in flight before any is used
            constexpr int kLoads = (kWinChunk + 31 + kWave - 1) / kWave;
            uint32_t bv[kLoads];
#pragma unroll
            for (int it = 0; it < kLoads; ++it) {
                const int q = lane + it * kWave;
                bv[it] = bases[lo + p0 + min(q, cb - 1)];   // clamped: no branch per load
            }
#pragma unroll
            for (int it = 0; it < kLoads; ++it) {
                const int q = lane + it * kWave;
                if (q < cb) {
                    bad |= bv[it] > 3u ? kKmBadBase : 0;
                    s_base[wv][q] = (uint8_t)(bv[it] & 3u);
                }
            }
            wave_lds_sync();
            const int j0 = lane * kWinPer;
            if (j0 < cw) {
                uint64_t fwd = 0, rc = 0;
                for (int q = 0; q < k - 1; ++q) {
                    const uint32_t b = s_base[wv][j0 + q];
                    fwd = (fwd << 2) | b;
                    rc = (rc >> 2) | ((uint64_t)(3u - b) << (2 * (k - 1)));
                }
                for (int j = j0; j < j0 + kWinPer && j < cw; ++j) {
                    const uint32_t b = s_base[wv][j + k - 1];
                    fwd = ((fwd << 2) | b) & mask;
                    rc = (rc >> 2) | ((uint64_t)(3u - b) << (2 * (k - 1)));
                    s_key[wv][j] = rc < fwd ? (rc | (1ull << kStrandBit)) : fwd;
                }
            }
            wave_lds_sync();
            for (int q = lane; q < cw; q += kWave) {
                keys[base + p0 + q] = s_key[wv][q];
                wid[base + p0 + q] = (uint32_t)(base + p0 + q);
            }
            wave_lds_sync();
        }
    }
    bad = wave_or_i32(bad);
    if (lane == 0 && bad) atomicOr(flags, bad);
}

// ---------------------------------------------------------------------------
// Runs of equal k-mers
// ---------------------------------------------------------------------------
// The read of window w (the last i with woff[i] <= w; woff[n] = W > w):
// rtab[w >> kRtabShift] is the read holding window (w >> kRtabShift) <<
// kRtabShift, and the reads from there on are stepped through (two loads
// for reads longer than 2^kRtabShift windows, instead of a binary search of
// some 18 dependent loads).
constexpr int kRtabShift = 12;
__device__ __forceinline__ int64_t read_of(const uint32_t* rtab, const int64_t* woff, int64_t w) {
    int64_t r = rtab[w >> kRtabShift];
    while (woff[r + 1] <= w) ++r;
    return r;
}

// rtab[b] = the read holding window b << kRtabShift, for every b below
// ceil(W / 2^kRtabShift): each read writes the b whose window it holds.
__global__ void k_km_rtab(const int64_t* __restrict__ woff, int64_t n, uint32_t* __restrict__ rtab) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t a = woff[i], z = woff[i + 1];
        for (int64_t b = (a + (int64_t(1) << kRtabShift) - 1) >> kRtabShift; (b << kRtabShift) < z; ++b)
            rtab[b] = (uint32_t)i;
    }
}

// The first element h <= e of e's run (equal codes under `mask`), or -1
// when the run holds more than hi elements before e (then it is not
// reliable).
__device__ __forceinline__ int64_t run_head(const uint64_t* keys, uint64_t mask, int64_t e, int32_t hi) {
    const uint64_t c = keys[e] & mask;
    int64_t h = e;
    for (int32_t s = 0; h > 0 && (keys[h - 1] & mask) == c; ++s) {
        if (s >= hi) return -1;
        --h;
    }
    return h;
}

// rel[e] = 1 where e starts a run (equal codes under `mask`) of length in
// [lo, hi] (the length read at most hi + 1 elements far); such a run's
// first window (its k-mer's first occurrence) is marked in `first`, one bit
// per window.
__global__ void k_km_runs(const uint64_t* __restrict__ keys, const uint32_t* __restrict__ wid, int64_t W,
                          uint64_t mask, int32_t lo, int32_t hi, int32_t* __restrict__ rel,
                          uint32_t* __restrict__ first) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < W; e += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t c = keys[e] & mask;
        int32_t r = 0;
        if (e == 0 || (keys[e - 1] & mask) != c) {
            int64_t len = 1;
            while (len <= hi && e + len < W && (keys[e + len] & mask) == c) ++len;
            r = (len >= lo && len <= hi) ? 1 : 0;
            if (r) {
                const uint32_t w = wid[e];
                atomicOr(&first[w >> 5], 1u << (w & 31));
            }
        }
        rel[e] = r;
    }
}

// Marked windows per 32-bit word of the bitmap.
__global__ void k_km_popc(const uint32_t* __restrict__ first, int64_t nwords, int32_t* __restrict__ cnt) {
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nwords;
         q += (int64_t)gridDim.x * blockDim.x)
        cnt[q] = __popc(first[q]);
}

// For every reliable run (first element h): its column, the marked windows
// before its first window (wbase: the words' exclusive scan), kept in
// colof[h]; and its entry count (its kept elements, from the scan kpos of
// the keep flags) in ccount[column].
__global__ void k_km_columns(const uint64_t* __restrict__ keys, const uint32_t* __restrict__ wid, int64_t W,
                             uint64_t mask, int32_t hi, const int32_t* __restrict__ rel,
                             const uint32_t* __restrict__ first, const int64_t* __restrict__ wbase,
                             const int64_t* __restrict__ kpos, int64_t* __restrict__ colof,
                             int32_t* __restrict__ ccount) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < W; e += (int64_t)gridDim.x * blockDim.x) {
        if (!rel[e]) continue;
        const uint64_t c = keys[e] & mask;
        int64_t len = 1;
        while (len <= hi && e + len < W && (keys[e + len] & mask) == c) ++len;
        const uint32_t w = wid[e];
        const int64_t col = wbase[w >> 5] + __popc(first[w >> 5] & ((1u << (w & 31)) - 1u));
        colof[e] = col;
        ccount[col] = (int32_t)(kpos[e + len] - kpos[e]);
    }
}

// keep[e] = 1 for the first element of each read inside a reliable run (the
// run is in window order: an element is its read's first in the run iff
// the element before it holds a window of an earlier read); rd[e] = the
// read of every element of a reliable run.
__global__ void k_km_keep(const uint64_t* __restrict__ keys, const uint32_t* __restrict__ wid, int64_t W,
                          uint64_t mask, const uint32_t* __restrict__ rtab, const int64_t* __restrict__ woff,
                          int32_t hi, const int32_t* __restrict__ rel, int32_t* __restrict__ keep,
                          uint32_t* __restrict__ rd) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < W; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t h = run_head(keys, mask, e, hi);
        int32_t k = 0;
        if (h >= 0 && rel[h]) {
            const int64_t r = read_of(rtab, woff, wid[e]);
            k = (h == e || (int64_t)wid[e - 1] < woff[r]) ? 1 : 0;
            rd[e] = (uint32_t)r;
        }
        keep[e] = k;
    }
}

// The kept elements as A entries in (column, read) order: key = read,
// value = (column << 32) | (position, or (position << 1) | strand), at the
// column's first slot (cstart) plus the element's rank among its run's kept
// elements; a reliable run's first element also writes the run's k-mer to
// codes.
__global__ void k_km_emit(const uint64_t* __restrict__ keys, const uint32_t* __restrict__ wid, int64_t W,
                          uint64_t mask, const uint32_t* __restrict__ rd, const int64_t* __restrict__ woff,
                          int32_t hi, const int64_t* __restrict__ colof, const int64_t* __restrict__ cstart,
                          const int32_t* __restrict__ keep, const int64_t* __restrict__ kpos, int strand_bit,
                          uint32_t* __restrict__ rkey, uint64_t* __restrict__ rval, uint64_t* __restrict__ codes) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < W; e += (int64_t)gridDim.x * blockDim.x) {
        if (!keep[e]) continue;
        const int64_t h = run_head(keys, mask, e, hi);   // >= 0: kept elements lie in reliable runs
        const uint64_t key = keys[e];
        const int64_t col = colof[h];
        if (h == e) codes[col] = key & mask;
        const int64_t w = wid[e];
        const int64_t r = rd[e];
        const int64_t pos = w - woff[r];
        const uint32_t strand = (uint32_t)(key >> kStrandBit);
        const uint32_t v = strand_bit ? (uint32_t)((pos << 1) | strand) : (uint32_t)pos;
        const int64_t o = cstart[col] + (kpos[e] - kpos[h]);
        rkey[o] = (uint32_t)r;
        rval[o] = ((uint64_t)(uint32_t)col << 32) | v;
    }
}

// A's row pointers from the entries sorted by read: rowptr[r] = the first
// entry of a read >= r.
__global__ void k_km_rowptr(const uint32_t* __restrict__ rkey, int64_t nnz, int64_t n, int64_t* __restrict__ rowptr) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e <= nnz;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r0 = e == 0 ? 0 : (int64_t)rkey[e - 1] + 1;
        const int64_t r1 = e == nnz ? n : (int64_t)rkey[e];
        for (int64_t r = r0; r <= r1; ++r) rowptr[r] = e;
    }
}

__global__ void k_km_split(const uint64_t* __restrict__ rval, int64_t nnz, int32_t* __restrict__ col,
                           int32_t* __restrict__ val) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t x = rval[e];
        col[e] = (int32_t)(x >> 32);
        val[e] = (int32_t)(uint32_t)x;
    }
}

static const char* describe_km_bad(int32_t bad) {
    if (bad & kKmBadOffsets) return "read offsets are not a valid offset array over the bases";
    if (bad & kKmBadBase) return "a base is outside 0..3";
    return "malformed input";
}

int kmer_matrix_run(const uint8_t* bases, const int64_t* offsets, int64_t n, int64_t nbases, int32_t k, int32_t lo,
                    int32_t hi, uint32_t flags, dibella_csr_out* A, uint64_t** codes_out, int64_t* m_out,
                    Arena& ar) {
    hipStream_t st = ar.stream();
    std::memset(A, 0, sizeof(*A));
    *codes_out = nullptr;
    *m_out = 0;
    if (n < 0 || nbases < 0 || k < 1 || k > 31 || lo < 1 || hi < lo) {
        set_error("dibella_kmer_matrix: sizes must be non-negative, k in [1, 31], 1 <= lo <= hi");
        return DIBELLA_EINVAL;
    }
    if (n >= (int64_t(1) << 31)) {
        set_error("dibella_kmer_matrix: reads must be < 2^31");
        return DIBELLA_EOVERFLOW;
    }
    if ((n > 0 && !offsets) || (nbases > 0 && !bases)) {
        set_error("dibella_kmer_matrix: null pointer");
        return DIBELLA_EINVAL;
    }
    const int strand_bit = (flags & DIBELLA_KMER_STRAND) ? 1 : 0;
    A->nrows = n;
    int32_t* d_flags;
    int64_t *wc, *woff;
    DB_TRY(ar.work_n(1, &d_flags));
    DB_TRY(ar.work_n(std::max<int64_t>(n, 1), &wc));
    DB_TRY(ar.work_n(n + 1, &woff));
    DB_TRY(fill_i32(d_flags, 0, 1, st));
    int tok = -1;
    DB_TRY(timing_begin(kPhKmerWindows, st, &tok));
    if (n > 0) {
        hipLaunchKernelGGL(k_km_count, dim3(grid_for(n, 256, 4096)), dim3(256), 0, st, offsets, n, nbases, k, wc,
                           d_flags);
        DB_HIP(hipGetLastError());
    }
    DB_TRY(timing_end(tok, st));
    DB_TRY(scan_exclusive(wc, woff, n, nullptr, ar));
    // ---- sync 1: the window count, the offsets' check
    HostStage& hst = host_stage();
    DB_TRY(hst.reserve(64));
    int64_t* h = static_cast<int64_t*>(hst.ptr);
    DB_HIP(hipMemcpyAsync(h, woff + n, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    DB_HIP(hipMemcpyAsync(h + 1, d_flags, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    DB_TRY(sync_stream(st));
    const int64_t W = h[0];
    const int32_t bad0 = *reinterpret_cast<int32_t*>(h + 1);
    DB_TRY(stage_done(st));
    if (bad0) {
        set_error(std::string("dibella_kmer_matrix: ") + describe_km_bad(bad0));
        return DIBELLA_EINVAL;
    }
    if (W >= (int64_t(1) << 32)) {
        set_error("dibella_kmer_matrix: 2^32 or more windows");
        return DIBELLA_EOVERFLOW;
    }
    // ---- windows, sort by k-mer, runs, kept elements (released before the
    // second sort)
    uint32_t* rkey[2] = {nullptr, nullptr};
    uint64_t* rval[2] = {nullptr, nullptr};
    int64_t m = 0, nnz = 0;
    uint64_t* codes = nullptr;
    {
        Arena wk(ar.alloc_fn(), ar.free_fn(), ar.alloc_ctx(), st);
        uint64_t *keys[2];
        uint32_t *wid[2], *rtab;
        int32_t *rel, *keep;
        int64_t *colof, *kpos;
        DB_TRY(wk.work_n(std::max<int64_t>(W, 1), &keys[0]));
        DB_TRY(wk.work_n(std::max<int64_t>(W, 1), &keys[1]));
        DB_TRY(wk.work_n(std::max<int64_t>(W, 1), &wid[0]));
        DB_TRY(wk.work_n(std::max<int64_t>(W, 1), &wid[1]));
        DB_TRY(wk.work_n(ceil_div(W, int64_t(1) << kRtabShift) + 1, &rtab));
        if (n > 0 && W > 0) {
            hipLaunchKernelGGL(k_km_rtab, dim3(grid_for(n, 256, 4096)), dim3(256), 0, st, woff, n, rtab);
            DB_HIP(hipGetLastError());
        }
        constexpr int WPB = 4;
        DB_TRY(timing_begin(kPhKmerWindows, st, &tok));
        if (n > 0 && W > 0) {
            hipLaunchKernelGGL(k_km_windows<WPB>, dim3(grid_for(n, WPB, 1 << 16)), dim3(WPB * kWave), 0, st, bases,
                               offsets, woff, n, k, keys[0], wid[0], d_flags);
            DB_HIP(hipGetLastError());
        }
        DB_TRY(timing_end(tok, st));
        int in_b = 0;
        DB_TRY(radix_sort(keys[0], wid[0], keys[1], wid[1], W, 2 * k, &in_b, wk));
        const uint64_t* sk = keys[in_b];
        const uint32_t* sw = wid[in_b];
        DB_TRY(wk.work_n(std::max<int64_t>(W, 1), &rel));
        DB_TRY(wk.work_n(W + 1, &colof));
        DB_TRY(wk.work_n(std::max<int64_t>(W, 1), &keep));
        DB_TRY(wk.work_n(W + 1, &kpos));
        // one bit per window: the first windows of the reliable k-mers
        const int64_t nwords = ceil_div(std::max<int64_t>(W, 1), int64_t(32));
        uint32_t* first;
        DB_TRY(wk.work_n(nwords, &first));
        DB_TRY(fill_i32(reinterpret_cast<int32_t*>(first), 0, nwords, st));
        const int grid = grid_for(W, 256, 1 << 16);
        const uint64_t cmask = (1ull << (2 * k)) - 1;   // k <= 31: the code bits
        uint32_t* rd;
        DB_TRY(wk.work_n(std::max<int64_t>(W, 1), &rd));
        DB_TRY(timing_begin(kPhKmerRuns, st, &tok));
        if (W > 0) {
            hipLaunchKernelGGL(k_km_runs, dim3(grid), dim3(256), 0, st, sk, sw, W, cmask, lo, hi, rel, first);
            hipLaunchKernelGGL(k_km_keep, dim3(grid), dim3(256), 0, st, sk, sw, W, cmask, rtab, woff, hi, rel, keep,
                               rd);
            DB_HIP(hipGetLastError());
        }
        DB_TRY(scan_exclusive(rel, colof, W, nullptr, wk));
        DB_TRY(scan_exclusive(keep, kpos, W, nullptr, wk));
        DB_TRY(timing_end(tok, st));
        // ---- sync 2: k-mers, entries, the bases' check
        DB_TRY(hst.reserve(64));
        int64_t* h2 = static_cast<int64_t*>(hst.ptr);
        DB_HIP(hipMemcpyAsync(h2, colof + W, sizeof(int64_t), hipMemcpyDeviceToHost, st));
        DB_HIP(hipMemcpyAsync(h2 + 1, kpos + W, sizeof(int64_t), hipMemcpyDeviceToHost, st));
        DB_HIP(hipMemcpyAsync(h2 + 2, d_flags, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        DB_TRY(sync_stream(st));
        m = h2[0];
        nnz = h2[1];
        const int32_t bad = *reinterpret_cast<int32_t*>(h2 + 2);
        DB_TRY(stage_done(st));
        if (bad) {
            set_error(std::string("dibella_kmer_matrix: ") + describe_km_bad(bad));
            return DIBELLA_EINVAL;
        }
        if (m >= (int64_t(1) << 31)) {
            set_error("dibella_kmer_matrix: 2^31 or more reliable k-mers");
            return DIBELLA_EOVERFLOW;
        }
        DB_TRY(ar.output_n(m, &codes));
        DB_TRY(ar.work_n(std::max<int64_t>(nnz, 1), &rkey[0]));
        DB_TRY(ar.work_n(std::max<int64_t>(nnz, 1), &rkey[1]));
        DB_TRY(ar.work_n(std::max<int64_t>(nnz, 1), &rval[0]));
        DB_TRY(ar.work_n(std::max<int64_t>(nnz, 1), &rval[1]));
        // columns by first occurrence, and each column's first entry slot
        int32_t *wcnt, *ccount;
        int64_t *wbase, *cstart;
        DB_TRY(wk.work_n(nwords, &wcnt));
        DB_TRY(wk.work_n(nwords + 1, &wbase));
        DB_TRY(wk.work_n(std::max<int64_t>(m, 1), &ccount));
        DB_TRY(wk.work_n(m + 1, &cstart));
        DB_TRY(timing_begin(kPhKmerRuns, st, &tok));
        if (W > 0) {
            hipLaunchKernelGGL(k_km_popc, dim3(grid_for(nwords, 256, 1 << 16)), dim3(256), 0, st, first, nwords,
                               wcnt);
            DB_HIP(hipGetLastError());
        }
        DB_TRY(scan_exclusive(wcnt, wbase, nwords, nullptr, wk));
        if (W > 0) {
            hipLaunchKernelGGL(k_km_columns, dim3(grid), dim3(256), 0, st, sk, sw, W, cmask, hi, rel, first, wbase,
                               kpos, colof, ccount);
            DB_HIP(hipGetLastError());
        }
        DB_TRY(scan_exclusive(ccount, cstart, m, nullptr, wk));
        if (W > 0) {
            hipLaunchKernelGGL(k_km_emit, dim3(grid), dim3(256), 0, st, sk, sw, W, cmask, rd, woff, hi, colof, cstart,
                               keep, kpos, strand_bit, rkey[0], rval[0], codes);
            DB_HIP(hipGetLastError());
        }
        DB_TRY(timing_end(tok, st));
    }
    // ---- entries by read (stable: columns stay in order inside a row)
    int in_b = 0;
    DB_TRY(radix_sort(rkey[0], rval[0], rkey[1], rval[1], nnz, std::max(1, ceil_log2_i64(std::max<int64_t>(n, 2))),
                      &in_b, ar));
    int64_t* rowptr;
    int32_t *col, *val;
    DB_TRY(ar.output_n(n + 1, &rowptr));
    DB_TRY(ar.output_n(nnz, &col));
    DB_TRY(ar.output_n(nnz, &val));
    DB_TRY(timing_begin(kPhKmerRows, st, &tok));
    hipLaunchKernelGGL(k_km_rowptr, dim3(grid_for(nnz + 1, 256, 1 << 16)), dim3(256), 0, st, rkey[in_b], nnz, n,
                       rowptr);
    DB_HIP(hipGetLastError());
    if (nnz > 0) {
        hipLaunchKernelGGL(k_km_split, dim3(grid_for(nnz, 256, 1 << 16)), dim3(256), 0, st, rval[in_b], nnz, col,
                           val);
        DB_HIP(hipGetLastError());
    }
    DB_TRY(timing_end(tok, st));
    A->nrows = n;
    A->ncols = m;
    A->nnz = nnz;
    A->rowptr = rowptr;
    A->col = col;
    A->val = val;
    *codes_out = codes;
    *m_out = m;
    return DIBELLA_OK;
}

}  // namespace dibella
