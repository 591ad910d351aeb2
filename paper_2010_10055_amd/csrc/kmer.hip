// A from the reads (Sec. IV-C; Alg. diBELLA 2D, KmerCounter and GenerateA):
// every window of k bases of every read is a k-mer, counted under its
// canonical form (the smaller 2-bit code of the k-mer and of its reverse
// complement; bases A0 C1 G2 T3, the first base most significant); k-mers
// whose count over all windows lies in [lo, hi] are reliable and, in
// increasing code order, are A's columns; A_ic is the smallest position of
// k-mer c in read i, or (position << 1) | strand (1: the read holds the
// canonical k-mer reverse complemented).
//
// On the device, with no hashing: every window's canonical code is sorted
// (stable LSD radix sort, 8-bit digits, keys and window numbers), so equal
// k-mers form runs in window order; a run's length is its frequency (read
// from its first element, at most hi + 1 steps), reliable runs are numbered
// by a scan, and the first element of each read within a reliable run
// (stable order: the read's smallest position) becomes an entry
// (read, column, value).  A second stable radix sort by read turns the
// entries, which are in column order, into A's rows with their columns in
// order.  Two host synchronisations: the window count (to size the sort)
// and the reliable k-mers and entries (to size A).
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
// in which every wave ranks its lanes among equal digits with 8 ballots,
// waves follow each other through LDS counters, and each element goes to
// its digit's running slot: ranks follow input order inside a tile and
// tiles follow input order, so every pass is stable.
// ---------------------------------------------------------------------------
constexpr int kSortBlock = 256;
constexpr int kSortItems = 16;
constexpr int kTile = kSortBlock * kSortItems;

template <class K>
__global__ __launch_bounds__(kSortBlock) void k_km_upsweep(const K* __restrict__ keys, int64_t n, int shift,
                                                           int64_t ntiles, int32_t* __restrict__ counts) {
    __shared__ int32_t hist[256];
    hist[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kTile;
    for (int q = 0; q < kSortItems; ++q) {
        const int64_t e = base + (int64_t)q * kSortBlock + threadIdx.x;
        if (e < n) atomicAdd(&hist[(uint32_t)(keys[e] >> shift) & 255u], 1);
    }
    __syncthreads();
    counts[(int64_t)threadIdx.x * ntiles + blockIdx.x] = hist[threadIdx.x];
}

template <class K, class V>
__global__ __launch_bounds__(kSortBlock) void k_km_downsweep(const K* __restrict__ kin, const V* __restrict__ vin,
                                                             int64_t n, int shift, int64_t ntiles,
                                                             const int64_t* __restrict__ offsets,
                                                             K* __restrict__ kout, V* __restrict__ vout) {
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
    K keyr[kSortItems];
    V valr[kSortItems];
#pragma unroll
    for (int sub = 0; sub < kSortItems; ++sub) {
        const int64_t e = min(base + (int64_t)sub * kSortBlock + tid, n - 1);   // clamped: no branch per load
        keyr[sub] = kin[e];
        valr[sub] = vin[e];
    }
#pragma unroll
    for (int sub = 0; sub < kSortItems; ++sub) {
        const bool valid = base + (int64_t)sub * kSortBlock + tid < n;
        const int d = (int)((uint32_t)(keyr[sub] >> shift) & 255u);
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
            kout[pos] = keyr[sub];
            vout[pos] = valr[sub];
        }
    }
}

// Sorts (ka, va) by the low `bits` bits of the keys with (kb, vb) as the
// other buffer; *in_b = 1 if the result ended in (kb, vb).
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
    K *kin = ka, *kout = kb;
    V *vin = va, *vout = vb;
    int tok = -1;
    DB_TRY(timing_begin(kPhKmerSort, st, &tok));
    for (int p = 0; p < passes; ++p) {
        hipLaunchKernelGGL(k_km_upsweep<K>, dim3((unsigned)ntiles), dim3(kSortBlock), 0, st, kin, n, 8 * p, ntiles,
                           counts);
        DB_HIP(hipGetLastError());
        DB_TRY(scan_exclusive_ws(counts, offsets, 256 * ntiles, nullptr, scan_ws, st));
        hipLaunchKernelGGL((k_km_downsweep<K, V>), dim3((unsigned)ntiles), dim3(kSortBlock), 0, st, kin, vin, n,
                           8 * p, ntiles, offsets, kout, vout);
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

// Every window of read i at woff[i] + p: its canonical code, its number and
// its strand bit (one bit per window, set with the wave's ballot).  One
// wave per read; lane l takes positions l, l + 64, ...: the k base loads of
// the wave read one contiguous run of bytes each.
template <int WPB>
__global__ __launch_bounds__(WPB* kWave) void k_km_windows(const uint8_t* __restrict__ bases,
                                                           const int64_t* __restrict__ off,
                                                           const int64_t* __restrict__ woff, int64_t n, int32_t k,
                                                           uint64_t* __restrict__ keys, uint32_t* __restrict__ wid,
                                                           uint32_t* __restrict__ sbits, int32_t* __restrict__ flags) {
    const int lane = lane_id();
    int32_t bad = 0;
    for (int64_t i = (int64_t)blockIdx.x * WPB + __builtin_amdgcn_readfirstlane(wave_id()); i < n;
         i += (int64_t)gridDim.x * WPB) {
        const int64_t lo = off[i], base = woff[i], nw = woff[i + 1] - base;
        for (int64_t p0 = 0; p0 < nw; p0 += kWave) {
            const int64_t p = p0 + lane;
            const bool valid = p < nw;
            uint64_t fwd = 0, rc = 0;
            if (valid) {
                for (int q = 0; q < k; ++q) {
                    uint32_t b = bases[lo + p + q];
                    bad |= b > 3u ? kKmBadBase : 0;
                    b &= 3u;
                    fwd = (fwd << 2) | b;
                    rc |= (uint64_t)(3u - b) << (2 * q);
                }
                keys[base + p] = rc < fwd ? rc : fwd;
                wid[base + p] = (uint32_t)(base + p);
            }
            const uint64_t mask = __ballot(valid && rc < fwd);
            // bits of windows base + p0 .. + 63, spread over up to three words
            const int64_t w0 = base + p0;
            const int sh = (int)(w0 & 31);
            const int64_t word = w0 >> 5;
            if (lane < 3 && mask) {
                uint32_t part;
                if (lane == 0) part = (uint32_t)(mask << sh);
                else if (lane == 1) part = sh ? (uint32_t)(mask >> (32 - sh)) : (uint32_t)(mask >> 32);
                else part = sh ? (uint32_t)(mask >> (64 - sh)) : 0u;
                if (part) atomicOr(&sbits[word + lane], part);
            }
        }
    }
    bad = wave_or_i32(bad);
    if (lane == 0 && bad) atomicOr(flags, bad);
}

// ---------------------------------------------------------------------------
// Runs of equal k-mers
// ---------------------------------------------------------------------------
// The first element h <= e of e's run, or -1 when the run holds more than
// hi elements before e (then it is not reliable).
__device__ __forceinline__ int64_t run_head(const uint64_t* keys, int64_t e, int32_t hi) {
    const uint64_t c = keys[e];
    int64_t h = e;
    for (int32_t s = 0; h > 0 && keys[h - 1] == c; ++s) {
        if (s >= hi) return -1;
        --h;
    }
    return h;
}

// rel[e] = 1 where e starts a run of length in [lo, hi] (the length read at
// most hi + 1 elements far).
__global__ void k_km_runs(const uint64_t* __restrict__ keys, int64_t W, int32_t lo, int32_t hi,
                          int32_t* __restrict__ rel) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < W; e += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t c = keys[e];
        int32_t r = 0;
        if (e == 0 || keys[e - 1] != c) {
            int64_t len = 1;
            while (len <= hi && e + len < W && keys[e + len] == c) ++len;
            r = (len >= lo && len <= hi) ? 1 : 0;
        }
        rel[e] = r;
    }
}

// The read of window w: the last i with woff[i] <= w (woff[n] = W > w).
__device__ __forceinline__ int64_t read_of(const int64_t* woff, int64_t n, int64_t w) {
    int64_t a = 0, b = n;   // woff[a] <= w < woff[b]
    while (b - a > 1) {
        const int64_t m = (a + b) >> 1;
        if (woff[m] <= w) a = m;
        else b = m;
    }
    return a;
}

// keep[e] = 1 for the first element of each read inside a reliable run
// (the run is in window order: the element before e, if in the run, has a
// smaller window, of the same read iff it is not before the read's first).
__global__ void k_km_keep(const uint64_t* __restrict__ keys, const uint32_t* __restrict__ wid, int64_t W,
                          const int64_t* __restrict__ woff, int64_t n, int32_t hi, const int32_t* __restrict__ rel,
                          int32_t* __restrict__ keep) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < W; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t h = run_head(keys, e, hi);
        int32_t k = 0;
        if (h >= 0 && rel[h]) k = (h == e || (int64_t)wid[e - 1] < woff[read_of(woff, n, wid[e])]) ? 1 : 0;
        keep[e] = k;
    }
}

// The kept elements as A entries in (column, read) order: key = read,
// value = (column << 32) | (position, or (position << 1) | strand).
__global__ void k_km_emit(const uint64_t* __restrict__ keys, const uint32_t* __restrict__ wid, int64_t W,
                          const int64_t* __restrict__ woff, int64_t n, int32_t hi, const int64_t* __restrict__ colof,
                          const int32_t* __restrict__ keep, const int64_t* __restrict__ kpos,
                          const uint32_t* __restrict__ sbits, int strand_bit, uint32_t* __restrict__ rkey,
                          uint64_t* __restrict__ rval) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < W; e += (int64_t)gridDim.x * blockDim.x) {
        if (!keep[e]) continue;
        const int64_t h = run_head(keys, e, hi);   // >= 0: kept elements lie in reliable runs
        const int64_t w = wid[e];
        const int64_t r = read_of(woff, n, w);
        const int64_t pos = w - woff[r];
        const uint32_t strand = (sbits[w >> 5] >> (w & 31)) & 1u;
        const uint32_t v = strand_bit ? (uint32_t)((pos << 1) | strand) : (uint32_t)pos;
        const int64_t o = kpos[e];
        rkey[o] = (uint32_t)r;
        rval[o] = ((uint64_t)(uint32_t)colof[h] << 32) | v;
    }
}

// codes[column] = the reliable run's k-mer.
__global__ void k_km_codes(const uint64_t* __restrict__ keys, int64_t W, const int32_t* __restrict__ rel,
                           const int64_t* __restrict__ colof, uint64_t* __restrict__ codes) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < W; e += (int64_t)gridDim.x * blockDim.x)
        if (rel[e]) codes[colof[e]] = keys[e];
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
        uint32_t *wid[2], *sbits;
        int32_t *rel, *keep;
        int64_t *colof, *kpos;
        DB_TRY(wk.work_n(std::max<int64_t>(W, 1), &keys[0]));
        DB_TRY(wk.work_n(std::max<int64_t>(W, 1), &keys[1]));
        DB_TRY(wk.work_n(std::max<int64_t>(W, 1), &wid[0]));
        DB_TRY(wk.work_n(std::max<int64_t>(W, 1), &wid[1]));
        DB_TRY(wk.work_n(ceil_div(W, 32) + 3, &sbits));
        DB_TRY(fill_i32(reinterpret_cast<int32_t*>(sbits), 0, ceil_div(W, 32) + 3, st));
        constexpr int WPB = 4;
        DB_TRY(timing_begin(kPhKmerWindows, st, &tok));
        if (n > 0 && W > 0) {
            hipLaunchKernelGGL(k_km_windows<WPB>, dim3(grid_for(n, WPB, 1 << 16)), dim3(WPB * kWave), 0, st, bases,
                               offsets, woff, n, k, keys[0], wid[0], sbits, d_flags);
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
        const int grid = grid_for(W, 256, 1 << 16);
        DB_TRY(timing_begin(kPhKmerRuns, st, &tok));
        if (W > 0) {
            hipLaunchKernelGGL(k_km_runs, dim3(grid), dim3(256), 0, st, sk, W, lo, hi, rel);
            DB_HIP(hipGetLastError());
        }
        DB_TRY(scan_exclusive(rel, colof, W, nullptr, wk));
        if (W > 0) {
            hipLaunchKernelGGL(k_km_keep, dim3(grid), dim3(256), 0, st, sk, sw, W, woff, n, hi, rel, keep);
            DB_HIP(hipGetLastError());
        }
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
        DB_TRY(timing_begin(kPhKmerRuns, st, &tok));
        if (W > 0) {
            hipLaunchKernelGGL(k_km_codes, dim3(grid), dim3(256), 0, st, sk, W, rel, colof, codes);
            hipLaunchKernelGGL(k_km_emit, dim3(grid), dim3(256), 0, st, sk, sw, W, woff, n, hi, colof, keep, kpos,
                               sbits, strand_bit, rkey[0], rval[0]);
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
