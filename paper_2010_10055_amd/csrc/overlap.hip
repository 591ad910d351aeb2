// C = A * A^T over the overlap semiring (Sec. IV-D): for every pair of reads
// (i, j) the number of shared reliable k-mers and the position pairs of the
// two smallest shared k-mer columns.
//
// Pipeline (one launch per step for all sets of a batch):
//   validate A and lay out its (column, read|position) pairs  ->  bucketed
//   counting sort by column in two or three passes: A^T and one record per
//   column (a column of two pairs carries them)  ->  per A entry its segment word (per
//   XCD column slice), products per row, row bins  ->  symbolic  ->  bins by
//   output size  ->  scan to C's row pointers  ->  numeric.
// Symbolic and numeric walk the products of one row per workgroup:
//   * bitmap path (sets whose read count fits an LDS bitmap): the symbolic
//     phase marks every column j in 1..4 bit planes ("seen >= p times"); the
//     plane of min_shared lists the output columns already in order.  The
//     numeric phase maps a column to its output rank with a per-word
//     popcount prefix.
//   * hash path (larger sets): LDS hash tables of (j, count) in the symbolic
//     phase (compacted and bitonic-sorted to give the output columns), a
//     small LDS hash from j to output rank in the numeric phase.
//   The symbolic phase stores each row's output columns in a scratch range;
//   the numeric phase counts and keeps the two smallest-k seeds per column.
// Rows too dense for LDS go through expand-sort-compress (ESC): products are
// expanded in k-mer order, stably radix sorted by j and compressed by runs.
#include "common.hpp"

#include <algorithm>
#include <cstring>

namespace dibella {

struct OvSet {
    const int64_t* a_rowptr;
    const int32_t* a_col;
    const int32_t* a_val;
    int64_t n, m, nnz;
    int64_t row_base, col_base, nnz_base;
    int64_t read_base;   // read id of the set's first row (a block of rows of a larger A: its first row)
    int64_t nreads;      // reads on the A^T side: C's columns (n, or the whole A's rows for a block)
    int32_t min_shared;
    int32_t id_bits;   // bits needed for a read id of this set (ESC radix passes)
    int32_t words;     // 32-bit words of a bitmap over the set's reads
    int32_t use_bits;  // 1: bitmap path, 0: hash path
    int64_t* c_rowptr;
    int32_t* c_col;
    int32_t* c_count;
    int32_t* c_seed;
};

constexpr int kMaxLog2 = 16;   // first-level symbolic classes (log2 table size)
constexpr int kMaxBins = 32;   // numeric bins: hash bins then bitmap bins
constexpr int kBitsClass = 0;  // symbolic class index used for bitmap rows

struct OvCounters {
    int64_t products;
    int64_t max_flops;
    int64_t esc_flops;
    int32_t sym_count[kMaxLog2];   // rows per symbolic class
    int32_t num_count[kMaxBins];   // rows per numeric bin
    int32_t retry_rows;            // hash rows that overflowed the first table
    int32_t esc_rows;
    int32_t overflow_rows;         // hash rows that overflowed the retry table too
    int32_t pad;
    int32_t qhead[64];             // work-queue heads of the persistent launches
};

// Queue heads: symbolic bitmap, symbolic hash classes, retry, numeric bins.
constexpr int kQSymBits = 0, kQSymHash = 1, kQRetry = 1 + kMaxLog2, kQNumeric = 2 + kMaxLog2;
static_assert(kQNumeric + kMaxBins <= 64, "queue heads");

// Persistent workgroups drain a queue of `count` items: the next item index,
// or -1 once the queue is empty.  Contains barriers (uniform).
__device__ __forceinline__ int next_item(int32_t* head, int count, int32_t* s_item) {
    if (threadIdx.x == 0) *s_item = atomicAdd(head, 1);
    __syncthreads();
    const int w = *s_item;
    __syncthreads();
    return w < count ? w : -1;
}

// Numeric bins: bin b holds rows with output size in (d[b-1], d[b]];
// bins [0, nh) serve the hash path, bins [nh, nh + nb) the bitmap path.
struct NumBins {
    int32_t nh, nb;
    int32_t d[kMaxBins];
};

enum : int32_t {
    kBadRowptr = 1,
    kBadCol = 2,
    kUnsorted = 4,
    kNegative = 8,
    kLongRow = 16,
};

constexpr uint64_t kEmpty64 = ~0ull;
constexpr int kMaxPlanes = 4;

// Open addressing with linear probing over T slots (any T): the start slot
// is the high part of (j * golden) * T.
__device__ __forceinline__ uint32_t hash_slot(int32_t j, uint32_t T) {
    return (uint32_t)(((uint64_t)((uint32_t)j * 0x9E3779B1u) * (uint64_t)T) >> 32);
}

// Insert key j; returns its slot, or -1 if all T slots were probed.
__device__ __forceinline__ int table_insert(int32_t* keys, uint32_t T, int32_t j) {
    uint32_t h = hash_slot(j, T);
    for (uint32_t p = 0; p < T; ++p) {
        const int32_t k = keys[h];
        if (k == j) return (int)h;
        if (k == -1) {
            const int32_t old = atomicCAS(&keys[h], -1, j);
            if (old == -1 || old == j) return (int)h;
        }
        if (++h == T) h = 0;
    }
    return -1;
}

// Slot of key j, or -1 if absent.
__device__ __forceinline__ int table_find(const int32_t* keys, uint32_t T, int32_t j) {
    uint32_t h = hash_slot(j, T);
    for (uint32_t p = 0; p < T; ++p) {
        const int32_t k = keys[h];
        if (k == j) return (int)h;
        if (k == -1) return -1;
        if (++h == T) h = 0;
    }
    return -1;
}

// Count one more occurrence of j in a table of u64 slots (j << 32) | count:
// insertion is a 64-bit CAS, the count a 64-bit add.  Returns the slot or -1
// (table full); *fresh = 1 if this call created the entry.
__device__ __forceinline__ int table64_add(uint64_t* tab, uint32_t T, int32_t j, int* fresh, uint32_t amount = 1) {
    uint32_t h = hash_slot(j, T);
    const uint64_t mine = ((uint64_t)(uint32_t)j << 32) | amount;
    *fresh = 0;
    for (uint32_t p = 0; p < T; ++p) {
        uint64_t v = tab[h];
        if (v == kEmpty64) {
            v = atomicCAS(&tab[h], kEmpty64, mine);
            if (v == kEmpty64) {
                *fresh = 1;
                return (int)h;
            }
        }
        if ((int32_t)(v >> 32) == j) {
            atomicAdd(&tab[h], (uint64_t)amount);
            return (int)h;
        }
        if (++h == T) h = 0;
    }
    return -1;
}

// Slots for `keys` distinct keys at a load of at most load_pct percent,
// rounded up to a multiple of 64.
__host__ __device__ __forceinline__ int64_t table_slots(int64_t keys, int load_pct) {
    const int64_t need = (keys * 100 + load_pct - 1) / load_pct;
    return ((need + 63) / 64) * 64;
}

// Bit planes of the bitmap path: plane p has bit j set once j was seen
// more than p times.  With min_shared <= kMaxPlanes planes the last plane
// is the output set.
__device__ __forceinline__ void planes_mark(uint32_t* B, int words, int planes, int32_t j) {
    const int w = j >> 5;
    const uint32_t bit = 1u << (j & 31);
    for (int p = 0; p < planes; ++p) {
        const uint32_t old = atomicOr(&B[p * words + w], bit);
        if (!(old & bit)) break;
    }
}

// Column slices for the segment pass: the global columns are cut into
// `count` ranges of about equal width, slice(c) = (c * mul) >> 32 with
// mul = floor(2^32 * count / total columns), so slice(c) < count and is
// monotone in c.  Each XCD gathers from one slice's share of the A^T column
// records at a time.
struct SliceMap {
    int32_t count;   // 0: no slices
    uint32_t mul;
};

// A^T column records (8 B per column): (start << 24) | length; a column of
// exactly two pairs (r0, p0), (r1, p1) instead holds
// kPairTag | ((p0 ^ p1) << 24) | (r0 ^ r1) (reads < 2^24, positions
// < 2^31).  An A entry's segment word is its column's record: an entry of
// a two-pair column, knowing its own read and position, recovers the other
// pair, so the walk has both products of the entry (itself and the other
// read) without gathering A^T.
constexpr uint64_t kPairTag = 1ull << 63;
__host__ __device__ __forceinline__ int slice_of(int64_t c, SliceMap sm) {
    return (int)(((uint64_t)c * sm.mul) >> 32);
}

// ---------------------------------------------------------------------------
// Step 1: validate A (one wave per row) and lay out its entries as pairs
// over the global entry space: key = global column, value =
// (position << 32) | read.  Grouping the pairs by key gives A^T.  With
// slices, the row's slice boundaries are recorded as well, slice-major:
// bnd[s * rows + g] = first entry of row g (relative to its start) whose
// column lies in slice s or later, for s = 0..count (s = count: the row
// length).  Without `keys` only the checks and the boundaries are made (A^T
// is then built column range by column range from the boundaries).
// ---------------------------------------------------------------------------
constexpr int kKeysIlp = 8;

// Workgroup b runs on XCD b mod 8 (dispatch is round-robin over the 8 XCDs):
// numbering the workgroups XCD by XCD gives each XCD one contiguous range of
// rows, so that the slice-major boundary writes of neighbouring rows (one
// 64-byte line holds 16 of them) meet in one L2.
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t grid) {
    return (grid & 7) ? b : (b & 7) * (grid >> 3) + (b >> 3);
}

template <int WPB>
__global__ __launch_bounds__(WPB* kWave) void k_ov_keys(const OvSet* __restrict__ sets, int nsets,
                                                        const int64_t* __restrict__ set_base, int64_t total_rows,
                                                        uint32_t* __restrict__ keys, uint64_t* __restrict__ pays,
                                                        int32_t* __restrict__ flags, int checks, SliceMap sm,
                                                        int32_t* __restrict__ bnd) {
    const int lane = lane_id();
    // the row, its set and the set's fields are wave-uniform: kept in scalar
    // registers so that the entry loads do not wait on them
    for (int64_t g = xcd_block(blockIdx.x, gridDim.x) * WPB + __builtin_amdgcn_readfirstlane(wave_id());
         g < total_rows; g += (int64_t)gridDim.x * WPB) {
        const int s = find_set(set_base, nsets, g);
        const OvSet S = sets[s];
        const int64_t i = g - S.row_base;
        const int64_t lo = S.a_rowptr[i], hi = S.a_rowptr[i + 1];
        int32_t bad = 0;
        if (i == 0 && lo != 0) bad |= kBadRowptr;
        if (i == S.n - 1 && hi != S.nnz) bad |= kBadRowptr;
        if (lo < 0 || hi < lo || hi > S.nnz) {
            bad |= kBadRowptr;
        } else if (hi - lo >= (int64_t(1) << 30)) {
            bad |= kLongRow;
        } else {
            int32_t prev_last = 0;   // column of the entry before this step's first
            int prev_sl = -1;        // slice of the entry before this step's first
            int32_t* rb = sm.count ? bnd + g : nullptr;   // boundary b at rb[b * total_rows]
            for (int64_t e0 = lo; e0 < hi; e0 += (int64_t)kWave * kKeysIlp) {
                int32_t kk[kKeysIlp], vv[kKeysIlp];
#pragma unroll
                for (int q = 0; q < kKeysIlp; ++q) {
                    const int64_t e = min(e0 + q * kWave + lane, hi - 1);   // clamped: no branch per load
                    kk[q] = gload(S.a_col + e);
                    vv[q] = gload(S.a_val + e);
                }
#pragma unroll
                for (int q = 0; q < kKeysIlp; ++q) {
                    const int64_t e = e0 + q * kWave + lane;
                    const bool in = e < hi;
                    const int32_t k = kk[q];
                    const bool ok = k >= 0 && k < S.m;
                    if (checks) {
                        // previous entry's column: from the lane below, or from
                        // the last lane of the previous group of 64
                        const int32_t up = __shfl_up(k, 1, kWave);
                        const int32_t prev = lane ? up : prev_last;
                        if (in && e > lo && prev >= k) bad |= kUnsorted;
                        if (in && vv[q] < 0) bad |= kNegative;
                        prev_last = __shfl(k, kWave - 1, kWave);
                    }
                    if (in) {
                        if (!ok) bad |= kBadCol;
                        // invalid columns get key 0: the call fails before A^T is used
                        if (keys) {
                            keys[S.nnz_base + e] = ok ? (uint32_t)(S.col_base + k) : 0u;
                            pays[S.nnz_base + e] = ((uint64_t)(uint32_t)vv[q] << 32) | (uint64_t)(uint32_t)i;
                        }
                    }
                    if (rb) {
                        // slices this entry opens: (slice of the previous entry, own slice];
                        // an unsorted or invalid row writes an incomplete table, but the
                        // call fails at the first synchronisation and every read of the
                        // table is clamped to the row
                        const int sl = ok ? slice_of(S.col_base + k, sm) : prev_sl;
                        const int up = __shfl_up(sl, 1, kWave);
                        const int psl = lane ? up : prev_sl;
                        if (in)
                            for (int b = max(psl, -1) + 1; b <= sl; ++b) rb[(int64_t)b * total_rows] = (int32_t)(e - lo);
                        prev_sl = __shfl(sl, kWave - 1, kWave);
                    }
                }
            }
            if (rb)
                for (int b = prev_sl + 1 + lane; b <= sm.count; b += kWave) rb[(int64_t)b * total_rows] = (int32_t)(hi - lo);
        }
        bad = wave_or_i32(bad);
        if (lane == 0 && bad) atomicOr(&flags[s], bad);
    }
}

// Products of an A entry whose column has record r.
__device__ __forceinline__ int64_t rec_products(uint64_t r) {
    return (r & kPairTag) ? 2 : (int64_t)(r & 0xFFFFFFull);
}

// ---------------------------------------------------------------------------
// Step 2: group the pairs by column with a bucketed counting sort, in two
// levels while the buckets (at most kMaxBuckets of 2^low columns, low <= 13)
// fit one partition, else in three:
//   k_ov_part_count   per workgroup (one or more chunks of kChunk pairs), a
//                     bucket histogram (bucket = key >> low), stored
//                     bucket-major;
//   scan              -> first output slot of every (bucket, workgroup);
//   k_ov_part_scatter per chunk, the pairs are ordered by bucket in LDS and
//                     written out as runs, so that stores coalesce;
//   (three levels: the first partition makes segments of 2^lowc columns;
//   the same two kernels in segmented mode then partition every segment
//   into buckets of 2^12 columns, see PartSeg)
//   k_ov_bucket_sort  one workgroup per bucket counts its pairs per column in
//                     LDS in staged sweeps of 2^12 columns, scans the counts
//                     into the column starts, places each (read, position)
//                     in LDS, writes the sweep out as one run and writes
//                     every column's record (its segment, or its two pairs;
//                     see kPairTag).
// The order inside an A^T row is left free: nothing downstream depends on it.
// Every pass takes the same chunks, so a malformed A (reported after the
// first synchronisation) can only over-count: writes are clamped to `cap`.
// ---------------------------------------------------------------------------
constexpr int kPartBlock = 1024;
constexpr int kPartIlp = 8;
constexpr int kChunk = kPartBlock * kPartIlp;
constexpr int kBucketBlock = 1024;
constexpr int64_t kMaxBuckets = 3840;
constexpr int kTwoLevelLow = 13;  // two levels: buckets of at most 2^13 columns
constexpr int kStageBits = 12;    // staged sweeps: 2^12 columns ...
constexpr int kStageCap = 17408;  // ... and at most this many pairs placed in LDS
constexpr int kCoarseLow = 20;    // three levels: segments of 2^20 columns (or wider, see the driver)

inline size_t part_scatter_lds(int64_t nbuckets) {
    return (size_t)kChunk * 12 + (size_t)nbuckets * 16;
}

// Segmented partition (the middle level of the three-level transpose): the
// input is already grouped by coarse bucket (segment c holds the pairs of
// columns [c << lowc, (c + 1) << lowc)), and every segment is partitioned on
// its own into F = 2^(lowc - low) fine buckets.  Segment c is cut into
// nch_c = chunk_base[c + 1] - chunk_base[c] chunks of kChunk pairs; its count
// table is fine-bucket-major over its chunks, starting at entry
// chunk_base[c] * F, so that one exclusive scan over all tables gives every
// (segment, fine bucket, chunk) its output position directly.
struct PartSeg {
    const int64_t* seg_start;    // [nseg + 1] first pair of each segment
    const int64_t* chunk_base;   // [nseg + 1] first chunk of each segment
    int32_t nseg;
};

// Pair range and count-table layout of one chunk.  Flat mode: chunk
// blockIdx.x * per_block + c over [0, n), table entry of bucket b at
// b * gridDim.x + blockIdx.x.  Segmented mode (one chunk per workgroup): the
// workgroup's chunk u within its segment sg, table entry of bucket b at
// chunk_base[sg] * nbuckets + b * nch_sg + u.  Returns false when the
// workgroup has no chunk.
struct ChunkPos {
    int64_t c0, c1;        // pairs [c0, c1)
    int64_t tab0, tstride; // table entry of bucket b: tab0 + b * tstride
};
template <bool SEG>
__device__ __forceinline__ bool chunk_pos(int64_t n, int per_block, int c, int nbuckets, const PartSeg& ps,
                                          ChunkPos* cp) {
    if (!SEG) {
        cp->c0 = ((int64_t)blockIdx.x * per_block + c) * kChunk;
        cp->c1 = min(cp->c0 + kChunk, n);
        cp->tab0 = blockIdx.x;
        cp->tstride = gridDim.x;
        return cp->c0 < n;
    }
    const int64_t q = blockIdx.x;
    if (q >= ps.chunk_base[ps.nseg]) return false;
    const int sg = find_set(ps.chunk_base, ps.nseg, q);
    const int64_t cb = ps.chunk_base[sg], nch = ps.chunk_base[sg + 1] - cb;
    cp->c0 = ps.seg_start[sg] + (q - cb) * kChunk;
    cp->c1 = min(cp->c0 + kChunk, ps.seg_start[sg + 1]);
    cp->tab0 = cb * nbuckets + (q - cb);
    cp->tstride = nch;
    return true;
}

// Bucket of a key: flat mode, key >> low clamped into range (keys of a
// malformed A may be unset); segmented mode, its fine bucket within the
// segment.
template <bool SEG>
__device__ __forceinline__ uint32_t bucket_of(uint32_t key, int low, int nbuckets) {
    return SEG ? (key >> low) & (uint32_t)(nbuckets - 1) : min(key >> low, (uint32_t)nbuckets - 1u);
}

// Adds `valid` lanes to hist[b] with one LDS atomic per run of consecutive
// lanes of the wave that share b (neighbouring pairs often share a bucket:
// a row's columns cluster when columns follow first occurrence, and one
// atomic per lane on one address would serialise).  Invalid lanes are the
// wave's last ones.
__device__ __forceinline__ void wave_run_add(uint32_t* hist, uint32_t b, bool valid) {
    const int lane = (int)(threadIdx.x & (kWave - 1));
    const uint32_t prev = __shfl_up(b, 1, kWave);
    const bool head = lane == 0 || prev != b;
    const uint64_t heads = __ballot(head);
    const uint64_t valids = __ballot(valid);
    if (head) {
        const uint64_t above = lane == kWave - 1 ? 0ull : heads & ~((2ull << lane) - 1ull);
        const uint64_t upto = above ? (above & (0ull - above)) - 1ull : ~0ull;   // lanes below the next head
        const uint32_t cnt = (uint32_t)__popcll(valids & upto & ~((1ull << lane) - 1ull));
        if (cnt) atomicAdd(&hist[b], cnt);
    }
}

template <bool SEG>
__global__ __launch_bounds__(kPartBlock) void k_ov_part_count(const uint32_t* __restrict__ keys, int64_t n,
                                                              int per_block, int low, int nbuckets,
                                                              PartSeg ps, int32_t* __restrict__ counts) {
    extern __shared__ __align__(16) unsigned char smem[];
    uint32_t* hist = reinterpret_cast<uint32_t*>(smem);
    ChunkPos cp;
    if (SEG && !chunk_pos<SEG>(n, 1, 0, nbuckets, ps, &cp)) {
        // surplus workgroups (the grid is sized from a bound) zero the unused
        // tail of the table, which the scan reads
        const int64_t q = (int64_t)blockIdx.x - ps.chunk_base[ps.nseg];
        const int64_t t0 = (ps.chunk_base[ps.nseg] + q) * nbuckets;
        for (int b = threadIdx.x; b < nbuckets; b += kPartBlock) counts[t0 + b] = 0;
        return;
    }
    for (int b = threadIdx.x; b < nbuckets; b += kPartBlock) hist[b] = 0u;
    __syncthreads();
    for (int c = 0; c < (SEG ? 1 : per_block); ++c) {
        if (!chunk_pos<SEG>(n, per_block, c, nbuckets, ps, &cp)) break;
        const int64_t c0 = cp.c0, c1 = cp.c1;
        uint32_t kk[kPartIlp];
#pragma unroll
        for (int q = 0; q < kPartIlp; ++q) kk[q] = keys[min(c0 + q * kPartBlock + threadIdx.x, c1 - 1)];
#pragma unroll
        for (int q = 0; q < kPartIlp; ++q)
            wave_run_add(hist, bucket_of<SEG>(kk[q], low, nbuckets), c0 + q * kPartBlock + threadIdx.x < c1);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < nbuckets; b += kPartBlock) counts[cp.tab0 + (int64_t)b * cp.tstride] = (int32_t)hist[b];
}

// K: the width of the keys written out; the next pass reads only their low
// bits, so where it needs at most 16 of them (buckets of at most 2^15
// columns sorted in staged sweeps) 16-bit keys halve the key bytes of both
// passes.  SEG: segmented mode (see PartSeg; one chunk per workgroup, a
// surplus workgroup does nothing).
template <bool SEG, class K>
__global__ __launch_bounds__(kPartBlock) void k_ov_part_scatter(
    const uint32_t* __restrict__ keys, const uint64_t* __restrict__ pays, int64_t n, int per_block, int low,
    int nbuckets, PartSeg ps, const int64_t* __restrict__ offsets, int64_t cap, K* __restrict__ skey,
    uint64_t* __restrict__ spay) {
    extern __shared__ __align__(16) unsigned char smem[];
    uint64_t* st_pay = reinterpret_cast<uint64_t*>(smem);                 // [kChunk]
    uint32_t* st_key = reinterpret_cast<uint32_t*>(st_pay + kChunk);      // [kChunk]
    uint32_t* lcnt = st_key + kChunk;                                     // [nbuckets] count, then cursor
    uint32_t* loff = lcnt + nbuckets;                                     // [nbuckets] chunk-local start
    int64_t* gpos = reinterpret_cast<int64_t*>(loff + nbuckets);          // [nbuckets], 8-byte aligned
    __shared__ uint32_t s_tmp[kPartBlock / kWave + 1];
    ChunkPos cp;
    if (!chunk_pos<SEG>(n, per_block, 0, nbuckets, ps, &cp)) return;   // uniform over the workgroup
    for (int b = threadIdx.x; b < nbuckets; b += kPartBlock) gpos[b] = offsets[cp.tab0 + (int64_t)b * cp.tstride];
    const int per = (nbuckets + kPartBlock - 1) / kPartBlock;
    const int b0 = threadIdx.x * per;
    for (int c = 0; c < (SEG ? 1 : per_block); ++c) {
        if (c > 0 && !chunk_pos<SEG>(n, per_block, c, nbuckets, ps, &cp)) break;
        const int64_t c0 = cp.c0, c1 = cp.c1;
        for (int b = threadIdx.x; b < nbuckets; b += kPartBlock) lcnt[b] = 0u;
        __syncthreads();
        uint32_t kk[kPartIlp], rk[kPartIlp];
        uint64_t pp[kPartIlp];
#pragma unroll
        for (int q = 0; q < kPartIlp; ++q) {
            const int64_t e = min(c0 + q * kPartBlock + threadIdx.x, c1 - 1);
            // flat mode: keys of a malformed A may be unset, the bucket is clamped into range
            kk[q] = SEG ? keys[e] : min(keys[e], ((uint32_t)nbuckets << low) - 1u);
            pp[q] = pays[e];
        }
        // rank of each pair among the chunk's pairs of its bucket
#pragma unroll
        for (int q = 0; q < kPartIlp; ++q)
            rk[q] = atomicAdd(&lcnt[bucket_of<SEG>(kk[q], low, nbuckets)],
                              c0 + q * kPartBlock + threadIdx.x < c1 ? 1u : 0u);
        __syncthreads();
        // chunk-local bucket starts: each thread scans a run of consecutive buckets
        uint32_t local = 0;
        for (int q = 0; q < per; ++q)
            if (b0 + q < nbuckets) local += lcnt[b0 + q];
        uint32_t tot;
        uint32_t run = block_exclusive_sum<kPartBlock>(local, s_tmp, &tot);
        for (int q = 0; q < per; ++q) {
            if (b0 + q >= nbuckets) break;
            loff[b0 + q] = run;
            run += lcnt[b0 + q];
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < kPartIlp; ++q) {
            if (c0 + q * kPartBlock + threadIdx.x >= c1) continue;
            const uint32_t slot = loff[bucket_of<SEG>(kk[q], low, nbuckets)] + rk[q];
            st_key[slot] = kk[q];
            st_pay[slot] = pp[q];
        }
        __syncthreads();
        // consecutive slots of one bucket go to consecutive output positions
        for (uint32_t slot = threadIdx.x; slot < tot; slot += kPartBlock) {
            const uint32_t key = st_key[slot];
            const int b = (int)bucket_of<SEG>(key, low, nbuckets);
            const int64_t pos = gpos[b] + (slot - loff[b]);
            if (pos < cap) {
                skey[pos] = (K)key;
                spay[pos] = st_pay[slot];
            }
        }
        __syncthreads();
        // the next chunk of this workgroup continues after this one's runs
        for (int b = threadIdx.x; b < nbuckets; b += kPartBlock) gpos[b] += lcnt[b];
    }
}

// Three-level transpose, between the levels: the segments (coarse buckets)
// from the first level's scanned table and their chunk counts, scanned into
// chunk_base (one workgroup).
constexpr int kSegChunkBlock = 1024;
__global__ __launch_bounds__(kSegChunkBlock) void k_ov_seg_chunks(const int64_t* __restrict__ offs1, int64_t npart1,
                                                                  int nseg, int64_t cap,
                                                                  int64_t* __restrict__ seg_start,
                                                                  int64_t* __restrict__ chunk_base) {
    __shared__ int64_t s_tmp[kSegChunkBlock / kWave + 1];
    int64_t carry = 0;
    for (int c0 = 0; c0 <= nseg; c0 += kSegChunkBlock) {
        const int c = c0 + (int)threadIdx.x;
        int64_t st = 0, nch = 0;
        if (c <= nseg) {
            st = min(offs1[(int64_t)c * npart1], cap);
            seg_start[c] = st;
            if (c < nseg) nch = (min(offs1[(int64_t)(c + 1) * npart1], cap) - st + kChunk - 1) / kChunk;
        }
        int64_t tot;
        const int64_t ex = block_exclusive_sum<kSegChunkBlock>(nch, s_tmp, &tot);
        if (c <= nseg) chunk_base[c] = carry + ex;
        carry += tot;
    }
}

// Start of every fine bucket b = sg * F + f (its first chunk's table entry
// in the scanned second-level table), and the end of the last one.
__global__ void k_ov_fine_start(const int64_t* __restrict__ offs2, const int64_t* __restrict__ chunk_base, int nseg,
                                int F, int64_t nfine, int64_t* __restrict__ fine_start) {
    for (int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b <= nfine; b += (int64_t)gridDim.x * blockDim.x) {
        const int64_t sg = b / F, f = b % F;
        int64_t e;
        if (sg >= nseg) e = chunk_base[nseg] * F;
        else e = chunk_base[sg] * F + f * (chunk_base[sg + 1] - chunk_base[sg]);
        fine_start[b] = offs2[e];
    }
}

// A^T over column ranges (one set): the range [c0, c1) holds the columns of
// slices [s0, s1), so row g's entries in it are [bnd[s0][g], bnd[s1][g]).
// Boundaries of a row that failed validation may be incomplete: they are
// clamped to the row, and the call fails before A^T is read.
__device__ __forceinline__ int2 range_of_row(const int32_t* bnd, int64_t stride, int64_t g, int s0, int s1,
                                             int32_t L) {
    const int32_t a = min(max(bnd[(int64_t)s0 * stride + g], 0), L);
    const int32_t z = min(max(bnd[(int64_t)s1 * stride + g], a), L);
    return make_int2(a, z);
}

// Entries per row in the range, and the range's total.
__global__ __launch_bounds__(256) void k_ov_range_count(const OvSet* __restrict__ sets, int64_t rows,
                                                        const int32_t* __restrict__ bnd, int s0, int s1,
                                                        int32_t* __restrict__ cnt) {
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < rows; g += (int64_t)gridDim.x * blockDim.x) {
        const OvSet& S = sets[0];
        const int64_t lo = S.a_rowptr[g], hi = S.a_rowptr[g + 1];
        const int32_t L = (lo < 0 || hi < lo || hi > S.nnz || hi - lo >= (int64_t(1) << 30)) ? 0 : (int32_t)(hi - lo);
        const int2 r = range_of_row(bnd, rows, g, s0, s1, L);
        cnt[g] = r.y - r.x;
    }
}

// The range's pairs, row by row at off[g]: key = column - c0 (0 for a column
// outside the range, which only a row that failed validation has), value =
// (position << 32) | read.  Nothing is written at or past `cap` (the pairs
// the host sized the buffers for; only an invalid A has more).
__global__ __launch_bounds__(256) void k_ov_range_keys(const OvSet* __restrict__ sets, int64_t rows,
                                                       const int32_t* __restrict__ bnd, int s0, int s1, int64_t c0,
                                                       int64_t c1, const int64_t* __restrict__ off, int64_t cap,
                                                       uint32_t* __restrict__ keys, uint64_t* __restrict__ pays) {
    const int lane = lane_id();
    for (int64_t g = (int64_t)blockIdx.x * (blockDim.x / kWave) + __builtin_amdgcn_readfirstlane(wave_id());
         g < rows; g += (int64_t)gridDim.x * (blockDim.x / kWave)) {
        const OvSet& S = sets[0];
        const int64_t lo = S.a_rowptr[g], hi = S.a_rowptr[g + 1];
        const int32_t L = (lo < 0 || hi < lo || hi > S.nnz || hi - lo >= (int64_t(1) << 30)) ? 0 : (int32_t)(hi - lo);
        const int2 r = range_of_row(bnd, rows, g, s0, s1, L);
        const int64_t o = off[g] - r.x;
        for (int32_t q = r.x + lane; q < r.y; q += kWave) {
            if (o + q >= cap) break;
            const int32_t k = gload(S.a_col + lo + q);
            const int32_t v = gload(S.a_val + lo + q);
            keys[o + q] = (k >= c0 && k < c1) ? (uint32_t)(k - c0) : 0u;
            pays[o + q] = ((uint64_t)(uint32_t)v << 32) | (uint64_t)(uint32_t)g;
        }
    }
}

// One workgroup per bucket of 2^low columns (first pair at
// start[b * stride], 16-bit keys holding at least the low `low` bits), sorted
// in sweeps of 2^sub columns (sub = min(low, 12)): per sweep the pairs of its
// columns are counted, placed in LDS and written out as one contiguous run
// (coalesced) when they fit kStageCap, else placed directly.  Only a staged
// sweep writes the two-pair records (otherwise every column gets its
// segment).  The pairs land in at[] at their input positions; a record's
// start is that position plus rec_base (A^T built column range by column
// range: `at` points at the range's first slot, rec_base is its index).
__global__ __launch_bounds__(kBucketBlock) void k_ov_bucket_sort(
    const int64_t* __restrict__ start, int64_t stride, int low, int sub, int64_t total_m, int64_t cap,
    const uint16_t* __restrict__ skey, const uint64_t* __restrict__ spay, uint64_t* __restrict__ rec,
    uint64_t* __restrict__ at, int64_t rec_base) {
    extern __shared__ __align__(16) unsigned char smem[];
    uint32_t* hist = reinterpret_cast<uint32_t*>(smem);
    uint64_t* stage = reinterpret_cast<uint64_t*>(hist + (1 << sub));
    __shared__ int64_t s_tmp[kBucketBlock / kWave + 1];
    const int b = blockIdx.x;
    const int sweeps = 1 << (low - sub);
    const int bins = 1 << sub;
    const uint32_t lmask = (uint32_t)(1u << low) - 1u, smask = (uint32_t)bins - 1u;
    const int64_t bs = min(start[(int64_t)b * stride], cap);
    const int64_t be = min(start[(int64_t)(b + 1) * stride], cap);
    const int64_t col_b = (int64_t)b << low;
    const int per = bins >= kBucketBlock ? bins / kBucketBlock : 1;
    const int c0 = threadIdx.x * per;
    int64_t base = bs;   // first slot of this sweep's columns
    for (int h = 0; h < sweeps; ++h) {
        for (int c = threadIdx.x; c < bins; c += kBucketBlock) hist[c] = 0u;
        __syncthreads();
        for (int64_t e0 = bs; e0 < be; e0 += kBucketBlock * kPartIlp) {
            uint32_t kk[kPartIlp];
#pragma unroll
            for (int q = 0; q < kPartIlp; ++q)
                kk[q] = skey[min(e0 + q * kBucketBlock + threadIdx.x, be - 1)] & lmask;   // clamped: no branch
#pragma unroll
            for (int q = 0; q < kPartIlp; ++q)
                atomicAdd(&hist[kk[q] & smask],
                          (e0 + q * kBucketBlock + threadIdx.x < be && (int)(kk[q] >> sub) == h) ? 1u : 0u);
        }
        __syncthreads();
        // exclusive scan of the bins: each thread owns `per` consecutive bins
        int64_t local = 0;
        for (int q = 0; q < per; ++q)
            if (c0 + q < bins) local += hist[c0 + q];
        int64_t tot;
        int64_t run = block_exclusive_sum<kBucketBlock>(local, s_tmp, &tot);
        const int64_t col0 = col_b + ((int64_t)h << sub);
        for (int q = 0; q < per; ++q) {
            const int c = c0 + q;
            if (c >= bins) break;
            const uint32_t n_c = hist[c];
            hist[c] = (uint32_t)(base + run);   // becomes the cursor of column c (< 2^32)
            run += n_c;
        }
        const bool staged = tot <= kStageCap;
        __syncthreads();
        for (int64_t e0 = bs; e0 < be; e0 += kBucketBlock * kPartIlp) {
            uint32_t kk[kPartIlp], pos[kPartIlp];
            uint64_t pp[kPartIlp];
#pragma unroll
            for (int q = 0; q < kPartIlp; ++q) {
                const int64_t e = min(e0 + q * kBucketBlock + threadIdx.x, be - 1);   // clamped: no branch
                kk[q] = skey[e] & lmask;
                pp[q] = (int)(kk[q] >> sub) == h ? spay[e] : 0ull;
            }
            bool mine[kPartIlp];
#pragma unroll
            for (int q = 0; q < kPartIlp; ++q) {
                mine[q] = e0 + q * kBucketBlock + threadIdx.x < be && (int)(kk[q] >> sub) == h;
                pos[q] = atomicAdd(&hist[kk[q] & smask], mine[q] ? 1u : 0u);
            }
#pragma unroll
            for (int q = 0; q < kPartIlp; ++q) {
                if (!mine[q]) continue;
                if (staged) stage[pos[q] - base] = pp[q];
                else if (pos[q] < cap) at[pos[q]] = pp[q];
            }
        }
        __syncthreads();
        if (staged)
            for (int64_t q = threadIdx.x; q < tot; q += kBucketBlock)
                if (base + q < cap) at[base + q] = stage[q];
        // column records: the cursors now hold the column ends, so column c
        // spans [end of c - 1, end of c); a column of two pairs carries them
        // (from the stage) so that a walk needs no A^T gather for it
        for (int q = 0; q < per; ++q) {
            const int c = c0 + q;
            if (c >= bins || col0 + c >= total_m) break;
            const uint32_t end = hist[c];
            const uint32_t first = c ? hist[c - 1] : (uint32_t)base;
            const uint32_t n_c = end - first;
            uint64_t r = ((uint64_t)(first + rec_base) << 24) | (uint64_t)n_c;
            if (staged && n_c == 2) {
                const uint64_t x = stage[first - base] ^ stage[first - base + 1];   // pairs: (pos << 32) | read
                r = kPairTag | ((x >> 32) << 24) | (x & 0xFFFFFFull);
            }
            rec[col0 + c] = r;
        }
        base += tot;
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Step 3: each A entry's segment word (its column's record), products per
// row, the row's scratch range bound, and bin rows for the symbolic phase:
// bitmap-path rows in one class, hash-path rows by first-level table size.
// k_ov_scatter: a workgroup owns kRowsPerBlock consecutive rows (one wave
// per row at a time); bin counts and totals are gathered in LDS and
// published with one global atomic per workgroup and counter.  With column
// slices the segment words come from k_ov_seg_slices first and k_ov_scatter
// only sums its products per (slice, row).
// ---------------------------------------------------------------------------
constexpr int kRowsPerBlock = 64;
constexpr int kSegWaves = 16;
constexpr int kSegIlp = 8;

// Sliced segment pass.  Workgroups are handed to the XCDs round-robin
// (workgroup b runs on XCD b mod 8), so workgroup b takes slice
// 8 * round + (b mod 8): at any time each XCD gathers column records from
// one slice only (at most 16 MB; with columns in first-occurrence order a
// row's records cluster, so the lines one workgroup touches are far fewer),
// instead of every XCD gathering from all of them.  A workgroup covers the
// sub-ranges of kSliceRows rows in its slice; those are short (a row spreads
// its entries over the slices), so the workgroup numbers their entries consecutively
// (a scan of the 64 lengths) and every thread takes entries by number,
// kSliceIlp at a time, finding the row with a search over the 64 starts:
// consecutive threads read consecutive columns and write consecutive
// segment words.  Products per (slice, row) go to part[slice * rows + row]
// (32 bits, saturated at 2^31: a row that large fails the call anyway);
// k_ov_scatter sums them.
constexpr int kSliceRows = 64;
constexpr int kSliceBlock = 256;
constexpr int kSliceIlp = 4;
constexpr int kMaxSlices = 8192;                   // 2^32 columns at kSliceCols each
// 2^21 columns (16 MB of records) per slice: with columns in first-occurrence
// order, wider slices cut a row into fewer sub-ranges and write a smaller
// boundary table (2^19 columns, one L2's worth, suited columns in code order)
constexpr int64_t kSliceCols = int64_t(1) << 21;
// a readable word for the loads of rows with no entries in a slice (their
// values are never used)
__device__ const int32_t kSliceNone[1] = {0};

__global__ __launch_bounds__(kSliceBlock) void k_ov_seg_slices(
    const OvSet* __restrict__ sets, int nsets, const int64_t* __restrict__ set_base, int64_t total_rows,
    int64_t groups, SliceMap sm, const int32_t* __restrict__ bnd, int64_t bnd_stride, const uint64_t* __restrict__ rec,
    uint64_t* __restrict__ seg, uint32_t* __restrict__ part) {
    __shared__ int32_t s_pre[kSliceRows + 1];      // first flat number of each row's sub-range
    __shared__ int64_t s_first[kSliceRows];        // global entry of the row's first entry in the slice
    __shared__ const int32_t* s_col[kSliceRows];   // its column
    __shared__ int64_t s_cb[kSliceRows], s_m[kSliceRows];
    __shared__ unsigned long long s_prod[kSliceRows];
    __shared__ int32_t s_tmp[kSliceBlock / kWave + 1];
    const int64_t b = blockIdx.x;
    const int sl = (int)((b / 8) / groups) * 8 + (int)(b % 8);
    const int64_t row0 = ((b / 8) % groups) * kSliceRows;
    if (sl >= sm.count) return;   // uniform over the workgroup
    int32_t len = 0;
    if (threadIdx.x < kSliceRows) {
        const int r = threadIdx.x;
        const int64_t g = row0 + r;
        s_first[r] = 0;
        s_col[r] = kSliceNone;
        s_cb[r] = 0;
        s_m[r] = 0;
        s_prod[r] = 0;
        if (g < total_rows) {
            const int s = find_set(set_base, nsets, g);
            const OvSet& S = sets[s];
            const int64_t i = g - S.row_base;
            const int64_t lo = S.a_rowptr[i], hi = S.a_rowptr[i + 1];
            if (!(lo < 0 || hi < lo || hi > S.nnz || hi - lo >= (int64_t(1) << 30))) {
                const int32_t L = (int32_t)(hi - lo);
                const int32_t a = min(max(bnd[(int64_t)sl * bnd_stride + g], 0), L);
                const int32_t z = min(max(bnd[(int64_t)(sl + 1) * bnd_stride + g], a), L);
                len = z - a;
                s_first[r] = S.nnz_base + lo + a;
                if (z > a) s_col[r] = S.a_col + lo + a;
                s_cb[r] = S.col_base;
                s_m[r] = S.m;
            }
        }
    }
    // sub-range lengths are below 2^30 each and the call's entries below
    // 2^31, so the workgroup's numbering fits 32 bits
    int32_t tot;
    const int32_t ex = block_exclusive_sum<kSliceBlock>(len, s_tmp, &tot);
    if (threadIdx.x < kSliceRows) s_pre[threadIdx.x] = ex;
    __syncthreads();
    for (int32_t q0 = threadIdx.x; q0 < tot; q0 += kSliceBlock * kSliceIlp) {
        // unconditional loads from clamped addresses: no load waits on another
        int rr[kSliceIlp];
        int32_t oo[kSliceIlp], kk[kSliceIlp];
#pragma unroll
        for (int u = 0; u < kSliceIlp; ++u) {
            const int32_t q = min(q0 + u * kSliceBlock, tot - 1);
            rr[u] = upper_index(s_pre, kSliceRows, q);   // the last row starting at or before q: non-empty
            oo[u] = q - s_pre[rr[u]];
            kk[u] = gload_nt(s_col[rr[u]] + oo[u]);
        }
        uint64_t rc[kSliceIlp];
#pragma unroll
        for (int u = 0; u < kSliceIlp; ++u) {
            const bool ok = kk[u] >= 0 && kk[u] < s_m[rr[u]];
            rc[u] = gload(rec + (ok ? s_cb[rr[u]] + kk[u] : 0));
        }
#pragma unroll
        for (int u = 0; u < kSliceIlp; ++u) {
            if (q0 + u * kSliceBlock >= tot) continue;
            const bool ok = kk[u] >= 0 && kk[u] < s_m[rr[u]];
            const uint64_t sg = ok ? rc[u] : 0ull;   // invalid column: empty segment
            atomicAdd(&s_prod[rr[u]], (unsigned long long)rec_products(sg));
            seg[s_first[rr[u]] + oo[u]] = sg;   // ordinary store: L2 merges the lines
        }
    }
    __syncthreads();
    if (threadIdx.x < kSliceRows) {
        const int64_t g = row0 + threadIdx.x;
        const unsigned long long p = s_prod[threadIdx.x];
        if (g < total_rows) part[(int64_t)sl * total_rows + g] = (uint32_t)(p < (1ull << 31) ? p : (1ull << 31));
    }
}

template <int WPB>
__global__ __launch_bounds__(WPB* kWave) void k_ov_scatter(
    const OvSet* __restrict__ sets, int nsets, const int64_t* __restrict__ set_base, int64_t total_rows,
    const uint64_t* __restrict__ rec, uint64_t* __restrict__ seg, int64_t* __restrict__ flops_row,
    int64_t* __restrict__ sbound, int32_t* __restrict__ sym_list,
    OvCounters* __restrict__ ctr, int first_log2, int load_pct, const uint32_t* __restrict__ part, int nslices) {
    __shared__ int32_t s_cnt[kMaxLog2], s_base[kMaxLog2];
    __shared__ int32_t s_bin[kRowsPerBlock], s_pos[kRowsPerBlock];
    __shared__ unsigned long long s_prod;
    __shared__ int64_t s_max;
    const int lane = lane_id();
    if (threadIdx.x < kMaxLog2) s_cnt[threadIdx.x] = 0;
    if (threadIdx.x == 0) {
        s_prod = 0;
        s_max = 0;
    }
    __syncthreads();
    const int64_t row0 = (int64_t)blockIdx.x * kRowsPerBlock;
    // rows are wave-uniform (scalar registers); kSegIlp entries per lane per
    // step with all column loads, then all row-pointer gathers, in flight
    for (int r = __builtin_amdgcn_readfirstlane(wave_id()); r < kRowsPerBlock; r += WPB) {
        const int64_t g = row0 + r;
        if (g >= total_rows) {
            if (lane == 0) s_bin[r] = -1;
            continue;
        }
        const int s = find_set(set_base, nsets, g);
        const OvSet S = sets[s];
        const int64_t i = g - S.row_base;
        const int64_t lo = S.a_rowptr[i], hi = S.a_rowptr[i + 1];
        int64_t fl = 0;
        if (part) {
            // the segments are written by the sliced pass: sum its partial products
            for (int q = lane; q < nslices; q += kWave) fl += part[(int64_t)q * total_rows + g];
        } else if (!(lo < 0 || hi < lo || hi > S.nnz || hi - lo >= (int64_t(1) << 30))) {
            for (int64_t e0 = lo; e0 < hi; e0 += (int64_t)kWave * kSegIlp) {
                int32_t kk[kSegIlp];
                uint64_t rc[kSegIlp];
#pragma unroll
                for (int q = 0; q < kSegIlp; ++q) kk[q] = gload(S.a_col + min(e0 + q * kWave + lane, hi - 1));
#pragma unroll
                for (int q = 0; q < kSegIlp; ++q) {
                    const int32_t k = kk[q];
                    const int64_t gk = (k >= 0 && k < S.m) ? S.col_base + k : 0;   // in range for the load
                    rc[q] = rec[gk];
                }
#pragma unroll
                for (int q = 0; q < kSegIlp; ++q) {
                    const int64_t e = e0 + q * kWave + lane;
                    if (e >= hi) continue;
                    if (!(kk[q] >= 0 && kk[q] < S.m)) rc[q] = 0ull;   // invalid column: empty segment
                    const uint64_t sg = rc[q];
                    fl += rec_products(sg);
                    seg[S.nnz_base + e] = sg;
                }
            }
        }
        fl = wave_sum(fl);
        if (lane == 0) {
            flops_row[g] = fl;
            // scratch range for the row's output columns: at most
            // min(products / min_shared, reads) of them
            const int64_t bound = fl / S.min_shared;
            sbound[g] = bound < S.nreads ? bound : S.nreads;
            s_bin[r] = -1;
            if (fl > 0) {
                atomicAdd(&s_prod, (unsigned long long)fl);
                atomic_max(&s_max, fl);
                int lg = kBitsClass;
                if (!S.use_bits) {
                    const int64_t keys = fl < S.nreads ? fl : S.nreads;
                    lg = ceil_log2_i64((keys * 100 + load_pct - 1) / load_pct);
                    lg = lg < 6 ? 6 : (lg > first_log2 ? first_log2 : lg);
                }
                s_bin[r] = lg;
                s_pos[r] = atomicAdd(&s_cnt[lg], 1);
            }
        }
    }
    __syncthreads();
    if (threadIdx.x < kMaxLog2 && s_cnt[threadIdx.x] > 0)
        s_base[threadIdx.x] = atomicAdd(&ctr->sym_count[threadIdx.x], s_cnt[threadIdx.x]);
    if (threadIdx.x == kWave && s_prod > 0) {
        atomic_add(&ctr->products, (int64_t)s_prod);
        atomic_max(&ctr->max_flops, s_max);
    }
    __syncthreads();
    for (int r = threadIdx.x; r < kRowsPerBlock; r += WPB * kWave) {
        const int b = s_bin[r];
        if (b >= 0) sym_list[(int64_t)b * total_rows + s_base[b] + s_pos[r]] = (int32_t)(row0 + r);
    }
}

// ---------------------------------------------------------------------------
// Shared product walk: the A entries t of row i are taken in chunks of
// walk_chunk_of(BLOCK) entries (two per thread); seg[t] gives the A^T
// segment (start, length) of entry t, and the products of the chunk are
// numbered t-major.  Products are handed out in windows of
// walk_win_of(BLOCK): every thread first writes its entries' chunk indices
// over their products' slots of the window (an LDS expansion, so that a
// product finds its entry with one LDS read), then each thread takes
// walk_per(BLOCK) products and issues all their gathers of A^T pairs before
// handing them to f(t, (j, p_j), q), so that several independent loads are
// in flight per thread.  The segments of the next chunk are loaded before
// the gathers of the current one, so the two loads overlap instead of
// following each other.  The block must call it uniformly.  `stop` (LDS
// flag) abandons the walk.  LDS: c_base (one int64 per chunk entry: segment
// start minus the entry's first product number, so a product q of entry t
// sits at A^T[c_base[t] + q]) and tbuf (one u16 per window product), carved
// from the front of the dynamic LDS by walk_lds().
// ---------------------------------------------------------------------------
__host__ __device__ constexpr int walk_chunk_of(int block) { return 2 * block; }
__host__ __device__ constexpr int walk_win_of(int block) { return block * 8 < 4096 ? block * 8 : 4096; }
__host__ __device__ constexpr size_t walk_lds(int block) {
    return (size_t)walk_chunk_of(block) * 8 + (size_t)walk_win_of(block) * 2;
}
__host__ __device__ constexpr int walk_per(int block) { return walk_win_of(block) / block; }
// the ESC expansion's static walk area
constexpr int kWalkChunk = 512;
constexpr int kWalkWin = 2048;

// Loads the segments of the chunk's entries owned by this thread (length 0
// past the end of the row) and, given the row's positions, their positions.
template <int BLOCK>
__device__ __forceinline__ void walk_load(const uint64_t* __restrict__ rseg, const int32_t* __restrict__ rval,
                                          int cbase, int cl, uint64_t (&sg)[walk_chunk_of(BLOCK) / BLOCK],
                                          int32_t (&pv)[walk_chunk_of(BLOCK) / BLOCK]) {
    constexpr int E = walk_chunk_of(BLOCK) / BLOCK;
#pragma unroll
    for (int u = 0; u < E; ++u) {
        const int e = (int)threadIdx.x * E + u;
        sg[u] = e < cl ? rseg[cbase + e] : 0ull;
        pv[u] = (rval && e < cl) ? rval[cbase + e] : 0;
    }
}

// Numbers the chunk's products (t-major) from its loaded segment words,
// writes c_base and returns the chunk's product count.  An entry of a
// two-pair column (kPairTag) has two products, itself and the other pair;
// the other pair follows from the column's XORs and the entry's own read
// and position (position 0 unless the row's positions were loaded), and its
// c_base holds it as kInlineBase - ((position << 24) | read) (< 2^55), at or
// below -2^62, far below every real base (those exceed -2^31).  Each thread keeps its
// entries' offsets and lengths for the window fills.
constexpr int64_t kInlineBase = -(int64_t(1) << 62);
constexpr int64_t kInlineBelow = -(int64_t(1) << 32);
__device__ __forceinline__ int2 inline_pair(int64_t cb) {
    const uint64_t v = (uint64_t)(kInlineBase - cb);
    return make_int2((int)(v & 0xFFFFFFull), (int)(v >> 24));
}
// Chunk-local counts are 32-bit: a row's products stay below 2^31 (a call
// with a larger row fails before any walk), and 64-bit counters here had
// cost the walking kernels a third of their occupancy in registers.
template <int BLOCK>
__device__ __forceinline__ int32_t walk_chunk(const uint64_t (&sg)[walk_chunk_of(BLOCK) / BLOCK],
                                              const int32_t (&pv)[walk_chunk_of(BLOCK) / BLOCK], int32_t self,
                                              int64_t* c_base, int64_t* s_tmp,
                                              int32_t (&my_off)[walk_chunk_of(BLOCK) / BLOCK],
                                              int32_t (&my_len)[walk_chunk_of(BLOCK) / BLOCK]) {
    constexpr int E = walk_chunk_of(BLOCK) / BLOCK;
    int32_t local = 0;
#pragma unroll
    for (int u = 0; u < E; ++u) {
        my_len[u] = (sg[u] & kPairTag) ? 2 : (int32_t)(sg[u] & 0xFFFFFFull);
        local += my_len[u];
    }
    int32_t tot;
    int32_t run = block_exclusive_sum<BLOCK>(local, reinterpret_cast<int32_t*>(s_tmp), &tot);
#pragma unroll
    for (int u = 0; u < E; ++u) {
        int64_t cb = (int64_t)(sg[u] >> 24) - run;
        if (sg[u] & kPairTag) {
            const uint64_t read = (sg[u] ^ (uint64_t)(uint32_t)self) & 0xFFFFFFull;
            const uint64_t pos = ((sg[u] >> 24) ^ (uint64_t)(uint32_t)pv[u]) & 0x7FFFFFFFull;
            cb = kInlineBase - (int64_t)((pos << 24) | read);
        }
        c_base[(int)threadIdx.x * E + u] = cb;
        my_off[u] = run;
        run += my_len[u];
    }
    return tot;
}

// Writes the chunk index of every product of the window [w0, w1); the
// second product of a two-pair entry (its other pair) is flagged with bit 15.
template <int BLOCK>
__device__ __forceinline__ void walk_fill(uint16_t* tbuf, const int64_t* c_base, int32_t w0, int32_t w1,
                                          const int32_t (&my_off)[walk_chunk_of(BLOCK) / BLOCK],
                                          const int32_t (&my_len)[walk_chunk_of(BLOCK) / BLOCK]) {
    constexpr int E = walk_chunk_of(BLOCK) / BLOCK;
    static_assert(walk_chunk_of(BLOCK) <= 0x8000, "chunk index below the flag bit");
#pragma unroll
    for (int u = 0; u < E; ++u) {
        const int idx = (int)threadIdx.x * E + u;
        const int32_t a = max(my_off[u], w0), b = min(my_off[u] + my_len[u], w1);
        const int32_t second = c_base[idx] <= kInlineBelow ? my_off[u] + 1 : -1;
        for (int32_t q = a; q < b; ++q) tbuf[q - w0] = (uint16_t)(idx | (q == second ? 0x8000 : 0));
    }
}

// rf(tt, jp, cbase, qb) once per round: product u of the round (u < PER)
// is entry cbase + (tt[u] & 0x7FFF) of the row with pair jp[u] = (j, p_j)
// and number qb + u * BLOCK, or absent (tt[u] < 0).  self: the row's read.
// rval: the row's positions, loaded with the segments so that the other
// pair of a two-pair column comes with its position (without it that
// position reads wrong: for callers that use only j).  own: given, the
// row's own products come with their positions too (else 0).  PER: gathers
// per thread and round (a kernel short of registers takes fewer).
template <int BLOCK, int PER, class RF>
__device__ __forceinline__ void walk_rounds(const uint64_t* __restrict__ rseg, int L,
                                            const int2* __restrict__ at, int64_t* c_base, uint16_t* tbuf,
                                            int64_t* s_tmp, const int32_t* stop, int32_t self,
                                            const int32_t* __restrict__ rval, const int32_t* __restrict__ own,
                                            RF&& rf) {
    constexpr int CH = walk_chunk_of(BLOCK), WIN = walk_win_of(BLOCK);
    static_assert(CH % BLOCK == 0 && CH <= 65536, "chunk index kept in 16 bits");
    constexpr int E = walk_chunk_of(BLOCK) / BLOCK;
    static_assert(WIN % (PER * BLOCK) == 0, "whole gather rounds per window");
    int32_t done = 0;   // products of earlier chunks
    uint64_t sg[E];
    int32_t pv[E];
    walk_load<BLOCK>(rseg, rval, 0, min(CH, L), sg, pv);
    for (int cbase = 0; cbase < L; cbase += CH) {
        int32_t my_off[E], my_len[E];
        const int32_t tot = walk_chunk<BLOCK>(sg, pv, self, c_base, s_tmp, my_off, my_len);
        const int nbase = cbase + CH;
        walk_load<BLOCK>(rseg, rval, nbase, nbase < L ? min(CH, L - nbase) : 0, sg, pv);
        for (int32_t w0 = 0; w0 < tot; w0 += WIN) {
            const int32_t w1 = min(w0 + WIN, tot);
            walk_fill<BLOCK>(tbuf, c_base, w0, w1, my_off, my_len);
            __syncthreads();
            for (int32_t q0 = w0 + (int32_t)threadIdx.x; q0 < w1; q0 += BLOCK * PER) {
                if (stop && __hip_atomic_load(stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) break;
                // The round's LDS reads are issued together (indices clamped,
                // so that no branch separates them and one wait covers them),
                // then the pairs of two-pair columns are decoded, then the
                // gathers go out: a register that a load in flight targets is
                // never written by an instruction after that load.
                int tt[PER];
                int64_t cb[PER];
                int2 jp[PER];
#pragma unroll
                for (int u = 0; u < PER; ++u) {
                    const int32_t q = q0 + u * BLOCK;
                    const int tv = tbuf[min(q, w1 - 1) - w0];
                    tt[u] = q < w1 ? tv : -1;
                }
#pragma unroll
                for (int u = 0; u < PER; ++u) cb[u] = c_base[tt[u] < 0 ? 0 : (tt[u] & 0x7FFF)];
#pragma unroll
                for (int u = 0; u < PER; ++u)
                    if (tt[u] >= 0 && cb[u] <= kInlineBelow)
                        jp[u] = (tt[u] & 0x8000) ? inline_pair(cb[u])   // the column's other pair
                                                 : make_int2(self, own ? own[cbase + (tt[u] & 0x7FFF)] : 0);
#pragma unroll
                for (int u = 0; u < PER; ++u)
                    if (tt[u] >= 0 && cb[u] > kInlineBelow) jp[u] = at[cb[u] + q0 + u * BLOCK];
                rf(tt, jp, cbase, done + q0);
            }
            __syncthreads();
            if (stop && __hip_atomic_load(stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) break;
        }
        done += tot;
        if (tot == 0) __syncthreads();   // c_base is rewritten by the next chunk
        if (stop && __hip_atomic_load(stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) break;
    }
}

// f(t, (j, p_j), q) for every product, in turn (see walk_rounds).
template <int BLOCK, int PER = walk_per(BLOCK), class F>
__device__ __forceinline__ void walk_products(const uint64_t* __restrict__ rseg, int L,
                                              const int2* __restrict__ at, int64_t* c_base, uint16_t* tbuf,
                                              int64_t* s_tmp, const int32_t* stop, int32_t self,
                                              const int32_t* __restrict__ rval, const int32_t* __restrict__ own,
                                              F&& f) {
    walk_rounds<BLOCK, PER>(rseg, L, at, c_base, tbuf, s_tmp, stop, self, rval, own,
                            [&](const int (&tt)[PER], const int2 (&jp)[PER], int cbase, int32_t qb) {
#pragma unroll
                                for (int u = 0; u < PER; ++u) {
                                    if (tt[u] < 0) continue;
                                    f(cbase + (tt[u] & 0x7FFF), jp[u], (int64_t)(qb + u * BLOCK));
                                }
                            });
}

// ---------------------------------------------------------------------------
// Symbolic phase, bitmap path.  Per row: mark every product's j in the bit
// planes; the output columns are the set bits of plane min_shared - 1,
// written to the row's scratch range in increasing order.
// LDS: chunk arrays | planes x words u32.
// ---------------------------------------------------------------------------
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_ov_sym_bits(
    const OvSet* __restrict__ sets, int nsets, const int64_t* __restrict__ set_base,
    const int32_t* __restrict__ list, const uint64_t* __restrict__ seg, const int2* __restrict__ at,
    const int64_t* __restrict__ soff, int32_t* __restrict__ scratch, int64_t* __restrict__ nnzrow,
    int32_t* __restrict__ distinct, int32_t* __restrict__ qhead, int count) {
    extern __shared__ __align__(16) unsigned char smem[];
    int64_t* c_base = reinterpret_cast<int64_t*>(smem);
    uint16_t* tbuf = reinterpret_cast<uint16_t*>(c_base + walk_chunk_of(BLOCK));
    uint32_t* B = reinterpret_cast<uint32_t*>(smem + walk_lds(BLOCK));
    __shared__ int64_t s_tmp[BLOCK / kWave + 1];
    __shared__ int32_t s_item;
    for (int item = next_item(qhead, count, &s_item); item >= 0; item = next_item(qhead, count, &s_item)) {
    const int64_t g = list[item];
    const int s = find_set(set_base, nsets, g);
    const OvSet& S = sets[s];
    const int64_t i = g - S.row_base;
    const int64_t lo = S.a_rowptr[i];
    const int L = (int)(S.a_rowptr[i + 1] - lo);
    const int words = S.words;
    const int planes = S.min_shared;
    for (int q = threadIdx.x; q < planes * words; q += BLOCK) B[q] = 0u;
    __syncthreads();
    // the diagonal (j = i) is a product of every entry of the row: it is
    // left out of the walk (one LDS address hit by every segment) and set
    // from its closed form, count = L
    const int32_t self = (int32_t)(S.read_base + i);
    walk_products<BLOCK>(seg + S.nnz_base + lo, L, at, c_base, tbuf, s_tmp, nullptr, self, nullptr, nullptr,
                         [&](int, int2 jp, int64_t) {
                             if (jp.x != self) planes_mark(B, words, planes, jp.x);
                         });
    __syncthreads();
    if (threadIdx.x == 0)
        for (int p = 0; p < planes && p < L; ++p) B[p * words + (self >> 5)] |= 1u << (self & 31);
    __syncthreads();
    // one block scan: each thread owns a run of consecutive words and counts
    // the distinct columns (plane 0) in the high half and the output
    // columns (last plane) in the low half of one 64-bit value
    const uint32_t* out_plane = B + (planes - 1) * words;
    const int per = (words + BLOCK - 1) / BLOCK;
    const int w0 = (int)threadIdx.x * per, w1 = min(w0 + per, words);
    int64_t both = 0;
    for (int w = w0; w < w1; ++w) both += ((int64_t)__popc(B[w]) << 32) | (int64_t)__popc(out_plane[w]);
    int64_t tot;
    int64_t pos = block_exclusive_sum<BLOCK>(both, s_tmp, &tot) & 0xFFFFFFFFll;
    int32_t* out = scratch + soff[g];
    for (int w = w0; w < w1; ++w) {
        uint32_t bits = out_plane[w];
        while (bits) {
            const int b = __ffs(bits) - 1;
            out[pos++] = (w << 5) | b;
            bits &= bits - 1;
        }
    }
    if (threadIdx.x == 0) {
        nnzrow[g] = tot & 0xFFFFFFFFll;
        distinct[g] = (int32_t)(tot >> 32);
    }
    __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Symbolic phase, hash path.  Per row: count every j in an LDS hash table
// whose slot is one u64 = (j << 32) | count, then compact the entries with
// count >= min_shared to the front of the table, bitonic-sort them by j (the
// high word) and store the sorted columns in the row's scratch range.
// Work items come from `list` (count = *dcount if given, else hcount).  The
// first level uses a table sized for min(products, n) keys capped at a
// modest size; a row that exceeds the load limit is queued for the retry
// level (one large table per workgroup); at the retry level an overflowing
// row is marked for expand-sort-compress (distinct = -1).
// LDS: chunk arrays | T u64.
// ---------------------------------------------------------------------------
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_ov_sym_hash(
    const OvSet* __restrict__ sets, int nsets, const int64_t* __restrict__ set_base,
    const int32_t* __restrict__ list, const int32_t* __restrict__ dcount, int hcount, int T, int limit,
    int retry_level, int32_t* __restrict__ retry_list, const uint64_t* __restrict__ seg,
    const int2* __restrict__ at, const int64_t* __restrict__ soff, int32_t* __restrict__ scratch,
    int64_t* __restrict__ nnzrow, int32_t* __restrict__ distinct, OvCounters* __restrict__ ctr,
    int32_t* __restrict__ qhead) {
    extern __shared__ __align__(16) unsigned char smem[];
    int64_t* c_base = reinterpret_cast<int64_t*>(smem);
    uint16_t* tbuf = reinterpret_cast<uint16_t*>(c_base + walk_chunk_of(BLOCK));
    uint64_t* tab = reinterpret_cast<uint64_t*>(smem + walk_lds(BLOCK));
    __shared__ int64_t s_tmp[BLOCK / kWave + 1];
    __shared__ int32_t s_nd, s_ovf, s_item;
    const int items = dcount ? *dcount : hcount;
    for (int w = next_item(qhead, items, &s_item); w >= 0; w = next_item(qhead, items, &s_item)) {
        const int64_t g = list[w];
        const int s = find_set(set_base, nsets, g);
        const OvSet& S = sets[s];
        const int64_t i = g - S.row_base;
        const int64_t lo = S.a_rowptr[i];
        const int L = (int)(S.a_rowptr[i + 1] - lo);
        for (int q = threadIdx.x; q < T; q += BLOCK) tab[q] = kEmpty64;
        if (threadIdx.x == 0) {
            s_nd = 0;
            s_ovf = 0;
        }
        __syncthreads();
        const int32_t self = (int32_t)(S.read_base + i);
        walk_products<BLOCK>(seg + S.nnz_base + lo, L, at, c_base, tbuf, s_tmp, &s_ovf, self, nullptr, nullptr,
                             [&](int, int2 jp, int64_t) {
                                 if (jp.x == self) return;   // the diagonal: added once below
                                 int fresh;
                                 const int slot = table64_add(tab, (uint32_t)T, jp.x, &fresh);
                                 if (slot < 0) {
                                     s_ovf = 1;
                                     return;
                                 }
                                 if (fresh && atomicAdd(&s_nd, 1) + 1 > limit) s_ovf = 1;
                             });
        __syncthreads();
        if (threadIdx.x == 0 && !s_ovf && L > 0) {   // the diagonal, count L
            int fresh;
            const int slot = table64_add(tab, (uint32_t)T, self, &fresh, (uint32_t)L);
            if (slot < 0 || (fresh && ++s_nd > limit)) s_ovf = 1;
        }
        __syncthreads();
        if (s_ovf) {
            if (threadIdx.x == 0) {
                if (retry_level == 0) {
                    retry_list[atomicAdd(&ctr->retry_rows, 1)] = (int32_t)g;
                } else {
                    nnzrow[g] = 0;
                    distinct[g] = -1;
                    atomicAdd(&ctr->overflow_rows, 1);
                }
            }
            __syncthreads();
            continue;
        }
        // in-place compaction of the selected entries (each moves left)
        const uint32_t ms = (uint32_t)S.min_shared;
        int64_t nsel = 0;
        for (int c = 0; c < T; c += BLOCK) {
            const int q = c + threadIdx.x;
            const uint64_t v = q < T ? tab[q] : kEmpty64;
            const int64_t take = (v != kEmpty64 && (uint32_t)v >= ms) ? 1 : 0;
            int64_t tot;
            const int64_t ex = block_exclusive_sum<BLOCK>(take, s_tmp, &tot);   // barriers: all reads done
            if (take) tab[nsel + ex] = v;
            nsel += tot;
            __syncthreads();
        }
        int P = 1;
        while (P < nsel) P <<= 1;
        for (int q = (int)nsel + threadIdx.x; q < P; q += BLOCK) tab[q] = kEmpty64;
        __syncthreads();
        for (int k = 2; k <= P; k <<= 1) {
            for (int jj = k >> 1; jj > 0; jj >>= 1) {
                for (int idx = threadIdx.x; idx < P; idx += BLOCK) {
                    const int ixj = idx ^ jj;
                    if (ixj > idx) {
                        const uint64_t a = tab[idx], b = tab[ixj];
                        if ((a > b) == ((idx & k) == 0)) {
                            tab[idx] = b;
                            tab[ixj] = a;
                        }
                    }
                }
                __syncthreads();
            }
        }
        int32_t* out = scratch + soff[g];
        for (int r = threadIdx.x; r < nsel; r += BLOCK) out[r] = (int32_t)(tab[r] >> 32);
        if (threadIdx.x == 0) {
            nnzrow[g] = nsel;
            distinct[g] = s_nd;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Bins for the numeric phase by output size and path, ESC routing.
// ---------------------------------------------------------------------------
constexpr int kBinBlock = 256;

__global__ __launch_bounds__(kBinBlock) void k_ov_bin_numeric(
    const OvSet* __restrict__ sets, int nsets, const int64_t* __restrict__ set_base, int64_t total_rows,
    const int64_t* __restrict__ flops_row, const int32_t* __restrict__ distinct,
    const int64_t* __restrict__ nnzrow, int32_t* __restrict__ num_list, int32_t* __restrict__ esc_list,
    int64_t* __restrict__ esc_off, OvCounters* __restrict__ ctr, NumBins bins) {
    __shared__ int32_t s_cnt[kMaxBins + 1], s_base[kMaxBins + 1];   // last slot: ESC
    __shared__ unsigned long long s_flops;
    __shared__ int64_t s_flops_base;
    if (threadIdx.x <= kMaxBins) s_cnt[threadIdx.x] = 0;
    if (threadIdx.x == 0) s_flops = 0;
    __syncthreads();
    const int64_t g = blockIdx.x * (int64_t)kBinBlock + threadIdx.x;
    int b = -1, pos = 0;
    int64_t foff = 0;
    if (g < total_rows) {
        const int64_t fl = flops_row[g];
        const int64_t nz = nnzrow[g];
        const bool bits = sets[find_set(set_base, nsets, g)].use_bits;
        const int b0 = bits ? bins.nh : 0;
        const int b1 = bits ? bins.nh + bins.nb : bins.nh;
        if (fl > 0 && (distinct[g] < 0 || b1 == b0 || nz > bins.d[b1 - 1])) {
            b = kMaxBins;
            foff = (int64_t)atomicAdd(&s_flops, (unsigned long long)fl);
        } else if (nz > 0) {
            b = b0;
            while (bins.d[b] < nz) ++b;
        }
        if (b >= 0) pos = atomicAdd(&s_cnt[b], 1);
    }
    __syncthreads();
    if (threadIdx.x < kMaxBins && s_cnt[threadIdx.x] > 0)
        s_base[threadIdx.x] = atomicAdd(&ctr->num_count[threadIdx.x], s_cnt[threadIdx.x]);
    if (threadIdx.x == kMaxBins && s_cnt[kMaxBins] > 0) {
        s_base[kMaxBins] = atomicAdd(&ctr->esc_rows, s_cnt[kMaxBins]);
        s_flops_base = atomic_add(&ctr->esc_flops, (int64_t)s_flops);
    }
    __syncthreads();
    if (b == kMaxBins) {
        esc_list[s_base[b] + pos] = (int32_t)g;
        esc_off[g] = s_flops_base + foff;
    } else if (b >= 0) {
        num_list[(int64_t)b * total_rows + s_base[b] + pos] = (int32_t)g;
    }
}


// ---------------------------------------------------------------------------
// Numeric phase.  The row's output columns are its sorted list in scratch;
// one pass over the products counts every listed j and keeps its two
// smallest seed candidates (t << 32) | p_j, t = index of k in row i
// (monotone in k), with an atomicMin cascade (the value displaced from m1
// moves on to m2).  The rank r of a listed column j comes from
//   bitmap path: a bitmap of the listed columns and a per-word popcount
//                prefix: r = prefix[j / 32] + popcount(lower bits of word);
//   hash path:   a small LDS hash from j to r.
// LDS: chunk arrays | m1, m2 (D u64) | cnt (D i32) | map (bitmap path:
// u32 words, then a u16 rank prefix per word).
// ---------------------------------------------------------------------------
template <int BLOCK, bool BITS>
__global__ __launch_bounds__(BLOCK) void k_ov_numeric(
    const OvSet* __restrict__ sets, int nsets, const int64_t* __restrict__ set_base,
    const int32_t* __restrict__ list, int Dmax, int load_pct, const int64_t* __restrict__ nnzrow,
    const int64_t* __restrict__ soff, const int32_t* __restrict__ scratch, const uint64_t* __restrict__ seg,
    const int2* __restrict__ at, const int64_t* __restrict__ G, int words_max, int32_t* __restrict__ qhead,
    int count) {
    extern __shared__ __align__(16) unsigned char smem[];
    int64_t* c_base = reinterpret_cast<int64_t*>(smem);
    uint16_t* tbuf = reinterpret_cast<uint16_t*>(c_base + walk_chunk_of(BLOCK));
    uint64_t* m1 = reinterpret_cast<uint64_t*>(smem + walk_lds(BLOCK));
    uint64_t* m2 = m1 + Dmax;
    int32_t* cnt = reinterpret_cast<int32_t*>(m2 + Dmax);
    int32_t* map = cnt + Dmax;   // BITS: bitmap (words) + prefix (words); else keys (T) + rank (T)
    __shared__ int64_t s_tmp[BLOCK / kWave + 1];
    __shared__ int32_t s_item;
    // BITS: the bitmap is cleared once here; each row then clears only the
    // words of its own columns when it is done
    if (BITS) {
        uint32_t* bm0 = reinterpret_cast<uint32_t*>(cnt + Dmax);
        for (int q = threadIdx.x; q < words_max; q += BLOCK) bm0[q] = 0u;
    }
    for (int item = next_item(qhead, count, &s_item); item >= 0; item = next_item(qhead, count, &s_item)) {
    const int64_t g = list[item];
    const int s = find_set(set_base, nsets, g);
    const OvSet& S = sets[s];
    const int64_t i = g - S.row_base;
    const int64_t lo = S.a_rowptr[i];
    const int L = (int)(S.a_rowptr[i + 1] - lo);
    const int nsel = (int)nnzrow[g];
    const int32_t* sel = scratch + soff[g];
    const uint32_t T = BITS ? 0u : (uint32_t)table_slots(nsel, load_pct);
    uint32_t* bm = reinterpret_cast<uint32_t*>(map);
    uint16_t* pre = reinterpret_cast<uint16_t*>(map + words_max);   // ranks < num_max_entries <= 8192
    int32_t* keys = map;
    int32_t* rank = map + T;
    if (!BITS) {
        for (uint32_t q = threadIdx.x; q < T; q += BLOCK) keys[q] = -1;
        __syncthreads();
    }
    for (int r = threadIdx.x; r < nsel; r += BLOCK) {
        const int32_t j = sel[r];
        if (BITS) {
            // sel is sorted: the first listed column of a word has the
            // word's smallest rank, so no scan over the words is needed
            atomicOr(&bm[j >> 5], 1u << (j & 31));
            if (r == 0 || (sel[r - 1] >> 5) != (j >> 5)) pre[j >> 5] = (uint16_t)r;
        } else {
            const int slot = table_insert(keys, T, j);
            if (slot >= 0) rank[slot] = r;
        }
        cnt[r] = 0;
        m1[r] = kEmpty64;
        m2[r] = kEmpty64;
    }
    __syncthreads();
    const int32_t self = (int32_t)(S.read_base + i);   // the diagonal is written from its closed form below
    // four gathers per round: eight would take the registers of half the
    // workgroups.  A round's products first look up their output ranks and
    // the current second seeds (LDS reads only, issued together), then count
    // and update the seeds.
    constexpr int NP = 4;
    walk_rounds<BLOCK, NP>(seg + S.nnz_base + lo, L, at, c_base, tbuf, s_tmp, nullptr, self, S.a_val + lo,
                           nullptr, [&](const int (&tt)[NP], const int2 (&jp)[NP], int cbase, int32_t) {
        // (the reads are unconditional, at index 0 for an absent product, so
        // that no branch keeps them apart)
        int r[NP];
#pragma unroll
        for (int u = 0; u < NP; ++u) {
            const bool live = tt[u] >= 0 && jp[u].x != self;
            const int32_t j = live ? jp[u].x : 0;
            if (BITS) {
                const uint32_t word = bm[j >> 5];
                const uint32_t bit = 1u << (j & 31);
                const int p = (int)pre[j >> 5];
                r[u] = (live && (word & bit)) ? p + __popc(word & (bit - 1u)) : -1;
            } else {
                r[u] = -1;
                if (live) {
                    const int slot = table_find(keys, T, j);
                    if (slot >= 0) r[u] = rank[slot];
                }
            }
        }
        uint64_t cur[NP];
#pragma unroll
        for (int u = 0; u < NP; ++u)
            cur[u] = __hip_atomic_load(&m2[r[u] < 0 ? 0 : r[u]], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
#pragma unroll
        for (int u = 0; u < NP; ++u) {
            if (r[u] < 0) continue;
            atomicAdd(&cnt[r[u]], 1);
            const uint64_t x = ((uint64_t)(uint32_t)(cbase + (tt[u] & 0x7FFF)) << 32) | (uint64_t)(uint32_t)jp[u].y;
            // m2 only decreases: a candidate above it (here, above a value it
            // held earlier in the round) can never be one of the two smallest
            // (all candidates of a column differ in t), so most products
            // skip the cascade
            if (x > cur[u]) continue;
            const uint64_t old = atomicMin(&m1[r[u]], x);
            const uint64_t rej = old > x ? old : x;
            if (rej != kEmpty64) atomicMin(&m2[r[u]], rej);
        }
    });
    __syncthreads();
    const int64_t off = G[g] - G[S.row_base];
    int4* seed4 = reinterpret_cast<int4*>(S.c_seed);
    for (int r = threadIdx.x; r < nsel; r += BLOCK) {
        const int32_t j = sel[r];
        int32_t c, pi0, pj0, pi1 = -1, pj1 = -1;
        if (j == self) {
            // C_ii: every entry of the row pairs with itself; the seeds are
            // its first two entries
            c = L;
            pi0 = pj0 = S.a_val[lo];
            if (L >= 2) pi1 = pj1 = S.a_val[lo + 1];
        } else if (m1[r] == kEmpty64) {
            // a listed column always has a candidate; never index with the sentinel
            c = cnt[r];
            pi0 = pj0 = -1;
        } else {
            const uint64_t a = m1[r], b = m2[r];
            c = cnt[r];
            pi0 = S.a_val[lo + (int64_t)(a >> 32)];
            pj0 = (int32_t)(uint32_t)a;
            if (b != kEmpty64) {
                pi1 = S.a_val[lo + (int64_t)(b >> 32)];
                pj1 = (int32_t)(uint32_t)b;
            }
        }
        S.c_col[off + r] = j;
        S.c_count[off + r] = c;
        seed4[off + r] = make_int4(pi0, pj0, pi1, pj1);
        if (BITS) bm[j >> 5] = 0u;   // every read of the bitmap is done (barrier after the walk)
    }
    __syncthreads();
    }
}

__global__ void k_ov_set_totals(const OvSet* __restrict__ sets, int nsets, const int64_t* __restrict__ G,
                                int64_t* __restrict__ set_nnz) {
    for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < nsets; s += gridDim.x * blockDim.x) {
        const OvSet& S = sets[s];
        set_nnz[s] = G[S.row_base + S.n] - G[S.row_base];
    }
}

__global__ void k_ov_write_rowptr(const OvSet* __restrict__ sets, int nsets,
                                  const int64_t* __restrict__ set_base, int64_t total_rows,
                                  const int64_t* __restrict__ G) {
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < total_rows + nsets;
         g += (int64_t)gridDim.x * blockDim.x) {
        if (g < total_rows) {
            const int s = find_set(set_base, nsets, g);
            const OvSet& S = sets[s];
            S.c_rowptr[g - S.row_base] = G[g] - G[S.row_base];
        } else {
            const OvSet& S = sets[g - total_rows];
            S.c_rowptr[S.n] = G[S.row_base + S.n] - G[S.row_base];
        }
    }
}

// ---------------------------------------------------------------------------
// ESC (expand - sort - compress) for rows too dense for an LDS table.
// ---------------------------------------------------------------------------
constexpr int kEscBlock = 256;

__global__ __launch_bounds__(kEscBlock) void k_esc_expand(
    const OvSet* __restrict__ sets, int nsets, const int64_t* __restrict__ set_base,
    const int32_t* __restrict__ list, const int64_t* __restrict__ esc_off, const uint64_t* __restrict__ seg,
    const int2* __restrict__ at, uint32_t* __restrict__ keys0, uint64_t* __restrict__ pay0) {
    static_assert(walk_chunk_of(kEscBlock) == kWalkChunk && walk_win_of(kEscBlock) == kWalkWin, "walk area");
    __shared__ int64_t c_base[kWalkChunk];
    __shared__ uint16_t tbuf[kWalkWin];
    __shared__ int64_t s_tmp[kEscBlock / kWave + 1];
    const int64_t g = list[blockIdx.x];
    const int s = find_set(set_base, nsets, g);
    const OvSet& S = sets[s];
    const int64_t i = g - S.row_base;
    const int64_t lo = S.a_rowptr[i];
    const int L = (int)(S.a_rowptr[i + 1] - lo);
    const int64_t base = esc_off[g];
    // products land at their t-major index, so the expansion is ordered by k
    walk_products<kEscBlock>(seg + S.nnz_base + lo, L, at, c_base, tbuf, s_tmp, nullptr, (int32_t)(S.read_base + i),
                             S.a_val + lo, S.a_val + lo, [&](int t, int2 jp, int64_t q) {
                                 keys0[base + q] = (uint32_t)jp.x;
                                 pay0[base + q] = ((uint64_t)(uint32_t)t << 32) | (uint64_t)(uint32_t)jp.y;
                             });
}

// Stable LSD radix sort (8-bit digits) of one row's expanded products by j.
__global__ __launch_bounds__(kEscBlock) void k_esc_sort(
    const OvSet* __restrict__ sets, int nsets, const int64_t* __restrict__ set_base,
    const int32_t* __restrict__ list, const int64_t* __restrict__ esc_off,
    const int64_t* __restrict__ flops_row, uint32_t* __restrict__ keys0, uint64_t* __restrict__ pay0,
    uint32_t* __restrict__ keys1, uint64_t* __restrict__ pay1) {
    constexpr int W = kEscBlock / kWave;
    __shared__ int32_t hist[256];
    __shared__ int32_t base_d[256];
    __shared__ int32_t wcnt[W][256];
    __shared__ int32_t wpre[W][256];
    __shared__ int32_t s_tmp[W + 1];
    const int64_t g = list[blockIdx.x];
    const int s = find_set(set_base, nsets, g);
    const int bits = sets[s].id_bits;
    const int64_t base = esc_off[g];
    const int64_t F = flops_row[g];
    uint32_t* ka = keys0 + base;
    uint64_t* pa = pay0 + base;
    uint32_t* kb = keys1 + base;
    uint64_t* pb = pay1 + base;
    const int w = wave_id();
    const int tid = threadIdx.x;
    const int passes = (bits + 7) / 8;
    for (int pass = 0; pass < passes; ++pass) {
        const int shift = 8 * pass;
        hist[tid] = 0;
        for (int q = 0; q < W; ++q) wcnt[q][tid] = 0;
        __syncthreads();
        for (int64_t e = tid; e < F; e += kEscBlock) atomicAdd(&hist[(ka[e] >> shift) & 255u], 1);
        __syncthreads();
        int32_t tot;
        const int32_t ex = block_exclusive_sum<kEscBlock>(hist[tid], s_tmp, &tot);
        base_d[tid] = ex;
        __syncthreads();
        for (int64_t tile = 0; tile < F; tile += kEscBlock) {
            const int64_t e = tile + tid;
            const bool valid = e < F;
            const uint32_t key = valid ? ka[e] : 0u;
            const uint64_t pay = valid ? pa[e] : 0ull;
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
                int32_t acc = base_d[tid];
                for (int q = 0; q < W; ++q) {
                    wpre[q][tid] = acc;
                    acc += wcnt[q][tid];
                    wcnt[q][tid] = 0;
                }
                base_d[tid] = acc;
            }
            __syncthreads();
            if (valid) {
                const int32_t pos = wpre[w][d] + rank;
                kb[pos] = key;
                pb[pos] = pay;
            }
            __syncthreads();
        }
        uint32_t* tk = ka; ka = kb; kb = tk;
        uint64_t* tp = pa; pa = pb; pb = tp;
    }
    if (passes & 1) {  // result sits in the second buffer: move it back
        for (int64_t e = tid; e < F; e += kEscBlock) {
            keys0[base + e] = ka[e];
            pay0[base + e] = pa[e];
        }
    }
}

// Runs of equal keys in one sorted ESC row, tile by tile: each element learns
// the start of its run from an inclusive max-scan of start positions (carried
// across tiles); the run's last element then knows its length.
template <int BLOCK>
__device__ __forceinline__ int64_t block_inclusive_max(int64_t v, int64_t* tmp) {
    constexpr int W = BLOCK / kWave;
    const int lane = lane_id(), w = wave_id();
    for (int d = 1; d < kWave; d <<= 1) {
        const int64_t y = __shfl_up(v, d, kWave);
        if (lane >= d) v = y > v ? y : v;
    }
    if (lane == kWave - 1) tmp[w] = v;
    __syncthreads();
    int64_t pre = -1;
    for (int q = 0; q < w; ++q) pre = tmp[q] > pre ? tmp[q] : pre;
    __syncthreads();
    (void)W;
    return v > pre ? v : pre;
}

__global__ __launch_bounds__(kEscBlock) void k_esc_count(
    const OvSet* __restrict__ sets, int nsets, const int64_t* __restrict__ set_base,
    const int32_t* __restrict__ list, const int64_t* __restrict__ esc_off,
    const int64_t* __restrict__ flops_row, const uint32_t* __restrict__ keys0,
    int64_t* __restrict__ nnzrow, int32_t* __restrict__ distinct) {
    __shared__ int64_t s_tmp[kEscBlock / kWave + 1];
    __shared__ int64_t s_red, s_last;
    const int64_t g = list[blockIdx.x];
    const int s = find_set(set_base, nsets, g);
    const int32_t ms = sets[s].min_shared;
    const uint32_t* k = keys0 + esc_off[g];
    const int64_t F = flops_row[g];
    int64_t runs = 0, sel = 0, carry = -1;
    for (int64_t tile = 0; tile < F; tile += kEscBlock) {
        const int64_t e = tile + threadIdx.x;
        const bool in = e < F;
        const bool start = in && (e == 0 || k[e] != k[e - 1]);
        const bool end = in && (e == F - 1 || k[e + 1] != k[e]);
        int64_t st = block_inclusive_max<kEscBlock>(start ? e : -1, s_tmp);
        st = st > carry ? st : carry;
        if (end) {
            ++runs;
            if (e - st + 1 >= ms) ++sel;
        }
        if (threadIdx.x == kEscBlock - 1) s_last = st;
        __syncthreads();
        carry = s_last;
        __syncthreads();
    }
    runs = block_sum_lds(runs, &s_red);
    sel = block_sum_lds(sel, &s_red);
    if (threadIdx.x == 0) {
        nnzrow[g] = sel;
        distinct[g] = (int32_t)(runs < 0x7fffffff ? runs : 0x7fffffff);
    }
}

__global__ __launch_bounds__(kEscBlock) void k_esc_emit(
    const OvSet* __restrict__ sets, int nsets, const int64_t* __restrict__ set_base,
    const int32_t* __restrict__ list, const int64_t* __restrict__ esc_off,
    const int64_t* __restrict__ flops_row, const uint32_t* __restrict__ keys0,
    const uint64_t* __restrict__ pay0, const int64_t* __restrict__ G) {
    __shared__ int64_t s_tmp[kEscBlock / kWave + 1];
    __shared__ int64_t s_last;
    const int64_t g = list[blockIdx.x];
    const int s = find_set(set_base, nsets, g);
    const OvSet& S = sets[s];
    const int64_t i = g - S.row_base;
    const int64_t lo = S.a_rowptr[i];
    const uint32_t* k = keys0 + esc_off[g];
    const uint64_t* p = pay0 + esc_off[g];
    const int64_t F = flops_row[g];
    const int64_t off0 = G[g] - G[S.row_base];
    int4* seed4 = reinterpret_cast<int4*>(S.c_seed);
    int64_t carry = -1, written = 0;
    for (int64_t tile = 0; tile < F; tile += kEscBlock) {
        const int64_t e = tile + threadIdx.x;
        const bool in = e < F;
        const bool start = in && (e == 0 || k[e] != k[e - 1]);
        const bool end = in && (e == F - 1 || k[e + 1] != k[e]);
        int64_t st = block_inclusive_max<kEscBlock>(start ? e : -1, s_tmp);
        st = st > carry ? st : carry;
        const int64_t rl = end ? e - st + 1 : 0;
        const int64_t take = (end && rl >= S.min_shared) ? 1 : 0;
        int64_t tot;
        const int64_t ex = block_exclusive_sum<kEscBlock>(take, s_tmp, &tot);
        if (take) {
            const int64_t o = off0 + written + ex;
            const uint64_t a = p[st];
            int32_t pi1 = -1, pj1 = -1;
            if (rl >= 2) {
                const uint64_t b = p[st + 1];
                pi1 = S.a_val[lo + (int64_t)(b >> 32)];
                pj1 = (int32_t)(uint32_t)b;
            }
            S.c_col[o] = (int32_t)k[e];
            S.c_count[o] = (int32_t)rl;
            seed4[o] = make_int4(S.a_val[lo + (int64_t)(a >> 32)], (int32_t)(uint32_t)a, pi1, pj1);
        }
        written += tot;
        if (threadIdx.x == kEscBlock - 1) s_last = st;
        __syncthreads();
        carry = s_last;
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Host driver
// ---------------------------------------------------------------------------
// Dynamic LDS budget per workgroup: the 160 KB of a gfx950 CU minus room
// for the kernels' static LDS.
constexpr size_t kLdsLimit = 158 * 1024;

static size_t sym_hash_lds(int block, int T) { return walk_lds(block) + (size_t)T * 8; }
static size_t sym_bits_lds(int block, int planes, int words) {
    return walk_lds(block) + (size_t)planes * words * 4;
}
// Numeric LDS for rows with at most D output entries: chunk arrays,
// m1/m2/cnt, and the column map (bitmap + prefix, or hash keys + ranks).
static size_t num_lds(int block, int D, int load_pct, bool bits, int words) {
    // bitmap path: u32 bitmap words + u16 rank prefixes; hash path: keys + ranks
    const size_t map = bits ? (((size_t)words * 6 + 7) & ~(size_t)7) : (size_t)table_slots(D, load_pct) * 8;
    return walk_lds(block) + (size_t)D * 20 + map;
}

// Workgroup width for a launch whose LDS footprint is `lds` at 256 threads:
// few workgroups fit a CU when the footprint is large, so those get more
// threads (more loads in flight per CU).
static int wide_block(int base, size_t lds) {
    if (lds > 80 * 1024) return 1024;
    if (lds > 40 * 1024) return std::max(base, 512);
    return base;
}

// A launch asking for more LDS than a workgroup may hold is refused here.
static int check_lds(size_t lds) {
    if (lds > kLdsLimit) {
        set_error("internal: launch needs " + std::to_string(lds) + " bytes of LDS");
        return DIBELLA_EDEVICE;
    }
    return DIBELLA_OK;
}

template <int BLOCK>
static int allow_lds_ov() {
    // the attribute calls are idempotent: threads racing here may both make them
    static std::atomic<bool> done{false};
    if (!done.load(std::memory_order_acquire)) {
        DB_HIP(hipFuncSetAttribute((const void*)k_ov_sym_hash<BLOCK>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)kLdsLimit));
        DB_HIP(hipFuncSetAttribute((const void*)k_ov_sym_bits<BLOCK>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)kLdsLimit));
        DB_HIP(hipFuncSetAttribute((const void*)k_ov_numeric<BLOCK, true>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsLimit));
        DB_HIP(hipFuncSetAttribute((const void*)k_ov_numeric<BLOCK, false>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsLimit));
        done.store(true, std::memory_order_release);
    }
    return DIBELLA_OK;
}

struct OvWork {   // device arrays shared by the launches of one call
    const OvSet* d_sets;
    int nsets;
    const int64_t* d_base;
    int32_t* retry_list;
    const uint64_t* seg;
    const int2* at;
    const int64_t* soff;
    int32_t* scratch;
    int64_t* nnzrow;
    int32_t* distinct;
    OvCounters* ctr;
    const int64_t* G;
};

struct SymArgs {
    const int32_t* list;
    const int32_t* dcount;
    int hcount, grid, T, limit, level, queue;
};

// Workgroups of a persistent launch: what fits the GPU at once (LDS and
// waves per CU), never more than the items.
static int persistent_grid(int count, int block, size_t lds) {
    static std::atomic<int> cus_cached{0};
    int cus = cus_cached.load(std::memory_order_relaxed);
    if (!cus) {
        int dev = 0;
        hipDeviceProp_t prop;
        cus = (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
                  ? prop.multiProcessorCount
                  : 256;
        cus_cached.store(cus, std::memory_order_relaxed);
    }
    const int by_lds = (int)std::max<size_t>(1, (160 * 1024) / (lds + 1024));
    const int by_waves = std::max(1, 2048 / block);
    const int64_t g = (int64_t)cus * std::min(by_lds, by_waves);
    return (int)std::max<int64_t>(1, std::min<int64_t>(count, g));
}

template <int BLOCK>
static int launch_sym_hash(const OvWork& W, const SymArgs& a, hipStream_t st) {
    DB_TRY(allow_lds_ov<BLOCK>());
    const size_t lds = sym_hash_lds(BLOCK, a.T);
    DB_TRY(check_lds(lds));
    const int grid = a.dcount ? a.grid : persistent_grid(a.hcount, BLOCK, lds);
    hipLaunchKernelGGL(k_ov_sym_hash<BLOCK>, dim3(grid), dim3(BLOCK), lds, st, W.d_sets,
                       W.nsets, W.d_base, a.list, a.dcount, a.hcount, a.T, a.limit, a.level, W.retry_list, W.seg,
                       W.at, W.soff, W.scratch, W.nnzrow, W.distinct, W.ctr, &W.ctr->qhead[a.queue]);
    DB_HIP(hipGetLastError());
    return DIBELLA_OK;
}

template <int BLOCK>
static int launch_sym_bits(const OvWork& W, const int32_t* list, int count, int planes, int words,
                           hipStream_t st) {
    DB_TRY(allow_lds_ov<BLOCK>());
    const size_t lds = sym_bits_lds(BLOCK, planes, words);
    DB_TRY(check_lds(lds));
    hipLaunchKernelGGL(k_ov_sym_bits<BLOCK>, dim3(persistent_grid(count, BLOCK, lds)), dim3(BLOCK), lds, st,
                       W.d_sets, W.nsets, W.d_base, list, W.seg, W.at, W.soff, W.scratch, W.nnzrow, W.distinct,
                       &W.ctr->qhead[kQSymBits], count);
    DB_HIP(hipGetLastError());
    return DIBELLA_OK;
}

template <int BLOCK>
static int launch_numeric(const OvWork& W, const int32_t* list, int count, int D, int load_pct, bool bits,
                          int words, int queue, hipStream_t st) {
    DB_TRY(allow_lds_ov<BLOCK>());
    const size_t lds = num_lds(BLOCK, D, load_pct, bits, words);
    DB_TRY(check_lds(lds));
    const int grid = persistent_grid(count, BLOCK, lds);
    int32_t* qh = &W.ctr->qhead[queue];
    if (bits)
        hipLaunchKernelGGL((k_ov_numeric<BLOCK, true>), dim3(grid), dim3(BLOCK), lds, st, W.d_sets, W.nsets,
                           W.d_base, list, D, load_pct, W.nnzrow, W.soff, W.scratch, W.seg, W.at, W.G, words, qh,
                           count);
    else
        hipLaunchKernelGGL((k_ov_numeric<BLOCK, false>), dim3(grid), dim3(BLOCK), lds, st, W.d_sets, W.nsets,
                           W.d_base, list, D, load_pct, W.nnzrow, W.soff, W.scratch, W.seg, W.at, W.G, 0, qh,
                           count);
    DB_HIP(hipGetLastError());
    return DIBELLA_OK;
}

#define DB_DISPATCH_BLOCK(block, fn, ...)                          \
    switch (block) {                                               \
        case 64: return fn<64>(__VA_ARGS__);                       \
        case 128: return fn<128>(__VA_ARGS__);                     \
        case 512: return fn<512>(__VA_ARGS__);                     \
        case 1024: return fn<1024>(__VA_ARGS__);                   \
        default: return fn<256>(__VA_ARGS__);                      \
    }

static int dispatch_sym_hash(int block, const OvWork& W, const SymArgs& a, hipStream_t st) {
    DB_DISPATCH_BLOCK(block, launch_sym_hash, W, a, st);
}
static int dispatch_sym_bits(int block, const OvWork& W, const int32_t* list, int count, int planes, int words,
                             hipStream_t st) {
    DB_DISPATCH_BLOCK(block, launch_sym_bits, W, list, count, planes, words, st);
}
static int dispatch_numeric(int block, const OvWork& W, const int32_t* list, int count, int D, int load_pct,
                            bool bits, int words, int queue, hipStream_t st) {
    DB_DISPATCH_BLOCK(block, launch_numeric, W, list, count, D, load_pct, bits, words, queue, st);
}

// Numeric bin bounds that fit the LDS: hash bins, then bitmap bins for a
// bitmap of `words` words (none if words == 0).
static NumBins numeric_bins(const dibella_tuning& tn, int words) {
    // few, wide bins: each bin is one launch, and launches cost a tail each
    static const int bounds[] = {256, 1024, 2048, 4096, 8192};
    NumBins b;
    std::memset(&b, 0, sizeof(b));
    int k = 0;   // next free entry of b.d
    for (int pass = 0; pass < 2; ++pass) {
        const bool bits = pass == 1;
        if (bits && words == 0) break;
        int n = 0, last = 0;
        for (int d : bounds) {
            if (d > tn.num_max_entries) break;
            if (num_lds(1024, d, tn.load_pct, bits, words) > kLdsLimit) break;
            b.d[k++] = d;
            ++n;
            last = d;
        }
        if (tn.num_max_entries > last && num_lds(1024, tn.num_max_entries, tn.load_pct, bits, words) <= kLdsLimit) {
            b.d[k++] = tn.num_max_entries;
            ++n;
        }
        if (bits) b.nb = n; else b.nh = n;
    }
    return b;
}

static const char* describe_bad(int32_t bad) {
    if (bad & kBadRowptr) return "row pointers are not a valid CSR row pointer array";
    if (bad & kBadCol) return "a column index is outside [0, ncols)";
    if (bad & kUnsorted) return "columns are not strictly increasing within a row";
    if (bad & kNegative) return "a position value is negative";
    if (bad & kLongRow) return "a row has 2^30 or more entries";
    return "malformed matrix";
}

// Host layout of a call's sets: checked sizes, global row, column and entry
// bases, and the largest bitmap over the bitmap-path sets.
struct OvLayout {
    std::vector<OvSet> hs;
    std::vector<int64_t> base;   // first global row of each set, then the total
    int64_t total_rows = 0, total_m = 0, total_nnz = 0;
    int bits_words = 0, bits_planes = 0;
};

// Whether a set of n reads takes the bitmap path.
static int32_t use_bits_for(int64_t nreads, int32_t min_shared, const dibella_tuning& tn) {
    const int32_t words = (int32_t)((nreads + 31) / 32);
    return (min_shared <= kMaxPlanes && words <= tn.bits_max_words &&
            sym_bits_lds(1024, min_shared, words) <= kLdsLimit)
               ? 1
               : 0;
}

static int ov_layout(const dibella_csr* A, int nsets, const int32_t* min_shared, const dibella_tuning& tn,
                     OvLayout& L) {
    L.hs.assign(nsets, OvSet{});
    L.base.assign(nsets + 1, 0);
    for (int s = 0; s < nsets; ++s) {
        const dibella_csr& a = A[s];
        if (a.nrows < 0 || a.ncols < 0 || a.nnz < 0) {
            set_error("set " + std::to_string(s) + ": negative size");
            return DIBELLA_EINVAL;
        }
        if (min_shared[s] < 1) {
            set_error("set " + std::to_string(s) + ": min_shared must be >= 1");
            return DIBELLA_EINVAL;
        }
        if (a.nrows >= (int64_t(1) << 24) || a.nnz >= (int64_t(1) << 40) ||
            a.ncols >= (int64_t(1) << 40)) {
            set_error("set " + std::to_string(s) + ": nrows must be < 2^24 and nnz, ncols < 2^40");
            return DIBELLA_EOVERFLOW;
        }
        if ((a.nrows > 0 && !a.rowptr) || (a.nnz > 0 && (!a.col || !a.val))) {
            set_error("set " + std::to_string(s) + ": null pointer");
            return DIBELLA_EINVAL;
        }
        if (a.nrows == 0 && a.nnz != 0) {
            set_error("set " + std::to_string(s) + ": entries in a matrix without rows");
            return DIBELLA_EINVAL;
        }
        OvSet& o = L.hs[s];
        std::memset(&o, 0, sizeof(o));
        o.a_rowptr = a.rowptr;
        o.a_col = a.col;
        o.a_val = a.val;
        o.n = a.nrows;
        o.m = a.ncols;
        o.nnz = a.nnz;
        o.row_base = L.total_rows;
        o.col_base = L.total_m;
        o.nnz_base = L.total_nnz;
        o.read_base = 0;
        o.nreads = a.nrows;
        o.min_shared = min_shared[s];
        o.id_bits = std::max(1, ceil_log2_i64(std::max<int64_t>(a.nrows, 2)));
        o.words = (int32_t)((a.nrows + 31) / 32);
        o.use_bits = use_bits_for(a.nrows, min_shared[s], tn);
        if (o.use_bits) {
            L.bits_words = std::max(L.bits_words, o.words);
            L.bits_planes = std::max(L.bits_planes, (int)o.min_shared);
        }
        L.base[s] = L.total_rows;
        L.total_rows += a.nrows;
        L.total_m += a.ncols;
        L.total_nnz += a.nnz;
    }
    L.base[nsets] = L.total_rows;
    if (L.total_rows >= (int64_t(1) << 31) || L.total_nnz >= (int64_t(1) << 32) ||
        L.total_m >= (int64_t(1) << 32)) {
        set_error("batch too large: total rows must be < 2^31, total columns and total nnz < 2^32");
        return DIBELLA_EOVERFLOW;
    }
    return DIBELLA_OK;
}

// Column slices for the segment pass: 8 per round, each at most kSliceCols
// columns wide; only where the column records outgrow an L2 and the slice
// tables ((2S + 1) int32 per row) stay within max(4 nnz, 2^24) entries
// (total_nnz < 2^31 keeps a workgroup's flat entry numbers in 32 bits).
static SliceMap slice_plan(int64_t total_m, int64_t total_rows, int64_t total_nnz) {
    SliceMap sm{0, 0u};
    const int64_t S = ceil_div(total_m, 8 * kSliceCols) * 8;
    if (total_rows > 0 && total_nnz > 0 && total_nnz < (int64_t(1) << 31) && total_m >= 4 * kSliceCols &&
        S <= kMaxSlices && (2 * S + 1) * total_rows <= std::max<int64_t>(4 * total_nnz, int64_t(1) << 24)) {
        sm.count = (int32_t)S;
        sm.mul = (uint32_t)(((uint64_t)S << 32) / (uint64_t)total_m);
    }
    return sm;
}

// A^T of a call's sets and the slice table of their rows: what the row
// phases read.
struct OvTransposed {
    const uint64_t* rec = nullptr;   // per column: its record (at least one slot)
    const int2* at = nullptr;        // A^T pairs (read, position), column by column
    const int32_t* bnd = nullptr;    // slice boundaries of every row, slice-major
    int64_t bnd_stride = 0;          // rows per slice in bnd
    SliceMap sm{0, 0u};
    const int32_t* d_flags = nullptr;   // per set: the validation flags k_ov_keys raised
    int nsets = 0;
};

// Bucketed counting sort of N pairs by key (column in [0, M)): keys_a /
// pays_a hold them; keys_b / pays_b are the partition passes' second
// buffers.  Writes A^T to at_dest (the range's first slot; it may be pays_a
// for a two-level sort or pays_b for a three-level one, the buffer the last
// pass does not read) and every column's record to rec[0, M), starts
// counted from rec_base.  Two levels (partition the pairs into buckets of
// 2^low columns, then a staged counting sort per bucket) while the buckets
// fit one partition; three levels beyond that (partition into segments of
// 2^lowc columns, partition every segment into buckets of 2^12 columns,
// staged sort per bucket), so that every bucket is sorted in staged sweeps
// with 16-bit keys and its two-pair columns carry their pairs.  Tables come
// from `scr`.
struct SortPlan {
    int low, lowc, fine_per, per_block;
    bool three;
    int64_t nbuckets, nsort, nchunks, npart, nchunks2, ncount2;
};

static SortPlan sort_plan(int64_t M, int64_t N) {
    SortPlan P{};
    const int col_bits = ceil_log2_i64(std::max<int64_t>(M, 2));
    // buckets of at most 2^13 columns: the last level then sorts each in two
    // staged sweeps (2^14 took four sweeps, each re-reading the bucket's
    // keys, and left a half-empty last round of workgroups on mid)
    P.low = std::min(kTwoLevelLow, std::max(10, col_bits - 8));
    P.three = ceil_div(M, int64_t(1) << kTwoLevelLow) > kMaxBuckets;
    P.lowc = kCoarseLow;
    if (P.three) {
        P.low = kStageBits;
        while (ceil_div(M, int64_t(1) << P.lowc) > kMaxBuckets) ++P.lowc;
    }
    P.fine_per = P.three ? 1 << (P.lowc - P.low) : 0;                          // buckets per segment
    P.nbuckets = ceil_div(M, int64_t(1) << (P.three ? P.lowc : P.low));       // first level
    P.nsort = ceil_div(M, int64_t(1) << P.low);                               // sorted by the last level
    P.nchunks = ceil_div(N, kChunk);
    // A first-level workgroup takes several chunks when that keeps the
    // (bucket, workgroup) count table small beside A.
    P.per_block = 1;
    while (P.nbuckets * ceil_div(P.nchunks, P.per_block) > std::max<int64_t>(int64_t(1) << 22, N / 8))
        P.per_block *= 2;
    P.npart = ceil_div(P.nchunks, P.per_block);   // first-level workgroups
    // second level: one chunk per workgroup, segments cut separately (at
    // most one partial chunk per segment)
    P.nchunks2 = P.three ? P.nchunks + P.nbuckets : 0;
    P.ncount2 = P.nchunks2 * P.fine_per;
    return P;
}

// Bytes of the tables sort_pairs takes from its arena (plus the keys and
// pairs buffers: 2 * 4 + 2 * 8 per pair, counted by the caller).
static size_t sort_table_bytes(const SortPlan& P) {
    auto pad = [](size_t b) { return Arena::padded(b); };
    size_t est = pad(4 * P.nbuckets * P.npart) + pad(8 * (P.nbuckets * P.npart + 1));
    if (P.three)
        est += pad(4 * P.ncount2) + pad(8 * (P.ncount2 + 1)) + 2 * pad(8 * (P.nbuckets + 1)) +
               pad(8 * (P.nbuckets * P.fine_per + 1));
    est += 2 * pad(8 * scan_workspace_elems(std::max({P.nbuckets * P.npart, P.ncount2, int64_t(1)}))) +
           8 * Arena::padded(1);
    return est;
}

static int sort_pairs(const SortPlan& P, int64_t M, int64_t N, uint32_t* keys_a, uint32_t* keys_b, uint64_t* pays_a,
                      uint64_t* pays_b, uint64_t* at_dest, uint64_t* rec, int64_t rec_base, Arena& scr) {
    hipStream_t st = scr.stream();
    if (N == 0) return DIBELLA_OK;
    int tok = -1;
    static std::atomic<bool> lds_ok{false};
    if (!lds_ok.load(std::memory_order_acquire)) {
        DB_HIP(hipFuncSetAttribute((const void*)k_ov_part_scatter<false, uint16_t>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsLimit));
        DB_HIP(hipFuncSetAttribute((const void*)k_ov_part_scatter<false, uint32_t>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsLimit));
        DB_HIP(hipFuncSetAttribute((const void*)k_ov_part_scatter<true, uint16_t>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsLimit));
        DB_HIP(hipFuncSetAttribute((const void*)k_ov_bucket_sort, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)kLdsLimit));
        lds_ok.store(true, std::memory_order_release);
    }
    const bool three = P.three;
    const int low = P.low, lowc = P.lowc, fine_per = P.fine_per, per_block = P.per_block;
    const int64_t nbuckets = P.nbuckets, npart = P.npart, nchunks2 = P.nchunks2, ncount2 = P.ncount2;
    const PartSeg flat{nullptr, nullptr, 0};
    int32_t* pcounts;
    int64_t* poffs;
    const int64_t ncount = nbuckets * npart;
    DB_TRY(scr.work_n(ncount, &pcounts));
    DB_TRY(scr.work_n(ncount + 1, &poffs));
    const int low1 = three ? lowc : low;
    DB_TRY(timing_begin(kPhPartCount, st, &tok));
    hipLaunchKernelGGL(k_ov_part_count<false>, dim3((unsigned)npart), dim3(kPartBlock), (size_t)nbuckets * 4, st,
                       keys_a, N, per_block, low1, (int)nbuckets, flat, pcounts);
    DB_HIP(hipGetLastError());
    DB_TRY(timing_end(tok, st));
    DB_TRY(scan_exclusive(pcounts, poffs, ncount, nullptr, scr));
    uint16_t* keys_a16 = reinterpret_cast<uint16_t*>(keys_a);
    uint16_t* keys_b16 = reinterpret_cast<uint16_t*>(keys_b);
    DB_TRY(timing_begin(kPhPartScatter, st, &tok));
    if (!three)   // the last level reads the low `low` <= 13 bits: 16-bit keys
        hipLaunchKernelGGL((k_ov_part_scatter<false, uint16_t>), dim3((unsigned)npart), dim3(kPartBlock),
                           part_scatter_lds(nbuckets), st, keys_a, pays_a, N, per_block, low1, (int)nbuckets, flat,
                           poffs, N, keys_b16, pays_b);
    else          // the second level needs lowc bits
        hipLaunchKernelGGL((k_ov_part_scatter<false, uint32_t>), dim3((unsigned)npart), dim3(kPartBlock),
                           part_scatter_lds(nbuckets), st, keys_a, pays_a, N, per_block, low1, (int)nbuckets, flat,
                           poffs, N, keys_b, pays_b);
    DB_HIP(hipGetLastError());
    DB_TRY(timing_end(tok, st));
    const int64_t* sort_start = poffs;   // first pair of bucket b: sort_start[b * sort_stride]
    int64_t sort_stride = npart;
    const uint16_t* sort_keys = keys_b16;
    const uint64_t* sort_pays = pays_b;
    if (three) {
        int64_t *seg_start, *chunk_base, *fine_start, *poffs2;
        int32_t* pcounts2;
        DB_TRY(scr.work_n(nbuckets + 1, &seg_start));
        DB_TRY(scr.work_n(nbuckets + 1, &chunk_base));
        DB_TRY(scr.work_n(nbuckets * fine_per + 1, &fine_start));
        DB_TRY(scr.work_n(ncount2, &pcounts2));
        DB_TRY(scr.work_n(ncount2 + 1, &poffs2));
        hipLaunchKernelGGL(k_ov_seg_chunks, dim3(1), dim3(kSegChunkBlock), 0, st, poffs, npart, (int)nbuckets, N,
                           seg_start, chunk_base);
        DB_HIP(hipGetLastError());
        const PartSeg ps{seg_start, chunk_base, (int32_t)nbuckets};
        DB_TRY(timing_begin(kPhPart2Count, st, &tok));
        hipLaunchKernelGGL(k_ov_part_count<true>, dim3((unsigned)nchunks2), dim3(kPartBlock), (size_t)fine_per * 4,
                           st, keys_b, N, 1, low, fine_per, ps, pcounts2);
        DB_HIP(hipGetLastError());
        DB_TRY(timing_end(tok, st));
        DB_TRY(scan_exclusive(pcounts2, poffs2, ncount2, nullptr, scr));
        DB_TRY(timing_begin(kPhPart2Scatter, st, &tok));
        hipLaunchKernelGGL((k_ov_part_scatter<true, uint16_t>), dim3((unsigned)nchunks2), dim3(kPartBlock),
                           part_scatter_lds(fine_per), st, keys_b, pays_b, N, 1, low, fine_per, ps, poffs2, N,
                           keys_a16, pays_a);
        DB_HIP(hipGetLastError());
        DB_TRY(timing_end(tok, st));
        hipLaunchKernelGGL(k_ov_fine_start, dim3(grid_for(nbuckets * fine_per + 1, 256, 4096)), dim3(256), 0, st,
                           poffs2, chunk_base, (int)nbuckets, fine_per, nbuckets * fine_per, fine_start);
        DB_HIP(hipGetLastError());
        sort_start = fine_start;
        sort_stride = 1;
        sort_keys = keys_a16;
        sort_pays = pays_a;
    }
    // staged sweeps of 2^12 columns (one sweep for buckets of at most that)
    DB_TRY(timing_begin(kPhBucketSort, st, &tok));
    hipLaunchKernelGGL((k_ov_bucket_sort), dim3((unsigned)P.nsort), dim3(kBucketBlock),
                       ((size_t)4 << kStageBits) + (size_t)8 * kStageCap, st, sort_start, sort_stride, low,
                       std::min(low, kStageBits), M, N, sort_keys, sort_pays, rec, at_dest, rec_base);
    DB_HIP(hipGetLastError());
    DB_TRY(timing_end(tok, st));
    return DIBELLA_OK;
}

// Steps O0 and O1 over every set of L (on the device as d_sets, d_base):
// validate A, build A^T and, with slices, the rows' slice boundaries.  The
// results come from `ar` (they live as long as it); the partition passes'
// keys and pairs come from a scratch arena released on return (its frees
// are ordered on the stream after the kernels that use them).  With
// col_ranges > 1 (one set with slices only) A^T is built over that many
// column ranges of whole slices, one after the other, each range's pairs
// gathered from the rows by their slice boundaries, so that the partition
// buffers hold one range's pairs at a time.
static int ov_transpose(const OvLayout& L, const OvSet* d_sets, const int64_t* d_base, uint32_t flags, Arena& ar,
                        OvTransposed* T, int col_ranges = 1) {
    hipStream_t st = ar.stream();
    const int nsets = (int)L.hs.size();
    const int64_t total_rows = L.total_rows, total_m = L.total_m, total_nnz = L.total_nnz;
    const SliceMap sm = slice_plan(total_m, total_rows, total_nnz);
    const int K = (nsets == 1 && sm.count > 0 && total_nnz > 0) ? std::max(1, std::min(col_ranges, (int)sm.count)) : 1;
    // ---- what the row phases keep: one reservation
    {
        auto pad = [](size_t b) { return Arena::padded(b); };
        size_t est = pad(4 * nsets) + pad(8 * std::max<int64_t>(total_m, 1)) + pad(8 * total_nnz) + 4 * Arena::padded(1);
        if (sm.count) est += pad(4 * total_rows * (sm.count + 1));
        DB_TRY(ar.reserve(est));
    }
    int32_t* d_flags;
    uint64_t* rec;
    uint64_t* at = nullptr;   // A^T (K > 1: its own buffer; else the last pass's output buffer, below)
    int32_t* bnd = nullptr;
    DB_TRY(ar.work_n(nsets, &d_flags));
    DB_TRY(ar.work_n(std::max<int64_t>(total_m, 1), &rec));
    if (K > 1) DB_TRY(ar.work_n(total_nnz, &at));
    if (sm.count) DB_TRY(ar.work_n((size_t)total_rows * (sm.count + 1), &bnd));
    DB_TRY(fill_i32(d_flags, 0, nsets, st));
    int tok = -1;
    constexpr int WPB = 4;
    const int grid_rows = grid_for(total_rows, WPB, 1 << 16);
    const int checks = (flags & DIBELLA_NO_VALIDATE) ? 0 : 1;
    // empty segments where no pass writes them (the bucket sort writes every
    // column of a range with entries)
    if (total_nnz == 0) DB_TRY(fill_i32(reinterpret_cast<int32_t*>(rec), 0, 2 * std::max<int64_t>(total_m, 1), st));

    if (K == 1) {
        const SortPlan P = sort_plan(total_m, total_nnz);
        Arena scr(ar.alloc_fn(), ar.free_fn(), ar.alloc_ctx(), st);
        DB_TRY(scr.reserve(2 * Arena::padded(4 * total_nnz) + Arena::padded(8 * total_nnz) + sort_table_bytes(P)));
        uint32_t *keys_a, *keys_b;
        uint64_t* pays_x;   // the pairs buffer that does not end as A^T
        DB_TRY(scr.work_n(total_nnz, &keys_a));
        DB_TRY(scr.work_n(total_nnz, &keys_b));
        DB_TRY(scr.work_n(total_nnz, &pays_x));
        uint64_t* at_out;
        DB_TRY(ar.work_n(total_nnz, &at_out));
        // the three-level sort ends in the second pairs buffer, the two-level
        // one in the first
        uint64_t* pays_a = P.three ? pays_x : at_out;
        uint64_t* pays_b = P.three ? at_out : pays_x;
        if (total_nnz > 0) DB_TRY(fill_i32(reinterpret_cast<int32_t*>(keys_a), 0, total_nnz, st));   // keys of skipped entries
        if (total_rows > 0) {
            DB_TRY(timing_begin(kPhKeys, st, &tok));
            hipLaunchKernelGGL(k_ov_keys<WPB>, dim3(grid_rows), dim3(WPB * kWave), 0, st, d_sets, nsets, d_base,
                               total_rows, keys_a, pays_a, d_flags, checks, sm, bnd);
            DB_HIP(hipGetLastError());
            DB_TRY(timing_end(tok, st));
        }
        DB_TRY(sort_pairs(P, total_m, total_nnz, keys_a, keys_b, pays_a, pays_b, at_out, rec, 0, scr));
        at = at_out;
    } else {
        // checks and slice boundaries only
        DB_TRY(timing_begin(kPhKeys, st, &tok));
        hipLaunchKernelGGL(k_ov_keys<WPB>, dim3(grid_rows), dim3(WPB * kWave), 0, st, d_sets, nsets, d_base,
                           total_rows, (uint32_t*)nullptr, (uint64_t*)nullptr, d_flags, checks, sm, bnd);
        DB_HIP(hipGetLastError());
        DB_TRY(timing_end(tok, st));
        // range k: slices [S k / K, S (k + 1) / K); its first column is the
        // first c with slice_of(c) >= that slice
        std::vector<int> s_of(K + 1);
        std::vector<int64_t> c_of(K + 1);
        for (int k = 0; k <= K; ++k) {
            s_of[k] = (int)((int64_t)sm.count * k / K);
            const uint64_t num = (uint64_t)s_of[k] << 32;
            c_of[k] = k == K ? total_m : std::min<int64_t>(total_m, (int64_t)((num + sm.mul - 1) / sm.mul));
        }
        // every range's pair count, read at one synchronisation
        int32_t* cnt;
        int64_t* off;
        DB_TRY(ar.work_n(total_rows, &cnt));
        DB_TRY(ar.work_n((size_t)(total_rows + 1) * K, &off));
        for (int k = 0; k < K; ++k) {
            hipLaunchKernelGGL(k_ov_range_count, dim3(grid_for(total_rows, 256, 4096)), dim3(256), 0, st, d_sets,
                               total_rows, bnd, s_of[k], s_of[k + 1], cnt);
            DB_HIP(hipGetLastError());
            DB_TRY(scan_exclusive(cnt, off + (int64_t)(total_rows + 1) * k, total_rows, nullptr, ar));
        }
        HostStage& hst = host_stage();
        DB_TRY(hst.reserve(sizeof(int64_t) * K + 64));
        int64_t* h_tot = static_cast<int64_t*>(hst.ptr);
        for (int k = 0; k < K; ++k)
            DB_HIP(hipMemcpyAsync(h_tot + k, off + (int64_t)(total_rows + 1) * k + total_rows, sizeof(int64_t),
                                  hipMemcpyDeviceToHost, st));
        DB_TRY(sync_stream(st));
        std::vector<int64_t> tot(h_tot, h_tot + K);
        DB_TRY(stage_done(st));
        int64_t base = 0;
        for (int k = 0; k < K; ++k) {
            const int64_t M = c_of[k + 1] - c_of[k], N = std::min(tot[k], total_nnz - base);
            if (M <= 0) continue;
            if (N <= 0) {
                DB_TRY(fill_i32(reinterpret_cast<int32_t*>(rec + c_of[k]), 0, 2 * M, st));
                continue;
            }
            const SortPlan P = sort_plan(M, N);
            Arena scr(ar.alloc_fn(), ar.free_fn(), ar.alloc_ctx(), st);
            DB_TRY(scr.reserve(2 * Arena::padded(4 * N) + 2 * Arena::padded(8 * N) + sort_table_bytes(P)));
            uint32_t *keys_a, *keys_b;
            uint64_t *pays_a, *pays_b;
            DB_TRY(scr.work_n(N, &keys_a));
            DB_TRY(scr.work_n(N, &keys_b));
            DB_TRY(scr.work_n(N, &pays_a));
            DB_TRY(scr.work_n(N, &pays_b));
            DB_TRY(timing_begin(kPhKeys, st, &tok));
            hipLaunchKernelGGL(k_ov_range_keys, dim3(grid_for(total_rows, 4, 1 << 16)), dim3(256), 0, st, d_sets,
                               total_rows, bnd, s_of[k], s_of[k + 1], c_of[k], c_of[k + 1],
                               off + (int64_t)(total_rows + 1) * k, N, keys_a, pays_a);
            DB_HIP(hipGetLastError());
            DB_TRY(timing_end(tok, st));
            DB_TRY(sort_pairs(P, M, N, keys_a, keys_b, pays_a, pays_b, at + base, rec + c_of[k], base, scr));
            base += N;
        }
    }
    T->rec = rec;
    T->at = total_nnz > 0 ? reinterpret_cast<const int2*>(at) : nullptr;
    T->bnd = bnd;
    T->bnd_stride = total_rows;
    T->sm = sm;
    T->d_flags = d_flags;
    T->nsets = nsets;
    return DIBELLA_OK;
}

// Steps O2-O4 for the rows of R (on the device as d_rsets, d_rbase; every
// set's A entries and columns are those T was built from, its rows those
// whose outputs C receives): row costs and bins, symbolic, numeric.  `bnd`
// is T's slice table at the first row of R (R's rows are consecutive rows
// of T's); seg_entries: the A entries of R's rows.  C's arrays are outputs
// of `ar`, or its workspace when c_as_work.
static int ov_rows(OvLayout& R, OvSet* d_rsets, const int64_t* d_rbase, const OvTransposed& T, const int32_t* bnd,
                   int64_t seg_entries, dibella_overlap_out* C, Arena& ar, bool c_as_work) {
    hipStream_t st = ar.stream();
    const dibella_tuning tn = tuning();
    dibella_stats& stt = stats();
    const int nsets = (int)R.hs.size();
    const int64_t total_rows = R.total_rows;
    const int64_t rows_nnz = seg_entries;   // one segment word per A entry of R's rows
    const SliceMap sm = T.sm;
    const NumBins bins = numeric_bins(tn, R.bits_words);
    if (bins.nh == 0) {
        set_error("tuning leaves no numeric table that fits the LDS");
        return DIBELLA_EINVAL;
    }
    const int64_t slice_groups = ceil_div(total_rows, kSliceRows);
    // ---- workspace: one reservation for everything requested before the
    // first synchronisation (allocator calls cost host time each)
    {
        auto pad = [](size_t b) { return Arena::padded(b); };
        size_t est = pad(sizeof(OvCounters)) + pad(8 * nsets) + pad(8 * rows_nnz);
        est += 7 * pad(8 * (total_rows + 1)) + 3 * pad(4 * total_rows);
        est += pad(4 * total_rows * kMaxLog2) + pad(4 * total_rows * kMaxBins);
        if (sm.count) est += pad(4 * total_rows * sm.count);
        est += 2 * pad(8 * scan_workspace_elems(std::max<int64_t>(total_rows, 1))) + 16 * Arena::padded(1);
        DB_TRY(ar.reserve(est));
    }
    OvCounters* d_ctr;
    int64_t* d_set_nnz;
    uint64_t* seg;
    int64_t *flops_row, *nnzrow, *G, *esc_off, *sbound, *soff;
    int32_t *distinct, *sym_list, *num_list, *esc_list, *retry_list;
    DB_TRY(ar.work_n(1, &d_ctr));
    DB_TRY(ar.work_n(nsets, &d_set_nnz));
    DB_TRY(ar.work_n(rows_nnz, &seg));
    DB_TRY(ar.work_n(total_rows, &flops_row));
    DB_TRY(ar.work_n(total_rows, &nnzrow));
    DB_TRY(ar.work_n(total_rows + 1, &G));
    DB_TRY(ar.work_n(total_rows, &esc_off));
    DB_TRY(ar.work_n(total_rows, &sbound));
    DB_TRY(ar.work_n(total_rows + 1, &soff));
    DB_TRY(ar.work_n(total_rows, &distinct));
    DB_TRY(ar.work_n((size_t)total_rows * kMaxLog2, &sym_list));
    DB_TRY(ar.work_n((size_t)total_rows * kMaxBins, &num_list));
    DB_TRY(ar.work_n(total_rows, &esc_list));
    DB_TRY(ar.work_n(total_rows, &retry_list));
    uint32_t* part = nullptr;
    if (sm.count) DB_TRY(ar.work_n((size_t)total_rows * sm.count, &part));

    HostStage& hst = host_stage();
    const size_t desc_bytes = sizeof(OvSet) * nsets;
    const size_t back_bytes = sizeof(OvCounters) + sizeof(int32_t) * T.nsets + sizeof(int64_t) * (nsets + 1);
    DB_TRY(hst.reserve(desc_bytes + back_bytes + 64));
    char* hbuf = static_cast<char*>(hst.ptr);
    DB_TRY(fill_i32(reinterpret_cast<int32_t*>(d_ctr), 0, sizeof(OvCounters) / 4, st));
    DB_TRY(fill_i64(nnzrow, 0, total_rows, st));
    DB_TRY(fill_i32(distinct, 0, total_rows, st));

    // ---- row costs + scratch ranges
    int tok = -1;
    if (total_rows > 0) {
        DB_TRY(timing_begin(kPhSegments, st, &tok));
        if (sm.count) {
            const int64_t nblk = (int64_t)(sm.count / 8) * 8 * slice_groups;
            hipLaunchKernelGGL(k_ov_seg_slices, dim3((unsigned)nblk), dim3(kSliceBlock), 0, st, d_rsets, nsets,
                               d_rbase, total_rows, slice_groups, sm, bnd, T.bnd_stride, T.rec, seg, part);
            DB_HIP(hipGetLastError());
        }
        hipLaunchKernelGGL(k_ov_scatter<kSegWaves>, dim3((unsigned)ceil_div(total_rows, kRowsPerBlock)),
                           dim3(kSegWaves * kWave), 0, st, d_rsets, nsets, d_rbase, total_rows, T.rec, seg,
                           flops_row, sbound, sym_list, d_ctr, tn.sym_first_log2, tn.load_pct, part, sm.count);
        DB_HIP(hipGetLastError());
        DB_TRY(timing_end(tok, st));
    }
    DB_TRY(scan_exclusive(sbound, soff, total_rows, nullptr, ar));
    // ---- sync 1: validity, bin sizes, scratch size
    char* back = hbuf + desc_bytes;
    OvCounters* h_ctr = reinterpret_cast<OvCounters*>(back);
    int32_t* h_flags = reinterpret_cast<int32_t*>(back + sizeof(OvCounters));
    int64_t* h_set_nnz = reinterpret_cast<int64_t*>(back + sizeof(OvCounters) + sizeof(int32_t) * T.nsets);
    DB_HIP(hipMemcpyAsync(h_ctr, d_ctr, sizeof(OvCounters), hipMemcpyDeviceToHost, st));
    DB_HIP(hipMemcpyAsync(h_flags, T.d_flags, sizeof(int32_t) * T.nsets, hipMemcpyDeviceToHost, st));
    DB_HIP(hipMemcpyAsync(h_set_nnz + nsets, soff + total_rows, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    DB_TRY(sync_stream(st));
    const int64_t scratch_words = h_set_nnz[nsets];
    for (int s = 0; s < T.nsets; ++s) {
        if (h_flags[s]) {
            set_error("set " + std::to_string(s) + ": " + describe_bad(h_flags[s]));
            return (h_flags[s] & kLongRow) && !(h_flags[s] & ~kLongRow) ? DIBELLA_EOVERFLOW
                                                                          : DIBELLA_EINVAL;
        }
    }
    if (h_ctr->max_flops >= (int64_t(1) << 31)) {
        set_error("a row needs 2^31 or more semiring products");
        return DIBELLA_EOVERFLOW;
    }
    stt.products += h_ctr->products;
    int32_t* scratch;
    DB_TRY(ar.work_n(scratch_words, &scratch));
    OvWork W{d_rsets, nsets, d_rbase, retry_list, seg, T.at, soff, scratch, nnzrow, distinct, d_ctr, G};

    // ---- symbolic: bitmap rows; hash rows by first-level table (largest
    // first), then the retry level
    if (h_ctr->sym_count[kBitsClass] > 0) {
        const int count = h_ctr->sym_count[kBitsClass];
        const int blk = wide_block(tn.sym_block, sym_bits_lds(256, R.bits_planes, R.bits_words));
        DB_TRY(timing_begin(kPhSymBits, st, &tok));
        DB_TRY(dispatch_sym_bits(blk, W, sym_list + (int64_t)kBitsClass * total_rows, count, R.bits_planes,
                                 R.bits_words, st));
        DB_TRY(timing_end(tok, st));
    }
    bool any_hash = false;
    for (int lg = tn.sym_first_log2; lg >= 6; --lg) {
        const int count = h_ctr->sym_count[lg];
        if (!count) continue;
        any_hash = true;
        const int Tn = 1 << lg;
        const int limit = (int)((int64_t)Tn * tn.load_pct / 100);
        DB_TRY(timing_begin(kPhSymHash, st, &tok));
        DB_TRY(dispatch_sym_hash(wide_block(tn.sym_block, sym_hash_lds(256, Tn)), W,
                                 SymArgs{sym_list + (int64_t)lg * total_rows, nullptr, count, count, Tn, limit, 0,
                                         kQSymHash + lg},
                                 st));
        DB_TRY(timing_end(tok, st));
    }
    if (any_hash) {
        const int Tn = 1 << tn.sym_max_log2;
        const int limit = (int)((int64_t)Tn * tn.load_pct / 100);
        const int grid = (int)std::min<int64_t>(total_rows, 512);
        DB_TRY(timing_begin(kPhSymHash, st, &tok));
        DB_TRY(dispatch_sym_hash(wide_block(tn.sym_block, sym_hash_lds(256, Tn)), W,
                                 SymArgs{retry_list, &d_ctr->retry_rows, 0, grid, Tn, limit, 1, kQRetry}, st));
        DB_TRY(timing_end(tok, st));
    }
    if (total_rows > 0) {
        hipLaunchKernelGGL(k_ov_bin_numeric, dim3((unsigned)ceil_div(total_rows, kBinBlock)), dim3(kBinBlock), 0, st,
                           d_rsets, nsets, d_rbase, total_rows, flops_row, distinct, nnzrow, num_list, esc_list,
                           esc_off, d_ctr, bins);
        DB_HIP(hipGetLastError());
    }
    DB_TRY(scan_exclusive(nnzrow, G, total_rows, nullptr, ar));
    hipLaunchKernelGGL(k_ov_set_totals, dim3(grid_for(nsets, 64, 1024)), dim3(64), 0, st, d_rsets, nsets, G,
                       d_set_nnz);
    DB_HIP(hipGetLastError());
    DB_HIP(hipMemcpyAsync(h_ctr, d_ctr, sizeof(OvCounters), hipMemcpyDeviceToHost, st));
    DB_HIP(hipMemcpyAsync(h_set_nnz, d_set_nnz, sizeof(int64_t) * nsets, hipMemcpyDeviceToHost, st));
    DB_TRY(sync_stream(st));  // sync 2

    // ---- ESC rows
    const int esc_rows = h_ctr->esc_rows;
    stt.esc_rows += esc_rows;
    uint32_t *keys0 = nullptr, *keys1 = nullptr;
    uint64_t *pay0 = nullptr, *pay1 = nullptr;
    if (esc_rows > 0) {
        const int64_t ef = h_ctr->esc_flops;
        DB_TRY(ar.work_n(ef, &keys0));
        DB_TRY(ar.work_n(ef, &keys1));
        DB_TRY(ar.work_n(ef, &pay0));
        DB_TRY(ar.work_n(ef, &pay1));
        DB_TRY(timing_begin(kPhEsc, st, &tok));
        hipLaunchKernelGGL(k_esc_expand, dim3(esc_rows), dim3(kEscBlock), 0, st, d_rsets, nsets, d_rbase,
                           esc_list, esc_off, seg, T.at, keys0, pay0);
        hipLaunchKernelGGL(k_esc_sort, dim3(esc_rows), dim3(kEscBlock), 0, st, d_rsets, nsets, d_rbase,
                           esc_list, esc_off, flops_row, keys0, pay0, keys1, pay1);
        DB_HIP(hipGetLastError());
        DB_TRY(timing_end(tok, st));
        if (h_ctr->overflow_rows > 0) {
            hipLaunchKernelGGL(k_esc_count, dim3(esc_rows), dim3(kEscBlock), 0, st, d_rsets, nsets, d_rbase,
                               esc_list, esc_off, flops_row, keys0, nnzrow, distinct);
            DB_HIP(hipGetLastError());
            DB_TRY(scan_exclusive(nnzrow, G, total_rows, nullptr, ar));
            hipLaunchKernelGGL(k_ov_set_totals, dim3(grid_for(nsets, 64, 1024)), dim3(64), 0, st, d_rsets,
                               nsets, G, d_set_nnz);
            DB_HIP(hipGetLastError());
            DB_HIP(hipMemcpyAsync(h_set_nnz, d_set_nnz, sizeof(int64_t) * nsets, hipMemcpyDeviceToHost, st));
            DB_TRY(sync_stream(st));  // sync 3 (only with rows that overflow the retry table)
        }
    }

    // ---- outputs
    for (int s = 0; s < nsets; ++s) {
        const int64_t nz = h_set_nnz[s];
        OvSet& o = R.hs[s];
        auto take = [&](auto n, auto** p) { return c_as_work ? ar.work_n(n, p) : ar.output_n(n, p); };
        DB_TRY(take(o.n + 1, &o.c_rowptr));
        DB_TRY(take(nz, &o.c_col));
        DB_TRY(take(nz, &o.c_count));
        DB_TRY(take(4 * nz, &o.c_seed));
        C[s].nrows = o.n;
        C[s].ncols = o.nreads;
        C[s].nnz = nz;
        C[s].rowptr = o.c_rowptr;
        C[s].col = o.c_col;
        C[s].count = o.c_count;
        C[s].seed = o.c_seed;
    }
    std::memcpy(hbuf, R.hs.data(), sizeof(OvSet) * nsets);
    DB_HIP(hipMemcpyAsync(d_rsets, hbuf, sizeof(OvSet) * nsets, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_ov_write_rowptr, dim3(grid_for(total_rows + nsets, 256, 4096)), dim3(256), 0, st,
                       d_rsets, nsets, d_rbase, total_rows, G);
    DB_HIP(hipGetLastError());
    // numeric bins (largest tables first) spread over the caller's stream and
    // the side streams, so that the few rows of the large bins overlap with
    // the many of the small ones instead of leaving the GPU to a tail
    SideStreams* side = nullptr;
    DB_TRY(side_streams(&side));
    int tok_all = -1;
    DB_TRY(timing_begin(kPhNumericAll, st, &tok_all));
    DB_TRY(side->begin(st));
    {
        // the side streams are joined back into st on every way out of this
        // block, so that no failure leaves work queued on them behind the
        // workspace the caller's allocator reclaims
        struct Join {
            SideStreams* side;
            hipStream_t st;
            bool joined;
            ~Join() {
                if (!joined) (void)side->end(st);
            }
        } join{side, st, false};
        int lane_k = 0;
        for (int b = bins.nh + bins.nb - 1; b >= 0; --b) {
            const int count = h_ctr->num_count[b];
            if (!count) continue;
            const bool bits = b >= bins.nh;
            const int D = bins.d[b];
            const int blk = wide_block(tn.num_block, num_lds(256, D, tn.load_pct, bits, R.bits_words));
            hipStream_t ls = lane_k == 0 ? st : side->s[lane_k - 1];
            lane_k = (lane_k + 1) % (kSideStreams + 1);
            DB_TRY(timing_begin(kPhNumeric, ls, &tok));
            DB_TRY(dispatch_numeric(blk, W, num_list + (int64_t)b * total_rows, count, D, tn.load_pct, bits,
                                    R.bits_words, kQNumeric + b, ls));
            DB_TRY(timing_end(tok, ls));
        }
        join.joined = true;
        DB_TRY(side->end(st));
    }
    DB_TRY(timing_end(tok_all, st));
    if (esc_rows > 0) {
        DB_TRY(timing_begin(kPhEsc, st, &tok));
        hipLaunchKernelGGL(k_esc_emit, dim3(esc_rows), dim3(kEscBlock), 0, st, d_rsets, nsets, d_rbase,
                           esc_list, esc_off, flops_row, keys0, pay0, G);
        DB_HIP(hipGetLastError());
        DB_TRY(timing_end(tok, st));
    }
    DB_TRY(stage_done(st));
    return DIBELLA_OK;
}

// Uploads a layout's sets and row bases into `ar`.
static int upload_sets(const OvLayout& L, Arena& ar, OvSet** d_sets, int64_t** d_base) {
    hipStream_t st = ar.stream();
    const int nsets = (int)L.hs.size();
    DB_TRY(ar.work_n(nsets, d_sets));
    DB_TRY(ar.work_n(nsets + 1, d_base));
    HostStage& hst = host_stage();
    const size_t desc_bytes = sizeof(OvSet) * nsets + sizeof(int64_t) * (nsets + 1);
    DB_TRY(hst.reserve(desc_bytes + 64));
    char* hbuf = static_cast<char*>(hst.ptr);
    std::memcpy(hbuf, L.hs.data(), sizeof(OvSet) * nsets);
    std::memcpy(hbuf + sizeof(OvSet) * nsets, L.base.data(), sizeof(int64_t) * (nsets + 1));
    DB_HIP(hipMemcpyAsync(*d_sets, hbuf, sizeof(OvSet) * nsets, hipMemcpyHostToDevice, st));
    DB_HIP(hipMemcpyAsync(*d_base, hbuf + sizeof(OvSet) * nsets, sizeof(int64_t) * (nsets + 1),
                          hipMemcpyHostToDevice, st));
    DB_TRY(stage_done(st));
    return DIBELLA_OK;
}

int overlap_run(const dibella_csr* A, int nsets, const int32_t* min_shared, dibella_overlap_out* C,
                uint32_t flags, Arena& ar) {
    const dibella_tuning tn = tuning();
    OvLayout L;
    DB_TRY(ov_layout(A, nsets, min_shared, tn, L));
    for (int s = 0; s < nsets; ++s) {
        C[s].nrows = A[s].nrows;
        C[s].ncols = A[s].nrows;
        C[s].nnz = 0;
        C[s].rowptr = nullptr;
        C[s].col = nullptr;
        C[s].count = nullptr;
        C[s].seed = nullptr;
    }
    if (numeric_bins(tn, L.bits_words).nh == 0) {
        set_error("tuning leaves no numeric table that fits the LDS");
        return DIBELLA_EINVAL;
    }
    OvSet* d_sets;
    int64_t* d_base;
    DB_TRY(upload_sets(L, ar, &d_sets, &d_base));
    OvTransposed T;
    DB_TRY(ov_transpose(L, d_sets, d_base, flags, ar, &T));
    stats().products = 0;
    stats().esc_rows = 0;
    return ov_rows(L, d_sets, d_base, T, T.bnd, L.total_nnz, C, ar, false);
}

// out[i] = in[i] + add for i in [0, n]: a block's row pointers placed after
// the entries of the blocks before it.
__global__ void k_shift_rowptr(const int64_t* __restrict__ in, int64_t n, int64_t add, int64_t* __restrict__ out) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = in[i] + add;
}

int overlap_graph_blocked_run(const dibella_csr* A, int32_t min_shared, const int32_t* read_len, int32_t k,
                              int32_t min_overlap, int32_t max_drift, int32_t min_density, int64_t block_rows,
                              dibella_csr_out* R, int32_t* nblocks, Arena& ar) {
    hipStream_t st = ar.stream();
    std::memset(R, 0, sizeof(*R));
    *nblocks = 0;
    if (block_rows < 1) {
        set_error("dibella_overlap_graph_blocked: block_rows must be >= 1");
        return DIBELLA_EINVAL;
    }
    if (k < 1 || k > 32 || min_overlap < 0) {
        set_error("dibella_overlap_graph_blocked: k must be in [1, 32] and min_overlap >= 0");
        return DIBELLA_EINVAL;
    }
    const dibella_tuning tn = tuning();
    OvLayout L;
    DB_TRY(ov_layout(A, 1, &min_shared, tn, L));
    if (numeric_bins(tn, L.bits_words).nh == 0) {
        set_error("tuning leaves no numeric table that fits the LDS");
        return DIBELLA_EINVAL;
    }
    const int64_t n = A->nrows;
    if (n > 0 && !read_len) {
        set_error("dibella_overlap_graph_blocked: null pointer");
        return DIBELLA_EINVAL;
    }
    OvSet* d_sets;
    int64_t* d_base;
    DB_TRY(upload_sets(L, ar, &d_sets, &d_base));
    // A^T over as many column ranges as there are blocks of rows, so that
    // its partition buffers shrink with the blocks too
    const int64_t nb = n > 0 ? ceil_div(n, block_rows) : 0;
    OvTransposed T;
    DB_TRY(ov_transpose(L, d_sets, d_base, 0u, ar, &T, (int)std::min<int64_t>(nb, 1 << 20)));
    stats().products = 0;
    stats().esc_rows = 0;
    // A's row pointers on the host (every block's first entry) and A's
    // validation flags: a block's segment words are indexed from its first
    // entry, so A must be known valid before any block runs
    std::vector<int64_t> rp(n + 1, 0);
    if (n > 0) {
        HostStage& hst = host_stage();
        DB_TRY(hst.reserve(sizeof(int64_t) * (n + 1) + 64));
        int32_t* h_flag = reinterpret_cast<int32_t*>(static_cast<char*>(hst.ptr) + sizeof(int64_t) * (n + 1));
        DB_HIP(hipMemcpyAsync(hst.ptr, A->rowptr, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToHost, st));
        DB_HIP(hipMemcpyAsync(h_flag, T.d_flags, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        DB_TRY(sync_stream(st));
        std::memcpy(rp.data(), hst.ptr, sizeof(int64_t) * (n + 1));
        const int32_t bad = *h_flag;
        DB_TRY(stage_done(st));
        if (bad) {
            set_error("set 0: " + std::string(describe_bad(bad)));
            return (bad & kLongRow) && !(bad & ~kLongRow) ? DIBELLA_EOVERFLOW : DIBELLA_EINVAL;
        }
    }
    std::vector<dibella_csr_out> parts(nb);
    int64_t total = 0;
    for (int64_t b = 0; b < nb; ++b) {
        const int64_t r0 = b * block_rows, r1 = std::min(n, r0 + block_rows);
        OvLayout B;
        B.hs = L.hs;
        OvSet& o = B.hs[0];
        o.a_rowptr = A->rowptr + r0;
        o.n = r1 - r0;
        o.row_base = 0;
        o.nnz_base = -rp[r0];   // segment words of the block's entries from 0
        o.read_base = r0;
        B.base = {0, r1 - r0};
        B.total_rows = r1 - r0;
        B.total_m = L.total_m;
        B.total_nnz = rp[r1] - rp[r0];
        B.bits_words = L.bits_words;
        B.bits_planes = L.bits_planes;
        // the block's workspace and rows of C are released at the end of
        // the block (in stream order: the next block's work comes after)
        Arena blk(ar.alloc_fn(), ar.free_fn(), ar.alloc_ctx(), st);
        OvSet* d_bs;
        int64_t* d_bb;
        DB_TRY(upload_sets(B, blk, &d_bs, &d_bb));
        dibella_overlap_out Cb;
        DB_TRY(ov_rows(B, d_bs, d_bb, T, T.bnd ? T.bnd + r0 : nullptr, B.total_nnz, &Cb, blk, true));
        DB_TRY(r_from_seeds_run(&Cb, r0, read_len, k, min_overlap, max_drift, min_density, &parts[b], blk, ar,
                                true));
        total += parts[b].nnz;
    }
    // R: the blocks' rows one after the other
    int64_t* rrp;
    int32_t *rcol, *rval;
    DB_TRY(ar.output_n(n + 1, &rrp));
    DB_TRY(ar.output_n(total, &rcol));
    DB_TRY(ar.output_n(total, &rval));
    if (n == 0) DB_TRY(fill_i64(rrp, 0, 1, st));
    int64_t off = 0;
    for (int64_t b = 0; b < nb; ++b) {
        const int64_t r0 = b * block_rows;
        const dibella_csr_out& P = parts[b];
        hipLaunchKernelGGL(k_shift_rowptr, dim3(grid_for(P.nrows + 1, 256, 1024)), dim3(256), 0, st, P.rowptr,
                           P.nrows, off, rrp + r0);
        DB_HIP(hipGetLastError());
        if (P.nnz > 0) {
            DB_HIP(hipMemcpyAsync(rcol + off, P.col, sizeof(int32_t) * P.nnz, hipMemcpyDeviceToDevice, st));
            DB_HIP(hipMemcpyAsync(rval + off, P.val, sizeof(int32_t) * P.nnz, hipMemcpyDeviceToDevice, st));
        }
        off += P.nnz;
    }
    R->nrows = R->ncols = n;
    R->nnz = total;
    R->rowptr = rrp;
    R->col = rcol;
    R->val = rval;
    *nblocks = (int32_t)nb;
    return DIBELLA_OK;
}

}  // namespace dibella
