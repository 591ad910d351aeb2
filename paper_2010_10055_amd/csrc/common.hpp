// Shared host and device helpers of the HIP library (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "dibella.h"

namespace dibella {

constexpr int kWave = 64;

// ---------------------------------------------------------------------------
// Errors
// ---------------------------------------------------------------------------
void set_error(const std::string& msg);
std::string& error_slot();

#define DB_HIP(expr)                                                                  \
    do {                                                                              \
        hipError_t _e = (expr);                                                       \
        if (_e != hipSuccess) {                                                       \
            ::dibella::set_error(std::string(#expr) + ": " + hipGetErrorString(_e));  \
            return DIBELLA_EDEVICE;                                                   \
        }                                                                             \
    } while (0)

#define DB_TRY(expr)                        \
    do {                                    \
        int _s = (expr);                    \
        if (_s != DIBELLA_OK) return _s;    \
    } while (0)

// ---------------------------------------------------------------------------
// Tuning (process wide) and per-thread statistics
// ---------------------------------------------------------------------------
dibella_tuning tuning();                    // a copy of the process-wide tunables (under a lock)
void tuning_store(const dibella_tuning& t);
dibella_stats& stats();

// ---------------------------------------------------------------------------
// Allocation through the caller's callbacks (or hipMallocAsync), released
// in reverse order when the call ends.  Outputs are kept unless the call
// fails.
// ---------------------------------------------------------------------------
class Arena {
  public:
    Arena(dibella_alloc_fn a, dibella_free_fn f, void* ctx, hipStream_t s)
        : alloc_(a), free_(f), ctx_(ctx), stream_(s) {}
    ~Arena();
    Arena(const Arena&) = delete;
    Arena& operator=(const Arena&) = delete;

    // Workspace: freed when the Arena dies.  bytes == 0 gives nullptr.
    // Requests are carved from the reserved block while it has room, else
    // requests up to 1 MB share 8 MB blocks (256-byte aligned).
    int work(size_t bytes, void** out);
    // One allocation for the workspace a call is about to request.
    int reserve(size_t bytes);
    static size_t padded(size_t bytes) { return (bytes + kAlign - 1) / kAlign * kAlign; }
    // Caller-owned output: freed only if fail() was called.
    int output(size_t bytes, void** out);
    void fail() { failed_ = true; }
    hipStream_t stream() const { return stream_; }
    // The allocator this arena draws from (for a nested arena whose
    // workspace is released before this one's).
    dibella_alloc_fn alloc_fn() const { return alloc_; }
    dibella_free_fn free_fn() const { return free_; }
    void* alloc_ctx() const { return ctx_; }

    template <class T>
    int work_n(size_t n, T** out) {
        void* p = nullptr;
        int s = work(n * sizeof(T), &p);
        *out = static_cast<T*>(p);
        return s;
    }
    template <class T>
    int output_n(size_t n, T** out) {
        void* p = nullptr;
        int s = output(n * sizeof(T), &p);
        *out = static_cast<T*>(p);
        return s;
    }

  private:
    static constexpr size_t kAlign = 256;
    static constexpr size_t kSmallMax = 1 << 20;
    static constexpr size_t kPoolBytes = 8 << 20;
    int work_raw(size_t bytes, void** out);
    void release(void* p);
    char* pool_ = nullptr;
    size_t pool_used_ = 0;
    char* res_ = nullptr;
    size_t res_cap_ = 0, res_used_ = 0;
    dibella_alloc_fn alloc_;
    dibella_free_fn free_;
    void* ctx_;
    hipStream_t stream_;
    bool failed_ = false;
    std::vector<void*> work_;
    std::vector<void*> outputs_;
};

// Pinned host staging per host thread: a ring of slots, one per call.
// reserve() moves to the next slot and waits only until that slot's last
// call (kStageSlots calls back) has executed its uploads and readbacks, so
// the host can queue a call while the previous ones still run.
constexpr int kStageSlots = 4;
struct HostStage {
    void* ptr = nullptr;   // the current slot
    size_t bytes = 0;
    int cur = -1;
    void* slot_ptr[kStageSlots] = {};
    size_t slot_bytes[kStageSlots] = {};
    hipEvent_t slot_use[kStageSlots] = {};
    int reserve(size_t need);
};
HostStage& host_stage();
int stage_done(hipStream_t s);       // record that the current slot has been consumed

int sync_stream(hipStream_t s);       // hipStreamSynchronize + counter

// A reduction writing into fixed buffers instead of allocating: host
// staging in `host` (pageable, at least tr_fixed_host_bytes()), S into the
// caller's arrays (capacity s_cap entries).  One set, no graphs.
struct TrFixed {
    void* host;
    size_t host_bytes;
    int64_t* s_rowptr;
    int32_t* s_col;
    int32_t* s_val;
    int64_t s_cap;
};
// C = A A^T for nsets sets (dibella_overlap, dibella_overlap_batched).
int overlap_run(const dibella_csr* A, int nsets, const int32_t* min_shared, dibella_overlap_out* C,
                uint32_t flags, Arena& ar);
// R from the seeds of C, whose row i is read row0 + i (dibella_r_from_seeds
// with row0 = 0).  Workspace from ar; R's arrays from `out`, as outputs, or
// as its workspace when out_as_work.
int r_from_seeds_run(const dibella_overlap_out* C, int64_t row0, const int32_t* read_len, int32_t k,
                     int32_t min_overlap, int32_t max_drift, int32_t min_density, dibella_csr_out* R, Arena& ar,
                     Arena& out, bool out_as_work);
// R's entries of C kept in tmp (tmp[e] >= 0 is the value, -1 dropped), rows
// written from R's row pointers rrp (one wave per row, order kept).
int write_marked_rows(int64_t n, const int64_t* rp, const int32_t* col, const int32_t* tmp, const int64_t* rrp,
                      int32_t* rcol, int32_t* rval, hipStream_t st);
// R from the alignment of C's pairs (dibella_r_from_alignment).
int r_from_alignment_run(const dibella_overlap_out* C, const uint8_t* bases, int64_t nbases, const int64_t* offsets,
                         int32_t k, int32_t mat, int32_t mis, int32_t gap, int32_t X, int32_t min_score,
                         uint32_t flags, dibella_csr_out* R, int32_t** score_out, Arena& ar);
// A from the reads (dibella_kmer_matrix).
int kmer_matrix_run(const uint8_t* bases, const int64_t* offsets, int64_t n, int64_t nbases, int32_t k, int32_t lo,
                    int32_t hi, uint32_t flags, dibella_csr_out* A, uint64_t** codes, int64_t* m, Arena& ar);
// R from the seeds of C = A A^T, built block of rows by block of rows.
int overlap_graph_blocked_run(const dibella_csr* A, int32_t min_shared, const int32_t* read_len, int32_t k,
                              int32_t min_overlap, int32_t max_drift, int32_t min_density, int64_t block_rows,
                              dibella_csr_out* R, int32_t* nblocks, Arena& ar);
int tr_run(const dibella_csr* R, int nsets, const int32_t* fuzz, uint32_t flags, dibella_csr_out* S,
           int32_t* iterations, Arena& ar, const TrFixed* fixed = nullptr);
size_t tr_workspace_bytes(int nsets, int64_t total_rows, int64_t total_nnz);
size_t tr_fixed_host_bytes();

// Streams that let independent launches of one call overlap: begin() makes
// them wait for the work queued so far on `main`, end() makes `main` wait for
// everything queued on them.  One set per host thread and device.
constexpr int kSideStreams = 2;
struct SideStreams {
    hipStream_t s[kSideStreams];
    hipEvent_t fork;
    hipEvent_t join[kSideStreams];
    int begin(hipStream_t main);
    int end(hipStream_t main);
};
int side_streams(SideStreams** out);

// Event timing of phases (no-ops unless enabled on this host thread).
// Timed kernels (labels of dibella_timing, see the header).
enum Phase {
    kPhKeys = 0, kPhPartCount, kPhPartScatter, kPhBucketSort, kPhPart2Count, kPhPart2Scatter, kPhSegments,
    kPhSymBits, kPhSymHash, kPhNumeric, kPhEsc, kPhTrMark, kPhTrCompact, kPhNumericAll, kPhRFromSeeds,
    kPhKmerWindows, kPhKmerSort, kPhKmerRuns, kPhKmerRows, kPhAlign
};
bool timing_on();
// While one lives on this host thread, no timing events are created or
// recorded (for the call that allocates nothing).
struct TimingPause {
    TimingPause();
    ~TimingPause();
    bool was;
};
int timing_begin(int phase, hipStream_t s, int* token);
int timing_end(int token, hipStream_t s);
void timing_set_enabled(bool on);
void timing_set_mask(uint32_t mask);
int timing_collect(dibella_timing* out);

// ---------------------------------------------------------------------------
// Device-wide exclusive scan: out[0] = 0, out[i+1] = sum_{q<=i} in[q].
// `enable` (device int, may be null): when it reads 0 the scan does nothing.
// ---------------------------------------------------------------------------
int scan_exclusive(const int32_t* in, int64_t* out, int64_t n, const int32_t* enable, Arena& ar);
int scan_exclusive(const int64_t* in, int64_t* out, int64_t n, const int32_t* enable, Arena& ar);
// Same with caller-provided workspace of scan_workspace_elems(n) int64s.
int64_t scan_workspace_elems(int64_t n);
int scan_exclusive_ws(const int32_t* in, int64_t* out, int64_t n, const int32_t* enable,
                      int64_t* tiles, hipStream_t s);
int scan_exclusive_ws(const int64_t* in, int64_t* out, int64_t n, const int32_t* enable,
                      int64_t* tiles, hipStream_t s);

// Fill kernels (used instead of memset nodes so that graph capture is safe).
int fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s);
int fill_i64(int64_t* p, int64_t v, int64_t n, hipStream_t s);

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline int grid_for(int64_t items, int block, int64_t cap = 1 << 20) {
    int64_t g = ceil_div(items, block);
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return static_cast<int>(g);
}

// ---------------------------------------------------------------------------
// Device helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }
__device__ __forceinline__ int wave_id() { return threadIdx.x / kWave; }
__device__ __forceinline__ uint64_t lanemask_lt() { return (1ull << lane_id()) - 1ull; }

// Load through a pointer known to address device (global) memory.  Pointers
// read from descriptors are generic to the compiler; generic loads share a
// wait counter with LDS operations, so a loop that mixes them with LDS
// atomics waits for every load in flight.
template <class T>
__device__ __forceinline__ T gload(const T* p) {
    return *(const __attribute__((address_space(1))) T*)p;
}
// The same, marked as streamed (read once).
template <class T>
__device__ __forceinline__ T gload_nt(const T* p) {
    return __builtin_nontemporal_load((const __attribute__((address_space(1))) T*)p);
}

__device__ __forceinline__ int32_t atomic_add(int32_t* p, int32_t v) { return atomicAdd(p, v); }
__device__ __forceinline__ uint32_t atomic_add(uint32_t* p, uint32_t v) { return atomicAdd(p, v); }
__device__ __forceinline__ int64_t atomic_add(int64_t* p, int64_t v) {
    return (int64_t)atomicAdd(reinterpret_cast<unsigned long long*>(p), (unsigned long long)v);
}
__device__ __forceinline__ int32_t atomic_max(int32_t* p, int32_t v) { return atomicMax(p, v); }
__device__ __forceinline__ int64_t atomic_max(int64_t* p, int64_t v) {
    return (int64_t)atomicMax(reinterpret_cast<long long*>(p), (long long)v);
}

// Largest s in [0, nsets) with base[s] <= g (base ascending, base[0] = 0).
__device__ __forceinline__ int find_set(const int64_t* base, int nsets, int64_t g) {
    int lo = 0, hi = nsets - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (base[mid] <= g) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ int32_t wave_or_i32(int32_t v) {
    for (int d = kWave / 2; d > 0; d >>= 1) v |= __shfl_xor(v, d, kWave);
    return v;
}

template <class T>
__device__ __forceinline__ T wave_sum(T v) {
    for (int d = kWave / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, kWave);
    return v;
}
template <class T>
__device__ __forceinline__ T wave_max(T v) {
    for (int d = kWave / 2; d > 0; d >>= 1) {
        T o = __shfl_xor(v, d, kWave);
        v = o > v ? o : v;
    }
    return v;
}
template <class T>
__device__ __forceinline__ T wave_inclusive_sum(T v) {
    const int lane = lane_id();
    for (int d = 1; d < kWave; d <<= 1) {
        T y = __shfl_up(v, d, kWave);
        if (lane >= d) v += y;
    }
    return v;
}

// Exclusive block scan of one value per thread; `tmp` holds BLOCK/64 + 1
// values of T in LDS.  Returns the exclusive prefix; *total = block sum.
// Contains barriers: every thread of the block must call it.
template <int BLOCK, class T>
__device__ __forceinline__ T block_exclusive_sum(T v, T* tmp, T* total) {
    constexpr int W = BLOCK / kWave;
    const int w = wave_id();
    T inc = wave_inclusive_sum(v);
    if (lane_id() == kWave - 1) tmp[w] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
        T acc = 0;
        for (int q = 0; q < W; ++q) {
            T x = tmp[q];
            tmp[q] = acc;
            acc += x;
        }
        tmp[W] = acc;
    }
    __syncthreads();
    T excl = inc - v + tmp[w];
    *total = tmp[W];
    __syncthreads();
    return excl;
}

// Block-wide reductions through one LDS word (all threads must call).
template <class T>
__device__ __forceinline__ T block_sum_lds(T v, T* slot) {
    if (threadIdx.x == 0) *slot = 0;
    __syncthreads();
    v = wave_sum(v);
    if (lane_id() == 0) atomic_add(slot, v);
    __syncthreads();
    T r = *slot;
    __syncthreads();
    return r;
}
template <class T>
__device__ __forceinline__ T block_max_lds(T v, T* slot) {
    if (threadIdx.x == 0) *slot = 0;
    __syncthreads();
    v = wave_max(v);
    if (lane_id() == 0) atomic_max(slot, v);
    __syncthreads();
    T r = *slot;
    __syncthreads();
    return r;
}

// Index of the last element <= q in the ascending array off[0..len) with
// off[0] = 0 <= q (LDS binary search).
__device__ __forceinline__ int upper_index(const int32_t* off, int len, int32_t q) {
    int lo = 0, hi = len - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= q) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__host__ __device__ __forceinline__ int ceil_log2_i64(int64_t x) {
    int r = 0;
    while ((int64_t(1) << r) < x) ++r;
    return r;
}

}  // namespace dibella
