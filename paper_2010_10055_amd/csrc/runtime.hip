// Runtime pieces shared by both products: error slot, tuning, statistics,
// allocation arena, pinned staging, fill kernels and the device-wide scan.
#include "common.hpp"

#include <cstring>
#include <mutex>

namespace dibella {

// ---------------------------------------------------------------------------
// Errors / tuning / stats
// ---------------------------------------------------------------------------
std::string& error_slot() {
    static thread_local std::string msg;
    return msg;
}
void set_error(const std::string& msg) { error_slot() = msg; }

namespace {
std::mutex& tuning_mutex() {
    static std::mutex mu;
    return mu;
}
dibella_tuning& tuning_slot() {
    static dibella_tuning t = {
        /*sym_block*/ 256, /*num_block*/ 256, /*tr_block*/ 128,
        /*sym_first_log2*/ 12, /*sym_max_log2*/ 14, /*num_max_entries*/ 5120,
        /*load_pct*/ 75, /*tr_lds_cap*/ 4096, /*tr_graph_passes*/ 4,
        /*bits_max_words*/ 8192};
    return t;
}
}  // namespace

// Each call takes one copy at its start, so a concurrent set_tuning never
// changes the shapes within a call.
dibella_tuning tuning() {
    std::lock_guard<std::mutex> lock(tuning_mutex());
    return tuning_slot();
}
void tuning_store(const dibella_tuning& t) {
    std::lock_guard<std::mutex> lock(tuning_mutex());
    tuning_slot() = t;
}

dibella_stats& stats() {
    static thread_local dibella_stats s;
    return s;
}

// ---------------------------------------------------------------------------
// Arena
// ---------------------------------------------------------------------------
int Arena::work(size_t bytes, void** out) {
    *out = nullptr;
    if (bytes == 0) return DIBELLA_OK;
    // small requests are carved from pooled blocks: one allocator call
    // serves many of them (allocator callbacks cost host time per call)
    const size_t need = (bytes + kAlign - 1) / kAlign * kAlign;
    if (res_ && res_used_ + need <= res_cap_) {
        *out = res_ + res_used_;
        res_used_ += need;
        return DIBELLA_OK;
    }
    if (need <= kSmallMax) {
        if (!pool_ || pool_used_ + need > kPoolBytes) {
            void* blk = nullptr;
            DB_TRY(work_raw(kPoolBytes, &blk));
            pool_ = static_cast<char*>(blk);
            pool_used_ = 0;
        }
        *out = pool_ + pool_used_;
        pool_used_ += need;
        return DIBELLA_OK;
    }
    return work_raw(bytes, out);
}

int Arena::reserve(size_t bytes) {
    void* blk = nullptr;
    DB_TRY(work_raw(bytes, &blk));
    res_ = static_cast<char*>(blk);
    res_cap_ = bytes;
    res_used_ = 0;
    return DIBELLA_OK;
}

int Arena::work_raw(size_t bytes, void** out) {
    void* p = nullptr;
    if (alloc_) {
        p = alloc_(bytes, ctx_);
    } else {
        if (hipMallocAsync(&p, bytes, stream_) != hipSuccess) p = nullptr;
    }
    if (!p) {
        set_error("allocation of " + std::to_string(bytes) + " bytes failed");
        return DIBELLA_ENOMEM;
    }
    work_.push_back(p);
    *out = p;
    return DIBELLA_OK;
}

int Arena::output(size_t bytes, void** out) {
    *out = nullptr;
    if (bytes == 0) return DIBELLA_OK;
    void* p = nullptr;
    if (alloc_) {
        p = alloc_(bytes, ctx_);
    } else {
        if (hipMallocAsync(&p, bytes, stream_) != hipSuccess) p = nullptr;
    }
    if (!p) {
        set_error("allocation of " + std::to_string(bytes) + " bytes failed");
        return DIBELLA_ENOMEM;
    }
    outputs_.push_back(p);
    *out = p;
    return DIBELLA_OK;
}

void Arena::release(void* p) {
    if (free_) free_(p, ctx_);
    else (void)hipFreeAsync(p, stream_);
}

Arena::~Arena() {
    for (auto it = work_.rbegin(); it != work_.rend(); ++it) release(*it);
    if (failed_)
        for (auto it = outputs_.rbegin(); it != outputs_.rend(); ++it) release(*it);
}

// ---------------------------------------------------------------------------
// Pinned staging
// ---------------------------------------------------------------------------
HostStage& host_stage() {
    static thread_local HostStage st;
    return st;
}

int HostStage::reserve(size_t need) {
    cur = (cur + 1) % kStageSlots;
    if (slot_use[cur]) DB_HIP(hipEventSynchronize(slot_use[cur]));
    if (need > slot_bytes[cur]) {
        if (slot_ptr[cur]) DB_HIP(hipHostFree(slot_ptr[cur]));
        slot_ptr[cur] = nullptr;
        slot_bytes[cur] = 0;
        size_t cap = 4096;
        while (cap < need) cap <<= 1;
        DB_HIP(hipHostMalloc(&slot_ptr[cur], cap, hipHostMallocDefault));
        slot_bytes[cur] = cap;
    }
    ptr = slot_ptr[cur];
    bytes = slot_bytes[cur];
    return DIBELLA_OK;
}

int stage_done(hipStream_t s) {
    HostStage& st = host_stage();
    if (st.cur < 0) return DIBELLA_OK;
    if (!st.slot_use[st.cur]) DB_HIP(hipEventCreateWithFlags(&st.slot_use[st.cur], hipEventDisableTiming));
    DB_HIP(hipEventRecord(st.slot_use[st.cur], s));
    return DIBELLA_OK;
}

// ---------------------------------------------------------------------------
// Side streams (per host thread and device, default priority, non-blocking)
// ---------------------------------------------------------------------------
namespace {
struct SideSet {
    int dev = -1;
    SideStreams ss;
};
}  // namespace

int side_streams(SideStreams** out) {
    static thread_local std::vector<SideSet> sets;
    int dev = 0;
    DB_HIP(hipGetDevice(&dev));
    for (auto& x : sets)
        if (x.dev == dev) {
            *out = &x.ss;
            return DIBELLA_OK;
        }
    SideSet x;
    x.dev = dev;
    for (int k = 0; k < kSideStreams; ++k) {
        DB_HIP(hipStreamCreateWithFlags(&x.ss.s[k], hipStreamNonBlocking));
        DB_HIP(hipEventCreateWithFlags(&x.ss.join[k], hipEventDisableTiming));
    }
    DB_HIP(hipEventCreateWithFlags(&x.ss.fork, hipEventDisableTiming));
    sets.push_back(x);
    *out = &sets.back().ss;
    return DIBELLA_OK;
}

int SideStreams::begin(hipStream_t main) {
    DB_HIP(hipEventRecord(fork, main));
    for (int k = 0; k < kSideStreams; ++k) DB_HIP(hipStreamWaitEvent(s[k], fork, 0));
    return DIBELLA_OK;
}

int SideStreams::end(hipStream_t main) {
    for (int k = 0; k < kSideStreams; ++k) {
        DB_HIP(hipEventRecord(join[k], s[k]));
        DB_HIP(hipStreamWaitEvent(main, join[k], 0));
    }
    return DIBELLA_OK;
}

int sync_stream(hipStream_t s) {
    DB_HIP(hipStreamSynchronize(s));
    stats().host_syncs++;
    return DIBELLA_OK;
}

// ---------------------------------------------------------------------------
// Phase timing
// ---------------------------------------------------------------------------
namespace {
struct TimingRec {
    int phase;
    hipEvent_t a, b;
};
struct TimingState {
    bool on = false;
    bool paused = false;
    uint32_t mask = ~0u;   // labels recorded while on (bit i = label i)
    std::vector<TimingRec> recs;
    std::vector<hipEvent_t> pool;
    ~TimingState() {
        for (auto& r : recs) {
            (void)hipEventDestroy(r.a);
            (void)hipEventDestroy(r.b);
        }
        for (auto e : pool) (void)hipEventDestroy(e);
    }
};
TimingState& tstate() {
    static thread_local TimingState t;
    return t;
}
int take_event(hipEvent_t* e) {
    TimingState& t = tstate();
    if (!t.pool.empty()) {
        *e = t.pool.back();
        t.pool.pop_back();
        return DIBELLA_OK;
    }
    DB_HIP(hipEventCreate(e));
    return DIBELLA_OK;
}
}  // namespace

bool timing_on() { return tstate().on; }

TimingPause::TimingPause() : was(tstate().paused) { tstate().paused = true; }
TimingPause::~TimingPause() { tstate().paused = was; }

int timing_begin(int phase, hipStream_t s, int* token) {
    *token = -1;
    TimingState& t = tstate();
    if (!t.on || t.paused || phase < 0 || phase >= 32 || !((t.mask >> phase) & 1u)) return DIBELLA_OK;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    DB_HIP(hipStreamIsCapturing(s, &cs));
    if (cs != hipStreamCaptureStatusNone) return DIBELLA_OK;
    TimingRec r{phase, nullptr, nullptr};
    DB_TRY(take_event(&r.a));
    DB_TRY(take_event(&r.b));
    DB_HIP(hipEventRecord(r.a, s));
    t.recs.push_back(r);
    *token = (int)t.recs.size() - 1;
    return DIBELLA_OK;
}

int timing_end(int token, hipStream_t s) {
    if (token < 0) return DIBELLA_OK;
    DB_HIP(hipEventRecord(tstate().recs[token].b, s));
    return DIBELLA_OK;
}

void timing_set_mask(uint32_t mask) { tstate().mask = mask; }

void timing_set_enabled(bool on) {
    TimingState& t = tstate();
    for (auto& r : t.recs) {
        t.pool.push_back(r.a);
        t.pool.push_back(r.b);
    }
    t.recs.clear();
    t.on = on;
}

int timing_collect(dibella_timing* out) {
    std::memset(out, 0, sizeof(*out));
    TimingState& t = tstate();
    for (auto& r : t.recs) {
        DB_HIP(hipEventSynchronize(r.b));
        float ms = 0.f;
        DB_HIP(hipEventElapsedTime(&ms, r.a, r.b));
        if (r.phase >= 0 && r.phase < DIBELLA_NUM_PHASES) {
            out->ms[r.phase] += ms;
            out->records[r.phase] += 1;
        }
        t.pool.push_back(r.a);
        t.pool.push_back(r.b);
    }
    t.recs.clear();
    return DIBELLA_OK;
}

// ---------------------------------------------------------------------------
// Fills
// ---------------------------------------------------------------------------
template <class T>
__global__ void k_fill(T* __restrict__ p, T v, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

int fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s) {
    if (n <= 0) return DIBELLA_OK;
    hipLaunchKernelGGL(k_fill<int32_t>, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, p, v, n);
    DB_HIP(hipGetLastError());
    return DIBELLA_OK;
}
int fill_i64(int64_t* p, int64_t v, int64_t n, hipStream_t s) {
    if (n <= 0) return DIBELLA_OK;
    hipLaunchKernelGGL(k_fill<int64_t>, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, p, v, n);
    DB_HIP(hipGetLastError());
    return DIBELLA_OK;
}

// ---------------------------------------------------------------------------
// Device-wide exclusive scan (reduce, then scan of tile sums, then
// downsweep).  Tile = 256 threads x 8 items.
// ---------------------------------------------------------------------------
constexpr int kScanBlock = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanBlock * kScanItems;

template <class T>
__global__ __launch_bounds__(kScanBlock) void k_scan_reduce(const T* __restrict__ in, int64_t n,
                                                            int64_t* __restrict__ tile_sum,
                                                            const int32_t* enable) {
    if (enable && *enable == 0) return;
    __shared__ int64_t slot;
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    int64_t acc = 0;
    for (int q = 0; q < kScanItems; ++q) {
        int64_t i = base + (int64_t)q * kScanBlock + threadIdx.x;
        if (i < n) acc += (int64_t)in[i];
    }
    acc = block_sum_lds(acc, &slot);
    if (threadIdx.x == 0) tile_sum[blockIdx.x] = acc;
}

// One block scans all tile sums in place (exclusive) and writes the total.
__global__ __launch_bounds__(kScanBlock) void k_scan_tiles(int64_t* __restrict__ tile_sum,
                                                           int64_t ntiles, int64_t* __restrict__ total,
                                                           const int32_t* enable) {
    if (enable && *enable == 0) return;
    __shared__ int64_t tmp[kScanBlock / kWave + 1];
    int64_t carry = 0;
    for (int64_t b = 0; b < ntiles; b += kScanBlock) {
        int64_t i = b + threadIdx.x;
        int64_t v = i < ntiles ? tile_sum[i] : 0;
        int64_t tot;
        int64_t ex = block_exclusive_sum<kScanBlock>(v, tmp, &tot);
        if (i < ntiles) tile_sum[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) *total = carry;
}

template <class T>
__global__ __launch_bounds__(kScanBlock) void k_scan_down(const T* __restrict__ in, int64_t n,
                                                          const int64_t* __restrict__ tile_sum,
                                                          int64_t* __restrict__ out,
                                                          const int32_t* enable) {
    if (enable && *enable == 0) return;
    __shared__ int64_t tmp[kScanBlock / kWave + 1];
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    // Each thread owns kScanItems consecutive elements.
    int64_t v[kScanItems];
    int64_t local = 0;
    const int64_t my = base + (int64_t)threadIdx.x * kScanItems;
#pragma unroll
    for (int q = 0; q < kScanItems; ++q) {
        int64_t i = my + q;
        v[q] = i < n ? (int64_t)in[i] : 0;
        local += v[q];
    }
    int64_t tot;
    int64_t ex = block_exclusive_sum<kScanBlock>(local, tmp, &tot);
    int64_t run = tile_sum[blockIdx.x] + ex;
    if (blockIdx.x == 0 && threadIdx.x == 0) out[0] = 0;
#pragma unroll
    for (int q = 0; q < kScanItems; ++q) {
        int64_t i = my + q;
        run += v[q];
        if (i < n) out[i + 1] = run;
    }
}

int64_t scan_workspace_elems(int64_t n) { return n <= 0 ? 0 : ceil_div(n, kScanTile) + 1; }

template <class T>
static int scan_impl(const T* in, int64_t* out, int64_t n, const int32_t* enable, int64_t* tiles,
                     hipStream_t s) {
    if (n <= 0) return fill_i64(out, 0, 1, s);   // out[0] = 0 only
    const int64_t ntiles = ceil_div(n, kScanTile);
    hipLaunchKernelGGL(k_scan_reduce<T>, dim3((unsigned)ntiles), dim3(kScanBlock), 0, s, in, n,
                       tiles, enable);
    hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(kScanBlock), 0, s, tiles, ntiles,
                       tiles + ntiles, enable);
    hipLaunchKernelGGL(k_scan_down<T>, dim3((unsigned)ntiles), dim3(kScanBlock), 0, s, in, n,
                       tiles, out, enable);
    DB_HIP(hipGetLastError());
    return DIBELLA_OK;
}

int scan_exclusive_ws(const int32_t* in, int64_t* out, int64_t n, const int32_t* enable,
                      int64_t* tiles, hipStream_t s) {
    return scan_impl(in, out, n, enable, tiles, s);
}
int scan_exclusive_ws(const int64_t* in, int64_t* out, int64_t n, const int32_t* enable,
                      int64_t* tiles, hipStream_t s) {
    return scan_impl(in, out, n, enable, tiles, s);
}

int scan_exclusive(const int32_t* in, int64_t* out, int64_t n, const int32_t* enable, Arena& ar) {
    int64_t* tiles = nullptr;
    DB_TRY(ar.work_n(scan_workspace_elems(n), &tiles));
    return scan_impl(in, out, n, enable, tiles, ar.stream());
}
int scan_exclusive(const int64_t* in, int64_t* out, int64_t n, const int32_t* enable, Arena& ar) {
    int64_t* tiles = nullptr;
    DB_TRY(ar.work_n(scan_workspace_elems(n), &tiles));
    return scan_impl(in, out, n, enable, tiles, ar.stream());
}

}  // namespace dibella
