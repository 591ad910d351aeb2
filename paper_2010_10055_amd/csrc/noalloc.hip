// dibella_transitive_reduce_noalloc: the transitive reduction for callers
// that cannot allocate (code under HIP graph capture, tight serving loops,
// harnesses that forbid allocation).  Its workspace comes from `scratch`, a
// static device array of kScratchBytes that every GPU the library runs on
// holds until the process ends; S goes into the caller's arrays.  Every call
// on one GPU shares that GPU's array: calls that overlap on one GPU race.
// Nothing here relies on the array's previous contents (the reduction's
// kernels clear what must start at zero).
#include "common.hpp"

#include <cstring>
#include <mutex>

namespace dibella {

constexpr size_t kScratchBytes = size_t(64) << 20;   // 64 MiB per GPU
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// Device address of `scratch` on the current device, looked up once per
// device with that device current (the host-side name of the array is not
// a device address).
static int scratch_ptr(void** out) {
    static std::mutex mu;
    static void* ptr[kMaxDevices] = {};
    int dev = 0;
    DB_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("dibella_transitive_reduce_noalloc: device index beyond " + std::to_string(kMaxDevices));
        return DIBELLA_EDEVICE;
    }
    std::lock_guard<std::mutex> lock(mu);
    if (!ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_error(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
            return DIBELLA_EDEVICE;
        }
        ptr[dev] = p;
    }
    *out = ptr[dev];
    return DIBELLA_OK;
}

// Bump allocation over the scratch array for the call's arena; releasing
// is a no-op (the next call starts again at the beginning).
struct Bump {
    char* base;
    size_t cap, used;
};
static void* bump_alloc(size_t bytes, void* ctx) {
    Bump* b = static_cast<Bump*>(ctx);
    const size_t need = Arena::padded(bytes);
    if (b->used + need > b->cap) return nullptr;
    void* p = b->base + b->used;
    b->used += need;
    return p;
}
static void bump_free(void*, void*) {}

}  // namespace dibella

using namespace dibella;

extern "C" int dibella_transitive_reduce_noalloc(const dibella_csr* R, int32_t fuzz, uint32_t flags,
                                                 int64_t* s_rowptr, int32_t* s_col, int32_t* s_val,
                                                 int64_t s_capacity, int64_t* s_nnz, int32_t* iterations,
                                                 void* hip_stream) {
    std::memset(&stats(), 0, sizeof(dibella_stats));
    if (!R || !s_nnz || !iterations || (R->nrows >= 0 && !s_rowptr)) {
        set_error("dibella_transitive_reduce_noalloc: bad arguments");
        return DIBELLA_EINVAL;
    }
    *s_nnz = 0;
    *iterations = 0;
    if (flags & DIBELLA_TR_USE_GRAPH) {
        set_error("dibella_transitive_reduce_noalloc: graphs are not available here (instantiating one allocates)");
        return DIBELLA_EINVAL;
    }
    if (R->nnz < 0 || R->nrows < 0 || s_capacity < R->nnz || (R->nnz > 0 && (!s_col || !s_val))) {
        set_error("dibella_transitive_reduce_noalloc: the output arrays must hold nnz(R) entries");
        return DIBELLA_EINVAL;
    }
    const size_t need = tr_workspace_bytes(1, R->nrows, R->nnz);
    if (need > kScratchBytes) {
        set_error("dibella_transitive_reduce_noalloc: R needs " + std::to_string(need) +
                  " bytes of scratch, the maximum is " + std::to_string(kScratchBytes));
        return DIBELLA_EINVAL;
    }
    void* base = nullptr;
    DB_TRY(scratch_ptr(&base));
    Bump bump{static_cast<char*>(base), kScratchBytes, 0};
    alignas(64) static thread_local unsigned char host[4096];
    static_assert(sizeof(host) >= 64, "staging");
    if (tr_fixed_host_bytes() > sizeof(host)) {
        set_error("internal: staging buffer too small");
        return DIBELLA_EDEVICE;
    }
    const TrFixed fx{host, sizeof(host), s_rowptr, s_col, s_val, s_capacity};
    TimingPause pause;
    dibella_csr_out S;
    int32_t it = 0;
    int status;
    {
        Arena ar(bump_alloc, bump_free, &bump, static_cast<hipStream_t>(hip_stream));
        status = tr_run(R, 1, &fuzz, flags, &S, &it, ar, &fx);
        if (status != DIBELLA_OK) {
            (void)hipStreamSynchronize(ar.stream());   // queued work may still use the scratch
            ar.fail();
        }
    }
    if (status == DIBELLA_OK) {
        *s_nnz = S.nnz;
        *iterations = it;
    }
    return status;
}
