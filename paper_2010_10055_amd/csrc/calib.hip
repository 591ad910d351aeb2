// Reference kernels of known HBM traffic.  They are not part of the library:
// the benchmark profiles them beside the library's kernels to learn how the
// L2-to-memory request counters weigh each access pattern (full-line
// streams, one touch per 64 or 128 bytes, random 4-byte gathers), and so to
// turn those counters into bytes.
//
// Every entry point takes device pointers and a HIP stream, launches one
// kernel and returns 0, or -1 on a bad argument or launch error.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

constexpr int kBlock = 256;
constexpr int kGrid = 256 * 16;   // 16 workgroups per CU

// Guards a reduction against dead-code elimination without writing: the
// inputs are all ones, so the sum is never this value.
constexpr float kNever = -1.0f;

__global__ __launch_bounds__(kBlock) void k_calib_read(const float4* __restrict__ x, int64_t n4,
                                                       float* __restrict__ out) {
    float acc = 0.f;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n4; i += (int64_t)gridDim.x * kBlock) {
        const float4 v = x[i];
        acc += v.x + v.y + v.z + v.w;
    }
    if (acc == kNever) out[0] = acc;
}

__global__ __launch_bounds__(kBlock) void k_calib_write(float4* __restrict__ y, int64_t n4, float v) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n4; i += (int64_t)gridDim.x * kBlock)
        y[i] = make_float4(v, v, v, v);
}

__global__ __launch_bounds__(kBlock) void k_calib_copy(const float4* __restrict__ x, float4* __restrict__ y,
                                                       int64_t n4) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n4; i += (int64_t)gridDim.x * kBlock)
        y[i] = x[i];
}

// One 4-byte read every STRIDE bytes (a template parameter, so that each
// stride is a kernel of its own name in a profile).
template <int STRIDE>
__global__ __launch_bounds__(kBlock) void k_calib_stride(const float* __restrict__ x, int64_t count,
                                                         float* __restrict__ out) {
    float acc = 0.f;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < count; i += (int64_t)gridDim.x * kBlock)
        acc += x[i * (STRIDE / 4)];
    if (acc == kNever) out[0] = acc;
}

// SplitMix64's output function (Steele, Lea and Flood, 2014): a bijective
// mix of a counter, here the source of random indices with no index stream.
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// `count` random 4-byte reads over x[0, n).
__global__ __launch_bounds__(kBlock) void k_calib_gather(const float* __restrict__ x, int64_t n, int64_t count,
                                                         uint64_t seed, float* __restrict__ out) {
    float acc = 0.f;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < count; i += (int64_t)gridDim.x * kBlock)
        acc += x[mix64(seed + (uint64_t)i) % (uint64_t)n];
    if (acc == kNever) out[0] = acc;
}

int done() { return hipGetLastError() == hipSuccess ? 0 : -1; }

}  // namespace

extern "C" {

// Reads `bytes` (a multiple of 16) from x.
int calib_read(const void* x, int64_t bytes, void* out, void* stream) {
    if (!x || !out || bytes <= 0 || bytes % 16) return -1;
    hipLaunchKernelGGL(k_calib_read, dim3(kGrid), dim3(kBlock), 0, (hipStream_t)stream,
                       (const float4*)x, bytes / 16, (float*)out);
    return done();
}

// Writes `bytes` (a multiple of 16) to y.
int calib_write(void* y, int64_t bytes, void* stream) {
    if (!y || bytes <= 0 || bytes % 16) return -1;
    hipLaunchKernelGGL(k_calib_write, dim3(kGrid), dim3(kBlock), 0, (hipStream_t)stream, (float4*)y, bytes / 16,
                       1.0f);
    return done();
}

// Copies `bytes` (a multiple of 16) from x to y.
int calib_copy(const void* x, void* y, int64_t bytes, void* stream) {
    if (!x || !y || bytes <= 0 || bytes % 16) return -1;
    hipLaunchKernelGGL(k_calib_copy, dim3(kGrid), dim3(kBlock), 0, (hipStream_t)stream, (const float4*)x,
                       (float4*)y, bytes / 16);
    return done();
}

// Reads one float every `stride_bytes` (64 or 128) over `bytes` of x.
int calib_stride(const void* x, int64_t bytes, int32_t stride_bytes, void* out, void* stream) {
    if (!x || !out || bytes <= 0 || (stride_bytes != 64 && stride_bytes != 128)) return -1;
    if (stride_bytes == 64)
        hipLaunchKernelGGL(k_calib_stride<64>, dim3(kGrid), dim3(kBlock), 0, (hipStream_t)stream, (const float*)x,
                           bytes / 64, (float*)out);
    else
        hipLaunchKernelGGL(k_calib_stride<128>, dim3(kGrid), dim3(kBlock), 0, (hipStream_t)stream,
                           (const float*)x, bytes / 128, (float*)out);
    return done();
}

// `count` random 4-byte reads over `bytes` of x.
int calib_gather(const void* x, int64_t bytes, int64_t count, uint64_t seed, void* out, void* stream) {
    if (!x || !out || bytes < 4 || count <= 0) return -1;
    hipLaunchKernelGGL(k_calib_gather, dim3(kGrid), dim3(kBlock), 0, (hipStream_t)stream, (const float*)x,
                       bytes / 4, count, seed, (float*)out);
    return done();
}

}  // extern "C"
