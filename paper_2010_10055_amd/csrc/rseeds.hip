// Overlap graph R from the seeds stored in C (Sec. IV-E: the reduction's
// overlap suffix and orientation are derived in place from the coordinates
// stored with each read pair; Sec. IV-D: C keeps two k-mer positions per
// pair).  The first seed of C_ij is the pair (p_i << 1 | strand_i,
// p_j << 1 | strand_j) of the smallest shared k-mer column, strand saying
// whether the read holds the canonical k-mer as is or reverse complemented.
// Extending the seed without gaps places read j (reverse complemented if the
// strands differ) at offset d in read i's frame:
//   d = p_i - p_j                   (same strand)
//   d = p_i + p_j + k - L_j         (reverse-complementary pair)
// With max_drift >= 0 the second seed must place the pair in the same
// relative orientation at an offset within max_drift bases of the first
// (else the entry is dropped).  The overlap spans [max(0, d),
// min(L_i, d + L_j)).  Pairs overlapping by fewer than min_overlap bases are
// dropped, and with min_density > 0 so are pairs sharing fewer than
// min_density k-mers per 10 kbp of overlap (count * 10000 < min_density *
// overlap: a repeat shared by two reads that do not overlap gives k-mers
// along the repeat only).  A contained overlap is kept with value 0, and
// otherwise the four categories of overlap give the entry
//   read i first (forward / inner):   suffix d + L_j - L_i, code (0, rc)
//   read j first (reverse / outer):   suffix -d,            code (1, 1 - rc)
// packed (suffix << 2) | code.  Two passes, one wave per row: the first
// computes every entry's value (or -1 when dropped) and the row's count,
// a scan gives R's row pointers, the second compacts with wave ballots.
// C may hold a block of consecutive rows of the whole matrix: row i of C is
// then read row0 + i, and its columns range over all reads.
#include "common.hpp"

#include <cstring>

namespace dibella {

enum : int32_t {
    kRsBadRowptr = 1,
    kRsBadCol = 2,
    kRsUnsorted = 4,
    kRsBadSeed = 8,
    kRsBadLength = 16,
};

constexpr int32_t kRsMaxLen = 1 << 28;   // suffixes stay below 2^28, as the reduction requires

// Offset of read j in read i's frame from one seed (a, b); rc: the pair is
// reverse-complementary.
__device__ __forceinline__ int64_t rs_offset(int32_t a, int32_t b, int64_t lj, int32_t k, bool* rc) {
    *rc = (a & 1) != (b & 1);
    const int64_t pi = a >> 1, pj = b >> 1;
    return *rc ? pi + pj + k - lj : pi - pj;
}

template <int WPB>
__global__ __launch_bounds__(WPB* kWave) void k_rs_mark(int64_t n, int64_t row0, int64_t ncols, int64_t nnz,
                                                        const int64_t* __restrict__ rp,
                                                        const int32_t* __restrict__ col,
                                                        const int32_t* __restrict__ count,
                                                        const int32_t* __restrict__ seed,
                                                        const int32_t* __restrict__ len, int32_t k, int32_t min_ov,
                                                        int32_t max_drift, int32_t min_density,
                                                        int32_t* __restrict__ tmp,
                                                        int64_t* __restrict__ cnt, int32_t* __restrict__ flags) {
    const int lane = lane_id();
    for (int64_t i = (int64_t)blockIdx.x * WPB + __builtin_amdgcn_readfirstlane(wave_id()); i < n;
         i += (int64_t)gridDim.x * WPB) {
        const int64_t lo = rp[i], hi = rp[i + 1];
        int32_t bad = 0;
        int64_t kept = 0;
        if ((i == 0 && lo != 0) || (i == n - 1 && hi != nnz) || lo < 0 || hi < lo || hi > nnz) {
            bad |= kRsBadRowptr;
        } else {
            const int64_t li = len[row0 + i];
            if (li < 0 || li >= kRsMaxLen) bad |= kRsBadLength;
            for (int64_t e = lo + lane; e < hi; e += kWave) {
                const int32_t j = col[e];
                int32_t out = -1;
                if (j < 0 || j >= ncols) {
                    bad |= kRsBadCol;
                } else {
                    if (e > lo && col[e - 1] >= j) bad |= kRsUnsorted;
                    if (j != row0 + i) {
                        const int32_t a = seed[4 * e], b = seed[4 * e + 1];
                        const int32_t a1 = seed[4 * e + 2], b1 = seed[4 * e + 3];
                        const int64_t lj = len[j];
                        if (lj < 0 || lj >= kRsMaxLen) bad |= kRsBadLength;
                        const bool second = a1 >= 0 && b1 >= 0;
                        if (a < 0 || b < 0 || (a >> 1) + k > li || (b >> 1) + k > lj ||
                            (max_drift >= 0 && second && ((a1 >> 1) + k > li || (b1 >> 1) + k > lj))) {
                            bad |= kRsBadSeed;
                        } else {
                            bool rc, rc1 = false;
                            const int64_t d = rs_offset(a, b, lj, k, &rc);
                            const int64_t d1 = second ? rs_offset(a1, b1, lj, k, &rc1) : 0;
                            // the second seed must agree (when asked for)
                            const bool agree = max_drift < 0 ||
                                               (second && rc1 == rc && d1 - d <= max_drift && d - d1 <= max_drift);
                            const int64_t ov = min(li, d + lj) - max(d, (int64_t)0);
                            const bool dense =
                                min_density <= 0 || (int64_t)count[e] * 10000 >= (int64_t)min_density * ov;
                            if (agree && dense && ov >= min_ov) {
                                if (ov == li || ov == lj) {
                                    out = 0;   // contained overlap
                                } else if (d > 0) {
                                    out = (int32_t)(((d + lj - li) << 2) | (rc ? 1 : 0));
                                } else {
                                    out = (int32_t)(((-d) << 2) | (rc ? 2 : 3));
                                }
                            }
                        }
                    }
                }
                tmp[e] = out;
                kept += out >= 0 ? 1 : 0;
            }
        }
        bad = wave_or_i32(bad);
        kept = wave_sum(kept);
        if (lane == 0) {
            cnt[i] = bad ? 0 : kept;
            if (bad) atomicOr(flags, bad);
        }
    }
}

template <int WPB>
__global__ __launch_bounds__(WPB* kWave) void k_rs_write(int64_t n, const int64_t* __restrict__ rp,
                                                         const int32_t* __restrict__ col,
                                                         const int32_t* __restrict__ tmp,
                                                         const int64_t* __restrict__ rrp, int32_t* __restrict__ rcol,
                                                         int32_t* __restrict__ rval) {
    const int lane = lane_id();
    for (int64_t i = (int64_t)blockIdx.x * WPB + __builtin_amdgcn_readfirstlane(wave_id()); i < n;
         i += (int64_t)gridDim.x * WPB) {
        const int64_t lo = rp[i], hi = rp[i + 1];
        int64_t out = rrp[i];
        for (int64_t b = lo; b < hi; b += kWave) {
            const int64_t e = b + lane;
            const int32_t v = e < hi ? tmp[e] : -1;
            const uint64_t mask = __ballot(v >= 0);
            if (v >= 0) {
                const int64_t pos = out + __popcll(mask & lanemask_lt());
                rcol[pos] = col[e];
                rval[pos] = v;
            }
            out += __popcll(mask);
        }
    }
}

int write_marked_rows(int64_t n, const int64_t* rp, const int32_t* col, const int32_t* tmp, const int64_t* rrp,
                      int32_t* rcol, int32_t* rval, hipStream_t st) {
    constexpr int WPB = 4;
    hipLaunchKernelGGL(k_rs_write<WPB>, dim3(grid_for(n, WPB, 1 << 16)), dim3(WPB * kWave), 0, st, n, rp, col, tmp,
                       rrp, rcol, rval);
    DB_HIP(hipGetLastError());
    return DIBELLA_OK;
}

static const char* describe_rs_bad(int32_t bad) {
    if (bad & kRsBadRowptr) return "row pointers of C are not a valid CSR row pointer array";
    if (bad & kRsBadCol) return "a column index of C is outside [0, ncols)";
    if (bad & kRsUnsorted) return "columns of C are not strictly increasing within a row";
    if (bad & kRsBadLength) return "a read length is negative or >= 2^28";
    if (bad & kRsBadSeed) return "a seed of an off-diagonal entry is missing or lies outside its read";
    return "malformed input";
}

int r_from_seeds_run(const dibella_overlap_out* C, int64_t row0, const int32_t* read_len, int32_t k,
                     int32_t min_overlap, int32_t max_drift, int32_t min_density, dibella_csr_out* R, Arena& ar,
                     Arena& out, bool out_as_work) {
    hipStream_t st = ar.stream();
    std::memset(R, 0, sizeof(*R));
    const int64_t n = C->nrows, nnz = C->nnz, ncols = C->ncols;
    if (n < 0 || nnz < 0 || row0 < 0 || ncols < row0 + n || k < 1 || k > 32 || min_overlap < 0) {
        set_error("dibella_r_from_seeds: C must have non-negative sizes and a column per read of its rows, "
                  "k in [1, 32], min_overlap >= 0");
        return DIBELLA_EINVAL;
    }
    if (ncols >= (int64_t(1) << 31) || nnz >= (int64_t(1) << 40)) {
        set_error("dibella_r_from_seeds: nrows must be < 2^31 and nnz < 2^40");
        return DIBELLA_EOVERFLOW;
    }
    if ((n > 0 && (!C->rowptr || !read_len)) || (nnz > 0 && (!C->col || !C->seed || !C->count))) {
        set_error("dibella_r_from_seeds: null pointer");
        return DIBELLA_EINVAL;
    }
    if (n == 0 && nnz != 0) {
        set_error("dibella_r_from_seeds: entries in a matrix without rows");
        return DIBELLA_EINVAL;
    }
    R->nrows = n;
    R->ncols = ncols;
    int32_t* tmp;
    int64_t* cnt;
    int32_t* d_flags;
    int64_t* rrp;
    DB_TRY(ar.work_n(nnz, &tmp));
    DB_TRY(ar.work_n(n, &cnt));
    DB_TRY(ar.work_n(1, &d_flags));
    // R's row pointers: their size is known before the sync
    DB_TRY(out_as_work ? out.work_n(n + 1, &rrp) : out.output_n(n + 1, &rrp));
    DB_TRY(fill_i32(d_flags, 0, 1, st));
    constexpr int WPB = 4;
    int tok = -1;
    DB_TRY(timing_begin(kPhRFromSeeds, st, &tok));
    if (n > 0) {
        hipLaunchKernelGGL(k_rs_mark<WPB>, dim3(grid_for(n, WPB, 1 << 16)), dim3(WPB * kWave), 0, st, n, row0,
                           ncols, nnz,
                           C->rowptr, C->col, C->count, C->seed, read_len, k, min_overlap, max_drift, min_density,
                           tmp, cnt, d_flags);
        DB_HIP(hipGetLastError());
    }
    DB_TRY(timing_end(tok, st));
    DB_TRY(scan_exclusive(cnt, rrp, n, nullptr, ar));
    HostStage& hst = host_stage();
    DB_TRY(hst.reserve(64));
    int64_t* h = static_cast<int64_t*>(hst.ptr);
    DB_HIP(hipMemcpyAsync(h, rrp + n, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    DB_HIP(hipMemcpyAsync(h + 1, d_flags, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    DB_TRY(sync_stream(st));
    const int32_t bad = *reinterpret_cast<int32_t*>(h + 1);
    if (bad) {
        set_error(std::string("dibella_r_from_seeds: ") + describe_rs_bad(bad));
        return DIBELLA_EINVAL;
    }
    const int64_t rnnz = h[0];
    int32_t *rcol, *rval;
    DB_TRY(out_as_work ? out.work_n(rnnz, &rcol) : out.output_n(rnnz, &rcol));
    DB_TRY(out_as_work ? out.work_n(rnnz, &rval) : out.output_n(rnnz, &rval));
    if (n > 0 && rnnz > 0) {
        DB_TRY(timing_begin(kPhRFromSeeds, st, &tok));
        DB_TRY(write_marked_rows(n, C->rowptr, C->col, tmp, rrp, rcol, rval, st));
        DB_TRY(timing_end(tok, st));
    }
    DB_TRY(stage_done(st));
    R->nnz = rnnz;
    R->rowptr = rrp;
    R->col = rcol;
    R->val = rval;
    return DIBELLA_OK;
}

}  // namespace dibella
