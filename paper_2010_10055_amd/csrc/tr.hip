// Transitive reduction of the overlap graph (Sec. IV-E): passes of
//   N = R^2 over MinPlus with the walk check, v = row max of R, M = v + x,
//   I = (M >= N) with the end-head check, R = R minus I
// until a pass deletes nothing.
//
// N is only needed where R has an entry (I is read on the pattern of R), so
// a pass computes N on that pattern: row i of R sits in LDS (sorted
// columns, values, running minima), every walk i -> k -> j streams row k of
// R, probes j in row i by binary search and folds the packed key
// (sum << 2 | end code) with an LDS atomicMin.  Row max, the comparison and
// the keep flags are fused into the same kernel; a wave-ballot compaction
// then writes the surviving entries into the other buffer.  A device-side
// update kernel counts deletions per set and clears the "active" flag that
// makes every later kernel return at once, so passes can be captured in a
// HIP graph and replayed without host round trips.
#include "common.hpp"

#include <algorithm>
#include <cstring>

namespace dibella {

struct TrSet {
    const int64_t* r_rowptr;
    const int32_t* r_col;
    const int32_t* r_val;
    int64_t n, nnz;
    int64_t row_base, nnz_base;
    int32_t fuzz;
    int32_t pad;
    int64_t* s_rowptr;
    int32_t* s_col;
    int32_t* s_val;
};

constexpr int kTrace = 64;

struct TrState {
    int32_t any_active;
    int32_t result_buf;
    int32_t pass;
    int32_t max_passes;
    int64_t triples_pass;
    int64_t triples_total;
    int32_t bin_count[3];   // small / medium / big rows
    int32_t pad;
    int64_t trace_nnz[kTrace];
    int64_t trace_triples[kTrace];
};

enum : int32_t { kTrBadRowptr = 1, kTrBadCol = 2, kTrUnsorted = 4, kTrDiagonal = 8, kTrBigOverhang = 16 };

constexpr uint32_t kInf = 0xFFFFFFFFu;
constexpr int kSmallCap = 512;
constexpr size_t kTrLdsLimit = 150 * 1024;
constexpr int kTrWin = 2048;   // walks per LDS expansion window
constexpr int kTrPer = 4;      // walks per thread in flight

// Hash slots for a row of at most `cap` entries (load <= 1/2).
__host__ __device__ constexpr int tr_hash_slots(int cap) {
    int h = 1;
    while (h < 2 * cap) h <<= 1;
    return h;
}
__device__ __forceinline__ uint32_t tr_hash(int32_t j, int slots) {
    return ((uint32_t)j * 0x9E3779B1u) >> (32 - __ffs(slots) + 1) & (uint32_t)(slots - 1);
}
// Dynamic LDS of a pass launch: chunk arrays, the row (col, val, N), the
// hash of its columns (MODE 0) and the expansion window.
__host__ __device__ constexpr size_t tr_mark_lds(int block, int cap) {
    return (size_t)block * 16 + (size_t)cap * 12 + (cap ? (size_t)tr_hash_slots(cap) * 4 : 0) + (size_t)kTrWin * 2;
}

// ---------------------------------------------------------------------------
// Validation and the contained-overlap drop (wave per row).
// ---------------------------------------------------------------------------
template <int WPB>
__global__ __launch_bounds__(WPB* kWave) void k_tr_validate(const TrSet* __restrict__ sets, int nsets,
                                                            const int64_t* __restrict__ set_base,
                                                            int64_t total_rows, int64_t* __restrict__ keepcnt,
                                                            uint8_t* __restrict__ rowok,
                                                            int32_t* __restrict__ flags) {
    const int lane = lane_id();
    for (int64_t g = (int64_t)blockIdx.x * WPB + wave_id(); g < total_rows;
         g += (int64_t)gridDim.x * WPB) {
        const int s = find_set(set_base, nsets, g);
        const TrSet& S = sets[s];
        const int64_t i = g - S.row_base;
        const int64_t lo = S.r_rowptr[i], hi = S.r_rowptr[i + 1];
        int32_t bad = 0;
        int64_t kept = 0;
        if (i == 0 && lo != 0) bad |= kTrBadRowptr;
        if (i == S.n - 1 && hi != S.nnz) bad |= kTrBadRowptr;
        if (lo < 0 || hi < lo || hi > S.nnz || hi - lo >= (int64_t(1) << 30)) {
            bad |= kTrBadRowptr;
        } else {
            for (int64_t e = lo + lane; e < hi; e += kWave) {
                const int32_t c = S.r_col[e];
                const int32_t v = S.r_val[e];
                if (c < 0 || c >= S.n) bad |= kTrBadCol;
                if (c == i) bad |= kTrDiagonal;
                if (e > lo && S.r_col[e - 1] >= c) bad |= kTrUnsorted;
                if ((v >> 2) >= (1 << 28)) bad |= kTrBigOverhang;
                if ((v >> 2) > 0) ++kept;
            }
        }
        bad = wave_or_i32(bad);
        kept = wave_sum(kept);
        if (lane == 0) {
            rowok[g] = bad ? 0 : 1;
            keepcnt[g] = bad ? 0 : kept;
            if (bad) atomicOr(&flags[s], bad);
        }
    }
}

constexpr int kRowsPerBlock = 64;

// Copy the entries with positive overhang; bin every non-empty row by
// length (LDS counters, one global atomic per workgroup and bin).
template <int WPB>
__global__ __launch_bounds__(WPB* kWave) void k_tr_init_copy(
    const TrSet* __restrict__ sets, int nsets, const int64_t* __restrict__ set_base, int64_t total_rows,
    const uint8_t* __restrict__ rowok, const int64_t* __restrict__ rp, int32_t* __restrict__ ci,
    int32_t* __restrict__ va, int32_t* __restrict__ lists, TrState* __restrict__ state, int mid_cap) {
    __shared__ int32_t s_cnt[3], s_base[3];
    __shared__ int32_t s_bin[kRowsPerBlock], s_pos[kRowsPerBlock];
    const int lane = lane_id();
    if (threadIdx.x < 3) s_cnt[threadIdx.x] = 0;
    __syncthreads();
    const int64_t row0 = (int64_t)blockIdx.x * kRowsPerBlock;
    for (int r = wave_id(); r < kRowsPerBlock; r += WPB) {
        const int64_t g = row0 + r;
        if (g >= total_rows) {
            if (lane == 0) s_bin[r] = -1;
            continue;
        }
        const int64_t out0 = rp[g];
        const int64_t L = rp[g + 1] - out0;
        if (rowok[g]) {
            const int s = find_set(set_base, nsets, g);
            const TrSet& S = sets[s];
            const int64_t i = g - S.row_base;
            const int64_t lo = S.r_rowptr[i], hi = S.r_rowptr[i + 1];
            int64_t out = out0;
            for (int64_t b = lo; b < hi; b += kWave) {
                const int64_t e = b + lane;
                int32_t c = 0, v = 0;
                bool k = false;
                if (e < hi) {
                    c = S.r_col[e];
                    v = S.r_val[e];
                    k = (v >> 2) > 0;
                }
                const uint64_t mask = __ballot(k);
                if (k) {
                    const int64_t pos = out + __popcll(mask & lanemask_lt());
                    ci[pos] = c;
                    va[pos] = v;
                }
                out += __popcll(mask);
            }
        }
        if (lane == 0) {
            s_bin[r] = -1;
            if (L > 0) {
                const int bin = L <= kSmallCap ? 0 : (L <= mid_cap ? 1 : 2);
                s_bin[r] = bin;
                s_pos[r] = atomicAdd(&s_cnt[bin], 1);
            }
        }
    }
    __syncthreads();
    if (threadIdx.x < 3 && s_cnt[threadIdx.x] > 0)
        s_base[threadIdx.x] = atomicAdd(&state->bin_count[threadIdx.x], s_cnt[threadIdx.x]);
    __syncthreads();
    for (int r = threadIdx.x; r < kRowsPerBlock; r += WPB * kWave) {
        const int b = s_bin[r];
        if (b >= 0) lists[(int64_t)b * total_rows + s_base[b] + s_pos[r]] = (int32_t)(row0 + r);
    }
}

// The passes run only if every set passed validation: a malformed call is
// reported after the first synchronisation, with no pass having run (every
// pass kernel returns at once while nothing is active).
__global__ void k_tr_init_state(TrState* __restrict__ state, const int64_t* __restrict__ rp,
                                int64_t total_rows, int32_t max_passes, int32_t nsets,
                                const int32_t* __restrict__ flags) {
    __shared__ int32_t s_bad;
    if (threadIdx.x == 0) s_bad = 0;
    __syncthreads();
    for (int s = threadIdx.x; s < nsets; s += blockDim.x)
        if (flags[s]) atomicOr(&s_bad, 1);
    __syncthreads();
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        state->any_active = (nsets > 0 && !s_bad) ? 1 : 0;
        state->result_buf = 0;
        state->pass = 0;
        state->max_passes = max_passes;
        state->triples_pass = 0;
        state->triples_total = 0;
        state->trace_nnz[0] = rp[total_rows];
    }
}

// ---------------------------------------------------------------------------
// One pass over one row: N on the pattern of the row, row max, comparison,
// keep flags.  MODE 0: row in LDS; MODE 1: row read from global memory and
// minima kept in `nbuf` (rows longer than the LDS cap).
// ---------------------------------------------------------------------------
template <int BLOCK, int MODE>
__device__ __forceinline__ void tr_row(const TrSet* __restrict__ sets, int nsets,
                                       const int64_t* __restrict__ set_base, int64_t g,
                                       const int64_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                       const int32_t* __restrict__ va, uint8_t* __restrict__ keep,
                                       int64_t* __restrict__ keepcnt, uint32_t* __restrict__ nbuf,
                                       const int32_t* __restrict__ active, int64_t* __restrict__ deleted,
                                       TrState* __restrict__ state, uint32_t flags, int32_t* s_col,
                                       int32_t* s_val, uint32_t* s_N, int32_t* s_hash, int hslots,
                                       int64_t* c_start, int64_t* c_off, uint16_t* tbuf,
                                       int64_t* s_tmp, int64_t* s_red64, int32_t* s_red32, int* out_set,
                                       int64_t* out_deleted, int64_t* out_triples) {
    const int s = find_set(set_base, nsets, g);
    const int64_t base = sets[s].row_base;
    const int32_t fuzz = sets[s].fuzz;
    const int64_t lo = rp[g];
    const int L = (int)(rp[g + 1] - lo);
    if (threadIdx.x == 0) {
        *out_set = s;
        *out_deleted = 0;
        *out_triples = 0;
    }
    if (!active[s]) {
        for (int u = threadIdx.x; u < L; u += BLOCK) keep[lo + u] = 1;
        if (threadIdx.x == 0) keepcnt[g] = L;
        return;
    }
    const int32_t* col;
    const int32_t* val;
    uint32_t* N;
    int32_t vmax = 0;
    if (MODE == 0) {
        for (int u = threadIdx.x; u < L; u += BLOCK) {
            const int32_t v = va[lo + u];
            s_col[u] = ci[lo + u];
            s_val[u] = v;
            s_N[u] = kInf;
            vmax = max(vmax, v >> 2);
        }
        col = s_col;
        val = s_val;
        N = s_N;
        // LDS hash of the row's columns -> position in the row (linear probing)
        for (int h = threadIdx.x; h < hslots; h += BLOCK) s_hash[h] = -1;
        __syncthreads();
        for (int u = threadIdx.x; u < L; u += BLOCK) {
            uint32_t h = tr_hash(ci[lo + u], hslots);
            while (atomicCAS(&s_hash[h], -1, u) != -1) h = (h + 1) & (uint32_t)(hslots - 1);
        }
    } else {
        for (int u = threadIdx.x; u < L; u += BLOCK) {
            nbuf[lo + u] = kInf;
            vmax = max(vmax, va[lo + u] >> 2);
        }
        __threadfence();   // the minima live in global memory: make the resets visible device wide
        col = ci + lo;
        val = va + lo;
        N = nbuf + lo;
    }
    vmax = block_max_lds(vmax, s_red32);   // contains barriers
    const bool variant_b = flags & DIBELLA_TR_VARIANT_B;
    int64_t triples = 0;
    // walks i -> k -> j: the row's entries k in chunks of BLOCK, their walks
    // numbered k-major and handed out through an LDS expansion of entry
    // indices (one LDS read per walk), kTrPer walks per thread in flight
    for (int cbase = 0; cbase < L; cbase += BLOCK) {
        const int cl = min(BLOCK, L - cbase);
        int64_t deg = 0, st = 0;
        if ((int)threadIdx.x < cl) {
            const int64_t gk = base + col[cbase + threadIdx.x];
            st = rp[gk];
            deg = rp[gk + 1] - st;
        }
        int64_t tot;
        const int64_t ex = block_exclusive_sum<BLOCK>(deg, s_tmp, &tot);
        c_start[threadIdx.x] = st;
        c_off[threadIdx.x] = ex;
        triples += tot;
        for (int64_t w0 = 0; w0 < tot; w0 += kTrWin) {
            const int64_t w1 = min(w0 + (int64_t)kTrWin, tot);
            {
                const int64_t a = max(ex, w0), b = min(ex + deg, w1);
                for (int64_t q = a; q < b; ++q) tbuf[q - w0] = (uint16_t)threadIdx.x;
            }
            __syncthreads();
            for (int64_t q0 = w0 + threadIdx.x; q0 < w1; q0 += (int64_t)BLOCK * kTrPer) {
                int tt[kTrPer];
                int32_t vkj[kTrPer], jj[kTrPer];
#pragma unroll
                for (int u = 0; u < kTrPer; ++u) {
                    const int64_t q = q0 + (int64_t)u * BLOCK;
                    tt[u] = -1;
                    if (q < w1) {
                        const int t = tbuf[q - w0];
                        const int64_t f = c_start[t] + (q - c_off[t]);
                        tt[u] = t;
                        vkj[u] = va[f];
                        jj[u] = ci[f];
                    }
                }
#pragma unroll
                for (int u = 0; u < kTrPer; ++u) {
                    if (tt[u] < 0) continue;
                    const int32_t vik = val[cbase + tt[u]];
                    if ((vik & 1) != ((vkj[u] >> 1) & 1)) continue;   // heads at k not opposite: not a walk
                    const int32_t j = jj[u];
                    int x;
                    if (MODE == 0) {
                        uint32_t h = tr_hash(j, hslots);
                        for (;;) {
                            x = s_hash[h];
                            if (x < 0 || col[x] == j) break;
                            h = (h + 1) & (uint32_t)(hslots - 1);
                        }
                        if (x < 0) continue;
                    } else {
                        int a = 0, b = L;                               // lower_bound of j in the row
                        while (a < b) {
                            const int mid = (a + b) >> 1;
                            if (col[mid] < j) a = mid + 1; else b = mid;
                        }
                        if (a >= L || col[a] != j) continue;
                        x = a;
                    }
                    const uint32_t key = ((uint32_t)((vik >> 2) + (vkj[u] >> 2)) << 2) | (uint32_t)(vik & 2) |
                                         (uint32_t)(vkj[u] & 1);
                    if (variant_b && (key & 3u) != (uint32_t)(val[x] & 3)) continue;
                    atomicMin(&N[x], key);
                }
            }
            __syncthreads();
        }
        if (tot == 0) __syncthreads();   // c_start/c_off are rewritten by the next chunk
    }
    const bool edge_rule = flags & DIBELLA_TR_RULE_EDGE;
    int32_t kept = 0;
    for (int u = threadIdx.x; u < L; u += BLOCK) {
        const int32_t v = val[u];
        const uint32_t nk = MODE == 0 ? N[u] : atomicOr(&N[u], 0u);   // global minima: read at L2
        const int64_t M = (int64_t)(edge_rule ? (v >> 2) : vmax) + fuzz;
        const bool del = nk != kInf && (nk & 3u) == (uint32_t)(v & 3) && (int64_t)(nk >> 2) <= M;
        keep[lo + u] = del ? 0 : 1;
        kept += del ? 0 : 1;
    }
    kept = block_sum_lds(kept, s_red32);
    if (threadIdx.x == 0) {
        keepcnt[g] = kept;
        *out_set = s;
        *out_deleted = L - kept;
        *out_triples = triples;
    }
}

template <int BLOCK, int MODE>
__global__ __launch_bounds__(BLOCK) void k_tr_mark(
    const TrSet* __restrict__ sets, int nsets, const int64_t* __restrict__ set_base,
    const int32_t* __restrict__ list, int bin, int64_t total_rows, int cap, const int64_t* __restrict__ rp,
    const int32_t* __restrict__ ci, const int32_t* __restrict__ va, uint8_t* __restrict__ keep,
    int64_t* __restrict__ keepcnt, uint32_t* __restrict__ nbuf, const int32_t* __restrict__ active,
    int64_t* __restrict__ deleted, TrState* __restrict__ state, uint32_t flags) {
    if (state->any_active == 0) return;
    extern __shared__ __align__(16) unsigned char smem[];
    int64_t* c_start = reinterpret_cast<int64_t*>(smem);
    int64_t* c_off = c_start + BLOCK;
    int32_t* s_col = reinterpret_cast<int32_t*>(c_off + BLOCK);
    int32_t* s_val = s_col + (MODE == 0 ? cap : 0);
    uint32_t* s_N = reinterpret_cast<uint32_t*>(s_val + (MODE == 0 ? cap : 0));
    const int hslots = MODE == 0 ? tr_hash_slots(cap) : 0;
    int32_t* s_hash = reinterpret_cast<int32_t*>(s_N + (MODE == 0 ? cap : 0));
    uint16_t* tbuf = reinterpret_cast<uint16_t*>(s_hash + hslots);
    __shared__ int64_t s_tmp[BLOCK / kWave + 1];
    __shared__ int64_t s_red64;
    __shared__ int32_t s_red32;
    const int32_t count = state->bin_count[bin];
    const int32_t* rows = list + (int64_t)bin * total_rows;
    // deletions per set and walks are summed by thread 0 over the rows of
    // this workgroup and published when the set changes and at the end
    int cur_set = -1;
    int64_t acc_del = 0, acc_trip = 0;
    for (int32_t w = blockIdx.x; w < count; w += gridDim.x) {
        int rs;
        int64_t rd, rt;
        tr_row<BLOCK, MODE>(sets, nsets, set_base, rows[w], rp, ci, va, keep, keepcnt, nbuf, active,
                            deleted, state, flags, s_col, s_val, s_N, s_hash, hslots, c_start, c_off, tbuf,
                            s_tmp, &s_red64, &s_red32, &rs, &rd, &rt);
        if (threadIdx.x == 0) {
            if (rs != cur_set) {
                if (acc_del) atomic_add(&deleted[cur_set], acc_del);
                cur_set = rs;
                acc_del = 0;
            }
            acc_del += rd;
            acc_trip += rt;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (acc_del) atomic_add(&deleted[cur_set], acc_del);
        if (acc_trip) atomic_add(&state->triples_pass, acc_trip);
    }
}

// Wave per row: write the kept entries of src into dst.
template <int WPB>
__global__ __launch_bounds__(WPB* kWave) void k_tr_compact(
    int64_t total_rows, const int64_t* __restrict__ rp, const int32_t* __restrict__ ci,
    const int32_t* __restrict__ va, const uint8_t* __restrict__ keep, const int64_t* __restrict__ drp,
    int32_t* __restrict__ dci, int32_t* __restrict__ dva, const TrState* __restrict__ state) {
    if (state->any_active == 0) return;
    const int lane = lane_id();
    for (int64_t g = (int64_t)blockIdx.x * WPB + wave_id(); g < total_rows;
         g += (int64_t)gridDim.x * WPB) {
        const int64_t lo = rp[g], hi = rp[g + 1];
        int64_t out = drp[g];
        for (int64_t b = lo; b < hi; b += kWave) {
            const int64_t e = b + lane;
            const bool k = e < hi && keep[e];
            const uint64_t mask = __ballot(k);
            if (k) {
                const int64_t pos = out + __popcll(mask & lanemask_lt());
                dci[pos] = ci[e];
                dva[pos] = va[e];
            }
            out += __popcll(mask);
        }
    }
}

__global__ __launch_bounds__(256) void k_tr_update(const TrSet* __restrict__ sets, int nsets,
                                                   const int64_t* __restrict__ drp, int64_t total_rows,
                                                   int32_t* __restrict__ active, int32_t* __restrict__ iters,
                                                   int64_t* __restrict__ deleted, int64_t* __restrict__ set_nnz,
                                                   TrState* __restrict__ state) {
    if (state->any_active == 0) return;
    __shared__ int32_t any;
    if (threadIdx.x == 0) any = 0;
    __syncthreads();
    const int32_t maxp = state->max_passes;
    for (int s = threadIdx.x; s < nsets; s += blockDim.x) {
        const TrSet& S = sets[s];
        set_nnz[s] = drp[S.row_base + S.n] - drp[S.row_base];
        if (active[s]) {
            const int32_t it = iters[s] + 1;
            iters[s] = it;
            if (deleted[s] == 0 || (maxp > 0 && it >= maxp)) active[s] = 0;
            deleted[s] = 0;
        }
        if (active[s]) atomicOr(&any, 1);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int32_t p = state->pass;
        if (p + 1 < kTrace) state->trace_nnz[p + 1] = drp[total_rows];
        if (p < kTrace) state->trace_triples[p] = state->triples_pass;
        state->triples_total += state->triples_pass;
        state->triples_pass = 0;
        state->pass = p + 1;
        state->result_buf ^= 1;
        state->any_active = any;
    }
}

// Final copies into the per-set outputs.
__global__ void k_tr_out_rowptr(const TrSet* __restrict__ sets, int nsets, const int64_t* __restrict__ set_base,
                                int64_t total_rows, const int64_t* __restrict__ rp) {
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < total_rows + nsets;
         g += (int64_t)gridDim.x * blockDim.x) {
        if (g < total_rows) {
            const int s = find_set(set_base, nsets, g);
            const TrSet& S = sets[s];
            S.s_rowptr[g - S.row_base] = rp[g] - rp[S.row_base];
        } else {
            const TrSet& S = sets[g - total_rows];
            S.s_rowptr[S.n] = rp[S.row_base + S.n] - rp[S.row_base];
        }
    }
}

// Entry e of the combined result belongs to the set whose first entry
// rp[row_base] is the largest <= e.
__global__ void k_tr_out_entries(const TrSet* __restrict__ sets, int nsets, const int64_t* __restrict__ ent_base,
                                 int64_t total, const int32_t* __restrict__ ci, const int32_t* __restrict__ va) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        int lo = 0, hi = nsets - 1;
        while (lo < hi) {   // last set with ent_base <= e and a non-empty range
            const int mid = (lo + hi + 1) >> 1;
            if (ent_base[mid] <= e) lo = mid; else hi = mid - 1;
        }
        const TrSet& S = sets[lo];
        const int64_t d = e - ent_base[lo];
        S.s_col[d] = ci[e];
        S.s_val[d] = va[e];
    }
}

__global__ void k_tr_ent_base(const TrSet* __restrict__ sets, int nsets, const int64_t* __restrict__ rp,
                              int64_t* __restrict__ ent_base) {
    for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < nsets; s += gridDim.x * blockDim.x)
        ent_base[s] = rp[sets[s].row_base];
}

// ---------------------------------------------------------------------------
// Host driver
// ---------------------------------------------------------------------------
struct TrBuffers {
    int block;   // workgroup width of the mark kernel (the call's tuning)
    const TrSet* d_sets;
    const int64_t* d_base;
    int nsets;
    int64_t total_rows;
    int64_t* rp[2];
    int32_t* ci[2];
    int32_t* va[2];
    uint8_t* keep;
    int64_t* keepcnt;
    uint32_t* nbuf;
    int32_t* lists;
    int32_t* active;
    int32_t* iters;
    int64_t* deleted;
    int64_t* set_nnz;
    TrState* state;
    int64_t* scan_tiles;
    uint32_t flags;
    int grid[3];
    int mid_cap;
};

template <int BLOCK>
static int allow_lds() {
    static std::atomic<bool> done{false};   // idempotent: racing threads may both set it
    if (!done.load(std::memory_order_acquire)) {
        DB_HIP(hipFuncSetAttribute((const void*)k_tr_mark<BLOCK, 0>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)kTrLdsLimit));
        done.store(true, std::memory_order_release);
    }
    return DIBELLA_OK;
}

// Called outside graph capture so that the attribute calls are not recorded.
static int prepare_pass_kernels(int block) {
    switch (block) {
        case 64: return allow_lds<64>();
        case 128: return allow_lds<128>();
        case 512: return allow_lds<512>();
        default: return allow_lds<256>();
    }
}

template <int BLOCK>
static int launch_pass_marks(const TrBuffers& B, int src, hipStream_t st) {
    const size_t lds_small = tr_mark_lds(BLOCK, kSmallCap);
    const size_t lds_mid = tr_mark_lds(BLOCK, B.mid_cap);
    const size_t lds_big = tr_mark_lds(BLOCK, 0);
    int tok = -1;
    DB_TRY(timing_begin(kPhTrMark, st, &tok));
    if (B.grid[0] > 0)
        hipLaunchKernelGGL((k_tr_mark<BLOCK, 0>), dim3(B.grid[0]), dim3(BLOCK), lds_small, st, B.d_sets, B.nsets,
                           B.d_base, B.lists, 0, B.total_rows, kSmallCap, B.rp[src], B.ci[src], B.va[src], B.keep,
                           B.keepcnt, B.nbuf, B.active, B.deleted, B.state, B.flags);
    if (B.grid[1] > 0)
        hipLaunchKernelGGL((k_tr_mark<BLOCK, 0>), dim3(B.grid[1]), dim3(BLOCK), lds_mid, st, B.d_sets, B.nsets,
                           B.d_base, B.lists, 1, B.total_rows, B.mid_cap, B.rp[src], B.ci[src], B.va[src],
                           B.keep, B.keepcnt, B.nbuf, B.active, B.deleted, B.state, B.flags);
    if (B.grid[2] > 0)
        hipLaunchKernelGGL((k_tr_mark<BLOCK, 1>), dim3(B.grid[2]), dim3(BLOCK), lds_big, st, B.d_sets, B.nsets,
                           B.d_base, B.lists, 2, B.total_rows, 0, B.rp[src], B.ci[src], B.va[src], B.keep,
                           B.keepcnt, B.nbuf, B.active, B.deleted, B.state, B.flags);
    DB_HIP(hipGetLastError());
    DB_TRY(timing_end(tok, st));
    return DIBELLA_OK;
}

// Enqueue one pass reading buffer `src` and writing buffer 1 - src.
static int enqueue_pass(const TrBuffers& B, int src, hipStream_t st) {
    switch (B.block) {
        case 64: DB_TRY(launch_pass_marks<64>(B, src, st)); break;
        case 128: DB_TRY(launch_pass_marks<128>(B, src, st)); break;
        case 512: DB_TRY(launch_pass_marks<512>(B, src, st)); break;
        default: DB_TRY(launch_pass_marks<256>(B, src, st)); break;
    }
    const int dst = 1 - src;
    DB_TRY(scan_exclusive_ws(B.keepcnt, B.rp[dst], B.total_rows, &B.state->any_active, B.scan_tiles, st));
    constexpr int WPB = 4;
    int tok = -1;
    if (B.total_rows > 0) {
        DB_TRY(timing_begin(kPhTrCompact, st, &tok));
        hipLaunchKernelGGL(k_tr_compact<WPB>, dim3(grid_for(B.total_rows, WPB, 1 << 16)), dim3(WPB * kWave), 0, st,
                           B.total_rows, B.rp[src], B.ci[src], B.va[src], B.keep, B.rp[dst], B.ci[dst],
                           B.va[dst], B.state);
        DB_TRY(timing_end(tok, st));
    }
    hipLaunchKernelGGL(k_tr_update, dim3(1), dim3(256), 0, st, B.d_sets, B.nsets, B.rp[dst], B.total_rows,
                       B.active, B.iters, B.deleted, B.set_nnz, B.state);
    DB_HIP(hipGetLastError());
    return DIBELLA_OK;
}

static const char* describe_tr_bad(int32_t bad) {
    if (bad & kTrBadRowptr) return "row pointers are not a valid CSR row pointer array";
    if (bad & kTrBadCol) return "a column index is outside [0, nrows)";
    if (bad & kTrUnsorted) return "columns are not strictly increasing within a row";
    if (bad & kTrDiagonal) return "R has a diagonal entry";
    if (bad & kTrBigOverhang) return "an overhang is >= 2^28";
    return "malformed matrix";
}

// Passes are captured on a private stream (the legacy null stream cannot be
// captured) and the instantiated graph is launched on the caller's stream.
static int capture_stream(hipStream_t* out) {
    static thread_local hipStream_t cs = nullptr;
    if (!cs) DB_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    *out = cs;
    return DIBELLA_OK;
}

struct GraphHolder {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    ~GraphHolder() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
    }
};

// Workspace of a reduction call (one reservation; every request fits it).
size_t tr_workspace_bytes(int nsets, int64_t total_rows, int64_t total_nnz) {
    auto pad = [](size_t b) { return Arena::padded(b); };
    size_t est = pad(sizeof(TrSet) * nsets) + 8 * pad(8 * (nsets + 1)) + pad(sizeof(TrState));
    est += pad(8 * total_rows) + pad(total_rows) + pad(12 * total_rows) + 2 * pad(8 * (total_rows + 1));
    est += 4 * pad(4 * total_nnz) + pad(total_nnz) + pad(4 * total_nnz);
    est += 4 * pad(8 * scan_workspace_elems(total_rows + 1)) + 4096;
    return est;
}

// Pinned-free staging bytes of a one-set call with fixed buffers.
size_t tr_fixed_host_bytes() { return sizeof(TrSet) + 2 * sizeof(int64_t) + sizeof(TrState) + 16 + 64; }

int tr_run(const dibella_csr* R, int nsets, const int32_t* fuzz, uint32_t flags, dibella_csr_out* S,
           int32_t* iterations, Arena& ar, const TrFixed* fixed) {
    hipStream_t st = ar.stream();
    const dibella_tuning tn = tuning();
    dibella_stats& stt = stats();
    if (fixed && (nsets != 1 || (flags & DIBELLA_TR_USE_GRAPH))) {
        set_error("a reduction into fixed buffers takes one set and no graphs");
        return DIBELLA_EINVAL;
    }
    // one set: descriptors on the stack (no host allocation)
    TrSet hs_one;
    int64_t base_one[2] = {0, 0};
    std::vector<TrSet> hs_many;
    std::vector<int64_t> base_many;
    if (nsets > 1) {
        hs_many.resize(nsets);
        base_many.assign(nsets + 1, 0);
    }
    TrSet* hs = nsets > 1 ? hs_many.data() : &hs_one;
    int64_t* base = nsets > 1 ? base_many.data() : base_one;
    int64_t total_rows = 0, total_nnz = 0;
    for (int s = 0; s < nsets; ++s) {
        const dibella_csr& r = R[s];
        if (r.nrows < 0 || r.nnz < 0 || r.ncols != r.nrows) {
            set_error("set " + std::to_string(s) + ": R must be square with non-negative sizes");
            return DIBELLA_EINVAL;
        }
        if (fuzz[s] < 0 || fuzz[s] >= (1 << 30)) {
            set_error("set " + std::to_string(s) + ": fuzz must be in [0, 2^30)");
            return DIBELLA_EINVAL;
        }
        if (r.nrows >= (int64_t(1) << 31) || r.nnz >= (int64_t(1) << 40)) {
            set_error("set " + std::to_string(s) + ": nrows must be < 2^31 and nnz < 2^40");
            return DIBELLA_EOVERFLOW;
        }
        if ((r.nrows > 0 && !r.rowptr) || (r.nnz > 0 && (!r.col || !r.val))) {
            set_error("set " + std::to_string(s) + ": null pointer");
            return DIBELLA_EINVAL;
        }
        if (r.nrows == 0 && r.nnz != 0) {
            set_error("set " + std::to_string(s) + ": entries in a matrix without rows");
            return DIBELLA_EINVAL;
        }
        TrSet& t = hs[s];
        std::memset(&t, 0, sizeof(t));
        t.r_rowptr = r.rowptr;
        t.r_col = r.col;
        t.r_val = r.val;
        t.n = r.nrows;
        t.nnz = r.nnz;
        t.row_base = total_rows;
        t.nnz_base = total_nnz;
        t.fuzz = fuzz[s];
        base[s] = total_rows;
        total_rows += r.nrows;
        total_nnz += r.nnz;
    }
    base[nsets] = total_rows;
    if (total_rows >= (int64_t(1) << 31)) {
        set_error("batch too large: total rows must be < 2^31");
        return DIBELLA_EOVERFLOW;
    }
    for (int s = 0; s < nsets; ++s) {
        S[s].nrows = R[s].nrows;
        S[s].ncols = R[s].nrows;
        S[s].nnz = 0;
        S[s].rowptr = nullptr;
        S[s].col = nullptr;
        S[s].val = nullptr;
        iterations[s] = 0;
    }

    TrBuffers B;
    std::memset(&B, 0, sizeof(B));
    B.block = tn.tr_block;
    TrSet* d_sets;
    int64_t* d_base;
    int32_t* d_flags;
    int64_t* ent_base;
    uint8_t* rowok;
    // one reservation for the call's workspace (allocator calls cost host time each)
    DB_TRY(ar.reserve(tr_workspace_bytes(nsets, total_rows, total_nnz)));
    DB_TRY(ar.work_n(nsets, &d_sets));
    DB_TRY(ar.work_n(nsets + 1, &d_base));
    DB_TRY(ar.work_n(nsets, &d_flags));
    DB_TRY(ar.work_n(nsets, &ent_base));
    DB_TRY(ar.work_n(nsets, &B.active));
    DB_TRY(ar.work_n(nsets, &B.iters));
    DB_TRY(ar.work_n(nsets, &B.deleted));
    DB_TRY(ar.work_n(nsets, &B.set_nnz));
    DB_TRY(ar.work_n(1, &B.state));
    DB_TRY(ar.work_n(total_rows, &B.keepcnt));
    DB_TRY(ar.work_n(total_rows, &rowok));
    DB_TRY(ar.work_n((size_t)3 * total_rows, &B.lists));
    for (int b = 0; b < 2; ++b) {
        DB_TRY(ar.work_n(total_rows + 1, &B.rp[b]));
        DB_TRY(ar.work_n(total_nnz, &B.ci[b]));
        DB_TRY(ar.work_n(total_nnz, &B.va[b]));
    }
    DB_TRY(ar.work_n(total_nnz, &B.keep));
    DB_TRY(ar.work_n(total_nnz, &B.nbuf));
    DB_TRY(ar.work_n(scan_workspace_elems(total_rows), &B.scan_tiles));
    B.d_sets = d_sets;
    B.d_base = d_base;
    B.nsets = nsets;
    B.total_rows = total_rows;
    B.flags = flags;
    // rows up to mid_cap are kept in LDS; the cap shrinks until the launch fits
    B.mid_cap = std::max(tn.tr_lds_cap, kSmallCap);
    while (B.mid_cap > kSmallCap && tr_mark_lds(tn.tr_block, B.mid_cap) > kTrLdsLimit) B.mid_cap -= 512;

    const size_t desc_bytes = sizeof(TrSet) * nsets + sizeof(int64_t) * (nsets + 1);
    const size_t back_bytes = sizeof(TrState) + (sizeof(int32_t) * 2 + sizeof(int64_t)) * nsets;
    char* hbuf;
    if (fixed) {   // pageable caller memory: the copies below complete before they return
        if (fixed->host_bytes < desc_bytes + back_bytes + 64) {
            set_error("internal: fixed host staging too small");
            return DIBELLA_EDEVICE;
        }
        hbuf = static_cast<char*>(fixed->host);
    } else {
        HostStage& hst = host_stage();
        DB_TRY(hst.reserve(desc_bytes + back_bytes + 64));
        hbuf = static_cast<char*>(hst.ptr);
    }
    std::memcpy(hbuf, hs, sizeof(TrSet) * nsets);
    std::memcpy(hbuf + sizeof(TrSet) * nsets, base, sizeof(int64_t) * (nsets + 1));
    DB_HIP(hipMemcpyAsync(d_sets, hbuf, sizeof(TrSet) * nsets, hipMemcpyHostToDevice, st));
    DB_HIP(hipMemcpyAsync(d_base, hbuf + sizeof(TrSet) * nsets, sizeof(int64_t) * (nsets + 1),
                          hipMemcpyHostToDevice, st));
    DB_TRY(fill_i32(d_flags, 0, nsets, st));
    DB_TRY(fill_i32(B.active, 1, nsets, st));
    DB_TRY(fill_i32(B.iters, 0, nsets, st));
    DB_TRY(fill_i64(B.deleted, 0, nsets, st));
    DB_TRY(fill_i32(reinterpret_cast<int32_t*>(B.state), 0, sizeof(TrState) / 4, st));

    constexpr int WPB = 4;
    const int grid_rows = grid_for(total_rows, WPB, 1 << 16);
    if (total_rows > 0) {
        hipLaunchKernelGGL(k_tr_validate<WPB>, dim3(grid_rows), dim3(WPB * kWave), 0, st, d_sets, nsets, d_base,
                           total_rows, B.keepcnt, rowok, d_flags);
        DB_HIP(hipGetLastError());
    }
    DB_TRY(scan_exclusive_ws(B.keepcnt, B.rp[0], total_rows, nullptr, B.scan_tiles, st));
    if (total_rows > 0) {
        hipLaunchKernelGGL(k_tr_init_copy<WPB>, dim3((unsigned)ceil_div(total_rows, kRowsPerBlock)),
                           dim3(WPB * kWave), 0, st, d_sets, nsets, d_base,
                           total_rows, rowok, B.rp[0], B.ci[0], B.va[0], B.lists, B.state, B.mid_cap);
        DB_HIP(hipGetLastError());
    }
    const uint32_t maxp = flags >> 16;
    hipLaunchKernelGGL(k_tr_init_state, dim3(1), dim3(64), 0, st, B.state, B.rp[0], total_rows, (int32_t)maxp,
                       nsets, d_flags);
    DB_HIP(hipGetLastError());

    char* back = hbuf + desc_bytes;
    TrState* h_state = reinterpret_cast<TrState*>(back);
    int32_t* h_flags = reinterpret_cast<int32_t*>(back + sizeof(TrState));
    int32_t* h_iters = h_flags + nsets;
    int64_t* h_set_nnz = reinterpret_cast<int64_t*>(back + sizeof(TrState) + sizeof(int32_t) * 2 * nsets);
    auto read_back = [&]() -> int {
        DB_HIP(hipMemcpyAsync(h_state, B.state, sizeof(TrState), hipMemcpyDeviceToHost, st));
        DB_HIP(hipMemcpyAsync(h_flags, d_flags, sizeof(int32_t) * nsets, hipMemcpyDeviceToHost, st));
        DB_HIP(hipMemcpyAsync(h_iters, B.iters, sizeof(int32_t) * nsets, hipMemcpyDeviceToHost, st));
        DB_HIP(hipMemcpyAsync(h_set_nnz, B.set_nnz, sizeof(int64_t) * nsets, hipMemcpyDeviceToHost, st));
        return sync_stream(st);
    };
    // Persistent grids sized from bounds the host knows (the bin sizes are
    // read on the device), so the first passes follow validation without a
    // synchronisation: at most nnz / (cap + 1) rows are longer than a cap.
    {
        const int occ = 8;   // resident blocks per CU assumed when sizing persistent grids
        const int64_t cap_grid = 256 * occ * 4;
        const int64_t bound[3] = {total_rows, total_nnz / (kSmallCap + 1), total_nnz / (B.mid_cap + 1)};
        for (int b = 0; b < 3; ++b) B.grid[b] = (int)std::min(bound[b], cap_grid);
    }
    auto check_valid = [&]() -> int {
        for (int s = 0; s < nsets; ++s) {
            if (h_flags[s]) {
                set_error("set " + std::to_string(s) + ": " + describe_tr_bad(h_flags[s]));
                return DIBELLA_EINVAL;
            }
        }
        return DIBELLA_OK;
    };

    DB_TRY(prepare_pass_kernels(B.block));
    {
        if (flags & DIBELLA_TR_USE_GRAPH) {
            int U = std::max(1, std::min(16, tn.tr_graph_passes));
            if (U & 1) U += 1;   // even: every replay starts from buffer 0
            GraphHolder gh;
            hipStream_t cs;
            DB_TRY(capture_stream(&cs));
            DB_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
            int cap_status = DIBELLA_OK;
            for (int u = 0; u < U && cap_status == DIBELLA_OK; ++u) cap_status = enqueue_pass(B, u & 1, cs);
            hipGraph_t g = nullptr;
            const hipError_t end = hipStreamEndCapture(cs, &g);
            gh.graph = g;
            if (cap_status != DIBELLA_OK) return cap_status;
            DB_HIP(end);
            DB_HIP(hipGraphInstantiate(&gh.exec, gh.graph, nullptr, nullptr, 0));
            while (true) {
                DB_HIP(hipGraphLaunch(gh.exec, st));
                DB_TRY(read_back());
                DB_TRY(check_valid());
                if (!h_state->any_active) break;
                if (h_state->pass > total_nnz + 2) {
                    set_error("transitive reduction did not converge");
                    return DIBELLA_EDEVICE;
                }
            }
        } else {
            // two passes per host synchronisation: a pass after convergence
            // returns at once (every pass kernel checks the active flag),
            // and a reduction that converges in two passes syncs once
            while (true) {
                DB_TRY(enqueue_pass(B, 0, st));
                DB_TRY(enqueue_pass(B, 1, st));
                DB_TRY(read_back());
                DB_TRY(check_valid());
                if (!h_state->any_active) break;
                if (h_state->pass > total_nnz + 2) {   // every productive pass deletes an entry
                    set_error("transitive reduction did not converge");
                    return DIBELLA_EDEVICE;
                }
            }
        }
    }
    const int res = h_state->result_buf;
    stt.passes = h_state->pass;
    stt.triples = h_state->triples_total;
    stt.trace_len = std::min(h_state->pass + 1, kTrace);
    for (int p = 0; p < stt.trace_len; ++p) stt.nnz_trace[p] = h_state->trace_nnz[p];
    for (int p = 0; p < std::min(h_state->pass, kTrace); ++p) stt.triples_trace[p] = h_state->trace_triples[p];

    // ---- outputs
    for (int s = 0; s < nsets; ++s) {
        const int64_t nz = h_state->pass > 0 ? h_set_nnz[s] : 0;
        if (fixed) {
            if (nz > fixed->s_cap) {   // cannot happen while the capacity holds nnz(R)
                set_error("internal: S exceeds the given capacity");
                return DIBELLA_EDEVICE;
            }
            hs[s].s_rowptr = fixed->s_rowptr;
            hs[s].s_col = nz ? fixed->s_col : nullptr;
            hs[s].s_val = nz ? fixed->s_val : nullptr;
        } else {
            DB_TRY(ar.output_n(R[s].nrows + 1, &hs[s].s_rowptr));
            DB_TRY(ar.output_n(nz, &hs[s].s_col));
            DB_TRY(ar.output_n(nz, &hs[s].s_val));
        }
        S[s].nnz = nz;
        S[s].rowptr = hs[s].s_rowptr;
        S[s].col = hs[s].s_col;
        S[s].val = hs[s].s_val;
        iterations[s] = h_iters[s];
    }
    std::memcpy(hbuf, hs, sizeof(TrSet) * nsets);
    DB_HIP(hipMemcpyAsync(d_sets, hbuf, sizeof(TrSet) * nsets, hipMemcpyHostToDevice, st));
    int64_t total_out = 0;
    for (int s = 0; s < nsets; ++s) total_out += S[s].nnz;
    hipLaunchKernelGGL(k_tr_out_rowptr, dim3(grid_for(total_rows + nsets, 256, 4096)), dim3(256), 0, st, d_sets,
                       nsets, d_base, total_rows, B.rp[res]);
    hipLaunchKernelGGL(k_tr_ent_base, dim3(grid_for(nsets, 64, 1024)), dim3(64), 0, st, d_sets, nsets, B.rp[res],
                       ent_base);
    if (total_out > 0)
        hipLaunchKernelGGL(k_tr_out_entries, dim3(grid_for(total_out, 256, 8192)), dim3(256), 0, st, d_sets, nsets,
                           ent_base, total_out, B.ci[res], B.va[res]);
    DB_HIP(hipGetLastError());
    if (!fixed) DB_TRY(stage_done(st));
    return DIBELLA_OK;
}

}  // namespace dibella
