// C = A * A^T over the overlap semiring (Sec. IV-D): for every pair of reads
// (i, j) the number of shared reliable k-mers and the position pairs of the
// two smallest shared k-mer columns.
//
// Pipeline (one launch per step for all sets of a batch):
//   validate + column histogram  ->  scan  ->  scatter A^T (read, pos) pairs,
//   per-entry A^T segment (start, length) and per-row products  ->  bins by
//   products  ->  symbolic (LDS hash of distinct j, counts)  ->  bins by
//   distinct count  ->  scan to row pointers  ->  numeric (LDS hash with
//   count and min-2 seeds, bitonic sort by j, coalesced write).
//   Rows whose distinct columns do not fit an LDS table go through
//   expand-sort-compress (ESC): products are expanded in k-mer order, stably
//   radix sorted by j and compressed by runs.
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
    int32_t min_shared;
    int32_t id_bits;  // bits needed for a read id of this set (ESC radix passes)
    int64_t* c_rowptr;
    int32_t* c_col;
    int32_t* c_count;
    int32_t* c_seed;
};

constexpr int kMaxLog2 = 16;

struct OvCounters {
    int64_t products;
    int64_t max_flops;
    int64_t esc_flops;
    int32_t sym_count[kMaxLog2];
    int32_t num_count[kMaxLog2];
    int32_t esc_rows;
    int32_t overflow_rows;
};

enum : int32_t {
    kBadRowptr = 1,
    kBadCol = 2,
    kUnsorted = 4,
    kNegative = 8,
    kLongRow = 16,
};

constexpr uint64_t kEmpty64 = ~0ull;

__device__ __forceinline__ uint32_t hash_slot(int32_t j, int logT) {
    return ((uint32_t)j * 0x9E3779B1u) >> (32 - logT);
}

__device__ __forceinline__ int32_t wave_or(int32_t v) {
    for (int d = kWave / 2; d > 0; d >>= 1) v |= __shfl_xor(v, d, kWave);
    return v;
}

// Insert key j into an open-addressing table (linear probing).  Returns the
// slot, or -1 if no slot was found within T probes.  *fresh = 1 if this
// call created the entry.
__device__ __forceinline__ int table_insert(int32_t* keys, int logT, int32_t j, int* fresh) {
    const uint32_t mask = (1u << logT) - 1u;
    uint32_t h = hash_slot(j, logT);
    *fresh = 0;
    for (uint32_t p = 0; p <= mask; ++p) {
        int32_t k = keys[h];
        if (k == j) return (int)h;
        if (k == -1) {
            int32_t old = atomicCAS(&keys[h], -1, j);
            if (old == -1) {
                *fresh = 1;
                return (int)h;
            }
            if (old == j) return (int)h;
        }
        h = (h + 1u) & mask;
    }
    return -1;
}

// ---------------------------------------------------------------------------
// Step 1: validate A, histogram of columns (one wave per row).
// ---------------------------------------------------------------------------
template <int WPB>
__global__ __launch_bounds__(WPB* kWave) void k_ov_hist(const OvSet* __restrict__ sets, int nsets,
                                                        const int64_t* __restrict__ set_base,
                                                        int64_t total_rows, int32_t* __restrict__ cnt,
                                                        int32_t* __restrict__ flags, int checks) {
    const int lane = lane_id();
    for (int64_t g = (int64_t)blockIdx.x * WPB + wave_id(); g < total_rows;
         g += (int64_t)gridDim.x * WPB) {
        const int s = find_set(set_base, nsets, g);
        const OvSet& S = sets[s];
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
            for (int64_t e = lo + lane; e < hi; e += kWave) {
                const int32_t k = S.a_col[e];
                if (k < 0 || k >= S.m) {
                    bad |= kBadCol;
                } else {
                    atomicAdd(&cnt[S.col_base + k], 1);
                }
                if (checks) {
                    if (e > lo && S.a_col[e - 1] >= k) bad |= kUnsorted;
                    if (S.a_val[e] < 0) bad |= kNegative;
                }
            }
        }
        bad = wave_or(bad);
        if (lane == 0 && bad) atomicOr(&flags[s], bad);
    }
}

// ---------------------------------------------------------------------------
// Step 3: scatter A^T, record each A entry's A^T segment, products per row,
// and bin rows for the symbolic phase by table size.
// ---------------------------------------------------------------------------
template <int WPB>
__global__ __launch_bounds__(WPB* kWave) void k_ov_scatter(
    const OvSet* __restrict__ sets, int nsets, const int64_t* __restrict__ set_base, int64_t total_rows,
    const int64_t* __restrict__ t_rowptr, int32_t* __restrict__ cnt, int2* __restrict__ at,
    uint64_t* __restrict__ seg, int64_t* __restrict__ flops_row, int32_t* __restrict__ sym_list,
    OvCounters* __restrict__ ctr, int min_log2, int max_log2, int load_log2) {
    const int lane = lane_id();
    for (int64_t g = (int64_t)blockIdx.x * WPB + wave_id(); g < total_rows;
         g += (int64_t)gridDim.x * WPB) {
        const int s = find_set(set_base, nsets, g);
        const OvSet& S = sets[s];
        const int64_t i = g - S.row_base;
        const int64_t lo = S.a_rowptr[i], hi = S.a_rowptr[i + 1];
        int64_t fl = 0;
        if (!(lo < 0 || hi < lo || hi > S.nnz || hi - lo >= (int64_t(1) << 30))) {
            for (int64_t e = lo + lane; e < hi; e += kWave) {
                const int32_t k = S.a_col[e];
                uint64_t sg = 0;
                if (k >= 0 && k < S.m) {
                    const int64_t gk = S.col_base + k;
                    const int64_t t0 = t_rowptr[gk];
                    const int64_t len = t_rowptr[gk + 1] - t0;
                    const int32_t slot = atomicSub(&cnt[gk], 1) - 1;
                    at[t0 + slot] = make_int2((int32_t)i, S.a_val[e]);
                    sg = ((uint64_t)t0 << 24) | (uint64_t)len;
                    fl += len;
                }
                seg[S.nnz_base + e] = sg;
            }
        }
        fl = wave_sum(fl);
        if (lane == 0) {
            flops_row[g] = fl;
            if (fl > 0) {
                atomic_add(&ctr->products, fl);
                atomic_max(&ctr->max_flops, fl);
                const int64_t keys = fl < S.n ? fl : S.n;
                int lg = ceil_log2_i64(keys) + load_log2;
                lg = lg < min_log2 ? min_log2 : (lg > max_log2 ? max_log2 : lg);
                const int32_t pos = atomicAdd(&ctr->sym_count[lg], 1);
                sym_list[(int64_t)lg * total_rows + pos] = (int32_t)g;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Shared product walk: for each A entry t of row i (in chunks of BLOCK) the
// A^T segment seg[t]; products are numbered t-major, and f(t, e) is called
// for product e of A^T belonging to entry t.  The block must call it
// uniformly.  `stop` (LDS flag) lets the callee abandon the walk.
// ---------------------------------------------------------------------------
template <int BLOCK, class F>
__device__ __forceinline__ void walk_products(const uint64_t* __restrict__ rseg, int L, int64_t* c_start,
                                              int64_t* c_off, int64_t* s_tmp, const int32_t* stop,
                                              F&& f) {
    for (int cbase = 0; cbase < L; cbase += BLOCK) {
        const int cl = min(BLOCK, L - cbase);
        int64_t len = 0, st = 0;
        if ((int)threadIdx.x < cl) {
            const uint64_t sg = rseg[cbase + threadIdx.x];
            st = (int64_t)(sg >> 24);
            len = (int64_t)(sg & 0xFFFFFFull);
        }
        int64_t tot;
        const int64_t ex = block_exclusive_sum<BLOCK>(len, s_tmp, &tot);
        c_start[threadIdx.x] = st;
        c_off[threadIdx.x] = ex;
        __syncthreads();
        for (int64_t q = threadIdx.x; q < tot; q += BLOCK) {
            if (stop && *(volatile const int32_t*)stop) break;
            int lo = 0, hi = cl - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (c_off[mid] <= q) lo = mid; else hi = mid - 1;
            }
            f(cbase + lo, c_start[lo] + (q - c_off[lo]), q);
        }
        __syncthreads();
        if (stop && *(volatile const int32_t*)stop) break;
    }
}

// ---------------------------------------------------------------------------
// Symbolic phase: distinct j per row and how many reach min_shared.
// ---------------------------------------------------------------------------
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_ov_symbolic(
    const OvSet* __restrict__ sets, int nsets, const int64_t* __restrict__ set_base,
    const int32_t* __restrict__ list, int logT, int limit, const uint64_t* __restrict__ seg,
    const int2* __restrict__ at, int64_t* __restrict__ nnzrow, int32_t* __restrict__ distinct,
    OvCounters* __restrict__ ctr) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int T = 1 << logT;
    int64_t* c_start = reinterpret_cast<int64_t*>(smem);
    int64_t* c_off = c_start + BLOCK;
    int32_t* keys = reinterpret_cast<int32_t*>(c_off + BLOCK);
    int32_t* cnt = keys + T;
    __shared__ int64_t s_tmp[BLOCK / kWave + 1];
    __shared__ int32_t s_nd, s_ovf, s_red;

    const int64_t g = list[blockIdx.x];
    const int s = find_set(set_base, nsets, g);
    const OvSet& S = sets[s];
    const int64_t i = g - S.row_base;
    const int64_t lo = S.a_rowptr[i];
    const int L = (int)(S.a_rowptr[i + 1] - lo);
    for (int q = threadIdx.x; q < T; q += BLOCK) {
        keys[q] = -1;
        cnt[q] = 0;
    }
    if (threadIdx.x == 0) {
        s_nd = 0;
        s_ovf = 0;
    }
    __syncthreads();
    walk_products<BLOCK>(seg + S.nnz_base + lo, L, c_start, c_off, s_tmp, &s_ovf,
                         [&](int, int64_t e, int64_t) {
                             const int32_t j = at[e].x;
                             int fresh;
                             const int slot = table_insert(keys, logT, j, &fresh);
                             if (slot < 0) {
                                 s_ovf = 1;
                                 return;
                             }
                             atomicAdd(&cnt[slot], 1);
                             if (fresh && atomicAdd(&s_nd, 1) + 1 >= limit) s_ovf = 1;
                         });
    __syncthreads();
    if (s_ovf) {
        if (threadIdx.x == 0) {
            nnzrow[g] = 0;
            distinct[g] = -1;
            atomicAdd(&ctr->overflow_rows, 1);
        }
        return;
    }
    int32_t mine = 0;
    for (int q = threadIdx.x; q < T; q += BLOCK)
        if (keys[q] != -1 && cnt[q] >= S.min_shared) ++mine;
    const int32_t tot = block_sum_lds(mine, &s_red);
    if (threadIdx.x == 0) {
        nnzrow[g] = tot;
        distinct[g] = s_nd;
    }
}

// ---------------------------------------------------------------------------
// Bins for the numeric phase, ESC routing.
// ---------------------------------------------------------------------------
__global__ void k_ov_bin_numeric(int64_t total_rows, const int64_t* __restrict__ flops_row,
                                 const int32_t* __restrict__ distinct, int32_t* __restrict__ num_list,
                                 int32_t* __restrict__ esc_list, int64_t* __restrict__ esc_off,
                                 OvCounters* __restrict__ ctr, int min_log2, int max_log2, int load_log2) {
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < total_rows;
         g += (int64_t)gridDim.x * blockDim.x) {
        const int64_t fl = flops_row[g];
        if (fl <= 0) continue;
        const int32_t d = distinct[g];
        const int lg = ceil_log2_i64(d < 1 ? 1 : d) + load_log2;
        if (d < 0 || lg > max_log2) {
            const int32_t pos = atomicAdd(&ctr->esc_rows, 1);
            esc_list[pos] = (int32_t)g;
            esc_off[g] = atomic_add(&ctr->esc_flops, fl);
        } else {
            const int l = lg < min_log2 ? min_log2 : lg;
            const int32_t pos = atomicAdd(&ctr->num_count[l], 1);
            num_list[(int64_t)l * total_rows + pos] = (int32_t)g;
        }
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
// Numeric phase: counts and the two smallest-k seeds per (i, j), sorted
// output.  A seed candidate is packed as (t << 32) | p_j where t is the
// index of k in row i (monotone in k); the two smallest survive an
// atomicMin cascade (the value displaced from m1 moves on to m2).
// ---------------------------------------------------------------------------
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_ov_numeric(
    const OvSet* __restrict__ sets, int nsets, const int64_t* __restrict__ set_base,
    const int32_t* __restrict__ list, int logT, const uint64_t* __restrict__ seg,
    const int2* __restrict__ at, const int64_t* __restrict__ G) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int T = 1 << logT;
    uint64_t* m1 = reinterpret_cast<uint64_t*>(smem);
    uint64_t* m2 = m1 + T;
    uint64_t* sortbuf = m2 + T;                                   // T/2
    int64_t* c_start = reinterpret_cast<int64_t*>(sortbuf + T / 2);
    int64_t* c_off = c_start + BLOCK;
    int32_t* keys = reinterpret_cast<int32_t*>(c_off + BLOCK);
    int32_t* cnt = keys + T;
    __shared__ int64_t s_tmp[BLOCK / kWave + 1];
    __shared__ int32_t s_nsel;

    const int64_t g = list[blockIdx.x];
    const int s = find_set(set_base, nsets, g);
    const OvSet& S = sets[s];
    const int64_t i = g - S.row_base;
    const int64_t lo = S.a_rowptr[i];
    const int L = (int)(S.a_rowptr[i + 1] - lo);
    for (int q = threadIdx.x; q < T; q += BLOCK) {
        keys[q] = -1;
        cnt[q] = 0;
        m1[q] = kEmpty64;
        m2[q] = kEmpty64;
    }
    if (threadIdx.x == 0) s_nsel = 0;
    __syncthreads();
    walk_products<BLOCK>(seg + S.nnz_base + lo, L, c_start, c_off, s_tmp, nullptr,
                         [&](int t, int64_t e, int64_t) {
                             const int2 jp = at[e];
                             int fresh;
                             const int slot = table_insert(keys, logT, jp.x, &fresh);
                             if (slot < 0) return;  // cannot happen: the table holds 2x the distinct keys
                             atomicAdd(&cnt[slot], 1);
                             const uint64_t x = ((uint64_t)(uint32_t)t << 32) | (uint64_t)(uint32_t)jp.y;
                             const uint64_t old = atomicMin(&m1[slot], x);
                             const uint64_t rej = old > x ? old : x;
                             if (rej != kEmpty64) atomicMin(&m2[slot], rej);
                         });
    __syncthreads();
    for (int q = threadIdx.x; q < T; q += BLOCK) {
        if (keys[q] != -1 && cnt[q] >= S.min_shared) {
            const int p = atomicAdd(&s_nsel, 1);
            sortbuf[p] = ((uint64_t)(uint32_t)keys[q] << 32) | (uint64_t)q;
        }
    }
    __syncthreads();
    const int nsel = s_nsel;
    int P = 1;
    while (P < nsel) P <<= 1;
    for (int q = nsel + threadIdx.x; q < P; q += BLOCK) sortbuf[q] = kEmpty64;
    __syncthreads();
    // bitonic sort of sortbuf[0, P) ascending
    for (int k = 2; k <= P; k <<= 1) {
        for (int jj = k >> 1; jj > 0; jj >>= 1) {
            for (int idx = threadIdx.x; idx < P; idx += BLOCK) {
                const int ixj = idx ^ jj;
                if (ixj > idx) {
                    const uint64_t a = sortbuf[idx], b = sortbuf[ixj];
                    const bool up = (idx & k) == 0;
                    if ((a > b) == up) {
                        sortbuf[idx] = b;
                        sortbuf[ixj] = a;
                    }
                }
            }
            __syncthreads();
        }
    }
    const int64_t off = G[g] - G[S.row_base];
    int4* seed4 = reinterpret_cast<int4*>(S.c_seed);
    for (int r = threadIdx.x; r < nsel; r += BLOCK) {
        const int slot = (int)(uint32_t)sortbuf[r];
        const uint64_t a = m1[slot], b = m2[slot];
        const int32_t pi0 = S.a_val[lo + (int64_t)(a >> 32)];
        const int32_t pj0 = (int32_t)(uint32_t)a;
        int32_t pi1 = -1, pj1 = -1;
        if (b != kEmpty64) {
            pi1 = S.a_val[lo + (int64_t)(b >> 32)];
            pj1 = (int32_t)(uint32_t)b;
        }
        S.c_col[off + r] = keys[slot];
        S.c_count[off + r] = cnt[slot];
        seed4[off + r] = make_int4(pi0, pj0, pi1, pj1);
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
    __shared__ int64_t c_start[kEscBlock], c_off[kEscBlock];
    __shared__ int64_t s_tmp[kEscBlock / kWave + 1];
    const int64_t g = list[blockIdx.x];
    const int s = find_set(set_base, nsets, g);
    const OvSet& S = sets[s];
    const int64_t i = g - S.row_base;
    const int64_t lo = S.a_rowptr[i];
    const int L = (int)(S.a_rowptr[i + 1] - lo);
    const int64_t base = esc_off[g];
    // walk_products numbers products per chunk; keep a running base so that
    // the expanded order is t-major over the whole row.
    int64_t chunk_base = 0;
    for (int cbase = 0; cbase < L; cbase += kEscBlock) {
        const int cl = min(kEscBlock, L - cbase);
        int64_t len = 0, st = 0;
        if ((int)threadIdx.x < cl) {
            const uint64_t sg = seg[S.nnz_base + lo + cbase + threadIdx.x];
            st = (int64_t)(sg >> 24);
            len = (int64_t)(sg & 0xFFFFFFull);
        }
        int64_t tot;
        const int64_t ex = block_exclusive_sum<kEscBlock>(len, s_tmp, &tot);
        c_start[threadIdx.x] = st;
        c_off[threadIdx.x] = ex;
        __syncthreads();
        for (int64_t q = threadIdx.x; q < tot; q += kEscBlock) {
            int a = 0, b = cl - 1;
            while (a < b) {
                const int mid = (a + b + 1) >> 1;
                if (c_off[mid] <= q) a = mid; else b = mid - 1;
            }
            const int2 jp = at[c_start[a] + (q - c_off[a])];
            const int64_t dst = base + chunk_base + q;
            keys0[dst] = (uint32_t)jp.x;
            pay0[dst] = ((uint64_t)(uint32_t)(cbase + a) << 32) | (uint64_t)(uint32_t)jp.y;
        }
        chunk_base += tot;
        __syncthreads();
    }
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

__device__ __forceinline__ int64_t run_length(const uint32_t* k, int64_t e, int64_t F) {
    int64_t r = e + 1;
    while (r < F && k[r] == k[e]) ++r;
    return r - e;
}

__global__ __launch_bounds__(kEscBlock) void k_esc_count(
    const OvSet* __restrict__ sets, int nsets, const int64_t* __restrict__ set_base,
    const int32_t* __restrict__ list, const int64_t* __restrict__ esc_off,
    const int64_t* __restrict__ flops_row, const uint32_t* __restrict__ keys0,
    int64_t* __restrict__ nnzrow, int32_t* __restrict__ distinct) {
    __shared__ int64_t s_red;
    const int64_t g = list[blockIdx.x];
    const int s = find_set(set_base, nsets, g);
    const int32_t ms = sets[s].min_shared;
    const uint32_t* k = keys0 + esc_off[g];
    const int64_t F = flops_row[g];
    int64_t runs = 0, sel = 0;
    for (int64_t e = threadIdx.x; e < F; e += kEscBlock) {
        if (e == 0 || k[e] != k[e - 1]) {
            ++runs;
            if (run_length(k, e, F) >= ms) ++sel;
        }
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
    int64_t carry = 0;
    for (int64_t tile = 0; tile < F; tile += kEscBlock) {
        const int64_t e = tile + threadIdx.x;
        int64_t rl = 0;
        int64_t take = 0;
        if (e < F && (e == 0 || k[e] != k[e - 1])) {
            rl = run_length(k, e, F);
            take = rl >= S.min_shared ? 1 : 0;
        }
        int64_t tot;
        const int64_t ex = block_exclusive_sum<kEscBlock>(take, s_tmp, &tot);
        if (take) {
            const int64_t o = off0 + carry + ex;
            const uint64_t a = p[e];
            int32_t pi1 = -1, pj1 = -1;
            if (rl >= 2) {
                const uint64_t b = p[e + 1];
                pi1 = S.a_val[lo + (int64_t)(b >> 32)];
                pj1 = (int32_t)(uint32_t)b;
            }
            S.c_col[o] = (int32_t)k[e];
            S.c_count[o] = (int32_t)rl;
            seed4[o] = make_int4(S.a_val[lo + (int64_t)(a >> 32)], (int32_t)(uint32_t)a, pi1, pj1);
        }
        carry += tot;
    }
}

// ---------------------------------------------------------------------------
// Host driver
// ---------------------------------------------------------------------------
template <int BLOCK>
static size_t sym_lds(int logT) { return (size_t)BLOCK * 16 + ((size_t)8 << logT); }
template <int BLOCK>
static size_t num_lds(int logT) {
    return ((size_t)1 << logT) * (8 + 8 + 4 + 4 + 4) + (size_t)BLOCK * 16;
}

template <int BLOCK>
static int launch_symbolic(const OvSet* d_sets, int nsets, const int64_t* d_base, const int32_t* list,
                           int count, int logT, int limit, const uint64_t* seg, const int2* at,
                           int64_t* nnzrow, int32_t* distinct, OvCounters* ctr, hipStream_t st) {
    const size_t lds = sym_lds<BLOCK>(logT);
    (void)hipFuncSetAttribute((const void*)k_ov_symbolic<BLOCK>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k_ov_symbolic<BLOCK>, dim3(count), dim3(BLOCK), lds, st, d_sets, nsets, d_base,
                       list, logT, limit, seg, at, nnzrow, distinct, ctr);
    DB_HIP(hipGetLastError());
    return DIBELLA_OK;
}

template <int BLOCK>
static int launch_numeric(const OvSet* d_sets, int nsets, const int64_t* d_base, const int32_t* list,
                          int count, int logT, const uint64_t* seg, const int2* at, const int64_t* G,
                          hipStream_t st) {
    const size_t lds = num_lds<BLOCK>(logT);
    (void)hipFuncSetAttribute((const void*)k_ov_numeric<BLOCK>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k_ov_numeric<BLOCK>, dim3(count), dim3(BLOCK), lds, st, d_sets, nsets, d_base,
                       list, logT, seg, at, G);
    DB_HIP(hipGetLastError());
    return DIBELLA_OK;
}

static int dispatch_symbolic(int block, const OvSet* d_sets, int nsets, const int64_t* d_base,
                             const int32_t* list, int count, int logT, int limit, const uint64_t* seg,
                             const int2* at, int64_t* nnzrow, int32_t* distinct, OvCounters* ctr,
                             hipStream_t st) {
    switch (block) {
        case 64: return launch_symbolic<64>(d_sets, nsets, d_base, list, count, logT, limit, seg, at, nnzrow, distinct, ctr, st);
        case 128: return launch_symbolic<128>(d_sets, nsets, d_base, list, count, logT, limit, seg, at, nnzrow, distinct, ctr, st);
        case 512: return launch_symbolic<512>(d_sets, nsets, d_base, list, count, logT, limit, seg, at, nnzrow, distinct, ctr, st);
        default: return launch_symbolic<256>(d_sets, nsets, d_base, list, count, logT, limit, seg, at, nnzrow, distinct, ctr, st);
    }
}

static int dispatch_numeric(int block, const OvSet* d_sets, int nsets, const int64_t* d_base,
                            const int32_t* list, int count, int logT, const uint64_t* seg, const int2* at,
                            const int64_t* G, hipStream_t st) {
    switch (block) {
        case 64: return launch_numeric<64>(d_sets, nsets, d_base, list, count, logT, seg, at, G, st);
        case 128: return launch_numeric<128>(d_sets, nsets, d_base, list, count, logT, seg, at, G, st);
        case 512: return launch_numeric<512>(d_sets, nsets, d_base, list, count, logT, seg, at, G, st);
        default: return launch_numeric<256>(d_sets, nsets, d_base, list, count, logT, seg, at, G, st);
    }
}

static const char* describe_bad(int32_t bad) {
    if (bad & kBadRowptr) return "row pointers are not a valid CSR row pointer array";
    if (bad & kBadCol) return "a column index is outside [0, ncols)";
    if (bad & kUnsorted) return "columns are not strictly increasing within a row";
    if (bad & kNegative) return "a position value is negative";
    if (bad & kLongRow) return "a row has 2^30 or more entries";
    return "malformed matrix";
}

int overlap_run(const dibella_csr* A, int nsets, const int32_t* min_shared, dibella_overlap_out* C,
                uint32_t flags, Arena& ar) {
    hipStream_t st = ar.stream();
    const dibella_tuning tn = tuning();
    dibella_stats& stt = stats();
    // ---- host checks and set layout
    std::vector<OvSet> hs(nsets);
    std::vector<int64_t> base(nsets + 1, 0);
    int64_t total_rows = 0, total_m = 0, total_nnz = 0;
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
        OvSet& o = hs[s];
        std::memset(&o, 0, sizeof(o));
        o.a_rowptr = a.rowptr;
        o.a_col = a.col;
        o.a_val = a.val;
        o.n = a.nrows;
        o.m = a.ncols;
        o.nnz = a.nnz;
        o.row_base = total_rows;
        o.col_base = total_m;
        o.nnz_base = total_nnz;
        o.min_shared = min_shared[s];
        o.id_bits = std::max(1, ceil_log2_i64(std::max<int64_t>(a.nrows, 2)));
        base[s] = total_rows;
        total_rows += a.nrows;
        total_m += a.ncols;
        total_nnz += a.nnz;
    }
    base[nsets] = total_rows;
    if (total_rows >= (int64_t(1) << 31) || total_nnz >= (int64_t(1) << 40)) {
        set_error("batch too large: total rows must be < 2^31 and total nnz < 2^40");
        return DIBELLA_EOVERFLOW;
    }
    for (int s = 0; s < nsets; ++s) {
        C[s].nrows = A[s].nrows;
        C[s].ncols = A[s].nrows;
        C[s].nnz = 0;
        C[s].rowptr = nullptr;
        C[s].col = nullptr;
        C[s].count = nullptr;
        C[s].seed = nullptr;
    }

    // ---- workspace
    OvSet* d_sets;
    int64_t* d_base;
    int32_t* d_flags;
    OvCounters* d_ctr;
    int64_t* d_set_nnz;
    DB_TRY(ar.work_n(nsets, &d_sets));
    DB_TRY(ar.work_n(nsets + 1, &d_base));
    DB_TRY(ar.work_n(nsets, &d_flags));
    DB_TRY(ar.work_n(1, &d_ctr));
    DB_TRY(ar.work_n(nsets, &d_set_nnz));
    int32_t* cnt;
    int64_t* t_rowptr;
    int2* at;
    uint64_t* seg;
    int64_t *flops_row, *nnzrow, *G, *esc_off;
    int32_t *distinct, *sym_list, *num_list, *esc_list;
    DB_TRY(ar.work_n(total_m, &cnt));
    DB_TRY(ar.work_n(total_m + 1, &t_rowptr));
    DB_TRY(ar.work_n(total_nnz, &at));
    DB_TRY(ar.work_n(total_nnz, &seg));
    DB_TRY(ar.work_n(total_rows, &flops_row));
    DB_TRY(ar.work_n(total_rows, &nnzrow));
    DB_TRY(ar.work_n(total_rows + 1, &G));
    DB_TRY(ar.work_n(total_rows, &esc_off));
    DB_TRY(ar.work_n(total_rows, &distinct));
    DB_TRY(ar.work_n((size_t)total_rows * kMaxLog2, &sym_list));
    DB_TRY(ar.work_n((size_t)total_rows * kMaxLog2, &num_list));
    DB_TRY(ar.work_n(total_rows, &esc_list));

    // ---- upload descriptors
    HostStage& hst = host_stage();
    const size_t desc_bytes = sizeof(OvSet) * nsets + sizeof(int64_t) * (nsets + 1);
    const size_t back_bytes = sizeof(OvCounters) + sizeof(int32_t) * nsets + sizeof(int64_t) * nsets;
    DB_TRY(hst.reserve(desc_bytes + back_bytes + 64));
    char* hbuf = static_cast<char*>(hst.ptr);
    std::memcpy(hbuf, hs.data(), sizeof(OvSet) * nsets);
    std::memcpy(hbuf + sizeof(OvSet) * nsets, base.data(), sizeof(int64_t) * (nsets + 1));
    DB_HIP(hipMemcpyAsync(d_sets, hbuf, sizeof(OvSet) * nsets, hipMemcpyHostToDevice, st));
    DB_HIP(hipMemcpyAsync(d_base, hbuf + sizeof(OvSet) * nsets, sizeof(int64_t) * (nsets + 1),
                          hipMemcpyHostToDevice, st));
    DB_TRY(fill_i32(d_flags, 0, nsets, st));
    DB_TRY(fill_i32(reinterpret_cast<int32_t*>(d_ctr), 0, sizeof(OvCounters) / 4, st));
    DB_TRY(fill_i32(cnt, 0, total_m, st));
    DB_TRY(fill_i64(nnzrow, 0, total_rows, st));
    DB_TRY(fill_i32(distinct, 0, total_rows, st));

    // ---- validate + transpose + row costs
    int tok = -1;
    DB_TRY(timing_begin(kPhTranspose, st, &tok));
    constexpr int WPB = 4;
    const int grid_rows = grid_for(total_rows, WPB, 1 << 16);
    const int checks = (flags & DIBELLA_NO_VALIDATE) ? 0 : 1;
    if (total_rows > 0) {
        hipLaunchKernelGGL(k_ov_hist<WPB>, dim3(grid_rows), dim3(WPB * kWave), 0, st, d_sets, nsets,
                           d_base, total_rows, cnt, d_flags, checks);
        DB_HIP(hipGetLastError());
    }
    DB_TRY(scan_exclusive(cnt, t_rowptr, total_m, nullptr, ar));
    const int min_log2 = tn.min_table_log2, load_log2 = tn.load_log2;
    if (total_rows > 0) {
        hipLaunchKernelGGL(k_ov_scatter<WPB>, dim3(grid_rows), dim3(WPB * kWave), 0, st, d_sets, nsets,
                           d_base, total_rows, t_rowptr, cnt, at, seg, flops_row, sym_list, d_ctr,
                           min_log2, tn.sym_max_log2, load_log2);
        DB_HIP(hipGetLastError());
    }
    DB_TRY(timing_end(tok, st));
    // ---- sync 1: validity and bin sizes
    char* back = hbuf + desc_bytes;
    OvCounters* h_ctr = reinterpret_cast<OvCounters*>(back);
    int32_t* h_flags = reinterpret_cast<int32_t*>(back + sizeof(OvCounters));
    int64_t* h_set_nnz = reinterpret_cast<int64_t*>(back + sizeof(OvCounters) + sizeof(int32_t) * nsets);
    DB_HIP(hipMemcpyAsync(h_ctr, d_ctr, sizeof(OvCounters), hipMemcpyDeviceToHost, st));
    DB_HIP(hipMemcpyAsync(h_flags, d_flags, sizeof(int32_t) * nsets, hipMemcpyDeviceToHost, st));
    DB_TRY(sync_stream(st));
    for (int s = 0; s < nsets; ++s) {
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
    stt.products = h_ctr->products;

    // ---- symbolic, largest tables first
    const int sym_max = tn.sym_max_log2;
    for (int lg = sym_max; lg >= min_log2; --lg) {
        const int count = h_ctr->sym_count[lg];
        if (!count) continue;
        const int T = 1 << lg;
        int limit = T + 1;  // smaller tables are sized to never fill
        if (lg == sym_max) limit = std::min(T * 3 / 4, T - tn.sym_block - 1);
        DB_TRY(timing_begin(kPhSymbolic, st, &tok));
        DB_TRY(dispatch_symbolic(tn.sym_block, d_sets, nsets, d_base, sym_list + (int64_t)lg * total_rows,
                                 count, lg, limit, seg, at, nnzrow, distinct, d_ctr, st));
        DB_TRY(timing_end(tok, st));
    }
    if (total_rows > 0) {
        hipLaunchKernelGGL(k_ov_bin_numeric, dim3(grid_for(total_rows, 256, 4096)), dim3(256), 0, st,
                           total_rows, flops_row, distinct, num_list, esc_list, esc_off, d_ctr, min_log2,
                           tn.num_max_log2, load_log2);
        DB_HIP(hipGetLastError());
    }
    DB_TRY(scan_exclusive(nnzrow, G, total_rows, nullptr, ar));
    hipLaunchKernelGGL(k_ov_set_totals, dim3(grid_for(nsets, 64, 1024)), dim3(64), 0, st, d_sets, nsets, G,
                       d_set_nnz);
    DB_HIP(hipGetLastError());
    DB_HIP(hipMemcpyAsync(h_ctr, d_ctr, sizeof(OvCounters), hipMemcpyDeviceToHost, st));
    DB_HIP(hipMemcpyAsync(h_set_nnz, d_set_nnz, sizeof(int64_t) * nsets, hipMemcpyDeviceToHost, st));
    DB_TRY(sync_stream(st));  // sync 2

    // ---- ESC rows
    const int esc_rows = h_ctr->esc_rows;
    stt.esc_rows = esc_rows;
    uint32_t *keys0 = nullptr, *keys1 = nullptr;
    uint64_t *pay0 = nullptr, *pay1 = nullptr;
    if (esc_rows > 0) {
        const int64_t ef = h_ctr->esc_flops;
        DB_TRY(ar.work_n(ef, &keys0));
        DB_TRY(ar.work_n(ef, &keys1));
        DB_TRY(ar.work_n(ef, &pay0));
        DB_TRY(ar.work_n(ef, &pay1));
        DB_TRY(timing_begin(kPhEsc, st, &tok));
        hipLaunchKernelGGL(k_esc_expand, dim3(esc_rows), dim3(kEscBlock), 0, st, d_sets, nsets, d_base,
                           esc_list, esc_off, seg, at, keys0, pay0);
        hipLaunchKernelGGL(k_esc_sort, dim3(esc_rows), dim3(kEscBlock), 0, st, d_sets, nsets, d_base,
                           esc_list, esc_off, flops_row, keys0, pay0, keys1, pay1);
        DB_HIP(hipGetLastError());
        DB_TRY(timing_end(tok, st));
        if (h_ctr->overflow_rows > 0) {
            hipLaunchKernelGGL(k_esc_count, dim3(esc_rows), dim3(kEscBlock), 0, st, d_sets, nsets, d_base,
                               esc_list, esc_off, flops_row, keys0, nnzrow, distinct);
            DB_HIP(hipGetLastError());
            DB_TRY(scan_exclusive(nnzrow, G, total_rows, nullptr, ar));
            hipLaunchKernelGGL(k_ov_set_totals, dim3(grid_for(nsets, 64, 1024)), dim3(64), 0, st, d_sets,
                               nsets, G, d_set_nnz);
            DB_HIP(hipGetLastError());
            DB_HIP(hipMemcpyAsync(h_set_nnz, d_set_nnz, sizeof(int64_t) * nsets, hipMemcpyDeviceToHost, st));
            DB_TRY(sync_stream(st));  // sync 3 (only with overflowing rows)
        }
    }

    // ---- outputs
    for (int s = 0; s < nsets; ++s) {
        const int64_t nz = h_set_nnz[s];
        DB_TRY(ar.output_n(A[s].nrows + 1, &hs[s].c_rowptr));
        DB_TRY(ar.output_n(nz, &hs[s].c_col));
        DB_TRY(ar.output_n(nz, &hs[s].c_count));
        DB_TRY(ar.output_n(4 * nz, &hs[s].c_seed));
        C[s].nnz = nz;
        C[s].rowptr = hs[s].c_rowptr;
        C[s].col = hs[s].c_col;
        C[s].count = hs[s].c_count;
        C[s].seed = hs[s].c_seed;
    }
    std::memcpy(hbuf, hs.data(), sizeof(OvSet) * nsets);
    DB_HIP(hipMemcpyAsync(d_sets, hbuf, sizeof(OvSet) * nsets, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_ov_write_rowptr, dim3(grid_for(total_rows + nsets, 256, 4096)), dim3(256), 0, st,
                       d_sets, nsets, d_base, total_rows, G);
    DB_HIP(hipGetLastError());
    const int num_max = tn.num_max_log2;
    for (int lg = num_max; lg >= min_log2; --lg) {
        const int count = h_ctr->num_count[lg];
        if (!count) continue;
        DB_TRY(timing_begin(kPhNumeric, st, &tok));
        DB_TRY(dispatch_numeric(tn.num_block, d_sets, nsets, d_base, num_list + (int64_t)lg * total_rows,
                                count, lg, seg, at, G, st));
        DB_TRY(timing_end(tok, st));
    }
    if (esc_rows > 0) {
        DB_TRY(timing_begin(kPhEsc, st, &tok));
        hipLaunchKernelGGL(k_esc_emit, dim3(esc_rows), dim3(kEscBlock), 0, st, d_sets, nsets, d_base,
                           esc_list, esc_off, flops_row, keys0, pay0, G);
        DB_HIP(hipGetLastError());
        DB_TRY(timing_end(tok, st));
    }
    DB_TRY(stage_done(st));
    return DIBELLA_OK;
}

}  // namespace dibella
