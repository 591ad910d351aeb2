// Seed-and-extend alignment of every candidate pair of C, and the overlap
// graph R from the alignment ends (Sec. IV-D: each entry of C is aligned in
// place, and the entries whose score is below the threshold are pruned,
// leaving R; Sec. IV-E: the suffix and orientation the reduction needs come
// from the alignment coordinates, by the four overlap categories).
//
// Each off-diagonal entry C_ij is aligned from its first seed, the k-mer at
// p_i in read i and p_j in read j.  When the strands of the seed differ the
// pair is reverse complementary and read j is taken reverse complemented
// (j'), the k-mer then sitting at q = L_j - k - p_j in j' (else q = p_j).
// The seed is extended to the right (i after p_i + k against j' after
// q + k) and to the left (i before p_i against j' before q, both read
// backwards) by X-drop extension (Zhang, Schwartz, Wagner and Miller, 2000)
// with linear scores: T(x, y) = the best score of aligning the first x
// bases of one side with the first y of the other, T(0, 0) = 0, a match
// `match`, a mismatch `mismatch`, a base against a gap `gap`.  The table is
// filled anti-diagonal by anti-diagonal (d = x + y); on anti-diagonal d only
// cells with a live predecessor are considered (x or x - 1 on d - 1, x - 1
// on d - 2), and a cell scoring below the best score of the earlier
// anti-diagonals minus X is dead.  An extension ends when two anti-diagonals
// in a row hold no live cell, at the sequence ends, or before an
// anti-diagonal that would consider more than 256 cells.  Its result is the
// best score and the first cell (anti-diagonal order, then x order) that
// reaches it.  The pair's score is left + k * match + right; entries
// scoring below min_score are pruned.  The alignment spans [b_i, e_i) of i
// and [b_j, e_j) of j'; r_i = L_i - e_i and r_j = L_j - e_j are the
// unaligned right ends.  A read whose unaligned ends both lie within the
// other's (b_j >= b_i and r_j >= r_i, or the reverse) is contained: value
// 0.  Otherwise read i first (b_i > b_j): suffix r_j - r_i, code (0, rc);
// read j first: suffix b_j - b_i, code (1, 1 - rc); value (suffix << 2) |
// code, the layout of the transitive reduction.
//
// Work: every extension (two per entry) is a task; groups of G lanes (16, 32
// or 64 of a wave) take tasks from a device counter and walk one
// anti-diagonal per step, G cells at a time.  The three live anti-diagonals
// of a group are rings of 256 scores in LDS indexed by x mod 256 (a live
// range never spans more), and the bases of the two sides are staged in
// LDS rings of 1024 positions, refilled 512 at a time as the band moves
// forward.  A group that finishes takes its next task in the same loop while
// the other groups of its wave go on.
#include "common.hpp"

#include <algorithm>
#include <atomic>
#include <cstring>

namespace dibella {

enum : int32_t {
    kAlBadRowptr = 1,
    kAlBadCol = 2,
    kAlUnsorted = 4,
    kAlBadSeed = 8,
    kAlBadOffsets = 16,
    kAlBadBase = 32,
};

constexpr int kAlBand = 256;     // most cells one anti-diagonal may consider
constexpr int kAlWin = 1024;     // staged bases per side (ring by position)
constexpr int kAlFill = 512;     // bases staged per refill
constexpr int32_t kAlDead = INT32_MIN;
constexpr int64_t kAlMaxLen = int64_t(1) << 28;

// ---------------------------------------------------------------------------
// Checks of the reads: offsets run from 0 to nbases without going back,
// every read is shorter than 2^28 bases and every base is 0..3.
// ---------------------------------------------------------------------------
__global__ void k_al_offsets(const int64_t* __restrict__ off, int64_t n, int64_t nbases, int32_t* flags) {
    int32_t bad = 0;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
        const int64_t a = off[r], b = off[r + 1];
        if (a < 0 || b < a || b > nbases || b - a >= kAlMaxLen) bad = kAlBadOffsets;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0 && (off[0] != 0 || off[n] != nbases)) bad = kAlBadOffsets;
    if (bad) atomicOr(flags, bad);
}

__global__ void k_al_bases(const uint8_t* __restrict__ bases, int64_t head, int64_t nvec, int64_t nbases,
                           int32_t* flags) {
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, stride = (int64_t)gridDim.x * blockDim.x;
    uint32_t acc = 0;
    const uint4* v = reinterpret_cast<const uint4*>(bases + head);
    for (int64_t w = tid; w < nvec; w += stride) {
        const uint4 x = v[w];
        acc |= x.x | x.y | x.z | x.w;
    }
    // the bytes before the first 16-byte boundary and after the last
    const int64_t tail0 = head + nvec * 16;
    for (int64_t p = tid; p < head + (nbases - tail0); p += stride) {
        const int64_t at = p < head ? p : tail0 + (p - head);
        acc |= bases[at];
    }
    if (acc & 0xFCFCFCFCu) atomicOr(flags, kAlBadBase);
}

// ---------------------------------------------------------------------------
// Checks of C (one wave per row): row pointers, columns in range and
// increasing, seeds of off-diagonal entries present and inside their reads.
// Writes the row of every entry for the extension tasks.
// ---------------------------------------------------------------------------
template <int WPB>
__global__ __launch_bounds__(WPB* kWave) void k_al_rows(int64_t n, int64_t ncols, int64_t nnz,
                                                        const int64_t* __restrict__ rp,
                                                        const int32_t* __restrict__ col,
                                                        const int32_t* __restrict__ seed,
                                                        const int64_t* __restrict__ off, int32_t k,
                                                        int32_t* __restrict__ row_of, int32_t* flags) {
    const int lane = lane_id();
    for (int64_t i = (int64_t)blockIdx.x * WPB + __builtin_amdgcn_readfirstlane(wave_id()); i < n;
         i += (int64_t)gridDim.x * WPB) {
        const int64_t lo = rp[i], hi = rp[i + 1];
        int32_t bad = 0;
        if ((i == 0 && lo != 0) || (i == n - 1 && hi != nnz) || lo < 0 || hi < lo || hi > nnz) {
            bad |= kAlBadRowptr;
        } else {
            const int64_t li = off[i + 1] - off[i];
            for (int64_t e = lo + lane; e < hi; e += kWave) {
                const int32_t j = col[e];
                row_of[e] = (int32_t)i;
                if (j < 0 || j >= ncols) {
                    bad |= kAlBadCol;
                    continue;
                }
                if (e > lo && col[e - 1] >= j) bad |= kAlUnsorted;
                if (j == i) continue;
                const int32_t a = seed[4 * e], b = seed[4 * e + 1];
                const int64_t lj = off[j + 1] - off[j];
                if (a < 0 || b < 0 || (a >> 1) + (int64_t)k > li || (b >> 1) + (int64_t)k > lj) bad |= kAlBadSeed;
            }
        }
        bad = wave_or_i32(bad);
        if (lane == 0 && bad) atomicOr(flags, bad);
    }
}

// ---------------------------------------------------------------------------
// The extensions.  Task t: entry t >> 1, right side (t even) or left side.
// Result per task: {best score, x end, y end, 0}.
// ---------------------------------------------------------------------------
struct AlSide {
    int64_t s0;    // index in bases of position 0
    int32_t dir;   // +1 or -1 per position
    int32_t comp;  // complement the bases
    int32_t len;   // positions
};

template <int G>
__device__ __forceinline__ int32_t group_max(int32_t v) {
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) {
        const int32_t w = __shfl_xor(v, o, G);
        v = w > v ? w : v;
    }
    return v;
}

// The maximum over a group of G lanes (G = 16, 32 or 64), in every lane of
// the group, without shuffles through LDS: lane swaps inside quads and
// mirrors inside rows of 16 (DPP), the two rows of 32 lanes by a swizzle,
// the two halves of a wave by reading one lane of each.
template <int G>
__device__ __forceinline__ int32_t group_max_dpp(int32_t v) {
    static_assert(G == 16 || G == 32 || G == 64, "groups of 16, 32 or 64 lanes");
    v = max(v, __builtin_amdgcn_update_dpp(v, v, 0xB1, 0xF, 0xF, false));    // quad_perm [1, 0, 3, 2]
    v = max(v, __builtin_amdgcn_update_dpp(v, v, 0x4E, 0xF, 0xF, false));    // quad_perm [2, 3, 0, 1]
    v = max(v, __builtin_amdgcn_update_dpp(v, v, 0x141, 0xF, 0xF, false));   // mirror within half rows
    v = max(v, __builtin_amdgcn_update_dpp(v, v, 0x140, 0xF, 0xF, false));   // mirror within rows
    if (G >= 32) v = max(v, __builtin_amdgcn_ds_swizzle(v, 0x401F));          // lane ^ 16 within 32
    if (G == 64) v = max(__builtin_amdgcn_readlane(v, 0), __builtin_amdgcn_readlane(v, 32));
    return v;
}

__device__ __forceinline__ void lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Stage positions [from, min(from + FILL, side.len)) of a side into its ring
// of WIN positions.
template <int G, int WIN = kAlWin, int FILL = kAlFill>
__device__ __forceinline__ void al_stage(uint8_t* ring, const uint8_t* __restrict__ bases, const AlSide& s,
                                         int32_t from, int gl) {
    const int32_t to = min(from + FILL, s.len);
#pragma unroll 4
    for (int32_t p = from + gl; p < to; p += G) {
        uint8_t b = bases[s.s0 + (int64_t)s.dir * p];
        ring[p & (WIN - 1)] = s.comp ? (uint8_t)(3 - b) : b;
    }
}

// Make positions [lo, hi] of a side readable from its ring, the staged range
// being [vl, wh) (at most WIN positions): a band below the staged range
// restarts it at lo; then blocks of FILL positions are staged until hi is
// covered.  A band spans at most WIN - FILL positions, so the ring keeps all
// of [lo, hi].  Returns whether anything was staged.
template <int G, int WIN = kAlWin, int FILL = kAlFill>
__device__ __forceinline__ bool al_cover(uint8_t* ring, const uint8_t* __restrict__ bases, const AlSide& s,
                                         int32_t lo, int32_t hi, int32_t& vl, int32_t& wh, int gl) {
    bool staged = false;
    if (lo < vl) vl = lo, wh = lo;
    while (hi >= wh && wh < s.len) {
        al_stage<G, WIN, FILL>(ring, bases, s, wh, gl);
        wh += FILL;
        vl = max(vl, wh - WIN);
        staged = true;
    }
    return staged;
}

// The two sides of extension `task` (entry task >> 1; right side for an even
// task, left side for an odd one) of the off-diagonal entry C_ij with first
// seed (a, b): read i against read j, or its reverse complement when the
// seed's strands differ.
__device__ __forceinline__ void al_sides(int64_t task, int32_t i, int32_t j, int32_t a, int32_t b,
                                         const int64_t* __restrict__ off, int32_t k, AlSide& A, AlSide& B) {
    const int64_t oi = off[i], oj = off[j];
    const int32_t li = (int32_t)(off[i + 1] - oi), lj = (int32_t)(off[j + 1] - oj);
    const bool rc = ((a ^ b) & 1) != 0;
    const int32_t pi = a >> 1, pj = b >> 1;
    const int32_t q = rc ? lj - k - pj : pj;
    if ((task & 1) == 0) {
        A = AlSide{oi + pi + k, 1, 0, li - pi - k};
        B = rc ? AlSide{oj + (lj - 1 - q - k), -1, 1, lj - q - k} : AlSide{oj + q + k, 1, 0, lj - q - k};
    } else {
        A = AlSide{oi + pi - 1, -1, 0, pi};
        B = rc ? AlSide{oj + (lj - q), 1, 1, q} : AlSide{oj + q - 1, -1, 0, q};
    }
}

template <int G>
__global__ __launch_bounds__(kWave) void k_al_extend(int64_t ntasks, const int64_t* __restrict__ list,
                                                     const unsigned long long* __restrict__ list_count,
                                                     const int32_t* __restrict__ row_of,
                                                     const int32_t* __restrict__ col,
                                                     const int32_t* __restrict__ seed,
                                                     const uint8_t* __restrict__ bases,
                                                     const int64_t* __restrict__ off, int32_t k, int32_t mat,
                                                     int32_t mis, int32_t gap, int32_t X,
                                                     unsigned long long* __restrict__ next,
                                                     int4* __restrict__ ext) {
    // next[0]: the next task; next[1]: cells considered, over all
    // extensions.  With a list, the tasks are list[0, *list_count) and
    // next[0] counts through the list.
    constexpr int NG = kWave / G;
    constexpr uint64_t kMask = G == 64 ? ~0ull : ((1ull << (G & 63)) - 1);   // a group's lanes, from bit 0
    __shared__ int32_t s_score[NG][3][kAlBand];
    __shared__ uint8_t s_base[NG][2][kAlWin];
    const int lane = threadIdx.x;
    const int grp = lane / G, gl = lane % G;
    const int leader = grp * G;
    int32_t(*ring)[kAlBand] = s_score[grp];
    uint8_t* wa = s_base[grp][0];
    uint8_t* wb = s_base[grp][1];

    // group state (the same in every lane of the group)
    bool busy = false, done = false;
    int64_t task = 0;
    AlSide A{}, B{};
    int32_t d = 0, r0 = 0;                 // current anti-diagonal and its ring (d mod 3)
    int32_t lo1 = 0, hi1 = -1, lo2 = 0, hi2 = -1;   // live ranges of d - 1 and d - 2
    int32_t best = 0, bx = 0, bd = 0;      // best score, its x and anti-diagonal
    int32_t vlA = 0, whA = 0, vlB = 0, whB = 0;   // staged positions [vl, wh) of each side
    unsigned long long cells = 0;          // cells this group considered

    const int64_t nt = list ? (int64_t)*list_count : ntasks;
    for (;;) {
        if (!busy && !done) {
            unsigned long long t = 0;
            if (gl == 0) t = atomicAdd(next, 1ull);
            t = __shfl(t, leader, kWave);
            if ((int64_t)t >= nt) {
                done = true;
            } else {
                task = list ? list[t] : (int64_t)t;
                const int64_t e = task >> 1;
                const int32_t i = row_of[e], j = col[e];
                if (i == j) {
                    if (gl == 0) ext[task] = make_int4(0, 0, 0, 0);
                } else {
                    al_sides(task, i, j, seed[4 * e], seed[4 * e + 1], off, k, A, B);
                    // anti-diagonal 0: the cell (0, 0)
                    if (gl == 0) ring[0][0] = 0;
                    d = 0;
                    r0 = 0;
                    lo1 = 0, hi1 = 0, lo2 = 0, hi2 = -1;
                    best = 0, bx = 0, bd = 0;
                    vlA = 0, whA = 0, vlB = 0, whB = 0;
                    busy = true;
                    lds_sync();
                }
            }
        }
        // leave once every group of the wave has run out of tasks
        if (__ballot(!done) == 0) {
            if (gl == 0 && cells) atomicAdd(next + 1, cells);
            break;
        }
        if (!busy) continue;

        // one anti-diagonal
        ++d;
        r0 = r0 == 2 ? 0 : r0 + 1;
        const int r1 = r0 == 0 ? 2 : r0 - 1, r2 = r1 == 0 ? 2 : r1 - 1;
        const int32_t m = A.len, n = B.len;
        bool finish = d > m + n || (lo1 > hi1 && lo2 > hi2);
        int32_t from = INT32_MAX, to = INT32_MIN;
        if (!finish) {
            if (lo1 <= hi1) from = lo1, to = hi1 + 1;
            if (lo2 <= hi2) from = min(from, lo2 + 1), to = max(to, hi2 + 1);
            from = max(from, max(d - n, 0));
            to = min(to, min(m, d));
            if (from <= to && to - from + 1 > kAlBand) finish = true;
        }
        if (!finish && from > to) {            // no cell to consider: an empty anti-diagonal
            lo2 = lo1, hi2 = hi1;
            lo1 = 0, hi1 = -1;
            continue;
        }
        if (!finish) {
            // stage the bases the cells read: positions x - 1 in [from - 1, to - 1]
            // of side A and y - 1 in [d - to - 1, d - from - 1] of side B
            bool staged = false;
            if (to >= 1) staged |= al_cover<G>(wa, bases, A, max(from - 1, 0), to - 1, vlA, whA, gl);
            if (d - from >= 1) staged |= al_cover<G>(wb, bases, B, max(d - to - 1, 0), d - from - 1, vlB, whB, gl);
            if (staged) lds_sync();
            cells += (unsigned long long)(to - from + 1);
            const int32_t floor_ = best - X;
            int32_t nlo = 0, nhi = -1, dbest = kAlDead, dx = 0;
            for (int32_t c0 = from; c0 <= to; c0 += G) {
                const int32_t x = c0 + gl, y = d - x;
                int32_t v = kAlDead;
                if (x <= to) {
                    if (x >= 1 && y >= 1 && x - 1 >= lo2 && x - 1 <= hi2) {
                        const int32_t p = ring[r2][(x - 1) & (kAlBand - 1)];
                        if (p != kAlDead)
                            v = p + (wa[(x - 1) & (kAlWin - 1)] == wb[(y - 1) & (kAlWin - 1)] ? mat : mis);
                    }
                    if (x >= 1 && x - 1 >= lo1 && x - 1 <= hi1) {
                        const int32_t p = ring[r1][(x - 1) & (kAlBand - 1)];
                        if (p != kAlDead && p + gap > v) v = p + gap;
                    }
                    if (y >= 1 && x >= lo1 && x <= hi1) {
                        const int32_t p = ring[r1][x & (kAlBand - 1)];
                        if (p != kAlDead && p + gap > v) v = p + gap;
                    }
                    if (v != kAlDead && v < floor_) v = kAlDead;
                    ring[r0][x & (kAlBand - 1)] = v;
                }
                const uint64_t live = (__ballot(v != kAlDead) >> leader) & kMask;
                if (live) {
                    if (nlo > nhi) nlo = c0 + __builtin_ctzll(live);
                    nhi = c0 + 63 - __builtin_clzll(live);
                    const int32_t cmax = group_max<G>(v);
                    if (cmax > dbest) {
                        const uint64_t at =
                            (__ballot(v == cmax) >> leader) & kMask;
                        dbest = cmax;
                        dx = c0 + __builtin_ctzll(at);
                    }
                }
            }
            lds_sync();
            lo2 = lo1, hi2 = hi1;
            lo1 = nlo, hi1 = nhi;
            if (nlo <= nhi && dbest > best) best = dbest, bx = dx, bd = d;
            continue;
        }
        // the extension is over
        if (gl == 0) ext[task] = make_int4(best, bx, bd - bx, 0);
        busy = false;
    }
}

// ---------------------------------------------------------------------------
// The extensions, fast path: an extension whose anti-diagonals never ask for
// more than G * C cells (the common case: an extension keeps about
// 2X / (match - gap) cells live).  Each lane of a group of G holds C cells
// of the current anti-diagonal, x = from + lane + G * h for h < C; the two
// earlier anti-diagonals stay in registers (a lane's cells there counted
// from that anti-diagonal's first considered cell) and are read across lanes
// by shuffles, so no score goes through LDS; only the bases are staged, in
// rings of kBandWin positions.  Two cells a lane halve the groups' share of
// the per-step bookkeeping (range update, staging checks, ballots, group
// maximum), which runs once per group and step whatever C is.  The cells
// considered, the dead ones, the ranges and the best cell are exactly the
// general kernel's.  An extension that would consider more than G * C cells
// on one anti-diagonal is appended to `fb` (fb_count[0] entries) and left to
// the general kernel, which redoes it from the start; its cells are counted
// there only.
// ---------------------------------------------------------------------------
constexpr int kBandWin = 256;
constexpr int kBandFill = 128;

template <int G, int C>
__global__ __launch_bounds__(kWave) void k_al_band(int64_t ntasks, const int32_t* __restrict__ row_of,
                                                   const int32_t* __restrict__ col,
                                                   const int32_t* __restrict__ seed,
                                                   const uint8_t* __restrict__ bases,
                                                   const int64_t* __restrict__ off, int32_t k, int32_t mat,
                                                   int32_t mis, int32_t gap, int32_t X,
                                                   unsigned long long* __restrict__ next, int4* __restrict__ ext,
                                                   int64_t* __restrict__ fb,
                                                   unsigned long long* __restrict__ fb_count) {
    // next[0]: the next task; next[1]: cells considered by finished extensions
    constexpr int NG = kWave / G;
    constexpr int BW = G * C;   // cells a group holds: lane l holds cells from + l + G * h, h < C
    constexpr uint64_t kMask = G == 64 ? ~0ull : ((1ull << (G & 63)) - 1);
    static_assert(C == 1 || C == 2, "one or two cells per lane");
    static_assert(BW <= 64, "a group's cells fit one 64-bit mask");
    static_assert(BW <= kBandWin - kBandFill, "a band fits the staged bases");
    constexpr int LG = G == 16 ? 4 : G == 32 ? 5 : 6;
    __shared__ uint8_t s_base[NG][2][kBandWin];
    const int lane = threadIdx.x;
    const int grp = lane / G, gl = lane % G;
    const int leader = grp * G;
    uint8_t* wa = s_base[grp][0];
    uint8_t* wb = s_base[grp][1];

    // group state (the same in every lane of the group)
    bool busy = false, done = false;
    int64_t task = 0;
    AlSide A{}, B{};
    int32_t d = 0;
    int32_t lo1 = 0, hi1 = -1, lo2 = 0, hi2 = -1;   // live ranges of d - 1 and d - 2
    int32_t f1 = 0, f2 = 0;                          // their first considered cells
    int32_t best = 0, bx = 0, bd = 0;
    int32_t vlA = 0, whA = 0, vlB = 0, whB = 0;
    unsigned long long tcells = 0, cells = 0;
    // this lane's cells of d - 1 and d - 2
    int32_t v1[C], v2[C];
#pragma unroll
    for (int h = 0; h < C; ++h) v1[h] = v2[h] = kAlDead;

    for (;;) {
        if (!busy && !done) {
            unsigned long long t = 0;
            if (gl == 0) t = atomicAdd(next, 1ull);
            t = __shfl(t, leader, kWave);
            if ((int64_t)t >= ntasks) {
                done = true;
            } else {
                task = (int64_t)t;
                const int64_t e = task >> 1;
                const int32_t i = row_of[e], j = col[e];
                if (i == j) {
                    if (gl == 0) ext[task] = make_int4(0, 0, 0, 0);
                } else {
                    al_sides(task, i, j, seed[4 * e], seed[4 * e + 1], off, k, A, B);
                    // anti-diagonal 0: the cell (0, 0)
                    d = 0;
                    lo1 = 0, hi1 = 0, f1 = 0;
                    lo2 = 0, hi2 = -1, f2 = 0;
#pragma unroll
                    for (int h = 0; h < C; ++h) {
                        v1[h] = (gl == 0 && h == 0) ? 0 : kAlDead;
                        v2[h] = kAlDead;
                    }
                    best = 0, bx = 0, bd = 0;
                    vlA = 0, whA = 0, vlB = 0, whB = 0;
                    tcells = 0;
                    busy = true;
                }
            }
        }
        // leave once every group of the wave has run out of tasks
        if (__ballot(!done) == 0) {
            if (gl == 0 && cells) atomicAdd(next + 1, cells);
            break;
        }
        if (!busy) continue;

        ++d;
        const int32_t m = A.len, n = B.len;
        bool finish = d > m + n || (lo1 > hi1 && lo2 > hi2);
        int32_t from = INT32_MAX, to = INT32_MIN;
        if (!finish) {
            if (lo1 <= hi1) from = lo1, to = hi1 + 1;
            if (lo2 <= hi2) from = min(from, lo2 + 1), to = max(to, hi2 + 1);
            from = max(from, max(d - n, 0));
            to = min(to, min(m, d));
            if (from <= to && to - from + 1 > kAlBand) finish = true;
        }
        if (!finish && from > to) {            // no cell to consider: an empty anti-diagonal
            lo2 = lo1, hi2 = hi1, f2 = f1;
            lo1 = 0, hi1 = -1;
#pragma unroll
            for (int h = 0; h < C; ++h) v2[h] = v1[h], v1[h] = kAlDead;
            continue;
        }
        if (!finish && to - from + 1 > BW) {   // wider than the group holds: the general kernel redoes it
            if (gl == 0) fb[atomicAdd(fb_count, 1ull)] = task;
            busy = false;
            continue;
        }
        if (!finish) {
            // stage the bases the cells read: positions x - 1 in [from - 1, to - 1]
            // of side A and y - 1 in [d - to - 1, d - from - 1] of side B
            bool staged = false;
            if (to >= 1)
                staged |= al_cover<G, kBandWin, kBandFill>(wa, bases, A, max(from - 1, 0), to - 1, vlA, whA, gl);
            if (d - from >= 1)
                staged |= al_cover<G, kBandWin, kBandFill>(wb, bases, B, max(d - to - 1, 0), d - from - 1, vlB, whB,
                                                           gl);
            if (staged) lds_sync();
            tcells += (unsigned long long)(to - from + 1);
            // the predecessors of cell c = gl + G * h: x - 1 on d - 2 (index
            // c + from - f2 - 1 there), x - 1 and x on d - 1 (c + from - f1 - 1,
            // c + from - f1).  Index t sits in lane t mod G, part t / G: the
            // lane is the same for every h, so one shuffle per part serves all.
            int32_t pd[C], pl[C], pu[C];
#pragma unroll
            for (int h = 0; h < C; ++h) pd[h] = pl[h] = pu[h] = kAlDead;
            const int od = from - f2 - 1, ol = from - f1 - 1, ou = from - f1;
#pragma unroll
            for (int q = 0; q < C; ++q) {
                const int32_t sd = __shfl(v2[q], gl + od, G);
                const int32_t sl = __shfl(v1[q], gl + ol, G);
                const int32_t su = __shfl(v1[q], gl + ou, G);
#pragma unroll
                for (int h = 0; h < C; ++h) {
                    if (C == 1 || ((gl + G * h + od) >> LG) == q) pd[h] = sd;
                    if (C == 1 || ((gl + G * h + ol) >> LG) == q) pl[h] = sl;
                    if (C == 1 || ((gl + G * h + ou) >> LG) == q) pu[h] = su;
                }
            }
            int32_t v[C];
#pragma unroll
            for (int h = 0; h < C; ++h) {
                const int32_t x = from + gl + G * h, y = d - x;
                const uint8_t ca = wa[(x - 1) & (kBandWin - 1)], cb = wb[(y - 1) & (kBandWin - 1)];
                int32_t w = kAlDead;
                if (x <= to) {
                    if (x >= 1 && y >= 1 && x - 1 >= lo2 && x - 1 <= hi2 && pd[h] != kAlDead)
                        w = pd[h] + (ca == cb ? mat : mis);
                    if (x >= 1 && x - 1 >= lo1 && x - 1 <= hi1 && pl[h] != kAlDead && pl[h] + gap > w) w = pl[h] + gap;
                    if (y >= 1 && x >= lo1 && x <= hi1 && pu[h] != kAlDead && pu[h] + gap > w) w = pu[h] + gap;
                    if (w != kAlDead && w < best - X) w = kAlDead;
                }
                v[h] = w;
            }
            uint64_t live = 0;
#pragma unroll
            for (int h = 0; h < C; ++h) live |= ((__ballot(v[h] != kAlDead) >> leader) & kMask) << (G * h);
            lo2 = lo1, hi2 = hi1, f2 = f1;
            f1 = from;
#pragma unroll
            for (int h = 0; h < C; ++h) v2[h] = v1[h], v1[h] = v[h];
            if (live) {
                lo1 = from + __builtin_ctzll(live);
                hi1 = from + 63 - __builtin_clzll(live);
                int32_t vm = v[0];
#pragma unroll
                for (int h = 1; h < C; ++h) vm = max(vm, v[h]);
                const int32_t dmax = group_max_dpp<G>(vm);
                if (dmax > best) {
                    uint64_t at = 0;
#pragma unroll
                    for (int h = 0; h < C; ++h) at |= ((__ballot(v[h] == dmax) >> leader) & kMask) << (G * h);
                    best = dmax, bx = from + __builtin_ctzll(at), bd = d;
                }
            } else {
                lo1 = 0, hi1 = -1;
            }
            continue;
        }
        // the extension is over
        if (gl == 0) ext[task] = make_int4(best, bx, bd - bx, 0);
        cells += tcells;
        busy = false;
    }
}

// ---------------------------------------------------------------------------
// Scores and R's values from the two extensions of every entry (one wave
// per row); entries below min_score get -1.
// ---------------------------------------------------------------------------
template <int WPB>
__global__ __launch_bounds__(WPB* kWave) void k_al_values(int64_t n, const int64_t* __restrict__ rp,
                                                          const int32_t* __restrict__ col,
                                                          const int32_t* __restrict__ seed,
                                                          const int64_t* __restrict__ off,
                                                          const int4* __restrict__ ext, int32_t k, int32_t mat,
                                                          int32_t min_score, int32_t* __restrict__ tmp,
                                                          int32_t* __restrict__ score, int64_t* __restrict__ cnt) {
    const int lane = lane_id();
    for (int64_t i = (int64_t)blockIdx.x * WPB + __builtin_amdgcn_readfirstlane(wave_id()); i < n;
         i += (int64_t)gridDim.x * WPB) {
        const int64_t lo = rp[i], hi = rp[i + 1];
        const int64_t li = off[i + 1] - off[i];
        int64_t kept = 0;
        for (int64_t e = lo + lane; e < hi; e += kWave) {
            const int32_t j = col[e];
            int32_t out = -1, sc = 0;
            if (j != i) {
                const int4 R = ext[2 * e], L = ext[2 * e + 1];
                sc = L.x + k * mat + R.x;
                if (sc >= min_score) {
                    const int32_t a = seed[4 * e], b = seed[4 * e + 1];
                    const int64_t lj = off[j + 1] - off[j];
                    const bool rc = ((a ^ b) & 1) != 0;
                    const int64_t pi = a >> 1, q = rc ? lj - k - (b >> 1) : (b >> 1);
                    const int64_t bi = pi - L.y, ei = pi + k + R.y, bj = q - L.z, ej = q + k + R.z;
                    const int64_t ri = li - ei, rj = lj - ej;
                    if ((bj >= bi && rj >= ri) || (bi >= bj && ri >= rj)) {
                        out = 0;
                    } else if (bi > bj) {
                        out = (int32_t)(((rj - ri) << 2) | (rc ? 1 : 0));
                    } else {
                        out = (int32_t)(((bj - bi) << 2) | (rc ? 2 : 3));
                    }
                }
            }
            tmp[e] = out;
            if (score) score[e] = sc;
            kept += out >= 0 ? 1 : 0;
        }
        kept = wave_sum(kept);
        if (lane == 0) cnt[i] = kept;
    }
}

static const char* describe_al_bad(int32_t bad) {
    if (bad & kAlBadOffsets)
        return "offsets must run from 0 to nbases, never decreasing, with every read shorter than 2^28 bases";
    if (bad & kAlBadBase) return "a base is outside 0..3";
    if (bad & kAlBadRowptr) return "row pointers of C are not a valid CSR row pointer array";
    if (bad & kAlBadCol) return "a column index of C is outside [0, ncols)";
    if (bad & kAlUnsorted) return "columns of C are not strictly increasing within a row";
    if (bad & kAlBadSeed) return "a seed of an off-diagonal entry is missing or lies outside its read";
    return "malformed input";
}

// Cells a group of the fast path holds (0: no fast path) from the band an
// extension keeps live, about 2X / (match - gap) cells, with room to spare:
// 16 is one cell a lane in groups of 16, 32 two cells a lane in groups of 16,
// 64 one cell a lane in groups of 64.
static int al_band_group(int32_t mat, int32_t gap, int32_t X) {
    const int64_t band = 2 * (int64_t)X / (mat - gap);
    return band <= 10 ? 16 : band <= 24 ? 32 : band <= 48 ? 64 : 0;
}

// Lanes per extension of the general kernel: about the band an extension
// keeps live, 2X / (match - gap) cells.
static int al_group(int32_t mat, int32_t gap, int32_t X, uint32_t flags) {
    const uint32_t g = flags & DIBELLA_ALIGN_GROUP_MASK;
    if (g == DIBELLA_ALIGN_GROUP_16) return 16;
    if (g == DIBELLA_ALIGN_GROUP_32) return 32;
    if (g == DIBELLA_ALIGN_GROUP_64) return 64;
    const int64_t band = 2 * (int64_t)X / (mat - gap);
    return band <= 16 ? 16 : band <= 40 ? 32 : 64;
}

static int al_cus() {
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
    return cus;
}

// One wave per workgroup; as many waves as the tasks need, up to 32 per CU.
static int al_band_grid(int64_t ntasks, int G) {
    const int64_t waves = ceil_div(ntasks, kWave / G);
    return (int)std::max<int64_t>(1, std::min<int64_t>(waves, (int64_t)al_cus() * 32));
}

static int al_grid(int64_t ntasks, int G) {
    const int cus = al_cus();
    const int ng = kWave / G;
    const size_t lds = (size_t)ng * (3 * kAlBand * sizeof(int32_t) + 2 * kAlWin);
    const int per_cu = (int)std::max<size_t>(1, std::min<size_t>(32, (160 * 1024) / lds));
    const int64_t waves = ceil_div(ntasks, ng);
    return (int)std::max<int64_t>(1, std::min<int64_t>(waves, (int64_t)cus * per_cu));
}

int r_from_alignment_run(const dibella_overlap_out* C, const uint8_t* bases, int64_t nbases, const int64_t* offsets,
                         int32_t k, int32_t mat, int32_t mis, int32_t gap, int32_t X, int32_t min_score,
                         uint32_t flags, dibella_csr_out* R, int32_t** score_out, Arena& ar) {
    hipStream_t st = ar.stream();
    std::memset(R, 0, sizeof(*R));
    if (score_out) *score_out = nullptr;
    const int64_t n = C->nrows, nnz = C->nnz;
    if (n < 0 || nnz < 0 || C->ncols != n || nbases < 0 || k < 1 || k > 32 || mat < 1 || mat > 7 || mis < -1024 ||
        mis > 0 || gap < -1024 || gap > -1 || X < 0 || X > (1 << 20) || (flags & ~DIBELLA_ALIGN_GROUP_MASK) ||
        (flags & DIBELLA_ALIGN_GROUP_MASK) > DIBELLA_ALIGN_GROUP_64) {
        set_error("dibella_r_from_alignment: C must be square with non-negative sizes; k in [1, 32], match in "
                  "[1, 7], mismatch in [-1024, 0], gap in [-1024, -1], xdrop in [0, 2^20], known flags");
        return DIBELLA_EINVAL;
    }
    if (n >= (int64_t(1) << 31) || nnz >= (int64_t(1) << 40)) {
        set_error("dibella_r_from_alignment: nrows must be < 2^31 and nnz < 2^40");
        return DIBELLA_EOVERFLOW;
    }
    if (!offsets || (n > 0 && !C->rowptr) || (nnz > 0 && (!C->col || !C->seed)) || (nbases > 0 && !bases)) {
        set_error("dibella_r_from_alignment: null pointer");
        return DIBELLA_EINVAL;
    }
    if (n == 0 && nnz != 0) {
        set_error("dibella_r_from_alignment: entries in a matrix without rows");
        return DIBELLA_EINVAL;
    }
    R->nrows = n;
    R->ncols = n;
    int32_t *row_of, *tmp, *d_flags, *score = nullptr;
    int64_t *cnt, *rrp;
    int4* ext;
    unsigned long long* next;
    DB_TRY(ar.work_n(nnz, &row_of));
    DB_TRY(ar.work_n(nnz, &tmp));
    DB_TRY(ar.work_n(2 * nnz, &ext));
    DB_TRY(ar.work_n(n, &cnt));
    DB_TRY(ar.work_n(2, &d_flags));
    // next: [0] fast-path task counter, [1] its cells, [2] extensions handed
    // to the general kernel, [3] the general kernel's task counter, [4] its cells
    DB_TRY(ar.work_n(6, &next));
    DB_TRY(ar.output_n(n + 1, &rrp));
    if (score_out) DB_TRY(ar.output_n(nnz, &score));
    DB_TRY(fill_i32(d_flags, 0, 2, st));
    DB_TRY(fill_i64(reinterpret_cast<int64_t*>(next), 0, 6, st));
    constexpr int WPB = 4;
    int tok = -1;
    // checks of the reads and of C
    hipLaunchKernelGGL(k_al_offsets, dim3(grid_for(std::max<int64_t>(n, 1), 256, 4096)), dim3(256), 0, st,
                       offsets, n, nbases, d_flags);
    DB_HIP(hipGetLastError());
    if (nbases > 0) {
        const int64_t head = std::min<int64_t>(nbases, (16 - (int64_t)(reinterpret_cast<uintptr_t>(bases) & 15)) & 15);
        const int64_t nvec = (nbases - head) / 16;
        hipLaunchKernelGGL(k_al_bases, dim3(grid_for(std::max<int64_t>(nvec, 1), 256, 8192)), dim3(256), 0, st, bases,
                           head, nvec, nbases, d_flags);
        DB_HIP(hipGetLastError());
    }
    // (the checks of C read the offsets only within their n + 1 entries, so
    // they run before the offsets are known to be valid)
    if (n > 0) {
        hipLaunchKernelGGL(k_al_rows<WPB>, dim3(grid_for(n, WPB, 1 << 16)), dim3(WPB * kWave), 0, st, n, n, nnz,
                           C->rowptr, C->col, C->seed, offsets, k, row_of, d_flags + 1);
        DB_HIP(hipGetLastError());
    }
    HostStage& hst = host_stage();
    DB_TRY(hst.reserve(64));
    int32_t* h = static_cast<int32_t*>(hst.ptr);
    DB_HIP(hipMemcpyAsync(h, d_flags, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    DB_TRY(sync_stream(st));
    if (h[0] || h[1]) {   // the reads' problems first: they make C's seed checks meaningless
        set_error(std::string("dibella_r_from_alignment: ") + describe_al_bad(h[0] ? h[0] : h[1]));
        return DIBELLA_EINVAL;
    }
    // the extensions: the fast path over every task, then the general kernel
    // over those it handed on (or, with a group width asked for, the general
    // kernel over every task)
    const int64_t ntasks = 2 * nnz;
    if (ntasks > 0) {
        const int FG = (flags & DIBELLA_ALIGN_GROUP_MASK) ? 0 : al_band_group(mat, gap, X);
        const int G = FG ? 64 : al_group(mat, gap, X, flags);
        int64_t* fb = nullptr;
        const int64_t* list = nullptr;
        const unsigned long long* list_count = nullptr;
        DB_TRY(timing_begin(kPhAlign, st, &tok));
        if (FG) {
            DB_TRY(ar.work_n(ntasks, &fb));
            const int grid = al_band_grid(ntasks, FG == 32 ? 16 : FG);
            if (FG == 16)
                hipLaunchKernelGGL((k_al_band<16, 1>), dim3(grid), dim3(kWave), 0, st, ntasks, row_of, C->col,
                                   C->seed, bases, offsets, k, mat, mis, gap, X, next, ext, fb, next + 2);
            else if (FG == 32)
                hipLaunchKernelGGL((k_al_band<16, 2>), dim3(grid), dim3(kWave), 0, st, ntasks, row_of, C->col,
                                   C->seed, bases, offsets, k, mat, mis, gap, X, next, ext, fb, next + 2);
            else
                hipLaunchKernelGGL((k_al_band<64, 1>), dim3(grid), dim3(kWave), 0, st, ntasks, row_of, C->col,
                                   C->seed, bases, offsets, k, mat, mis, gap, X, next, ext, fb, next + 2);
            DB_HIP(hipGetLastError());
            list = fb;
            list_count = next + 2;
        }
        // with a list, its length is on the device: a grid of a few waves per
        // CU drains it (waves with nothing to take leave at once)
        const int grid = FG ? std::min(al_grid(ntasks, G), al_cus() * 4) : al_grid(ntasks, G);
        if (G == 16)
            hipLaunchKernelGGL(k_al_extend<16>, dim3(grid), dim3(kWave), 0, st, ntasks, list, list_count, row_of,
                               C->col, C->seed, bases, offsets, k, mat, mis, gap, X, next + 3, ext);
        else if (G == 32)
            hipLaunchKernelGGL(k_al_extend<32>, dim3(grid), dim3(kWave), 0, st, ntasks, list, list_count, row_of,
                               C->col, C->seed, bases, offsets, k, mat, mis, gap, X, next + 3, ext);
        else
            hipLaunchKernelGGL(k_al_extend<64>, dim3(grid), dim3(kWave), 0, st, ntasks, list, list_count, row_of,
                               C->col, C->seed, bases, offsets, k, mat, mis, gap, X, next + 3, ext);
        DB_HIP(hipGetLastError());
        DB_TRY(timing_end(tok, st));
    }
    if (n > 0) {
        hipLaunchKernelGGL(k_al_values<WPB>, dim3(grid_for(n, WPB, 1 << 16)), dim3(WPB * kWave), 0, st, n,
                           C->rowptr, C->col, C->seed, offsets, ext, k, mat, min_score, tmp, score, cnt);
        DB_HIP(hipGetLastError());
    }
    DB_TRY(scan_exclusive(cnt, rrp, n, nullptr, ar));
    int64_t* h64 = reinterpret_cast<int64_t*>(h + 2);
    DB_HIP(hipMemcpyAsync(h64, rrp + n, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    DB_HIP(hipMemcpyAsync(h64 + 1, next, 5 * sizeof(int64_t), hipMemcpyDeviceToHost, st));
    DB_TRY(sync_stream(st));
    const int64_t rnnz = h64[0];
    stats().cells = h64[2] + h64[5];
    int32_t *rcol, *rval;
    DB_TRY(ar.output_n(rnnz, &rcol));
    DB_TRY(ar.output_n(rnnz, &rval));
    if (n > 0 && rnnz > 0) DB_TRY(write_marked_rows(n, C->rowptr, C->col, tmp, rrp, rcol, rval, st));
    DB_TRY(stage_done(st));
    R->nnz = rnnz;
    R->rowptr = rrp;
    R->col = rcol;
    R->val = rval;
    if (score_out) *score_out = score;
    return DIBELLA_OK;
}

}  // namespace dibella
