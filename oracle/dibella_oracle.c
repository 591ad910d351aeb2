/*
 * Plain CPU oracle for the two semiring sparse products of diBELLA 2D.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct
 * reference that the tests, the smoke check and the CPU-baseline leg of the
 * benchmark compare against.  It shares no code, header or table with the
 * HIP library, and the library never calls it.
 *
 * Everything is integer arithmetic.  Matrices are CSR with int64 row
 * pointers and int32 column indices and values (the layouts the generator
 * documents).  Output arrays are malloc'd here and released with
 * oracle_free().
 *
 * Overlap (Sec. IV-D): C = A * A^T where A_ik is the position of k-mer k in
 * read i.  The semiring's multiply pairs up the two positions of a shared
 * k-mer; its add counts shared k-mers and appends another position pair while
 * fewer than two are stored.  Appending is done in increasing k-mer order, so
 * the kept pairs are those of the two smallest shared k-mer columns (the
 * order the paper leaves to the library is fixed this way).
 *
 * Transitive reduction (Sec. IV-E, Algorithm "TransitiveReduction" and the
 * MinPlus semiring): repeat { N = R^2 over MinPlus with the walk check;
 * v = row max of R; v += x; M = R with row i's entries replaced by v_i;
 * I = (M >= N) with the end-orientation check; R = R minus I } until nnz(R)
 * stops changing.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_VARIANT_B 0x1u  /* N only over paths whose end code matches R_ij */
#define ORACLE_RULE_EDGE 0x2u  /* M_ij = overhang(R_ij) + x instead of row max + x */

void oracle_free(void* p) { free(p); }

static void* xmalloc(size_t bytes) { return malloc(bytes ? bytes : 1); }

/* ------------------------------------------------------------------------ */
/* A^T by a stable bucket pass over the rows of A (Algorithm diBELLA 2D,     */
/* Transpose): row k of A^T lists (read j, position) in increasing j.        */
/* ------------------------------------------------------------------------ */
static void transpose(int64_t n, int64_t m, const int64_t* rowptr, const int32_t* col,
                      const int32_t* val, int64_t* t_rowptr, int32_t* t_read, int32_t* t_pos) {
    int64_t* fill = (int64_t*)xmalloc(sizeof(int64_t) * (size_t)(m + 1));
    memset(t_rowptr, 0, sizeof(int64_t) * (size_t)(m + 1));
    for (int64_t e = 0; e < rowptr[n]; ++e) t_rowptr[col[e] + 1]++;
    for (int64_t k = 0; k < m; ++k) t_rowptr[k + 1] += t_rowptr[k];
    memcpy(fill, t_rowptr, sizeof(int64_t) * (size_t)(m + 1));
    for (int64_t i = 0; i < n; ++i)
        for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
            int64_t d = fill[col[e]]++;
            t_read[d] = (int32_t)i;
            t_pos[d] = val[e];
        }
    free(fill);
}

static int cmp_i32(const void* a, const void* b) {
    int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
    return (x > y) - (x < y);
}

/* A^T into caller arrays t_rowptr[m+1], t_read[nnz], t_pos[nnz], so that
 * several row ranges (threads) can share one transpose. */
int oracle_transpose(int64_t n, int64_t m, const int64_t* rowptr, const int32_t* col,
                     const int32_t* val, int64_t* t_rowptr, int32_t* t_read, int32_t* t_pos) {
    transpose(n, m, rowptr, col, val, t_rowptr, t_read, t_pos);
    return 0;
}

/* Rows `sel[0..nsel)` of C = A A^T (nsel < 0: all rows, in order), given
 * A^T (as built by oracle_transpose; it is only read).
 * Per row: walk k in A_i in increasing order, and for every (j, p_j) in row k
 * of A^T, add 1 to the count of C_ij and append (A_ik, p_j) while fewer than
 * two pairs are stored.  Keep entries with count >= min_shared, sorted by j.
 * Outputs: out_rowptr[nrows_out+1], *out_col, *out_count, *out_seed (4 per
 * entry: p_i0, p_j0, p_i1, p_j1, -1 where absent). */
int oracle_overlap_rows_t(int64_t n, int64_t m, const int64_t* rowptr, const int32_t* col,
                          const int32_t* val, const int64_t* t_rowptr, const int32_t* t_read,
                          const int32_t* t_pos, int32_t min_shared, const int64_t* sel, int64_t nsel,
                          int64_t* out_rowptr, int32_t** out_col, int32_t** out_count,
                          int32_t** out_seed, int64_t* out_nnz) {
    (void)m;
    int32_t* count = (int32_t*)calloc((size_t)(n ? n : 1), sizeof(int32_t));
    int32_t* seeds = (int32_t*)xmalloc(sizeof(int32_t) * 4 * (size_t)(n ? n : 1));
    int32_t* touched = (int32_t*)xmalloc(sizeof(int32_t) * (size_t)(n ? n : 1));
    int64_t nrows_out = nsel < 0 ? n : nsel;
    int64_t cap = 1024, nnz = 0;
    int32_t* oc = (int32_t*)xmalloc(sizeof(int32_t) * (size_t)cap);
    int32_t* on = (int32_t*)xmalloc(sizeof(int32_t) * (size_t)cap);
    int32_t* os = (int32_t*)xmalloc(sizeof(int32_t) * 4 * (size_t)cap);
    out_rowptr[0] = 0;
    for (int64_t r = 0; r < nrows_out; ++r) {
        int64_t i = nsel < 0 ? r : sel[r];
        int64_t nt = 0;
        for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
            int32_t k = col[e];
            for (int64_t f = t_rowptr[k]; f < t_rowptr[k + 1]; ++f) {
                int32_t j = t_read[f];
                if (count[j] == 0) {
                    touched[nt++] = j;
                    seeds[4 * j + 0] = seeds[4 * j + 1] = seeds[4 * j + 2] = seeds[4 * j + 3] = -1;
                }
                int32_t c = count[j]++;
                if (c < 2) {                  /* concatenate while fewer than two */
                    seeds[4 * j + 2 * c + 0] = val[e];
                    seeds[4 * j + 2 * c + 1] = t_pos[f];
                }
            }
        }
        qsort(touched, (size_t)nt, sizeof(int32_t), cmp_i32);
        for (int64_t q = 0; q < nt; ++q) {
            int32_t j = touched[q];
            if (count[j] >= min_shared) {
                if (nnz == cap) {
                    cap *= 2;
                    oc = (int32_t*)realloc(oc, sizeof(int32_t) * (size_t)cap);
                    on = (int32_t*)realloc(on, sizeof(int32_t) * (size_t)cap);
                    os = (int32_t*)realloc(os, sizeof(int32_t) * 4 * (size_t)cap);
                }
                oc[nnz] = j;
                on[nnz] = count[j];
                memcpy(os + 4 * nnz, seeds + 4 * j, 4 * sizeof(int32_t));
                nnz++;
            }
            count[j] = 0;
        }
        out_rowptr[r + 1] = nnz;
    }
    free(count); free(seeds); free(touched);
    *out_col = oc; *out_count = on; *out_seed = os; *out_nnz = nnz;
    return 0;
}

/* The same, building A^T first (one call, one transpose). */
int oracle_overlap_rows(int64_t n, int64_t m, const int64_t* rowptr, const int32_t* col,
                        const int32_t* val, int32_t min_shared, const int64_t* sel, int64_t nsel,
                        int64_t* out_rowptr, int32_t** out_col, int32_t** out_count,
                        int32_t** out_seed, int64_t* out_nnz) {
    int64_t nnz_a = rowptr[n];
    int64_t* t_rowptr = (int64_t*)xmalloc(sizeof(int64_t) * (size_t)(m + 1));
    int32_t* t_read = (int32_t*)xmalloc(sizeof(int32_t) * (size_t)nnz_a);
    int32_t* t_pos = (int32_t*)xmalloc(sizeof(int32_t) * (size_t)nnz_a);
    transpose(n, m, rowptr, col, val, t_rowptr, t_read, t_pos);
    int r = oracle_overlap_rows_t(n, m, rowptr, col, val, t_rowptr, t_read, t_pos, min_shared, sel,
                                  nsel, out_rowptr, out_col, out_count, out_seed, out_nnz);
    free(t_rowptr); free(t_read); free(t_pos);
    return r;
}

int oracle_overlap(int64_t n, int64_t m, const int64_t* rowptr, const int32_t* col,
                   const int32_t* val, int32_t min_shared, int64_t* out_rowptr,
                   int32_t** out_col, int32_t** out_count, int32_t** out_seed, int64_t* out_nnz) {
    return oracle_overlap_rows(n, m, rowptr, col, val, min_shared, NULL, -1, out_rowptr,
                               out_col, out_count, out_seed, out_nnz);
}

/* ------------------------------------------------------------------------ */
/* Transitive reduction                                                      */
/* ------------------------------------------------------------------------ */
/* R value: (overhang << 2) | (o_src << 1) | o_dst.                          */
static int32_t oh_of(int32_t v) { return v >> 2; }
static int32_t src_of(int32_t v) { return (v >> 1) & 1; }
static int32_t dst_of(int32_t v) { return v & 1; }
static int32_t code_of(int32_t v) { return v & 3; }

#define INF_KEY 0xFFFFFFFFu

/* MinPlus semiring of the reduction.  An N value is the pair (sum of
 * overhangs, end code) packed as (sum << 2) | code, so that Add = min picks
 * the shortest suffix (ties broken by the code).  Multiply returns a+b only
 * if the walk i -> k -> j is valid, i.e. both heads at k point opposite ways:
 * k is left by the orientation it was entered with (dst(R_ik) == src(R_kj)).
 * The end code of the walk is (src(R_ik), dst(R_kj)). */
static uint32_t minplus_multiply(int32_t r_ik, int32_t r_kj) {
    if (dst_of(r_ik) != src_of(r_kj)) return INF_KEY;          /* Id() */
    uint32_t sum = (uint32_t)(oh_of(r_ik) + oh_of(r_kj));
    return (sum << 2) | (uint32_t)(src_of(r_ik) << 1) | (uint32_t)dst_of(r_kj);
}
static uint32_t minplus_add(uint32_t a, uint32_t b) { return a < b ? a : b; }

/* N = R^2 (one CSR, rows sorted).  Under variant B only entries on the
 * pattern of R whose end code equals that of R_ij are accumulated. */
static void square(int64_t n, const int64_t* rp, const int32_t* ci, const int32_t* va,
                   uint32_t flags, int64_t** n_rp, int32_t** n_ci, uint32_t** n_va,
                   int64_t* walks) {
    uint32_t* acc = (uint32_t*)xmalloc(sizeof(uint32_t) * (size_t)(n ? n : 1));
    int32_t* rcode = (int32_t*)xmalloc(sizeof(int32_t) * (size_t)(n ? n : 1));
    int32_t* touched = (int32_t*)xmalloc(sizeof(int32_t) * (size_t)(n ? n : 1));
    for (int64_t j = 0; j < n; ++j) { acc[j] = INF_KEY; rcode[j] = -1; }
    int64_t cap = 1024, nnz = 0;
    int64_t* orp = (int64_t*)xmalloc(sizeof(int64_t) * (size_t)(n + 1));
    int32_t* oci = (int32_t*)xmalloc(sizeof(int32_t) * (size_t)cap);
    uint32_t* ova = (uint32_t*)xmalloc(sizeof(uint32_t) * (size_t)cap);
    orp[0] = 0;
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t e = rp[i]; e < rp[i + 1]; ++e) rcode[ci[e]] = code_of(va[e]);
        int64_t nt = 0;
        for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
            int32_t k = ci[e];
            *walks += rp[k + 1] - rp[k];
            for (int64_t f = rp[k]; f < rp[k + 1]; ++f) {
                int32_t j = ci[f];
                uint32_t key = minplus_multiply(va[e], va[f]);
                if (key == INF_KEY) continue;
                if ((flags & ORACLE_VARIANT_B) && (rcode[j] < 0 || (int32_t)(key & 3u) != rcode[j]))
                    continue;
                if (acc[j] == INF_KEY) touched[nt++] = j;
                acc[j] = minplus_add(acc[j], key);
            }
        }
        qsort(touched, (size_t)nt, sizeof(int32_t), cmp_i32);
        for (int64_t q = 0; q < nt; ++q) {
            if (nnz == cap) {
                cap *= 2;
                oci = (int32_t*)realloc(oci, sizeof(int32_t) * (size_t)cap);
                ova = (uint32_t*)realloc(ova, sizeof(uint32_t) * (size_t)cap);
            }
            oci[nnz] = touched[q];
            ova[nnz] = acc[touched[q]];
            nnz++;
            acc[touched[q]] = INF_KEY;
        }
        for (int64_t e = rp[i]; e < rp[i + 1]; ++e) rcode[ci[e]] = -1;
        orp[i + 1] = nnz;
    }
    free(acc); free(rcode); free(touched);
    *n_rp = orp; *n_ci = oci; *n_va = ova;
}

/* Value of sparse N at (i, j) or INF_KEY (binary search in the sorted row). */
static uint32_t lookup(const int64_t* rp, const int32_t* ci, const uint32_t* va, int64_t i, int32_t j) {
    int64_t lo = rp[i], hi = rp[i + 1];
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (ci[mid] < j) lo = mid + 1; else hi = mid;
    }
    return (lo < rp[i + 1] && ci[lo] == j) ? va[lo] : INF_KEY;
}

/* S = TransitiveReduction(R, x).  Entries with overhang <= 0 are contained
 * overlaps and are dropped first.  `iterations` counts executed passes,
 * including the final pass that deletes nothing.  nnz_trace (if non-NULL,
 * room for max_trace values) receives nnz(R) after the drop and after every
 * pass; *walks counts the walks i -> k -> j enumerated by all squarings. */
int oracle_transitive_reduce(int64_t n, const int64_t* rowptr, const int32_t* col,
                             const int32_t* val, int32_t fuzz, uint32_t flags,
                             int64_t* out_rowptr, int32_t** out_col, int32_t** out_val,
                             int64_t* out_nnz, int32_t* iterations, int64_t* nnz_trace,
                             int32_t max_trace, int64_t* walks) {
    int64_t nnz = 0;
    *walks = 0;
    int64_t* rp = (int64_t*)xmalloc(sizeof(int64_t) * (size_t)(n + 1));
    int32_t* ci = (int32_t*)xmalloc(sizeof(int32_t) * (size_t)(rowptr[n] ? rowptr[n] : 1));
    int32_t* va = (int32_t*)xmalloc(sizeof(int32_t) * (size_t)(rowptr[n] ? rowptr[n] : 1));
    rp[0] = 0;
    for (int64_t i = 0; i < n; ++i) {           /* contained overlaps are discarded */
        for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e)
            if (oh_of(val[e]) > 0) { ci[nnz] = col[e]; va[nnz] = val[e]; nnz++; }
        rp[i + 1] = nnz;
    }
    int32_t ntrace = 0;
    if (nnz_trace && ntrace < max_trace) nnz_trace[ntrace++] = nnz;
    int32_t* v = (int32_t*)xmalloc(sizeof(int32_t) * (size_t)(n ? n : 1));
    int32_t iter = 0;
    int64_t prev;
    do {
        prev = nnz;
        iter++;
        int64_t* n_rp; int32_t* n_ci; uint32_t* n_va;
        square(n, rp, ci, va, flags, &n_rp, &n_ci, &n_va, walks);  /* N = R^2 */
        for (int64_t i = 0; i < n; ++i) {                         /* v = Reduce(Row, 0, max) */
            v[i] = 0;
            for (int64_t e = rp[i]; e < rp[i + 1]; ++e)
                if (oh_of(va[e]) > v[i]) v[i] = oh_of(va[e]);
        }
        for (int64_t i = 0; i < n; ++i)                           /* v = Apply(v, +x) on nonzeros */
            if (v[i] != 0) v[i] += fuzz;
        int64_t w = 0;
        int64_t row_start = 0;
        for (int64_t i = 0; i < n; ++i) {
            for (int64_t e = row_start; e < rp[i + 1]; ++e) {
                /* M = DimApply(R, v): row i of R takes v_i (or R_ij + x under the edge rule) */
                int64_t mij = (flags & ORACLE_RULE_EDGE) ? (int64_t)oh_of(va[e]) + fuzz : (int64_t)v[i];
                uint32_t nij = lookup(n_rp, n_ci, n_va, i, ci[e]);
                /* I = M >= N, on entries present in both, with matching end heads */
                int transitive = nij != INF_KEY && (int32_t)(nij & 3u) == code_of(va[e]) &&
                                 (int64_t)(nij >> 2) <= mij;
                if (!transitive) { ci[w] = ci[e]; va[w] = va[e]; w++; }   /* R = R .* !I */
            }
            row_start = rp[i + 1];
            rp[i + 1] = w;
        }
        nnz = w;
        free(n_rp); free(n_ci); free(n_va);
        if (nnz_trace && ntrace < max_trace) nnz_trace[ntrace++] = nnz;
    } while (nnz != prev);
    free(v);
    memcpy(out_rowptr, rp, sizeof(int64_t) * (size_t)(n + 1));
    free(rp);
    *out_col = ci; *out_val = va; *out_nnz = nnz; *iterations = iter;
    return 0;
}

/* One pass of the reduction on R as given (no contained-overlap drop):
 * writes mark[e] = 1 for every entry found transitive.  Rows other than
 * those in sel[0..nsel) are not examined (nsel < 0: all rows).  Used to
 * check sampled rows of large inputs. */
int oracle_tr_pass_marks(int64_t n, const int64_t* rowptr, const int32_t* col,
                         const int32_t* val, int32_t fuzz, uint32_t flags,
                         const int64_t* sel, int64_t nsel, uint8_t* mark) {
    uint32_t* acc = (uint32_t*)xmalloc(sizeof(uint32_t) * (size_t)(n ? n : 1));
    int32_t* rcode = (int32_t*)xmalloc(sizeof(int32_t) * (size_t)(n ? n : 1));
    for (int64_t j = 0; j < n; ++j) { acc[j] = INF_KEY; rcode[j] = -1; }
    int64_t rows = nsel < 0 ? n : nsel;
    for (int64_t r = 0; r < rows; ++r) {
        int64_t i = nsel < 0 ? r : sel[r];
        for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) rcode[col[e]] = code_of(val[e]);
        for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {   /* row i of N = R^2 */
            int32_t k = col[e];
            for (int64_t f = rowptr[k]; f < rowptr[k + 1]; ++f) {
                int32_t j = col[f];
                uint32_t key = minplus_multiply(val[e], val[f]);
                if (key == INF_KEY) continue;
                if ((flags & ORACLE_VARIANT_B) && (rcode[j] < 0 || (int32_t)(key & 3u) != rcode[j]))
                    continue;
                acc[j] = minplus_add(acc[j], key);
            }
        }
        int32_t vi = 0;
        for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e)
            if (oh_of(val[e]) > vi) vi = oh_of(val[e]);
        if (vi != 0) vi += fuzz;
        for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
            int64_t mij = (flags & ORACLE_RULE_EDGE) ? (int64_t)oh_of(val[e]) + fuzz : (int64_t)vi;
            uint32_t nij = acc[col[e]];
            mark[e] = (uint8_t)(nij != INF_KEY && (int32_t)(nij & 3u) == code_of(val[e]) &&
                                (int64_t)(nij >> 2) <= mij);
        }
        for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
            int32_t k = col[e];
            for (int64_t f = rowptr[k]; f < rowptr[k + 1]; ++f) acc[col[f]] = INF_KEY;
            rcode[col[e]] = -1;
        }
    }
    free(acc); free(rcode);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Overlap graph R from the seeds stored in C (Sec. IV-D, IV-E)             */
/* ------------------------------------------------------------------------ */
/* The reduction needs, per read pair, the overlap suffix and the overlap
 * orientation, derived in place from the alignment coordinates stored with
 * the pair.  Here the coordinates are the first stored seed of C_ij, with no
 * alignment in between: each seed value is (position << 1) | strand, where
 * strand says whether the read holds the shared canonical k-mer as is (0) or
 * as its reverse complement (1).  The two reads are reverse-complementary
 * iff the strands differ.  Extending the seed without gaps to both read ends
 * places read j (reverse complemented if the pair is) in the frame of read
 * i at offset d: d = p_i - p_j, or d = p_i + p_j + k - L_j for a
 * reverse-complementary pair.  The alignment then starts at s_i = max(0, d)
 * in i and s_j = max(0, -d) in j, and the overlap has length
 * min(L_i, d + L_j) - max(0, d).  With max_drift >= 0 a pair is kept only
 * if C holds its second seed too, placing the pair in the same relative
 * orientation at an offset within max_drift bases of the first (two
 * independent k-mers agree on the overlap; an unrelated second hit does
 * not).  With min_density > 0 a pair is kept only if it shares at least
 * min_density k-mers per 10 kbp of its overlap (count * 10000 >=
 * min_density * overlap): a true overlap shares k-mers all along its
 * length at a rate the error rate fixes, a pair that only shares a repeat
 * does so along the repeat alone.  Both tests stand in for the alignment
 * that prunes C into R.  Pairs whose overlap is shorter than min_overlap
 * are not kept.  A contained overlap (the overlap is all of one
 * read) is kept with value 0 (the reduction discards it).  Otherwise the
 * four categories of overlap give the pair's code and suffix:
 *   not reverse complement, s_i > s_j: forward  -> code (0,0), suffix of j past i
 *   not reverse complement, s_i < s_j: reverse  -> code (1,1), suffix of j before i
 *   reverse complement,     s_i > s_j: inner    -> code (0,1), suffix of j past i
 *   reverse complement,     s_i < s_j: outer    -> code (1,0), suffix of j before i
 * (s_i > s_j: read i comes first in its own frame, so the walk i -> j keeps
 * i as sequenced and continues with j in the pair's relative orientation;
 * otherwise the walk i -> j runs the other way and takes both reads
 * reverse complemented.)  The diagonal of C is not part of R.
 * Output: R as CSR with val = (suffix << 2) | code, rows sorted.  Returns 0,
 * or -1 if a seed of an off-diagonal entry is missing or outside its read. */
/* Offset of read j in read i's frame from one seed (a, b), and whether the
 * pair is reverse-complementary. */
static int64_t seed_offset(int32_t a, int32_t b, int64_t lj, int32_t k, int* rc) {
    int64_t pi = a >> 1, pj = b >> 1;
    *rc = (a & 1) != (b & 1);
    return *rc ? pi + pj + k - lj : pi - pj;
}

int oracle_r_from_seeds(int64_t n, const int64_t* c_rowptr, const int32_t* c_col,
                        const int32_t* c_count, const int32_t* c_seed, const int32_t* read_len,
                        int32_t k, int32_t min_overlap, int32_t max_drift, int32_t min_density,
                        int64_t* out_rowptr, int32_t** out_col, int32_t** out_val,
                        int64_t* out_nnz) {
    int64_t cap = c_rowptr[n] ? c_rowptr[n] : 1, nnz = 0;
    int32_t* oc = (int32_t*)xmalloc(sizeof(int32_t) * (size_t)cap);
    int32_t* ov = (int32_t*)xmalloc(sizeof(int32_t) * (size_t)cap);
    out_rowptr[0] = 0;
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t e = c_rowptr[i]; e < c_rowptr[i + 1]; ++e) {
            int64_t j = c_col[e];
            if (j == i) continue;
            int32_t a = c_seed[4 * e + 0], b = c_seed[4 * e + 1];
            int64_t li = read_len[i], lj = read_len[j];
            if (a < 0 || b < 0) { free(oc); free(ov); return -1; }
            int64_t pi = a >> 1, pj = b >> 1;
            if (pi + k > li || pj + k > lj) { free(oc); free(ov); return -1; }
            int rc;
            int64_t d = seed_offset(a, b, lj, k, &rc);
            if (max_drift >= 0) {                            /* the second seed must agree */
                int32_t a1 = c_seed[4 * e + 2], b1 = c_seed[4 * e + 3];
                if (a1 < 0 || b1 < 0) continue;
                if ((a1 >> 1) + k > li || (b1 >> 1) + k > lj) { free(oc); free(ov); return -1; }
                int rc1;
                int64_t d1 = seed_offset(a1, b1, lj, k, &rc1);
                if (rc1 != rc || d1 - d > max_drift || d - d1 > max_drift) continue;
            }
            int64_t lo = d > 0 ? d : 0, hi = d + lj < li ? d + lj : li;
            int64_t overlap = hi - lo;
            if (overlap < min_overlap) continue;
            if (min_density > 0 && (int64_t)c_count[e] * 10000 < (int64_t)min_density * overlap) continue;
            int32_t value;
            if (overlap == li || overlap == lj) {
                value = 0;                                   /* contained overlap */
            } else {
                int64_t si = d > 0 ? d : 0, sj = d < 0 ? -d : 0;
                int64_t suffix;
                int32_t code;
                if (si > sj) {                               /* forward or inner */
                    suffix = d + lj - li;
                    code = rc ? 1 : 0;                       /* (0,0) or (0,1) */
                } else {                                     /* reverse or outer */
                    suffix = -d;
                    code = rc ? 2 : 3;                       /* (1,0) or (1,1) */
                }
                value = (int32_t)((suffix << 2) | code);
            }
            oc[nnz] = (int32_t)j;
            ov[nnz] = value;
            nnz++;
        }
        out_rowptr[i + 1] = nnz;
    }
    *out_col = oc; *out_val = ov; *out_nnz = nnz;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* A from the reads: k-mer counting, reliable k-mers, A (Sec. IV-C, Alg.     */
/* diBELLA 2D: KmerCounter and GenerateA)                                    */
/* ------------------------------------------------------------------------ */
/* Every window of k bases (p + k <= L_i) of every read is a k-mer.  Bases
 * are 2-bit codes A0 C1 G2 T3, the first base the most significant.  Its
 * canonical form is the smaller of its code and its reverse complement's
 * (the complement of each base, in reverse order); its strand is 1 when the
 * reverse complement is the smaller (the read holds the canonical k-mer
 * reverse complemented), else 0.  The frequency of a canonical k-mer is the
 * number of windows of all reads that have it (repeats inside a read
 * count); it is reliable when lo <= frequency <= hi.  The reliable k-mers
 * are A's columns in the order of their first occurrence in the reads: by
 * the first read holding the k-mer, then by the k-mer's smallest position
 * in that read (the paper fixes no column order; this one makes the k-mers
 * one read holds consecutive columns).  A_ic = the smallest position of
 * k-mer c in read i, or (position << 1) | strand (the strand at that
 * position) when strand_bit is set.
 * Outputs: rowptr[n+1], *out_col, *out_val (nnz each), *out_codes (m
 * reliable codes, codes[c] the k-mer of column c), *out_m, *out_nnz.
 * Returns 0, -1 for k outside [1, 31], lo < 1, hi < lo or a base outside
 * 0..3. */
typedef struct {
    uint64_t code;
    int64_t read;
    int64_t pos;
    int32_t strand;
} oracle_window;

static int cmp_window(const void* a, const void* b) {
    const oracle_window* x = (const oracle_window*)a;
    const oracle_window* y = (const oracle_window*)b;
    if (x->code != y->code) return x->code < y->code ? -1 : 1;
    if (x->read != y->read) return x->read < y->read ? -1 : 1;
    return (x->pos > y->pos) - (x->pos < y->pos);
}

typedef struct {
    int64_t read;
    int64_t col;
    int32_t val;
} oracle_entry;

/* a reliable k-mer: its windows win[a, b) (sorted), first occurrence first */
typedef struct {
    int64_t a, b;
} oracle_run;

static const oracle_window* g_runs_win;   /* the windows the runs index (qsort has no context) */

static int cmp_run_first(const void* x, const void* y) {
    const oracle_window* p = &g_runs_win[((const oracle_run*)x)->a];
    const oracle_window* q = &g_runs_win[((const oracle_run*)y)->a];
    if (p->read != q->read) return p->read < q->read ? -1 : 1;
    return (p->pos > q->pos) - (p->pos < q->pos);
}

static int cmp_entry(const void* a, const void* b) {
    const oracle_entry* x = (const oracle_entry*)a;
    const oracle_entry* y = (const oracle_entry*)b;
    if (x->read != y->read) return x->read < y->read ? -1 : 1;
    return (x->col > y->col) - (x->col < y->col);
}

int oracle_kmer_matrix(int64_t n, const uint8_t* bases, const int64_t* offsets, int32_t k, int32_t lo,
                       int32_t hi, int32_t strand_bit, int64_t* out_rowptr, int32_t** out_col,
                       int32_t** out_val, uint64_t** out_codes, int64_t* out_m, int64_t* out_nnz) {
    if (k < 1 || k > 31 || lo < 1 || hi < lo) return -1;
    /* every window: its canonical code, read, position and strand */
    int64_t W = 0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t L = offsets[i + 1] - offsets[i];
        if (L >= k) W += L - k + 1;
    }
    oracle_window* win = (oracle_window*)xmalloc(sizeof(oracle_window) * (size_t)(W ? W : 1));
    int64_t w = 0;
    for (int64_t i = 0; i < n; ++i) {
        const uint8_t* s = bases + offsets[i];
        int64_t L = offsets[i + 1] - offsets[i];
        for (int64_t p = 0; p + k <= L; ++p) {
            uint64_t fwd = 0, rc = 0;
            for (int32_t q = 0; q < k; ++q) {
                if (s[p + q] > 3) { free(win); return -1; }
                fwd = (fwd << 2) | s[p + q];                          /* first base most significant */
                rc |= (uint64_t)(3 - s[p + q]) << (2 * q);            /* complement, reversed */
            }
            win[w].code = rc < fwd ? rc : fwd;
            win[w].strand = rc < fwd;
            win[w].read = i;
            win[w].pos = p;
            ++w;
        }
    }
    W = w;   /* the windows filled (equal to the count above) */
    qsort(win, (size_t)W, sizeof(oracle_window), cmp_window);
    /* frequencies (runs of equal codes) and the reliable k-mers; within a run
     * the windows are in (read, position) order, so a run's first window is
     * the k-mer's first occurrence and the first window of a read in a run
     * has the read's smallest position */
    oracle_run* runs = (oracle_run*)xmalloc(sizeof(oracle_run) * (size_t)(W ? W : 1));
    int64_t m = 0, nnz = 0;
    for (int64_t a = 0; a < W;) {
        int64_t b = a;
        while (b < W && win[b].code == win[a].code) ++b;
        int64_t freq = b - a;
        if (freq >= lo && freq <= hi) {
            runs[m].a = a;
            runs[m].b = b;
            ++m;
        }
        a = b;
    }
    /* columns: the reliable k-mers by first occurrence */
    g_runs_win = win;
    qsort(runs, (size_t)m, sizeof(oracle_run), cmp_run_first);
    g_runs_win = NULL;
    oracle_entry* ent = (oracle_entry*)xmalloc(sizeof(oracle_entry) * (size_t)(W ? W : 1));
    uint64_t* codes = (uint64_t*)xmalloc(sizeof(uint64_t) * (size_t)(m ? m : 1));
    for (int64_t c = 0; c < m; ++c) {
        codes[c] = win[runs[c].a].code;
        for (int64_t e = runs[c].a; e < runs[c].b; ++e) {
            if (e > runs[c].a && win[e].read == win[e - 1].read) continue;   /* not the read's first */
            ent[nnz].read = win[e].read;
            ent[nnz].col = c;
            ent[nnz].val = strand_bit ? (int32_t)((win[e].pos << 1) | win[e].strand) : (int32_t)win[e].pos;
            ++nnz;
        }
    }
    free(runs);
    free(win);
    qsort(ent, (size_t)nnz, sizeof(oracle_entry), cmp_entry);
    int32_t* oc = (int32_t*)xmalloc(sizeof(int32_t) * (size_t)(nnz ? nnz : 1));
    int32_t* ov = (int32_t*)xmalloc(sizeof(int32_t) * (size_t)(nnz ? nnz : 1));
    for (int64_t i = 0; i <= n; ++i) out_rowptr[i] = 0;
    for (int64_t e = 0; e < nnz; ++e) {
        out_rowptr[ent[e].read + 1]++;
        oc[e] = (int32_t)ent[e].col;
        ov[e] = ent[e].val;
    }
    for (int64_t i = 0; i < n; ++i) out_rowptr[i + 1] += out_rowptr[i];
    free(ent);
    *out_col = oc; *out_val = ov; *out_codes = codes; *out_m = m; *out_nnz = nnz;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Seed-and-extend alignment of C's read pairs and the graph R it gives     */
/* (Sec. IV-D: each nonzero of C is aligned by extending its seed, and      */
/* pruned when the score does not reach a threshold; Sec. IV-E: R's suffix   */
/* and orientation come from the alignment coordinates)                     */
/* ------------------------------------------------------------------------ */
/* X-drop extension (Zhang, Schwartz, Wagner and Miller, 2000) of a against
 * b from their starts: T(i, j) is the best score of aligning a[0, i) with
 * b[0, j) (match `mat`, mismatch `mis`, a base against a gap `gap`; T(0, 0) =
 * 0), computed anti-diagonal by anti-diagonal (d = i + j).  On anti-diagonal
 * d the cells considered are those reachable from a live cell of d - 1 (i
 * or i - 1 there) or d - 2 (i - 1 there); a cell whose score is below the
 * best score of the earlier anti-diagonals minus X is dead, as are cells
 * with no live predecessor.  The best score and the first cell (in
 * anti-diagonal order, then i order) reaching it are the result.  The
 * extension stops when two anti-diagonals in a row have no live cell, at
 * the sequences' ends, or when the cells to consider on one anti-diagonal
 * would exceed ORACLE_XD_BAND (then it keeps what it has). */
#define ORACLE_XD_BAND 256
#define ORACLE_XD_DEAD INT64_MIN

static int64_t xdrop_extend(const uint8_t* a, int64_t m, const uint8_t* b, int64_t n, int32_t mat, int32_t mis,
                            int32_t gap, int32_t X, int64_t* ea, int64_t* eb) {
    int64_t* dg[3];   /* anti-diagonals d - 2, d - 1, d, indexed by i */
    for (int t = 0; t < 3; ++t) {
        dg[t] = (int64_t*)xmalloc(sizeof(int64_t) * (size_t)(m + 1));
        for (int64_t i = 0; i <= m; ++i) dg[t][i] = ORACLE_XD_DEAD;
    }
    int64_t lo[3], hi[3];   /* live range of each kept anti-diagonal (lo > hi: none) */
    int64_t best = 0;
    *ea = 0; *eb = 0;
    /* d = 0: the cell (0, 0) */
    dg[2][0] = 0; lo[2] = 0; hi[2] = 0;
    lo[1] = 1; hi[1] = 0;   /* d = -1: none */
    lo[0] = 1; hi[0] = 0;   /* d = -2: none */
    for (int64_t d = 1; d <= m + n; ++d) {
        /* shift: d - 1 becomes d - 2, d becomes d - 1 */
        int64_t* old = dg[0];
        for (int64_t i = (lo[0] <= hi[0] ? lo[0] : 1); i <= hi[0]; ++i) old[i] = ORACLE_XD_DEAD;
        dg[0] = dg[1]; lo[0] = lo[1]; hi[0] = hi[1];
        dg[1] = dg[2]; lo[1] = lo[2]; hi[1] = hi[2];
        dg[2] = old;
        if (lo[0] > hi[0] && lo[1] > hi[1]) { lo[2] = 1; hi[2] = 0; break; }   /* two dead anti-diagonals */
        int64_t from = INT64_MAX, to = INT64_MIN;
        if (lo[1] <= hi[1]) { from = lo[1]; to = hi[1] + 1; }
        if (lo[0] <= hi[0]) { if (lo[0] + 1 < from) from = lo[0] + 1; if (hi[0] + 1 > to) to = hi[0] + 1; }
        if (from < d - n) from = d - n;
        if (from < 0) from = 0;
        if (to > m) to = m;
        if (to > d) to = d;
        lo[2] = 1; hi[2] = 0;
        if (from > to) continue;
        if (to - from + 1 > ORACLE_XD_BAND) break;
        int64_t dbest = ORACLE_XD_DEAD, di = -1;
        for (int64_t i = from; i <= to; ++i) {
            int64_t j = d - i, v = ORACLE_XD_DEAD;
            if (i >= 1 && j >= 1 && dg[0][i - 1] != ORACLE_XD_DEAD)
                v = dg[0][i - 1] + (a[i - 1] == b[j - 1] ? mat : mis);
            if (i >= 1 && dg[1][i - 1] != ORACLE_XD_DEAD && dg[1][i - 1] + gap > v) v = dg[1][i - 1] + gap;
            if (j >= 1 && dg[1][i] != ORACLE_XD_DEAD && dg[1][i] + gap > v) v = dg[1][i] + gap;
            if (v != ORACLE_XD_DEAD && v < best - X) v = ORACLE_XD_DEAD;   /* x-drop */
            dg[2][i] = v;
            if (v != ORACLE_XD_DEAD) {
                if (lo[2] > hi[2]) lo[2] = i;
                hi[2] = i;
                if (v > dbest) { dbest = v; di = i; }
            }
        }
        if (dbest != ORACLE_XD_DEAD && dbest > best) { best = dbest; *ea = di; *eb = d - di; }
    }
    for (int t = 0; t < 3; ++t) free(dg[t]);
    return best;
}

/* For every off-diagonal entry of C (seeds (position << 1) | strand as in
 * oracle_r_from_seeds): read j is taken as sequenced, or reverse
 * complemented when the strands differ (j'); the first seed's k-mer sits at
 * p_i in read i and at q = p_j, or L_j - k - p_j in j'.  The seed (k
 * matches) is extended to the right (i after p_i + k against j' after
 * q + k) and to the left (the reversed prefixes before p_i and q) by X-drop
 * extension; the score is the two extensions' plus k * mat, and the
 * alignment spans [bi, ei) of i and [bj, ej) of j'.  Pairs scoring below
 * min_score are pruned.  The rest give R's entry from the alignment ends:
 * one read contained in the other (its unaligned ends both within the
 * other's) -> value 0; else read i first (bi > bj): suffix (L_j - ej) -
 * (L_i - ei), code (0, rc); else suffix bj - bi, code (1, 1 - rc).
 * Outputs as oracle_r_from_seeds, plus score[nnz(C)] (the score of every
 * entry of C, 0 on the diagonal).  Returns 0, or -1 for a missing or
 * out-of-range seed, a base outside 0..3 in any read, a read length of 2^28
 * or more, or scores outside match in [1, 7], mismatch in [-1024, 0], gap in
 * [-1024, -1], X in [0, 2^20] (the ranges keep every score within 32 bits). */
static uint8_t seq_at(const uint8_t* s, int64_t L, int rc, int64_t x) {
    return rc ? (uint8_t)(3 - s[L - 1 - x]) : s[x];
}

int oracle_r_from_alignment(int64_t n, const int64_t* c_rowptr, const int32_t* c_col, const int32_t* c_seed,
                            const uint8_t* bases, const int64_t* offsets, int32_t k, int32_t mat, int32_t mis,
                            int32_t gap, int32_t X, int32_t min_score, int64_t* out_rowptr, int32_t** out_col,
                            int32_t** out_val, int32_t* out_score, int64_t* out_nnz) {
    if (k < 1 || k > 32 || mat < 1 || mat > 7 || mis < -1024 || mis > 0 || gap < -1024 || gap > -1 || X < 0 ||
        X > (1 << 20))
        return -1;
    for (int64_t r = 0; r < n; ++r) {
        if (offsets[r + 1] - offsets[r] < 0 || offsets[r + 1] - offsets[r] >= ((int64_t)1 << 28)) return -1;
        for (int64_t x = offsets[r]; x < offsets[r + 1]; ++x)
            if (bases[x] > 3) return -1;
    }
    int64_t cap = 1024, nnz = 0;
    int32_t* oc = (int32_t*)xmalloc(sizeof(int32_t) * (size_t)cap);
    int32_t* ov = (int32_t*)xmalloc(sizeof(int32_t) * (size_t)cap);
    out_rowptr[0] = 0;
    for (int64_t i = 0; i < n; ++i) {
        const uint8_t* si = bases + offsets[i];
        int64_t li = offsets[i + 1] - offsets[i];
        for (int64_t e = c_rowptr[i]; e < c_rowptr[i + 1]; ++e) {
            int32_t j = c_col[e];
            out_score[e] = 0;
            if (j == (int32_t)i) continue;
            const uint8_t* sj = bases + offsets[j];
            int64_t lj = offsets[j + 1] - offsets[j];
            int32_t a = c_seed[4 * e + 0], b = c_seed[4 * e + 1];
            if (a < 0 || b < 0 || (a >> 1) + k > li || (b >> 1) + k > lj) {
                free(oc); free(ov);
                return -1;
            }
            int rc = (a & 1) != (b & 1);
            int64_t pi = a >> 1, q = rc ? lj - k - (b >> 1) : (b >> 1);
            /* the oriented sequences of the two extensions */
            int64_t mr = li - pi - k, nr = lj - q - k, ml = pi, nl = q;
            uint8_t* ar = (uint8_t*)xmalloc((size_t)(mr + 1));
            uint8_t* br = (uint8_t*)xmalloc((size_t)(nr + 1));
            uint8_t* al = (uint8_t*)xmalloc((size_t)(ml + 1));
            uint8_t* bl = (uint8_t*)xmalloc((size_t)(nl + 1));
            for (int64_t x = 0; x < mr; ++x) ar[x] = si[pi + k + x];
            for (int64_t x = 0; x < nr; ++x) br[x] = seq_at(sj, lj, rc, q + k + x);
            for (int64_t x = 0; x < ml; ++x) al[x] = si[pi - 1 - x];
            for (int64_t x = 0; x < nl; ++x) bl[x] = seq_at(sj, lj, rc, q - 1 - x);
            int64_t ear, ebr, eal, ebl;
            int64_t sr = xdrop_extend(ar, mr, br, nr, mat, mis, gap, X, &ear, &ebr);
            int64_t sl = xdrop_extend(al, ml, bl, nl, mat, mis, gap, X, &eal, &ebl);
            free(ar); free(br); free(al); free(bl);
            int64_t score = sl + (int64_t)k * mat + sr;
            out_score[e] = (int32_t)score;
            if (score < min_score) continue;
            int64_t bi = pi - eal, ei = pi + k + ear, bj = q - ebl, ej = q + k + ebr;
            int64_t ri = li - ei, rj = lj - ej;   /* unaligned right ends */
            int32_t val;
            if ((bj >= bi && rj >= ri) || (bi >= bj && ri >= rj)) {
                val = 0;                                            /* contained */
            } else if (bi > bj) {
                val = (int32_t)(((rj - ri) << 2) | (rc ? 1 : 0));  /* i first */
            } else {
                val = (int32_t)(((bj - bi) << 2) | (rc ? 2 : 3));  /* j first */
            }
            if (nnz == cap) {
                cap *= 2;
                oc = (int32_t*)realloc(oc, sizeof(int32_t) * (size_t)cap);
                ov = (int32_t*)realloc(ov, sizeof(int32_t) * (size_t)cap);
            }
            oc[nnz] = j;
            ov[nnz] = val;
            ++nnz;
        }
        out_rowptr[i + 1] = nnz;
    }
    *out_col = oc; *out_val = ov; *out_nnz = nnz;
    return 0;
}

/* X-drop extension of a against b (for the tests). */
int64_t oracle_xdrop_extend(const uint8_t* a, int64_t m, const uint8_t* b, int64_t n, int32_t mat, int32_t mis,
                            int32_t gap, int32_t X, int64_t* ea, int64_t* eb) {
    return xdrop_extend(a, m, b, n, mat, mis, gap, X, ea, eb);
}
