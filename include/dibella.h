/*
 * dibella.h -- C ABI of the MI355X (gfx950) library for the two semiring
 * sparse products of diBELLA 2D (Guidi et al., "Parallel String Graph
 * Construction and Transitive Reduction for De Novo Genome Assembly",
 * arXiv 2010.10055).
 *
 *   dibella_overlap            C = A * A^T over the overlap semiring
 *                              (Sec. IV-D, Algorithm "diBELLA 2D": Transpose
 *                              and the candidate overlap matrix).
 *   dibella_transitive_reduce  S = transitive reduction of the overlap graph R
 *                              (Sec. IV-E, Algorithm "TransitiveReduction" and
 *                              the MinPlus semiring algorithm).
 *   *_batched                  the same for many independent sets in one
 *                              set of launches.
 *   dibella_r_from_seeds       the overlap graph R from the seeds stored in C
 *                              (Sec. IV-D, IV-E).
 *   dibella_r_from_alignment   R from a seed-and-extend alignment of every
 *                              pair of C and the pruning of low scores
 *                              (Sec. IV-D: Apply(C, Alignment()), Prune;
 *                              Sec. IV-E for R's values).
 *   dibella_overlap_graph_blocked
 *                              R from A with C formed one block of reads at a
 *                              time (Sec. VIII, future work).
 *   dibella_transitive_reduce_noalloc
 *                              the reduction for callers that cannot allocate.
 *   dibella_kmer_matrix        A from the reads: k-mer counting, reliable
 *                              k-mers, A (Sec. IV-C; Algorithm "diBELLA 2D":
 *                              KmerCounter and GenerateA).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - All matrix pointers are DEVICE pointers on the current HIP device.
 *   Inputs are borrowed and never written.
 * - CSR: rowptr int64[nrows+1] with rowptr[0] = 0 and rowptr[nrows] = nnz,
 *   col int32 strictly increasing inside a row, val int32.
 * - Every kernel and copy is enqueued on `hip_stream` (NULL = the null
 *   stream).  On return the outputs are fully described (sizes and pointers)
 *   but their contents are ready only once the stream reaches that point.
 * - Outputs and workspace are obtained through `alloc(bytes, ctx)` and
 *   released through `free(p, ctx)`.  Workspace is released before the call
 *   returns while work may still be queued, so the allocator must be stream
 *   ordered on `hip_stream` (PyTorch's caching allocator on the current
 *   stream is; so is the built-in hipMallocAsync/hipFreeAsync used when
 *   alloc == NULL).  Output buffers belong to the caller.  A zero-byte
 *   request is never made: empty outputs come back as NULL.
 * - Return value: DIBELLA_OK or a negative status.  On error no output is
 *   returned (everything allocated by the call has been released) and
 *   dibella_last_error() describes the problem.
 * - Calls on different streams from different host threads are independent.
 */
#ifndef DIBELLA_H
#define DIBELLA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DIBELLA_OK          0
#define DIBELLA_EINVAL     (-1)  /* malformed matrix or argument */
#define DIBELLA_ENOMEM     (-2)  /* the allocator returned NULL */
#define DIBELLA_EDEVICE    (-3)  /* a HIP call failed (message in last_error) */
#define DIBELLA_EOVERFLOW  (-4)  /* sizes beyond the index widths */

/* Flags of the transitive reduction. */
#define DIBELLA_TR_VARIANT_B   0x1u  /* N_ij only over walks whose end heads match R_ij */
#define DIBELLA_TR_RULE_EDGE   0x2u  /* M_ij = overhang(R_ij) + fuzz (default: row max + fuzz) */
#define DIBELLA_NO_VALIDATE    0x4u  /* skip the structural checks of the input */
#define DIBELLA_TR_USE_GRAPH   0x8u  /* run the passes as captured HIP graphs */
/* Flag of dibella_kmer_matrix. */
#define DIBELLA_KMER_STRAND    0x1u  /* values (position << 1) | strand */
/* Flags of dibella_r_from_alignment: lanes per extension of the general
 * kernel, run over every extension (0 = a register-band fast path with
 * lanes chosen from the scores and X, the general kernel redoing the
 * extensions whose band outgrows it; the results are the same). */
#define DIBELLA_ALIGN_GROUP_16   0x1u
#define DIBELLA_ALIGN_GROUP_32   0x2u
#define DIBELLA_ALIGN_GROUP_64   0x3u
#define DIBELLA_ALIGN_GROUP_MASK 0x3u
/* Bits 16..31: stop after this many passes (0 = run to the fixed point). */
#define DIBELLA_TR_MAX_PASSES(n) (((uint32_t)(n) & 0xFFFFu) << 16)

typedef struct {
    int64_t nrows, ncols, nnz;
    const int64_t* rowptr;
    const int32_t* col;
    const int32_t* val;
} dibella_csr;

/* C = A A^T: per entry the number of shared k-mers and two seed pairs
 * seed[4e..4e+3] = (pos in read i, pos in read j) for the smallest shared
 * k-mer column, then for the second smallest; -1 where absent. */
typedef struct {
    int64_t nrows, ncols, nnz;
    int64_t* rowptr;
    int32_t* col;
    int32_t* count;
    int32_t* seed;
} dibella_overlap_out;

typedef struct {
    int64_t nrows, ncols, nnz;
    int64_t* rowptr;
    int32_t* col;
    int32_t* val;
} dibella_csr_out;

typedef void* (*dibella_alloc_fn)(size_t bytes, void* ctx);
typedef void (*dibella_free_fn)(void* p, void* ctx);

/*
 * dibella_overlap -- candidate overlap matrix C = A * A^T (Sec. IV-D).
 *
 * A: reads x reliable k-mers; A_ik = start of k-mer k in read i (>= 0).
 * The multiply of the semiring pairs the two positions of a shared k-mer;
 * the add counts shared k-mers and keeps the position pairs of the two
 * smallest shared k-mer columns (the paper keeps two position pairs per
 * read pair and leaves which ones to the library; this fixes it so C_ji is
 * C_ij with each pair swapped).  Entries with count < min_shared are not stored; the diagonal
 * is kept.  C rows are sorted by column.  Output arrays: rowptr[n+1],
 * col/count[nnz], seed[4*nnz].
 * Errors: EINVAL for a malformed A (rowptr, column order or range, negative
 * value) or min_shared < 1; EOVERFLOW if nrows >= 2^24 (two-pair column
 * records hold read ids in 24 bits), if a row needs 2^31 semiring products
 * or more, or if the entries or the columns of all sets of one call add up
 * to 2^32 or more.
 * Host synchronisation: two stream syncs (three if some row needs more
 * distinct columns than one LDS table holds): the first reads the
 * validation flags, the row-cost classes and the output-column scratch
 * size, the second the exact size of C, so that neither C nor the scratch
 * is allocated at its upper bound.
 */
int dibella_overlap(const dibella_csr* A, int32_t min_shared, dibella_overlap_out* C,
                    dibella_alloc_fn alloc, dibella_free_fn free_fn, void* ctx,
                    void* hip_stream);

/*
 * dibella_transitive_reduce -- string graph S from the overlap graph R
 * (Sec. IV-E).
 *
 * R: square; R_ij = the overlap of read i followed by read j, packed as
 * (overhang << 2) | (o_i << 1) | o_j where overhang is the suffix of j past
 * the overlap and o = 0/1 says the read is walked as sequenced / reverse
 * complemented.  Entries with overhang <= 0 are contained overlaps and are
 * discarded first.  Then passes repeat until a pass deletes nothing:
 *   N_ij = min over k of (overhang_ik + overhang_kj, end code) taken only over
 *          valid walks (the heads at k are opposite: o_k of R_ik equals o_k of
 *          R_kj), computed on the pattern of R;
 *   v_i  = max overhang in row i;  M_ij = v_i + fuzz (RULE_EDGE: overhang_ij + fuzz);
 *   delete R_ij where N_ij exists, its end code equals that of R_ij and
 *   its overhang sum <= M_ij; all deletions of a pass at once.
 * *iterations = passes executed, counting the final pass that deletes
 * nothing.  S has R's layout.
 * Errors: EINVAL for a malformed or non-square R, a diagonal entry, an
 * overhang >= 2^28, or fuzz outside [0, 2^30).
 * Host synchronisation: one stream sync per two passes (per captured graph
 * of passes with DIBELLA_TR_USE_GRAPH); the first also reads the validity
 * of R, and a malformed R runs no pass.  A reduction that converges in two
 * passes syncs once.
 */
int dibella_transitive_reduce(const dibella_csr* R, int32_t fuzz, uint32_t flags,
                              dibella_csr_out* S, int32_t* iterations,
                              dibella_alloc_fn alloc, dibella_free_fn free_fn, void* ctx,
                              void* hip_stream);

/*
 * Batched forms: nsets independent problems (arrays of nsets descriptors,
 * per-set min_shared / fuzz / iterations) processed by the same kernels in
 * one set of launches; every set's result is bit-identical to its own
 * single call.  Work items are the rows of all sets, ordered by estimated
 * cost and drained from a device queue.
 */
int dibella_overlap_batched(const dibella_csr* A, int32_t nsets, const int32_t* min_shared,
                            dibella_overlap_out* C, dibella_alloc_fn alloc,
                            dibella_free_fn free_fn, void* ctx, void* hip_stream);

int dibella_transitive_reduce_batched(const dibella_csr* R, int32_t nsets, const int32_t* fuzz,
                                      uint32_t flags, dibella_csr_out* S, int32_t* iterations,
                                      dibella_alloc_fn alloc, dibella_free_fn free_fn,
                                      void* ctx, void* hip_stream);

/*
 * dibella_r_from_seeds -- overlap graph R from the seeds stored in C
 * (Sec. IV-E: the reduction's overlap suffix and orientation are derived in
 * place from the coordinates stored with each read pair; Sec. IV-D: C keeps
 * two k-mer positions per pair).  It stands between the two products where
 * the paper aligns and prunes, without aligning (dibella_r_from_alignment
 * aligns).
 *
 * C: the output of dibella_overlap (borrowed, never written; col, count and
 * seed are read) for an A whose
 * values are (position << 1) | strand, strand = 1 where the read holds the
 * reverse complement of the canonical k-mer.  read_len: device int32[n],
 * the length of every read, in [0, 2^28).  k: the k-mer length, 1..32.
 * For every off-diagonal entry, its first seed (smallest shared k-mer)
 * places read j in read i's frame by ungapped extension: offset
 * d = p_i - p_j, or p_i + p_j + k - L_j if the strands differ (the pair is
 * reverse complementary).  With max_drift >= 0 the second seed must exist
 * and place the pair in the same relative orientation at an offset within
 * max_drift bases of d (two k-mers agreeing on the overlap, standing in for
 * the alignment that prunes C); max_drift < 0 uses the first seed alone.
 * The overlap [max(0, d), min(L_i, d + L_j)) must
 * span at least min_overlap bases, else the entry is dropped; with
 * min_density > 0 the pair must also share at least min_density k-mers per
 * 10 kbp of that overlap (count * 10000 >= min_density * overlap: a true
 * overlap shares k-mers all along it, a pair that only shares a repeat does
 * not).  These tests stand in for the alignment that prunes C.  A contained
 * overlap is kept with value 0 (the reduction discards it).  Otherwise the
 * four overlap categories give val = (suffix << 2) | (o_i << 1) | o_j:
 *   read i first (forward, inner):   suffix d + L_j - L_i, code (0, rc)
 *   read j first (reverse, outer):   suffix -d,            code (1, 1 - rc)
 * R is n x n in dibella_transitive_reduce's layout, rows sorted.
 * Errors: EINVAL for a malformed C (row pointers, column range or order),
 * a missing seed or one outside its read (position + k > length), a read
 * length outside [0, 2^28), k outside [1, 32] or min_overlap < 0;
 * EOVERFLOW if nrows >= 2^31.
 * Host synchronisation: one stream sync (to size R).
 */
int dibella_r_from_seeds(const dibella_overlap_out* C, const int32_t* read_len, int32_t k,
                         int32_t min_overlap, int32_t max_drift, int32_t min_density,
                         dibella_csr_out* R, dibella_alloc_fn alloc, dibella_free_fn free_fn,
                         void* ctx, void* hip_stream);

/*
 * dibella_r_from_alignment -- R from a seed-and-extend alignment of every
 * pair of C (Sec. IV-D: the alignment is an element-wise operation on C
 * that flags each entry by its score, and the entries scoring below the
 * threshold are pruned; Sec. IV-E: the suffix and orientation of each kept
 * pair come from its alignment coordinates).
 *
 * C: the output of dibella_overlap (square, borrowed; col and seed are
 * read) for an A whose values are (position << 1) | strand.  bases: device
 * uint8[nbases], 2-bit codes A0 C1 G2 T3, the reads back to back; offsets:
 * device int64[n + 1], read i = bases[offsets[i], offsets[i + 1]),
 * offsets[0] = 0, offsets[n] = nbases, non-decreasing, every read shorter
 * than 2^28 bases.  For every off-diagonal entry C_ij the first seed (p_i,
 * p_j) is extended both ways by X-drop extension (Zhang et al., 2000) of
 * read i against read j, or its reverse complement j' when the seed's
 * strands differ (the k-mer then sits at q = L_j - k - p_j in j', else
 * q = p_j): to the right from p_i + k and q + k, to the left from p_i and q
 * backwards.  Linear scores: match in [1, 7], mismatch in [-1024, 0], gap in
 * [-1024, -1] per base against a gap; cells of the extension table are
 * taken anti-diagonal by anti-diagonal, only those with a live predecessor
 * on the two previous anti-diagonals, and a cell scoring below the best of
 * the earlier anti-diagonals minus xdrop (in [0, 2^20]) is dead.  An
 * extension stops after two anti-diagonals without a live cell, at the
 * sequence ends, or before an anti-diagonal that would consider more than
 * 256 cells; it gives its best score and the first cell reaching it
 * (anti-diagonal order, then position in read i).  The pair's score is
 * left + k * match + right; entries below min_score are dropped.  With the
 * alignment spanning [b_i, e_i) of i and [b_j, e_j) of j' and r = L - e the
 * unaligned right ends: one read's unaligned ends both within the other's
 * (b_j >= b_i and r_j >= r_i, or b_i >= b_j and r_i >= r_j): contained,
 * value 0; else read i first (b_i > b_j): suffix r_j - r_i, code (0, rc);
 * else suffix b_j - b_i, code (1, 1 - rc); val = (suffix << 2) | code.
 * R: n x n in dibella_transitive_reduce's layout, rows sorted, allocated
 * through alloc.  score (may be NULL): *score receives device int32[nnz(C)],
 * allocated through alloc, the score of every entry of C (0 on the
 * diagonal; NULL when C is empty).  flags: DIBELLA_ALIGN_GROUP_* or 0
 * (the lanes used never change the result).
 * Errors: EINVAL for a malformed C (row pointers, column range or order), a
 * non-square C, a missing seed or one outside its read, malformed offsets, a
 * base outside 0..3, k outside [1, 32], scores or xdrop outside their
 * ranges, unknown flags; EOVERFLOW if nrows >= 2^31 or nnz >= 2^40.
 * Host synchronisation: two stream syncs (the checks of the reads and of C;
 * the size of R).
 */
int dibella_r_from_alignment(const dibella_overlap_out* C, const uint8_t* bases, int64_t nbases,
                             const int64_t* offsets, int32_t k, int32_t match, int32_t mismatch,
                             int32_t gap, int32_t xdrop, int32_t min_score, uint32_t flags,
                             dibella_csr_out* R, int32_t** score, dibella_alloc_fn alloc,
                             dibella_free_fn free_fn, void* ctx, void* hip_stream);

/*
 * dibella_overlap_graph_blocked -- the overlap graph R of A with C formed
 * one block of rows at a time (Sec. VIII: to bound memory, only a region
 * of the candidate overlap matrix exists at any time, and its spurious
 * entries are removed before the next region is formed; Sec. IV-D, IV-E
 * for the two steps).  A^T is built once.  Then for every block of
 * block_rows consecutive reads (the last one shorter), that block's rows of
 * C = A A^T are formed exactly as dibella_overlap forms them, turned into
 * their rows of R exactly as dibella_r_from_seeds does, and released before
 * the next block.  The result equals dibella_r_from_seeds(dibella_overlap(A,
 * min_shared), read_len, k, min_overlap, max_drift, min_density) entry for
 * entry.
 *
 * A, min_shared: as dibella_overlap (one set).  read_len, k, min_overlap,
 * max_drift, min_density: as dibella_r_from_seeds.  block_rows >= 1 (a
 * value >= nrows gives one block).  R: n x n, allocated through alloc;
 * *nblocks (may be NULL) receives the number of blocks.  Where A has enough
 * columns for the sliced segment pass, A^T is itself built over as many
 * column ranges as there are blocks (at most one per slice), one range's
 * partition buffers at a time.  Peak workspace: A^T (8 bytes per entry),
 * the column records and slice table, plus the larger of one column range's
 * partition buffers and one block's row-phase workspace and C rows, plus R
 * so far.
 * Errors: those of dibella_overlap and dibella_r_from_seeds; EINVAL for
 * block_rows < 1.  Host synchronisation: one stream sync for the column
 * ranges' sizes (with column ranges), one to read A's row pointers, then per
 * block the syncs of dibella_overlap's row phases (two, or three on
 * retry-table overflow) and one of dibella_r_from_seeds.
 */
int dibella_overlap_graph_blocked(const dibella_csr* A, int32_t min_shared, const int32_t* read_len,
                                  int32_t k, int32_t min_overlap, int32_t max_drift,
                                  int32_t min_density, int64_t block_rows, dibella_csr_out* R,
                                  int32_t* nblocks, dibella_alloc_fn alloc, dibella_free_fn free_fn,
                                  void* ctx, void* hip_stream);

/*
 * dibella_transitive_reduce_noalloc -- dibella_transitive_reduce for callers
 * that cannot allocate (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  It makes no device or pinned host
 * allocation: its workspace is a static device array of 64 MiB that every
 * GPU the library runs on holds until the process ends, and S goes into the
 * caller's arrays.  Same semantics, flags and errors as
 * dibella_transitive_reduce for one set, plus:
 *   s_rowptr: int64[nrows + 1]; s_col, s_val: int32[s_capacity] with
 *   s_capacity >= nnz(R) (S never has more entries than R); on return
 *   *s_nnz = nnz(S) and *iterations = passes.
 *   EINVAL if the capacity is below nnz(R), if DIBELLA_TR_USE_GRAPH is set
 *   (instantiating a graph allocates), or if R needs more than the 64 MiB of
 *   workspace (about 21 bytes per entry and 37 per row).
 * Every call on one GPU uses that GPU's array: calls that overlap on one GPU
 * (different streams or host threads) race and must be serialised by the
 * caller.  No timing records are taken during the call.
 */
int dibella_transitive_reduce_noalloc(const dibella_csr* R, int32_t fuzz, uint32_t flags,
                                      int64_t* s_rowptr, int32_t* s_col, int32_t* s_val,
                                      int64_t s_capacity, int64_t* s_nnz, int32_t* iterations,
                                      void* hip_stream);

/*
 * dibella_kmer_matrix -- A from the reads (Sec. IV-C; Algorithm "diBELLA 2D":
 * KmerCounter and GenerateA).
 *
 * bases: device uint8[nbases], 2-bit codes A0 C1 G2 T3, the reads back to
 * back; offsets: device int64[n + 1], read i = bases[offsets[i],
 * offsets[i + 1]) (offsets[0] = 0, offsets[n] = nbases, non-decreasing).
 * Every window of k bases of a read (position p, p + k <= length) is a
 * k-mer; its canonical form is the smaller of its code (first base most
 * significant) and its reverse complement's, its strand 1 when the reverse
 * complement is the smaller.  A k-mer's frequency is its number of windows
 * over all reads (repeats inside a read count); it is reliable when
 * lo <= frequency <= hi.  The reliable k-mers are A's columns in the order
 * of their first occurrence: by the first read holding the k-mer, then by
 * its smallest position in that read (the paper fixes no column order;
 * this one gives the k-mers of a read consecutive columns, so the rows of
 * A^T that one read's products visit lie side by side in memory).  A_ic =
 * the smallest position of k-mer c in read i, or (position << 1) | strand
 * (the strand at that position) with DIBELLA_KMER_STRAND.  A: n x m, rows
 * sorted, allocated through alloc; *codes: device uint64[m], codes[c] = the
 * canonical code of column c, allocated through alloc (NULL when m = 0).
 * Errors: EINVAL for k outside [1, 31], lo < 1, hi < lo, malformed offsets
 * or a base outside 0..3; EOVERFLOW for n >= 2^31, 2^32 windows or more, or
 * 2^31 reliable k-mers or more.
 * Host synchronisation: two stream syncs (the window count; the k-mer and
 * entry counts).
 */
int dibella_kmer_matrix(const uint8_t* bases, const int64_t* offsets, int64_t nreads, int64_t nbases,
                        int32_t k, int32_t lo, int32_t hi, uint32_t flags, dibella_csr_out* A,
                        uint64_t** codes, dibella_alloc_fn alloc, dibella_free_fn free_fn, void* ctx,
                        void* hip_stream);

/* Message of the last nonzero status returned on this host thread. */
const char* dibella_last_error(void);

/* Launch shapes and table sizes.  Values outside the supported sets are
 * rejected with EINVAL.  The setting is process wide; change it only while
 * no call is running. */
typedef struct {
    int32_t sym_block;        /* threads per workgroup, symbolic phase: 64,128,256,512 */
    int32_t num_block;        /* numeric phase: 64,128,256,512 */
    int32_t tr_block;         /* reduction pass: 64,128,256,512 */
    int32_t sym_first_log2;   /* first symbolic LDS hash table, log2 slots: 8..13; rows
                                 that overflow it are retried with the retry table */
    int32_t sym_max_log2;     /* retry table, log2 slots: sym_first_log2..14; rows that
                                 overflow it go to expand-sort-compress */
    int32_t num_max_entries;  /* most output entries a row may have in the numeric LDS path:
                                 256..8192 (capped by the LDS); larger rows go to ESC */
    int32_t load_pct;         /* hash-table load limit in percent: 40..85 */
    int32_t tr_lds_cap;       /* longest row kept in LDS by a pass: 512..8192 (lowered in
                                 steps of 512 until the pass fits the LDS: 6144 at 512
                                 threads); longer rows keep their minima in global memory */
    int32_t tr_graph_passes;  /* passes per captured graph: 1..16 */
    int32_t bits_max_words;   /* bitmap path for sets with at most 32 * this many reads
                                 (and min_shared <= 4): 0..8192; 0 = hash path only */
} dibella_tuning;

int dibella_get_tuning(dibella_tuning* out);
int dibella_set_tuning(const dibella_tuning* t);

/* Counters of the last call on this host thread (for measurement). */
typedef struct {
    int64_t products;         /* overlap: semiring multiplies = sum_k (col count)^2 */
    int64_t esc_rows;         /* overlap: rows handled by expand-sort-compress */
    int64_t host_syncs;       /* stream synchronisations made by the call */
    int64_t triples;          /* reduction: walks i->k->j examined, all passes */
    int32_t passes;           /* reduction: passes run (max over sets) */
    int32_t trace_len;        /* entries used in nnz_trace / triples_trace */
    int64_t nnz_trace[64];    /* reduction: total nnz after the contained drop, then after each pass */
    int64_t triples_trace[64];/* reduction: triples examined in each pass */
    int64_t cells;            /* alignment: extension-table cells considered, both sides of
                                 every pair (dibella_r_from_alignment) */
} dibella_stats;

int dibella_last_stats(dibella_stats* out);

/* Kernel timing with HIP events recorded on the caller's stream around each
 * launch of the main kernels (per host thread).  One record per launch:
 *   0 keys          validation of A and its (column, read|position) pairs
 *   1 part_count    bucketed transpose: bucket histogram per chunk of pairs
 *   2 part_scatter  bucketed transpose: pairs grouped by bucket
 *   3 bucket_sort   bucketed transpose: per bucket, a counting sort by column
 *                   in staged sweeps giving the A^T entries and one record
 *                   per column
 *   4 part2_count   three-level transpose (very many columns): per chunk of
 *                   a segment, its bucket histogram
 *   5 part2_scatter three-level transpose: pairs of each segment grouped by
 *                   bucket
 *   6 segments      A^T segment per A entry, products per row, row bins
 *   7 sym_bits      symbolic phase, bitmap path
 *   8 sym_hash      symbolic phase, hash path (one launch per table size)
 *   9 numeric       numeric phase (one launch per output-size bin)
 *  10 esc           expand-sort-compress kernels of dense rows
 *  11 tr_mark       reduction pass: N on the pattern of R, row max, compare
 *  12 tr_compact    reduction pass: compaction of the kept entries
 *  13 numeric_phase the whole numeric phase of one call, first launch to
 *                   last (its launches overlap on several streams, so the
 *                   sum of the records of label 9 exceeds this)
 *  14 r_from_seeds  overlap graph from the seeds of C (both passes)
 *  15 kmer_windows  A from the reads: window counts and canonical codes
 *  16 kmer_sort     A from the reads: the radix sorts (by k-mer, by read)
 *  17 kmer_runs     A from the reads: frequencies, columns, kept entries
 *  18 kmer_rows     A from the reads: row pointers, columns and values
 *  19 align         R from the alignment: the X-drop extensions of all pairs
 * Passes run as captured graphs are not timed.  Enabling clears the
 * accumulators; collect waits for the recorded events, returns the summed
 * milliseconds and number of records per label, and clears them. */
#define DIBELLA_NUM_PHASES 20
typedef struct {
    double ms[DIBELLA_NUM_PHASES];
    int64_t records[DIBELLA_NUM_PHASES];
} dibella_timing;

int dibella_timing_enable(int on);
/* Labels recorded while timing is enabled on this host thread: bit i selects
 * label i (all labels by default).  A launch whose label is not selected
 * records no events and costs no host time.  Bits at DIBELLA_NUM_PHASES or
 * above are rejected with EINVAL.  Records already taken are kept. */
int dibella_timing_select(uint32_t label_mask);
int dibella_timing_collect(dibella_timing* out);

#ifdef __cplusplus
}
#endif
#endif /* DIBELLA_H */
