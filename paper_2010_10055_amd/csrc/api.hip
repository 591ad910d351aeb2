// extern "C" entry points of include/dibella.h: argument checks, statistics
// reset, and the stream / allocator plumbing around the two drivers.
#include "common.hpp"

#include <cstring>

using namespace dibella;

namespace {

void reset_stats() { std::memset(&stats(), 0, sizeof(dibella_stats)); }

// On failure: wait for everything already enqueued (it may still reference
// workspace and staging), then let the arena release outputs too.
template <class Fn>
int guarded(Arena& ar, Fn&& fn) {
    int s = fn();
    if (s != DIBELLA_OK) {
        (void)hipStreamSynchronize(ar.stream());
        ar.fail();
    }
    return s;
}

}  // namespace

extern "C" {

int dibella_overlap(const dibella_csr* A, int32_t min_shared, dibella_overlap_out* C, dibella_alloc_fn alloc,
                    dibella_free_fn free_fn, void* ctx, void* hip_stream) {
    return dibella_overlap_batched(A, 1, &min_shared, C, alloc, free_fn, ctx, hip_stream);
}

int dibella_overlap_batched(const dibella_csr* A, int32_t nsets, const int32_t* min_shared,
                            dibella_overlap_out* C, dibella_alloc_fn alloc, dibella_free_fn free_fn, void* ctx,
                            void* hip_stream) {
    reset_stats();
    if (!A || !C || !min_shared || nsets < 0 || (alloc == nullptr) != (free_fn == nullptr)) {
        set_error("dibella_overlap: bad arguments");
        return DIBELLA_EINVAL;
    }
    if (nsets == 0) return DIBELLA_OK;
    int status;
    {
        Arena ar(alloc, free_fn, ctx, static_cast<hipStream_t>(hip_stream));
        status = guarded(ar, [&] { return overlap_run(A, nsets, min_shared, C, 0u, ar); });
    }
    if (status != DIBELLA_OK)
        for (int s = 0; s < nsets; ++s) std::memset(&C[s], 0, sizeof(C[s]));
    return status;
}

int dibella_transitive_reduce(const dibella_csr* R, int32_t fuzz, uint32_t flags, dibella_csr_out* S,
                              int32_t* iterations, dibella_alloc_fn alloc, dibella_free_fn free_fn, void* ctx,
                              void* hip_stream) {
    return dibella_transitive_reduce_batched(R, 1, &fuzz, flags, S, iterations, alloc, free_fn, ctx, hip_stream);
}

int dibella_transitive_reduce_batched(const dibella_csr* R, int32_t nsets, const int32_t* fuzz, uint32_t flags,
                                      dibella_csr_out* S, int32_t* iterations, dibella_alloc_fn alloc,
                                      dibella_free_fn free_fn, void* ctx, void* hip_stream) {
    reset_stats();
    if (!R || !S || !fuzz || !iterations || nsets < 0 || (alloc == nullptr) != (free_fn == nullptr)) {
        set_error("dibella_transitive_reduce: bad arguments");
        return DIBELLA_EINVAL;
    }
    if (nsets == 0) return DIBELLA_OK;
    int status;
    {
        Arena ar(alloc, free_fn, ctx, static_cast<hipStream_t>(hip_stream));
        status = guarded(ar, [&] { return tr_run(R, nsets, fuzz, flags, S, iterations, ar); });
    }
    if (status != DIBELLA_OK)
        for (int s = 0; s < nsets; ++s) {
            std::memset(&S[s], 0, sizeof(S[s]));
            iterations[s] = 0;
        }
    return status;
}

int dibella_r_from_seeds(const dibella_overlap_out* C, const int32_t* read_len, int32_t k, int32_t min_overlap,
                         int32_t max_drift, int32_t min_density, dibella_csr_out* R, dibella_alloc_fn alloc,
                         dibella_free_fn free_fn, void* ctx, void* hip_stream) {
    reset_stats();
    if (!C || !R || (alloc == nullptr) != (free_fn == nullptr)) {
        set_error("dibella_r_from_seeds: bad arguments");
        return DIBELLA_EINVAL;
    }
    if (C->ncols != C->nrows) {
        set_error("dibella_r_from_seeds: C must be square");
        return DIBELLA_EINVAL;
    }
    int status;
    {
        Arena ar(alloc, free_fn, ctx, static_cast<hipStream_t>(hip_stream));
        status = guarded(ar, [&] {
            return r_from_seeds_run(C, 0, read_len, k, min_overlap, max_drift, min_density, R, ar, ar, false);
        });
    }
    if (status != DIBELLA_OK) std::memset(R, 0, sizeof(*R));
    return status;
}

int dibella_overlap_graph_blocked(const dibella_csr* A, int32_t min_shared, const int32_t* read_len, int32_t k,
                                  int32_t min_overlap, int32_t max_drift, int32_t min_density, int64_t block_rows,
                                  dibella_csr_out* R, int32_t* nblocks, dibella_alloc_fn alloc,
                                  dibella_free_fn free_fn, void* ctx, void* hip_stream) {
    reset_stats();
    if (!A || !R || (alloc == nullptr) != (free_fn == nullptr)) {
        set_error("dibella_overlap_graph_blocked: bad arguments");
        return DIBELLA_EINVAL;
    }
    int32_t nb = 0;
    int status;
    {
        Arena ar(alloc, free_fn, ctx, static_cast<hipStream_t>(hip_stream));
        status = guarded(ar, [&] {
            return overlap_graph_blocked_run(A, min_shared, read_len, k, min_overlap, max_drift, min_density,
                                             block_rows, R, &nb, ar);
        });
    }
    if (status != DIBELLA_OK) std::memset(R, 0, sizeof(*R));
    if (nblocks) *nblocks = status == DIBELLA_OK ? nb : 0;
    return status;
}

int dibella_kmer_matrix(const uint8_t* bases, const int64_t* offsets, int64_t nreads, int64_t nbases, int32_t k,
                        int32_t lo, int32_t hi, uint32_t flags, dibella_csr_out* A, uint64_t** codes,
                        dibella_alloc_fn alloc, dibella_free_fn free_fn, void* ctx, void* hip_stream) {
    reset_stats();
    if (!A || !codes || (alloc == nullptr) != (free_fn == nullptr) || (flags & ~DIBELLA_KMER_STRAND)) {
        set_error("dibella_kmer_matrix: bad arguments");
        return DIBELLA_EINVAL;
    }
    int64_t m = 0;
    int status;
    {
        Arena ar(alloc, free_fn, ctx, static_cast<hipStream_t>(hip_stream));
        status = guarded(ar, [&] {
            return kmer_matrix_run(bases, offsets, nreads, nbases, k, lo, hi, flags, A, codes, &m, ar);
        });
    }
    if (status != DIBELLA_OK) {
        std::memset(A, 0, sizeof(*A));
        *codes = nullptr;
    }
    return status;
}

int dibella_r_from_alignment(const dibella_overlap_out* C, const uint8_t* bases, int64_t nbases,
                             const int64_t* offsets, int32_t k, int32_t match, int32_t mismatch, int32_t gap,
                             int32_t xdrop, int32_t min_score, uint32_t flags, dibella_csr_out* R, int32_t** score,
                             dibella_alloc_fn alloc, dibella_free_fn free_fn, void* ctx, void* hip_stream) {
    reset_stats();
    if (!C || !R || (alloc == nullptr) != (free_fn == nullptr)) {
        set_error("dibella_r_from_alignment: bad arguments");
        return DIBELLA_EINVAL;
    }
    int status;
    {
        Arena ar(alloc, free_fn, ctx, static_cast<hipStream_t>(hip_stream));
        status = guarded(ar, [&] {
            return r_from_alignment_run(C, bases, nbases, offsets, k, match, mismatch, gap, xdrop, min_score, flags,
                                        R, score, ar);
        });
    }
    if (status != DIBELLA_OK) {
        std::memset(R, 0, sizeof(*R));
        if (score) *score = nullptr;
    }
    return status;
}

const char* dibella_last_error(void) { return error_slot().c_str(); }

int dibella_get_tuning(dibella_tuning* out) {
    if (!out) return DIBELLA_EINVAL;
    *out = tuning();
    return DIBELLA_OK;
}

int dibella_set_tuning(const dibella_tuning* t) {
    auto block_ok = [](int b) { return b == 64 || b == 128 || b == 256 || b == 512; };
    if (!t || !block_ok(t->sym_block) || !block_ok(t->num_block) || !block_ok(t->tr_block) ||
        t->sym_first_log2 < 8 || t->sym_first_log2 > 13 || t->sym_max_log2 < t->sym_first_log2 ||
        t->sym_max_log2 > 14 || t->num_max_entries < 256 || t->num_max_entries > 8192 ||
        t->load_pct < 40 || t->load_pct > 85 || t->tr_lds_cap < 512 || t->tr_lds_cap > 8192 ||
        t->tr_graph_passes < 1 || t->tr_graph_passes > 16 || t->bits_max_words < 0 ||
        t->bits_max_words > 8192) {
        set_error("dibella_set_tuning: value outside the supported range");
        return DIBELLA_EINVAL;
    }
    tuning_store(*t);
    return DIBELLA_OK;
}

int dibella_timing_enable(int on) {
    timing_set_enabled(on != 0);
    return DIBELLA_OK;
}

int dibella_timing_select(uint32_t label_mask) {
    if (label_mask >> DIBELLA_NUM_PHASES) return DIBELLA_EINVAL;
    timing_set_mask(label_mask);
    return DIBELLA_OK;
}

int dibella_timing_collect(dibella_timing* out) {
    if (!out) return DIBELLA_EINVAL;
    return timing_collect(out);
}

int dibella_last_stats(dibella_stats* out) {
    if (!out) return DIBELLA_EINVAL;
    *out = stats();
    return DIBELLA_OK;
}

}  // extern "C"
