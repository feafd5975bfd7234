/*
 * swsearch.h - C ABI of the MI355X (gfx950) Smith-Waterman protein database search.
 *
 * The library computes, for one or many protein queries, the optimal local
 * alignment score S of every subject of a device-resident protein database
 * under Smith-Waterman with Gotoh affine gaps (Sec. II-B, Eq. 1-3 of
 * Costanzo et al., "Comparing Performance and Portability between CUDA and
 * SYCL for Protein Database Search on NVIDIA, AMD, and Intel GPUs"):
 *
 *   H[i][j] = max(0, H[i-1][j-1] + SM(Q[i], D[j]), E[i][j], F[i][j])
 *   E[i][j] = max(H[i][j-1] - Go, E[i][j-1] - Ge)
 *   F[i][j] = max(H[i-1][j] - Go, F[i-1][j] - Ge)
 *   H = E = F = 0 on row 0 and column 0;  S = max(0, max H).
 *
 * Only scores are computed (linear space); the top-ranked subjects can then be
 * selected (Sec. II-B, "all alignment scores are calculated first and optimal
 * alignments are computed only for top-ranked database sequences").
 *
 * Scores are exact int32 values for every input: internally most cells run in
 * saturating 16-bit lanes, and any subject whose 16-bit score reaches the
 * saturation value is recomputed with 32-bit cells.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Residue codes are int8 values 0..A-1, where A is the database's alphabet
 *    size (sw_pack_opts.alphabet; by default A = 20, the amino acids in the
 *    order ARNDCQEGHILKMFPSTWYV).  Any other value in a query or database is
 *    an error (SW_E_RESIDUE).
 *  - The substitution matrix is int8[A][A], row-major, indexed
 *    [query residue][subject residue], in host memory.
 *  - Gap penalties are Go = gap_open >= 0 and Ge = gap_extend >= 0; a gap run
 *    of k residues costs Go + (k-1)*Ge when Ge <= Go (the recurrence itself
 *    is what is computed for any Go, Ge >= 0).  Negative values: SW_E_INVALID.
 *  - "d_" pointers are device memory of the device that was current when the
 *    database was packed; "h_" pointers are host memory.  The caller owns every
 *    pointer it passes.  The library allocates device memory behind an sw_db
 *    handle only for calls that are not given it: a caller can own all of it
 *    by packing with sw_db_pack_into and searching with sw_search_ws and
 *    sw_search_batch_ws (sizes from sw_db_pack_bytes and
 *    sw_batch_workspace_bytes); the handle then holds host memory only.
 *  - All work is enqueued on the given HIP stream and the call returns without
 *    waiting for it, except where stated.  Outputs are valid once the stream
 *    has completed.  Host input arrays may be reused as soon as a call returns.
 *  - Errors are returned as negative sw_status codes; a text description of
 *    the most recent error of the calling thread is available from
 *    sw_last_error().  No call aborts the process.
 *  - A handle may be used from one host thread at a time and by at most one
 *    search in flight at a time (searches reuse the handle's device workspace).
 */
#ifndef SWSEARCH_H
#define SWSEARCH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t sw_status;
enum {
    SW_OK = 0,
    SW_E_INVALID = -1,      /* null pointer, negative size or penalty, mismatched database */
    SW_E_RESIDUE = -2,      /* residue code outside the alphabet */
    SW_E_NOMEM = -3,        /* device or host allocation failed */
    SW_E_HIP = -4,          /* a HIP runtime call failed; see sw_last_error() */
    SW_E_UNSUPPORTED = -5,  /* request outside the implemented limits (e.g. k > 1024) */
    SW_E_SIZE = -6          /* a caller buffer is too small */
};

/* Opaque packed database.  Created by sw_db_pack, released by sw_db_free. */
typedef struct sw_db sw_db;

/* Stream type: a hipStream_t passed as an opaque pointer (NULL = default stream). */
typedef void* sw_stream;

/* Packing options; zero-initialise for defaults. */
typedef struct {
    int32_t max_qlen;         /* unused hint, 0 */
    int32_t force_lanes;      /* test hook: 0 = planner decides; 1,2,4,...,64 = every pair of
                                 subjects is swept by this many cooperating lanes */
    int32_t rerun_threshold;  /* test hook: 0 = the largest, 31744 (0x7C00) minus the search's 16-bit
                                 bias c = minus the matrix's lowest score (4 for BLOSUM62); a smaller
                                 value sends every pair whose 16-bit score reaches it to the exact
                                 32-bit recompute */
    int32_t rows_per_lane;    /* tuning: 0 = planner decides; 4, 8 or 16 query rows per lane */
    int32_t unit_share;       /* tuning: largest work unit as a fraction of one persistent wave's
                                 share of a search, in 1/1000; 0 = default (250) */
    int32_t lane_pack;        /* tuning, batched and multi-query forms: 0 or 1 = the two 16-bit halves
                                 of a lane hold two subjects; 2 = they hold two queries (queries are
                                 paired by length; a single query always uses subject pairs) */
    int32_t alphabet;         /* residue codes 0..alphabet-1: 0 = 20 (the standard amino acids
                                 ARNDCQEGHILKMFPSTWYV); up to 24 (e.g. plus B, Z, X, *).  Substitution
                                 matrices passed with this database are int8[alphabet * alphabet].
                                 Fixed at packing; sw_db_tune ignores it. */
    int32_t rerun_cap;        /* test hook: 0 = default; > 0 = at most this many flagged (query, subject
                                 pair) entries in the recompute's list.  Pairs flagged beyond the list are
                                 kept as one bit each and recomputed all the same, so scores never
                                 depend on it; it exists to exercise that path. */
    int32_t poison;           /* test hook: 1 = every flagged pair's 16-bit scores are written as
                                 -1,000,000,007 before the recompute overwrites them, so a pair the
                                 recompute missed would show; 0 = off. */
    int32_t align_tiles;      /* tuning, alignments: 0 = pairs whose query and subject both have at least
                                 2,048 residues fill their matrix as tiles of 256 query rows by 128-256
                                 subject columns over the whole GPU, the others on one workgroup each;
                                 1 = every pair on one workgroup; 2 = every pair as tiles.  The
                                 alignments are the same for every setting. */
} sw_pack_opts;

/*
 * sw_db_pack - build a device-resident, search-ready image of a protein database.
 *   d_residues : device int8, the subjects concatenated; subject k occupies
 *                d_residues[h_offsets[k] .. h_offsets[k+1]).
 *   h_offsets  : host int64[n + 1], non-decreasing, h_offsets[0] >= 0.
 *   n          : number of subjects (>= 0).
 *   opts       : may be NULL.
 *   out        : receives the handle.
 * The image sorts subjects by length and interleaves them for coalesced loads;
 * it is independent of the query and the scoring parameters.  This call
 * synchronises the stream (packing is a one-time setup step) and validates
 * every residue code: SW_E_RESIDUE if any is outside 0..alphabet-1.
 */
sw_status sw_db_pack(const int8_t* d_residues, const int64_t* h_offsets, int64_t n,
                     const sw_pack_opts* opts, sw_stream stream, sw_db** out);

/*
 * sw_db_pack_bytes - device bytes of the packed image of a database with these
 * offsets (the same for any options): the interleaved residues plus about
 * 20 bytes per subject of tables, of which 8 per subject are used while
 * packing only.
 *
 * sw_db_pack_into - sw_db_pack into a caller-owned device buffer d_db of
 * db_bytes >= sw_db_pack_bytes (SW_E_SIZE otherwise), 256-byte aligned
 * (SW_E_INVALID otherwise).  The handle keeps host-side tables only and never
 * frees d_db, which must outlive the handle.
 */
sw_status sw_db_pack_bytes(const int64_t* h_offsets, int64_t n, const sw_pack_opts* opts, int64_t* bytes);
sw_status sw_db_pack_into(const int8_t* d_residues, const int64_t* h_offsets, int64_t n,
                          const sw_pack_opts* opts, void* d_db, int64_t db_bytes, sw_stream stream,
                          sw_db** out);

/*
 * sw_db_tune - change the tuning knobs and test hooks of a packed database
 * (every field of opts but max_qlen and alphabet).  Synchronises the handle's
 * device and drops cached plans and graphs.  Results are bit-identical for
 * every setting; only speed changes.
 */
sw_status sw_db_tune(sw_db* db, const sw_pack_opts* opts);

/* Releases the handle and its device memory (after synchronising its device). */
void sw_db_free(sw_db* db);

/* Number of subjects, total residues and device bytes the handle itself allocated (0 for a
   handle packed with sw_db_pack_into and searched only through the _ws calls). */
sw_status sw_db_info(const sw_db* db, int64_t* n, int64_t* residues, int64_t* device_bytes);

/*
 * sw_search - scores of one query against every subject (the "plain" form).
 *   h_query    : host int8[qlen], residue codes (validated on the host).
 *   qlen       : >= 0; qlen == 0 gives all-zero scores.
 *   db         : packed database.
 *   h_offsets  : the offsets the database was packed with, or NULL.  When
 *                given they are checked against the handle (same n, same
 *                first and last offset and the same 64-bit hash of all n + 1
 *                values, an O(n) pass on the host): SW_E_INVALID otherwise.
 *                NULL skips the check (the caller vouches for them).
 *   n          : number of subjects; must equal the handle's.
 *   h_subst    : host int8[A*A] substitution matrix.
 *   gap_open, gap_extend : Go, Ge >= 0.
 *   d_scores_out : device int32[n]; receives S for each subject in the
 *                original database order.
 * The work is enqueued on `stream`.  The first search of a query length plans
 * it on the host and copies the plan to the handle's device memory with a
 * synchronous copy (later searches of that length reuse it); sw_search_ws
 * sends the plan with the query, in stream order, instead.
 */
sw_status sw_search(const int8_t* h_query, int32_t qlen, sw_db* db, const int64_t* h_offsets,
                    int64_t n, const int8_t* h_subst, int32_t gap_open, int32_t gap_extend,
                    int32_t* d_scores_out, sw_stream stream);

/*
 * sw_search_ws - sw_search on a caller-owned device workspace d_workspace of
 * ws_bytes >= sw_batch_workspace_bytes(db, {0, qlen}, 1, 0, 0) bytes,
 * 256-byte aligned.  Allocates no device memory.  The workspace holds the
 * boundary rows between passes, the query profile, the staged query and work
 * items, the recompute list and counters; it must stay untouched until the
 * stream has completed the search (and until sw_last_stats, which reads the
 * counters from it).  Results are identical to sw_search.
 */
sw_status sw_search_ws(const int8_t* h_query, int32_t qlen, sw_db* db, const int64_t* h_offsets, int64_t n,
                       const int8_t* h_subst, int32_t gap_open, int32_t gap_extend, int32_t* d_scores_out,
                       void* d_workspace, int64_t ws_bytes, sw_stream stream);

/*
 * sw_topk - the k best subjects of one score vector (Sec. II-B: alignments are
 * computed only for top-ranked subjects), ordered by score descending, then by
 * subject index ascending.  When k > n the tail is padded with score -1 and
 * index -1.
 *   d_scores : device int32[n].      k : 1..1024.
 *   d_top_scores : device int32[k].   d_top_index : device int64[k].
 */
sw_status sw_topk(const int32_t* d_scores, int64_t n, int32_t k,
                  int32_t* d_top_scores, int64_t* d_top_index, sw_stream stream);

/*
 * sw_topk_ws - sw_topk with a caller-owned device workspace, which lets a long
 * score vector be cut into pieces whose own top k are merged in a second
 * launch (hundreds of workgroups instead of one).  Same results as sw_topk.
 * sw_topk_ws_bytes gives the workspace size for n and k (0: one launch is
 * used, the workspace may be NULL).  d_workspace NULL always takes one launch;
 * a non-NULL workspace smaller than required is SW_E_SIZE.  Any int32 scores
 * are ordered correctly (sw_topk too), negative ones included.
 */
sw_status sw_topk_ws_bytes(int64_t n, int32_t k, int64_t* bytes);
sw_status sw_topk_ws(const int32_t* d_scores, int64_t n, int32_t k, int32_t* d_top_scores, int64_t* d_top_index,
                     void* d_workspace, int64_t ws_bytes, sw_stream stream);

/*
 * sw_topk_noalloc - sw_topk_ws without any allocation, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops).
 * The piece workspace is a fixed 4 MiB device array inside the library, one
 * copy per device, held until the process ends; the call itself makes no
 * hipMalloc, hipFree or other allocation.  Same arguments and results as
 * sw_topk (k in 1..1024, any n), on the current device.  Calls that overlap
 * on one device share its array and race: keep them on one stream or order
 * them with events.  A workspace need beyond the array would be SW_E_SIZE; a
 * row needs at most 256 pieces x k x 12 bytes + 256, so none does.
 */
sw_status sw_topk_noalloc(const int32_t* d_scores, int64_t n, int32_t k, int32_t* d_top_scores,
                          int64_t* d_top_index, sw_stream stream);

/*
 * sw_search_batch - scores of nq queries against every subject in one
 * persistent launch sequence (the "batched" form), plus each query's top k.
 *   h_queries  : host int8, the queries concatenated.
 *   h_qoffsets : host int64[nq + 1], non-decreasing.
 *   k          : 0 (no top-k) or 1..1024.
 *   d_scores   : device int32[nq * n] (row q = query q, original subject order),
 *                or NULL to keep only the top k (then k must be >= 1).
 *   d_top_scores : device int32[nq * k] or NULL when k == 0.
 *   d_top_index  : device int64[nq * k] or NULL when k == 0.
 * A batch shape (query lengths, penalties, k, output and workspace
 * addresses, stream) that comes twice in a row is captured as a HIP graph on
 * the second call and replayed on later calls with that shape; a shape seen
 * once is enqueued directly.  A new query-length mix waits for the stream's
 * earlier work (the handle's plan buffer is replaced).
 */
sw_status sw_search_batch(const int8_t* h_queries, const int64_t* h_qoffsets, int32_t nq,
                          sw_db* db, const int8_t* h_subst, int32_t gap_open, int32_t gap_extend,
                          int32_t k, int32_t* d_scores, int32_t* d_top_scores, int64_t* d_top_index,
                          sw_stream stream);

/*
 * sw_batch_workspace_bytes - device bytes of the workspace of one search of
 * the nq queries with offsets h_qoffsets (lengths matter, contents do not):
 * sw_search_batch_ws with top k (0..1024), or sw_search_ws when nq == 1 and
 * k == 0.  scores_in_ws != 0 adds room for the nq score rows, needed when the
 * batched call is given d_scores == NULL.  Plans the batch (the plan is kept
 * for the next call with the same lengths).
 *
 * sw_search_batch_ws - sw_search_batch on a caller-owned workspace of
 * ws_bytes >= that size (SW_E_SIZE otherwise), 256-byte aligned.  Allocates
 * no device memory; the captured graph of a batch shape is tied to the
 * workspace address (another address captures again).  The plan travels
 * with the queries into the workspace, in stream order, so the call does not
 * wait for earlier work, and calls may be queued back to back on one stream
 * (a serving loop keeps the next batch queued while one runs).  Queries are
 * staged through a ring of four pinned host buffers per handle: a call waits
 * only until the staging copy of the call four before it on the handle has
 * run.  The workspace must stay untouched until the stream has completed the
 * call.
 */
sw_status sw_batch_workspace_bytes(sw_db* db, const int64_t* h_qoffsets, int32_t nq, int32_t k,
                                   int32_t scores_in_ws, int64_t* bytes);
sw_status sw_search_batch_ws(const int8_t* h_queries, const int64_t* h_qoffsets, int32_t nq, sw_db* db,
                             const int8_t* h_subst, int32_t gap_open, int32_t gap_extend, int32_t k,
                             int32_t* d_scores, int32_t* d_top_scores, int64_t* d_top_index,
                             void* d_workspace, int64_t ws_bytes, sw_stream stream);

/*
 * sw_search_multi - one launch sequence in which each query scores one chunk of
 * the database (the building block of continuous batching in a serving loop).
 * The length-sorted groups of 128 subjects are dealt round-robin into nchunks
 * chunks: chunk c holds groups c, c + nchunks, c + 2*nchunks, ..., so every
 * chunk has the same length mix.  Query q scores the subjects of chunk
 * h_chunk[q] and writes those entries of its own score vector h_d_scores[q]
 * (device int32[n], original subject order); entries of other chunks are left
 * untouched.  After one call per chunk (in any order, in any mix of queries)
 * the vector holds every score.  A zero-length query fills its whole vector
 * with 0.
 *   h_chunk    : host int32[nq], each in 0..nchunks-1.
 *   h_d_scores : host array of nq device pointers.
 * Synchronises the stream before planning (the plan buffer is reused).
 */
sw_status sw_search_multi(const int8_t* h_queries, const int64_t* h_qoffsets, int32_t nq, const int32_t* h_chunk,
                          int32_t nchunks, sw_db* db, const int8_t* h_subst, int32_t gap_open, int32_t gap_extend,
                          int32_t* const* h_d_scores, sw_stream stream);

/* Alignment modes of sw_search_mode. */
enum { SW_LOCAL = 0, SW_GLOBAL = 1, SW_SEMIGLOBAL = 2 };

/*
 * sw_search_mode - scores of one query against every subject in one of three
 * modes.  SW_LOCAL is sw_search (Smith-Waterman, Sec. II-B, Eq. 1-3).  The
 * other two drop the 0 of Eq. 1 and put gap runs on the borders,
 * H[i][0] = g(i) with g(k) = -(Go + (k-1) * min(Go, Ge)), g(0) = 0, E[i][0] =
 * F[0][j] = minus infinity:
 *   SW_GLOBAL      H[0][j] = g(j), S = H[m][n] (both sequences end to end);
 *   SW_SEMIGLOBAL  H[0][j] = 0, S = max over j of H[m][j] (the whole query
 *                  against any stretch of the subject).
 * Scores may be negative.  Cells are 16-bit with a bias and a check that
 * every H of a pair stayed in the exact range; pairs that left it are
 * recomputed in 32-bit cells, so every score is exact.  SW_GLOBAL with
 * Ge <= Go and a query of at most about 3,100 residues (at 10/2) stores
 * H[i][j] - g(j) in its cells, which keeps every subject's row-0 gap run in
 * range; otherwise subjects whose row-0 gap run leaves the range run in 32-bit
 * cells from the start.  SW_E_UNSUPPORTED if Go + (qlen + longest subject) * max(Go, Ge)
 * could leave +-2^29.  Other arguments and errors as for sw_search;
 * sw_last_stats reports the 16-bit launch (out[0], out[2]) and, in out[4] and
 * out[5], the launches beside it (long pairs of a short query at 4 or 8 rows
 * per lane, and the 32-bit subjects).
 */
sw_status sw_search_mode(int32_t mode, const int8_t* h_query, int32_t qlen, sw_db* db, const int64_t* h_offsets,
                         int64_t n, const int8_t* h_subst, int32_t gap_open, int32_t gap_extend,
                         int32_t* d_scores_out, sw_stream stream);

/* One optimal local alignment (see sw_align). */
typedef struct {
    int32_t score;            /* S of the pair */
    int32_t q_begin, q_end;   /* aligned query residues [q_begin, q_end), 0-based */
    int64_t subject;          /* subject index, as requested */
    int64_t s_begin, s_end;   /* aligned subject residues [s_begin, s_end), 0-based */
    int64_t n_ops;            /* operations written for this alignment */
} sw_alignment;

/*
 * sw_align - the optimal local alignment of one query against each of nsub
 * chosen subjects (Sec. II-B: a database search keeps alignments only for its
 * top-ranked subjects, recovered by tracing back from the cell holding S).
 *   h_query, qlen : as for sw_search (qlen <= 2^20).
 *   h_subjects    : host int64[nsub], subject indices 0..n-1 (repeats allowed).
 *   h_out         : host sw_alignment[nsub].
 *   h_ops         : host char[nsub * ops_stride]; alignment k's operations go
 *                   to h_ops[k * ops_stride ...], first aligned residue pair
 *                   first: 'M' = query and subject residue aligned, 'I' = query
 *                   residue against a gap, 'D' = subject residue against a gap.
 *                   A maximal run of k gap operations of one kind costs
 *                   Go + (k-1) * min(Go, Ge), the cost the recurrence charges.
 *   ops_stride    : >= qlen + the longest requested subject (SW_E_SIZE otherwise).
 * Among alignments of equal score the one returned ends at the first cell
 * with H = S in row-major order and, tracing back, prefers the diagonal, then
 * the horizontal gap (E), then the vertical gap (F), and a gap that opens
 * over one that extends.  S = 0 gives an empty alignment (all fields 0).
 * Synchronous: the work runs on `stream` and the call returns when the host
 * buffers are filled.  Device memory: about qlen x subject length bytes per
 * pair, in rounds of pairs that fit 4 GiB (a larger single pair runs alone).
 * A pair fills its matrix on one workgroup, or as tiles over the whole GPU
 * (pairs with both sides >= 2,048 residues by default; sw_pack_opts.align_tiles);
 * the alignment is the same either way.
 */
sw_status sw_align(const int8_t* h_query, int32_t qlen, sw_db* db, const int64_t* h_subjects, int32_t nsub,
                   const int8_t* h_subst, int32_t gap_open, int32_t gap_extend, sw_alignment* h_out, char* h_ops,
                   int64_t ops_stride, sw_stream stream);

/*
 * sw_align_batch - sw_align for several queries in one call, e.g. the top hits
 * of every query of a batched search (Sec. II-B).  Query q is
 * h_queries[h_qoffsets[q] .. h_qoffsets[q+1]) and is aligned against the
 * subjects h_subjects[h_soffsets[q] - h_soffsets[0] .. h_soffsets[q+1] -
 * h_soffsets[0]).  The pairs of all queries share the launches, longest
 * first, so many queries' alignments run at once; each result equals what
 * sw_align returns for that query and subject.
 *   h_qoffsets : host int64[nq + 1], non-decreasing; each query <= 2^20 residues.
 *   h_soffsets : host int64[nq + 1], non-decreasing, h_soffsets[0] >= 0;
 *                P = h_soffsets[nq] - h_soffsets[0] pairs.
 *   h_out      : host sw_alignment[P], in the order of h_subjects.
 *   h_ops      : host char[P * ops_stride], as for sw_align.
 *   ops_stride : >= query length + subject length for every pair (SW_E_SIZE).
 * Errors as for sw_align; nq = 0 does nothing.  Synchronous, with the same
 * device memory rounds as sw_align.
 */
sw_status sw_align_batch(const int8_t* h_queries, const int64_t* h_qoffsets, int32_t nq, sw_db* db,
                         const int64_t* h_subjects, const int64_t* h_soffsets, const int8_t* h_subst, int32_t gap_open,
                         int32_t gap_extend, sw_alignment* h_out, char* h_ops, int64_t ops_stride, sw_stream stream);

/*
 * sw_pair - the Smith-Waterman score (Eq. 1-3) of one pair of long sequences,
 * spread over the whole GPU (intra-task parallelism, Sec. II-B; one-to-one
 * alignment of long sequences, Sec. III-A).  The matrix is cut into tiles of
 * 256 query rows by 128 or 256 subject columns; the tiles of one
 * anti-diagonal are independent and run in one launch (one wave each), so a
 * pair of m x n residues takes about m/256 + n/256 launches and no
 * workgroup waits for another.  int32 cells.
 *   h_query, h_subject : host residue codes 0..alphabet-1 (validated).
 *   alphabet           : 0 (= 20) or 1..24;  h_subst : host int8[alphabet^2].
 *   d_score            : device int32, receives S (0 for an empty sequence).
 *   d_workspace        : device, 256-byte aligned, ws_bytes >= sw_pair_workspace_bytes
 *                        (about 8 (m + n) bytes plus the sequences); may be NULL when
 *                        either length is 0.
 * SW_E_UNSUPPORTED when 127 x min(m, n) could exceed int32.  Asynchronous on
 * the stream; the workspace must stay untouched until it completes.
 */
sw_status sw_pair_workspace_bytes(int64_t qlen, int64_t slen, int64_t* bytes);
sw_status sw_pair(const int8_t* h_query, int64_t qlen, const int8_t* h_subject, int64_t slen, int32_t alphabet,
                  const int8_t* h_subst, int32_t gap_open, int32_t gap_extend, int32_t* d_score,
                  void* d_workspace, int64_t ws_bytes, sw_stream stream);

/* Human-readable name of a status code (static string). */
const char* sw_status_str(sw_status s);
/* Description of the most recent error on the calling thread ("" if none). */
const char* sw_last_error(void);

/*
 * Execution statistics of the most recent search on the handle (read after the
 * stream has completed):
 *   out[0] = work items of the bulk 16-bit launch,  out[1] = (query, subject
 *   pair) entries flagged for the 32-bit recompute (saturated or, in the
 *   end-to-end modes, out of the exact range),  out[2] = rows per lane (R) of
 *   the bulk launch,  out[3] = persistent waves launched,  out[4] = work items
 *   of the side launch (long pairs of a short query),  out[5] = rows per lane
 *   of the side launch,  out[6] = pairs the 32-bit recompute computed (equals
 *   out[1] after every search),  out[7] = flagged pairs beyond the recompute
 *   list's capacity (recomputed from their flag bits).
 * This call synchronises the handle's device.
 */
sw_status sw_last_stats(sw_db* db, int64_t out[8]);

/*
 * Kernel timing for benchmarks.  When enabled, every search on the handle
 * records a pair of HIP events on the caller's stream around its 16-bit sweep
 * launch (the dominant kernel).  sw_kernel_times synchronises the handle's
 * device, writes up to cap elapsed times in milliseconds (oldest first) to
 * ms_out, sets *count to the number written and forgets them.  At most 4096
 * launches are remembered; older ones are dropped.
 */
sw_status sw_profile_kernels(sw_db* db, int32_t enable);
sw_status sw_kernel_times(sw_db* db, float* ms_out, int32_t cap, int32_t* count);

#ifdef __cplusplus
}
#endif
#endif /* SWSEARCH_H */
