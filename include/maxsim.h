/*
 * maxsim.h -- C ABI of the MI355X (gfx950) TileMaxSim scoring library.
 *
 * The library implements late-interaction MaxSim scoring (Eq. (1) of
 * "TileMaxSim: IO-Aware GPU MaxSim Scoring with Dimension Tiling and Fused
 * Product Quantization", arXiv 2606.26439):
 *
 *     score(Q, D) = sum_{i < Nq} max_{j < Nd} q_i . d_j
 *
 * fused so that every document token is read from HBM once (Sec. 3.2.3 and
 * Theorem 1), with 128-wide dimension chunks accumulated in FP32 before the
 * max (Evaluation, "Embedding Dimension Scaling"), PQ scoring through
 * per-query lookup tables held in LDS (Sec. 4.2-4.3), top-k selection, the
 * unfused comparator that materialises S = Q D^T (Sec. 2.3, Eq. io_naive),
 * and the per-token input conversion the precision forms need.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Every data pointer is a DEVICE pointer (HBM of the current HIP device)
 *   owned by the caller. The library never frees or retains it beyond the
 *   stream-ordered work it enqueues. Descriptor structs are HOST memory and
 *   are read only during the call.
 * - Calls are asynchronous on `stream` (a hipStream_t; NULL = the null
 *   stream). Host-visible argument errors return a non-zero status BEFORE
 *   anything is enqueued; MAXSIM_EHIP reports a failed launch.
 * - Token sets are CSR-packed: tokens[n_tokens, dim] row-major, row stride
 *   dim * element_size bytes, base address 16-byte aligned; set s owns rows
 *   offsets[s] .. offsets[s+1]-1, offsets[0] = 0 and non-decreasing (int64).
 * - Scores are FP32. A document with no tokens scores -inf (a max over an
 *   empty set); a query with no tokens scores 0 (an empty sum). Each score is
 *   produced by exactly one wavefront with a fixed reduction order, so
 *   results are bit-reproducible run to run and independent of batching.
 * - The error text of the last failing call on the calling thread is
 *   returned by maxsim_last_error().
 */
#ifndef MAXSIM_H
#define MAXSIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MAXSIM_ABI_VERSION 1

typedef void* maxsim_stream_t; /* hipStream_t */

typedef enum {
  MAXSIM_OK = 0,
  MAXSIM_EINVAL = 1,       /* bad pointer, size, alignment or inconsistent descriptor */
  MAXSIM_EUNSUPPORTED = 2, /* valid request outside what the kernels handle */
  MAXSIM_EWORKSPACE = 3,   /* workspace missing or smaller than *_workspace_size() */
  MAXSIM_EHIP = 4,         /* a HIP runtime call or kernel launch failed */
  MAXSIM_EDEVCHECK = 5     /* maxsim_check found device-side input violations */
} maxsim_status;

typedef enum {
  MAXSIM_F32 = 0,
  MAXSIM_BF16 = 1,
  MAXSIM_F16 = 2,
  MAXSIM_F8E4M3 = 3 /* OCP E4M3FN codes with one FP32 power-of-two scale per token */
} maxsim_dtype;

/*
 * A CSR set of token-vector sets (documents or queries). Q in R^{Nq x d} and
 * D in R^{Nd x d} of Eq. (1), one set each.
 *   dtype     element type of `tokens`.
 *   dim       d; a multiple of 16, 16 <= dim <= 1024 (the kernels work in
 *             d-chunks of 64, 128 or 256 and zero-extend the last chunk, which
 *             adds exact zeros: the scores equal those of the zero-padded rows).
 *   n_sets    number of sets; n_tokens = offsets[n_sets] (host copies, so the
 *             library needs no device-to-host read).
 *   max_len   host upper bound on tokens per set. For queries it selects the
 *             kernel's query-token capacity and must be <= 64; a query that
 *             exceeds it on the device gets NaN scores.
 *   scales    FP8 only: [n_tokens] FP32 per-token scales, each a normal power
 *             of two; the token's value is code * scale. NULL otherwise.
 * Token values must be finite: a NaN or infinite element gives unspecified
 * scores for the sets it meets (never an out-of-bounds access).
 */
typedef struct {
  int32_t dtype;
  int32_t dim;
  int64_t n_sets;
  int64_t n_tokens;
  int32_t max_len;
  int32_t reserved;
  const void* tokens;
  const int64_t* offsets;
  const float* scales;
} maxsim_csr;

/*
 * Candidate lists: query a is scored against documents
 * doc_ids[offsets[a] .. offsets[a+1]-1] (int32 ids into the document set);
 * n_total = offsets[n_queries] on the host. A NULL maxsim_candidates* means
 * every query against every document, scores laid out [n_queries, n_docs].
 * Ids outside [0, n_docs) are the caller's error (not checked on device).
 */
typedef struct {
  const int64_t* offsets;
  const int32_t* doc_ids;
  int64_t n_total;
} maxsim_candidates;

/*
 * PQ-compressed documents (Sec. 4.1): token t is the concatenation over
 * m < M of centroid codebooks[m, codes[t, m], :] (dsub values each), so
 * dim = M * dsub.
 *   M in {4, 8, 16}; 1 <= K <= 256; 1 <= dsub <= 32.
 *   cb_dtype MAXSIM_F16 or MAXSIM_F32 for codebooks[M, K, dsub].
 *   codes [n_tokens, M] uint8; offsets [n_docs + 1] int64 as for maxsim_csr.
 */
typedef struct {
  int32_t M;
  int32_t K;
  int32_t dsub;
  int32_t cb_dtype;
  const void* codebooks;
  const uint8_t* codes;
  const int64_t* offsets;
  int64_t n_docs;
  int64_t n_tokens;
} maxsim_pq_docs;

/*
 * Residual-compressed documents (the centroid plus quantized-residual form of
 * the PLAID/WARP indexes named in the paper's Related Work and WARP
 * comparison): token t is
 *   x_t[k] = centroids[centroid_ids[t], k] + weights[code(t, k)],
 * where code(t, k) is the nbits-wide field at bit k * nbits of row t of
 * `residuals` (row_bytes = dim * nbits / 8; fields fill each byte from its
 * least significant bit up).
 *   dim in {64, 128, 256}; nbits in {1, 2, 4}; 1 <= n_centroids < 2^24.
 *   centroids    [n_centroids, dim] F16, 16-byte aligned.
 *   weights      [2^nbits] F16: the residual value of each code.
 *   centroid_ids [n_tokens] int32; ids outside [0, n_centroids) are the
 *                caller's error (the kernel clamps them, so they only give
 *                wrong scores; maxsim_validate_residual detects them).
 *   residuals    [n_tokens, row_bytes] uint8, 16-byte aligned.
 *   offsets      [n_docs + 1] int64 as for maxsim_csr.
 */
typedef struct {
  int32_t dim;
  int32_t nbits;
  int64_t n_centroids;
  const void* centroids;
  const void* weights;
  const int32_t* centroid_ids;
  const uint8_t* residuals;
  const int64_t* offsets;
  int64_t n_docs;
  int64_t n_tokens;
} maxsim_residual_docs;

int maxsim_abi_version(void);
const char* maxsim_last_error(void);

/*
 * Input preparation for the precision forms (Evaluation, "Precision"; FP8 is
 * this library's addition). Converts src[n_tokens, dim] FP32 into `dtype`:
 *   BF16 / F16: round to nearest even per element; `scales` must be NULL.
 *   F8E4M3: per token, s = 2^k with k the smallest integer such that
 *           max_u |x_u| <= 448 * 2^k (s = 1 for an all-zero token), written to
 *           scales[t]; codes = E4M3FN(x / s), round to nearest even.
 *   F32: plain copy.
 * dim: a multiple of 16, 16 <= dim <= 1024 (else MAXSIM_EUNSUPPORTED).
 * dst has n_tokens * dim elements of `dtype`.
 */
maxsim_status maxsim_quantize(const float* src, int64_t n_tokens, int32_t dim, int32_t dtype,
                              void* dst, float* scales, maxsim_stream_t stream);

/*
 * Fused MaxSim (Algorithm 3, "V2-MQ", with BQ = Nq so each document byte is
 * read once; Theorem 1). Many queries of uneven Nq (<= 64) against ragged
 * documents in one persistent launch.
 *   queries, docs  same dtype and dim. For F8E4M3 both carry scales; S_ij is
 *                  scaled by s_q[i] * s_d[j] (exact, powers of two).
 *   cand           NULL: scores[a * n_docs + b]; else scores[p] for each pair
 *                  index p of the candidate lists.
 *   workspace      maxsim_score_workspace_size() bytes (may be 0 -> NULL ok).
 */
size_t maxsim_score_workspace_size(const maxsim_csr* queries, const maxsim_csr* docs,
                                   const maxsim_candidates* cand);
maxsim_status maxsim_score(const maxsim_csr* queries, const maxsim_csr* docs,
                           const maxsim_candidates* cand, float* scores, void* workspace,
                           size_t ws_bytes, maxsim_stream_t stream);

/*
 * Unfused comparator (Sec. 2.1 two-step decomposition, Eq. io_naive): first
 * S = D Q^T for every document token and query token, written to HBM in FP32
 * inside `workspace`, then a second kernel reads S back for the max over
 * document tokens and the sum over query tokens. Same arguments and results
 * as maxsim_score; candidates are not supported (EUNSUPPORTED).
 * The workspace size is n_q * n_tokens * (16-column blocks of max_len) * 64
 * bytes; when that overflows size_t the size call returns SIZE_MAX and the
 * scoring call EUNSUPPORTED.
 */
size_t maxsim_score_unfused_workspace_size(const maxsim_csr* queries, const maxsim_csr* docs);
maxsim_status maxsim_score_unfused(const maxsim_csr* queries, const maxsim_csr* docs,
                                   float* scores, void* workspace, size_t ws_bytes,
                                   maxsim_stream_t stream);

/*
 * Fused PQ scoring (Sec. 4.2-4.3): per query, the table
 * T[i, m, k] = q_i[m*dsub:(m+1)*dsub] . C[m, k] is built in LDS (FP32), then
 * each document token scores sum_m T[i, m, c_jm], followed by the running
 * max over tokens and the sum over query tokens. Codes are read from HBM;
 * decompressed vectors are never written.
 *   queries  dtype F16 or F32, dim = M * dsub, max_len <= 64.
 *   cand     as for maxsim_score.
 */
size_t maxsim_pq_score_workspace_size(const maxsim_csr* queries, const maxsim_pq_docs* docs,
                                      const maxsim_candidates* cand);
maxsim_status maxsim_pq_score(const maxsim_csr* queries, const maxsim_pq_docs* docs,
                              const maxsim_candidates* cand, float* scores, void* workspace,
                              size_t ws_bytes, maxsim_stream_t stream);

/*
 * MaxSim over residual-compressed documents: Eq. (1) on the decoded tokens,
 * computed as q_i . x_j = q_i . C[id_j] + q_i . r_j. The call first builds
 * the table P[c, i] = C[c] . q_i (FP32, every centroid against every query
 * token of the batch) in `workspace`; the fused scorer then reads each
 * token's id and packed residual once, gathers P[id_j, i], decodes the
 * residual in registers and adds q_i . r_j before the max over tokens and the
 * sum over query tokens. Decoded vectors are never written.
 *   queries    F16, same dim, max_len <= 64. Each query owns
 *              W = 16 * nqb table columns, nqb = ceil(max_len / 16) rounded
 *              up to a power of two; n_centroids and n_queries * W must stay
 *              below 2^24 and their product below 2^32 (else
 *              MAXSIM_EUNSUPPORTED).
 *   cand       as for maxsim_score.
 *   workspace  maxsim_residual_score_workspace_size() bytes:
 *              n_centroids * n_queries * W * 4, rounded up to 256.
 */
size_t maxsim_residual_score_workspace_size(const maxsim_csr* queries,
                                            const maxsim_residual_docs* docs,
                                            const maxsim_candidates* cand);
maxsim_status maxsim_residual_score(const maxsim_csr* queries, const maxsim_residual_docs* docs,
                                    const maxsim_candidates* cand, float* scores,
                                    void* workspace, size_t ws_bytes, maxsim_stream_t stream);

/*
 * Top-k per segment (the torch.topk step of the paper's end-to-end pipeline,
 * Evaluation "End-to-End Retrieval Latency"). Segment s is
 * scores[seg_offsets[s] .. seg_offsets[s+1]-1]; ids (int32, same indexing)
 * name the entries, or NULL for the index within the segment. Output rows
 * out_scores[s * k ..], out_ids[s * k ..] hold the k best entries ordered by
 * score descending, then id ascending (exact, deterministic); a segment with
 * fewer than k entries is padded with score -inf and id -1. NaN ranks below
 * -inf. 1 <= k <= 1024; n_total = seg_offsets[n_segments] (host copy).
 */
size_t maxsim_topk_workspace_size(int64_t n_segments, int32_t k);
maxsim_status maxsim_topk(const float* scores, const int64_t* seg_offsets, int64_t n_segments,
                          int64_t n_total, const int32_t* ids, int32_t k, float* out_scores,
                          int32_t* out_ids, void* workspace, size_t ws_bytes,
                          maxsim_stream_t stream);

/*
 * Fused scoring with the top-k in the scorer's epilogue (the retrieval step
 * of the paper's end-to-end pipeline, Evaluation "End-to-End Retrieval
 * Latency", for the whole collection as in the large-scale extrapolation):
 * the same scores as maxsim_score, but none is stored. Each workgroup of the
 * scoring launch keeps its scores' ranking keys on chip and selects the k best
 * of each query's share of its range (exact radix select); a second, small
 * launch merges the per-workgroup parts of every query.
 *   queries, docs, cand  as for maxsim_score.
 *   k                    1 <= k <= 1024.
 *   out_scores, out_ids  [n_queries * k] device arrays: row a holds query a's
 *                        k best documents by score descending, then id
 *                        ascending, padded with (-inf, -1); ids are document
 *                        indices, or the candidate ids with candidate lists.
 *                        Bit-identical to maxsim_score followed by
 *                        maxsim_topk over per-query segments (ids NULL, or the
 *                        candidate doc_ids).
 *   workspace            maxsim_score_topk_workspace_size() bytes, 16-byte
 *                        aligned, contents ignored: per-workgroup parts and a
 *                        4-byte key per (query, document) pair for workgroups
 *                        whose range does not fit their LDS (SIZE_MAX: too
 *                        large for the address space).
 * Errors: as maxsim_score; k out of range -> MAXSIM_EINVAL; workspace short
 * -> MAXSIM_EWORKSPACE. Asynchronous on `stream` (two launches).
 */
size_t maxsim_score_topk_workspace_size(const maxsim_csr* queries, const maxsim_csr* docs,
                                        const maxsim_candidates* cand, int32_t k);
maxsim_status maxsim_score_topk(const maxsim_csr* queries, const maxsim_csr* docs,
                                const maxsim_candidates* cand, int32_t k, float* out_scores,
                                int32_t* out_ids, void* workspace, size_t ws_bytes,
                                maxsim_stream_t stream);

/*
 * maxsim_score_topk for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same two launches and the same results, bit for bit, with
 * the workspace taken from a fixed scratch array of
 * MAXSIM_NOALLOC_SCRATCH_BYTES that the library holds on each GPU it runs on
 * until the process ends. The call allocates nothing; the caller still owns
 * the queries, documents, candidates and outputs (as for maxsim_score_topk).
 *   queries, docs, cand, k, out_scores, out_ids, stream
 *                        as for maxsim_score_topk.
 * Errors: as maxsim_score_topk; a problem whose
 * maxsim_score_topk_workspace_size() exceeds MAXSIM_NOALLOC_SCRATCH_BYTES ->
 * MAXSIM_EWORKSPACE (nothing enqueued). The scratch needs no clearing
 * between calls (every word a launch reads was written earlier in the same
 * call) and keeps the last call's contents. All calls on one GPU share its
 * scratch: calls that overlap on one GPU (on different streams, or from
 * different host threads without ordering) race and give undefined results.
 */
#define MAXSIM_NOALLOC_SCRATCH_BYTES (64u * 1024u * 1024u)
maxsim_status maxsim_score_topk_noalloc(const maxsim_csr* queries, const maxsim_csr* docs,
                                        const maxsim_candidates* cand, int32_t k,
                                        float* out_scores, int32_t* out_ids,
                                        maxsim_stream_t stream);

/*
 * Tile/launch-shape autotuner (Evaluation, "Tile Size Sensitivity"): times
 * every candidate launch configuration of the fused kernel on the given
 * problem with HIP events (synchronises `stream`), keeps the fastest for the
 * key (dtype, dim, query-token capacity), and, if cache_path is not NULL,
 * rewrites that JSON file with every tuned key. maxsim_score then uses the
 * tuned configuration for matching keys. Writes a one-line JSON report of
 * the timings to report (if not NULL, up to report_len bytes).
 */
maxsim_status maxsim_autotune(const maxsim_csr* queries, const maxsim_csr* docs,
                              const maxsim_candidates* cand, float* scores, void* workspace,
                              size_t ws_bytes, maxsim_stream_t stream, int32_t reps,
                              const char* cache_path, char* report, size_t report_len);
/* Loads tuned configurations written by maxsim_autotune,
 * maxsim_pq_autotune or maxsim_residual_autotune (missing file: OK, no-op). */
maxsim_status maxsim_load_tune_cache(const char* cache_path);

/*
 * PQ scorer choice (Sec. 4.3 Phase 2, and the same scores through the ADC
 * identity of Sec. 4.2): maxsim_pq_score runs either the per-query table
 * kernel (variant 0) or a decode-into-MFMA kernel (variant 1: the codebooks
 * sit in LDS, each 16-token document tile is rebuilt from them into matrix
 * operands and contracted with up to 8 x 16 query tokens per wave). Variant 1
 * applies to F16 queries and codebooks with dsub in {8, 16, 32} and
 * 16 * ceil(max_len / 16) * dim <= 1024 after rounding the block count up to
 * a power of two; untuned keys use it whenever it applies. This call times
 * both (synchronises `stream`) on the given problem, keeps the faster for the
 * key (M, dsub, query blocks, candidates or not), rewrites cache_path (if not
 * NULL) and writes a one-line JSON report. Workspace as for maxsim_pq_score
 * with the table kernel (trials that need more are skipped).
 */
maxsim_status maxsim_pq_autotune(const maxsim_csr* queries, const maxsim_pq_docs* docs,
                                 const maxsim_candidates* cand, float* scores, void* workspace,
                                 size_t ws_bytes, maxsim_stream_t stream, int32_t reps,
                                 const char* cache_path, char* report, size_t report_len);

/*
 * Residual scorer tuning: the fused residual kernel keeps a ring of document
 * tiles in flight (centroid ids loaded several tiles ahead of the table
 * gathers they address, which run ahead of the matrix work); this call times
 * each ring shape on the given problem (synchronises `stream`), keeps the
 * fastest for the key (nbits, dim, query blocks, candidates or not),
 * rewrites cache_path (if not NULL) with every tuned key and writes a
 * one-line JSON report. Workspace as for maxsim_residual_score.
 */
maxsim_status maxsim_residual_autotune(const maxsim_csr* queries,
                                       const maxsim_residual_docs* docs,
                                       const maxsim_candidates* cand, float* scores,
                                       void* workspace, size_t ws_bytes, maxsim_stream_t stream,
                                       int32_t reps, const char* cache_path, char* report,
                                       size_t report_len);

/*
 * Device-side input checks. The scoring calls trust what lives in device
 * memory (reading it on the host would cost a device-to-host copy per call),
 * so a caller can check it once, e.g. when a document pool is built or before
 * a batch is scored. maxsim_validate enqueues, on `stream`, kernels that clear
 * *flags (a device int32 owned by the caller) and then OR into it one bit per
 * violated rule:
 *   MAXSIM_CHECK_DOC_OFFSETS    docs->offsets: offsets[0] == 0, non-decreasing,
 *                               offsets[n_sets] == n_tokens
 *   MAXSIM_CHECK_QUERY_OFFSETS  the same for queries
 *   MAXSIM_CHECK_QUERY_LENGTH   a query longer than queries->max_len
 *   MAXSIM_CHECK_CAND_OFFSETS   cand->offsets: 0 first, non-decreasing, n_total last
 *   MAXSIM_CHECK_CAND_IDS       a candidate id outside [0, n_docs)
 *   MAXSIM_CHECK_FP8_SCALES     an FP8 token scale that is not a normal power of two
 *   MAXSIM_CHECK_PQ_CODES       a PQ code >= K
 *   MAXSIM_CHECK_CENTROID_IDS   a residual document's centroid id outside
 *                               [0, n_centroids)
 * queries and cand may be NULL (not checked). Every access stays inside the
 * declared array sizes whatever the contents. maxsim_validate_pq does the same
 * for PQ documents (offsets and codes), maxsim_validate_residual for
 * residual-compressed documents (offsets and centroid ids). maxsim_check synchronises `stream`,
 * reads *flags and returns MAXSIM_EDEVCHECK, with the violated rules named in
 * maxsim_last_error(), if any bit is set (MAXSIM_OK otherwise).
 */
#define MAXSIM_CHECK_DOC_OFFSETS 1
#define MAXSIM_CHECK_QUERY_OFFSETS 2
#define MAXSIM_CHECK_QUERY_LENGTH 4
#define MAXSIM_CHECK_CAND_OFFSETS 8
#define MAXSIM_CHECK_CAND_IDS 16
#define MAXSIM_CHECK_FP8_SCALES 32
#define MAXSIM_CHECK_PQ_CODES 64
#define MAXSIM_CHECK_CENTROID_IDS 128
maxsim_status maxsim_validate(const maxsim_csr* queries, const maxsim_csr* docs,
                              const maxsim_candidates* cand, int32_t* flags,
                              maxsim_stream_t stream);
maxsim_status maxsim_validate_pq(const maxsim_csr* queries, const maxsim_pq_docs* docs,
                                 const maxsim_candidates* cand, int32_t* flags,
                                 maxsim_stream_t stream);
maxsim_status maxsim_validate_residual(const maxsim_csr* queries,
                                       const maxsim_residual_docs* docs,
                                       const maxsim_candidates* cand, int32_t* flags,
                                       maxsim_stream_t stream);
maxsim_status maxsim_check(const int32_t* flags, maxsim_stream_t stream);

/*
 * Measured HBM read ceiling (for reporting the scorers against what the
 * device sustains as well as against its published peak; the paper reports
 * utilisation against the published peak, Evaluation "Memory Bandwidth
 * Utilization"). Streams `bytes` of buf (16-byte aligned; whole 4 KiB tiles
 * are read) with 16-byte loads, one contiguous share per wave, and writes one
 * XOR checksum per wave to sink (sink_len >= 4 entries; the grid is
 * min(sink_len / 4, 8 * CUs) workgroups of 4 waves).
 *   variant 0: lane-contiguous loads; 1: the same, non-temporal;
 *           2: the fused scorer's 16-row tile pattern; 3: the same,
 *           non-temporal; 4: lane-contiguous non-temporal loads straight
 *           into LDS, read back from LDS; 5: variant 4 with 4 KiB tiles
 *           dealt round-robin to the waves instead of one share per wave.
 */
maxsim_status maxsim_stream_probe(const void* buf, size_t bytes, int32_t variant, uint32_t* sink,
                                  int64_t sink_len, maxsim_stream_t stream);

/*
 * Measured LDS gather ceiling, the bound of the PQ scorers: the table kernel
 * gathers lookup-table entries from LDS (Sec. 4.3 Phase 2) and the
 * decode-into-MFMA kernel gathers codebook rows (the ADC identity, Sec. 4.2).
 * One workgroup of 16 waves per CU (grid min(sink_len / 16, CUs)) fills a
 * table of table_bytes (65536 or 131072) in LDS, then streams `bytes` of
 * buf (16-byte aligned; whole 1 KiB units, non-temporal) and turns every
 * 4-byte word into 8 table indices, each read by one LDS instruction:
 *   variant 0: random 4-byte reads, 4 passes per word (128 reads per lane per
 *              16 bytes streamed);
 *   variant 1: random 16-byte reads (32 per lane per 16 bytes);
 *   variant 2: 16-byte reads whose 16 lanes per quarter-wave hit 16 distinct
 *              16-byte bank groups (conflict-free; 32 per lane per 16 bytes).
 * Writes one XOR checksum per wave to sink (sink_len >= 16). Time it with
 * events: reads = bytes / 16 * (variant 0 ? 128 : 32).
 */
maxsim_status maxsim_lds_probe(const void* buf, size_t bytes, int32_t variant,
                               int32_t table_bytes, uint32_t* sink, int64_t sink_len,
                               maxsim_stream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* MAXSIM_H */
