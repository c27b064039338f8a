// kernels.h -- host-visible launch interfaces of the kernel translation units.
// Only the library's own sources include this header.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

// Arguments of the fused scorer and the unfused comparator (device pointers).
struct FusedParams {
  const char* q_tok;
  const int64_t* q_off;
  const float* q_scales;
  int64_t n_q;
  const char* d_tok;
  const int64_t* d_off;
  const float* d_scales;
  int64_t n_docs;
  const int64_t* cand_off;  // nullptr: every query against every doc
  const int32_t* cand_ids;
  float* scores;
  int64_t n_pairs;           // number of (query, doc) scores
  int64_t tokens_per_query;  // d_off[n_docs] (host copy)
  int32_t dim;
  int32_t nch;        // ceil(dim / DCH): d-chunks per row
  int32_t row_bytes;  // dim * element size (row stride in HBM)
  // Query units: without candidate lists a unit is `group` consecutive
  // queries that share every document tile read (query a of unit u is
  // u * group + a, its tokens in blocks a * bpq .. a * bpq + bpq - 1 of 16);
  // with candidate lists a unit is one query (group 1, bpq = query blocks).
  int32_t group;
  int32_t bpq;
  // 64-byte column groups of a query row in LDS: nch * DCH * element size /
  // 64 (the row zero-extended to whole chunks)
  int32_t ncg;
  int64_t n_units;   // ceil(n_q / group)
  int64_t n_upairs;  // work pairs: n_units * n_docs, or the candidate count
  // Fused top-k (topk_k > 0): a score is not stored; its ranking key goes to
  // LDS at byte lds_keys_off of the dynamic LDS (key_cap slots): one array
  // indexed from the workgroup's first pair when its whole range fits, else
  // the slots of the wave that computed it (key_cap / NW per wave), or
  // key_spill[pair * group + query of the unit] when the wave's range does
  // not fit either; after its
  // waves finish, the workgroup writes the top-k keys of each query's part of
  // its range to slot (workgroup + unit) * group + query of part_keys (k keys)
  // and part_cnt, and its first work pair to wg_lo[workgroup].
  int32_t topk_k;
  int32_t sel_cap;       // sort-buffer keys of the selection (power of two >= max(k, 64))
  int32_t key_cap;       // LDS key slots of the workgroup (a multiple of its wave count)
  int32_t lds_keys_off;  // bytes; the wave ranges follow the key slots
  uint32_t* key_spill;   // [n_upairs * group]
  int64_t* wg_lo;        // [grid]
  uint64_t* part_keys;   // [(grid + n_units) * group * topk_k]
  uint32_t* part_cnt;    // [(grid + n_units) * group]
};

// Merge of the fused scorer's per-workgroup top-k parts (one workgroup per
// query): the k best keys of every part that covers the query.
struct MergeParams {
  const int64_t* cand_off;  // nullptr: every query against every doc
  int64_t n_q;
  int64_t n_docs;
  int64_t n_upairs;
  int32_t group;
  int32_t grid;  // workgroups of the scoring launch
  int32_t k;
  int32_t pad;
  const int64_t* wg_lo;
  const uint64_t* part_keys;
  const uint32_t* part_cnt;
  float* out_scores;  // [n_q * k]
  int32_t* out_ids;   // [n_q * k]
};
// LDS bytes the fused scorer's top-k epilogue needs at offset 0 (it reuses
// the query and ring area once every wave has finished), for a sort buffer
// of sel_cap keys.
size_t fused_topk_scratch_bytes(int sel_cap);
constexpr int MERGE_MAX_GRID = 4096;
hipError_t launch_topk_merge(const MergeParams& M, hipStream_t s);

typedef hipError_t (*fused_launch_fn)(const FusedParams&, int grid, size_t lds, hipStream_t);
typedef int (*fused_occ_fn)(size_t lds);
struct FusedFns {
  fused_launch_fn launch;
  fused_occ_fn occupancy;
  bool stage;
};

// dt: maxsim_dtype; nqb: query blocks of 16 (1, 2, 4, 8); dch: 64, 128 or 256;
// pf: prefetch depth (2, 3, 4); nw: waves per workgroup (4, 8); qm: where the
// query operand lives (0: one LDS copy per workgroup, 1: VGPRs, d in one
// chunk; 2: one LDS copy per wave);
// stage: document tiles arrive through a per-wave LDS ring (pf slots of
// 16 rows x dch elements per wave, after the query block) instead of VGPRs.
// rt: document rows per step (16; 32 for FP8 with staged tiles and Q in VGPRs).
FusedFns fused_kernel_fns(int dt, int nqb, int dch, int pf, int nw, int qm, bool stage, int rt);

hipError_t launch_unfused(int dt, int nqb, int dch, const FusedParams& P, float* S, int cus,
                          size_t lds, hipStream_t s);

// ---- PQ ----
struct PqParams {
  const char* q_tok;  // F16 or F32 query tokens
  const int64_t* q_off;
  int64_t n_q;
  int32_t q_f32;     // 1: FP32 query tokens, 0: FP16
  int32_t cb_f32;    // 1: FP32 codebooks, 0: FP16
  const void* codebooks;  // [M, K, dsub]
  const uint8_t* codes;   // [T, M]
  const int64_t* d_off;
  int64_t n_docs;
  const int64_t* cand_off;
  const int32_t* cand_ids;
  float* scores;    // final scores
  float* partial;   // [n_slices, n_pairs] when n_slices > 1, else nullptr
  int64_t n_pairs;
  int64_t tokens_per_query;
  int32_t M, K, dsub, dim;
  int32_t qt;        // query tokens per slice (LUT rows)
  int32_t n_slices;  // ceil(max Nq / qt)
  int32_t n_chunks;  // doc-range chunks per (query, slice) or per query group
  int32_t nw;        // waves per workgroup (8 or 16)
  // decode-into-MFMA variant only
  int32_t bpq;    // 16-column query blocks per query (ceil(max Nq / 16))
  int32_t group;  // queries per work item
  int32_t nqb;    // query blocks per wave (group * bpq)
  int32_t pad;
};
hipError_t launch_pq(const PqParams& P, int max_nq, hipStream_t s);
// Decode-into-MFMA PQ scorer: F16 queries and codebooks, dsub in {8, 16, 32};
// lds = M * K * dsub * 2 bytes; nqb in {1, 2, 4, 8} with nqb * M * dsub <= 1024.
hipError_t launch_pq_mfma(const PqParams& P, size_t lds, hipStream_t s);

// ---- residual-compressed documents ----
struct ResParams {
  const void* q_tok;  // F16 [n_qtok, dim]
  const int64_t* q_off;
  int64_t n_q;
  int64_t n_qtok;         // q_off[n_q] (host copy)
  const void* centroids;  // F16 [n_centroids, dim]
  int64_t n_centroids;
  const void* weights;  // F16 [2^nbits]
  const int32_t* ids;   // [T] centroid id per document token
  const uint8_t* residuals;  // [T, dim * nbits / 8] packed codes
  const int64_t* d_off;
  int64_t n_docs;
  const int64_t* cand_off;
  const int32_t* cand_ids;
  float* scores;
  float* table;  // workspace: [n_centroids, n_cols] FP32
  const char* zero_row;  // set by launch_residual: 1 KiB of device zeros
  int64_t n_cols;        // n_q * 16 * nqb: each query owns 16 * nqb columns
  int32_t dim;    // 64, 128 or 256
  int32_t nbits;  // 1, 2 or 4
  int32_t nqb;    // 16-column query blocks (1, 2, 4)
  int32_t n_chunks;  // document-range chunks per query
  int32_t pipe;      // load-pipeline variant, 0 .. RES_PIPES - 1
  int32_t pad;
};
constexpr int RES_PIPES = 4;
// Builds the centroid-query table, then scores (grid n_q * n_chunks).
hipError_t launch_residual(const ResParams& P, hipStream_t s);

// ---- top-k ----
hipError_t launch_topk(const float* scores, const int64_t* seg_off, int64_t n_seg, int64_t n_total,
                       const int32_t* ids, int k, float* out_scores, int32_t* out_ids, void* ws,
                       hipStream_t s);
size_t topk_ws_bytes(int64_t n_seg, int k);

// ---- input conversion ----
hipError_t launch_quantize(const float* src, int64_t n_tokens, int dim, int dt, void* dst,
                           float* scales, hipStream_t s);

// ---- measured read ceiling ----
hipError_t launch_stream_probe(const void* buf, size_t bytes, int variant, uint32_t* sink,
                               int grid, hipStream_t s);
// ---- measured LDS gather ceiling (grid: one workgroup of 16 waves per CU) ----
hipError_t launch_lds_probe(const void* buf, size_t bytes, int variant, int table_bytes,
                            uint32_t* sink, int grid, hipStream_t s);

// ---- device-side input checks (flags: caller's device int32) ----
hipError_t launch_clear_flags(int32_t* flags, hipStream_t s);
hipError_t launch_check_offsets(const int64_t* off, int64_t n, int64_t n_tokens, int max_len,
                                int bit_off, int bit_len, int32_t* flags, hipStream_t s);
hipError_t launch_check_ids(const int32_t* ids, int64_t n, int64_t n_docs, int bit,
                            int32_t* flags, hipStream_t s);
hipError_t launch_check_scales(const float* sc, int64_t n, int bit, int32_t* flags, hipStream_t s);
hipError_t launch_check_codes(const uint8_t* codes, int64_t n, int K, int bit, int32_t* flags,
                              hipStream_t s);

// ---- device properties ----
int device_cu_count();
