/*
 * maxsim_oracle.c -- plain, slow, single-threaded FP64 reference for the
 * TileMaxSim hot path (arXiv 2606.26439).
 *
 * THIS IS TEST INFRASTRUCTURE. Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it. The GPU library shares no
 * code, header, table or helper with this file, and this file includes
 * nothing from the GPU library.
 *
 * Every function follows the paper's definitions directly, with no blocking,
 * fusion or reordering:
 *   - oracle_maxsim        : Eq. (1), MaxSim(Q,D) = sum_i max_j q_i . d_j
 *                            (Background, "Multi-Vector Retrieval and MaxSim").
 *                            The fused kernels only change memory-access order
 *                            and the d>128 variant only splits the dot product
 *                            into 128-wide partial sums (Evaluation, "Embedding
 *                            Dimension Scaling"), so Eq. (1) is the exact
 *                            target for every plain path.
 *   - oracle_pq_decode     : the "Decompress" step of the PQ pipeline (Sec. 4.1):
 *                            a token's vector is the concatenation of its M
 *                            selected centroids.
 *   - oracle_pq_lut_build  : Phase 1 of Sec. 4.3, the distance table
 *                            T[i,m,k] = q_i[m*dsub:(m+1)*dsub] . C[m,k].
 *   - oracle_pq_lut_score  : Phase 2 of Sec. 4.3: s_ij = sum_m T[i,m,c_jm],
 *                            running max over j, sum over i.
 *   - oracle_residual_decode: centroid plus per-dimension quantized residual
 *                            (the compressed form of the PLAID/WARP indexes
 *                            named in Related Work); scoring then applies
 *                            Eq. (1) to the decoded vectors.
 *   - oracle_topk          : order by (score descending, id ascending), keep k.
 *   - oracle_round_*       : IEEE-style round-to-nearest-even into binary16,
 *                            bfloat16 and OCP FP8 E4M3FN, written from the
 *                            formats' definitions (precision of the inputs,
 *                            Evaluation "Precision").
 *   - oracle_quant_e4m3    : per-token power-of-two scale s with
 *                            amax <= 448*s minimal, then E4M3FN(x/s).
 *
 * Conventions where the paper is silent:
 *   - a document with no tokens has max over an empty set = -inf, so its
 *     score is -inf when the query has at least one token;
 *   - a query with no tokens has an empty sum, score 0;
 *   - candidate lists select documents by id; NULL means every document.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

int oracle_abi_version(void) { return 1; }

/* ------------------------------------------------------------------ */
/* Eq. (1): MaxSim over CSR-packed token sets.                         */
/* ------------------------------------------------------------------ */

/* score(Q, D) for one query token set and one document token set. */
static double maxsim_one(const double* q, int64_t nq, const double* d, int64_t nd,
                         int32_t dim) {
  double total = 0.0;
  for (int64_t i = 0; i < nq; ++i) {
    double best = -INFINITY;
    for (int64_t j = 0; j < nd; ++j) {
      double dot = 0.0;
      for (int32_t k = 0; k < dim; ++k) dot += q[i * dim + k] * d[j * dim + k];
      if (dot > best) best = dot;
    }
    total += best;
  }
  return total;
}

/*
 * Queries: q_tok[q_off[n_q], dim], query a owns rows q_off[a] .. q_off[a+1]-1.
 * Docs:    d_tok[d_off[n_docs], dim], doc b owns rows d_off[b] .. d_off[b+1]-1.
 * Candidates: if cand_off is NULL, every query is scored against every doc and
 *   scores[a * n_docs + b] is written. Otherwise query a is scored against
 *   docs cand_ids[cand_off[a] .. cand_off[a+1]-1] and scores[p] is written for
 *   each pair index p in that range.
 * Returns 0, or -1 on an out-of-range candidate id.
 */
int oracle_maxsim(const double* q_tok, const int64_t* q_off, int64_t n_q,
                  const double* d_tok, const int64_t* d_off, int64_t n_docs,
                  int32_t dim, const int64_t* cand_off, const int32_t* cand_ids,
                  double* scores) {
  for (int64_t a = 0; a < n_q; ++a) {
    const double* q = q_tok + q_off[a] * dim;
    int64_t nq = q_off[a + 1] - q_off[a];
    if (cand_off == NULL) {
      for (int64_t b = 0; b < n_docs; ++b) {
        scores[a * n_docs + b] =
            maxsim_one(q, nq, d_tok + d_off[b] * dim, d_off[b + 1] - d_off[b], dim);
      }
    } else {
      for (int64_t p = cand_off[a]; p < cand_off[a + 1]; ++p) {
        int64_t b = cand_ids[p];
        if (b < 0 || b >= n_docs) return -1;
        scores[p] = maxsim_one(q, nq, d_tok + d_off[b] * dim, d_off[b + 1] - d_off[b], dim);
      }
    }
  }
  return 0;
}

/* ------------------------------------------------------------------ */
/* Product quantization (Sec. 4).                                      */
/* ------------------------------------------------------------------ */

/* Decompress: out[t, m*dsub + u] = C[m, codes[t, m], u]. */
int oracle_pq_decode(const uint8_t* codes, int64_t n_tokens, int32_t M, int32_t K,
                     int32_t dsub, const double* codebooks, double* out) {
  for (int64_t t = 0; t < n_tokens; ++t) {
    for (int32_t m = 0; m < M; ++m) {
      int32_t c = codes[t * M + m];
      if (c >= K) return -1;
      for (int32_t u = 0; u < dsub; ++u)
        out[t * (int64_t)M * dsub + m * dsub + u] =
            codebooks[((int64_t)m * K + c) * dsub + u];
    }
  }
  return 0;
}

/* Phase 1: T[i, m, k] = sum_u q[i, m*dsub + u] * C[m, k, u]. */
void oracle_pq_lut_build(const double* q, int64_t nq, int32_t M, int32_t K, int32_t dsub,
                         const double* codebooks, double* table) {
  int32_t dim = M * dsub;
  for (int64_t i = 0; i < nq; ++i)
    for (int32_t m = 0; m < M; ++m)
      for (int32_t k = 0; k < K; ++k) {
        double acc = 0.0;
        for (int32_t u = 0; u < dsub; ++u)
          acc += q[i * dim + m * dsub + u] * codebooks[((int64_t)m * K + k) * dsub + u];
        table[(i * M + m) * K + k] = acc;
      }
}

/*
 * Phase 2 for one query (its table already built): for each selected doc,
 * s_ij = sum_m T[i, m, c_jm]; score = sum_i max_j s_ij.
 * doc_sel: if NULL, score docs 0..n_sel-1; else score docs doc_sel[0..n_sel-1].
 */
int oracle_pq_lut_score(const double* table, int64_t nq, int32_t M, int32_t K,
                        const uint8_t* codes, const int64_t* d_off, int64_t n_docs,
                        const int32_t* doc_sel, int64_t n_sel, double* scores) {
  for (int64_t p = 0; p < n_sel; ++p) {
    int64_t b = doc_sel ? doc_sel[p] : p;
    if (b < 0 || b >= n_docs) return -1;
    double total = 0.0;
    for (int64_t i = 0; i < nq; ++i) {
      double best = -INFINITY;
      for (int64_t j = d_off[b]; j < d_off[b + 1]; ++j) {
        double s = 0.0;
        for (int32_t m = 0; m < M; ++m) {
          int32_t c = codes[j * M + m];
          if (c >= K) return -1;
          s += table[(i * M + m) * K + c];
        }
        if (s > best) best = s;
      }
      total += best;
    }
    scores[p] = total;
  }
  return 0;
}

/* ------------------------------------------------------------------ */
/* Residual-compressed documents (the centroid + per-dimension         */
/* quantized residual representation of the PLAID/WARP indexes the     */
/* paper integrates with, Related Work and the WARP comparison).       */
/* ------------------------------------------------------------------ */

/*
 * Decompress: token t is centroid ids[t] plus a residual whose dimension k is
 * weights[code(t, k)], where code(t, k) is the nbits-wide field at bit
 * k * nbits of the token's packed row (row_bytes = dim * nbits / 8 bytes;
 * fields fill each byte from its least significant bit up):
 *   out[t, k] = centroids[ids[t], k] + weights[code(t, k)].
 * Returns 0, or -1 on a centroid id outside [0, n_centroids).
 */
int oracle_residual_decode(const int32_t* ids, const uint8_t* residuals, int64_t n_tokens,
                           int32_t dim, int32_t nbits, int32_t n_centroids,
                           const double* centroids, const double* weights, double* out) {
  const int64_t row_bytes = (int64_t)dim * nbits / 8;
  const uint32_t field_mask = (1u << nbits) - 1u;
  for (int64_t t = 0; t < n_tokens; ++t) {
    const int32_t c = ids[t];
    if (c < 0 || c >= n_centroids) return -1;
    for (int32_t k = 0; k < dim; ++k) {
      const int64_t bit = (int64_t)k * nbits;
      const uint32_t byte = residuals[t * row_bytes + bit / 8];
      const uint32_t code = (byte >> (bit % 8)) & field_mask;
      out[t * dim + k] = centroids[(int64_t)c * dim + k] + weights[code];
    }
  }
  return 0;
}

/* ------------------------------------------------------------------ */
/* Top-k: (score descending, id ascending).                            */
/* ------------------------------------------------------------------ */

typedef struct { double s; int64_t id; } scored_id;

static int cmp_scored(const void* a, const void* b) {
  const scored_id* x = (const scored_id*)a;
  const scored_id* y = (const scored_id*)b;
  if (x->s > y->s) return -1;
  if (x->s < y->s) return 1;
  if (x->id < y->id) return -1;
  if (x->id > y->id) return 1;
  return 0;
}

/*
 * scores[n] with ids[n] (NULL: id = position). Writes the first min(k, n)
 * entries of the ordering to out_ids / out_scores and pads the rest with
 * id -1 and score -inf. Returns 0, or -1 on allocation failure.
 */
int oracle_topk(const double* scores, const int64_t* ids, int64_t n, int64_t k,
                int64_t* out_ids, double* out_scores) {
  scored_id* v = (scored_id*)malloc((size_t)(n > 0 ? n : 1) * sizeof(scored_id));
  if (!v) return -1;
  for (int64_t i = 0; i < n; ++i) {
    v[i].s = scores[i];
    v[i].id = ids ? ids[i] : i;
  }
  qsort(v, (size_t)n, sizeof(scored_id), cmp_scored);
  for (int64_t r = 0; r < k; ++r) {
    if (r < n) {
      out_ids[r] = v[r].id;
      out_scores[r] = v[r].s;
    } else {
      out_ids[r] = -1;
      out_scores[r] = -INFINITY;
    }
  }
  free(v);
  return 0;
}

/* ------------------------------------------------------------------ */
/* Number formats: round-to-nearest-even from the format definitions.  */
/* ------------------------------------------------------------------ */

/*
 * A binary format with p explicit mantissa bits and minimum normal exponent
 * emin has, for |x| in [2^e, 2^(e+1)) with e >= emin, spacing 2^(e-p); below
 * 2^emin the spacing is 2^(emin-p) (subnormals). Rounding |x| to a multiple of
 * that spacing with ties to even is rint() in the default rounding mode.
 * The input is a float widened to double, so every step below is exact.
 */
static double round_rne(double x, int p, int emin) {
  if (x == 0.0 || !isfinite(x)) return x;
  double ax = fabs(x);
  int e;
  frexp(ax, &e); /* ax = f * 2^e, f in [0.5, 1) so floor(log2 ax) = e-1 */
  e -= 1;
  if (e < emin) e = emin;
  double quantum = ldexp(1.0, e - p);
  double r = rint(ax / quantum) * quantum;
  return x < 0 ? -r : r;
}

/* Encode a value already representable in (p, emin, bias) into sign|exp|mant. */
static uint32_t encode_bits(double v, int p, int emin, int bias, int total_bits) {
  uint32_t sign = signbit(v) ? 1u : 0u;
  double av = fabs(v);
  uint32_t expf = 0, mant = 0;
  if (isinf(av)) {
    expf = (1u << (total_bits - 1 - p)) - 1u;
    mant = 0;
  } else if (av == 0.0) {
    expf = 0;
    mant = 0;
  } else {
    int e;
    frexp(av, &e);
    e -= 1;
    if (e < emin) { /* subnormal */
      expf = 0;
      mant = (uint32_t)(av / ldexp(1.0, emin - p));
    } else {
      expf = (uint32_t)(e + bias);
      mant = (uint32_t)(av / ldexp(1.0, e - p)) - (1u << p);
    }
  }
  return (sign << (total_bits - 1)) | (expf << p) | mant;
}

static double decode_bits(uint32_t bits, int p, int emin, int bias, int total_bits,
                          int has_inf) {
  uint32_t sign = (bits >> (total_bits - 1)) & 1u;
  uint32_t expf = (bits >> p) & ((1u << (total_bits - 1 - p)) - 1u);
  uint32_t mant = bits & ((1u << p) - 1u);
  uint32_t expmax = (1u << (total_bits - 1 - p)) - 1u;
  double v;
  if (has_inf && expf == expmax) {
    v = mant ? NAN : INFINITY;
  } else if (!has_inf && expf == expmax && mant == (1u << p) - 1u) {
    v = NAN; /* E4M3FN: S.1111.111 is NaN, no infinities */
  } else if (expf == 0) {
    v = ldexp((double)mant, emin - p);
  } else {
    v = ldexp((double)((1u << p) + mant), (int)expf - bias - p);
  }
  return sign ? -v : v;
}

/* binary16: p = 10, emin = -14, bias 15, max finite 65504, overflow -> inf. */
void oracle_round_f16(const float* x, int64_t n, uint16_t* bits) {
  for (int64_t i = 0; i < n; ++i) {
    double v = isnan(x[i]) ? NAN : round_rne((double)x[i], 10, -14);
    if (isnan(v)) {
      bits[i] = 0x7E00;
      continue;
    }
    if (fabs(v) > 65504.0) v = copysign(INFINITY, v);
    bits[i] = (uint16_t)encode_bits(v, 10, -14, 15, 16);
  }
}

void oracle_decode_f16(const uint16_t* bits, int64_t n, double* out) {
  for (int64_t i = 0; i < n; ++i) out[i] = decode_bits(bits[i], 10, -14, 15, 16, 1);
}

/* bfloat16: p = 7, emin = -126, bias 127; overflow past the largest finite -> inf. */
void oracle_round_bf16(const float* x, int64_t n, uint16_t* bits) {
  const double bf16_max = ldexp(255.0, 120); /* (2 - 2^-7) * 2^127 */
  for (int64_t i = 0; i < n; ++i) {
    double v = isnan(x[i]) ? NAN : round_rne((double)x[i], 7, -126);
    if (isnan(v)) {
      bits[i] = 0x7FC0;
      continue;
    }
    if (fabs(v) > bf16_max) v = copysign(INFINITY, v);
    bits[i] = (uint16_t)encode_bits(v, 7, -126, 127, 16);
  }
}

void oracle_decode_bf16(const uint16_t* bits, int64_t n, double* out) {
  for (int64_t i = 0; i < n; ++i) out[i] = decode_bits(bits[i], 7, -126, 127, 16, 1);
}

/* OCP FP8 E4M3FN: p = 3, emin = -6, bias 7, max finite 448, no inf; saturate. */
static uint8_t e4m3_from_double(double x) {
  double v = round_rne(x, 3, -6);
  if (fabs(v) > 448.0) v = copysign(448.0, v);
  return (uint8_t)encode_bits(v, 3, -6, 7, 8);
}

void oracle_round_e4m3(const float* x, int64_t n, uint8_t* bits) {
  for (int64_t i = 0; i < n; ++i) bits[i] = e4m3_from_double((double)x[i]);
}

void oracle_decode_e4m3(const uint8_t* bits, int64_t n, double* out) {
  for (int64_t i = 0; i < n; ++i) out[i] = decode_bits(bits[i], 3, -6, 7, 8, 0);
}

/*
 * Per-token FP8 quantization: s = 2^k with k the smallest integer such that
 * amax <= 448 * 2^k (s = 1 for an all-zero token); code = E4M3FN(x / s).
 * Dividing by a power of two is exact in double, and 448 * 2^k is exact, so
 * the comparisons that pick k are exact.
 */
void oracle_quant_e4m3(const float* x, int64_t n_tokens, int32_t dim, uint8_t* codes,
                       float* scales) {
  for (int64_t t = 0; t < n_tokens; ++t) {
    double amax = 0.0;
    for (int32_t u = 0; u < dim; ++u) {
      double a = fabs((double)x[t * dim + u]);
      if (a > amax) amax = a;
    }
    int k = 0;
    if (amax > 0.0) {
      k = ilogb(amax) - 8;
      while (amax > ldexp(448.0, k)) ++k;
      while (amax <= ldexp(448.0, k - 1)) --k;
    }
    double s = ldexp(1.0, k);
    scales[t] = (float)s;
    for (int32_t u = 0; u < dim; ++u)
      codes[t * dim + u] = e4m3_from_double((double)x[t * dim + u] / s);
  }
}
