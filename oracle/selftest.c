/*
 * selftest.c -- drives every oracle function over small and edge-case inputs
 * so the oracle can be built and run under the host AddressSanitizer and
 * UndefinedBehaviorSanitizer (tests/test_oracle_sanitized.py builds it with
 * gcc -fsanitize=address,undefined). Test infrastructure only.
 *
 * Each check states a value fixed by the definitions (Eq. (1), the PQ
 * decompression of Sec. 4.1, the formats' bit layouts); a failure prints the
 * case and exits non-zero.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_maxsim(const double* q_tok, const int64_t* q_off, int64_t n_q, const double* d_tok,
                  const int64_t* d_off, int64_t n_docs, int32_t dim, const int64_t* cand_off,
                  const int32_t* cand_ids, double* scores);
int oracle_pq_decode(const uint8_t* codes, int64_t n_tokens, int32_t M, int32_t K, int32_t dsub,
                     const double* codebooks, double* out);
void oracle_pq_lut_build(const double* q, int64_t nq, int32_t M, int32_t K, int32_t dsub,
                         const double* codebooks, double* table);
int oracle_pq_lut_score(const double* table, int64_t nq, int32_t M, int32_t K,
                        const uint8_t* codes, const int64_t* d_off, int64_t n_docs,
                        const int32_t* doc_sel, int64_t n_sel, double* scores);
int oracle_residual_decode(const int32_t* ids, const uint8_t* residuals, int64_t n_tokens,
                           int32_t dim, int32_t nbits, int32_t n_centroids,
                           const double* centroids, const double* weights, double* out);
int oracle_topk(const double* scores, const int64_t* ids, int64_t n, int64_t k, int64_t* out_ids,
                double* out_scores);
void oracle_round_f16(const float* x, int64_t n, uint16_t* bits);
void oracle_decode_f16(const uint16_t* bits, int64_t n, double* out);
void oracle_round_bf16(const float* x, int64_t n, uint16_t* bits);
void oracle_decode_bf16(const uint16_t* bits, int64_t n, double* out);
void oracle_round_e4m3(const float* x, int64_t n, uint8_t* bits);
void oracle_decode_e4m3(const uint8_t* bits, int64_t n, double* out);
void oracle_quant_e4m3(const float* x, int64_t n_tokens, int32_t dim, uint8_t* codes,
                       float* scales);

static int failures = 0;
#define CHECK(cond, ...)                  \
  do {                                    \
    if (!(cond)) {                        \
      fprintf(stderr, "FAIL: " __VA_ARGS__); \
      fprintf(stderr, "\n");              \
      ++failures;                         \
    }                                     \
  } while (0)

static void test_maxsim(void) {
  /* dim 2; query tokens (1,0), (0,1); doc 0 = {(2,1), (0,3)}, doc 1 empty,
   * doc 2 = {(-1,-1)}: scores max(2,0)+max(1,3) = 5, -inf, -1 + -1 = -2 */
  const double q[] = {1, 0, 0, 1};
  const int64_t q_off[] = {0, 2, 2}; /* second query is empty */
  const double d[] = {2, 1, 0, 3, -1, -1};
  const int64_t d_off[] = {0, 2, 2, 3};
  double s[6];
  CHECK(oracle_maxsim(q, q_off, 2, d, d_off, 3, 2, NULL, NULL, s) == 0, "maxsim rc");
  CHECK(s[0] == 5.0 && isinf(s[1]) && s[1] < 0 && s[2] == -2.0, "maxsim values %g %g %g", s[0],
        s[1], s[2]);
  CHECK(s[3] == 0.0 && s[4] == 0.0 && s[5] == 0.0, "empty query scores 0");
  const int64_t c_off[] = {0, 2, 3};
  const int32_t c_ids[] = {2, 0, 1};
  double sc[3];
  CHECK(oracle_maxsim(q, q_off, 2, d, d_off, 3, 2, c_off, c_ids, sc) == 0, "cand rc");
  CHECK(sc[0] == -2.0 && sc[1] == 5.0 && sc[2] == 0.0, "cand values");
  const int32_t bad_ids[] = {3, 0, 1};
  CHECK(oracle_maxsim(q, q_off, 2, d, d_off, 3, 2, c_off, bad_ids, sc) == -1, "bad id rejected");
}

static void test_pq(void) {
  /* M = 2, K = 3, dsub = 2: centroid (m, k) = (10m + k, -(10m + k)) */
  double cb[2 * 3 * 2];
  for (int m = 0; m < 2; ++m)
    for (int k = 0; k < 3; ++k) {
      cb[(m * 3 + k) * 2 + 0] = 10 * m + k;
      cb[(m * 3 + k) * 2 + 1] = -(10 * m + k);
    }
  const uint8_t codes[] = {2, 1, 0, 0, 1, 2};
  double dec[3 * 4];
  CHECK(oracle_pq_decode(codes, 3, 2, 3, 2, cb, dec) == 0, "decode rc");
  CHECK(dec[0] == 2 && dec[1] == -2 && dec[2] == 11 && dec[3] == -11, "decode token 0");
  CHECK(dec[8] == 1 && dec[10] == 12 && dec[11] == -12, "decode token 2");
  const uint8_t bad[] = {3, 0};
  CHECK(oracle_pq_decode(bad, 1, 2, 3, 2, cb, dec) == -1, "code >= K rejected");
  const double q[] = {1, 0, 0, 1, 0, 0, 0, 0}; /* 2 query tokens, dim 4 */
  double table[2 * 2 * 3];
  oracle_pq_lut_build(q, 2, 2, 3, 2, cb, table);
  /* T[i, m, k] at (i*M + m)*K + k: q0 = (1,0 | 0,1), q1 = 0 */
  CHECK(table[(0 * 2 + 0) * 3 + 2] == 2.0 && table[(0 * 2 + 1) * 3 + 1] == -11.0, "table");
  CHECK(table[(1 * 2 + 1) * 3 + 2] == 0.0, "table of a zero query token");
  const int64_t d_off[] = {0, 2, 2, 3};
  double s[3];
  CHECK(oracle_pq_lut_score(table, 2, 2, 3, codes, d_off, 3, NULL, 3, s) == 0, "lut rc");
  /* doc 0, q0: token 0 (codes 2, 1) 2 - 11 = -9, token 1 (codes 0, 0)
   * 0 - 10 = -10, max -9; q1 is zero: max 0; score -9 */
  CHECK(s[0] == -9.0, "lut doc 0 %g", s[0]);
  CHECK(isinf(s[1]) && s[1] < 0, "lut empty doc");
  const int32_t sel[] = {2, 7};
  CHECK(oracle_pq_lut_score(table, 2, 2, 3, codes, d_off, 3, sel, 2, s) == -1, "lut bad id");
}

static void test_residual(void) {
  /* dim 4, 2 bits: byte 0xE4 holds codes 0, 1, 2, 3 (low bits first) */
  const double cen[] = {1, 2, 3, 4, 0, 0, 0, 0};
  const double w[] = {-0.5, -0.25, 0.25, 0.5};
  const int32_t ids[] = {0, 1};
  const uint8_t res[] = {0xE4, 0x1B};
  double out[8];
  CHECK(oracle_residual_decode(ids, res, 2, 4, 2, 2, cen, w, out) == 0, "residual rc");
  CHECK(out[0] == 0.5 && out[1] == 1.75 && out[2] == 3.25 && out[3] == 4.5, "residual token 0");
  CHECK(out[4] == 0.5 && out[5] == 0.25 && out[6] == -0.25 && out[7] == -0.5, "residual token 1");
  const int32_t bad[] = {2};
  CHECK(oracle_residual_decode(bad, res, 1, 4, 2, 2, cen, w, out) == -1, "residual bad id");
  /* dim 2, 4 bits: byte 0x21 holds codes 1, 2 */
  const double w16[16] = {0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 15};
  const uint8_t r4[] = {0x21};
  const double c2[] = {0.5, 0.5};
  const int32_t z[] = {0};
  CHECK(oracle_residual_decode(z, r4, 1, 2, 4, 1, c2, w16, out) == 0 && out[0] == 1.5 &&
            out[1] == 2.5,
        "residual 4-bit fields");
}

static void test_topk(void) {
  const double s[] = {1.0, 3.0, 3.0, -INFINITY, 2.0};
  const int64_t ids[] = {10, 7, 4, 1, 9};
  int64_t oi[8];
  double os[8];
  CHECK(oracle_topk(s, ids, 5, 8, oi, os) == 0, "topk rc");
  CHECK(oi[0] == 4 && oi[1] == 7 && oi[2] == 9 && oi[3] == 10 && oi[4] == 1, "topk order");
  CHECK(oi[5] == -1 && isinf(os[7]), "topk padding");
  CHECK(oracle_topk(s, NULL, 0, 2, oi, os) == 0 && oi[0] == -1, "topk empty");
}

static void test_formats(void) {
  const float x[] = {1.0f, -2.5f, 65504.0f, 65520.0f, 5.9604645e-8f, 1e-9f, 0.0f, 3.3333333f};
  uint16_t h[8];
  double v[8];
  oracle_round_f16(x, 8, h);
  oracle_decode_f16(h, 8, v);
  CHECK(h[0] == 0x3C00 && h[1] == 0xC100 && h[2] == 0x7BFF, "f16 bits");
  CHECK(h[3] == 0x7C00, "f16 overflow to inf");
  CHECK(h[4] == 0x0001 && h[5] == 0x0000, "f16 subnormal / underflow");
  CHECK(v[7] == 3.333984375, "f16 rounding %g", v[7]);
  uint16_t b[8];
  oracle_round_bf16(x, 8, b);
  oracle_decode_bf16(b, 8, v);
  CHECK(b[0] == 0x3F80 && b[1] == 0xC020, "bf16 bits");
  CHECK(v[7] == 3.328125, "bf16 rounding %g", v[7]);
  const float y[] = {448.0f, 500.0f, -1.0f, 0.001953125f, 0.0f, 0.3f};
  uint8_t e[6];
  double w[6];
  oracle_round_e4m3(y, 6, e);
  oracle_decode_e4m3(e, 6, w);
  CHECK(e[0] == 0x7E && w[0] == 448.0, "e4m3 max");
  CHECK(w[1] == 448.0, "e4m3 saturates");
  CHECK(e[2] == 0xB8, "e4m3 -1");
  CHECK(e[3] == 0x01 && w[3] == 0.001953125, "e4m3 min subnormal");
  CHECK(w[5] == 0.3125, "e4m3 rounding %g", w[5]);
  const float t[] = {0, 0, 0, 0, 1000.0f, -3.0f, 0.5f, 0.0f};
  uint8_t c[8];
  float sc[2];
  oracle_quant_e4m3(t, 2, 4, c, sc);
  CHECK(sc[0] == 1.0f, "zero token scale 1");
  CHECK(sc[1] == 4.0f, "scale 2^k with 1000 <= 448 * 2^k minimal: %g", sc[1]);
}

int main(void) {
  test_maxsim();
  test_pq();
  test_residual();
  test_topk();
  test_formats();
  if (failures) {
    fprintf(stderr, "%d check(s) failed\n", failures);
    return 1;
  }
  printf("oracle selftest: ok\n");
  return 0;
}
