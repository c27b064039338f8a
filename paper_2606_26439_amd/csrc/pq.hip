// pq.hip -- fused PQ scoring with the distance table in LDS (Sec. 4.2-4.3).
//
// Work item = (doc chunk, query, query-token slice). Its workgroup
//   1. builds the slice's table T[m][k][i] = q_i[m-th subspace] . C[m, k] in
//      LDS (FP32; i fastest so the QT query-token lanes of one doc token read
//      QT consecutive words: one conflict-free LDS access per (token, m));
//   2. streams its chunk of documents: each wave takes whole documents; lane
//      (i, jj) = (lane % QT, lane / QT) scores query token i against doc token
//      jj of each group of 64/QT tokens: s = sum_m T[m][c_m][i], running max
//      in a VGPR; rows past the document's end are clamped to its last token
//      (a duplicate never changes a max);
//   3. at a document's end: xor-shuffles finish the max over the token
//      sub-slots and sum the slice's query tokens; one lane stores the
//      slice's partial score.
// Codes are read from HBM once per (query, slice); chunk-major item order
// lets the workgroups resident at one time share a chunk's codes in L2/MALL.
// Several slices are summed by a second kernel in slice order, so the result
// does not depend on scheduling.
#include "device_common.h"
#include "kernels.h"

namespace {

constexpr int PQ_NW = 8;

template <int M>
struct CodeVec;
template <>
struct CodeVec<4> {
  typedef uint32_t type;
  __device__ static uint32_t byte(type v, int m) { return (v >> (8 * m)) & 0xFF; }
};
template <>
struct CodeVec<8> {
  typedef uint2 type;
  __device__ static uint32_t byte(type v, int m) {
    return ((m < 4 ? v.x : v.y) >> (8 * (m & 3))) & 0xFF;
  }
};
template <>
struct CodeVec<16> {
  typedef uint4 type;
  __device__ static uint32_t byte(type v, int m) {
    uint32_t w = m < 4 ? v.x : (m < 8 ? v.y : (m < 12 ? v.z : v.w));
    return (w >> (8 * (m & 3))) & 0xFF;
  }
};

__device__ __forceinline__ float ld_f(const void* p, int64_t i, bool f32) {
  return f32 ? ((const float*)p)[i] : (float)((const _Float16*)p)[i];
}

template <int M, int QT>
__global__ __launch_bounds__(PQ_NW * 64) void pq_fused_kernel(PqParams P) {
  extern __shared__ float lut[];  // [M][K][QT], then the query slice [QT][dim]
  typedef typename CodeVec<M>::type cvec;
  constexpr int DPW = 64 / QT;  // doc tokens per wave iteration
  const int lane = lane_id();
  const int qi = lane % QT, jj = lane / QT;
  const int wave = uniform(threadIdx.x >> 6);
  const int K = P.K, dsub = P.dsub, dim = P.dim;

  const int64_t item = blockIdx.x;
  const int sl = (int)(item % P.n_slices);
  const int64_t a = (item / P.n_slices) % P.n_q;
  const int64_t chunk = item / ((int64_t)P.n_slices * P.n_q);

  // pair range of this item
  int64_t p0, p1, pair_base;
  if (P.cand_off == nullptr) {
    pair_base = a * P.n_docs;
    p0 = pair_base + (P.n_docs * chunk) / P.n_chunks;
    p1 = pair_base + (P.n_docs * (chunk + 1)) / P.n_chunks;
  } else {
    pair_base = 0;
    int64_t c0 = P.cand_off[a], c1 = P.cand_off[a + 1];
    p0 = c0 + ((c1 - c0) * chunk) / P.n_chunks;
    p1 = c0 + ((c1 - c0) * (chunk + 1)) / P.n_chunks;
  }
  if (p0 >= p1) return;  // uniform for the whole workgroup

  const int64_t q0 = P.q_off[a];
  const int nq = (int)(P.q_off[a + 1] - q0);
  int nq_slice = nq - sl * QT;
  nq_slice = nq_slice < 0 ? 0 : (nq_slice > QT ? QT : nq_slice);

  // ---- Phase 1: the slice's table ----
  float* qs = lut + (size_t)M * K * QT;
  const int nthreads = PQ_NW * 64;
  for (int e = threadIdx.x; e < QT * dim; e += nthreads) {
    int i = e / dim, u = e - i * dim;
    qs[e] = i < nq_slice ? ld_f(P.q_tok, (q0 + sl * QT + i) * dim + u, P.q_f32) : 0.f;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < M * K * QT; e += nthreads) {
    int i = e % QT;
    int mk = e / QT;  // m * K + k
    int m = mk / K;
    const float* qrow = qs + i * dim + m * dsub;
    float acc = 0.f;
    for (int u = 0; u < dsub; ++u)
      acc = fmaf(qrow[u], ld_f(P.codebooks, (int64_t)mk * dsub + u, P.cb_f32), acc);
    lut[e] = acc;
  }
  __syncthreads();

  // ---- Phase 2: lookup, max over doc tokens, sum over the slice ----
  float* out = P.n_slices > 1 ? P.partial + (int64_t)sl * P.n_pairs : P.scores;
  const cvec* codes = (const cvec*)P.codes;
  for (int64_t p = p0 + wave; p < p1; p += PQ_NW) {
    int64_t b = P.cand_off == nullptr ? p - pair_base : (int64_t)P.cand_ids[p];
    const int64_t t0 = P.d_off[b];
    const int nd = (int)(P.d_off[b + 1] - t0);
    if (nd == 0) {
      if (lane == 0) out[p] = nq_slice > 0 ? -__builtin_inff() : 0.f;
      continue;
    }
    float mx = -__builtin_inff();
    for (int base = 0; base < nd; base += 2 * DPW) {
      int j0 = base + jj, j1 = base + DPW + jj;
      j0 = j0 < nd ? j0 : nd - 1;
      j1 = j1 < nd ? j1 : nd - 1;
      cvec c0 = codes[t0 + j0];
      cvec c1 = codes[t0 + j1];
      float s0 = 0.f, s1 = 0.f;
#pragma unroll
      for (int m = 0; m < M; ++m) {
        s0 += lut[(m * K + (int)CodeVec<M>::byte(c0, m)) * QT + qi];
        s1 += lut[(m * K + (int)CodeVec<M>::byte(c1, m)) * QT + qi];
      }
      mx = fmaxf(mx, fmaxf(s0, s1));
    }
#pragma unroll
    for (int off = QT; off < 64; off <<= 1) mx = fmaxf(mx, xor_shfl(mx, off));
    float v = mx;
#pragma unroll
    for (int off = QT / 2; off >= 1; off >>= 1) v += xor_shfl(v, off);
    if (lane == 0) out[p] = v;
  }
}

__global__ __launch_bounds__(256) void pq_slice_sum_kernel(const float* __restrict__ partial,
                                                           float* __restrict__ scores,
                                                           int64_t n_pairs, int n_slices) {
  for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < n_pairs;
       p += (int64_t)gridDim.x * 256) {
    float s = partial[p];
    for (int sl = 1; sl < n_slices; ++sl) s += partial[(int64_t)sl * n_pairs + p];
    scores[p] = s;
  }
}

template <int M, int QT>
hipError_t launch_pq_t(const PqParams& P, hipStream_t s) {
  size_t lds = ((size_t)M * P.K * QT + (size_t)QT * P.dim) * sizeof(float);
  auto k = pq_fused_kernel<M, QT>;
  if (lds > 64 * 1024) {
    hipError_t e =
        hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  int64_t items = (int64_t)P.n_chunks * P.n_q * P.n_slices;
  hipLaunchKernelGGL(k, dim3((unsigned)items), dim3(PQ_NW * 64), lds, s, P);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || P.n_slices <= 1) return e;
  int64_t blocks = (P.n_pairs + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(pq_slice_sum_kernel, dim3((unsigned)blocks), dim3(256), 0, s,
                     (const float*)P.partial, P.scores, P.n_pairs, P.n_slices);
  return hipGetLastError();
}

template <int M>
hipError_t launch_pq_m(const PqParams& P, hipStream_t s) {
  switch (P.qt) {
    case 8: return launch_pq_t<M, 8>(P, s);
    case 16: return launch_pq_t<M, 16>(P, s);
    case 32: return launch_pq_t<M, 32>(P, s);
    default: return launch_pq_t<M, 64>(P, s);
  }
}

}  // namespace

hipError_t launch_pq(const PqParams& P, int max_nq, hipStream_t s) {
  (void)max_nq;
  switch (P.M) {
    case 4: return launch_pq_m<4>(P, s);
    case 8: return launch_pq_m<8>(P, s);
    default: return launch_pq_m<16>(P, s);
  }
}
