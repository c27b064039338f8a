// pq.hip -- fused PQ scoring with the distance table in LDS (Sec. 4.2-4.3).
//
// Work item = (doc chunk, query, query-token slice). Its workgroup
//   1. builds the slice's table T[i, m, k] = q_i[m-th subspace] . C[m, k] in
//      LDS (FP32, stored [k][m][i]: the entries of 4 query tokens for one
//      (k, m) are 16 contiguous bytes);
//   2. streams its chunk of documents: each wave takes whole documents; lane
//      (qq, jj) = (lane % (QT/4), lane / (QT/4)) scores query tokens
//      4qq..4qq+3 against doc token jj of each group of 64/(QT/4) tokens:
//      per subspace one ds_read_b128 brings the 4 entries T[m][c_m][4qq..],
//      so the code byte and the address are computed once per 4 lookups;
//      running maxima stay in VGPRs; rows past the document's end are clamped
//      to its last token (a duplicate never changes a max); the codes of the
//      next token group are loaded while the current one is scored;
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

constexpr int PQ_MAX_DSUB = 32;  // centroid length limit of the table build

template <int M>
struct CodeVec;
// byte(v, m): the code of subspace m; rotate(v, r): the same codes moved down
// by r bytes (0 <= r < 4), so byte(rotate(v, r), m) = byte(v, (m + r) % M).
template <>
struct CodeVec<4> {
  typedef uint32_t type;
  __device__ static uint32_t byte(type v, int m) { return __builtin_amdgcn_ubfe(v, 8 * m, 8); }
  __device__ static type rotate(type v, int r) { return __builtin_amdgcn_alignbit(v, v, 8 * r); }
};
template <>
struct CodeVec<8> {
  typedef uint2 type;
  __device__ static uint32_t byte(type v, int m) {
    return __builtin_amdgcn_ubfe(m < 4 ? v.x : v.y, 8 * (m & 3), 8);
  }
  __device__ static type rotate(type v, int r) {
    return make_uint2(__builtin_amdgcn_alignbit(v.y, v.x, 8 * r),
                      __builtin_amdgcn_alignbit(v.x, v.y, 8 * r));
  }
};
template <>
struct CodeVec<16> {
  typedef uint4 type;
  __device__ static uint32_t byte(type v, int m) {
    uint32_t w = m < 4 ? v.x : (m < 8 ? v.y : (m < 12 ? v.z : v.w));
    return __builtin_amdgcn_ubfe(w, 8 * (m & 3), 8);
  }
  __device__ static type rotate(type v, int r) {
    return make_uint4(__builtin_amdgcn_alignbit(v.y, v.x, 8 * r),
                      __builtin_amdgcn_alignbit(v.z, v.y, 8 * r),
                      __builtin_amdgcn_alignbit(v.w, v.z, 8 * r),
                      __builtin_amdgcn_alignbit(v.x, v.w, 8 * r));
  }
};

template <int M, int QT, bool QF32, bool CBF32, int PQ_NW>
__global__ __launch_bounds__(PQ_NW * 64) void pq_fused_kernel(PqParams P) {
  extern __shared__ float lut[];  // [M][K][QT], then the query slice [QT][dim]
  typedef typename CodeVec<M>::type cvec;
  constexpr int QQ = QT / 4;    // lanes per doc token (4 query tokens each)
  constexpr int DPW = 64 / QQ;  // doc tokens per wave iteration
  const int lane = lane_id();
  const int qq = lane % QQ, jj = lane / QQ;
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

  // ---- Phase 1: the slice's table, stored [k][m][i] ----
  float* qs = lut + (size_t)M * K * QT;
  const int nthreads = PQ_NW * 64;
  for (int e = threadIdx.x; e < QT * dim; e += nthreads) {
    int i = e / dim, u = e - i * dim;
    float v = 0.f;
    if (i < nq_slice) {
      int64_t idx = (q0 + sl * QT + i) * dim + u;
      v = QF32 ? ((const float*)P.q_tok)[idx] : (float)((const _Float16*)P.q_tok)[idx];
    }
    qs[e] = v;
  }
  __syncthreads();
  // one thread per (m, k): its centroid is read once (vector loads) and
  // dotted with the QT query-token slices, which every thread of the
  // workgroup reads from LDS in the same order (broadcast)
  for (int mk = threadIdx.x; mk < M * K; mk += nthreads) {
    const int m = mk / K, k = mk - m * K;
    float c[PQ_MAX_DSUB];
#pragma unroll
    for (int u = 0; u < PQ_MAX_DSUB; ++u) {
      c[u] = 0.f;
      if (u < dsub) {
        if constexpr (CBF32)
          c[u] = ((const float*)P.codebooks)[(int64_t)mk * dsub + u];
        else
          c[u] = (float)((const _Float16*)P.codebooks)[(int64_t)mk * dsub + u];
      }
    }
    for (int i = 0; i < QT; ++i) {
      const float* qrow = qs + i * dim + m * dsub;
      float acc = 0.f;
#pragma unroll
      for (int u = 0; u < PQ_MAX_DSUB; ++u)
        if (u < dsub) acc = fmaf(qrow[u], c[u], acc);
      lut[(k * M + m) * QT + i] = acc;
    }
  }
  __syncthreads();

  // ---- Phase 2: lookup, max over doc tokens, sum over the slice ----
  // lane (qq, jj): query tokens 4qq..4qq+3 of the slice against doc token jj
  // of each group of DPW tokens; one 16-byte LDS read brings the 4 entries.
  float* out = P.n_slices > 1 ? P.partial + (int64_t)sl * P.n_pairs : P.scores;
  const cvec* codes = (const cvec*)P.codes;
  // Row (k, m) of the table is QT*4 bytes at (k*M + m)*QT*4. The doc tokens
  // that share an LDS pass visit the subspaces in rotated orders (token jj
  // starts at subspace jj mod RG), so in any one read their rows fall in
  // different bank groups whatever their codes are.
  constexpr int RG0 = (64 / QT) < M ? (64 / QT) : M;
  constexpr int RG = RG0 < 4 ? RG0 : 4;  // rotate() moves by fewer than 4 bytes
  constexpr int KROW = M * QT * 4;  // bytes per centroid index k
  constexpr int KSH = __builtin_ctz(KROW);
  static_assert((1 << KSH) == KROW, "table row must be a power of two");
  const int rot = jj % RG;
  int mbase[M];
#pragma unroll
  for (int m = 0; m < M; ++m) mbase[m] = ((m + rot) % M) * QT * 4 + qq * 16;
  const char* lut_c = (const char*)lut;

  // Cursor over (document, token group) steps of this wave's documents
  // (p0 + wave, p0 + wave + NW, ...). Document offsets come from scalar loads
  // one document ahead; code loads run PF groups ahead in a ring of
  // registers, each refill issuing exactly one load (a zero row when idle).
  const bool has_cand = P.cand_off != nullptr;
  auto doc_of = [&](int64_t pp) -> int64_t {
    return has_cand ? (int64_t)sload_i32(P.cand_ids, pp) : pp - pair_base;
  };
  int64_t cp = p0 + wave;
  int64_t ct0 = 0, nx_s = 0, nx_e = 0;
  int cnd = 0, cbase = 0;
  if (cp < p1) {
    int64_t b0 = doc_of(cp);
    ct0 = sload_i64(P.d_off, b0);
    cnd = (int)(sload_i64(P.d_off, b0 + 1) - ct0);
    if (cp + PQ_NW < p1) {
      int64_t b1 = doc_of(cp + PQ_NW);
      nx_s = sload_i64(P.d_off, b1);
      nx_e = sload_i64(P.d_off, b1 + 1);
    }
  }
  auto next_doc = [&]() {
    cp += PQ_NW;
    cbase = 0;
    ct0 = nx_s;
    cnd = (int)(nx_e - nx_s);
    if (cp + PQ_NW < p1) {
      int64_t b1 = doc_of(cp + PQ_NW);
      nx_s = sload_i64(P.d_off, b1);
      nx_e = sload_i64(P.d_off, b1 + 1);
    }
  };
  constexpr int F_VALID = 1, F_EMPTY = 2, F_DLAST = 4;
  const cvec* const zero = (const cvec*)zero_row_ptr();
  auto fill = [&](cvec& cv, int& fl, int64_t& pp) {
    const cvec* src = zero;
    int f = 0;
    pp = cp;
    if (cp < p1) {
      if (cnd == 0) {
        f = F_VALID | F_EMPTY;
      } else {
        int j = cbase + jj;
        src = codes + ct0 + (j < cnd ? j : cnd - 1);
        f = F_VALID | (cbase + DPW >= cnd ? F_DLAST : 0);
      }
    }
    cv = *src;
    fl = f;
    if (cp < p1) {
      if (cnd == 0 || cbase + DPW >= cnd)
        next_doc();
      else
        cbase += DPW;
    }
  };

  float mx0 = -__builtin_inff(), mx1 = mx0, mx2 = mx0, mx3 = mx0;
  auto consume = [&](const cvec& cv, int fl, int64_t pp) {
    if (!(fl & F_VALID)) return;
    if (fl & F_EMPTY) {
      if (lane == 0) out[pp] = nq_slice > 0 ? -__builtin_inff() : 0.f;
      return;
    }
    const cvec cr = CodeVec<M>::rotate(cv, rot);  // byte m of cr = code of subspace (m + rot) % M
    float4 v = *(const float4*)(lut_c + (CodeVec<M>::byte(cr, 0) << KSH) + mbase[0]);
    float s0 = v.x, s1 = v.y, s2 = v.z, s3 = v.w;
#pragma unroll
    for (int m = 1; m < M; ++m) {
      v = *(const float4*)(lut_c + (CodeVec<M>::byte(cr, m) << KSH) + mbase[m]);
      s0 += v.x;
      s1 += v.y;
      s2 += v.z;
      s3 += v.w;
    }
    mx0 = fmaxf(mx0, s0);
    mx1 = fmaxf(mx1, s1);
    mx2 = fmaxf(mx2, s2);
    mx3 = fmaxf(mx3, s3);
    if (fl & F_DLAST) {
#pragma unroll
      for (int off = QQ; off < 64; off <<= 1) {
        mx0 = fmaxf(mx0, xor_shfl(mx0, off));
        mx1 = fmaxf(mx1, xor_shfl(mx1, off));
        mx2 = fmaxf(mx2, xor_shfl(mx2, off));
        mx3 = fmaxf(mx3, xor_shfl(mx3, off));
      }
      float v = (mx0 + mx1) + (mx2 + mx3);
#pragma unroll
      for (int off = QQ / 2; off >= 1; off >>= 1) v += xor_shfl(v, off);
      if (lane == 0) out[pp] = v;
      mx0 = mx1 = mx2 = mx3 = -__builtin_inff();
    }
  };

  // four ring slots, written out so each keeps its own registers
  cvec r0, r1, r2, r3;
  int f0, f1, f2, f3;
  int64_t q0p, q1p, q2p, q3p;
  fill(r0, f0, q0p);
  fill(r1, f1, q1p);
  fill(r2, f2, q2p);
  fill(r3, f3, q3p);
  if (f0 & F_VALID) {
    while (true) {
      consume(r0, f0, q0p);
      fill(r0, f0, q0p);
      consume(r1, f1, q1p);
      fill(r1, f1, q1p);
      consume(r2, f2, q2p);
      fill(r2, f2, q2p);
      consume(r3, f3, q3p);
      fill(r3, f3, q3p);
      if (!(f0 & F_VALID)) break;
    }
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

template <int M, int QT, bool QF32, bool CBF32>
hipError_t launch_pq_t(const PqParams& P, hipStream_t s) {
  size_t lds = ((size_t)M * P.K * QT + (size_t)QT * P.dim) * sizeof(float);
  auto k = P.nw == 16 ? pq_fused_kernel<M, QT, QF32, CBF32, 16> : pq_fused_kernel<M, QT, QF32, CBF32, 8>;
  if (lds > 64 * 1024) {
    hipError_t e =
        hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  int64_t items = (int64_t)P.n_chunks * P.n_q * P.n_slices;
  hipLaunchKernelGGL(k, dim3((unsigned)items), dim3(P.nw * 64), lds, s, P);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || P.n_slices <= 1) return e;
  int64_t blocks = (P.n_pairs + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(pq_slice_sum_kernel, dim3((unsigned)blocks), dim3(256), 0, s,
                     (const float*)P.partial, P.scores, P.n_pairs, P.n_slices);
  return hipGetLastError();
}

template <int M, bool QF32, bool CBF32>
hipError_t launch_pq_qt(const PqParams& P, hipStream_t s) {
  switch (P.qt) {
    case 8: return launch_pq_t<M, 8, QF32, CBF32>(P, s);
    case 16: return launch_pq_t<M, 16, QF32, CBF32>(P, s);
    case 32: return launch_pq_t<M, 32, QF32, CBF32>(P, s);
    default: return launch_pq_t<M, 64, QF32, CBF32>(P, s);
  }
}

template <int M>
hipError_t launch_pq_m(const PqParams& P, hipStream_t s) {
  if (P.q_f32) return P.cb_f32 ? launch_pq_qt<M, true, true>(P, s) : launch_pq_qt<M, true, false>(P, s);
  return P.cb_f32 ? launch_pq_qt<M, false, true>(P, s) : launch_pq_qt<M, false, false>(P, s);
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
