// fused_inst.hip -- host launchers of the fused scorer and of the unfused
// comparator for one element type. The build compiles this file once per
// type with -DFUSED_DT=<maxsim_dtype>, so the four types compile in parallel.
#include "fused_impl.h"

#ifndef FUSED_DT
#error "FUSED_DT must be defined"
#endif

namespace {

constexpr int DT = FUSED_DT;

template <int NQB, int DCH, int PF, int NW, int QM, bool STAGE, int RT = 16>
hipError_t launch_fused_t(const FusedParams& P, int grid, size_t lds, hipStream_t s) {
  auto k = fused_detail::fused_maxsim_kernel<DT, NQB, DCH, PF, NW, QM, STAGE, RT>;
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k, dim3(grid), dim3(NW * 64), lds, s, P);
  return hipGetLastError();
}

template <int NQB, int DCH, int PF, int NW, int QM, bool STAGE, int RT = 16>
int occupancy_fused_t(size_t lds) {
  auto k = fused_detail::fused_maxsim_kernel<DT, NQB, DCH, PF, NW, QM, STAGE, RT>;
  if (lds > 64 * 1024 &&
      hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) !=
          hipSuccess)
    return 0;
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, NW * 64, lds) != hipSuccess) return 0;
  return nb;
}

template <int NQB, int DCH, int PF, int NW, bool STAGE>
FusedFns pick_q(int qm, int rt) {
  if (rt == 32) {
    // 32-row steps: FP8 only (narrow rows), staged, query operand in VGPRs
    if constexpr (DT == DT_FP8 && STAGE && DCH != 256) {
      if (qm == fused_detail::Q_REGS)
        return {launch_fused_t<NQB, DCH, PF, NW, fused_detail::Q_REGS, STAGE, 32>,
                occupancy_fused_t<NQB, DCH, PF, NW, fused_detail::Q_REGS, STAGE, 32>, STAGE};
    }
    return {nullptr, nullptr, STAGE};
  }
  if constexpr (DCH == 256) {
    // wide chunks: LDS-staged, query operand in LDS (d >= 512), at most 4
    // query blocks, 1- and 2-byte elements
    if constexpr (DT == DT_F32 || NQB == 8 || !STAGE) {
      return {nullptr, nullptr, STAGE};
    } else {
      if (qm == fused_detail::Q_WAVE)
        return {launch_fused_t<NQB, DCH, PF, NW, fused_detail::Q_WAVE, STAGE>,
                occupancy_fused_t<NQB, DCH, PF, NW, fused_detail::Q_WAVE, STAGE>, STAGE};
      if (qm == fused_detail::Q_SHARED)
        return {launch_fused_t<NQB, DCH, PF, NW, fused_detail::Q_SHARED, STAGE>,
                occupancy_fused_t<NQB, DCH, PF, NW, fused_detail::Q_SHARED, STAGE>, STAGE};
      return {nullptr, nullptr, STAGE};
    }
  } else if constexpr (NQB == 8) {
    // eight query blocks only with the query operand in VGPRs, and only for
    // 1- and 2-byte elements (the host never asks for anything else)
    if constexpr (DT == DT_F32) {
      return {nullptr, nullptr, STAGE};
    } else {
      if (qm != fused_detail::Q_REGS) return {nullptr, nullptr, STAGE};
      return {launch_fused_t<NQB, DCH, PF, NW, fused_detail::Q_REGS, STAGE>,
              occupancy_fused_t<NQB, DCH, PF, NW, fused_detail::Q_REGS, STAGE>, STAGE};
    }
  } else {
    if (qm == fused_detail::Q_REGS)
      return {launch_fused_t<NQB, DCH, PF, NW, fused_detail::Q_REGS, STAGE>,
              occupancy_fused_t<NQB, DCH, PF, NW, fused_detail::Q_REGS, STAGE>, STAGE};
    if (qm == fused_detail::Q_WAVE)
      return {launch_fused_t<NQB, DCH, PF, NW, fused_detail::Q_WAVE, STAGE>,
              occupancy_fused_t<NQB, DCH, PF, NW, fused_detail::Q_WAVE, STAGE>, STAGE};
    return {launch_fused_t<NQB, DCH, PF, NW, fused_detail::Q_SHARED, STAGE>,
            occupancy_fused_t<NQB, DCH, PF, NW, fused_detail::Q_SHARED, STAGE>, STAGE};
  }
}

template <int NQB, int DCH, int PF, bool STAGE>
FusedFns pick_nw(int nw, int qm, int rt) {
  return nw == 8 ? pick_q<NQB, DCH, PF, 8, STAGE>(qm, rt) : pick_q<NQB, DCH, PF, 4, STAGE>(qm, rt);
}

template <int NQB, int DCH, bool STAGE>
FusedFns pick_pf(int pf, int nw, int qm, int rt) {
  if (pf == 2) return pick_nw<NQB, DCH, 2, STAGE>(nw, qm, rt);
  if (pf == 3) return pick_nw<NQB, DCH, 3, STAGE>(nw, qm, rt);
  return pick_nw<NQB, DCH, 4, STAGE>(nw, qm, rt);
}

template <int NQB, int DCH>
FusedFns pick_stage(int pf, int nw, int qm, bool stage, int rt) {
  return stage ? pick_pf<NQB, DCH, true>(pf, nw, qm, rt) : pick_pf<NQB, DCH, false>(pf, nw, qm, rt);
}

template <int NQB>
FusedFns pick_dch(int dch, int pf, int nw, int qm, bool stage, int rt) {
  if (dch == 64) return pick_stage<NQB, 64>(pf, nw, qm, stage, rt);
  if (dch == 256) return pick_stage<NQB, 256>(pf, nw, qm, stage, rt);
  return pick_stage<NQB, 128>(pf, nw, qm, stage, rt);
}

template <int NQB, int DCH, int NW, int PF>
hipError_t launch_sim_matrix(const FusedParams& P, float* S, int cus, size_t lds, hipStream_t s) {
  auto k1 = fused_detail::sim_matrix_kernel<DT, NQB, DCH, NW, PF>;
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)k1,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  int occ = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k1, NW * 64, lds);
  if (e != hipSuccess) return e;
  if (occ < 1) return hipErrorInvalidConfiguration;
  // one resident wave per run of tiles: every workgroup starts at once
  const int64_t tiles = (P.tokens_per_query + 15) / 16;
  int64_t grid = (int64_t)occ * cus;
  if (grid * NW > tiles) grid = (tiles + NW - 1) / NW;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(k1, dim3((unsigned)grid, (unsigned)P.n_q), dim3(NW * 64), lds, s, P, S);
  return hipGetLastError();
}

// Unfused comparator: S to HBM, then the segmented max / sum read back.
// `lds` is the staged query's size; the LDS ring of the S kernel is added
// here (4 waves with 3 steps in flight each, or 2 waves with 2 when that
// does not fit beside a large query operand).
template <int NQB, int DCH>
hipError_t launch_unfused_t(const FusedParams& P, float* S, int cus, size_t lds, hipStream_t s) {
  constexpr size_t LDS_MAX = 160 * 1024;  // gfx950 LDS per workgroup
  const size_t big = lds + fused_detail::stage_ring_bytes<DT, DCH, 3, 4>();
  const size_t small = lds + fused_detail::stage_ring_bytes<DT, DCH, 2, 2>();
  hipError_t e;
  if (big <= LDS_MAX)
    e = launch_sim_matrix<NQB, DCH, 4, 3>(P, S, cus, big, s);
  else if (small <= LDS_MAX)
    e = launch_sim_matrix<NQB, DCH, 2, 2>(P, S, cus, small, s);
  else
    return hipErrorInvalidValue;
  if (e != hipSuccess) return e;
  constexpr int NQP = NQB * 16;
  int64_t blocks = (P.n_pairs + 3) / 4;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(fused_detail::seg_maxsum_kernel<NQP>, dim3((unsigned)blocks), dim3(256), 0, s,
                     P, (const float*)S);
  return hipGetLastError();
}

template <int NQB>
hipError_t unfused_dch(const FusedParams& P, float* S, int cus, size_t lds, int dch,
                       hipStream_t s) {
  return dch == 64 ? launch_unfused_t<NQB, 64>(P, S, cus, lds, s)
                   : launch_unfused_t<NQB, 128>(P, S, cus, lds, s);
}

}  // namespace

#define CAT2(a, b) a##b
#define CAT(a, b) CAT2(a, b)

FusedFns CAT(fused_kernel_fns_, FUSED_DT)(int nqb, int dch, int pf, int nw, int qm,
                                           bool stage, int rt) {
  if (nqb == 1) return pick_dch<1>(dch, pf, nw, qm, stage, rt);
  if (nqb == 2) return pick_dch<2>(dch, pf, nw, qm, stage, rt);
  if (nqb == 8) return pick_dch<8>(dch, pf, nw, qm, stage, rt);
  return pick_dch<4>(dch, pf, nw, qm, stage, rt);
}

hipError_t CAT(launch_unfused_, FUSED_DT)(int nqb, int dch, const FusedParams& P, float* S,
                                           int cus, size_t lds, hipStream_t s) {
  if (nqb == 1) return unfused_dch<1>(P, S, cus, lds, dch, s);
  if (nqb == 2) return unfused_dch<2>(P, S, cus, lds, dch, s);
  return unfused_dch<4>(P, S, cus, lds, dch, s);
}
