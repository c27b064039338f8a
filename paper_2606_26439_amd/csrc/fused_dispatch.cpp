// fused_dispatch.cpp -- routes a fused/unfused launch to the translation unit
// compiled for its element type.
#include "kernels.h"

FusedFns fused_kernel_fns_0(int, int, int, int, int, bool, int);
FusedFns fused_kernel_fns_1(int, int, int, int, int, bool, int);
FusedFns fused_kernel_fns_2(int, int, int, int, int, bool, int);
FusedFns fused_kernel_fns_3(int, int, int, int, int, bool, int);
hipError_t launch_unfused_0(int, int, const FusedParams&, float*, int, size_t, hipStream_t);
hipError_t launch_unfused_1(int, int, const FusedParams&, float*, int, size_t, hipStream_t);
hipError_t launch_unfused_2(int, int, const FusedParams&, float*, int, size_t, hipStream_t);
hipError_t launch_unfused_3(int, int, const FusedParams&, float*, int, size_t, hipStream_t);

FusedFns fused_kernel_fns(int dt, int nqb, int dch, int pf, int nw, int qm, bool stage, int rt) {
  switch (dt) {
    case 0: return fused_kernel_fns_0(nqb, dch, pf, nw, qm, stage, rt);
    case 1: return fused_kernel_fns_1(nqb, dch, pf, nw, qm, stage, rt);
    case 2: return fused_kernel_fns_2(nqb, dch, pf, nw, qm, stage, rt);
    default: return fused_kernel_fns_3(nqb, dch, pf, nw, qm, stage, rt);
  }
}

hipError_t launch_unfused(int dt, int nqb, int dch, const FusedParams& P, float* S, int cus,
                          size_t lds, hipStream_t s) {
  switch (dt) {
    case 0: return launch_unfused_0(nqb, dch, P, S, cus, lds, s);
    case 1: return launch_unfused_1(nqb, dch, P, S, cus, lds, s);
    case 2: return launch_unfused_2(nqb, dch, P, S, cus, lds, s);
    default: return launch_unfused_3(nqb, dch, P, S, cus, lds, s);
  }
}
