// One instance of the fused scorer for the assembly check of its cross-lane
// swaps (tests/test_swap_asm.py): FP16, two query blocks, 128-wide chunks,
// three steps in flight, four waves, query operand in VGPRs, LDS-staged
// tiles, 16-row steps. Compiled to assembly only; never linked.
#include "../paper_2606_26439_amd/csrc/fused_impl.h"

template __global__ void fused_detail::fused_maxsim_kernel<DT_F16, 2, 128, 3, 4, fused_detail::Q_REGS,
                                                           true, 16>(FusedParams);
