// r2r_async_wide.hip - the asynchronous-staging transform kernels with the
// wide register budget (FP64, length 512, DFT and DCT-IV types; see
// async_launch.h for why they have a unit of their own).
#include <hip/hip_runtime.h>

#include "async_launch.h"

namespace poisson_dev {

hipError_t async_wide_launch(const R2RFastArgs<double>& a, int kind, int inverse,
                             hipStream_t stream) {
  using C = FastVar<256, 0>;
  void (*k)(R2RFastArgs<double>) = nullptr;
  switch (kind * 2 + inverse) {
#define POISSON_AW(K_, I_)                                                                   \
  case K_ * 2 + I_:                                                                          \
    static_assert(AsyncBudget<double, C, K_>::WIDE, "wide kernels only");                   \
    k = a.g.layout == 0 ? r2r_async_kernel<double, C, K_, I_, 0>                            \
                        : r2r_async_kernel<double, C, K_, I_, 1>;                           \
    break;
    POISSON_AW(0, 0) POISSON_AW(0, 1) POISSON_AW(3, 0) POISSON_AW(3, 1) POISSON_AW(4, 0)
    POISSON_AW(4, 1)
#undef POISSON_AW
    default: return hipErrorInvalidValue;
  }
  hipLaunchKernelGGL(k, dim3(async_resident_blocks(reinterpret_cast<const void*>(k), a.g.ntiles)),
                     dim3(512), 0, stream, a);
  return hipGetLastError();
}

hipError_t regstage_launch(const R2RFastArgs<double>& a, int kind, int inverse, bool hinted,
                           hipStream_t stream) {
  if (a.g.layout != 0) return hipErrorInvalidValue;
  void (*k)(R2RFastArgs<double>) = nullptr;
  switch (kind * 2 + inverse) {
#define POISSON_RS(K_, I_)                                                                    \
  case K_ * 2 + I_:                                                                          \
    k = hinted ? r2r_regstage_kernel<double, RegStageCfg, K_, I_, true>                     \
               : r2r_regstage_kernel<double, RegStageCfg, K_, I_, false>;                   \
    break;
    POISSON_RS(0, 0) POISSON_RS(0, 1) POISSON_RS(1, 0) POISSON_RS(1, 1) POISSON_RS(2, 0)
    POISSON_RS(2, 1) POISSON_RS(3, 0) POISSON_RS(3, 1) POISSON_RS(4, 0) POISSON_RS(4, 1)
#undef POISSON_RS
    default: return hipErrorInvalidValue;
  }
  hipLaunchKernelGGL(k, dim3(async_resident_blocks(reinterpret_cast<const void*>(k), a.g.ntiles)),
                     dim3(512), 0, stream, a);
  return hipGetLastError();
}

}  // namespace poisson_dev
