// r2r_async.hip - instantiations and launches of the asynchronous-staging
// transform kernels (r2r_fast.h) other than the wide ones (see
// async_launch.h).
#include <hip/hip_runtime.h>

#include "async_launch.h"

namespace poisson_dev {
namespace {

template <typename T, typename C>
hipError_t launch(const R2RFastArgs<T>& a, int kind, int inverse, hipStream_t st) {
  void (*k)(R2RFastArgs<T>) = nullptr;
  switch (kind * 2 + inverse) {
#define POISSON_AK(K_, I_)                                                                   \
  case K_ * 2 + I_:                                                                          \
    if constexpr (AsyncBudget<T, C, K_>::WIDE) return async_wide_launch(a, K_, I_, st);      \
    else k = a.g.layout == 0 ? r2r_async_tight_kernel<T, C, K_, I_, 0>                      \
                             : r2r_async_tight_kernel<T, C, K_, I_, 1>;                     \
    break;
    POISSON_AK(0, 0) POISSON_AK(0, 1) POISSON_AK(1, 0) POISSON_AK(1, 1) POISSON_AK(2, 0)
    POISSON_AK(2, 1) POISSON_AK(3, 0) POISSON_AK(3, 1) POISSON_AK(4, 0) POISSON_AK(4, 1)
#undef POISSON_AK
    default: return hipErrorInvalidValue;
  }
  hipLaunchKernelGGL(k, dim3(async_resident_blocks(reinterpret_cast<const void*>(k), a.g.ntiles)),
                     dim3(512), 0, st, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_m(const R2RFastArgs<T>& a, int M, int shape, int kind, int inverse,
                    hipStream_t st) {
  switch (M * 4 + shape) {
    case 128 * 4 + 0: return launch<T, AsyncVar<128, 0>>(a, kind, inverse, st);
    case 128 * 4 + 1: return launch<T, AsyncVar<128, 1>>(a, kind, inverse, st);
    case 256 * 4 + 0: return launch<T, AsyncVar<256, 0>>(a, kind, inverse, st);
    case 256 * 4 + 1: return launch<T, AsyncVar<256, 1>>(a, kind, inverse, st);
    case 256 * 4 + 2:   // FP32 only: the FP64 tile and stage would not fit in LDS
      if constexpr (sizeof(T) == 4) return launch<T, AsyncVar<256, 2>>(a, kind, inverse, st);
      return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t async_transform_launch(const R2RFastArgs<double>& a, int M, int shape, int kind,
                                  int inverse, hipStream_t stream) {
  return launch_m<double>(a, M, shape, kind, inverse, stream);
}

hipError_t async_transform_launch(const R2RFastArgs<float>& a, int M, int shape, int kind,
                                  int inverse, hipStream_t stream) {
  return launch_m<float>(a, M, shape, kind, inverse, stream);
}

}  // namespace poisson_dev
