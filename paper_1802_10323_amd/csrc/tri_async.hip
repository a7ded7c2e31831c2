// tri_async.hip - instantiations and launches of the asynchronous-staging
// elimination kernels (tri_fast.h), in a translation unit of their own like
// the staging transforms (see async_launch.h).
#include <hip/hip_runtime.h>

#include "async_launch.h"
#include "tri_fast.h"

namespace poisson_dev {
namespace {

template <typename T, int RPC, int P>
hipError_t launch(const TriFastArgs<T>& a, hipStream_t st) {
  void (*k)(TriFastArgs<T>) =
      a.g.layout == 0 ? tri_async_kernel<T, RPC, P, 0> : tri_async_kernel<T, RPC, P, 1>;
  hipLaunchKernelGGL(k, dim3(async_resident_blocks(reinterpret_cast<const void*>(k), a.g.ntiles)),
                     dim3(512), 0, st, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_n(const TriFastArgs<T>& a, int n, hipStream_t st) {
  switch (n) {
    case 64: return launch<T, 4, 16>(a, st);
    case 96: return launch<T, 6, 16>(a, st);
    case 128: return launch<T, 8, 16>(a, st);
    case 192: return launch<T, 12, 16>(a, st);
    case 256: return launch<T, 8, 32>(a, st);
    case 384: return launch<T, 6, 64>(a, st);
    case 512: return launch<T, 8, 64>(a, st);
    default: return hipErrorInvalidValue;
  }
}

template <typename T, int RPC, int P>
hipError_t launch_direct(const TriFastArgs<T>& a, hipStream_t st) {
  if constexpr ((RPC * sizeof(T)) % 16 != 0) {
    return hipErrorInvalidValue;
  } else {
    // whole groups of 64 / P lines only
    if (a.g.layout != 1 || a.g.nlines % (64 / P) != 0) return hipErrorInvalidValue;
    void (*k)(TriFastArgs<T>) = tri_direct_kernel<T, RPC, P>;
    const long long groups = (long long)a.g.nlines / (64 / P);
    hipLaunchKernelGGL(k, dim3(direct_blocks(reinterpret_cast<const void*>(k), (groups + 3) / 4)),
                       dim3(256), 0, st, a);
    return hipGetLastError();
  }
}

template <typename T>
hipError_t launch_direct_n(const TriFastArgs<T>& a, int n, hipStream_t st) {
  switch (n) {
    case 64: return launch_direct<T, 4, 16>(a, st);
    case 96: return launch_direct<T, 6, 16>(a, st);
    case 128: return launch_direct<T, 8, 16>(a, st);
    case 192: return launch_direct<T, 12, 16>(a, st);
    case 256: return launch_direct<T, 8, 32>(a, st);
    case 384: return launch_direct<T, 6, 64>(a, st);
    case 512: return launch_direct<T, 8, 64>(a, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t direct_elimination_launch(const TriFastArgs<double>& a, int n, hipStream_t stream) {
  return launch_direct_n<double>(a, n, stream);
}

hipError_t direct_elimination_launch(const TriFastArgs<float>& a, int n, hipStream_t stream) {
  return launch_direct_n<float>(a, n, stream);
}

hipError_t async_elimination_launch(const TriFastArgs<double>& a, int n, hipStream_t stream) {
  return launch_n<double>(a, n, stream);
}

hipError_t async_elimination_launch(const TriFastArgs<float>& a, int n, hipStream_t stream) {
  return launch_n<float>(a, n, stream);
}

}  // namespace poisson_dev
