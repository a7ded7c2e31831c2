// poisson.hip - host side of the gfx950 Poisson solver: plans, tables,
// launches and the C ABI declared in include/poisson.h.
//
// The solve follows the three steps of Sec. 2.1 (forward transforms along the
// two transformed axes, Gauss elimination of Eq. (poi_reduced) along the third,
// backward transforms), each step one HBM sweep of the field by one kernel.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "poisson.h"
#include "r2r_kernel.h"
#include "r2r_fast.h"
#include "tridiag_kernel.h"
#include "tri_fast.h"
#include "batch_kernels.h"
#include "async_launch.h"
#include "refine_kernels.h"
#include "projection.h"
#include "navier_stokes.h"
#include "plane_kernels.h"

using namespace poisson_dev;

// ------------------------------------------------------------------ errors

static thread_local int g_err = 0;
static thread_local char g_msg[512] = "";

static int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
static int fail(int code, const char* fmt, ...) {
  g_err = code;
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_msg, sizeof(g_msg), fmt, ap);
  va_end(ap);
  return code;
}

#define HIP_TRY(expr)                                                              \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess)                                                          \
      return fail(POISSON_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_));    \
  } while (0)

// The solve kernels move two neighbouring points of a line with one 16-byte
// access, so a field they work on must be 16-byte aligned (hipMalloc and
// torch allocations are; a view at an odd element offset is not).  Returns
// POISSON_EINVAL, naming the argument, when it is not.
static int misaligned(const void* ptr, const char* what) {
  if ((reinterpret_cast<uintptr_t>(ptr) & 15) == 0) return POISSON_OK;
  return fail(POISSON_EINVAL, "%s must be 16-byte aligned", what);
}

extern "C" int last_error(void) { return g_err; }
extern "C" const char* last_error_message(void) { return g_msg; }

// ------------------------------------------------------------------ constants

static constexpr int R2R_NT = 512;
static constexpr int R2R_EMAX_D = 8;    // complex values per thread, FP64
static constexpr int R2R_EMAX_F = 16;   // complex values per thread, FP32
static constexpr int TRI_NT = 512;
static constexpr int MAX_TRANSFORM_N = 1024;
static constexpr int MAX_SOLVE_N = 512;
static constexpr size_t LDS_LIMIT = 160 * 1024;

// ------------------------------------------------------------------ tables

// cos and sin of pi*M/(4n) for an integer M: the angle is reduced exactly
// (in integers) to [0, pi/4] before the library call, so symmetric angles
// give exactly symmetric values.
static void cos_sin_quarter(long long M, long long n, double& c, double& s) {
  const long long turn = 8 * n;
  M %= turn;
  if (M < 0) M += turn;
  double ss = 1.0, sc = 1.0;
  if (M > 4 * n) { M = turn - M; ss = -1.0; }      // theta -> 2 pi - theta
  if (M > 2 * n) { M = 4 * n - M; sc = -1.0; }     // theta -> pi - theta
  bool swap = false;
  if (M > n) { M = 2 * n - M; swap = true; }       // theta -> pi/2 - theta
  const double th = M_PI * (double)M / (4.0 * (double)n);
  double cc = std::cos(th), sn = std::sin(th);
  if (swap) std::swap(cc, sn);
  c = sc * cc;
  s = ss * sn;
}

// e^{-i pi M/(4n)}
static cplx<double> expm(long long M, long long n) {
  double c, s;
  cos_sin_quarter(M, n, c, s);
  return {c, -s};
}

// Table 1: lambda_q = -4 sin^2(theta_q), theta_q = pi M_q / (4n).
static double eigenvalue(int kind, int n, int q) {
  long long M;
  if (kind == BC_DD_NODE || kind == BC_NN_NODE) {   // theta = pi(q+1)/(2(n+1)), pi q/(2(n-1))
    double c, s;
    if (kind == BC_DD_NODE) cos_sin_quarter(2LL * (q + 1), n + 1, c, s);
    else cos_sin_quarter(2LL * q, n - 1, c, s);
    return -4.0 * s * s;
  }
  switch (kind) {
    case BC_PERIODIC: M = 4LL * ((q + 1) / 2); break;   // wavenumber of storage slot q
    case BC_NN: M = 2LL * q; break;
    case BC_DD: M = 2LL * (q + 1); break;
    default: M = 2LL * q + 1; break;                      // ND and DN
  }
  double c, s;
  cos_sin_quarter(M, n, c, s);
  return -4.0 * s * s;
}

static bool factor_radices(int m, std::vector<int>& radices) {
  radices.clear();
  int e2 = 0;
  while (m % 2 == 0) { m /= 2; ++e2; }
  int n8 = e2 / 3, rem = e2 % 3, n4 = 0, n2 = 0;
  if (rem == 1) { if (n8 > 0) { --n8; n4 = 2; } else n2 = 1; }
  if (rem == 2) n4 = 1;
  for (int i = 0; i < n8; ++i) radices.push_back(8);
  for (int i = 0; i < n4; ++i) radices.push_back(4);
  for (int i = 0; i < n2; ++i) radices.push_back(2);
  for (int p : {3, 5})
    while (m % p == 0) { m /= p; radices.push_back(p); }
  return m == 1 && radices.size() <= 16;
}

// ------------------------------------------------------------------ plan

struct AxisTables {           // one transformed axis
  int axis = 0, n = 0, kind = 0, m = 0;
  std::vector<int> radices;
  size_t off_d = 0, off_f = 0;   // byte offsets of the twiddle block (FP64 / FP32)
};

struct poisson_plan {
  int dims[3];
  int bc[3];
  double h[3];                 // uniform spacing (x, y) ; z uses dz
  std::vector<double> dz;
  bool z_uniform;
  double shift = 0.0;          // Helmholtz shift: (A + shift) Phi = f
  bool generic_r2r = false;    // POISSON_GENERIC_R2R=1: size-generic transform kernel only
  bool generic_tri = false;    // POISSON_GENERIC_TRI=1: size-generic elimination kernel only
  int grid_cap = 0;            // POISSON_GRID_CAP=B: at most B blocks per stage launch (0: none)
  int rk3_kernel = 0;          // POISSON_RK3_KERNEL: 0 fused (default), 1 "tiled", 2 "simple"
  bool rk3_general = false;    // POISSON_RK3_GENERAL=1: the fused kernel's general z loop on whole tiles too
  bool plane_off = false;      // POISSON_PLANE=0: no small-plane transforms
  char* plane_mats = nullptr;  // small grids: dense transform matrices (FP64, then FP32)
  size_t plane_off_f = 0;      // byte offset of the FP32 copy in plane_mats
  int t1, t2, s;
  bool singular, s_periodic;
  int device;
  AxisTables ax[2];
  // elimination axis tables
  size_t off_tri_d = 0, off_tri_f = 0;     // a, b, c, w   (4 n_s)
  // Lines whose length has no size-specialised kernel are run in the kernel
  // of the next specialised length pad_n (0: not padded), with the tables
  // extended by decoupled rows (see plan_create).
  int pad_n = 0;
  size_t off_tri_pad = 0;                  // a, b, c, w   (4 pad_n), FP64
  size_t off_lam_d = 0, off_lam_f = 0;     // lamu, lamv
  size_t off_ops[3] = {0, 0, 0};           // per axis: a, b, c, h (FP64, residual)
  size_t off_proj[3] = {0, 0, 0};          // per axis: 1/h (n), 1/centre distance (n + 1)
  int nu = 0, nv = 0;
  int P = 1, lcmax = 1;
  char* dtab = nullptr;        // device tables
  size_t tab_bytes = 0;
  // refinement
  int mode = POISSON_FP64;
  double tol = 1e-10;
  int max_iters = 8;
  double* f64 = nullptr;       // FP64 copy of f
  float* e32 = nullptr;        // FP32 residual / correction
  bool ws_external = false;    // f64 / e32 lent by the owner (a server slot), not freed here
  double* stats = nullptr;     // device reduction slots
  double* stats_host = nullptr;
  size_t ws_bytes = 0;
  int last_iters = 1;
  double last_rel = 0.0;
  int last_converged = 1;
};

static size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }
// Non-staggered (node) boundary pairs: DST-I / DCT-I transforms.
static bool node_pair(int kind) { return kind == BC_DD_NODE || kind == BC_NN_NODE; }
static constexpr size_t align_up_c(size_t v, size_t a) { return (v + a - 1) / a * a; }

// ------------------------------------------------------------------ variants

// Elimination chunking: rows per chunk x chunks per line.
template <int RPC_, int P_>
struct TriCfg {
  static constexpr int RPC = RPC_, P = P_;
};

static constexpr int kFastVariants = 8;   // transform: tile shape x radix order, + staging forms
static constexpr int kAsyncVariant = 4;   // 4, 5, 6: asynchronous staging in tile shape 0, 1, 2
static constexpr int kRegStageVariant = 7;  // register-staged 32-line tiles (FP64, 512, strided)
static constexpr int kTriVariants = 4;    // elimination: two chunkings, staging, direct
static constexpr int kTriAsyncVariant = 2;
static constexpr int kTriDirectVariant = 3;   // contiguous lines, registers only

// Call f(FastVar<M, V>{}) for a specialised transform length; -1 otherwise.
template <typename F>
static long long with_fast_cfg(int M, int V, F&& f) {
  switch (M * 4 + (V & 3)) {
#define POISSON_FV(M_, V_) case M_ * 4 + V_: return f(FastVar<M_, V_>{});
#define POISSON_FM(M_) POISSON_FV(M_, 0) POISSON_FV(M_, 1) POISSON_FV(M_, 2) POISSON_FV(M_, 3)
    POISSON_FM(16) POISSON_FM(32) POISSON_FM(48) POISSON_FM(64)
    POISSON_FM(96) POISSON_FM(128) POISSON_FM(192) POISSON_FM(256)
    // single solves only (the batched kernel takes the lengths above)
    POISSON_FM(72) POISSON_FM(80) POISSON_FM(144) POISSON_FM(160)
#undef POISSON_FM
#undef POISSON_FV
    default: return -1;
  }
}

// Call f(TriCfg<RPC, P>{}) for a specialised elimination length; -1 otherwise.
template <typename F>
static long long with_tri_cfg(int n, int V, F&& f) {
  switch (n * 2 + (V & 1)) {
#define POISSON_TV(N_, V_, R_, P_) case N_ * 2 + V_: return f(TriCfg<R_, P_>{});
    POISSON_TV(64, 0, 4, 16) POISSON_TV(64, 1, 2, 32)
    POISSON_TV(96, 0, 6, 16) POISSON_TV(96, 1, 3, 32)
    POISSON_TV(128, 0, 8, 16) POISSON_TV(128, 1, 4, 32)
    POISSON_TV(192, 0, 12, 16) POISSON_TV(192, 1, 6, 32)
    POISSON_TV(256, 0, 8, 32) POISSON_TV(256, 1, 16, 16)
    POISSON_TV(384, 0, 6, 64) POISSON_TV(384, 1, 12, 32)
    POISSON_TV(512, 0, 8, 64) POISSON_TV(512, 1, 16, 32)
#undef POISSON_TV
    default: return -1;
  }
}

// Variants chosen by the autotuner, per device, kernel family (0 transform,
// 1 elimination), element size, length and layout (0 strided, 1
// contiguous); variant 0 where nothing was tuned.
static std::mutex g_tune_mu;
static std::map<std::tuple<int, int, int, int, int>, int> g_tune;

// Variant used where nothing was tuned.  Transforms: the asynchronous-staging
// form for the lengths it is compiled for, else variant 0.  Its tile shape:
// shape 1 (half the lines per tile, so that twice the blocks fit in a CU's
// LDS) for FP64 length 256 and for FP32 length 512 on the contiguous axis,
// where the extra overlap pays most; shape 2 (32 lines) for FP32 length 512
// on the strided axes, whose tile rows are then 128 bytes long; else shape
// 0, whose wider tile rows use each DRAM page better.
static int default_choice(int family, int bytes, int n, int layout) {
  if (family == 1) {
    // elimination: the direct form on contiguous lines (the 512^3 cube's
    // lines of 512 points: 0.438 against 0.509 ms in FP64, 0.337 against
    // 0.420 ms for the staging form in FP32); the second chunking (shorter
    // interface reduction) on strided lines of 384 points, and of 256
    // points in FP32
    if (layout == 1) return kTriDirectVariant;
    return layout == 0 && (n == 384 || (bytes == 4 && n == 256)) ? 1 : 0;
  }
  if (n != 128 && n != 256) return 0;
  // FP64 length 512 on a strided axis: the register-staged 32-line tile,
  // whose 256-byte rows use each DRAM page better (measured on the 512^3
  // cube, forward + backward: z 1.037 against 1.086 ms, y 0.876 against
  // 0.895 ms for the LDS-staged 16-line tile)
  if (bytes == 8 && n == 256 && layout == 0) return kRegStageVariant;
  int shape = 0;
  if (bytes == 8 && n == 128) shape = 1;
  if (bytes == 4 && n == 256) shape = layout == 1 ? 1 : 2;
  return kAsyncVariant + shape;
}

static int tuned_choice(int family, int bytes, int n, int layout) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  const auto it = g_tune.find(std::make_tuple(dev, family, bytes, n, layout));
  return it == g_tune.end() ? default_choice(family, bytes, n, layout) : it->second;
}

static void set_tuned_choice(int family, int bytes, int n, int layout, int v) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune[std::make_tuple(dev, family, bytes, n, layout)] = v;
}

static int lds_setup_once() {
  static std::once_flag once;
  static int status = 0;
  std::call_once(once, [] {
    hipError_t e = hipSuccess;
#define ALLOW(k) if (e == hipSuccess) e = hipFuncSetAttribute((const void*)(k), hipFuncAttributeMaxDynamicSharedMemorySize, (int)LDS_LIMIT)
    ALLOW((r2r_kernel<double, R2R_EMAX_D, R2R_NT>));
    ALLOW((r2r_kernel<float, R2R_EMAX_F, R2R_NT>));
    for (int M : {16, 32, 48, 64, 72, 80, 96, 128, 144, 160, 192, 256})
      for (int V = 0; V < 4; ++V)
        with_fast_cfg(M, V, [&](auto cfg) {
          using C = decltype(cfg);
          ALLOW((r2r_fast_kernel<double, C>));
          ALLOW((r2r_fast_kernel<float, C>));
          return 0LL;
        });
    ALLOW((tridiag_kernel<double, 4, TRI_NT>));
    ALLOW((tridiag_kernel<double, 8, TRI_NT>));
    ALLOW((tridiag_kernel<float, 4, TRI_NT>));
    ALLOW((tridiag_kernel<float, 8, TRI_NT>));
    for (int n : {64, 96, 128, 192, 256, 384, 512})
      for (int V = 0; V < 2; ++V)
        with_tri_cfg(n, V, [&](auto cfg) {
          using C = decltype(cfg);
          ALLOW((tri_fast_kernel<double, C::RPC, C::P, 0>));
          ALLOW((tri_fast_kernel<double, C::RPC, C::P, 1>));
          ALLOW((tri_fast_kernel<float, C::RPC, C::P, 0>));
          ALLOW((tri_fast_kernel<float, C::RPC, C::P, 1>));
          return 0LL;
        });
    ALLOW((tri_fast_kernel<double, 2, 16, 0>));
    ALLOW((tri_fast_kernel<float, 2, 16, 0>));
    ALLOW((tri_fast_kernel<double, 3, 16, 0>));
    ALLOW((tri_fast_kernel<float, 3, 16, 0>));
    ALLOW((plane_transform_kernel<double, false>));
    ALLOW((plane_transform_kernel<double, true>));
    ALLOW((plane_transform_kernel<float, false>));
    ALLOW((plane_transform_kernel<float, true>));
    ALLOW((batch_r2r_kernel<double>));
    ALLOW((batch_tri_kernel<double>));
    ALLOW((batch_r2r_kernel<float>));
    ALLOW((batch_tri_kernel<float>));
#undef ALLOW
    status = e == hipSuccess ? 0 : fail(POISSON_EHIP, "hipFuncSetAttribute: %s", hipGetErrorString(e));
  });
  return status;
}

static int ilog2(int v) {
  int l = 0;
  while ((1 << (l + 1)) <= v) ++l;
  return l;
}
static int pow2_ceil_log(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

// Geometry of the lines along axis `axis` (0 = x, 1 = y, 2 = z) of an
// nx x ny x nz field, with at most 2^lognl_max lines per tile.
static LineGeom make_geom(int axis, const int* dims, int lognl_max) {
  LineGeom g{};
  const long long nx = dims[0], ny = dims[1], nz = dims[2];
  if (axis == 0) {
    g.layout = 1;
    g.n = dims[0];
    g.sp = 1;
    g.nlines = (int)(ny * nz);
    g.lognl = std::min(lognl_max, pow2_ceil_log(g.nlines));
    g.logtpl = std::min(6, pow2_ceil_log(g.n));
    g.ntiles = (g.nlines + (1 << g.lognl) - 1) >> g.lognl;
  } else {
    g.layout = 0;
    g.n = dims[axis];
    g.sp = axis == 1 ? nx : nx * ny;
    g.nx = (int)nx;
    g.nb = axis == 1 ? (int)nz : (int)ny;
    g.sb = axis == 1 ? nx * ny : nx;
    g.logtxw = std::min(lognl_max, pow2_ceil_log(g.nx));
    g.lognbt = std::min(lognl_max - g.logtxw, pow2_ceil_log(g.nb));
    g.lognl = g.logtxw + g.lognbt;
    g.tiles_x = (g.nx + (1 << g.logtxw) - 1) >> g.logtxw;
    g.ntiles = g.tiles_x * ((g.nb + (1 << g.lognbt) - 1) >> g.lognbt);
  }
  return g;
}

// ceil(2^32 / d) for 1 < d < 2^16 (0 for d = 1: never used)
static unsigned div_magic(int d) {
  return d > 1 ? (unsigned)((((unsigned long long)1 << 32) + d - 1) / d) : 0u;
}

static thread_local int t_grid_cap = 0;
int poisson_dev::grid_cap_blocks() { return t_grid_cap; }

// Persistent grid: as many blocks as can be resident at once (CUs x blocks
// per CU for this kernel, block size and LDS), each looping over tiles, so
// that no block pays launch and set-up more than once per launch.
static int resident_grid(const void* fn, int block, size_t lds, long long ntiles) {
  static std::mutex mu;
  static std::vector<std::pair<std::pair<const void*, size_t>, std::pair<int, int>>> cache;
  int dev = 0;
  (void)hipGetDevice(&dev);
  int per_cu = 0, cus = 0;
  {
    std::lock_guard<std::mutex> lk(mu);
    for (auto& e : cache)
      if (e.first.first == fn && e.first.second == lds + (size_t)dev * 0x100000000ull) {
        per_cu = e.second.first;
        cus = e.second.second;
      }
  }
  if (!cus) {
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) cus = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, block, lds) != hipSuccess) per_cu = 1;
    per_cu = std::max(per_cu, 1);
    std::lock_guard<std::mutex> lk(mu);
    cache.push_back({{fn, lds + (size_t)dev * 0x100000000ull}, {per_cu, cus}});
  }
  long long blocks = (long long)cus * per_cu;
  const int cap = grid_cap_blocks();
  if (cap > 0) blocks = std::min<long long>(blocks, cap);
  return (int)std::min<long long>(ntiles, blocks);
}

// ------------------------------------------------------------------ launches

// Launch arguments of the size-specialised transform kernel (r2r_fast.h)
// of configuration C.
template <typename T, typename C>
static R2RFastArgs<T> fast_args(const poisson_plan* p, const AxisTables& A, int inverse, T* data,
                                const double* skip, double* out64 = nullptr) {
  constexpr int M = C::M;
  R2RFastArgs<T> a{};
  a.data = data;
  a.g = make_geom(A.axis, p->dims, ilog2(C::NL));
  a.kind = A.kind;
  a.inverse = inverse;
  if (!inverse) a.scale = (T)1;
  else a.scale = (T)(node_pair(A.kind) ? 1.0 / (2.0 * A.m) : A.kind <= BC_DD ? 1.0 / A.n : 1.0 / (2.0 * A.n));
  const cplx<T>* tw = reinterpret_cast<const cplx<T>*>(p->dtab + (sizeof(T) == 8 ? A.off_d : A.off_f));
  a.tw_fft = tw;
  a.tw_split = tw + M;
  a.tw_quarter = tw + 2 * M + 1;
  a.tw_pre = tw + 3 * M + 2;
  a.tw_post = tw + 4 * M + 2;
  a.skip = skip;
  a.out64 = out64;
  return a;
}

template <typename T, typename C>
static int launch_fast(const poisson_plan* p, const AxisTables& A, int inverse, T* data,
                       hipStream_t st, const double* skip, double* out64 = nullptr) {
  const R2RFastArgs<T> a = fast_args<T, C>(p, A, inverse, data, skip, out64);
  const size_t lds = fast_lds_bytes<T, C>();
  const void* fn = reinterpret_cast<const void*>(&r2r_fast_kernel<T, C>);
  hipLaunchKernelGGL((r2r_fast_kernel<T, C>), dim3(resident_grid(fn, 512, lds, a.g.ntiles)),
                     dim3(512), lds, st, a);
  HIP_TRY(hipGetLastError());
  return POISSON_OK;
}

// Asynchronous-staging form (r2r_fast.h) for lengths 2M, M in {128, 256};
// -1 if it does not apply (length, or strided rows that do not split into
// 16-byte pieces).
// Staging-transform tile shapes compiled for length M = n/2 in type T.
template <typename T>
static bool async_shape_exists(int m, int shape) {
  if (m != 128 && m != 256) return false;
  return shape == 0 || shape == 1 || (shape == 2 && m == 256 && sizeof(T) == 4);
}

template <typename T>
static int launch_async(const poisson_plan* p, const AxisTables& A, int shape, int inverse,
                        T* data, hipStream_t st, const double* skip, double* out64 = nullptr) {
  if (A.m != 128 && A.m != 256) return -1;
  if (A.axis != 0 && p->dims[0] % (int)(16 / sizeof(T)) != 0) return -1;
  if (!async_shape_exists<T>(A.m, shape)) return -1;
  R2RFastArgs<T> a;
  switch (A.m * 4 + shape) {
    case 128 * 4 + 0: a = fast_args<T, AsyncVar<128, 0>>(p, A, inverse, data, skip, out64); break;
    case 128 * 4 + 1: a = fast_args<T, AsyncVar<128, 1>>(p, A, inverse, data, skip, out64); break;
    case 256 * 4 + 0: a = fast_args<T, AsyncVar<256, 0>>(p, A, inverse, data, skip, out64); break;
    case 256 * 4 + 1: a = fast_args<T, AsyncVar<256, 1>>(p, A, inverse, data, skip, out64); break;
    default: a = fast_args<T, AsyncVar<256, 2>>(p, A, inverse, data, skip, out64); break;
  }
  const hipError_t e = async_transform_launch(a, A.m, shape, A.kind, inverse, st);
  if (e != hipSuccess)
    return fail(POISSON_EHIP, "staging transform launch: %s", hipGetErrorString(e));
  return POISSON_OK;
}

// True if the asynchronous-staging form in tile shape `shape` applies to
// axis A in type T.
template <typename T>
static bool async_applies(const poisson_plan* p, const AxisTables& A, int shape) {
  return async_shape_exists<T>(A.m, shape) &&
         (A.axis == 0 || p->dims[0] % (int)(16 / sizeof(T)) == 0);
}

// True if the register-staged form applies to axis A in type T: FP64,
// length 512, strided axis, nx a multiple of 32 (a tile is 32 consecutive x
// of one band, and every line of every tile exists, so its stores need no
// branch) and element offsets within a tile's lines that fit 32 bits.  The
// launch also needs a 16-byte aligned field (pairs of lines are read with
// 16-byte loads).
template <typename T>
static bool regstage_applies(const poisson_plan* p, const AxisTables& A) {
  if (sizeof(T) != 8 || A.m != 256 || A.axis == 0 || p->dims[0] % 32) return false;
  const long long sp = A.axis == 1 ? (long long)p->dims[0] : (long long)p->dims[0] * p->dims[1];
  return 32 + (long long)A.n * sp < (1LL << 32);
}

// Specialised transform of axis A in variant V (-1: the length has none).
template <typename T>
static int launch_fast_variant(const poisson_plan* p, const AxisTables& A, int V, int inverse,
                               T* data, hipStream_t st, const double* skip,
                               double* out64 = nullptr) {
  if (V == kRegStageVariant) {
    if constexpr (sizeof(T) == 8) {
      if (regstage_applies<T>(p, A) && (reinterpret_cast<uintptr_t>(data) & 15) == 0) {
        const R2RFastArgs<T> a = fast_args<T, RegStageCfg>(p, A, inverse, data, skip);
        // nontemporal accesses on fields at least twice the 256 MB
        // Infinity Cache (smaller ones can stay there between stages)
        const bool hinted = (double)p->dims[0] * p->dims[1] * p->dims[2] * sizeof(T) >=
                            (double)(512u << 20);
        const hipError_t e = regstage_launch(a, A.kind, inverse, hinted, st);
        if (e != hipSuccess)
          return fail(POISSON_EHIP, "register-staged transform launch: %s", hipGetErrorString(e));
        return POISSON_OK;
      }
    }
    V = kAsyncVariant;   // elsewhere: the LDS-staged form (itself variant 0 where it does not apply)
  }
  if (V >= kAsyncVariant) {
    const int rc = launch_async<T>(p, A, V - kAsyncVariant, inverse, data, st, skip, out64);
    if (rc != -1) return rc;
    V = 0;
  }
  return (int)with_fast_cfg(A.m, V, [&](auto cfg) {
    return (long long)launch_fast<T, decltype(cfg)>(p, A, inverse, data, st, skip, out64);
  });
}

// out64 (FP32 only): write the widened result there instead of in place.
template <typename T>
static int launch_r2r(const poisson_plan* p, int role, int inverse, T* data, hipStream_t st,
                      const double* skip = nullptr, double* out64 = nullptr) {
  const AxisTables& A = p->ax[role];
  if constexpr (sizeof(T) == 8) out64 = nullptr;
  t_grid_cap = p->grid_cap;
  if (!p->generic_r2r && !node_pair(A.kind)) {
    const int rc = launch_fast_variant<T>(p, A, tuned_choice(0, sizeof(T), A.m, A.axis == 0),
                                          inverse, data, st, skip, out64);
    if (rc != -1) return rc;
  }
  constexpr int EMAX = sizeof(T) == 8 ? R2R_EMAX_D : R2R_EMAX_F;
  const int cap_reals = 2 * EMAX * R2R_NT;
  const int rows = 2 * A.m;   // tile rows per line (node pairs: their extension)
  const int lognl_max = ilog2(std::max(1, std::min(cap_reals / rows, R2R_NT)));
  R2RArgs<T> a{};
  a.data = data;
  a.g = make_geom(A.axis, p->dims, lognl_max);
  a.kind = A.kind;
  a.inverse = inverse;
  a.m = A.m;
  a.npass = (int)A.radices.size();
  int Ns = 1;
  for (int i = 0; i < a.npass; ++i) {
    a.radix[i] = A.radices[i];
    a.ns_magic[i] = div_magic(Ns);
    Ns *= A.radices[i];
  }
  a.nlp = (1 << a.g.lognl) | 1;
  a.n_magic = div_magic(A.n);
  if (!inverse) a.scale = (T)1;
  else a.scale = (T)(node_pair(A.kind) ? 1.0 / (2.0 * A.m) : A.kind <= BC_DD ? 1.0 / A.n : 1.0 / (2.0 * A.n));
  const char* base = p->dtab + (sizeof(T) == 8 ? A.off_d : A.off_f);
  const cplx<T>* tw = reinterpret_cast<const cplx<T>*>(base);
  a.tw_fft = tw;
  a.tw_split = tw + A.m;
  a.tw_quarter = tw + 2 * A.m + 1;
  a.tw_pre = tw + 3 * A.m + 2;
  a.tw_post = tw + 4 * A.m + 2;
  a.skip = skip;
  a.out64 = out64;
  const size_t lds = (size_t)rows * a.nlp * sizeof(T);
  if (lds > LDS_LIMIT) return fail(POISSON_EUNSUPPORTED, "transform tile needs %zu B of LDS", lds);
  const void* fn = reinterpret_cast<const void*>(&r2r_kernel<T, EMAX, R2R_NT>);
  hipLaunchKernelGGL((r2r_kernel<T, EMAX, R2R_NT>),
                     dim3(resident_grid(fn, R2R_NT, lds, a.g.ntiles)), dim3(R2R_NT), lds, st, a);
  HIP_TRY(hipGetLastError());
  return POISSON_OK;
}

// Launch arguments of the size-specialised elimination kernel (tri_fast.h).
template <typename T, int RPC, int P>
static TriFastArgs<T> tri_fast_args(const poisson_plan* p, T* data, const double* skip) {
  using L = TriFastLayout<T, RPC, P>;
  TriFastArgs<T> a{};
  a.data = data;
  a.g = make_geom(p->s, p->dims, ilog2(L::NL));
  a.periodic = p->s_periodic;
  a.singular = p->singular;
  a.nu = p->nu;
  a.nv = p->nv;
  // FP64 tables for both field precisions (the recurrences run in FP64);
  // a padded plan's tables have L::N = pad_n rows
  const double* tri = reinterpret_cast<const double*>(
      p->dtab + (p->pad_n && p->pad_n == L::N ? p->off_tri_pad : p->off_tri_d));
  a.nreal = p->dims[p->s];
  a.a = tri;
  a.b = tri + L::N;
  a.c = tri + 2 * L::N;
  a.w = tri + 3 * L::N;
  const double* lam = reinterpret_cast<const double*>(p->dtab + p->off_lam_d);
  a.lamu = lam;
  a.lamv = lam + p->nu;
  a.skip = skip;
  return a;
}

template <typename T, int RPC, int P>
static int launch_tri_fast(const poisson_plan* p, T* data, hipStream_t st, const double* skip) {
  using L = TriFastLayout<T, RPC, P>;
  const TriFastArgs<T> a = tri_fast_args<T, RPC, P>(p, data, skip);
  const size_t lds = tri_fast_lds_bytes<T, RPC, P>();
  // one kernel per layout (strided, contiguous)
  void (*k)(TriFastArgs<T>) =
      a.g.layout == 0 ? tri_fast_kernel<T, RPC, P, 0> : tri_fast_kernel<T, RPC, P, 1>;
  const void* fn = reinterpret_cast<const void*>(k);
  hipLaunchKernelGGL(k, dim3(resident_grid(fn, L::NT, lds, a.g.ntiles)), dim3(L::NT), lds, st, a);
  HIP_TRY(hipGetLastError());
  return POISSON_OK;
}

// True if the staging elimination applies in type T (strided rows must split
// into 16-byte pieces).
template <typename T>
static bool tri_async_applies(const poisson_plan* p) {
  return p->s == 0 || p->dims[0] % (int)(16 / sizeof(T)) == 0;
}

// True if the direct elimination applies: contiguous lines whose chunks (of
// the variant-0 chunking) are whole 16-byte pieces, a 16-byte aligned field,
// and a line count that splits into whole groups of 64 / P lines.
template <typename T>
static bool tri_direct_applies(const poisson_plan* p, const T* data) {
  if (p->s != 0 || (reinterpret_cast<uintptr_t>(data) & 15) != 0) return false;
  const long long rpc = with_tri_cfg(p->dims[0], 0, [](auto cfg) {
    return (long long)decltype(cfg)::RPC;
  });
  const long long lanes = with_tri_cfg(p->dims[0], 0, [](auto cfg) {
    return (long long)decltype(cfg)::P;
  });
  // whole groups of 64 / P lines (a wave's lines per step)
  return rpc > 0 && (rpc * (long long)sizeof(T)) % 16 == 0 &&
         ((long long)p->dims[1] * p->dims[2]) % (64 / lanes) == 0;
}

// Specialised elimination in variant V (-1: the length has none).
template <typename T>
static int launch_tri_variant(const poisson_plan* p, int V, T* data, hipStream_t st,
                              const double* skip) {
  if (V == kTriDirectVariant) {
    if (tri_direct_applies<T>(p, data)) {
      const int n = p->dims[p->s];
      const long long rc = with_tri_cfg(n, 0, [&](auto cfg) {
        using C = decltype(cfg);
        const TriFastArgs<T> a = tri_fast_args<T, C::RPC, C::P>(p, data, skip);
        const hipError_t e = direct_elimination_launch(a, n, st);
        return (long long)(e == hipSuccess ? POISSON_OK
                                           : fail(POISSON_EHIP, "direct elimination launch: %s",
                                                  hipGetErrorString(e)));
      });
      if (rc != -1) return (int)rc;
    }
    V = 0;
  }
  if (V == kTriAsyncVariant) {
    if (tri_async_applies<T>(p)) {
      const int n = p->dims[p->s];
      const long long rc = with_tri_cfg(n, 0, [&](auto cfg) {
        using C = decltype(cfg);
        const TriFastArgs<T> a = tri_fast_args<T, C::RPC, C::P>(p, data, skip);
        const hipError_t e = async_elimination_launch(a, n, st);
        return (long long)(e == hipSuccess ? POISSON_OK
                                           : fail(POISSON_EHIP, "staging elimination launch: %s",
                                                  hipGetErrorString(e)));
      });
      if (rc != -1) return (int)rc;
    }
    V = 0;
  }
  return (int)with_tri_cfg(p->dims[p->s], V, [&](auto cfg) {
    using C = decltype(cfg);
    return (long long)launch_tri_fast<T, C::RPC, C::P>(p, data, st, skip);
  });
}

// True if lines of n points have size-specialised elimination kernels.
static bool tri_fast_length(int n) {
  return with_tri_cfg(n, 0, [](auto) { return 0LL; }) == 0;
}

// Complex length M of the size-specialised transform kernel for axis A, or
// 0 if its length has none, among the lengths the batched kernel takes
// (single solves also have 72, 80, 144 and 160).
static int r2r_fast_length(const AxisTables& A) {
  if (node_pair(A.kind)) return 0;
  switch (A.m) {
    case 16: case 32: case 48: case 64: case 96: case 128: case 192: case 256: return A.m;
    default: return 0;
  }
}

template <typename T>
static int launch_tridiag(const poisson_plan* p, T* data, hipStream_t st,
                          const double* skip = nullptr) {
  t_grid_cap = p->grid_cap;
  if (p->pad_n) {   // padded lines: the plain chunked kernel of length pad_n
    return (int)with_tri_cfg(p->pad_n, 0, [&](auto cfg) {
      using C = decltype(cfg);
      return (long long)launch_tri_fast<T, C::RPC, C::P>(p, data, st, skip);
    });
  }
  if (!p->generic_tri) {
    const int n = p->dims[p->s];
    // small grids (transforms as dense matrices): lines of 32 or 48 points in
    // the 16-lane chunking, instead of the size-generic kernel
    if (p->plane_mats && n == 32) return launch_tri_fast<T, 2, 16>(p, data, st, skip);
    if (p->plane_mats && n == 48) return launch_tri_fast<T, 3, 16>(p, data, st, skip);
    const int rc = launch_tri_variant<T>(p, tuned_choice(1, sizeof(T), n, p->s == 0), data, st, skip);
    if (rc != -1) return rc;
  }
  TriArgs<T> a{};
  a.data = data;
  const int lines = TRI_NT / p->P;            // lines covered by the block's threads
  a.g = make_geom(p->s, p->dims, ilog2(lines));
  a.P = p->P;
  a.lcmax = p->lcmax;
  a.nlp = lines | 1;
  a.cpitch = (p->lcmax * a.nlp) | 1;
  a.n_magic = div_magic(p->dims[p->s]);
  a.periodic = p->s_periodic;
  a.singular = p->singular;
  a.nu = p->nu;
  const size_t ns = (size_t)p->dims[p->s];
  const T* tri = reinterpret_cast<const T*>(p->dtab + (sizeof(T) == 8 ? p->off_tri_d : p->off_tri_f));
  a.a = tri;
  a.b = tri + ns;
  a.c = tri + 2 * ns;
  a.w = tri + 3 * ns;
  const T* lam = reinterpret_cast<const T*>(p->dtab + (sizeof(T) == 8 ? p->off_lam_d : p->off_lam_f));
  a.lamu = lam;
  a.lamv = lam + p->nu;
  a.skip = skip;
  // tile + row-offset table (one int per row)
  const size_t lds = align_up((size_t)p->P * a.cpitch * sizeof(T), 16) + (size_t)ns * sizeof(int);
  if (lds > LDS_LIMIT) return fail(POISSON_EUNSUPPORTED, "elimination tile needs %zu B of LDS", lds);
  const dim3 block(TRI_NT);
  if (p->lcmax - 1 <= 4) {
    const void* fn = reinterpret_cast<const void*>(&tridiag_kernel<T, 4, TRI_NT>);
    hipLaunchKernelGGL((tridiag_kernel<T, 4, TRI_NT>),
                       dim3(resident_grid(fn, TRI_NT, lds, a.g.ntiles)), block, lds, st, a);
  } else {
    const void* fn = reinterpret_cast<const void*>(&tridiag_kernel<T, 8, TRI_NT>);
    hipLaunchKernelGGL((tridiag_kernel<T, 8, TRI_NT>),
                       dim3(resident_grid(fn, TRI_NT, lds, a.g.ntiles)), block, lds, st, a);
  }
  HIP_TRY(hipGetLastError());
  return POISSON_OK;
}

// The three steps of Sec. 2.1: forward transforms t1 then t2, elimination
// along s, backward transforms t2 then t1.  out64 (FP32 only): the last
// launch writes the widened solution there instead of in place.
// Both transforms of one direction on a small grid (plane_kernels.h).
template <typename T>
static int launch_plane(const poisson_plan* p, bool inverse, T* data, hipStream_t st,
                        const double* skip, double* out64) {
  const int nx = p->dims[0], ny = p->dims[1];
  const size_t n2x = (size_t)nx * nx, n2y = (size_t)ny * ny;
  const T* m = reinterpret_cast<const T*>(p->plane_mats + (sizeof(T) == 8 ? 0 : p->plane_off_f));
  // order: forward x, forward y, backward x, backward y
  const T* mx = m + (inverse ? n2x + n2y : 0);
  const T* my = mx + n2x;
  const size_t lds = (2 * (size_t)nx * ny + n2x + n2y) * sizeof(T);
  if (inverse)
    hipLaunchKernelGGL((plane_transform_kernel<T, true>), dim3(p->dims[2]), dim3(PLANE_NT), lds, st,
                       data, out64, mx, my, nx, ny, skip);
  else
    hipLaunchKernelGGL((plane_transform_kernel<T, false>), dim3(p->dims[2]), dim3(PLANE_NT), lds, st,
                       data, out64, mx, my, nx, ny, skip);
  HIP_TRY(hipGetLastError());
  return POISSON_OK;
}

template <typename T>
static int solve_typed(const poisson_plan* p, T* data, hipStream_t st,
                       const double* skip = nullptr, double* out64 = nullptr) {
  int rc;
  if (p->plane_mats) {             // small grid: both transforms of a direction in one launch
    if ((rc = launch_plane<T>(p, false, data, st, skip, nullptr))) return rc;
    if ((rc = launch_tridiag<T>(p, data, st, skip))) return rc;
    return launch_plane<T>(p, true, data, st, skip, sizeof(T) == 8 ? nullptr : out64);
  }
  if ((rc = launch_r2r<T>(p, 0, 0, data, st, skip))) return rc;
  if ((rc = launch_r2r<T>(p, 1, 0, data, st, skip))) return rc;
  if ((rc = launch_tridiag<T>(p, data, st, skip))) return rc;
  if ((rc = launch_r2r<T>(p, 1, 1, data, st, skip))) return rc;
  if ((rc = launch_r2r<T>(p, 0, 1, data, st, skip, out64))) return rc;
  return POISSON_OK;
}

// Dense transform matrices of a small grid's two transformed axes (x and
// y), FP64 then FP32, in plane_mats: forward x, forward y, backward x,
// backward y, each n x n with row j the transform of unit vector j.  They
// are made by running the plan's own transform kernels (same tables, same
// variants) on the unit vectors, laid out as contiguous lines.
static int build_plane_matrices(poisson_plan* p) {
  const int n[2] = {p->dims[0], p->dims[1]};
  const int nmax = std::max(n[0], n[1]);
  double* tmp = nullptr;
  if (hipMalloc(&tmp, (size_t)nmax * nmax * sizeof(double)) != hipSuccess)
    return fail(POISSON_ENOMEM, "transform matrix scratch allocation failed");
  std::vector<double> h, eye;
  int rc = POISSON_OK;
  for (int inv = 0; inv < 2 && rc == POISSON_OK; ++inv)
    for (int r = 0; r < 2 && rc == POISSON_OK; ++r) {
      const int m = n[r];
      const size_t mm = (size_t)m * m;
      eye.assign(mm, 0.0);
      for (int j = 0; j < m; ++j) eye[(size_t)j * m + j] = 1.0;
      if (hipMemcpy(tmp, eye.data(), mm * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
        rc = fail(POISSON_EHIP, "transform matrix upload failed");
        break;
      }
      poisson_plan q = *p;            // the same tables; m lines of m contiguous points
      q.dims[0] = m;
      q.dims[1] = m;
      q.dims[2] = 1;
      q.ax[r].axis = 0;
      q.grid_cap = 0;
      q.plane_mats = nullptr;
      if ((rc = launch_r2r<double>(&q, r, inv, tmp, nullptr))) break;
      const size_t off = h.size();
      h.resize(off + mm);
      if (hipMemcpy(h.data() + off, tmp, mm * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess)
        rc = fail(POISSON_EHIP, "transform matrix download failed");
    }
  (void)hipFree(tmp);
  if (rc != POISSON_OK) return rc;
  const std::vector<float> hf(h.begin(), h.end());
  const size_t bytes_d = h.size() * sizeof(double);
  const size_t off_f = align_up(bytes_d, 256);
  const size_t total = off_f + hf.size() * sizeof(float);
  if (hipMalloc(&p->plane_mats, total) != hipSuccess)
    return fail(POISSON_ENOMEM, "transform matrix allocation (%zu B) failed", total);
  if (hipMemcpy(p->plane_mats, h.data(), bytes_d, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(p->plane_mats + off_f, hf.data(), hf.size() * sizeof(float), hipMemcpyHostToDevice) !=
          hipSuccess) {
    (void)hipFree(p->plane_mats);
    p->plane_mats = nullptr;
    return fail(POISSON_EHIP, "transform matrix upload failed");
  }
  p->plane_off_f = off_f;
  p->tab_bytes += total;
  return POISSON_OK;
}

// ------------------------------------------------------------------ plan_create

// Cell widths along axis q (x and y uniform, z from dz).
static std::vector<double> axis_widths(const poisson_plan* p, int q) {
  if (q == 2) return p->dz;
  return std::vector<double>(p->dims[q], p->h[q]);
}

// Rows of the 1D staggered operator on cell widths h (finite-volume form:
// centre distances are the mean of neighbouring widths; at a wall the ghost
// cell mirrors the edge cell, so a Neumann face adds +a_0 / +c_{n-1} to the
// diagonal and a Dirichlet face subtracts it; a periodic axis keeps a_0 and
// c_{n-1} as the wrap couplings).  out = [a | b | c | h], each n long.
static void axis_rows(const std::vector<double>& hs, int kind, double* out) {
  const int n = (int)hs.size();
  if (node_pair(kind)) {   // uniform node spacing: zero beyond DD ends, mirrored beyond NN ends
    double* a = out;
    double* b = a + n;
    double* c = b + n;
    double* w = c + n;
    const double inv = 1.0 / (hs[0] * hs[0]);
    for (int k = 0; k < n; ++k) {
      a[k] = k > 0 ? inv : 0.0;
      c[k] = k < n - 1 ? inv : 0.0;
      b[k] = -2.0 * inv;
      w[k] = hs[k];
    }
    if (kind == BC_NN_NODE && n > 1) {
      c[0] = 2.0 * inv;
      a[n - 1] = 2.0 * inv;
    }
    return;
  }
  const bool periodic = kind == BC_PERIODIC;
  std::vector<double> dc(n + 1);
  for (int k = 1; k < n; ++k) dc[k] = 0.5 * (hs[k - 1] + hs[k]);
  if (periodic) dc[0] = dc[n] = 0.5 * (hs[n - 1] + hs[0]);
  else { dc[0] = hs[0]; dc[n] = hs[n - 1]; }
  double* a = out;
  double* b = a + n;
  double* c = b + n;
  double* w = c + n;
  for (int k = 0; k < n; ++k) {
    a[k] = 1.0 / (hs[k] * dc[k]);
    c[k] = 1.0 / (hs[k] * dc[k + 1]);
    b[k] = -(a[k] + c[k]);
    w[k] = hs[k];
  }
  if (!periodic) {
    const bool low_n = kind == BC_NN || kind == BC_ND;
    const bool high_n = kind == BC_NN || kind == BC_DN;
    b[0] += low_n ? a[0] : -a[0];
    b[n - 1] += high_n ? c[n - 1] : -c[n - 1];
    a[0] = 0.0;
    c[n - 1] = 0.0;
  }
}

static bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

// Chunks per line of the elimination kernel: a power of two (the interface
// reduction is cyclic on a periodic axis), every chunk >= 2 rows, at most 8
// rows per chunk (64 chunks = one line per wavefront for long lines).
static int choose_chunks(int n, int& P, int& lcmax) {
  P = 1;
  while (P < 32 && n >= 4 * P) P *= 2;
  if ((n + P - 1) / P > 8 && n >= 2 * 64) P = 64;
  lcmax = (n + P - 1) / P;
  return lcmax - 1 <= 8 ? 0 : -1;
}

extern "C" poisson_plan* plan_create(int nx, int ny, int nz, double dx, double dy, const double* dz,
                                     int bc_x, int bc_y, int bc_z) {
  return plan_create_helmholtz(nx, ny, nz, dx, dy, dz, bc_x, bc_y, bc_z, 0.0);
}

extern "C" poisson_plan* plan_create_helmholtz(int nx, int ny, int nz, double dx, double dy,
                                               const double* dz, int bc_x, int bc_y, int bc_z,
                                               double shift) {
  g_err = 0;
  g_msg[0] = 0;
  if (nx < 1 || ny < 1 || nz < 1) { fail(POISSON_EINVAL, "sizes must be >= 1 (got %d %d %d)", nx, ny, nz); return nullptr; }
  if (!dz) { fail(POISSON_EINVAL, "dz is NULL"); return nullptr; }
  if (!finite_pos(dx) || !finite_pos(dy)) { fail(POISSON_EINVAL, "dx, dy must be finite and > 0"); return nullptr; }
  const int bcs[3] = {bc_x, bc_y, bc_z};
  for (int i = 0; i < 3; ++i)
    if (bcs[i] < BC_PERIODIC || bcs[i] > BC_NN_NODE) { fail(POISSON_EINVAL, "boundary pair %d out of range on axis %d", bcs[i], i); return nullptr; }
  if (!std::isfinite(shift) || shift > 0.0) { fail(POISSON_EINVAL, "the Helmholtz shift must be finite and <= 0"); return nullptr; }
  for (int k = 0; k < nz; ++k)
    if (!finite_pos(dz[k])) { fail(POISSON_EINVAL, "dz[%d] must be finite and > 0", k); return nullptr; }
  if ((long long)nx * ny * nz > (1LL << 34)) { fail(POISSON_EUNSUPPORTED, "grid too large"); return nullptr; }

  poisson_plan* p = new poisson_plan();
  p->dims[0] = nx; p->dims[1] = ny; p->dims[2] = nz;
  for (int i = 0; i < 3; ++i) p->bc[i] = bcs[i];
  p->h[0] = dx; p->h[1] = dy; p->h[2] = dz[0];
  p->dz.assign(dz, dz + nz);
  p->z_uniform = true;
  {
    const char* env = std::getenv("POISSON_GENERIC_R2R");
    p->generic_r2r = env && env[0] == '1';
    env = std::getenv("POISSON_GENERIC_TRI");
    p->generic_tri = env && env[0] == '1';
    env = std::getenv("POISSON_GRID_CAP");
    p->grid_cap = env ? std::max(0, std::atoi(env)) : 0;
    env = std::getenv("POISSON_PLANE");
    p->plane_off = env && env[0] == '0';
    env = std::getenv("POISSON_RK3_KERNEL");
    p->rk3_kernel = !env ? 0 : std::strcmp(env, "tiled") == 0 ? 1 : std::strcmp(env, "simple") == 0 ? 2 : 0;
    env = std::getenv("POISSON_RK3_GENERAL");
    p->rk3_general = env && std::strcmp(env, "1") == 0;
  }
  for (int k = 1; k < nz; ++k) if (dz[k] != dz[0]) p->z_uniform = false;
  p->shift = shift;
  if (node_pair(bc_z) && !p->z_uniform) {
    fail(POISSON_EUNSUPPORTED, "a node boundary pair needs a uniform spacing (z)");
    delete p;
    return nullptr;
  }

  // axis roles (elimination axis s; the others transformed, in x, y, z order).
  // All periodic: eliminate along the contiguous x (lines in registers, no
  // strided pass) when y and z take the DFT, else along z.
  auto dft_length = [](int n) {
    std::vector<int> r;
    return n >= 2 && n % 2 == 0 && n <= MAX_TRANSFORM_N && factor_radices(n / 2, r);
  };
  if (!p->z_uniform || bc_z != BC_PERIODIC) p->s = 2;
  else if (bc_x != BC_PERIODIC) p->s = 0;
  else if (bc_y != BC_PERIODIC) p->s = 1;
  else if (dft_length(ny) && dft_length(nz)) p->s = 0;
  else p->s = 2;
  int t[2], nt = 0;
  for (int i = 0; i < 3; ++i) if (i != p->s) t[nt++] = i;
  p->t1 = t[0];
  p->t2 = t[1];
  p->singular = shift == 0.0;
  for (int i = 0; i < 3; ++i)
    if (bcs[i] != BC_PERIODIC && bcs[i] != BC_NN && bcs[i] != BC_NN_NODE) p->singular = false;
  p->s_periodic = bcs[p->s] == BC_PERIODIC;
  if (p->singular && (node_pair(bc_x) || node_pair(bc_y) || node_pair(bc_z))) {
    fail(POISSON_EUNSUPPORTED, "a singular problem with a node boundary pair (no Dirichlet face, no shift)");
    delete p;
    return nullptr;
  }

  auto reject = [&](int code, const char* msg, int a) { fail(code, msg, a); delete p; return (poisson_plan*)nullptr; };
  for (int r = 0; r < 2; ++r) {
    AxisTables& A = p->ax[r];
    A.axis = t[r];
    A.n = p->dims[A.axis];
    A.kind = bcs[A.axis];
    if (node_pair(A.kind)) {   // DST-I / DCT-I through a real DFT of length 2m
      A.m = A.kind == BC_DD_NODE ? A.n + 1 : A.n - 1;
      if (A.m < 1 || 2 * A.m > MAX_TRANSFORM_N)
        return reject(POISSON_EUNSUPPORTED, "node axis length %d out of range", A.n);
      if (!factor_radices(A.m, A.radices))
        return reject(POISSON_EUNSUPPORTED, "node axis length %d: its FFT length has a prime factor > 5", A.n);
      continue;
    }
    if (A.n % 2 || A.n < 2 || A.n > MAX_TRANSFORM_N)
      return reject(POISSON_EUNSUPPORTED, "transformed axis length %d must be even and in [2, 1024]", A.n);
    A.m = A.n / 2;
    if (!factor_radices(A.m, A.radices))
      return reject(POISSON_EUNSUPPORTED, "transformed axis length %d: n/2 has a prime factor > 5", A.n);
  }
  const int ns = p->dims[p->s];
  if (ns > MAX_SOLVE_N) return reject(POISSON_EUNSUPPORTED, "elimination axis length %d > 512", ns);
  if (p->s_periodic && ns < 3) return reject(POISSON_EUNSUPPORTED, "periodic elimination axis needs n >= 3 (got %d)", ns);
  if (choose_chunks(ns, p->P, p->lcmax))
    return reject(POISSON_EUNSUPPORTED, "elimination axis length %d not supported", ns);
  p->nu = p->dims[t[0]];
  p->nv = p->dims[t[1]];

  // host tables
  std::vector<char> host;
  auto push = [&](const void* src, size_t bytes) {
    const size_t off = align_up(host.size(), 256);
    host.resize(off + bytes);
    std::memcpy(host.data() + off, src, bytes);
    return off;
  };
  for (int r = 0; r < 2; ++r) {
    AxisTables& A = p->ax[r];
    const int m = A.m, n = 2 * m;   // n: the real length of the FFT (node pairs: their extension)
    std::vector<cplx<double>> tw;
    for (int t = 0; t < m; ++t) tw.push_back(expm(16LL * t, n));        // e^{-2 pi i t/m}
    for (int k = 0; k <= m; ++k) tw.push_back(expm(8LL * k, n));        // e^{-2 pi i k/n}
    for (int k = 0; k <= m; ++k) tw.push_back(expm(2LL * k, n));        // e^{-i pi k/(2n)}
    for (int j = 0; j < m; ++j) tw.push_back(expm(4LL * j + 1, n));     // e^{-i pi (4j+1)/(4n)}
    for (int k = 0; k < m; ++k) tw.push_back(expm(4LL * k, n));         // e^{-i pi k/n}
    std::vector<cplx<float>> twf(tw.size());
    for (size_t i = 0; i < tw.size(); ++i) twf[i] = {(float)tw[i].re, (float)tw[i].im};
    A.off_d = push(tw.data(), tw.size() * sizeof(cplx<double>));
    A.off_f = push(twf.data(), twf.size() * sizeof(cplx<float>));
  }
  {
    const int ns_ = ns;
    std::vector<double> tri(4 * ns_);
    axis_rows(axis_widths(p, p->s), bcs[p->s], tri.data());
    for (int k = 0; k < ns_; ++k) tri[ns_ + k] += shift;   // the Helmholtz shift joins every diagonal
    std::vector<float> trif(tri.begin(), tri.end());
    p->off_tri_d = push(tri.data(), tri.size() * sizeof(double));
    p->off_tri_f = push(trif.data(), trif.size() * sizeof(float));
    // Padding: a line of ns < N points, N the next specialised length (at most
    // 3/2 ns), solved as a line of N whose last N - ns rows are decoupled
    // (a = c = 0, diagonal -1: with the shifts mu <= 0 of the transformed
    // axes no pivot of theirs comes near 0) and whose right-hand side there
    // is 0, so they come out 0 and leave the first ns unknowns those of the
    // real line.  Only for non-periodic lines (the real last row then has no
    // coupling past it) of non-singular plans (the gauge pins the line's
    // last row).
    if (!p->s_periodic && !p->singular && !p->generic_tri && !tri_fast_length(ns_)) {
      for (const int cand : {64, 96, 128, 192, 256, 384, 512}) {
        if (cand >= ns_ && 2 * cand <= 3 * ns_) {
          p->pad_n = cand;
          break;
        }
      }
    }
    if (p->pad_n) {
      const int N = p->pad_n;
      std::vector<double> pad(4 * (size_t)N, 0.0);
      for (int k = 0; k < N; ++k) {
        const bool real = k < ns_;
        pad[k] = real ? tri[k] : 0.0;                          // a
        pad[N + k] = real ? tri[ns_ + k] : -1.0;               // b (shift included)
        pad[2 * N + k] = real ? tri[2 * ns_ + k] : 0.0;        // c
        pad[3 * N + k] = real ? tri[3 * ns_ + k] : 0.0;        // w
      }
      p->off_tri_pad = push(pad.data(), pad.size() * sizeof(double));
    }
    for (int q = 0; q < 3; ++q) {
      std::vector<double> ops(4 * (size_t)p->dims[q]);
      axis_rows(axis_widths(p, q), bcs[q], ops.data());
      if (q == 0)   // the residual's operator: the shift once, on the x rows
        for (int k = 0; k < p->dims[0]; ++k) ops[p->dims[0] + k] += shift;
      p->off_ops[q] = push(ops.data(), ops.size() * sizeof(double));
    }
    for (int q = 0; q < 3; ++q) {   // projection: 1/h per cell, 1/centre distance per face
      const std::vector<double> hs = axis_widths(p, q);
      const int n = (int)hs.size();
      std::vector<double> t(2 * (size_t)n + 1);
      for (int k = 0; k < n; ++k) t[k] = 1.0 / hs[k];
      double* idc = t.data() + n;
      for (int f = 1; f < n; ++f) idc[f] = 1.0 / (0.5 * (hs[f - 1] + hs[f]));
      if (bcs[q] == BC_PERIODIC) {
        idc[0] = idc[n] = 1.0 / (0.5 * (hs[n - 1] + hs[0]));
      } else {
        idc[0] = 1.0 / hs[0];
        idc[n] = 1.0 / hs[n - 1];
      }
      p->off_proj[q] = push(t.data(), t.size() * sizeof(double));
    }
    std::vector<double> lam;
    for (int r = 0; r < 2; ++r) {
      const AxisTables& A = p->ax[r];
      const double hh = p->h[A.axis];
      for (int q = 0; q < A.n; ++q) lam.push_back(eigenvalue(A.kind, A.n, q) / (hh * hh));
    }
    std::vector<float> lamf(lam.begin(), lam.end());
    p->off_lam_d = push(lam.data(), lam.size() * sizeof(double));
    p->off_lam_f = push(lamf.data(), lamf.size() * sizeof(float));
  }
  p->tab_bytes = host.size();
  if (hipGetDevice(&p->device) != hipSuccess) { fail(POISSON_EHIP, "hipGetDevice failed"); delete p; return nullptr; }
  if (lds_setup_once()) { delete p; return nullptr; }
  if (hipMalloc(&p->dtab, p->tab_bytes) != hipSuccess) { fail(POISSON_ENOMEM, "table allocation (%zu B) failed", p->tab_bytes); delete p; return nullptr; }
  if (hipMemcpy(p->dtab, host.data(), p->tab_bytes, hipMemcpyHostToDevice) != hipSuccess) {
    fail(POISSON_EHIP, "table upload failed");
    (void)hipFree(p->dtab);
    delete p;
    return nullptr;
  }
  // small grid transformed along x and y: the transforms as dense matrices
  if (p->s == 2 && !p->plane_off && !p->generic_r2r && p->dims[0] <= PLANE_NMAX &&
      p->dims[1] <= PLANE_NMAX) {
    if (build_plane_matrices(p)) {
      (void)hipFree(p->dtab);
      delete p;
      return nullptr;
    }
  }
  return p;
}

static void free_workspace(poisson_plan* p) {
  if (p->f64 && !p->ws_external) (void)hipFree(p->f64);
  if (p->e32 && !p->ws_external) (void)hipFree(p->e32);
  p->ws_external = false;
  if (p->stats) (void)hipFree(p->stats);
  if (p->stats_host) (void)hipHostFree(p->stats_host);
  p->f64 = nullptr;
  p->e32 = nullptr;
  p->stats = nullptr;
  p->stats_host = nullptr;
  p->ws_bytes = 0;
}

extern "C" void plan_destroy(poisson_plan* p) {
  if (!p) return;
  free_workspace(p);
  if (p->dtab) (void)hipFree(p->dtab);
  if (p->plane_mats) (void)hipFree(p->plane_mats);
  delete p;
}

static size_t field_points(const poisson_plan* p) {
  return (size_t)p->dims[0] * p->dims[1] * p->dims[2];
}

extern "C" size_t plan_workspace_bytes(const poisson_plan* p) {
  if (!p) return 0;
  size_t ws = p->ws_bytes;
  if (p->mode == POISSON_FP32_REFINED && ws == 0)
    ws = field_points(p) * (sizeof(double) + sizeof(float)) + 4096;
  return p->tab_bytes + ws;
}

extern "C" int plan_roles(const poisson_plan* p, int roles[3]) {
  if (!p || !roles) return fail(POISSON_EINVAL, "null argument");
  roles[0] = p->t1;
  roles[1] = p->t2;
  roles[2] = p->s;
  return POISSON_OK;
}

extern "C" int transform_stage(poisson_plan* p, int role, int inverse, double* field, hipStream_t st) {
  if (!p || !field) return fail(POISSON_EINVAL, "null argument");
  if (int rc = misaligned(field, "field")) return rc;
  if (role < 0 || role > 1) return fail(POISSON_EINVAL, "role must be 0 or 1");
  return launch_r2r<double>(p, role, inverse ? 1 : 0, field, st);
}

extern "C" int tridiag_stage(poisson_plan* p, double* field, hipStream_t st) {
  if (!p || !field) return fail(POISSON_EINVAL, "null argument");
  if (int rc = misaligned(field, "field")) return rc;
  return launch_tridiag<double>(p, field, st);
}

// ------------------------------------------------------------------ refinement

extern "C" int plan_set_precision(poisson_plan* p, int mode, double tol, int max_iters) {
  if (!p) return fail(POISSON_EINVAL, "null plan");
  if (mode != POISSON_FP64 && mode != POISSON_FP32_REFINED) return fail(POISSON_EINVAL, "unknown precision mode %d", mode);
  if (mode == POISSON_FP32_REFINED) {
    if (!(tol > 0.0) || !std::isfinite(tol)) return fail(POISSON_EINVAL, "tol must be finite and > 0");
    if (max_iters < 1 || max_iters > 64) return fail(POISSON_EINVAL, "max_iters must be in [1, 64]");
    if (!p->f64) {
      const size_t N = field_points(p);
      if (hipMalloc(&p->f64, N * sizeof(double)) != hipSuccess ||
          hipMalloc(&p->e32, N * sizeof(float)) != hipSuccess ||
          hipMalloc(&p->stats, REFINE_STAT_SLOTS * sizeof(double)) != hipSuccess ||
          hipHostMalloc(&p->stats_host, REFINE_STAT_SLOTS * sizeof(double), hipHostMallocDefault) != hipSuccess) {
        free_workspace(p);
        return fail(POISSON_ENOMEM, "refinement workspace allocation failed");
      }
      p->ws_bytes = N * (sizeof(double) + sizeof(float)) + REFINE_STAT_SLOTS * sizeof(double);
    }
    p->tol = tol;
    p->max_iters = max_iters;
  }
  p->mode = mode;
  return POISSON_OK;
}

static int solve_refined(poisson_plan* p, double* rhs, hipStream_t st);

extern "C" int solve(poisson_plan* p, double* rhs, hipStream_t st) {
  if (!p || !rhs) return fail(POISSON_EINVAL, "null argument");
  if (int rc = misaligned(rhs, "rhs")) return rc;
  if (p->mode == POISSON_FP32_REFINED) return solve_refined(p, rhs, st);
  p->last_iters = 1;
  p->last_rel = 0.0;
  p->last_converged = 1;
  return solve_typed<double>(p, rhs, st);
}

// Status of a refined solve from its status block, copied to host memory at
// the end of its stream: the FP32 solves run (sweeps that ran have
// ||e||^2 >= 0), the last relative update, and whether it converged.
static bool refine_status_decode(const double* h, int max_iters, int* iters, double* rel) {
  int it = 1;
  for (int sweep = 1; sweep < max_iters; ++sweep)
    if (h[4 + 2 * sweep] >= 0.0) ++it;
  *iters = it;
  *rel = h[3];
  return h[2] != 0.0;
}

extern "C" int solve_status(poisson_plan* p, int* iters, double* rel) {
  if (!p) return fail(POISSON_EINVAL, "null plan");
  if (p->mode == POISSON_FP32_REFINED && p->stats_host)
    p->last_converged = refine_status_decode(p->stats_host, p->max_iters, &p->last_iters, &p->last_rel);
  if (iters) *iters = p->last_iters;
  if (rel) *rel = p->last_rel;
  return p->last_converged ? POISSON_OK : POISSON_ENOTCONVERGED;
}

// Workspace of a refined solve: the FP64 copy of f, the FP32 residual /
// correction field and the status block (REFINE_STAT_SLOTS doubles).  A
// plan's own (plan_set_precision), lent by a server slot, or the library's
// static scratch array (solve_refined_noalloc).
struct RefineWork {
  double* f64;
  float* e32;
  double* stats;
  double tol;
  int max_iters;
};

static RefineWork plan_work(const poisson_plan* p) {
  return RefineWork{p->f64, p->e32, p->stats, p->tol, p->max_iters};
}

static RefineGeom refine_geom(const poisson_plan* p, double* stats) {
  RefineGeom G{};
  for (int q = 0; q < 3; ++q) {
    const int n = p->dims[q];
    const double* base = reinterpret_cast<const double*>(p->dtab + p->off_ops[q]);
    G.ax[q] = OpAxis{base, base + n, base + 2 * n, base + 3 * n, n};
  }
  G.npts = (long long)field_points(p);
  G.stats = stats;
  return G;
}

// FP32 solve + FP64 refinement (fixed launch sequence; sweeps after
// convergence return at once through the device skip flag):
//   f~ = f (minus its weighted mean if singular), Phi = solve32(f~);
//   repeat: r = f~ - A Phi (FP64), e = solve32(r), Phi += e (FP64);
//   finally, if singular, remove the weighted mean of Phi (FP64).
// Pieces of the refined solve (the batched form runs the same kernel bodies
// for all its instances at once, refine_kernels.h).
struct RefineLaunch {
  long long N;
  RefineGeom G;
  int nb;
  ResidualGrid rg;
};

static RefineLaunch refine_launch(const poisson_plan* p, double* stats) {
  RefineLaunch r;
  r.N = (long long)field_points(p);
  r.G = refine_geom(p, stats);
  r.nb = (int)std::min<long long>(REFINE_BLOCKS, (r.N + REFINE_NT - 1) / REFINE_NT);
  r.rg = residual_grid(p->dims[0], p->dims[1], p->dims[2]);
  return r;
}

// Nontemporal accesses in the refinement sweeps on fields of at least
// 512 MiB (twice the 256 MB Infinity Cache).
static bool refine_hinted(const poisson_plan* p) {
  return (double)p->dims[0] * p->dims[1] * p->dims[2] * sizeof(double) >= (double)(512u << 20);
}

// Status reset, projection of f if singular, the FP64 copy of f and its FP32 cast.
static int refine_begin(const poisson_plan* p, const RefineWork& W, double* rhs, hipStream_t st) {
  const RefineLaunch r = refine_launch(p, W.stats);
  hipLaunchKernelGGL(refine_init_kernel, dim3(1), dim3(256), 0, st, W.stats);
  if (p->singular) {
    hipLaunchKernelGGL(refine_wsum_kernel, dim3(r.nb), dim3(REFINE_NT), 0, st, (const double*)rhs, r.G);
    hipLaunchKernelGGL(refine_mean_kernel, dim3(1), dim3(REFINE_NT), 0, st, W.stats, r.nb);
  }
  hipLaunchKernelGGL(refine_hinted(p) ? refine_prep_kernel<true> : refine_prep_kernel<false>,
                     dim3(r.nb), dim3(REFINE_NT), 0, st, (const double*)rhs,
                     W.f64, W.e32, (const double*)W.stats, (int)p->singular, r.N);
  HIP_TRY(hipGetLastError());
  return POISSON_OK;
}

// Sweep `sweep` before its FP32 solve: the FP64 residual into e32.
static int refine_sweep_begin(const poisson_plan* p, const RefineWork& W, double* rhs,
                              hipStream_t st) {
  const RefineLaunch r = refine_launch(p, W.stats);
  hipLaunchKernelGGL(refine_hinted(p) ? refine_residual_kernel<true> : refine_residual_kernel<false>,
                     dim3(r.rg.blocks), dim3(REFINE_NT), 0, st,
                     (const double*)rhs, (const double*)W.f64, W.e32, r.G, r.rg);
  HIP_TRY(hipGetLastError());
  return POISSON_OK;
}

// Sweep `sweep` after its FP32 solve: Phi += e and the convergence test.
static int refine_sweep_end(const poisson_plan* p, const RefineWork& W, double* rhs, int sweep,
                            hipStream_t st) {
  const RefineLaunch r = refine_launch(p, W.stats);
  hipLaunchKernelGGL(refine_hinted(p) ? refine_update_kernel<true> : refine_update_kernel<false>,
                     dim3(r.nb), dim3(REFINE_NT), 0, st, rhs,
                     (const float*)W.e32, r.G);
  hipLaunchKernelGGL(refine_status_kernel, dim3(1), dim3(REFINE_NT), 0, st, W.stats, r.nb, sweep,
                     W.tol);
  HIP_TRY(hipGetLastError());
  return POISSON_OK;
}

// Gauge of a singular problem.
static int refine_end(const poisson_plan* p, const RefineWork& W, double* rhs, hipStream_t st) {
  const RefineLaunch r = refine_launch(p, W.stats);
  if (p->singular) {
    hipLaunchKernelGGL(refine_wsum_kernel, dim3(r.nb), dim3(REFINE_NT), 0, st, (const double*)rhs, r.G);
    hipLaunchKernelGGL(refine_mean_kernel, dim3(1), dim3(REFINE_NT), 0, st, W.stats, r.nb);
    hipLaunchKernelGGL(refine_shift_kernel, dim3(r.nb), dim3(REFINE_NT), 0, st, rhs,
                       (const double*)W.stats, r.N);
  }
  HIP_TRY(hipGetLastError());
  return POISSON_OK;
}

// The whole refined solve on workspace W.
static int run_refined(const poisson_plan* p, const RefineWork& W, double* rhs, hipStream_t st) {
  int rc;
  if ((rc = refine_begin(p, W, rhs, st))) return rc;
  // the first FP32 solve's last pass writes Phi (widened) into rhs
  if ((rc = solve_typed<float>(p, W.e32, st, nullptr, rhs))) return rc;
  for (int sweep = 1; sweep < W.max_iters; ++sweep) {
    if ((rc = refine_sweep_begin(p, W, rhs, st))) return rc;
    if ((rc = solve_typed<float>(p, W.e32, st, W.stats))) return rc;
    if ((rc = refine_sweep_end(p, W, rhs, sweep, st))) return rc;
  }
  return refine_end(p, W, rhs, st);
}

// The plan's refined solve, and the status copy for solve_status.
static int solve_refined(poisson_plan* p, double* rhs, hipStream_t st) {
  const RefineWork W = plan_work(p);
  const int rc = run_refined(p, W, rhs, st);
  if (rc) return rc;
  HIP_TRY(hipMemcpyAsync(p->stats_host, p->stats, REFINE_PARTIALS * sizeof(double),
                         hipMemcpyDeviceToHost, st));
  return POISSON_OK;
}

// ------------------------------------------------------------------ no-allocation refined solve

// Workspace of solve_refined_noalloc: one array per device, allocated when
// the library's code object is loaded and held until the process ends.
// In host code `scratch` names a host-side stand-in; its device address is
// taken once per device (hipGetSymbolAddress) and only that address is used.
static constexpr size_t kScratchBytes = size_t(256) << 20;
static constexpr size_t kScratchStatsBytes = align_up_c(REFINE_STAT_SLOTS * sizeof(double), 256);
static __device__ __align__(256) char scratch[kScratchBytes];

static constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static char* g_scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on the current device (taken on the first
// call on that device).
static int scratch_address(char** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(POISSON_EUNSUPPORTED, "device %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    char* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(POISSON_EHIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    g_scratch_dev[dev] = ptr;
  }
  *out = g_scratch_dev[dev];
  return POISSON_OK;
}

extern "C" size_t refined_noalloc_max_points(void) {
  return (kScratchBytes - kScratchStatsBytes) / (sizeof(double) + sizeof(float));
}

// status_out[0] = FP32 solves run, [1] = 1 if converged else 0, [2] = last
// relative update (device memory of the caller).
__global__ void refine_report_kernel(const double* __restrict__ stats, int max_iters,
                                     double* __restrict__ out) {
  if (threadIdx.x != 0) return;
  int it = 1;
  for (int sweep = 1; sweep < max_iters; ++sweep)
    if (stats[4 + 2 * sweep] >= 0.0) ++it;
  out[0] = (double)it;
  out[1] = stats[2] != 0.0 ? 1.0 : 0.0;
  out[2] = stats[3];
}

extern "C" int solve_refined_noalloc(poisson_plan* p, double* rhs, double tol, int max_iters,
                                     double* status_out, hipStream_t st) {
  if (!p || !rhs) return fail(POISSON_EINVAL, "null argument");
  if (int rc = misaligned(rhs, "rhs")) return rc;
  if (!(tol > 0.0) || !std::isfinite(tol)) return fail(POISSON_EINVAL, "tol must be finite and > 0");
  if (max_iters < 1 || max_iters > REFINE_MAX_SWEEPS)
    return fail(POISSON_EINVAL, "max_iters must be in [1, %d]", REFINE_MAX_SWEEPS);
  const size_t N = field_points(p);
  if (N > refined_noalloc_max_points())
    return fail(POISSON_EUNSUPPORTED,
                "grid of %zu points exceeds the no-allocation workspace (%zu points, %zu B)", N,
                refined_noalloc_max_points(), kScratchBytes);
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev != p->device) return fail(POISSON_EINVAL, "plan lives on device %d, current is %d", p->device, dev);
  char* base = nullptr;
  if (int rc = scratch_address(&base)) return rc;
  RefineWork W;
  W.stats = reinterpret_cast<double*>(base);
  W.f64 = reinterpret_cast<double*>(base + kScratchStatsBytes);
  W.e32 = reinterpret_cast<float*>(base + kScratchStatsBytes + N * sizeof(double));
  W.tol = tol;
  W.max_iters = max_iters;
  if (int rc = run_refined(p, W, rhs, st)) return rc;
  if (status_out) {
    hipLaunchKernelGGL(refine_report_kernel, dim3(1), dim3(64), 0, st, (const double*)W.stats,
                       max_iters, status_out);
    HIP_TRY(hipGetLastError());
  }
  return POISSON_OK;
}

// ------------------------------------------------------------------ projection

static ProjGeom proj_geom(const poisson_plan* p) {
  ProjGeom G{};
  for (int q = 0; q < 3; ++q) {
    const int n = p->dims[q];
    const double* t = reinterpret_cast<const double*>(p->dtab + p->off_proj[q]);
    const int kind = p->bc[q];
    G.ax[q] = ProjAxis{t, t + n, n, kind != BC_PERIODIC ? 1 : 0,
                       kind == BC_DD || kind == BC_DN ? 1 : 0, kind == BC_DD || kind == BC_ND ? 1 : 0};
  }
  G.npts = (long long)field_points(p);
  return G;
}

// z-marching tiles of the projection kernels: 64 x 4 columns, PROJ_KC planes
static dim3 proj_tiles(const poisson_plan* p) {
  return dim3((p->dims[0] + PROJ_TX - 1) / PROJ_TX, (p->dims[1] + PROJ_TY - 1) / PROJ_TY,
              (p->dims[2] + PROJ_KC - 1) / PROJ_KC);
}

// u = u_in - gamma_dt grad(phi), p += phi (z-marching tiles; in place when u_in == u)
static int launch_proj_update(const poisson_plan* p, const double* phi, double gamma_dt,
                              const double* ui, const double* vi, const double* wi, double* u,
                              double* v, double* w, double* pres, hipStream_t st) {
  hipLaunchKernelGGL(proj_update_zmarch_kernel, proj_tiles(p), dim3(PROJ_NT), 0, st, phi, gamma_dt, ui, vi, wi,
                     u, v, w, pres, proj_geom(p));
  HIP_TRY(hipGetLastError());
  return POISSON_OK;
}

static bool staggered_plan(const poisson_plan* p) {
  return !node_pair(p->bc[0]) && !node_pair(p->bc[1]) && !node_pair(p->bc[2]);
}

extern "C" int projection_rhs(poisson_plan* p, const double* u, const double* v, const double* w,
                              double gamma_dt, double* rhs, hipStream_t st) {
  if (!p || !u || !v || !w || !rhs) return fail(POISSON_EINVAL, "null argument");
  if (!staggered_plan(p)) return fail(POISSON_EUNSUPPORTED, "projection needs staggered boundary pairs");
  if (!(gamma_dt != 0.0) || !std::isfinite(gamma_dt)) return fail(POISSON_EINVAL, "gamma_dt must be finite and non-zero");
  hipLaunchKernelGGL(proj_rhs_kernel, proj_tiles(p), dim3(PROJ_NT), 0, st, u, v, w,
                     1.0 / gamma_dt, rhs, proj_geom(p));
  HIP_TRY(hipGetLastError());
  return POISSON_OK;
}

extern "C" int projection_update(poisson_plan* p, const double* phi, double gamma_dt, double* u,
                                 double* v, double* w, double* pres, hipStream_t st) {
  if (!p || !phi || !u || !v || !w || !pres) return fail(POISSON_EINVAL, "null argument");
  if (!staggered_plan(p)) return fail(POISSON_EUNSUPPORTED, "projection needs staggered boundary pairs");
  if (!std::isfinite(gamma_dt)) return fail(POISSON_EINVAL, "gamma_dt must be finite");
  return launch_proj_update(p, phi, gamma_dt, u, v, w, u, v, w, pres, st);
}

extern "C" int pressure_correction(poisson_plan* p, double* u, double* v, double* w, double* pres,
                                   double gamma_dt, double* phi, hipStream_t st) {
  int rc;
  if (phi && (rc = misaligned(phi, "phi"))) return rc;
  if ((rc = projection_rhs(p, u, v, w, gamma_dt, phi, st))) return rc;
  if ((rc = solve(p, phi, st))) return rc;
  return projection_update(p, phi, gamma_dt, u, v, w, pres, st);
}

// ------------------------------------------------------------------ Navier-Stokes step

static constexpr double kRK3Alpha[3] = {8.0 / 15.0, 5.0 / 12.0, 3.0 / 4.0};
static constexpr double kRK3Beta[3] = {0.0, -17.0 / 60.0, -5.0 / 12.0};

// A plan the time step runs on: periodic along every axis, uniform widths.
static int rk3_plan_check(const poisson_plan* p) {
  if (p->bc[0] != BC_PERIODIC || p->bc[1] != BC_PERIODIC || p->bc[2] != BC_PERIODIC)
    return fail(POISSON_EUNSUPPORTED, "the time step needs a plan periodic along every axis");
  if (!p->z_uniform) return fail(POISSON_EUNSUPPORTED, "the time step needs uniform widths along z");
  if (p->shift != 0.0) return fail(POISSON_EUNSUPPORTED, "the time step needs a Poisson (unshifted) plan");
  return POISSON_OK;
}

// Arguments of substep k's prediction: AD buffers as described at
// rk3_predict, no correction.
static RK3Args rk3_args(const poisson_plan* p, int k, double dt, double nu, const double* vel,
                        double* work, double* ad, const double* pres) {
  const long long N = (long long)field_points(p);
  const double dx = p->h[0], dy = p->h[1], dz = p->dz[0];
  RK3Args A;
  A.vel = vel;
  A.p = pres;
  // two AD buffers: substep 1 writes the first, substep 2 reads it and
  // writes the second (a tile also reads the previous AD of faces that its
  // neighbours own and overwrite), substep 3 reads the second
  A.ad_prev = k == 3 ? ad + 3 * N : ad;
  A.ad = k == 1 ? ad : ad + 3 * N;
  A.star = work;
  A.phi_prev = nullptr;
  A.p_out = nullptr;
  A.c_gdt = 0.0;
  A.idx = 1.0 / dx;
  A.idy = 1.0 / dy;
  A.idz = 1.0 / dz;
  A.kx = nu / (dx * dx);
  A.ky = nu / (dy * dy);
  A.kz = nu / (dz * dz);
  const double alpha = kRK3Alpha[k - 1], beta = kRK3Beta[k - 1];
  A.a_dt = dt * alpha;
  A.b_dt = dt * beta;
  A.g_dt = dt * (alpha + beta);
  A.nx = p->dims[0];
  A.ny = p->dims[1];
  A.nz = p->dims[2];
  A.npts = N;
  return A;
}

static dim3 rk3_tiles(const RK3Args& A) {
  return dim3((A.nx + RK3_TX - 1) / RK3_TX, (A.ny + RK3_TY - 1) / RK3_TY, (A.nz + RK3_KC - 1) / RK3_KC);
}

// The fused prediction of substep k (with the previous substep's
// correction when `correct`); rhs = div(u*) / (gamma_k dt).
static int launch_predict_div(const RK3Args& A, int k, bool correct, double* rhs, hipStream_t st,
                              bool general) {
  const dim3 tiles = rk3_tiles(A);
  const double inv_gdt = 1.0 / A.g_dt;
  // whole tiles and z ranges: the branch-free form of the z loop
  const bool full = A.nx % RK3_TX == 0 && A.ny % RK3_TY == 0 && A.nz % RK3_KC == 0 && !general;
  auto go = [&](auto full_c) {
    constexpr bool F = decltype(full_c)::value;
    if (k == 1)
      hipLaunchKernelGGL((rk3_predict_div_kernel<false, true, false, F>), tiles, dim3(RK3_NT), 0, st, A, rhs, inv_gdt);
    else if (k == 2 && !correct)
      hipLaunchKernelGGL((rk3_predict_div_kernel<true, true, false, F>), tiles, dim3(RK3_NT), 0, st, A, rhs, inv_gdt);
    else if (k == 2)
      hipLaunchKernelGGL((rk3_predict_div_kernel<true, true, true, F>), tiles, dim3(RK3_NT), 0, st, A, rhs, inv_gdt);
    else if (!correct)
      hipLaunchKernelGGL((rk3_predict_div_kernel<true, false, false, F>), tiles, dim3(RK3_NT), 0, st, A, rhs, inv_gdt);
    else
      hipLaunchKernelGGL((rk3_predict_div_kernel<true, false, true, F>), tiles, dim3(RK3_NT), 0, st, A, rhs, inv_gdt);
  };
  if (full) go(std::true_type{});
  else go(std::false_type{});
  HIP_TRY(hipGetLastError());
  return POISSON_OK;
}

static int rk3_check(const poisson_plan* p, int k, double dt, double nu) {
  if (k < 1 || k > 3) return fail(POISSON_EINVAL, "substep %d is not 1, 2 or 3", k);
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(POISSON_EINVAL, "dt must be finite and positive");
  if (!(nu >= 0.0) || !std::isfinite(nu)) return fail(POISSON_EINVAL, "nu must be finite and >= 0");
  return rk3_plan_check(p);
}

extern "C" int rk3_predict(poisson_plan* p, int k, double dt, double nu, const double* vel, double* work,
                           double* ad, const double* pres, double* rhs, hipStream_t st) {
  if (!p || !vel || !work || !ad || !pres || !rhs) return fail(POISSON_EINVAL, "null argument");
  if (int rc = rk3_check(p, k, dt, nu)) return rc;
  const long long N = (long long)field_points(p);
  const RK3Args A = rk3_args(p, k, dt, nu, vel, work, ad, pres);
  // AD_prev is read when beta_k != 0 (k = 2, 3); AD is kept for the next
  // substep (k = 1, 2): the first substep of the next step does not read it
  const double gdt = A.g_dt;
  const dim3 tiles = rk3_tiles(A);
  if (p->rk3_kernel == 0) {        // prediction and right-hand side in one sweep
    if (int rc = launch_predict_div(A, k, false, rhs, st, p->rk3_general)) return rc;
  } else {
    if (p->rk3_kernel == 2) {
      const int blocks = (int)std::max<long long>(1, std::min<long long>(RK3_BLOCKS, (N + RK3_NT - 1) / RK3_NT));
      if (k == 1)
        hipLaunchKernelGGL((rk3_predict_kernel<false, true>), dim3(blocks), dim3(RK3_NT), 0, st, A);
      else if (k == 2)
        hipLaunchKernelGGL((rk3_predict_kernel<true, true>), dim3(blocks), dim3(RK3_NT), 0, st, A);
      else
        hipLaunchKernelGGL((rk3_predict_kernel<true, false>), dim3(blocks), dim3(RK3_NT), 0, st, A);
    } else {
      if (k == 1)
        hipLaunchKernelGGL((rk3_predict_tiled_kernel<false, true>), tiles, dim3(RK3_NT), 0, st, A);
      else if (k == 2)
        hipLaunchKernelGGL((rk3_predict_tiled_kernel<true, true>), tiles, dim3(RK3_NT), 0, st, A);
      else
        hipLaunchKernelGGL((rk3_predict_tiled_kernel<true, false>), tiles, dim3(RK3_NT), 0, st, A);
    }
    HIP_TRY(hipGetLastError());
    // right-hand side of the pressure equation, div(u*) / (gamma dt), in a sweep of its own
    hipLaunchKernelGGL(proj_rhs_kernel, proj_tiles(p), dim3(PROJ_NT), 0, st, (const double*)work,
                       (const double*)(work + N), (const double*)(work + 2 * N), 1.0 / gdt, rhs, proj_geom(p));
    HIP_TRY(hipGetLastError());
  }
  return POISSON_OK;
}

extern "C" int rk3_substep(poisson_plan* p, int k, double dt, double nu, double* vel, double* work,
                           double* ad, double* pres, double* phi, hipStream_t st) {
  if (phi)
    if (int rc = misaligned(phi, "phi")) return rc;
  if (int rc = rk3_predict(p, k, dt, nu, vel, work, ad, pres, phi, st)) return rc;
  const long long N = (long long)field_points(p);
  const double gdt = (kRK3Alpha[k - 1] + kRK3Beta[k - 1]) * dt;
  if (int rc = solve(p, phi, st)) return rc;
  return launch_proj_update(p, phi, gdt, work, work + N, work + 2 * N, vel, vel + N, vel + 2 * N, pres, st);
}

extern "C" int rk3_step(poisson_plan* p, double dt, double nu, double* vel, double* work, double* ad,
                        double* pres, double* phi, double* scratch, hipStream_t st) {
  if (!p || !vel || !work || !ad || !pres || !phi || !scratch) return fail(POISSON_EINVAL, "null argument");
  if (int rc = misaligned(phi, "phi")) return rc;
  if (int rc = misaligned(scratch, "scratch")) return rc;
  if (int rc = rk3_check(p, 1, dt, nu)) return rc;
  if (p->rk3_kernel != 0) {        // the other prediction kernels: substep by substep
    for (int k = 1; k <= 3; ++k)
      if (int rc = rk3_substep(p, k, dt, nu, vel, work, ad, pres, phi, st)) return rc;
    return POISSON_OK;
  }
  // Each substep's projection is applied by the next substep's prediction
  // as it reads the planes (u* alternates between work and vel, p between
  // pres and the first half of scratch, Phi between phi and its second
  // half); the third substep's projection is the update sweep.
  const long long N = (long long)field_points(p);
  double* p2 = scratch;
  double* phi2 = scratch + N;
  auto gdt = [&](int k) { return (kRK3Alpha[k - 1] + kRK3Beta[k - 1]) * dt; };
  RK3Args A = rk3_args(p, 1, dt, nu, vel, work, ad, pres);          // vel -> work (u*1)
  if (int rc = launch_predict_div(A, 1, false, phi, st, p->rk3_general)) return rc;
  if (int rc = solve(p, phi, st)) return rc;                        // Phi1
  A = rk3_args(p, 2, dt, nu, work, vel, ad, pres);                  // u*1, Phi1, p -> vel (u*2), p2
  A.phi_prev = phi;
  A.p_out = p2;
  A.c_gdt = gdt(1);
  if (int rc = launch_predict_div(A, 2, true, phi2, st, p->rk3_general)) return rc;
  if (int rc = solve(p, phi2, st)) return rc;                       // Phi2
  A = rk3_args(p, 3, dt, nu, vel, work, ad, p2);                    // u*2, Phi2, p2 -> work (u*3), pres
  A.phi_prev = phi2;
  A.p_out = pres;
  A.c_gdt = gdt(2);
  if (int rc = launch_predict_div(A, 3, true, phi, st, p->rk3_general)) return rc;
  if (int rc = solve(p, phi, st)) return rc;                        // Phi3
  return launch_proj_update(p, phi, gdt(3), work, work + N, work + 2 * N, vel, vel + N, vel + 2 * N,
                            pres, st);
}

// ------------------------------------------------------------------ batch

extern "C" int batch_solve(poisson_plan* const* plans, double* const* rhs, int count, hipStream_t st) {
  if (count < 0 || (count > 0 && (!plans || !rhs))) return fail(POISSON_EINVAL, "bad batch arguments");
  for (int i = 0; i < count; ++i) {
    if (!plans[i] || !rhs[i]) return fail(POISSON_EINVAL, "null plan or field at batch index %d", i);
    if (int rc = misaligned(rhs[i], "every batch field")) return rc;
    for (int j = 0; j < i; ++j)
      if (plans[j] == plans[i] && plans[i]->mode == POISSON_FP32_REFINED)
        return fail(POISSON_EINVAL, "refined plan at batch index %d appears twice", i);
  }
  bool specialised = true;
  for (int i = 0; i < count && specialised; ++i) {
    const poisson_plan* p = plans[i];
    specialised = r2r_fast_length(p->ax[0]) && r2r_fast_length(p->ax[1]) &&
                  tri_fast_length(p->dims[p->s]) && !p->generic_r2r && !p->generic_tri &&
                  p->mode == plans[0]->mode;
  }
  if (count > 0 && specialised) {
    poisson_batch* b = batch_create(plans, count);
    if (!b) return g_err;
    int rc = batch_bind(b, rhs);
    if (!rc) rc = batch_launch(b, st, 0);
    const hipError_t e = hipStreamSynchronize(st);
    batch_destroy(b);
    if (rc) return rc;
    if (e != hipSuccess) return fail(POISSON_EHIP, "hipStreamSynchronize: %s", hipGetErrorString(e));
    return POISSON_OK;
  }
  for (int i = 0; i < count; ++i) {
    const int rc = solve(plans[i], rhs[i], st);
    if (rc) return rc;
  }
  return POISSON_OK;
}

// ------------------------------------------------------------------ batched launches

// Pipeline steps of a solve (Sec. 2.1): forward t1, forward t2, elimination,
// backward t2, backward t1, as (transform role or -1, inverse).
static const int kStepRole[5] = {0, 1, -1, 1, 0};
static const int kStepInverse[5] = {0, 0, 0, 1, 1};
static constexpr int kMaxSteps = 10;

// A batch of FP64 plans has the five steps of a solve.  A batch of
// FP32 + refinement plans has ten: the steps of the first FP32 solve (its
// last one writes the widened solution into the caller's field) and those
// of the later sweeps' solves (each job skips once its plan has converged).
struct poisson_batch {
  int device = 0;
  bool fp32 = false;                  // FP32 + refinement plans
  int nsteps = 5;
  std::vector<poisson_plan*> plans;
  std::vector<int> order[5];          // instances in job order, per pipeline step
  int njobs[kMaxSteps] = {};
  int items[kMaxSteps] = {};
  size_t lds[kMaxSteps] = {};
  size_t off[kMaxSteps] = {};         // byte offset of each step's job array
  size_t bytes = 0;
  char* djobs = nullptr;              // device job arrays (all steps)
  int force[5] = {-1, -1, -1, -1, -1};  // variant of every job of a step (-1: per-length table)
  std::vector<double*> rhs;           // bound fields
  RefineJob* drefine = nullptr;       // refined batch: per-instance refinement jobs (device)
  int refine_eblocks = 0;             // blocks of its element-wise launches
  int refine_rblocks = 0;             // blocks of its residual launch
  bool bound = false;
  hipStream_t cap = nullptr;          // private stream for graph capture
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

// Job tables of one step in element type T.
template <typename T>
static void batch_step_jobs(poisson_batch* b, int k, double* const* rhs, std::vector<char>& host) {
  const int ps = k % 5;                       // pipeline step
  const bool sweep = k >= 5;                  // later sweeps of a refined batch
  int first = 0;
  size_t lds = 0;
  for (size_t j = 0; j < b->order[ps].size(); ++j) {
    const int i = b->order[ps][j];
    poisson_plan* p = b->plans[i];
    T* data = b->fp32 ? reinterpret_cast<T*>(p->e32) : reinterpret_cast<T*>(rhs ? rhs[i] : nullptr);
    const double* skip = sweep ? p->stats : nullptr;
    double* out64 = b->fp32 && !sweep && ps == 4 && rhs ? rhs[i] : nullptr;
    if (kStepRole[ps] >= 0) {
      const AxisTables& A = p->ax[kStepRole[ps]];
      BatchR2RJob<T> J{};
      J.M = A.m;
      J.V = b->force[ps] >= 0 ? b->force[ps] : tuned_choice(0, sizeof(T), A.m, A.axis == 0);
      if (J.V >= 4) J.V = 0;   // the batched kernel has the synchronous variants
      with_fast_cfg(J.M, J.V, [&](auto cfg) {
        using C = decltype(cfg);
        J.a = fast_args<T, C>(p, A, kStepInverse[ps], data, skip, out64);
        lds = std::max(lds, fast_lds_bytes<T, C>());
        return 0LL;
      });
      J.first = first;
      first += J.a.g.ntiles;
      std::memcpy(host.data() + b->off[k] + j * sizeof(J), &J, sizeof(J));
    } else {
      const int n = p->dims[p->s];
      BatchTriJob<T> J{};
      const int tv = b->force[ps] >= 0 ? b->force[ps] : tuned_choice(1, sizeof(T), n, p->s == 0);
      J.key = 2 * n + (tv < 2 ? tv : 0);   // the batched kernel has the synchronous chunkings
      with_tri_cfg(n, J.key & 1, [&](auto cfg) {
        using C = decltype(cfg);
        J.a = tri_fast_args<T, C::RPC, C::P>(p, data, skip);
        lds = std::max(lds, tri_fast_lds_bytes<T, C::RPC, C::P>());
        return 0LL;
      });
      J.first = first;
      first += J.a.g.ntiles;
      std::memcpy(host.data() + b->off[k] + j * sizeof(J), &J, sizeof(J));
    }
  }
  b->items[k] = first;
  b->lds[k] = lds;
}

// Job tables of every step for the given fields (null fields: sizes only),
// with the variants chosen now (the batch's own choice for a step if it has
// one, else the per-length table); sets item counts and LDS sizes.
static void batch_jobs(poisson_batch* b, double* const* rhs, std::vector<char>& host) {
  host.assign(b->bytes, 0);
  for (int k = 0; k < b->nsteps; ++k) {
    if (b->fp32) batch_step_jobs<float>(b, k, rhs, host);
    else batch_step_jobs<double>(b, k, rhs, host);
  }
}

extern "C" poisson_batch* batch_create(poisson_plan* const* plans, int count) {
  if (count < 1 || !plans) { fail(POISSON_EINVAL, "a batch needs at least one plan"); return nullptr; }
  if (lds_setup_once()) return nullptr;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) { fail(POISSON_EHIP, "hipGetDevice failed"); return nullptr; }
  for (int i = 0; i < count; ++i) {
    const poisson_plan* p = plans[i];
    if (!p) { fail(POISSON_EINVAL, "null plan at batch index %d", i); return nullptr; }
    if (p->device != dev) { fail(POISSON_EINVAL, "plan %d lives on another device", i); return nullptr; }
    if (p->mode != plans[0]->mode) {
      fail(POISSON_EUNSUPPORTED, "a batch takes plans of one precision mode (index %d differs)", i);
      return nullptr;
    }
    if (p->mode == POISSON_FP32_REFINED && (!p->f64 || !p->e32)) {
      fail(POISSON_EINVAL, "refined plan %d has no workspace", i);
      return nullptr;
    }
    for (int r = 0; r < 2; ++r)
      if (!r2r_fast_length(p->ax[r])) {
        fail(POISSON_EUNSUPPORTED, "plan %d: transform length %d has no size-specialised kernel", i, p->ax[r].n);
        return nullptr;
      }
    if (!tri_fast_length(p->dims[p->s])) {
      fail(POISSON_EUNSUPPORTED, "plan %d: elimination length %d has no size-specialised kernel", i, p->dims[p->s]);
      return nullptr;
    }
  }
  for (int i = 0; i < count; ++i)
    for (int j = 0; j < i; ++j)
      if (plans[i] == plans[j] && plans[i]->mode == POISSON_FP32_REFINED) {
        fail(POISSON_EINVAL, "refined plan %d appears twice (one workspace per plan)", i);
        return nullptr;
      }
  poisson_batch* b = new poisson_batch();
  b->device = dev;
  b->fp32 = plans[0]->mode == POISSON_FP32_REFINED;
  b->nsteps = b->fp32 ? 10 : 5;
  b->plans.assign(plans, plans + count);
  for (int k = 0; k < 5; ++k) {
    std::vector<int>& ord = b->order[k];
    for (int i = 0; i < count; ++i) ord.push_back(i);
    // group jobs that share LDS tables: transforms by length and type class
    // (twiddles), eliminations by length
    auto key = [&](int i) {
      const poisson_plan* p = plans[i];
      if (kStepRole[k] >= 0) {
        const AxisTables& A = p->ax[kStepRole[k]];
        return A.m * 2 + (A.kind >= BC_ND ? 1 : 0);
      }
      return p->dims[p->s];
    };
    std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return key(x) < key(y); });
  }
  size_t bytes = 0;
  for (int k = 0; k < b->nsteps; ++k) {
    const bool r2r = kStepRole[k % 5] >= 0;
    const size_t job = b->fp32 ? (r2r ? sizeof(BatchR2RJob<float>) : sizeof(BatchTriJob<float>))
                               : (r2r ? sizeof(BatchR2RJob<double>) : sizeof(BatchTriJob<double>));
    b->njobs[k] = count;
    bytes = align_up(bytes, 64);
    b->off[k] = bytes;
    bytes += (size_t)count * job;
  }
  b->bytes = bytes;
  std::vector<char> host;
  batch_jobs(b, nullptr, host);       // item counts
  if (hipMalloc(&b->djobs, b->bytes) != hipSuccess ||
      (b->fp32 && hipMalloc(&b->drefine, count * sizeof(RefineJob)) != hipSuccess)) {
    fail(POISSON_ENOMEM, "batch job tables: hipMalloc failed");
    if (b->djobs) (void)hipFree(b->djobs);
    delete b;
    return nullptr;
  }
  return b;
}

// Job tables for the bound fields to the device (synchronous).  The
// captured launches carry the LDS size, grid and item count of each step:
// when the variants changed them, capture again at the next launch.
static int batch_upload(poisson_batch* b) {
  size_t lds_before[kMaxSteps];
  int items_before[kMaxSteps];
  std::memcpy(lds_before, b->lds, sizeof(lds_before));
  std::memcpy(items_before, b->items, sizeof(items_before));
  std::vector<char> host;
  batch_jobs(b, b->rhs.data(), host);
  if (b->exec && (std::memcmp(lds_before, b->lds, sizeof(lds_before)) != 0 ||
                  std::memcmp(items_before, b->items, sizeof(items_before)) != 0)) {
    (void)hipGraphExecDestroy(b->exec);
    (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
  }
  HIP_TRY(hipMemcpy(b->djobs, host.data(), b->bytes, hipMemcpyHostToDevice));
  if (b->fp32) {
    // refinement jobs: each instance's kernels on its own block range, with
    // the block counts of its single-plan launches (same reductions)
    std::vector<RefineJob> jobs(b->plans.size());
    int fe = 0, fr = 0;
    for (size_t i = 0; i < b->plans.size(); ++i) {
      const poisson_plan* p = b->plans[i];
      const RefineLaunch r = refine_launch(p, p->stats);
      RefineJob& J = jobs[i];
      J.G = r.G;
      J.phi = b->rhs[i];
      J.f64 = p->f64;
      J.e32 = p->e32;
      J.singular = p->singular ? 1 : 0;
      J.nb = r.nb;
      J.rg = r.rg;
      J.first_e = fe;
      J.first_r = fr;
      J.max_iters = p->max_iters;
      J.tol = p->tol;
      fe += r.nb;
      fr += r.rg.blocks;    // a multiple of 8: every job starts XCD-aligned
    }
    b->refine_eblocks = fe;
    b->refine_rblocks = fr;
    HIP_TRY(hipMemcpy(b->drefine, jobs.data(), jobs.size() * sizeof(RefineJob),
                      hipMemcpyHostToDevice));
  }
  b->bound = true;
  return POISSON_OK;
}

extern "C" int batch_bind(poisson_batch* b, double* const* rhs) {
  if (!b || !rhs) return fail(POISSON_EINVAL, "null argument");
  for (size_t i = 0; i < b->plans.size(); ++i)
    if (!rhs[i]) return fail(POISSON_EINVAL, "null field at batch index %zu", i);
    else if (int rc = misaligned(rhs[i], "every batch field")) return rc;
  b->rhs.assign(rhs, rhs + b->plans.size());
  if (b->exec) {
    // the refinement kernels around the batched steps take the fields as
    // arguments: a captured sequence of a refined batch is for the old ones
    if (b->fp32) {
      (void)hipGraphExecDestroy(b->exec);
      (void)hipGraphDestroy(b->graph);
      b->exec = nullptr;
      b->graph = nullptr;
    }
  }
  return batch_upload(b);
}

// One persistent launch of step k (k >= 5: the sweep tables of a refined batch).
template <typename T>
static int batch_enqueue_typed(poisson_batch* b, int k, hipStream_t st) {
  if (b->items[k] == 0) return POISSON_OK;
  t_grid_cap = 0;   // batched launches are never capped
  const size_t lds = b->lds[k];
  if (kStepRole[k % 5] >= 0) {
    const auto* jobs = reinterpret_cast<const BatchR2RJob<T>*>(b->djobs + b->off[k]);
    const void* fn = reinterpret_cast<const void*>(&batch_r2r_kernel<T>);
    hipLaunchKernelGGL(batch_r2r_kernel<T>, dim3(resident_grid(fn, 512, lds, b->items[k])),
                       dim3(512), lds, st, jobs, b->njobs[k], b->items[k]);
  } else {
    const auto* jobs = reinterpret_cast<const BatchTriJob<T>*>(b->djobs + b->off[k]);
    const void* fn = reinterpret_cast<const void*>(&batch_tri_kernel<T>);
    hipLaunchKernelGGL(batch_tri_kernel<T>, dim3(resident_grid(fn, 512, lds, b->items[k])),
                       dim3(512), lds, st, jobs, b->njobs[k], b->items[k]);
  }
  HIP_TRY(hipGetLastError());
  return POISSON_OK;
}

static int batch_enqueue_step(poisson_batch* b, int k, hipStream_t st) {
  return b->fp32 ? batch_enqueue_typed<float>(b, k, st) : batch_enqueue_typed<double>(b, k, st);
}

// The whole batched solve: the five steps (FP64), or the refined sequence:
// per instance the refinement kernels (cheap, one field each), between them
// the FP32 solves as batched steps over all instances.
static int batch_enqueue(poisson_batch* b, hipStream_t st) {
  int rc;
  if (!b->fp32) {
    for (int k = 0; k < 5; ++k)
      if ((rc = batch_enqueue_step(b, k, st))) return rc;
    return POISSON_OK;
  }
  const int n = (int)b->plans.size();
  int sweeps = 1;
  bool singular = false;
  for (const poisson_plan* p : b->plans) {
    sweeps = std::max(sweeps, p->max_iters);
    singular = singular || p->singular;
  }
  const RefineJob* jobs = b->drefine;
  const dim3 blk(REFINE_NT);
  // the refinement kernels of all instances, one launch per kind (each
  // instance on its own block range, as in its single-plan launch)
  hipLaunchKernelGGL(refine_batch_init, dim3(n), dim3(256), 0, st, jobs);
  if (singular) {
    hipLaunchKernelGGL(refine_batch_wsum, dim3(b->refine_eblocks), blk, 0, st, jobs, n);
    hipLaunchKernelGGL(refine_batch_mean, dim3(n), blk, 0, st, jobs);
  }
  hipLaunchKernelGGL(refine_batch_prep, dim3(b->refine_eblocks), blk, 0, st, jobs, n);
  HIP_TRY(hipGetLastError());
  for (int k = 0; k < 5; ++k)
    if ((rc = batch_enqueue_step(b, k, st))) return rc;
  for (int sweep = 1; sweep < sweeps; ++sweep) {
    hipLaunchKernelGGL(refine_batch_residual, dim3(b->refine_rblocks), blk, 0, st, jobs, n, sweep);
    HIP_TRY(hipGetLastError());
    for (int k = 5; k < 10; ++k)
      if ((rc = batch_enqueue_step(b, k, st))) return rc;
    hipLaunchKernelGGL(refine_batch_update, dim3(b->refine_eblocks), blk, 0, st, jobs, n);
    hipLaunchKernelGGL(refine_batch_status, dim3(n), blk, 0, st, jobs, sweep);
    HIP_TRY(hipGetLastError());
  }
  if (singular) {
    hipLaunchKernelGGL(refine_batch_wsum, dim3(b->refine_eblocks), blk, 0, st, jobs, n);
    hipLaunchKernelGGL(refine_batch_mean, dim3(n), blk, 0, st, jobs);
    hipLaunchKernelGGL(refine_batch_shift, dim3(b->refine_eblocks), blk, 0, st, jobs, n);
  }
  HIP_TRY(hipGetLastError());
  for (const poisson_plan* p : b->plans)
    HIP_TRY(hipMemcpyAsync(p->stats_host, p->stats, REFINE_PARTIALS * sizeof(double),
                           hipMemcpyDeviceToHost, st));
  return POISSON_OK;
}

extern "C" int batch_launch(poisson_batch* b, hipStream_t st, int use_graph) {
  if (!b) return fail(POISSON_EINVAL, "null batch");
  if (!b->bound) return fail(POISSON_EINVAL, "batch has no fields bound (batch_bind)");
  if (!use_graph) return batch_enqueue(b, st);
  if (!b->exec) {
    // capture the launches once on a private stream; the job tables live in
    // device memory, so later batch_bind calls of an FP64 batch need no
    // re-capture
    if (!b->cap) HIP_TRY(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
    HIP_TRY(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
    const int rc = batch_enqueue(b, b->cap);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(b->cap, &g);
    if (rc) { if (g) (void)hipGraphDestroy(g); return rc; }
    if (e != hipSuccess) return fail(POISSON_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
    b->graph = g;
    HIP_TRY(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
  }
  HIP_TRY(hipGraphLaunch(b->exec, st));
  return POISSON_OK;
}

extern "C" void batch_destroy(poisson_batch* b) {
  if (!b) return;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  if (b->djobs) (void)hipFree(b->djobs);
  if (b->drefine) (void)hipFree(b->drefine);
  delete b;
}

// ------------------------------------------------------------------ autotuner

__global__ void fill_kernel(double* x, long long n, double v) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    x[i] = v;
}

// Average time (ms) of `reps` calls of launch() on st, after one untimed call.
template <typename F>
static double time_launches(hipStream_t st, int reps, F&& launch, int& rc) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  rc = POISSON_OK;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    rc = fail(POISSON_EHIP, "hipEventCreate failed");
    if (e0) (void)hipEventDestroy(e0);
    return 0.0;
  }
  rc = launch();
  if (!rc && hipEventRecord(e0, st) != hipSuccess) rc = fail(POISSON_EHIP, "hipEventRecord failed");
  for (int r = 0; r < reps && !rc; ++r) rc = launch();
  float ms = 0.0f;
  if (!rc && (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
              hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
    rc = fail(POISSON_EHIP, "event timing failed");
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return rc ? 0.0 : (double)ms / reps;
}

template <typename T>
static int autotune_typed(poisson_plan* p, double* scratch, int reps, hipStream_t st,
                          double* report) {
  T* data = reinterpret_cast<T*>(scratch);
  const long long N = (long long)field_points(p);
  int rc = POISSON_OK;
  auto reset = [&]() -> int {
    hipLaunchKernelGGL(fill_kernel, dim3(1024), dim3(256), 0, st, scratch, N * (long long)sizeof(T) / 8, 0.5);
    HIP_TRY(hipGetLastError());
    return POISSON_OK;
  };
  for (int role = 0; role < 2; ++role) {
    const AxisTables& A = p->ax[role];
    if (!r2r_fast_length(A)) continue;
    int best = 0;
    double best_ms = 1e300;
    for (int V = 0; V < kFastVariants; ++V) {
      if (V == kRegStageVariant) {
        if (!regstage_applies<T>(p, A)) continue;
      } else if (V >= kAsyncVariant && !async_applies<T>(p, A, V - kAsyncVariant)) {
        continue;
      }
      if ((rc = reset())) return rc;
      // forward then backward: the field keeps its size over the repetitions
      const double ms = time_launches(st, reps, [&]() -> int {
        int r = launch_fast_variant<T>(p, A, V, 0, data, st, nullptr);
        if (!r) r = launch_fast_variant<T>(p, A, V, 1, data, st, nullptr);
        return r;
      }, rc);
      if (rc) return rc;
      if (report) report[role * kFastVariants + V] = ms;
      if (ms < best_ms) { best_ms = ms; best = V; }
    }
    set_tuned_choice(0, sizeof(T), A.m, A.axis == 0, best);
  }
  const int n = p->dims[p->s];
  if (tri_fast_length(n)) {
    int best = 0;
    double best_ms = 1e300;
    for (int V = 0; V < kTriVariants; ++V) {
      if (V == kTriAsyncVariant && !tri_async_applies<T>(p)) continue;
      if (V == kTriDirectVariant && !tri_direct_applies<T>(p, data)) continue;
      if ((rc = reset())) return rc;
      const double ms = time_launches(st, reps, [&]() -> int {
        return launch_tri_variant<T>(p, V, data, st, nullptr);
      }, rc);
      if (rc) return rc;
      if (report) report[2 * kFastVariants + V] = ms;
      if (ms < best_ms) { best_ms = ms; best = V; }
    }
    set_tuned_choice(1, sizeof(T), n, p->s == 0, best);
  }
  return POISSON_OK;
}

extern "C" int plan_autotune(poisson_plan* p, double* scratch, int reps, hipStream_t st,
                             double* report) {
  if (!p || !scratch) return fail(POISSON_EINVAL, "null argument");
  if (int rc = misaligned(scratch, "scratch")) return rc;
  if (reps < 1 || reps > 1000) return fail(POISSON_EINVAL, "reps must be in [1, 1000]");
  if (lds_setup_once()) return g_err;
  if (report)
    for (int i = 0; i < 2 * (2 * kFastVariants + kTriVariants); ++i) report[i] = -1.0;
  int rc = autotune_typed<double>(p, scratch, reps, st, report);
  if (!rc) rc = autotune_typed<float>(p, scratch, reps, st,
                                      report ? report + 2 * kFastVariants + kTriVariants : nullptr);
  return rc;
}

// Choice per step of a bound batch: every job of the step in the variant of
// the per-length table, or all in one synchronous variant.  A batch launch
// runs at the occupancy of its largest job configuration (its LDS), so the
// fastest variant of each instance alone is not always the fastest mix.
static constexpr int kBatchCandidates = 5;   // table, then variants 0-3 (elimination: 0-1)

extern "C" int batch_autotune(poisson_batch* b, int reps, hipStream_t st, double* report) {
  if (!b) return fail(POISSON_EINVAL, "null batch");
  if (!b->bound) return fail(POISSON_EINVAL, "batch has no fields bound (batch_bind)");
  if (reps < 1 || reps > 1000) return fail(POISSON_EINVAL, "reps must be in [1, 1000]");
  if (report)
    for (int i = 0; i < 5 * kBatchCandidates; ++i) report[i] = -1.0;
  HIP_TRY(hipStreamSynchronize(st));   // nothing of the batch in flight before its tables change
  auto reset = [&]() -> int {
    for (size_t i = 0; i < b->plans.size(); ++i)
      hipLaunchKernelGGL(fill_kernel, dim3(256), dim3(256), 0, st, b->rhs[i],
                         (long long)field_points(b->plans[i]), 0.5);
    HIP_TRY(hipGetLastError());
    return POISSON_OK;
  };
  int rc = POISSON_OK;
  for (int k = 0; k < 5; ++k) {
    const int count = kStepRole[k] >= 0 ? 4 : 2;
    int best = -1;
    double best_ms = 1e300;
    for (int c = -1; c < count; ++c) {
      b->force[k] = c;
      if ((rc = batch_upload(b)) || (rc = reset())) return rc;
      const double ms = time_launches(st, reps, [&]() { return batch_enqueue_step(b, k, st); }, rc);
      if (rc) return rc;
      if (report) report[k * kBatchCandidates + c + 1] = ms;
      if (ms < best_ms) { best_ms = ms; best = c; }
    }
    b->force[k] = best;
  }
  return batch_upload(b);
}

extern "C" int set_tuned_variant(int family, int n, int layout, int fp64, int variant) {
  if (family != 0 && family != 1) return fail(POISSON_EINVAL, "family must be 0 or 1");
  const int count = family == 0 ? kFastVariants : kTriVariants;
  if (variant < 0 || variant >= count) return fail(POISSON_EINVAL, "variant must be in [0, %d)", count);
  const bool ok = family == 0 ? (n % 2 == 0 && with_fast_cfg(n / 2, 0, [](auto) { return 0LL; }) == 0)
                              : tri_fast_length(n);
  if (!ok) return fail(POISSON_EUNSUPPORTED, "length %d has no size-specialised kernels", n);
  set_tuned_choice(family, fp64 ? 8 : 4, family == 0 ? n / 2 : n, layout ? 1 : 0, variant);
  return POISSON_OK;
}

extern "C" int tuned_variant(int family, int n, int layout, int fp64) {
  if (family != 0 && family != 1) return fail(POISSON_EINVAL, "family must be 0 or 1");
  const int len = family == 0 ? n / 2 : n;   // transforms are keyed by M = n/2
  return tuned_choice(family, fp64 ? 8 : 4, len, layout ? 1 : 0);
}

// ------------------------------------------------------------------ server

#include "server.h"
