// Batched explicit Runge-Kutta stepping of the Galerkin system dc/dt = Q(c)
// (Section 2.3: with the identity mass matrix the weak form is an ODE system per
// spatial cell; the relaxation experiments of Section 5 integrate it with an
// explicit Runge-Kutta scheme).
//
// Every stage is one apply of the collision operator on the whole batch,
// followed by a fused element-wise combination y = c + dt * sum_j a_sj k_j; the
// step ends with c += dt * sum_j b_j k_j.  The invariant rows of every stage
// evaluation are checked in FP64 on the device (running maximum of |k_s| on the
// mass, momentum and energy rows, kept in the workspace), so the in-loop check
// costs no host synchronization; the maximum is read once at the end.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>

#include "../../include/wefq.h"
#include "wefq_core.h"

namespace wefq {

// Butcher tableaux of the explicit schemes: a[s][j] (j < s), b[s].
struct Tableau {
  int stages;
  double a[4][4];
  double b[4];
};

static const Tableau* tableau(int scheme) {
  static const Tableau euler = {1, {{0}}, {1.0}};
  static const Tableau heun = {2, {{0}, {1.0}}, {0.5, 0.5}};
  static const Tableau ssp3 = {3, {{0}, {1.0}, {0.25, 0.25}}, {1.0 / 6.0, 1.0 / 6.0, 2.0 / 3.0}};
  static const Tableau rk4 = {4, {{0}, {0.5}, {0.0, 0.5}, {0.0, 0.0, 1.0}},
                              {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0}};
  switch (scheme) {
    case WEFQ_RK_EULER: return &euler;
    case WEFQ_RK_HEUN: return &heun;
    case WEFQ_RK_SSP3: return &ssp3;
    case WEFQ_RK_CLASSIC4: return &rk4;
    default: return nullptr;
  }
}

template <typename T>
struct CombineParams {
  const T* c;              // [B][ldc]
  T* out;                  // [B][ldo]
  const T* k[4];           // stage derivatives, [B][N] each
  double coef[4];          // dt * tableau weight per stage (0 for absent terms)
  int nk;
  int64_t B, N, ldc, ldo;
};

// out = c + sum_j coef_j k_j, terms added in stage order (FMA in the element type).
template <typename T>
__global__ __launch_bounds__(256) void rk_combine_kernel(CombineParams<T> p) {
  const int64_t total = p.B * p.N;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = i / p.N, n = i - b * p.N;
    T v = p.c[b * p.ldc + n];
    for (int j = 0; j < p.nk; ++j) v = fma((T)p.coef[j], p.k[j][i], v);
    p.out[b * p.ldo + n] = v;
  }
}

// Running FP64 maximum of |k| over the invariant rows of every cell.  The value is
// non-negative, so its IEEE bit pattern orders like an unsigned integer (NaN above
// +inf, so a NaN propagates).
template <typename T>
__global__ __launch_bounds__(256) void rk_invariant_kernel(const T* k, int64_t B, int64_t N, int NK, int L,
                                                         unsigned long long* maxbits) {
  __shared__ unsigned long long red[256];
  int rows[5] = {0, 1, NK, 2 * NK, 3 * NK};
  int nrows = 1 + (NK > 1 ? 1 : 0);
  if (L >= 1) { rows[nrows] = NK; rows[nrows + 1] = 2 * NK; rows[nrows + 2] = 3 * NK; nrows += 3; }
  unsigned long long m = 0;
  for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < B; b += (int64_t)gridDim.x * blockDim.x)
    for (int i = 0; i < nrows; ++i) {
      const double v = fabs((double)k[b * N + rows[i]]);
      const unsigned long long u = (unsigned long long)__double_as_longlong(v);
      m = u > m ? u : m;
    }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int st = blockDim.x / 2; st > 0; st >>= 1) {
    if (threadIdx.x < st) red[threadIdx.x] = red[threadIdx.x + st] > red[threadIdx.x] ? red[threadIdx.x + st] : red[threadIdx.x];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicMax(maxbits, red[0]);
}

__global__ void rk_reset_kernel(unsigned long long* maxbits) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *maxbits = 0ull;
}

static int64_t grid_for(int64_t work) {
  int64_t g = (work + 255) / 256;
  return g < 1 ? 1 : (g > 16384 ? 16384 : g);
}

template <typename T>
static hipError_t rk_run(wefq_core* h, int precision, const Tableau& tb, T* c, int64_t B, int64_t ld, double dt,
                         int nsteps, char* work, hipStream_t s) {
  const int64_t N = h->N;
  unsigned long long* maxbits = reinterpret_cast<unsigned long long*>(work);
  T* y = reinterpret_cast<T*>(work + 256);
  T* k[4];
  for (int j = 0; j < tb.stages; ++j) k[j] = y + (size_t)(j + 1) * B * N;
  hipLaunchKernelGGL(rk_reset_kernel, dim3(1), dim3(64), 0, s, maxbits);
  hipError_t e = hipGetLastError();
  const int64_t cgrid = grid_for(B * N), igrid = grid_for(B);
  for (int step = 0; step < nsteps && e == hipSuccess; ++step) {
    for (int st = 0; st < tb.stages && e == hipSuccess; ++st) {
      // stage input: c itself for the first stage, else c + dt sum_j a_sj k_j
      const T* in = c;
      int64_t ldin = ld;
      if (st > 0) {
        CombineParams<T> p;
        p.c = c; p.out = y; p.nk = st; p.B = B; p.N = N; p.ldc = ld; p.ldo = N;
        for (int j = 0; j < 4; ++j) { p.k[j] = j < st ? k[j] : nullptr; p.coef[j] = j < st ? dt * tb.a[st][j] : 0.0; }
        hipLaunchKernelGGL(rk_combine_kernel<T>, dim3((unsigned)cgrid), dim3(256), 0, s, p);
        e = hipGetLastError();
        in = y;
        ldin = N;
      }
      if (e != hipSuccess) break;
      e = precision == WEFQ_FP64_NAIVE ? launch_apply_fp64(h, (const double*)in, (double*)k[st], B, ldin, N, s)
                                       : launch_apply_mfma(h, precision, in, k[st], B, ldin, N, s);
      if (e != hipSuccess) break;
      hipLaunchKernelGGL(rk_invariant_kernel<T>, dim3((unsigned)igrid), dim3(256), 0, s, k[st], B, N, h->NK, h->L,
                         maxbits);
      e = hipGetLastError();
    }
    if (e != hipSuccess) break;
    CombineParams<T> p;
    p.c = c; p.out = c; p.nk = tb.stages; p.B = B; p.N = N; p.ldc = ld; p.ldo = ld;
    for (int j = 0; j < 4; ++j) { p.k[j] = j < tb.stages ? k[j] : nullptr; p.coef[j] = j < tb.stages ? dt * tb.b[j] : 0.0; }
    hipLaunchKernelGGL(rk_combine_kernel<T>, dim3((unsigned)cgrid), dim3(256), 0, s, p);
    e = hipGetLastError();
  }
  return e;
}

// Fixed device scratch of wefq_rk_integrate_noalloc: the check state and the stage buffers,
// laid out as the caller-owned workspace of wefq_rk_integrate.  Every device the library runs
// on holds its own copy until the process ends.  Host code never passes this name to a
// kernel (on the host it is only a stand-in for the symbol); it uses the device address that
// hipGetSymbolAddress returns, looked up once per device.
static __device__ __align__(256) char rk_scratch[WEFQ_RK_NOALLOC_BYTES];

static std::mutex rk_scratch_mu;
static char* rk_scratch_ptr[64];

// Device address of rk_scratch on the current device (the caller has selected it).
static hipError_t rk_scratch_address(int device, char** out) {
  if (device < 0 || device >= 64) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(rk_scratch_mu);
  if (!rk_scratch_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(rk_scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    rk_scratch_ptr[device] = static_cast<char*>(p);
  }
  *out = rk_scratch_ptr[device];
  return hipSuccess;
}

}  // namespace wefq

using namespace wefq;

static wefq_status rk_fail(wefq_status st, const std::string& msg) {
  set_error(msg);
  return st;
}

static bool rk_precision_ok(const wefq_core* h, int precision) {
  if (precision != WEFQ_FP64 && precision != WEFQ_FP32 && precision != WEFQ_BF16X3 && precision != WEFQ_FP64_NAIVE)
    return false;
  const unsigned need = precision == WEFQ_FP64_NAIVE ? (unsigned)WEFQ_FP64 : (unsigned)precision;
  return (h->precisions & need) != 0;
}

extern "C" {

wefq_status wefq_rk_workspace(wefq_handle h, int32_t precision, int32_t scheme, int64_t B, int64_t* bytes) {
  if (!h || !bytes) return rk_fail(WEFQ_EINVAL, "null argument");
  const Tableau* tb = tableau(scheme);
  if (!tb) return rk_fail(WEFQ_EINVAL, "unknown Runge-Kutta scheme");
  if (!rk_precision_ok(h, precision)) return rk_fail(WEFQ_EINVAL, "precision unknown or not prepared for this core");
  if (B < 0) return rk_fail(WEFQ_EINVAL, "negative batch size");
  const int64_t elem = (precision == WEFQ_FP64 || precision == WEFQ_FP64_NAIVE) ? 8 : 4;
  *bytes = 256 + (int64_t)(tb->stages + 1) * B * h->N * elem;
  return WEFQ_OK;
}

}  // extern "C"

// Shared by wefq_rk_integrate (caller workspace) and wefq_rk_integrate_noalloc (the fixed
// device scratch, work == nullptr): argument checks, the stepping, the optional readback.
static wefq_status rk_integrate_impl(wefq_handle h, int32_t precision, int32_t scheme, void* c, int64_t B, int64_t ld,
                                     double dt, int32_t nsteps, void* work, int64_t work_bytes, double* max_invariant,
                                     void* stream, bool fixed_scratch) {
  if (!h) return rk_fail(WEFQ_EINVAL, "null handle");
  const Tableau* tb = tableau(scheme);
  if (!tb) return rk_fail(WEFQ_EINVAL, "unknown Runge-Kutta scheme");
  if (!rk_precision_ok(h, precision)) return rk_fail(WEFQ_EINVAL, "precision unknown or not prepared for this core");
  if (B < 0 || nsteps < 0) return rk_fail(WEFQ_EINVAL, "negative batch size or step count");
  if (!(dt == dt) || dt > 1e300 || dt < -1e300) return rk_fail(WEFQ_EINVAL, "time step must be finite");
  if (max_invariant) *max_invariant = 0.0;
  if (B == 0 || nsteps == 0) return WEFQ_OK;
  if (!c || (!work && !fixed_scratch)) return rk_fail(WEFQ_EINVAL, "null coefficient or workspace pointer");
  if (ld < h->N) return rk_fail(WEFQ_EINVAL, "leading dimension smaller than N");
  const int64_t elem = (precision == WEFQ_FP64 || precision == WEFQ_FP64_NAIVE) ? 8 : 4;
  const int64_t need = 256 + (int64_t)(tb->stages + 1) * B * h->N * elem;
  if (fixed_scratch && need > (int64_t)WEFQ_RK_NOALLOC_BYTES)
    return rk_fail(WEFQ_EBUDGET, "batch needs " + std::to_string(need) + " bytes of stage buffers, more than the " +
                                     std::to_string((long long)WEFQ_RK_NOALLOC_BYTES) +
                                     "-byte fixed scratch (WEFQ_RK_NOALLOC_BYTES); use wefq_rk_integrate");
  if (hipSetDevice(h->device) != hipSuccess) return rk_fail(WEFQ_EHIP, "hipSetDevice failed");
  if (fixed_scratch) {
    char* p = nullptr;
    const hipError_t e = rk_scratch_address(h->device, &p);
    if (e != hipSuccess) return rk_fail(WEFQ_EHIP, std::string("fixed scratch address: ") + hipGetErrorString(e));
    work = p;
    work_bytes = (int64_t)WEFQ_RK_NOALLOC_BYTES;
  }
  if (((uintptr_t)c & (uintptr_t)(elem - 1)) || ((uintptr_t)work & 255))
    return rk_fail(WEFQ_EINVAL, "c must be aligned to the element size and the workspace to 256 bytes");
  if (work_bytes < need) return rk_fail(WEFQ_EINVAL, "workspace smaller than wefq_rk_workspace reports");
  const char* cb = (const char*)c;
  const char* wb = (const char*)work;
  if (cb < wb + need && wb < cb + (size_t)B * ld * elem) return rk_fail(WEFQ_EINVAL, "c and the workspace overlap");
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = elem == 8 ? rk_run<double>(h, precision, *tb, (double*)c, B, ld, dt, nsteps, (char*)work, s)
                           : rk_run<float>(h, precision, *tb, (float*)c, B, ld, dt, nsteps, (char*)work, s);
  if (e != hipSuccess) return rk_fail(WEFQ_EHIP, std::string("Runge-Kutta launch failed: ") + hipGetErrorString(e));
  if (max_invariant) {
    unsigned long long bits = 0;
    e = hipMemcpyAsync(&bits, work, sizeof(bits), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return rk_fail(WEFQ_EHIP, std::string("invariant check readback: ") + hipGetErrorString(e));
    double v;
    static_assert(sizeof(v) == sizeof(bits), "double is 64-bit");
    __builtin_memcpy(&v, &bits, sizeof(v));
    *max_invariant = v;
  }
  return WEFQ_OK;
}

extern "C" {

wefq_status wefq_rk_integrate(wefq_handle h, int32_t precision, int32_t scheme, void* c, int64_t B, int64_t ld,
                              double dt, int32_t nsteps, void* work, int64_t work_bytes, double* max_invariant,
                              void* stream) {
  return rk_integrate_impl(h, precision, scheme, c, B, ld, dt, nsteps, work, work_bytes, max_invariant, stream,
                           false);
}

wefq_status wefq_rk_integrate_noalloc(wefq_handle h, int32_t precision, int32_t scheme, void* c, int64_t B,
                                      int64_t ld, double dt, int32_t nsteps, double* max_invariant, void* stream) {
  return rk_integrate_impl(h, precision, scheme, c, B, ld, dt, nsteps, nullptr, 0, max_invariant, stream, true);
}

}  // extern "C"
