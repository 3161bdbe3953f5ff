// Attainable arithmetic rates of the device, measured with kernels that do nothing else:
// chains of matrix-core instructions (FP32 and FP64 16x16x4, BF16 16x16x32) or of unpacked
// vector fused multiply-adds (FP32, FP64), with no memory traffic but one store per lane at the
// end.  They give the measured peaks that a kernel's algorithmic rate is set against, beside
// the datasheet figures.
#include <hip/hip_runtime.h>

#include <string>

#include "../../include/wefq.h"
#include "wefq_core.h"

namespace wefq {

typedef float p4f __attribute__((ext_vector_type(4)));
typedef double p4d __attribute__((ext_vector_type(4)));
typedef __bf16 p8bf __attribute__((ext_vector_type(8)));

constexpr int kProbeBlock = 256;
constexpr int kUnroll = 16;        // matrix instructions per loop trip
constexpr int kValuChains = 8;     // independent chains per lane (vector ALU)

template <int KIND>
__global__ __launch_bounds__(kProbeBlock) void peak_kernel(double* out, int iters, float seed) {
  const int64_t gid = (int64_t)blockIdx.x * kProbeBlock + threadIdx.x;
  const float t = (float)threadIdx.x * 1e-7f;
  double result = 0.0;
  // Matrix cores: one dependent chain per wave, kUnroll instructions per loop trip.  The
  // 8 waves of each SIMD interleave their chains, which keeps its matrix pipe busy; one
  // chain also keeps the compiler from shuffling accumulators between register files
  // inside the loop, which several chains per wave provoke.
  if constexpr (KIND == WEFQ_PROBE_MFMA_F32) {
    p4f c = {0.f, 0.f, 0.f, 0.f};
    const float a = seed + t, b = seed - t;
    for (int i = 0; i < iters; ++i)
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) c = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    result = (double)c[0] + c[1] + c[2] + c[3];
  } else if constexpr (KIND == WEFQ_PROBE_MFMA_F64) {
    p4d c = {0.0, 0.0, 0.0, 0.0};
    const double a = seed + t, b = seed - t;
    for (int i = 0; i < iters; ++i)
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) c = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    result = c[0] + c[1] + c[2] + c[3];
  } else if constexpr (KIND == WEFQ_PROBE_MFMA_BF16) {
    p4f c = {0.f, 0.f, 0.f, 0.f};
    p8bf a, b;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      a[e] = (__bf16)(seed + t * (float)e);
      b[e] = (__bf16)(seed - t * (float)e);
    }
    for (int i = 0; i < iters; ++i)
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    result = (double)c[0] + c[1] + c[2] + c[3];
  } else if constexpr (KIND == WEFQ_PROBE_VALU_F32) {
    // x <- x * m + a with |m| < 1 stays bounded; the chains are independent
    float x[kValuChains];
#pragma unroll
    for (int c = 0; c < kValuChains; ++c) x[c] = seed + t * (float)c;
    const float m = 0.9999f - t, a = seed * 1e-4f;
    for (int i = 0; i < iters; ++i)
#pragma unroll
      for (int c = 0; c < kValuChains; ++c) x[c] = __builtin_fmaf(x[c], m, a);
#pragma unroll
    for (int c = 0; c < kValuChains; ++c) result += x[c];
  } else {
    double x[kValuChains];
#pragma unroll
    for (int c = 0; c < kValuChains; ++c) x[c] = (double)seed + (double)t * c;
    const double m = 0.9999 - (double)t, a = (double)seed * 1e-4;
    for (int i = 0; i < iters; ++i)
#pragma unroll
      for (int c = 0; c < kValuChains; ++c) x[c] = __builtin_fma(x[c], m, a);
#pragma unroll
    for (int c = 0; c < kValuChains; ++c) result += x[c];
  }
  out[gid] = result;
}

// FLOP of one loop iteration of one wave (a multiply-add counts 2)
static double probe_flop_per_wave_iter(int kind) {
  switch (kind) {
    case WEFQ_PROBE_MFMA_F32:
    case WEFQ_PROBE_MFMA_F64: return kUnroll * 16.0 * 16 * 4 * 2;
    case WEFQ_PROBE_MFMA_BF16: return kUnroll * 16.0 * 16 * 32 * 2;
    default: return kValuChains * 64.0 * 2;
  }
}

static int probe_iters(int kind) {
  switch (kind) {
    case WEFQ_PROBE_MFMA_F32:
    case WEFQ_PROBE_MFMA_F64: return 1024;
    case WEFQ_PROBE_MFMA_BF16: return 4096;
    default: return 16384;
  }
}

template <int KIND>
static void launch_kind(int grid, double* out, int iters, float seed, hipStream_t s) {
  hipLaunchKernelGGL(peak_kernel<KIND>, dim3(grid), dim3(kProbeBlock), 0, s, out, iters, seed);
}

static void launch_probe(int kind, int grid, double* out, int iters, hipStream_t s) {
  const float seed = 1e-3f;
  switch (kind) {
    case WEFQ_PROBE_MFMA_F32: launch_kind<WEFQ_PROBE_MFMA_F32>(grid, out, iters, seed, s); break;
    case WEFQ_PROBE_MFMA_F64: launch_kind<WEFQ_PROBE_MFMA_F64>(grid, out, iters, seed, s); break;
    case WEFQ_PROBE_MFMA_BF16: launch_kind<WEFQ_PROBE_MFMA_BF16>(grid, out, iters, seed, s); break;
    case WEFQ_PROBE_VALU_F32: launch_kind<WEFQ_PROBE_VALU_F32>(grid, out, iters, seed, s); break;
    default: launch_kind<WEFQ_PROBE_VALU_F64>(grid, out, iters, seed, s); break;
  }
}

}  // namespace wefq

using namespace wefq;

extern "C" wefq_status wefq_peak_probe(int32_t device, int32_t kind, double* tflops, void* stream) {
  if (!tflops) { set_error("null output pointer"); return WEFQ_EINVAL; }
  *tflops = 0.0;
  if (kind < WEFQ_PROBE_MFMA_F32 || kind > WEFQ_PROBE_VALU_F64) { set_error("unknown probe kind"); return WEFQ_EINVAL; }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) { set_error("no HIP device available"); return WEFQ_EHIP; }
  if (device < 0 || device >= ndev) { set_error("device ordinal out of range"); return WEFQ_EINVAL; }
  if (hipSetDevice(device) != hipSuccess) { set_error("hipSetDevice failed"); return WEFQ_EHIP; }
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cus <= 0) {
    set_error("cannot read the compute unit count");
    return WEFQ_EHIP;
  }
  const int grid = cus * 8;                      // 8 workgroups of 4 waves per CU: 8 waves per SIMD
  const int iters = probe_iters(kind);
  hipStream_t s = (hipStream_t)stream;
  double* out = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipMalloc(&out, (size_t)grid * kProbeBlock * sizeof(double));
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  float best_ms = 0.0f;
  if (e == hipSuccess) {
    launch_probe(kind, grid, out, iters, s);    // warm-up (clocks, code load)
    e = hipGetLastError();
  }
  for (int rep = 0; rep < 5 && e == hipSuccess; ++rep) {
    e = hipEventRecord(e0, s);
    if (e != hipSuccess) break;
    launch_probe(kind, grid, out, iters, s);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e == hipSuccess && ms > 0.0f && (best_ms == 0.0f || ms < best_ms)) best_ms = ms;
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (out) (void)hipFree(out);
  if (e != hipSuccess) { set_error(std::string("peak probe: ") + hipGetErrorString(e)); return WEFQ_EHIP; }
  if (best_ms <= 0.0f) { set_error("peak probe: no timing"); return WEFQ_EHIP; }
  const double waves = (double)grid * (kProbeBlock / 64);
  *tflops = probe_flop_per_wave_iter(kind) * iters * waves / (best_ms * 1e-3) / 1e12;
  return WEFQ_OK;
}
