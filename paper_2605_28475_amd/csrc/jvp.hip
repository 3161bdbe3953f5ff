// Two-input forms of the collision operator.  The Jacobian-vector product
// out = J(c) d = Q(c, d) + Q(d, c),
// the derivative of Q at c in the direction d (with Q(f, g) the bilinear form whose
// diagonal is Q(f, f), Section 2.3).  It is the apply kernel with two inputs: per
// slice the coupling accumulates sum_z g_z (c_{k2,q2z} d_{k3,q3z} + d_{k2,q2z} c_{k3,q3z}),
// which the merged radial tiles contract exactly as they do f (x) f.  The bilinear form
// Q(f, g) itself adds the antisymmetric part: the coupling sum_z g_z (f_x (x) g_y -
// g_x (x) f_y) contracted with the partner tiles D of the merged channels.  Both cell
// tiles sit in LDS, so the default tile holds at most half as many cells as for Q(f, f).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/wefq.h"
#include "wefq_core.h"
#include "apply_tile.h"

namespace wefq {

// FP32 launches run 12 waves per workgroup (768 threads, three per SIMD; the two cell tiles
// fill the LDS, so one workgroup holds a compute unit), 16 up to 5x5 quadrants (1,024 threads,
// four per SIMD, whose registers fit 128); FP64 launches 8.  Measured on one MI355X, J(c) d in
// FP32, 8 -> 12 waves: K = L = 12 with 65,536 cells 66.4 -> 62.4 ms, K = L = 16 with 8,192 cells
// 59.2 -> 51.3 ms, K = L = 8 with 65,536 cells 7.08 -> 6.02 ms, K = L = 10 and 14 11% and 10%
// faster; 12 -> 16 waves: K = L = 8 6.06 -> 5.72 ms, K = L = 9 with 32,768 cells 4.86 -> 4.59 ms,
// K = L = 6 equal; in FP64 the 12-wave instances spill.
template <int H, int MODE> constexpr int jvp_waves() { return MODE == 0 ? (H <= 5 ? 16 : 12) : 8; }

template <int H, int SLOTS, int RT, int MODE, bool ANTI>
__global__ __launch_bounds__((64 * jvp_waves<H, MODE>())) void apply_jvp_kernel(MfmaParams p) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  __shared__ int unit_ctr;
  mfma_tile<H, SLOTS, RT, MODE, true, ANTI, jvp_waves<H, MODE>()>(p, (int64_t)blockIdx.x, (int)blockIdx.y, lds_raw,
                                                               &unit_ctr);
}

template <int H, int SLOTS, int RT, int MODE>
static hipError_t launch_jvp_t(const MfmaParams& p, bool anti, int64_t ntiles, size_t lds, hipStream_t s) {
  auto k = anti ? apply_jvp_kernel<H, SLOTS, RT, MODE, true> : apply_jvp_kernel<H, SLOTS, RT, MODE, false>;
  hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k, dim3((unsigned)ntiles, (unsigned)p.nsplit), dim3((64 * jvp_waves<H, MODE>())), lds, s, p);
  return hipGetLastError();
}

// Eight output states per column group (tiles of 2 cells) exist for FP64 at H >= 7 only:
// there two FP64 tiles of 4 cells no longer fit LDS (K = L >= 13).  At H >= 8, where the
// apply's work units hold 4 output states, these launches take a second unit list with 8.
template <int H, int RT, int MODE>
static hipError_t launch_jvp_s(const MfmaParams& p, bool anti, int slots, int64_t ntiles, size_t lds,
                               hipStream_t s) {
  switch (slots) {
    case 1: return launch_jvp_t<H, 1, RT, MODE>(p, anti, ntiles, lds, s);
    case 2: return launch_jvp_t<H, 2, RT, MODE>(p, anti, ntiles, lds, s);
    case 4: return launch_jvp_t<H, 4, RT, MODE>(p, anti, ntiles, lds, s);
    case 8:
      if constexpr (MODE == 2 && H >= 7) return launch_jvp_t<H, 8, RT, MODE>(p, anti, ntiles, lds, s);
      return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
}

template <int H>
static hipError_t launch_jvp_h(const MfmaParams& p, bool anti, int mode, int slots, int rt, int64_t ntiles,
                               size_t lds, hipStream_t s) {
  if (rt == 2) {
    if constexpr (H >= 8) {
      if (mode == 0) return launch_jvp_s<H, 2, 0>(p, anti, slots, ntiles, lds, s);
      if (mode == 2) return launch_jvp_s<H, 2, 2>(p, anti, slots, ntiles, lds, s);
    }
    return hipErrorInvalidValue;
  }
  if (mode == 0) return launch_jvp_s<H, 1, 0>(p, anti, slots, ntiles, lds, s);
  if (mode == 2) return launch_jvp_s<H, 1, 2>(p, anti, slots, ntiles, lds, s);
  return hipErrorInvalidValue;
}

// One two-input launch: symmetric coupling with the merged tiles (anti = false), or the
// antisymmetric coupling with the partner tiles, combined into out (anti = true).
static hipError_t launch_two(const wefq_core* h, bool anti, int precision, const void* f, const void* g, void* out,
                             int64_t B, int64_t ldf, int64_t ldg, int64_t ldo, hipStream_t s) {
  if (B == 0) return hipSuccess;
  const int mode = mfma_mode(precision);
  if (mode != 0 && mode != 2) return hipErrorInvalidValue;
  const size_t elem = mode == 2 ? 8 : 4;
  int slots = 0;
  for (int sl : {1, 2, 4, 8}) {
    if (sl == 8 && (mode != 2 || h->H < 7)) break;
    if (2 * tile_lds_bytes(h, sl, elem) <= (size_t)h->lds_limit) { slots = sl; break; }
  }
  if (slots == 0) return hipErrorInvalidValue;
  MfmaParams p;
  p.f = f; p.g = g; p.Q = out; p.B = B; p.ldf = ldf; p.ldg = ldg; p.ldq = ldo;
  p.NK = h->NK; p.NQ = h->NQ; p.N = h->N;
  p.nunits = h->nunits; p.units = h->d_units; p.chan_begin = h->d_chan_begin;
  p.slice_off = h->d_slice_off; p.sptr = h->d_sptr; p.spair = h->d_spair; p.mq = h->d_mq; p.mq_pad = h->d_mq_pad;
  p.mg = h->d_mg; p.mg64 = h->d_mg64;
  p.Rt32 = anti ? h->d_Dt32 : h->d_Rt32; p.Rt64 = anti ? h->d_Dt64 : h->d_Rt64;
  p.R16_32 = anti ? h->d_D16_32 : h->d_R16_32; p.R16_64 = anti ? h->d_D16_64 : h->d_R16_64;
  p.Rhi = nullptr; p.Rlo = nullptr;
  if (slots == 8 && h->d_units8) { p.units = h->d_units8; p.nunits = h->nunits8; }
  const int TB = 16 / slots;
  const int64_t ntiles = (B + TB - 1) / TB;
  p.nsplit = tile_splits(h, ntiles, p.nunits, 1, 0);
  if (p.nsplit > 1 && p.nsplit > p.nunits / 4) p.nsplit = p.nunits / 4 > 1 ? p.nunits / 4 : 1;
  const size_t lds = 2 * tile_lds_bytes(h, slots, elem);
  // a launch holds at most 2^32 - 1 threads: larger batches run as several launches of whole
  // tiles (each cell's result does not depend on its batch)
  const int64_t max_cells = max_cells_per_launch(TB, 1024);   // the largest block of any instance
  if (B > max_cells) {
    for (int64_t c0 = 0; c0 < B; c0 += max_cells) {
      const int64_t nc = (B - c0) < max_cells ? (B - c0) : max_cells;
      const hipError_t e = launch_two(h, anti, precision, (const char*)f + c0 * ldf * elem,
                                      (const char*)g + c0 * ldg * elem, (char*)out + c0 * ldo * elem, nc, ldf, ldg,
                                      ldo, s);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  switch (h->H) {
    case 1: return launch_jvp_h<1>(p, anti, mode, slots, h->RT, ntiles, lds, s);
    case 2: return launch_jvp_h<2>(p, anti, mode, slots, h->RT, ntiles, lds, s);
    case 3: return launch_jvp_h<3>(p, anti, mode, slots, h->RT, ntiles, lds, s);
    case 4: return launch_jvp_h<4>(p, anti, mode, slots, h->RT, ntiles, lds, s);
    case 5: return launch_jvp_h<5>(p, anti, mode, slots, h->RT, ntiles, lds, s);
    case 6: return launch_jvp_h<6>(p, anti, mode, slots, h->RT, ntiles, lds, s);
    case 7: return launch_jvp_h<7>(p, anti, mode, slots, h->RT, ntiles, lds, s);
    case 8: return launch_jvp_h<8>(p, anti, mode, slots, h->RT, ntiles, lds, s);
    case 9: return launch_jvp_h<9>(p, anti, mode, slots, h->RT, ntiles, lds, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_apply_jvp(const wefq_core* h, int precision, const void* c, const void* d, void* out,
                            int64_t B, int64_t ldc, int64_t ldd, int64_t ldo, hipStream_t s) {
  return launch_two(h, false, precision, c, d, out, B, ldc, ldd, ldo, s);
}

// Q(f, g) = (R~ Phi_S + D Phi_A) / 2: the symmetric launch writes R~ Phi_S = J(f) g, the
// antisymmetric one adds D Phi_A and halves, on the same stream.
hipError_t launch_apply_qfg(const wefq_core* h, int precision, const void* f, const void* g, void* out,
                            int64_t B, int64_t ldf, int64_t ldg, int64_t ldo, hipStream_t s) {
  hipError_t e = launch_two(h, false, precision, f, g, out, B, ldf, ldg, ldo, s);
  if (e != hipSuccess) return e;
  return launch_two(h, true, precision, f, g, out, B, ldf, ldg, ldo, s);
}

}  // namespace wefq
