// Contraction kernels for Q(f, f) (Section 4.5) and the FP64 conservation check.
//
// apply_fp64_kernel   the plain FP64 comparator: the paper's naive contraction
//                     (eq. full_discrete_sum as written), one thread per output
//                     (cell, q1, k1), looping over the COO rows of q1 and k2, k3;
//                     no channel merging, no tiling, no matrix cores.
// apply_mfma_kernel   angular-first contraction (Section 4.5.4) re-laid for CDNA4
//                     (the per-tile code is mfma_tile in apply_tile.h):
//   * a workgroup owns a tile of 16 cells (8 or 4 when f does not fit in LDS; then
//     the 16 MFMA columns are 8 cells x 2 or 4 cells x 4 output states) and stages
//     their coefficients in LDS, rows (q, k) by cells;
//   * the COO rows (q1,q2,q3) and (q1,q3,q2) are merged (exact for Q(f,f)), so
//     channel (l1,l2,l3) with l2 < l3 carries R^{(l1l2l3)}_{k1k2k3} + R^{(l1l3l2)}_{k1k3k2};
//   * per slice (channel, q1) the intermediate Phi^{(c,q1)}_{k2k3} =
//     sum_z g_z f_{k2,q2z} f_{k3,q3z} (angular coupling, on the VALU) is built by
//     wave-uniform integer-indexed gathers from LDS straight into the MFMA
//     B-operand layout: lane group r = lane/16 owns the (k2,k3) quadrant
//     (r/2, r%2) of the NK x NK grid, lane%16 is the MFMA column (cell); rows
//     sharing q2 are applied in pairs, one outer product per pair;
//   * the radial contraction Q_{k1,q1} += sum R^{(c)}_{k1,(k2k3)} Phi_{(k2k3)}
//     runs on v_mfma_f32_16x16x4_f32 (FP32), v_mfma_f64_16x16x4_f64 (FP64) or as
//     three split hi/lo BF16 v_mfma_f32_16x16x32_bf16 products with FP32
//     accumulation (BF16X3); for NK = 17 the last radial row is a VALU dot product;
//   * the wave keeps the 16x16 accumulator tiles of a group of q1 values of
//     one l1 across all channels of that l1 (the channel reduction), so every
//     output is produced by one wave in a fixed order: results are bitwise
//     independent of the other cells in the batch;
//   * waves pull (l1, q1-group) work units from an LDS counter, largest first; a
//     launch with few tiles deals each tile's units to several workgroups.
// The mass, momentum and energy rows of Q come out as exact zeros because those rows of the
// core are zero (Section 4.4): every product on them is 0 x finite.  They are stored as
// computed, so the FP64 conservation check below tests the zeroing and the row mapping.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/wefq.h"
#include "wefq_core.h"
#include "apply_tile.h"

namespace wefq {

struct Fp64Params {
  const double* f;
  double* Q;
  int64_t B, ldf, ldq;
  int NK, N, nchunk;
  const double* R;
  const int* q1ptr;
  const int* ent_c;
  const uint32_t* ent_q;
  const double* ent_g;
};

// A wavefront holds 64 cells computing the same output (q1, k1): the COO rows
// and the rows of R they address are wave-uniform (scalar loads shared by the
// 64 cells); each lane reads its own cell's coefficients.
__global__ __launch_bounds__(256) void apply_fp64_kernel(Fp64Params p) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t ncb = (p.B + 63) / 64;
  const int64_t cb = blockIdx.x % ncb;
  const int n = (int)(blockIdx.x / ncb) * 4 + w;
  if (n >= p.N) return;
  const int64_t b = cb * 64 + lane;
  const bool active = b < p.B;
  const int NK = p.NK, NK2 = NK * NK;
  const int q1 = n / NK, k1 = n - (n / NK) * NK;
  const double* fb = p.f + (active ? b : 0) * p.ldf;
  double acc = 0.0;
  const int e1 = p.q1ptr[q1 + 1];
  for (int e = p.q1ptr[q1]; e < e1; ++e) {
    const uint32_t qq = p.ent_q[e];
    const double* f2 = fb + (int)(qq & 0xffffu) * NK;
    const double* f3 = fb + (int)(qq >> 16) * NK;
    const double* Rr = p.R + (int64_t)p.ent_c[e] * NK2 * NK + (int64_t)k1 * NK2;
    double s = 0.0;
    for (int k2 = 0; k2 < NK; ++k2) {
      double t = 0.0;
      for (int k3 = 0; k3 < NK; ++k3) t = fma(Rr[k2 * NK + k3], f3[k3], t);
      s = fma(f2[k2], t, s);
    }
    acc = fma(p.ent_g[e], s, acc);
  }
  if (active) p.Q[b * p.ldq + n] = acc;
}

hipError_t launch_apply_fp64(const wefq_core* h, const double* f, double* Q, int64_t B,
                             int64_t ldf, int64_t ldq, hipStream_t s) {
  if (B == 0) return hipSuccess;
  Fp64Params p;
  p.f = f; p.Q = Q; p.ldf = ldf; p.ldq = ldq;
  p.NK = h->NK; p.N = h->N; p.nchunk = (h->N + 3) / 4;
  p.R = h->dR64; p.q1ptr = h->d_q1ptr; p.ent_c = h->d_ent_c; p.ent_q = h->d_ent_q; p.ent_g = h->d_ent_g;
  // a launch holds at most 2^32 - 1 threads (grid x block): 256-thread blocks, nchunk per
  // 64 cells
  const int64_t maxcells = max_cells_per_launch(64, 256, p.nchunk);
  for (int64_t b0 = 0; b0 < B; b0 += maxcells) {
    const int64_t nb = B - b0 < maxcells ? B - b0 : maxcells;
    Fp64Params q = p;
    q.f = f + b0 * ldf; q.Q = Q + b0 * ldq; q.B = nb;
    const int64_t blocks = ((nb + 63) / 64) * p.nchunk;
    hipLaunchKernelGGL(apply_fp64_kernel, dim3((unsigned)blocks), dim3(256), 0, s, q);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// WAVES = 8, 12 or 16 waves per workgroup (launches of up to 512, 768 or 1,024 threads); 16 only
// for quadrants up to 5x5, whose registers fit the 128 per lane of four waves per SIMD.
template <int H, int SLOTS, int RT, int MODE, int WAVES>
__global__ __launch_bounds__(64 * WAVES) void apply_mfma_kernel(MfmaParams p) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  __shared__ int unit_ctr;
  mfma_tile<H, SLOTS, RT, MODE, false, false, WAVES>(p, (int64_t)blockIdx.x, (int)blockIdx.y, lds_raw, &unit_ctr);
}

// The instance for a block size: 8 waves up to 512 threads, 12 up to 768, 16 up to 1,024
// (null where it does not exist).
template <int H, int SLOTS, int RT, int MODE>
static const void* kernel_t(int block) {
  if (block <= 512) return (const void*)apply_mfma_kernel<H, SLOTS, RT, MODE, 8>;
  if (block <= 768) return (const void*)apply_mfma_kernel<H, SLOTS, RT, MODE, 12>;
  if constexpr (H <= 5) {
    if (block <= 1024) return (const void*)apply_mfma_kernel<H, SLOTS, RT, MODE, 16>;
  }
  return nullptr;
}

// One instance per (H, slots, RT, mode, waves), chosen at run time; the launch dispatch below
// and the attribute queries (spills, residency) see the same kernels.
template <int H, int RT, int MODE>
static const void* kernel_s(int slots, int block) {
  switch (slots) {
    case 1: return kernel_t<H, 1, RT, MODE>(block);
    case 2: return kernel_t<H, 2, RT, MODE>(block);
    case 4: return kernel_t<H, 4, RT, MODE>(block);
    default: return nullptr;
  }
}

template <int H>
static const void* kernel_h(int mode, int slots, int rt, int block) {
  if (rt == 2) {
    if constexpr (H >= 8) {
      switch (mode) {
        case 0: return kernel_s<H, 2, 0>(slots, block);
        case 1: return kernel_s<H, 2, 1>(slots, block);
        case 2: return kernel_s<H, 2, 2>(slots, block);
      }
    }
    return nullptr;
  }
  switch (mode) {
    case 0: return kernel_s<H, 1, 0>(slots, block);
    case 1: return kernel_s<H, 1, 1>(slots, block);
    case 2: return kernel_s<H, 1, 2>(slots, block);
  }
  return nullptr;
}

static const void* mfma_kernel(const wefq_core* h, int mode, int slots, int block) {
  switch (h->H) {
    case 1: return kernel_h<1>(mode, slots, h->RT, block);
    case 2: return kernel_h<2>(mode, slots, h->RT, block);
    case 3: return kernel_h<3>(mode, slots, h->RT, block);
    case 4: return kernel_h<4>(mode, slots, h->RT, block);
    case 5: return kernel_h<5>(mode, slots, h->RT, block);
    case 6: return kernel_h<6>(mode, slots, h->RT, block);
    case 7: return kernel_h<7>(mode, slots, h->RT, block);
    case 8: return kernel_h<8>(mode, slots, h->RT, block);
    case 9: return kernel_h<9>(mode, slots, h->RT, block);
    default: return nullptr;
  }
}

int mfma_spill_bytes(const wefq_core* h, int mode, int slots, int block) {
  const void* k = mfma_kernel(h, mode, slots, block);
  hipFuncAttributes a;
  if (!k || hipFuncGetAttributes(&a, k) != hipSuccess) return -1;
  return (int)a.localSizeBytes;
}

int mfma_blocks_per_cu(const wefq_core* h, int mode, int slots, int block) {
  const void* k = mfma_kernel(h, mode, slots, block);
  if (!k) return 0;
  const size_t lds = tile_lds_bytes(h, slots, mode == 2 ? 8 : 4);
  int n = 0;
  if (hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k, block, lds) != hipSuccess)
    return 0;
  return n;
}

hipError_t launch_apply_mfma(const wefq_core* h, int precision, const void* f, void* Q, int64_t B,
                             int64_t ldf, int64_t ldq, hipStream_t s) {
  if (B == 0) return hipSuccess;
  MfmaParams p;
  p.f = f; p.g = nullptr; p.Q = Q; p.B = B; p.ldf = ldf; p.ldg = 0; p.ldq = ldq;
  p.NK = h->NK; p.NQ = h->NQ; p.N = h->N;
  p.nunits = h->nunits; p.units = h->d_units; p.chan_begin = h->d_chan_begin;
  p.slice_off = h->d_slice_off; p.sptr = h->d_sptr; p.spair = h->d_spair; p.mq = h->d_mq; p.mq_pad = h->d_mq_pad;
  p.mg = h->d_mg; p.mg64 = h->d_mg64;
  p.Rt32 = h->d_Rt32; p.Rt64 = h->d_Rt64; p.Rhi = h->d_Rhi; p.Rlo = h->d_Rlo;
  p.R16_32 = h->d_R16_32; p.R16_64 = h->d_R16_64;
  const int mode = mfma_mode(precision);
  if (mode < 0) return hipErrorInvalidValue;
  const int slots = h->slots[mode], block = h->block[mode];
  if (slots == 0) return hipErrorInvalidValue;
  const int TB = 16 / slots;
  const int64_t ntiles = (B + TB - 1) / TB;
  p.nsplit = tile_splits(h, ntiles, p.nunits, h->split_per_cu[mode],
                         (int64_t)h->cu_count * h->resident_per_cu[mode]);
  if (use_units2(h, mode, slots, p.nsplit, block)) { p.units = h->d_units2; p.nunits = h->nunits2; }
  const size_t lds = tile_lds_bytes(h, slots, mode == 2 ? 8 : 4);
  // a launch holds at most 2^32 - 1 threads: larger batches run as several launches of whole
  // tiles (each cell's result does not depend on its batch)
  const int64_t max_cells = max_cells_per_launch(TB, block);
  if (B > max_cells) {
    for (int64_t c0 = 0; c0 < B; c0 += max_cells) {
      const int64_t nc = (B - c0) < max_cells ? (B - c0) : max_cells;
      const size_t esz = mode == 2 ? 8 : 4;
      const hipError_t e = launch_apply_mfma(h, precision, (const char*)f + c0 * ldf * esz,
                                             (char*)Q + c0 * ldq * esz, nc, ldf, ldq, s);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  const void* k = mfma_kernel(h, mode, slots, block);
  if (!k) return hipErrorInvalidValue;
  hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  void* args[] = {&p};
  return hipLaunchKernel(k, dim3((unsigned)ntiles, (unsigned)p.nsplit), dim3(block), args, lds, s);
}

// ---------------------------------------------------------------- conservation check
__global__ void check_kernel(const void* Q, int precision, int64_t B, int64_t ldq, int NK, int L,
                             double* out) {
  __shared__ double red[256];
  double m = 0.0;
  int rows[5] = {0, 1, NK, 2 * NK, 3 * NK};
  int nrows = 1 + (NK > 1 ? 1 : 0);
  if (L >= 1) { rows[nrows] = NK; rows[nrows + 1] = 2 * NK; rows[nrows + 2] = 3 * NK; nrows += 3; }
  for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < B; b += (int64_t)gridDim.x * blockDim.x) {
    for (int i = 0; i < nrows; ++i) {
      double v = (precision == WEFQ_FP64 || precision == WEFQ_FP64_NAIVE) ? ((const double*)Q)[b * ldq + rows[i]]
                                                                           : (double)((const float*)Q)[b * ldq + rows[i]];
      v = fabs(v);
      m = (v > m || v != v) ? v : m;
    }
  }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int st = blockDim.x / 2; st > 0; st >>= 1) {
    if (threadIdx.x < st) {
      double a = red[threadIdx.x], b2 = red[threadIdx.x + st];
      red[threadIdx.x] = (b2 > a || b2 != b2) ? b2 : a;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

hipError_t launch_check(const wefq_core* h, int precision, const void* Q, int64_t B, int64_t ldq,
                        hipStream_t s) {
  hipLaunchKernelGGL(check_kernel, dim3(h->check_blocks), dim3(256), 0, s, Q, precision, B, ldq,
                     h->NK, h->L, h->d_check);
  return hipGetLastError();
}

}  // namespace wefq
