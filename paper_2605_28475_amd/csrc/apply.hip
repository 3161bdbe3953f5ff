// Contraction kernels for Q(f, f) (Section 4.5) and the FP64 conservation check.
//
// apply_fp64_kernel   the plain FP64 comparator: the paper's naive contraction
//                     (eq. full_discrete_sum as written), one thread per output
//                     (cell, q1, k1), looping over the COO rows of q1 and k2, k3;
//                     no channel merging, no tiling, no matrix cores.
// apply_mfma_kernel   angular-first contraction (Section 4.5.4) re-laid for CDNA4:
//   * a workgroup owns a tile of 16 cells (8 when f does not fit in LDS; then
//     the 16 MFMA columns are 8 cells x 2 output states) and stages their
//     coefficients in LDS as fs[n][cell];
//   * the COO rows (q1,q2,q3) and (q1,q3,q2) are merged (exact for Q(f,f)), so
//     channel (l1,l2,l3) with l2 < l3 carries R^{(l1l2l3)}_{k1k2k3} + R^{(l1l3l2)}_{k1k3k2};
//   * per slice (channel, q1) the intermediate Phi^{(c,q1)}_{k2k3} =
//     sum_z g_z f_{k2,q2z} f_{k3,q3z} (angular coupling, FP32 VALU) is built by
//     wave-uniform integer-indexed gathers from LDS straight into the MFMA
//     B-operand layout: lane group r = lane/16 owns the (k2,k3) quadrant
//     (r/2, r%2) of the NK x NK grid, lane%16 is the MFMA column (cell);
//   * the radial contraction Q_{k1,q1} += sum R^{(c)}_{k1,(k2k3)} Phi_{(k2k3)}
//     runs on v_mfma_f32_16x16x4_f32 (FP32) or as three split hi/lo BF16
//     v_mfma_f32_16x16x32_bf16 products with FP32 accumulation (BF16X3);
//   * the wave keeps the 16x16 accumulator tiles of a group of q1 values of
//     one l1 across all channels of that l1 (the channel reduction), so every
//     output is produced by one wave in a fixed order: results are bitwise
//     independent of the other cells in the batch;
//   * waves pull (l1, q1-group) work units from an LDS counter, largest first.
// The mass, momentum and energy rows are stored as exact zeros (Section 4.4).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/wefq.h"
#include "wefq_core.h"

namespace wefq {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

__device__ inline bool invariant_row(int q1, int k1) {
  return (q1 == 0 && k1 <= 1) || (q1 >= 1 && q1 <= 3 && k1 == 0);
}

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
  if (active) p.Q[b * p.ldq + n] = invariant_row(q1, k1) ? 0.0 : acc;
}

hipError_t launch_apply_fp64(const wefq_core* h, const double* f, double* Q, int64_t B,
                             int64_t ldf, int64_t ldq, hipStream_t s) {
  if (B == 0) return hipSuccess;
  Fp64Params p;
  p.f = f; p.Q = Q; p.ldf = ldf; p.ldq = ldq;
  p.NK = h->NK; p.N = h->N; p.nchunk = (h->N + 3) / 4;
  p.R = h->dR64; p.q1ptr = h->d_q1ptr; p.ent_c = h->d_ent_c; p.ent_q = h->d_ent_q; p.ent_g = h->d_ent_g;
  const int64_t maxcells = (int64_t)64 * (0x7fffffff / p.nchunk);
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

struct MfmaParams {
  const void* f;
  void* Q;
  int64_t B, ldf, ldq;
  int NK, NQ, N;
  int nunits;
  const int* units;        // [nunits][3]
  const int* chan_begin;   // [L+2]
  const int* slice_off;    // [NTm]
  const int* sptr;         // slices + 1
  const uint32_t* mq;      // q2*NK | (q3*NK) << 16 (row offsets of the two gathered states)
  const float* mg;         // merged weights (FP32 / BF16X3)
  const double* mg64;      // merged weights (FP64)
  const float* Rt32;       // [NTm][RT][H*H][64]
  const double* Rt64;      // [NTm][RT][H*H][64]
  const uint16_t* Rhi;     // [NTm][RT][U][64][8]
  const uint16_t* Rlo;
};

// output states per work unit (fewer when NK > 16 needs two accumulator row tiles)
__host__ __device__ constexpr int gq_for(int H) { return H >= 8 ? 4 : 8; }
typedef double v4d __attribute__((ext_vector_type(4)));

// MODE 0: FP32 MFMA, 1: split BF16x3 MFMA, 2: FP64 MFMA.
template <int MODE> struct ModeTraits;
template <> struct ModeTraits<0> { typedef float T; typedef v4f acc_t; };
template <> struct ModeTraits<1> { typedef float T; typedef v4f acc_t; };
template <> struct ModeTraits<2> { typedef double T; typedef v4d acc_t; };

template <int H, int SLOTS, int RT, int MODE>
__global__ __launch_bounds__(512) void apply_mfma_kernel(MfmaParams p) {
  typedef typename ModeTraits<MODE>::T T;
  typedef typename ModeTraits<MODE>::acc_t acc_t;
  constexpr int TB = 16 / SLOTS;
  constexpr int HH = H * H;
  constexpr int U = (HH + 7) / 8;
  constexpr int GQ = gq_for(H);
  constexpr int NP = GQ / SLOTS > 0 ? GQ / SLOTS : 1;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  T* fs = reinterpret_cast<T*>(lds_raw);
  __shared__ int unit_ctr;
  const T* f = static_cast<const T*>(p.f);
  T* Qo = static_cast<T*>(p.Q);
  const int NK = p.NK;
  const int64_t cell0 = (int64_t)blockIdx.x * TB;
  // stage the coefficient tile: fs[n * TB + cell]
  for (int idx = threadIdx.x; idx < TB * p.N; idx += blockDim.x) {
    const int cl = idx / p.N, n = idx - cl * p.N;
    const int64_t cell = cell0 + cl;
    fs[n * TB + cl] = (cell < p.B) ? f[cell * p.ldf + n] : T(0);
  }
  if (threadIdx.x == 0) unit_ctr = 0;
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int r = lane >> 4, j = lane & 15;
  const int h2 = r >> 1, h3 = r & 1;
  const int cellj = j % TB, slot = j / TB;
  // lane group r covers k2 in [k2s, k2s+H) and k3 in [k3s, k3s+H): the lower half
  // starts at 0, the upper at NK-H (for odd NK the middle row is in both halves;
  // the R tile holds zero for the copy in the upper half), so every gather is a
  // per-lane base plus a compile-time offset.
  const int k2s = h2 ? NK - H : 0, k3s = h3 ? NK - H : 0;
  const T* lane_u = fs + k2s * TB + cellj;
  const T* lane_w = fs + k3s * TB + cellj;
  // read-only routing rows: through the constant address space so that
  // wave-uniform rows are fetched with scalar loads
  typedef const __attribute__((address_space(4))) uint32_t cu32;
  typedef const __attribute__((address_space(4))) float cf32;
  typedef const __attribute__((address_space(4))) double cf64;
  cu32* mq = (cu32*)p.mq;
  cf32* mg = (cf32*)p.mg;
  cf64* mg64 = (cf64*)p.mg64;
  while (true) {
    int u = 0;
    if (lane == 0) u = atomicAdd(&unit_ctr, 1);
    u = __shfl(u, 0);
    if (u >= p.nunits) break;
    const int l1 = p.units[3 * u], qb = p.units[3 * u + 1], nq = p.units[3 * u + 2];
    acc_t acc[NP][RT];
#pragma unroll
    for (int gi = 0; gi < NP; ++gi)
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) acc[gi][rt] = (acc_t){0, 0, 0, 0};
    const int cb = p.chan_begin[l1], ce = p.chan_begin[l1 + 1];
    for (int ct = cb; ct < ce; ++ct) {
      const int soff = p.slice_off[ct] - l1 * l1;
#pragma unroll
      for (int gi = 0; gi < NP; ++gi) {
        if (gi * SLOTS >= nq) break;
        const int qi = gi * SLOTS + slot;
        const bool qvalid = qi < nq;
        const int s = soff + qb + (qvalid ? qi : 0);
        int e0 = p.sptr[s], e1 = p.sptr[s + 1];
        if (!qvalid) e1 = e0;
        T phi[U * 8];
#pragma unroll
        for (int t = 0; t < U * 8; ++t) phi[t] = T(0);
        if (SLOTS == 1) {               // the slice is shared by the whole wave
          e0 = __builtin_amdgcn_readfirstlane(e0);
          e1 = __builtin_amdgcn_readfirstlane(e1);
          if (e0 < e1) {
            uint32_t qq = mq[e0];
            T gg = MODE == 2 ? (T)mg64[e0] : (T)mg[e0];
            for (int e = e0; e < e1; ++e) {
              // prefetch the next row (the arrays carry tail slack)
              const uint32_t qn = mq[e + 1];
              const T gn = MODE == 2 ? (T)mg64[e + 1] : (T)mg[e + 1];
              const T* pu = lane_u + (int)(qq & 0xffffu) * TB;
              const T* pw = lane_w + (int)(qq >> 16) * TB;
              T uu[H], ww[H];
#pragma unroll
              for (int a = 0; a < H; ++a) { uu[a] = gg * pu[a * TB]; ww[a] = pw[a * TB]; }
#pragma unroll
              for (int a = 0; a < H; ++a)
#pragma unroll
                for (int b = 0; b < H; ++b) phi[a * H + b] = fma(uu[a], ww[b], phi[a * H + b]);
              qq = qn; gg = gn;
            }
          }
        } else {
          const int len = e1 - e0;
          int maxlen = len;
#pragma unroll
          for (int off = TB; off < 16; off <<= 1) {
            const int o = __shfl_xor(maxlen, off);
            maxlen = maxlen > o ? maxlen : o;
          }
          for (int i = 0; i < maxlen; ++i) {
            const bool in = i < len;
            const int e = in ? e0 + i : e0;
            const uint32_t qq = in ? mq[e] : 0u;
            const T gg = in ? (MODE == 2 ? (T)mg64[e] : (T)mg[e]) : T(0);
            const T* pu = lane_u + (int)(qq & 0xffffu) * TB;
            const T* pw = lane_w + (int)(qq >> 16) * TB;
            T uu[H], ww[H];
#pragma unroll
            for (int a = 0; a < H; ++a) { uu[a] = gg * pu[a * TB]; ww[a] = pw[a * TB]; }
#pragma unroll
            for (int a = 0; a < H; ++a)
#pragma unroll
              for (int b = 0; b < H; ++b) phi[a * H + b] = fma(uu[a], ww[b], phi[a * H + b]);
          }
        }
        if constexpr (MODE == 0) {
#pragma unroll
          for (int rt = 0; rt < RT; ++rt) {
            const float* At = p.Rt32 + ((int64_t)(ct * RT + rt) * HH) * 64 + lane;
#pragma unroll
            for (int t0 = 0; t0 < HH; t0 += 8) {
              float av[8];
#pragma unroll
              for (int t = 0; t < 8; ++t) av[t] = (t0 + t < HH) ? At[(t0 + t) * 64] : 0.0f;
              __builtin_amdgcn_sched_barrier(0);
#pragma unroll
              for (int t = 0; t < 8; ++t)
                if (t0 + t < HH)
                  acc[gi][rt] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[t], phi[t0 + t], acc[gi][rt], 0, 0, 0);
            }
          }
        } else if constexpr (MODE == 2) {
#pragma unroll
          for (int rt = 0; rt < RT; ++rt) {
            const double* At = p.Rt64 + ((int64_t)(ct * RT + rt) * HH) * 64 + lane;
#pragma unroll
            for (int t0 = 0; t0 < HH; t0 += 8) {
              double av[8];
#pragma unroll
              for (int t = 0; t < 8; ++t) av[t] = (t0 + t < HH) ? At[(t0 + t) * 64] : 0.0;
              __builtin_amdgcn_sched_barrier(0);
#pragma unroll
              for (int t = 0; t < 8; ++t)
                if (t0 + t < HH)
                  acc[gi][rt] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[t], phi[t0 + t], acc[gi][rt], 0, 0, 0);
            }
          }
        } else {
#pragma unroll
          for (int uu8 = 0; uu8 < U; ++uu8) {
            v8bf bh, bl;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
              const float x = phi[uu8 * 8 + e];
              const __bf16 xh = (__bf16)x;
              bh[e] = xh;
              bl[e] = (__bf16)(x - (float)xh);
            }
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) {
              const int64_t off = (((int64_t)(ct * RT + rt) * U + uu8) * 64 + lane) * 8;
              const v8bf ah = *reinterpret_cast<const v8bf*>(p.Rhi + off);
              const v8bf al = *reinterpret_cast<const v8bf*>(p.Rlo + off);
              acc[gi][rt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc[gi][rt], 0, 0, 0);
              acc[gi][rt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc[gi][rt], 0, 0, 0);
              acc[gi][rt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc[gi][rt], 0, 0, 0);
            }
          }
        }
      }
    }
    // write the accumulator tiles: column lane%16; output register i holds row
    // 4*(lane/16)+i for the FP32 and BF16 forms and row lane/16+4*i for the FP64 form
    const int64_t cell = cell0 + cellj;
#pragma unroll
    for (int gi = 0; gi < NP; ++gi) {
      const int qi = gi * SLOTS + slot;
      if (qi >= nq || cell >= p.B) continue;
      const int q1 = qb + qi;
      T* dst = Qo + cell * p.ldq + (int64_t)q1 * NK;
#pragma unroll
      for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int k1 = rt * 16 + (MODE == 2 ? r + 4 * i : 4 * r + i);
          if (k1 < NK) dst[k1] = invariant_row(q1, k1) ? T(0) : (T)acc[gi][rt][i];
        }
    }
  }
}

template <int H, int SLOTS, int RT, int MODE>
static hipError_t launch_mfma_t(const MfmaParams& p, int64_t ntiles, int block, size_t lds, hipStream_t s) {
  auto k = apply_mfma_kernel<H, SLOTS, RT, MODE>;
  hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k, dim3((unsigned)ntiles), dim3(block), lds, s, p);
  return hipGetLastError();
}

template <int H, int RT, int MODE>
static hipError_t launch_mfma_s(const MfmaParams& p, int slots, int64_t ntiles, int block, size_t lds,
                                hipStream_t s) {
  switch (slots) {
    case 1: return launch_mfma_t<H, 1, RT, MODE>(p, ntiles, block, lds, s);
    case 2: return launch_mfma_t<H, 2, RT, MODE>(p, ntiles, block, lds, s);
    case 4: return launch_mfma_t<H, 4, RT, MODE>(p, ntiles, block, lds, s);
    default: return hipErrorInvalidValue;
  }
}

template <int H>
static hipError_t launch_mfma_h(const MfmaParams& p, int mode, int slots, int rt, int64_t ntiles, int block,
                                size_t lds, hipStream_t s) {
  if (rt == 2) {
    if constexpr (H >= 8) {
      switch (mode) {
        case 0: return launch_mfma_s<H, 2, 0>(p, slots, ntiles, block, lds, s);
        case 1: return launch_mfma_s<H, 2, 1>(p, slots, ntiles, block, lds, s);
        case 2: return launch_mfma_s<H, 2, 2>(p, slots, ntiles, block, lds, s);
      }
    }
    return hipErrorInvalidValue;
  }
  switch (mode) {
    case 0: return launch_mfma_s<H, 1, 0>(p, slots, ntiles, block, lds, s);
    case 1: return launch_mfma_s<H, 1, 1>(p, slots, ntiles, block, lds, s);
    case 2: return launch_mfma_s<H, 1, 2>(p, slots, ntiles, block, lds, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_apply_mfma(const wefq_core* h, int precision, const void* f, void* Q, int64_t B,
                             int64_t ldf, int64_t ldq, hipStream_t s) {
  if (B == 0) return hipSuccess;
  MfmaParams p;
  p.f = f; p.Q = Q; p.B = B; p.ldf = ldf; p.ldq = ldq;
  p.NK = h->NK; p.NQ = h->NQ; p.N = h->N;
  p.nunits = h->nunits; p.units = h->d_units; p.chan_begin = h->d_chan_begin;
  p.slice_off = h->d_slice_off; p.sptr = h->d_sptr; p.mq = h->d_mq; p.mg = h->d_mg; p.mg64 = h->d_mg64;
  p.Rt32 = h->d_Rt32; p.Rt64 = h->d_Rt64; p.Rhi = h->d_Rhi; p.Rlo = h->d_Rlo;
  const int mode = precision == WEFQ_FP64 ? 2 : (precision == WEFQ_BF16X3 ? 1 : 0);
  const int slots = mode == 2 ? h->SLOTS64 : h->SLOTS;
  if (slots == 0) return hipErrorInvalidValue;
  const int TB = 16 / slots;
  const int64_t ntiles = (B + TB - 1) / TB;
  const size_t lds = (size_t)h->N * TB * (mode == 2 ? 8 : 4);
  switch (h->H) {
    case 1: return launch_mfma_h<1>(p, mode, slots, h->RT, ntiles, h->block, lds, s);
    case 2: return launch_mfma_h<2>(p, mode, slots, h->RT, ntiles, h->block, lds, s);
    case 3: return launch_mfma_h<3>(p, mode, slots, h->RT, ntiles, h->block, lds, s);
    case 4: return launch_mfma_h<4>(p, mode, slots, h->RT, ntiles, h->block, lds, s);
    case 5: return launch_mfma_h<5>(p, mode, slots, h->RT, ntiles, h->block, lds, s);
    case 6: return launch_mfma_h<6>(p, mode, slots, h->RT, ntiles, h->block, lds, s);
    case 7: return launch_mfma_h<7>(p, mode, slots, h->RT, ntiles, h->block, lds, s);
    case 8: return launch_mfma_h<8>(p, mode, slots, h->RT, ntiles, h->block, lds, s);
    case 9: return launch_mfma_h<9>(p, mode, slots, h->RT, ntiles, h->block, lds, s);
    default: return hipErrorInvalidValue;
  }
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
      double v = (precision == 1 || precision == 8) ? ((const double*)Q)[b * ldq + rows[i]]
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
