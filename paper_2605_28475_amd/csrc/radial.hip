// The radial-first ordering of the factorized sum (Section 4.5.3), in FP64.
//
// Pass 1 contracts the radial core with the two gathered states for every distinct
// (channel, q2, q3) triple of the real-Gaunt table, into the dense intermediate
//   Psi^{k1}_{q2 q3 c} = sum_{k2, k3} R^{(c)}_{k1 k2 k3} f_{k2 q2} f_{k3 q3},
// sum-factorized as t_{k1 k2} = sum_k3 R_{k1 k2 k3} f_{k3 q3}, Psi^{k1} = sum_k2 t_{k1 k2} f_{k2 q2}.
// Pass 2 streams the table grouped by output state:
//   Q_{k1 q1} = sum_{z : q1z = q1} g_z Psi^{k1}_{q2z q3z c_z}.
// Psi lives in a caller-provided workspace in HBM, [group][k1][cell] with cells fastest, so
// a batch is processed in chunks of cells that fit the workspace; each chunk of f is first
// transposed into the workspace, [n][cell], so that both passes read coalesced.  Every
// wavefront of a pass works on one group (pass 1) or one output mode (pass 2) for 64 cells,
// so the core and the table entries are read through the scalar cache.  This is a reference
// ordering: its cost is the write and re-read of Psi (groups x NK doubles per cell) and one
// NK^3 contraction per group instead of one per (channel, q1) slice.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/wefq.h"
#include "wefq_core.h"
#include "apply_tile.h"

namespace wefq {

struct RadialParams {
  const double* f;
  double* Q;
  int64_t ldf, ldq;
  int64_t c0, nc;          // this chunk: cells [c0, c0 + nc)
  int NK, N, ngroups, Bp;  // Bp: chunk width padded to a multiple of 64
  const double* R;         // zeroed core [c][k1][k2][k3]
  const int* grp_c;        // [ngroups] channel of each group
  const uint32_t* grp_q;   // [ngroups] q2 | q3 << 16
  const int* q1ptr;        // [NQ + 1] table rows grouped by q1
  const int* row_grp;      // [N_G] group of each row
  const double* row_g;     // [N_G] real Gaunt weight of each row
  double* fT;              // workspace: [N][Bp]
  double* psi;             // workspace: [ngroups][NK][Bp]
};

typedef const __attribute__((address_space(4))) double cdbl;
typedef const __attribute__((address_space(4))) int cint;
typedef const __attribute__((address_space(4))) uint32_t cu32;

// fT[n][cell] = f[c0 + cell][n]; zero for the pad cells [nc, Bp).  32 x 32 tiles through LDS.
__global__ __launch_bounds__(256) void radial_transpose_kernel(RadialParams p) {
  __shared__ double tile[32][33];
  const int n0 = blockIdx.x * 32, b0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int r = ty; r < 32; r += 8) {
    const int cell = b0 + r, n = n0 + tx;
    double v = 0.0;
    if (cell < p.nc && n < p.N) v = p.f[(p.c0 + cell) * p.ldf + n];
    tile[r][tx] = v;
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int n = n0 + r, cell = b0 + tx;
    if (n < p.N && cell < p.Bp) p.fT[(int64_t)n * p.Bp + cell] = tile[tx][r];
  }
}

template <int NK>
__global__ __launch_bounds__(256) void radial_psi_kernel(RadialParams p) {
  const int64_t tid = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int wpg = p.Bp >> 6;
  const int64_t wave = tid >> 6;
  const int grp = __builtin_amdgcn_readfirstlane((int)(wave / wpg));
  if (grp >= p.ngroups) return;
  const int cell = (int)((wave % wpg) * 64 + (tid & 63));
  const int c = ((cint*)p.grp_c)[grp];
  const uint32_t qq = ((cu32*)p.grp_q)[grp];
  const int q2 = qq & 0xffff, q3 = qq >> 16;
  cdbl* R = (cdbl*)p.R + (int64_t)c * NK * NK * NK;
  double f2[NK], f3[NK];
#pragma unroll
  for (int k = 0; k < NK; ++k) {
    f2[k] = p.fT[(int64_t)(q2 * NK + k) * p.Bp + cell];
    f3[k] = p.fT[(int64_t)(q3 * NK + k) * p.Bp + cell];
  }
  double* out = p.psi + (int64_t)grp * NK * p.Bp + cell;
  for (int k1 = 0; k1 < NK; ++k1) {
    double acc = 0.0;
#pragma unroll
    for (int k2 = 0; k2 < NK; ++k2) {
      double t = 0.0;
#pragma unroll
      for (int k3 = 0; k3 < NK; ++k3) t += R[(k1 * NK + k2) * NK + k3] * f3[k3];
      acc += t * f2[k2];
    }
    __builtin_nontemporal_store(acc, out + (int64_t)k1 * p.Bp);   // streamed: read once, by pass 2
  }
}

__global__ __launch_bounds__(256) void radial_gather_kernel(RadialParams p) {
  const int64_t tid = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int wpg = p.Bp >> 6;
  const int64_t wave = tid >> 6;
  const int n = __builtin_amdgcn_readfirstlane((int)(wave / wpg));
  if (n >= p.N) return;
  const int cell = (int)((wave % wpg) * 64 + (tid & 63));
  const int q1 = n / p.NK, k1 = n % p.NK;
  // four independent partial sums keep four Psi loads in flight per lane
  const double* col = p.psi + (int64_t)k1 * p.Bp + cell;
  const int64_t gstride = (int64_t)p.NK * p.Bp;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  const int z1 = ((cint*)p.q1ptr)[q1 + 1];
  int z = ((cint*)p.q1ptr)[q1];
  for (; z + 3 < z1; z += 4) {
    a0 += ((cdbl*)p.row_g)[z] * col[((cint*)p.row_grp)[z] * gstride];
    a1 += ((cdbl*)p.row_g)[z + 1] * col[((cint*)p.row_grp)[z + 1] * gstride];
    a2 += ((cdbl*)p.row_g)[z + 2] * col[((cint*)p.row_grp)[z + 2] * gstride];
    a3 += ((cdbl*)p.row_g)[z + 3] * col[((cint*)p.row_grp)[z + 3] * gstride];
  }
  for (; z < z1; ++z) a0 += ((cdbl*)p.row_g)[z] * col[((cint*)p.row_grp)[z] * gstride];
  double acc = (a0 + a1) + (a2 + a3);
  if (cell < p.nc) p.Q[(p.c0 + cell) * p.ldq + n] = acc;
}

template <int NK>
static void launch_psi(const RadialParams& p, hipStream_t s) {
  const int64_t threads = (int64_t)p.ngroups * p.Bp;
  hipLaunchKernelGGL(radial_psi_kernel<NK>, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, p);
}

int64_t radial_bytes_per_cell(const wefq_core* h) { return ((int64_t)h->N + (int64_t)h->rad_groups * h->NK) * 8; }

hipError_t launch_apply_radial(const wefq_core* h, const double* f, double* Q, int64_t B, int64_t ldf, int64_t ldq,
                               void* work, int64_t chunk, hipStream_t s) {
  if (B == 0) return hipSuccess;
  RadialParams p;
  p.f = f; p.Q = Q; p.ldf = ldf; p.ldq = ldq;
  p.NK = h->NK; p.N = h->N; p.ngroups = h->rad_groups;
  p.Bp = (int)chunk;
  p.R = h->dR64; p.grp_c = h->d_rad_grp_c; p.grp_q = h->d_rad_grp_q;
  p.q1ptr = h->d_rad_q1ptr; p.row_grp = h->d_rad_row_grp; p.row_g = h->d_rad_row_g;
  p.fT = (double*)work;
  p.psi = p.fT + (int64_t)h->N * chunk;
  for (int64_t c0 = 0; c0 < B; c0 += chunk) {
    RadialParams q = p;
    q.c0 = c0;
    q.nc = B - c0 < chunk ? B - c0 : chunk;
    hipLaunchKernelGGL(radial_transpose_kernel, dim3((unsigned)((h->N + 31) / 32), (unsigned)(chunk / 32)), dim3(256),
                       0, s, q);
    switch (h->NK) {
      case 1: launch_psi<1>(q, s); break;
      case 2: launch_psi<2>(q, s); break;
      case 3: launch_psi<3>(q, s); break;
      case 4: launch_psi<4>(q, s); break;
      case 5: launch_psi<5>(q, s); break;
      case 6: launch_psi<6>(q, s); break;
      case 7: launch_psi<7>(q, s); break;
      case 8: launch_psi<8>(q, s); break;
      case 9: launch_psi<9>(q, s); break;
      case 10: launch_psi<10>(q, s); break;
      case 11: launch_psi<11>(q, s); break;
      case 12: launch_psi<12>(q, s); break;
      case 13: launch_psi<13>(q, s); break;
      case 14: launch_psi<14>(q, s); break;
      case 15: launch_psi<15>(q, s); break;
      case 16: launch_psi<16>(q, s); break;
      case 17: launch_psi<17>(q, s); break;
      default: return hipErrorInvalidValue;
    }
    const int64_t threads = (int64_t)h->N * chunk;
    hipLaunchKernelGGL(radial_gather_kernel, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, q);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace wefq
