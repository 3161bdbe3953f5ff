// Dense Cartesian contraction (Section 4.5.1, the paper's comparison baseline):
//   Q_a1 = sum_{a2, a3} C_{a1 a2 a3} f_a2 f_a3
// with the full weak-form tensor C of N^3 entries, assembled from the factorized form
// C_{(k1 q1)(k2 q2)(k3 q3)} = g_{q1 q2 q3} R^{(c)}_{k1 k2 k3} (eq. wigner-eckart-factorization,
// Section 4.1).  The contraction is one dense product per batch: the N x N^2 matrix C times
// the N^2 x cells matrix f (x) f, whose columns are generated on the fly from f in LDS, on
// the FP64 matrix cores.  It exists to measure the dense ordering against the factorized
// ones on the same chip, not as a product path.
//
// Layout of C in device memory (caller-owned, wefq_dense_bytes):
//   rows a1 in tiles of 16 (NA = 16 ceil(N/16) rows, the padding rows zero);
//   the inner index kappa = a2 * N4 + a3 with a3 padded to N4 = 4 ceil(N/4) (zeros);
//   element (a1, kappa) at ((a1/16) * KC + kappa/4) * 64 + (a1 % 16) + 16 (kappa % 4),
//   KC = N N4 / 4: one v_mfma_f64_16x16x4 A operand is 64 consecutive doubles, one per lane.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "../../include/wefq.h"
#include "wefq_core.h"

namespace wefq {

typedef double v4d_t __attribute__((ext_vector_type(4)));

struct DenseShape {
  int64_t N, NA, N4, KC;
};

static DenseShape dense_shape(const wefq_core* h) {
  DenseShape d;
  d.N = h->N;
  d.NA = (d.N + 15) / 16 * 16;
  d.N4 = (d.N + 3) / 4 * 4;
  d.KC = d.N * d.N4 / 4;
  return d;
}

int64_t dense_bytes(const wefq_core* h) {
  const DenseShape d = dense_shape(h);
  return d.NA * d.N * d.N4 * 8;
}

__global__ __launch_bounds__(256) void dense_zero_kernel(double2* C, int64_t n2) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n2; i += (int64_t)gridDim.x * blockDim.x)
    C[i] = make_double2(0.0, 0.0);
}

struct AssembleParams {
  double* C;
  const double* R;          // [N_T][NK][NK][NK], zeroed
  const int* q1ptr;         // COO rows grouped by q1
  const int* ent_c;
  const uint32_t* ent_q;    // q2 | q3 << 16
  const double* ent_g;
  int NK;
  int64_t KC, N4;
};

// Block (q1, y) writes the entries of the COO rows of q1: every (q1, q2, q3) occurs once in
// the table, so every entry of C is written by at most one thread.
__global__ __launch_bounds__(256) void dense_assemble_kernel(AssembleParams p) {
  const int q1 = blockIdx.x;
  const int NK = p.NK, NK3 = NK * NK * NK;
  const int e0 = p.q1ptr[q1], e1 = p.q1ptr[q1 + 1];
  const int64_t total = (int64_t)(e1 - e0) * NK3;
  for (int64_t t = (int64_t)blockIdx.y * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.y * blockDim.x) {
    const int e = e0 + (int)(t / NK3);
    const int r = (int)(t - (int64_t)(e - e0) * NK3);
    const int k1 = r / (NK * NK), k2 = (r / NK) % NK, k3 = r % NK;
    const uint32_t qq = p.ent_q[e];
    const int64_t a1 = (int64_t)q1 * NK + k1;
    const int64_t a2 = (int64_t)(qq & 0xffffu) * NK + k2;
    const int64_t a3 = (int64_t)(qq >> 16) * NK + k3;
    const int64_t kappa = a2 * p.N4 + a3;
    const int64_t idx = ((a1 >> 4) * p.KC + (kappa >> 2)) * 64 + (a1 & 15) + 16 * (kappa & 3);
    p.C[idx] = p.ent_g[e] * p.R[(int64_t)p.ent_c[e] * NK3 + r];
  }
}

struct DenseParams {
  const double* C;
  const double* f;
  double* Q;
  int64_t B, ldf, ldq;
  int64_t N, N4, KC;
  int a1_tiles;             // NA / 16
  int waves;                // a1 tiles per workgroup (one per wave)
  int groups;               // ceil(a1_tiles / waves)
  int cell_tiles;           // ceil(B / 16)
};

// One workgroup: a tile of 16 cells (f transposed into LDS, fT[a][cell], zero beyond N and B)
// and `waves` tiles of 16 output rows a1, one per wave.  A wave walks kappa in steps of 4:
// the A operand is 64 consecutive doubles of C, the B operand f_a2 f_a3 for its cell (column
// lane % 16) and a3 = 4 (kappa/4 mod N4/4) + lane/16.  Workgroups are ordered so that the
// ones a chiplet (XCD, blocks b = x mod 8) runs at the same time share their rows of C and
// differ in cells, which lets its L2 serve C to several of them.
__global__ __launch_bounds__(1024) void dense_contract_kernel(DenseParams p) {
  extern __shared__ __align__(16) double fT[];
  const int64_t total = (int64_t)p.groups * p.cell_tiles;
  const int64_t b = blockIdx.x, x = b & 7, i = b >> 3;
  int64_t start = 0;
  for (int y = 0; y < x; ++y) start += (total - y + 7) / 8;
  const int64_t item = start + i;
  if (i >= (total - x + 7) / 8 || item >= total) return;      // uniform over the workgroup
  const int group = (int)(item / p.cell_tiles);
  const int64_t ct = item - (int64_t)group * p.cell_tiles;
  const int64_t cell0 = ct * 16;
  for (int64_t t = threadIdx.x; t < p.N4 * 16; t += blockDim.x) {
    const int64_t a = t >> 4, c = t & 15, cell = cell0 + c;
    fT[t] = (a < p.N && cell < p.B) ? p.f[cell * p.ldf + a] : 0.0;
  }
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int t1 = group * p.waves + wave;
  if (t1 >= p.a1_tiles) return;
  const int j = lane & 15, kk = lane >> 4;
  const double* A = p.C + (int64_t)t1 * p.KC * 64 + lane;
  const int64_t nc3 = p.N4 / 4;
  v4d_t acc = {0.0, 0.0, 0.0, 0.0};
  for (int64_t a2 = 0; a2 < p.N; ++a2) {
    const double fa2 = fT[a2 * 16 + j];
    const double* Aa = A + a2 * nc3 * 64;
    const double* fb = fT + kk * 16 + j;
    int64_t c = 0;
    for (; c + 4 <= nc3; c += 4) {
      double av[4], bv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        av[u] = Aa[(c + u) * 64];
        bv[u] = fa2 * fb[(c + u) * 64];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], bv[u], acc, 0, 0, 0);
    }
    for (; c < nc3; ++c) {
      const double av = Aa[c * 64];
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, fa2 * fb[c * 64], acc, 0, 0, 0);
    }
  }
  // output register i holds row lane/16 + 4 i of the tile, column lane % 16
  const int64_t cell = cell0 + j;
  if (cell < p.B) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t a1 = (int64_t)t1 * 16 + kk + 4 * r;
      if (a1 < p.N) p.Q[cell * p.ldq + a1] = acc[r];
    }
  }
}

hipError_t launch_dense_assemble(const wefq_core* h, double* C, hipStream_t s) {
  const DenseShape d = dense_shape(h);
  const int64_t n2 = dense_bytes(h) / 16;
  hipLaunchKernelGGL(dense_zero_kernel, dim3(4096), dim3(256), 0, s, reinterpret_cast<double2*>(C), n2);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  AssembleParams p;
  p.C = C; p.R = h->dR64; p.q1ptr = h->d_q1ptr; p.ent_c = h->d_ent_c; p.ent_q = h->d_ent_q; p.ent_g = h->d_ent_g;
  p.NK = h->NK; p.KC = d.KC; p.N4 = d.N4;
  hipLaunchKernelGGL(dense_assemble_kernel, dim3((unsigned)h->NQ, 64), dim3(256), 0, s, p);
  return hipGetLastError();
}

// Dynamic LDS of the contraction kernel: the transposed f tile.
size_t dense_lds_bytes(const wefq_core* h) { return (size_t)dense_shape(h).N4 * 16 * 8; }

hipError_t launch_dense_contract(const wefq_core* h, const double* C, const double* f, double* Q, int64_t B,
                                 int64_t ldf, int64_t ldq, hipStream_t s) {
  if (B == 0) return hipSuccess;
  const DenseShape d = dense_shape(h);
  DenseParams p;
  p.C = C; p.f = f; p.Q = Q; p.ldf = ldf; p.ldq = ldq;
  p.N = d.N; p.N4 = d.N4; p.KC = d.KC;
  p.a1_tiles = (int)(d.NA / 16);
  // at most 16 waves per workgroup, spread evenly over the groups of row tiles
  p.groups = (p.a1_tiles + 15) / 16;
  p.waves = (p.a1_tiles + p.groups - 1) / p.groups;
  const size_t lds = dense_lds_bytes(h);
  hipError_t e = hipFuncSetAttribute((const void*)dense_contract_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return e;
  // at most 2^31 - 1 workgroups per launch: larger batches run as several launches
  const int64_t max_tiles = 0x7fffffffLL / p.groups;
  for (int64_t c0 = 0; c0 < B; c0 += max_tiles * 16) {
    DenseParams q = p;
    q.B = B - c0 < max_tiles * 16 ? B - c0 : max_tiles * 16;
    q.f = f + c0 * ldf;
    q.Q = Q + c0 * ldq;
    q.cell_tiles = (int)((q.B + 15) / 16);
    const int64_t blocks = (int64_t)q.groups * q.cell_tiles;
    hipLaunchKernelGGL(dense_contract_kernel, dim3((unsigned)blocks), dim3(64 * q.waves), lds, s, q);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace wefq

using namespace wefq;

static wefq_status dense_fail(wefq_status st, const std::string& msg) {
  set_error(msg);
  return st;
}

static wefq_status dense_ready(wefq_handle h) {
  if (!h) return dense_fail(WEFQ_EINVAL, "null handle");
  if (!(h->precisions & WEFQ_FP64) || !h->dR64 || !h->d_q1ptr)
    return dense_fail(WEFQ_EINVAL, "the dense contraction needs a core built with WEFQ_FP64");
  if (dense_lds_bytes(h) > (size_t)h->lds_limit)
    return dense_fail(WEFQ_EUNSUPPORTED, "N too large for the dense contraction's LDS tile of f (N <= 1280)");
  return WEFQ_OK;
}

extern "C" {

wefq_status wefq_dense_bytes(wefq_handle h, int64_t* bytes) {
  if (!bytes) return dense_fail(WEFQ_EINVAL, "null output pointer");
  const wefq_status st = dense_ready(h);
  if (st != WEFQ_OK) return st;
  *bytes = dense_bytes(h);
  return WEFQ_OK;
}

wefq_status wefq_dense_assemble(wefq_handle h, void* C, int64_t C_bytes, void* stream) {
  const wefq_status st = dense_ready(h);
  if (st != WEFQ_OK) return st;
  if (!C || ((uintptr_t)C & 255)) return dense_fail(WEFQ_EINVAL, "C must be non-null and 256-byte aligned");
  if (C_bytes < dense_bytes(h)) return dense_fail(WEFQ_EINVAL, "C smaller than wefq_dense_bytes reports");
  if (hipSetDevice(h->device) != hipSuccess) return dense_fail(WEFQ_EHIP, "hipSetDevice failed");
  const hipError_t e = launch_dense_assemble(h, static_cast<double*>(C), (hipStream_t)stream);
  if (e != hipSuccess) return dense_fail(WEFQ_EHIP, std::string("dense assembly failed: ") + hipGetErrorString(e));
  return WEFQ_OK;
}

wefq_status wefq_apply_Q_dense(wefq_handle h, const void* C, int64_t C_bytes, const double* f, double* Q, int64_t B,
                               int64_t ld_f, int64_t ld_q, void* stream) {
  const wefq_status st = dense_ready(h);
  if (st != WEFQ_OK) return st;
  if (B < 0) return dense_fail(WEFQ_EINVAL, "negative batch size");
  if (B == 0) return WEFQ_OK;
  if (!C || ((uintptr_t)C & 255)) return dense_fail(WEFQ_EINVAL, "C must be non-null and 256-byte aligned");
  if (C_bytes < dense_bytes(h)) return dense_fail(WEFQ_EINVAL, "C smaller than wefq_dense_bytes reports");
  if (!f || !Q) return dense_fail(WEFQ_EINVAL, "null input or output pointer");
  if (ld_f < h->N || ld_q < h->N) return dense_fail(WEFQ_EINVAL, "leading dimension smaller than N");
  if (((uintptr_t)f | (uintptr_t)Q) & 7) return dense_fail(WEFQ_EINVAL, "f and Q must be aligned to 8 bytes");
  const char* fb = (const char*)f; const char* qb = (const char*)Q; const char* cb = (const char*)C;
  const size_t fn = (size_t)B * ld_f * 8, qn = (size_t)B * ld_q * 8, cn = (size_t)dense_bytes(h);
  if ((fb < qb + qn && qb < fb + fn) || (cb < qb + qn && qb < cb + cn))
    return dense_fail(WEFQ_EINVAL, "Q must not overlap f or C");
  if (hipSetDevice(h->device) != hipSuccess) return dense_fail(WEFQ_EHIP, "hipSetDevice failed");
  const hipError_t e = launch_dense_contract(h, static_cast<const double*>(C), f, Q, B, ld_f, ld_q,
                                             (hipStream_t)stream);
  if (e != hipSuccess) return dense_fail(WEFQ_EHIP, std::string("dense contraction failed: ") + hipGetErrorString(e));
  return WEFQ_OK;
}

}  // extern "C"
