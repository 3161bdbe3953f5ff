// Internal representation of a built core (the opaque wefq_handle).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdlib>
#include <string>
#include <vector>

#include "../../include/wefq.h"
#include "wefq_host.h"

struct wefq_core {
  int device = 0;
  int model = 0;
  int K = 0, L = 0, NK = 0, NQ = 0, N = 0;
  int NT = 0, NG = 0, NS = 0;          // paper counts
  int NTm = 0, NGm = 0, NSm = 0;       // merged counts
  double gamma = 0.0, b0 = 0.0;
  std::vector<double> beta;            // Legendre coefficients of the angular factor; empty: isotropic
  unsigned precisions = 0;
  int64_t quad_nodes = 0;
  int rad_pad = 0, ang_pad = 0;        // extra Gauss nodes beyond the exact counts (self-convergence)
  int64_t device_bytes = 0;
  std::vector<wefq::Channel> chans;
  std::vector<double> R64;             // host copy, zeroed, [c][k1][k2][k3]
  std::vector<double> R64raw;          // before the invariant-row zeroing (bilinear tables, serialization)

  // FP64 plain path: COO rows grouped by q1 (CSR), paper channel ids
  // radial-first ordering (reference path): distinct (channel, q2, q3) groups of the table
  int rad_groups = 0;
  int* d_rad_grp_c = nullptr;          // [rad_groups]
  uint32_t* d_rad_grp_q = nullptr;     // [rad_groups] q2 | q3 << 16
  int* d_rad_q1ptr = nullptr;          // [NQ + 1]
  int* d_rad_row_grp = nullptr;        // [N_G], rows grouped by q1
  double* d_rad_row_g = nullptr;       // [N_G]

  double* dR64 = nullptr;
  int* d_q1ptr = nullptr;              // NQ + 1
  int* d_ent_c = nullptr;              // N_G
  uint32_t* d_ent_q = nullptr;         // q2 | q3 << 16
  double* d_ent_g = nullptr;

  // MFMA path (merged channels sorted by l1)
  int H = 0, RT = 0;                   // quadrant size; RT == 2 marks NK = 17 (row 16 on the VALU)
  int slots[3] = {0, 0, 0};            // tile shape per mode (0 FP32, 1 BF16X3, 2 FP64): the cell
  int block[3] = {512, 512, 512};      // tile is 16/slots cells; block = threads per workgroup
  int split_per_cu[3] = {1, 1, 1};     // split workgroups per compute unit for small batches
  int resident_per_cu[3] = {1, 1, 1};  // workgroups of the mode's kernel resident per compute unit
  int* d_chan_begin = nullptr;         // L + 2: merged channels of l1 are [begin[l1], begin[l1+1])
  int* d_slice_off = nullptr;          // NTm: first slice of the merged channel
  int* d_sptr = nullptr;               // NSm(all (c,m1)) + 1
  int* d_spair = nullptr;              // per slice: first single row (rows before it come in q2 pairs)
  uint32_t* d_mq = nullptr;            // merged entries, two words each: q2*NK, q3*NK
  uint32_t* d_mq_pad = nullptr;        // the same with the padded pitch NK+1 (tiles with pad rows)
  float* d_mg = nullptr;               // merged weights
  double* d_mg64 = nullptr;            // merged weights, FP64
  float* d_Rt32 = nullptr;             // [NTm][ceil(H*H/4)][64][4]  (rows k1 < 16)
  double* d_Rt64 = nullptr;            // [NTm][ceil(H*H/2)][64][2]
  float* d_R16_32 = nullptr;           // NK = 17: row k1 = 16, [NTm][4][4 ceil(H*H/4)]
  double* d_R16_64 = nullptr;
  float* d_Dt32 = nullptr;             // antisymmetric partner tiles (bilinear form), layout of d_Rt32
  double* d_Dt64 = nullptr;
  float* d_D16_32 = nullptr;
  double* d_D16_64 = nullptr;
  uint16_t* d_Rhi = nullptr;           // [NTm][ceil(H*H/8)][64][8] bf16 bits
  uint16_t* d_Rlo = nullptr;
  int* d_units = nullptr;              // [nunits][UNIT_STRIDE]: l1, count, q1 values
  int nunits = 0;
  long alloc_count = 0;                // device allocations so far (failure-path test hook)
  int* d_units8 = nullptr;             // units of 8 output states (FP64 two-input tiles, H >= 7)
  int nunits8 = 0;
  int* d_units2 = nullptr;             // units of 2 output states (short launches, see unit_list)
  int nunits2 = 0;
  int GQ = 0;                          // q1 per unit
  double tile_cost = 0.0;              // estimated cost of one full 16-cell tile (scheduling only)
  int lds_limit = 0;                   // usable LDS bytes per workgroup
  int cu_count = 256;                  // compute units of the device

  // conservation check scratch
  double* d_check = nullptr;
  int check_blocks = 256;

  std::vector<void*> allocations;
};

namespace wefq {

// ints per work-unit record of the apply kernels: l1, count, up to 8 q1 values
constexpr int UNIT_STRIDE = 10;

// LDS layout of a cell tile (shared by the host tables and the kernels).  Rows are
// (q, k), TB cells per row, one block of NK rows per q.  Lane groups of the lower half
// of k read rows [0, H) of a block, those of the upper half H rows from `upper`.  The two
// halves start an odd number of rows apart, so that rows of 16, 8 or 4 cells read by
// the two halves fall into different LDS banks:
//  * odd NK, odd H: the upper half starts at k = H; its last row (k = NK) has zero
//    weight and reads the next block's first row, or after the last block one zero
//    tail row;
//  * odd NK, even H: it starts at k = NK - H = H - 1; that first row, shared with the
//    lower half, has zero weight;
//  * even NK: it starts at k = H; when H is even, one zero pad row per block sits between
//    k = H - 1 and k = H, which also makes the block pitch NK + 1 odd (the rows of different
//    output states' q blocks then fall into different banks as often as odd NK allows).
//    every_tile = false keeps the pad to 16-cell tiles (the halves of 8- and 4-cell tiles
//    are then H rows apart): the persistent plan kernel, whose one body holds every tile
//    shape, measured slower with the pad code in its 8- and 4-cell shapes.
__host__ __device__ inline int tile_pad_rows(int NK, int H, int TB, bool every_tile = true) {
  return (!(NK & 1) && !(H & 1) && (every_tile || TB == 16)) ? 1 : 0;
}
__host__ __device__ inline int tile_tail_rows(int NK, int H) { return ((NK & 1) && (H & 1)) ? 1 : 0; }
__host__ __device__ inline int tile_upper_k(int NK, int H) { return ((NK & 1) && !(H & 1)) ? NK - H : H; }
__host__ __device__ inline int tile_upper_row(int NK, int H, int TB, bool every_tile = true) {
  return tile_upper_k(NK, H) + tile_pad_rows(NK, H, TB, every_tile);
}

// Output states per work unit, for every quadrant size.  Units of 4 states give each wave
// shorter serial chains than 8 and balance a tile's waves better; the kernels then hold 4
// accumulator groups instead of 8, which was faster again in FP64 (5% at K = L = 12) and at
// small truncations.  Tiles with 8 output states per column group take units of 8.
constexpr int kUnitStates = 4;

// Workgroups per cell tile for a launch of ntiles tiles over a list of nunits work units.
// Every output row still belongs to one unit and one wave, so the split never changes
// results; every workgroup keeps at least 4 units for its 8 waves.
// * Below one tile per compute unit, each tile's units are split to about one workgroup per
//   compute unit (latency mode).
// * per_cu is 2 where two workgroups of the kernel fit on a compute unit and its quadrants
//   are 4x4 or larger (set at core build), else 1: a launch of one to per_cu tiles per
//   compute unit then splits its tiles to about per_cu workgroups per compute unit.  (Below
//   one tile per compute unit the units per workgroup run short of its 8 waves first: at
//   K = L = 8 with 1,024 cells, targeting two per unit cost 17%.)
// * resident > 0 (workgroups resident on the device at once): a launch whose tiles leave
//   the last round of workgroups partly empty splits them n ways, n <= 4, for the fewest
//   rounds per tile, ceil(ntiles n / resident) / n, charged 4% per extra split.  Measured at
//   K = L = 16 with 315 tiles on 256 compute units: 19.6 ms unsplit, 13.8 ms in 4; at
//   K = L = 12 with 375 tiles: 5.29 ms, 4.06 ms in 2; whole rounds (512, 1,024, 4,096 tiles)
//   stay unsplit.
inline int tile_splits(const wefq_core* h, int64_t ntiles, int nunits, int per_cu, int64_t resident) {
  const int64_t cus = (int64_t)h->cu_count;
  const int64_t cap = nunits / 4 > 1 ? nunits / 4 : 1;
  if (ntiles <= 0) return 1;
  const int64_t target = (per_cu > 1 && ntiles >= cus) ? cus * per_cu : cus;
  if (ntiles < target) {
    const int64_t want = (target + ntiles - 1) / ntiles;
    return (int)(want < cap ? want : cap);
  }
  if (resident <= 0) return 1;
  int best = 1;
  double best_t = (double)((ntiles + resident - 1) / resident);
  for (int n = 2; n <= 4 && n <= cap; ++n) {
    const double rounds = (double)((ntiles * n + resident - 1) / resident);
    const double t = rounds / n * (1.0 + 0.04 * (n - 1));
    if (t < best_t) { best_t = t; best = n; }
  }
  return best;
}

// Units of 2 output states for a launch whose workgroups would hold fewer than 2 units of 4
// per wave (one slot per column group, FP32 and BF16x3): more, shorter units even out the
// waves' chains.  Measured on one MI355X against units of 4 (ms): K = L = 8, 4,096 cells, FP32
// 0.315 -> 0.297 and BF16x3 0.265 -> 0.240; K = L = 12, 1,024 cells, FP32 0.917 -> 0.775.  At 2
// or more units of 4 per wave they were equal or slower (K = L = 8 with 8,192 cells: 0.549 ->
// 0.568 ms; K = L = 12 with 8,192: 4.92 -> 5.05 ms), and slower in FP64 (0.540 -> 0.555 ms at
// K = L = 8, 4,096 cells), whose R tile is loaded per unit and channel.  Every output row
// still belongs to one unit and one wave and is summed in the same order: the choice never
// changes results.
inline bool use_units2(const wefq_core* h, int mode, int slots, int nsplit, int block) {
  if (!h->d_units2 || mode == 2 || slots != 1) return false;
  const int64_t waves = (int64_t)nsplit * (block / 64);
  return (int64_t)h->nunits < 2 * waves;
}

// Kernel mode of a precision: 0 FP32, 1 BF16X3, 2 FP64 (tiled); -1 otherwise.
inline int mfma_mode(int precision) {
  return precision == WEFQ_FP32 ? 0 : precision == WEFQ_BF16X3 ? 1 : precision == WEFQ_FP64 ? 2 : -1;
}

// LDS bytes of one coefficient tile of 16/slots cells.
inline size_t tile_lds_bytes(const wefq_core* h, int slots, size_t elem, bool every_tile = true) {
  const int TB = 16 / slots;
  const int pd = tile_pad_rows(h->NK, h->H, TB, every_tile);
  return ((size_t)h->NQ * (h->NK + pd) + tile_tail_rows(h->NK, h->H)) * TB * elem;
}

// Error reporting helper (thread-local message).
void set_error(const std::string& msg);

// Test hook for the failure paths: with WEFQ_TEST_FAIL_DEVICE_ALLOC=n in the environment, the
// n-th device allocation of a handle's tables (counted from 1) and every later one fail as if
// the device were out of memory.
inline bool injected_alloc_failure(wefq_core* h) {
  const char* e = std::getenv("WEFQ_TEST_FAIL_DEVICE_ALLOC");
  if (!e) return false;
  const long n = std::atol(e);
  return n > 0 && ++h->alloc_count >= n;
}

// Allocate device memory recorded in the handle.
template <typename T>
T* dev_alloc(wefq_core* h, size_t count) {
  void* p = nullptr;
  if (count == 0) count = 1;
  if (injected_alloc_failure(h)) return nullptr;
  if (hipMalloc(&p, count * sizeof(T)) != hipSuccess) return nullptr;
  h->allocations.push_back(p);
  h->device_bytes += (int64_t)(count * sizeof(T));
  return (T*)p;
}

// FP64 radial core on the device: fills h->R64 (not yet zeroed) on the host.
// Returns false (with set_error) on failure.
bool build_radial_core(wefq_core* h, const std::vector<CooRow>& coo, hipStream_t stream);

// Upload routing tables / MFMA tiles for the requested precisions.
bool prepare_apply_tables(wefq_core* h, const std::vector<CooRow>& coo, hipStream_t stream);

// Kernel launchers (apply.hip).
hipError_t launch_apply_fp64(const wefq_core* h, const double* f, double* Q, int64_t B,
                             int64_t ldf, int64_t ldq, hipStream_t s);
hipError_t launch_apply_mfma(const wefq_core* h, int precision, const void* f, void* Q,
                             int64_t B, int64_t ldf, int64_t ldq, hipStream_t s);
// Private (scratch) bytes per lane of the MFMA kernel instance of a tile shape and block size
// (the 12-wave instance above 512 threads): nonzero when it spills registers.  Returns -1 for
// a shape with no instance.
int mfma_spill_bytes(const wefq_core* h, int mode, int slots, int block);
// Workgroups of the apply kernel for (mode, slots) resident per compute unit at the given
// block size with its LDS tile; 0 when the query fails.
int mfma_blocks_per_cu(const wefq_core* h, int mode, int slots, int block);
// Jacobian-vector product out = J(c) d = Q(c, d) + Q(d, c) for FP32 or FP64 (jvp.hip).
hipError_t launch_apply_jvp(const wefq_core* h, int precision, const void* c, const void* d, void* out,
                            int64_t B, int64_t ldc, int64_t ldd, int64_t ldo, hipStream_t s);
// Bilinear form out = Q(f, g) for FP32 or FP64 (jvp.hip; needs the WEFQ_PREP_BILINEAR tables).
hipError_t launch_apply_qfg(const wefq_core* h, int precision, const void* f, const void* g, void* out,
                            int64_t B, int64_t ldf, int64_t ldg, int64_t ldo, hipStream_t s);
hipError_t launch_check(const wefq_core* h, int precision, const void* Q, int64_t B,
                        int64_t ldq, hipStream_t s);
// Radial-first ordering, FP64 (radial.hip; needs the WEFQ_PREP_RADIAL tables).  work holds
// chunk * radial_bytes_per_cell(h) bytes; chunk is a multiple of 64.
int64_t radial_bytes_per_cell(const wefq_core* h);
hipError_t launch_apply_radial(const wefq_core* h, const double* f, double* Q, int64_t B, int64_t ldf, int64_t ldq,
                               void* work, int64_t chunk, hipStream_t s);

}  // namespace wefq
