// Uneven batches in one persistent launch (several cores of different size and
// collision model in one kernel), captured once in a HIP graph.
//
// A plan is a list of segments (core, precision, f, Q, B, tile shape).  Its
// work list holds one item per (segment, cell tile), or several per tile when a
// tile's cost exceeds a third of a workgroup's fair share (the tile's work units
// are then dealt round-robin to the items), sorted by decreasing estimated cost,
// so the largest items start first and the last ones are short.  The persistent kernel
// runs as many workgroups as fit on the device at once; each pulls items from
// a device counter and runs the same per-tile code as the standalone apply
// (same arithmetic order, hence bitwise the same per-cell results), selecting
// the tile geometry of the item's core (8- and 4-cell tiles of even NK and even H
// without the standalone layout's pad rows: only LDS addresses differ).
// plan_reset_kernel clears the counter (a kernel node, so replays of the captured
// graph need no memset node).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/wefq.h"
#include "apply_tile.h"
#include "wefq_core.h"

namespace wefq {

struct SegDesc {
  MfmaParams p;
  int H, SLOTS, RT, pad;
};

struct PlanParams {
  const SegDesc* segs;
  const int64_t* items;     // seg << 48 | split << 40 | tile
  int nitems;
  int* counter;
};

__global__ void plan_reset_kernel(int* counter) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *counter = 0;
}

#define WEFQ_TILE_CASE(H_, S_, R_)                                                                        \
  case (H_) * 100 + (S_) * 10 + (R_):                                                                     \
    mfma_tile<H_, S_, R_, MODE, false, false, WAVES, false, true>(sd.p, tile, split, lds_raw, &unit_ctr); \
    break;
#define WEFQ_TILE_CASES_H(H_) WEFQ_TILE_CASE(H_, 1, 1) WEFQ_TILE_CASE(H_, 2, 1) WEFQ_TILE_CASE(H_, 4, 1)

// Builds of the persistent kernel (VARIANT):
//  * kAll: 8 waves (256 or 512 threads), every tile shape.  One body holding them all spills
//    registers in BF16x3 (8 bytes per lane) and FP64 (572);
//  * kWide: 12 waves (768 threads, three per SIMD, 168 registers), FP32 quadrants up to 5x5
//    and 7x7 with one output state per column group and 9x9 with two and the 17th radial row
//    (the default FP32 shapes of K = 0..9, 12 and 16).  These compile together without spill;
//    adding 6x6 spilled 32 bytes per lane, adding 7x7 and 8x8 with two output states 100;
//  * kWide2: 12 waves, FP32 quadrants 6x6 with one output state per column group and 7x7 and
//    8x8 with two (the default shapes of K = 10, 11 and 13 to 15), 8 bytes of spill per lane;
//  * kDefaults: 8 waves, the BF16x3 or FP64 shapes the core build picks by default on this
//    device (BF16x3: 1x1 to 7x7 with one output state per column group, 7x7 to 9x9 with two,
//    no spill; FP64: 1x1 to 5x5 with one, 6x6 and 7x7 with two, 7x7 to 9x9 with four, 300
//    bytes).  Plans of these shapes measured 4-6% faster than with kAll.
enum { kAll = 0, kWide = 1, kDefaults = 2, kWide2 = 3 };

// The shape lists (H, SLOTS, RT) of the restricted builds; the kernel's switch and the host's
// membership tests are both generated from them.
#define WEFQ_WIDE_SHAPES(X) X(1, 1, 1) X(2, 1, 1) X(3, 1, 1) X(4, 1, 1) X(5, 1, 1) X(7, 1, 1) X(9, 2, 2)
#define WEFQ_WIDE2_SHAPES(X) X(6, 1, 1) X(7, 2, 1) X(8, 2, 1)
#define WEFQ_BF16_DEFAULT_SHAPES(X) \
  X(1, 1, 1) X(2, 1, 1) X(3, 1, 1) X(4, 1, 1) X(5, 1, 1) X(6, 1, 1) X(7, 1, 1) X(7, 2, 1) X(8, 2, 1) X(9, 2, 2)
#define WEFQ_FP64_DEFAULT_SHAPES(X) \
  X(1, 1, 1) X(2, 1, 1) X(3, 1, 1) X(4, 1, 1) X(5, 1, 1) X(6, 2, 1) X(7, 2, 1) X(7, 4, 1) X(8, 4, 1) X(9, 4, 2)
#define WEFQ_SHAPE_IS(H_, S_, R_) || (H == (H_) && SLOTS == (S_) && RT == (R_))

__host__ __device__ constexpr bool wide_plan_shape(int H, int SLOTS, int RT) {
  return false WEFQ_WIDE_SHAPES(WEFQ_SHAPE_IS);
}
__host__ __device__ constexpr bool wide2_plan_shape(int H, int SLOTS, int RT) {
  return false WEFQ_WIDE2_SHAPES(WEFQ_SHAPE_IS);
}
__host__ __device__ constexpr bool default_plan_shape(int mode, int H, int SLOTS, int RT) {
  return mode == 1 ? (false WEFQ_BF16_DEFAULT_SHAPES(WEFQ_SHAPE_IS))
                   : mode == 2 ? (false WEFQ_FP64_DEFAULT_SHAPES(WEFQ_SHAPE_IS)) : false;
}

template <int MODE, int VARIANT>
__global__ __launch_bounds__(VARIANT == kWide || VARIANT == kWide2 ? 768 : 512) void apply_persistent_kernel(
    PlanParams pp) {
  constexpr int WAVES = VARIANT == kWide || VARIANT == kWide2 ? 12 : 8;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  __shared__ int unit_ctr;
  __shared__ int item_sh;
  while (true) {
    if (threadIdx.x == 0) item_sh = atomicAdd(pp.counter, 1);
    __syncthreads();
    const int it = item_sh;
    __syncthreads();
    if (it >= pp.nitems) break;
    const int64_t code = pp.items[it];
    const SegDesc& sd = pp.segs[(int)(code >> 48)];
    const int split = (int)((code >> 40) & 0xff);
    const int64_t tile = code & ((1LL << 40) - 1);
    if constexpr (VARIANT == kWide) {
      switch (sd.H * 100 + sd.SLOTS * 10 + sd.RT) {
        WEFQ_WIDE_SHAPES(WEFQ_TILE_CASE)
        default: break;
      }
    } else if constexpr (VARIANT == kWide2) {
      switch (sd.H * 100 + sd.SLOTS * 10 + sd.RT) {
        WEFQ_WIDE2_SHAPES(WEFQ_TILE_CASE)
        default: break;
      }
    } else if constexpr (VARIANT == kDefaults && MODE == 1) {
      switch (sd.H * 100 + sd.SLOTS * 10 + sd.RT) {
        WEFQ_BF16_DEFAULT_SHAPES(WEFQ_TILE_CASE)
        default: break;
      }
    } else if constexpr (VARIANT == kDefaults) {
      switch (sd.H * 100 + sd.SLOTS * 10 + sd.RT) {
        WEFQ_FP64_DEFAULT_SHAPES(WEFQ_TILE_CASE)
        default: break;
      }
    } else {
      switch (sd.H * 100 + sd.SLOTS * 10 + sd.RT) {
        WEFQ_TILE_CASES_H(1) WEFQ_TILE_CASES_H(2) WEFQ_TILE_CASES_H(3)
        WEFQ_TILE_CASES_H(4) WEFQ_TILE_CASES_H(5) WEFQ_TILE_CASES_H(6)
        WEFQ_TILE_CASES_H(7) WEFQ_TILE_CASES_H(8) WEFQ_TILE_CASES_H(9)
        WEFQ_TILE_CASE(8, 1, 2) WEFQ_TILE_CASE(8, 2, 2) WEFQ_TILE_CASE(8, 4, 2)
        WEFQ_TILE_CASE(9, 1, 2) WEFQ_TILE_CASE(9, 2, 2) WEFQ_TILE_CASE(9, 4, 2)
        default: break;
      }
    }
    __syncthreads();                 // the tile's LDS is reused by the next item
  }
}

}  // namespace wefq

using namespace wefq;

struct wefq_plan_s {
  int device = 0;
  int mode = 0;
  int block = 512;
  int variant = kAll;
  int grid = 0;
  size_t lds = 0;
  int nitems = 0;
  SegDesc* d_segs = nullptr;
  int64_t* d_items = nullptr;
  int* d_counter = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  const void* kernel = nullptr;
};

static wefq_status plan_fail(wefq_status st, const std::string& msg) {
  set_error(msg);
  return st;
}

static void plan_free(wefq_plan_s* p) {
  if (!p) return;
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->d_segs) (void)hipFree(p->d_segs);
  if (p->d_items) (void)hipFree(p->d_items);
  if (p->d_counter) (void)hipFree(p->d_counter);
  delete p;
}

// Kernel of a plan precision (mode 0 FP32, 1 BF16X3, 2 FP64) and build (kWide: FP32 only).
static const void* persistent_kernel(int mode, int variant) {
  if (variant == kWide) return (const void*)apply_persistent_kernel<0, kWide>;
  if (variant == kWide2) return (const void*)apply_persistent_kernel<0, kWide2>;
  if (variant == kDefaults && mode == 1) return (const void*)apply_persistent_kernel<1, kDefaults>;
  if (variant == kDefaults && mode == 2) return (const void*)apply_persistent_kernel<2, kDefaults>;
  return mode == 0 ? (const void*)apply_persistent_kernel<0, kAll>
         : mode == 1 ? (const void*)apply_persistent_kernel<1, kAll> : (const void*)apply_persistent_kernel<2, kAll>;
}

static hipError_t launch_persistent(int mode, int variant, int block, int grid, size_t lds, hipStream_t s,
                                    PlanParams pp) {
  void* args[] = {&pp};
  hipError_t e = hipLaunchKernel(persistent_kernel(mode, variant), dim3(grid), dim3(block), args, lds, s);
  return e != hipSuccess ? e : hipGetLastError();
}

static hipError_t plan_enqueue(const wefq_plan_s* p, hipStream_t s) {
  hipLaunchKernelGGL(plan_reset_kernel, dim3(1), dim3(64), 0, s, p->d_counter);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_persistent(p->mode, p->variant, p->block, p->grid, p->lds, s,
                           PlanParams{p->d_segs, p->d_items, p->nitems, p->d_counter});
}

// A batch of segments made into a work list: the per-segment parameters and the item codes,
// largest first.
struct WorkList {
  int mode = 0;
  int device = -1;
  size_t lds = 0;
  std::vector<SegDesc> descs;
  std::vector<int64_t> codes;
};

// The 12-wave build whose tile shapes cover every segment of an FP32 work list, or kAll when
// none does.
static int wide_variant(const WorkList& w) {
  if (w.mode != 0) return kAll;
  bool a = true, b = true;
  for (const SegDesc& d : w.descs) {
    a = a && wide_plan_shape(d.H, d.SLOTS, d.RT);
    b = b && wide2_plan_shape(d.H, d.SLOTS, d.RT);
  }
  return a ? kWide : (b ? kWide2 : kAll);
}
static bool all_wide(const WorkList& w) { return wide_variant(w) != kAll; }

// The build of the persistent kernel for a work list at a block size (768 needs all_wide).
static int kernel_variant(const WorkList& w, int block) {
  if (block == 768) return wide_variant(w);
  if (w.mode == 0) return kAll;
  for (const SegDesc& d : w.descs)
    if (!default_plan_shape(w.mode, d.H, d.SLOTS, d.RT)) return kAll;
  return kDefaults;
}

// Validate the segments and build their descriptors (any mix of cores of one precision on one
// device).  Items are made by make_items once the residency is known.
static wefq_status describe_segments(int32_t nseg, const wefq_segment* segs, WorkList& w,
                                     std::vector<int64_t>& seg_tiles, std::vector<double>& seg_cost,
                                     std::vector<int>& seg_units) {
  if (!segs || nseg <= 0) return plan_fail(WEFQ_EINVAL, "at least one segment is needed");
  const int prec = segs[0].precision;
  if (prec != WEFQ_FP32 && prec != WEFQ_BF16X3 && prec != WEFQ_FP64)
    return plan_fail(WEFQ_EINVAL, "plan precision must be FP32, BF16X3 or FP64");
  const int mode = prec == WEFQ_FP64 ? 2 : (prec == WEFQ_BF16X3 ? 1 : 0);
  const size_t elem = mode == 2 ? 8 : 4;
  const int device = segs[0].core ? segs[0].core->device : -1;
  if (nseg >= (1 << 15)) return plan_fail(WEFQ_EINVAL, "too many segments");
  w.mode = mode;
  w.device = device;
  w.lds = 0;
  w.descs.assign(nseg, SegDesc());
  seg_tiles.assign(nseg, 0);
  seg_cost.assign(nseg, 0.0);
  seg_units.assign(nseg, 0);
  for (int i = 0; i < nseg; ++i) {
    const wefq_segment& g = segs[i];
    wefq_core* h = g.core;
    if (!h) return plan_fail(WEFQ_EINVAL, "null core in segment");
    if (h->device != device) return plan_fail(WEFQ_EINVAL, "all segments must use cores on one device");
    if (g.precision != prec) return plan_fail(WEFQ_EINVAL, "all segments of a plan use one precision");
    if (!(h->precisions & (unsigned)prec)) return plan_fail(WEFQ_EINVAL, "precision was not prepared for a core");
    if (g.B < 0) return plan_fail(WEFQ_EINVAL, "negative segment size");
    if (g.B > 0 && (!g.f || !g.Q)) return plan_fail(WEFQ_EINVAL, "null segment buffer");
    if (g.ld_f < h->N || g.ld_q < h->N) return plan_fail(WEFQ_EINVAL, "leading dimension smaller than N");
    if (((uintptr_t)g.f | (uintptr_t)g.Q) & (elem - 1)) return plan_fail(WEFQ_EINVAL, "buffers must be aligned to the element size");
    int slots = g.slots ? g.slots : h->slots[mode];
    if (slots != 1 && slots != 2 && slots != 4) return plan_fail(WEFQ_EINVAL, "slots must be 0, 1, 2 or 4");
    const int TB = 16 / slots;
    const size_t need = tile_lds_bytes(h, slots, elem, false);
    if (need > (size_t)h->lds_limit) return plan_fail(WEFQ_EUNSUPPORTED, "segment tile does not fit in LDS");
    w.lds = std::max(w.lds, need);
    SegDesc& d = w.descs[i];
    std::memset(&d, 0, sizeof(d));
    MfmaParams& p = d.p;
    p.f = g.f; p.g = nullptr; p.Q = g.Q; p.B = g.B; p.ldf = g.ld_f; p.ldg = 0; p.ldq = g.ld_q;
    p.NK = h->NK; p.NQ = h->NQ; p.N = h->N;
    p.nunits = h->nunits; p.nsplit = 1; p.units = h->d_units; p.chan_begin = h->d_chan_begin;
    p.slice_off = h->d_slice_off; p.sptr = h->d_sptr; p.spair = h->d_spair; p.mq = h->d_mq; p.mq_pad = h->d_mq_pad;
    p.mg = h->d_mg; p.mg64 = h->d_mg64;
    p.Rt32 = h->d_Rt32; p.Rt64 = h->d_Rt64; p.Rhi = h->d_Rhi; p.Rlo = h->d_Rlo;
    p.R16_32 = h->d_R16_32; p.R16_64 = h->d_R16_64;
    d.H = h->H; d.SLOTS = slots; d.RT = h->RT;
    const int64_t ntiles = (g.B + TB - 1) / TB;
    if (ntiles >= (1LL << 40)) return plan_fail(WEFQ_EINVAL, "segment too large");
    seg_tiles[i] = ntiles;
    seg_cost[i] = h->tile_cost * (double)TB / 16.0;
    seg_units[i] = h->nunits;
  }
  return WEFQ_OK;
}

// Work items: (segment, cell tile, split), largest first.  A tile whose cost exceeds a third of a
// workgroup's fair share is split over several workgroups (its work units dealt round-robin, as
// in a small-batch launch), so that the last items are short.
static wefq_status make_items(WorkList& w, const std::vector<int64_t>& seg_tiles, const std::vector<double>& seg_cost,
                              const std::vector<int>& seg_units, int resident) {
  const int nseg = (int)w.descs.size();
  double total = 0.0;
  for (int i = 0; i < nseg; ++i) total += seg_cost[i] * (double)seg_tiles[i];
  const double target = total / (3.0 * (double)resident);
  std::vector<std::pair<double, int64_t>> items;
  for (int i = 0; i < nseg; ++i) {
    int ns = 1;
    if (target > 0.0 && seg_cost[i] > target) {
      const int cap = std::max(1, std::min(255, seg_units[i] / 4));
      ns = (int)std::min<double>(cap, std::ceil(seg_cost[i] / target));
    }
    w.descs[i].p.nsplit = ns;
    for (int64_t t = 0; t < seg_tiles[i]; ++t)
      for (int sp = 0; sp < ns; ++sp)
        items.push_back({seg_cost[i] / ns, ((int64_t)i << 48) | ((int64_t)sp << 40) | t});
  }
  if (items.size() > 0x7fffffffULL) return plan_fail(WEFQ_EINVAL, "too many work items");
  std::stable_sort(items.begin(), items.end(),
                   [](const std::pair<double, int64_t>& a, const std::pair<double, int64_t>& b) { return a.first > b.first; });
  w.codes.resize(items.size());
  for (size_t i = 0; i < items.size(); ++i) w.codes[i] = items[i].second;
  return WEFQ_OK;
}

// Workgroups of a persistent kernel build resident per compute unit at (block, lds), and the
// compute unit count of the current device.
static void residency(int mode, int variant, int block, size_t lds, int device, int* per_cu, int* cus) {
  *per_cu = 0;
  *cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, persistent_kernel(mode, variant), block, lds) != hipSuccess ||
      *per_cu < 1)
    *per_cu = 1;
  if (hipDeviceGetAttribute(cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || *cus < 1) *cus = 1;
}

extern "C" {

wefq_status wefq_plan_create(int32_t nseg, const wefq_segment* segs, int32_t block, void* stream,
                             wefq_plan* out) {
  if (!out || !segs || nseg <= 0) return plan_fail(WEFQ_EINVAL, "plan needs at least one segment and an output");
  *out = nullptr;
  if (block != 256 && block != 512 && block != 768) return plan_fail(WEFQ_EINVAL, "block must be 256, 512 or 768");
  WorkList w;
  std::vector<int64_t> seg_tiles;
  std::vector<double> seg_cost;
  std::vector<int> seg_units;
  wefq_status st = describe_segments(nseg, segs, w, seg_tiles, seg_cost, seg_units);
  if (st != WEFQ_OK) return st;
  if (block == 768 && !all_wide(w))
    return plan_fail(WEFQ_EINVAL, "block 768 runs FP32 plans whose tile shapes all belong to one 12-wave build");
  const int mode = w.mode, device = w.device;
  const size_t lds = w.lds;
  if (hipSetDevice(device) != hipSuccess) return plan_fail(WEFQ_EHIP, "hipSetDevice failed");
  const int variant = kernel_variant(w, block);
  const void* k = persistent_kernel(mode, variant);
  if (hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
    return plan_fail(WEFQ_EHIP, "cannot reserve LDS for the persistent kernel");
  int per_cu = 0, cus = 0;
  residency(mode, variant, block, lds, device, &per_cu, &cus);
  st = make_items(w, seg_tiles, seg_cost, seg_units, per_cu * cus);
  if (st != WEFQ_OK) return st;
  const std::vector<SegDesc>& descs = w.descs;
  const std::vector<int64_t>& codes = w.codes;
  wefq_plan_s* pl = new (std::nothrow) wefq_plan_s();
  if (!pl) return plan_fail(WEFQ_ENOMEM, "host allocation failed");
  pl->device = device; pl->mode = mode; pl->block = block; pl->variant = variant; pl->lds = lds;
  pl->nitems = (int)codes.size();
  bool ok = hipMalloc(&pl->d_segs, sizeof(SegDesc) * nseg) == hipSuccess &&
            hipMalloc(&pl->d_items, sizeof(int64_t) * std::max<size_t>(1, codes.size())) == hipSuccess &&
            hipMalloc(&pl->d_counter, sizeof(int) * 64) == hipSuccess;
  if (!ok) { plan_free(pl); return plan_fail(WEFQ_ENOMEM, "device allocation failed"); }
  hipStream_t s = (hipStream_t)stream;
  ok = hipMemcpyAsync(pl->d_segs, descs.data(), sizeof(SegDesc) * nseg, hipMemcpyHostToDevice, s) == hipSuccess &&
       (codes.empty() || hipMemcpyAsync(pl->d_items, codes.data(), sizeof(int64_t) * codes.size(),
                                        hipMemcpyHostToDevice, s) == hipSuccess) &&
       hipStreamSynchronize(s) == hipSuccess;
  if (!ok) { plan_free(pl); return plan_fail(WEFQ_EHIP, "plan upload failed"); }
  pl->kernel = k;
  pl->grid = std::max(1, std::min(per_cu * cus, std::max(1, pl->nitems)));
  // capture {reset, persistent kernel} once; replays launch the instantiated graph
  hipStream_t cs = nullptr;
  ok = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) == hipSuccess &&
       hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess;
  if (ok) {
    hipError_t e = plan_enqueue(pl, cs);
    hipError_t e2 = hipStreamEndCapture(cs, &pl->graph);
    ok = e == hipSuccess && e2 == hipSuccess &&
         hipGraphInstantiate(&pl->exec, pl->graph, nullptr, nullptr, 0) == hipSuccess;
  }
  if (cs) (void)hipStreamDestroy(cs);
  if (!ok) { plan_free(pl); return plan_fail(WEFQ_EHIP, "graph capture of the plan failed"); }
  *out = pl;
  return WEFQ_OK;
}

wefq_status wefq_plan_launch(wefq_plan p, void* stream) {
  if (!p) return plan_fail(WEFQ_EINVAL, "null plan");
  if (p->nitems == 0) return WEFQ_OK;
  if (hipSetDevice(p->device) != hipSuccess) return plan_fail(WEFQ_EHIP, "hipSetDevice failed");
  hipError_t e = hipGraphLaunch(p->exec, (hipStream_t)stream);
  if (e != hipSuccess) return plan_fail(WEFQ_EHIP, std::string("graph launch failed: ") + hipGetErrorString(e));
  return WEFQ_OK;
}

wefq_status wefq_plan_launch_direct(wefq_plan p, void* stream) {
  if (!p) return plan_fail(WEFQ_EINVAL, "null plan");
  if (p->nitems == 0) return WEFQ_OK;
  if (hipSetDevice(p->device) != hipSuccess) return plan_fail(WEFQ_EHIP, "hipSetDevice failed");
  hipError_t e = plan_enqueue(p, (hipStream_t)stream);
  if (e != hipSuccess) return plan_fail(WEFQ_EHIP, std::string("plan launch failed: ") + hipGetErrorString(e));
  return WEFQ_OK;
}

wefq_status wefq_plan_info(wefq_plan p, int64_t* work_items, int64_t* lds_bytes, int64_t* grid) {
  if (!p) return plan_fail(WEFQ_EINVAL, "null plan");
  if (work_items) *work_items = p->nitems;
  if (lds_bytes) *lds_bytes = (int64_t)p->lds;
  if (grid) *grid = p->grid;
  return WEFQ_OK;
}

wefq_status wefq_plan_destroy(wefq_plan p) {
  if (!p) return plan_fail(WEFQ_EINVAL, "null plan");
  (void)hipSetDevice(p->device);
  plan_free(p);
  return WEFQ_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- runners (continuous batching)
//
// A runner launches one persistent kernel per call over whatever segments the caller hands
// it: the serving loop's scheduling tick.  Its work lists go through a ring of slots, each a
// device buffer of descriptors, items and counter with a pinned host staging copy; a slot is
// reused once the event recorded after its last launch has completed, so the host waits only
// when every slot is still in flight.  Nothing is allocated per launch.

namespace {
constexpr int kRunnerSlots = 4;

struct RunnerSlot {
  SegDesc* d_segs = nullptr;
  int64_t* d_items = nullptr;
  int* d_counter = nullptr;
  SegDesc* h_segs = nullptr;       // pinned staging
  int64_t* h_items = nullptr;
  hipEvent_t done = nullptr;
  bool used = false;
};
}  // namespace

struct wefq_runner_s {
  int device = 0;
  int mode = 0;
  int block = 512;
  int max_items = 0, max_segments = 0;
  int next = 0;
  int64_t launches = 0;
  RunnerSlot slots[kRunnerSlots];
};

static void runner_free(wefq_runner_s* r) {
  if (!r) return;
  for (RunnerSlot& sl : r->slots) {
    if (sl.done) {
      (void)hipEventSynchronize(sl.done);
      (void)hipEventDestroy(sl.done);
    }
    if (sl.d_segs) (void)hipFree(sl.d_segs);
    if (sl.d_items) (void)hipFree(sl.d_items);
    if (sl.d_counter) (void)hipFree(sl.d_counter);
    if (sl.h_segs) (void)hipHostFree(sl.h_segs);
    if (sl.h_items) (void)hipHostFree(sl.h_items);
  }
  delete r;
}

extern "C" {

wefq_status wefq_runner_create(int32_t device, int32_t precision, int32_t max_segments, int32_t max_items,
                               int32_t block, wefq_runner* out) {
  if (!out) return plan_fail(WEFQ_EINVAL, "null output pointer");
  *out = nullptr;
  if (precision != WEFQ_FP32 && precision != WEFQ_BF16X3 && precision != WEFQ_FP64)
    return plan_fail(WEFQ_EINVAL, "runner precision must be FP32, BF16X3 or FP64");
  if (block != 256 && block != 512 && block != 768) return plan_fail(WEFQ_EINVAL, "block must be 256, 512 or 768");
  if (block == 768 && precision != WEFQ_FP32) return plan_fail(WEFQ_EINVAL, "block 768 runs FP32 runners only");
  if (max_segments < 1 || max_segments >= (1 << 15) || max_items < 1)
    return plan_fail(WEFQ_EINVAL, "max_segments must be in [1, 32767] and max_items >= 1");
  if (hipSetDevice(device) != hipSuccess) return plan_fail(WEFQ_EINVAL, "bad device ordinal");
  wefq_runner_s* r = new (std::nothrow) wefq_runner_s();
  if (!r) return plan_fail(WEFQ_ENOMEM, "host allocation failed");
  r->device = device;
  r->mode = precision == WEFQ_FP64 ? 2 : (precision == WEFQ_BF16X3 ? 1 : 0);
  r->block = block;
  r->max_items = max_items;
  r->max_segments = max_segments;
  bool ok = true;
  for (RunnerSlot& sl : r->slots) {
    ok = ok && hipMalloc(&sl.d_segs, sizeof(SegDesc) * max_segments) == hipSuccess &&
         hipMalloc(&sl.d_items, sizeof(int64_t) * max_items) == hipSuccess &&
         hipMalloc(&sl.d_counter, sizeof(int) * 64) == hipSuccess &&
         hipHostMalloc(&sl.h_segs, sizeof(SegDesc) * max_segments, hipHostMallocDefault) == hipSuccess &&
         hipHostMalloc(&sl.h_items, sizeof(int64_t) * max_items, hipHostMallocDefault) == hipSuccess &&
         hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) == hipSuccess;
    if (!ok) break;
  }
  if (!ok) { runner_free(r); return plan_fail(WEFQ_ENOMEM, "runner allocation failed"); }
  // the largest tile any core may bring: reserve the device's usable LDS once
  int dev_lds = 0;
  if (hipDeviceGetAttribute(&dev_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device) != hipSuccess || dev_lds <= 0)
    dev_lds = 65536;
  const int limit = std::min(dev_lds, 163840) - 512;
  // (every build a launch may pick: a runner of 768 threads launches the 8-wave kernel of 512
  // for batches with other tile shapes)
  bool lds_ok = true;
  for (const int v : {kAll, kDefaults, kWide, kWide2})
    if ((v != kWide && v != kWide2) || r->block == 768)
      lds_ok = lds_ok && hipFuncSetAttribute(persistent_kernel(r->mode, v), hipFuncAttributeMaxDynamicSharedMemorySize,
                                             limit) == hipSuccess;
  if (!lds_ok) {
    runner_free(r);
    return plan_fail(WEFQ_EHIP, "cannot reserve LDS for the persistent kernel");
  }
  *out = r;
  return WEFQ_OK;
}

wefq_status wefq_runner_launch(wefq_runner r, int32_t nseg, const wefq_segment* segs, void* stream) {
  if (!r) return plan_fail(WEFQ_EINVAL, "null runner");
  if (nseg < 0 || nseg > r->max_segments) return plan_fail(WEFQ_EINVAL, "segment count outside [0, max_segments]");
  if (nseg == 0) return WEFQ_OK;
  WorkList w;
  std::vector<int64_t> seg_tiles;
  std::vector<double> seg_cost;
  std::vector<int> seg_units;
  wefq_status st = describe_segments(nseg, segs, w, seg_tiles, seg_cost, seg_units);
  if (st != WEFQ_OK) return st;
  if (w.device != r->device) return plan_fail(WEFQ_EINVAL, "segments must use cores on the runner's device");
  if (w.mode != r->mode) return plan_fail(WEFQ_EINVAL, "segments must use the runner's precision");
  if (hipSetDevice(r->device) != hipSuccess) return plan_fail(WEFQ_EHIP, "hipSetDevice failed");
  const int block = (r->block == 768 && !all_wide(w)) ? 512 : r->block;
  const int variant = kernel_variant(w, block);
  int per_cu = 0, cus = 0;
  residency(r->mode, variant, block, w.lds, r->device, &per_cu, &cus);
  st = make_items(w, seg_tiles, seg_cost, seg_units, per_cu * cus);
  if (st != WEFQ_OK) return st;
  const int nitems = (int)w.codes.size();
  if (nitems > r->max_items) return plan_fail(WEFQ_EBUDGET, "the batch has more work items than the runner holds");
  if (nitems == 0) return WEFQ_OK;
  RunnerSlot& sl = r->slots[r->next];
  if (sl.used && hipEventSynchronize(sl.done) != hipSuccess)
    return plan_fail(WEFQ_EHIP, "waiting for a runner slot failed");
  std::memcpy(sl.h_segs, w.descs.data(), sizeof(SegDesc) * nseg);
  std::memcpy(sl.h_items, w.codes.data(), sizeof(int64_t) * nitems);
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = hipMemcpyAsync(sl.d_segs, sl.h_segs, sizeof(SegDesc) * nseg, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(sl.d_items, sl.h_items, sizeof(int64_t) * nitems, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(plan_reset_kernel, dim3(1), dim3(64), 0, s, sl.d_counter);
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    const int grid = std::max(1, std::min(per_cu * cus, nitems));
    e = launch_persistent(r->mode, variant, block, grid, w.lds, s,
                          PlanParams{sl.d_segs, sl.d_items, nitems, sl.d_counter});
  }
  // the slot is busy until everything enqueued above has run (also after a failed enqueue)
  const hipError_t er = hipEventRecord(sl.done, s);
  sl.used = er == hipSuccess;
  r->next = (r->next + 1) % kRunnerSlots;
  if (e != hipSuccess) return plan_fail(WEFQ_EHIP, std::string("runner launch failed: ") + hipGetErrorString(e));
  if (er != hipSuccess) return plan_fail(WEFQ_EHIP, "runner event record failed");
  ++r->launches;
  return WEFQ_OK;
}

wefq_status wefq_runner_destroy(wefq_runner r) {
  if (!r) return plan_fail(WEFQ_EINVAL, "null runner");
  (void)hipSetDevice(r->device);
  runner_free(r);
  return WEFQ_OK;
}

}  // extern "C"
