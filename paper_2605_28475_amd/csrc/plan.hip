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
// the tile geometry of the item's core.  plan_reset_kernel clears the counter
// (a kernel node, so replays of the captured graph need no memset node).
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

#define WEFQ_TILE_CASE(H_, S_, R_)                                       \
  case (H_) * 100 + (S_) * 10 + (R_):                                    \
    mfma_tile<H_, S_, R_, MODE>(sd.p, tile, split, lds_raw, &unit_ctr);  \
    break;
#define WEFQ_TILE_CASES_H(H_) WEFQ_TILE_CASE(H_, 1, 1) WEFQ_TILE_CASE(H_, 2, 1) WEFQ_TILE_CASE(H_, 4, 1)

template <int MODE>
__global__ __launch_bounds__(512) void apply_persistent_kernel(PlanParams pp) {
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
    switch (sd.H * 100 + sd.SLOTS * 10 + sd.RT) {
      WEFQ_TILE_CASES_H(1) WEFQ_TILE_CASES_H(2) WEFQ_TILE_CASES_H(3)
      WEFQ_TILE_CASES_H(4) WEFQ_TILE_CASES_H(5) WEFQ_TILE_CASES_H(6)
      WEFQ_TILE_CASES_H(7) WEFQ_TILE_CASES_H(8) WEFQ_TILE_CASES_H(9)
      WEFQ_TILE_CASE(8, 1, 2) WEFQ_TILE_CASE(8, 2, 2) WEFQ_TILE_CASE(8, 4, 2)
      WEFQ_TILE_CASE(9, 1, 2) WEFQ_TILE_CASE(9, 2, 2) WEFQ_TILE_CASE(9, 4, 2)
      default: break;
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

static hipError_t plan_enqueue(const wefq_plan_s* p, hipStream_t s) {
  hipLaunchKernelGGL(plan_reset_kernel, dim3(1), dim3(64), 0, s, p->d_counter);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  PlanParams pp{p->d_segs, p->d_items, p->nitems, p->d_counter};
  switch (p->mode) {
    case 0: hipLaunchKernelGGL(apply_persistent_kernel<0>, dim3(p->grid), dim3(p->block), p->lds, s, pp); break;
    case 1: hipLaunchKernelGGL(apply_persistent_kernel<1>, dim3(p->grid), dim3(p->block), p->lds, s, pp); break;
    default: hipLaunchKernelGGL(apply_persistent_kernel<2>, dim3(p->grid), dim3(p->block), p->lds, s, pp); break;
  }
  return hipGetLastError();
}

extern "C" {

wefq_status wefq_plan_create(int32_t nseg, const wefq_segment* segs, int32_t block, void* stream,
                             wefq_plan* out) {
  if (!out || !segs || nseg <= 0) return plan_fail(WEFQ_EINVAL, "plan needs at least one segment and an output");
  *out = nullptr;
  if (block != 256 && block != 512) return plan_fail(WEFQ_EINVAL, "block must be 256 or 512");
  const int prec = segs[0].precision;
  if (prec != WEFQ_FP32 && prec != WEFQ_BF16X3 && prec != WEFQ_FP64)
    return plan_fail(WEFQ_EINVAL, "plan precision must be FP32, BF16X3 or FP64");
  const int mode = prec == WEFQ_FP64 ? 2 : (prec == WEFQ_BF16X3 ? 1 : 0);
  const size_t elem = mode == 2 ? 8 : 4;
  const int device = segs[0].core ? segs[0].core->device : -1;
  if (nseg >= (1 << 15)) return plan_fail(WEFQ_EINVAL, "too many segments");
  std::vector<SegDesc> descs(nseg);
  std::vector<int64_t> seg_tiles(nseg);
  std::vector<double> seg_cost(nseg);
  std::vector<int> seg_units(nseg);
  size_t lds = 0;
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
    const size_t need = tile_lds_bytes(h, slots, elem);
    if (need > (size_t)h->lds_limit) return plan_fail(WEFQ_EUNSUPPORTED, "segment tile does not fit in LDS");
    lds = std::max(lds, need);
    SegDesc& d = descs[i];
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
  if (hipSetDevice(device) != hipSuccess) return plan_fail(WEFQ_EHIP, "hipSetDevice failed");
  const void* k = mode == 0 ? (const void*)apply_persistent_kernel<0>
                  : mode == 1 ? (const void*)apply_persistent_kernel<1> : (const void*)apply_persistent_kernel<2>;
  if (hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
    return plan_fail(WEFQ_EHIP, "cannot reserve LDS for the persistent kernel");
  int per_cu = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, block, lds) != hipSuccess || per_cu < 1) per_cu = 1;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cus < 1) cus = 1;
  // Work items: (segment, cell tile, split), largest first.  A tile whose cost exceeds a
  // third of a workgroup's fair share is split over several workgroups (its work units
  // dealt round-robin, as in a small-batch launch), so that the last items are short.
  double total = 0.0;
  for (int i = 0; i < nseg; ++i) total += seg_cost[i] * (double)seg_tiles[i];
  const double target = total / (3.0 * (double)per_cu * (double)cus);
  std::vector<std::pair<double, int64_t>> items;
  for (int i = 0; i < nseg; ++i) {
    int ns = 1;
    if (target > 0.0 && seg_cost[i] > target) {
      const int cap = std::max(1, std::min(255, seg_units[i] / 4));
      ns = (int)std::min<double>(cap, std::ceil(seg_cost[i] / target));
    }
    descs[i].p.nsplit = ns;
    for (int64_t t = 0; t < seg_tiles[i]; ++t)
      for (int sp = 0; sp < ns; ++sp)
        items.push_back({seg_cost[i] / ns, ((int64_t)i << 48) | ((int64_t)sp << 40) | t});
  }
  if (items.size() > 0x7fffffffULL) return plan_fail(WEFQ_EINVAL, "too many work items");
  std::stable_sort(items.begin(), items.end(),
                   [](const std::pair<double, int64_t>& a, const std::pair<double, int64_t>& b) { return a.first > b.first; });
  wefq_plan_s* pl = new (std::nothrow) wefq_plan_s();
  if (!pl) return plan_fail(WEFQ_ENOMEM, "host allocation failed");
  pl->device = device; pl->mode = mode; pl->block = block; pl->lds = lds; pl->nitems = (int)items.size();
  std::vector<int64_t> codes(items.size());
  for (size_t i = 0; i < items.size(); ++i) codes[i] = items[i].second;
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
