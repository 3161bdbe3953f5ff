// Per-tile angular-first contraction shared by the standalone and persistent
// apply kernels (see apply.hip for the design notes).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "wefq_core.h"

namespace wefq {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef __bf16 v2bf __attribute__((ext_vector_type(2)));
typedef float v2f __attribute__((ext_vector_type(2)));

struct MfmaParams {
  const void* f;
  const void* g;           // second input of the Jacobian-vector product (unused otherwise)
  void* Q;
  int64_t B, ldf, ldg, ldq;
  int NK, NQ, N;
  int nunits;
  int nsplit;              // workgroups sharing one cell tile; each takes every nsplit-th unit
  const int* units;        // [nunits][UNIT_STRIDE]: l1, count, q1 values
  const int* chan_begin;   // [L+2]
  const int* slice_off;    // [NTm]
  const int* sptr;         // slices + 1
  const int* spair;        // per slice: first single row; rows [sptr[s], spair[s]) are q2 pairs
  const uint32_t* mq;      // [rows][2]: q2*NKp, q3*NKp, the LDS row offsets of the two gathered states
                           // (swapped in the second row of a pair: a pair reads as u, a, b, u)
  const uint32_t* mq_pad;  // the same with the padded row pitch (tiles with a pad row per block)
  const float* mg;         // merged weights (FP32 / BF16X3)
  const double* mg64;      // merged weights (FP64)
  const float* Rt32;       // [NTm][ceil(H*H/4)][64][4]: rows k1 < 16 in the MFMA A-operand
                           // layout, 4 steps t per lane and load
  const double* Rt64;      // [NTm][ceil(H*H/2)][64][2]
  const uint16_t* Rhi;     // [NTm][U][64][8]
  const uint16_t* Rlo;
  const float* R16_32;     // NK = 17 only: row k1 = 16 of R per lane group, [NTm][4][4 ceil(H*H/4)]
  const double* R16_64;
};

// output states per work unit (the same for every quadrant size)
__host__ __device__ constexpr int gq_for(int) { return kUnitStates; }

typedef double v4d __attribute__((ext_vector_type(4)));
typedef double v2d __attribute__((ext_vector_type(2)));

// MODE 0: FP32 MFMA, 1: split BF16x3 MFMA, 2: FP64 MFMA.
template <int MODE> struct ModeTraits;
template <> struct ModeTraits<0> { typedef float T; typedef v4f acc_t; };
template <> struct ModeTraits<1> { typedef float T; typedef v4f acc_t; };
template <> struct ModeTraits<2> { typedef double T; typedef v4d acc_t; };

// The LDS rows one coupling step reads: the q2 row u and the q3 rows a (and b for a
// pair) of the first input; with two inputs also the same rows of the second (g).
template <typename T, int H, bool TWO>
struct Rows {
  T u[H], a[H], b[H];
  T ug[TWO ? H : 1], ag[TWO ? H : 1], bg[TWO ? H : 1];
};

// Phi += u (x) w (or Phi -= u (x) w) over an H x H quadrant.
template <int H, bool NEG = false, typename T>
__device__ __forceinline__ void outer_product(T* phi, const T* u, const T* w) {
#pragma unroll
  for (int a = 0; a < H; ++a)
#pragma unroll
    for (int b = 0; b < H; ++b) phi[a * H + b] = fma(NEG ? -u[a] : u[a], w[b], phi[a * H + b]);
}

// One cell tile: stage f, then process the (l1, q1-group) work units split, split + nsplit, ...
// (all of them when nsplit = 1).  Each output row belongs to one unit, so splitting a tile
// over several workgroups changes neither the work per row nor its order.
// WAVES: waves per workgroup the instance is built for, 8, 12 (three per SIMD, which leaves each
// lane 168 registers: the 12-wave instances hoist the R tile only up to 6x6 quadrants) or 16
// (four per SIMD, 128 registers; quadrants up to 5x5).
// PAD_ALL: the tile layout's pad rows in tiles of every width (false: 16-cell tiles only).
// AHEAD: FP32 tiles whose R tile streams load each batch of it one batch ahead of its MFMAs
// (the persistent plan kernel: 2% faster there; the standalone kernel at K = L = 12 ran 12%
// slower with it).
// TWO: two inputs f, g; the coupling is symmetric, sum w (f_x (x) g_y + g_x (x) f_y), or with
// ANTI antisymmetric, sum w (f_x (x) g_y - g_x (x) f_y), contracted with the tiles the caller
// passes as the A operand, and the result combined as out = (out + result) / 2.
template <int H, int SLOTS, int RT, int MODE, bool TWO = false, bool ANTI = false, int WAVES = 8,
          bool PAD_ALL = true, bool AHEAD = false>
__device__ __forceinline__ void mfma_tile(const MfmaParams& p, int64_t tile, int split, unsigned char* lds_raw,
                                          int* unit_ctr_p) {
  typedef typename ModeTraits<MODE>::T T;
  typedef typename ModeTraits<MODE>::acc_t acc_t;
  constexpr int TB = 16 / SLOTS;
  constexpr int HH = H * H;
  constexpr int U = (HH + 7) / 8;
  constexpr int Q4 = (HH + 3) / 4, Q2 = (HH + 1) / 2;   // vector loads of the A-operand tiles
  constexpr int GQ = gq_for(H);
  constexpr int NP = GQ / SLOTS > 0 ? GQ / SLOTS : 1;
  // The two-buffer coupling pipeline (below) where it was measured faster: FP32 at quadrants
  // of 6 to 8 and BF16x3 from 6 up, one input.  It costs 3H (pairs) more registers, which
  // spill in FP64, cost occupancy below 6x6, and made FP32 at 9x9 slower (K = L = 16: 73.3
  // against 62.6 ms).
  constexpr bool PIPE = !TWO && ((MODE == 0 && H >= 6 && H <= 8) || (MODE == 1 && H >= 6));
  T* fs = reinterpret_cast<T*>(lds_raw);
  int& unit_ctr = *unit_ctr_p;
  T* Qo = static_cast<T*>(p.Q);
  const int NK = p.NK;
  const int64_t cell0 = tile * TB;
  // stage the coefficient tile: fs[(q * NKp + k + pd * (k >= H)) * TB + cell], with the
  // zero pad and tail rows of the layout described with tile_upper_row
  // (with two inputs the second tile follows the first, gofs elements later)
  const int pd = tile_pad_rows(NK, H, TB, PAD_ALL);
  const int NKp = NK + pd;
  const int tail = tile_tail_rows(NK, H);
  const int gofs = TWO ? (p.NQ * NKp + tail) * TB : 0;
#pragma unroll
  for (int in = 0; in < (TWO ? 2 : 1); ++in) {
    const T* src = static_cast<const T*>(in ? p.g : p.f);
    const int64_t ld = in ? p.ldg : p.ldf;
    T* dst = fs + in * gofs;
    for (int idx = threadIdx.x; idx < TB * p.N; idx += blockDim.x) {
      const int cl = idx / p.N, n = idx - cl * p.N;
      const int q = n / NK, k = n - q * NK;
      const int64_t cell = cell0 + cl;
      dst[(q * NKp + k + (k >= H ? pd : 0)) * TB + cl] = (cell < p.B) ? src[cell * ld + n] : T(0);
    }
    if (pd)
      for (int idx = threadIdx.x; idx < TB * p.NQ; idx += blockDim.x) {
        const int q = idx / TB, cl = idx - q * TB;
        dst[(q * NKp + H) * TB + cl] = T(0);
      }
    if (tail && threadIdx.x < TB) dst[p.NQ * NKp * TB + threadIdx.x] = T(0);
  }
  if (threadIdx.x == 0) unit_ctr = 0;
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int r = lane >> 4, j = lane & 15;
  const int h2 = r >> 1, h3 = r & 1;
  const int cellj = j % TB, slot = j / TB;
  // lane group r covers the rows [k2s, k2s+H) for k2 and [k3s, k3s+H) for k3 of every
  // q block: the lower half starts at row 0, the upper half at tile_upper_row (the R
  // tile gives zero weight to its rows outside [H, NK)), so every gather is a per-lane
  // base plus a compile-time offset.
  const int up = tile_upper_row(NK, H, TB, PAD_ALL);
  const int k2s = h2 ? up : 0, k3s = h3 ? up : 0;
  const T* lane_u = fs + k2s * TB + cellj;
  const T* lane_w = fs + k3s * TB + cellj;
  // read-only routing rows: through the constant address space so that
  // wave-uniform rows are fetched with scalar loads
  typedef const __attribute__((address_space(4))) uint32_t cu32;
  typedef const __attribute__((address_space(4))) float cf32;
  typedef const __attribute__((address_space(4))) double cf64;
  // (the work-unit and slice tables too: their indices are wave-uniform, and scalar
  // loads keep them off the vector-memory counter that the R-tile loads occupy)
  typedef const __attribute__((address_space(4))) int ci32;
  ci32* units = (ci32*)p.units;
  ci32* chan_begin = (ci32*)p.chan_begin;
  ci32* slice_off = (ci32*)p.slice_off;
  ci32* sptr = (ci32*)p.sptr;
  ci32* spair = (ci32*)p.spair;
  cu32* mq = (cu32*)(pd ? p.mq_pad : p.mq);
  cf32* mg = (cf32*)p.mg;
  cf64* mg64 = (cf64*)p.mg64;
  // the same rows through vector loads: an offset the compiler cannot prove uniform (a zero
  // produced by a register move it cannot see through) makes every access a vector load
  // (indexing a uniform base with a lane-varying 32-bit index lets the loads use a scalar base
  // and a 32-bit vector offset)
  // (the pipelined loops walk them with running pointers, one add per pointer and step)
  int vz;
  asm volatile("v_mov_b32 %0, 0" : "=v"(vz));
  const uint32_t* mqv = (pd ? p.mq_pad : p.mq) + vz;   // two words per row
  const T* mgv = (MODE == 2 ? reinterpret_cast<const T*>(p.mg64) : reinterpret_cast<const T*>(p.mg)) + vz;
  while (true) {
    int u = 0;
    if (lane == 0) u = atomicAdd(&unit_ctr, 1);
    u = __builtin_amdgcn_readfirstlane(__shfl(u, 0)) * p.nsplit + split;
    if (u >= p.nunits) break;
    // unit record: l1, count, then the unit's q1 values; with several output states
    // per MFMA column group, consecutive entries hold m1 and -m1, whose slices have
    // similar lengths, so the masked coupling loops waste little
    const int ub = UNIT_STRIDE * u;
    const int l1 = units[ub], nq = units[ub + 1];
    // RT == 2 marks NK = 17: rows 0..15 on MFMA, row 16 as a VALU dot product
    acc_t acc[NP];
    T acc16[NP];
#pragma unroll
    for (int gi = 0; gi < NP; ++gi) { acc[gi] = (acc_t){0, 0, 0, 0}; acc16[gi] = T(0); }
    const int cb = chan_begin[l1], ce = chan_begin[l1 + 1];
    for (int ct = cb; ct < ce; ++ct) {
      const int soff = slice_off[ct] - l1 * l1;
      // The channel's R tile is the MFMA A operand for every q1 of the unit.  When
      // registers allow, it is loaded once per channel ahead of the first coupling,
      // so its latency hides behind the VALU work; otherwise it streams in batches.
      constexpr bool HOIST = MODE == 2 ? (H <= 4) : (H <= (WAVES > 8 ? 6 : 7));
      float a32[HOIST && MODE == 0 ? Q4 * 4 : 1];
      double a64[HOIST && MODE == 2 ? Q2 * 2 : 1];
      v8bf ahi[HOIST && MODE == 1 ? U : 1], alo[HOIST && MODE == 1 ? U : 1];
      if constexpr (HOIST && MODE == 0) {
        const v4f* At = reinterpret_cast<const v4f*>(p.Rt32) + (int64_t)ct * Q4 * 64 + lane;
#pragma unroll
        for (int q = 0; q < Q4; ++q) {
          const v4f x = At[q * 64];
#pragma unroll
          for (int i = 0; i < 4; ++i) a32[4 * q + i] = x[i];
        }
      } else if constexpr (HOIST && MODE == 2) {
        const v2d* At = reinterpret_cast<const v2d*>(p.Rt64) + (int64_t)ct * Q2 * 64 + lane;
#pragma unroll
        for (int q = 0; q < Q2; ++q) {
          const v2d x = At[q * 64];
          a64[2 * q] = x[0];
          a64[2 * q + 1] = x[1];
        }
      } else if constexpr (HOIST && MODE == 1) {
#pragma unroll
        for (int uu8 = 0; uu8 < U; ++uu8) {
          const int64_t off = (((int64_t)ct * U + uu8) * 64 + lane) * 8;
          ahi[uu8] = *reinterpret_cast<const v8bf*>(p.Rhi + off);
          alo[uu8] = *reinterpret_cast<const v8bf*>(p.Rlo + off);
        }
      }
#pragma unroll
      for (int gi = 0; gi < NP; ++gi) {
        if (gi * SLOTS >= nq) break;
        // The first batch of a streamed FP32 R tile is loaded before the coupling and stays in
        // flight during it (up to 7x7 quadrants; at 8x8 and 9x9 the 12-wave kernels spill with
        // it).  K = L = 12 with 65,536 cells 37.6 -> 36.8 ms, K = L = 13 15.5 -> 15.2 ms.
        constexpr bool FIRST = MODE == 0 && !HOIST && !AHEAD && H <= 7;
        v4f first0 = (v4f){0, 0, 0, 0}, first1 = (v4f){0, 0, 0, 0};
        if constexpr (FIRST) {
          const v4f* At = reinterpret_cast<const v4f*>(p.Rt32) + (int64_t)ct * Q4 * 64 + lane;
          first0 = At[0];
          if (4 < HH) first1 = At[64];
        }
        T phi[U * 8];
#pragma unroll
        for (int t = 0; t < U * 8; ++t) phi[t] = T(0);
        // The slice's rows come as pairs sharing q2, then single rows.  A pair adds
        // f_{k2,q2} (g_a f_{k3,q3a} + g_b f_{k3,q3b}) to Phi: one outer product for
        // two rows.  A single adds (g f_{k2,q2}) f_{k3,q3}.  With two inputs c, d (the
        // Jacobian-vector product) each product x (x) y becomes c_x (x) d_y + d_x (x) c_y.
        auto weight = [&](int e) -> T { return MODE == 2 ? (T)mg64[e] : (T)mg[e]; };
        // A step's routing: the LDS row offsets of the q2 row (u) and of the q3 rows (a, and b
        // for a pair), each a word of its own, so that an address is one shift-and-add from
        // the lane's base; and the weights.
        struct Route { uint32_t u, a, b; T ga, gb; };
        auto gather = [&](const Route& rt, Rows<T, H, TWO>& x, bool pair) {
          const T* pu = lane_u + (int)rt.u * TB;
          const T* pa = lane_w + (int)rt.a * TB;
          const T* pb = lane_w + (int)rt.b * TB;
#pragma unroll
          for (int a = 0; a < H; ++a) {
            x.u[a] = pu[a * TB];
            x.a[a] = pa[a * TB];
            if (pair) x.b[a] = pb[a * TB];
            if constexpr (TWO) {
              x.ug[a] = pu[gofs + a * TB];
              x.ag[a] = pa[gofs + a * TB];
              if (pair) x.bg[a] = pb[gofs + a * TB];
            }
          }
        };
        auto pair_acc = [&](T ga, T gb, const Rows<T, H, TWO>& x) {
          T wf[H];
#pragma unroll
          for (int b = 0; b < H; ++b) wf[b] = fma(gb, x.b[b], ga * x.a[b]);
          if constexpr (TWO) {
            T wg[H];
#pragma unroll
            for (int b = 0; b < H; ++b) wg[b] = fma(gb, x.bg[b], ga * x.ag[b]);
            outer_product<H>(phi, x.u, wg);
            outer_product<H, ANTI>(phi, x.ug, wf);
          } else {
            outer_product<H>(phi, x.u, wf);
          }
        };
        auto single_acc = [&](T gg, const Rows<T, H, TWO>& x) {
          T uu[H];
#pragma unroll
          for (int a = 0; a < H; ++a) uu[a] = gg * x.u[a];
          if constexpr (TWO) {
            T ug[H];
#pragma unroll
            for (int a = 0; a < H; ++a) ug[a] = gg * x.ug[a];
            outer_product<H>(phi, uu, x.ag);
            outer_product<H, ANTI>(phi, ug, x.a);
          } else {
            outer_product<H>(phi, uu, x.a);
          }
        };
        // Software pipeline over the slice's rows: two row buffers, A and B, alternate, so
        // that while one accumulates its outer product the LDS gathers of the other are in
        // flight (the loops are unrolled by two rows or pairs, with scheduling barriers that
        // keep each gather ahead of the previous row's arithmetic).  The routing rows (offsets
        // and weights) come through vector loads two rows ahead: a scalar load there would
        // share the LDS counter, and every wait for it would also wait for all gathers in
        // flight.  The arrays carry 8 entries of tail slack (row offset 0, weight 0).
        // maxrows: steps (rows or pairs) of the longest slice among the wave's lanes; fetch(i, rt):
        // routing of step i of this lane's slice (zero weight past its end); pair: two rows per step.
        auto pipeline = [&](int maxrows, auto fetch, bool pair) {
          if (maxrows <= 0) return;
          Route r0, r1;
          fetch(0, r0);
          fetch(1, r1);
          Rows<T, H, TWO> A, B;
          gather(r0, A, pair);
          int i = 0;
          for (; i + 1 < maxrows; i += 2) {
            Route r2, r3;
            fetch(i + 2, r2);
            gather(r1, B, pair);
            __builtin_amdgcn_sched_barrier(0);
            if (pair) pair_acc(r0.ga, r0.gb, A); else single_acc(r0.ga, A);
            __builtin_amdgcn_sched_barrier(0);
            fetch(i + 3, r3);
            gather(r2, A, pair);
            __builtin_amdgcn_sched_barrier(0);
            if (pair) pair_acc(r1.ga, r1.gb, B); else single_acc(r1.ga, B);
            __builtin_amdgcn_sched_barrier(0);
            r0 = r2;
            r1 = r3;
          }
          if (i < maxrows) {
            if (pair) pair_acc(r0.ga, r0.gb, A); else single_acc(r0.ga, A);
          }
        };
        if constexpr (PIPE && SLOTS == 1) {     // the slice is shared by the whole wave
          const int s = soff + units[ub + 2 + gi];
          const int e0 = sptr[s], e1 = sptr[s + 1], ep = spair[s];
          const int np_ = (ep - e0) >> 1, ns_ = e1 - ep;
          // rows are fetched in order, up to two steps past the end (within the table's slack);
          // a pair is rows (q2, q3a), (q2, q3b), stored as words u, a, b, u
          const uint32_t* pq = mqv + 2 * e0;
          const T* pw = mgv + e0;
          pipeline(np_, [&](int, Route& rt) {
            rt.u = pq[0]; rt.a = pq[1]; rt.b = pq[2]; rt.ga = pw[0]; rt.gb = pw[1];
            pq += 4; pw += 2;
          }, true);
          pq = mqv + 2 * ep;
          pw = mgv + ep;
          pipeline(ns_, [&](int, Route& rt) {
            rt.u = pq[0]; rt.a = pq[1]; rt.b = 0u; rt.ga = pw[0]; rt.gb = T(0);
            pq += 2; pw += 1;
          }, false);
        } else if constexpr (PIPE) {
          // Lanes of different output states walk different slices: every lane fetches its
          // own slot's rows (lane-varying addresses, vector loads); the loops run to the
          // longest slot, and rows past a slot's end carry weight zero and row offset 0.
          int se0[SLOTS], sep[SLOTS], se1[SLOTS];
          int maxp = 0, maxs = 0;
#pragma unroll
          for (int sl = 0; sl < SLOTS; ++sl) {
            const int qs = gi * SLOTS + sl;
            se0[sl] = se1[sl] = sep[sl] = 0;
            if (qs < nq) {
              const int ss = soff + units[ub + 2 + qs];
              se0[sl] = sptr[ss];
              se1[sl] = sptr[ss + 1];
              sep[sl] = spair[ss];
            }
            const int np_s = (sep[sl] - se0[sl]) >> 1, ns_s = se1[sl] - sep[sl];
            maxp = maxp > np_s ? maxp : np_s;
            maxs = maxs > ns_s ? maxs : ns_s;
          }
          int my0 = 0, myp = 0, my1 = 0;
#pragma unroll
          for (int sl = 0; sl < SLOTS; ++sl)
            if (slot == sl) { my0 = se0[sl]; myp = sep[sl]; my1 = se1[sl]; }
          const int my_np = (myp - my0) >> 1, my_ns = my1 - myp;
          // each lane's pointers stop at the end of its slot's rows, where they still read
          // valid table entries (the slot's singles, the next slice, or the slack); those
          // reads are masked
          const uint32_t* pq = mqv + 2 * my0;
          const T* pw = mgv + my0;
          pipeline(maxp, [&](int i, Route& rt) {
            const bool in = i < my_np;
            const uint32_t xu = pq[0], xa = pq[1], xb = pq[2];
            const T ya = pw[0], yb = pw[1];
            rt.u = in ? xu : 0u; rt.a = in ? xa : 0u; rt.b = in ? xb : 0u;
            rt.ga = in ? ya : T(0); rt.gb = in ? yb : T(0);
            pq += in ? 4 : 0; pw += in ? 2 : 0;
          }, true);
          pq = mqv + 2 * myp;
          pw = mgv + myp;
          pipeline(maxs, [&](int i, Route& rt) {
            const bool in = i < my_ns;
            const uint32_t xu = pq[0], xa = pq[1];
            const T ya = pw[0];
            rt.u = in ? xu : 0u; rt.a = in ? xa : 0u; rt.b = 0u; rt.ga = in ? ya : T(0); rt.gb = T(0);
            pq += in ? 2 : 0; pw += in ? 1 : 0;
          }, false);
        } else if constexpr (SLOTS == 1) {
          // Without the two row buffers (where registers do not allow them): one row's
          // gathers ahead, routing rows through scalar loads
          const int s = soff + units[ub + 2 + gi];
          const int e0 = sptr[s], e1 = sptr[s + 1], ep = spair[s];
          // software pipeline: the gathers of the next row (pair) are in flight
          // while the outer product of the current one accumulates (the arrays
          // carry tail slack, whose row offsets point at LDS row 0)
          auto pair_route = [&](int e) {
            return Route{mq[2 * e], mq[2 * e + 1], mq[2 * e + 2], weight(e), weight(e + 1)};
          };
          auto single_route = [&](int e) { return Route{mq[2 * e], mq[2 * e + 1], 0u, weight(e), T(0)}; };
          if (e0 < ep) {
            Route rc = pair_route(e0);
            Rows<T, H, TWO> cur;
            gather(rc, cur, true);
            for (int e = e0; e < ep; e += 2) {
              const Route rn = pair_route(e + 2);
              Rows<T, H, TWO> nxt;
              gather(rn, nxt, true);
              pair_acc(rc.ga, rc.gb, cur);
              cur = nxt;
              rc = rn;
            }
          }
          if (ep < e1) {
            Route rc = single_route(ep);
            Rows<T, H, TWO> cur;
            gather(rc, cur, false);
            for (int e = ep; e < e1; ++e) {
              const Route rn = single_route(e + 1);
              Rows<T, H, TWO> nxt;
              gather(rn, nxt, false);
              single_acc(rc.ga, cur);
              cur = nxt;
              rc = rn;
            }
          }
        } else {
          // Lanes of different output states walk different slices: every lane fetches its
          // own slot's rows through vector loads, walking running pointers that stop at the
          // end of the slot's rows (where they still read valid entries: the slot's singles,
          // the next slice, or the table's slack) and masking past it; the loops run to the
          // longest slot, and rows past a slot's end carry weight zero and row offset 0 (all
          // such lanes then read the same LDS row: a broadcast, not a bank conflict).
          int se0[SLOTS], sep[SLOTS], se1[SLOTS];
          int maxp = 0, maxs = 0;
#pragma unroll
          for (int sl = 0; sl < SLOTS; ++sl) {
            const int qs = gi * SLOTS + sl;
            se0[sl] = se1[sl] = sep[sl] = 0;
            if (qs < nq) {
              const int ss = soff + units[ub + 2 + qs];
              se0[sl] = sptr[ss];
              se1[sl] = sptr[ss + 1];
              sep[sl] = spair[ss];
            }
            const int np_s = (sep[sl] - se0[sl]) >> 1, ns_s = se1[sl] - sep[sl];
            maxp = maxp > np_s ? maxp : np_s;
            maxs = maxs > ns_s ? maxs : ns_s;
          }
          int my0 = 0, myp = 0, my1 = 0;
#pragma unroll
          for (int sl = 0; sl < SLOTS; ++sl)
            if (slot == sl) { my0 = se0[sl]; myp = sep[sl]; my1 = se1[sl]; }
          const int my_np = (myp - my0) >> 1, my_ns = my1 - myp;
          const uint32_t* pqp = mqv + 2 * my0;
          const T* pwp = mgv + my0;
          const uint32_t* pqs = mqv + 2 * myp;
          const T* pws = mgv + myp;
          auto fetch_pair = [&](int i, Route& rt) {
            const bool in = i < my_np;
            const uint32_t xu = pqp[0], xa = pqp[1], xb = pqp[2];
            const T ya = pwp[0], yb = pwp[1];
            rt.u = in ? xu : 0u; rt.a = in ? xa : 0u; rt.b = in ? xb : 0u;
            rt.ga = in ? ya : T(0); rt.gb = in ? yb : T(0);
            pqp += in ? 4 : 0; pwp += in ? 2 : 0;
          };
          auto fetch_single = [&](int i, Route& rt) {
            const bool in = i < my_ns;
            const uint32_t xu = pqs[0], xa = pqs[1];
            const T y = pws[0];
            rt.u = in ? xu : 0u; rt.a = in ? xa : 0u; rt.b = 0u; rt.ga = in ? y : T(0); rt.gb = T(0);
            pqs += in ? 2 : 0; pws += in ? 1 : 0;
          };
          if (maxp > 0) {
            Route rc;
            Rows<T, H, TWO> cur;
            fetch_pair(0, rc);
            gather(rc, cur, true);
            for (int i = 0; i < maxp; ++i) {
              Route rn;
              Rows<T, H, TWO> nxt;
              fetch_pair(i + 1, rn);
              gather(rn, nxt, true);
              pair_acc(rc.ga, rc.gb, cur);
              cur = nxt;
              rc = rn;
            }
          }
          if (maxs > 0) {
            Route rc;
            Rows<T, H, TWO> cur;
            fetch_single(0, rc);
            gather(rc, cur, false);
            for (int i = 0; i < maxs; ++i) {
              Route rn;
              Rows<T, H, TWO> nxt;
              fetch_single(i + 1, rn);
              gather(rn, nxt, false);
              single_acc(rc.ga, cur);
              cur = nxt;
              rc = rn;
            }
          }
        }
        // Radial contraction of the slice on the matrix cores.  The wave raises its
        // issue priority for the MFMA block, so the matrix core is refilled promptly
        // while the other wave of the SIMD issues its coupling VALU work; the priority
        // switches also keep the compiler from hoisting this block's operand
        // preparation into the coupling loops (which spills registers at H = 9).
        __builtin_amdgcn_s_setprio(1);
        if constexpr (HOIST && MODE == 0) {
#pragma unroll
          for (int t = 0; t < HH; ++t)
            acc[gi] = __builtin_amdgcn_mfma_f32_16x16x4f32(a32[t], phi[t], acc[gi], 0, 0, 0);
        } else if constexpr (HOIST && MODE == 2) {
#pragma unroll
          for (int t = 0; t < HH; ++t)
            acc[gi] = __builtin_amdgcn_mfma_f64_16x16x4f64(a64[t], phi[t], acc[gi], 0, 0, 0);
        } else if constexpr (MODE == 0 && AHEAD) {
          // the streamed R tile, 8 steps per batch, the next batch's loads issued ahead of the
          // current batch's MFMAs
          const v4f* At = reinterpret_cast<const v4f*>(p.Rt32) + (int64_t)ct * Q4 * 64 + lane;
          v4f x0 = At[0];
          v4f x1 = (4 < HH) ? At[64] : (v4f){0, 0, 0, 0};
#pragma unroll
          for (int t0 = 0; t0 < HH; t0 += 8) {
            v4f n0 = (v4f){0, 0, 0, 0}, n1 = (v4f){0, 0, 0, 0};
            if (t0 + 8 < HH) n0 = At[((t0 + 8) / 4) * 64];
            if (t0 + 12 < HH) n1 = At[((t0 + 8) / 4 + 1) * 64];
            float av[8];
#pragma unroll
            for (int t = 0; t < 4; ++t) { av[t] = x0[t]; av[t + 4] = x1[t]; }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int t = 0; t < 8; ++t)
              if (t0 + t < HH) acc[gi] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[t], phi[t0 + t], acc[gi], 0, 0, 0);
            x0 = n0;
            x1 = n1;
          }
        } else if constexpr (MODE == 0) {
          const v4f* At = reinterpret_cast<const v4f*>(p.Rt32) + (int64_t)ct * Q4 * 64 + lane;
#pragma unroll
          for (int t0 = 0; t0 < HH; t0 += 8) {
            float av[8];
            const v4f x0 = (FIRST && t0 == 0) ? first0 : At[(t0 / 4) * 64];
            const v4f x1 = (FIRST && t0 == 0) ? first1 : (t0 + 4 < HH) ? At[(t0 / 4 + 1) * 64] : (v4f){0, 0, 0, 0};
#pragma unroll
            for (int t = 0; t < 4; ++t) { av[t] = x0[t]; av[t + 4] = x1[t]; }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int t = 0; t < 8; ++t)
              if (t0 + t < HH) acc[gi] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[t], phi[t0 + t], acc[gi], 0, 0, 0);
          }
        } else if constexpr (MODE == 2) {
          const v2d* At = reinterpret_cast<const v2d*>(p.Rt64) + (int64_t)ct * Q2 * 64 + lane;
#pragma unroll
          for (int t0 = 0; t0 < HH; t0 += 8) {
            double av[8];
#pragma unroll
            for (int t = 0; t < 8; t += 2) {
              const v2d x = (t0 + t < HH) ? At[((t0 + t) / 2) * 64] : (v2d){0.0, 0.0};
              av[t] = x[0];
              av[t + 1] = x[1];
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int t = 0; t < 8; ++t)
              if (t0 + t < HH) acc[gi] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[t], phi[t0 + t], acc[gi], 0, 0, 0);
          }
        } else {
          // the streamed hi/lo R tiles, the next step's loads issued ahead of the current
          // step's MFMAs (against loads in the step: K = L = 12 with 65,536 cells 32.3 -> 31.6 ms,
          // K = L = 14 with 16,384 cells 23.2 -> 22.1 ms, K = L = 10 1.5% slower)
          const int64_t off0 = ((int64_t)ct * U * 64 + lane) * 8;
          v8bf ahn = HOIST ? ahi[0] : *reinterpret_cast<const v8bf*>(p.Rhi + off0);
          v8bf aln = HOIST ? alo[0] : *reinterpret_cast<const v8bf*>(p.Rlo + off0);
#pragma unroll
          for (int uu8 = 0; uu8 < U; ++uu8) {
            const v8bf ah = ahn, al = aln;
            if (uu8 + 1 < U) {
              const int64_t offn = off0 + (int64_t)(uu8 + 1) * 64 * 8;
              ahn = HOIST ? ahi[HOIST ? uu8 + 1 : 0] : *reinterpret_cast<const v8bf*>(p.Rhi + offn);
              aln = HOIST ? alo[HOIST ? uu8 + 1 : 0] : *reinterpret_cast<const v8bf*>(p.Rlo + offn);
            }
            // split hi/lo two values at a time: one packed round-to-nearest conversion gives
            // both hi halves, which are unpacked back to FP32 by a shift and a mask
            v8bf bh, bl;
#pragma unroll
            for (int e = 0; e < 8; e += 2) {
              const float x0 = phi[uu8 * 8 + e], x1 = phi[uu8 * 8 + e + 1];
              const v2bf h = __builtin_convertvector((v2f){x0, x1}, v2bf);
              const uint32_t hb = __builtin_bit_cast(uint32_t, h);
              const float h0 = __builtin_bit_cast(float, hb << 16);
              const float h1 = __builtin_bit_cast(float, hb & 0xffff0000u);
              const v2bf l = __builtin_convertvector((v2f){x0 - h0, x1 - h1}, v2bf);
              bh[e] = h[0]; bh[e + 1] = h[1];
              bl[e] = l[0]; bl[e + 1] = l[1];
            }
            acc[gi] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc[gi], 0, 0, 0);
            acc[gi] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc[gi], 0, 0, 0);
            acc[gi] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc[gi], 0, 0, 0);
          }
        }
        __builtin_amdgcn_s_setprio(0);
        if constexpr (RT == 2) {
          // row k1 = 16: partial dot product over this lane group's quadrant, then
          // the four lane groups of a column (lanes j, j+16, j+32, j+48) are summed
          T part = T(0);
          // (the row is padded to 4 ceil(HH/4) values, so whole vectors load)
          if constexpr (MODE == 2) {
            const v2d* r16 = reinterpret_cast<const v2d*>(p.R16_64 + ((int64_t)ct * 4 + r) * (Q4 * 4));
#pragma unroll
            for (int q = 0; q < Q2; ++q) {
              const v2d x = r16[q];
              part = fma(x[0], phi[2 * q], part);
              if (2 * q + 1 < HH) part = fma(x[1], phi[2 * q + 1], part);
            }
          } else {
            const v4f* r16 = reinterpret_cast<const v4f*>(p.R16_32 + ((int64_t)ct * 4 + r) * (Q4 * 4));
#pragma unroll
            for (int q = 0; q < Q4; ++q) {
              const v4f x = r16[q];
#pragma unroll
              for (int i = 0; i < 4; ++i)
                if (4 * q + i < HH) part = fma((T)x[i], phi[4 * q + i], part);
            }
          }
          part += __shfl_xor(part, 16);
          part += __shfl_xor(part, 32);
          acc16[gi] += part;
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
      const int q1 = units[ub + 2 + qi];
      T* dst = Qo + cell * p.ldq + (int64_t)q1 * NK;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int k1 = MODE == 2 ? r + 4 * i : 4 * r + i;
        if (k1 < NK) {
          T v = (T)acc[gi][i];
          // The invariant rows of Q(f, f) and J(c) d come out exactly 0 from the core, whose
          // invariant rows are zero (every product there is 0 x finite), so they are stored as
          // computed and the conservation check tests the zeroing.  The antisymmetric part keeps
          // its momentum and energy rows; its mass row, zero only up to rounding in the unzeroed
          // core, is stored as 0.
          if constexpr (ANTI) dst[k1] = (q1 == 0 && k1 == 0) ? T(0) : T(0.5) * (dst[k1] + v);
          else dst[k1] = v;
        }
      }
      if (RT == 2 && r == 0) dst[16] = ANTI ? T(0.5) * (dst[16] + acc16[gi]) : acc16[gi];
    }
  }
}

}  // namespace wefq
