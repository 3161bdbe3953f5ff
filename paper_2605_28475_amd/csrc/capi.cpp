// C ABI of the wefq library: core construction, table preparation, dispatch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/wefq.h"
#include "wefq_core.h"

namespace wefq {

static thread_local std::string g_last_error;
void set_error(const std::string& msg) { g_last_error = msg; }

static uint16_t bf16_bits(float x) {       // round to nearest even
  uint32_t u;
  std::memcpy(&u, &x, 4);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
static float bf16_to_float(uint16_t b) {
  uint32_t u = (uint32_t)b << 16;
  float x;
  std::memcpy(&x, &u, 4);
  return x;
}

static void zero_invariants(wefq_core* h) {
  const int NK = h->NK;
  const size_t blk = (size_t)NK * NK * NK;
  for (int c = 0; c < h->NT; ++c) {
    double* R = h->R64.data() + c * blk;
    const Channel& ch = h->chans[c];
    if (ch.l1 == 0 || ch.l1 == 1)                      // mass (l1=0), momentum (l1=1): k1 = 0
      for (int i = 0; i < NK * NK; ++i) R[i] = 0.0;
    if (ch.l1 == 0 && NK > 1)                          // energy: k1 = 1
      for (int i = 0; i < NK * NK; ++i) R[NK * NK + i] = 0.0;
    if (ch.l1 == 0 && ch.l2 == 0 && ch.l3 == 0)        // detailed balance: R_{k1,0,0} = 0
      for (int k1 = 0; k1 < NK; ++k1) R[(size_t)k1 * NK * NK] = 0.0;
  }
}

template <typename T>
static bool upload(wefq_core* h, T*& dst, const std::vector<T>& src, hipStream_t s) {
  dst = dev_alloc<T>(h, src.size());
  if (!dst) { set_error("device allocation failed"); return false; }
  if (src.empty()) return true;
  // The source is often a block-scoped host vector that dies right after this call, and an
  // early return on a later failure destroys the rest: wait for the copy here, so that no
  // source has to outlive its call (a few dozen waits at build time).
  if (hipMemcpyAsync(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess) {
    set_error("host to device copy failed");
    return false;
  }
  return true;
}

// Split workgroups per compute unit for small batches (tile_splits): 2 where two workgroups
// of the mode's kernel fit on a compute unit at its tile shape and its quadrants are 4x4 or
// larger, else 1.  A second resident workgroup doubles the waves that hide the coupling's
// latency, at the price of staging each tile twice; measured at 4,096 cells it gained 14-15%
// at K = L = 8 and 2-7% at K = L = 6 (FP32, BF16x3) and lost 10-33% at K = L = 4, whose
// tiles are too small to repay the staging; where two do not fit (FP64 from 4x4 quadrants
// up, every precision from K = L = 10) the second workgroup only queues, and lost up to 70%.
static int split_target(const wefq_core* h, int mode) {
  if (h->slots[mode] == 0 || h->H < 4) return 1;
  return mfma_blocks_per_cu(h, mode, h->slots[mode], h->block[mode]) >= 2 ? 2 : 1;
}

// Workgroups of the mode's kernel resident per compute unit at its tile shape (at least 1).
static int resident_blocks(const wefq_core* h, int mode) {
  if (h->slots[mode] == 0) return 1;
  const int n = mfma_blocks_per_cu(h, mode, h->slots[mode], h->block[mode]);
  return n > 1 ? n : 1;
}

bool prepare_apply_tables(wefq_core* h, const std::vector<CooRow>& coo, hipStream_t s) {
  const int NK = h->NK, NQ = h->NQ, L = h->L;
  const size_t blk = (size_t)NK * NK * NK;
  // ---- FP64 plain path: rows grouped by q1 (stable: keeps channel order)
  std::vector<int> order(coo.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    if (coo[a].q1 != coo[b].q1) return coo[a].q1 < coo[b].q1;
    return coo[a].c < coo[b].c;
  });
  std::vector<int> q1ptr(NQ + 1, 0), ec(coo.size());
  std::vector<uint32_t> eq(coo.size());
  std::vector<double> eg(coo.size());
  for (size_t i = 0; i < order.size(); ++i) {
    const CooRow& r = coo[order[i]];
    q1ptr[r.q1 + 1]++;
    ec[i] = r.c;
    eq[i] = (uint32_t)r.q2 | ((uint32_t)r.q3 << 16);
    eg[i] = r.g;
  }
  for (int q = 0; q < NQ; ++q) q1ptr[q + 1] += q1ptr[q];
  if (!upload(h, h->dR64, h->R64, s) || !upload(h, h->d_q1ptr, q1ptr, s) || !upload(h, h->d_ent_c, ec, s) ||
      !upload(h, h->d_ent_q, eq, s) || !upload(h, h->d_ent_g, eg, s))
    return false;
  // ---- radial-first ordering: distinct (channel, q2, q3) groups in table order, and the
  // rows grouped by q1 (the order above) pointing at their group
  if (h->precisions & WEFQ_PREP_RADIAL) {
    std::unordered_map<int64_t, int> gid;
    gid.reserve(coo.size());
    std::vector<int> grp_c, row_grp(coo.size());
    std::vector<uint32_t> grp_q;
    std::vector<int> grp_of_row(coo.size());
    for (size_t z = 0; z < coo.size(); ++z) {
      const CooRow& r = coo[z];
      const int64_t key = ((int64_t)r.c * NQ + r.q2) * NQ + r.q3;
      auto it = gid.find(key);
      if (it == gid.end()) {
        it = gid.emplace(key, (int)grp_c.size()).first;
        grp_c.push_back(r.c);
        grp_q.push_back((uint32_t)r.q2 | ((uint32_t)r.q3 << 16));
      }
      grp_of_row[z] = it->second;
    }
    for (size_t i = 0; i < order.size(); ++i) row_grp[i] = grp_of_row[order[i]];
    h->rad_groups = (int)grp_c.size();
    if (!upload(h, h->d_rad_grp_c, grp_c, s) || !upload(h, h->d_rad_grp_q, grp_q, s) ||
        !upload(h, h->d_rad_q1ptr, q1ptr, s) || !upload(h, h->d_rad_row_grp, row_grp, s) ||
        !upload(h, h->d_rad_row_g, eg, s))
      return false;
  }
  // ---- merged channels (l2 <= l3), in paper order (sorted by l1)
  std::vector<int> cidx((L + 1) * (L + 1) * (L + 1), -1);
  for (int c = 0; c < h->NT; ++c) {
    const Channel& ch = h->chans[c];
    cidx[(ch.l1 * (L + 1) + ch.l2) * (L + 1) + ch.l3] = c;
  }
  std::vector<int> mchan;                      // paper channel of each merged channel
  std::vector<int> merged_of(h->NT, -1);
  for (int c = 0; c < h->NT; ++c)
    if (h->chans[c].l2 <= h->chans[c].l3) { merged_of[c] = (int)mchan.size(); mchan.push_back(c); }
  const int NTm = (int)mchan.size();
  h->NTm = NTm;
  std::vector<double> Rm((size_t)NTm * blk);
  for (int m = 0; m < NTm; ++m) {
    const Channel& ch = h->chans[mchan[m]];
    const double* Ra = h->R64.data() + (size_t)mchan[m] * blk;
    const double* Rb = ch.l2 < ch.l3 ? h->R64.data() + (size_t)cidx[(ch.l1 * (L + 1) + ch.l3) * (L + 1) + ch.l2] * blk : Ra;
    double sc = ch.l2 < ch.l3 ? 1.0 : 0.5;
    for (int k1 = 0; k1 < NK; ++k1)
      for (int k2 = 0; k2 < NK; ++k2)
        for (int k3 = 0; k3 < NK; ++k3)
          Rm[(size_t)m * blk + ((size_t)k1 * NK + k2) * NK + k3] =
              ch.l2 < ch.l3 ? Ra[((size_t)k1 * NK + k2) * NK + k3] + Rb[((size_t)k1 * NK + k3) * NK + k2]
                            : sc * (Ra[((size_t)k1 * NK + k2) * NK + k3] + Ra[((size_t)k1 * NK + k3) * NK + k2]);
  }
  // Antisymmetric partner of the merged core, for the bilinear form Q(f, g):
  // D = R^{(l1l2l3)}_{k1k2k3} - R^{(l1l3l2)}_{k1k3k2} (l2 < l3), (R_{k1k2k3} - R_{k1k3k2}) / 2 (l2 = l3),
  // so that Q(f, g) = (R~ Phi_S + D Phi_A) / 2 with Phi_S, Phi_A the symmetric and
  // antisymmetric two-input couplings.
  // D is built from the core before the invariant-row zeroing, except the mass row
  // (exactly zero for every pair of inputs); its momentum and energy rows carry the
  // part of Q(f, g) that is antisymmetric in f and g.
  const bool wantD = (h->precisions & WEFQ_PREP_BILINEAR) != 0;
  std::vector<double> Dm;
  if (wantD) {
    Dm.resize((size_t)NTm * blk);
    for (int m = 0; m < NTm; ++m) {
      const Channel& ch = h->chans[mchan[m]];
      const double* Ra = h->R64raw.data() + (size_t)mchan[m] * blk;
      const double* Rb = ch.l2 < ch.l3 ? h->R64raw.data() + (size_t)cidx[(ch.l1 * (L + 1) + ch.l3) * (L + 1) + ch.l2] * blk : Ra;
      const double sc = ch.l2 < ch.l3 ? 1.0 : 0.5;
      for (int k1 = 0; k1 < NK; ++k1)
        for (int k2 = 0; k2 < NK; ++k2)
          for (int k3 = 0; k3 < NK; ++k3)
            Dm[(size_t)m * blk + ((size_t)k1 * NK + k2) * NK + k3] =
                (ch.l1 == 0 && k1 == 0) ? 0.0 : sc * (Ra[((size_t)k1 * NK + k2) * NK + k3] - Rb[((size_t)k1 * NK + k3) * NK + k2]);
    }
  }
  std::vector<int> chan_begin(L + 2, 0);
  for (int m = 0; m < NTm; ++m) chan_begin[h->chans[mchan[m]].l1 + 1]++;
  for (int l = 0; l <= L; ++l) chan_begin[l + 1] += chan_begin[l];
  // slices (merged channel, m1) with merged rows
  std::vector<std::vector<std::pair<uint32_t, double>>> slices;
  std::vector<int> slice_off(NTm);
  for (int m = 0; m < NTm; ++m) {
    slice_off[m] = (int)slices.size();
    slices.resize(slices.size() + 2 * h->chans[mchan[m]].l1 + 1);
  }
  int ngm = 0;
  for (const CooRow& r : coo) {
    int m = merged_of[r.c];
    if (m < 0) continue;                        // carried by the partner channel
    const Channel& ch = h->chans[r.c];
    double g = r.g;
    if (ch.l2 == ch.l3) {
      if (r.q2 > r.q3) continue;
      if (r.q2 < r.q3) g *= 2.0;
    }
    // entries carry the LDS row offsets q*NK of the two gathered states
    slices[slice_off[m] + (r.q1 - ch.l1 * ch.l1)].push_back(
        {(uint32_t)(r.q2 * NK) | ((uint32_t)(r.q3 * NK) << 16), g});
    ++ngm;
  }
  // Within a slice, rows that share q2 are stored as consecutive pairs first (the
  // kernel folds a pair into one outer product: f_{.,q2} x (g_a f_{.,q3a} + g_b f_{.,q3b})),
  // then the remaining single rows; spair[s] is the first single row of slice s.
  std::vector<int> sptr(slices.size() + 1, 0), spair(slices.size(), 0);
  std::vector<uint32_t> mq;
  std::vector<float> mg;
  std::vector<double> mg64;
  int nsm = 0;
  typedef std::pair<uint32_t, double> Ent;
  for (size_t i = 0; i < slices.size(); ++i) {
    auto& sl = slices[i];
    std::sort(sl.begin(), sl.end(), [](const Ent& a, const Ent& b) {
      return (a.first & 0xffff) != (b.first & 0xffff) ? (a.first & 0xffff) < (b.first & 0xffff) : (a.first >> 16) < (b.first >> 16);
    });
    std::vector<Ent> singles;
    for (size_t a = 0; a < sl.size();) {
      size_t b = a;
      while (b < sl.size() && (sl[b].first & 0xffff) == (sl[a].first & 0xffff)) ++b;
      for (; a + 1 < b; a += 2)
        for (size_t t = a; t < a + 2; ++t) { mq.push_back(sl[t].first); mg.push_back((float)sl[t].second); mg64.push_back(sl[t].second); }
      if (a < b) singles.push_back(sl[a++]);
    }
    spair[i] = (int)mq.size();
    std::sort(singles.begin(), singles.end(), [](const Ent& a, const Ent& b) {
      return (a.first >> 16) != (b.first >> 16) ? (a.first >> 16) < (b.first >> 16) : (a.first & 0xffff) < (b.first & 0xffff);
    });
    for (auto& e : singles) { mq.push_back(e.first); mg.push_back((float)e.second); mg64.push_back(e.second); }
    sptr[i + 1] = (int)mq.size();
    if (!sl.empty()) ++nsm;
  }
  for (int pad = 0; pad < 8; ++pad) { mq.push_back(0u); mg.push_back(0.0f); mg64.push_back(0.0); }  // tail slack
  h->NGm = ngm;
  h->NSm = nsm;
  // The device tables hold each row's two LDS row offsets as words of their own (q2*pitch,
  // q3*pitch), so that the kernel forms an address with one shift-and-add; the pitch is NK,
  // and NK+1 for tiles with a pad row per q block.  The second row of a pair stores
  // its two words swapped (q3b first), so that a pair's three distinct offsets u = q2, a =
  // q3a, b = q3b are its first three words and come in one load.
  auto unpack_rows = [&](uint32_t pitch) {
    std::vector<uint32_t> o(2 * mq.size());
    for (size_t i = 0; i < mq.size(); ++i) {
      o[2 * i] = (mq[i] & 0xffffu) / NK * pitch;
      o[2 * i + 1] = (mq[i] >> 16) / NK * pitch;
    }
    for (size_t sl = 0; sl + 1 < sptr.size(); ++sl)
      for (int e = sptr[sl]; e + 1 < spair[sl]; e += 2) std::swap(o[2 * (e + 1)], o[2 * (e + 1) + 1]);
    return o;
  };
  const std::vector<uint32_t> mq_rows = unpack_rows((uint32_t)NK);
  std::vector<uint32_t> mq_pad;
  if (tile_pad_rows(NK, (NK + 1) / 2, 8)) mq_pad = unpack_rows((uint32_t)(NK + 1));
  // MFMA geometry
  h->H = (NK + 1) / 2;
  h->RT = NK > 16 ? 2 : 1;
  if (hipDeviceGetAttribute(&h->cu_count, hipDeviceAttributeMultiprocessorCount, h->device) != hipSuccess ||
      h->cu_count <= 0)
    h->cu_count = 256;
  int dev_lds = 0;
  if (hipDeviceGetAttribute(&dev_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, h->device) != hipSuccess || dev_lds <= 0)
    dev_lds = 65536;
  const size_t limit = (size_t)std::min(dev_lds, 163840) - 512;
  h->lds_limit = (int)limit;
  // Default tile shape per mode: the fewest output states sharing the 16 MFMA
  // columns (largest cell tile, fewest coefficient-tile reloads per cell) whose
  // LDS tile fits and whose kernel instance spills at most a few registers; when
  // every fitting instance spills more, the largest fitting tile.  (Measured at
  // K = L = 12 and 16: a 44-byte spill costs less than doubling the tile reloads,
  // a 268-byte spill costs more.)
  constexpr int kMaxSpillBytes = 128;
  auto pick_slots = [&](int mode) {
    const size_t elem = mode == 2 ? 8 : 4;
    int first_fit = 0;
    for (int sl : {1, 2, 4}) {
      if (tile_lds_bytes(h, sl, elem) > limit) continue;
      if (!first_fit) first_fit = sl;
      const int spill = mfma_spill_bytes(h, mode, sl, 512);
      if (spill >= 0 && spill <= kMaxSpillBytes) return sl;
    }
    return first_fit;
  };
  for (int mode = 0; mode < 3; ++mode) h->slots[mode] = pick_slots(mode);
  const int H = h->H, HH = H * H, RT = h->RT, UU = (HH + 7) / 8;   // RT == 2: NK = 17
  // FP32 tiles hold 4 steps t per lane ([NTm][Q4][64][4]) and FP64 tiles 2 ([NTm][Q2][64][2]),
  // so that the kernels load them as vectors; the row-16 vectors are padded to 4 Q4 values
  const int Q4 = (HH + 3) / 4, Q2 = (HH + 1) / 2, HHp = 4 * Q4;
  auto idx32 = [&](int m, int t, int ln) { return (((size_t)m * Q4 + t / 4) * 64 + ln) * 4 + t % 4; };
  auto idx64 = [&](int m, int t, int ln) { return (((size_t)m * Q2 + t / 2) * 64 + ln) * 2 + t % 2; };
  // A-operand value for lane group r at step t: the group's quadrant starts at k = 0
  // (lower half) or k = tile_upper_k (upper half); upper-half rows outside [H, NK), the
  // one shared with the lower half or the one past the end, have zero weight.
  const int uk = tile_upper_k(NK, H);
  auto Tval = [&](const std::vector<double>& M, int m, int k1, int t, int r) -> double {
    if (t >= HH || k1 >= NK) return 0.0;
    int a = t / H, b = t % H;
    int h2 = r >> 1, h3 = r & 1;
    int k2 = (h2 ? uk : 0) + a, k3 = (h3 ? uk : 0) + b;
    if (k2 >= NK || k3 >= NK) return 0.0;
    if (h2 && k2 < H) return 0.0;
    if (h3 && k3 < H) return 0.0;
    return M[(size_t)m * blk + ((size_t)k1 * NK + k2) * NK + k3];
  };
  auto Rval = [&](int m, int k1, int t, int r) -> double { return Tval(Rm, m, k1, t, r); };
  bool want32 = h->precisions & WEFQ_FP32, want16 = h->precisions & WEFQ_BF16X3, want64 = h->precisions & WEFQ_FP64;
  if ((want32 && h->slots[0] == 0) || (want16 && h->slots[1] == 0) || (want64 && h->slots[2] == 0)) {
    set_error("coefficient tile does not fit in LDS for this truncation");
    return false;
  }
  // NK = 17: row k1 = 16 of every merged channel per lane group, for the VALU dot product
  std::vector<double> r16;
  if (RT == 2) {
    r16.assign((size_t)NTm * 4 * HHp, 0.0);
    for (int m = 0; m < NTm; ++m)
      for (int r = 0; r < 4; ++r)
        for (int t = 0; t < HH; ++t) r16[((size_t)m * 4 + r) * HHp + t] = Rval(m, 16, t, r);
  }
  if (want64) {
    std::vector<double> t64((size_t)NTm * Q2 * 64 * 2, 0.0);
    for (int m = 0; m < NTm; ++m)
      for (int t = 0; t < HH; ++t)
        for (int ln = 0; ln < 64; ++ln) t64[idx64(m, t, ln)] = Rval(m, ln & 15, t, ln >> 4);
    if (!upload(h, h->d_Rt64, t64, s) || !upload(h, h->d_mg64, mg64, s)) return false;
    if (RT == 2 && !upload(h, h->d_R16_64, r16, s)) return false;
  }
  if ((want32 || want16) && RT == 2) {
    std::vector<float> r16f(r16.begin(), r16.end());
    if (!upload(h, h->d_R16_32, r16f, s)) return false;
  }
  if (want32) {
    std::vector<float> t32((size_t)NTm * Q4 * 64 * 4, 0.0f);
    for (int m = 0; m < NTm; ++m)
      for (int t = 0; t < HH; ++t)
        for (int ln = 0; ln < 64; ++ln) t32[idx32(m, t, ln)] = (float)Rval(m, ln & 15, t, ln >> 4);
    if (!upload(h, h->d_Rt32, t32, s)) return false;
  }
  if (wantD) {                // the antisymmetric tiles in the same layouts (FP64 and FP32)
    std::vector<double> d16;
    if (RT == 2) {
      d16.assign((size_t)NTm * 4 * HHp, 0.0);
      for (int m = 0; m < NTm; ++m)
        for (int r = 0; r < 4; ++r)
          for (int t = 0; t < HH; ++t) d16[((size_t)m * 4 + r) * HHp + t] = Tval(Dm, m, 16, t, r);
    }
    std::vector<double> t64((size_t)NTm * Q2 * 64 * 2, 0.0);
    std::vector<float> t32((size_t)NTm * Q4 * 64 * 4, 0.0f);
    for (int m = 0; m < NTm; ++m)
      for (int t = 0; t < HH; ++t)
        for (int ln = 0; ln < 64; ++ln) {
          const double v = Tval(Dm, m, ln & 15, t, ln >> 4);
          t64[idx64(m, t, ln)] = v;
          t32[idx32(m, t, ln)] = (float)v;
        }
    if ((want64 && !upload(h, h->d_Dt64, t64, s)) || (want32 && !upload(h, h->d_Dt32, t32, s))) return false;
    if (RT == 2) {
      std::vector<float> d16f(d16.begin(), d16.end());
      if ((want64 && !upload(h, h->d_D16_64, d16, s)) || (want32 && !upload(h, h->d_D16_32, d16f, s))) return false;
    }
  }
  if (want16) {
    std::vector<uint16_t> hi((size_t)NTm * UU * 64 * 8), lo(hi.size());
    for (int m = 0; m < NTm; ++m)
      for (int u = 0; u < UU; ++u)
        for (int ln = 0; ln < 64; ++ln)
          for (int e = 0; e < 8; ++e) {
            double v = Rval(m, ln & 15, u * 8 + e, ln >> 4);
            uint16_t bh = bf16_bits((float)v);
            uint16_t bl = bf16_bits((float)(v - (double)bf16_to_float(bh)));
            size_t idx = (((size_t)m * UU + u) * 64 + ln) * 8 + e;
            hi[idx] = bh; lo[idx] = bl;
          }
    if (!upload(h, h->d_Rhi, hi, s) || !upload(h, h->d_Rlo, lo, s)) return false;
  }
  // work units: (l1, up to GQ output states q1), largest estimated cost first.  Within
  // l1 the states are listed as m1, -m1 for m1 = 1..l1, then m1 = 0, so that a group
  // of output states sharing the MFMA columns holds slices of similar length.
  struct Unit { int l1, nq; int q[UNIT_STRIDE - 2]; double cost; };
  auto build_units = [&](int GQ, std::vector<int>& uarr, double& total_cost) -> int {
    std::vector<Unit> units;
    for (int l1 = 0; l1 <= L; ++l1) {
      std::vector<int> order;
      for (int m = 1; m <= l1; ++m) { order.push_back(l1 * l1 + l1 + m); order.push_back(l1 * l1 + l1 - m); }
      order.push_back(l1 * l1 + l1);
      for (size_t i0 = 0; i0 < order.size(); i0 += GQ) {
        Unit un{l1, 0, {}, 0.0};
        un.nq = (int)std::min<size_t>(GQ, order.size() - i0);
        for (int i = 0; i < un.nq; ++i) un.q[i] = order[i0 + i];
        for (int m = chan_begin[l1]; m < chan_begin[l1 + 1]; ++m)
          for (int i = 0; i < un.nq; ++i) {
            const int si = slice_off[m] + un.q[i] - l1 * l1;
            const int npair = (spair[si] - sptr[si]) / 2, nsingle = sptr[si + 1] - spair[si];
            un.cost += (double)npair * (HH + 5 * H) + (double)nsingle * (HH + 3 * H) + HH * RT * 8.0;
          }
        units.push_back(un);
      }
    }
    std::stable_sort(units.begin(), units.end(), [](const Unit& a, const Unit& b) { return a.cost > b.cost; });
    total_cost = 0.0;
    for (auto& u : units) {
      uarr.push_back(u.l1);
      uarr.push_back(u.nq);
      for (int i = 0; i < UNIT_STRIDE - 2; ++i) uarr.push_back(u.q[i]);
      total_cost += u.cost;
    }
    return (int)units.size();
  };
  // Units hold kUnitStates = 4 output states: a wave then runs a shorter serial chain, and
  // the units of a tile balance better over its 8 waves.  Against units of 8 this measured
  // 5-45% faster for K <= 8 at every batch size from 256 to 65,536 cells, up to 47% faster
  // at K = 10 and 12 below 4,096 cells, and equal at K = 10 and 12 on larger batches;
  // results are bitwise the same.
  h->GQ = kUnitStates;
  std::vector<int> uarr;
  h->nunits = build_units(h->GQ, uarr, h->tile_cost);
  // Default block: 256 threads when a tile holds fewer than 16 work units, too few to keep 8
  // waves busy.  Measured with 9 to 12 units (K = L = 4 and 5; K = 8, 12, 16 at L = 2 to 4):
  // 256 threads were 1-33% faster in 18 of 20 cases and 2% slower in 2; with 16 units
  // (K = L = 6) it was mixed, with 57 (K = 4, L = 13) 1.5-1.9x slower.
  // Otherwise the block of 512, 768 (12 waves, three per SIMD) or 1,024 threads (16 waves, four
  // per SIMD; quadrants up to 5x5) whose instance of the mode's tile shape spills at most 64
  // bytes per lane and keeps the most waves resident per compute unit, the larger block on a
  // tie.  A tile that fills the LDS leaves one workgroup per compute unit, and the third wave
  // per SIMD hides more of the coupling's gather latency behind the other waves' arithmetic;
  // where several workgroups fit, one larger workgroup stages each tile once and its waves share
  // one work-unit counter.  Measured (ms, 512 -> 768 threads): K = L = 12 FP32 65,536 cells
  // 39.6 -> 37.3, BF16x3 31.3 -> 30.9; K = L = 10 FP32 32,768 cells 7.63 -> 6.89; K = L = 14 FP32
  // 16,384 cells 29.0 -> 24.7; K = L = 16 FP32 62.9 -> 59.1 (a 56-byte spill); K = L = 8 FP64
  // 65,536 cells 7.68 -> 6.83.  Instances that spill more were much slower (K = L = 12 FP64:
  // 77.0 -> 91.3 ms).  At K = L = 8 in FP32, where two 8-wave workgroups fit, 768 threads were
  // slower (3.66 -> 4.07 ms) and 1,024 equal at 65,536 cells (3.65 ms) and faster on small
  // batches (4,096 cells 0.291 -> 0.278 ms, 2,048 cells 0.192 -> 0.162 ms).
  constexpr int kWideMaxSpill = 64;
  for (int mode = 0; mode < 3; ++mode) {
    int blk = h->nunits < 16 ? 256 : 512;
    if (blk == 512 && h->slots[mode]) {
      const int sl = h->slots[mode];
      int best = 8 * mfma_blocks_per_cu(h, mode, sl, 512);
      for (const int cand : {768, 1024}) {
        const int spill = mfma_spill_bytes(h, mode, sl, cand);
        if (spill < 0 || spill > kWideMaxSpill) continue;          // no instance, or it spills
        const int waves = cand / 64 * mfma_blocks_per_cu(h, mode, sl, cand);
        if (waves >= best) { best = waves; blk = cand; }
      }
    }
    h->block[mode] = blk;
    h->split_per_cu[mode] = split_target(h, mode);
    h->resident_per_cu[mode] = resident_blocks(h, mode);
  }
  // the FP64 two-input tiles of 2 cells carry 8 output states per column group (H >= 7):
  // they get units of 8
  if (H >= 7 && want64) {
    std::vector<int> u8;
    double c8 = 0.0;
    h->nunits8 = build_units(8, u8, c8);
    if (!upload(h, h->d_units8, u8, s)) return false;
  }
  {
    std::vector<int> u2;
    double c2 = 0.0;
    h->nunits2 = build_units(2, u2, c2);
    if (!upload(h, h->d_units2, u2, s)) return false;
  }
  if (!upload(h, h->d_units, uarr, s) || !upload(h, h->d_chan_begin, chan_begin, s) ||
      !upload(h, h->d_slice_off, slice_off, s) || !upload(h, h->d_sptr, sptr, s) ||
      !upload(h, h->d_spair, spair, s) ||
      !upload(h, h->d_mq, mq_rows, s) || !upload(h, h->d_mg, mg, s))
    return false;
  if (mq_pad.empty()) h->d_mq_pad = h->d_mq;
  else if (!upload(h, h->d_mq_pad, mq_pad, s)) return false;
  h->d_check = dev_alloc<double>(h, h->check_blocks);
  if (!h->d_check) { set_error("device allocation failed"); return false; }
  return hipStreamSynchronize(s) == hipSuccess;
}

}  // namespace wefq

using namespace wefq;

static wefq_status fail(wefq_status st, const std::string& msg) {
  set_error(msg);
  return st;
}

static void free_core(wefq_core* h) {
  if (!h) return;
  for (void* p : h->allocations) (void)hipFree(p);
  delete h;
}

extern "C" {

const char* wefq_last_error(void) { return g_last_error.c_str(); }

// Validate the core parameters and make an empty handle with its channel and COO tables.
static wefq_status new_core(int32_t model, double gamma_in, double b0, int32_t K, int32_t L, uint32_t precisions,
                            int32_t device, int32_t n_beta, const double* beta, wefq_core** out,
                            std::vector<CooRow>& coo) {
  *out = nullptr;
  if (K < 0 || K > 16 || L < 0 || L > 16) return fail(WEFQ_EUNSUPPORTED, "Kmax and Lmax must lie in [0, 16]");
  if (n_beta < 0 || n_beta > WEFQ_MAX_BETA) return fail(WEFQ_EINVAL, "n_beta must lie in [0, WEFQ_MAX_BETA]");
  if (n_beta > 0 && !beta) return fail(WEFQ_EINVAL, "null angular factor with n_beta > 0");
  for (int j = 0; j < n_beta; ++j)
    if (!std::isfinite(beta[j])) return fail(WEFQ_EINVAL, "non-finite angular factor coefficient");
  double gamma;
  switch (model) {
    case WEFQ_MAXWELL: gamma = 0.0; break;
    case WEFQ_HARD_SPHERE: gamma = 1.0; break;
    case WEFQ_VHS: gamma = gamma_in; break;
    default: return fail(WEFQ_EINVAL, "unknown collision model");
  }
  if (!(gamma >= 0.0 && gamma <= 2.0)) return fail(WEFQ_EINVAL, "gamma must lie in [0, 2]");
  unsigned prec = precisions ? precisions : (WEFQ_FP64 | WEFQ_FP32 | WEFQ_BF16X3);
  if (prec & ~63u) return fail(WEFQ_EINVAL, "unknown precision bits");
  if (prec & (WEFQ_FP64_NAIVE | WEFQ_PREP_RADIAL)) prec |= WEFQ_FP64;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return fail(WEFQ_EHIP, "no HIP device available");
  if (device < 0 || device >= ndev) return fail(WEFQ_EINVAL, "device ordinal out of range");
  if (hipSetDevice(device) != hipSuccess) return fail(WEFQ_EHIP, "hipSetDevice failed");
  wefq_core* h = new (std::nothrow) wefq_core();
  if (!h) return fail(WEFQ_ENOMEM, "host allocation failed");
  h->device = device;
  h->model = model;
  h->K = K; h->L = L; h->NK = h->K + 1; h->NQ = (h->L + 1) * (h->L + 1);
  h->N = h->NK * h->NQ;
  h->gamma = gamma;
  h->b0 = b0 > 0 ? b0 : 1.0 / (4.0 * 3.141592653589793238462643383279502884);
  h->precisions = prec;
  if (n_beta > 0) h->beta.assign(beta, beta + n_beta);
  h->chans = enumerate_channels(h->L);
  h->NT = (int)h->chans.size();
  coo = build_coo(h->L);
  h->NG = (int)coo.size();
  std::vector<char> seen((size_t)h->NT * h->NQ, 0);
  int ns = 0;
  for (auto& r : coo) if (!seen[(size_t)r.c * h->NQ + r.q1]) { seen[(size_t)r.c * h->NQ + r.q1] = 1; ++ns; }
  h->NS = ns;
  *out = h;
  return WEFQ_OK;
}

// From the raw core in h->R64: keep a copy (bilinear tables, serialization), zero the
// invariant rows (Section 4.4) and prepare the device tables.
static wefq_status finish_core(wefq_core* h, const std::vector<CooRow>& coo, hipStream_t s, wefq_handle* out) {
  h->R64raw = h->R64;
  zero_invariants(h);
  if (!prepare_apply_tables(h, coo, s)) { free_core(h); return WEFQ_ENOMEM; }
  *out = h;
  return WEFQ_OK;
}

wefq_status wefq_build_core(const wefq_core_desc* desc, void* stream, wefq_handle* out) {
  try {
    if (!desc || !out) return fail(WEFQ_EINVAL, "null descriptor or output pointer");
    *out = nullptr;
    wefq_core* h = nullptr;
    std::vector<CooRow> coo;
    if (desc->rad_pad < 0 || desc->rad_pad > 64 || desc->ang_pad < 0 || desc->ang_pad > 64)
      return fail(WEFQ_EINVAL, "rad_pad and ang_pad must lie in [0, 64]");
    wefq_status st = new_core(desc->model, desc->gamma, desc->b0, desc->Kmax, desc->Lmax, desc->precisions,
                              desc->device, desc->n_beta, desc->beta, &h, coo);
    if (st != WEFQ_OK) return st;
    h->rad_pad = desc->rad_pad;
    h->ang_pad = desc->ang_pad;
    hipStream_t s = (hipStream_t)stream;
    if (!build_radial_core(h, coo, s)) { free_core(h); return WEFQ_EHIP; }
    return finish_core(h, coo, s, out);
  } catch (const std::exception& e) {
    return fail(WEFQ_EINVAL, std::string("exception in core build: ") + e.what());
  } catch (...) {
    return fail(WEFQ_EINVAL, "unknown exception in core build");
  }
}

wefq_status wefq_core_info_get(wefq_handle h, wefq_core_info* info) {
  if (!h || !info) return fail(WEFQ_EINVAL, "null handle or info pointer");
  info->N = h->N; info->NK = h->NK; info->NQ = h->NQ;
  info->N_T = h->NT; info->N_G = h->NG; info->N_S = h->NS;
  info->N_T_merged = h->NTm; info->N_G_merged = h->NGm; info->N_S_merged = h->NSm;
  info->quad_nodes = h->quad_nodes;
  info->device_bytes = h->device_bytes;
  double nk = h->NK;
  info->flop_alg_per_cell = 2.0 * nk * nk * h->NG + 2.0 * nk * nk * nk * h->NS;
  info->gamma = h->gamma; info->b0 = h->b0;
  info->model = h->model;
  info->n_beta = (int64_t)h->beta.size();
  for (int j = 0; j < WEFQ_MAX_BETA; ++j) info->beta[j] = j < (int)h->beta.size() ? h->beta[j] : 0.0;
  info->radial_groups = h->rad_groups;
  info->rad_pad = h->rad_pad;
  info->ang_pad = h->ang_pad;
  return WEFQ_OK;
}

wefq_status wefq_mode_index(wefq_handle h, int32_t k, int32_t l, int32_t m, int64_t* n) {
  if (!h || !n) return fail(WEFQ_EINVAL, "null handle or output pointer");
  if (k < 0 || k > h->K || l < 0 || l > h->L || m < -l || m > l)
    return fail(WEFQ_EINVAL, "mode (k, l, m) outside the truncation");
  *n = (int64_t)(l * l + l + m) * h->NK + k;
  return WEFQ_OK;
}

wefq_status wefq_core_download_R(wefq_handle h, double* host_R, int64_t count) {
  if (!h || !host_R) return fail(WEFQ_EINVAL, "null handle or output pointer");
  if (count != (int64_t)h->R64.size()) return fail(WEFQ_EINVAL, "count must equal N_T * NK^3");
  std::memcpy(host_R, h->R64.data(), h->R64.size() * sizeof(double));
  return WEFQ_OK;
}

// ---- serialization: the raw radial core and its parameters
//
// File layout (native byte order): CoreFileHeader; for version 2 (a core with an angular
// factor) a CoreFileAngular record; then N_T * NK^3 doubles of the core before the
// invariant-row zeroing, [c][k1][k2][k3] in the paper's channel order.  An isotropic
// core is written as version 1.  The checksum is the 64-bit FNV-1a hash of the payload
// bytes.
struct CoreFileHeader {
  char magic[8];
  uint32_t version, header_bytes;
  int32_t model, K, L, NT, NK, pad;
  double gamma, b0;
  int64_t quad_nodes;
  uint64_t count, checksum;
};
struct CoreFileAngular {
  int32_t n_beta, pad;
  double beta[WEFQ_MAX_BETA];
};
static const char kCoreMagic[8] = {'W', 'E', 'F', 'Q', 'C', 'O', 'R', 'E'};

static uint64_t fnv1a(const void* data, size_t n) {
  const unsigned char* p = static_cast<const unsigned char*>(data);
  uint64_t hsh = 1469598103934665603ull;
  for (size_t i = 0; i < n; ++i) { hsh ^= p[i]; hsh *= 1099511628211ull; }
  return hsh;
}

wefq_status wefq_core_save(wefq_handle h, const char* path) {
  if (!h || !path) return fail(WEFQ_EINVAL, "null handle or path");
  if (h->R64raw.size() != h->R64.size()) return fail(WEFQ_EINVAL, "the core holds no raw radial tensor");
  CoreFileHeader hd;
  std::memset(&hd, 0, sizeof(hd));
  std::memcpy(hd.magic, kCoreMagic, 8);
  const bool angular = !h->beta.empty();
  CoreFileAngular an;
  std::memset(&an, 0, sizeof(an));
  an.n_beta = (int32_t)h->beta.size();
  for (size_t j = 0; j < h->beta.size(); ++j) an.beta[j] = h->beta[j];
  hd.version = angular ? 2 : 1;
  hd.header_bytes = sizeof(CoreFileHeader) + (angular ? sizeof(CoreFileAngular) : 0);
  hd.model = h->model; hd.K = h->K; hd.L = h->L; hd.NT = h->NT; hd.NK = h->NK;
  hd.gamma = h->gamma; hd.b0 = h->b0; hd.quad_nodes = h->quad_nodes;
  hd.count = h->R64raw.size();
  hd.checksum = fnv1a(h->R64raw.data(), h->R64raw.size() * sizeof(double));
  FILE* fp = std::fopen(path, "wb");
  if (!fp) return fail(WEFQ_EINVAL, std::string("cannot open for writing: ") + path);
  bool ok = std::fwrite(&hd, sizeof(hd), 1, fp) == 1 &&
            (!angular || std::fwrite(&an, sizeof(an), 1, fp) == 1) &&
            std::fwrite(h->R64raw.data(), sizeof(double), h->R64raw.size(), fp) == h->R64raw.size();
  ok = (std::fclose(fp) == 0) && ok;
  if (!ok) return fail(WEFQ_EINVAL, std::string("write failed: ") + path);
  return WEFQ_OK;
}

wefq_status wefq_core_load(const char* path, uint32_t precisions, int32_t device, void* stream, wefq_handle* out) {
  try {
    if (!path || !out) return fail(WEFQ_EINVAL, "null path or output pointer");
    *out = nullptr;
    FILE* fp = std::fopen(path, "rb");
    if (!fp) return fail(WEFQ_EINVAL, std::string("cannot open: ") + path);
    CoreFileHeader hd;
    CoreFileAngular an;
    std::memset(&an, 0, sizeof(an));
    std::vector<double> raw;
    bool ok = std::fread(&hd, sizeof(hd), 1, fp) == 1 && std::memcmp(hd.magic, kCoreMagic, 8) == 0 &&
              (hd.version == 1 || hd.version == 2) &&
              hd.header_bytes == sizeof(CoreFileHeader) + (hd.version == 2 ? sizeof(CoreFileAngular) : 0) &&
              hd.K >= 0 && hd.K <= 16 && hd.L >= 0 && hd.L <= 16 && hd.NK == hd.K + 1 &&
              hd.count == (uint64_t)hd.NT * hd.NK * hd.NK * hd.NK && hd.NT > 0;
    if (ok && hd.version == 2)
      ok = std::fread(&an, sizeof(an), 1, fp) == 1 && an.n_beta >= 1 && an.n_beta <= WEFQ_MAX_BETA;
    if (ok) {
      raw.resize(hd.count);
      ok = std::fread(raw.data(), sizeof(double), raw.size(), fp) == raw.size() && std::fgetc(fp) == EOF &&
           fnv1a(raw.data(), raw.size() * sizeof(double)) == hd.checksum;
    }
    std::fclose(fp);
    if (!ok) return fail(WEFQ_EINVAL, std::string("not a valid core file (header, size or checksum): ") + path);
    wefq_core* h = nullptr;
    std::vector<CooRow> coo;
    wefq_status st = new_core(hd.model, hd.gamma, hd.b0, hd.K, hd.L, precisions, device, an.n_beta, an.beta, &h, coo);
    if (st != WEFQ_OK) return st;
    if (h->NT != hd.NT) { free_core(h); return fail(WEFQ_EINVAL, "channel count does not match the truncation"); }
    h->R64 = std::move(raw);
    h->quad_nodes = hd.quad_nodes;
    return finish_core(h, coo, (hipStream_t)stream, out);
  } catch (const std::exception& e) {
    return fail(WEFQ_EINVAL, std::string("exception in core load: ") + e.what());
  }
}

static wefq_status check_batch(wefq_handle h, int32_t precision, const void* a, const void* b, int64_t B,
                               int64_t lda, int64_t ldb) {
  if (!h) return fail(WEFQ_EINVAL, "null handle");
  if (precision != WEFQ_FP64 && precision != WEFQ_FP32 && precision != WEFQ_BF16X3 && precision != WEFQ_FP64_NAIVE)
    return fail(WEFQ_EINVAL, "unknown precision");
  unsigned need = precision == WEFQ_FP64_NAIVE ? (unsigned)WEFQ_FP64 : (unsigned)precision;
  if (!(h->precisions & need)) return fail(WEFQ_EINVAL, "precision was not prepared for this core");
  if (B < 0) return fail(WEFQ_EINVAL, "negative batch size");
  if (B == 0) return WEFQ_OK;
  if (!a) return fail(WEFQ_EINVAL, "null input pointer");
  if (lda < h->N || ldb < h->N) return fail(WEFQ_EINVAL, "leading dimension smaller than N");
  const uintptr_t align = (precision == WEFQ_FP64 || precision == WEFQ_FP64_NAIVE) ? 7 : 3;
  if (((uintptr_t)a & align) || (b && ((uintptr_t)b & align)))
    return fail(WEFQ_EINVAL, "pointers must be aligned to the element size");
  return WEFQ_OK;
}

wefq_status wefq_apply_Q(wefq_handle h, int32_t precision, const void* f, void* Q, int64_t B, int64_t ld_f,
                         int64_t ld_q, void* stream) {
  wefq_status st = check_batch(h, precision, f, Q, B, ld_f, ld_q);
  if (st != WEFQ_OK || B == 0) return st;
  if (!Q) return fail(WEFQ_EINVAL, "null output pointer");
  size_t es = (precision == WEFQ_FP64 || precision == WEFQ_FP64_NAIVE) ? 8 : 4;
  const char* fb = (const char*)f; const char* qb = (const char*)Q;
  if (fb < qb + (size_t)B * ld_q * es && qb < fb + (size_t)B * ld_f * es)
    return fail(WEFQ_EINVAL, "f and Q must not overlap");
  if (hipSetDevice(h->device) != hipSuccess) return fail(WEFQ_EHIP, "hipSetDevice failed");
  hipError_t e;
  if (precision == WEFQ_FP64_NAIVE)
    e = launch_apply_fp64(h, (const double*)f, (double*)Q, B, ld_f, ld_q, (hipStream_t)stream);
  else
    e = launch_apply_mfma(h, precision, f, Q, B, ld_f, ld_q, (hipStream_t)stream);
  if (e != hipSuccess) return fail(WEFQ_EHIP, std::string("kernel launch failed: ") + hipGetErrorString(e));
  return WEFQ_OK;
}

static const int64_t kRadialMaxChunk = 65536;

wefq_status wefq_radial_workspace(wefq_handle h, int64_t chunk, int64_t* bytes) {
  if (!h || !bytes) return fail(WEFQ_EINVAL, "null handle or output pointer");
  if (!(h->precisions & WEFQ_PREP_RADIAL)) return fail(WEFQ_EINVAL, "the core was built without WEFQ_PREP_RADIAL");
  if (chunk < 1) return fail(WEFQ_EINVAL, "chunk must be >= 1");
  const int64_t c = std::min<int64_t>((chunk + 63) / 64 * 64, kRadialMaxChunk);
  *bytes = c * radial_bytes_per_cell(h);
  return WEFQ_OK;
}

wefq_status wefq_apply_Q_radial(wefq_handle h, const double* f, double* Q, int64_t B, int64_t ld_f, int64_t ld_q,
                                void* work, int64_t work_bytes, void* stream) {
  wefq_status st = check_batch(h, WEFQ_FP64, f, Q, B, ld_f, ld_q);
  if (st != WEFQ_OK || B == 0) return st;
  if (!(h->precisions & WEFQ_PREP_RADIAL)) return fail(WEFQ_EINVAL, "the core was built without WEFQ_PREP_RADIAL");
  if (!Q) return fail(WEFQ_EINVAL, "null output pointer");
  if (!work || ((uintptr_t)work & 255)) return fail(WEFQ_EINVAL, "workspace must be non-null and 256-byte aligned");
  const int64_t per_cell = radial_bytes_per_cell(h);
  const int64_t chunk = std::min<int64_t>(work_bytes / per_cell / 64 * 64, kRadialMaxChunk);
  if (chunk < 64) return fail(WEFQ_EINVAL, "workspace smaller than one 64-cell chunk");
  const char* fb = (const char*)f; const char* qb = (const char*)Q; const char* wb = (const char*)work;
  const size_t fn = (size_t)B * ld_f * 8, qn = (size_t)B * ld_q * 8, wn = (size_t)chunk * per_cell;
  if ((fb < qb + qn && qb < fb + fn) || (fb < wb + wn && wb < fb + fn) || (qb < wb + wn && wb < qb + qn))
    return fail(WEFQ_EINVAL, "f, Q and the workspace must not overlap");
  if (hipSetDevice(h->device) != hipSuccess) return fail(WEFQ_EHIP, "hipSetDevice failed");
  hipError_t e = launch_apply_radial(h, f, Q, B, ld_f, ld_q, work, chunk, (hipStream_t)stream);
  if (e != hipSuccess) return fail(WEFQ_EHIP, std::string("kernel launch failed: ") + hipGetErrorString(e));
  return WEFQ_OK;
}

// Validation shared by the two-input entry points.
static wefq_status check_two(wefq_handle h, int32_t precision, const void* c, const void* d, void* out, int64_t B,
                             int64_t ld_c, int64_t ld_d, int64_t ld_out) {
  if (h && precision != WEFQ_FP64 && precision != WEFQ_FP32)
    return fail(WEFQ_EINVAL, "the two-input forms run in FP64 or FP32");
  wefq_status st = check_batch(h, precision, c, d, B, ld_c, ld_d);
  if (st != WEFQ_OK || B == 0) return st;
  if (!d || !out) return fail(WEFQ_EINVAL, "null direction or output pointer");
  if (ld_out < h->N) return fail(WEFQ_EINVAL, "leading dimension smaller than N");
  const size_t es = precision == WEFQ_FP64 ? 8 : 4;
  if ((uintptr_t)out & (es - 1)) return fail(WEFQ_EINVAL, "pointers must be aligned to the element size");
  const char* ob = (const char*)out;
  const size_t on = (size_t)B * ld_out * es;
  for (const void* in : {c, d}) {
    const char* ib = (const char*)in;
    const size_t inn = (size_t)B * (in == c ? ld_c : ld_d) * es;
    if (ib < ob + on && ob < ib + inn) return fail(WEFQ_EINVAL, "the output must not overlap c or d");
  }
  // the smallest two-input tile: 2 cells x 8 output states (FP64, H >= 7), else 4 x 4
  const int max_slots = (precision == WEFQ_FP64 && h->H >= 7) ? 8 : 4;
  if (2 * tile_lds_bytes(h, max_slots, es) > (size_t)h->lds_limit)
    return fail(WEFQ_EUNSUPPORTED, "two coefficient tiles do not fit in LDS for this truncation");
  return WEFQ_OK;
}

wefq_status wefq_apply_J(wefq_handle h, int32_t precision, const void* c, const void* d, void* out, int64_t B,
                         int64_t ld_c, int64_t ld_d, int64_t ld_out, void* stream) {
  wefq_status st = check_two(h, precision, c, d, out, B, ld_c, ld_d, ld_out);
  if (st != WEFQ_OK || B == 0) return st;
  if (hipSetDevice(h->device) != hipSuccess) return fail(WEFQ_EHIP, "hipSetDevice failed");
  hipError_t e = launch_apply_jvp(h, precision, c, d, out, B, ld_c, ld_d, ld_out, (hipStream_t)stream);
  if (e != hipSuccess) return fail(WEFQ_EHIP, std::string("kernel launch failed: ") + hipGetErrorString(e));
  return WEFQ_OK;
}

wefq_status wefq_apply_Qfg(wefq_handle h, int32_t precision, const void* f, const void* g, void* out, int64_t B,
                           int64_t ld_f, int64_t ld_g, int64_t ld_out, void* stream) {
  wefq_status st = check_two(h, precision, f, g, out, B, ld_f, ld_g, ld_out);
  if (st != WEFQ_OK || B == 0) return st;
  if (!(h->precisions & WEFQ_PREP_BILINEAR))
    return fail(WEFQ_EINVAL, "the bilinear-form tables were not prepared (WEFQ_PREP_BILINEAR)");
  if (hipSetDevice(h->device) != hipSuccess) return fail(WEFQ_EHIP, "hipSetDevice failed");
  hipError_t e = launch_apply_qfg(h, precision, f, g, out, B, ld_f, ld_g, ld_out, (hipStream_t)stream);
  if (e != hipSuccess) return fail(WEFQ_EHIP, std::string("kernel launch failed: ") + hipGetErrorString(e));
  return WEFQ_OK;
}

wefq_status wefq_check_conservation(wefq_handle h, int32_t precision, const void* Q, int64_t B, int64_t ld_q,
                                    double* max_abs, void* stream) {
  if (!max_abs) return fail(WEFQ_EINVAL, "null result pointer");
  wefq_status st = check_batch(h, precision, Q, nullptr, B, ld_q, ld_q);
  if (st != WEFQ_OK) return st;
  *max_abs = 0.0;
  if (B == 0) return WEFQ_OK;
  if (hipSetDevice(h->device) != hipSuccess) return fail(WEFQ_EHIP, "hipSetDevice failed");
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = launch_check(h, precision, Q, B, ld_q, s);
  std::vector<double> part(h->check_blocks);
  if (e == hipSuccess) e = hipMemcpyAsync(part.data(), h->d_check, part.size() * 8, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(WEFQ_EHIP, std::string("conservation check: ") + hipGetErrorString(e));
  double m = 0.0;
  for (double v : part) m = (v > m || v != v) ? v : m;
  *max_abs = m;
  return WEFQ_OK;
}

wefq_status wefq_tune_set(wefq_handle h, int32_t precision, int32_t slots, int32_t block) {
  if (!h) return fail(WEFQ_EINVAL, "null handle");
  const int mode = mfma_mode(precision);
  if (mode < 0) return fail(WEFQ_EINVAL, "tile shapes exist for FP64, FP32 and BF16X3");
  if (slots != 1 && slots != 2 && slots != 4) return fail(WEFQ_EINVAL, "slots must be 1, 2 or 4");
  if (block != 256 && block != 512 && block != 768 && block != 1024)
    return fail(WEFQ_EINVAL, "block must be 256, 512, 768 or 1024");
  const size_t elem = mode == 2 ? 8 : 4;
  if (tile_lds_bytes(h, slots, elem) > (size_t)h->lds_limit)
    return fail(WEFQ_EUNSUPPORTED, "tile of 16/slots cells does not fit in LDS");
  // the attribute and residency queries below run on the current device
  if (hipSetDevice(h->device) != hipSuccess) return fail(WEFQ_EHIP, "hipSetDevice failed");
  if (mfma_spill_bytes(h, mode, slots, block) < 0)
    return fail(WEFQ_EINVAL, "no kernel instance for this tile shape at this block size (1024: quadrants up to 5x5)");
  h->slots[mode] = slots;
  h->block[mode] = block;
  h->split_per_cu[mode] = split_target(h, mode);
  h->resident_per_cu[mode] = resident_blocks(h, mode);
  return WEFQ_OK;
}

wefq_status wefq_tune_get(wefq_handle h, int32_t precision, int32_t* slots, int32_t* block) {
  if (!h || !slots || !block) return fail(WEFQ_EINVAL, "null argument");
  const int mode = mfma_mode(precision);
  if (mode < 0) return fail(WEFQ_EINVAL, "tile shapes exist for FP64, FP32 and BF16X3");
  *slots = h->slots[mode];
  *block = h->block[mode];
  return WEFQ_OK;
}

wefq_status wefq_destroy(wefq_handle h) {
  if (!h) return fail(WEFQ_EINVAL, "null handle");
  (void)hipSetDevice(h->device);
  free_core(h);
  return WEFQ_OK;
}

wefq_status wefq_host_coo(int32_t Lmax, int64_t* count, int32_t* q1, int32_t* q2, int32_t* q3, int32_t* channel,
                          double* g) {
  try {
    if (!count) return fail(WEFQ_EINVAL, "null count pointer");
    if (Lmax < 0 || Lmax > 16) return fail(WEFQ_EUNSUPPORTED, "Lmax must lie in [0, 16]");
    std::vector<CooRow> rows = build_coo(Lmax);
    if (!q1 && !q2 && !q3 && !channel && !g) { *count = (int64_t)rows.size(); return WEFQ_OK; }
    if (*count < (int64_t)rows.size()) return fail(WEFQ_EINVAL, "output arrays too small");
    for (size_t i = 0; i < rows.size(); ++i) {
      if (q1) q1[i] = rows[i].q1;
      if (q2) q2[i] = rows[i].q2;
      if (q3) q3[i] = rows[i].q3;
      if (channel) channel[i] = rows[i].c;
      if (g) g[i] = rows[i].g;
    }
    *count = (int64_t)rows.size();
    return WEFQ_OK;
  } catch (...) {
    return fail(WEFQ_EINVAL, "exception while building the COO table");
  }
}

wefq_status wefq_host_gauss(int32_t kind, int32_t n, double alpha, double* x, double* w) {
  try {
    if (!x || !w) return fail(WEFQ_EINVAL, "null output pointer");
    if ((kind != 0 && kind != 1) || n < 1 || n > 512 || (kind == 1 && alpha <= -1.0))
      return fail(WEFQ_EINVAL, "bad quadrature request");
    std::vector<double> xs, ws;
    gauss_rule(kind, n, alpha, xs, ws);
    std::memcpy(x, xs.data(), n * 8);
    std::memcpy(w, ws.data(), n * 8);
    return WEFQ_OK;
  } catch (...) {
    return fail(WEFQ_EINVAL, "quadrature failed");
  }
}

}  // extern "C"
