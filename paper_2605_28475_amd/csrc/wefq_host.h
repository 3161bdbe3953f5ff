// Host-side tables of the factorized operator: channels, real Gaunt weights,
// COO routing table, merged slices and Gauss quadrature rules.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace wefq {

// Interaction channel (l1, l2, l3) of Section 4.1: triangle rule, even sum.
struct Channel { int l1, l2, l3; };

// One COO row of the real Gaunt table (Section 4.2), 0-based indices.
struct CooRow { int q1, q2, q3, c; double g; };

// Channels in the paper's enumeration: l1 outer, l2 middle, l3 inner.
std::vector<Channel> enumerate_channels(int L);

// Wigner 3j symbol (j1 j2 j3; m1 m2 m3) from Racah's closed form, evaluated
// in extended precision.
long double wigner3j(int j1, int j2, int j3, int m1, int m2, int m3);

// Real Gaunt weight g(q1,q2,q3) = int Y_q1 Y_q2 Y_q3 dOmega for the real
// harmonics Y_{l,0}=Y_l^0, Y_{l,m>0}=sqrt2(-1)^m Re Y_l^m, Y_{l,m<0}=sqrt2(-1)^m Im Y_l^|m|,
// obtained from the complex Gaunt coefficient by the unitary complex-to-real map.
double real_gaunt(int l1, int m1, int l2, int m2, int l3, int m3);

// COO table in the paper's order (q3 slowest, q2, q1 fastest); |g| <= tol dropped.
std::vector<CooRow> build_coo(int L, double tol = 1e-12);

// Gauss rules.  kind 0: Gauss-Legendre on [-1,1]; kind 1: generalized
// Gauss-Laguerre with weight x^alpha e^{-x} on [0, inf).
void gauss_rule(int kind, int n, double alpha, std::vector<double>& x, std::vector<double>& w);

// Most threads one kernel launch may hold (grid size times block size).
constexpr int64_t max_launch_threads() { return 0xffffffffLL; }

// Cells of one launch of a kernel that runs one workgroup of `block` threads per tile of
// `tile_cells` cells (times `blocks_per_tile` workgroups): larger batches are split into
// launches of at most this many cells.
inline int64_t max_cells_per_launch(int64_t tile_cells, int64_t block, int64_t blocks_per_tile = 1) {
  return max_launch_threads() / (block * blocks_per_tile) * tile_cells;
}

inline int q_of(int l, int m) { return l * l + l + m; }
inline int l_of_q(int q) { int l = 0; while ((l + 1) * (l + 1) <= q) ++l; return l; }

}  // namespace wefq
