// FP64 assembly of the radial kinematic core R^{(c)}_{k1 k2 k3} on the GPU.
//
// Definition (Sections 3.2-3.3, 4.1): with the real Gaunt weights g and the
// weak-form tensor C of Section 2.3, R^{(c)} = sum_m g C / sum_m g^2 over the
// channel's COO rows.  sum_m g C is a rotation-invariant 8-D integral.  Instead
// of the paper's privileged frame (v along z) with 2-D Duffy patches that tame
// the cone singularity of u^gamma, the integral is written in centre-of-mass /
// relative variables G = (v+w)/2, u = v - w, where that singular factor is a
// pure power of the coordinate u and is absorbed exactly into a generalized
// Gauss-Laguerre weight (the device the paper uses for its energy variable):
//   sum_m g C = b0 (2pi)^-3 8pi^2 int G^2 e^{-G^2} dG int u^{2+gamma} e^{-u^2/4} du
//               int_{-1}^{1} dmu  I_c(G, u, mu)
// with G along z and u_hat = (sqrt(1-mu^2), 0, mu) (rotation invariance removes
// the remaining angles).  At each node
//   I_c = [sigG_c h_{k1 l1}(G, u/2) - sigL_c P_{k1 l1}(|v|^2)] P_{k2 l2}(|v|^2) P_{k3 l3}(|w|^2)
//   v = G z + u u_hat/2,  w = G z - u u_hat/2,  P_kl(r^2) = N_kl L_k^{(l+1/2)}(r^2/2)
//   sigG_c = Y_l1,0(z) sum_m g(l1 0, l2 m, l3 m) S_l2m(v) S_l3m(w)      (gain)
//   sigL_c = 4pi Y_l1,0(z) Y_l2,0(z) g(l1 0, l2 0, l3 0) Y_l3,0(z) Pi_l3(v,w) |v|^{l1+l2-l3}  (loss)
// S_lm are real solid harmonics, Pi_l(a,b) = (|a||b|)^l P_l(a.b/|a||b|), and
// h_kl(G, r) Y_lm(G_hat) = int_{S^2} phi_klm(G + r n) dn is the gain sphere
// average of the test function (Funk-Hecke: it commutes with rotations), a 1-D
// Gauss-Legendre integral.  All integrands are polynomials in (G^2, u^2, mu)
// times the weights, so every rule is exact: the result carries only rounding.
//
// With an angular factor, B = b0 u^gamma beta(cos chi), cos chi = u_hat . n, the gain
// sphere average A_klm(G, u_hat, r) = int dn beta(u_hat . n) phi_klm(G z + r n) is no
// longer h_kl(G, r) Y_lm(G_hat): it is integrated directly at every node, with n measured
// from u_hat (Gauss-Legendre in cos chi weighted by beta, trapezoid in the azimuth; exact
// for a polynomial beta), for every cos-type (l, m >= 0) -- v, w and u_hat lie in the x-z
// plane, so sin-type terms vanish by the y -> -y reflection.  The gain of a channel is
// then sum_{m1,m2,m3 >= 0} g(l1 m1, l2 m2, l3 m3) A_{k1 l1 m1} S_l2m2(v) S_l3m3(w), and the
// loss is scaled by int dn beta(u_hat . n) / (4 pi).  The outer rules are unchanged: A is
// a polynomial of the same degree in (G, r) and of degree <= min(J, 2 k1 + l1) in u_hat.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <vector>

#include "wefq_core.h"

namespace wefq {

struct NodeParams {
  int P, K, L, NK, nnu;
  const double* G;       // [P]
  const double* u;       // [P]
  const double* mu;      // [P]
  const double* nu;      // [nnu]
  const double* wnu;     // [nnu]
  const double* Nkl;     // [L+1][NK] radial normalization
  const double* NlmR;    // [(L+1)(L+2)/2] real solid-harmonic normalization (m >= 0)
  double* Pv;            // [L+1][NK][P]
  double* Pw;            // [L+1][NK][P]
  double* Hg;            // [L+1][NK][P]
  double* Sv;            // [(L+1)(L+2)/2][P]
  double* Sw;            // [(L+1)(L+2)/2][P]
  double* Bi;            // [L+1][P]
  double* V2;            // [P]
};

// Laguerre L_k^{(a)}(x) for k = 0..K into out[k*stride].
__device__ inline void laguerre_all(int K, double a, double x, double* out, long stride, double scale_k0,
                                    const double* nk) {
  double p0 = 1.0, p1 = 1.0 + a - x;
  out[0] = nk[0] * p0 * scale_k0;
  if (K >= 1) out[stride] = nk[1] * p1 * scale_k0;
  for (int k = 1; k < K; ++k) {
    double p2 = ((2 * k + 1 + a - x) * p1 - (k + a) * p0) / (k + 1);
    p0 = p1; p1 = p2;
    out[(long)(k + 1) * stride] = nk[k + 1] * p1 * scale_k0;
  }
}

// Thread per (node, l): radial values, gain averages, solid harmonics.
__global__ void core_nodes_kernel(NodeParams p) {
  long tid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  long P = p.P;
  if (tid >= P * (p.L + 1)) return;
  int l = (int)(tid / P);
  long i = tid % P;
  double G = p.G[i], u = p.u[i], mu = p.mu[i];
  double st = sqrt(fmax(0.0, 1.0 - mu * mu));
  double vx = 0.5 * u * st, vz = G + 0.5 * u * mu;
  double wx = -vx, wz = G - 0.5 * u * mu;
  double v2 = vx * vx + vz * vz, w2 = wx * wx + wz * wz;
  double a = l + 0.5;
  const double* nk = p.Nkl + (long)l * p.NK;
  laguerre_all(p.K, a, 0.5 * v2, p.Pv + ((long)l * p.NK) * P + i, P, 1.0, nk);
  laguerre_all(p.K, a, 0.5 * w2, p.Pw + ((long)l * p.NK) * P + i, P, 1.0, nk);
  // gain: h_kl(G, r) = 2pi N_kl int dnu L_k((|x|^2)/2) Pi_l0(x), x = G z + r n(nu)
  double r = 0.5 * u;
  double acc[17];
  for (int k = 0; k <= p.K; ++k) acc[k] = 0.0;
  for (int j = 0; j < p.nnu; ++j) {
    double nu = p.nu[j];
    double xz = G + r * nu;
    double x2 = G * G + r * r + 2.0 * G * r * nu;
    // solid Legendre |x|^l P_l(x_z/|x|) by the three-term recurrence
    double s0 = 1.0, s1 = xz;
    double sl = (l == 0) ? 1.0 : xz;
    for (int t = 1; t < l; ++t) {
      double s2 = ((2 * t + 1) * xz * s1 - t * x2 * s0) / (t + 1);
      s0 = s1; s1 = s2; sl = s2;
    }
    double xx = 0.5 * x2;
    double q0 = 1.0, q1 = 1.0 + a - xx;
    double wj = p.wnu[j] * sl;
    acc[0] += wj * q0;
    if (p.K >= 1) acc[1] += wj * q1;
    for (int k = 1; k < p.K; ++k) {
      double q2 = ((2 * k + 1 + a - xx) * q1 - (k + a) * q0) / (k + 1);
      q0 = q1; q1 = q2;
      acc[k + 1] += wj * q1;
    }
  }
  const double twopi = 6.283185307179586476925286766559;
  for (int k = 0; k <= p.K; ++k) p.Hg[((long)l * p.NK + k) * P + i] = twopi * nk[k] * acc[k];
  // real solid harmonics S_lm (m >= 0, cos type) of v and w in the x-z plane:
  // S_lm = N_lm x^m Pi_lm(z, r^2), Pi_mm = (2m-1)!!, Pi_{m+1,m} = (2m+1) z Pi_mm,
  // (l-m) Pi_lm = (2l-1) z Pi_{l-1,m} - (l+m-1) r^2 Pi_{l-2,m}.
  for (int m = 0; m <= l; ++m) {
    double dfac = 1.0;
    for (int t = 1; t <= m; ++t) dfac *= (2 * t - 1);
    double pv0 = dfac, pw0 = dfac, pv1 = 0, pw1 = 0, pv = dfac, pw = dfac;
    if (l > m) {
      pv1 = (2 * m + 1) * vz * dfac; pw1 = (2 * m + 1) * wz * dfac;
      pv = pv1; pw = pw1;
      for (int t = m + 2; t <= l; ++t) {
        double nv = ((2 * t - 1) * vz * pv1 - (t + m - 1) * v2 * pv0) / (t - m);
        double nw = ((2 * t - 1) * wz * pw1 - (t + m - 1) * w2 * pw0) / (t - m);
        pv0 = pv1; pv1 = nv; pw0 = pw1; pw1 = nw;
        pv = nv; pw = nw;
      }
    }
    double xm_v = 1.0, xm_w = 1.0;
    for (int t = 0; t < m; ++t) { xm_v *= vx; xm_w *= wx; }
    int lm = l * (l + 1) / 2 + m;
    p.Sv[(long)lm * P + i] = p.NlmR[lm] * xm_v * pv;
    p.Sw[(long)lm * P + i] = p.NlmR[lm] * xm_w * pw;
  }
  // bi-solid Legendre Pi_l(v, w) = (|v||w|)^l P_l(cos beta)
  double vw = vx * wx + vz * wz, b = v2 * w2;
  double b0 = 1.0, b1 = vw, bl = (l == 0) ? 1.0 : vw;
  for (int t = 1; t < l; ++t) {
    double b2 = ((2 * t + 1) * vw * b1 - t * b * b0) / (t + 1);
    b0 = b1; b1 = b2; bl = b2;
  }
  p.Bi[(long)l * P + i] = bl;
  if (l == 0) p.V2[i] = v2;
}

struct GainParams {
  int P, K, L, NK, nt, ne;
  const double* G;       // [P]
  const double* u;       // [P]
  const double* mu;      // [P]
  const double* t;       // [nt] Gauss-Legendre nodes in cos chi
  const double* wt;      // [nt] weight * beta(t) * 2pi / ne
  const double* ce;      // [ne] cos of the azimuth nodes
  const double* se;      // [ne] sin of the azimuth nodes
  const double* Nkl;     // [L+1][NK]
  const double* NlmR;    // [(L+1)(L+2)/2]
  double* A;             // [(L+1)(L+2)/2][NK][P] gain averages A_klm
};

// 1/n for n = 1..17: the recurrences below divide only by these small integers.
__constant__ double kRecip[18] = {0.0,       1.0,       1.0 / 2,  1.0 / 3,  1.0 / 4,  1.0 / 5,
                                  1.0 / 6,   1.0 / 7,   1.0 / 8,  1.0 / 9,  1.0 / 10, 1.0 / 11,
                                  1.0 / 12,  1.0 / 13,  1.0 / 14, 1.0 / 15, 1.0 / 16, 1.0 / 17};

// Thread per (node, l, m >= 0): the beta-weighted gain sphere average of phi_klm for all k.
// Threads of a wavefront share (l, m) except at P boundaries, so the loops are uniform.
__global__ __launch_bounds__(256) void core_gain_angular_kernel(GainParams p) {
  const long P = p.P;
  const int NLM = (p.L + 1) * (p.L + 2) / 2;
  const long tid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= P * NLM) return;
  const int lm = (int)(tid / P);
  const long i = tid % P;
  int l = 0;
  while ((l + 1) * (l + 2) / 2 <= lm) ++l;
  const int m = lm - l * (l + 1) / 2;
  const double G = p.G[i], r = 0.5 * p.u[i], mu = p.mu[i];
  const double st = sqrt(fmax(0.0, 1.0 - mu * mu));
  const double a = l + 0.5;
  double dfac = 1.0;
  for (int j = 1; j <= m; ++j) dfac *= (2 * j - 1);
  double acc[17];
#pragma unroll
  for (int k = 0; k < 17; ++k) acc[k] = 0.0;
  for (int it = 0; it < p.nt; ++it) {
    const double t = p.t[it], sn = sqrt(fmax(0.0, 1.0 - t * t));
    // n = t u_hat + sn (cos eps e1 + sin eps e2): u_hat = (st, 0, mu), e1 = (mu, 0, -st), e2 = y
    const double bx = t * st, bz = t * mu, cx = sn * mu, cz = -sn * st;
    for (int ie = 0; ie < p.ne; ++ie) {
      const double ce = p.ce[ie], se = p.se[ie];
      const double xx = r * (bx + cx * ce), xy = r * sn * se, xz = G + r * (bz + cz * ce);
      const double x2 = xx * xx + xy * xy + xz * xz;
      // cos-type solid harmonic: Re((x + i y)^m) Pi_lm(z, |x|^2)
      double re = 1.0, im = 0.0;
      for (int j = 0; j < m; ++j) {
        const double nr = re * xx - im * xy;
        im = re * xy + im * xx;
        re = nr;
      }
      double pl = dfac;
      if (l > m) {
        double p0 = dfac, p1 = (2 * m + 1) * xz * dfac;
        pl = p1;
        for (int j = m + 2; j <= l; ++j) {
          const double p2 = ((2 * j - 1) * xz * p1 - (j + m - 1) * x2 * p0) * kRecip[j - m];
          p0 = p1; p1 = p2; pl = p2;
        }
      }
      const double w = p.wt[it] * re * pl;
      const double xh = 0.5 * x2;
      double q0 = 1.0, q1 = 1.0 + a - xh;
      acc[0] += w;
      if (p.K >= 1) acc[1] += w * q1;
#pragma unroll
      for (int k = 1; k < 16; ++k) {
        if (k < p.K) {
          const double q2 = ((2 * k + 1 + a - xh) * q1 - (k + a) * q0) * kRecip[k + 1];
          q0 = q1; q1 = q2;
          acc[k + 1] += w * q1;
        }
      }
    }
  }
  const double* nk = p.Nkl + (long)l * p.NK;
  const double nlm = p.NlmR[lm];
#pragma unroll
  for (int k = 0; k < 17; ++k)
    if (k <= p.K) p.A[((long)lm * p.NK + k) * P + i] = nlm * nk[k] * acc[k];
}

struct ChanParams {
  int P, NK, L;
  const double* W;       // [P] node weights
  const double* Pv;
  const double* Pw;
  const double* Hg;
  const double* Sv;
  const double* Sw;
  const double* Bi;
  const double* V2;
  const int* cl;          // [NT][3]
  const double* gz;       // [NT][L+1]: g(l1 0, l2 m, l3 m) * Y_l1,0(z)
  const double* gl;       // [NT]: 4pi Y_l1,0 Y_l2,0 Y_l3,0 (z) g(l1 0, l2 0, l3 0)
  const double* invS;     // [NT]
  double* R;              // [NT][NK^3]
  const double* A;        // angular factor: gain averages [(L+1)(L+2)/2][NK][P]; null when isotropic
  const int* eoff;        // [NT*17+1] ranges of the cos-type Gaunt entries per (channel, m1)
  const int* emm;         // m2 | m3 << 8 (all m >= 0)
  const double* eg;       // g(l1 m1, l2 m2, l3 m3)
};

constexpr int NODE_BLOCK = 64;
constexpr int ROW = 18;                    // LDS row stride in doubles: 16-byte aligned rows

// One workgroup per channel; thread t owns the (k1, k2) pair t and all NK values of k3,
// held in registers (NK is a template parameter so that the accumulators are not
// indexed at run time).
template <int NK>
__global__ __launch_bounds__(320) void core_accumulate_kernel(ChanParams p) {
  const int c = blockIdx.x;
  const int l1 = p.cl[3 * c], l2 = p.cl[3 * c + 1], l3 = p.cl[3 * c + 2];
  const long P = p.P;
  __shared__ __align__(16) double sX[NODE_BLOCK][ROW];
  __shared__ __align__(16) double sA[NODE_BLOCK][ROW];
  __shared__ __align__(16) double sB[NODE_BLOCK][ROW];
  __shared__ double sig[NODE_BLOCK][2];
  __shared__ double sS[NODE_BLOCK][17];     // per-node gain sums over m2, m3 for each m1
  const int t = threadIdx.x;
  const int k1 = t / NK, k2 = t % NK;
  const bool active = t < NK * NK;
  double acc[NK];
#pragma unroll
  for (int k = 0; k < NK; ++k) acc[k] = 0.0;
  const int mmax = l2 < l3 ? l2 : l3;
  const int epow = (l1 + l2 - l3) / 2;
  for (long p0 = 0; p0 < P; p0 += NODE_BLOCK) {
    int nb = (int)((P - p0) < NODE_BLOCK ? (P - p0) : NODE_BLOCK);
    if (p.A) {
      // gain sums per (node, m1), spread over the whole workgroup
      for (int w = t; w < nb * (l1 + 1); w += blockDim.x) {
        const int j = w % nb, m1 = w / nb;
        const long i = p0 + j;
        double a = 0.0;
        for (int e = p.eoff[c * 17 + m1]; e < p.eoff[c * 17 + m1 + 1]; ++e) {
          const int mm = p.emm[e];
          a += p.eg[e] * p.Sv[(long)(l2 * (l2 + 1) / 2 + (mm & 255)) * P + i] *
               p.Sw[(long)(l3 * (l3 + 1) / 2 + (mm >> 8)) * P + i];
        }
        sS[j][m1] = a * p.W[i];
      }
    }
    if (t < nb) {
      long i = p0 + t;
      double sg = 0.0;
      if (!p.A) {
        for (int m = 0; m <= mmax; ++m)
          sg += p.gz[(long)c * (p.L + 1) + m] * p.Sv[(long)(l2 * (l2 + 1) / 2 + m) * P + i] *
                p.Sw[(long)(l3 * (l3 + 1) / 2 + m) * P + i];
      }
      double vp = 1.0, v2 = p.V2[i];
      for (int e = 0; e < epow; ++e) vp *= v2;
      double sl = p.gl[c] * p.Bi[(long)l3 * P + i] * vp;
      sig[t][0] = sg * p.W[i];
      sig[t][1] = sl * p.W[i];
    }
    __syncthreads();
    for (int e = t; e < nb * NK; e += blockDim.x) {
      int j = e / NK, k = e % NK;
      long i = p0 + j;
      double gain;
      if (p.A) {
        gain = 0.0;
        for (int m1 = 0; m1 <= l1; ++m1)
          gain += sS[j][m1] * p.A[((long)(l1 * (l1 + 1) / 2 + m1) * NK + k) * P + i];
      } else {
        gain = sig[j][0] * p.Hg[((long)l1 * NK + k) * P + i];
      }
      sX[j][k] = gain - sig[j][1] * p.Pv[((long)l1 * NK + k) * P + i];
      sA[j][k] = p.Pv[((long)l2 * NK + k) * P + i];
      sB[j][k] = p.Pw[((long)l3 * NK + k) * P + i];
    }
    __syncthreads();
    if (active) {
      for (int j = 0; j < nb; ++j) {
        const double xa = sX[j][k1] * sA[j][k2];
#pragma unroll
        for (int k3 = 0; k3 < NK; ++k3) acc[k3] += xa * sB[j][k3];
      }
    }
    __syncthreads();
  }
  if (active) {
    const double s = p.invS[c];
#pragma unroll
    for (int k3 = 0; k3 < NK; ++k3)
      p.R[(long)c * NK * NK * NK + ((long)k1 * NK + k2) * NK + k3] = acc[k3] * s;
  }
}

static void launch_accumulate(int NK, int NT, hipStream_t stream, const ChanParams& cp) {
  const dim3 grid(NT), block(((NK * NK + 63) / 64) * 64);
  switch (NK) {
#define WEFQ_ACC_CASE(n) \
    case n: hipLaunchKernelGGL(core_accumulate_kernel<n>, grid, block, 0, stream, cp); break;
    WEFQ_ACC_CASE(1) WEFQ_ACC_CASE(2) WEFQ_ACC_CASE(3) WEFQ_ACC_CASE(4) WEFQ_ACC_CASE(5) WEFQ_ACC_CASE(6)
    WEFQ_ACC_CASE(7) WEFQ_ACC_CASE(8) WEFQ_ACC_CASE(9) WEFQ_ACC_CASE(10) WEFQ_ACC_CASE(11) WEFQ_ACC_CASE(12)
    WEFQ_ACC_CASE(13) WEFQ_ACC_CASE(14) WEFQ_ACC_CASE(15) WEFQ_ACC_CASE(16) WEFQ_ACC_CASE(17)
#undef WEFQ_ACC_CASE
    default: break;
  }
}

#define HIPCHK(x)                                                                    \
  do {                                                                               \
    hipError_t e_ = (x);                                                             \
    if (e_ != hipSuccess) {                                                          \
      set_error(std::string("HIP error in core build: ") + hipGetErrorString(e_));   \
      return false;                                                                  \
    }                                                                                \
  } while (0)

bool build_radial_core(wefq_core* h, const std::vector<CooRow>& coo, hipStream_t stream) {
  const int K = h->K, L = h->L, NK = h->NK, NT = h->NT;
  const int D = 2 * K + L;
  // point counts exact for the polynomial degree 3D of the integrand (Section 3.3), plus the
  // caller's padding: rad_pad more points in each radial rule, ang_pad more in each angular one
  const int nsig = (3 * D) / 2 / 2 + 1 + h->rad_pad;
  const int nmu = (3 * D) / 2 + 1 + h->ang_pad;
  const int nnu = (K + L) / 2 + 1 + h->ang_pad;
  std::vector<double> xs, ws, xu, wu, xm, wm, xn, wn;
  gauss_rule(1, nsig, 0.5, xs, ws);                  // sigma = G^2, weight sigma^{1/2} e^{-sigma}
  gauss_rule(1, nsig, 0.5 * (1.0 + h->gamma), xu, wu); // s = u^2/4, weight s^{(1+gamma)/2} e^{-s}
  gauss_rule(0, nmu, 0.0, xm, wm);
  gauss_rule(0, nnu, 0.0, xn, wn);
  const long P = (long)nsig * nsig * nmu;
  h->quad_nodes = P;
  // angular factor: beta-weighted Gauss-Legendre rule in cos chi (exact to degree D + J,
  // the degree of phi(G + r n) in n plus that of beta) and a trapezoid rule of D + 1
  // azimuths (exact for trigonometric degree D)
  const bool angular = !h->beta.empty();
  const int J = angular ? (int)h->beta.size() - 1 : 0;
  const int nt = angular ? (D + J) / 2 + 1 + h->ang_pad : 0, ne = angular ? D + 1 + h->ang_pad : 0;
  std::vector<double> tt, wt, ce, se;
  double loss_scale = 1.0;                           // int dn beta(u_hat . n) / (4 pi)
  if (angular) {
    const double pi_ = 3.141592653589793238462643383279502884;
    std::vector<double> w_t;
    gauss_rule(0, nt, 0.0, tt, w_t);
    wt.resize(nt);
    double bint = 0.0;
    for (int a = 0; a < nt; ++a) {
      double p0 = 1.0, p1 = tt[a], b = h->beta[0];
      for (int j = 1; j <= J; ++j) {
        b += h->beta[j] * p1;
        const double p2 = ((2 * j + 1) * tt[a] * p1 - j * p0) / (j + 1);
        p0 = p1; p1 = p2;
      }
      wt[a] = w_t[a] * b * 2 * pi_ / ne;
      bint += w_t[a] * b;
    }
    loss_scale = 2 * pi_ * bint / (4 * pi_);
    ce.resize(ne); se.resize(ne);
    for (int j = 0; j < ne; ++j) { ce[j] = std::cos(2 * pi_ * j / ne); se[j] = std::sin(2 * pi_ * j / ne); }
  }
  const double pi = 3.141592653589793238462643383279502884;
  const double pref = h->b0 * std::pow(2 * pi, -3.0) * 8 * pi * pi * 0.5 * std::pow(2.0, 2.0 + h->gamma);
  std::vector<double> G(P), U(P), MU(P), W(P);
  long n = 0;
  for (int a = 0; a < nsig; ++a)
    for (int b = 0; b < nsig; ++b)
      for (int c = 0; c < nmu; ++c, ++n) {
        G[n] = std::sqrt(xs[a]);
        U[n] = 2.0 * std::sqrt(xu[b]);
        MU[n] = xm[c];
        W[n] = pref * ws[a] * wu[b] * wm[c];
      }
  // radial and angular normalizations
  std::vector<double> Nkl((L + 1) * NK), NlmR((L + 1) * (L + 2) / 2);
  for (int l = 0; l <= L; ++l)
    for (int k = 0; k < NK; ++k)
      Nkl[l * NK + k] = std::exp(0.5 * (1.5 * std::log(2 * pi) + std::lgamma(k + 1.0) -
                                        (l + 0.5) * std::log(2.0) - std::lgamma(k + l + 1.5)));
  for (int l = 0; l <= L; ++l)
    for (int m = 0; m <= l; ++m) {
      double r = (2 * l + 1) / (4 * pi) * std::exp(std::lgamma(l - m + 1.0) - std::lgamma(l + m + 1.0));
      NlmR[l * (l + 1) / 2 + m] = std::sqrt(m == 0 ? r : 2 * r);
    }
  // per-channel Gaunt factors
  std::vector<int> cl(3 * NT);
  std::vector<double> gz((size_t)NT * (L + 1), 0.0), gl(NT), invS(NT, 0.0);
  for (const CooRow& r : coo) invS[r.c] += r.g * r.g;
  for (int c = 0; c < NT; ++c) {
    const Channel& ch = h->chans[c];
    cl[3 * c] = ch.l1; cl[3 * c + 1] = ch.l2; cl[3 * c + 2] = ch.l3;
    double y1 = std::sqrt((2 * ch.l1 + 1) / (4 * pi));
    double y2 = std::sqrt((2 * ch.l2 + 1) / (4 * pi));
    double y3 = std::sqrt((2 * ch.l3 + 1) / (4 * pi));
    for (int m = 0; m <= std::min(ch.l2, ch.l3); ++m)
      gz[(size_t)c * (L + 1) + m] = y1 * real_gaunt(ch.l1, 0, ch.l2, m, ch.l3, m);
    gl[c] = 4 * pi * loss_scale * y1 * y2 * y3 * real_gaunt(ch.l1, 0, ch.l2, 0, ch.l3, 0);
    invS[c] = invS[c] > 0 ? 1.0 / invS[c] : 0.0;
  }
  const int NLM = (L + 1) * (L + 2) / 2;
  // cos-type Gaunt entries for the angular gain, grouped by (channel, m1): the COO rows with
  // m1, m2, m3 >= 0
  std::vector<int> eoff((size_t)NT * 17 + 1, 0), emm;
  std::vector<double> eg;
  if (angular) {
    std::vector<std::vector<std::pair<int, double>>> per((size_t)NT * 17);
    for (const CooRow& r : coo) {
      const int l1 = l_of_q(r.q1), l2 = l_of_q(r.q2), l3 = l_of_q(r.q3);
      const int m1 = r.q1 - l1 * l1 - l1, m2 = r.q2 - l2 * l2 - l2, m3 = r.q3 - l3 * l3 - l3;
      if (m1 < 0 || m2 < 0 || m3 < 0) continue;
      per[(size_t)r.c * 17 + m1].push_back({m2 | (m3 << 8), r.g});
    }
    for (size_t b = 0; b < per.size(); ++b) {
      eoff[b + 1] = eoff[b] + (int)per[b].size();
      for (auto& e : per[b]) { emm.push_back(e.first); eg.push_back(e.second); }
    }
  }
  // device buffers (temporary)
  std::vector<void*> tmp;
  auto dalloc = [&](size_t bytes) -> double* {
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
    tmp.push_back(p);
    return (double*)p;
  };
  auto cleanup = [&]() { for (void* p : tmp) (void)hipFree(p); };
  double *dG = dalloc(P * 8), *dU = dalloc(P * 8), *dMU = dalloc(P * 8), *dW = dalloc(P * 8);
  double *dnu = dalloc(nnu * 8), *dwnu = dalloc(nnu * 8), *dNkl = dalloc(Nkl.size() * 8), *dNlm = dalloc(NlmR.size() * 8);
  size_t rad = (size_t)(L + 1) * NK * P;
  double *dPv = dalloc(rad * 8), *dPw = dalloc(rad * 8), *dHg = dalloc(rad * 8);
  double *dSv = dalloc((size_t)NLM * P * 8), *dSw = dalloc((size_t)NLM * P * 8);
  double *dBi = dalloc((size_t)(L + 1) * P * 8), *dV2 = dalloc(P * 8);
  double *dgz = dalloc(gz.size() * 8), *dgl = dalloc(NT * 8), *dinvS = dalloc(NT * 8);
  int* dcl = (int*)dalloc(cl.size() * sizeof(int));
  double* dR = dalloc((size_t)NT * NK * NK * NK * 8);
  double *dA = nullptr, *dtt = nullptr, *dwt = nullptr, *dce = nullptr, *dse = nullptr, *deg = nullptr;
  int *deoff = nullptr, *demm = nullptr;
  if (angular) {
    dA = dalloc((size_t)NLM * NK * P * 8);
    dtt = dalloc(nt * 8); dwt = dalloc(nt * 8); dce = dalloc(ne * 8); dse = dalloc(ne * 8);
    deoff = (int*)dalloc(eoff.size() * sizeof(int));
    demm = (int*)dalloc(std::max<size_t>(1, emm.size()) * sizeof(int));
    deg = dalloc(std::max<size_t>(1, eg.size()) * 8);
  }
  for (void* p : tmp)
    if (!p) { cleanup(); set_error("device allocation failed in core build"); return false; }
  bool ok = true;
  auto up = [&](void* d, const void* s, size_t bytes) {
    if (ok && hipMemcpyAsync(d, s, bytes, hipMemcpyHostToDevice, stream) != hipSuccess) ok = false;
  };
  up(dG, G.data(), P * 8); up(dU, U.data(), P * 8); up(dMU, MU.data(), P * 8); up(dW, W.data(), P * 8);
  up(dnu, xn.data(), nnu * 8); up(dwnu, wn.data(), nnu * 8);
  up(dNkl, Nkl.data(), Nkl.size() * 8); up(dNlm, NlmR.data(), NlmR.size() * 8);
  up(dgz, gz.data(), gz.size() * 8); up(dgl, gl.data(), NT * 8); up(dinvS, invS.data(), NT * 8);
  up(dcl, cl.data(), cl.size() * sizeof(int));
  if (angular) {
    up(dtt, tt.data(), nt * 8); up(dwt, wt.data(), nt * 8); up(dce, ce.data(), ne * 8); up(dse, se.data(), ne * 8);
    up(deoff, eoff.data(), eoff.size() * sizeof(int));
    if (!emm.empty()) { up(demm, emm.data(), emm.size() * sizeof(int)); up(deg, eg.data(), eg.size() * 8); }
  }
  if (!ok) { cleanup(); set_error("upload failed in core build"); return false; }
  NodeParams np{(int)P, K, L, NK, nnu, dG, dU, dMU, dnu, dwnu, dNkl, dNlm, dPv, dPw, dHg, dSv, dSw, dBi, dV2};
  long threads = P * (L + 1);
  hipLaunchKernelGGL(core_nodes_kernel, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, stream, np);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) { cleanup(); set_error(std::string("core node kernel: ") + hipGetErrorString(e)); return false; }
  if (angular) {
    GainParams gp{(int)P, K, L, NK, nt, ne, dG, dU, dMU, dtt, dwt, dce, dse, dNkl, dNlm, dA};
    const long gthreads = P * NLM;
    hipLaunchKernelGGL(core_gain_angular_kernel, dim3((unsigned)((gthreads + 255) / 256)), dim3(256), 0, stream, gp);
    e = hipGetLastError();
    if (e != hipSuccess) { cleanup(); set_error(std::string("core gain kernel: ") + hipGetErrorString(e)); return false; }
  }
  ChanParams cp{(int)P, NK, L, dW, dPv, dPw, dHg, dSv, dSw, dBi, dV2, dcl, dgz, dgl, dinvS, dR,
                dA, deoff, demm, deg};
  launch_accumulate(NK, NT, stream, cp);
  e = hipGetLastError();
  if (e != hipSuccess) { cleanup(); set_error(std::string("core accumulate kernel: ") + hipGetErrorString(e)); return false; }
  h->R64.assign((size_t)NT * NK * NK * NK, 0.0);
  e = hipMemcpyAsync(h->R64.data(), dR, h->R64.size() * 8, hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  cleanup();
  if (e != hipSuccess) { set_error(std::string("core build: ") + hipGetErrorString(e)); return false; }
  return true;
}

}  // namespace wefq
