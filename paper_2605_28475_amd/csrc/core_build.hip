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
};

constexpr int NODE_BLOCK = 32;

// One workgroup per channel; thread t owns the (k1, k2) pair t and all k3.
__global__ void core_accumulate_kernel(ChanParams p) {
  const int c = blockIdx.x;
  const int NK = p.NK;
  const int l1 = p.cl[3 * c], l2 = p.cl[3 * c + 1], l3 = p.cl[3 * c + 2];
  const long P = p.P;
  __shared__ double sX[NODE_BLOCK][17];
  __shared__ double sA[NODE_BLOCK][17];
  __shared__ double sB[NODE_BLOCK][17];
  __shared__ double sig[NODE_BLOCK][2];
  const int t = threadIdx.x;
  const int k1 = t / NK, k2 = t % NK;
  const bool active = t < NK * NK;
  double acc[17];
  for (int k = 0; k < 17; ++k) acc[k] = 0.0;
  const int mmax = l2 < l3 ? l2 : l3;
  const int epow = (l1 + l2 - l3) / 2;
  for (long p0 = 0; p0 < P; p0 += NODE_BLOCK) {
    int nb = (int)((P - p0) < NODE_BLOCK ? (P - p0) : NODE_BLOCK);
    if (t < nb) {
      long i = p0 + t;
      double sg = 0.0;
      for (int m = 0; m <= mmax; ++m)
        sg += p.gz[(long)c * (p.L + 1) + m] * p.Sv[(long)(l2 * (l2 + 1) / 2 + m) * P + i] *
              p.Sw[(long)(l3 * (l3 + 1) / 2 + m) * P + i];
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
      sX[j][k] = sig[j][0] * p.Hg[((long)l1 * NK + k) * P + i] - sig[j][1] * p.Pv[((long)l1 * NK + k) * P + i];
      sA[j][k] = p.Pv[((long)l2 * NK + k) * P + i];
      sB[j][k] = p.Pw[((long)l3 * NK + k) * P + i];
    }
    __syncthreads();
    if (active) {
      for (int j = 0; j < nb; ++j) {
        double xa = sX[j][k1] * sA[j][k2];
        for (int k3 = 0; k3 < NK; ++k3) acc[k3] += xa * sB[j][k3];
      }
    }
    __syncthreads();
  }
  if (active) {
    double s = p.invS[c];
    for (int k3 = 0; k3 < NK; ++k3)
      p.R[(long)c * NK * NK * NK + ((long)k1 * NK + k2) * NK + k3] = acc[k3] * s;
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
  const int nsig = (3 * D) / 2 / 2 + 1;
  const int nmu = (3 * D) / 2 + 1;
  const int nnu = (K + L) / 2 + 1;
  std::vector<double> xs, ws, xu, wu, xm, wm, xn, wn;
  gauss_rule(1, nsig, 0.5, xs, ws);                  // sigma = G^2, weight sigma^{1/2} e^{-sigma}
  gauss_rule(1, nsig, 0.5 * (1.0 + h->gamma), xu, wu); // s = u^2/4, weight s^{(1+gamma)/2} e^{-s}
  gauss_rule(0, nmu, 0.0, xm, wm);
  gauss_rule(0, nnu, 0.0, xn, wn);
  const long P = (long)nsig * nsig * nmu;
  h->quad_nodes = P;
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
    gl[c] = 4 * pi * y1 * y2 * y3 * real_gaunt(ch.l1, 0, ch.l2, 0, ch.l3, 0);
    invS[c] = invS[c] > 0 ? 1.0 / invS[c] : 0.0;
  }
  const int NLM = (L + 1) * (L + 2) / 2;
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
  if (!ok) { cleanup(); set_error("upload failed in core build"); return false; }
  NodeParams np{(int)P, K, L, NK, nnu, dG, dU, dMU, dnu, dwnu, dNkl, dNlm, dPv, dPw, dHg, dSv, dSw, dBi, dV2};
  long threads = P * (L + 1);
  hipLaunchKernelGGL(core_nodes_kernel, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, stream, np);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) { cleanup(); set_error(std::string("core node kernel: ") + hipGetErrorString(e)); return false; }
  ChanParams cp{(int)P, NK, L, dW, dPv, dPw, dHg, dSv, dSw, dBi, dV2, dcl, dgz, dgl, dinvS, dR};
  int bs = ((NK * NK + 63) / 64) * 64;
  hipLaunchKernelGGL(core_accumulate_kernel, dim3(NT), dim3(bs), 0, stream, cp);
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
