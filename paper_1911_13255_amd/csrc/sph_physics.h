// Per-particle and per-pair physics of the multi-resolution SPH FSI method in
// FP32, as device functions shared by the kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "sph_types.h"

namespace mrsph {

// Wendland C2 kernel with support 2h (the paper's "5th-order Wendland",
// Section 4 preamble): W = alpha (1 - q/2)^4 (1 + 2q), dW/dr = -5 alpha q (1 - q/2)^3 / h.
__device__ __forceinline__ void wendland(float r, float inv_h, float alpha, float &W, float &dW) {
  float q = r * inv_h;
  float t = 1.0f - 0.5f * q;
  float t3 = t * t * t;
  W = alpha * t3 * t * (1.0f + 2.0f * q);
  dW = -5.0f * alpha * q * t3 * inv_h;
}

__device__ __forceinline__ float wendland_dW(float r, float inv_h, float alpha) {
  float q = r * inv_h;
  float t = 1.0f - 0.5f * q;
  return -5.0f * alpha * q * t * t * t * inv_h;
}

// Tait equation of state (Section 2.1) as a function of eps = rho/rho0 - 1.
// For gamma = 7, (1+eps)^7 - 1 is expanded by the binomial theorem so that
// small density excesses keep full FP32 relative precision.
__device__ __forceinline__ float eos_p(float eps, const ScenePar &P) {
  if (P.gamma == 7.0f) {
    float poly = 7.0f + eps * (21.0f + eps * (35.0f + eps * (35.0f + eps * (21.0f + eps * (7.0f + eps)))));
    return P.p_coef * eps * poly;
  }
  return P.p_coef * expm1f(P.gamma * log1pf(eps));
}

// The same inside pair loops: `tait7` is true when every lane of the
// wavefront belongs to a gamma = 7 scene (a uniform branch, so the general
// power is not evaluated beside the polynomial).
__device__ __forceinline__ float eos_p_pair(float eps, const ScenePar &P, bool tait7) {
  if (tait7) {
    float poly = 7.0f + eps * (21.0f + eps * (35.0f + eps * (35.0f + eps * (21.0f + eps * (7.0f + eps)))));
    return P.p_coef * eps * poly;
  }
  return eos_p(eps, P);
}

// Reciprocal with the hardware approximation (1 ulp); for pair-loop
// quotients that do not have to round like the coupling force's.
__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
// Square root with the hardware approximation (1 ulp), same use.
__device__ __forceinline__ float fast_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }

// Inverse: eps of the density at pressure p, with the bracket
// 1 + gamma p / (rho0 c^2) clipped at 0 (zero density under extreme tension).
__device__ __forceinline__ float eos_eps(float p, const ScenePar &P) {
  float s = P.gam_inv_rho0c2 * p;
  if (s <= -1.0f) return -1.0f;
  return expm1f(log1pf(s) / P.gamma);
}

template <int DIM>
__device__ __forceinline__ float dotv(const float *a, const float *b) {
  float s = a[0] * b[0] + a[1] * b[1];
  if (DIM == 3) s += a[2] * b[2];
  return s;
}

// Inter-particle Riemann problem along e = e_ij, left state i, right state j
// (Section 2.2; linearised acoustic solver with a limited dissipation):
//   U_L = -v_i.e, U_R = -v_j.e, rho_bar = (rho_i + rho_j)/2,
//   P* = (p_i + p_j)/2 + rho_bar beta (U_L - U_R)/2, beta = min(3 max(U_L - U_R, 0), c),
//   U* = (U_L + U_R)/2 + (p_i - p_j) / (2 rho_bar c),
//   v* = (v_i + v_j)/2 - (U* - (U_L + U_R)/2) e.
// riemann = 0 selects the simple averages.
template <int DIM>
__device__ __forceinline__ float riemann_pressure(const ScenePar &P, float rho_i, float rho_j, float p_i,
                                                  float p_j, const float *vi, const float *vj,
                                                  const float *e) {
  float pavg = 0.5f * (p_i + p_j);
  if (!P.riemann) return pavg;
  float UL = -dotv<DIM>(vi, e), UR = -dotv<DIM>(vj, e);
  float du = UL - UR;
  float beta = fminf(3.0f * fmaxf(du, 0.0f), P.c);
  return pavg + 0.5f * (0.5f * (rho_i + rho_j)) * beta * du;
}

// (v_i - v*) . e, the projection that the continuity equation needs.
template <int DIM>
__device__ __forceinline__ float riemann_dv_dot_e(const ScenePar &P, float rho_i, float rho_j, float p_i,
                                                  float p_j, const float *vi, const float *vj,
                                                  const float *e) {
  // v_i - v* = (v_i - v_j)/2 + (U* - (U_L+U_R)/2) e, and e.e = 1
  float half = 0.5f * (dotv<DIM>(vi, e) - dotv<DIM>(vj, e));
  if (!P.riemann) return half;
  return half + (p_i - p_j) * fast_rcp((rho_i + rho_j) * P.c);  // / (2 rho_bar c)
}

// Force on fluid particle i from one wall or solid particle a, at h_F
// (Section 3.1, coupling forces; Section 3.2, imaginary pressure and velocity
// from the time-averaged solid state):
//   f = -2 V_i V_a (p_i rho_d + p_d rho_i)/(rho_i + rho_d) grad_i W
//       + 2 eta V_i V_a (v_i - v_d) / (|r_ia| + 0.01 h) dW/dr,
//   p_d = p_i + rho_i max(0, (abar - g).n) (r_ia . n),  v_d = 2 vbar - v_i.
// The solid side calls the same function with the same arguments and takes
// the negative; FP contraction is off so that both sides round identically.
template <int DIM>
__device__ __forceinline__ void coupling_force(const ScenePar &P, float m_i, float eh_i, float p_i,
                                                        const float *v_i, const float *rv, float4 bpos,
                                                        float4 bvbar, float4 bnrm, float *f, float *fp = nullptr) {
#pragma clang fp contract(off)
  float r2 = rv[0] * rv[0] + rv[1] * rv[1];
  if (DIM == 3) r2 += rv[2] * rv[2];
  float r = sqrtf(r2);
  float dW = wendland_dW(r, P.inv_hf, P.alpha_f);
  float rho_i = P.rho0 * (1.0f + eh_i);
  float V_i = m_i / rho_i;
  float V_a = bpos.w;
  float rn = rv[0] * bnrm.x + rv[1] * bnrm.y;
  if (DIM == 3) rn += rv[2] * bnrm.z;
  float p_d = p_i + rho_i * bvbar.w * rn;
  float rho_d = P.rho0 * (1.0f + eos_eps(p_d, P));
  float pf = (p_i * rho_d + p_d * rho_i) / (rho_i + rho_d);
  float cp = -2.0f * V_i * V_a * pf * dW / r;
  float cv = 2.0f * P.eta * V_i * V_a * dW / (r + 0.01f * P.hf);
  float vb[3] = {bvbar.x, bvbar.y, bvbar.z};
  for (int k = 0; k < DIM; ++k) {
    // v_i - v_d = 2 (v_i - vbar)
    float dv = 2.0f * (v_i[k] - vb[k]);
    f[k] = cp * rv[k] + cv * dv;
    if (fp) fp[k] = cp * rv[k];  // pressure part alone
  }
}

// ---------------------------------------------------------------- solid

// Solid stress (Section 2.1) as P B, from H = F - I, with
// C - I = H + H^T + H^T H and M = mu (C - I) + lambda q I:
//   material 0, Neo-Hookean: S = dW/dE = mu (I - C^-1) + lambda ln J C^-1,
//     evaluated as S = C^-1 M with q = ln J;
//   material 1, linear elastic in the Green-Lagrange strain (Kirchhoff):
//     S = lambda tr(E) I + 2 mu E = M with q = tr(E) = tr(C - I) / 2.
// Both forms keep the relative precision of small strains.  Returns
// P B = (I + H) S B and J = det(I + H).  T is float or double.
template <typename T>
__device__ __forceinline__ T log1p_t(T x);
template <>
__device__ __forceinline__ float log1p_t<float>(float x) { return log1pf(x); }
template <>
__device__ __forceinline__ double log1p_t<double>(double x) { return log1p(x); }

template <int DIM, typename T>
__device__ __forceinline__ void solid_PB(int material, const T *H, const T *B, T mu, T lam, T *PB, T &J) {
  T CmI[9];
  for (int i = 0; i < DIM; ++i)
    for (int j = 0; j < DIM; ++j) {
      T s = H[i * DIM + j] + H[j * DIM + i];
      for (int k = 0; k < DIM; ++k) s += H[k * DIM + i] * H[k * DIM + j];
      CmI[i * DIM + j] = s;
    }
  T Jm1;
  if (DIM == 2) {
    Jm1 = H[0] + H[3] + (H[0] * H[3] - H[1] * H[2]);
  } else {
    T tr = H[0] + H[4] + H[8];
    T m2 = (H[0] * H[4] - H[1] * H[3]) + (H[0] * H[8] - H[2] * H[6]) + (H[4] * H[8] - H[5] * H[7]);
    T d3 = H[0] * (H[4] * H[8] - H[5] * H[7]) - H[1] * (H[3] * H[8] - H[5] * H[6]) +
           H[2] * (H[3] * H[7] - H[4] * H[6]);
    Jm1 = tr + m2 + d3;
  }
  J = T(1) + Jm1;
  const bool nh = material != 1;
  T q;
  if (nh) {
    q = log1p_t<T>(Jm1);
  } else {
    q = T(0);
    for (int i = 0; i < DIM; ++i) q += CmI[i * DIM + i];
    q *= T(0.5);
  }
  T M[9];
  for (int i = 0; i < DIM; ++i)
    for (int j = 0; j < DIM; ++j) M[i * DIM + j] = mu * CmI[i * DIM + j] + (i == j ? lam * q : T(0));
  // C^-1 (Neo-Hookean) or the identity (linear elastic)
  T Ci[9];
  T inv = T(1) / (J * J);  // det C = J^2
  if (DIM == 2) {
    T c00 = T(1) + CmI[0], c11 = T(1) + CmI[3], c01 = CmI[1];
    Ci[0] = nh ? c11 * inv : T(1);
    Ci[1] = nh ? -c01 * inv : T(0);
    Ci[2] = nh ? -c01 * inv : T(0);
    Ci[3] = nh ? c00 * inv : T(1);
  } else {
    T C[9];
    for (int k = 0; k < 9; ++k) C[k] = CmI[k];
    C[0] += T(1);
    C[4] += T(1);
    C[8] += T(1);
    Ci[0] = (C[4] * C[8] - C[5] * C[7]) * inv;
    Ci[1] = (C[2] * C[7] - C[1] * C[8]) * inv;
    Ci[2] = (C[1] * C[5] - C[2] * C[4]) * inv;
    Ci[3] = (C[5] * C[6] - C[3] * C[8]) * inv;
    Ci[4] = (C[0] * C[8] - C[2] * C[6]) * inv;
    Ci[5] = (C[2] * C[3] - C[0] * C[5]) * inv;
    Ci[6] = (C[3] * C[7] - C[4] * C[6]) * inv;
    Ci[7] = (C[1] * C[6] - C[0] * C[7]) * inv;
    Ci[8] = (C[0] * C[4] - C[1] * C[3]) * inv;
    if (!nh)
      for (int k = 0; k < 9; ++k) Ci[k] = (k % 4 == 0) ? T(1) : T(0);
  }
  T S[9];
  for (int i = 0; i < DIM; ++i)
    for (int j = 0; j < DIM; ++j) {
      T s = T(0);
      for (int k = 0; k < DIM; ++k) s += Ci[i * DIM + k] * M[k * DIM + j];
      S[i * DIM + j] = s;
    }
  T Pm[9];
  for (int i = 0; i < DIM; ++i)
    for (int j = 0; j < DIM; ++j) {
      T s = S[i * DIM + j];
      for (int k = 0; k < DIM; ++k) s += H[i * DIM + k] * S[k * DIM + j];
      Pm[i * DIM + j] = s;
    }
  for (int i = 0; i < DIM; ++i)
    for (int j = 0; j < DIM; ++j) {
      T s = T(0);
      for (int k = 0; k < DIM; ++k) s += Pm[i * DIM + k] * B[k * DIM + j];
      PB[i * DIM + j] = s;
    }
}

}  // namespace mrsph
