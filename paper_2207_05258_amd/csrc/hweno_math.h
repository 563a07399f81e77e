// Device math of the L-HWENO hot path for gfx950 (header-only, templated on
// the real type).  Zhang & Zhao, arXiv 2207.05258, Section 2.
//
// Everything here is per-lane scalar code: the stencil work is a VALU problem
// (every interface has its own 4x4 eigenbasis, so there is no shared-operand
// contraction for MFMA).  The formulas are rearranged for few divisions:
//   * the convex combination of Sections 2.1/2.2 is evaluated with a single
//     division in FP64 (numerator and denominator scaled by the product of
//     the three (beta_l + eps)) and with hardware reciprocals in FP32;
//   * the Euler characteristic projection L = R^{-1} and back projection R
//     use the closed-form eigenvectors and their shared sub-expressions;
//   * the linear derivative flux h-hat = p0'^+ + p0'^- is pre-combined over
//     the four stencil points (one set of coefficients on F, U, A U_n, U_n).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

// math below is host+device so that it can be unit-checked on the CPU
#define HW_HD __host__ __device__ __forceinline__

namespace hweno {

enum { PH_LINADV = 0, PH_BURGERS = 1, PH_EULER = 2 };

template <int PHYS, int DIM>
struct Comps {
  static constexpr int M = (PHYS == PH_EULER) ? (DIM == 1 ? 3 : 4) : 1;
  static constexpr int NF = M * (1 + DIM);
};

template <typename T>
struct Weights {
  T g0, g1, g2;  // linear weights, positive, summing to one
  T eps;         // epsilon of the nonlinear weights
  T gs;          // g0 + g1 + g2
};

template <typename T>
struct Consts {
  Weights<T> rw;  // reconstruction weights gamma_l (Section 2.1)
  Weights<T> lw;  // limiter weights d_l (Section 2.2)
  T gm1;          // gamma_gas - 1
  T gam;          // gamma_gas
  T ax, ay;       // advection speeds (linear advection)
  int characteristic;
  int limiter_on;
  int limiter_char;  // Euler: limiter on characteristic fields of each cell
};

// Reciprocal, quotient and reciprocal square root of finite, positive,
// normal arguments (densities, squared sound speeds, sums of positive
// weights) without the IEEE special-case scaling of the library routines.
// FP32: the hardware instructions (1 ulp).  FP64: the hardware approximation
// (relative error about 2^-24 on gfx950, measured) refined by one Newton step,
// which leaves about 2^-48; a quotient gets one residual correction on top
// (about 1 ulp).  The host build of the math (CPU unit checks) divides.
template <typename T>
HW_HD T fast_rcp(T x);
template <>
HW_HD float fast_rcp<float>(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_rcpf(x);  // v_rcp_f32
#else
  return 1.0f / x;
#endif
}
template <>
HW_HD double fast_rcp<double>(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
  const double r = __builtin_amdgcn_rcp(x);  // v_rcp_f64
  return fma(r, fma(-x, r, 1.0), r);
#else
  return 1.0 / x;
#endif
}

template <typename T>
HW_HD T fast_div(T n, T d) {
#if defined(__HIP_DEVICE_COMPILE__)
  const T r = fast_rcp(d);
  const T q = n * r;
  if constexpr (sizeof(T) == 8) return fma(fma(-d, q, n), r, q);
  return q;
#else
  return n / d;
#endif
}

template <typename T>
HW_HD T fast_rsq(T x);
template <>
HW_HD float fast_rsq<float>(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_rsqf(x);  // v_rsq_f32
#else
  return 1.0f / sqrtf(x);
#endif
}
template <>
HW_HD double fast_rsq<double>(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
  const double y = __builtin_amdgcn_rsq(x);  // v_rsq_f64
  // y <- y (3 - x y^2) / 2
  return fma(0.5 * y, fma(-x * y, y, 1.0), y);
#else
  return 1.0 / sqrt(x);
#endif
}

// ---------------------------------------------------------------------------
// Convex combination shared by the reconstruction (Section 2.1) and the
// limiter (Section 2.2):
//   tau = (|b0-b1| + |b0-b2|)^2 / 4,  wbar_l = g_l (1 + tau/(b_l + eps)),
//   result = w0 (P0/g0 - g1/g0 P1 - g2/g0 P2) + w1 P1 + w2 P2, w = wbar/sum.
// With c_l = b_l + eps and e_l = 1 + tau/c_l this is
//   (e0 P0 + g1 P1 (e1-e0) + g2 P2 (e2-e0)) / (g0 e0 + g1 e1 + g2 e2).
// combine_c takes the c_l (FP64: callers fold eps into the sums that form the
// indicators), combine the b_l.
// ---------------------------------------------------------------------------
template <typename T>
HW_HD T combine_c(T P0, T P1, T P2, T c0, T c1, T c2, const Weights<T>& w) {
  T tau = fabs(c0 - c1) + fabs(c0 - c2);
  tau = T(0.25) * tau * tau;
  // numerator and denominator times P = c0 c1 c2 (one division):
  //   num = P P0 + tau (c1 c2 P0 + g1 P1 c2 (c0 - c1) + g2 P2 c1 (c0 - c2)),
  //   den = (g0 + g1 + g2) P + tau (g0 c1 c2 + g1 c0 c2 + g2 c0 c1)
  const T c12 = c1 * c2;
  const T P = c0 * c12;
  const T N = fma(c12, P0, fma(w.g1 * P1 * c2, c0 - c1, w.g2 * P2 * c1 * (c0 - c2)));
  const T D = fma(w.g0, c12, fma(w.g1, c0 * c2, w.g2 * (c0 * c1)));
  return fast_div(fma(P, P0, tau * N), fma(w.gs, P, tau * D));
}

template <typename T>
HW_HD T combine(T P0, T P1, T P2, T b0, T b1, T b2, const Weights<T>& w) {
  if constexpr (sizeof(T) == 8) {
    return combine_c(P0, P1, P2, b0 + w.eps, b1 + w.eps, b2 + w.eps, w);
  } else {
    // FP32: one reciprocal per weight (the products of the single-division
    // form lose FP32 accuracy when the indicators span many decades)
    T tau = fabs(b0 - b1) + fabs(b0 - b2);
    tau = T(0.25) * tau * tau;
    const T e0 = T(1) + tau * fast_rcp(b0 + w.eps);
    const T e1 = T(1) + tau * fast_rcp(b1 + w.eps);
    const T e2 = T(1) + tau * fast_rcp(b2 + w.eps);
    const T num = e0 * P0 + w.g1 * P1 * (e1 - e0) + w.g2 * P2 * (e2 - e0);
    const T den = w.g0 * e0 + w.g1 * e1 + w.g2 * e2;
    return num * fast_rcp(den);
  }
}

// Nonlinear HWENO value at x_{i+1/2} from the upwind ("+") data
// f_{i-1}, f_i, f_{i+1} and H_l = dx h_l (Section 2.1): candidate values of
// the quintic p0 and quadratics p1, p2, their smoothness indicators (beta2
// from its integral definition, eq. GHYZ) and the combination above.
template <typename T>
HW_HD T hw_plus(T fm, T f0, T fp, T Hm, T H0, T Hp,
                                     const Weights<T>& w) {
  const T s = fm + fp, dl = fm - fp, lap = s - T(2) * f0;
  const T Hs = Hm + Hp, Hd = Hm - Hp;
  const T p0 = T(11.0 / 60.0) * s + T(19.0 / 30.0) * f0 + T(0.05) * Hd + T(0.5) * H0;
  T p1, p2;
  if constexpr (sizeof(T) == 8) {
    const T q = T(5.0 / 6.0) * f0 + T(1.0 / 3.0) * H0;  // shared by p1 and p2
    p1 = T(1.0 / 6.0) * fm + (T(1.0 / 3.0) * H0 + q);
    p2 = T(1.0 / 6.0) * fp + q;
  } else {
    p1 = T(1.0 / 6.0) * (fm + T(5) * f0) + T(2.0 / 3.0) * H0;
    p2 = T(1.0 / 6.0) * (T(5) * f0 + fp) + T(1.0 / 3.0) * H0;
  }
  // beta_0 from the monomial coefficients a1..a5 of p0 in (x - x_i)/dx, i.e.
  //   (a1 + a3/4 + a5/16)^2 + 13/3 (a2 + 63/130 a4)^2 + 781/20 (a3 + 8825/10934 a5)^2
  //   + 1421461/2275 a4^2 + 21520059541/1377684 a5^2,
  // written as a sum of five squares of linear forms in (H0, Hd, lap, Hs, dl):
  // the first form reduces exactly to H0 (p0'(x_i) dx = H_i, a Hermite
  // condition), and each other one carries the square root of its weight.
  const T x1 = T(0.5284229075567874) * Hd + T(2.0976788148466414) * lap;  // sqrt(13/3)(33 Hd + 131 lap)/130
  const T x2 = T(-1.6032089149031234) * Hs + T(-12.66183557959969) * H0 +
               T(-7.934126704702969) * dl;                              // sqrt(781/20)(a3 + 8825/10934 a5)
  const T x4 = T(-6.249090043648465) * Hd + T(-12.49818008729693) * lap;  // sqrt(1421461/2275) a4
  const T x5 = T(31.24546092343706) * Hs + T(124.98184369374825) * H0 +
               T(93.73638277031118) * dl;                               // sqrt(21520059541/1377684) a5
  const T u1 = H0 - f0 + fm, u2 = H0 + f0 - fp;
  if constexpr (sizeof(T) == 8) {
    // the indicators with eps added, eps starting the sums
    const T h2e = H0 * H0 + w.eps;
    return combine_c(p0, p1, p2, h2e + x1 * x1 + x2 * x2 + x4 * x4 + x5 * x5,
                     h2e + T(13.0 / 3.0) * u1 * u1, h2e + T(13.0 / 3.0) * u2 * u2, w);
  } else {
    const T h2 = H0 * H0;
    const T b0 = h2 + x1 * x1 + x2 * x2 + x4 * x4 + x5 * x5;
    const T b1 = h2 + T(13.0 / 3.0) * u1 * u1;
    const T b2 = h2 + T(13.0 / 3.0) * u2 * u2;
    return combine(p0, p1, p2, b0, b1, b2, w);
  }
}

// HWENO limiter value v~_i (Section 2.2) from u_{i-1}, u_i, u_{i+1},
// v_{i-1}, v_{i+1}: quartic q0 and linear q1, q2, their derivatives at x_i
// and smoothness indicators.  h = dx, ih = 1/dx.
template <typename T>
HW_HD T limit1(T um, T u0, T up, T vm, T vp, T h, T ih,
                                    const Weights<T>& w) {
  const T Vs = h * (vm + vp), Vd = h * (vm - vp);
  const T lap = um - T(2) * u0 + up;
  const T D = up - um;
  const T a1 = T(0.75) * D - T(0.25) * Vs;  // = dx q0'(x_i)
  // beta_0 of q0 from its coefficients a1..a4,
  //   (a1 + a3/4)^2 + 13/3 (a2 + 63/130 a4)^2 + 781/20 a3^2 + 1421461/2275 a4^2,
  // as a sum of four squares of linear forms (weights' square roots folded in)
  const T x0 = T(11.0 / 16.0) * D - T(3.0 / 16.0) * Vs;                  // a1 + a3/4
  const T x1 = T(0.2682146576235209) * Vd + T(1.5772623149801082) * lap;  // sqrt(13/3)(a2 + 63/130 a4)
  const T x3 = T(1.5622499799967993) * (Vs - D);                         // sqrt(781/20) a3
  const T x4 = T(-6.249090043648465) * Vd + T(-12.49818008729693) * lap;  // sqrt(1421461/2275) a4
  const T d1 = u0 - um, d2 = up - u0;
  // the combination is linear in the candidates q_l' = (a1, d1, d2) / dx
  if constexpr (sizeof(T) == 8) {
    // the indicators with eps added, eps starting the sums
    return ih * combine_c(a1, d1, d2, x0 * x0 + w.eps + x1 * x1 + x3 * x3 + x4 * x4,
                          d1 * d1 + w.eps, d2 * d2 + w.eps, w);
  } else {
    return ih * combine(a1, d1, d2, x0 * x0 + x1 * x1 + x3 * x3 + x4 * x4, d1 * d1, d2 * d2, w);
  }
}

// ---------------------------------------------------------------------------
// Physics in a normal-direction frame.  For 2D Euler the components are
// ordered (rho, m_n, m_t, E): normal momentum first, so one code path serves
// both directions (y swaps the two momenta on load and store).
// ---------------------------------------------------------------------------

// flux F_n(U) and the chain-rule products A_n(U) Dn and A_n(U) Dt
// (h, xi, eta, theta of eq. EQ3), for one stencil point.
template <typename T, int PHYS, int M, bool MIXED>
HW_HD void point_fluxes(const T* U, const T* Dn, const T* Dt,
                                             const Consts<T>& k, T an, T* F,
                                             T* A, T* B) {
  if constexpr (PHYS == PH_EULER) {
    const T ir = fast_rcp(U[0]);
    const T un = U[1] * ir;
    const T ut = (M == 4) ? U[2] * ir : T(0);
    const T E = U[M - 1];
    const T q2 = un * un + ut * ut;
    const T p = k.gm1 * (E - T(0.5) * U[0] * q2);
    const T Ep = E + p;
    F[0] = U[1];
    F[1] = U[1] * un + p;
    if constexpr (M == 4) F[2] = U[1] * ut;
    F[M - 1] = un * Ep;
    auto jvp = [&](const T* D, T* out) {
      const T r = D[0], a = D[1], b = (M == 4) ? D[2] : T(0), e = D[M - 1];
      const T us = (a - un * r) * ir;
      const T ts = (b - ut * r) * ir;
      const T ps = k.gm1 * (e - un * a - ut * b + T(0.5) * q2 * r);
      out[0] = a;
      out[1] = a * un + U[1] * us + ps;
      if constexpr (M == 4) out[2] = a * ut + U[1] * ts;
      out[M - 1] = us * Ep + un * (e + ps);
    };
    jvp(Dn, A);
    if constexpr (MIXED) jvp(Dt, B);
  } else if constexpr (PHYS == PH_BURGERS) {
    F[0] = T(0.5) * U[0] * U[0];
    A[0] = U[0] * Dn[0];
    if constexpr (MIXED) B[0] = U[0] * Dt[0];
  } else {
    F[0] = an * U[0];
    A[0] = an * Dn[0];
    if constexpr (MIXED) B[0] = an * Dt[0];
  }
}

// Roe-averaged eigen-system of the normal flux Jacobian: right eigenvectors
// (1, un-c, ut, H-un c), (1, un, ut, q^2/2), (0, 0, 1, ut), (1, un+c, ut, H+un c)
// (1D drops ut), left eigenvectors = their inverse in closed form.
template <typename T, int M>
struct Eigen {
  T un, ut, H, c, ic, b1, b2, hq2;

  HW_HD void roe(const T* UL, const T* UR, T gm1) {
    // sqrt(rho) and 1/rho from one reciprocal square root per side
    const T qL = fast_rsq(UL[0]), qR = fast_rsq(UR[0]);
    const T sL = UL[0] * qL, sR = UR[0] * qR;
    const T irL = qL * qL, irR = qR * qR;
    const T uL = UL[1] * irL, uR = UR[1] * irR;
    const T tL = (M == 4) ? UL[2] * irL : T(0), tR = (M == 4) ? UR[2] * irR : T(0);
    const T pL = gm1 * (UL[M - 1] - T(0.5) * UL[0] * (uL * uL + tL * tL));
    const T pR = gm1 * (UR[M - 1] - T(0.5) * UR[0] * (uR * uR + tR * tR));
    const T HL = (UL[M - 1] + pL) * irL, HR = (UR[M - 1] + pR) * irR;
    const T iw = fast_rcp(sL + sR);
    const T wL = sL * iw, wR = sR * iw;
    un = wL * uL + wR * uR;
    ut = wL * tL + wR * tR;
    H = wL * HL + wR * HR;
    const T q2 = un * un + ut * ut;
    hq2 = T(0.5) * q2;
    const T c2 = gm1 * (H - hq2);
    ic = fast_rsq(c2);
    c = c2 * ic;
    b1 = gm1 * ic * ic;
    b2 = b1 * hq2;
  }

  // eigen-system at one state (what the Roe average of a state with itself gives)
  HW_HD void cell(const T* U, T gm1) {
    const T ir = fast_rcp(U[0]);
    un = U[1] * ir;
    ut = (M == 4) ? U[2] * ir : T(0);
    hq2 = T(0.5) * (un * un + ut * ut);
    const T p = gm1 * (U[M - 1] - U[0] * hq2);
    H = (U[M - 1] + p) * ir;
    const T c2 = gm1 * (H - hq2);
    ic = fast_rsq(c2);
    c = c2 * ic;
    b1 = gm1 * ic * ic;
    b2 = b1 * hq2;
  }

  // w = L x
  HW_HD void project(const T* x, T* w) const {
    if constexpr (M == 4) {
      const T phi = b2 * x[0] - b1 * (un * x[1] + ut * x[2] - x[3]);
      const T psi = (un * x[0] - x[1]) * ic;
      w[0] = T(0.5) * (phi + psi);
      w[1] = x[0] - phi;
      w[2] = x[2] - ut * x[0];
      w[3] = T(0.5) * (phi - psi);
    } else {
      const T phi = b2 * x[0] - b1 * (un * x[1] - x[2]);
      const T psi = (un * x[0] - x[1]) * ic;
      w[0] = T(0.5) * (phi + psi);
      w[1] = x[0] - phi;
      w[2] = T(0.5) * (phi - psi);
    }
  }

  // y = R w
  HW_HD void back(const T* w, T* y) const {
    if constexpr (M == 4) {
      const T s = w[0] + w[1] + w[3], dif = w[3] - w[0];
      y[0] = s;
      y[1] = un * s + c * dif;
      y[2] = ut * s + w[2];
      y[3] = H * (w[0] + w[3]) + un * c * dif + hq2 * w[1] + ut * w[2];
    } else {
      const T s = w[0] + w[1] + w[2], dif = w[2] - w[0];
      y[0] = s;
      y[1] = un * s + c * dif;
      y[2] = H * (w[0] + w[2]) + un * c * dif + hq2 * w[1];
    }
  }
};

// Characteristic variant of the limiter (a choice the paper leaves open for
// systems): the five stencil vectors u_{i-1}, u_i, u_{i+1}, v_{i-1}, v_{i+1}
// (normal frame) are projected with the left eigenvectors of the cell's own
// state, each characteristic field is limited as a scalar, and the right
// eigenvectors map the result back.
template <typename T, int M>
HW_HD void limit_char(const T* um, const T* u0, const T* up, const T* vm, const T* vp, T h, T ih,
                      const Weights<T>& w, T gm1, T* out) {
  Eigen<T, M> e;
  e.cell(u0, gm1);
  T a[M], b[M], c[M], dm[M], dp[M], z[M];
  e.project(um, a);
  e.project(u0, b);
  e.project(up, c);
  e.project(vm, dm);
  e.project(vp, dp);
#pragma unroll
  for (int q = 0; q < M; ++q) z[q] = limit1(a[q], b[q], c[q], dm[q], dp[q], h, ih, w);
  e.back(z, out);
}

// ---------------------------------------------------------------------------
// All fluxes of one interface x_{i+1/2} along the normal direction.
// Stencil points s = 0..3 are x_{i-1}, x_i, x_{i+1}, x_{i+2};
// ld(s, U, Dn, Dt) loads the state of point s in the normal frame.
// Outputs (normal frame): fh = f-hat (nonlinear, Section 2.1 with Remarks
// 2.1/2.2).  The two linear fluxes, h-hat (p0'^+ + p0'^-, component-wise)
// and the mixed flux of eq. (mixed) (only when MIXED), are sums of one term
// per stencil point; point s hands its terms to lin(s, c, dh, dx) as soon as
// they are formed (s = 0 first, then 1, 2, 3), so the caller can accumulate
// them where it stores them instead of keeping twelve partial sums live in
// registers across the nonlinear reconstructions.
//   alpha: global LF speed of this direction; h: cell size; ih = 1/h.
// ---------------------------------------------------------------------------
template <typename T, int PHYS, int M, bool MIXED, typename Loader, typename Lin>
HW_HD void interface_fluxes(const Loader& ld, const Lin& lin, T alpha, T h, T ih, T an,
                            const Consts<T>& k, T* fh) {
  constexpr bool CHARW = (PHYS == PH_EULER);
  Eigen<T, M> eg;
  const bool proj = CHARW && k.characteristic;
  if constexpr (CHARW) {
    if (proj) {
      T UL[M], UR[M], dn[M], dt[M];
      ld(1, UL, dn, dt);
      ld(2, UR, dn, dt);
      eg.roe(UL, UR, k.gm1);
    }
  }
  // split point data in characteristic fields: "+" side uses s = 0..2,
  // "-" side uses s = 1..3 (stored at s-1)
  T fP[3][M], HP[3][M], fM[3][M], HM[3][M];
  // linear derivative flux h-hat = p0'^+(f^+, h^+) + mirrored p0'^-(f^-, h^-),
  // expanded with f^+- = (F +- alpha U)/2, h^+- = (A Dn +- alpha Dn)/2:
  //   [F0 - 15F1 + 15F2 - F3 + alpha (U0 - U1 - U2 + U3)] / (8 dx)
  // + [A0 - 7A1 - 7A2 + A3 + alpha (D0 + 3D1 - 3D2 - D3)] / 24
  constexpr T cF[4] = {T(1), T(-15), T(15), T(-1)};
  constexpr T cU[4] = {T(1), T(-1), T(-1), T(1)};
  constexpr T cA[4] = {T(1), T(-7), T(-7), T(1)};
  constexpr T cD[4] = {T(1), T(3), T(-3), T(-1)};
  constexpr T cX[4] = {T(-1), T(7), T(7), T(-1)};
  const T hh2 = T(0.5) * h;
  const T i8 = T(0.125) * ih;
  // one stencil point: physics, linear-flux accumulation, split and projected data
  auto point = [&](const int s) {
    T U[M], Dn[M], Dt[M], F[M], A[M], B[M];
    ld(s, U, Dn, Dt);
    point_fluxes<T, PHYS, M, MIXED>(U, Dn, Dt, k, an, F, A, B);
#pragma unroll
    for (int c = 0; c < M; ++c) {
      const T dh = (cF[s] * F[c] + alpha * cU[s] * U[c]) * i8 +
                   (cA[s] * A[c] + alpha * cD[s] * Dn[c]) * T(1.0 / 24.0);
      const T dx = MIXED ? cX[s] * B[c] * T(1.0 / 12.0) : T(0);
      lin(s, c, dh, dx);
    }
    if (s <= 2) {
      T x[M], y[M];
#pragma unroll
      for (int c = 0; c < M; ++c) {
        x[c] = T(0.5) * (F[c] + alpha * U[c]);
        y[c] = hh2 * (A[c] + alpha * Dn[c]);
      }
      if (proj) {
        eg.project(x, fP[s]);
        eg.project(y, HP[s]);
      } else {
#pragma unroll
        for (int c = 0; c < M; ++c) {
          fP[s][c] = x[c];
          HP[s][c] = y[c];
        }
      }
    }
    if (s >= 1) {
      T x[M], y[M];
#pragma unroll
      for (int c = 0; c < M; ++c) {
        x[c] = T(0.5) * (F[c] - alpha * U[c]);
        y[c] = hh2 * (A[c] - alpha * Dn[c]);
      }
      if (proj) {
        eg.project(x, fM[s - 1]);
        eg.project(y, HM[s - 1]);
      } else {
#pragma unroll
        for (int c = 0; c < M; ++c) {
          fM[s - 1][c] = x[c];
          HM[s - 1][c] = y[c];
        }
      }
    }
  };
  // "+" side first (points 0..2), so its data die before point 3 is loaded
  point(0);
  point(1);
  point(2);
  T fc[M];
#pragma unroll
  for (int c = 0; c < M; ++c)
    fc[c] = hw_plus(fP[0][c], fP[1][c], fP[2][c], HP[0][c], HP[1][c], HP[2][c], k.rw);
  point(3);
  // "-" mirrored: i+2, i+1, i with derivative data negated (reflection about
  // the interface)
#pragma unroll
  for (int c = 0; c < M; ++c)
    fc[c] += hw_plus(fM[2][c], fM[1][c], fM[0][c], -HM[2][c], -HM[1][c], -HM[0][c], k.rw);
  if (proj) {
    eg.back(fc, fh);
  } else {
#pragma unroll
    for (int c = 0; c < M; ++c) fh[c] = fc[c];
  }
}

// wave speeds |u_n| + c (Euler), |u| (Burgers), |a| (linear advection) of
// one point in each direction, plus admissibility flags.
template <typename T, int PHYS, int DIM>
HW_HD void point_speeds(const T* U, const Consts<T>& k,
                                             T& sx, T& sy, uint32_t& flags) {
  if constexpr (PHYS == PH_EULER) {
    constexpr int M = Comps<PHYS, DIM>::M;
    const T r = U[0];
    const T ir = T(1) / r;
    const T u = U[1] * ir;
    const T v = (DIM == 2) ? U[2] * ir : T(0);
    const T p = k.gm1 * (U[M - 1] - T(0.5) * r * (u * u + v * v));
    const T c = sqrt(k.gam * p * ir);
    sx = fabs(u) + c;
    sy = (DIM == 2) ? fabs(v) + c : T(0);
    bool fin = true;
#pragma unroll
    for (int q = 0; q < M; ++q) fin = fin && isfinite(U[q]);
    if (!fin) flags |= 1u;
    if (!(r > T(0))) flags |= 2u;
    if (!(p > T(0))) flags |= 4u;
  } else if constexpr (PHYS == PH_BURGERS) {
    sx = fabs(U[0]);
    sy = (DIM == 2) ? sx : T(0);
    if (!isfinite(U[0])) flags |= 1u;
  } else {
    sx = fabs(k.ax);
    sy = (DIM == 2) ? fabs(k.ay) : T(0);
    if (!isfinite(U[0])) flags |= 1u;
  }
}

}  // namespace hweno
