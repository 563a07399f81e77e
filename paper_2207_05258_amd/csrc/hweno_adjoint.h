// Hand-written reverse-mode derivatives (vector-Jacobian products) of the
// device math in hweno_math.h: the discrete adjoint of the semi-discrete
// operator (eqs. odeH / ode2H with the reconstruction of Section 2.1) and of
// the limiter (Section 2.2), with the Lax-Friedrichs speeds held fixed.
//
// Conventions: every *_vjp function recomputes the forward quantities it
// needs from the same inputs and ACCUMULATES (+=) the input adjoints.
// |x| is differentiated as sign(x) with sign(0) = 0.
#pragma once

#include "hweno_math.h"

namespace hweno {

template <typename T>
HW_HD T sgn(T x) {
  return T((x > T(0)) - (x < T(0)));
}

// reverse of combine(): adjoints of P0, P1, P2 and b0, b1, b2 (overwritten);
// returns the forward value
template <typename T>
HW_HD T combine_vjp(T P0, T P1, T P2, T b0, T b1, T b2, const Weights<T>& w, T g,
                       T& gP0, T& gP1, T& gP2, T& gb0, T& gb1, T& gb2) {
  const T d01 = b0 - b1, d02 = b0 - b2;
  const T sa = fabs(d01) + fabs(d02);
  const T tau = T(0.25) * sa * sa;
  const T i0 = fast_rcp(b0 + w.eps), i1 = fast_rcp(b1 + w.eps), i2 = fast_rcp(b2 + w.eps);
  const T e0 = T(1) + tau * i0, e1 = T(1) + tau * i1, e2 = T(1) + tau * i2;
  const T iden = fast_rcp(w.g0 * e0 + w.g1 * e1 + w.g2 * e2);
  const T r = (e0 * P0 + w.g1 * P1 * (e1 - e0) + w.g2 * P2 * (e2 - e0)) * iden;
  const T gi = g * iden;
  gP0 = gi * e0;
  gP1 = gi * w.g1 * (e1 - e0);
  gP2 = gi * w.g2 * (e2 - e0);
  const T ge0 = gi * (P0 - w.g1 * P1 - w.g2 * P2 - w.g0 * r);
  const T ge1 = gi * w.g1 * (P1 - r);
  const T ge2 = gi * w.g2 * (P2 - r);
  const T gs = T(0.5) * sa * (ge0 * i0 + ge1 * i1 + ge2 * i2);  // d tau / d sa = sa / 2
  const T s01 = sgn(d01), s02 = sgn(d02);
  gb0 = -ge0 * tau * i0 * i0 + gs * (s01 + s02);
  gb1 = -ge1 * tau * i1 * i1 - gs * s01;
  gb2 = -ge2 * tau * i2 * i2 - gs * s02;
  return r;
}

// reverse of hw_plus(); returns the forward value hw_plus(...)
template <typename T>
HW_HD T hw_plus_vjp(T fm, T f0, T fp, T Hm, T H0, T Hp, const Weights<T>& w, T g, T& gfm,
                    T& gf0, T& gfp, T& gHm, T& gH0, T& gHp) {
  const T s = fm + fp, dl = fm - fp, lap = s - T(2) * f0;
  const T Hs = Hm + Hp, Hd = Hm - Hp;
  const T p0 = T(11.0 / 60.0) * s + T(19.0 / 30.0) * f0 + T(0.05) * Hd + T(0.5) * H0;
  const T p1 = T(1.0 / 6.0) * (fm + T(5) * f0) + T(2.0 / 3.0) * H0;
  const T p2 = T(1.0 / 6.0) * (T(5) * f0 + fp) + T(1.0 / 3.0) * H0;
  // beta_0 as the sum of squares of hw_plus(): H0 and four linear forms
  constexpr T c11 = T(0.5284229075567874), c12 = T(2.0976788148466414);
  constexpr T c21 = T(-1.6032089149031234), c22 = T(-12.66183557959969), c23 = T(-7.934126704702969);
  constexpr T c41 = T(-6.249090043648465), c42 = T(-12.49818008729693);
  constexpr T c51 = T(31.24546092343706), c52 = T(124.98184369374825), c53 = T(93.73638277031118);
  const T x1 = c11 * Hd + c12 * lap;
  const T x2 = c21 * Hs + c22 * H0 + c23 * dl;
  const T x4 = c41 * Hd + c42 * lap;
  const T x5 = c51 * Hs + c52 * H0 + c53 * dl;
  const T b0 = H0 * H0 + x1 * x1 + x2 * x2 + x4 * x4 + x5 * x5;
  const T u1 = H0 - f0 + fm, u2 = H0 + f0 - fp, h2 = H0 * H0;
  const T b1 = h2 + T(13.0 / 3.0) * u1 * u1;
  const T b2 = h2 + T(13.0 / 3.0) * u2 * u2;
  T gp0, gp1, gp2, gb0, gb1, gb2;
  const T value = combine_vjp(p0, p1, p2, b0, b1, b2, w, g, gp0, gp1, gp2, gb0, gb1, gb2);
  // smoothness indicators
  const T g2 = T(2) * gb0;
  const T gx1 = g2 * x1, gx2 = g2 * x2, gx4 = g2 * x4, gx5 = g2 * x5;
  const T gu1 = T(26.0 / 3.0) * u1 * gb1;
  const T gu2 = T(26.0 / 3.0) * u2 * gb2;
  T gH0_ = T(2) * H0 * (gb1 + gb2 + gb0) + gu1 + gu2 + c22 * gx2 + c52 * gx5;
  T gfm_ = gu1, gf0_ = gu2 - gu1, gfp_ = -gu2;
  // candidate values
  T gs_ = T(11.0 / 60.0) * gp0;
  gf0_ += T(19.0 / 30.0) * gp0;
  T gHd = T(0.05) * gp0;
  gH0_ += T(0.5) * gp0;
  gfm_ += T(1.0 / 6.0) * gp1;
  gf0_ += T(5.0 / 6.0) * gp1 + T(5.0 / 6.0) * gp2;
  gH0_ += T(2.0 / 3.0) * gp1 + T(1.0 / 3.0) * gp2;
  gfp_ += T(1.0 / 6.0) * gp2;
  // the linear forms of beta_0
  const T gHs = c21 * gx2 + c51 * gx5;
  const T gdl = c23 * gx2 + c53 * gx5;
  gHd += c11 * gx1 + c41 * gx4;
  const T glap = c12 * gx1 + c42 * gx4;
  gs_ += glap;
  gf0_ -= T(2) * glap;
  gfm += gfm_ + gs_ + gdl;
  gfp += gfp_ + gs_ - gdl;
  gf0 += gf0_;
  gHm += gHs + gHd;
  gHp += gHs - gHd;
  gH0 += gH0_;
  return value;
}

// reverse of limit1()
template <typename T>
HW_HD void limit1_vjp(T um, T u0, T up, T vm, T vp, T h, T ih, const Weights<T>& w, T g,
                      T& gum, T& gu0, T& gup, T& gvm, T& gvp) {
  const T Vs = h * (vm + vp), Vd = h * (vm - vp);
  const T lap = um - T(2) * u0 + up;
  const T D = up - um;
  const T a1 = T(0.75) * D - T(0.25) * Vs;
  // beta_0 as the sum of squares of limit1()
  constexpr T k11 = T(0.2682146576235209), k12 = T(1.5772623149801082), k3 = T(1.5622499799967993);
  constexpr T c41 = T(-6.249090043648465), c42 = T(-12.49818008729693);
  const T x0 = T(11.0 / 16.0) * D - T(3.0 / 16.0) * Vs;
  const T x1 = k11 * Vd + k12 * lap;
  const T x3 = k3 * (Vs - D);
  const T x4 = c41 * Vd + c42 * lap;
  const T b0 = x0 * x0 + x1 * x1 + x3 * x3 + x4 * x4;
  const T d1 = u0 - um, d2 = up - u0;
  T gP0, gP1, gP2, gb0, gb1, gb2;
  combine_vjp(a1 * ih, d1 * ih, d2 * ih, b0, d1 * d1, d2 * d2, w, g, gP0, gP1, gP2, gb0, gb1, gb2);
  const T gd1 = gP1 * ih + T(2) * d1 * gb1;
  const T gd2 = gP2 * ih + T(2) * d2 * gb2;
  const T g2 = T(2) * gb0;
  const T gx0 = g2 * x0, gx1 = g2 * x1, gx3 = g2 * x3, gx4 = g2 * x4;
  const T ga1 = gP0 * ih;
  const T gD = T(0.75) * ga1 + T(11.0 / 16.0) * gx0 - k3 * gx3;
  const T gVs = T(-0.25) * ga1 - T(3.0 / 16.0) * gx0 + k3 * gx3;
  const T gVd = k11 * gx1 + c41 * gx4;
  const T glap = k12 * gx1 + c42 * gx4;
  gup += gD + glap + gd2;
  gum += -gD + glap - gd1;
  gu0 += T(-2) * glap + gd1 - gd2;
  gvm += h * (gVs + gVd);
  gvp += h * (gVs - gVd);
}

// reverse of point_fluxes(): from adjoints of F, A = A_n Dn, B = A_n Dt
template <typename T, int PHYS, int M, bool MIXED>
HW_HD void point_fluxes_vjp(const T* U, const T* Dn, const T* Dt, const Consts<T>& k, T an,
                            const T* gF, const T* gA, const T* gB, T* gU, T* gDn, T* gDt) {
  if constexpr (PHYS == PH_EULER) {
    const T rho = U[0], mn = U[1], mt = (M == 4) ? U[2] : T(0), E = U[M - 1];
    const T ir = fast_rcp(rho);
    const T un = mn * ir, ut = mt * ir;
    const T q2 = un * un + ut * ut;
    const T p = k.gm1 * (E - T(0.5) * rho * q2);
    const T Ep = E + p;
    T grho = 0, gmn = 0, gmt = 0, gE = 0, gun = 0, gut = 0, gq2 = 0, gEp = 0, gp = 0, gir = 0;
    // F = (mn, mn un + p, mn ut, un Ep)
    gmn += gF[0] + un * gF[1];
    gun += mn * gF[1];
    gp += gF[1];
    if constexpr (M == 4) {
      gmn += ut * gF[2];
      gut += mn * gF[2];
    }
    gun += Ep * gF[M - 1];
    gEp += un * gF[M - 1];
    auto jvp_vjp = [&](const T* D, const T* go, T* gD) {
      const T r = D[0], a = D[1], b = (M == 4) ? D[2] : T(0), e = D[M - 1];
      const T us = (a - un * r) * ir;
      const T ts = (b - ut * r) * ir;
      const T ps = k.gm1 * (e - un * a - ut * b + T(0.5) * q2 * r);
      T gr = 0, ga = go[0], gb = 0, ge = 0, gus = 0, gts = 0, gps = 0;
      // out1 = a un + mn us + ps
      ga += un * go[1];
      gun += a * go[1];
      gmn += us * go[1];
      gus += mn * go[1];
      gps += go[1];
      if constexpr (M == 4) {  // out2 = a ut + mn ts
        ga += ut * go[2];
        gut += a * go[2];
        gmn += ts * go[2];
        gts += mn * go[2];
      }
      // out3 = us Ep + un (e + ps)
      gus += Ep * go[M - 1];
      gEp += us * go[M - 1];
      gun += (e + ps) * go[M - 1];
      ge += un * go[M - 1];
      gps += un * go[M - 1];
      // ps = gm1 (e - un a - ut b + q2 r / 2)
      const T gq = k.gm1 * gps;
      ge += gq;
      gun -= a * gq;
      ga -= un * gq;
      gut -= b * gq;
      gb -= ut * gq;
      gq2 += T(0.5) * r * gq;
      gr += T(0.5) * q2 * gq;
      // ts = (b - ut r) ir, us = (a - un r) ir
      gb += ir * gts;
      gut -= r * ir * gts;
      gr -= ut * ir * gts;
      gir += (b - ut * r) * gts;
      ga += ir * gus;
      gun -= r * ir * gus;
      gr -= un * ir * gus;
      gir += (a - un * r) * gus;
      gD[0] += gr;
      gD[1] += ga;
      if constexpr (M == 4) gD[2] += gb;
      gD[M - 1] += ge;
    };
    jvp_vjp(Dn, gA, gDn);
    if constexpr (MIXED) jvp_vjp(Dt, gB, gDt);
    gE += gEp;
    gp += gEp;
    gE += k.gm1 * gp;
    grho -= T(0.5) * k.gm1 * q2 * gp;
    gq2 -= T(0.5) * k.gm1 * rho * gp;
    gun += T(2) * un * gq2;
    gut += T(2) * ut * gq2;
    gmn += ir * gun;
    gir += mn * gun;
    gmt += ir * gut;
    gir += mt * gut;
    grho -= ir * ir * gir;
    gU[0] += grho;
    gU[1] += gmn;
    if constexpr (M == 4) gU[2] += gmt;
    gU[M - 1] += gE;
  } else if constexpr (PHYS == PH_BURGERS) {
    gU[0] += U[0] * gF[0] + Dn[0] * gA[0];
    gDn[0] += U[0] * gA[0];
    if constexpr (MIXED) {
      gU[0] += Dt[0] * gB[0];
      gDt[0] += U[0] * gB[0];
    }
  } else {
    gU[0] += an * gF[0];
    gDn[0] += an * gA[0];
    if constexpr (MIXED) gDt[0] += an * gB[0];
  }
}

// adjoints of the Roe eigen-system quantities used by project() / back()
template <typename T>
struct EigenAdj {
  T un = 0, ut = 0, H = 0, c = 0, ic = 0, b1 = 0, b2 = 0, hq2 = 0;
};

// reverse of Eigen::project(): gx = L^T gw, plus eigen-system adjoints
template <typename T, int M>
HW_HD void project_vjp(const Eigen<T, M>& e, const T* x, const T* gw, T* gx, EigenAdj<T>& ge) {
  if constexpr (M == 4) {
    const T gphi = T(0.5) * gw[0] - gw[1] + T(0.5) * gw[3];
    const T gpsi = T(0.5) * (gw[0] - gw[3]);
    gx[0] = e.b2 * gphi + e.un * e.ic * gpsi + gw[1] - e.ut * gw[2];
    gx[1] = -e.b1 * e.un * gphi - e.ic * gpsi;
    gx[2] = -e.b1 * e.ut * gphi + gw[2];
    gx[3] = e.b1 * gphi;
    ge.b2 += x[0] * gphi;
    ge.b1 -= (e.un * x[1] + e.ut * x[2] - x[3]) * gphi;
    ge.un += -e.b1 * x[1] * gphi + e.ic * x[0] * gpsi;
    ge.ut += -e.b1 * x[2] * gphi - x[0] * gw[2];
    ge.ic += (e.un * x[0] - x[1]) * gpsi;
  } else {
    const T gphi = T(0.5) * gw[0] - gw[1] + T(0.5) * gw[2];
    const T gpsi = T(0.5) * (gw[0] - gw[2]);
    gx[0] = e.b2 * gphi + e.un * e.ic * gpsi + gw[1];
    gx[1] = -e.b1 * e.un * gphi - e.ic * gpsi;
    gx[2] = e.b1 * gphi;
    ge.b2 += x[0] * gphi;
    ge.b1 -= (e.un * x[1] - x[2]) * gphi;
    ge.un += -e.b1 * x[1] * gphi + e.ic * x[0] * gpsi;
    ge.ic += (e.un * x[0] - x[1]) * gpsi;
  }
}

// reverse of Eigen::back(), in two parts: gw = R^T gy (needs no forward
// value), and the eigen-system adjoints (need the back-projected w)
template <typename T, int M>
HW_HD void back_T(const Eigen<T, M>& e, const T* gy, T* gw) {
  if constexpr (M == 4) {
    const T gs = gy[0] + e.un * gy[1] + e.ut * gy[2];
    const T gdif = e.c * gy[1] + e.un * e.c * gy[3];
    gw[0] = gs - gdif + e.H * gy[3];
    gw[1] = gs + e.hq2 * gy[3];
    gw[2] = gy[2] + e.ut * gy[3];
    gw[3] = gs + gdif + e.H * gy[3];
  } else {
    const T gs = gy[0] + e.un * gy[1];
    const T gdif = e.c * gy[1] + e.un * e.c * gy[2];
    gw[0] = gs - gdif + e.H * gy[2];
    gw[1] = gs + e.hq2 * gy[2];
    gw[2] = gs + gdif + e.H * gy[2];
  }
}

template <typename T, int M>
HW_HD void back_eigen_adj(const Eigen<T, M>& e, const T* w, const T* gy, EigenAdj<T>& ge) {
  if constexpr (M == 4) {
    const T s = w[0] + w[1] + w[3], dif = w[3] - w[0];
    ge.un += s * gy[1] + e.c * dif * gy[3];
    ge.c += dif * gy[1] + e.un * dif * gy[3];
    ge.ut += s * gy[2] + w[2] * gy[3];
    ge.H += (w[0] + w[3]) * gy[3];
    ge.hq2 += w[1] * gy[3];
  } else {
    const T s = w[0] + w[1] + w[2], dif = w[2] - w[0];
    ge.un += s * gy[1] + e.c * dif * gy[2];
    ge.c += dif * gy[1] + e.un * dif * gy[2];
    ge.H += (w[0] + w[2]) * gy[2];
    ge.hq2 += w[1] * gy[2];
  }
}

// reverse of Eigen::roe(): eigen-system adjoints -> adjoints of UL, UR (accumulated)
template <typename T, int M>
HW_HD void roe_vjp(const T* UL, const T* UR, T gm1, const EigenAdj<T>& g, T* gUL, T* gUR) {
  // the forward's arithmetic (Eigen::roe): sqrt(rho) and 1/rho from one
  // reciprocal square root per side
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
  const T un = wL * uL + wR * uR, ut = wL * tL + wR * tR, H = wL * HL + wR * HR;
  const T hq2 = T(0.5) * (un * un + ut * ut);
  const T c2 = gm1 * (H - hq2);
  const T ic = fast_rsq(c2);
  const T c = c2 * ic;
  const T b1 = gm1 * ic * ic;
  // b2 = b1 hq2, b1 = gm1 ic^2, ic = 1/c, c = sqrt(gm1 (H - hq2))
  const T gb1 = g.b1 + hq2 * g.b2;
  T ghq2 = g.hq2 + b1 * g.b2;
  const T gic = g.ic + T(2) * gm1 * ic * gb1;
  const T gc = g.c - ic * ic * gic;
  const T gcc = gm1 * T(0.5) * ic * gc;
  const T gH = g.H + gcc;
  ghq2 -= gcc;
  const T gun = g.un + un * ghq2, gut = g.ut + ut * ghq2;
  // Roe weights
  const T gwL = uL * gun + tL * gut + HL * gH, gwR = uR * gun + tR * gut + HR * gH;
  const T giw = sL * gwL + sR * gwR;
  const T gsL = iw * gwL - iw * iw * giw, gsR = iw * gwR - iw * iw * giw;
  // q = 1 / sqrt(rho): d sqrt(rho) / d rho = q / 2
  auto side = [&](const T* U, T ir, T q, T u, T t, T p, T w, T gs, T* gU) {
    const T gHs = w * gH, gu = w * gun, gt = w * gut;
    T gE = ir * gHs, gp = ir * gHs, gir = (U[M - 1] + p) * gHs;
    gE += gm1 * gp;
    T grho = -T(0.5) * gm1 * (u * u + t * t) * gp;
    const T gu2 = gu - gm1 * U[0] * u * gp;
    const T gt2 = gt - gm1 * U[0] * t * gp;
    const T gm = ir * gu2;
    gir += U[1] * gu2;
    T gn = 0;
    if constexpr (M == 4) {
      gn = ir * gt2;
      gir += U[2] * gt2;
    }
    grho += T(0.5) * gs * q - ir * ir * gir;
    gU[0] += grho;
    gU[1] += gm;
    if constexpr (M == 4) gU[2] += gn;
    gU[M - 1] += gE;
  };
  side(UL, irL, qL, uL, tL, pL, wL, gsL, gUL);
  side(UR, irR, qR, uR, tR, pR, wR, gsR, gUR);
}

// reverse of limit_char(): the adjoint gout of the limited derivative (normal
// frame) is mapped back through the right eigenvectors, the scalar limiters of
// the characteristic fields, the left-eigenvector projections of the five
// stencil vectors, and the cell's eigen-system.  That eigen-system is the Roe
// average of the cell with itself, so reversing roe() with both sides equal to
// u0 (both contributions into gu0) differentiates it exactly.  Results are
// accumulated into gum, gu0, gup, gvm, gvp.
template <typename T, int M>
HW_HD void limit_char_vjp(const T* um, const T* u0, const T* up, const T* vm, const T* vp, T h,
                          T ih, const Weights<T>& w, T gm1, const T* gout, T* gum, T* gu0,
                          T* gup, T* gvm, T* gvp) {
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
  EigenAdj<T> ge;
  T gz[M];
  back_T(e, gout, gz);
  back_eigen_adj(e, z, gout, ge);
  T ga[M], gb[M], gc[M], gdm[M], gdp[M];
#pragma unroll
  for (int q = 0; q < M; ++q) {
    ga[q] = gb[q] = gc[q] = gdm[q] = gdp[q] = T(0);
    limit1_vjp(a[q], b[q], c[q], dm[q], dp[q], h, ih, w, gz[q], ga[q], gb[q], gc[q], gdm[q], gdp[q]);
  }
  T gx[M];
  auto add = [&](const T* x, const T* gw, T* out) {
    project_vjp(e, x, gw, gx, ge);
#pragma unroll
    for (int q = 0; q < M; ++q) out[q] += gx[q];
  };
  add(um, ga, gum);
  add(u0, gb, gu0);
  add(up, gc, gup);
  add(vm, gdm, gvm);
  add(vp, gdp, gvp);
  roe_vjp<T, M>(u0, u0, gm1, ge, gu0, gu0);
}

// ---------------------------------------------------------------------------
// VJP of interface_fluxes(): given the adjoints of f-hat, h-hat and the mixed
// flux (normal frame), emit(s, mode, gU, gDn, gDt) receives adjoint
// contributions for the state of stencil point s.  mode EMIT_SET is the first
// contribution to point s (all fields), EMIT_ADD adds to all fields, EMIT_ADD_U
// adds to the U fields only (gDn, gDt are zero).  The "+" side (points 0..2)
// and the mirrored "-" side (points 1..3) are differentiated in separate
// passes, so that only one side's projected data and adjoints are live at a
// time; every point receives exactly one EMIT_SET, before any addition.  The
// eigen-system adjoint (through the Roe average) is linear in the per-side
// accumulations, so each side applies its share at its end: the accumulators
// never stay live across the two passes.
// ---------------------------------------------------------------------------
enum { EMIT_SET = 0, EMIT_ADD = 1, EMIT_ADD_U = 2 };

template <typename T, int PHYS, int M, bool MIXED, typename Loader, typename Emit, typename GH>
HW_HD void interface_vjp(const Loader& ld, T alpha, T h, T ih, T an, const Consts<T>& k,
                         const T* gfh, const GH& ghh, const GH& gxh, const Emit& emit) {
  constexpr bool CHARW = (PHYS == PH_EULER);
  const bool proj = CHARW && k.characteristic;
  Eigen<T, M> eg;
  if constexpr (CHARW) {
    if (proj) {
      T U1[M], U2[M], dn[M], dt[M];
      ld(1, U1, dn, dt);
      ld(2, U2, dn, dt);
      eg.roe(U1, U2, k.gm1);
    }
  }
  const T hh2 = T(0.5) * h;
  constexpr T cF[4] = {T(1), T(-15), T(15), T(-1)};
  constexpr T cU[4] = {T(1), T(-1), T(-1), T(1)};
  constexpr T cA[4] = {T(1), T(-7), T(-7), T(1)};
  constexpr T cD[4] = {T(1), T(3), T(-3), T(-1)};
  constexpr T cX[4] = {T(-1), T(7), T(7), T(-1)};
  const T i8 = T(0.125) * ih;
  EigenAdj<T> ge;
  T gfc[M];  // adjoint of the characteristic flux f-hat^+ + f-hat^-
  if (proj) {
    back_T(eg, gfh, gfc);
  } else {
#pragma unroll
    for (int c = 0; c < M; ++c) gfc[c] = gfh[c];
  }
  // split data x = (F +- alpha U)/2, y = dx/2 (A Dn +- alpha Dn) of point s
  auto split = [&](int s, T sign, T* U, T* Dn, T* Dt, T* x, T* y) {
    T F[M], A[M], B[M];
    ld(s, U, Dn, Dt);
    point_fluxes<T, PHYS, M, false>(U, Dn, Dt, k, an, F, A, B);
#pragma unroll
    for (int c = 0; c < M; ++c) {
      x[c] = T(0.5) * (F[c] + sign * alpha * U[c]);
      y[c] = hh2 * (A[c] + sign * alpha * Dn[c]);
    }
  };
  auto side = [&](const bool plus) {
    const int s0 = plus ? 0 : 1;
    const T sign = plus ? T(1) : T(-1);
    T fS[3][M], HS[3][M];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      T U[M], Dn[M], Dt[M], x[M], y[M];
      split(s0 + j, sign, U, Dn, Dt, x, y);
      if (proj) {
        eg.project(x, fS[j]);
        eg.project(y, HS[j]);
      } else {
#pragma unroll
        for (int c = 0; c < M; ++c) {
          fS[j][c] = x[c];
          HS[j][c] = y[c];
        }
      }
    }
    T gfS[3][M], gHS[3][M], fcs[M];
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
      for (int c = 0; c < M; ++c) gfS[j][c] = gHS[j][c] = T(0);
#pragma unroll
    for (int c = 0; c < M; ++c) {
      if (plus) {
        fcs[c] = hw_plus_vjp(fS[0][c], fS[1][c], fS[2][c], HS[0][c], HS[1][c], HS[2][c], k.rw,
                             gfc[c], gfS[0][c], gfS[1][c], gfS[2][c], gHS[0][c], gHS[1][c],
                             gHS[2][c]);
      } else {
        // mirrored: i+2, i+1, i with the derivative data negated
        T n2 = 0, n1 = 0, n0 = 0;
        fcs[c] = hw_plus_vjp(fS[2][c], fS[1][c], fS[0][c], -HS[2][c], -HS[1][c], -HS[0][c],
                             k.rw, gfc[c], gfS[2][c], gfS[1][c], gfS[0][c], n2, n1, n0);
        gHS[2][c] -= n2;
        gHS[1][c] -= n1;
        gHS[0][c] -= n0;
      }
    }
    // the back projection's eigen-system adjoint is linear in f-hat: add this side's part
    if (proj) back_eigen_adj(eg, fcs, gfh, ge);
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const int s = s0 + j;
      T U[M], Dn[M], Dt[M], x[M], y[M], gx[M], gy[M];
      split(s, sign, U, Dn, Dt, x, y);
      if (proj) {
        project_vjp(eg, x, gfS[j], gx, ge);
        project_vjp(eg, y, gHS[j], gy, ge);
      } else {
#pragma unroll
        for (int c = 0; c < M; ++c) {
          gx[c] = gfS[j][c];
          gy[c] = gHS[j][c];
        }
      }
      // the linear fluxes of points 0..2 are differentiated in the "+" pass,
      // point 3's in the "-" pass
      const bool lin = plus || s == 3;
      T gF[M], gA[M], gB[M], gUd[M], gDnd[M], gDtd[M];
#pragma unroll
      for (int c = 0; c < M; ++c) {
        gF[c] = T(0.5) * gx[c] + (lin ? cF[s] * i8 * ghh[c] : T(0));
        gUd[c] = sign * T(0.5) * alpha * gx[c] + (lin ? alpha * cU[s] * i8 * ghh[c] : T(0));
        gA[c] = hh2 * gy[c] + (lin ? cA[s] * T(1.0 / 24.0) * ghh[c] : T(0));
        gDnd[c] = sign * hh2 * alpha * gy[c] + (lin ? alpha * cD[s] * T(1.0 / 24.0) * ghh[c] : T(0));
        gB[c] = (MIXED && lin) ? cX[s] * T(1.0 / 12.0) * gxh[c] : T(0);
        gDtd[c] = T(0);
      }
      point_fluxes_vjp<T, PHYS, M, MIXED>(U, Dn, Dt, k, an, gF, gA, gB, gUd, gDnd, gDtd);
      emit(s, (plus || s == 3) ? EMIT_SET : EMIT_ADD, gUd, gDnd, gDtd);
    }
    if constexpr (CHARW) {
      if (proj) {
        T U1[M], U2[M], dn[M], dt[M], gU1[M], gU2[M], z[M];
        ld(1, U1, dn, dt);
        ld(2, U2, dn, dt);
#pragma unroll
        for (int c = 0; c < M; ++c) gU1[c] = gU2[c] = z[c] = T(0);
        roe_vjp<T, M>(U1, U2, k.gm1, ge, gU1, gU2);
        emit(1, EMIT_ADD_U, gU1, z, z);
        emit(2, EMIT_ADD_U, gU2, z, z);
        ge = EigenAdj<T>();
      }
    }
  };
  side(true);
  side(false);
}

}  // namespace hweno
