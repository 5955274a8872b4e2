// Element physics of the stabilised trilinear-hexahedron weak form (App. A,
// eq. weakstable) for a cube of edge h, written once for the residual, the exact
// Newton Jacobian apply, its transpose and the design sensitivity.
//
// Shape functions: N_a(xi) = prod_d (1 + s_ad xi_d) / 2 on [-1, 1]^3, local node
// a = ia + 2 ja + 4 ka with signs s_a = 2 (ia, ja, ka) - 1.  Quadrature: 2x2x2 Gauss
// points g s_q (g = 1/sqrt 3), numbered like the nodes, weight h^3 / 8 each.
//
// Everything goes through the hierarchical ("modal") basis
//   phi = (1, xi, eta, zeta, xi eta, xi zeta, eta zeta, xi eta zeta):
// nodal values -> modal coefficients is one 8-point Hadamard butterfly (24 adds), and
// Gauss-point values, gradients and the transposed test-function sums are again
// butterflies.  Because a trilinear field's x-derivative does not depend on x, the
// x-gradient takes only 4 distinct Gauss-point values (indexed by the (eta, zeta)
// signs), and likewise for y and z.  The centroid value and gradient equal the mean of
// the Gauss-point ones, which lets the SUPG centroid velocity be folded into the
// Gauss-point sums in the transposed apply.
//
// Header-only and free of HIP types, so the same code builds for gfx950 and, for
// checking, for the host.
#pragma once

#if defined(__HIPCC__)
#include <hip/hip_runtime.h>
#define NC_HD __host__ __device__ __forceinline__
#else
#include <cmath>
#define NC_HD inline
#endif

namespace nc {

template <typename T>
struct ElemConst {
  T W;         // h^3 / 8: Gauss weight times Jacobian determinant
  T dxi;       // 2 / h: reference-to-physical derivative factor
  T inv_mu;    // 1 / mu
  T beta;      // rho0 alpha g0 (buoyancy per unit temperature, along +z)
  T rcp;       // rho0 c_p
  T Q;         // volumetric source on the source box (everywhere by default)
  T inv_he2;   // 1 / h_e^2, h_e^2 = dx^2 + dy^2 + dz^2 = 3 h^2
  T tau3inv2;  // tau3^-2 = 16 / h_e^4
  int qi0, qi1, qj0, qj1, qk0, qk1;   // element index ranges (inclusive) carrying Q
  // the volumetric source of element (i, j, k)
  NC_HD T source(int i, int j, int k) const {
    if (Q == (T)0) return (T)0;   // uniform: no source, no per-element test
    return (i >= qi0 && i <= qi1 && j >= qj0 && j <= qj1 && k >= qk0 && k <= qk1) ? Q : (T)0;
  }
};

template <typename T>
NC_HD ElemConst<T> make_elem_const(double h, double rho0, double mu, double cp, double g0, double alpha, double Q) {
  ElemConst<T> c;
  const double he2 = 3.0 * h * h;
  c.W = (T)(h * h * h / 8.0);
  c.dxi = (T)(2.0 / h);
  c.inv_mu = (T)(1.0 / mu);
  c.beta = (T)(rho0 * alpha * g0);
  c.rcp = (T)(rho0 * cp);
  c.Q = (T)Q;
  c.inv_he2 = (T)(1.0 / he2);
  c.tau3inv2 = (T)(16.0 / (he2 * he2));
  c.qi0 = c.qj0 = c.qk0 = -(1 << 30);
  c.qi1 = c.qj1 = c.qk1 = 1 << 30;
  return c;
}

template <typename T> struct GC {
  static constexpr T g = (T)0.57735026918962576451;   // 1/sqrt(3)
  static constexpr T g2 = (T)(1.0 / 3.0);
  static constexpr T g3 = (T)0.19245008972987525484;  // 1/(3 sqrt 3)
};

// m[k] = sum_a phi_k(s_a) f[a]  (k in the modal order above, a in node order)
template <typename T>
NC_HD void hadamard_fwd(const T f[8], T m[8]) {
  const T s0 = f[1] + f[0], d0 = f[1] - f[0];
  const T s1 = f[3] + f[2], d1 = f[3] - f[2];
  const T s2 = f[5] + f[4], d2 = f[5] - f[4];
  const T s3 = f[7] + f[6], d3 = f[7] - f[6];
  const T ss0 = s1 + s0, sd0 = s1 - s0, ss1 = s3 + s2, sd1 = s3 - s2;
  const T ds0 = d1 + d0, dd0 = d1 - d0, ds1 = d3 + d2, dd1 = d3 - d2;
  m[0] = ss1 + ss0;
  m[3] = ss1 - ss0;
  m[2] = sd1 + sd0;
  m[6] = sd1 - sd0;
  m[1] = ds1 + ds0;
  m[5] = ds1 - ds0;
  m[4] = dd1 + dd0;
  m[7] = dd1 - dd0;
}

// v[q] = sum_k e[k] phi_k(s_q)  (values of a modal expansion at the 8 sign patterns)
template <typename T>
NC_HD void hadamard_inv(const T e[8], T v[8]) {
  const T am = e[0] - e[3], ap = e[0] + e[3];
  const T cm = e[2] - e[6], cp = e[2] + e[6];
  const T bm = e[1] - e[5], bp = e[1] + e[5];
  const T dm = e[4] - e[7], dp = e[4] + e[7];
  const T A0 = am - cm, B0 = bm - dm;
  const T A1 = am + cm, B1 = bm + dm;
  const T A2 = ap - cp, B2 = bp - dp;
  const T A3 = ap + cp, B3 = bp + dp;
  v[0] = A0 - B0; v[1] = A0 + B0;
  v[2] = A1 - B1; v[3] = A1 + B1;
  v[4] = A2 - B2; v[5] = A2 + B2;
  v[6] = A3 - B3; v[7] = A3 + B3;
}

// out[i + 2 j] = a + s_i b + s_j c + s_i s_j d,  s = -1, +1
template <typename T>
NC_HD void bilinear4(T a, T b, T c, T d, T out[4]) {
  const T cm = a - c, cp = a + c, dm = b - d, dp = b + d;
  out[0] = cm - dm;
  out[1] = cm + dm;
  out[2] = cp - dp;
  out[3] = cp + dp;
}

// Gauss-point index helpers: q = qx + 2 qy + 4 qz
NC_HD int jx_of(int q) { return ((q >> 1) & 1) + 2 * ((q >> 2) & 1); }   // (qy, qz)
NC_HD int jy_of(int q) { return (q & 1) + 2 * ((q >> 2) & 1); }          // (qx, qz)
NC_HD int jz_of(int q) { return (q & 1) + 2 * ((q >> 1) & 1); }          // (qx, qy)

// Physical gradient of a nodal trilinear field at the Gauss points (gx indexed by
// (qy, qz), gy by (qx, qz), gz by (qx, qy)) and at the centroid.  m: modal coefficients.
template <typename T>
NC_HD void grad_from_modal(const T m[8], const ElemConst<T>& c, T gx[4], T gy[4], T gz[4], T gc[3]) {
  const T s = c.dxi * (T)0.125;
  const T g = GC<T>::g, g2 = GC<T>::g2;
  bilinear4(s * m[1], s * g * m[4], s * g * m[5], s * g2 * m[7], gx);
  bilinear4(s * m[2], s * g * m[4], s * g * m[6], s * g2 * m[7], gy);
  bilinear4(s * m[3], s * g * m[5], s * g * m[6], s * g2 * m[7], gz);
  gc[0] = s * m[1];
  gc[1] = s * m[2];
  gc[2] = s * m[3];
}

// Values at the Gauss points and at the centroid from modal coefficients.
template <typename T>
NC_HD void val_from_modal(const T m[8], T v[8], T& vc) {
  const T s = (T)0.125, g = GC<T>::g, g2 = GC<T>::g2, g3 = GC<T>::g3;
  const T e[8] = {s * m[0], s * g * m[1], s * g * m[2], s * g * m[3],
                  s * g2 * m[4], s * g2 * m[5], s * g2 * m[6], s * g3 * m[7]};
  hadamard_inv(e, v);
  vc = e[0];
}

// r[a] += scale * sum_q [ N_a(q) s[q] + grad N_a(q) . F[q] ]   (s or F may be null)
template <typename T>
NC_HD void project(const T* s, const T* Fx, const T* Fy, const T* Fz, const ElemConst<T>& c, T scale, T r[8]) {
  const T g = GC<T>::g, g2 = GC<T>::g2, g3 = GC<T>::g3;
  T S[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (s) hadamard_fwd(s, S);
  T ax = 0, ayx = 0, azx = 0, ayzx = 0;    // sum Fx, sum s_y Fx, sum s_z Fx, sum s_y s_z Fx
  T ay = 0, axy = 0, azy = 0, axzy = 0;
  T az = 0, axz = 0, ayz = 0, axyz = 0;
  if (Fx) {
    const T p0 = Fx[0] + Fx[1], p1 = Fx[2] + Fx[3], p2 = Fx[4] + Fx[5], p3 = Fx[6] + Fx[7];
    ax = (p0 + p1) + (p2 + p3);
    ayx = (p1 + p3) - (p0 + p2);
    azx = (p2 + p3) - (p0 + p1);
    ayzx = (p0 + p3) - (p1 + p2);
  }
  if (Fy) {
    const T p0 = Fy[0] + Fy[2], p1 = Fy[1] + Fy[3], p2 = Fy[4] + Fy[6], p3 = Fy[5] + Fy[7];
    ay = (p0 + p1) + (p2 + p3);
    axy = (p1 + p3) - (p0 + p2);
    azy = (p2 + p3) - (p0 + p1);
    axzy = (p0 + p3) - (p1 + p2);
  }
  if (Fz) {
    const T p0 = Fz[0] + Fz[4], p1 = Fz[1] + Fz[5], p2 = Fz[2] + Fz[6], p3 = Fz[3] + Fz[7];
    az = (p0 + p1) + (p2 + p3);
    axz = (p1 + p3) - (p0 + p2);
    ayz = (p2 + p3) - (p0 + p1);
    axyz = (p0 + p3) - (p1 + p2);
  }
  const T d = c.dxi;
  const T sc = scale * (T)0.125;
  T rho[8];
  rho[0] = sc * S[0];
  rho[1] = sc * (g * S[1] + d * ax);
  rho[2] = sc * (g * S[2] + d * ay);
  rho[3] = sc * (g * S[3] + d * az);
  rho[4] = sc * (g2 * S[4] + d * g * (ayx + axy));
  rho[5] = sc * (g2 * S[5] + d * g * (azx + axz));
  rho[6] = sc * (g2 * S[6] + d * g * (azy + ayz));
  rho[7] = sc * (g3 * S[7] + d * g2 * (ayzx + axzy + axyz));
  T v[8];
  hadamard_inv(rho, v);
#pragma unroll
  for (int a = 0; a < 8; ++a) r[a] += v[a];
}

// Linearisation data of one element at the state (P, T): Darcy velocity per unit
// permeability uh = -(1/mu)(grad P - beta T e_z) at the Gauss points (Sec. 2.1,
// eq. finaldarcy with g = -g0 e_z), grad T, the convective term
// conv = rho0 c_p u . grad T - Q, the centroid velocity u0 and the SUPG parameter
// tau = (tau1^-2 + tau3^-2)^(-1/2) with tau1 = h_e / (2 |u0|), tau3 = h_e^2 / 4 (App. A).
template <typename T>
struct Lin {
  T uhx[4], uhy[4], uhz[8];
  T gTx[4], gTy[4], gTz[4];
  T Tq[8];
  T conv[8];
  T u0[3];
  T tau, dtau;      // tau and d tau / d(u0 . du0) = -4 tau^3 / h_e^2
  T k, kap;
};

template <typename T>
NC_HD void linearize_q(const T P[8], const T Tn[8], T k, T kap, T Q, const ElemConst<T>& c, Lin<T>& L) {
  T mP[8], mT[8];
  hadamard_fwd(P, mP);
  hadamard_fwd(Tn, mT);
  T gPx[4], gPy[4], gPz[4], gPc[3], gTc[3], Tc;
  grad_from_modal(mP, c, gPx, gPy, gPz, gPc);
  grad_from_modal(mT, c, L.gTx, L.gTy, L.gTz, gTc);
  val_from_modal(mT, L.Tq, Tc);
  L.k = k;
  L.kap = kap;
  const T im = c.inv_mu;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    L.uhx[j] = -im * gPx[j];
    L.uhy[j] = -im * gPy[j];
  }
#pragma unroll
  for (int q = 0; q < 8; ++q) L.uhz[q] = -im * (gPz[jz_of(q)] - c.beta * L.Tq[q]);
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int jx = jx_of(q), jy = jy_of(q), jz = jz_of(q);
    L.conv[q] = c.rcp * kap * (L.uhx[jx] * L.gTx[jx] + L.uhy[jy] * L.gTy[jy] + L.uhz[q] * L.gTz[jz]) - Q;
  }
  const T cm = kap * im;
  L.u0[0] = -cm * gPc[0];
  L.u0[1] = -cm * gPc[1];
  L.u0[2] = -cm * (gPc[2] - c.beta * Tc);
  const T s = (T)4 * (L.u0[0] * L.u0[0] + L.u0[1] * L.u0[1] + L.u0[2] * L.u0[2]) * c.inv_he2 + c.tau3inv2;
  const T tau = (T)1 / sqrt(s);
  L.tau = tau;
  L.dtau = (T)(-4) * tau * tau * tau * c.inv_he2;
}
// with the constant's source Q
template <typename T>
NC_HD void linearize(const T P[8], const T Tn[8], T k, T kap, const ElemConst<T>& c, Lin<T>& L) {
  linearize_q(P, Tn, k, kap, c.Q, c, L);
}

// Element rows of the residual (without the boundary flux and without the lumped-mass
// term M_a U_a of the velocity rows, which the caller adds at the node):
//   R_P,a = sum_q W grad N_a . (-u_q)
//   R_T,a = sum_q W [ N*_a conv_q + k grad N_a . grad T_q ],  N*_a = N_a + tau u0 . grad N_a
//   R_U,a = - sum_q W N_a u_q
template <typename T, bool WITH_U>
NC_HD void elem_residual(const Lin<T>& L, const ElemConst<T>& c, T rP[8], T rT[8], T rU[3][8]) {
  T FPx[8], FPy[8], FPz[8], FTx[8], FTy[8], FTz[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int jx = jx_of(q), jy = jy_of(q), jz = jz_of(q);
    const T ux = L.kap * L.uhx[jx], uy = L.kap * L.uhy[jy], uz = L.kap * L.uhz[q];
    FPx[q] = -ux; FPy[q] = -uy; FPz[q] = -uz;
    const T tc = L.tau * L.conv[q];
    FTx[q] = tc * L.u0[0] + L.k * L.gTx[jx];
    FTy[q] = tc * L.u0[1] + L.k * L.gTy[jy];
    FTz[q] = tc * L.u0[2] + L.k * L.gTz[jz];
  }
  project<T>(nullptr, FPx, FPy, FPz, c, c.W, rP);
  project<T>(L.conv, FTx, FTy, FTz, c, c.W, rT);
  if constexpr (WITH_U) {
    project<T>(FPx, nullptr, nullptr, nullptr, c, c.W, rU[0]);
    project<T>(FPy, nullptr, nullptr, nullptr, c, c.W, rU[1]);
    project<T>(FPz, nullptr, nullptr, nullptr, c, c.W, rU[2]);
  }
}

// Exact Newton Jacobian applied to a direction (p, t) of the P and T unknowns; the
// velocity columns (lumped mass on the diagonal) are added by the caller.
//   du_q = -(kappa/mu)(grad p_q - beta t_q e_z),  du0 likewise at the centroid,
//   dtau = -4 tau^3 / h_e^2 (u0 . du0),
//   dconv_q = rho0 c_p (du_q . grad T_q + u_q . grad t_q),
//   yP_a = sum_q W grad N_a . (-du_q)
//   yT_a = sum_q W [ N*_a dconv_q + (dtau u0 + tau du0) . grad N_a conv_q + k grad N_a . grad t_q ]
//   yU_a = -sum_q W N_a du_q
template <typename T, bool WITH_U>
NC_HD void elem_jv(const Lin<T>& L, const T p[8], const T t[8], const ElemConst<T>& c, T yP[8], T yT[8], T yU[3][8]) {
  T mp[8], mt[8];
  hadamard_fwd(p, mp);
  hadamard_fwd(t, mt);
  T gpx[4], gpy[4], gpz[4], gpc[3], gtx[4], gty[4], gtz[4], gtc[3], tq[8], tc;
  grad_from_modal(mp, c, gpx, gpy, gpz, gpc);
  grad_from_modal(mt, c, gtx, gty, gtz, gtc);
  val_from_modal(mt, tq, tc);
  const T cm = L.kap * c.inv_mu;
  const T du0x = -cm * gpc[0], du0y = -cm * gpc[1], du0z = -cm * (gpc[2] - c.beta * tc);
  const T dtau = L.dtau * (L.u0[0] * du0x + L.u0[1] * du0y + L.u0[2] * du0z);
  const T ax = dtau * L.u0[0] + L.tau * du0x;
  const T ay = dtau * L.u0[1] + L.tau * du0y;
  const T az = dtau * L.u0[2] + L.tau * du0z;
  T FPx[8], FPy[8], FPz[8], FTx[8], FTy[8], FTz[8], sT[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int jx = jx_of(q), jy = jy_of(q), jz = jz_of(q);
    const T dux = -cm * gpx[jx], duy = -cm * gpy[jy], duz = -cm * (gpz[jz] - c.beta * tq[q]);
    const T ux = L.kap * L.uhx[jx], uy = L.kap * L.uhy[jy], uz = L.kap * L.uhz[q];
    const T dconv = c.rcp * (dux * L.gTx[jx] + duy * L.gTy[jy] + duz * L.gTz[jz] + ux * gtx[jx] + uy * gty[jy] + uz * gtz[jz]);
    sT[q] = dconv;
    const T td = L.tau * dconv;
    FTx[q] = td * L.u0[0] + ax * L.conv[q] + L.k * gtx[jx];
    FTy[q] = td * L.u0[1] + ay * L.conv[q] + L.k * gty[jy];
    FTz[q] = td * L.u0[2] + az * L.conv[q] + L.k * gtz[jz];
    FPx[q] = -dux; FPy[q] = -duy; FPz[q] = -duz;
  }
  project<T>(nullptr, FPx, FPy, FPz, c, c.W, yP);
  project<T>(sT, FTx, FTy, FTz, c, c.W, yT);
  if constexpr (WITH_U) {
    project<T>(FPx, nullptr, nullptr, nullptr, c, c.W, yU[0]);
    project<T>(FPy, nullptr, nullptr, nullptr, c, c.W, yU[1]);
    project<T>(FPz, nullptr, nullptr, nullptr, c, c.W, yU[2]);
  }
}

// Transpose of elem_jv: given the adjoint weights (wP, wT, wU) of the element's rows,
// return the contributions to the P and T columns (the velocity columns only carry the
// lumped mass, added by the caller).  Derived by running the operations of elem_jv
// backwards; the centroid quantities are the mean of the Gauss-point ones, so their
// adjoints are spread as 1/8 onto every Gauss point.
template <typename T, bool WITH_U>
NC_HD void elem_jtw(const Lin<T>& L, const T wP[8], const T wT[8], const T wU[3][8], const ElemConst<T>& c,
                    T yP[8], T yT[8]) {
  T mwp[8], mwt[8];
  hadamard_fwd(wP, mwp);
  hadamard_fwd(wT, mwt);
  T gwpx[4], gwpy[4], gwpz[4], gwpc[3], gwtx[4], gwty[4], gwtz[4], gwtc[3], wtq[8], wtc;
  grad_from_modal(mwp, c, gwpx, gwpy, gwpz, gwpc);
  grad_from_modal(mwt, c, gwtx, gwty, gwtz, gwtc);
  val_from_modal(mwt, wtq, wtc);
  T wuq[3][8];
  if constexpr (WITH_U) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      T m[8], vc;
      hadamard_fwd(wU[d], m);
      val_from_modal(m, wuq[d], vc);
    }
  }
  const T W = c.W;
  const T cm = L.kap * c.inv_mu;
  T ub[3][8];            // adjoint of du_q
  T gtbx[8], gtby[8], gtbz[8];   // adjoint of grad t_q
  T taub = 0, u0b0 = 0, u0b1 = 0, u0b2 = 0;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int jx = jx_of(q), jy = jy_of(q), jz = jz_of(q);
    const T gx = gwtx[jx], gy = gwty[jy], gz = gwtz[jz];
    const T u0g = L.u0[0] * gx + L.u0[1] * gy + L.u0[2] * gz;
    const T dconvb = W * (wtq[q] + L.tau * u0g);             // adjoint of dconv_q
    const T wc = W * L.conv[q];
    taub += wc * u0g;
    u0b0 += wc * gx; u0b1 += wc * gy; u0b2 += wc * gz;
    const T ux = L.kap * L.uhx[jx], uy = L.kap * L.uhy[jy], uz = L.kap * L.uhz[q];
    const T rb = c.rcp * dconvb;
    gtbx[q] = W * L.k * gx + rb * ux;
    gtby[q] = W * L.k * gy + rb * uy;
    gtbz[q] = W * L.k * gz + rb * uz;
    ub[0][q] = -W * gwpx[jx] + rb * L.gTx[jx];
    ub[1][q] = -W * gwpy[jy] + rb * L.gTy[jy];
    ub[2][q] = -W * gwpz[jz] + rb * L.gTz[jz];
    if constexpr (WITH_U) {
      ub[0][q] -= W * wuq[0][q];
      ub[1][q] -= W * wuq[1][q];
      ub[2][q] -= W * wuq[2][q];
    }
  }
  // du0 enters through tau du0 . grad N and through dtau = L.dtau (u0 . du0)
  const T tb = taub * L.dtau;
  const T e0 = (T)0.125 * (L.tau * u0b0 + tb * L.u0[0]);
  const T e1 = (T)0.125 * (L.tau * u0b1 + tb * L.u0[1]);
  const T e2 = (T)0.125 * (L.tau * u0b2 + tb * L.u0[2]);
  T FPx[8], FPy[8], FPz[8], sT[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    // du = -cm (grad p - beta t e_z): adjoint to grad p is -cm ub, to t is cm beta ub_z
    FPx[q] = -cm * (ub[0][q] + e0);
    FPy[q] = -cm * (ub[1][q] + e1);
    FPz[q] = -cm * (ub[2][q] + e2);
    sT[q] = cm * c.beta * (ub[2][q] + e2);
  }
  project<T>(nullptr, FPx, FPy, FPz, c, (T)1, yP);
  project<T>(sT, gtbx, gtby, gtbz, c, (T)1, yT);
}

// Design sensitivity of one element: -lambda_e^T dR_e/dgamma with
// dR/dgamma = k'(gamma) dR/dk + kappa'(gamma) dR/dkappa (Sec. 5.2 RAMP derivatives).
//   lambda^T dR/dk     = sum_q W grad lT . grad T
//   lambda^T dR/dkappa = sum_q W [ -grad lP . uh - lU . uh + (lT + tau u0 . grad lT) rho0 c_p uh . grad T
//                                 + (dtau_dkappa u0 + tau uh0) . grad lT conv ]
// with uh = u / kappa and dtau_dkappa = -4 tau^3 / h_e^2 (u0 . uh0).  The velocity rows'
// lumped-mass term does not depend on the design.
template <typename T, bool WITH_U>
NC_HD T elem_sensitivity(const Lin<T>& L, const T lP[8], const T lT[8], const T lU[3][8], T dk, T dkap,
                         const ElemConst<T>& c) {
  T mlp[8], mlt[8];
  hadamard_fwd(lP, mlp);
  hadamard_fwd(lT, mlt);
  T glpx[4], glpy[4], glpz[4], glpc[3], gltx[4], glty[4], gltz[4], gltc[3], ltq[8], ltc;
  grad_from_modal(mlp, c, glpx, glpy, glpz, glpc);
  grad_from_modal(mlt, c, gltx, glty, gltz, gltc);
  val_from_modal(mlt, ltq, ltc);
  T luq[3][8];
  if constexpr (WITH_U) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      T m[8], vc;
      hadamard_fwd(lU[d], m);
      val_from_modal(m, luq[d], vc);
    }
  }
  const T ikap = (T)1 / L.kap;
  const T uh0x = L.u0[0] * ikap, uh0y = L.u0[1] * ikap, uh0z = L.u0[2] * ikap;
  const T dtau_k = L.dtau * (L.u0[0] * uh0x + L.u0[1] * uh0y + L.u0[2] * uh0z);
  const T bx = dtau_k * L.u0[0] + L.tau * uh0x;
  const T by = dtau_k * L.u0[1] + L.tau * uh0y;
  const T bz = dtau_k * L.u0[2] + L.tau * uh0z;
  T rk = 0, rkap = 0;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int jx = jx_of(q), jy = jy_of(q), jz = jz_of(q);
    const T gx = gltx[jx], gy = glty[jy], gz = gltz[jz];
    rk += gx * L.gTx[jx] + gy * L.gTy[jy] + gz * L.gTz[jz];
    const T uhx = L.uhx[jx], uhy = L.uhy[jy], uhz = L.uhz[q];
    T a = -(glpx[jx] * uhx + glpy[jy] * uhy + glpz[jz] * uhz);
    if constexpr (WITH_U) a -= luq[0][q] * uhx + luq[1][q] * uhy + luq[2][q] * uhz;
    const T star = ltq[q] + L.tau * (L.u0[0] * gx + L.u0[1] * gy + L.u0[2] * gz);
    a += star * c.rcp * (uhx * L.gTx[jx] + uhy * L.gTy[jy] + uhz * L.gTz[jz]);
    a += (bx * gx + by * gy + bz * gz) * L.conv[q];
    rkap += a;
  }
  return -c.W * (dk * rk + dkap * rkap);
}

// Velocity rows' coupling to the (P, T) columns alone: yU_a = -sum_q W N_a du_q with
// du_q = -(kappa/mu)(grad p_q - beta t_q e_z).  State independent (only kappa enters).
template <typename T>
NC_HD void elem_uproj(const T p[8], const T t[8], T kap, const ElemConst<T>& c, T yU[3][8]) {
  T mp[8], mt[8];
  hadamard_fwd(p, mp);
  hadamard_fwd(t, mt);
  T gpx[4], gpy[4], gpz[4], gpc[3], tq[8], tc;
  grad_from_modal(mp, c, gpx, gpy, gpz, gpc);
  val_from_modal(mt, tq, tc);
  const T cm = kap * c.inv_mu;
  T sx[8], sy[8], sz[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    sx[q] = cm * gpx[jx_of(q)];
    sy[q] = cm * gpy[jy_of(q)];
    sz[q] = cm * (gpz[jz_of(q)] - c.beta * tq[q]);
  }
  project<T>(sx, nullptr, nullptr, nullptr, c, c.W, yU[0]);
  project<T>(sy, nullptr, nullptr, nullptr, c, c.W, yU[1]);
  project<T>(sz, nullptr, nullptr, nullptr, c, c.W, yU[2]);
}

// Transpose of elem_uproj: contributions of velocity-row weights zu to the P and T columns.
template <typename T>
NC_HD void elem_uprojT(const T zu[3][8], T kap, const ElemConst<T>& c, T yP[8], T yT[8]) {
  T zq[3][8];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    T m[8], vc;
    hadamard_fwd(zu[d], m);
    val_from_modal(m, zq[d], vc);
  }
  const T cmw = kap * c.inv_mu * c.W;
  T Fx[8], Fy[8], Fz[8], s[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    Fx[q] = cmw * zq[0][q];
    Fy[q] = cmw * zq[1][q];
    Fz[q] = cmw * zq[2][q];
    s[q] = -cmw * c.beta * zq[2][q];
  }
  project<T>(nullptr, Fx, Fy, Fz, c, (T)1, yP);
  project<T>(s, nullptr, nullptr, nullptr, c, (T)1, yT);
}

// ===================================================================================
// Fast element operators in the modal basis.
//
// With the 2x2x2 Gauss rule on a cube the modal functions are orthogonal, which makes
// the state-independent parts of the element operator nearly diagonal:
//   sum_q grad phi_m . grad phi_n = K_m delta_mn,  K = (0, 8, 8, 8, 16/3, 16/3, 16/3, 8/3)
//   sum_q d(phi_m)/dzeta phi_n    = B_mn with B_30 = 8, B_51 = B_62 = 8/3, B_74 = 8/9
// so the pressure rows (Darcy stiffness and buoyancy) and the conduction part of the
// energy rows cost a handful of multiplies per element.  The streamline-upwind term and
// the derivative of the SUPG weight reduce to sums of the Hadamard transform of the
// Gauss-point convection (12 multiply-adds each, see modal_grad_dot).  Only the
// convective Gauss-point products remain per Gauss point.  The arithmetic is the same
// discrete operator as the Gauss-point form above.
// ===================================================================================

template <typename T> struct MC {
  static constexpr T K1 = (T)8, K4 = (T)(16.0 / 3.0), K7 = (T)(8.0 / 3.0);
  static constexpr T B0 = (T)8, B1 = (T)(8.0 / 3.0), B4 = (T)(8.0 / 9.0);
};

// rho += v (x) F: contributions of sum_q grad N_a(q) . v f(q) to the modal coefficients
// rho, where F = hadamard_fwd(f) (f given at the Gauss points), up to the factor dxi/8.
template <typename T>
NC_HD void modal_grad_dot(T vx, T vy, T vz, const T F[8], T rho[8]) {
  const T g = GC<T>::g, g2 = GC<T>::g2;
  rho[1] += vx * F[0];
  rho[2] += vy * F[0];
  rho[3] += vz * F[0];
  rho[4] += g * (vx * F[2] + vy * F[1]);
  rho[5] += g * (vx * F[3] + vz * F[1]);
  rho[6] += g * (vy * F[3] + vz * F[2]);
  rho[7] += g2 * (vx * F[6] + vy * F[5] + vz * F[4]);
}

// transpose of modal_grad_dot with respect to F
template <typename T>
NC_HD void modal_grad_dot_T_F(T vx, T vy, T vz, const T rb[8], T Fb[8]) {
  const T g = GC<T>::g, g2 = GC<T>::g2;
  Fb[0] += vx * rb[1] + vy * rb[2] + vz * rb[3];
  Fb[1] += g * (vy * rb[4] + vz * rb[5]);
  Fb[2] += g * (vx * rb[4] + vz * rb[6]);
  Fb[3] += g * (vx * rb[5] + vy * rb[6]);
  Fb[4] += g2 * vz * rb[7];
  Fb[5] += g2 * vy * rb[7];
  Fb[6] += g2 * vx * rb[7];
}

// transpose of modal_grad_dot with respect to v
template <typename T>
NC_HD void modal_grad_dot_T_v(const T F[8], const T rb[8], T& vx, T& vy, T& vz) {
  const T g = GC<T>::g, g2 = GC<T>::g2;
  vx = F[0] * rb[1] + g * (F[2] * rb[4] + F[3] * rb[5]) + g2 * F[6] * rb[7];
  vy = F[0] * rb[2] + g * (F[1] * rb[4] + F[3] * rb[6]) + g2 * F[5] * rb[7];
  vz = F[0] * rb[3] + g * (F[1] * rb[5] + F[2] * rb[6]) + g2 * F[4] * rb[7];
}

// transpose of bilinear4: (a, b, c, d) += sums of o weighted by 1, s_i, s_j, s_i s_j
template <typename T>
NC_HD void bilinear4_T(const T o[4], T& a, T& b, T& c, T& d) {
  a += (o[0] + o[1]) + (o[2] + o[3]);
  b += (o[1] + o[3]) - (o[0] + o[2]);
  c += (o[2] + o[3]) - (o[0] + o[1]);
  d += (o[0] + o[3]) - (o[1] + o[2]);
}

// Per-element linearisation data for the modal operators.
template <typename T>
struct LinM {
  T ux[4], uy[4], uz[8];       // Darcy velocity at the Gauss points
  T gTx[4], gTy[4], gTz[4];    // grad T at the Gauss points
  T C[8];                      // hadamard_fwd of conv_q = rho0 c_p u_q . grad T_q - Q
  T u0[3];                     // centroid velocity
  T tau, dtau;                 // SUPG parameter and d tau / d (u0 . du0)
  T k, cm;                     // conductivity and kappa / mu
  T mP[8], mT[8];              // modal coefficients of P and T (8 x)
};

// Gauss-point velocity of a (pressure, temperature) pair given by modal coefficients:
// u = -cm (grad p - beta t e_z); ux indexed by (qy, qz), uy by (qx, qz), uz by q.
template <typename T>
NC_HD void modal_velocity(const T mp[8], const T mt[8], T cm, const ElemConst<T>& c, T ux[4], T uy[4], T uz[8],
                          T u0[3]) {
  const T g = GC<T>::g, g2 = GC<T>::g2, g3 = GC<T>::g3;
  const T fu = -cm * c.dxi * (T)0.125;
  const T e1 = fu * mp[1], e2 = fu * mp[2], e3 = fu * mp[3];
  const T e4 = fu * g * mp[4], e5 = fu * g * mp[5], e6 = fu * g * mp[6], e7 = fu * g2 * mp[7];
  bilinear4(e1, e4, e5, e7, ux);
  bilinear4(e2, e4, e6, e7, uy);
  T uzp[4];
  bilinear4(e3, e5, e6, e7, uzp);
  const T ft = cm * c.beta * (T)0.125;
  const T et[8] = {ft * mt[0], ft * g * mt[1], ft * g * mt[2], ft * g * mt[3],
                   ft * g2 * mt[4], ft * g2 * mt[5], ft * g2 * mt[6], ft * g3 * mt[7]};
  T tq[8];
  hadamard_inv(et, tq);
#pragma unroll
  for (int q = 0; q < 8; ++q) uz[q] = uzp[jz_of(q)] + tq[q];
  u0[0] = e1;
  u0[1] = e2;
  u0[2] = e3 + et[0];
}

template <typename T>
NC_HD void lin_modal_q(const T P[8], const T Tn[8], T k, T kap, T Q, const ElemConst<T>& c, LinM<T>& L) {
  hadamard_fwd(P, L.mP);
  hadamard_fwd(Tn, L.mT);
  L.k = k;
  L.cm = kap * c.inv_mu;
  modal_velocity(L.mP, L.mT, L.cm, c, L.ux, L.uy, L.uz, L.u0);
  T gc[3];
  grad_from_modal(L.mT, c, L.gTx, L.gTy, L.gTz, gc);
  T conv[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int jx = jx_of(q), jy = jy_of(q), jz = jz_of(q);
    conv[q] = c.rcp * (L.ux[jx] * L.gTx[jx] + L.uy[jy] * L.gTy[jy] + L.uz[q] * L.gTz[jz]) - Q;
  }
  hadamard_fwd(conv, L.C);
  const T s = (T)4 * (L.u0[0] * L.u0[0] + L.u0[1] * L.u0[1] + L.u0[2] * L.u0[2]) * c.inv_he2 + c.tau3inv2;
  const T tau = (T)1 / sqrt(s);
  L.tau = tau;
  L.dtau = (T)(-4) * tau * tau * tau * c.inv_he2;
}
// with the constant's source Q
template <typename T>
NC_HD void lin_modal(const T P[8], const T Tn[8], T k, T kap, const ElemConst<T>& c, LinM<T>& L) {
  lin_modal_q(P, Tn, k, kap, c.Q, c, L);
}

// Pressure rows in modal form: rho_m = W cm [dxi^2/64 K_m mp_m - beta dxi/64 B mt]
template <typename T>
NC_HD void modal_prow(const T mp[8], const T mt[8], T cm, const ElemConst<T>& c, T rho[8]) {
  const T a = cm * c.W * c.dxi * c.dxi * (T)(1.0 / 64.0);
  const T b = cm * c.W * c.dxi * c.beta * (T)(1.0 / 64.0);
  rho[0] = (T)0;
  rho[1] = a * MC<T>::K1 * mp[1];
  rho[2] = a * MC<T>::K1 * mp[2];
  rho[3] = a * MC<T>::K1 * mp[3] - b * MC<T>::B0 * mt[0];
  rho[4] = a * MC<T>::K4 * mp[4];
  rho[5] = a * MC<T>::K4 * mp[5] - b * MC<T>::B1 * mt[1];
  rho[6] = a * MC<T>::K4 * mp[6] - b * MC<T>::B1 * mt[2];
  rho[7] = a * MC<T>::K7 * mp[7] - b * MC<T>::B4 * mt[4];
}

// Velocity rows: yU_a = -W sum_q N_a(q) u_q for u = (ux, uy, uzp[jz] + t-part), using
// that ux depends on (qy, qz) only (the x-sum of N_a is one), and likewise uy, uzp.  The
// temperature part of uz is projected in modal form (mass matrix diagonal).
template <typename T>
NC_HD void modal_urows(const T ux[4], const T uy[4], const T uzp[4], const T mt[8], T cmbeta, const ElemConst<T>& c,
                       T yU[3][8]) {
  const T g = GC<T>::g, g2 = GC<T>::g2, g4 = GC<T>::g2 * GC<T>::g2;
  const T w4 = -c.W * (T)0.25;
  T vx[4], vy[4], vz[4];
  {
    T a = 0, b = 0, cc = 0, d = 0;
    bilinear4_T(ux, a, b, cc, d);
    bilinear4(w4 * a, w4 * g * b, w4 * g * cc, w4 * g2 * d, vx);
  }
  {
    T a = 0, b = 0, cc = 0, d = 0;
    bilinear4_T(uy, a, b, cc, d);
    bilinear4(w4 * a, w4 * g * b, w4 * g * cc, w4 * g2 * d, vy);
  }
  {
    T a = 0, b = 0, cc = 0, d = 0;
    bilinear4_T(uzp, a, b, cc, d);
    bilinear4(w4 * a, w4 * g * b, w4 * g * cc, w4 * g2 * d, vz);
  }
  const T ft = -c.W * cmbeta * (T)0.125;
  const T et[8] = {ft * mt[0], ft * g2 * mt[1], ft * g2 * mt[2], ft * g2 * mt[3],
                   ft * g4 * mt[4], ft * g4 * mt[5], ft * g4 * mt[6], ft * g4 * g2 * mt[7]};
  T tz[8];
  hadamard_inv(et, tz);
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    const int ia = a & 1, ja = (a >> 1) & 1, ka = (a >> 2) & 1;
    yU[0][a] += vx[ja + 2 * ka];
    yU[1][a] += vy[ia + 2 * ka];
    yU[2][a] += vz[ia + 2 * ja] + tz[a];
  }
}

// Energy rows in modal form for a Gauss-point convection f with transform F: the
// Galerkin and streamline parts plus conduction k K_m mt_m:
//   rho_m = W/8 g^deg(m) F_m + W dxi/8 (tau u0) (x) F + W k dxi^2/64 K_m mt_m
template <typename T>
NC_HD void modal_trow(const T F[8], const T mt[8], const LinM<T>& L, const ElemConst<T>& c, T rho[8]) {
  const T g = GC<T>::g, g2 = GC<T>::g2, g3 = GC<T>::g3;
  const T w8 = c.W * (T)0.125;
  const T kd = L.k * c.W * c.dxi * c.dxi * (T)(1.0 / 64.0);
  rho[0] = w8 * F[0];
  rho[1] = w8 * g * F[1] + kd * MC<T>::K1 * mt[1];
  rho[2] = w8 * g * F[2] + kd * MC<T>::K1 * mt[2];
  rho[3] = w8 * g * F[3] + kd * MC<T>::K1 * mt[3];
  rho[4] = w8 * g2 * F[4] + kd * MC<T>::K4 * mt[4];
  rho[5] = w8 * g2 * F[5] + kd * MC<T>::K4 * mt[5];
  rho[6] = w8 * g2 * F[6] + kd * MC<T>::K4 * mt[6];
  rho[7] = w8 * g3 * F[7] + kd * MC<T>::K7 * mt[7];
  const T sd = w8 * c.dxi * L.tau;
  modal_grad_dot(sd * L.u0[0], sd * L.u0[1], sd * L.u0[2], F, rho);
}

template <typename T, bool WITH_U>
NC_HD void elem_residual_m(const LinM<T>& L, const ElemConst<T>& c, T rP[8], T rT[8], T rU[3][8]) {
  T rho[8];
  modal_prow(L.mP, L.mT, L.cm, c, rho);
  T v[8];
  hadamard_inv(rho, v);
#pragma unroll
  for (int a = 0; a < 8; ++a) rP[a] += v[a];
  modal_trow(L.C, L.mT, L, c, rho);
  hadamard_inv(rho, v);
#pragma unroll
  for (int a = 0; a < 8; ++a) rT[a] += v[a];
  if constexpr (WITH_U) {
    // split uz into its pressure part (bilinear in x, y) and temperature part
    T uzp[4];
    {
      const T g = GC<T>::g, g2 = GC<T>::g2;
      const T fu = -L.cm * c.dxi * (T)0.125;
      bilinear4(fu * L.mP[3], fu * g * L.mP[5], fu * g * L.mP[6], fu * g2 * L.mP[7], uzp);
    }
    modal_urows(L.ux, L.uy, uzp, L.mT, L.cm * c.beta, c, rU);
  }
}

// Exact Newton Jacobian times (p, t), modal form of elem_jv.
template <typename T, bool WITH_U>
NC_HD void elem_jv_m(const LinM<T>& L, const T p[8], const T t[8], const ElemConst<T>& c, T yP[8], T yT[8],
                     T yU[3][8]) {
  T mp[8], mt[8];
  hadamard_fwd(p, mp);
  hadamard_fwd(t, mt);
  T rho[8], v[8];
  modal_prow(mp, mt, L.cm, c, rho);
  hadamard_inv(rho, v);
#pragma unroll
  for (int a = 0; a < 8; ++a) yP[a] += v[a];
  T dux[4], duy[4], duz[8], du0[3];
  modal_velocity(mp, mt, L.cm, c, dux, duy, duz, du0);
  T gtx[4], gty[4], gtz[4], gtc[3];
  grad_from_modal(mt, c, gtx, gty, gtz, gtc);
  const T dtau = L.dtau * (L.u0[0] * du0[0] + L.u0[1] * du0[1] + L.u0[2] * du0[2]);
  T dconv[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int jx = jx_of(q), jy = jy_of(q), jz = jz_of(q);
    dconv[q] = c.rcp * (dux[jx] * L.gTx[jx] + duy[jy] * L.gTy[jy] + duz[q] * L.gTz[jz] + L.ux[jx] * gtx[jx] +
                        L.uy[jy] * gty[jy] + L.uz[q] * gtz[jz]);
  }
  T S[8];
  hadamard_fwd(dconv, S);
  modal_trow(S, mt, L, c, rho);
  const T sd = c.W * (T)0.125 * c.dxi;
  modal_grad_dot(sd * (dtau * L.u0[0] + L.tau * du0[0]), sd * (dtau * L.u0[1] + L.tau * du0[1]),
                 sd * (dtau * L.u0[2] + L.tau * du0[2]), L.C, rho);
  hadamard_inv(rho, v);
#pragma unroll
  for (int a = 0; a < 8; ++a) yT[a] += v[a];
  if constexpr (WITH_U) {
    T duzp[4];
    const T g = GC<T>::g, g2 = GC<T>::g2;
    const T fu = -L.cm * c.dxi * (T)0.125;
    bilinear4(fu * mp[3], fu * g * mp[5], fu * g * mp[6], fu * g2 * mp[7], duzp);
    modal_urows(dux, duy, duzp, mt, L.cm * c.beta, c, yU);
  }
}

// Transpose of elem_jv_m: contributions of the row weights (wP, wT, wU) to the P and T
// columns, obtained by running each step of elem_jv_m backwards.
template <typename T, bool WITH_U>
NC_HD void elem_jtw_m(const LinM<T>& L, const T wP[8], const T wT[8], const T wU[3][8], const ElemConst<T>& c,
                      T yP[8], T yT[8]) {
  const T g = GC<T>::g, g2 = GC<T>::g2, g3 = GC<T>::g3, g4 = GC<T>::g2 * GC<T>::g2;
  const T cm = L.cm;
  T rbP[8], rbT[8];
  hadamard_fwd(wP, rbP);
  hadamard_fwd(wT, rbT);
  T mbp[8] = {0, 0, 0, 0, 0, 0, 0, 0}, mbt[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  // pressure rows
  {
    const T a = cm * c.W * c.dxi * c.dxi * (T)(1.0 / 64.0);
    const T b = cm * c.W * c.dxi * c.beta * (T)(1.0 / 64.0);
    mbp[1] += a * MC<T>::K1 * rbP[1];
    mbp[2] += a * MC<T>::K1 * rbP[2];
    mbp[3] += a * MC<T>::K1 * rbP[3];
    mbp[4] += a * MC<T>::K4 * rbP[4];
    mbp[5] += a * MC<T>::K4 * rbP[5];
    mbp[6] += a * MC<T>::K4 * rbP[6];
    mbp[7] += a * MC<T>::K7 * rbP[7];
    mbt[0] -= b * MC<T>::B0 * rbP[3];
    mbt[1] -= b * MC<T>::B1 * rbP[5];
    mbt[2] -= b * MC<T>::B1 * rbP[6];
    mbt[4] -= b * MC<T>::B4 * rbP[7];
  }
  // energy rows: rho = w8 g^deg S + kd K mt + sd tau u0 (x) S + sd A (x) C
  const T w8 = c.W * (T)0.125;
  const T kd = L.k * c.W * c.dxi * c.dxi * (T)(1.0 / 64.0);
  T Sb[8] = {w8 * rbT[0], w8 * g * rbT[1], w8 * g * rbT[2], w8 * g * rbT[3],
             w8 * g2 * rbT[4], w8 * g2 * rbT[5], w8 * g2 * rbT[6], w8 * g3 * rbT[7]};
  mbt[1] += kd * MC<T>::K1 * rbT[1];
  mbt[2] += kd * MC<T>::K1 * rbT[2];
  mbt[3] += kd * MC<T>::K1 * rbT[3];
  mbt[4] += kd * MC<T>::K4 * rbT[4];
  mbt[5] += kd * MC<T>::K4 * rbT[5];
  mbt[6] += kd * MC<T>::K4 * rbT[6];
  mbt[7] += kd * MC<T>::K7 * rbT[7];
  const T sd = w8 * c.dxi;
  modal_grad_dot_T_F(sd * L.tau * L.u0[0], sd * L.tau * L.u0[1], sd * L.tau * L.u0[2], rbT, Sb);
  T Ab[3];
  modal_grad_dot_T_v(L.C, rbT, Ab[0], Ab[1], Ab[2]);
  Ab[0] *= sd; Ab[1] *= sd; Ab[2] *= sd;
  // A = dtau u0 + tau du0 with dtau = L.dtau (u0 . du0)
  const T ua = L.u0[0] * Ab[0] + L.u0[1] * Ab[1] + L.u0[2] * Ab[2];
  T du0b[3] = {L.tau * Ab[0] + L.dtau * ua * L.u0[0], L.tau * Ab[1] + L.dtau * ua * L.u0[1],
               L.tau * Ab[2] + L.dtau * ua * L.u0[2]};
  // S = hadamard_fwd(dconv)
  T dcb[8];
  hadamard_inv(Sb, dcb);
  // dconv = rcp (du . gT + u . gt)
  T duxb[4] = {0, 0, 0, 0}, duyb[4] = {0, 0, 0, 0}, duzb[8], gtxb[4] = {0, 0, 0, 0}, gtyb[4] = {0, 0, 0, 0},
    gtzb[4] = {0, 0, 0, 0};
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int jx = jx_of(q), jy = jy_of(q), jz = jz_of(q);
    const T r = c.rcp * dcb[q];
    duxb[jx] += r * L.gTx[jx];
    duyb[jy] += r * L.gTy[jy];
    duzb[q] = r * L.gTz[jz];
    gtxb[jx] += r * L.ux[jx];
    gtyb[jy] += r * L.uy[jy];
    gtzb[jz] += r * L.uz[q];
  }
  // velocity rows
  T duzpb[4] = {0, 0, 0, 0};
  if constexpr (WITH_U) {
    const T w4 = -c.W * (T)0.25;
    T ox[4], oy[4], oz[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      ox[i] = wU[0][2 * i] + wU[0][2 * i + 1];                    // sum over ia at (ja, ka) = i
      oy[i] = wU[1][(i & 1) + 4 * (i >> 1)] + wU[1][(i & 1) + 2 + 4 * (i >> 1)];   // sum over ja at (ia, ka)
      oz[i] = wU[2][i] + wU[2][i + 4];                            // sum over ka at (ia, ja)
    }
    {
      T a = 0, b = 0, cc = 0, d = 0;
      bilinear4_T(ox, a, b, cc, d);
      T tmp[4];
      bilinear4(w4 * a, w4 * g * b, w4 * g * cc, w4 * g2 * d, tmp);
#pragma unroll
      for (int j = 0; j < 4; ++j) duxb[j] += tmp[j];
    }
    {
      T a = 0, b = 0, cc = 0, d = 0;
      bilinear4_T(oy, a, b, cc, d);
      T tmp[4];
      bilinear4(w4 * a, w4 * g * b, w4 * g * cc, w4 * g2 * d, tmp);
#pragma unroll
      for (int j = 0; j < 4; ++j) duyb[j] += tmp[j];
    }
    {
      T a = 0, b = 0, cc = 0, d = 0;
      bilinear4_T(oz, a, b, cc, d);
      bilinear4(w4 * a, w4 * g * b, w4 * g * cc, w4 * g2 * d, duzpb);
    }
    T mwz[8];
    hadamard_fwd(wU[2], mwz);
    const T ft = -c.W * cm * c.beta * (T)0.125;
    mbt[0] += ft * mwz[0];
    mbt[1] += ft * g2 * mwz[1];
    mbt[2] += ft * g2 * mwz[2];
    mbt[3] += ft * g2 * mwz[3];
    mbt[4] += ft * g4 * mwz[4];
    mbt[5] += ft * g4 * mwz[5];
    mbt[6] += ft * g4 * mwz[6];
    mbt[7] += ft * g4 * g2 * mwz[7];
  }
  // uz = uzp[jz] + tq: tq from mt, uzp from mp
#pragma unroll
  for (int q = 0; q < 8; ++q) duzpb[jz_of(q)] += duzb[q];
  {
    const T ft = cm * c.beta * (T)0.125;
    T Tq[8];
    hadamard_fwd(duzb, Tq);
    mbt[0] += ft * Tq[0] + ft * du0b[2];      // centroid du0z = e3 + ft mt0
    mbt[1] += ft * g * Tq[1];
    mbt[2] += ft * g * Tq[2];
    mbt[3] += ft * g * Tq[3];
    mbt[4] += ft * g2 * Tq[4];
    mbt[5] += ft * g2 * Tq[5];
    mbt[6] += ft * g2 * Tq[6];
    mbt[7] += ft * g3 * Tq[7];
  }
  // ux = bilinear4(e1, e4, e5, e7), uy = bilinear4(e2, e4, e6, e7), uzp = bilinear4(e3, e5, e6, e7)
  {
    T e1 = du0b[0], e2 = du0b[1], e3 = du0b[2], e4 = 0, e5 = 0, e6 = 0, e7 = 0;
    bilinear4_T(duxb, e1, e4, e5, e7);
    bilinear4_T(duyb, e2, e4, e6, e7);
    bilinear4_T(duzpb, e3, e5, e6, e7);
    const T fu = -cm * c.dxi * (T)0.125;
    mbp[1] += fu * e1;
    mbp[2] += fu * e2;
    mbp[3] += fu * e3;
    mbp[4] += fu * g * e4;
    mbp[5] += fu * g * e5;
    mbp[6] += fu * g * e6;
    mbp[7] += fu * g2 * e7;
  }
  // grad t = bilinear4 of (s mt1, s g mt4, s g mt5, s g2 mt7) etc.
  {
    T e1 = 0, e2 = 0, e3 = 0, e4 = 0, e5 = 0, e6 = 0, e7 = 0;
    bilinear4_T(gtxb, e1, e4, e5, e7);
    bilinear4_T(gtyb, e2, e4, e6, e7);
    bilinear4_T(gtzb, e3, e5, e6, e7);
    const T s = c.dxi * (T)0.125;
    mbt[1] += s * e1;
    mbt[2] += s * e2;
    mbt[3] += s * e3;
    mbt[4] += s * g * e4;
    mbt[5] += s * g * e5;
    mbt[6] += s * g * e6;
    mbt[7] += s * g2 * e7;
  }
  T v[8];
  hadamard_inv(mbp, v);
#pragma unroll
  for (int a = 0; a < 8; ++a) yP[a] += v[a];
  hadamard_inv(mbt, v);
#pragma unroll
  for (int a = 0; a < 8; ++a) yT[a] += v[a];
}

// RAMP interpolation (Sec. 5.2, eqs. condRAMP and permRAMP) and derivatives.
template <typename T>
NC_HD void ramp(T gam, T k_f, T k_s, T q_c, T kap_f, T kap_s, T q_p, T& k, T& kap, T& dk, T& dkap) {
  const T dc = (T)1 + q_c * ((T)1 - gam);
  const T dp = (T)1 + q_p * gam;
  k = k_f + gam / dc * (k_s - k_f);
  kap = kap_s + ((T)1 - gam) / dp * (kap_f - kap_s);
  dk = (k_s - k_f) * ((T)1 + q_c) / (dc * dc);
  dkap = -(kap_f - kap_s) * ((T)1 + q_p) / (dp * dp);
}

}  // namespace nc
