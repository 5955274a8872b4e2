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
  T Q;         // uniform volumetric source
  T inv_he2;   // 1 / h_e^2, h_e^2 = dx^2 + dy^2 + dz^2 = 3 h^2
  T tau3inv2;  // tau3^-2 = 16 / h_e^4
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
NC_HD void linearize(const T P[8], const T Tn[8], T k, T kap, const ElemConst<T>& c, Lin<T>& L) {
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
    L.conv[q] = c.rcp * kap * (L.uhx[jx] * L.gTx[jx] + L.uhy[jy] * L.gTy[jy] + L.uhz[q] * L.gTz[jz]) - c.Q;
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
  if (WITH_U) {
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
  if (WITH_U) {
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
  if (WITH_U) {
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
    if (WITH_U) {
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
  if (WITH_U) {
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
    if (WITH_U) a -= luq[0][q] * uhx + luq[1][q] * uhy + luq[2][q] * uhz;
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
