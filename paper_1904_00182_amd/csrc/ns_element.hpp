// Element rows of the Navier-Stokes / Brinkman flow model (the full-flow model of the
// hybrid strategy, Sec. 6.4): the momentum equation of Sec. 2.1 (eq. app_NS, modified
// pressure, Boussinesq buoyancy) with a Brinkman friction a(gamma) u, incompressibility
// and the energy equation of eq. goveq, on equal-order trilinear elements with 2x2x2
// Gauss points:
//   momentum   sum_q detJ [ W_a r_m + mu grad N_a . (grad u + grad u^T) ]
//   continuity sum_q detJ [ N_a div u + (tau_m / rho0) grad N_a . r_m ]
//   energy     sum_q detJ [ N*_a (rho0 c_p u . grad T - Q) + k grad N_a . grad T ]
// r_m = rho0 (u . grad) u + grad P + a u + rho0 alpha g T (the strong momentum residual
// without the viscous term), W_a = N_a + tau_m u0 . grad N_a, N*_a = N_a + tau u0 . grad N_a,
// u0 the centroid velocity, h_e^2 = 3 h^2,
//   tau_m = (4 |u0|^2 / h_e^2 + 16 nu^2 / h_e^4 + (a / rho0)^2)^(-1/2),
//   tau   = (4 |u0|^2 / h_e^2 + 16 / h_e^4)^(-1/2)   (the energy parameter of App. A).
//
// The routine is written once over a scalar type S: double gives the residual, Dual (a
// value with one directional derivative) the exact Jacobian column or design derivative
// by forward-mode differentiation of the same arithmetic.
#pragma once

#include <hip/hip_runtime.h>

namespace nc {
namespace ns {

struct Dual {
  double v, d;
};
__device__ inline Dual operator+(Dual a, Dual b) { return Dual{a.v + b.v, a.d + b.d}; }
__device__ inline Dual operator-(Dual a, Dual b) { return Dual{a.v - b.v, a.d - b.d}; }
__device__ inline Dual operator*(Dual a, Dual b) { return Dual{a.v * b.v, a.v * b.d + a.d * b.v}; }
__device__ inline Dual operator*(double s, Dual a) { return Dual{s * a.v, s * a.d}; }
__device__ inline Dual operator*(Dual a, double s) { return Dual{s * a.v, s * a.d}; }
__device__ inline Dual operator+(Dual a, double s) { return Dual{a.v + s, a.d}; }
__device__ inline Dual operator+(double s, Dual a) { return Dual{a.v + s, a.d}; }
__device__ inline Dual operator-(Dual a, double s) { return Dual{a.v - s, a.d}; }
__device__ inline Dual& operator+=(Dual& a, Dual b) { a = a + b; return a; }

// s^(-1/2)
__device__ inline double rsqrt_(double s) { return 1.0 / sqrt(s); }
__device__ inline Dual rsqrt_(Dual s) {
  const double r = 1.0 / sqrt(s.v);
  return Dual{r, -0.5 * s.d * r * r * r};
}

template <class S> __device__ inline S lift(double v);
template <> __device__ inline double lift<double>(double v) { return v; }
template <> __device__ inline Dual lift<Dual>(double v) { return Dual{v, 0.0}; }

// Constants of one grid level.
struct NsConst {
  double h;        // element edge
  double rho, mu, cp;
  double bz;       // z component of rho0 alpha g (g = (0, 0, -g0)): -rho0 alpha g0
  double nu2;      // (mu / rho0)^2
  double he2;      // h_e^2 = 3 h^2
  double Q;        // volumetric source on the elements of the source box (every element
  int qi0, qi1, qj0, qj1, qk0, qk1;   // when the box covers the grid), inclusive ranges
  __host__ __device__ double source(int i, int j, int k) const {
    return (i >= qi0 && i <= qi1 && j >= qj0 && j <= qj1 && k >= qk0 && k <= qk1) ? Q : 0.0;
  }
};

// Gauss coordinates of the unit interval, (1 -+ 1/sqrt 3) / 2
constexpr double G0 = 0.21132486540518711775, G1 = 0.78867513459481288225;

// Element rows.  `in(a, f)` gives local node a's unknown f (0..2 velocity, 3 P, 4 T) as
// S, `out(a, f, v)` receives row (a, f); k and a are the element's conductivity and
// Brinkman coefficient, Q its source.
template <class S, class In, class Out>
__device__ inline void element_rows(const NsConst& c, S k, S a, double Q, const In& in, Out& out) {
  const double h = c.h, ih = 1.0 / h, detJ = h * h * h * 0.125;
  S v[8][5];
#pragma unroll
  for (int n = 0; n < 8; ++n)
#pragma unroll
    for (int f = 0; f < 5; ++f) v[n][f] = in(n, f);
  S u0[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    S s = v[0][i];
#pragma unroll
    for (int n = 1; n < 8; ++n) s += v[n][i];
    u0[i] = 0.125 * s;
  }
  const S uu = u0[0] * u0[0] + u0[1] * u0[1] + u0[2] * u0[2];
  const double ihe2 = 1.0 / c.he2;
  const S adv2 = 4.0 * ihe2 * uu;
  const S tau_m = rsqrt_(adv2 + 16.0 * c.nu2 * ihe2 * ihe2 + (1.0 / (c.rho * c.rho)) * (a * a));
  const S tau_t = rsqrt_(adv2 + 16.0 * ihe2 * ihe2);
  const S tm_rho = (1.0 / c.rho) * tau_m;
#pragma unroll 1
  for (int q = 0; q < 8; ++q) {
    const double gx = (q & 1) ? G1 : G0, gy = (q & 2) ? G1 : G0, gz = (q & 4) ? G1 : G0;
    // shape values and gradients of the eight nodes at this point
    double N[8], D[8][3];
#pragma unroll
    for (int n = 0; n < 8; ++n) {
      const double lx = (n & 1) ? gx : 1.0 - gx, ly = (n & 2) ? gy : 1.0 - gy, lz = (n & 4) ? gz : 1.0 - gz;
      const double dx = (n & 1) ? ih : -ih, dy = (n & 2) ? ih : -ih, dz = (n & 4) ? ih : -ih;
      N[n] = lx * ly * lz;
      D[n][0] = dx * ly * lz;
      D[n][1] = lx * dy * lz;
      D[n][2] = lx * ly * dz;
    }
    S uq[3], Gu[3][3], GP[3], Tq, GT[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      uq[i] = N[0] * v[0][i];
      GP[i] = D[0][i] * v[0][3];
      GT[i] = D[0][i] * v[0][4];
#pragma unroll
      for (int j = 0; j < 3; ++j) Gu[i][j] = D[0][j] * v[0][i];
    }
    Tq = N[0] * v[0][4];
#pragma unroll
    for (int n = 1; n < 8; ++n) {
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        uq[i] += N[n] * v[n][i];
        GP[i] += D[n][i] * v[n][3];
        GT[i] += D[n][i] * v[n][4];
#pragma unroll
        for (int j = 0; j < 3; ++j) Gu[i][j] += D[n][j] * v[n][i];
      }
      Tq += N[n] * v[n][4];
    }
    S rm[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const S conv = uq[0] * Gu[i][0] + uq[1] * Gu[i][1] + uq[2] * Gu[i][2];
      rm[i] = c.rho * conv + GP[i] + a * uq[i];
    }
    rm[2] += c.bz * Tq;
    const S div = Gu[0][0] + Gu[1][1] + Gu[2][2];
    const S cT = (c.rho * c.cp) * (uq[0] * GT[0] + uq[1] * GT[1] + uq[2] * GT[2]) - Q;
    S Sg[3][3];   // symmetric gradient grad u + grad u^T, times mu
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) Sg[i][j] = c.mu * (Gu[i][j] + Gu[j][i]);
#pragma unroll
    for (int n = 0; n < 8; ++n) {
      const S adv = u0[0] * D[n][0] + u0[1] * D[n][1] + u0[2] * D[n][2];
      const S Wm = N[n] + tau_m * adv;
      const S Wt = N[n] + tau_t * adv;
#pragma unroll
      for (int i = 0; i < 3; ++i)
        out(n, i, detJ * (Wm * rm[i] + D[n][0] * Sg[i][0] + D[n][1] * Sg[i][1] + D[n][2] * Sg[i][2]));
      out(n, 3, detJ * (N[n] * div + tm_rho * (D[n][0] * rm[0] + D[n][1] * rm[1] + D[n][2] * rm[2])));
      out(n, 4, detJ * (Wt * cT + k * (D[n][0] * GT[0] + D[n][1] * GT[1] + D[n][2] * GT[2])));
    }
  }
}

// Integrated energy weights int_e N*_a (the weight of the volumetric heat load) at the
// centroid velocity u0 of the element: the Gauss sum of N_a is h^3/8 and of grad N_a is
// +-h^2/4 per direction, so int N*_a = h^3/8 + tau (h^2/4) sum_d s_ad u0_d.
template <class S>
__device__ inline S load_weight(const NsConst& c, const S u0[3], int n) {
  const double ihe2 = 1.0 / c.he2;
  const S uu = u0[0] * u0[0] + u0[1] * u0[1] + u0[2] * u0[2];
  const S tau_t = rsqrt_(4.0 * ihe2 * uu + 16.0 * ihe2 * ihe2);
  const double q = 0.25 * c.h * c.h;
  const S adv = ((n & 1) ? q : -q) * u0[0] + ((n & 2) ? q : -q) * u0[1] + ((n & 4) ? q : -q) * u0[2];
  return c.h * c.h * c.h * 0.125 + tau_t * adv;
}

}  // namespace ns
}  // namespace nc
