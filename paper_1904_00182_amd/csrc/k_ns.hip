// Kernels of the Navier-Stokes / Brinkman solver (the full-flow model of the hybrid
// strategy, Sec. 6.4).  The Jacobian is assembled, not applied matrix-free: every element
// column comes from forward-mode differentiation of the element rows (ns_element.hpp),
// and the node-block matrix (27 neighbours x 5 x 5 per node, one plane per entry so that
// the threads of a wave read consecutive nodes) serves the operator, its transpose for
// the adjoint, the block-Jacobi smoother and the coarsest dense solve.  Element loops
// that scatter into nodes run colour by colour (the eight parities of (i, j, k)): elements
// of one colour share no node, so the accumulation needs no atomics and its order is
// fixed, and results are bitwise reproducible.
#include <cmath>

#include "kernels.hpp"
#include "ns_element.hpp"
#include "ns_kernels.hpp"

namespace nc {
namespace ns {

namespace {

constexpr int BS = 256;

inline int blocks(long n) { return (int)((n + BS - 1) / BS); }

__device__ inline void elem_ijk(const ColourGrid& cg, long t, int& i, int& j, int& k) {
  const int ii = (int)(t % cg.mx);
  const int jj = (int)((t / cg.mx) % cg.my);
  const int kk = (int)(t / ((long)cg.mx * cg.my));
  i = 2 * ii + cg.cx;
  j = 2 * jj + cg.cy;
  k = 2 * kk + cg.cz;
}

__device__ inline void elem_nodes(const Grid& g, int i, int j, int k, int nid[8]) {
#pragma unroll
  for (int n = 0; n < 8; ++n) nid[n] = g.node(i + (n & 1), j + ((n >> 1) & 1), k + (n >> 2));
}

__device__ inline void node_ijk(const Grid& g, long n, int& i, int& j, int& k) {
  i = (int)(n % (g.nx + 1));
  j = (int)((n / (g.nx + 1)) % (g.ny + 1));
  k = (int)(n / ((long)(g.nx + 1) * (g.ny + 1)));
}

// neighbour offset index o = (dx+1) + 3 (dy+1) + 9 (dz+1)
__device__ inline bool neighbour(const Grid& g, int i, int j, int k, int o, int& m) {
  const int a = i + o % 3 - 1, b = j + (o / 3) % 3 - 1, c = k + o / 9 - 1;
  if (a < 0 || a > g.nx || b < 0 || b > g.ny || c < 0 || c > g.nz) return false;
  m = g.node(a, b, c);
  return true;
}

template <typename T>
__global__ void fill_kernel(T* __restrict__ a, long n, T v) {
  for (long t = (long)blockIdx.x * BS + threadIdx.x; t < n; t += (long)gridDim.x * BS) a[t] = v;
}

// r += element rows of one colour
__global__ __launch_bounds__(BS) void residual_kernel(Grid g, NsConst c, ColourGrid cg, const double* __restrict__ coef,
                                                      const double* __restrict__ s, double* __restrict__ r) {
  const long t = (long)blockIdx.x * BS + threadIdx.x;
  if (t >= cg.count) return;
  int i, j, k, nid[8];
  elem_ijk(cg, t, i, j, k);
  elem_nodes(g, i, j, k, nid);
  const long e = g.elem(i, j, k);
  double acc[8][5];
#pragma unroll
  for (int n = 0; n < 8; ++n)
#pragma unroll
    for (int f = 0; f < 5; ++f) acc[n][f] = 0.0;
  auto in = [&](int n, int f) { return s[5 * (long)nid[n] + f]; };
  auto out = [&](int n, int f, double v) { acc[n][f] += v; };
  element_rows<double>(c, coef[2 * e], coef[2 * e + 1], c.source(i, j, k), in, out);
#pragma unroll
  for (int n = 0; n < 8; ++n)
#pragma unroll
    for (int f = 0; f < 5; ++f) r[5 * (long)nid[n] + f] += acc[n][f];
}

// patch flux on the T rows; constrained rows r = s - 0
__global__ void residual_finish_kernel(Grid g, Patch patch, const double* __restrict__ s, double* __restrict__ r) {
  const long n = (long)blockIdx.x * BS + threadIdx.x;
  if (n >= g.nodes()) return;
  int i, j, k;
  node_ijk(g, n, i, j, k);
  if (k == 0) {
    double fl = 0.0;
    for (int dj = -1; dj <= 0; ++dj)
      for (int di = -1; di <= 0; ++di) {
        const int fi = i + di, fj = j + dj;
        if (fi >= 0 && fi < g.nx && fj >= 0 && fj < g.ny && patch.has(fi, fj)) fl += 0.25 * patch.q_h * patch.h * patch.h;
      }
    r[5 * n + 4] -= fl;
  }
#pragma unroll
  for (int f = 0; f < 5; ++f)
    if (fixed(g, i, j, k, f)) r[5 * n + f] = s[5 * n + f];
}

// Jacobian columns of one colour, added into the node-block matrix of precision T, by
// forward-mode differentiation of the element rows with the work shared: a block holds AS_E elements of one colour
// and five waves, wave g the columns of field g (uniform across the wave), lane b * AS_E + le
// the column of node b of element le.  The primal quantities of each element and Gauss
// point (interpolated fields, strong momentum residual, divergence, energy residual,
// symmetric stress) are computed once into LDS; each column then needs only its tangents,
// which for the unit direction of (b, g) follow from N_b and grad N_b at the point:
//   g < 3:  u' = N_b e_g, (grad u)' = e_g grad N_b^T, u0' = e_g / 8
//   g = 3:  (grad P)' = grad N_b
//   g = 4:  T' = N_b, (grad T)' = grad N_b
// differentiating every product of the element rows (including tau_m and tau through u0).
constexpr int AS_E = 8;            // elements per block
constexpr int AS_Q = 26;           // primal doubles per Gauss point
constexpr int AS_X = 11;           // per-element doubles: u0, tau_m, tau, d tau_m / d u0, d tau / d u0

__device__ inline void shape_at(int q, int n, double ih, double& N, double D[3]) {
  const double gx = (q & 1) ? G1 : G0, gy = (q & 2) ? G1 : G0, gz = (q & 4) ? G1 : G0;
  const double lx = (n & 1) ? gx : 1.0 - gx, ly = (n & 2) ? gy : 1.0 - gy, lz = (n & 4) ? gz : 1.0 - gz;
  N = lx * ly * lz;
  D[0] = ((n & 1) ? ih : -ih) * ly * lz;
  D[1] = lx * ((n & 2) ? ih : -ih) * lz;
  D[2] = lx * ly * ((n & 4) ? ih : -ih);
}

template <typename T>
__global__ __launch_bounds__(5 * 64) void assemble_shared_kernel(Grid g, NsConst c, ColourGrid cg,
                                                                 const double* __restrict__ coef,
                                                                 const double* __restrict__ s, T* __restrict__ A,
                                                                 long N) {
  __shared__ double vals[AS_E][40];
  __shared__ double pq[AS_E][8][AS_Q];
  __shared__ double pe[AS_E][AS_X];
  __shared__ int nodes[AS_E][8];
  __shared__ double kc[AS_E], ac[AS_E];
  const int tid = threadIdx.x;
  const int fg = tid >> 6, lane = tid & 63;        // field of the columns, lane
  const int b = lane / AS_E, le = lane % AS_E;     // column node, element in the block
  const long e0 = (long)blockIdx.x * AS_E;
  const double h = c.h, ih = 1.0 / h, detJ = h * h * h * 0.125;
  // nodal values and ids
  {
    const int el = tid / 40, d = tid % 40;
    if (el < AS_E && e0 + el < cg.count) {
      int i, j, k;
      elem_ijk(cg, e0 + el, i, j, k);
      const int n = d / 5, f = d % 5;
      const int id = g.node(i + (n & 1), j + ((n >> 1) & 1), k + (n >> 2));
      vals[el][d] = s[5 * (long)id + f];
      if (f == 0) nodes[el][n] = id;
      if (d == 0) {
        const long e = g.elem(i, j, k);
        kc[el] = coef[2 * e];
        ac[el] = coef[2 * e + 1];
      }
    }
  }
  __syncthreads();
  // primal quantities per (element, Gauss point): the first wave
  if (fg == 0 && e0 + (lane >> 3) < cg.count) {
    const int el = lane >> 3, q = lane & 7;
    const double a = ac[el];
    double uq[3] = {0, 0, 0}, Gu[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}}, GP[3] = {0, 0, 0}, Tq = 0,
           GT[3] = {0, 0, 0};
    double u0[3] = {0, 0, 0};
    for (int n = 0; n < 8; ++n) {
      double Nn, D[3];
      shape_at(q, n, ih, Nn, D);
      const double* v = vals[el] + 5 * n;
      for (int i = 0; i < 3; ++i) {
        uq[i] += Nn * v[i];
        u0[i] += 0.125 * v[i];
        GP[i] += D[i] * v[3];
        GT[i] += D[i] * v[4];
        for (int jj = 0; jj < 3; ++jj) Gu[i][jj] += D[jj] * v[i];
      }
      Tq += Nn * v[4];
    }
    double* P = pq[el][q];
    double rm[3];
    for (int i = 0; i < 3; ++i)
      rm[i] = c.rho * (uq[0] * Gu[i][0] + uq[1] * Gu[i][1] + uq[2] * Gu[i][2]) + GP[i] + a * uq[i];
    rm[2] += c.bz * Tq;
    for (int i = 0; i < 3; ++i) {
      P[i] = uq[i];
      for (int jj = 0; jj < 3; ++jj) P[3 + 3 * i + jj] = Gu[i][jj];
      P[12 + i] = GT[i];
      P[15 + i] = rm[i];
    }
    P[18] = Gu[0][0] + Gu[1][1] + Gu[2][2];
    P[19] = (c.rho * c.cp) * (uq[0] * GT[0] + uq[1] * GT[1] + uq[2] * GT[2]);   // the source is subtracted below
    P[20] = c.mu * 2.0 * Gu[0][0];
    P[21] = c.mu * 2.0 * Gu[1][1];
    P[22] = c.mu * 2.0 * Gu[2][2];
    P[23] = c.mu * (Gu[0][1] + Gu[1][0]);
    P[24] = c.mu * (Gu[0][2] + Gu[2][0]);
    P[25] = c.mu * (Gu[1][2] + Gu[2][1]);
    if (q == 0) {
      const double ihe2 = 1.0 / c.he2;
      const double uu = u0[0] * u0[0] + u0[1] * u0[1] + u0[2] * u0[2];
      const double tm = 1.0 / sqrt(4.0 * ihe2 * uu + 16.0 * c.nu2 * ihe2 * ihe2 + a * a / (c.rho * c.rho));
      const double tt = 1.0 / sqrt(4.0 * ihe2 * uu + 16.0 * ihe2 * ihe2);
      double* X = pe[el];
      for (int i = 0; i < 3; ++i) {
        X[i] = u0[i];
        X[5 + i] = -4.0 * ihe2 * u0[i] * tm * tm * tm;
        X[8 + i] = -4.0 * ihe2 * u0[i] * tt * tt * tt;
      }
      X[3] = tm;
      X[4] = tt;
    }
  }
  __syncthreads();
  if (e0 + le >= cg.count) return;
  int ei, ej, ek;
  elem_ijk(cg, e0 + le, ei, ej, ek);
  const double Qe = c.source(ei, ej, ek);
  const double k = kc[le], a = ac[le];
  const double* X = pe[le];
  const double u0[3] = {X[0], X[1], X[2]};
  const double tm = X[3], tt = X[4];
  // tangents of u0, tau_m and tau for this column
  const double du0 = fg < 3 ? 0.125 : 0.0;
  const double dtm = fg < 3 ? 0.125 * X[5 + fg] : 0.0, dtt = fg < 3 ? 0.125 * X[8 + fg] : 0.0;
  const double irho = 1.0 / c.rho, rcp = c.rho * c.cp;
  double col[8][5];
#pragma unroll
  for (int n = 0; n < 8; ++n)
#pragma unroll
    for (int f = 0; f < 5; ++f) col[n][f] = 0.0;
#pragma unroll 1
  for (int q = 0; q < 8; ++q) {
    const double* P = pq[le][q];
    double Nb, Db[3];
    shape_at(q, b, ih, Nb, Db);
    const double uq[3] = {P[0], P[1], P[2]};
    const double rm[3] = {P[15], P[16], P[17]};
    const double cT = P[19] - Qe;
    // tangents of the point quantities
    double drm[3], ddiv = 0.0, dcT = 0.0, dGT[3] = {0, 0, 0};
    const double ub = uq[0] * Db[0] + uq[1] * Db[1] + uq[2] * Db[2];
    if (fg < 3) {
#pragma unroll
      for (int i = 0; i < 3; ++i) drm[i] = c.rho * Nb * P[3 + 3 * i + fg];
      drm[fg] += c.rho * ub + a * Nb;
      ddiv = Db[fg];
      dcT = rcp * Nb * P[12 + fg];
    } else if (fg == 3) {
#pragma unroll
      for (int i = 0; i < 3; ++i) drm[i] = Db[i];
    } else {
      drm[0] = drm[1] = 0.0;
      drm[2] = c.bz * Nb;
      dcT = rcp * ub;
#pragma unroll
      for (int i = 0; i < 3; ++i) dGT[i] = Db[i];
    }
#pragma unroll
    for (int n = 0; n < 8; ++n) {
      double Nn, Dn[3];
      shape_at(q, n, ih, Nn, Dn);
      const double adv = u0[0] * Dn[0] + u0[1] * Dn[1] + u0[2] * Dn[2];
      const double dadv = fg < 3 ? du0 * Dn[fg] : 0.0;
      const double Wm = Nn + tm * adv, dWm = dtm * adv + tm * dadv;
      const double Wt = Nn + tt * adv, dWt = dtt * adv + tt * dadv;
      const double Dnrm = Dn[0] * rm[0] + Dn[1] * rm[1] + Dn[2] * rm[2];
      const double Dndrm = Dn[0] * drm[0] + Dn[1] * drm[1] + Dn[2] * drm[2];
      // viscous tangent: mu (delta_ig Dn . Db + Dn_g Db_i) for a velocity column
      const double DnDb = Dn[0] * Db[0] + Dn[1] * Db[1] + Dn[2] * Db[2];
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        double vis = 0.0;
        if (fg < 3) vis = c.mu * ((i == fg ? DnDb : 0.0) + Dn[fg] * Db[i]);
        col[n][i] += detJ * (dWm * rm[i] + Wm * drm[i] + vis);
      }
      col[n][3] += detJ * (Nn * ddiv + irho * (dtm * Dnrm + tm * Dndrm));
      col[n][4] += detJ * (dWt * cT + Wt * dcT + k * (Dn[0] * dGT[0] + Dn[1] * dGT[1] + Dn[2] * dGT[2]));
    }
  }
  const int bx = b & 1, by = (b >> 1) & 1, bz = b >> 2;
#pragma unroll
  for (int n = 0; n < 8; ++n) {
    const int o = (bx - (n & 1) + 1) + 3 * (by - ((n >> 1) & 1) + 1) + 9 * (bz - (n >> 2) + 1);
    const int id = nodes[le][n];
    // a returnless atomic add (no round trip through the registers); within one colour no
    // other thread touches the entry, so the additions keep their launch order
#pragma unroll
    for (int f = 0; f < 5; ++f) unsafeAtomicAdd(A + (size_t)(o * 25 + f * 5 + fg) * N + id, (T)col[n][f]);
  }
}

// Constrained rows become identity rows, constrained columns zero (J~ = [[J_ff, 0], [0, I]])
template <typename T>
__global__ void fix_kernel(Grid g, T* __restrict__ A, long N) {
  const long n = (long)blockIdx.x * BS + threadIdx.x;
  if (n >= N) return;
  int i, j, k;
  node_ijk(g, n, i, j, k);
  bool rowfix[5];
#pragma unroll
  for (int f = 0; f < 5; ++f) rowfix[f] = fixed(g, i, j, k, f);
  for (int o = 0; o < 27; ++o) {
    int m;
    if (!neighbour(g, i, j, k, o, m)) continue;
    int mi, mj, mk;
    node_ijk(g, m, mi, mj, mk);
#pragma unroll
    for (int gg = 0; gg < 5; ++gg) {
      const bool colfix = fixed(g, mi, mj, mk, gg);
#pragma unroll
      for (int f = 0; f < 5; ++f) {
        if (rowfix[f]) A[(size_t)(o * 25 + f * 5 + gg) * N + n] = (T)((o == 13 && f == gg) ? 1.0 : 0.0);
        else if (colfix) A[(size_t)(o * 25 + f * 5 + gg) * N + n] = (T)0.0;
      }
    }
  }
}

// y = A x, y = b - A x, or one damped block-Jacobi sweep y = x + omega D^-1 (b - A x)
// (A^T and D^-T when TR); x, b, y node-interleaved [N][5].
template <typename TM, typename T, bool TR, int MODE>
__global__ __launch_bounds__(BS) void bsr_kernel(Grid g, const TM* __restrict__ A, const TM* __restrict__ Dinv,
                                                 const T* __restrict__ x, const T* __restrict__ b, T* __restrict__ y,
                                                 T omega, long N) {
  const long n = (long)blockIdx.x * BS + threadIdx.x;
  if (n >= N) return;
  int i, j, k;
  node_ijk(g, n, i, j, k);
  T acc[5] = {0, 0, 0, 0, 0};
#pragma unroll
  for (int o = 0; o < 27; ++o) {
    int m;
    if (!neighbour(g, i, j, k, o, m)) continue;
    T xm[5];
#pragma unroll
    for (int f = 0; f < 5; ++f) xm[f] = x[5 * (long)m + f];
    if (!TR) {
#pragma unroll
      for (int f = 0; f < 5; ++f)
#pragma unroll
        for (int gg = 0; gg < 5; ++gg) acc[f] += (T)A[(size_t)(o * 25 + f * 5 + gg) * N + n] * xm[gg];
    } else {
#pragma unroll
      for (int f = 0; f < 5; ++f)
#pragma unroll
        for (int gg = 0; gg < 5; ++gg) acc[gg] += (T)A[(size_t)((26 - o) * 25 + f * 5 + gg) * N + m] * xm[f];
    }
  }
  if (MODE == 0) {
#pragma unroll
    for (int f = 0; f < 5; ++f) y[5 * n + f] = acc[f];
    return;
  }
  T r[5];
#pragma unroll
  for (int f = 0; f < 5; ++f) r[f] = b[5 * n + f] - acc[f];
  if (MODE == 1) {
#pragma unroll
    for (int f = 0; f < 5; ++f) y[5 * n + f] = r[f];
    return;
  }
#pragma unroll
  for (int f = 0; f < 5; ++f) {
    T z = 0;
#pragma unroll
    for (int gg = 0; gg < 5; ++gg) z += (T)(TR ? Dinv[(size_t)(gg * 5 + f) * N + n] : Dinv[(size_t)(f * 5 + gg) * N + n]) * r[gg];
    y[5 * n + f] = x[5 * n + f] + omega * z;
  }
}

// constrained dofs of a five-field array set to 0
__global__ void mask_kernel(Grid g, double* __restrict__ s) {
  const long n = (long)blockIdx.x * BS + threadIdx.x;
  if (n >= g.nodes()) return;
  int i, j, k;
  node_ijk(g, n, i, j, k);
#pragma unroll
  for (int f = 0; f < 5; ++f)
    if (fixed(g, i, j, k, f)) s[5 * n + f] = 0.0;
}

// out[n][f] = sc.s[f] in[n][f], converting precision
template <typename Ta, typename Tb>
__global__ void scale_fields_kernel(const Ta* __restrict__ in, Tb* __restrict__ out, Field5 sc, long N) {
  const long t = (long)blockIdx.x * BS + threadIdx.x;
  if (t >= 5 * N) return;
  out[t] = (Tb)(sc.s[t % 5] * (double)in[t]);
}

// diagonal entries of A into d [N][5] (0 on constrained dofs)
template <typename TM>
__global__ void diagonal_kernel(Grid g, const TM* __restrict__ A, double* __restrict__ d, long N) {
  const long n = (long)blockIdx.x * BS + threadIdx.x;
  if (n >= N) return;
  int i, j, k;
  node_ijk(g, n, i, j, k);
#pragma unroll
  for (int f = 0; f < 5; ++f) d[5 * n + f] = fixed(g, i, j, k, f) ? 0.0 : (double)A[(size_t)(13 * 25 + f * 6) * N + n];
}

// x = omega D^-1 b (D^-T): the first sweep from a zero guess
template <typename T, bool TR>
__global__ void diag_scale_kernel(const T* __restrict__ Dinv, const T* __restrict__ b, T* __restrict__ x, T omega, long N) {
  const long n = (long)blockIdx.x * BS + threadIdx.x;
  if (n >= N) return;
  T r[5];
#pragma unroll
  for (int f = 0; f < 5; ++f) r[f] = b[5 * n + f];
#pragma unroll
  for (int f = 0; f < 5; ++f) {
    T z = 0;
#pragma unroll
    for (int gg = 0; gg < 5; ++gg) z += (TR ? Dinv[(size_t)(gg * 5 + f) * N + n] : Dinv[(size_t)(f * 5 + gg) * N + n]) * r[gg];
    x[5 * n + f] = omega * z;
  }
}

// Inverse of each node's 5 x 5 diagonal block (Gauss-Jordan, partial pivoting, float64)
template <typename T>
__global__ void diag_inverse_kernel(const T* __restrict__ A, T* __restrict__ Dinv, long N) {
  const long n = (long)blockIdx.x * BS + threadIdx.x;
  if (n >= N) return;
  double M[5][10];
#pragma unroll
  for (int f = 0; f < 5; ++f)
#pragma unroll
    for (int gg = 0; gg < 5; ++gg) {
      M[f][gg] = (double)A[(size_t)(13 * 25 + f * 5 + gg) * N + n];
      M[f][5 + gg] = f == gg ? 1.0 : 0.0;
    }
#pragma unroll
  for (int c = 0; c < 5; ++c) {
    int p = c;
    double best = fabs(M[c][c]);
#pragma unroll
    for (int r = c + 1; r < 5; ++r)
      if (fabs(M[r][c]) > best) { best = fabs(M[r][c]); p = r; }
#pragma unroll
    for (int r = 0; r < 5; ++r)
      if (r == p && p != c)
#pragma unroll
        for (int q = 0; q < 10; ++q) { const double t = M[c][q]; M[c][q] = M[r][q]; M[r][q] = t; }
    const double inv = 1.0 / M[c][c];
#pragma unroll
    for (int q = 0; q < 10; ++q) M[c][q] *= inv;
#pragma unroll
    for (int r = 0; r < 5; ++r) {
      if (r == c) continue;
      const double fct = M[r][c];
#pragma unroll
      for (int q = 0; q < 10; ++q) M[r][q] -= fct * M[c][q];
    }
  }
#pragma unroll
  for (int f = 0; f < 5; ++f)
#pragma unroll
    for (int gg = 0; gg < 5; ++gg) Dinv[(size_t)(f * 5 + gg) * N + n] = (T)M[f][5 + gg];
}

// bc = P^T rf on the free dofs of both grids (trilinear weights)
template <typename T>
__global__ void restrict_kernel(Grid gf, Grid gc, const T* __restrict__ rf, T* __restrict__ bc) {
  const long n = (long)blockIdx.x * BS + threadIdx.x;
  if (n >= gc.nodes()) return;
  int I, J, K;
  node_ijk(gc, n, I, J, K);
  double acc[5] = {0, 0, 0, 0, 0};
  for (int dk = -1; dk <= 1; ++dk)
    for (int dj = -1; dj <= 1; ++dj)
      for (int di = -1; di <= 1; ++di) {
        const int i = 2 * I + di, j = 2 * J + dj, k = 2 * K + dk;
        if (i < 0 || i > gf.nx || j < 0 || j > gf.ny || k < 0 || k > gf.nz) continue;
        const double w = (di ? 0.5 : 1.0) * (dj ? 0.5 : 1.0) * (dk ? 0.5 : 1.0);
        const long m = gf.node(i, j, k);
#pragma unroll
        for (int f = 0; f < 5; ++f)
          if (!fixed(gf, i, j, k, f)) acc[f] += w * (double)rf[5 * m + f];
      }
#pragma unroll
  for (int f = 0; f < 5; ++f) bc[5 * n + f] = fixed(gc, I, J, K, f) ? (T)0 : (T)acc[f];
}

// xf += P xc on the free dofs of the fine grid
template <typename T>
__global__ void prolong_kernel(Grid gf, Grid gc, const T* __restrict__ xc, T* __restrict__ xf) {
  const long n = (long)blockIdx.x * BS + threadIdx.x;
  if (n >= gf.nodes()) return;
  int i, j, k;
  node_ijk(gf, n, i, j, k);
  const int I0 = i >> 1, I1 = (i + 1) >> 1, J0 = j >> 1, J1 = (j + 1) >> 1, K0 = k >> 1, K1 = (k + 1) >> 1;
  double acc[5] = {0, 0, 0, 0, 0};
  for (int c = 0; c < 8; ++c) {
    const int I = (c & 1) ? I1 : I0, J = (c & 2) ? J1 : J0, K = (c & 4) ? K1 : K0;
    const long m = gc.node(I, J, K);
#pragma unroll
    for (int f = 0; f < 5; ++f) acc[f] += 0.125 * (double)xc[5 * m + f];
  }
#pragma unroll
  for (int f = 0; f < 5; ++f)
    if (!fixed(gf, i, j, k, f)) xf[5 * n + f] += (T)acc[f];
}

__global__ void inject_kernel(Grid gf, Grid gc, const double* __restrict__ sf, double* __restrict__ sc) {
  const long n = (long)blockIdx.x * BS + threadIdx.x;
  if (n >= gc.nodes()) return;
  int I, J, K;
  node_ijk(gc, n, I, J, K);
  const long m = gf.node(2 * I, 2 * J, 2 * K);
#pragma unroll
  for (int f = 0; f < 5; ++f) sc[5 * n + f] = sf[5 * m + f];
}

// dense row-major copy of the node-block matrix (D zeroed beforehand)
template <typename T>
__global__ void dense_kernel(Grid g, const T* __restrict__ A, double* __restrict__ D, long N) {
  const long t = (long)blockIdx.x * BS + threadIdx.x;
  if (t >= N * 27) return;
  const long n = t % N;
  const int o = (int)(t / N);
  int i, j, k, m;
  node_ijk(g, n, i, j, k);
  if (!neighbour(g, i, j, k, o, m)) return;
  const long nd = 5 * N;
  for (int f = 0; f < 5; ++f)
    for (int gg = 0; gg < 5; ++gg) D[(5 * n + f) * nd + 5 * (long)m + gg] = (double)A[(size_t)(o * 25 + f * 5 + gg) * N + n];
}

// coef[e][1] = a(gamma_e) = abar q gamma / (1 + q - gamma) (the solid's impermeability abar
// interpolated with penalty q), da[e] = abar q (1 + q) / (1 + q - gamma)^2
__global__ void brinkman_kernel(long E, double abar, double q, const double* __restrict__ gamma,
                                double* __restrict__ coef, double* __restrict__ da) {
  const long e = (long)blockIdx.x * BS + threadIdx.x;
  if (e >= E) return;
  const double g = gamma[e], den = 1.0 + q - g;
  coef[2 * e + 1] = abar * q * g / den;
  da[e] = abar * q * (1.0 + q) / (den * den);
}

__device__ inline double block_sum(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < BS / 64; ++w) t += red[w];
  return t;
}

// per-block partial sums of the compliance: patch flux times T plus the volumetric load
__global__ __launch_bounds__(BS) void objective_kernel(Grid g, NsConst c, Patch patch, const double* __restrict__ s,
                                                       double* __restrict__ part) {
  __shared__ double red[BS / 64];
  double acc = 0.0;
  for (long e = (long)blockIdx.x * BS + threadIdx.x; e < g.elems(); e += (long)gridDim.x * BS) {
    const int i = (int)(e % g.nx), j = (int)((e / g.nx) % g.ny), k = (int)(e / ((long)g.nx * g.ny));
    const double Q = c.source(i, j, k);
    if (Q != 0.0) {
      int nid[8];
      elem_nodes(g, i, j, k, nid);
      double u0[3] = {0, 0, 0};
      for (int n = 0; n < 8; ++n)
        for (int d = 0; d < 3; ++d) u0[d] += 0.125 * s[5 * (long)nid[n] + d];
      for (int n = 0; n < 8; ++n) acc += Q * load_weight<double>(c, u0, n) * s[5 * (long)nid[n] + 4];
    }
    if (k == 0 && patch.has(i, j)) {
      const double w = 0.25 * patch.q_h * patch.h * patch.h;
      for (int n = 0; n < 4; ++n) acc += w * s[5 * (long)g.node(i + (n & 1), j + (n >> 1), 0) + 4];
    }
  }
  const double t = block_sum(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

__global__ __launch_bounds__(BS) void sum_kernel(const double* __restrict__ part, int n, double* __restrict__ out) {
  __shared__ double red[BS / 64];
  double acc = 0.0;
  for (int t = threadIdx.x; t < n; t += BS) acc += part[t];
  const double t = block_sum(acc, red);
  if (threadIdx.x == 0) out[0] = t;
}

// d f / d s per node: the patch load on T, and the volumetric load's derivative through T
// and (via the weight's centroid velocity) u, v, w; constrained dofs zero
__global__ void objective_grad_kernel(Grid g, NsConst c, Patch patch, const double* __restrict__ s,
                                      double* __restrict__ g5) {
  const long n = (long)blockIdx.x * BS + threadIdx.x;
  if (n >= g.nodes()) return;
  int i, j, k;
  node_ijk(g, n, i, j, k);
  double out[5] = {0, 0, 0, 0, 0};
  if (k == 0)
    for (int dj = -1; dj <= 0; ++dj)
      for (int di = -1; di <= 0; ++di) {
        const int fi = i + di, fj = j + dj;
        if (fi >= 0 && fi < g.nx && fj >= 0 && fj < g.ny && patch.has(fi, fj)) out[4] += 0.25 * patch.q_h * patch.h * patch.h;
      }
  for (int ce = 0; ce < 8; ++ce) {
    const int ie = i - 1 + (ce & 1), je = j - 1 + ((ce >> 1) & 1), ke = k - 1 + (ce >> 2);
    if (ie < 0 || ie >= g.nx || je < 0 || je >= g.ny || ke < 0 || ke >= g.nz) continue;
    const double Q = c.source(ie, je, ke);
    if (Q == 0.0) continue;
    const int ln = (i - ie) + 2 * (j - je) + 4 * (k - ke);
    int nid[8];
    elem_nodes(g, ie, je, ke, nid);
    double u0[3] = {0, 0, 0};
    for (int a = 0; a < 8; ++a)
      for (int d = 0; d < 3; ++d) u0[d] += 0.125 * s[5 * (long)nid[a] + d];
    out[4] += Q * load_weight<double>(c, u0, ln);
    for (int d = 0; d < 3; ++d) {
      Dual ud[3];
      for (int q = 0; q < 3; ++q) ud[q] = Dual{u0[q], q == d ? 0.125 : 0.0};
      double acc = 0.0;
      for (int a = 0; a < 8; ++a) acc += load_weight<Dual>(c, ud, a).d * s[5 * (long)nid[a] + 4];
      out[d] += Q * acc;
    }
  }
#pragma unroll
  for (int f = 0; f < 5; ++f) g5[5 * n + f] = fixed(g, i, j, k, f) ? 0.0 : out[f];
}

// out[e] = -lambda_e^T d R_e / d gamma_e through k and the Brinkman coefficient a
__global__ __launch_bounds__(BS) void sensitivity_kernel(Grid g, NsConst c, const double* __restrict__ coef,
                                                         const double* __restrict__ dk, const double* __restrict__ da,
                                                         const double* __restrict__ s, const double* __restrict__ lam,
                                                         double* __restrict__ out) {
  const long e = (long)blockIdx.x * BS + threadIdx.x;
  if (e >= g.elems()) return;
  const int i = (int)(e % g.nx), j = (int)((e / g.nx) % g.ny), k = (int)(e / ((long)g.nx * g.ny));
  int nid[8];
  elem_nodes(g, i, j, k, nid);
  double l[8][5];
#pragma unroll
  for (int n = 0; n < 8; ++n) {
    const int ni = i + (n & 1), nj = j + ((n >> 1) & 1), nk = k + (n >> 2);
#pragma unroll
    for (int f = 0; f < 5; ++f) l[n][f] = fixed(g, ni, nj, nk, f) ? 0.0 : lam[5 * (long)nid[n] + f];
  }
  double acc = 0.0;
  auto in = [&](int n, int f) { return Dual{s[5 * (long)nid[n] + f], 0.0}; };
  auto outf = [&](int n, int f, Dual v) { acc += l[n][f] * v.d; };
  element_rows<Dual>(c, Dual{coef[2 * e], dk[e]}, Dual{coef[2 * e + 1], da[e]}, c.source(i, j, k), in, outf);
  out[e] = -acc;
}

}  // namespace

ColourGrid colour_grid(const Grid& g, int col) {
  ColourGrid cg;
  cg.cx = col & 1;
  cg.cy = (col >> 1) & 1;
  cg.cz = col >> 2;
  cg.mx = (g.nx - cg.cx + 1) / 2;
  cg.my = (g.ny - cg.cy + 1) / 2;
  cg.mz = (g.nz - cg.cz + 1) / 2;
  cg.count = (long)cg.mx * cg.my * cg.mz;
  return cg;
}

template <typename T>
void launch_fill(hipStream_t st, T* a, long n, T v) {
  launch(fill_kernel<T>, dim3(std::min(blocks(n), 8192)), dim3(BS), 0, st, a, n, v);
}

void launch_residual(hipStream_t st, const Grid& g, const NsConst& c, const Patch& patch, const double* coef,
                     const double* s, double* r) {
  launch_fill<double>(st, r, 5 * g.nodes(), 0.0);
  for (int col = 0; col < 8; ++col) {
    const ColourGrid cg = colour_grid(g, col);
    if (cg.count > 0) launch(residual_kernel, dim3(blocks(cg.count)), dim3(BS), 0, st, g, c, cg, coef, s, r);
  }
  launch(residual_finish_kernel, dim3(blocks(g.nodes())), dim3(BS), 0, st, g, patch, s, r);
}

template <typename T>
void launch_assemble(hipStream_t st, const Grid& g, const NsConst& c, const double* coef, const double* s, T* A) {
  const long N = g.nodes();
  launch_fill<T>(st, A, (long)NS_ENTRIES * N, (T)0);
  for (int col = 0; col < 8; ++col) {
    const ColourGrid cg = colour_grid(g, col);
    if (cg.count > 0)
      launch(assemble_shared_kernel<T>, dim3((unsigned)((cg.count + AS_E - 1) / AS_E)), dim3(5 * 64), 0, st, g, c, cg,
             coef, s, A, N);
  }
  launch(fix_kernel<T>, dim3(blocks(N)), dim3(BS), 0, st, g, A, N);
}

template <typename TM, typename T>
void launch_bsr(hipStream_t st, const Grid& g, const TM* A, const TM* Dinv, bool tr, int mode, const T* x, const T* b,
                T* y, T omega) {
  const long N = g.nodes();
  const dim3 gr(blocks(N));
#define NS_BSR(TRV, M) launch(bsr_kernel<TM, T, TRV, M>, gr, dim3(BS), 0, st, g, A, Dinv, x, b, y, omega, N)
  if (!tr) {
    if (mode == 0) NS_BSR(false, 0);
    else if (mode == 1) NS_BSR(false, 1);
    else NS_BSR(false, 2);
  } else {
    if (mode == 0) NS_BSR(true, 0);
    else if (mode == 1) NS_BSR(true, 1);
    else NS_BSR(true, 2);
  }
#undef NS_BSR
}

template <typename T>
void launch_diag_scale(hipStream_t st, const Grid& g, const T* Dinv, bool tr, T omega, const T* b, T* x) {
  const long N = g.nodes();
  if (tr) launch(diag_scale_kernel<T, true>, dim3(blocks(N)), dim3(BS), 0, st, Dinv, b, x, omega, N);
  else launch(diag_scale_kernel<T, false>, dim3(blocks(N)), dim3(BS), 0, st, Dinv, b, x, omega, N);
}

template <typename T>
void launch_diag_inverse(hipStream_t st, const Grid& g, const T* A, T* Dinv) {
  launch(diag_inverse_kernel<T>, dim3(blocks(g.nodes())), dim3(BS), 0, st, A, Dinv, g.nodes());
}

template <typename T>
void launch_restrict(hipStream_t st, const Grid& gf, const Grid& gc, const T* rf, T* bc) {
  launch(restrict_kernel<T>, dim3(blocks(gc.nodes())), dim3(BS), 0, st, gf, gc, rf, bc);
}

template <typename T>
void launch_prolong_add(hipStream_t st, const Grid& gf, const Grid& gc, const T* xc, T* xf) {
  launch(prolong_kernel<T>, dim3(blocks(gf.nodes())), dim3(BS), 0, st, gf, gc, xc, xf);
}

void launch_mask(hipStream_t st, const Grid& g, double* s) {
  launch(mask_kernel, dim3(blocks(g.nodes())), dim3(BS), 0, st, g, s);
}

template <typename Ta, typename Tb>
void launch_scale_fields(hipStream_t st, long N, const Ta* in, Tb* out, const Field5& sc) {
  launch(scale_fields_kernel<Ta, Tb>, dim3(blocks(5 * N)), dim3(BS), 0, st, in, out, sc, N);
}
template void launch_scale_fields<double, double>(hipStream_t, long, const double*, double*, const Field5&);
template void launch_scale_fields<double, float>(hipStream_t, long, const double*, float*, const Field5&);

template <typename TM>
void launch_diagonal(hipStream_t st, const Grid& g, const TM* A, double* d) {
  launch(diagonal_kernel<TM>, dim3(blocks(g.nodes())), dim3(BS), 0, st, g, A, d, g.nodes());
}
template void launch_diagonal<double>(hipStream_t, const Grid&, const double*, double*);
template void launch_diagonal<float>(hipStream_t, const Grid&, const float*, double*);

void launch_inject(hipStream_t st, const Grid& gf, const Grid& gc, const double* sf, double* sc) {
  launch(inject_kernel, dim3(blocks(gc.nodes())), dim3(BS), 0, st, gf, gc, sf, sc);
}

template <typename T>
void launch_dense(hipStream_t st, const Grid& g, const T* A, double* D) {
  const long N = g.nodes();
  launch_fill<double>(st, D, 25 * N * N, 0.0);
  launch(dense_kernel<T>, dim3(blocks(27 * N)), dim3(BS), 0, st, g, A, D, N);
}

void launch_brinkman(hipStream_t st, long E, double abar, double q, const double* gamma, double* coef, double* da) {
  launch(brinkman_kernel, dim3(blocks(E)), dim3(BS), 0, st, E, abar, q, gamma, coef, da);
}

void launch_objective(hipStream_t st, const Grid& g, const NsConst& c, const Patch& patch, const double* s, double* part,
                      double* out) {
  constexpr int NB = 1024;
  launch(objective_kernel, dim3(NB), dim3(BS), 0, st, g, c, patch, s, part);
  launch(sum_kernel, dim3(1), dim3(BS), 0, st, (const double*)part, NB, out);
}

void launch_objective_grad(hipStream_t st, const Grid& g, const NsConst& c, const Patch& patch, const double* s,
                           double* g5) {
  launch(objective_grad_kernel, dim3(blocks(g.nodes())), dim3(BS), 0, st, g, c, patch, s, g5);
}

void launch_sensitivity(hipStream_t st, const Grid& g, const NsConst& c, const double* coef, const double* dk,
                        const double* da, const double* s, const double* lam, double* out) {
  launch(sensitivity_kernel, dim3(blocks(g.elems())), dim3(BS), 0, st, g, c, coef, dk, da, s, lam, out);
}

#define NS_INST(T)                                                                                                    \
  template void launch_fill<T>(hipStream_t, T*, long, T);                                                              \
  template void launch_assemble<T>(hipStream_t, const Grid&, const NsConst&, const double*, const double*, T*);        \
  template void launch_bsr<T, T>(hipStream_t, const Grid&, const T*, const T*, bool, int, const T*, const T*, T*, T);  \
  template void launch_diag_scale<T>(hipStream_t, const Grid&, const T*, bool, T, const T*, T*);                       \
  template void launch_diag_inverse<T>(hipStream_t, const Grid&, const T*, T*);                                        \
  template void launch_restrict<T>(hipStream_t, const Grid&, const Grid&, const T*, T*);                               \
  template void launch_prolong_add<T>(hipStream_t, const Grid&, const Grid&, const T*, T*);                            \
  template void launch_dense<T>(hipStream_t, const Grid&, const T*, double*);
NS_INST(float)
NS_INST(double)
#undef NS_INST


}  // namespace ns
}  // namespace nc
