// Host build of the library's element header (paper_1904_00182_amd/csrc/element.hpp),
// used only by the CPU test-suite to check the element math against the oracle before
// any GPU run.  Element loops and the node-level finishing (lumped mass, boundary flux,
// constraints) are written out plainly here; the GPU kernels implement the same
// finishing independently.
#include <cmath>
#include <cstring>
#include <vector>
#include "../../paper_1904_00182_amd/csrc/element.hpp"

using namespace nc;

static int g_variant = 0;   // 0: Gauss-point element functions, 1: modal element functions

namespace {
struct Grid {
  int nx, ny, nz;
  double h, q_h, px0, px1, py0, py1;
  ElemConst<double> c;
  long node(int i, int j, int k) const { return i + (long)(nx + 1) * (j + (long)(ny + 1) * k); }
  bool tfix(int i, int j, int k) const { return i == 0 || i == nx || j == 0 || j == ny || k == nz; }
  bool pfix(int i, int j, int k) const { return i == 0 && j == 0 && k == nz; }
  double mass(int i, int j, int k) const {
    int m = (1 + (i > 0 && i < nx)) * (1 + (j > 0 && j < ny)) * (1 + (k > 0 && k < nz));
    return c.W * m;
  }
};

Grid make(const int* dims, const double* prm) {
  Grid g;
  g.nx = dims[0]; g.ny = dims[1]; g.nz = dims[2];
  g.h = prm[0];
  g.c = make_elem_const<double>(prm[0], prm[1], prm[2], prm[3], prm[4], prm[5], prm[6]);
  g.q_h = prm[7]; g.px0 = prm[8]; g.px1 = prm[9]; g.py0 = prm[10]; g.py1 = prm[11];
  return g;
}

template <class F>
void for_elems(const Grid& g, F f) {
  for (int k = 0; k < g.nz; ++k)
    for (int j = 0; j < g.ny; ++j)
      for (int i = 0; i < g.nx; ++i) {
        long n[8];
        for (int a = 0; a < 8; ++a) n[a] = g.node(i + (a & 1), j + ((a >> 1) & 1), k + ((a >> 2) & 1));
        f(i, j, k, i + (long)g.nx * (j + (long)g.ny * k), n);
      }
}
}  // namespace

extern "C" {

void hc_set_variant(int v) { g_variant = v; }

int hc_residual(const int* dims, const double* prm, const double* kk, const double* kap, const double* s, double* r) {
  Grid g = make(dims, prm);
  long N = (long)(g.nx + 1) * (g.ny + 1) * (g.nz + 1);
  std::memset(r, 0, sizeof(double) * 5 * N);
  for_elems(g, [&](int i, int j, int k, long e, const long* n) {
    double P[8], T[8], rP[8] = {0}, rT[8] = {0}, rU[3][8] = {{0}};
    for (int a = 0; a < 8; ++a) { P[a] = s[5 * n[a] + 3]; T[a] = s[5 * n[a] + 4]; }
    if (g_variant == 0) {
      Lin<double> L;
      linearize(P, T, kk[e], kap[e], g.c, L);
      elem_residual<double, true>(L, g.c, rP, rT, rU);
    } else {
      LinM<double> L;
      lin_modal(P, T, kk[e], kap[e], g.c, L);
      elem_residual_m<double, true>(L, g.c, rP, rT, rU);
    }
    if (k == 0) {
      double xc = (i + 0.5) * g.h, yc = (j + 0.5) * g.h;
      if (xc >= g.px0 && xc <= g.px1 && yc >= g.py0 && yc <= g.py1)
        for (int a = 0; a < 4; ++a) rT[a] -= g.q_h * g.h * g.h / 4.0;
    }
    for (int a = 0; a < 8; ++a) {
      for (int d = 0; d < 3; ++d) r[5 * n[a] + d] += rU[d][a];
      r[5 * n[a] + 3] += rP[a];
      r[5 * n[a] + 4] += rT[a];
    }
  });
  for (int k = 0; k <= g.nz; ++k)
    for (int j = 0; j <= g.ny; ++j)
      for (int i = 0; i <= g.nx; ++i) {
        long n = g.node(i, j, k);
        for (int d = 0; d < 3; ++d) r[5 * n + d] += g.mass(i, j, k) * s[5 * n + d];
        if (g.tfix(i, j, k)) r[5 * n + 4] = s[5 * n + 4];
        if (g.pfix(i, j, k)) r[5 * n + 3] = s[5 * n + 3];
      }
  return 0;
}

static void masked_copy(const Grid& g, const double* v, std::vector<double>& vm) {
  long N = (long)(g.nx + 1) * (g.ny + 1) * (g.nz + 1);
  vm.assign(v, v + 5 * N);
  for (int k = 0; k <= g.nz; ++k)
    for (int j = 0; j <= g.ny; ++j)
      for (int i = 0; i <= g.nx; ++i) {
        long n = g.node(i, j, k);
        if (g.tfix(i, j, k)) vm[5 * n + 4] = 0;
        if (g.pfix(i, j, k)) vm[5 * n + 3] = 0;
      }
}

static void finish(const Grid& g, const double* v, double* y) {
  for (int k = 0; k <= g.nz; ++k)
    for (int j = 0; j <= g.ny; ++j)
      for (int i = 0; i <= g.nx; ++i) {
        long n = g.node(i, j, k);
        for (int d = 0; d < 3; ++d) y[5 * n + d] += g.mass(i, j, k) * v[5 * n + d];
        if (g.tfix(i, j, k)) y[5 * n + 4] = v[5 * n + 4];
        if (g.pfix(i, j, k)) y[5 * n + 3] = v[5 * n + 3];
      }
}

int hc_jv(const int* dims, const double* prm, const double* kk, const double* kap, const double* s, const double* v, double* y) {
  Grid g = make(dims, prm);
  long N = (long)(g.nx + 1) * (g.ny + 1) * (g.nz + 1);
  std::vector<double> vm;
  masked_copy(g, v, vm);
  std::memset(y, 0, sizeof(double) * 5 * N);
  for_elems(g, [&](int, int, int, long e, const long* n) {
    double P[8], T[8], p[8], t[8], yP[8] = {0}, yT[8] = {0}, yU[3][8] = {{0}};
    for (int a = 0; a < 8; ++a) {
      P[a] = s[5 * n[a] + 3]; T[a] = s[5 * n[a] + 4];
      p[a] = vm[5 * n[a] + 3]; t[a] = vm[5 * n[a] + 4];
    }
    if (g_variant == 0) {
      Lin<double> L;
      linearize(P, T, kk[e], kap[e], g.c, L);
      elem_jv<double, true>(L, p, t, g.c, yP, yT, yU);
    } else {
      LinM<double> L;
      lin_modal(P, T, kk[e], kap[e], g.c, L);
      elem_jv_m<double, true>(L, p, t, g.c, yP, yT, yU);
    }
    for (int a = 0; a < 8; ++a) {
      for (int d = 0; d < 3; ++d) y[5 * n[a] + d] += yU[d][a];
      y[5 * n[a] + 3] += yP[a];
      y[5 * n[a] + 4] += yT[a];
    }
  });
  finish(g, v, y);
  return 0;
}

int hc_jtw(const int* dims, const double* prm, const double* kk, const double* kap, const double* s, const double* w, double* y) {
  Grid g = make(dims, prm);
  long N = (long)(g.nx + 1) * (g.ny + 1) * (g.nz + 1);
  std::vector<double> wm;
  masked_copy(g, w, wm);
  std::memset(y, 0, sizeof(double) * 5 * N);
  for_elems(g, [&](int, int, int, long e, const long* n) {
    double P[8], T[8], wP[8], wT[8], wU[3][8], yP[8] = {0}, yT[8] = {0};
    for (int a = 0; a < 8; ++a) {
      P[a] = s[5 * n[a] + 3]; T[a] = s[5 * n[a] + 4];
      wP[a] = wm[5 * n[a] + 3]; wT[a] = wm[5 * n[a] + 4];
      for (int d = 0; d < 3; ++d) wU[d][a] = wm[5 * n[a] + d];
    }
    if (g_variant == 0) {
      Lin<double> L;
      linearize(P, T, kk[e], kap[e], g.c, L);
      elem_jtw<double, true>(L, wP, wT, wU, g.c, yP, yT);
    } else {
      LinM<double> L;
      lin_modal(P, T, kk[e], kap[e], g.c, L);
      elem_jtw_m<double, true>(L, wP, wT, wU, g.c, yP, yT);
    }
    for (int a = 0; a < 8; ++a) {
      y[5 * n[a] + 3] += yP[a];
      y[5 * n[a] + 4] += yT[a];
    }
  });
  finish(g, w, y);
  return 0;
}

int hc_sens(const int* dims, const double* prm, const double* kk, const double* kap, const double* dk,
            const double* dkap, const double* s, const double* lam, double* out) {
  Grid g = make(dims, prm);
  std::vector<double> lm;
  masked_copy(g, lam, lm);
  for_elems(g, [&](int, int, int, long e, const long* n) {
    double P[8], T[8], lP[8], lT[8], lU[3][8];
    for (int a = 0; a < 8; ++a) {
      P[a] = s[5 * n[a] + 3]; T[a] = s[5 * n[a] + 4];
      lP[a] = lm[5 * n[a] + 3]; lT[a] = lm[5 * n[a] + 4];
      for (int d = 0; d < 3; ++d) lU[d][a] = lm[5 * n[a] + d];
    }
    Lin<double> L;
    linearize(P, T, kk[e], kap[e], g.c, L);
    out[e] = elem_sensitivity<double, true>(L, lP, lT, lU, dk[e], dkap[e], g.c);
  });
  return 0;
}
}
