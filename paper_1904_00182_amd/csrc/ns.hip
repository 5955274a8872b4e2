// Solver runtime of the Navier-Stokes / Brinkman flow model (the full-flow model of the
// hybrid strategy, Sec. 6.4) behind the nc_ns_* entry points of include/nc.h: context and
// workspace carving, the design chain, the assembled Jacobian hierarchy, flexible GMRES
// with a geometric-multigrid preconditioner (damped node-block Jacobi smoothing,
// rediscretised coarse levels at the injected state), damped Newton (Sec. 5.4), the
// adjoint solve and the sensitivities (Sec. 5.1).
//
// Precision: the Newton residual, the Krylov vectors and the operator of the Krylov
// solves are float64 (the level-0 Jacobian is assembled in float64); with NC_MIXED the
// multigrid hierarchy -- the smoother's matrices and node-block inverses, transfers and
// V-cycle vectors -- is float32.  The Krylov solve then converges to the requested float64
// residual, and the preconditioner's precision only changes the iteration count.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "kernels.hpp"
#include "ns_kernels.hpp"
#include "../../include/nc.h"

using namespace nc;
using namespace nc::ns;

namespace {

constexpr int NS_MAXLEV = 10;
constexpr size_t NS_ALIGN = 256;
constexpr int COARSE_SWEEPS = 20;   // coarsest level without a dense inverse

struct NsError {
  hipError_t e;
};
inline void ck(hipError_t e) {
  if (e != hipSuccess) throw NsError{e};
}

struct NsLevel {
  Grid g;
  double h;
  NsConst c;
  double* coef;   // [E][2]: conductivity k, Brinkman coefficient a (float64)
  double* st;     // [N][5] linearisation state (levels >= 1; level 0 uses the caller's s)
  void* A;        // [NS_ENTRIES][N] node-block Jacobian in the working precision
  void* Dinv;     // [25][N] inverse node blocks
  void *x, *x2, *b, *r;   // [N][5] V-cycle vectors
};

struct Carver {
  char* base;
  size_t off = 0;
  template <typename T>
  T* take(size_t count) {
    off = (off + NS_ALIGN - 1) / NS_ALIGN * NS_ALIGN;
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

double now() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

}  // namespace

struct nc_ns_ctx {
  nc_problem p;
  hipStream_t stream;
  char* ws_base;         // the caller's workspace (aligned) and the bytes the layout uses
  size_t ws_need;
  bool mixed;
  int L;
  NsLevel lev[NS_MAXLEV];
  double* A64;           // level-0 Jacobian in float64 (the same buffer as lev[0].A in NC_FP64)
  long N, E, n5, ld;
  int m;
  Patch patch;
  Regions reg;
  bool regions;
  long n_design;
  bool pde;
  HelmholtzPlan helm;
  double* helm_work;
  double *gamma, *dk, *da, *ftmp, *sens;
  float* coef32;         // float32 copy the RAMP kernel writes (unused here)
  bool dense;
  int ncoarse;
  double* Ad;            // coarsest inverse and its transpose
  int* perm;
  double* gjwork;
  double *V, *Z;         // Krylov basis and preconditioned vectors, float64
  double *part, *dres;
  double* hbuf;          // pinned host mirror of dres
  double *R, *d, *strial, *tmp5, *bs;
  // Krylov solves run on the row-equilibrated system S^-1 J~ (S^-1 J~^T) with S the root
  // mean square of each field's free diagonal entries (the continuity rows are smaller
  // than the momentum rows by about h^2); the preconditioner sees S v
  Field5 rs, rs_inv;
  long nfree[5];
  double omega;          // block-Jacobi damping in use: smooth_omega, or the fallback after a stall
  bool design_set;
  bool lin_valid;        // Jacobian hierarchy assembled at lin_s
  const double* lin_s;
  double t_setup;
};

namespace {

bool box_on(const double* b) { return b[1] > b[0] && b[3] > b[2] && b[5] > b[4]; }

void box_range(const double* b, const Grid& g, double h, int r[6]) {
  const int n[3] = {g.nx, g.ny, g.nz};
  for (int d = 0; d < 3; ++d) {
    int lo = n[d], hi = -1;
    for (int i = 0; i < n[d]; ++i) {
      const double c = (i + 0.5) * h;
      if (c >= b[2 * d] && c <= b[2 * d + 1]) {
        lo = std::min(lo, i);
        hi = std::max(hi, i);
      }
    }
    r[2 * d] = lo;
    r[2 * d + 1] = hi;
  }
}

bool valid(const nc_problem* p) {
  if (!p || p->nx < 1 || p->ny < 1 || p->nz < 1) return false;
  if ((double)(p->nx + 1) * (p->ny + 1) * (p->nz + 1) * 5 >= 2147483647.0) return false;
  if (p->mu <= 0 || p->rho0 <= 0 || p->kappa_s <= 0 || p->kappa_f <= 0 || p->k_f <= 0 || p->k_s <= 0) return false;
  if (p->precision != NC_FP64 && p->precision != NC_MIXED) return false;
  if (p->krylov_restart < 1 || p->krylov_restart > MAXC - 2) return false;
  if (!(p->krylov_rtol > 0) || !(p->adjoint_rtol > 0)) return false;
  if (!(p->newton_eta0 >= 0.0 && p->newton_eta0 < 1.0)) return false;
  if (p->smooth_pre < 1 || p->smooth_post < 0 || p->smooth_pre_coarse < 1 || p->smooth_post_coarse < 0) return false;
  if (!(p->smooth_omega > 0.0 && p->smooth_omega <= 2.0)) return false;
  if (p->filter_kind != NC_FILTER_CONE && p->filter_kind != NC_FILTER_PDE) return false;
  if ((p->sym_x != 0 && p->sym_x != 1) || (p->sym_y != 0 && p->sym_y != 1)) return false;
  if (!(p->filter_radius >= 0.0)) return false;
  return true;
}

int choose_levels(const nc_problem* p, Grid* gs) {
  gs[0] = Grid{p->nx, p->ny, p->nz, (p->sym_x ? 1 : 0) | (p->sym_y ? 2 : 0)};
  int L = 1;
  const int cap = p->levels > 0 ? std::min(p->levels, NS_MAXLEV) : NS_MAXLEV;
  while (L < cap) {
    const Grid& f = gs[L - 1];
    if ((f.nx & 1) || (f.ny & 1) || (f.nz & 1)) break;
    if (f.nx / 2 < 2 || f.ny / 2 < 2 || f.nz / 2 < 2) break;
    if (p->levels <= 0 && 5 * f.nodes() <= NC_DENSE_MAX) break;
    gs[L] = Grid{f.nx / 2, f.ny / 2, f.nz / 2, f.sym};
    ++L;
  }
  return L;
}

NsConst make_const(const nc_problem& p, double h, const Grid& g) {
  NsConst c;
  c.h = h;
  c.rho = p.rho0;
  c.mu = p.mu;
  c.cp = p.cp;
  c.bz = -p.rho0 * p.alpha * p.g0;
  c.nu2 = (p.mu / p.rho0) * (p.mu / p.rho0);
  c.he2 = 3.0 * h * h;
  c.Q = p.Q;
  c.qi0 = c.qj0 = c.qk0 = 0;
  c.qi1 = g.nx - 1;
  c.qj1 = g.ny - 1;
  c.qk1 = g.nz - 1;
  if (box_on(p.q_box)) {
    int r[6];
    box_range(p.q_box, g, h, r);
    c.qi0 = r[0]; c.qi1 = r[1]; c.qj0 = r[2]; c.qj1 = r[3]; c.qk0 = r[4]; c.qk1 = r[5];
  }
  return c;
}

size_t carve(nc_ns_ctx* c, char* base) {
  Carver cv{base};
  const nc_problem& p = c->p;
  Grid gs[NS_MAXLEV];
  c->L = choose_levels(&p, gs);
  c->mixed = p.precision == NC_MIXED;
  const size_t rs = c->mixed ? sizeof(float) : sizeof(double);
  const double h0 = p.h > 0 ? p.h : 1.0 / p.nx;
  for (int l = 0; l < c->L; ++l) {
    NsLevel& L = c->lev[l];
    L.g = gs[l];
    L.h = h0 * (1 << l);
    L.c = make_const(p, L.h, L.g);
    const long N = L.g.nodes(), E = L.g.elems();
    L.coef = cv.take<double>(2 * E);
    L.st = l > 0 ? cv.take<double>(5 * N) : nullptr;
    L.A = cv.take<char>((size_t)NS_ENTRIES * N * rs);
    L.Dinv = cv.take<char>(25 * N * rs);
    L.x = cv.take<char>(5 * N * rs);
    L.x2 = cv.take<char>(5 * N * rs);
    L.b = cv.take<char>(5 * N * rs);
    L.r = cv.take<char>(5 * N * rs);
  }
  c->N = gs[0].nodes();
  c->E = gs[0].elems();
  c->n5 = 5 * c->N;
  c->A64 = c->mixed ? cv.take<double>((size_t)NS_ENTRIES * c->N) : (double*)c->lev[0].A;
  c->reg = Regions{};
  c->reg.has_s = box_on(p.solid_box) ? 1 : 0;
  c->reg.has_d = box_on(p.design_box) ? 1 : 0;
  if (c->reg.has_s) box_range(p.solid_box, gs[0], h0, c->reg.s);
  if (c->reg.has_d) box_range(p.design_box, gs[0], h0, c->reg.d);
  c->regions = c->reg.has_s || c->reg.has_d;
  c->n_design = 0;
  for (int k = 0; k < gs[0].nz; ++k)
    for (int j = 0; j < gs[0].ny; ++j)
      for (int i = 0; i < gs[0].nx; ++i) c->n_design += c->reg.design(i, j, k) ? 1 : 0;
  c->gamma = cv.take<double>(c->E);
  c->dk = cv.take<double>(c->E);
  c->da = cv.take<double>(c->E);
  c->ftmp = cv.take<double>(c->E);
  c->sens = cv.take<double>(c->E);
  c->coef32 = cv.take<float>(2 * c->E);
  c->pde = p.filter_kind == NC_FILTER_PDE && p.filter_radius > 0.0;
  c->helm_work = cv.take<double>(c->pde ? 4 * c->N : 1);
  if (c->pde) c->helm = helmholtz_plan(h0, p.filter_radius, 1e-15);
  const Grid& gc = c->lev[c->L - 1].g;
  c->ncoarse = (int)(5 * gc.nodes());
  c->dense = c->ncoarse <= NC_DENSE_MAX;
  c->Ad = cv.take<double>(c->dense ? 2 * (size_t)c->ncoarse * c->ncoarse : 1);
  c->perm = cv.take<int>(c->dense ? 2 * c->ncoarse : 1);
  c->gjwork = cv.take<double>(c->dense ? 2 * c->ncoarse : 1);
  c->m = p.krylov_restart;
  c->ld = (c->n5 + 63) / 64 * 64;
  c->V = cv.take<double>((size_t)(c->m + 1) * c->ld);
  c->Z = cv.take<double>((size_t)c->m * c->ld);
  c->part = cv.take<double>((size_t)RED_BLOCKS * MAXC);
  c->dres = cv.take<double>(4 * MAXC);
  c->R = cv.take<double>(c->n5);
  c->d = cv.take<double>(c->n5);
  c->strial = cv.take<double>(c->n5);
  c->tmp5 = cv.take<double>(c->n5);
  c->bs = cv.take<double>(c->n5);
  for (int f = 0; f < 5; ++f) c->nfree[f] = 0;
  const Grid& g0 = gs[0];
  for (int k = 0; k <= g0.nz; ++k)
    for (int j = 0; j <= g0.ny; ++j)
      for (int i = 0; i <= g0.nx; ++i)
        for (int f = 0; f < 5; ++f) c->nfree[f] += fixed(g0, i, j, k, f) ? 0 : 1;
  return cv.off + NS_ALIGN;
}

void sync(nc_ns_ctx* c) { ck(hipStreamSynchronize(c->stream)); }

void fetch(nc_ns_ctx* c, const double* dev, int count) {
  ck(hipMemcpyAsync(c->hbuf, dev, sizeof(double) * count, hipMemcpyDeviceToHost, c->stream));
  sync(c);
}

double norm(nc_ns_ctx* c, const double* a) {
  launch_norm<double>(c->stream, a, c->n5, c->part, c->dres);
  fetch(c, c->dres, 1);
  return c->hbuf[0];
}

// per-field 2-norms of a (out[0..4]) and b (out[5..9])
void field_norms(nc_ns_ctx* c, const double* a, const double* b, double out[10]) {
  launch_field_norms(c->stream, a, b, c->N, c->part, c->dres);
  fetch(c, c->dres, 10);
  for (int f = 0; f < 10; ++f) out[f] = c->hbuf[f];
}

void apply_filter(nc_ns_ctx* c, const double* x, double* y, bool transpose) {
  const Grid& g = c->lev[0].g;
  if (c->pde) launch_pde_filter(c->stream, g, c->helm, x, y, c->helm_work);
  else launch_cone_filter(c->stream, g, c->p.filter_radius, x, y, transpose, c->ftmp);
}

void residual(nc_ns_ctx* c, const double* s, double* r) {
  const NsLevel& L0 = c->lev[0];
  nc::ns::launch_residual(c->stream, L0.g, L0.c, c->patch, L0.coef, s, r);
}

// Jacobian hierarchy at s: level 0 in float64 (and its working-precision copy), the
// coarser levels rediscretised at the injected state, node-block inverses, the coarsest
// dense inverse.
template <typename T>
void linearize_t(nc_ns_ctx* c, const double* s) {
  hipStream_t st = c->stream;
  const double t0 = now();
  NsLevel& L0 = c->lev[0];
  nc::ns::launch_assemble<double>(st, L0.g, L0.c, L0.coef, s, c->A64);
  launch_diagonal<double>(st, L0.g, c->A64, c->bs);
  {
    double dn[10];
    field_norms(c, c->bs, nullptr, dn);
    for (int f = 0; f < 5; ++f) {
      const double rms = c->nfree[f] > 0 ? dn[f] / std::sqrt((double)c->nfree[f]) : 1.0;
      c->rs.s[f] = rms > 0.0 && std::isfinite(rms) ? rms : 1.0;
      c->rs_inv.s[f] = 1.0 / c->rs.s[f];
    }
  }
  if (c->mixed) launch_convert<double, float>(st, c->A64, (float*)L0.A, (long)NS_ENTRIES * c->N, 1.0);
  const double* sf = s;
  for (int l = 1; l < c->L; ++l) {
    NsLevel& L = c->lev[l];
    nc::ns::launch_inject(st, c->lev[l - 1].g, L.g, sf, L.st);
    nc::ns::launch_assemble<T>(st, L.g, L.c, L.coef, L.st, (T*)L.A);
    sf = L.st;
  }
  for (int l = 0; l < c->L; ++l)
    nc::ns::launch_diag_inverse<T>(st, c->lev[l].g, (const T*)c->lev[l].A, (T*)c->lev[l].Dinv);
  if (c->dense) {
    const NsLevel& Lc = c->lev[c->L - 1];
    nc::ns::launch_dense<T>(st, Lc.g, (const T*)Lc.A, c->Ad);
    launch_gauss_jordan(st, c->Ad, c->ncoarse, c->perm, c->gjwork);
    launch_dense_transpose(st, c->Ad, c->Ad + (size_t)c->ncoarse * c->ncoarse, c->ncoarse);
  }
  ck(hipGetLastError());
  sync(c);
  c->t_setup += now() - t0;
  c->lin_valid = true;
  c->lin_s = s;
}

// The Krylov operator stays the float64 Jacobian in NC_MIXED as well: with a float32 one
// the Newton steps lose their quadratic convergence on these ill-conditioned systems
// (measured: 25 Newton steps instead of 3 on the 128x64x128 cavity).
void linearize(nc_ns_ctx* c, const double* s) {
  if (c->mixed) linearize_t<float>(c, s);
  else linearize_t<double>(c, s);
}

// One V-cycle from level l on lev[l].b with a zero initial guess; returns the buffer
// holding the result (lev[l].x or lev[l].x2).
template <typename T>
T* vcycle(nc_ns_ctx* c, int l, bool tr) {
  hipStream_t st = c->stream;
  NsLevel& L = c->lev[l];
  const T om = (T)c->omega;
  T* cur = (T*)L.x;
  T* nxt = (T*)L.x2;
  const T* A = (const T*)L.A;
  const T* Di = (const T*)L.Dinv;
  const T* b = (const T*)L.b;
  if (l == c->L - 1) {
    if (c->dense) {
      launch_dense_apply<T>(st, c->Ad, c->ncoarse, tr, b, cur);
      return cur;
    }
    nc::ns::launch_diag_scale<T>(st, L.g, Di, tr, om, b, cur);
    for (int k = 1; k < COARSE_SWEEPS; ++k) {
      nc::ns::launch_bsr<T, T>(st, L.g, A, Di, tr, 2, cur, b, nxt, om);
      std::swap(cur, nxt);
    }
    return cur;
  }
  const int npre = l == 0 ? c->p.smooth_pre : c->p.smooth_pre_coarse;
  const int npost = l == 0 ? c->p.smooth_post : c->p.smooth_post_coarse;
  nc::ns::launch_diag_scale<T>(st, L.g, Di, tr, om, b, cur);
  for (int k = 1; k < npre; ++k) {
    nc::ns::launch_bsr<T, T>(st, L.g, A, Di, tr, 2, cur, b, nxt, om);
    std::swap(cur, nxt);
  }
  nc::ns::launch_bsr<T, T>(st, L.g, A, Di, tr, 1, cur, b, (T*)L.r, om);
  NsLevel& C = c->lev[l + 1];
  nc::ns::launch_restrict<T>(st, L.g, C.g, (const T*)L.r, (T*)C.b);
  T* xc = vcycle<T>(c, l + 1, tr);
  nc::ns::launch_prolong_add<T>(st, L.g, C.g, xc, cur);
  for (int k = 0; k < npost; ++k) {
    nc::ns::launch_bsr<T, T>(st, L.g, A, Di, tr, 2, cur, b, nxt, om);
    std::swap(cur, nxt);
  }
  return cur;
}

// z = M^-1 (scale v) (M^-T when tr), float64 in and out; scale: the row scales S of the
// equilibrated Krylov system (or the identity)
void precondition(nc_ns_ctx* c, bool tr, const double* v, double* z, const Field5& scale) {
  hipStream_t st = c->stream;
  NsLevel& L0 = c->lev[0];
  if (c->mixed) {
    nc::ns::launch_scale_fields<double, float>(st, c->N, v, (float*)L0.b, scale);
    const float* x = vcycle<float>(c, 0, tr);
    launch_convert<float, double>(st, x, z, c->n5, 1.0);
  } else {
    nc::ns::launch_scale_fields<double, double>(st, c->N, v, (double*)L0.b, scale);
    const double* x = vcycle<double>(c, 0, tr);
    launch_convert<double, double>(st, x, z, c->n5, 1.0);
  }
}

const Field5 kUnit{{1.0, 1.0, 1.0, 1.0, 1.0}};

void apply(nc_ns_ctx* c, bool tr, const double* x, double* y) {
  nc::ns::launch_bsr<double, double>(c->stream, c->lev[0].g, c->A64, nullptr, tr, 0, x, nullptr, y, 0.0);
}

// y = S^-1 A x (A^T when tr): the operator of the equilibrated Krylov system
void apply_scaled(nc_ns_ctx* c, bool tr, const double* x, double* y) {
  apply(c, tr, x, y);
  nc::ns::launch_scale_fields<double, double>(c->stream, c->N, y, y, c->rs_inv);
}

// Right-preconditioned flexible GMRES(m) on S^-1 J~ x = S^-1 b (J~^T when tr) in float64,
// from x = 0, classical Gram-Schmidt with one reorthogonalisation; restarts from the true
// residual.  Returns the iterations (or -1 on a non-finite value); *relres the final
// relative residual of the equilibrated system.
int fgmres(nc_ns_ctx* c, bool tr, const double* b_in, double* x, double rtol, int maxit, double* relres,
           bool* stalled = nullptr) {
  hipStream_t st = c->stream;
  const long n = c->n5, ld = c->ld;
  const int m = c->m;
  double* V = c->V;
  double* Z = c->Z;
  double* dres = c->dres;
  double* b = c->bs;
  nc::ns::launch_scale_fields<double, double>(st, c->N, b_in, b, c->rs_inv);
  nc::ns::launch_fill<double>(st, x, n, 0.0);
  const double bnorm = norm(c, b);
  *relres = 0.0;
  if (bnorm == 0.0) return 0;
  if (!std::isfinite(bnorm)) return -1;
  launch_convert<double, double>(st, b, V, n, 1.0 / bnorm);
  double beta = bnorm;
  int total = 0;
  std::vector<double> H((m + 1) * m), cs(m), sn(m), g(m + 1), y(m);
  while (true) {
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int jend = 0;
    for (int j = 0; j < m; ++j) {
      double* vj = V + (long)j * ld;
      double* w = V + (long)(j + 1) * ld;
      double* zj = Z + (long)j * ld;
      precondition(c, tr, vj, zj, c->rs);
      apply_scaled(c, tr, zj, w);
      launch_mdot<double>(st, V, ld, j + 1, w, n, c->part, dres);
      launch_maxpy<double>(st, V, ld, j + 1, dres, -1.0, w, n, c->part, nullptr);
      launch_mdot<double>(st, V, ld, j + 1, w, n, c->part, dres + MAXC);
      launch_maxpy<double>(st, V, ld, j + 1, dres + MAXC, -1.0, w, n, c->part, dres + 2 * MAXC);
      fetch(c, dres, 3 * MAXC);
      const double* hs = c->hbuf;
      for (int i = 0; i <= j; ++i) H[i * m + j] = hs[i] + hs[MAXC + i];
      const double hn = hs[2 * MAXC];
      H[(j + 1) * m + j] = hn;
      if (hn > 0.0) launch_scale_inv<double>(st, dres + 2 * MAXC, w, w, n);
      for (int i = 0; i < j; ++i) {
        const double a = H[i * m + j], bb = H[(i + 1) * m + j];
        H[i * m + j] = cs[i] * a + sn[i] * bb;
        H[(i + 1) * m + j] = -sn[i] * a + cs[i] * bb;
      }
      const double a = H[j * m + j], bb = H[(j + 1) * m + j];
      const double r = std::hypot(a, bb);
      cs[j] = r > 0 ? a / r : 1.0;
      sn[j] = r > 0 ? bb / r : 0.0;
      H[j * m + j] = r;
      H[(j + 1) * m + j] = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      ++total;
      jend = j + 1;
      const double res = std::fabs(g[j + 1]) / bnorm;
      *relres = res;
      if (!std::isfinite(res)) return -1;
      if (res <= rtol || total >= maxit || hn == 0.0) break;
    }
    for (int i = jend - 1; i >= 0; --i) {
      double s = g[i];
      for (int k = i + 1; k < jend; ++k) s -= H[i * m + k] * y[k];
      y[i] = s / H[i * m + i];
    }
    std::memcpy(c->hbuf, y.data(), sizeof(double) * jend);
    ck(hipMemcpyAsync(dres + 3 * MAXC, c->hbuf, sizeof(double) * jend, hipMemcpyHostToDevice, st));
    launch_maxpy<double>(st, Z, ld, jend, dres + 3 * MAXC, 1.0, x, n, c->part, nullptr);
    // restart (or final check) from the true residual
    apply_scaled(c, tr, x, V);
    launch_rsub<double>(st, b, V, n);
    beta = norm(c, V);
    *relres = beta / bnorm;
    if (!std::isfinite(beta)) return -1;
    if (*relres <= rtol || total >= maxit) break;
    // a first cycle that has not halved the residual: the smoother's damping does not suit
    // this system (undamped node-block Jacobi diverges on the saddle-point blocks)
    if (stalled && total == jend && *relres > 0.5) {
      *stalled = true;
      return total;
    }
    launch_convert<double, double>(st, V, V, n, 1.0 / beta);
  }
  return total;
}

// fgmres, switching the context to the fallback damping for good (and solving again from
// zero) when the first restart cycle stalls; the fallback only ever damps more
int krylov(nc_ns_ctx* c, bool tr, const double* b, double* x, double rtol, double* relres) {
  const double fb = c->p.smooth_omega_fallback;
  bool stalled = false;
  int its = fgmres(c, tr, b, x, rtol, c->p.krylov_maxit, relres, fb > 0.0 && fb < c->omega ? &stalled : nullptr);
  if (its < 0 || !stalled) return its;
  c->omega = fb;
  const int more = fgmres(c, tr, b, x, rtol, c->p.krylov_maxit, relres);
  return more < 0 ? more : its + more;
}

// max over fields of |a_f| / |b_f| (0 where both vanish)
double field_ratio(const double* na, const double* nb) {
  double worst = 0.0;
  for (int f = 0; f < 5; ++f) worst = std::max(worst, na[f] / std::max(nb[f], 1e-300));
  return worst;
}

int newton(nc_ns_ctx* c, double* s, nc_info* info) {
  hipStream_t st = c->stream;
  const nc_problem& p = c->p;
  const NsLevel& L0 = c->lev[0];
  nc::ns::launch_mask(st, L0.g, s);
  residual(c, s, c->R);
  double nr[10];
  field_norms(c, c->R, nullptr, nr);
  double nrm = 0.0;
  for (int f = 0; f < 5; ++f) nrm += nr[f] * nr[f];
  nrm = std::sqrt(nrm);
  if (info) for (int f = 0; f < 5; ++f) info->res0[f] = nr[f];
  if (!std::isfinite(nrm)) return NC_ENAN;
  double prev = nrm;
  bool converged = false;
  int it = 0, ktot = 0;
  double relres = 0.0;
  for (; it < p.newton_maxit; ++it) {
    linearize(c, s);
    double eta = p.newton_eta0 > 0.0 ? p.newton_eta0 : p.krylov_rtol;
    if (it > 0 && p.newton_eta0 > 0.0) {
      const double ratio = nrm / prev;
      eta = std::min(p.newton_eta0, std::max(p.krylov_rtol, 0.9 * ratio * ratio));
    }
    const int its = krylov(c, false, c->R, c->d, eta, &relres);
    if (its < 0) return NC_ENAN;
    ktot += its;
    // full step s - d; a full step already below the tolerance in every field is taken
    // undamped and ends the iteration
    launch_axpy(st, -1.0, c->d, s, c->strial, c->n5);
    double nds[10];
    field_norms(c, c->d, c->strial, nds);
    const bool tiny = field_ratio(nds, nds + 5) <= p.newton_step_rtol;
    double lam = 1.0, nt = 0.0;
    while (true) {
      if (lam < 1.0) launch_axpy(st, -lam, c->d, s, c->strial, c->n5);
      residual(c, c->strial, c->tmp5);
      double ntf[10];
      field_norms(c, c->tmp5, nullptr, ntf);
      nt = 0.0;
      for (int f = 0; f < 5; ++f) nt += ntf[f] * ntf[f];
      nt = std::sqrt(nt);
      if (tiny || nt <= nrm || lam < 1.0 / 64) break;
      lam *= 0.5;
    }
    ck(hipMemcpyAsync(s, c->strial, sizeof(double) * c->n5, hipMemcpyDeviceToDevice, st));
    ck(hipMemcpyAsync(c->R, c->tmp5, sizeof(double) * c->n5, hipMemcpyDeviceToDevice, st));
    prev = nrm;
    nrm = nt;
    if (!std::isfinite(nrm)) return NC_ENAN;
    double rel[10];
    field_norms(c, c->d, s, rel);
    const double step = field_ratio(rel, rel + 5);
    if (info && it < NC_HIST_MAX) {
      info->hist_krylov[it] = its;
      double hr[10];
      field_norms(c, c->R, nullptr, hr);
      for (int f = 0; f < 5; ++f) info->hist_res[it][f] = hr[f];
      info->hist_len = it + 1;
    }
    if (lam == 1.0 && step <= p.newton_step_rtol) {
      converged = true;
      ++it;
      break;
    }
  }
  if (info) {
    info->newton_its = it;
    info->krylov_its = ktot;
    info->levels = c->L;
    info->krylov_f64 = 0;
    info->rel_res = relres;
    double fr[10];
    field_norms(c, c->R, nullptr, fr);
    for (int f = 0; f < 5; ++f) info->res[f] = fr[f];
  }
  c->lin_valid = false;   // the hierarchy is at the previous iterate
  return converged ? NC_OK : NC_NOT_CONVERGED;
}

int adjoint(nc_ns_ctx* c, const double* s, const double* rhs, double* lam, nc_info* info) {
  hipStream_t st = c->stream;
  linearize(c, s);
  ck(hipMemcpyAsync(c->tmp5, rhs, sizeof(double) * c->n5, hipMemcpyDeviceToDevice, st));
  nc::ns::launch_mask(st, c->lev[0].g, c->tmp5);
  double relres = 0.0;
  const int its = krylov(c, true, c->tmp5, lam, c->p.adjoint_rtol, &relres);
  if (its < 0) return NC_ENAN;
  nc::ns::launch_mask(st, c->lev[0].g, lam);
  if (info) {
    double r0[10];
    field_norms(c, c->tmp5, nullptr, r0);
    for (int f = 0; f < 5; ++f) info->res0[f] = r0[f];
    apply(c, true, lam, c->d);
    launch_rsub<double>(st, c->tmp5, c->d, c->n5);
    double rr[10];
    field_norms(c, c->d, nullptr, rr);
    for (int f = 0; f < 5; ++f) info->res[f] = rr[f];
    info->krylov_its = its;
    info->levels = c->L;
    info->krylov_f64 = 0;
    info->rel_res = relres;
    info->hist_len = 1;
    info->hist_krylov[0] = its;
    for (int f = 0; f < 5; ++f) info->hist_res[0][f] = rr[f];
  }
  return relres <= 10.0 * c->p.adjoint_rtol ? NC_OK : NC_NOT_CONVERGED;
}

template <class F>
int guarded(F f) {
  try {
    return f();
  } catch (const NsError&) {
    return NC_EHIP;
  } catch (const std::bad_alloc&) {
    return NC_EHIP;
  }
}

}  // namespace

// ====================================================================== C ABI
extern "C" {

size_t nc_ns_workspace_bytes(const nc_problem* p) {
  if (!valid(p)) return 0;
  nc_ns_ctx tmp;
  tmp.p = *p;
  if (tmp.p.h <= 0) tmp.p.h = 1.0 / p->nx;
  return carve(&tmp, nullptr);
}

int nc_ns_create(const nc_problem* p, void* workspace_dev, size_t bytes, void* stream, nc_ns_ctx** out) {
  if (!out || !valid(p) || !workspace_dev) return NC_EINVAL;
  *out = nullptr;
  return guarded([&]() {
    nc_ns_ctx* c = new nc_ns_ctx();
    c->p = *p;
    if (c->p.h <= 0) c->p.h = 1.0 / p->nx;
    const size_t need = carve(c, nullptr);
    if (bytes < need) {
      delete c;
      return NC_ENOMEM;
    }
    char* base = (char*)workspace_dev;
    const size_t mis = (size_t)((uintptr_t)base % NS_ALIGN);
    if (mis) base += NS_ALIGN - mis;
    carve(c, base);
    c->ws_base = base;
    c->ws_need = need;
    c->stream = (hipStream_t)stream;
    c->patch = Patch{c->p.q_h, c->p.patch_x0, c->p.patch_x1, c->p.patch_y0, c->p.patch_y1, c->p.h};
    c->design_set = false;
    c->lin_valid = false;
    c->lin_s = nullptr;
    c->omega = c->p.smooth_omega;
    c->t_setup = 0.0;
    c->hbuf = nullptr;
    if (hipHostMalloc((void**)&c->hbuf, sizeof(double) * 4 * MAXC, hipHostMallocDefault) != hipSuccess) {
      delete c;
      return NC_EHIP;
    }
    *out = c;
    return NC_OK;
  });
}

int nc_ns_set_problem(nc_ns_ctx* c, const nc_problem* p) {
  if (!c || !valid(p)) return NC_EINVAL;
  return guarded([&]() {
    nc_ns_ctx tmp;
    tmp.p = *p;
    if (tmp.p.h <= 0) tmp.p.h = 1.0 / p->nx;
    const size_t need = carve(&tmp, nullptr);
    bool same = need == c->ws_need && tmp.L == c->L && tmp.mixed == c->mixed && tmp.m == c->m &&
                tmp.dense == c->dense && tmp.pde == c->pde;
    for (int l = 0; same && l < c->L; ++l)
      same = tmp.lev[l].g.nx == c->lev[l].g.nx && tmp.lev[l].g.ny == c->lev[l].g.ny && tmp.lev[l].g.nz == c->lev[l].g.nz;
    if (!same) return NC_EINVAL;
    sync(c);
    c->p = tmp.p;
    carve(c, c->ws_base);   // the same layout: recomputes the level constants and regions only
    c->patch = Patch{c->p.q_h, c->p.patch_x0, c->p.patch_x1, c->p.patch_y0, c->p.patch_y1, c->p.h};
    c->omega = c->p.smooth_omega;
    c->design_set = false;
    c->lin_valid = false;
    return NC_OK;
  });
}

int nc_ns_destroy(nc_ns_ctx* c) {
  if (!c) return NC_EINVAL;
  (void)hipStreamSynchronize(c->stream);
  if (c->hbuf) (void)hipHostFree(c->hbuf);
  delete c;
  return NC_OK;
}

int nc_ns_set_design(nc_ns_ctx* c, const double* x) {
  if (!c || !x) return NC_EINVAL;
  return guarded([&]() {
    hipStream_t st = c->stream;
    const nc_problem& p = c->p;
    NsLevel& L0 = c->lev[0];
    apply_filter(c, x, c->gamma, false);
    if (c->regions) launch_passive(st, L0.g, c->reg, c->gamma);
    // conductivity RAMP (and a permeability that the next kernel overwrites)
    launch_ramp(st, c->E, c->gamma, p.k_f, p.k_s, p.q_c, p.kappa_f, 0.5 * p.kappa_f, p.q_p, L0.coef, c->coef32, c->dk,
                c->da);
    nc::ns::launch_brinkman(st, c->E, p.kappa_s, p.q_p, c->gamma, L0.coef, c->da);
    for (int l = 1; l < c->L; ++l)
      launch_average_coef<double>(st, c->lev[l - 1].g, c->lev[l].g, c->lev[l - 1].coef, c->lev[l].coef);
    ck(hipGetLastError());
    c->design_set = true;
    c->lin_valid = false;
    return NC_OK;
  });
}

int nc_ns_get_gamma(nc_ns_ctx* c, double* gamma) {
  if (!c || !gamma || !c->design_set) return NC_EINVAL;
  return guarded([&]() {
    ck(hipMemcpyAsync(gamma, c->gamma, sizeof(double) * c->E, hipMemcpyDeviceToDevice, c->stream));
    return NC_OK;
  });
}

int nc_ns_residual(nc_ns_ctx* c, const double* s, double* r) {
  if (!c || !s || !r || s == r || !c->design_set) return NC_EINVAL;
  return guarded([&]() {
    residual(c, s, r);
    ck(hipGetLastError());
    return NC_OK;
  });
}

int nc_ns_linearize(nc_ns_ctx* c, const double* s) {
  if (!c || !s || !c->design_set) return NC_EINVAL;
  return guarded([&]() {
    linearize(c, s);
    return NC_OK;
  });
}

int nc_ns_jac_apply(nc_ns_ctx* c, const double* v, double* y) {
  if (!c || !v || !y || v == y || !c->lin_valid) return NC_EINVAL;
  return guarded([&]() {
    apply(c, false, v, y);
    ck(hipGetLastError());
    return NC_OK;
  });
}

int nc_ns_jacT_apply(nc_ns_ctx* c, const double* w, double* y) {
  if (!c || !w || !y || w == y || !c->lin_valid) return NC_EINVAL;
  return guarded([&]() {
    apply(c, true, w, y);
    ck(hipGetLastError());
    return NC_OK;
  });
}

int nc_ns_precondition(nc_ns_ctx* c, int transpose, const double* v, double* z) {
  if (!c || !v || !z || v == z || !c->lin_valid) return NC_EINVAL;
  return guarded([&]() {
    precondition(c, transpose != 0, v, z, kUnit);
    ck(hipGetLastError());
    return NC_OK;
  });
}

int nc_ns_solve_state(nc_ns_ctx* c, double* s, nc_info* info) {
  if (!c || !s || !c->design_set) return NC_EINVAL;
  return guarded([&]() {
    const double t0 = now();
    c->t_setup = 0.0;
    if (info) std::memset(info, 0, sizeof(*info));
    const int r = newton(c, s, info);
    sync(c);
    if (info) {
      info->t_total = now() - t0;
      info->t_setup = c->t_setup;
      info->t_solve = info->t_total - info->t_setup;
    }
    return r;
  });
}

int nc_ns_objective(nc_ns_ctx* c, const double* s, double* f) {
  if (!c || !s || !f) return NC_EINVAL;
  return guarded([&]() {
    const NsLevel& L0 = c->lev[0];
    nc::ns::launch_objective(c->stream, L0.g, L0.c, c->patch, s, c->part, c->dres);
    fetch(c, c->dres, 1);
    *f = c->hbuf[0];
    return NC_OK;
  });
}

int nc_ns_objective_grad(nc_ns_ctx* c, const double* s, double* g) {
  if (!c || !s || !g) return NC_EINVAL;
  return guarded([&]() {
    const NsLevel& L0 = c->lev[0];
    nc::ns::launch_objective_grad(c->stream, L0.g, L0.c, c->patch, s, g);
    ck(hipGetLastError());
    return NC_OK;
  });
}

int nc_ns_solve_adjoint(nc_ns_ctx* c, const double* s, const double* rhs, double* lam, nc_info* info) {
  if (!c || !s || !rhs || !lam || rhs == lam || !c->design_set) return NC_EINVAL;
  return guarded([&]() {
    const double t0 = now();
    c->t_setup = 0.0;
    if (info) std::memset(info, 0, sizeof(*info));
    const int r = adjoint(c, s, rhs, lam, info);
    sync(c);
    if (info) {
      info->t_total = now() - t0;
      info->t_setup = c->t_setup;
      info->t_solve = info->t_total - info->t_setup;
    }
    return r;
  });
}

int nc_ns_sensitivity(nc_ns_ctx* c, const double* s, const double* lam, double* dfdx, double* dfdgamma) {
  if (!c || !s || !lam || !dfdx || !c->design_set) return NC_EINVAL;
  return guarded([&]() {
    hipStream_t st = c->stream;
    const NsLevel& L0 = c->lev[0];
    double* g = dfdgamma ? dfdgamma : c->sens;
    nc::ns::launch_sensitivity(st, L0.g, L0.c, L0.coef, c->dk, c->da, s, lam, g);
    if (c->regions) launch_design_mask(st, L0.g, c->reg, g, false, 0.0);
    apply_filter(c, g, dfdx, true);
    if (c->regions) launch_design_mask(st, L0.g, c->reg, dfdx, false, 0.0);
    ck(hipGetLastError());
    return NC_OK;
  });
}

}  // extern "C"
