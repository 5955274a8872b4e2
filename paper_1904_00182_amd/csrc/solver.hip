// Solver runtime behind the C ABI of include/nc.h: context and workspace carving, the
// multigrid hierarchy, flexible GMRES, the damped Newton iteration (Sec. 5.4), the
// adjoint solve with iterative refinement and the sensitivities (Sec. 5.1).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <type_traits>
#include <vector>

#include "kernels.hpp"
#include "../../include/nc.h"

using namespace nc;

namespace {

constexpr int MAXLEV = 10;
constexpr size_t ALIGN = 256;

struct Level {
  Grid g;
  double h;
  ElemConst<double> c64;
  ElemConst<float> c32;
  double* coef64;
  float* coef32;
  double* st64;
  float* st32;
  void* dinv;   // [N][4] in the working precision
  void* x;      // V-cycle iterate, ping-pong partner, right-hand side, residual: [N][2]
  void* x2;
  void* b;
  void* r;
};

struct Carver {
  char* base;
  size_t off = 0;
  template <typename T>
  T* take(size_t count) {
    off = (off + ALIGN - 1) / ALIGN * ALIGN;
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

struct HipError {
  hipError_t e;
};

// Kernel classes of the per-context event timer (nc_set_timing / nc_get_timing).
enum TimerClass {
  TC_RESIDUAL = 0, TC_JV, TC_JTW, TC_SMOOTH, TC_SMOOTH_T, TC_PT_RESID, TC_DIAG, TC_UPROJ, TC_TRANSFER,
  TC_COARSE, TC_MDOT, TC_MAXPY, TC_VECTOR, TC_SETUP, TC_SMOOTH_COARSE, TC_PT_RESID_COARSE, TC_COUNT
};
constexpr int TIMER_EVENTS = 8192;
constexpr int SETUP_REC = 8;   // hierarchy rebuilds timed before the event pool is drained

inline void ck(hipError_t e) {
  if (e != hipSuccess) throw HipError{e};
}

}  // namespace

struct nc_ctx {
  nc_problem p;
  hipStream_t stream;
  char* ws_base;         // the caller's workspace (aligned) and the bytes the layout uses
  size_t ws_need;
  bool mixed;
  int L;
  Level lev[MAXLEV];
  Patch patch;
  long N, E, n5;
  long ld;               // stride between Krylov vectors (2N rounded up to 64 for aligned vector loads)
  int m;                 // Krylov restart length
  // design chain
  double *gamma, *dk, *dkap, *ftmp, *sens;
  Regions reg;           // passive solid / fluid regions on the finest grid
  bool regions;          // any passive region
  long n_design;         // elements of the design domain
  bool pde;              // PDE (Helmholtz) density filter
  HelmholtzPlan helm;
  double* helm_work;     // its four node vectors
  // coarsest level
  double *emats, *A;
  int* perm;
  double* gjwork;
  int ncoarse;
  bool dense;            // coarsest level solved by the dense inverse (else smoothing only)
  // The coarsest inverse is built on a stream of its own, concurrently with the other
  // levels' setup and the first half of the first V-cycle, and the coarser levels' node-
  // block inverses on a second one, concurrently with the finest level's: `fork` (on
  // stream) orders both after the state injection, `join` (on side) and `join2` (on side2)
  // mark them done, and the pending flags say whether stream still has to wait for them
  // (before the first use of A, and before the first step down from the finest level).
  hipStream_t side, side2;
  hipEvent_t fork, join, join2;
  bool join_pending, join2_pending;
  // device time of the hierarchy rebuilds of one solve call (nc_info.t_setup): per
  // rebuild a start event on stream and an end event on each of the three streams
  hipEvent_t setup_ev[SETUP_REC][4];
  int setup_used;
  double setup_s;
  // Krylov space in the working precision
  void *V, *Z, *kx, *kb;
  // reductions
  double *part, *dres;
  double* hbuf;          // pinned host mirror of dres
  double* hslots;        // pinned: one Hessenberg column (h1, h2, norm) per Krylov iteration, then |b|
  std::vector<hipEvent_t> kev;   // completion of each Krylov iteration's column copy
  // float64 Newton / adjoint vectors
  double *R, *d, *strial, *ra, *tmp5;
  double* pt64;          // float64 (P, T) vector of the reduced solves
  // per-field row equilibration of the five-field system inside FGMRES
  Scale5<double> rows64;
  Scale5<float> rows32;
  // row weights of the Krylov solves (the equilibration above, reweighted per field in
  // the adjoint refinement)
  Scale5<double> krow64;
  Scale5<float> krow32;
  // bookkeeping
  bool design_set;
  bool hier_valid;       // multigrid hierarchy (node-block inverses, coarse inverse) built for this design
  bool rows_valid;       // rows64 / rows32 and res_floor computed for this design
  double res_floor;      // round-off floor of the scaled residual
  double omega;          // block-Jacobi damping in use: smooth_omega, or the fallback after a stall
  bool k64;              // NC_MIXED: Krylov vectors and operator in float64 (float32 V-cycle) after a
                         // float32 Krylov solve failed to converge
  bool reserve64;        // V64 / Z64 hold a float64 Krylov basis for that fallback
  double* V64;
  double* Z64;
  // optional event timing per kernel class
  bool timing;
  std::vector<hipEvent_t> ev;
  std::vector<int> ev_class;
  std::vector<double> ev_bytes;
  int ev_used;
  double t_ms[TC_COUNT];
  long t_cnt[TC_COUNT];
  double t_bytes[TC_COUNT];   // algorithmic bytes moved by the timed launches
};

namespace {

// ------------------------------------------------------------------ event timing
void timing_flush(nc_ctx* c) {
  if (!c->timing || c->ev_used == 0) return;
  ck(hipStreamSynchronize(c->side));   // timed launches on the setup streams
  ck(hipStreamSynchronize(c->side2));
  ck(hipEventSynchronize(c->ev[2 * c->ev_used - 1]));
  for (int k = 0; k < c->ev_used; ++k) {
    float ms = 0.f;
    ck(hipEventElapsedTime(&ms, c->ev[2 * k], c->ev[2 * k + 1]));
    c->t_ms[c->ev_class[k]] += ms;
    c->t_cnt[c->ev_class[k]] += 1;
    c->t_bytes[c->ev_class[k]] += c->ev_bytes[k];
  }
  c->ev_used = 0;
}

// RAII bracket around the launches of one kernel class; `bytes`: the algorithmic bytes
// the launches must move (inputs read once, outputs written once)
struct Timed {
  nc_ctx* c;
  int k;
  Timed(nc_ctx* ctx, int cls, double bytes = 0.0) : c(ctx), k(-1) {
    if (!c->timing) return;
    if (c->ev_used == TIMER_EVENTS / 2) timing_flush(c);
    k = c->ev_used++;
    c->ev_class[k] = cls;
    c->ev_bytes[k] = bytes;
    // bracket the scope; the first kernel launched in it re-records both events inside
    // its own dispatch (launch_timer), so the class time is that kernel's duration
    ck(hipEventRecord(c->ev[2 * k], c->stream));
    launch_timer() = LaunchTimer{c->ev[2 * k], c->ev[2 * k + 1]};
  }
  ~Timed() {
    if (k < 0) return;
    LaunchTimer& lt = launch_timer();
    if (lt.start) {   // no kernel in the scope
      (void)hipEventRecord(c->ev[2 * k + 1], c->stream);
      lt = LaunchTimer{};
    }
  }
};

// node and element counts of a level, for the byte counts of timed launches
double nn(const Grid& g) { return (double)(g.nx + 1) * (g.ny + 1) * (g.nz + 1); }
double ne(const Grid& g) { return (double)g.nx * g.ny * g.nz; }

// ------------------------------------------------------------------ setup helpers
// A box (x0, x1, y0, y1, z0, z1) is in use when x1 > x0, y1 > y0 and z1 > z0.
bool box_on(const double* b) { return b[1] > b[0] && b[3] > b[2] && b[5] > b[4]; }

// Inclusive element index ranges of the elements whose centre ((i + 1/2) h, ...) lies in
// the closed box; an empty range has lo > hi.
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

bool valid_problem(const nc_problem* p) {
  if (!p || p->nx < 1 || p->ny < 1 || p->nz < 1) return false;
  if ((double)(p->nx + 1) * (p->ny + 1) * (p->nz + 1) * 5 >= 2147483647.0) return false;   // 32-bit indices
  if ((double)(p->nx + 1) * (p->ny + 1) * 5 * 8 >= 4294967296.0) return false;   // 32-bit offsets in a layer
  if (p->mu <= 0 || p->kappa_s <= 0 || p->kappa_f <= 0 || p->k_f <= 0 || p->k_s <= 0) return false;
  if (p->precision != NC_FP64 && p->precision != NC_MIXED) return false;
  if (p->krylov_restart < 1 || p->krylov_restart > MAXC - 2) return false;
  if (!(p->krylov_rtol > 0) || !(p->krylov_rtol_mixed > 0) || !(p->adjoint_rtol > 0)) return false;
  if (p->gs_passes != 1 && p->gs_passes != 2) return false;
  if (p->coarse_tail != 0 && p->coarse_tail != 1) return false;
  if (p->f64_krylov_fallback != 0 && p->f64_krylov_fallback != 1) return false;
  if (!(p->newton_eta0 >= 0.0 && p->newton_eta0 < 1.0)) return false;
  if (p->smooth_pre < 1 || p->smooth_post < 0 || p->smooth_pre_coarse < 1 || p->smooth_post_coarse < 0) return false;
  if (!(p->smooth_omega > 0.0 && p->smooth_omega <= 2.0) || !(p->smooth_omega_fallback >= 0.0 && p->smooth_omega_fallback <= 2.0))
    return false;
  if (p->filter_kind != NC_FILTER_CONE && p->filter_kind != NC_FILTER_PDE) return false;
  if ((p->sym_x != 0 && p->sym_x != 1) || (p->sym_y != 0 && p->sym_y != 1)) return false;
  if (!(p->filter_radius >= 0.0)) return false;
  return true;
}

int choose_levels(const nc_problem* p, Grid* gs) {
  Grid g{p->nx, p->ny, p->nz, (p->sym_x ? 1 : 0) | (p->sym_y ? 2 : 0)};
  gs[0] = g;
  int L = 1;
  const int cap = p->levels > 0 ? std::min(p->levels, MAXLEV) : MAXLEV;
  while (L < cap) {
    const Grid& f = gs[L - 1];
    if ((f.nx & 1) || (f.ny & 1) || (f.nz & 1)) break;
    if (f.nx / 2 < 2 || f.ny / 2 < 2 || f.nz / 2 < 2) break;
    if (p->levels <= 0 && 2 * f.nodes() <= 300) break;
    gs[L] = Grid{f.nx / 2, f.ny / 2, f.nz / 2, f.sym};
    ++L;
  }
  return L;
}

// Lays out every device buffer in the workspace (base == nullptr: size query only).
size_t carve(nc_ctx* c, char* base) {
  Carver cv{base};
  const nc_problem& p = c->p;
  Grid gs[MAXLEV];
  c->L = choose_levels(&p, gs);
  c->mixed = p.precision == NC_MIXED;
  const size_t rs = c->mixed ? sizeof(float) : sizeof(double);
  const double h0 = p.h > 0 ? p.h : 1.0 / p.nx;
  for (int l = 0; l < c->L; ++l) {
    Level& L = c->lev[l];
    L.g = gs[l];
    L.h = h0 * (1 << l);
    L.c64 = make_elem_const<double>(L.h, p.rho0, p.mu, p.cp, p.g0, p.alpha, p.Q);
    L.c32 = make_elem_const<float>(L.h, p.rho0, p.mu, p.cp, p.g0, p.alpha, p.Q);
    if (box_on(p.q_box)) {   // the source only on the elements of the box (on every level)
      int r[6];
      box_range(p.q_box, L.g, L.h, r);
      L.c64.qi0 = L.c32.qi0 = r[0]; L.c64.qi1 = L.c32.qi1 = r[1];
      L.c64.qj0 = L.c32.qj0 = r[2]; L.c64.qj1 = L.c32.qj1 = r[3];
      L.c64.qk0 = L.c32.qk0 = r[4]; L.c64.qk1 = L.c32.qk1 = r[5];
    }
    const long N = L.g.nodes(), E = L.g.elems();
    L.coef64 = cv.take<double>(2 * E);
    L.coef32 = cv.take<float>(2 * E);
    L.st64 = cv.take<double>(2 * N);
    L.st32 = cv.take<float>(2 * N);
    L.dinv = cv.take<char>(4 * N * rs);
    L.x = cv.take<char>(2 * N * rs);
    L.x2 = cv.take<char>(2 * N * rs);
    L.b = cv.take<char>(2 * N * rs);
    L.r = cv.take<char>(2 * N * rs);
  }
  c->N = gs[0].nodes();
  c->E = gs[0].elems();
  // passive regions on the finest grid
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
  c->n5 = 5 * c->N;
  c->m = p.krylov_restart;
  c->gamma = cv.take<double>(c->E);
  c->dk = cv.take<double>(c->E);
  c->dkap = cv.take<double>(c->E);
  c->ftmp = cv.take<double>(c->E);
  c->sens = cv.take<double>(c->E);
  c->pde = p.filter_kind == NC_FILTER_PDE && p.filter_radius > 0.0;
  c->helm_work = cv.take<double>(c->pde ? 4 * c->N : 1);
  if (c->pde) c->helm = helmholtz_plan(h0, p.filter_radius, 1e-15);
  const Grid& gc = c->lev[c->L - 1].g;
  c->ncoarse = (int)(2 * gc.nodes());
  c->dense = c->ncoarse <= NC_DENSE_MAX;
  c->emats = cv.take<double>(c->dense ? gc.elems() * 256 : 1);
  c->A = cv.take<double>(c->dense ? 2 * (size_t)c->ncoarse * c->ncoarse : 1);   // inverse and its transpose
  c->perm = cv.take<int>(c->dense ? 2 * c->ncoarse : 1);
  c->gjwork = cv.take<double>(c->dense ? 2 * c->ncoarse : 1);
  c->ld = (2 * c->N + 63) / 64 * 64;   // Krylov vectors: the (P, T) system
  c->V = cv.take<char>((size_t)(c->m + 1) * c->ld * rs);
  c->Z = cv.take<char>((size_t)c->m * c->ld * rs);
  const bool reserve64 = c->mixed && p.f64_krylov_fallback != 0;
  c->V64 = cv.take<double>(reserve64 ? (size_t)(c->m + 1) * c->ld : 1);
  c->Z64 = cv.take<double>(reserve64 ? (size_t)c->m * c->ld : 1);
  c->reserve64 = reserve64;
  c->kx = cv.take<char>(2 * c->N * rs);
  c->kb = cv.take<char>(2 * c->N * rs);
  c->pt64 = cv.take<double>(2 * c->N);
  c->part = cv.take<double>(RED_BLOCKS * MAXC);   // per-block partial sums of the reductions
  c->dres = cv.take<double>(4 * MAXC);
  c->R = cv.take<double>(c->n5);
  c->d = cv.take<double>(c->n5);
  c->strial = cv.take<double>(c->n5);
  c->ra = cv.take<double>(c->n5);
  c->tmp5 = cv.take<double>(c->n5);
  return cv.off + ALIGN;
}

template <typename T>
LevelView<T> view(nc_ctx* c, int l);
template <>
LevelView<double> view<double>(nc_ctx* c, int l) {
  Level& L = c->lev[l];
  return LevelView<double>{L.g, L.c64, L.coef64, L.st64, (const double*)L.dinv};
}
template <>
LevelView<float> view<float>(nc_ctx* c, int l) {
  Level& L = c->lev[l];
  return LevelView<float>{L.g, L.c32, L.coef32, L.st32, (const float*)L.dinv};
}

void sync(nc_ctx* c) { ck(hipStreamSynchronize(c->stream)); }

void fetch(nc_ctx* c, const double* dev, int count) {
  ck(hipMemcpyAsync(c->hbuf, dev, sizeof(double) * count, hipMemcpyDeviceToHost, c->stream));
  sync(c);
}

// Make stream wait for the coarsest inverse built on the side stream, and for the coarser
// levels' node-block inverses.
void join_coarse(nc_ctx* c) {
  if (!c->join_pending) return;
  ck(hipStreamWaitEvent(c->stream, c->join, 0));
  c->join_pending = false;
}
void join_levels(nc_ctx* c) {
  if (!c->join2_pending) return;
  ck(hipStreamWaitEvent(c->stream, c->join2, 0));
  c->join2_pending = false;
}

// The context's density filter: y = F x, or F^T x when transpose (the PDE filter is
// symmetric; the cone filter's transpose goes through ftmp).
void apply_filter(nc_ctx* c, const double* x, double* y, bool transpose) {
  const Grid& g = c->lev[0].g;
  if (c->pde) launch_pde_filter(c->stream, g, c->helm, x, y, c->helm_work);
  else launch_cone_filter(c->stream, g, c->p.filter_radius, x, y, transpose, c->ftmp);
}

// dfdx = F^T dfdgamma for the filtered, passive-overwritten design: dfdgamma is zeroed
// on passive elements (their gamma is fixed) and dfdx off the design domain (those x are
// not design variables).
void pull_back(nc_ctx* c, double* dfdgamma, double* dfdx) {
  const Grid& g = c->lev[0].g;
  if (c->regions) launch_design_mask(c->stream, g, c->reg, dfdgamma, false, 0.0);
  apply_filter(c, dfdgamma, dfdx, true);
  if (c->regions) launch_design_mask(c->stream, g, c->reg, dfdx, false, 0.0);
}

// Adds the device time of the recorded hierarchy rebuilds to setup_s (each rebuild: from
// its start on stream to the last of its three streams' ends) and frees the event slots.
void setup_drain(nc_ctx* c) {
  for (int r = 0; r < c->setup_used; ++r) {
    float worst = 0.f;
    for (int k = 1; k < 4; ++k) {
      ck(hipEventSynchronize(c->setup_ev[r][k]));
      float ms = 0.f;
      ck(hipEventElapsedTime(&ms, c->setup_ev[r][0], c->setup_ev[r][k]));
      worst = std::max(worst, ms);
    }
    c->setup_s += 1e-3 * worst;
  }
  c->setup_used = 0;
}

// ------------------------------------------------------------------ linearisation
template <typename T>
void linearize_levels(nc_ctx* c) {
  hipStream_t st = c->stream;
  // the injection below overwrites what the previous setup on the side streams read
  join_coarse(c);
  join_levels(c);
  if (c->setup_used == SETUP_REC) setup_drain(c);
  hipEvent_t* sev = c->setup_ev[c->setup_used++];
  ck(hipEventRecord(sev[0], st));
  for (int l = 1; l < c->L; ++l) {
    if (sizeof(T) == 8)
      launch_inject_state<double>(st, c->lev[l - 1].g, c->lev[l].g, c->lev[l - 1].st64, c->lev[l].st64);
    else
      launch_inject_state<float>(st, c->lev[l - 1].g, c->lev[l].g, c->lev[l - 1].st32, c->lev[l].st32);
  }
  // after the injection (and every earlier reader of A and of the coarse levels on stream)
  if (c->dense || c->L > 1) ck(hipEventRecord(c->fork, st));
  if (c->L > 1) {
    ck(hipStreamWaitEvent(c->side2, c->fork, 0));
    for (int l = 1; l < c->L; ++l) {
      Timed tm(c, TC_SETUP);
      launch_diag_inverse<T>(c->side2, view<T>(c, l), (T*)c->lev[l].dinv, false);
    }
    ck(hipEventRecord(c->join2, c->side2));
    c->join2_pending = true;
  }
  ck(hipEventRecord(sev[2], c->L > 1 ? c->side2 : st));
  if (c->dense) {
    ck(hipStreamWaitEvent(c->side, c->fork, 0));
    { Timed tm(c, TC_SETUP); launch_coarse_assemble<T>(c->side, view<T>(c, c->L - 1), c->emats, c->A); }
    { Timed tm(c, TC_SETUP); launch_gauss_jordan(c->side, c->A, c->ncoarse, c->perm, c->gjwork); }
    { Timed tm(c, TC_SETUP); launch_dense_transpose(c->side, c->A, c->A + (size_t)c->ncoarse * c->ncoarse, c->ncoarse); }
    ck(hipEventRecord(c->join, c->side));
    c->join_pending = true;
  }
  ck(hipEventRecord(sev[3], c->dense ? c->side : st));
  {
    Timed tm(c, TC_SETUP);
    launch_diag_inverse<T>(st, view<T>(c, 0), (T*)c->lev[0].dinv, true);
  }
  ck(hipEventRecord(sev[1], st));
}

// Packs the (P, T) state used by the Jacobian applies; with `levels` also rebuilds the
// multigrid hierarchy (state injection, node-block inverses, coarsest inverse) at s.  The
// hierarchy only preconditions, so it may lag behind the state.
void linearize(nc_ctx* c, const double* s, bool levels) {
  hipStream_t st = c->stream;
  launch_pack_state<double>(st, c->lev[0].g, s, c->lev[0].st64);
  launch_pack_state<float>(st, c->lev[0].g, s, c->lev[0].st32);
  if (!levels) return;
  if (c->mixed) linearize_levels<float>(c);
  else linearize_levels<double>(c);
  c->hier_valid = true;
}

// ------------------------------------------------------------------ V-cycle
// x_ready: L.x already holds the first damped block-Jacobi step from a zero guess (fused
// into the restriction that produced L.b).
template <typename T>
void vcycle(nc_ctx* c, int l, bool tr, bool x_ready = false) {
  hipStream_t st = c->stream;
  Level& L = c->lev[l];
  const T om = (T)c->omega;
  LevelView<T> v = view<T>(c, l);
  const double sweep_bytes = sizeof(T) * (12 * nn(L.g) + 2 * ne(L.g));
  const int sweep_class = l == 0 ? (tr ? TC_SMOOTH_T : TC_SMOOTH) : TC_SMOOTH_COARSE;
  auto first_step = [&]() {
    if (x_ready) return;
    Timed tm(c, TC_TRANSFER, sizeof(T) * 8 * nn(L.g));
    launch_diag_scale<T>(st, L.g, (const T*)L.dinv, tr, om, (const T*)L.b, (T*)L.x);
  };
  auto sweep = [&]() {
    Timed tm(c, sweep_class, sweep_bytes);
    launch_pt_apply<T>(st, v, tr, MODE_SMOOTH, (const T*)L.x, (const T*)L.b, (T*)L.x2, om, l == 0);
    std::swap(L.x, L.x2);
  };
  if (l == c->L - 1) {
    if (c->dense) {
      join_coarse(c);
      Timed tm(c, TC_COARSE, (double)sizeof(T) * ((double)c->ncoarse * c->ncoarse + 2.0 * c->ncoarse));
      launch_dense_apply<T>(st, c->A, c->ncoarse, tr, (const T*)L.b, (T*)L.x);
    } else {
      first_step();
      for (int s = 1; s < 8; ++s) sweep();
    }
    return;
  }
  const int npre = l == 0 ? c->p.smooth_pre : c->p.smooth_pre_coarse;
  const int npost = l == 0 ? c->p.smooth_post : c->p.smooth_post_coarse;
  first_step();
  for (int s = 1; s < npre; ++s) sweep();
  { Timed tm(c, l == 0 ? TC_PT_RESID : TC_PT_RESID_COARSE, sizeof(T) * (8 * nn(L.g) + 2 * ne(L.g))); launch_pt_apply<T>(st, v, tr, MODE_RESID, (const T*)L.x, (const T*)L.b, (T*)L.r, om, l == 0); }
  Level& C = c->lev[l + 1];
  if (l == 0) join_levels(c);
  if (c->dense && c->p.coarse_tail && l + 2 == c->L - 1 && tail_cycle_fits<T>(L.g, C.g, c->lev[l + 2].g)) {
    // the rest of the cycle below this level in one workgroup
    const size_t n2 = (size_t)c->ncoarse * c->ncoarse;
    join_coarse(c);
    Timed tm(c, TC_COARSE, sizeof(T) * (6.0 * nn(L.g) + 8.0 * nn(C.g) + 2.0 * ne(C.g)) + 8.0 * n2);
    launch_tail_cycle<T>(st, L.g, (const T*)L.r, (T*)L.x, view<T>(c, l + 1), c->lev[l + 2].g, tr ? c->A + n2 : c->A,
                         tr, om, c->p.smooth_pre_coarse, c->p.smooth_post_coarse);
  } else {
    // the coarse level's first smoothing step rides along with the restriction, except on
    // a coarsest level solved by the dense inverse
    const bool fuse = !(l + 1 == c->L - 1 && c->dense);
    {
      Timed tm(c, TC_TRANSFER, sizeof(T) * (2 * nn(L.g) + (fuse ? 8 : 2) * nn(C.g)));
      launch_restrict<T>(st, L.g, C.g, (const T*)L.r, (T*)C.b, fuse ? (const T*)C.dinv : nullptr, tr, om, (T*)C.x);
    }
    vcycle<T>(c, l + 1, tr, fuse);
    { Timed tm(c, TC_TRANSFER, sizeof(T) * (4 * nn(L.g) + 2 * nn(C.g))); launch_prolong_add<T>(st, L.g, C.g, (const T*)C.x, (T*)L.x); }
  }
  for (int s = 0; s < npost; ++s) sweep();
}

// Block-Jacobi sweeps on the finest level after its first damped step (each swaps x, x2).
int level0_swaps(const nc_ctx* c) {
  if (c->L == 1) return c->dense ? 0 : 7;
  return std::max(0, c->p.smooth_pre - 1) + c->p.smooth_post;
}

// z = M^-1 v for the row-scaled (P, T) system D A (A^T when tr): one multigrid V-cycle
// on D^-1 v (rows = null: no scaling); with nrm, v is first normalised in place by the
// device scalar nrm[0].  The finest level's iterate buffers are routed so
// that the cycle's result ends in z.
template <typename T>
void precondition_pt(nc_ctx* c, bool tr, T* v, T* z, const Scale5<T>* rows, const double* nrm = nullptr) {
  hipStream_t st = c->stream;
  Level& L0 = c->lev[0];
  void* const xo = L0.x;
  void* const x2o = L0.x2;
  if (level0_swaps(c) % 2 == 0) L0.x = z;
  else L0.x2 = z;
  const T ip = rows ? (T)1 / rows->s[3] : (T)1, it = rows ? (T)1 / rows->s[4] : (T)1;
  {
    Timed tm(c, TC_VECTOR, sizeof(T) * 10 * nn(L0.g));
    launch_pc_in<T>(st, L0.g, v, nrm, ip, it, (const T*)L0.dinv, tr, (T)c->omega, (T*)L0.b, (T*)L0.x);
  }
  vcycle<T>(c, 0, tr, true);
  L0.x = xo;
  L0.x2 = x2o;
}

// y = D A x (A^T when tr), the operator of the (P, T) Krylov solve
template <typename T>
void apply_pt(nc_ctx* c, bool tr, const T* x, T* y, const Scale5<T>* rows) {
  Timed tm(c, tr ? TC_JTW : TC_JV, sizeof(T) * (6 * nn(c->lev[0].g) + 2 * ne(c->lev[0].g)));
  launch_pt_store<T>(c->stream, view<T>(c, 0), tr, x, y, rows);
}

template <typename T>
const Scale5<T>* row_scales(nc_ctx* c);
template <>
const Scale5<double>* row_scales<double>(nc_ctx* c) { return &c->krow64; }
template <>
const Scale5<float>* row_scales<float>(nc_ctx* c) { return &c->krow32; }

// Constant per-field row scales ~ 1 / (diagonal of each field's block): lumped mass for
// the velocity rows, (8h/3) kappa_mean/mu and (8h/3) k_mean for the P and T rows.
// They depend on the design only and are computed once per design; every solve starts its
// Krylov row weights from them.
double residual_floor(nc_ctx* c);
void compute_row_scales(nc_ctx* c) {
  if (!c->rows_valid) {
    const Level& L0 = c->lev[0];
    launch_coef_sums(c->stream, L0.coef64, c->E, c->part, c->dres);
    fetch(c, c->dres, 2);
    const double km = c->hbuf[0] / c->E, kapm = c->hbuf[1] / c->E;
    const double lap = 8.0 * L0.h / 3.0;
    const double du = 1.0 / (8.0 * L0.c64.W), dp = 1.0 / (lap * kapm / c->p.mu), dt = 1.0 / (lap * km);
    c->rows64 = Scale5<double>{{du, du, du, dp, dt}};
    c->rows32 = Scale5<float>{{(float)du, (float)du, (float)du, (float)dp, (float)dt}};
    c->res_floor = residual_floor(c);
    c->rows_valid = true;
  }
  c->krow64 = c->rows64;
  c->krow32 = c->rows32;
}

// ------------------------------------------------------------------ flexible GMRES
constexpr int HSLOT = 2 * MAXC + 8;   // doubles per Hessenberg slot: h1 [MAXC], h2 [MAXC], norm

// Solves D A x = b (A the (P, T) block of J~, A^T when tr, D the P and T row scales) from
// x = 0 with right preconditioning.  Each Arnoldi step orthogonalises by classical
// Gram-Schmidt (gs_passes times; two passes are "twice is enough", Kahan and Parlett)
// entirely on the device, and its reduction kernels also store the Hessenberg column in
// the step's own pinned host slot.  The host runs one step behind: it enqueues step j,
// then waits for and processes the column of step j-1 (Givens rotations, convergence
// test), so the device does not idle on the host's round trip -- except before a step
// predicted to end the solve, where it waits rather than enqueue a step that would be
// discarded.
bool debug_on();

//
// T is the precision of the Krylov vectors and of the operator, TP that of the V-cycle (a
// float64 basis with the float32 V-cycle is the NC_MIXED fallback, in its own reserve).
template <typename T, typename TP = T>
int fgmres(nc_ctx* c, bool tr, const T* b, T* x, double rtol, int maxit, double* relres, bool* stalled = nullptr) {
  hipStream_t st = c->stream;
  const Scale5<T>* rows = row_scales<T>(c);
  const long n = 2 * c->N, ld = c->ld;
  const int m = c->m;
  constexpr bool split = !std::is_same<T, TP>::value;
  T* V = split ? (T*)c->V64 : (T*)c->V;
  T* Z = split ? (T*)c->Z64 : (T*)c->Z;
  double* dres = c->dres;
  ck(hipMemsetAsync(x, 0, sizeof(T) * n, st));
  // |b| also goes to the pinned slot after the Hessenberg slots; the host reads it with
  // step 0's column rather than waiting for it here
  const double* hb = c->hslots + (size_t)MAXC * HSLOT;
  launch_norm<T>(st, b, n, c->part, dres, c->hslots + (size_t)MAXC * HSLOT);
  *relres = 0.0;
  launch_scale_inv<T>(st, dres, b, V, n);
  double bnorm = -1.0, beta = -1.0;
  bool no_rhs = false;
  int total = 0;
  std::vector<double> H((m + 1) * m), cs(m), sn(m), g(m + 1), y(m);
  const int passes = c->p.gs_passes;   // classical Gram-Schmidt passes per step (1 or 2)
  // enqueue Arnoldi step j: z_j = M^-1 v_j, w = D A z_j, two Gram-Schmidt passes, v_{j+1}
  auto enqueue = [&](int j) {
    T* vj = V + (long)j * ld;
    T* w = V + (long)(j + 1) * ld;
    T* zj = Z + (long)j * ld;
    // v_j arrives unnormalised from step j-1 (its norm is still in dres); step 0's is normal
    if constexpr (std::is_same<T, TP>::value) {
      precondition_pt<T>(c, tr, vj, zj, rows, j > 0 ? dres + 2 * MAXC : nullptr);
    } else {
      // normalise v_j in place and round a copy to the V-cycle's precision; the cycle's
      // result is widened into z_j (kb and kx are free: b and x are float64 here)
      TP* pv = (TP*)c->kb;
      TP* pz = (TP*)c->kx;
      {
        Timed tm(c, TC_VECTOR, (double)(2 * sizeof(T) + sizeof(TP)) * n);
        launch_normalize_copy<T, TP>(st, j > 0 ? dres + 2 * MAXC : nullptr, vj, pv, n);
      }
      precondition_pt<TP>(c, tr, pv, pz, row_scales<TP>(c), nullptr);
      {
        Timed tm(c, TC_VECTOR, (double)(sizeof(T) + sizeof(TP)) * n);
        launch_scale2<TP, T>(st, c->N, pz, zj, 1.0, 1.0);
      }
    }
    apply_pt<T>(c, tr, zj, w, rows);
    // the reductions store the Hessenberg column into the step's pinned slot as well
    double* hs = c->hslots + (size_t)j * HSLOT;
    for (int pass = 0; pass < passes; ++pass) {
      const bool last = pass == passes - 1;
      { Timed tm(c, TC_MDOT, sizeof(T) * (double)(j + 2) * n); launch_mdot<T>(st, V, ld, j + 1, w, n, c->part, dres + pass * MAXC, false, hs + pass * MAXC); }
      { Timed tm(c, TC_MAXPY, sizeof(T) * (double)(j + 3) * n);
        launch_maxpy<T>(st, V, ld, j + 1, dres + pass * MAXC, -1.0, w, n, c->part, last ? dres + 2 * MAXC : nullptr,
                        last ? hs + 2 * MAXC : nullptr); }
    }
    ck(hipEventRecord(c->kev[j], st));
  };
  // relative residuals of the last two processed steps, and whether the next step
  // processed is expected to end the solve
  double res_prev = -1.0, res_prev2 = -1.0;
  auto likely_done = [&]() -> bool {
    if (total + 1 >= maxit) return true;
    if (!(res_prev > 0.0 && res_prev2 > 0.0)) return false;
    return res_prev * (res_prev / res_prev2) <= rtol;
  };
  while (true) {
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int jend = 0;
    bool done = false, stop = false, bad = false;
    // process the column of step j; returns true when the cycle stops after it
    auto process = [&](int j) -> bool {
      ck(hipEventSynchronize(c->kev[j]));
      if (bnorm < 0.0) {   // the solve's first step: |b| arrived with it
        bnorm = hb[0];
        beta = bnorm;
        g[0] = beta;
        if (!(bnorm > 0.0)) {   // zero (x stays 0) or non-finite right-hand side
          no_rhs = true;
          done = true;
          return true;
        }
      }
      const double* hs = c->hslots + (size_t)j * HSLOT;
      for (int i = 0; i <= j; ++i) H[i * m + j] = passes == 2 ? hs[i] + hs[MAXC + i] : hs[i];
      const double hn = hs[2 * MAXC];
      H[(j + 1) * m + j] = hn;
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
      res_prev2 = res_prev;
      res_prev = res;
      if (!std::isfinite(res)) bad = true;
      if (bad || res <= rtol || total >= maxit || hn == 0.0) done = true;
      return done;
    };
    // Step j+1 is enqueued before step j is processed (so the device does not wait for the
    // host), unless step j is predicted to end the solve: then the host waits for step j
    // first, and enqueues step j+1 only if the solve goes on.  The prediction extrapolates
    // the last contraction of the residual; a wrong guess costs one host round trip, a
    // right one the whole discarded step.
    enqueue(0);
    for (int j = 0;; ++j) {
      const bool more = j + 1 < m;
      const bool spec = more && !likely_done();
      if (spec) enqueue(j + 1);
      stop = process(j);
      if (stop || !more) break;
      if (!spec) enqueue(j + 1);
    }
    if (no_rhs) return bnorm == 0.0 ? 0 : -1;
    if (bad) {
      sync(c);
      return -1;
    }
    for (int i = jend - 1; i >= 0; --i) {
      double s = g[i];
      for (int k = i + 1; k < jend; ++k) s -= H[i * m + k] * y[k];
      y[i] = s / H[i * m + i];
    }
    // the coefficients go through the pinned buffer: its last device-to-host use was
    // synchronised, and any later host write to it follows a synchronising fetch
    std::memcpy(c->hbuf, y.data(), sizeof(double) * jend);
    ck(hipMemcpyAsync(dres + 3 * MAXC, c->hbuf, sizeof(double) * jend, hipMemcpyHostToDevice, st));
    launch_maxpy<T>(st, Z, ld, jend, dres + 3 * MAXC, 1.0, x, n, c->part, nullptr);
    if (done) break;
    // a first cycle that has not halved the residual: the preconditioner does not work
    // for this system (undamped block Jacobi diverges on strongly convective blocks); the
    // caller may retry with more damping
    if (stalled && total == jend && *relres > 0.5) {
      *stalled = true;
      return total;
    }
    // restart from the true residual
    apply_pt<T>(c, tr, x, V, rows);
    launch_rsub<T>(st, b, V, n);
    launch_norm<T>(st, V, n, c->part, dres);
    fetch(c, dres, 1);
    beta = c->hbuf[0];
    if (debug_on())
      std::fprintf(stderr, "nc fgmres restart after %d: recurrence %.2e true %.2e\n", total, *relres, beta / bnorm);
    *relres = beta / bnorm;
    if (beta / bnorm <= rtol) break;
    launch_scale_inv<T>(st, dres, V, V, n);
  }
  return total;
}

// Solve of J~ d = r (J~^T d = r when tr) for five-field float64 r and d.  The P and T rows
// of J~ do not involve the velocity, so the velocity rows are eliminated exactly: the
// (P, T) system is solved in the working precision -- by FGMRES on the row-scaled system
// (krylov) or by one V-cycle (an error estimate) -- and the velocity part follows by
// back-substitution through the lumped mass in float64:
//   J~ d = r:    A d_PT = r_PT,               d_u = M^-1 (r_u - C d_PT)
//   J~^T d = r:  d_u = M^-1 r_u,              A^T d_PT = r_PT - C^T d_u
template <typename T>
int reduced_solve(nc_ctx* c, bool tr, const double* r, double* d, bool krylov, double rtol, double* relres) {
  hipStream_t st = c->stream;
  const Level& L0 = c->lev[0];
  const LevelView<double> v64 = view<double>(c, 0);
  const double sp = krylov ? c->krow64.s[3] : 1.0, stt = krylov ? c->krow64.s[4] : 1.0;
  T* kb = (T*)c->kb;
  T* kx = (T*)c->kx;
  const double ubytes = 8.0 * (12 * nn(L0.g) + ne(L0.g));
  const double vbytes = (8.0 + sizeof(T)) * 2 * nn(L0.g);
  if (!tr) {
    Timed tm(c, TC_VECTOR, vbytes);
    launch_pack_pt<T>(st, c->N, r, kb, sp, stt);
  } else {
    { Timed tm(c, TC_UPROJ, ubytes); launch_uprojT<double>(st, v64, r, c->pt64, d, nullptr); }
    { Timed tm(c, TC_VECTOR, vbytes); launch_scale2<double, T>(st, c->N, c->pt64, kb, sp, stt); }
  }
  int its = 0;
  if (krylov) {
    bool stalled = false;
    if (!c->k64) {
      const bool damp = c->p.smooth_omega_fallback > 0.0 && c->p.smooth_omega_fallback < c->omega;
      its = fgmres<T>(c, tr, kb, kx, rtol, c->p.krylov_maxit, relres, damp || c->reserve64 ? &stalled : nullptr);
      if (its < 0) return its;
      if (stalled && damp) {
        stalled = false;
        // switch this context to the fallback damping for good and solve again from zero
        if (debug_on()) std::fprintf(stderr, "nc fgmres stalled (relres %.2e): block-Jacobi damping %g -> %g\n", *relres,
                                     c->omega, c->p.smooth_omega_fallback);
        c->omega = c->p.smooth_omega_fallback;
        const int more = fgmres<T>(c, tr, kb, kx, rtol, c->p.krylov_maxit, relres);
        if (more < 0) return more;
        its += more;
      }
    }
    if constexpr (sizeof(T) < sizeof(double)) {
      // A float32 Krylov solve that ends unconverged: where the V-cycle amplifies a few
      // directions by orders of magnitude (the pressure inside a solid region whose
      // permeability is 1e5 below the fluid's, which the per-field row scales do not see),
      // the float32 rounding of the basis and of the operator is of the size of the
      // residual itself.  With the reserve, the context then keeps float64 Krylov vectors
      // and a float64 operator for good, with the float32 V-cycle as the preconditioner.
      // (a first restart cycle that did not halve the residual, with no stronger damping
      // left to try, takes the same way at once)
      if (c->reserve64 && (c->k64 || stalled || (*relres > rtol && its >= c->p.krylov_maxit))) {
        if (!c->k64 && debug_on())
          std::fprintf(stderr, "nc fgmres float32 unconverged (relres %.2e): float64 Krylov from now on\n", *relres);
        c->k64 = true;
        double* b64 = c->tmp5;   // free during a linear solve
        if (!tr) {
          Timed tm(c, TC_VECTOR, vbytes);
          launch_pack_pt<double>(st, c->N, r, b64, sp, stt);
        } else {
          Timed tm(c, TC_VECTOR, vbytes);
          launch_scale2<double, double>(st, c->N, c->pt64, b64, sp, stt);
        }
        const int more = fgmres<double, T>(c, tr, b64, c->pt64, rtol, c->p.krylov_maxit, relres);
        if (more < 0) return more;
        its += more;
        if (!tr) {
          Timed tm(c, TC_UPROJ, ubytes);
          launch_uproj<double>(st, v64, c->pt64, r, d, nullptr);
        } else {
          Timed tm(c, TC_VECTOR, vbytes);
          launch_unpack_pt<double>(st, L0.g, c->pt64, d);
        }
        return its;
      }
    }
  } else {
    precondition_pt<T>(c, tr, kb, kx, nullptr);
  }
  if (!tr) {
    { Timed tm(c, TC_VECTOR, vbytes); launch_scale2<T, double>(st, c->N, kx, c->pt64, 1.0, 1.0); }
    { Timed tm(c, TC_UPROJ, ubytes); launch_uproj<double>(st, v64, c->pt64, r, d, nullptr); }
  } else {
    Timed tm(c, TC_VECTOR, vbytes);
    launch_unpack_pt<T>(st, L0.g, kx, d);
  }
  return its;
}

// Relative residual, in float64 and with the Krylov row scales, of the (P, T) part of the
// last linear solve J~ d = r (its (P, T) solution is still in pt64).
double pt_true_relres(nc_ctx* c, const double* r) {
  hipStream_t st = c->stream;
  const long n = 2 * c->N;
  double* b64 = c->tmp5;       // D r_PT
  double* w64 = c->tmp5 + n;   // D A d_PT, then D (r_PT - A d_PT)
  launch_pack_pt<double>(st, c->N, r, b64, c->krow64.s[3], c->krow64.s[4]);
  apply_pt<double>(c, false, c->pt64, w64, &c->krow64);
  launch_norm<double>(st, b64, n, c->part, c->dres + 3 * MAXC);
  launch_rsub<double>(st, b64, w64, n);
  launch_norm<double>(st, w64, n, c->part, c->dres + 3 * MAXC + 1);
  ck(hipMemcpyAsync(c->hbuf, c->dres + 3 * MAXC, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
  sync(c);
  return c->hbuf[0] > 0.0 ? c->hbuf[1] / c->hbuf[0] : 0.0;
}

int linear_solve(nc_ctx* c, bool tr, const double* r, double* d, double rtol, double* relres) {
  return c->mixed ? reduced_solve<float>(c, tr, r, d, true, rtol, relres)
                  : reduced_solve<double>(c, tr, r, d, true, rtol, relres);
}

// Per-field error estimate of an approximate solution: e = one V-cycle solve of the
// residual r, returns max_f |e_f| / |x_f| over the fields with |x_f| > 0.
double error_estimate(nc_ctx* c, bool tr, const double* r, const double* x) {
  double dummy = 0.0;
  if (c->mixed) reduced_solve<float>(c, tr, r, c->tmp5, false, 0.0, &dummy);
  else reduced_solve<double>(c, tr, r, c->tmp5, false, 0.0, &dummy);
  launch_field_norms(c->stream, c->tmp5, x, c->N, c->part, c->dres);
  fetch(c, c->dres, 10);
  double worst = 0.0;
  for (int f = 0; f < 5; ++f)
    if (c->hbuf[5 + f] > 0) worst = std::max(worst, c->hbuf[f] / c->hbuf[5 + f]);
  return worst;
}

double norm64(nc_ctx* c, const double* a) {
  launch_norm<double>(c->stream, a, c->n5, c->part, c->dres);
  fetch(c, c->dres, 1);
  return c->hbuf[0];
}

// 2-norm of a five-field vector with the per-field row scales of the equilibrated system,
// from its fetched per-field norms fn[5] or computed
double scaled_from(const nc_ctx* c, const double* fn) {
  double s = 0.0;
  for (int f = 0; f < 5; ++f) {
    const double v = c->rows64.s[f] * fn[f];
    s += v * v;
  }
  return std::sqrt(s);
}
double scaled_norm(nc_ctx* c, const double* a) {
  launch_field_norms(c->stream, a, nullptr, c->N, c->part, c->dres);
  fetch(c, c->dres, 5);
  return scaled_from(c, c->hbuf);
}

// elements carrying the volumetric source on the finest grid
struct BoxRangeCount {
  long count;
};
BoxRangeCount source_count(const nc_ctx* c) {
  const Grid& g = c->lev[0].g;
  const ElemConst<double>& e = c->lev[0].c64;
  const long ni = std::max(0, std::min(e.qi1, g.nx - 1) - std::max(e.qi0, 0) + 1);
  const long nj = std::max(0, std::min(e.qj1, g.ny - 1) - std::max(e.qj0, 0) + 1);
  const long nk = std::max(0, std::min(e.qk1, g.nz - 1) - std::max(e.qk0, 0) + 1);
  return BoxRangeCount{ni * nj * nk};
}

// round-off floor of the scaled residual: 1e-12 of the scaled boundary-flux load
double residual_floor(nc_ctx* c) {
  launch_objective_grad(c->stream, c->lev[0].g, c->patch, c->tmp5);
  double fl = scaled_norm(c, c->tmp5);
  if (c->p.Q != 0.0) {   // the load of the volumetric source: |Q| h^3 per source element
    const BoxRangeCount n = source_count(c);
    fl += fabs(c->p.Q) * std::pow(c->lev[0].h, 3) * std::sqrt((double)n.count) * c->rows64.s[4];
  }
  return 1e-12 * fl;
}

// NC_DEBUG=1 prints the Newton and adjoint iterations to stderr (tracing aid)
bool debug_on() {
  static const bool on = std::getenv("NC_DEBUG") != nullptr;
  return on;
}

// ------------------------------------------------------------------ Newton
int newton(nc_ctx* c, double* s, nc_info* info) {
  hipStream_t st = c->stream;
  const nc_problem& p = c->p;
  const Level& L0 = c->lev[0];
  launch_mask_state(st, L0.g, s);
  compute_row_scales(c);
  const double floor = c->res_floor;
  launch_residual(st, L0.g, L0.c64, c->patch, L0.coef64, s, c->R);
  // merit function of the damped Newton iteration: the residual 2-norm with the per-field
  // row scales (the same root; the scaling keeps the small pressure rows visible)
  double rn = scaled_norm(c, c->R);
  if (!std::isfinite(rn)) return NC_ENAN;
  if (info) {
    for (int f = 0; f < 5; ++f) info->res0[f] = c->hbuf[f];   // per-field norms fetched by scaled_norm
    info->hist_len = 0;
  }
  const double lin_rtol = c->mixed ? p.krylov_rtol_mixed : p.krylov_rtol;
  int status = NC_NOT_CONVERGED;
  int kits = 0, it = 0;
  double relres = 0.0;
  int first_its = 0;
  double rn_last = rn;   // merit before the previous step
  for (it = 0; it < p.newton_maxit; ++it) {
    if (rn <= floor) { status = NC_OK; break; }   // already at the residual's round-off floor
    // inexact-Newton forcing term (Eisenstat and Walker's second choice): the first step
    // is solved only to newton_eta0, later ones to 0.9 (|R_k| / |R_k-1|)^2, never looser
    // than newton_eta0 nor tighter than the Krylov tolerance.  Far from the root the
    // linear solve need not beat the contraction the nonlinearity allows; near it the
    // ratio is small and the Krylov tolerance governs, so the final accuracy is unchanged.
    double eta = lin_rtol;
    if (p.newton_eta0 > lin_rtol) {
      const double q = rn / rn_last;
      eta = it == 0 ? p.newton_eta0 : std::min(p.newton_eta0, std::max(lin_rtol, 0.9 * q * q));
    }
    rn_last = rn;
    // rebuild the preconditioner on the first two steps (the first step moves the state
    // from the guess to near the root) or when the last solve needed many more iterations
    const bool rebuild = it < 2 || !c->hier_valid;
    linearize(c, s, rebuild);
    int its = linear_solve(c, false, c->R, c->d, eta, &relres);
    if (its < 0) return NC_ENAN;
    if (c->mixed && c->reserve64 && !c->k64) {
      // the float32 solve's own residual can hide a float64 residual far above it (its
      // operator's rounding, relative to a correction the V-cycle has amplified); then the
      // step goes on in float64 Krylov, for good
      const double rt = pt_true_relres(c, c->R);
      if (!(rt <= 10.0 * std::max(relres, eta))) {
        if (debug_on()) std::fprintf(stderr, "nc newton %d: float32 solve relres %.2e, float64 %.2e: float64 Krylov\n", it,
                                     relres, rt);
        c->k64 = true;
        const int more = linear_solve(c, false, c->R, c->d, eta, &relres);
        if (more < 0) return NC_ENAN;
        its += more;
      }
    }
    if (it == 1) first_its = its;
    if (it >= 2 && its > 2 * first_its + 4) c->hier_valid = false;
    kits += its;
    // d solves J d = R; the Newton step is -d.  Per-field size of the step relative to
    // the state, taken before the line search, fetched together with the residual of the
    // full step (the first trial of the line search)
    launch_field_norms(st, c->d, s, c->N, c->part, c->dres);
    launch_axpy(st, -1.0, c->d, s, c->strial, c->n5);
    { Timed tm(c, TC_RESIDUAL, 8.0 * (10 * nn(L0.g) + 2 * ne(L0.g))); launch_residual(st, L0.g, L0.c64, c->patch, L0.coef64, c->strial, c->tmp5); }
    launch_field_norms(st, c->tmp5, nullptr, c->N, c->part, c->dres + 16);
    fetch(c, c->dres, 21);
    double step = 0.0, step_pt = 0.0;
    for (int f = 0; f < 5; ++f) {
      const double sf = c->hbuf[5 + f], df = c->hbuf[f];
      const double r = sf > 0 ? df / sf : (df > 0 ? 1.0 : 0.0);
      step = std::max(step, r);
      if (f >= 3) step_pt = std::max(step_pt, r);
    }
    // a step this small in (P, T) is at the round-off level of the root, where the
    // residual norm is noise and no longer orders the iterates: it is taken in full
    const bool tiny = step_pt <= 1e3 * p.newton_step_rtol && relres <= 10.0 * lin_rtol;
    // inexact Newton: after a full step delta solved to relative residual eta, the error
    // left is about eta |delta| + O(|delta|^2); below the step tolerance no further step
    // is needed
    const bool predicted = relres <= 10.0 * lin_rtol && std::max(relres, step_pt) * step_pt <= p.newton_step_rtol;
    double lam = 1.0, rt = scaled_from(c, c->hbuf + 16);
    double fres[5];   // per-field norms of the accepted trial's residual
    for (int f = 0; f < 5; ++f) fres[f] = c->hbuf[16 + f];
    while (true) {
      if (lam < 1.0) {
        launch_axpy(st, -lam, c->d, s, c->strial, c->n5);
        { Timed tm(c, TC_RESIDUAL, 8.0 * (10 * nn(L0.g) + 2 * ne(L0.g))); launch_residual(st, L0.g, L0.c64, c->patch, L0.coef64, c->strial, c->tmp5); }
        rt = scaled_norm(c, c->tmp5);
        for (int f = 0; f < 5; ++f) fres[f] = c->hbuf[f];
      }
      if (!std::isfinite(rt)) return NC_ENAN;
      if (rt <= rn || rt <= floor || tiny || lam < 1.0 / 64) break;
      lam *= 0.5;
    }
    ck(hipMemcpyAsync(s, c->strial, sizeof(double) * c->n5, hipMemcpyDeviceToDevice, st));
    std::swap(c->R, c->tmp5);
    if (info && info->hist_len < NC_HIST_MAX) {
      info->hist_krylov[info->hist_len] = its;
      for (int f = 0; f < 5; ++f) info->hist_res[info->hist_len][f] = fres[f];
      ++info->hist_len;
    }
    const double rn_prev = rn;
    rn = rt;
    // converged: a full step below the step tolerance in every field, a residual at the
    // floor, or a tiny (P, T) step that no longer halves the residual (the iteration has
    // stagnated at the float64 round-off of the root; the velocity rows, a small
    // difference of large pressure and buoyancy terms, sit above the step tolerance there)
    if (debug_on())
      std::fprintf(stderr, "nc newton %d: krylov %d relres %.2e lam %g step %.2e step_pt %.2e merit %.3e -> %.3e floor %.2e\n",
                   it, its, relres, lam, step, step_pt, rn_prev, rn, floor);
    // (a small step from a linear solve that missed its tolerance says nothing about the
    // root: the step tests need the solve to have reached it)
    const bool solved = relres <= 10.0 * eta;
    if (lam == 1.0 && ((solved && step <= p.newton_step_rtol) || rn <= floor || predicted || (tiny && rn > 0.5 * rn_prev))) {
      status = NC_OK;
      ++it;
      break;
    }
  }
  if (info) {
    info->newton_its = it;
    info->krylov_its = kits;
    info->refine_its = 0;
    info->levels = c->L;
    info->krylov_f64 = c->k64 ? 1 : 0;
    info->rel_res = relres;
    launch_field_norms(st, c->R, nullptr, c->N, c->part, c->dres);
    fetch(c, c->dres, 5);
    for (int f = 0; f < 5; ++f) info->res[f] = c->hbuf[f];
  }
  return status;
}

// ------------------------------------------------------------------ adjoint
int adjoint(nc_ctx* c, const double* s, const double* rhs, double* lam, nc_info* info) {
  hipStream_t st = c->stream;
  const nc_problem& p = c->p;
  const Level& L0 = c->lev[0];
  linearize(c, s, !c->hier_valid);
  compute_row_scales(c);
  ck(hipMemcpyAsync(c->ra, rhs, sizeof(double) * c->n5, hipMemcpyDeviceToDevice, st));
  launch_mask_state(st, L0.g, c->ra);
  const double bn = scaled_norm(c, c->ra);
  if (!std::isfinite(bn)) return NC_ENAN;
  if (info) {
    for (int f = 0; f < 5; ++f) info->res0[f] = c->hbuf[f];
    for (int f = 0; f < 5; ++f) info->res[f] = c->hbuf[f];
    info->hist_len = 0;
    info->newton_its = info->krylov_its = info->refine_its = 0;
    info->levels = c->L;
    info->krylov_f64 = c->k64 ? 1 : 0;
    info->rel_res = bn == 0.0 ? 0.0 : 1.0;
  }
  ck(hipMemsetAsync(lam, 0, sizeof(double) * c->n5, st));
  if (bn == 0.0) return NC_OK;
  const double lin_rtol = c->mixed ? p.krylov_rtol_mixed : std::min(p.krylov_rtol, p.adjoint_rtol);
  int kits = 0, ref = 0, status = NC_NOT_CONVERGED;
  double relres = 0.0, rel = 1.0;
  // r = rhs - J^T lam, refined in float64 until the relative residual meets adjoint_rtol
  ck(hipMemcpyAsync(c->R, c->ra, sizeof(double) * c->n5, hipMemcpyDeviceToDevice, st));
  double rel_prev = 1.0;
  for (ref = 0; ref < 20; ++ref) {
    // float32 inner solves: the first to krylov_rtol_mixed, later ones to the reduction
    // still needed (with a factor 2 margin), not below what float32 sustains
    const double tol = c->mixed ? std::min(lin_rtol, std::max(1e-6, 0.5 * p.adjoint_rtol / rel)) : lin_rtol;
    const int its = linear_solve(c, true, c->R, c->d, tol, &relres);
    if (its < 0) return NC_ENAN;
    kits += its;
    launch_axpy(st, 1.0, c->d, lam, lam, c->n5);
    // per-field norms of lambda and of the new residual r = rhs - J^T lambda, one fetch
    launch_field_norms(st, lam, nullptr, c->N, c->part, c->dres);
    launch_jtw5<double>(st, view<double>(c, 0), lam, c->tmp5);
    launch_axpy(st, -1.0, c->tmp5, c->ra, c->R, c->n5);
    launch_field_norms(st, c->R, nullptr, c->N, c->part, c->dres + 16);
    fetch(c, c->dres, 21);
    // weight the (P, T) rows of later sweeps by 1 / |lambda_f|, relative to T, so that the
    // Krylov residual measures each field's relative error (the adjoint of the pressure
    // rows is small and otherwise under-resolved)
    {
      const double lp = c->hbuf[3], lt = c->hbuf[4];
      if (lp > 0 && lt > 0) {
        const double wgt = std::min(1e4, std::max(1e-4, lt / lp));
        c->krow64.s[3] = c->rows64.s[3] * wgt;
        c->krow32.s[3] = (float)c->krow64.s[3];
        if (debug_on()) std::fprintf(stderr, "nc adjoint sweep %d: P-row weight %.3e\n", ref, wgt);
      }
    }
    rel = scaled_from(c, c->hbuf + 16) / bn;
    if (!std::isfinite(rel)) return NC_ENAN;
    if (info && info->hist_len < NC_HIST_MAX) {
      info->hist_krylov[info->hist_len] = its;
      for (int f = 0; f < 5; ++f) info->hist_res[info->hist_len][f] = c->hbuf[16 + f];
      ++info->hist_len;
    }
    // converged when the (row-scaled) residual is small and one preconditioner application
    // predicts a per-field relative error below the same tolerance; when refinement stops
    // gaining (round-off floor) the error estimate alone decides
    const bool stalled = rel > 0.25 * rel_prev;
    if (rel <= p.adjoint_rtol || stalled) {
      const double est = error_estimate(c, true, c->R, lam);
      if (debug_on()) std::fprintf(stderr, "nc adjoint sweep %d: krylov %d rel %.2e est %.2e\n", ref, its, rel, est);
      if (est <= 10.0 * p.adjoint_rtol || (stalled && est <= 1e2 * p.adjoint_rtol)) {
        status = NC_OK;
        ++ref;
        break;
      }
      if (stalled && c->mixed && c->reserve64 && !c->k64) {
        // float32 inner solves no longer reduce the float64 residual: float64 Krylov from here
        if (debug_on()) std::fprintf(stderr, "nc adjoint sweep %d: refinement stalled, float64 Krylov\n", ref);
        c->k64 = true;
      } else if (stalled && ref > 2) {
        ++ref;
        break;
      }
    }
    rel_prev = rel;
  }
  if (info) {
    info->newton_its = 0;
    info->krylov_its = kits;
    info->refine_its = ref;
    info->levels = c->L;
    info->krylov_f64 = c->k64 ? 1 : 0;
    info->rel_res = rel;
    launch_field_norms(st, c->R, nullptr, c->N, c->part, c->dres);
    fetch(c, c->dres, 5);
    for (int f = 0; f < 5; ++f) info->res[f] = c->hbuf[f];
  }
  return status;
}

template <class F>
int guarded(F f) {
  try {
    return f();
  } catch (const HipError& e) {
    std::fprintf(stderr, "nc: HIP error %d (%s)\n", (int)e.e, hipGetErrorString(e.e));
    return NC_EHIP;
  } catch (const std::bad_alloc&) {
    return NC_ENOMEM;
  } catch (...) {
    return NC_EINVAL;
  }
}

double now() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace

// ------------------------------------------------------------------ static scratch
// Scratch of nc_dense_inverse_noalloc: 2 n doubles (step columns), then 2 n ints (pivot
// rows), for n up to NC_DENSE_MAX.  Each GPU holds its own copy until the process ends.
static_assert(2 * NC_DENSE_MAX * (sizeof(double) + sizeof(int)) <= NC_DENSE_NOALLOC_SCRATCH, "scratch too small");
static __device__ __align__(256) unsigned char scratch[NC_DENSE_NOALLOC_SCRATCH];

namespace {

// Device address of `scratch` on the current device, looked up once per device (host code
// must not pass the array's name itself: on the host it is only a stand-in symbol).
unsigned char* scratch_ptr() {
  static std::mutex mu;
  static std::vector<unsigned char*> ptrs;
  int dev = 0;
  ck(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(mu);
  if ((int)ptrs.size() <= dev) ptrs.resize(dev + 1, nullptr);
  if (!ptrs[dev]) {
    void* p = nullptr;
    ck(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) throw HipError{hipErrorInvalidSymbol};
    ptrs[dev] = (unsigned char*)p;
  }
  return ptrs[dev];
}

}  // namespace

// ====================================================================== C ABI
extern "C" {

void nc_problem_default(nc_problem* p, int nx, int ny, int nz) {
  std::memset(p, 0, sizeof(*p));
  p->nx = nx; p->ny = ny; p->nz = nz;
  p->h = 1.0 / nx;
  p->rho0 = p->mu = p->cp = p->g0 = 1.0;
  p->alpha = 1e3;
  p->k_f = 1.0; p->k_s = 100.0;
  p->kappa_f = 0.00513; p->kappa_s = 1e-4;
  p->q_c = 8.0; p->q_p = 8.0;
  p->q_h = 1.0;
  p->patch_x0 = 0.375; p->patch_x1 = 0.625; p->patch_y0 = 0.125; p->patch_y1 = 0.375;
  p->Q = 0.0;
  p->filter_radius = 0.0;
  p->precision = NC_FP64;
  p->levels = 0;
  p->newton_step_rtol = 1e-11;
  p->krylov_rtol = 1e-7;
  p->krylov_rtol_mixed = 6e-5;
  p->gs_passes = 1;
  p->coarse_tail = 1;
  p->adjoint_rtol = 3e-11;
  p->newton_maxit = 30;
  p->newton_eta0 = 3e-3;
  p->krylov_restart = 24;
  p->krylov_maxit = 400;
  p->smooth_pre = 2;
  p->smooth_post = 2;
  p->smooth_omega = 1.0;
  p->smooth_omega_fallback = 0.7;
  p->f64_krylov_fallback = 0;
  p->smooth_pre_coarse = 1;
  p->smooth_post_coarse = 1;
  p->filter_kind = NC_FILTER_CONE;
  p->sym_x = p->sym_y = 0;
  for (int d = 0; d < 6; ++d) p->q_box[d] = p->solid_box[d] = p->design_box[d] = 0.0;
}

size_t nc_workspace_bytes(const nc_problem* p) {
  if (!valid_problem(p)) return 0;
  nc_ctx tmp;
  tmp.p = *p;
  return carve(&tmp, nullptr);
}

// Frees what a context holds besides the caller's workspace, after its side stream drains.
static void release(nc_ctx* c) {
  for (hipStream_t s : {c->side, c->side2})
    if (s) {
      (void)hipStreamSynchronize(s);
      (void)hipStreamDestroy(s);
    }
  for (hipEvent_t e : {c->fork, c->join, c->join2})
    if (e) (void)hipEventDestroy(e);
  for (auto& r : c->setup_ev)
    for (hipEvent_t e : r)
      if (e) (void)hipEventDestroy(e);
  for (auto& e : c->ev) (void)hipEventDestroy(e);
  for (auto& e : c->kev)
    if (e) (void)hipEventDestroy(e);
  if (c->hbuf) (void)hipHostFree(c->hbuf);
  if (c->hslots) (void)hipHostFree(c->hslots);
  delete c;
}

int nc_create(const nc_problem* p, void* workspace_dev, size_t bytes, void* stream, nc_ctx** out) {
  if (!out || !valid_problem(p) || !workspace_dev) return NC_EINVAL;
  *out = nullptr;
  return guarded([&]() {
    nc_ctx* c = new nc_ctx();
    c->p = *p;
    if (c->p.h <= 0) c->p.h = 1.0 / p->nx;
    const size_t need = carve(c, nullptr);
    if (bytes < need) {
      delete c;
      return NC_ENOMEM;
    }
    char* base = (char*)workspace_dev;
    const size_t mis = (size_t)((uintptr_t)base % ALIGN);
    if (mis) base += ALIGN - mis;
    carve(c, base);
    c->ws_base = base;
    c->ws_need = need;
    c->stream = (hipStream_t)stream;
    c->patch = Patch{c->p.q_h, c->p.patch_x0, c->p.patch_x1, c->p.patch_y0, c->p.patch_y1, c->p.h};
    c->design_set = false;
    c->hier_valid = false;
    c->omega = c->p.smooth_omega;
    c->k64 = false;
    c->timing = false;
    c->ev_used = 0;
    c->join_pending = c->join2_pending = false;
    c->kev.resize(MAXC);
    for (auto& e : c->kev) e = nullptr;
    c->side = c->side2 = nullptr;
    c->fork = c->join = c->join2 = nullptr;
    c->hslots = c->hbuf = nullptr;
    c->setup_used = 0;
    c->setup_s = 0.0;
    for (auto& r : c->setup_ev)
      for (hipEvent_t& e : r) e = nullptr;
    bool ok = true;
    for (auto& r : c->setup_ev)
      for (hipEvent_t& e : r) ok = ok && hipEventCreate(&e) == hipSuccess;
    for (auto& e : c->kev) ok = ok && hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess;
    ok = ok && hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) == hipSuccess;
    ok = ok && hipStreamCreateWithFlags(&c->side2, hipStreamNonBlocking) == hipSuccess;
    ok = ok && hipEventCreateWithFlags(&c->fork, hipEventDisableTiming) == hipSuccess;
    ok = ok && hipEventCreateWithFlags(&c->join, hipEventDisableTiming) == hipSuccess;
    ok = ok && hipEventCreateWithFlags(&c->join2, hipEventDisableTiming) == hipSuccess;
    ok = ok && hipHostMalloc((void**)&c->hslots, sizeof(double) * (MAXC + 1) * HSLOT, hipHostMallocDefault) == hipSuccess;
    ok = ok && hipHostMalloc((void**)&c->hbuf, sizeof(double) * 4 * MAXC, hipHostMallocDefault) == hipSuccess;
    if (!ok) {
      release(c);
      return NC_EHIP;
    }
    *out = c;
    return NC_OK;
  });
}

int nc_set_problem(nc_ctx* c, const nc_problem* p) {
  if (!c || !valid_problem(p)) return NC_EINVAL;
  return guarded([&]() {
    nc_ctx tmp;
    tmp.p = *p;
    if (tmp.p.h <= 0) tmp.p.h = 1.0 / p->nx;
    const size_t need = carve(&tmp, nullptr);
    bool same = need == c->ws_need && tmp.L == c->L && tmp.pde == c->pde && tmp.mixed == c->mixed && tmp.m == c->m &&
                tmp.dense == c->dense;
    for (int l = 0; same && l < c->L; ++l)
      same = tmp.lev[l].g.nx == c->lev[l].g.nx && tmp.lev[l].g.ny == c->lev[l].g.ny && tmp.lev[l].g.nz == c->lev[l].g.nz;
    if (!same) return NC_EINVAL;
    // the setup streams may still read what the new parameters replace
    join_coarse(c);
    join_levels(c);
    c->p = tmp.p;
    carve(c, c->ws_base);   // the same layout: recomputes the level constants and regions only
    c->patch = Patch{c->p.q_h, c->p.patch_x0, c->p.patch_x1, c->p.patch_y0, c->p.patch_y1, c->p.h};
    c->omega = c->p.smooth_omega;
    c->k64 = false;
    c->design_set = false;
    c->hier_valid = false;
    c->rows_valid = false;
    return NC_OK;
  });
}

int nc_mma_update(nc_ctx* c, int iter, double* x, const double* dfdx, double g, const double* dgdx, double move,
                  double* state, double* lambda) {
  if (!c || !x || !dfdx || !dgdx || !state || iter < 1 || !(move > 0.0) || !std::isfinite(g)) return NC_EINVAL;
  if (c->n_design == 0) return NC_EINVAL;
  return guarded([&]() {
    hipStream_t st = c->stream;
    const Grid& gr = c->lev[0].g;
    launch_mma_prepare(st, gr, c->reg, iter, move, 0.0, 1.0, x, dfdx, dgdx, state, c->part, c->dres);
    fetch(c, c->dres, 1);
    const double b = c->hbuf[0] - g;   // the approximation at x equals g there
    // constraint approximation minus b at MMA_CAND multipliers
    auto eval = [&](const MmaCand& cand, double* con) {
      launch_mma_dual(st, gr, c->reg, cand, state, c->part, c->dres);
      fetch(c, c->dres, MMA_CAND);
      for (int k = 0; k < MMA_CAND; ++k) con[k] = c->hbuf[k] - b;
    };
    double con[MMA_CAND];
    MmaCand cand;
    // first pass: 0, a geometric grid over 1e-30 .. 1e30, and the limit lambda -> inf
    cand.v[0] = 0.0;
    for (int k = 1; k < MMA_CAND - 1; ++k) cand.v[k] = std::pow(10.0, -30.0 + 60.0 * (k - 1) / (MMA_CAND - 3));
    cand.v[MMA_CAND - 1] = INFINITY;
    eval(cand, con);
    double lam;
    if (!std::isfinite(con[0]) || !std::isfinite(con[MMA_CAND - 1])) throw HipError{hipErrorUnknown};
    if (con[0] <= 0.0) {
      lam = 0.0;
    } else if (con[MMA_CAND - 1] > 0.0) {
      lam = INFINITY;   // no point of the box satisfies the approximation: reduce it most
    } else {
      // bracket [lo, hi]: con(lo) > 0 >= con(hi); narrowed geometrically while it spans
      // more than a factor 2, then linearly, to a relative width of 1e-15
      int k = 1;
      while (con[k] > 0.0) ++k;
      double lo = cand.v[k - 1], hi = cand.v[k];
      for (int pass = 0; pass < 60 && hi - lo > 1e-15 * hi; ++pass) {
        const bool geo = lo > 0.0 && hi > 2.0 * lo;
        const double l0 = lo > 0.0 ? lo : hi * 1e-30;
        for (int m = 0; m < MMA_CAND; ++m) {
          const double t = (m + 1.0) / (MMA_CAND + 1.0);
          cand.v[m] = geo || lo == 0.0 ? l0 * std::pow(hi / l0, t) : lo + (hi - lo) * t;
        }
        eval(cand, con);
        double nlo = lo, nhi = hi;
        for (int m = 0; m < MMA_CAND; ++m) {
          if (con[m] > 0.0) nlo = cand.v[m];
          else { nhi = cand.v[m]; break; }
        }
        lo = nlo;
        hi = nhi;
      }
      lam = hi;
    }
    launch_mma_apply(st, gr, c->reg, iter, lam, x, state);
    ck(hipGetLastError());
    sync(c);
    if (lambda) *lambda = lam;
    return NC_OK;
  });
}

int nc_destroy(nc_ctx* c) {
  if (!c) return NC_EINVAL;
  (void)hipStreamSynchronize(c->stream);
  release(c);
  return NC_OK;
}

const char* nc_status_string(int s) {
  switch (s) {
    case NC_OK: return "ok";
    case NC_NOT_CONVERGED: return "not converged";
    case NC_EINVAL: return "invalid argument";
    case NC_ENOMEM: return "workspace too small";
    case NC_EHIP: return "HIP runtime error";
    case NC_ENAN: return "non-finite value encountered";
    default: return "unknown status";
  }
}

int nc_set_design(nc_ctx* c, const double* x) {
  if (!c || !x) return NC_EINVAL;
  return guarded([&]() {
    hipStream_t st = c->stream;
    const nc_problem& p = c->p;
    Level& L0 = c->lev[0];
    // the setup streams may still read the coefficients of the previous design
    join_coarse(c);
    join_levels(c);
    apply_filter(c, x, c->gamma, false);
    if (c->regions) launch_passive(st, L0.g, c->reg, c->gamma);
    launch_ramp(st, c->E, c->gamma, p.k_f, p.k_s, p.q_c, p.kappa_f, p.kappa_s, p.q_p, L0.coef64, L0.coef32, c->dk,
                c->dkap);
    for (int l = 1; l < c->L; ++l) {
      launch_average_coef<double>(st, c->lev[l - 1].g, c->lev[l].g, c->lev[l - 1].coef64, c->lev[l].coef64);
      launch_average_coef<float>(st, c->lev[l - 1].g, c->lev[l].g, c->lev[l - 1].coef32, c->lev[l].coef32);
    }
    ck(hipGetLastError());
    c->design_set = true;
    c->hier_valid = false;
    c->rows_valid = false;
    return NC_OK;
  });
}

int nc_get_gamma(nc_ctx* c, double* gamma) {
  if (!c || !gamma || !c->design_set) return NC_EINVAL;
  return guarded([&]() {
    ck(hipMemcpyAsync(gamma, c->gamma, sizeof(double) * c->E, hipMemcpyDeviceToDevice, c->stream));
    return NC_OK;
  });
}

int nc_filter_apply(nc_ctx* c, int transpose, const double* x, double* y) {
  if (!c || !x || !y || x == y) return NC_EINVAL;
  return guarded([&]() {
    apply_filter(c, x, y, transpose != 0);
    ck(hipGetLastError());
    return NC_OK;
  });
}

int nc_residual(nc_ctx* c, const double* s, double* r) {
  if (!c || !s || !r || !c->design_set) return NC_EINVAL;
  return guarded([&]() {
    const Level& L0 = c->lev[0];
    launch_residual(c->stream, L0.g, L0.c64, c->patch, L0.coef64, s, r);
    ck(hipGetLastError());
    return NC_OK;
  });
}

int nc_linearize(nc_ctx* c, const double* s) {
  if (!c || !s || !c->design_set) return NC_EINVAL;
  return guarded([&]() {
    linearize(c, s, false);
    ck(hipGetLastError());
    return NC_OK;
  });
}

int nc_jac_apply(nc_ctx* c, const double* v, double* y) {
  if (!c || !v || !y) return NC_EINVAL;
  return guarded([&]() { launch_jv5<double>(c->stream, view<double>(c, 0), v, y); ck(hipGetLastError()); return NC_OK; });
}
int nc_jacT_apply(nc_ctx* c, const double* w, double* y) {
  if (!c || !w || !y) return NC_EINVAL;
  return guarded([&]() { launch_jtw5<double>(c->stream, view<double>(c, 0), w, y); ck(hipGetLastError()); return NC_OK; });
}
int nc_jac_apply_f32(nc_ctx* c, const float* v, float* y) {
  if (!c || !v || !y) return NC_EINVAL;
  return guarded([&]() { launch_jv5<float>(c->stream, view<float>(c, 0), v, y); ck(hipGetLastError()); return NC_OK; });
}
int nc_jacT_apply_f32(nc_ctx* c, const float* w, float* y) {
  if (!c || !w || !y) return NC_EINVAL;
  return guarded([&]() { launch_jtw5<float>(c->stream, view<float>(c, 0), w, y); ck(hipGetLastError()); return NC_OK; });
}

int nc_solve_state(nc_ctx* c, double* s, nc_info* info) {
  if (!c || !s || !c->design_set) return NC_EINVAL;
  return guarded([&]() {
    const double t0 = now();
    c->setup_s = 0.0;
    c->setup_used = 0;   // rebuilds recorded by earlier calls are not this call's
    if (info) std::memset(info, 0, sizeof(*info));
    const int r = newton(c, s, info);
    sync(c);
    setup_drain(c);
    if (info) {
      info->t_total = now() - t0;
      info->t_setup = c->setup_s;
      info->t_solve = info->t_total - info->t_setup;
    }
    return r;
  });
}

int nc_objective(nc_ctx* c, const double* s, double* f) {
  if (!c || !s || !f || !c->design_set) return NC_EINVAL;
  return guarded([&]() {
    launch_objective(c->stream, c->lev[0].g, c->patch, c->lev[0].c64, c->lev[0].coef64, s, c->part, c->dres);
    fetch(c, c->dres, 1);
    *f = c->hbuf[0];
    return NC_OK;
  });
}

int nc_objective_grad(nc_ctx* c, const double* s, double* g) {
  if (!c || !g) return NC_EINVAL;
  if (c->p.Q != 0.0 && !s) return NC_EINVAL;   // the volumetric part depends on the state
  return guarded([&]() {
    const Level& L0 = c->lev[0];
    launch_objective_grad(c->stream, L0.g, c->patch, g);
    if (c->p.Q != 0.0) {
      launch_objective_grad_q(c->stream, L0.g, L0.c64, L0.coef64, s, g);
      launch_mask_state(c->stream, L0.g, g);
    }
    ck(hipGetLastError());
    return NC_OK;
  });
}

int nc_objective_sensitivity(nc_ctx* c, const double* s, const double* lam, double* dfdx, double* dfdgamma) {
  if (!c || !s || !lam || !dfdx || !c->design_set) return NC_EINVAL;
  return guarded([&]() {
    hipStream_t st = c->stream;
    const Level& L0 = c->lev[0];
    double* g = dfdgamma ? dfdgamma : c->sens;
    launch_sensitivity(st, L0.g, L0.c64, L0.coef64, c->dk, c->dkap, s, lam, g);
    if (c->p.Q != 0.0) launch_objective_dgamma(st, L0.g, L0.c64, L0.coef64, c->dkap, s, g);
    pull_back(c, g, dfdx);
    ck(hipGetLastError());
    return NC_OK;
  });
}

int nc_volume(nc_ctx* c, double* frac, double* dgdx) {
  if (!c || !frac || !c->design_set) return NC_EINVAL;
  if (c->n_design == 0) return NC_EINVAL;
  return guarded([&]() {
    hipStream_t st = c->stream;
    const Grid& g = c->lev[0].g;
    if (dgdx) {
      launch_design_mask(st, g, c->reg, c->sens, true, 1.0 / (double)c->n_design);
      apply_filter(c, c->sens, dgdx, true);
      launch_design_mask(st, g, c->reg, dgdx, false, 0.0);
    }
    launch_design_sum(st, g, c->reg, c->gamma, c->part, c->dres);
    fetch(c, c->dres, 1);
    *frac = c->hbuf[0] / (double)c->n_design;
    return NC_OK;
  });
}

int nc_solve_adjoint(nc_ctx* c, const double* s, const double* rhs, double* lam, nc_info* info) {
  if (!c || !s || !rhs || !lam || !c->design_set) return NC_EINVAL;
  return guarded([&]() {
    const double t0 = now();
    c->setup_s = 0.0;
    c->setup_used = 0;   // rebuilds recorded by earlier calls are not this call's
    if (info) std::memset(info, 0, sizeof(*info));
    const int r = adjoint(c, s, rhs, lam, info);
    sync(c);
    setup_drain(c);
    if (info) {
      info->t_total = now() - t0;
      info->t_setup = c->setup_s;
      info->t_solve = info->t_total - info->t_setup;
    }
    return r;
  });
}

int nc_sensitivity(nc_ctx* c, const double* s, const double* lam, double* dfdx, double* dfdgamma) {
  if (!c || !s || !lam || !dfdx || !c->design_set) return NC_EINVAL;
  return guarded([&]() {
    hipStream_t st = c->stream;
    const Level& L0 = c->lev[0];
    double* g = dfdgamma ? dfdgamma : c->sens;
    launch_sensitivity(st, L0.g, L0.c64, L0.coef64, c->dk, c->dkap, s, lam, g);
    pull_back(c, g, dfdx);
    ck(hipGetLastError());
    return NC_OK;
  });
}

int nc_set_timing(nc_ctx* c, int enable) {
  if (!c) return NC_EINVAL;
  return guarded([&]() {
    if (enable && c->ev.empty()) {
      c->ev.resize(TIMER_EVENTS);
      c->ev_class.resize(TIMER_EVENTS / 2);
      c->ev_bytes.resize(TIMER_EVENTS / 2);
      for (auto& e : c->ev) ck(hipEventCreate(&e));
    }
    if (c->timing) timing_flush(c);
    c->timing = enable != 0 && !c->ev.empty();
    c->ev_used = 0;
    for (int k = 0; k < TC_COUNT; ++k) { c->t_ms[k] = 0.0; c->t_cnt[k] = 0; c->t_bytes[k] = 0.0; }
    return NC_OK;
  });
}

int nc_get_timing(nc_ctx* c, double* ms, long* counts, double* bytes, int n) {
  if (!c || !ms || !counts || n < 1) return NC_EINVAL;
  return guarded([&]() {
    timing_flush(c);
    for (int k = 0; k < n; ++k) {
      ms[k] = k < TC_COUNT ? c->t_ms[k] : 0.0;
      counts[k] = k < TC_COUNT ? c->t_cnt[k] : 0;
      if (bytes) bytes[k] = k < TC_COUNT ? c->t_bytes[k] : 0.0;
    }
    return TC_COUNT;
  });
}

int nc_cone_filter(int nx, int ny, int nz, double radius, const double* x, double* y, int transpose, void* stream) {
  if (nx < 1 || ny < 1 || nz < 1 || !x || !y) return NC_EINVAL;
  if (transpose && radius > 0) return NC_EINVAL;   // the transpose needs a temporary; use a context
  return guarded([&]() {
    launch_cone_filter((hipStream_t)stream, Grid{nx, ny, nz}, radius, x, y, false, nullptr);
    ck(hipGetLastError());
    return NC_OK;
  });
}

int nc_precondition(nc_ctx* c, int transpose, const double* s, const double* v, double* z) {
  if (!c || !s || !v || !z || !c->design_set) return NC_EINVAL;
  return guarded([&]() {
    linearize(c, s, true);
    hipStream_t st = c->stream;
    if (c->mixed) {
      launch_scale2<double, float>(st, c->N, v, (float*)c->kb, 1.0, 1.0);
      precondition_pt<float>(c, transpose != 0, (float*)c->kb, (float*)c->kx, nullptr);
      launch_scale2<float, double>(st, c->N, (const float*)c->kx, z, 1.0, 1.0);
    } else {
      launch_scale2<double, double>(st, c->N, v, (double*)c->kb, 1.0, 1.0);
      precondition_pt<double>(c, transpose != 0, (double*)c->kb, (double*)c->kx, nullptr);
      launch_scale2<double, double>(st, c->N, (const double*)c->kx, z, 1.0, 1.0);
    }
    ck(hipGetLastError());
    return NC_OK;
  });
}

int nc_dense_inverse(double* a, int n, int* iwork, double* dwork, void* stream) {
  if (n < 1 || n > NC_DENSE_MAX || !a || !iwork || !dwork) return NC_EINVAL;
  return guarded([&]() {
    hipStream_t st = (hipStream_t)stream;
    launch_gauss_jordan(st, a, n, iwork, dwork);
    launch_dense_transpose(st, a, a + (size_t)n * n, n);
    ck(hipGetLastError());
    return NC_OK;
  });
}

int nc_dense_inverse_noalloc(double* a, int n, void* stream) {
  if (n < 1 || n > NC_DENSE_MAX || !a) return NC_EINVAL;
  return guarded([&]() {
    unsigned char* base = scratch_ptr();
    double* dwork = (double*)base;
    int* iwork = (int*)(base + 2 * (size_t)NC_DENSE_MAX * sizeof(double));
    hipStream_t st = (hipStream_t)stream;
    launch_gauss_jordan(st, a, n, iwork, dwork);
    launch_dense_transpose(st, a, a + (size_t)n * n, n);
    ck(hipGetLastError());
    return NC_OK;
  });
}

}  // extern "C"
