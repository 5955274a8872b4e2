// Host-side launchers of the solver's HIP kernels.  All launches are asynchronous on
// the given stream; device pointers only.
#pragma once

#include "common.hpp"

namespace nc {

enum ApplyMode { MODE_STORE = 0, MODE_RESID = 1, MODE_SMOOTH = 2 };

// ---- operator kernels (z-march over element columns, deterministic node accumulation)
// r = R~(s), float64, five fields per node (row a2)
void launch_residual(hipStream_t st, const Grid& g, const ElemConst<double>& c, const Patch& patch,
                     const double* coef, const double* s, double* r);
// y = J~ x (five fields) at the level's linearisation (row a4)
template <typename T>
void launch_jv5(hipStream_t st, const LevelView<T>& L, const T* x, T* y, const Scale5<T>* rows = nullptr);
// y = J~^T w (five fields) (row a5)
template <typename T>
void launch_jtw5(hipStream_t st, const LevelView<T>& L, const T* w, T* y, const Scale5<T>* rows = nullptr);
// y = D A x on the finest grid, A the (P, T) block of J~ (A^T when transposed), D the
// row scales rows->s[3], s[4] (identity when null): the operator of the Krylov solve
template <typename T>
void launch_pt_store(hipStream_t st, const LevelView<T>& L, bool transpose, const T* x, T* y, const Scale5<T>* rows);
// Two-field (P, T) operator of a multigrid level: y = A x, r = b - A x, or one damped
// block-Jacobi sweep y = x + omega D^-1 (b - A x); transpose selects A^T.
template <typename T>
void launch_pt_apply(hipStream_t st, const LevelView<T>& L, bool transpose, int mode, const T* x, const T* b,
                     T* y, T omega, bool fine);
// The bottom of a V-cycle in one workgroup, for a level L small enough (tail_cycle_fits)
// whose next level gc is the dense coarsest: from the residual ru of the level gu above,
// restriction into L with the first damped block-Jacobi step, npre - 1 further sweeps,
// residual, restriction to gc, x = ainv b there (ainv: the inverse, or its transpose for
// the transposed cycle), prolongation, npost sweeps, and xu += P x on gu.
template <typename T>
bool tail_cycle_fits(const Grid& gu, const Grid& g, const Grid& gc);
template <typename T>
void launch_tail_cycle(hipStream_t st, const Grid& gu, const T* ru, T* xu, const LevelView<T>& L, const Grid& gc,
                       const double* ainv, bool transpose, T omega, int npre, int npost);
// Inverse 2x2 (P, T) node blocks of the level Jacobian into dinv [N][4].
template <typename T>
void launch_diag_inverse(hipStream_t st, const LevelView<T>& L, T* dinv, bool fine);
// Preconditioner pieces coupling the velocity rows (block-triangular structure):
//   forward: z = [ (r_u - C x)/M ; x ] with x the (P, T) correction (constrained dofs: z = r)
// (r5 is divided by the row scales `rows` on input when given)
template <typename T>
void launch_uproj(hipStream_t st, const LevelView<T>& L, const T* x_pt, const T* r5, T* z5, const Scale5<T>* rows = nullptr);
//   transpose: z_u = r_u / M, b = r_PT - C^T z_u (masked)
template <typename T>
void launch_uprojT(hipStream_t st, const LevelView<T>& L, const T* r5, T* b_pt, T* z5, const Scale5<T>* rows = nullptr);

// ---- multigrid transfers and setup
template <typename T>
// bc = P^T rf (constrained coarse dofs zero); with dinv also xc = omega D^-1 bc (D^-T when
// transposed), the first block-Jacobi step of the coarse level from a zero guess
void launch_restrict(hipStream_t st, const Grid& fine, const Grid& coarse, const T* rf, T* bc, const T* dinv,
                     bool transpose, T omega, T* xc);
template <typename T>
void launch_prolong_add(hipStream_t st, const Grid& fine, const Grid& coarse, const T* xc, T* xf);
template <typename T>
void launch_inject_state(hipStream_t st, const Grid& fine, const Grid& coarse, const T* sf, T* sc);
template <typename T>
void launch_average_coef(hipStream_t st, const Grid& fine, const Grid& coarse, const T* cf, T* cc);
// coarsest level: element matrices, dense assembly (constrained rows/cols -> identity),
// in-place Gauss-Jordan inverse with partial pivoting, dense (transposed) mat-vec
template <typename T>
void launch_coarse_assemble(hipStream_t st, const LevelView<T>& L, double* elem_mats, double* A);
// In-place inverse of the dense n x n matrix A (row-major; A has room for 2 n^2 doubles),
// Gauss-Jordan with partial pivoting; perm: 2 n ints, work: 2 n doubles of scratch.
void launch_gauss_jordan(hipStream_t st, double* A, int n, int* perm, double* work);
void launch_dense_transpose(hipStream_t st, const double* A, double* At, int n);
template <typename T>
void launch_dense_apply(hipStream_t st, const double* Ainv, int n, bool transpose, const T* b, T* x);

// ---- state / vector helpers
template <typename T>
void launch_pack_state(hipStream_t st, const Grid& g, const double* s5, T* pt);           // (P, T) of s
// Preconditioner input of the (P, T) Krylov solve: b = v / (s_P, s_T) (row scales undone;
// constrained dofs 0) and the first damped block-Jacobi step x = omega D^-1 b (D^-T).
// With nrm (device scalar), v is first normalised in place: v <- v / nrm[0].
template <typename T>
void launch_pc_in(hipStream_t st, const Grid& g, T* v, const double* nrm, T inv_p, T inv_t, const T* dinv,
                  bool transpose, T omega, T* b, T* x);
// out[n][f] = s_f * r5[n][3 + f] (the (P, T) entries of a five-field float64 vector)
template <typename T>
void launch_pack_pt(hipStream_t st, long nodes, const double* r5, T* out, double s_p, double s_t);
// out[n][f] = s_f * in[n][f] for two-field vectors, converting precision
template <typename Ta, typename Tb>
void launch_scale2(hipStream_t st, long nodes, const Ta* in, Tb* out, double s_p, double s_t);
// v <- v / nrm[0] in place (when nrm is not null; nrm on the device) and out = v rounded to Tb
template <typename Ta, typename Tb>
void launch_normalize_copy(hipStream_t st, const double* nrm, Ta* v, Tb* out, long n);
// out5[n][3 + f] = x[n][f] (free dofs) or 0 (constrained dofs); velocity entries untouched
template <typename T>
void launch_unpack_pt(hipStream_t st, const Grid& g, const T* x, double* out5);
void launch_mask_state(hipStream_t st, const Grid& g, double* s5);                       // constrained -> 0
template <typename Ta, typename Tb>
void launch_convert(hipStream_t st, const Ta* a, Tb* b, long n, double scale);           // b = scale * a
void launch_axpy(hipStream_t st, double a, const double* x, const double* y, double* out, long n);  // out = a x + y

template <typename T>
void launch_diag_scale(hipStream_t st, const Grid& g, const T* dinv, bool transpose, T omega, const T* b, T* x);
template <typename T>
void launch_rsub(hipStream_t st, const T* b, T* out, long n);                          // out = b - out

// ---- reductions (deterministic: fixed grid, fixed order).  `part` is a scratch array of
// RED_BLOCKS * MAXC doubles for the per-block partial sums.
constexpr int RED_BLOCKS = 2048;
constexpr int MAXC = 32;
// out[c] = V[c] . w for c < cnt (and out[cnt] = w . w when with_norm); hout, when not
// null (pinned host memory), receives the same values from the same kernel
template <typename T>
void launch_mdot(hipStream_t st, const T* V, long ld, int cnt, const T* w, long n, double* part, double* out,
                 bool with_norm = false, double* hout = nullptr);
// w += sign * sum_c h[c] V[c]; if nrm_out != null also nrm_out[0] = ||w||_2 after the update
// (and hnrm_out[0], pinned host memory, when not null)
template <typename T>
void launch_maxpy(hipStream_t st, const T* V, long ld, int cnt, const double* h, double sign, T* w, long n,
                  double* part, double* nrm_out, double* hnrm_out = nullptr);
template <typename T>
void launch_scale_inv(hipStream_t st, const double* nrm, const T* w, T* v, long n);
// per-field 2-norms of [N][5] arrays: out[f] = ||a_f||, and if b != null out[5+f] = ||b_f||
void launch_field_norms(hipStream_t st, const double* a, const double* b, long nodes, double* part, double* out);
template <typename T>
void launch_norm(hipStream_t st, const T* a, long n, double* part, double* out, double* hout = nullptr);

// ---- design chain and sensitivities
void launch_cone_filter(hipStream_t st, const Grid& g, double radius, const double* x, double* y, bool transpose,
                        double* tmp);
void launch_ramp(hipStream_t st, long E, const double* gamma, double k_f, double k_s, double q_c, double kap_f,
                 double kap_s, double q_p, double* coef64, float* coef32, double* dk, double* dkap);
void launch_sensitivity(hipStream_t st, const Grid& g, const ElemConst<double>& c, const double* coef,
                        const double* dk, const double* dkap, const double* s5, const double* lam5, double* out);
// PDE (Helmholtz) density filter of Sec. 5.1 (k_filter.hip): Chebyshev steps planned from
// closed-form spectrum bounds of the Jacobi-preconditioned operator
constexpr int HELM_MAX_STEPS = 400;
struct HelmholtzPlan {
  double h, r;        // element edge, length scale r = R h / (2 sqrt 3)
  double lmin, lmax;  // spectrum bounds of D^-1 K_F
  int steps;          // Chebyshev steps for the error bound tol
};
HelmholtzPlan helmholtz_plan(double h, double radius, double tol);
// y = F x (F symmetric); work: 4 node vectors
void launch_pde_filter(hipStream_t st, const Grid& g, const HelmholtzPlan& pl, const double* x, double* y,
                       double* work);
// out[0] = sum_e k_e, out[1] = sum_e kappa_e
void launch_coef_sums(hipStream_t st, const double* coef, long E, double* part, double* out);
// objective: the patch-flux compliance plus the volumetric compliance of the source
// elements (c.source), sum_e f_tQ,e^T t_e with the SUPG weight
void launch_objective(hipStream_t st, const Grid& g, const Patch& patch, const ElemConst<double>& c, const double* coef,
                      const double* s5, double* part, double* out);
void launch_objective_grad(hipStream_t st, const Grid& g, const Patch& patch, double* g5);
// g5 += d (volumetric compliance) / d (P, T)
void launch_objective_grad_q(hipStream_t st, const Grid& g, const ElemConst<double>& c, const double* coef,
                             const double* s5, double* g5);
// out[e] += explicit d (volumetric compliance) / d gamma_e (through the permeability)
void launch_objective_dgamma(hipStream_t st, const Grid& g, const ElemConst<double>& c, const double* coef,
                             const double* dkap, const double* s5, double* out);

// ---- passive regions of the benchmark (Sec. 6.1): inclusive element index ranges
struct Regions {
  int s[6];        // passive solid (gamma = 1): i0, i1, j0, j1, k0, k1
  int d[6];        // design domain; outside it (and outside the solid) passive fluid
  int has_s, has_d;
  __host__ __device__ bool solid(int i, int j, int k) const {
    return has_s && i >= s[0] && i <= s[1] && j >= s[2] && j <= s[3] && k >= s[4] && k <= s[5];
  }
  __host__ __device__ bool design(int i, int j, int k) const {
    if (solid(i, j, k)) return false;
    return !has_d || (i >= d[0] && i <= d[1] && j >= d[2] && j <= d[3] && k >= d[4] && k <= d[5]);
  }
};
void launch_passive(hipStream_t st, const Grid& g, const Regions& rg, double* gamma);
// a = 0 off the design domain (set: a = fill on it, 0 off it)
void launch_design_mask(hipStream_t st, const Grid& g, const Regions& rg, double* a, bool set, double fill);
// ---- MMA design update (k_mma.hip); the caller's state holds NC_MMA_ROWS rows of E:
// previous two iterates, asymptotes, subproblem bounds, approximation coefficients
constexpr int MMA_CAND = 32;
struct MmaCand {
  double v[MMA_CAND];   // multipliers evaluated by one pass (inf: the limit lambda -> inf)
};
// coefficients of the subproblem at x; out[0] = sum of the constraint approximation at x
void launch_mma_prepare(hipStream_t st, const Grid& g, const Regions& rg, int iter, double move, double xmin,
                        double xmax, const double* x, const double* df, const double* dg, double* state, double* part,
                        double* out);
// out[c] = constraint approximation at x(lambda_c) (without its right-hand side)
void launch_mma_dual(hipStream_t st, const Grid& g, const Regions& rg, const MmaCand& lam, const double* state,
                     double* part, double* out);
void launch_mma_apply(hipStream_t st, const Grid& g, const Regions& rg, int iter, double lam, double* x, double* state);

// out[0] = sum of gamma over the design domain
void launch_design_sum(hipStream_t st, const Grid& g, const Regions& rg, const double* gamma, double* part,
                       double* out);

}  // namespace nc
