// Host-side launchers of the Navier-Stokes / Brinkman solver's kernels (k_ns.hip).  All
// launches are asynchronous on the given stream; device pointers only.
#pragma once

#include "common.hpp"
#include "ns_element.hpp"

namespace nc {
namespace ns {

// entries per node of the node-block matrix: 27 neighbours x 5 x 5, stored as planes
// A[(o * 25 + f * 5 + g) * N + n], o = (dx+1) + 3 (dy+1) + 9 (dz+1) the neighbour's offset
constexpr int NS_ENTRIES = 27 * 25;

// Dirichlet sets of the flow model: no slip on the walls (only u.n on a symmetry plane),
// the pressure level at (0, 0, nz), T as in the Darcy model.
__host__ __device__ inline bool fixed(const Grid& g, int i, int j, int k, int f) {
  if (f < 3) {
    const bool wall = i == 0 || j == 0 || k == 0 || k == g.nz || (i == g.nx && g.tx >= 0) || (j == g.ny && g.ty >= 0);
    return wall || (f == 0 && i == g.nx) || (f == 1 && j == g.ny);
  }
  if (f == 3) return g.pfix(i, j, k);
  return g.tfix(i, j, k);
}

// The elements of one colour (i, j, k parities cx, cy, cz): mx * my * mz of them.
struct ColourGrid {
  int cx, cy, cz, mx, my, mz;
  long count;
};
ColourGrid colour_grid(const Grid& g, int col);

template <typename T>
void launch_fill(hipStream_t st, T* a, long n, T v);
// r = R~(s): element rows (k, a per element in coef [E][2]), patch flux, constrained rows s
void launch_residual(hipStream_t st, const Grid& g, const NsConst& c, const Patch& patch, const double* coef,
                     const double* s, double* r);
// A = J~(s) in precision T (constrained rows identity, constrained columns zero)
template <typename T>
void launch_assemble(hipStream_t st, const Grid& g, const NsConst& c, const double* coef, const double* s, T* A);
// mode 0: y = A x; 1: y = b - A x; 2: y = x + omega D^-1 (b - A x); transposes when tr
template <typename TM, typename T>
void launch_bsr(hipStream_t st, const Grid& g, const TM* A, const TM* Dinv, bool tr, int mode, const T* x, const T* b,
                T* y, T omega);
template <typename T>
void launch_diag_scale(hipStream_t st, const Grid& g, const T* Dinv, bool tr, T omega, const T* b, T* x);
template <typename T>
void launch_diag_inverse(hipStream_t st, const Grid& g, const T* A, T* Dinv);
template <typename T>
void launch_restrict(hipStream_t st, const Grid& gf, const Grid& gc, const T* rf, T* bc);
template <typename T>
void launch_prolong_add(hipStream_t st, const Grid& gf, const Grid& gc, const T* xc, T* xf);
// five per-field factors
struct Field5 {
  double s[5];
};
// out[n][f] = sc.s[f] in[n][f] for [N][5] arrays (in == out allowed)
template <typename Ta, typename Tb>
void launch_scale_fields(hipStream_t st, long N, const Ta* in, Tb* out, const Field5& sc);
// d [N][5] = the diagonal of the node-block matrix A (0 on constrained dofs)
template <typename TM>
void launch_diagonal(hipStream_t st, const Grid& g, const TM* A, double* d);
// constrained dofs of s [N][5] set to 0
void launch_mask(hipStream_t st, const Grid& g, double* s);
void launch_inject(hipStream_t st, const Grid& gf, const Grid& gc, const double* sf, double* sc);
// D (5N x 5N, row-major) = A
template <typename T>
void launch_dense(hipStream_t st, const Grid& g, const T* A, double* D);
// Brinkman coefficient a(gamma) = abar q gamma / (1 + q - gamma) into coef[e][1] and its
// derivative into da (abar: the solid's impermeability, q: its RAMP penalty)
void launch_brinkman(hipStream_t st, long E, double abar, double q, const double* gamma, double* coef, double* da);
void launch_objective(hipStream_t st, const Grid& g, const NsConst& c, const Patch& patch, const double* s, double* part,
                      double* out);
void launch_objective_grad(hipStream_t st, const Grid& g, const NsConst& c, const Patch& patch, const double* s,
                           double* g5);
void launch_sensitivity(hipStream_t st, const Grid& g, const NsConst& c, const double* coef, const double* dk,
                        const double* da, const double* s, const double* lam, double* out);

}  // namespace ns
}  // namespace nc
