// Method of Moving Asymptotes for the volume-constrained design update (Sec. 5.1; move
// limit of Sec. 6.1), on the design elements of a context.  Svanberg's method with his
// standard asymptote rules; the separable convex subproblem with one constraint is solved
// through its dual, a concave function of one multiplier lambda >= 0 whose derivative is
// the constraint's approximation at x(lambda), non-increasing in lambda.  Each element's
// x(lambda) is closed form, so one pass over the elements evaluates the derivative at
// MMA_CAND multipliers at once; the host narrows the bracket by that factor per pass.
#include <cmath>

#include "kernels.hpp"

namespace nc {

namespace {

constexpr int BS = 256;
constexpr int MMA_BLOCKS = 1024;
constexpr double ASY_INIT = 0.5, ASY_INCR = 1.2, ASY_DECR = 0.7, ALBEFA = 0.1, RAA0 = 1e-5;

struct ElemIdx {
  int i, j, k;
};
__device__ inline ElemIdx elem_idx(const Grid& g, long e) {
  return ElemIdx{(int)(e % g.nx), (int)((e / g.nx) % g.ny), (int)(e / ((long)g.nx * g.ny))};
}

__device__ inline double wsum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Row r of the caller's MMA state [NC_MMA_ROWS][E]
__device__ inline double* row(double* st, long E, int r) { return st + (long)r * E; }

// p and q of an approximation with derivative d: (U - x)^2 (1.001 d+ + 0.001 d- + raa0),
// (x - L)^2 (0.001 d+ + 1.001 d- + raa0)
__device__ inline void pq(double d, double ux, double xl, double& p, double& q) {
  const double dp = d > 0.0 ? d : 0.0, dm = d < 0.0 ? -d : 0.0;
  p = ux * ux * (1.001 * dp + 0.001 * dm + RAA0);
  q = xl * xl * (0.001 * dp + 1.001 * dm + RAA0);
}

// Asymptotes, subproblem bounds and the approximations' coefficients of every design
// element; partial sums of the constraint approximation at x (for its right-hand side).
__global__ __launch_bounds__(BS) void mma_prepare_kernel(Grid g, Regions rg, int iter, double move, double xmin,
                                                         double xmax, const double* __restrict__ x,
                                                         const double* __restrict__ df, const double* __restrict__ dg,
                                                         double* __restrict__ st, double* __restrict__ part) {
  __shared__ double red[BS / 64];
  const long E = g.elems();
  const double span = xmax - xmin;
  double acc = 0.0;
  for (long e = (long)blockIdx.x * BS + threadIdx.x; e < E; e += (long)gridDim.x * BS) {
    const ElemIdx q = elem_idx(g, e);
    if (!rg.design(q.i, q.j, q.k)) continue;
    const double xe = x[e];
    double lo, up;
    if (iter <= 2) {
      lo = xe - ASY_INIT * span;
      up = xe + ASY_INIT * span;
    } else {
      const double x1 = row(st, E, 0)[e], x2 = row(st, E, 1)[e];
      const double sgn = (xe - x1) * (x1 - x2);
      const double fac = sgn > 0.0 ? ASY_INCR : (sgn < 0.0 ? ASY_DECR : 1.0);
      lo = xe - fac * (x1 - row(st, E, 2)[e]);
      up = xe + fac * (row(st, E, 3)[e] - x1);
      lo = fmin(fmax(lo, xe - 10.0 * span), xe - 0.01 * span);
      up = fmin(fmax(up, xe + 0.01 * span), xe + 10.0 * span);
    }
    const double al = fmax(fmax(xmin, lo + ALBEFA * (xe - lo)), xe - move);
    const double be = fmin(fmin(xmax, up - ALBEFA * (up - xe)), xe + move);
    const double ux = up - xe, xl = xe - lo;
    double p0, q0, p1, q1;
    pq(df[e], ux, xl, p0, q0);
    pq(dg[e], ux, xl, p1, q1);
    row(st, E, 2)[e] = lo;
    row(st, E, 3)[e] = up;
    row(st, E, 4)[e] = al;
    row(st, E, 5)[e] = be;
    row(st, E, 6)[e] = p0;
    row(st, E, 7)[e] = q0;
    row(st, E, 8)[e] = p1;
    row(st, E, 9)[e] = q1;
    acc += p1 / ux + q1 / xl;
  }
  acc = wsum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < BS / 64; ++w) t += red[w];
    part[blockIdx.x] = t;
  }
}

// x_e(lambda): the minimiser of (p0 + lambda p1)/(U - x) + (q0 + lambda q1)/(x - L) on
// [alpha, beta]; lambda = inf: of p1/(U - x) + q1/(x - L)
__device__ inline double x_of(double lam, double lo, double up, double al, double be, double p0, double q0, double p1,
                              double q1) {
  double P, Q;
  if (isinf(lam)) {
    P = p1;
    Q = q1;
  } else {
    P = p0 + lam * p1;
    Q = q0 + lam * q1;
  }
  const double sp = sqrt(P), sq = sqrt(Q);
  return fmin(fmax((sp * lo + sq * up) / (sp + sq), al), be);
}

// Constraint approximation at x(lambda_c) for MMA_CAND multipliers: per-block partials
// part[c * MMA_BLOCKS + block]
__global__ __launch_bounds__(BS) void mma_dual_kernel(Grid g, Regions rg, MmaCand lam, const double* __restrict__ st,
                                                      double* __restrict__ part) {
  __shared__ double red[BS / 64][MMA_CAND];
  const long E = g.elems();
  double acc[MMA_CAND];
#pragma unroll
  for (int c = 0; c < MMA_CAND; ++c) acc[c] = 0.0;
  for (long e = (long)blockIdx.x * BS + threadIdx.x; e < E; e += (long)gridDim.x * BS) {
    const ElemIdx q = elem_idx(g, e);
    if (!rg.design(q.i, q.j, q.k)) continue;
    const double lo = st[2 * E + e], up = st[3 * E + e], al = st[4 * E + e], be = st[5 * E + e];
    const double p0 = st[6 * E + e], q0 = st[7 * E + e], p1 = st[8 * E + e], q1 = st[9 * E + e];
#pragma unroll
    for (int c = 0; c < MMA_CAND; ++c) {
      const double xe = x_of(lam.v[c], lo, up, al, be, p0, q0, p1, q1);
      acc[c] += p1 / (up - xe) + q1 / (xe - lo);
    }
  }
#pragma unroll
  for (int c = 0; c < MMA_CAND; ++c) {
    const double v = wsum(acc[c]);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6][c] = v;
  }
  __syncthreads();
  if (threadIdx.x < MMA_CAND) {
    double t = 0.0;
    for (int w = 0; w < BS / 64; ++w) t += red[w][threadIdx.x];
    part[(long)threadIdx.x * MMA_BLOCKS + blockIdx.x] = t;
  }
}

// out[c] = sum over blocks of part[c][block], in a fixed order (one wave per column)
__global__ __launch_bounds__(BS) void mma_sum_kernel(const double* __restrict__ part, int ncol, double* __restrict__ out) {
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int c = w; c < ncol; c += BS / 64) {
    double s = 0.0;
    for (int b = lane; b < MMA_BLOCKS; b += 64) s += part[(long)c * MMA_BLOCKS + b];
    s = wsum(s);
    if (lane == 0) out[c] = s;
  }
}

// x <- x(lambda) on the design elements; the previous two iterates shift in the state
__global__ __launch_bounds__(BS) void mma_apply_kernel(Grid g, Regions rg, int iter, double lam, double* __restrict__ x,
                                                       double* __restrict__ st) {
  const long E = g.elems();
  const long e = (long)blockIdx.x * BS + threadIdx.x;
  if (e >= E) return;
  const ElemIdx q = elem_idx(g, e);
  if (!rg.design(q.i, q.j, q.k)) return;
  const double xn = x_of(lam, st[2 * E + e], st[3 * E + e], st[4 * E + e], st[5 * E + e], st[6 * E + e], st[7 * E + e],
                         st[8 * E + e], st[9 * E + e]);
  const double xe = x[e];
  st[E + e] = iter <= 1 ? xe : st[e];
  st[e] = xe;
  x[e] = xn;
}

}  // namespace

void launch_mma_prepare(hipStream_t st, const Grid& g, const Regions& rg, int iter, double move, double xmin,
                        double xmax, const double* x, const double* df, const double* dg, double* state, double* part,
                        double* out) {
  launch(mma_prepare_kernel, dim3(MMA_BLOCKS), dim3(BS), 0, st, g, rg, iter, move, xmin, xmax, x, df, dg, state, part);
  launch(mma_sum_kernel, dim3(1), dim3(BS), 0, st, (const double*)part, 1, out);
}

void launch_mma_dual(hipStream_t st, const Grid& g, const Regions& rg, const MmaCand& lam, const double* state,
                     double* part, double* out) {
  launch(mma_dual_kernel, dim3(MMA_BLOCKS), dim3(BS), 0, st, g, rg, lam, state, part);
  launch(mma_sum_kernel, dim3(1), dim3(BS), 0, st, (const double*)part, MMA_CAND, out);
}

void launch_mma_apply(hipStream_t st, const Grid& g, const Regions& rg, int iter, double lam, double* x, double* state) {
  launch(mma_apply_kernel, dim3((unsigned)((g.elems() + BS - 1) / BS)), dim3(BS), 0, st, g, rg, iter, lam, x, state);
}

}  // namespace nc
