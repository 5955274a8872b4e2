// PDE (Helmholtz) density filter of Sec. 5.1: -r^2 lap y + y = x with Neumann walls,
// r = R h / (2 sqrt 3), on the trilinear nodal field y, Galerkin with the consistent mass:
//   K_F y = B x,  K_F = int (r^2 grad N_a . grad N_b + N_a N_b),  B_ae = int_e N_a = h^3 / 8,
// and gamma_e = the mean of y over element e = the average of its eight nodal values.
//
// Solver.  The grid is uniform, so K_F is one constant 27-point stencil; Jacobi
// preconditioning makes it well conditioned independently of h for a fixed R (R = 2.5:
// condition number 3.3), with spectrum bounds known in closed form (see
// helmholtz_plan).  A Chebyshev iteration with those bounds needs no inner products:
// every step is one fused node kernel (stencil apply, iterate and residual update, next
// direction), the step coefficients are host constants, there is no host round trip and
// the result is bitwise reproducible.
#include <algorithm>
#include <cmath>
#include <utility>

#include "kernels.hpp"

namespace nc {

namespace {

constexpr int BS = 256;   // threads per block of the node and element kernels
inline int blocks_for(long n) { return (int)((n + BS - 1) / BS); }

// Entry (a, b) of the element matrix r^2 int grad N_a . grad N_b + int N_a N_b of a cube of
// edge h, by the coincidence pattern p = s_x + 2 s_y + 4 s_z of local nodes a and b
// (s_d = 1 when they share the d coordinate).  With the 1D linear-element matrices
// k(same) = 1/h, k(diff) = -1/h, m(same) = h/3, m(diff) = h/6, the entry is
// r^2 (k_x m_y m_z + m_x k_y m_z + m_x m_y k_z) + m_x m_y m_z.
void element_pattern(double h, double r, double a[8]) {
  for (int p = 0; p < 8; ++p) {
    double k[3], m[3];
    for (int d = 0; d < 3; ++d) {
      const bool same = (p >> d) & 1;
      k[d] = same ? 1.0 / h : -1.0 / h;
      m[d] = same ? h / 3.0 : h / 6.0;
    }
    a[p] = r * r * (k[0] * m[1] * m[2] + m[0] * k[1] * m[2] + m[0] * m[1] * k[2]) + m[0] * m[1] * m[2];
  }
}

struct HelmCoef {
  double a[8];   // element pattern entries
};

// n / d for 0 <= n < 2^31 by a multiply-high and a shift (division by an invariant
// integer, Granlund and Montgomery): q = (mulhi(n, m) + n) >> s with s = ceil(log2 d),
// m = floor(2^32 (2^s - d) / d) + 1.
struct FastDiv {
  unsigned d, m, s;
  FastDiv() = default;
  explicit FastDiv(unsigned div) : d(div), m(0), s(0) {
    while ((1ull << s) < div) ++s;
    m = (unsigned)(((1ull << 32) * ((1ull << s) - div)) / div + 1);
  }
  __device__ unsigned div(unsigned n) const {
    const unsigned hi = (unsigned)(((unsigned long long)n * m) >> 32);
    return (unsigned)(((unsigned long long)hi + n) >> s);
  }
};

struct NodeGrid {
  Grid g;
  FastDiv nx1, nxy;   // divisions by nx + 1 and (nx + 1)(ny + 1)
};

struct NodeIdx {
  int i, j, k, n;
  bool ok;
};
// Workgroups are dispatched round-robin over the chip's 8 XCDs, each with its own L2; the
// logical block order gives XCD x (hardware blocks x, x + 8, ...) one contiguous range of
// nodes, so a node's neighbours one row or plane away are mostly in the same L2.
__device__ inline unsigned xcd_block() {
  const unsigned nb = gridDim.x, b = blockIdx.x, x = b % 8, q = nb / 8, rem = nb % 8;
  return x * q + (x < rem ? x : rem) + b / 8;
}
__device__ inline NodeIdx node_idx(const NodeGrid& ng) {
  const unsigned n = xcd_block() * blockDim.x + threadIdx.x;
  NodeIdx q{0, 0, 0, (int)n, n < (unsigned)ng.g.nodes()};
  if (!q.ok) return q;
  const unsigned k = ng.nxy.div(n), rem = n - k * ng.nxy.d;
  const unsigned j = ng.nx1.div(rem);
  q.k = (int)k;
  q.j = (int)j;
  q.i = (int)(rem - j * ng.nx1.d);
  return q;
}

// b = s_in * (sum of x over the elements around each node); the iteration starts from
// y = 0: residual b, first direction b / (theta D).
__global__ __launch_bounds__(BS) void helm_init_kernel(NodeGrid ng, double s_in, double a_diag, double inv_theta,
                                                       const double* __restrict__ x, double* __restrict__ y,
                                                       double* __restrict__ r, double* __restrict__ d) {
  const Grid& g = ng.g;
  const NodeIdx q = node_idx(ng);
  if (!q.ok) return;
  double b = 0.0;
  for (int ez = q.k - 1; ez <= q.k; ++ez) {
    if (ez < 0 || ez >= g.nz) continue;
    for (int ey = q.j - 1; ey <= q.j; ++ey) {
      if (ey < 0 || ey >= g.ny) continue;
      for (int ex = q.i - 1; ex <= q.i; ++ex) {
        if (ex < 0 || ex >= g.nx) continue;
        b += x[g.elem(ex, ey, ez)];
      }
    }
  }
  b *= s_in;
  const int n = g.node(q.i, q.j, q.k);
  y[n] = 0.0;
  r[n] = b;
  d[n] = inv_theta * b / (g.valence(q.i, q.j, q.k) * a_diag);
}

// One Chebyshev step, y += d, r -= K_F d, d' = c1 d + c2 D^-1 r, with the direction staged
// in LDS: a workgroup of CT_X x CT_Y threads owns a CT_X x CT_Y tile of node columns over a
// chunk of CT_Z node planes and stages the CT_Z + 2 planes of d it touches (the tile and a
// one-node halo, zero off the grid) in LDS, so that each value of d is read from memory
// about once instead of once per neighbour.  Every load of the chunk (d, and the own nodes'
// y and r) is issued before the first LDS store and the workgroup waits at one barrier, so
// the memory latency is paid once per chunk rather than once per plane.  Row n of K_F:
// neighbour n + o couples through the elements the two share; each of them contributes the
// same pattern entry (s_d = [o_d == 0]), and their number is the product over d of 2 (o_d = 0,
// node inside in d), 1 (o_d = 0 on a wall, or o_d = +-1 with the neighbour on the grid) or 0
// (neighbour off the grid); an interior row is the constant 27-point stencil.  Summed in a
// fixed order, so results are bitwise reproducible.
constexpr int CT_X = 32, CT_Y = 8, CT_Z = 4, CT_LX = CT_X + 2, CT_LY = CT_Y + 2;
constexpr int CT_THREADS = CT_X * CT_Y, CT_PLANE = CT_LX * CT_LY;
constexpr int CT_SLOTS = (CT_PLANE + CT_THREADS - 1) / CT_THREADS;  // plane values per thread

__global__ __launch_bounds__(CT_THREADS) void helm_cheb_tiled_kernel(Grid g, HelmCoef c, double c1, double c2,
                                                                    int tiles, const double* __restrict__ d,
                                                                    double* __restrict__ d_next,
                                                                    double* __restrict__ y, double* __restrict__ r) {
  __shared__ double buf[CT_Z + 2][CT_PLANE];
  // workgroups are dealt to the eight XCDs in turn; the logical block id is chosen so that
  // each XCD runs a contiguous range of them, and tiles that share halo planes and cache
  // lines share that XCD's L2
  const int nb = (int)gridDim.x, xcd = (int)blockIdx.x % 8, q8 = nb / 8, rem8 = nb % 8;
  const int lb = xcd * q8 + min(xcd, rem8) + (int)blockIdx.x / 8;
  const int tile = lb % tiles, chunk = lb / tiles;
  const int tx = threadIdx.x % CT_X, ty = threadIdx.x / CT_X;
  const int ntx = (g.nx + CT_X) / CT_X;                      // tiles over the nx + 1 node columns
  const int gi0 = (tile % ntx) * CT_X, gj0 = (tile / ntx) * CT_Y;
  const int i = gi0 + tx, j = gj0 + ty;
  const int K0 = chunk * CT_Z, nk = min(CT_Z, g.nz + 1 - K0);
  const bool own = i <= g.nx && j <= g.ny;
  // planes K0 - 1 .. K0 + CT_Z of d; a plane beyond nz (the last chunk's tail) reads as zero
  double v[CT_Z + 2][CT_SLOTS];
#pragma unroll
  for (int p = 0; p < CT_Z + 2; ++p) {
    const int k = K0 - 1 + p;
    const bool zin = k >= 0 && k <= g.nz;
#pragma unroll
    for (int s = 0; s < CT_SLOTS; ++s) {
      const int t = (int)threadIdx.x + s * CT_THREADS;
      const int gi = gi0 - 1 + t % CT_LX, gj = gj0 - 1 + t / CT_LX;
      v[p][s] = (t < CT_PLANE && zin && gi >= 0 && gi <= g.nx && gj >= 0 && gj <= g.ny) ? d[g.node(gi, gj, k)] : 0.0;
    }
  }
  double yv[CT_Z], rv[CT_Z];
#pragma unroll
  for (int p = 0; p < CT_Z; ++p) {
    const bool ok = own && p < nk;
    const int n = ok ? g.node(i, j, K0 + p) : 0;
    yv[p] = ok ? y[n] : 0.0;
    rv[p] = ok ? r[n] : 0.0;
  }
#pragma unroll
  for (int p = 0; p < CT_Z + 2; ++p)
#pragma unroll
    for (int s = 0; s < CT_SLOTS; ++s) {
      const int t = (int)threadIdx.x + s * CT_THREADS;
      if (t < CT_PLANE) buf[p][t] = v[p][s];
    }
  __syncthreads();
  if (!own) return;
  // count factors of the element-count row in x and y (offset -1, 0, +1)
  double cxy[3][3];
  {
    double cx[3], cy[3];
    for (int o = -1; o <= 1; ++o) {
      cx[o + 1] = o == 0 ? ((i > 0 && i < g.nx) ? 2.0 : 1.0) : ((i + o >= 0 && i + o <= g.nx) ? 1.0 : 0.0);
      cy[o + 1] = o == 0 ? ((j > 0 && j < g.ny) ? 2.0 : 1.0) : ((j + o >= 0 && j + o <= g.ny) ? 1.0 : 0.0);
    }
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) cxy[a][b] = cx[b] * cy[a];
  }
  const int li = tx + 1, lj = ty + 1;
#pragma unroll
  for (int p = 0; p < CT_Z; ++p) {
    if (p >= nk) break;
    const int k = K0 + p;
    double acc = 0.0;
#pragma unroll
    for (int oz = -1; oz <= 1; ++oz) {
      const double cz = oz == 0 ? ((k > 0 && k < g.nz) ? 2.0 : 1.0) : ((k + oz >= 0 && k + oz <= g.nz) ? 1.0 : 0.0);
      const double* pl = buf[p + 1 + oz];
#pragma unroll
      for (int oy = -1; oy <= 1; ++oy)
#pragma unroll
        for (int ox = -1; ox <= 1; ++ox) {
          const int e = (ox == 0) + 2 * (oy == 0) + 4 * (oz == 0);
          acc += cz * cxy[oy + 1][ox + 1] * c.a[e] * pl[(li + ox) + CT_LX * (lj + oy)];
        }
    }
    const double dn = buf[p + 1][li + CT_LX * lj];
    const double diag = cxy[1][1] * ((k > 0 && k < g.nz) ? 2.0 : 1.0) * c.a[7];
    const int n = g.node(i, j, k);
    y[n] = yv[p] + dn;
    const double rn = rv[p] - acc;
    r[n] = rn;
    d_next[n] = c1 * dn + c2 * rn / diag;
  }
}

// out_e = s_out * sum of (y + d) over the element's eight nodes (the last direction is
// added here rather than by another step)
__global__ __launch_bounds__(BS) void helm_out_kernel(Grid g, double s_out, const double* __restrict__ y,
                                                      const double* __restrict__ d, double* __restrict__ out) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= g.elems()) return;
  const int i = (int)(e % g.nx), j = (int)((e / g.nx) % g.ny), k = (int)(e / ((long)g.nx * g.ny));
  double s = 0.0;
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const int n = g.node(i + (c & 1), j + ((c >> 1) & 1), k + ((c >> 2) & 1));
    s += y[n] + d[n];
  }
  out[e] = s_out * s;
}

}  // namespace

// Chebyshev plan for radius R (element lengths) on a grid of edge h.  The symbol of
// D^-1 K_F (D its diagonal) on the cosine modes is
//   [r^2 sum_d k_d prod_(d' != d) m_d' + prod_d m_d] / D0,
//   k_d = (2/h)(1 - c_d), m_d = (h/3)(2 + c_d), c_d = cos(theta_d), D0 = 8 (r^2 h/3 + h^3/27),
// and on a uniform grid with Neumann walls those modes are the eigenvectors (the wall rows
// are half rows), so its eigenvalues lie between the symbol's extremes over c in [-1, 1]^3.
// The symbol is affine in each c_d, so they are attained at the cube's eight vertices.
HelmholtzPlan helmholtz_plan(double h, double radius, double tol) {
  HelmholtzPlan pl{};
  pl.h = h;
  pl.r = radius * h / (2.0 * std::sqrt(3.0));
  double lo = 1e300, hi = 0.0;
  const double r2 = pl.r * pl.r, D0 = 8.0 * (r2 * h / 3.0 + h * h * h / 27.0);
  for (int v = 0; v < 8; ++v) {
    double k[3], m[3];
    for (int d = 0; d < 3; ++d) {
      const double cd = ((v >> d) & 1) ? 1.0 : -1.0;
      k[d] = 2.0 / h * (1.0 - cd);
      m[d] = h / 3.0 * (2.0 + cd);
    }
    const double s = (r2 * (k[0] * m[1] * m[2] + m[0] * k[1] * m[2] + m[0] * m[1] * k[2]) + m[0] * m[1] * m[2]) / D0;
    lo = std::fmin(lo, s);
    hi = std::fmax(hi, s);
  }
  pl.lmin = lo;
  pl.lmax = hi;
  // error after k steps <= 1 / T_k(theta / delta) = 2 sigma^k / (1 + sigma^2k),
  // sigma = (sqrt(kappa) - 1) / (sqrt(kappa) + 1)
  const double kappa = hi / lo, sk = std::sqrt(kappa);
  const double sigma = (sk - 1.0) / (sk + 1.0);
  int steps = 1;
  while (steps < HELM_MAX_STEPS && 2.0 * std::pow(sigma, steps) > tol) ++steps;
  pl.steps = steps;
  return pl;
}

// y = F x with F = h^-3 B^T K_F^-1 B (symmetric, so also the sensitivity map F^T).
// work: 4 node vectors (iterate, residual, two directions).
void launch_pde_filter(hipStream_t st, const Grid& g, const HelmholtzPlan& pl, const double* x, double* y,
                       double* work) {
  const long N = g.nodes();
  double* yy = work;
  double* rr = work + N;
  double* d0 = work + 2 * N;
  double* d1 = work + 3 * N;
  HelmCoef c;
  element_pattern(pl.h, pl.r, c.a);
  NodeGrid ng{g, FastDiv((unsigned)(g.nx + 1)), FastDiv((unsigned)((g.nx + 1) * (g.ny + 1)))};
  // Chebyshev acceleration (Saad, Iterative Methods for Sparse Linear Systems, Alg. 12.1)
  // with the Jacobi preconditioner on [lmin, lmax]
  const double theta = 0.5 * (pl.lmax + pl.lmin), delta = 0.5 * (pl.lmax - pl.lmin);
  const double sigma1 = theta / delta;
  const double h3 = pl.h * pl.h * pl.h;
  launch(helm_init_kernel, dim3(blocks_for(N)), dim3(BS), 0, st, ng, h3 / 8.0, c.a[7], 1.0 / theta, x, yy, rr, d0);
  double rho = 1.0 / sigma1;
  // tiles of CT_X x CT_Y node columns times z chunks of CT_Z node planes
  const int tiles = ((g.nx + CT_X) / CT_X) * ((g.ny + CT_Y) / CT_Y);
  const int chunks = (g.nz + CT_Z) / CT_Z;
  for (int s = 0; s < pl.steps; ++s) {
    const double rho_next = 1.0 / (2.0 * sigma1 - rho);
    launch(helm_cheb_tiled_kernel, dim3((unsigned)(tiles * chunks)), dim3(CT_X * CT_Y), 0, st, g, c, rho_next * rho,
           2.0 * rho_next / delta, tiles, (const double*)d0, d1, yy, rr);
    rho = rho_next;
    std::swap(d0, d1);
  }
  launch(helm_out_kernel, dim3(blocks_for(g.elems())), dim3(BS), 0, st, g, 1.0 / 8.0, (const double*)yy,
         (const double*)d0, y);
}

}  // namespace nc
