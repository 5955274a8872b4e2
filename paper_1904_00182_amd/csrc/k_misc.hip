// Multigrid transfers and setup, dense coarse solve, vector kernels, deterministic
// reductions, design chain (cone filter, RAMP), sensitivities and the objective.
#include <utility>

#include "kernels.hpp"
#include "transfer.hpp"

namespace nc {

constexpr int BS = 256;

static inline int blocks_for(long n, int bs = BS) {
  long b = (n + bs - 1) / bs;
  return (int)std::max<long>(1, std::min<long>(b, 65535L * 32));
}

// ------------------------------------------------------------------ transfers
// Node kernels run on a 2-D grid: blockIdx.y is the node plane k, the x dimension covers
// the (nx+1)(ny+1) nodes of the plane (one 32-bit division per thread).
struct PlaneIdx {
  int i, j, k;
  bool ok;
};
__device__ inline PlaneIdx plane_idx(const Grid& g) {
  const int p = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  const int row = g.nx + 1;
  PlaneIdx r;
  r.k = (int)blockIdx.y;
  r.j = p / row;
  r.i = p - r.j * row;
  r.ok = r.j <= g.ny;
  return r;
}
static inline dim3 plane_grid(const Grid& g, int bs) {
  return dim3((unsigned)ceil_div((long)(g.nx + 1) * (g.ny + 1), bs), (unsigned)(g.nz + 1));
}

// Restriction by the transpose of trilinear prolongation (full weighting), constrained
// coarse dofs set to zero; one thread per coarse node.  With dinv, also the first damped
// block-Jacobi step of the coarse level from a zero guess, x = omega D^-1 b (D^-T b when
// transposed).
template <typename T>
__global__ __launch_bounds__(128) void restrict_kernel(Grid fine, Grid coarse, const T* __restrict__ rf, T* __restrict__ bc,
                                const T* __restrict__ dinv, int transpose, T omega, T* __restrict__ xc) {
  const PlaneIdx q = plane_idx(coarse);
  if (!q.ok) return;
  const int I = q.i, J = q.j, K = q.k;
  TAcc<T> sp, stt;
  restrict_taps(fine, I, J, K, rf, sp, stt);
  using P2 = typename Pair<T>::type;
  const int n = coarse.node(I, J, K);
  const T bp = coarse.pfix(I, J, K) ? (T)0 : (T)sp;
  const T bt = coarse.tfix(I, J, K) ? (T)0 : (T)stt;
  reinterpret_cast<P2*>(bc)[n] = P2{bp, bt};
  if (dinv) {
    const typename Quad<T>::type D = reinterpret_cast<const typename Quad<T>::type*>(dinv)[n];
    reinterpret_cast<P2*>(xc)[n] =
        P2{omega * (D.x * bp + (transpose ? D.z : D.y) * bt), omega * ((transpose ? D.y : D.z) * bp + D.w * bt)};
  }
}

// Trilinear prolongation added to the fine iterate; one thread per pair of fine nodes
// (2m, j, k), (2m + 1, j, k) along x.
template <typename T>
__global__ __launch_bounds__(256) void prolong_kernel(Grid fine, Grid coarse, const T* __restrict__ xc, T* __restrict__ xf) {
  const int p = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  const int row = coarse.nx + 1;   // pairs per fine row; the last pair has its even node only
  const int j = p / row, m = p - j * row, k = (int)blockIdx.y;
  if (j > fine.ny) return;
  TAcc<T> sp[2], stt[2];
  prolong_taps_pair(coarse, m, j, k, xc, sp, stt);
  using P2 = typename Pair<T>::type;
  P2* x = reinterpret_cast<P2*>(xf);
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int i = 2 * m + h;
    if (i > fine.nx) break;
    const int n = fine.node(i, j, k);
    P2 v = x[n];
    if (!fine.pfix(i, j, k)) v.x += (T)sp[h];
    if (!fine.tfix(i, j, k)) v.y += (T)stt[h];
    x[n] = v;
  }
}

template <typename T>
__global__ void inject_kernel(Grid fine, Grid coarse, const T* __restrict__ sf, T* __restrict__ sc) {
  const long n = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= coarse.nodes()) return;
  const int I = (int)(n % (coarse.nx + 1));
  const int J = (int)((n / (coarse.nx + 1)) % (coarse.ny + 1));
  const int K = (int)(n / ((long)(coarse.nx + 1) * (coarse.ny + 1)));
  const long m = fine.node(2 * I, 2 * J, 2 * K);
  sc[2 * n] = sf[2 * m];
  sc[2 * n + 1] = sf[2 * m + 1];
}

template <typename T>
__global__ void average_coef_kernel(Grid fine, Grid coarse, const T* __restrict__ cf, T* __restrict__ cc) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= coarse.elems()) return;
  const int I = (int)(e % coarse.nx);
  const int J = (int)((e / coarse.nx) % coarse.ny);
  const int K = (int)(e / ((long)coarse.nx * coarse.ny));
  double k = 0.0, kap = 0.0;
  for (int c = 0; c < 8; ++c) {
    const long f = fine.elem(2 * I + (c & 1), 2 * J + ((c >> 1) & 1), 2 * K + ((c >> 2) & 1));
    k += (double)cf[2 * f];
    kap += (double)cf[2 * f + 1];
  }
  cc[2 * e] = (T)(0.125 * k);
  cc[2 * e + 1] = (T)(0.125 * kap);
}

template <typename T>
void launch_restrict(hipStream_t st, const Grid& fine, const Grid& coarse, const T* rf, T* bc, const T* dinv,
                     bool transpose, T omega, T* xc) {
  launch(restrict_kernel<T>, plane_grid(coarse, 128), dim3(128), 0, st, fine, coarse, rf, bc, dinv,
                     transpose ? 1 : 0, omega, xc);
}
template <typename T>
void launch_prolong_add(hipStream_t st, const Grid& fine, const Grid& coarse, const T* xc, T* xf) {
  const dim3 grid((unsigned)ceil_div((long)(coarse.nx + 1) * (fine.ny + 1), 256), (unsigned)(fine.nz + 1));
  launch(prolong_kernel<T>, grid, dim3(256), 0, st, fine, coarse, xc, xf);
}
template <typename T>
void launch_inject_state(hipStream_t st, const Grid& fine, const Grid& coarse, const T* sf, T* sc) {
  launch(inject_kernel<T>, dim3(blocks_for(coarse.nodes())), dim3(BS), 0, st, fine, coarse, sf, sc);
}
template <typename T>
void launch_average_coef(hipStream_t st, const Grid& fine, const Grid& coarse, const T* cf, T* cc) {
  launch(average_coef_kernel<T>, dim3(blocks_for(coarse.elems())), dim3(BS), 0, st, fine, coarse, cf, cc);
}

// ------------------------------------------------------------------ coarsest level
// Element Jacobian columns of the (P, T) operator: mats[e][col][row], 16 x 16, local dof
// index 2 a + field.
template <typename T>
__global__ __launch_bounds__(BS) void elem_matrix_kernel(LevelView<T> L, double* __restrict__ mats) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long E = L.g.elems();
  if (t >= E * 16) return;
  const long e = t / 16;
  const int col = (int)(t % 16);
  const int i = (int)(e % L.g.nx), j = (int)((e / L.g.nx) % L.g.ny), k = (int)(e / ((long)L.g.nx * L.g.ny));
  T P[8], Tn[8], p[8], tt[8];
  for (int a = 0; a < 8; ++a) {
    const long n = L.g.node(i + (a & 1), j + ((a >> 1) & 1), k + ((a >> 2) & 1));
    P[a] = L.st[2 * n];
    Tn[a] = L.st[2 * n + 1];
    p[a] = (T)0;
    tt[a] = (T)0;
  }
  if (col & 1) tt[col >> 1] = (T)1; else p[col >> 1] = (T)1;
  Lin<T> lin;
  linearize_q(P, Tn, L.coef[2 * e], L.coef[2 * e + 1], L.c.source(i, j, k), L.c, lin);
  T yP[8] = {0}, yT[8] = {0}, yU[3][8];
  elem_jv<T, false>(lin, p, tt, L.c, yP, yT, yU);
  double* m = mats + (e * 16 + col) * 16;
  for (int a = 0; a < 8; ++a) {
    m[2 * a] = (double)yP[a];
    m[2 * a + 1] = (double)yT[a];
  }
}

// Dense assembly, one thread per entry A[r][c] (row-major), constrained rows and
// columns replaced by the identity.
__global__ void dense_assemble_kernel(Grid g, const double* __restrict__ mats, double* __restrict__ A) {
  const long n = 2 * g.nodes();
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * n) return;
  const long r = t / n, c = t % n;
  const long nr = r / 2, nc_ = c / 2;
  const int fr = (int)(r % 2), fc = (int)(c % 2);
  const int ir = (int)(nr % (g.nx + 1)), jr = (int)((nr / (g.nx + 1)) % (g.ny + 1)), kr = (int)(nr / ((long)(g.nx + 1) * (g.ny + 1)));
  const int ic = (int)(nc_ % (g.nx + 1)), jc = (int)((nc_ / (g.nx + 1)) % (g.ny + 1)), kc = (int)(nc_ / ((long)(g.nx + 1) * (g.ny + 1)));
  const bool rfix = fr == 0 ? g.pfix(ir, jr, kr) : g.tfix(ir, jr, kr);
  const bool cfix = fc == 0 ? g.pfix(ic, jc, kc) : g.tfix(ic, jc, kc);
  if (rfix || cfix) {
    A[t] = (r == c) ? 1.0 : 0.0;
    return;
  }
  double s = 0.0;
  // elements containing node r: lower corner (ir - ar, jr - br, kr - cr)
  for (int cr = 0; cr < 2; ++cr)
    for (int br = 0; br < 2; ++br)
      for (int ar = 0; ar < 2; ++ar) {
        const int ei = ir - ar, ej = jr - br, ek = kr - cr;
        if (ei < 0 || ej < 0 || ek < 0 || ei >= g.nx || ej >= g.ny || ek >= g.nz) continue;
        const int ac = ic - ei, bc = jc - ej, ccz = kc - ek;
        if (ac < 0 || ac > 1 || bc < 0 || bc > 1 || ccz < 0 || ccz > 1) continue;
        const long e = g.elem(ei, ej, ek);
        const int la_r = ar + 2 * br + 4 * cr, la_c = ac + 2 * bc + 4 * ccz;
        s += mats[(e * 16 + 2 * la_c + fc) * 16 + 2 * la_r + fr];
      }
  A[t] = s;
}

template <typename T>
void launch_coarse_assemble(hipStream_t st, const LevelView<T>& L, double* elem_mats, double* A) {
  const long E = L.g.elems();
  launch(elem_matrix_kernel<T>, dim3(blocks_for(E * 16)), dim3(BS), 0, st, L, elem_mats);
  const long n = 2 * L.g.nodes();
  launch(dense_assemble_kernel, dim3(blocks_for(n * n)), dim3(BS), 0, st, L.g, elem_mats, A);
}

// In-place Gauss-Jordan inversion with partial pivoting: for pivot step k, the pivot p is
// the first row r >= k of largest |A[r][k]|; rows k and p are interchanged, the pivot row is
// scaled by 1 / A[p][k] (its column-k entry replaced by 1 first), and every other row r
// subtracts A[r][k] times it (its column-k entry replaced by 0 first), which builds the
// inverse in place.  The row interchanges are undone as column interchanges in reverse
// order at the end.

// The same inversion with the matrix held in registers, for n <= GJS_NMAX, and without row
// interchanges: the pivot of step k is the row p_k of largest |A[r][k]| among the rows
// not yet used as pivots (ties: lowest lane, then lowest slot; a NaN counts as largest).
// Row p_k is scaled and every other row eliminated exactly as above.  Column k then holds
// the column of the inverse that belongs to row p_k, so after n steps entry (r, c) is
// (A^-1)[s(r)][p_c], s(r) being the step that took row r as pivot: the write-back applies
// both permutations at once.
// Row r belongs to lane r % 64 (slot r / 64) of every wave, column c to wave c % 16 (slot
// c / 16).  In step k the wave holding column k finds the pivot with a wave reduction and
// puts the column and the pivot index in LDS (two buffers, so one barrier per step); each
// wave reads the pivot row's entries of its own columns from lane p % 64 with readlane.
constexpr int GJS_RI = 3, GJS_NW = 16, GJS_CJ = 10, GJS_NMAX = GJS_NW * GJS_CJ;   // 64 * GJS_RI >= GJS_NMAX

__device__ inline double readlane_f64(double x, int l) {
  const long long b = __double_as_longlong(x);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)b, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

__global__ __launch_bounds__(1024) void gauss_jordan_small_kernel(double* __restrict__ A, int n, int* __restrict__ perm) {
  __shared__ double colk[2][64 * GJS_RI];
  __shared__ int spiv[2];
  __shared__ int sp[GJS_NMAX];   // pivot row of each step
  __shared__ int ss[GJS_NMAX];   // step at which each row was the pivot
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  double a[GJS_RI][GJS_CJ];
#pragma unroll
  for (int i = 0; i < GJS_RI; ++i)
#pragma unroll
    for (int j = 0; j < GJS_CJ; ++j) {
      const int r = lane + 64 * i, c = w + GJS_NW * j;
      a[i][j] = (r < n && c < n) ? A[(long)r * n + c] : 0.0;
    }
  unsigned used = 0;   // bit i: row lane + 64 i is padding or has been a pivot
#pragma unroll
  for (int i = 0; i < GJS_RI; ++i)
    if (lane + 64 * i >= n) used |= 1u << i;
#pragma unroll
  for (int j0 = 0; j0 < GJS_CJ; ++j0) {
    for (int wk = 0; wk < GJS_NW && wk + GJS_NW * j0 < n; ++wk) {
      const int k = wk + GJS_NW * j0, buf = k & 1;
      if (w == wk) {
        double best = -1.0;
        int bi = -1;
#pragma unroll
        for (int i = 0; i < GJS_RI; ++i) {
          double v = fabs(a[i][j0]);
          if (v != v) v = __builtin_inf();
          if (!((used >> i) & 1u) && v > best) { best = v; bi = lane + 64 * i; }
        }
        // at least one row is unused (k < n), so the maximum is >= 0 and names one
        double m = best;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
        const unsigned long long hit = __ballot(best == m);
        const int src = __builtin_amdgcn_readfirstlane(__builtin_ctzll(hit));
        const int p = __builtin_amdgcn_readlane(bi, src);
#pragma unroll
        for (int i = 0; i < GJS_RI; ++i) colk[buf][lane + 64 * i] = a[i][j0];
        if (lane == 0) spiv[buf] = p;
      }
      __syncthreads();
      const int p = __builtin_amdgcn_readfirstlane(spiv[buf]);
      const int pl = p & 63, pi = p >> 6;
      if (threadIdx.x == 0) { sp[k] = p; ss[p] = k; perm[k] = p; }
      const double ipv = 1.0 / colk[buf][p];
      double f[GJS_RI];
#pragma unroll
      for (int i = 0; i < GJS_RI; ++i) f[i] = colk[buf][lane + 64 * i] * ipv;
      double pr[GJS_CJ];   // row p in this wave's columns (wave-uniform)
      if (pi == 0) {
#pragma unroll
        for (int j = 0; j < GJS_CJ; ++j) pr[j] = readlane_f64(a[0][j], pl);
      } else if (pi == 1) {
#pragma unroll
        for (int j = 0; j < GJS_CJ; ++j) pr[j] = readlane_f64(a[1][j], pl);
      } else {
#pragma unroll
        for (int j = 0; j < GJS_CJ; ++j) pr[j] = readlane_f64(a[2][j], pl);
      }
#pragma unroll
      for (int i = 0; i < GJS_RI; ++i)
#pragma unroll
        for (int j = 0; j < GJS_CJ; ++j) a[i][j] = fma(-f[i], pr[j], a[i][j]);
      if (w == wk) {
#pragma unroll
        for (int i = 0; i < GJS_RI; ++i) a[i][j0] = -f[i];
      }
      if (lane == pl) {
        used |= 1u << pi;
#pragma unroll
        for (int i = 0; i < GJS_RI; ++i)
          if (i == pi) {
#pragma unroll
            for (int j = 0; j < GJS_CJ; ++j) a[i][j] = (w == wk && j == j0) ? ipv : pr[j] * ipv;
          }
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < GJS_RI; ++i)
#pragma unroll
    for (int j = 0; j < GJS_CJ; ++j) {
      const int r = lane + 64 * i, c = w + GJS_NW * j;
      if (r < n && c < n) A[(long)ss[r] * n + sp[c]] = a[i][j];
    }
}

// The same inversion for larger n over many workgroups, one launch per pivot step: every
// block picks the pivot of column k from a contiguous copy of that column (same rule as
// above), then all blocks update the matrix from Ain into Aout (two buffers, no in-place
// hazards) with the same operations, and copy the new column k + 1 out.
__global__ __launch_bounds__(256) void gj_column_kernel(const double* __restrict__ A, int n, int k,
                                                         double* __restrict__ col) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n) col[r] = A[(long)r * n + k];
}
__global__ __launch_bounds__(256) void gj_step_kernel(const double* __restrict__ Ain, double* __restrict__ Aout,
                                                       const double* __restrict__ colk, double* __restrict__ colnext,
                                                       int n, int k, int* __restrict__ perm) {
  __shared__ int sp;
  if (threadIdx.x < 64) {
    double best = -1.0;
    int bi = k;
    for (int r = k + (int)threadIdx.x; r < n; r += 64) {
      const double v = fabs(colk[r]);
      if (v > best) { best = v; bi = r; }
    }
    for (int off = 32; off > 0; off >>= 1) {
      const double ov = __shfl_down(best, off, 64);
      const int oi = __shfl_down(bi, off, 64);
      if (ov > best || (ov == best && oi < bi)) { best = ov; bi = oi; }
    }
    if (threadIdx.x == 0) sp = bi;
  }
  __syncthreads();
  const int p = sp;
  if (blockIdx.x == 0 && threadIdx.x == 0) perm[k] = p;
  const double ipv = 1.0 / Ain[(long)p * n + k];
  const double fk = Ain[(long)k * n + k];
  const int nn = n * n;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < nn; t += gridDim.x * blockDim.x) {
    const int r = t / n, c = t - r * n;
    const double pr = (c == k ? 1.0 : Ain[(long)p * n + c]) * ipv;
    double v;
    if (r == k) v = pr;
    else if (r == p) v = (c == k ? 0.0 : Ain[(long)k * n + c]) - fk * pr;
    else v = (c == k ? 0.0 : Ain[t]) - colk[r] * pr;
    Aout[t] = v;
    if (c == k + 1) colnext[r] = v;
  }
}
// inverse column map of the interchanges undone in reverse order (one block)
__global__ __launch_bounds__(1024) void gj_colmap_kernel(const int* __restrict__ perm, int n, int* __restrict__ inv) {
  extern __shared__ int sidx[];
  for (int j = threadIdx.x; j < n; j += blockDim.x) sidx[j] = j;
  __syncthreads();
  if (threadIdx.x == 0)
    for (int k = n - 1; k >= 0; --k) {
      const int q = perm[k], tmp = sidx[k];
      sidx[k] = sidx[q];
      sidx[q] = tmp;
    }
  __syncthreads();
  for (int j = threadIdx.x; j < n; j += blockDim.x) inv[sidx[j]] = j;
}
__global__ __launch_bounds__(256) void gj_permute_kernel(const double* __restrict__ src, double* __restrict__ dst,
                                                          int n, const int* __restrict__ inv) {
  const int nn = n * n;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < nn; t += gridDim.x * blockDim.x) {
    const int r = t / n, c = t - r * n;
    dst[(long)r * n + inv[c]] = src[t];
  }
}
__global__ __launch_bounds__(256) void copy_f64_kernel(const double* __restrict__ a, double* __restrict__ b, long n) {
  for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x) b[t] = a[t];
}

void launch_gauss_jordan(hipStream_t st, double* A, int n, int* perm, double* work) {
  if (n <= GJS_NMAX) {
    launch(gauss_jordan_small_kernel, dim3(1), dim3(1024), 0, st, A, n, perm);
    return;
  }
  // A holds 2 n^2 doubles (the inverse and, later, its transpose): both halves serve as
  // the step buffers here; work holds two columns, perm 2 n ints
  double* buf[2] = {A, A + (long)n * n};
  const int nb = std::min(1024, ceil_div((long)n * n, 256));
  launch(gj_column_kernel, dim3(ceil_div(n, 256)), dim3(256), 0, st, (const double*)A, n, 0, work);
  for (int k = 0; k < n; ++k)
    launch(gj_step_kernel, dim3(nb), dim3(256), 0, st, (const double*)buf[k & 1], buf[(k + 1) & 1],
           (const double*)(work + (long)(k & 1) * n), work + (long)((k + 1) & 1) * n, n, k, perm);
  launch(gj_colmap_kernel, dim3(1), dim3(1024), sizeof(int) * n, st, (const int*)perm, n, perm + n);
  double* src = buf[n & 1];
  double* dst = buf[(n + 1) & 1];
  launch(gj_permute_kernel, dim3(nb), dim3(256), 0, st, (const double*)src, dst, n, (const int*)(perm + n));
  if (dst != A) launch(copy_f64_kernel, dim3(nb), dim3(256), 0, st, (const double*)dst, A, (long)n * n);
}

// x = Ainv b (one wave per row) or x = Ainv^T b (one thread per column)
template <typename T>
__global__ void dense_apply_kernel(const double* __restrict__ Ainv, int n, int transpose, const T* __restrict__ b,
                                   T* __restrict__ x) {
  if (!transpose) {
    const int row = (int)((blockIdx.x * (long)blockDim.x + threadIdx.x) / 64);
    const int lane = threadIdx.x & 63;
    if (row >= n) return;
    double s = 0.0;
    for (int c = lane; c < n; c += 64) s += Ainv[(long)row * n + c] * (double)b[c];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if (lane == 0) x[row] = (T)s;
  } else {
    const int col = blockIdx.x * blockDim.x + threadIdx.x;
    if (col >= n) return;
    double s = 0.0;
    for (int r = 0; r < n; ++r) s += Ainv[(long)r * n + col] * (double)b[r];
    x[col] = (T)s;
  }
}

// Ainv holds A^-1 followed by (A^-1)^T (row-major n x n each); both products read rows.
template <typename T>
void launch_dense_apply(hipStream_t st, const double* Ainv, int n, bool transpose, const T* b, T* x) {
  const double* M = transpose ? Ainv + (long)n * n : Ainv;
  launch(dense_apply_kernel<T>, dim3(ceil_div((long)n * 64, BS)), dim3(BS), 0, st, M, n, 0, b, x);
}

__global__ void transpose_kernel(const double* __restrict__ A, double* __restrict__ At, int n) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long)n * n) return;
  const long r = t / n, c = t % n;
  At[c * n + r] = A[t];
}
void launch_dense_transpose(hipStream_t st, const double* A, double* At, int n) {
  launch(transpose_kernel, dim3(blocks_for((long)n * n)), dim3(BS), 0, st, A, At, n);
}

// ------------------------------------------------------------------ state / vectors
template <typename T>
__global__ void pack_state_kernel(long N, const double* __restrict__ s5, T* __restrict__ pt) {
  const long n = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  pt[2 * n] = (T)s5[5 * n + 3];
  pt[2 * n + 1] = (T)s5[5 * n + 4];
}
template <typename T>
void launch_pack_state(hipStream_t st, const Grid& g, const double* s5, T* pt) {
  launch(pack_state_kernel<T>, dim3(blocks_for(g.nodes())), dim3(BS), 0, st, g.nodes(), s5, pt);
}

// Preconditioner input of the (P, T) Krylov solve (see kernels.hpp)
template <typename T>
__global__ void pc_in_kernel(Grid g, T* __restrict__ v, const double* __restrict__ nrm, T inv_p, T inv_t,
                             const T* __restrict__ dinv, int transpose, T omega, T* __restrict__ b, T* __restrict__ x) {
  using P2 = typename Pair<T>::type;
  using Q4 = typename Quad<T>::type;
  const PlaneIdx q = plane_idx(g);
  if (!q.ok) return;
  const int n = g.node(q.i, q.j, q.k);
  const P2 vv = reinterpret_cast<const P2*>(v)[n];
  T vp = vv.x, vt = vv.y;
  if (nrm) {   // normalise the new Krylov vector in place (v <- v / |v|)
    const double s = 1.0 / nrm[0];
    vp = (T)(s * (double)vp);
    vt = (T)(s * (double)vt);
    reinterpret_cast<P2*>(v)[n] = P2{vp, vt};
  }
  const T bp = g.pfix(q.i, q.j, q.k) ? (T)0 : inv_p * vp;
  const T bt = g.tfix(q.i, q.j, q.k) ? (T)0 : inv_t * vt;
  reinterpret_cast<P2*>(b)[n] = P2{bp, bt};
  const Q4 D = reinterpret_cast<const Q4*>(dinv)[n];
  reinterpret_cast<P2*>(x)[n] =
      P2{omega * (D.x * bp + (transpose ? D.z : D.y) * bt), omega * ((transpose ? D.y : D.z) * bp + D.w * bt)};
}
template <typename T>
void launch_pc_in(hipStream_t st, const Grid& g, T* v, const double* nrm, T inv_p, T inv_t, const T* dinv,
                  bool transpose, T omega, T* b, T* x) {
  launch(pc_in_kernel<T>, plane_grid(g, 256), dim3(256), 0, st, g, v, nrm, inv_p, inv_t, dinv, transpose ? 1 : 0,
         omega, b, x);
}

template <typename T>
__global__ void pack_pt_kernel(long nodes, const double* __restrict__ r5, T* __restrict__ out, double s_p, double s_t) {
  for (long n = (long)blockIdx.x * blockDim.x + threadIdx.x; n < nodes; n += (long)gridDim.x * blockDim.x) {
    out[2 * n] = (T)(s_p * r5[5 * n + 3]);
    out[2 * n + 1] = (T)(s_t * r5[5 * n + 4]);
  }
}
template <typename T>
void launch_pack_pt(hipStream_t st, long nodes, const double* r5, T* out, double s_p, double s_t) {
  launch(pack_pt_kernel<T>, dim3(std::min(blocks_for(nodes), 4096)), dim3(BS), 0, st, nodes, r5, out, s_p,
                     s_t);
}

template <typename Ta, typename Tb>
__global__ void scale2_kernel(long nodes, const Ta* __restrict__ in, Tb* __restrict__ out, double s_p, double s_t) {
  for (long n = (long)blockIdx.x * blockDim.x + threadIdx.x; n < nodes; n += (long)gridDim.x * blockDim.x) {
    out[2 * n] = (Tb)(s_p * (double)in[2 * n]);
    out[2 * n + 1] = (Tb)(s_t * (double)in[2 * n + 1]);
  }
}
template <typename Ta, typename Tb>
void launch_scale2(hipStream_t st, long nodes, const Ta* in, Tb* out, double s_p, double s_t) {
  launch((scale2_kernel<Ta, Tb>), dim3(std::min(blocks_for(nodes), 4096)), dim3(BS), 0, st, nodes, in, out,
                     s_p, s_t);
}

template <typename Ta, typename Tb>
__global__ void normalize_copy_kernel(const double* __restrict__ nrm, Ta* v, Tb* __restrict__ out, long n) {
  const double s = nrm ? 1.0 / nrm[0] : 1.0;
  for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x) {
    const Ta a = nrm ? (Ta)(s * (double)v[t]) : v[t];
    if (nrm) v[t] = a;
    out[t] = (Tb)a;
  }
}
template <typename Ta, typename Tb>
void launch_normalize_copy(hipStream_t st, const double* nrm, Ta* v, Tb* out, long n) {
  launch((normalize_copy_kernel<Ta, Tb>), dim3(std::min(blocks_for(n), 4096)), dim3(BS), 0, st, nrm, v, out, n);
}

template <typename T>
__global__ void unpack_pt_kernel(Grid g, const T* __restrict__ x, double* __restrict__ out5) {
  const PlaneIdx q = plane_idx(g);
  if (!q.ok) return;
  const int n = g.node(q.i, q.j, q.k);
  out5[5 * (long)n + 3] = g.pfix(q.i, q.j, q.k) ? 0.0 : (double)x[2 * n];
  out5[5 * (long)n + 4] = g.tfix(q.i, q.j, q.k) ? 0.0 : (double)x[2 * n + 1];
}
template <typename T>
void launch_unpack_pt(hipStream_t st, const Grid& g, const T* x, double* out5) {
  launch(unpack_pt_kernel<T>, plane_grid(g, 256), dim3(256), 0, st, g, x, out5);
}

__global__ void mask_state_kernel(Grid g, double* __restrict__ s5) {
  const long n = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= g.nodes()) return;
  const int i = (int)(n % (g.nx + 1)), j = (int)((n / (g.nx + 1)) % (g.ny + 1)), k = (int)(n / ((long)(g.nx + 1) * (g.ny + 1)));
  if (g.pfix(i, j, k)) s5[5 * n + 3] = 0.0;
  if (g.tfix(i, j, k)) s5[5 * n + 4] = 0.0;
  if (g.ufix(i, j, 0)) s5[5 * n] = 0.0;
  if (g.ufix(i, j, 1)) s5[5 * n + 1] = 0.0;
}
void launch_mask_state(hipStream_t st, const Grid& g, double* s5) {
  launch(mask_state_kernel, dim3(blocks_for(g.nodes())), dim3(BS), 0, st, g, s5);
}

template <typename Ta, typename Tb>
__global__ void convert_kernel(const Ta* __restrict__ a, Tb* __restrict__ b, long n, double scale) {
  for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x)
    b[t] = (Tb)(scale * (double)a[t]);
}
template <typename Ta, typename Tb>
void launch_convert(hipStream_t st, const Ta* a, Tb* b, long n, double scale) {
  launch((convert_kernel<Ta, Tb>), dim3(std::min(blocks_for(n), 4096)), dim3(BS), 0, st, a, b, n, scale);
}

__global__ void axpy_kernel(double a, const double* __restrict__ x, const double* __restrict__ y, double* __restrict__ out, long n) {
  for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x)
    out[t] = a * x[t] + y[t];
}
void launch_axpy(hipStream_t st, double a, const double* x, const double* y, double* out, long n) {
  launch(axpy_kernel, dim3(std::min(blocks_for(n), 4096)), dim3(BS), 0, st, a, x, y, out, n);
}


// x = omega D^-1 b (or D^-T): the first damped block-Jacobi sweep from a zero iterate
template <typename T>
__global__ void diag_scale_kernel(long N, const T* __restrict__ dinv, int transpose, T omega, const T* __restrict__ b,
                                  T* __restrict__ x) {
  const long n = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  const T* D = dinv + 4 * n;
  const T bp = b[2 * n], bt = b[2 * n + 1];
  if (!transpose) {
    x[2 * n] = omega * (D[0] * bp + D[1] * bt);
    x[2 * n + 1] = omega * (D[2] * bp + D[3] * bt);
  } else {
    x[2 * n] = omega * (D[0] * bp + D[2] * bt);
    x[2 * n + 1] = omega * (D[1] * bp + D[3] * bt);
  }
}
template <typename T>
void launch_diag_scale(hipStream_t st, const Grid& g, const T* dinv, bool transpose, T omega, const T* b, T* x) {
  launch(diag_scale_kernel<T>, dim3(blocks_for(g.nodes())), dim3(BS), 0, st, g.nodes(), dinv,
                     transpose ? 1 : 0, omega, b, x);
}

// out = b - out  (restart residual)
template <typename T>
__global__ void rsub_kernel(const T* __restrict__ b, T* __restrict__ out, long n) {
  for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x)
    out[t] = b[t] - out[t];
}
template <typename T>
void launch_rsub(hipStream_t st, const T* b, T* out, long n) {
  launch(rsub_kernel<T>, dim3(std::min(blocks_for(n), 4096)), dim3(BS), 0, st, b, out, n);
}

// ------------------------------------------------------------------ reductions
__device__ inline double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Vector loads of 16 bytes: 4 floats or 2 doubles per lane.
template <typename T> struct Vec16;
template <> struct Vec16<float> { using type = float4; static constexpr int W = 4; };
template <> struct Vec16<double> { using type = double2; static constexpr int W = 2; };

__device__ inline double hsum(float4 a, float4 b) {
  return (double)a.x * b.x + (double)a.y * b.y + (double)a.z * b.z + (double)a.w * b.w;
}
__device__ inline double hsum(double2 a, double2 b) { return a.x * b.x + a.y * b.y; }

// Multi-dot and multi-axpy of the Krylov solver.
//
// Both kernels split the vectors into one contiguous chunk per block and walk it in
// sub-tiles of KBS x KT<T>::U 16-byte vectors.  The multi-dot keeps the sub-tile of w in
// registers and streams the basis vectors in groups of KGT<T>::G, issuing each group's loads
// before the previous group is used (two groups of KT<T>::U loads in flight per thread), so
// w and every basis vector are read once and the memory system does not wait on the
// reductions; each wave reduces its partial dot products and its lane 0 adds them to the
// wave's own row of LDS sums (no barrier between groups); the block adds the wave rows in
// order at the end.  Every block but the last covers whole sub-tiles.  Full sub-tiles take
// unguarded vector loads, so the loads of a group are all in flight together.  A second,
// one-block launch adds the per-block sums in block order, so results are deterministic;
// the launch boundary makes the partials visible across the chip's L2 caches (a
// device-scope fence per block, with the atomic ticket of a last-block scheme, costs far
// more here).  The multi-axpy updates its sub-tile of w with all basis vectors in float64
// and writes it back once, with the norm of the result reduced the same way.
constexpr int KBS = 256;   // threads per block
// 16-byte vectors per thread and sub-tile: 3072 float32 / 2048 float64 elements per sub-tile
// (the 529 sub-tiles of 4096 float32 elements that a 1M-element (P, T) vector made with
// 512-thread blocks needed two rounds of the 512 resident blocks; 705 sub-tiles of 3072
// fit in one round of 1024)
template <typename T>
struct KT {
  static constexpr int U = sizeof(T) == 4 ? 3 : 4;
};
// basis vectors per group; two groups are in flight at a time (the next group's loads are
// issued before the current group is used), so that the memory system never waits for a
// group's reductions
template <typename T>
struct KGT {
  static constexpr int G = 2;                          // multi-dot
  static constexpr int GA = 1;                         // multi-axpy (its float64 accumulators take the rest)
};
// blocks: at most RED_BLOCKS (partials of column c at part[c * RED_BLOCKS + b])

// out[c] = sum over b < nblk of part[c * stride + b] for c < ncol, in a fixed order
// (sqrt of the column sum for c >= sqrt_from).  One block: (column, 16 lanes), each lane
// with 8 independent loads in flight.
__global__ __launch_bounds__(KBS) void reduce_cols_kernel(const double* __restrict__ part, long stride, int nblk,
                                                          int ncol, int sqrt_from, double* __restrict__ out,
                                                          double* __restrict__ hout) {
  constexpr int LN = 16;
  for (int c0 = 0; c0 < ncol; c0 += KBS / LN) {
    const int c = c0 + (int)(threadIdx.x / LN), sub = threadIdx.x % LN;
    double s = 0.0;
    if (c < ncol) {
      const double* pc = part + (long)c * stride;
      double a[8] = {0, 0, 0, 0, 0, 0, 0, 0};
      int b = sub;
      for (; b + 7 * LN < nblk; b += 8 * LN) {
#pragma unroll
        for (int q = 0; q < 8; ++q) a[q] += pc[b + q * LN];
      }
      for (; b < nblk; b += LN) a[0] += pc[b];
      s = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
    }
#pragma unroll
    for (int off = LN / 2; off > 0; off >>= 1) s += __shfl_down(s, off, LN);
    if (sub == 0 && c < ncol) {
      const double v = c >= sqrt_from ? sqrt(s) : s;
      out[c] = v;
      if (hout) hout[c] = v;
    }
  }
}

// 16-byte vector idx of p: a plain vector load when FULL (the caller has checked that the
// whole sub-tile lies below lim <= n / W), else zero-filled at and past lim and n.
template <bool FULL, typename T>
__device__ inline typename Vec16<T>::type load16(const T* __restrict__ p, long idx, long lim, long nv, long n) {
  using V16 = typename Vec16<T>::type;
  constexpr int VW = Vec16<T>::W;
  if (FULL || (idx < nv && idx < lim)) return reinterpret_cast<const V16*>(p)[idx];
  V16 r;
  T* pr = reinterpret_cast<T*>(&r);
#pragma unroll
  for (int q = 0; q < VW; ++q) {
    const long e = idx * VW + q;
    pr[q] = (idx < lim && e < n) ? p[e] : (T)0;
  }
  return r;
}

// Contiguous chunk of 16-byte vectors of block b, [beg, end): whole sub-tiles, so that only
// the last block ends in a partial one
template <typename T>
__device__ inline void block_chunk(long nvt, long& beg, long& end) {
  constexpr long SUB = (long)KBS * KT<T>::U;
  const long per = ((nvt + gridDim.x - 1) / gridDim.x + SUB - 1) / SUB * SUB;
  beg = (long)blockIdx.x * per;
  end = beg + per < nvt ? beg + per : nvt;
}

// One group of the multi-dot's basis vectors (column c0 + g; past cnt, w itself for the
// norm column or as filler)
template <bool FULL, typename T>
__device__ __attribute__((always_inline)) inline void mdot_load(const T* __restrict__ V, long ld, int cnt,
                                                                const T* __restrict__ w, int c0, long base, long end,
                                                                long nv, long n,
                                                                typename Vec16<T>::type (&vt)[KGT<T>::G][KT<T>::U]) {
#pragma unroll
  for (int g = 0; g < KGT<T>::G; ++g) {
    const T* v = c0 + g < cnt ? V + (long)(c0 + g) * ld : w;
#pragma unroll
    for (int u = 0; u < KT<T>::U; ++u) vt[g][u] = load16<FULL>(v, base + u * KBS + threadIdx.x, end, nv, n);
  }
}
template <typename T>
__device__ __attribute__((always_inline)) inline void mdot_use(const typename Vec16<T>::type (&vt)[KGT<T>::G][KT<T>::U],
                                                               const typename Vec16<T>::type (&wt)[KT<T>::U], int c0,
                                                               int ncol, double (*wpart)[MAXC + 1]) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int g = 0; g < KGT<T>::G; ++g) {
    double s = 0.0;
#pragma unroll
    for (int u = 0; u < KT<T>::U; ++u) s += hsum(vt[g][u], wt[u]);
    s = wave_sum(s);
    if (lane == 0 && c0 + g < ncol) wpart[wv][c0 + g] += s;
  }
}

// One sub-tile of the multi-dot: lane 0 of each wave adds the wave's partial dot products
// to its own row of wpart (fixed order, no barrier).
template <bool FULL, typename T>
__device__ inline void mdot_subtile(const T* __restrict__ V, long ld, int cnt, int ncol, const T* __restrict__ w,
                                    long base, long end, long nv, long n, double (*wpart)[MAXC + 1]) {
  using V16 = typename Vec16<T>::type;
  constexpr int G = KGT<T>::G;
  V16 wt[KT<T>::U];
#pragma unroll
  for (int u = 0; u < KT<T>::U; ++u) wt[u] = load16<FULL>(w, base + u * KBS + threadIdx.x, end, nv, n);
  V16 va[G][KT<T>::U], vb[G][KT<T>::U];
  mdot_load<FULL>(V, ld, cnt, w, 0, base, end, nv, n, va);
  for (int c0 = 0; c0 < ncol; c0 += 2 * G) {
    if (c0 + G < ncol) mdot_load<FULL>(V, ld, cnt, w, c0 + G, base, end, nv, n, vb);
    mdot_use<T>(va, wt, c0, ncol, wpart);
    if (c0 + 2 * G < ncol) mdot_load<FULL>(V, ld, cnt, w, c0 + 2 * G, base, end, nv, n, va);
    if (c0 + G < ncol) mdot_use<T>(vb, wt, c0 + G, ncol, wpart);
  }
}

// out[c] = V[c] . w for c < cnt; with `with_norm` also out[cnt] = w . w
template <typename T>
__global__ __launch_bounds__(KBS) __attribute__((amdgpu_waves_per_eu(4))) void mdot_kernel(
    const T* __restrict__ V, long ld, int cnt, const T* __restrict__ w, long n, int with_norm,
    double* __restrict__ part) {
  constexpr int VW = Vec16<T>::W;
  __shared__ double wpart[KBS / 64][MAXC + 1];
  const int ncol = cnt + with_norm;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0)
    for (int c = 0; c <= MAXC; ++c) wpart[wv][c] = 0.0;
  const long nv = n / VW, nvt = (n + VW - 1) / VW;
  long beg, end;
  block_chunk<T>(nvt, beg, end);
  const long lim = end < nv ? end : nv;
  for (long base = beg; base < end; base += (long)KBS * KT<T>::U) {
    if (base + (long)KBS * KT<T>::U <= lim) mdot_subtile<true>(V, ld, cnt, ncol, w, base, end, nv, n, wpart);
    else mdot_subtile<false>(V, ld, cnt, ncol, w, base, end, nv, n, wpart);
  }
  __syncthreads();
  if ((int)threadIdx.x < ncol) {
    double s = 0.0;
#pragma unroll
    for (int w2 = 0; w2 < KBS / 64; ++w2) s += wpart[w2][threadIdx.x];
    part[(long)threadIdx.x * RED_BLOCKS + blockIdx.x] = s;
  }
}

// blocks for streaming n elements: one sub-tile each, at most RED_BLOCKS
template <typename T>
static int stream_blocks(long n) {
  const long nvt = (n + Vec16<T>::W - 1) / Vec16<T>::W;
  const long sub = (long)KBS * KT<T>::U;
  return (int)std::max<long>(1, std::min<long>(RED_BLOCKS, (nvt + sub - 1) / sub));
}

template <typename T>
void launch_mdot(hipStream_t st, const T* V, long ld, int cnt, const T* w, long n, double* part, double* out,
                 bool with_norm, double* hout) {
  const int nb = stream_blocks<T>(n);
  const int ncol = cnt + (with_norm ? 1 : 0);
  launch(mdot_kernel<T>, dim3(nb), dim3(KBS), 0, st, V, ld, cnt, w, n, with_norm ? 1 : 0, part);
  launch(reduce_cols_kernel, dim3(1), dim3(KBS), 0, st, part, (long)RED_BLOCKS, nb, ncol, ncol, out, hout);
}

// out[c] = sum over blocks of part[b][c] in a fixed order; sqrt if do_sqrt.  One block of
// 1024 threads: (column, 32 lanes), each lane with 8 independent loads in flight.
__global__ __launch_bounds__(1024) void reduce_parts_kernel(const double* __restrict__ part, int nblk, int cnt,
                                                            double* __restrict__ out, int do_sqrt,
                                                            double* __restrict__ hout) {
  const int c = threadIdx.x >> 5, sub = threadIdx.x & 31;
  double a[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (c < cnt) {
    int b = sub;
    for (; b + 7 * 32 < nblk; b += 8 * 32) {
#pragma unroll
      for (int q = 0; q < 8; ++q) a[q] += part[(b + q * 32) * MAXC + c];
    }
    for (; b < nblk; b += 32) a[0] += part[b * MAXC + c];
  }
  double s = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
  for (int off = 16; off > 0; off >>= 1) s += __shfl_down(s, off, 32);
  if (sub == 0 && c < cnt) {
    const double v = do_sqrt ? sqrt(s) : s;
    out[c] = v;
    if (hout) hout[c] = v;
  }
}

// One group of the multi-axpy's basis vectors (rows past cnt re-read row c0 with weight 0)
template <bool FULL, typename T>
__device__ __attribute__((always_inline)) inline void maxpy_load(const T* __restrict__ V, long ld, int cnt, int c0,
                                                                 long base, long end, long nv, long n,
                                                                 typename Vec16<T>::type (&vt)[KGT<T>::GA][KT<T>::U]) {
#pragma unroll
  for (int g = 0; g < KGT<T>::GA; ++g) {
    const T* v = V + (long)(c0 + g < cnt ? c0 + g : c0) * ld;
#pragma unroll
    for (int u = 0; u < KT<T>::U; ++u) vt[g][u] = load16<FULL>(v, base + u * KBS + threadIdx.x, end, nv, n);
  }
}
template <typename T>
__device__ __attribute__((always_inline)) inline void maxpy_use(const typename Vec16<T>::type (&vt)[KGT<T>::GA][KT<T>::U],
                                                                const double* hs, int cnt, int c0,
                                                                double (&a)[KT<T>::U][Vec16<T>::W]) {
#pragma unroll
  for (int g = 0; g < KGT<T>::GA; ++g) {
    const double hc = c0 + g < cnt ? hs[c0 + g] : 0.0;
#pragma unroll
    for (int u = 0; u < KT<T>::U; ++u) {
      const T* pv = reinterpret_cast<const T*>(&vt[g][u]);
#pragma unroll
      for (int q = 0; q < Vec16<T>::W; ++q) a[u][q] += hc * (double)pv[q];
    }
  }
}

// One sub-tile of the multi-axpy; returns the partial sum of squares of the result.
template <bool FULL, typename T>
__device__ inline double maxpy_subtile(const T* __restrict__ V, long ld, int cnt, const double* hs, T* __restrict__ w,
                                       long base, long end, long nv, long n) {
  using V16 = typename Vec16<T>::type;
  constexpr int VW = Vec16<T>::W;
  double a[KT<T>::U][VW];
#pragma unroll
  for (int u = 0; u < KT<T>::U; ++u) {
    const V16 wv = load16<FULL>(w, base + u * KBS + threadIdx.x, end, nv, n);
    const T* pw = reinterpret_cast<const T*>(&wv);
#pragma unroll
    for (int q = 0; q < VW; ++q) a[u][q] = (double)pw[q];
  }
  constexpr int G = KGT<T>::GA;
  V16 va[G][KT<T>::U], vb[G][KT<T>::U];
  maxpy_load<FULL>(V, ld, cnt, 0, base, end, nv, n, va);
  for (int c0 = 0; c0 < cnt; c0 += 2 * G) {
    if (c0 + G < cnt) maxpy_load<FULL>(V, ld, cnt, c0 + G, base, end, nv, n, vb);
    maxpy_use<T>(va, hs, cnt, c0, a);
    if (c0 + 2 * G < cnt) maxpy_load<FULL>(V, ld, cnt, c0 + 2 * G, base, end, nv, n, va);
    if (c0 + G < cnt) maxpy_use<T>(vb, hs, cnt, c0 + G, a);
  }
  double nrm = 0.0;
#pragma unroll
  for (int u = 0; u < KT<T>::U; ++u) {
    const long idx = base + u * KBS + threadIdx.x;
    V16 wv;
    T* pw = reinterpret_cast<T*>(&wv);
#pragma unroll
    for (int q = 0; q < VW; ++q) {
      pw[q] = (T)a[u][q];
      nrm += (double)pw[q] * (double)pw[q];
    }
    if (FULL || (idx < nv && idx < end)) {
      reinterpret_cast<V16*>(w)[idx] = wv;
    } else if (idx < end) {
#pragma unroll
      for (int q = 0; q < VW; ++q)
        if (idx * VW + q < n) w[idx * VW + q] = pw[q];
    }
  }
  return nrm;
}

// w += sign * sum_c h[c] V[c]; with nrm_out also nrm_out[0] = |w| (after the update)
template <typename T>
__global__ __launch_bounds__(KBS) __attribute__((amdgpu_waves_per_eu(4))) void maxpy_kernel(
    const T* __restrict__ V, long ld, int cnt, const double* __restrict__ h, double sign, T* __restrict__ w, long n,
    double* __restrict__ part) {
  constexpr int VW = Vec16<T>::W;
  __shared__ double hs[MAXC];
  __shared__ double red[KBS / 64];
  if ((int)threadIdx.x < cnt) hs[threadIdx.x] = sign * h[threadIdx.x];
  __syncthreads();
  const long nv = n / VW, nvt = (n + VW - 1) / VW;
  long beg, end;
  block_chunk<T>(nvt, beg, end);
  const long lim = end < nv ? end : nv;
  double nrm = 0.0;
  for (long base = beg; base < end; base += (long)KBS * KT<T>::U) {
    if (base + (long)KBS * KT<T>::U <= lim) nrm += maxpy_subtile<true>(V, ld, cnt, hs, w, base, end, nv, n);
    else nrm += maxpy_subtile<false>(V, ld, cnt, hs, w, base, end, nv, n);
  }
  if (part) {
    const double s = wave_sum(nrm);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
      double tot = 0.0;
      for (int w2 = 0; w2 < KBS / 64; ++w2) tot += red[w2];
      part[blockIdx.x] = tot;
    }
  }
}

template <typename T>
void launch_maxpy(hipStream_t st, const T* V, long ld, int cnt, const double* h, double sign, T* w, long n, double* part,
                  double* nrm_out, double* hnrm_out) {
  const int nb = stream_blocks<T>(n);
  launch(maxpy_kernel<T>, dim3(nb), dim3(KBS), 0, st, V, ld, cnt, h, sign, w, n,
                     nrm_out ? part : nullptr);
  if (nrm_out)
    launch(reduce_cols_kernel, dim3(1), dim3(KBS), 0, st, part, (long)RED_BLOCKS, nb, 1, 0, nrm_out, hnrm_out);
}

template <typename T>
__global__ void scale_inv_kernel(const double* __restrict__ nrm, const T* __restrict__ w, T* __restrict__ v, long n) {
  const double s = 1.0 / nrm[0];
  for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x)
    v[t] = (T)(s * (double)w[t]);
}
template <typename T>
void launch_scale_inv(hipStream_t st, const double* nrm, const T* w, T* v, long n) {
  launch(scale_inv_kernel<T>, dim3(std::min(blocks_for(n), 4096)), dim3(BS), 0, st, nrm, w, v, n);
}

template <typename T>
__global__ __launch_bounds__(BS) void norm_kernel(const T* __restrict__ a, long n, double* __restrict__ part) {
  __shared__ double red[BS / 64];
  double s = 0.0;
  for (long t = (long)blockIdx.x * BS + threadIdx.x; t < n; t += (long)gridDim.x * BS) {
    const double v = (double)a[t];
    s += v * v;
  }
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double tot = 0.0;
    for (int w2 = 0; w2 < BS / 64; ++w2) tot += red[w2];
    part[blockIdx.x * MAXC] = tot;
  }
}
template <typename T>
void launch_norm(hipStream_t st, const T* a, long n, double* part, double* out, double* hout) {
  launch(norm_kernel<T>, dim3(RED_BLOCKS), dim3(BS), 0, st, a, n, part);
  launch(reduce_parts_kernel, dim3(1), dim3(1024), 0, st, part, RED_BLOCKS, 1, out, 1, hout);
}

__global__ __launch_bounds__(BS) void field_norms_kernel(const double* __restrict__ a, const double* __restrict__ b,
                                                         long nodes, double* __restrict__ part) {
  __shared__ double red[BS / 64][10];
  double s[10];
#pragma unroll
  for (int f = 0; f < 10; ++f) s[f] = 0.0;
  for (long n = (long)blockIdx.x * BS + threadIdx.x; n < nodes; n += (long)gridDim.x * BS) {
#pragma unroll
    for (int f = 0; f < 5; ++f) {
      const double v = a[5 * n + f];
      s[f] += v * v;
      if (b) {
        const double u = b[5 * n + f];
        s[5 + f] += u * u;
      }
    }
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int f = 0; f < 10; ++f) {
    const double t = wave_sum(s[f]);
    if (lane == 0) red[wid][f] = t;
  }
  __syncthreads();
  if (threadIdx.x < 10) {
    double tot = 0.0;
    for (int w2 = 0; w2 < BS / 64; ++w2) tot += red[w2][threadIdx.x];
    part[blockIdx.x * MAXC + threadIdx.x] = tot;
  }
}
void launch_field_norms(hipStream_t st, const double* a, const double* b, long nodes, double* part, double* out) {
  launch(field_norms_kernel, dim3(RED_BLOCKS), dim3(BS), 0, st, a, b, nodes, part);
  launch(reduce_parts_kernel, dim3(1), dim3(1024), 0, st, part, RED_BLOCKS, 10, out, 1, (double*)nullptr);
}

// ------------------------------------------------------------------ design chain
// Cone filter y_e = sum_j w_ej x_j / sum_j w_ej, w_ej = max(0, R - |c_e - c_j| / h) over
// in-grid elements.  Transpose: y_j = sum_e w_ej (x_e / W_e), done as tmp_e = x_e / W_e
// followed by the unnormalised symmetric stencil.
__device__ inline double cone_weight_sum(const Grid& g, int i, int j, int k, double R, int r) {
  double ws = 0.0;
  for (int dk = -r; dk <= r; ++dk)
    for (int dj = -r; dj <= r; ++dj)
      for (int di = -r; di <= r; ++di) {
        const double w = R - sqrt((double)(di * di + dj * dj + dk * dk));
        const int a = i + di, b = j + dj, c = k + dk;
        if (w > 0.0 && a >= 0 && a < g.nx && b >= 0 && b < g.ny && c >= 0 && c < g.nz) ws += w;
      }
  return ws;
}

__global__ void cone_kernel(Grid g, double R, int r, const double* __restrict__ x, double* __restrict__ y, int mode) {
  // mode 0: normalised forward; 1: divide by W (first pass of the transpose);
  // 2: unnormalised stencil (second pass of the transpose)
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= g.elems()) return;
  const int i = (int)(e % g.nx), j = (int)((e / g.nx) % g.ny), k = (int)(e / ((long)g.nx * g.ny));
  if (mode == 1) {
    y[e] = x[e] / cone_weight_sum(g, i, j, k, R, r);
    return;
  }
  double s = 0.0, ws = 0.0;
  for (int dk = -r; dk <= r; ++dk)
    for (int dj = -r; dj <= r; ++dj)
      for (int di = -r; di <= r; ++di) {
        const double w = R - sqrt((double)(di * di + dj * dj + dk * dk));
        const int a = i + di, b = j + dj, c = k + dk;
        if (w > 0.0 && a >= 0 && a < g.nx && b >= 0 && b < g.ny && c >= 0 && c < g.nz) {
          s += w * x[g.elem(a, b, c)];
          ws += w;
        }
      }
  y[e] = mode == 0 ? s / ws : s;
}

void launch_cone_filter(hipStream_t st, const Grid& g, double radius, const double* x, double* y, bool transpose,
                        double* tmp) {
  const long E = g.elems();
  if (radius <= 0.0) {
    (void)hipMemcpyAsync(y, x, sizeof(double) * E, hipMemcpyDeviceToDevice, st);
    return;
  }
  const int r = (int)ceil(radius);
  if (!transpose) {
    launch(cone_kernel, dim3(blocks_for(E)), dim3(BS), 0, st, g, radius, r, x, y, 0);
  } else {
    launch(cone_kernel, dim3(blocks_for(E)), dim3(BS), 0, st, g, radius, r, x, tmp, 1);
    launch(cone_kernel, dim3(blocks_for(E)), dim3(BS), 0, st, g, radius, r, tmp, y, 2);
  }
}

__global__ void ramp_kernel(long E, const double* __restrict__ gam, double k_f, double k_s, double q_c, double kap_f,
                            double kap_s, double q_p, double* __restrict__ c64, float* __restrict__ c32,
                            double* __restrict__ dk, double* __restrict__ dkap) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= E) return;
  double k, kap, a, b;
  ramp<double>(gam[e], k_f, k_s, q_c, kap_f, kap_s, q_p, k, kap, a, b);
  c64[2 * e] = k;
  c64[2 * e + 1] = kap;
  c32[2 * e] = (float)k;
  c32[2 * e + 1] = (float)kap;
  dk[e] = a;
  dkap[e] = b;
}
void launch_ramp(hipStream_t st, long E, const double* gamma, double k_f, double k_s, double q_c, double kap_f,
                 double kap_s, double q_p, double* coef64, float* coef32, double* dk, double* dkap) {
  launch(ramp_kernel, dim3(blocks_for(E)), dim3(BS), 0, st, E, gamma, k_f, k_s, q_c, kap_f, kap_s, q_p,
                     coef64, coef32, dk, dkap);
}

// ------------------------------------------------------------------ sensitivities
__global__ __launch_bounds__(BS) void sensitivity_kernel(Grid g, ElemConst<double> c, const double* __restrict__ coef,
                                   const double* __restrict__ dk, const double* __restrict__ dkap,
                                   const double* __restrict__ s5, const double* __restrict__ l5, double* __restrict__ out) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= g.elems()) return;
  const int i = (int)(e % g.nx), j = (int)((e / g.nx) % g.ny), k = (int)(e / ((long)g.nx * g.ny));
  double P[8], Tn[8], lP[8], lT[8], lU[3][8];
  for (int a = 0; a < 8; ++a) {
    const int ii = i + (a & 1), jj = j + ((a >> 1) & 1), kk = k + ((a >> 2) & 1);
    const long n = g.node(ii, jj, kk);
    P[a] = s5[5 * n + 3];
    Tn[a] = s5[5 * n + 4];
    lP[a] = g.pfix(ii, jj, kk) ? 0.0 : l5[5 * n + 3];
    lT[a] = g.tfix(ii, jj, kk) ? 0.0 : l5[5 * n + 4];
    for (int d = 0; d < 3; ++d) lU[d][a] = g.ufix(ii, jj, d) ? 0.0 : l5[5 * n + d];
  }
  Lin<double> L;
  linearize_q(P, Tn, coef[2 * e], coef[2 * e + 1], c.source(i, j, k), c, L);
  out[e] = elem_sensitivity<double, true>(L, lP, lT, lU, dk[e], dkap[e], c);
}
void launch_sensitivity(hipStream_t st, const Grid& g, const ElemConst<double>& c, const double* coef,
                        const double* dk, const double* dkap, const double* s5, const double* lam5, double* out) {
  launch(sensitivity_kernel, dim3(blocks_for(g.elems())), dim3(BS), 0, st, g, c, coef, dk, dkap, s5, lam5, out);
}

// ------------------------------------------------------------------ coefficient means
__global__ __launch_bounds__(BS) void coef_sum_kernel(const double* __restrict__ coef, long E, double* __restrict__ part) {
  __shared__ double red[BS / 64][2];
  double a = 0.0, b = 0.0;
  for (long e = (long)blockIdx.x * BS + threadIdx.x; e < E; e += (long)gridDim.x * BS) {
    a += coef[2 * e];
    b += coef[2 * e + 1];
  }
  a = wave_sum(a);
  b = wave_sum(b);
  if ((threadIdx.x & 63) == 0) { red[threadIdx.x >> 6][0] = a; red[threadIdx.x >> 6][1] = b; }
  __syncthreads();
  if (threadIdx.x < 2) {
    double tot = 0.0;
    for (int w2 = 0; w2 < BS / 64; ++w2) tot += red[w2][threadIdx.x];
    part[blockIdx.x * MAXC + threadIdx.x] = tot;
  }
}
void launch_coef_sums(hipStream_t st, const double* coef, long E, double* part, double* out) {
  launch(coef_sum_kernel, dim3(RED_BLOCKS), dim3(BS), 0, st, coef, E, part);
  launch(reduce_parts_kernel, dim3(1), dim3(1024), 0, st, part, RED_BLOCKS, 2, out, 0, (double*)nullptr);
}

// ------------------------------------------------------------------ objective
// Volumetric compliance of one element, f_e = sum_a T_a int_e N*_a Q (Sec. 5.1 eq. objdiscr
// with f_tQ of App. A).  For the trilinear element int_e N_a = h^3 / 8 and
// int_e grad N_a = h^3 grad N_a(x_c), so f_e = Q h^3 (T_c + tau u0 . grad T_c) with the
// centroid values; with its derivatives by the nodal P and T (u0 and tau depend on them)
// and by the permeability (u0 = kappa w).
struct QElem {
  double f, dP[8], dT[8], dkap;
};
__device__ QElem q_element(const ElemConst<double>& c, double Q, double kap, const double P[8], const double Tn[8]) {
  const double q4 = 0.125 * c.dxi;   // 1 / (4 h): |d N_a / d x_d| at the centroid
  double gP[3] = {0.0, 0.0, 0.0}, G[3] = {0.0, 0.0, 0.0}, Tc = 0.0;
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    const double sx = (a & 1) ? q4 : -q4, sy = (a & 2) ? q4 : -q4, sz = (a & 4) ? q4 : -q4;
    gP[0] += sx * P[a]; gP[1] += sy * P[a]; gP[2] += sz * P[a];
    G[0] += sx * Tn[a]; G[1] += sy * Tn[a]; G[2] += sz * Tn[a];
    Tc += 0.125 * Tn[a];
  }
  const double im = c.inv_mu;
  const double w[3] = {-im * gP[0], -im * gP[1], -im * (gP[2] - c.beta * Tc)};   // u0 / kappa
  const double u0[3] = {kap * w[0], kap * w[1], kap * w[2]};
  const double tau = 1.0 / sqrt(4.0 * (u0[0] * u0[0] + u0[1] * u0[1] + u0[2] * u0[2]) * c.inv_he2 + c.tau3inv2);
  const double t3 = -4.0 * tau * tau * tau * c.inv_he2;     // d tau = t3 (u0 . d u0)
  const double uG = u0[0] * G[0] + u0[1] * G[1] + u0[2] * G[2];
  const double QV = Q * 8.0 * c.W;                          // Q h^3
  QElem r;
  r.f = QV * (Tc + tau * uG);
  const double cm = kap * im;
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    const double sx = (a & 1) ? q4 : -q4, sy = (a & 2) ? q4 : -q4, sz = (a & 4) ? q4 : -q4;
    // d u0 / d P_a = -(kappa / mu) grad N_a(x_c)
    const double dux = -cm * sx, duy = -cm * sy, duz = -cm * sz;
    r.dP[a] = QV * (uG * t3 * (u0[0] * dux + u0[1] * duy + u0[2] * duz) + tau * (G[0] * dux + G[1] * duy + G[2] * duz));
    // d u0 / d T_a = (kappa / mu) beta N_a(x_c) e_z
    const double dTz = cm * c.beta * 0.125;
    r.dT[a] = QV * (0.125 + tau * (u0[0] * sx + u0[1] * sy + u0[2] * sz) + uG * t3 * u0[2] * dTz + tau * G[2] * dTz);
  }
  r.dkap = QV * (uG * t3 * (u0[0] * w[0] + u0[1] * w[1] + u0[2] * w[2]) + tau * (G[0] * w[0] + G[1] * w[1] + G[2] * w[2]));
  return r;
}

// the source box of c clamped to the grid: [i0, i1] x [j0, j1] x [k0, k1], count 0 if empty
struct BoxRange {
  int i0, i1, j0, j1, k0, k1;
  long count;
};
__host__ __device__ inline BoxRange source_range(const Grid& g, const ElemConst<double>& c) {
  BoxRange b;
  b.i0 = c.qi0 < 0 ? 0 : c.qi0; b.i1 = c.qi1 > g.nx - 1 ? g.nx - 1 : c.qi1;
  b.j0 = c.qj0 < 0 ? 0 : c.qj0; b.j1 = c.qj1 > g.ny - 1 ? g.ny - 1 : c.qj1;
  b.k0 = c.qk0 < 0 ? 0 : c.qk0; b.k1 = c.qk1 > g.nz - 1 ? g.nz - 1 : c.qk1;
  const long ni = b.i1 - b.i0 + 1, nj = b.j1 - b.j0 + 1, nk = b.k1 - b.k0 + 1;
  b.count = (c.Q == 0.0 || ni <= 0 || nj <= 0 || nk <= 0) ? 0 : ni * nj * nk;
  return b;
}
__device__ inline void element_nodes(const Grid& g, const double* s5, int i, int j, int k, double P[8], double Tn[8]) {
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    const long n = g.node(i + (a & 1), j + ((a >> 1) & 1), k + ((a >> 2) & 1));
    P[a] = s5[5 * n + 3];
    Tn[a] = s5[5 * n + 4];
  }
}

// f = sum over patch faces of q_h h^2/4 (T of the face's four nodes) + the volumetric
// compliance of the source elements
__global__ __launch_bounds__(BS) void objective_kernel(Grid g, Patch pa, ElemConst<double> c, const double* __restrict__ coef,
                                                       const double* __restrict__ s5, double* __restrict__ part) {
  __shared__ double red[BS / 64];
  double s = 0.0;
  const long F = (long)g.nx * g.ny;
  for (long f = (long)blockIdx.x * BS + threadIdx.x; f < F; f += (long)gridDim.x * BS) {
    const int i = (int)(f % g.nx), j = (int)(f / g.nx);
    if (!pa.has(i, j)) continue;
    const double w = pa.q_h * pa.h * pa.h * 0.25;
    for (int c = 0; c < 4; ++c) s += w * s5[5 * g.node(i + (c & 1), j + (c >> 1), 0) + 4];
  }
  const BoxRange b = source_range(g, c);
  const long ni = b.i1 - b.i0 + 1, nj = b.j1 - b.j0 + 1;
  for (long t = (long)blockIdx.x * BS + threadIdx.x; t < b.count; t += (long)gridDim.x * BS) {
    const int i = b.i0 + (int)(t % ni), j = b.j0 + (int)((t / ni) % nj), k = b.k0 + (int)(t / (ni * nj));
    double P[8], Tn[8];
    element_nodes(g, s5, i, j, k, P, Tn);
    s += q_element(c, c.Q, coef[2 * g.elem(i, j, k) + 1], P, Tn).f;
  }
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double tot = 0.0;
    for (int w2 = 0; w2 < BS / 64; ++w2) tot += red[w2];
    part[blockIdx.x * MAXC] = tot;
  }
}
void launch_objective(hipStream_t st, const Grid& g, const Patch& patch, const ElemConst<double>& c, const double* coef,
                      const double* s5, double* part, double* out) {
  launch(objective_kernel, dim3(RED_BLOCKS), dim3(BS), 0, st, g, patch, c, coef, s5, part);
  launch(reduce_parts_kernel, dim3(1), dim3(1024), 0, st, part, RED_BLOCKS, 1, out, 0, (double*)nullptr);
}

__global__ void objective_grad_kernel(Grid g, Patch pa, double* __restrict__ g5) {
  const long n = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= g.nodes()) return;
  const int i = (int)(n % (g.nx + 1)), j = (int)((n / (g.nx + 1)) % (g.ny + 1)), k = (int)(n / ((long)(g.nx + 1) * (g.ny + 1)));
  double v = 0.0;
  if (k == 0 && !g.tfix(i, j, k)) {
    const double w = pa.q_h * pa.h * pa.h * 0.25;
    for (int c = 0; c < 4; ++c) {
      const int fi = i - (c & 1), fj = j - (c >> 1);
      if (fi >= 0 && fi < g.nx && fj >= 0 && fj < g.ny && pa.has(fi, fj)) v += w;
    }
  }
  for (int f = 0; f < 4; ++f) g5[5 * n + f] = 0.0;
  g5[5 * n + 4] = v;
}
void launch_objective_grad(hipStream_t st, const Grid& g, const Patch& patch, double* g5) {
  launch(objective_grad_kernel, dim3(blocks_for(g.nodes())), dim3(BS), 0, st, g, patch, g5);
}

// g5 += d (volumetric compliance) / d (P, T): each node gathers the derivatives of the
// source elements around it, in a fixed order; constrained entries are left to the caller
__global__ __launch_bounds__(BS) void objective_grad_q_kernel(Grid g, ElemConst<double> c, const double* __restrict__ coef,
                                                              const double* __restrict__ s5, double* __restrict__ g5) {
  const long n = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= g.nodes()) return;
  const int i = (int)(n % (g.nx + 1)), j = (int)((n / (g.nx + 1)) % (g.ny + 1)), k = (int)(n / ((long)(g.nx + 1) * (g.ny + 1)));
  double dp = 0.0, dt = 0.0;
  for (int a = 7; a >= 0; --a) {   // element (i, j, k) - offset(a) has this node as its corner a
    const int ei = i - (a & 1), ej = j - ((a >> 1) & 1), ek = k - ((a >> 2) & 1);
    if (ei < 0 || ei >= g.nx || ej < 0 || ej >= g.ny || ek < 0 || ek >= g.nz) continue;
    const double Q = c.source(ei, ej, ek);
    if (Q == 0.0) continue;
    double P[8], Tn[8];
    element_nodes(g, s5, ei, ej, ek, P, Tn);
    const QElem r = q_element(c, Q, coef[2 * g.elem(ei, ej, ek) + 1], P, Tn);
    dp += r.dP[a];
    dt += r.dT[a];
  }
  g5[5 * n + 3] += dp;
  g5[5 * n + 4] += dt;
}
void launch_objective_grad_q(hipStream_t st, const Grid& g, const ElemConst<double>& c, const double* coef,
                             const double* s5, double* g5) {
  launch(objective_grad_q_kernel, dim3(blocks_for(g.nodes())), dim3(BS), 0, st, g, c, coef, s5, g5);
}

// out[e] += d (volumetric compliance) / d gamma_e = d f_e / d kappa * d kappa / d gamma
__global__ __launch_bounds__(BS) void objective_dgamma_kernel(Grid g, ElemConst<double> c, const double* __restrict__ coef,
                                                              const double* __restrict__ dkap, const double* __restrict__ s5,
                                                              double* __restrict__ out) {
  const BoxRange b = source_range(g, c);
  const long ni = b.i1 - b.i0 + 1, nj = b.j1 - b.j0 + 1;
  for (long t = (long)blockIdx.x * BS + threadIdx.x; t < b.count; t += (long)gridDim.x * BS) {
    const int i = b.i0 + (int)(t % ni), j = b.j0 + (int)((t / ni) % nj), k = b.k0 + (int)(t / (ni * nj));
    double P[8], Tn[8];
    element_nodes(g, s5, i, j, k, P, Tn);
    const long e = g.elem(i, j, k);
    out[e] += q_element(c, c.Q, coef[2 * e + 1], P, Tn).dkap * dkap[e];
  }
}
void launch_objective_dgamma(hipStream_t st, const Grid& g, const ElemConst<double>& c, const double* coef,
                             const double* dkap, const double* s5, double* out) {
  const long cnt = source_range(g, c).count;
  if (cnt == 0) return;
  launch(objective_dgamma_kernel, dim3(blocks_for(cnt)), dim3(BS), 0, st, g, c, coef, dkap, s5, out);
}

// ------------------------------------------------------------------ passive regions
// gamma = 1 on passive solid, 0 on passive fluid (outside the design domain)
__global__ __launch_bounds__(BS) void passive_kernel(Grid g, Regions rg, double* __restrict__ gamma) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= g.elems()) return;
  const int i = (int)(e % g.nx), j = (int)((e / g.nx) % g.ny), k = (int)(e / ((long)g.nx * g.ny));
  if (rg.solid(i, j, k)) gamma[e] = 1.0;
  else if (!rg.design(i, j, k)) gamma[e] = 0.0;
}
void launch_passive(hipStream_t st, const Grid& g, const Regions& rg, double* gamma) {
  launch(passive_kernel, dim3(blocks_for(g.elems())), dim3(BS), 0, st, g, rg, gamma);
}
// a[e] = 0 off the design domain; with fill: a[e] = design ? fill : 0
__global__ __launch_bounds__(BS) void design_mask_kernel(Grid g, Regions rg, double* __restrict__ a, int set, double fill) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= g.elems()) return;
  const int i = (int)(e % g.nx), j = (int)((e / g.nx) % g.ny), k = (int)(e / ((long)g.nx * g.ny));
  const bool d = rg.design(i, j, k);
  if (set) a[e] = d ? fill : 0.0;
  else if (!d) a[e] = 0.0;
}
void launch_design_mask(hipStream_t st, const Grid& g, const Regions& rg, double* a, bool set, double fill) {
  launch(design_mask_kernel, dim3(blocks_for(g.elems())), dim3(BS), 0, st, g, rg, a, set ? 1 : 0, fill);
}
// out[0] = sum of gamma over the design domain
__global__ __launch_bounds__(BS) void design_sum_kernel(Grid g, Regions rg, const double* __restrict__ gamma,
                                                        double* __restrict__ part) {
  __shared__ double red[BS / 64];
  double s = 0.0;
  for (long e = (long)blockIdx.x * BS + threadIdx.x; e < g.elems(); e += (long)gridDim.x * BS) {
    const int i = (int)(e % g.nx), j = (int)((e / g.nx) % g.ny), k = (int)(e / ((long)g.nx * g.ny));
    if (rg.design(i, j, k)) s += gamma[e];
  }
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double tot = 0.0;
    for (int w2 = 0; w2 < BS / 64; ++w2) tot += red[w2];
    part[blockIdx.x * MAXC] = tot;
  }
}
void launch_design_sum(hipStream_t st, const Grid& g, const Regions& rg, const double* gamma, double* part,
                       double* out) {
  launch(design_sum_kernel, dim3(RED_BLOCKS), dim3(BS), 0, st, g, rg, gamma, part);
  launch(reduce_parts_kernel, dim3(1), dim3(1024), 0, st, part, RED_BLOCKS, 1, out, 0, (double*)nullptr);
}

// ------------------------------------------------------------------ instantiations
#define NC_INST(T)                                                                                   \
  template void launch_restrict<T>(hipStream_t, const Grid&, const Grid&, const T*, T*, const T*, bool, T, T*); \
  template void launch_prolong_add<T>(hipStream_t, const Grid&, const Grid&, const T*, T*);         \
  template void launch_inject_state<T>(hipStream_t, const Grid&, const Grid&, const T*, T*);        \
  template void launch_average_coef<T>(hipStream_t, const Grid&, const Grid&, const T*, T*);        \
  template void launch_coarse_assemble<T>(hipStream_t, const LevelView<T>&, double*, double*);      \
  template void launch_dense_apply<T>(hipStream_t, const double*, int, bool, const T*, T*);         \
  template void launch_pack_state<T>(hipStream_t, const Grid&, const double*, T*);                  \
  template void launch_pc_in<T>(hipStream_t, const Grid&, T*, const double*, T, T, const T*, bool, T, T*, T*); \
  template void launch_pack_pt<T>(hipStream_t, long, const double*, T*, double, double);             \
  template void launch_unpack_pt<T>(hipStream_t, const Grid&, const T*, double*);                    \
  template void launch_mdot<T>(hipStream_t, const T*, long, int, const T*, long, double*, double*, bool, double*); \
  template void launch_maxpy<T>(hipStream_t, const T*, long, int, const double*, double, T*, long, double*, double*, double*); \
  template void launch_scale_inv<T>(hipStream_t, const double*, const T*, T*, long);                \
  template void launch_norm<T>(hipStream_t, const T*, long, double*, double*, double*);            \
  template void launch_diag_scale<T>(hipStream_t, const Grid&, const T*, bool, T, const T*, T*);    \
  template void launch_rsub<T>(hipStream_t, const T*, T*, long);
NC_INST(double)
NC_INST(float)
#undef NC_INST
template void launch_convert<double, float>(hipStream_t, const double*, float*, long, double);
template void launch_convert<float, double>(hipStream_t, const float*, double*, long, double);
template void launch_convert<double, double>(hipStream_t, const double*, double*, long, double);
template void launch_convert<float, float>(hipStream_t, const float*, float*, long, double);
template void launch_scale2<double, float>(hipStream_t, long, const double*, float*, double, double);
template void launch_scale2<float, double>(hipStream_t, long, const float*, double*, double, double);
template void launch_scale2<double, double>(hipStream_t, long, const double*, double*, double, double);
template void launch_normalize_copy<double, float>(hipStream_t, const double*, double*, float*, long);

}  // namespace nc
