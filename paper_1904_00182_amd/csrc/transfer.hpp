// Grid-transfer stencils of the multigrid hierarchy, shared by the stand-alone transfer
// kernels and the single-workgroup bottom of the V-cycle so that both do the same
// arithmetic.  Level l + 1 halves every grid dimension of level l; fine node (2I, 2J, 2K)
// coincides with coarse node (I, J, K).
#pragma once

#include "common.hpp"

namespace nc {

// Accumulator of the transfer stencils for T-valued vectors: float64 also for float32
// vectors (summing the taps in float32 cost up to 30 % more Krylov iterations of the
// mixed-precision solves, with erratic counts from grid to grid).
template <typename T>
using TAcc = double;

// Full weighting (the transpose of trilinear prolongation, weights 1, 1/2, 1/4, 1/8) of the
// fine (P, T) vector rf at coarse node (I, J, K), summed in the caller's accumulator type A
// (the weights are exact in it): the 27 taps are clamped into the grid with weight 0
// outside it, so every load is independent of the others.
template <typename A, typename T>
__device__ inline void restrict_taps(const Grid& fine, int I, int J, int K, const T* rf, A& sp, A& stt) {
  int ix[3], jy[3], kz[3];
  A wx[3], wy[3], wz[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int i = 2 * I + d - 1, j = 2 * J + d - 1, k = 2 * K + d - 1;
    const A w = d == 1 ? (A)1 : (A)0.5;
    ix[d] = min(max(i, 0), fine.nx);
    jy[d] = min(max(j, 0), fine.ny);
    kz[d] = min(max(k, 0), fine.nz);
    wx[d] = (i >= 0 && i <= fine.nx) ? w : (A)0;
    wy[d] = (j >= 0 && j <= fine.ny) ? w : (A)0;
    wz[d] = (k >= 0 && k <= fine.nz) ? w : (A)0;
  }
  sp = (A)0;
  stt = (A)0;
#pragma unroll
  for (int dk = 0; dk < 3; ++dk)
#pragma unroll
    for (int dj = 0; dj < 3; ++dj)
#pragma unroll
      for (int di = 0; di < 3; ++di) {
        const A w = wz[dk] * wy[dj] * wx[di];
        const auto r = reinterpret_cast<const typename Pair<T>::type*>(rf)[fine.node(ix[di], jy[dj], kz[dk])];
        sp += w * (A)r.x;
        stt += w * (A)r.y;
      }
}

// Trilinear interpolation of the coarse (P, T) vector xc at fine node (i, j, k), in the
// caller's accumulator type A: the eight coarse taps are loaded together (a tap repeated
// with weight 0 where the fine node lies on a coarse plane).
template <typename A, typename T>
__device__ inline void prolong_taps(const Grid& coarse, int i, int j, int k, const T* xc, A& sp, A& stt) {
  const int i0 = i >> 1, i1 = (i + 1) >> 1, j0 = j >> 1, j1 = (j + 1) >> 1, k0 = k >> 1, k1 = (k + 1) >> 1;
  const A h = (A)0.5;
  const A wi[2] = {(i & 1) ? h : (A)1, (i & 1) ? h : (A)0};
  const A wj[2] = {(j & 1) ? h : (A)1, (j & 1) ? h : (A)0};
  const A wk[2] = {(k & 1) ? h : (A)1, (k & 1) ? h : (A)0};
  sp = (A)0;
  stt = (A)0;
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const A w = wi[a] * wj[b] * wk[c];
        const auto v = reinterpret_cast<const typename Pair<T>::type*>(xc)[coarse.node(a ? i1 : i0, b ? j1 : j0, c ? k1 : k0)];
        sp += w * (A)v.x;
        stt += w * (A)v.y;
      }
}

// prolong_taps for the fine node pair (2m, j, k), (2m + 1, j, k) at once: both read coarse
// columns m and m + 1 only, so the pair loads eight taps instead of sixteen; each node's sum
// takes the same terms in the same order as prolong_taps.  Node 2m + 1 exists only for
// m < coarse.nx (its values are then left unset).
template <typename A, typename T>
__device__ inline void prolong_taps_pair(const Grid& coarse, int m, int j, int k, const T* xc, A sp[2], A stt[2]) {
  const int m1 = min(m + 1, coarse.nx);
  const int j0 = j >> 1, j1 = (j + 1) >> 1, k0 = k >> 1, k1 = (k + 1) >> 1;
  const A h = (A)0.5;
  const A wj[2] = {(j & 1) ? h : (A)1, (j & 1) ? h : (A)0};
  const A wk[2] = {(k & 1) ? h : (A)1, (k & 1) ? h : (A)0};
  const A we[2] = {(A)1, (A)0}, wo[2] = {h, h};   // wi of the even and the odd node
  sp[0] = sp[1] = (A)0;
  stt[0] = stt[1] = (A)0;
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int jj = b ? j1 : j0, kk = c ? k1 : k0;
      const auto v0 = reinterpret_cast<const typename Pair<T>::type*>(xc)[coarse.node(m, jj, kk)];
      const auto v1 = reinterpret_cast<const typename Pair<T>::type*>(xc)[coarse.node(m1, jj, kk)];
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const A w = we[a] * wj[b] * wk[c];
        sp[0] += w * (A)v0.x;   // the even node's taps are column m twice
        stt[0] += w * (A)v0.y;
        const auto& v = a ? v1 : v0;
        const A wodd = wo[a] * wj[b] * wk[c];
        sp[1] += wodd * (A)v.x;
        stt[1] += wodd * (A)v.y;
      }
    }
}

}  // namespace nc
