// Grid-transfer stencils of the multigrid hierarchy, shared by the stand-alone transfer
// kernels and the single-workgroup bottom of the V-cycle so that both do the same
// arithmetic.  Level l + 1 halves every grid dimension of level l; fine node (2I, 2J, 2K)
// coincides with coarse node (I, J, K).
#pragma once

#include "common.hpp"

namespace nc {

// Full weighting (the transpose of trilinear prolongation, weights 1, 1/2, 1/4, 1/8) of the
// fine (P, T) vector rf at coarse node (I, J, K): the 27 taps are clamped into the grid
// with weight 0 outside it, so every load is independent of the others.
template <typename T>
__device__ inline void restrict_taps(const Grid& fine, int I, int J, int K, const T* rf, double& sp,
                                     double& stt) {
  int ix[3], jy[3], kz[3];
  double wx[3], wy[3], wz[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int i = 2 * I + d - 1, j = 2 * J + d - 1, k = 2 * K + d - 1;
    const double w = d == 1 ? 1.0 : 0.5;
    ix[d] = min(max(i, 0), fine.nx);
    jy[d] = min(max(j, 0), fine.ny);
    kz[d] = min(max(k, 0), fine.nz);
    wx[d] = (i >= 0 && i <= fine.nx) ? w : 0.0;
    wy[d] = (j >= 0 && j <= fine.ny) ? w : 0.0;
    wz[d] = (k >= 0 && k <= fine.nz) ? w : 0.0;
  }
  sp = 0.0;
  stt = 0.0;
#pragma unroll
  for (int dk = 0; dk < 3; ++dk)
#pragma unroll
    for (int dj = 0; dj < 3; ++dj)
#pragma unroll
      for (int di = 0; di < 3; ++di) {
        const double w = wz[dk] * wy[dj] * wx[di];
        const int m = fine.node(ix[di], jy[dj], kz[dk]);
        sp += w * (double)rf[2 * m];
        stt += w * (double)rf[2 * m + 1];
      }
}

// Trilinear interpolation of the coarse (P, T) vector xc at fine node (i, j, k): the eight
// coarse taps are loaded together (a tap repeated with weight 0 where the fine node lies
// on a coarse plane).
template <typename T>
__device__ inline void prolong_taps(const Grid& coarse, int i, int j, int k, const T* xc, double& sp,
                                    double& stt) {
  const int i0 = i >> 1, i1 = (i + 1) >> 1, j0 = j >> 1, j1 = (j + 1) >> 1, k0 = k >> 1, k1 = (k + 1) >> 1;
  const double wi[2] = {(i & 1) ? 0.5 : 1.0, (i & 1) ? 0.5 : 0.0};
  const double wj[2] = {(j & 1) ? 0.5 : 1.0, (j & 1) ? 0.5 : 0.0};
  const double wk[2] = {(k & 1) ? 0.5 : 1.0, (k & 1) ? 0.5 : 0.0};
  sp = 0.0;
  stt = 0.0;
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const double w = wi[a] * wj[b] * wk[c];
        const int m = coarse.node(a ? i1 : i0, b ? j1 : j0, c ? k1 : k0);
        sp += w * (double)xc[2 * m];
        stt += w * (double)xc[2 * m + 1];
      }
}

}  // namespace nc
