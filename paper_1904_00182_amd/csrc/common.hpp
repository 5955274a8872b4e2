// Shared device/host definitions of the solver library: grid views, constraint
// predicates, launch helpers.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <cstddef>
#include <cstdint>

#include "element.hpp"

namespace nc {

// Structured grid of one multigrid level: nx*ny*nz cubes, nodes (nx+1)(ny+1)(nz+1).
struct Grid {
  int nx, ny, nz;
  __host__ __device__ long nodes() const { return (long)(nx + 1) * (ny + 1) * (nz + 1); }
  __host__ __device__ long elems() const { return (long)nx * ny * nz; }
  // 32-bit indices: grids are limited to fewer than 2^31 / 5 nodes (checked at context creation)
  __host__ __device__ int node(int i, int j, int k) const { return i + (nx + 1) * (j + (ny + 1) * k); }
  __host__ __device__ int elem(int i, int j, int k) const { return i + nx * (j + ny * k); }
  // Dirichlet sets of the cavity: T on the vertical walls and the top, P at (0, 0, nz).
  __host__ __device__ bool tfix(int i, int j, int k) const { return i == 0 || i == nx || j == 0 || j == ny || k == nz; }
  __host__ __device__ bool pfix(int i, int j, int k) const { return i == 0 && j == 0 && k == nz; }
  // number of elements sharing node (i, j, k)
  __host__ __device__ int valence(int i, int j, int k) const {
    return (1 + (i > 0 && i < nx)) * (1 + (j > 0 && j < ny)) * (1 + (k > 0 && k < nz));
  }
};

// A node's (P, T) pair and its 2x2 block as single aligned vectors (the [N][2] and [N][4]
// layouts start every node on a multiple of the vector size).
template <typename T> struct Pair;
template <> struct Pair<float> { using type = float2; };
template <> struct Pair<double> { using type = double2; };
template <typename T> struct Quad;
template <> struct Quad<float> { using type = float4; };
template <> struct Quad<double> { using type = double4; };

// Read-only view of one level's linearisation for the operator kernels.
template <typename T>
struct LevelView {
  Grid g;
  ElemConst<T> c;
  const T* coef;   // [E][2]: conductivity k, permeability kappa
  const T* st;     // [N][2]: linearisation state (P, T)
  const T* dinv;   // [N][4]: inverse of the 2x2 (P, T) node block of the Jacobian, row major
};

// Constant per-field row scaling (u, v, w, P, T) used to equilibrate the five-field
// system inside the Krylov solver; the identity for the public entry points.
template <typename T>
struct Scale5 {
  T s[5];
};

// Heat-flux patch on the bottom face (boundary load of eq. weakstable).
struct Patch {
  double q_h, x0, x1, y0, y1, h;
  __host__ __device__ bool has(int i, int j) const {
    const double xc = (i + 0.5) * h, yc = (j + 0.5) * h;
    return xc >= x0 && xc <= x1 && yc >= y0 && yc <= y1;
  }
};

inline int ceil_div(long a, long b) { return (int)((a + b - 1) / b); }

// Optional timing of the next kernel launch of the calling thread: when start is set, the
// next launch() records its begin and end into (start, stop) as part of its own dispatch
// (exact kernel duration, no marker packets around it) and clears the pair.
struct LaunchTimer {
  hipEvent_t start = nullptr, stop = nullptr;
};
inline LaunchTimer& launch_timer() {
  static thread_local LaunchTimer t;
  return t;
}

template <typename F, typename... Args>
inline void launch(F kernel, dim3 grid, dim3 block, unsigned shm, hipStream_t st, Args... args) {
  LaunchTimer& lt = launch_timer();
  if (lt.start) {
    hipExtLaunchKernelGGL(kernel, grid, block, shm, st, lt.start, lt.stop, 0, args...);
    lt.start = lt.stop = nullptr;
  } else {
    hipLaunchKernelGGL(kernel, grid, block, shm, st, args...);
  }
}

}  // namespace nc
