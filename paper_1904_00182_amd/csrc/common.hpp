// Shared device/host definitions of the solver library: grid views, constraint
// predicates, launch helpers.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <cstddef>
#include <cstdint>

#include "element.hpp"

namespace nc {

// One z-layer of an array as a buffer resource: entries are addressed by a 32-bit byte
// offset within the layer (one layer of a five-field float64 array stays below 4 GiB,
// checked at context creation), and the layer base is a scalar operand, so a thread's
// offsets are computed once and reused from layer to layer.  Reads past the layer's end
// return zero instead of touching other memory.
template <typename T>
struct LayerRef {
  __amdgpu_buffer_rsrc_t r;
  // 0x00020000: the third descriptor word of the gfx9-family raw buffer (32-bit data format)
  __device__ LayerRef(const T* base, unsigned entries)
      : r(__builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(base), 0, (int)(entries * (unsigned)sizeof(T)), 0x00020000)) {}
  // base[idx .. idx + sizeof(V) / sizeof(T)) as one V
  template <typename V = T>
  __device__ V ld(unsigned idx) const {
    const int off = (int)(idx * (unsigned)sizeof(T));
    if constexpr (sizeof(V) == 4) return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
    else if constexpr (sizeof(V) == 8) return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
    else if constexpr (sizeof(V) == 16) return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
    else {
      static_assert(sizeof(V) == 32, "4, 8, 16 or 32 bytes");
      using U4 = unsigned __attribute__((ext_vector_type(4)));
      struct {
        U4 lo, hi;
      } w{__builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0), __builtin_amdgcn_raw_buffer_load_b128(r, off + 16, 0, 0)};
      return __builtin_bit_cast(V, w);
    }
  }
  template <typename V = T>
  __device__ void st(unsigned idx, const V& v) const {
    const int off = (int)(idx * (unsigned)sizeof(T));
    using U2 = unsigned __attribute__((ext_vector_type(2)));
    using U4 = unsigned __attribute__((ext_vector_type(4)));
    if constexpr (sizeof(V) == 4) __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, off, 0, 0);
    else if constexpr (sizeof(V) == 8) __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(U2, v), r, off, 0, 0);
    else {
      static_assert(sizeof(V) == 16, "4, 8 or 16 bytes");
      __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(U4, v), r, off, 0, 0);
    }
  }
};

// Structured grid of one multigrid level: nx*ny*nz cubes, nodes (nx+1)(ny+1)(nz+1).
struct Grid {
  int nx, ny, nz;
  int sym = 0;   // bit 0: the wall x = Lx is a symmetry plane, bit 1: the wall y = Ly
  // the index of the x (y) wall where T is held, -1 when that wall is a symmetry plane
  int tx = (sym & 1) ? -1 : nx, ty = (sym & 2) ? -1 : ny;
  __host__ __device__ long nodes() const { return (long)(nx + 1) * (ny + 1) * (nz + 1); }
  __host__ __device__ long elems() const { return (long)nx * ny * nz; }
  // 32-bit indices: grids are limited to fewer than 2^31 / 5 nodes (checked at context creation)
  __host__ __device__ int node(int i, int j, int k) const { return i + (nx + 1) * (j + (ny + 1) * k); }
  __host__ __device__ int elem(int i, int j, int k) const { return i + nx * (j + ny * k); }
  // The same indices split into a z-layer and a position within it: node (i, j, k) of an
  // [N][nf] array is entry nf * col(i, j) of layer(a, nf, k), element (i, j, k) of an [E][nf]
  // array entry nf * ecol(i, j) of elayer(a, nf, k).  k must be the same for the whole
  // wavefront (the z-march's layer is), which keeps the layer resource in scalar registers.
  __host__ __device__ unsigned col(int i, int j) const { return (unsigned)(i + (nx + 1) * j); }
  __host__ __device__ unsigned ecol(int i, int j) const { return (unsigned)(i + nx * j); }
  template <typename P>
  __device__ LayerRef<P> layer(const P* a, int nf, int k) const {
    const unsigned len = (unsigned)nf * (unsigned)(nx + 1) * (unsigned)(ny + 1);
    return LayerRef<P>(a + (size_t)len * k, len);
  }
  template <typename P>
  __device__ LayerRef<P> elayer(const P* a, int nf, int k) const {
    const unsigned len = (unsigned)nf * (unsigned)nx * (unsigned)ny;
    return LayerRef<P>(a + (size_t)len * k, len);
  }
  // Dirichlet sets of the cavity: T on the vertical walls and the top (a symmetry plane is
  // insulated instead), P at (0, 0, nz), and the normal velocity on a symmetry plane (its
  // projection there is the mean over both sides of an odd field).
  __host__ __device__ bool tfix(int i, int j, int k) const { return i == 0 || i == tx || j == 0 || j == ty || k == nz; }
  __host__ __device__ bool ufix(int i, int j, int d) const {
    return (d == 0 && tx < 0 && i == nx) || (d == 1 && ty < 0 && j == ny);
  }
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
