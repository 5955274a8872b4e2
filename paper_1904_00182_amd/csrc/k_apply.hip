// Operator kernels: residual, Jacobian, transposed Jacobian, multigrid smoother and the
// velocity-coupling pieces of the preconditioner.
//
// Work decomposition ("z-march").  A workgroup of TX x TY threads covers a tile of TX x
// TY element columns and marches up in z through KZ + 1 element layers.  Thread (tx, ty)
// computes element (I0 - 1 + tx, J0 - 1 + ty, k) of every layer in registers (modal
// element operators of element.hpp) and owns node column (I0 - 1 + tx, J0 - 1 + ty) for
// tx, ty >= 1 -- the lower-left node of its own element.  Each node gathers the
// contributions of its four elements per layer through LDS (the three neighbours'
// corners) and the contribution of the layer below from a register accumulator, always
// in the same order, so results are bitwise reproducible and no atomics are needed.
// Elements on the tile's lower x / y edge and the layer below the z chunk are recomputed
// by the neighbouring workgroup; the tile shape is chosen per grid to keep that halo and
// idle lanes small.
#include <algorithm>
#include <cstdlib>
#include <array>
#include <cstdio>
#include <map>
#include <mutex>
#include <stdexcept>
#include <type_traits>

#include "kernels.hpp"
#include "transfer.hpp"

namespace nc {

constexpr unsigned NXCD = 8;   // accelerator complex dies of the MI355X

// Occupancy floor of an operator's z-march (waves per SIMD the register allocation must
// leave room for): Op::MIN_WAVES where the operator sets it, else 1.
template <class Op, class = void>
struct MinWaves {
  static constexpr int value = 1;
};
template <class Op>
struct MinWaves<Op, std::void_t<decltype(Op::MIN_WAVES)>> {
  static constexpr int value = Op::MIN_WAVES;
};

// Largest workgroup of an operator's z-march: Op::MAX_THREADS where the operator sets it,
// else 256.
template <class Op, class = void>
struct MaxThreads {
  static constexpr int value = 256;
};
template <class Op>
struct MaxThreads<Op, std::void_t<decltype(Op::MAX_THREADS)>> {
  static constexpr int value = Op::MAX_THREADS;
};

// Operators whose finish can take the node's own values loaded ahead (Op::prefetch,
// Op::finish_pre), and the type that holds them (a placeholder for the others)
template <class Op, class = void>
struct PreOf {
  using type = char;
  static constexpr bool value = false;
};
template <class Op>
struct PreOf<Op, std::void_t<typename Op::Pre>> {
  using type = typename Op::Pre;
  static constexpr bool value = true;
};

// Shape of a z-march launch: tiles of tx x ty threads (tx * ty <= the kernel's NT, the
// workgroup rounded up to whole wavefronts) and the nz + 1 node planes split into `chunks`
// z ranges of as equal length as possible.
struct ZShape {
  int tx, ty, chunks;
};

// FINE: 1 for launches on the finest grid, 0 on coarser multigrid levels (the same code;
// separate instantiations keep the two apart in kernel traces).
template <class Op, int NT, int FINE>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(MinWaves<Op>::value)))
void zmarch_kernel(const Op op, const ZShape zs) {
  using T = typename Op::real;
  constexpr int NI = Op::NIN, NO = Op::NOUT;
  __shared__ T xch[6 * NO * NT];
  const int TX = zs.tx;
  const int tid = threadIdx.x, ty = tid / TX, tx = tid - ty * TX;
  const bool active = ty < zs.ty;   // lanes past the tile in its last wavefront idle
  const int nx = op.g.nx, ny = op.g.ny, nz = op.g.nz;
  // XCD-aware tile order: workgroups are dispatched round-robin over the XCDs by linear id,
  // so id w runs on XCD w % NXCD; give each XCD one contiguous range of tiles (x fastest,
  // then y, then z chunks) so that tiles sharing halo nodes share that XCD's L2
  const unsigned nbx = gridDim.x, nby = gridDim.y, total = nbx * nby * gridDim.z;
  const unsigned wid = blockIdx.x + nbx * (blockIdx.y + nby * blockIdx.z);
  const unsigned per = total / NXCD, rem = total % NXCD, xcd = wid % NXCD, kk = wid / NXCD;
  const unsigned tile = xcd < rem ? xcd * (per + 1) + kk : rem * (per + 1) + (xcd - rem) * per + kk;
  const int bx = (int)(tile % nbx), by = (int)((tile / nbx) % nby), bz = (int)(tile / (nbx * nby));
  const int i = bx * (TX - 1) - 1 + tx;
  const int j = by * (zs.ty - 1) - 1 + ty;
  // node planes [K0, K1) of this chunk
  const int K0 = (int)((long)bz * (nz + 1) / zs.chunks), K1 = (int)((long)(bz + 1) * (nz + 1) / zs.chunks);
  const bool colok = active && i >= 0 && i < nx && j >= 0 && j < ny;
  const bool owner = active && tx >= 1 && ty >= 1 && i <= nx && j <= ny;
  const int kbeg = K0 > 0 ? K0 - 1 : 0;
  const int kend = K1 - 1;
  T acc[NO];
#pragma unroll
  for (int f = 0; f < NO; ++f) acc[f] = (T)0;
  T nd[8][NI];
  bool have_lo = false;
  for (int kl = kbeg; kl <= kend; ++kl) {
    T out[8][NO];
#pragma unroll
    for (int a = 0; a < 8; ++a)
#pragma unroll
      for (int f = 0; f < NO; ++f) out[a][f] = (T)0;
    if (colok && kl < nz) {
      if (!have_lo) {
#pragma unroll
        for (int cc = 0; cc < 4; ++cc) op.load(i + (cc & 1), j + (cc >> 1), kl, nd[cc]);
      }
#pragma unroll
      for (int cc = 0; cc < 4; ++cc) op.load(i + (cc & 1), j + (cc >> 1), kl + 1, nd[4 + cc]);
      op.element(i, j, kl, nd, out);
#pragma unroll
      for (int cc = 0; cc < 4; ++cc)
#pragma unroll
        for (int f = 0; f < NI; ++f) nd[cc][f] = nd[4 + cc][f];
      have_lo = true;
    }
#pragma unroll
    for (int ka = 0; ka < 2; ++ka)
#pragma unroll
      for (int cc = 0; cc < 3; ++cc)
#pragma unroll
        for (int f = 0; f < NO; ++f) xch[((ka * 3 + cc) * NO + f) * NT + tid] = out[cc + 1 + 4 * ka][f];
    __syncthreads();
    if (owner) {
      const int tl = tid - 1, td = tid - TX, tld = tid - TX - 1;
      T v[NO];
#pragma unroll
      for (int f = 0; f < NO; ++f)
        v[f] = acc[f] + out[0][f] + xch[(0 * NO + f) * NT + tl] + xch[(1 * NO + f) * NT + td] +
               xch[(2 * NO + f) * NT + tld];
      if (kl >= K0) op.finish(i, j, kl, v);
#pragma unroll
      for (int f = 0; f < NO; ++f)
        acc[f] = out[4][f] + xch[(3 * NO + f) * NT + tl] + xch[(4 * NO + f) * NT + td] + xch[(5 * NO + f) * NT + tld];
    }
    __syncthreads();
  }
}

// The z-march with one node plane per workgroup (KZ = 1) computes two element layers one
// after the other: the layer below the plane (recomputed, as the halo) and its own.  On
// the small coarse grids that take KZ = 1 that serial pair sets the launch time, so there
// a workgroup of TX x TY x 2 threads computes both layers at once (threadIdx.z = 0: layer
// K - 1, 1: layer K) and the owner of node (i, j, K) adds the eight contributions in the
// z-march's order -- the four from the layer below, then the four from its own layer --
// so the results are the same bit for bit.  Used on grids of at most 16384 elements.
template <class Op, int TX, int TY>
__global__ __launch_bounds__(TX* TY * 2) void zpair_kernel(const Op op) {
  using T = typename Op::real;
  constexpr int NI = Op::NIN, NO = Op::NOUT, NT = TX * TY;
  static_assert(NT % 64 == 0, "each wavefront on one layer");
  __shared__ T xch[2][4 * NO * NT];   // [layer][corner][field][thread]: the corners on plane K
  // threadIdx.z is the same across a wavefront (TX * TY is a multiple of 64): reading it as
  // a scalar keeps the layer addressing of the operator in scalar registers
  const int tx = threadIdx.x, ty = threadIdx.y, tz = __builtin_amdgcn_readfirstlane(threadIdx.z), tid = tx + TX * ty;
  const int nx = op.g.nx, ny = op.g.ny, nz = op.g.nz;
  const unsigned nbx = gridDim.x, nby = gridDim.y, total = nbx * nby * gridDim.z;
  const unsigned wid = blockIdx.x + nbx * (blockIdx.y + nby * blockIdx.z);
  const unsigned per = total / NXCD, rem = total % NXCD, xcd = wid % NXCD, kk = wid / NXCD;
  const unsigned tile = xcd < rem ? xcd * (per + 1) + kk : rem * (per + 1) + (xcd - rem) * per + kk;
  const int bx = (int)(tile % nbx), by = (int)((tile / nbx) % nby), K = (int)(tile / (nbx * nby));
  const int i = bx * (TX - 1) - 1 + tx;
  const int j = by * (TY - 1) - 1 + ty;
  const int kl = K - 1 + tz;
  // the owner's own node values are loaded now, so that their latency hides behind the
  // element arithmetic instead of following it
  const bool own = tz == 1 && tx >= 1 && ty >= 1 && i <= nx && j <= ny;
  typename PreOf<Op>::type pre{};
  if constexpr (PreOf<Op>::value) {
    if (own) pre = op.prefetch(i, j, K);
  }
  T out[8][NO];
#pragma unroll
  for (int a = 0; a < 8; ++a)
#pragma unroll
    for (int f = 0; f < NO; ++f) out[a][f] = (T)0;
  if (i >= 0 && i < nx && j >= 0 && j < ny && kl >= 0 && kl < nz) {
    T nd[8][NI];
#pragma unroll
    for (int cc = 0; cc < 4; ++cc) {
      op.load(i + (cc & 1), j + (cc >> 1), kl, nd[cc]);
      op.load(i + (cc & 1), j + (cc >> 1), kl + 1, nd[4 + cc]);
    }
    op.element(i, j, kl, nd, out);
  }
  // layer K - 1 gives its top corners to plane K, layer K its bottom corners
#pragma unroll
  for (int cc = 0; cc < 4; ++cc)
#pragma unroll
    for (int f = 0; f < NO; ++f) xch[tz][(cc * NO + f) * NT + tid] = out[cc + 4 * (1 - tz)][f];
  __syncthreads();
  if (own) {
    const int tl = tid - 1, td = tid - TX, tld = tid - TX - 1;
    T v[NO];
#pragma unroll
    for (int f = 0; f < NO; ++f) {
      const T acc = xch[0][(0 * NO + f) * NT + tid] + xch[0][(1 * NO + f) * NT + tl] +
                    xch[0][(2 * NO + f) * NT + td] + xch[0][(3 * NO + f) * NT + tld];
      v[f] = acc + xch[1][(0 * NO + f) * NT + tid] + xch[1][(1 * NO + f) * NT + tl] +
             xch[1][(2 * NO + f) * NT + td] + xch[1][(3 * NO + f) * NT + tld];
    }
    if constexpr (PreOf<Op>::value) op.finish_pre(i, j, K, v, pre);
    else op.finish(i, j, K, v);
  }
}

// Tile shapes of the coarse levels (threads in x, y); a tile owns (TX-1) x (TY-1) node
// columns.
struct TileCfg {
  int tx, ty;
};
constexpr int NTILES = 3;
constexpr TileCfg TILES[NTILES] = {{16, 16}, {32, 8}, {8, 8}};

// Fewest launched lanes over the grid's tiles; NC_TILE=<index> forces a shape.
static int pick_tile(const Grid& g) {
  static const int forced = [] {
    const char* e = std::getenv("NC_TILE");
    return e ? std::atoi(e) : -1;
  }();
  if (forced >= 0 && forced < NTILES) return forced;
  long best = -1;
  int bi = 0;
  for (int c = 0; c < NTILES; ++c) {
    const long lanes = (long)TILES[c].tx * TILES[c].ty;
    const long cost = lanes * ceil_div(g.nx + 1, TILES[c].tx - 1) * ceil_div(g.ny + 1, TILES[c].ty - 1);
    if (best < 0 || cost < best) { best = cost; bi = c; }
  }
  return bi;
}

// Shape of the z-march on the finest grid, chosen per grid and kernel from a timing model.
// A wavefront's element layer takes a fixed VALU time per SIMD, so a layer step of the
// busiest CU takes w = (wavefronts it holds over all rounds) / 4 of those units, but no
// less than LAT units however few wavefronts share a SIMD (latency no longer hidden; 2.4
// fits the 128 x 64 x 128 sweep timings), plus w / 4 that latency does not hide either;
// the launch takes a chunk's planes + 1 such steps.  Ties go to more resident wavefronts
// (occupancy calculator), then to fewer lanes.  Tile
// widths are free between 8 and NT / 8 so that the (TX-1) x (TY-1) owned columns can
// divide the node plane with little left over: 11 x 23 threads in 26 chunks for 129 x 65 x
// 129 nodes (26.0 us per fine sweep, against 29.1 us for 16 x 16 tiles in 22 chunks, which
// launch 1.4 lanes per element column).  NC_ZSHAPE=tx,ty,chunks forces a shape.
template <class Op, int NT>
static ZShape fine_shape(const Grid& g) {
  static const ZShape forced = [] {
    ZShape z{0, 0, 0};
    const char* e = std::getenv("NC_ZSHAPE");
    if (e && std::sscanf(e, "%d,%d,%d", &z.tx, &z.ty, &z.chunks) != 3) z = ZShape{0, 0, 0};
    return z;
  }();
  if (forced.tx >= 2 && forced.ty >= 2 && forced.tx * forced.ty <= NT && forced.chunks >= 1 &&
      forced.chunks <= g.nz + 1)
    return forced;
  static std::mutex mu;
  static std::map<std::array<int, 4>, ZShape> cache;
  int dev = 0, cus = 0;
  (void)hipGetDevice(&dev);
  std::lock_guard<std::mutex> lock(mu);
  const std::array<int, 4> key{g.nx, g.ny, g.nz, dev};
  const auto hit = cache.find(key);
  if (hit != cache.end()) return hit->second;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 256;
  int resident[NT / 64 + 1] = {0};   // workgroups per CU by wavefronts per workgroup
  for (int w = 1; w <= NT / 64; ++w) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void*>(zmarch_kernel<Op, NT, 1>),
                                                     64 * w, 0) != hipSuccess || nb < 1)
      nb = 1;
    resident[w] = nb;
  }
  constexpr double LAT = 2.4;
  double best = -1;
  long best_live = 0, best_lanes = 0;
  ZShape bz{16, 16, 1};
  for (int tx = 8; tx <= NT / 8; ++tx)
    for (int ty = 8; tx * ty <= NT; ++ty) {
      const int waves = ceil_div(tx * ty, 64);
      const long tiles = (long)ceil_div(g.nx + 1, tx - 1) * ceil_div(g.ny + 1, ty - 1);
      for (int ch = 1; ch <= g.nz + 1; ++ch) {
        const long per_cu = (tiles * ch + cus - 1) / cus;
        const int kz = ceil_div(g.nz + 1, ch);
        const double w = (double)(per_cu * waves) / 4.0;
        const double cost = (kz + 1) * (std::max(LAT, w) + 0.25 * w);
        const long live = std::min<long>(per_cu, resident[waves]) * waves;
        const long lanes = tiles * ch * waves;
        const bool better = best < 0 || cost < best * (1 - 1e-9) ||
                            (cost <= best * (1 + 1e-9) && (live > best_live || (live == best_live && lanes < best_lanes)));
        if (better) {
          best = cost;
          best_live = live;
          best_lanes = lanes;
          bz = ZShape{tx, ty, ch};
        }
      }
    }
  cache[key] = bz;
  return bz;
}

template <class Op, int FINE = 1>
static void run_zmarch_fine(hipStream_t st, const Op& op) {
  constexpr int NT = MaxThreads<Op>::value;
  const Grid& g = op.g;
  const ZShape zs = fine_shape<Op, NT>(g);
  const dim3 grid(ceil_div(g.nx + 1, zs.tx - 1), ceil_div(g.ny + 1, zs.ty - 1), zs.chunks);
  launch((zmarch_kernel<Op, NT, FINE>), grid, dim3(64 * ceil_div(zs.tx * zs.ty, 64)), 0, st, op, zs);
}

template <class Op, int TX, int TY>
static void run_zmarch_coarse(hipStream_t st, const Op& op) {
  constexpr int NT = MaxThreads<Op>::value;
  const Grid& g = op.g;
  const int tiles_x = ceil_div(g.nx + 1, TX - 1);
  const int tiles_y = ceil_div(g.ny + 1, TY - 1);
  // z chunks on the coarse levels: about `target` workgroups over the device
  // (NC_ZBLOCKS_COARSE overrides) with at least `kzmin` node planes per chunk (NC_KZMIN
  // overrides).  A thread's serial work is KZ + 1 element layers, so short chunks cut the
  // latency of launches on small grids at the price of recomputing more halo layers.
  static const int target = [] {
    const char* e = std::getenv("NC_ZBLOCKS_COARSE");
    return e ? std::max(1, std::atoi(e)) : 1024;
  }();
  static const int kzmin = [] {
    const char* e = std::getenv("NC_KZMIN");
    return e ? std::max(1, std::atoi(e)) : 1;
  }();
  const int want = std::max(1, target * 256 / (TX * TY) / std::max(1, tiles_x * tiles_y));
  const int KZ = std::max(kzmin, ceil_div(g.nz + 1, want));
  const int chunks = ceil_div(g.nz + 1, KZ);
  // paired layers win where the launch is latency bound (32x16x32 6.8 -> 6.1 us,
  // 16x8x16 6.4 -> 5.5 us) and lose where it has work to fill the chip (64x32x64
  // 11.5 -> 14.0 us)
  if (KZ == 1 && g.elems() <= 16384) {
    launch((zpair_kernel<Op, TX, TY>), dim3(tiles_x, tiles_y, g.nz + 1), dim3(TX, TY, 2), 0, st, op);
    return;
  }
  static_assert(TX * TY <= NT, "coarse tiles fit the kernel's workgroup");
  launch((zmarch_kernel<Op, NT, 0>), dim3(tiles_x, tiles_y, chunks), dim3(TX * TY), 0, st, op,
         ZShape{TX, TY, chunks});
}

template <class Op, int FINE = 1>
static void run_zmarch(hipStream_t st, const Op& op) {
  // coarse levels with more than 16384 elements take the finest grid's shape model too
  // (64 x 32 x 64: 14 x 18 threads in 65 chunks instead of 8 x 8 tiles, the level's sweeps
  // and residuals 2.7 -> 2.35 ms per 128 x 64 x 128 step); smaller ones the fixed tiles
  // and, where KZ = 1, the paired-layer kernel (NC_TILE forces the fixed tiles everywhere)
  static const bool tile_forced = std::getenv("NC_TILE") != nullptr;
  if constexpr (FINE) {
    run_zmarch_fine(st, op);
  } else if (op.g.elems() > 16384 && !tile_forced) {
    run_zmarch_fine<Op, 0>(st, op);
  } else {
    switch (pick_tile(op.g)) {
      case 0: run_zmarch_coarse<Op, 16, 16>(st, op); break;
      case 1: run_zmarch_coarse<Op, 32, 8>(st, op); break;
      default: run_zmarch_coarse<Op, 8, 8>(st, op); break;
    }
  }
}

// ------------------------------------------------------------------ residual (float64)
struct ResidualOp {
  using real = double;
  static constexpr int NIN = 2, NOUT = 5;
  Grid g;
  ElemConst<double> c;
  Patch patch;
  const double* coef;
  const double* s;
  double* r;
  __device__ void load(int i, int j, int k, double in[NIN]) const {
    const long n = g.node(i, j, k);
    in[0] = s[5 * n + 3];
    in[1] = s[5 * n + 4];
  }
  __device__ void element(int i, int j, int k, const double nd[8][NIN], double out[8][NOUT]) const {
    double P[8], Tn[8];
#pragma unroll
    for (int a = 0; a < 8; ++a) { P[a] = nd[a][0]; Tn[a] = nd[a][1]; }
    const long e = g.elem(i, j, k);
    LinM<double> L;
    lin_modal_q(P, Tn, coef[2 * e], coef[2 * e + 1], c.source(i, j, k), c, L);
    double rP[8] = {0}, rT[8] = {0}, rU[3][8] = {{0}};
    elem_residual_m<double, true>(L, c, rP, rT, rU);
    if (k == 0 && patch.has(i, j)) {
      const double fl = patch.q_h * patch.h * patch.h * 0.25;
#pragma unroll
      for (int a = 0; a < 4; ++a) rT[a] -= fl;
    }
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      out[a][0] = rU[0][a]; out[a][1] = rU[1][a]; out[a][2] = rU[2][a];
      out[a][3] = rP[a]; out[a][4] = rT[a];
    }
  }
  __device__ void finish(int i, int j, int k, const double v[NOUT]) const {
    const long n = g.node(i, j, k);
    const double M = c.W * g.valence(i, j, k);
#pragma unroll
    for (int d = 0; d < 3; ++d) r[5 * n + d] = g.ufix(i, j, d) ? s[5 * n + d] : v[d] + M * s[5 * n + d];
    r[5 * n + 3] = g.pfix(i, j, k) ? s[5 * n + 3] : v[3];
    r[5 * n + 4] = g.tfix(i, j, k) ? s[5 * n + 4] : v[4];
  }
};

void launch_residual(hipStream_t st, const Grid& g, const ElemConst<double>& c, const Patch& patch,
                     const double* coef, const double* s, double* r) {
  ResidualOp op{g, c, patch, coef, s, r};
  run_zmarch(st, op);
}

// ------------------------------------------------------------------ Jacobian applies
// NF: fields per node of the direction/output arrays (5 on the fine level, 2 in the
// (P, T) multigrid hierarchy).  XP: the level has a volumetric source or symmetry planes
// (per-element source, symmetry-plane velocity rows); without them the element code is the
// plain cavity's, with no per-element tests in the loop.
template <typename T, int NF, int MODE, bool XP = false>
struct JvOp {
  using real = T;
  static constexpr int MIN_WAVES = 2;   // two waves per SIMD also for the float64 five-field applies
  static_assert(NF == 2 || MODE == MODE_STORE, "five-field applies store only");
  static constexpr int NIN = 4, NOUT = NF;
  Grid g;
  ElemConst<T> c;
  const T* coef;
  const T* st;
  const T* x;
  const T* b;
  const T* dinv;
  T* y;
  T omega;
  Scale5<T> rs;   // output row scales (five-field mode)
  __device__ void load(int i, int j, int k, T in[NIN]) const {
    using P2 = typename Pair<T>::type;
    const unsigned n = g.col(i, j);
    const P2 s = g.layer(st, 2, k).template ld<P2>(2 * n);
    const auto xk = g.layer(x, NF, k);
    T p, t;
    if constexpr (NF == 2) {
      const P2 v = xk.template ld<P2>(2 * n);
      p = v.x;
      t = v.y;
    } else {
      p = xk.template ld<T>(NF * n + NF - 2);
      t = xk.template ld<T>(NF * n + NF - 1);
    }
    if (g.pfix(i, j, k)) p = (T)0;
    if (g.tfix(i, j, k)) t = (T)0;
    in[0] = s.x;
    in[1] = s.y;
    in[2] = p;
    in[3] = t;
  }
  __device__ void element(int i, int j, int k, const T nd[8][NIN], T out[8][NOUT]) const {
    T P[8], Tn[8], p[8], t[8];
#pragma unroll
    for (int a = 0; a < 8; ++a) { P[a] = nd[a][0]; Tn[a] = nd[a][1]; p[a] = nd[a][2]; t[a] = nd[a][3]; }
    const auto kc = g.elayer(coef, 2, k).template ld<typename Pair<T>::type>(2 * g.ecol(i, j));
    LinM<T> L;
    lin_modal_q(P, Tn, kc.x, kc.y, XP ? c.source(i, j, k) : (T)0, c, L);
    T yP[8] = {0}, yT[8] = {0}, yU[3][8] = {{0}};
    elem_jv_m<T, NF == 5>(L, p, t, c, yP, yT, yU);
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      if constexpr (NF == 5) { out[a][0] = yU[0][a]; out[a][1] = yU[1][a]; out[a][2] = yU[2][a]; }
      out[a][NF - 2] = yP[a];
      out[a][NF - 1] = yT[a];
    }
  }
  // the node's own values that finish reads (x for a sweep, b, D^-1), loadable ahead of it
  struct Pre {
    typename Pair<T>::type xn{}, bn{};
    typename Quad<T>::type D{};
  };
  __device__ Pre prefetch(int i, int j, int k) const {
    Pre q;
    if constexpr (NF == 2) {
      using P2 = typename Pair<T>::type;
      const unsigned n = g.col(i, j);
      if constexpr (MODE == MODE_SMOOTH) {
        q.xn = g.layer(x, 2, k).template ld<P2>(2 * n);
        q.D = g.layer(dinv, 4, k).template ld<typename Quad<T>::type>(4 * n);
      }
      if constexpr (MODE != MODE_STORE) q.bn = g.layer(b, 2, k).template ld<P2>(2 * n);
    }
    return q;
  }
  __device__ void finish(int i, int j, int k, const T v[NOUT]) const { finish_pre(i, j, k, v, prefetch(i, j, k)); }
  __device__ void finish_pre(int i, int j, int k, const T v[NOUT], const Pre& pre) const {
    using P2 = typename Pair<T>::type;
    const unsigned n = g.col(i, j);
    const auto xk = g.layer(x, NF, k);
    const auto yk = g.layer(y, NF, k);
    const bool pf = g.pfix(i, j, k), tf = g.tfix(i, j, k);
    if constexpr (NF == 5) {
      const T M = c.W * (T)g.valence(i, j, k);
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const T xd = xk.template ld<T>(5 * n + d);
        yk.template st<T>(5 * n + d, rs.s[d] * (XP && g.ufix(i, j, d) ? xd : v[d] + M * xd));
      }
      const T ap = pf ? xk.template ld<T>(5 * n + 3) : v[3];
      const T at = tf ? xk.template ld<T>(5 * n + 4) : v[4];
      yk.template st<T>(5 * n + 3, rs.s[3] * ap);
      yk.template st<T>(5 * n + 4, rs.s[4] * at);
    } else {
      // x at the node itself: needed by the sweep, otherwise only at constrained dofs
      const P2 xn = pre.xn;
      const T ap = pf ? (MODE == MODE_SMOOTH ? xn.x : xk.template ld<T>(2 * n)) : v[0];
      const T at = tf ? (MODE == MODE_SMOOTH ? xn.y : xk.template ld<T>(2 * n + 1)) : v[1];
      if (MODE == MODE_STORE) {
        yk.template st<P2>(2 * n, P2{rs.s[3] * ap, rs.s[4] * at});
      } else {
        const P2 bn = pre.bn;
        const T rp = bn.x - ap, rt = bn.y - at;
        if (MODE == MODE_RESID) {
          yk.template st<P2>(2 * n, P2{rp, rt});
        } else {
          const auto D = pre.D;
          yk.template st<P2>(2 * n, P2{xn.x + omega * (D.x * rp + D.y * rt), xn.y + omega * (D.z * rp + D.w * rt)});
        }
      }
    }
  }
};

template <typename T, int NF, int MODE, bool XP = false>
struct JtwOp {
  using real = T;
  static constexpr int MIN_WAVES = 2;   // two waves per SIMD also for the float64 five-field applies
  static_assert(NF == 2 || MODE == MODE_STORE, "five-field applies store only");
  static constexpr int NIN = NF == 5 ? 7 : 4, NOUT = 2;
  Grid g;
  ElemConst<T> c;
  const T* coef;
  const T* st;
  const T* x;     // weights w
  const T* b;
  const T* dinv;
  T* y;
  T omega;
  Scale5<T> rs;   // output row scales (five-field mode)
  __device__ void load(int i, int j, int k, T in[NIN]) const {
    using P2 = typename Pair<T>::type;
    const unsigned n = g.col(i, j);
    const P2 s = g.layer(st, 2, k).template ld<P2>(2 * n);
    const auto xk = g.layer(x, NF, k);
    T p, t;
    if constexpr (NF == 2) {
      const P2 v = xk.template ld<P2>(2 * n);
      p = v.x;
      t = v.y;
    } else {
      p = xk.template ld<T>(NF * n + NF - 2);
      t = xk.template ld<T>(NF * n + NF - 1);
#pragma unroll
      for (int d = 0; d < 3; ++d) in[4 + d] = XP && g.ufix(i, j, d) ? (T)0 : xk.template ld<T>(5 * n + d);
    }
    if (g.pfix(i, j, k)) p = (T)0;
    if (g.tfix(i, j, k)) t = (T)0;
    in[0] = s.x;
    in[1] = s.y;
    in[2] = p;
    in[3] = t;
  }
  __device__ void element(int i, int j, int k, const T nd[8][NIN], T out[8][NOUT]) const {
    T P[8], Tn[8], wP[8], wT[8], wU[3][8];
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      P[a] = nd[a][0]; Tn[a] = nd[a][1]; wP[a] = nd[a][2]; wT[a] = nd[a][3];
      if constexpr (NF == 5) { wU[0][a] = nd[a][4]; wU[1][a] = nd[a][5]; wU[2][a] = nd[a][6]; }
    }
    const auto kc = g.elayer(coef, 2, k).template ld<typename Pair<T>::type>(2 * g.ecol(i, j));
    LinM<T> L;
    lin_modal_q(P, Tn, kc.x, kc.y, XP ? c.source(i, j, k) : (T)0, c, L);
    T yP[8] = {0}, yT[8] = {0};
    elem_jtw_m<T, NF == 5>(L, wP, wT, wU, c, yP, yT);
#pragma unroll
    for (int a = 0; a < 8; ++a) { out[a][0] = yP[a]; out[a][1] = yT[a]; }
  }
  // the node's own values that finish reads (x for a sweep, b, D^-1), loadable ahead of it
  struct Pre {
    typename Pair<T>::type xn{}, bn{};
    typename Quad<T>::type D{};
  };
  __device__ Pre prefetch(int i, int j, int k) const {
    Pre q;
    if constexpr (NF == 2) {
      using P2 = typename Pair<T>::type;
      const unsigned n = g.col(i, j);
      if constexpr (MODE == MODE_SMOOTH) {
        q.xn = g.layer(x, 2, k).template ld<P2>(2 * n);
        q.D = g.layer(dinv, 4, k).template ld<typename Quad<T>::type>(4 * n);
      }
      if constexpr (MODE != MODE_STORE) q.bn = g.layer(b, 2, k).template ld<P2>(2 * n);
    }
    return q;
  }
  __device__ void finish(int i, int j, int k, const T v[NOUT]) const { finish_pre(i, j, k, v, prefetch(i, j, k)); }
  __device__ void finish_pre(int i, int j, int k, const T v[NOUT], const Pre& pre) const {
    using P2 = typename Pair<T>::type;
    const unsigned n = g.col(i, j);
    const auto xk = g.layer(x, NF, k);
    const auto yk = g.layer(y, NF, k);
    const bool pf = g.pfix(i, j, k), tf = g.tfix(i, j, k);
    if constexpr (NF == 5) {
      const T M = c.W * (T)g.valence(i, j, k);
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const T xd = xk.template ld<T>(5 * n + d);
        yk.template st<T>(5 * n + d, rs.s[d] * (XP && g.ufix(i, j, d) ? xd : M * xd));
      }
      const T ap = pf ? xk.template ld<T>(5 * n + 3) : v[0];
      const T at = tf ? xk.template ld<T>(5 * n + 4) : v[1];
      yk.template st<T>(5 * n + 3, rs.s[3] * ap);
      yk.template st<T>(5 * n + 4, rs.s[4] * at);
    } else {
      // x at the node itself: needed by the sweep, otherwise only at constrained dofs
      const P2 xn = pre.xn;
      const T ap = pf ? (MODE == MODE_SMOOTH ? xn.x : xk.template ld<T>(2 * n)) : v[0];
      const T at = tf ? (MODE == MODE_SMOOTH ? xn.y : xk.template ld<T>(2 * n + 1)) : v[1];
      if (MODE == MODE_STORE) {
        yk.template st<P2>(2 * n, P2{rs.s[3] * ap, rs.s[4] * at});
      } else {
        const P2 bn = pre.bn;
        const T rp = bn.x - ap, rt = bn.y - at;
        if (MODE == MODE_RESID) {
          yk.template st<P2>(2 * n, P2{rp, rt});
        } else {
          const auto D = pre.D;   // (D^-1)^T
          yk.template st<P2>(2 * n, P2{xn.x + omega * (D.x * rp + D.z * rt), xn.y + omega * (D.y * rp + D.w * rt)});
        }
      }
    }
  }
};

template <typename T>
static Scale5<T> ones_or(const Scale5<T>* s) {
  return s ? *s : Scale5<T>{{(T)1, (T)1, (T)1, (T)1, (T)1}};
}

// whether a level needs the extended element code (source or symmetry planes)
template <typename T>
static bool extended(const LevelView<T>& L) { return L.c.Q != (T)0 || L.g.sym != 0; }

template <typename T>
void launch_jv5(hipStream_t st, const LevelView<T>& L, const T* x, T* y, const Scale5<T>* rows) {
  if (extended(L)) {
    JvOp<T, 5, MODE_STORE, true> op{L.g, L.c, L.coef, L.st, x, nullptr, nullptr, y, (T)0, ones_or(rows)};
    run_zmarch(st, op);
  } else {
    JvOp<T, 5, MODE_STORE> op{L.g, L.c, L.coef, L.st, x, nullptr, nullptr, y, (T)0, ones_or(rows)};
    run_zmarch(st, op);
  }
}
template <typename T>
void launch_jtw5(hipStream_t st, const LevelView<T>& L, const T* w, T* y, const Scale5<T>* rows) {
  if (extended(L)) {
    JtwOp<T, 5, MODE_STORE, true> op{L.g, L.c, L.coef, L.st, w, nullptr, nullptr, y, (T)0, ones_or(rows)};
    run_zmarch(st, op);
  } else {
    JtwOp<T, 5, MODE_STORE> op{L.g, L.c, L.coef, L.st, w, nullptr, nullptr, y, (T)0, ones_or(rows)};
    run_zmarch(st, op);
  }
}

// y = D J_PT x (J_PT^T when transposed) on the finest grid: the (P, T) block of the
// Jacobian, constrained rows and columns the identity, rows scaled by rows->s[3], s[4]
template <typename T>
void launch_pt_store(hipStream_t st, const LevelView<T>& L, bool transpose, const T* x, T* y, const Scale5<T>* rows) {
#define NC_STORE(OP, X)                                                                     \
  {                                                                                         \
    OP<T, 2, MODE_STORE, X> op{L.g, L.c, L.coef, L.st, x, nullptr, nullptr, y, (T)0, ones_or(rows)}; \
    run_zmarch<OP<T, 2, MODE_STORE, X>, 1>(st, op);                                          \
  }
  const bool xp = extended(L);
  if (!transpose) {
    if (xp) NC_STORE(JvOp, true) else NC_STORE(JvOp, false)
  } else {
    if (xp) NC_STORE(JtwOp, true) else NC_STORE(JtwOp, false)
  }
#undef NC_STORE
}

template <typename T>
void launch_pt_apply(hipStream_t st, const LevelView<T>& L, bool transpose, int mode, const T* x, const T* b, T* y,
                     T omega, bool fine) {
#define NC_PTX(OP, M, X)                                                                     \
  {                                                                                         \
    OP<T, 2, M, X> op{L.g, L.c, L.coef, L.st, x, b, L.dinv, y, omega, ones_or<T>(nullptr)};  \
    if (fine) run_zmarch<OP<T, 2, M, X>, 1>(st, op); else run_zmarch<OP<T, 2, M, X>, 0>(st, op); \
  }
#define NC_PT(OP, M)                      \
  {                                       \
    if (xp) NC_PTX(OP, M, true)           \
    else NC_PTX(OP, M, false)             \
  }
  const bool xp = extended(L);
  if (!transpose) {
    if (mode == MODE_STORE) NC_PT(JvOp, MODE_STORE)
    else if (mode == MODE_RESID) NC_PT(JvOp, MODE_RESID)
    else NC_PT(JvOp, MODE_SMOOTH)
  } else {
    if (mode == MODE_STORE) NC_PT(JtwOp, MODE_STORE)
    else if (mode == MODE_RESID) NC_PT(JtwOp, MODE_RESID)
    else NC_PT(JtwOp, MODE_SMOOTH)
  }
#undef NC_PT
#undef NC_PTX
}

// ------------------------------------------------------------------ bottom of the V-cycle
// The last smoothed level and the dense coarsest level in one workgroup.  On grids this
// small each launch of the per-step path is latency bound (one wave's serial element work
// plus the launch itself), so here the whole bottom of the cycle -- restriction into the
// level with its first damped step, further pre-sweeps, residual, restriction to the
// coarsest level, the dense solve, prolongation, post-sweeps and the prolongation into
// the level above -- runs with the level's vectors in LDS, one element per thread per
// pass and a barrier between passes.  With PF the level's node-block inverses, state
// and coefficients are staged in LDS too.  Global loads are batched so that many are in
// flight at once: inside one workgroup their latency, not bandwidth, sets the time.  The
// element and node arithmetic is that of JvOp / JtwOp on two fields; each node sums its
// elements' contributions in corner order, so results do not depend on timing.
template <typename T>
struct TailArgs {
  Grid gu;              // level above
  const T* ru;          // its residual, restricted into this level
  T* xu;                // its iterate, to which the prolonged correction is added
  LevelView<T> lv;      // this level
  Grid gc;              // coarsest level
  const double* ainv;   // coarsest inverse (its transpose for the transposed cycle), row-major
  T omega;
  int npre, npost;
};

constexpr int TAIL_THREADS = 512, TAIL_LDS_MAX = 65536;

// LDS bytes: element contributions [E][8][2] (the coarsest vectors reuse them), the level's
// b, x, y [N][2]; with the prefetch also D^-1 [N][4], the state [N][2], coefficients [E][2]
template <typename T>
static size_t tail_lds_bytes(const Grid& g, const Grid& gc, bool pf) {
  const size_t con = std::max<size_t>(16 * (size_t)g.elems(), 4 * (size_t)gc.nodes());
  return sizeof(T) * (con + 6 * (size_t)g.nodes() + (pf ? 6 * (size_t)g.nodes() + 2 * (size_t)g.elems() : 0));
}

// (i, j, k) of a linear index n = i + nx1 (j + ny1 k) in a box of nx1 x ny1 x ... points.
// The two divisions take a float estimate of the quotient and one correction step, exact
// for n < 2^22 (the tail's grids are far smaller), in place of the integer division
// sequences that otherwise dominate the tail's index arithmetic.
struct TailIdx {
  int d1, d2;
  float r1, r2;
  __device__ TailIdx(int nx1, int ny1) : d1(nx1), d2(nx1 * ny1), r1(1.0f / (float)nx1), r2(1.0f / (float)(nx1 * ny1)) {}
  __device__ static int div(int n, int d, float r, int& rem) {
    int q = (int)((float)n * r);
    rem = n - q * d;
    if (rem < 0) {
      --q;
      rem += d;
    } else if (rem >= d) {
      ++q;
      rem -= d;
    }
    return q;
  }
  __device__ void operator()(int n, int& i, int& j, int& k) const {
    int rem;
    k = div(n, d2, r2, rem);
    j = div(rem, d1, r1, i);
  }
};

template <typename T, bool TR, bool PF, bool XP>
__global__ __launch_bounds__(TAIL_THREADS) void tail_cycle_kernel(const TailArgs<T> a) {
  extern __shared__ __align__(16) unsigned char tail_smem[];
  const Grid g = a.lv.g, gc = a.gc, gu = a.gu;
  const int N = (int)g.nodes(), E = (int)g.elems(), Nc = (int)gc.nodes(), Nu = (int)gu.nodes();
  const int nc2 = 2 * Nc;
  T* con = (T*)tail_smem;   // [E][8 corners][2]; during the coarse correction bc, xc [Nc][2]
  T* b = con + max(16 * E, 2 * nc2);
  T* x = b + 2 * N;
  T* y = x + 2 * N;
  T* sD = y + 2 * N;        // prefetched D^-1 [N][4], state [N][2], coefficients [E][2]
  T* sSt = sD + 4 * N;
  T* sCoef = sSt + 2 * N;
  T* bc = con;
  T* xc = con + nc2;
  const int t = threadIdx.x;
  const T om = a.omega;
  const TailIdx node_g(g.nx + 1, g.ny + 1), elem_g(g.nx, g.ny), node_gc(gc.nx + 1, gc.ny + 1),
      node_gu(gu.nx + 1, gu.ny + 1);
  if constexpr (PF) {
    for (int m = t; m < 4 * N; m += TAIL_THREADS) sD[m] = a.lv.dinv[m];
    for (int m = t; m < 2 * N; m += TAIL_THREADS) sSt[m] = a.lv.st[m];
    for (int m = t; m < 2 * E; m += TAIL_THREADS) sCoef[m] = a.lv.coef[m];
  }
  const T* D = PF ? (const T*)sD : a.lv.dinv;
  const T* ST = PF ? (const T*)sSt : a.lv.st;
  const T* CO = PF ? (const T*)sCoef : a.lv.coef;
  for (int n = t; n < N; n += TAIL_THREADS) {
    int I, J, K;
    node_g(n, I, J, K);
    TAcc<T> sp, stt;
    restrict_taps(gu, I, J, K, a.ru, sp, stt);
    const T bp = g.pfix(I, J, K) ? (T)0 : (T)sp;
    const T bt = g.tfix(I, J, K) ? (T)0 : (T)stt;
    b[2 * n] = bp;
    b[2 * n + 1] = bt;
    const T* d = a.lv.dinv + 4 * n;
    x[2 * n] = om * (d[0] * bp + d[TR ? 2 : 1] * bt);
    x[2 * n + 1] = om * (d[TR ? 1 : 2] * bp + d[3] * bt);
  }
  __syncthreads();
  // passes: pre - 1 further sweeps, the residual (followed by the coarse correction), then
  // the post-sweeps; a sweep writes y from x and the two swap
  const int pre = max(a.npre, 1) - 1, passes = pre + 1 + a.npost;
  for (int q = 0; q < passes; ++q) {
    for (int e = t; e < E; e += TAIL_THREADS) {
      int i, j, k;
      elem_g(e, i, j, k);
      T P[8], Tn[8], p[8], w[8];
#pragma unroll
      for (int c8 = 0; c8 < 8; ++c8) {
        const int ni = i + (c8 & 1), nj = j + ((c8 >> 1) & 1), nk = k + (c8 >> 2);
        const int n = g.node(ni, nj, nk);
        P[c8] = ST[2 * n];
        Tn[c8] = ST[2 * n + 1];
        p[c8] = g.pfix(ni, nj, nk) ? (T)0 : x[2 * n];
        w[c8] = g.tfix(ni, nj, nk) ? (T)0 : x[2 * n + 1];
      }
      LinM<T> L;
      lin_modal_q(P, Tn, CO[2 * e], CO[2 * e + 1], XP ? a.lv.c.source(i, j, k) : (T)0, a.lv.c, L);
      T yP[8] = {0}, yT[8] = {0}, yU[3][8] = {{0}};
      if constexpr (TR) elem_jtw_m<T, false>(L, p, w, yU, a.lv.c, yP, yT);
      else elem_jv_m<T, false>(L, p, w, a.lv.c, yP, yT, yU);
#pragma unroll
      for (int c8 = 0; c8 < 8; ++c8) {
        con[(8 * e + c8) * 2] = yP[c8];
        con[(8 * e + c8) * 2 + 1] = yT[c8];
      }
    }
    __syncthreads();
    const bool resid = q == pre;
    for (int n = t; n < N; n += TAIL_THREADS) {
      int I, J, K;
      node_g(n, I, J, K);
      T vp = (T)0, vt = (T)0;
#pragma unroll
      for (int c8 = 0; c8 < 8; ++c8) {
        const int ei = I - (c8 & 1), ej = J - ((c8 >> 1) & 1), ek = K - (c8 >> 2);
        if (ei >= 0 && ei < g.nx && ej >= 0 && ej < g.ny && ek >= 0 && ek < g.nz) {
          const int e = g.elem(ei, ej, ek);
          vp += con[(8 * e + c8) * 2];
          vt += con[(8 * e + c8) * 2 + 1];
        }
      }
      const T ap = g.pfix(I, J, K) ? x[2 * n] : vp;
      const T at = g.tfix(I, J, K) ? x[2 * n + 1] : vt;
      const T rp = b[2 * n] - ap, rt = b[2 * n + 1] - at;
      if (resid) {
        y[2 * n] = rp;
        y[2 * n + 1] = rt;
      } else {
        const T* d = D + 4 * n;
        y[2 * n] = x[2 * n] + om * (d[0] * rp + d[TR ? 2 : 1] * rt);
        y[2 * n + 1] = x[2 * n + 1] + om * (d[TR ? 1 : 2] * rp + d[3] * rt);
      }
    }
    __syncthreads();
    if (!resid) {
      T* tmp = x;
      x = y;
      y = tmp;
      continue;
    }
    // coarse correction: restrict the residual, solve densely, prolong into x
    for (int n = t; n < Nc; n += TAIL_THREADS) {
      int I, J, K;
      node_gc(n, I, J, K);
      TAcc<T> sp, stt;
      restrict_taps(g, I, J, K, (const T*)y, sp, stt);
      bc[2 * n] = gc.pfix(I, J, K) ? (T)0 : (T)sp;
      bc[2 * n + 1] = gc.tfix(I, J, K) ? (T)0 : (T)stt;
    }
    __syncthreads();
    // eight lanes per row, combined by a butterfly inside the eight lanes; each lane loads
    // its next TAIL_DU entries of the row before it multiplies any, so that a row costs
    // one memory latency per 8 x TAIL_DU columns (the inverse is read from memory on every
    // launch)
    constexpr int TAIL_DU = 20;
    for (int row = t >> 3; row < nc2; row += TAIL_THREADS / 8) {
      const double* arow = a.ainv + (long)row * nc2;
      double s = 0.0;
      for (int c0 = t & 7; c0 < nc2; c0 += 8 * TAIL_DU) {
        double av[TAIL_DU];
#pragma unroll
        for (int u = 0; u < TAIL_DU; ++u) av[u] = c0 + 8 * u < nc2 ? arow[c0 + 8 * u] : 0.0;
#pragma unroll
        for (int u = 0; u < TAIL_DU; ++u)
          if (c0 + 8 * u < nc2) s += av[u] * (double)bc[c0 + 8 * u];
      }
      s += __shfl_xor(s, 1, 8);
      s += __shfl_xor(s, 2, 8);
      s += __shfl_xor(s, 4, 8);
      if ((t & 7) == 0) xc[row] = (T)s;
    }
    __syncthreads();
    for (int n = t; n < N; n += TAIL_THREADS) {
      int I, J, K;
      node_g(n, I, J, K);
      TAcc<T> sp, stt;
      prolong_taps(gc, I, J, K, (const T*)xc, sp, stt);
      if (!g.pfix(I, J, K)) x[2 * n] += (T)sp;
      if (!g.tfix(I, J, K)) x[2 * n + 1] += (T)stt;
    }
    __syncthreads();
  }
  // prolongation into the level above, TAIL_B nodes per thread per batch: the batch's
  // loads of the upper iterate are issued before any of its stores
  constexpr int TAIL_B = 8;
  for (int base = 0; base < Nu; base += TAIL_B * TAIL_THREADS) {
    T up[TAIL_B], ut[TAIL_B];
#pragma unroll
    for (int r = 0; r < TAIL_B; ++r) {
      const int n = base + r * TAIL_THREADS + t;
      up[r] = n < Nu ? a.xu[2 * n] : (T)0;
      ut[r] = n < Nu ? a.xu[2 * n + 1] : (T)0;
    }
#pragma unroll
    for (int r = 0; r < TAIL_B; ++r) {
      const int n = base + r * TAIL_THREADS + t;
      if (n < Nu) {
        int i, j, k;
        node_gu(n, i, j, k);
        TAcc<T> sp, stt;
        prolong_taps(g, i, j, k, (const T*)x, sp, stt);
        if (!gu.pfix(i, j, k)) a.xu[2 * n] = up[r] + (T)sp;
        if (!gu.tfix(i, j, k)) a.xu[2 * n + 1] = ut[r] + (T)stt;
      }
    }
  }
}

template <typename T>
bool tail_cycle_fits(const Grid& gu, const Grid& g, const Grid& gc) {
  return g.elems() <= TAIL_THREADS && gu.nodes() <= 65536 && tail_lds_bytes<T>(g, gc, false) <= TAIL_LDS_MAX;
}

template <typename T>
void launch_tail_cycle(hipStream_t st, const Grid& gu, const T* ru, T* xu, const LevelView<T>& L, const Grid& gc,
                       const double* ainv, bool transpose, T omega, int npre, int npost) {
  if (!tail_cycle_fits<T>(gu, L.g, gc)) throw std::runtime_error("tail cycle does not fit one workgroup");
  const TailArgs<T> a{gu, ru, xu, L, gc, ainv, omega, npre, npost};
  const bool pf = tail_lds_bytes<T>(L.g, gc, true) <= TAIL_LDS_MAX;
  const size_t lds = tail_lds_bytes<T>(L.g, gc, pf);
  const dim3 grid(1), block(TAIL_THREADS);
  // XP: the level carries a volumetric source (symmetry planes change only the constraint
  // sets of the (P, T) system, which the grid's predicates cover)
  const bool xp = L.c.Q != (T)0;
  if (transpose) {
    if (pf) {
      if (xp) launch(tail_cycle_kernel<T, true, true, true>, grid, block, lds, st, a);
      else launch(tail_cycle_kernel<T, true, true, false>, grid, block, lds, st, a);
    } else {
      if (xp) launch(tail_cycle_kernel<T, true, false, true>, grid, block, lds, st, a);
      else launch(tail_cycle_kernel<T, true, false, false>, grid, block, lds, st, a);
    }
  } else {
    if (pf) {
      if (xp) launch(tail_cycle_kernel<T, false, true, true>, grid, block, lds, st, a);
      else launch(tail_cycle_kernel<T, false, true, false>, grid, block, lds, st, a);
    } else {
      if (xp) launch(tail_cycle_kernel<T, false, false, true>, grid, block, lds, st, a);
      else launch(tail_cycle_kernel<T, false, false, false>, grid, block, lds, st, a);
    }
  }
}

// ------------------------------------------------------------------ block diagonal
template <typename T>
struct DiagOp {
  using real = T;
  static constexpr int NIN = 2, NOUT = 4;
  Grid g;
  ElemConst<T> c;
  const T* coef;
  const T* st;
  T* dinv;
  __device__ void load(int i, int j, int k, T in[NIN]) const {
    const long n = g.node(i, j, k);
    in[0] = st[2 * n];
    in[1] = st[2 * n + 1];
  }
  __device__ void element(int i, int j, int k, const T nd[8][NIN], T out[8][NOUT]) const {
    T P[8], Tn[8];
#pragma unroll
    for (int a = 0; a < 8; ++a) { P[a] = nd[a][0]; Tn[a] = nd[a][1]; }
    const long e = g.elem(i, j, k);
    LinM<T> L;
    lin_modal_q(P, Tn, coef[2 * e], coef[2 * e + 1], c.source(i, j, k), c, L);
    // float32: unrolled, so that the compiler folds the unit inputs through the transforms
    // (the float64 instance would then hold too many values and spill, so it loops)
    if constexpr (sizeof(T) == 4) {
#pragma unroll
      for (int a = 0; a < 8; ++a)
#pragma unroll
        for (int fld = 0; fld < 2; ++fld) column(L, a, fld, out);
    } else {
#pragma nounroll
      for (int a = 0; a < 8; ++a)
        for (int fld = 0; fld < 2; ++fld) column(L, a, fld, out);
    }
  }
  // the block entries of corner a from the element's response to a unit (P or T) input there
  __device__ __attribute__((always_inline)) void column(const LinM<T>& L, int a, int fld, T out[8][NOUT]) const {
    T p[8] = {0}, t[8] = {0}, yP[8] = {0}, yT[8] = {0}, yU[3][8];
    if (fld == 0) p[a] = (T)1; else t[a] = (T)1;
    elem_jv_m<T, false>(L, p, t, c, yP, yT, yU);
    // row-major block [dRP/dP, dRP/dT; dRT/dP, dRT/dT]
    out[a][fld] = yP[a];
    out[a][2 + fld] = yT[a];
  }
  __device__ void finish(int i, int j, int k, const T v[NOUT]) const {
    T pp = v[0], pt = v[1], tp = v[2], tt = v[3];
    if (g.tfix(i, j, k)) { tp = (T)0; tt = (T)1; pt = (T)0; }
    if (g.pfix(i, j, k)) { pp = (T)1; pt = (T)0; tp = (T)0; }
    const T idet = (T)1 / (pp * tt - pt * tp);
    T* D = dinv + 4 * g.node(i, j, k);
    D[0] = tt * idet;
    D[1] = -pt * idet;
    D[2] = -tp * idet;
    D[3] = pp * idet;
  }
};

template <typename T>
void launch_diag_inverse(hipStream_t st, const LevelView<T>& L, T* dinv, bool fine) {
  DiagOp<T> op{L.g, L.c, L.coef, L.st, dinv};
  if (fine) run_zmarch<DiagOp<T>, 1>(st, op);
  else run_zmarch<DiagOp<T>, 0>(st, op);
}

// ------------------------------------------------------------------ velocity coupling
template <typename T>
struct UprojOp {
  using real = T;
  static constexpr int NIN = 2, NOUT = 3;
  Grid g;
  ElemConst<T> c;
  const T* coef;
  const T* xpt;
  const T* r5;
  T* z5;
  Scale5<T> inv;   // 1 / row scale of r5
  __device__ void load(int i, int j, int k, T in[NIN]) const {
    const long n = g.node(i, j, k);
    in[0] = g.pfix(i, j, k) ? (T)0 : xpt[2 * n];
    in[1] = g.tfix(i, j, k) ? (T)0 : xpt[2 * n + 1];
  }
  __device__ void element(int i, int j, int k, const T nd[8][NIN], T out[8][NOUT]) const {
    T p[8], t[8], yU[3][8] = {{0}};
#pragma unroll
    for (int a = 0; a < 8; ++a) { p[a] = nd[a][0]; t[a] = nd[a][1]; }
    elem_uproj<T>(p, t, coef[2 * g.elem(i, j, k) + 1], c, yU);
#pragma unroll
    for (int a = 0; a < 8; ++a) { out[a][0] = yU[0][a]; out[a][1] = yU[1][a]; out[a][2] = yU[2][a]; }
  }
  __device__ void finish(int i, int j, int k, const T v[NOUT]) const {
    const long n = g.node(i, j, k);
    const T iM = (T)1 / (c.W * (T)g.valence(i, j, k));
#pragma unroll
    for (int d = 0; d < 3; ++d)
      z5[5 * n + d] = g.ufix(i, j, d) ? inv.s[d] * r5[5 * n + d] : (inv.s[d] * r5[5 * n + d] - v[d]) * iM;
    z5[5 * n + 3] = g.pfix(i, j, k) ? inv.s[3] * r5[5 * n + 3] : xpt[2 * n];
    z5[5 * n + 4] = g.tfix(i, j, k) ? inv.s[4] * r5[5 * n + 4] : xpt[2 * n + 1];
  }
};

template <typename T>
struct UprojTOp {
  using real = T;
  static constexpr int NIN = 3, NOUT = 2;
  Grid g;
  ElemConst<T> c;
  const T* coef;
  const T* r5;
  T* bpt;
  T* z5;
  Scale5<T> inv;   // 1 / row scale of r5
  __device__ void load(int i, int j, int k, T in[NIN]) const {
    const long n = g.node(i, j, k);
    const T iM = (T)1 / (c.W * (T)g.valence(i, j, k));
#pragma unroll
    for (int d = 0; d < 3; ++d) in[d] = g.ufix(i, j, d) ? (T)0 : inv.s[d] * r5[5 * n + d] * iM;
  }
  __device__ void element(int i, int j, int k, const T nd[8][NIN], T out[8][NOUT]) const {
    T zu[3][8], yP[8] = {0}, yT[8] = {0};
#pragma unroll
    for (int a = 0; a < 8; ++a) { zu[0][a] = nd[a][0]; zu[1][a] = nd[a][1]; zu[2][a] = nd[a][2]; }
    elem_uprojT<T>(zu, coef[2 * g.elem(i, j, k) + 1], c, yP, yT);
#pragma unroll
    for (int a = 0; a < 8; ++a) { out[a][0] = yP[a]; out[a][1] = yT[a]; }
  }
  __device__ void finish(int i, int j, int k, const T v[NOUT]) const {
    const long n = g.node(i, j, k);
    const T iM = (T)1 / (c.W * (T)g.valence(i, j, k));
#pragma unroll
    for (int d = 0; d < 3; ++d) z5[5 * n + d] = inv.s[d] * r5[5 * n + d] * (g.ufix(i, j, d) ? (T)1 : iM);
    bpt[2 * n] = g.pfix(i, j, k) ? (T)0 : inv.s[3] * r5[5 * n + 3] - v[0];
    bpt[2 * n + 1] = g.tfix(i, j, k) ? (T)0 : inv.s[4] * r5[5 * n + 4] - v[1];
  }
};

template <typename T>
static Scale5<T> inverse_or_ones(const Scale5<T>* s) {
  Scale5<T> r = ones_or<T>(nullptr);
  if (s)
    for (int f = 0; f < 5; ++f) r.s[f] = (T)1 / s->s[f];
  return r;
}
template <typename T>
void launch_uproj(hipStream_t st, const LevelView<T>& L, const T* x_pt, const T* r5, T* z5, const Scale5<T>* rows) {
  UprojOp<T> op{L.g, L.c, L.coef, x_pt, r5, z5, inverse_or_ones(rows)};
  run_zmarch(st, op);
}
template <typename T>
void launch_uprojT(hipStream_t st, const LevelView<T>& L, const T* r5, T* b_pt, T* z5, const Scale5<T>* rows) {
  UprojTOp<T> op{L.g, L.c, L.coef, r5, b_pt, z5, inverse_or_ones(rows)};
  run_zmarch(st, op);
}

#define NC_INST(T)                                                                                  \
  template void launch_jv5<T>(hipStream_t, const LevelView<T>&, const T*, T*, const Scale5<T>*);    \
  template void launch_jtw5<T>(hipStream_t, const LevelView<T>&, const T*, T*, const Scale5<T>*);   \
  template void launch_pt_apply<T>(hipStream_t, const LevelView<T>&, bool, int, const T*, const T*, T*, T, bool); \
  template bool tail_cycle_fits<T>(const Grid&, const Grid&, const Grid&);                            \
  template void launch_tail_cycle<T>(hipStream_t, const Grid&, const T*, T*, const LevelView<T>&, const Grid&,     \
                                     const double*, bool, T, int, int);                                \
  template void launch_pt_store<T>(hipStream_t, const LevelView<T>&, bool, const T*, T*, const Scale5<T>*);       \
  template void launch_diag_inverse<T>(hipStream_t, const LevelView<T>&, T*, bool);                 \
  template void launch_uproj<T>(hipStream_t, const LevelView<T>&, const T*, const T*, T*, const Scale5<T>*); \
  template void launch_uprojT<T>(hipStream_t, const LevelView<T>&, const T*, T*, T*, const Scale5<T>*);
NC_INST(double)
NC_INST(float)
#undef NC_INST

}  // namespace nc
