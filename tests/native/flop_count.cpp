// Floating-point operation count of the library's element kernels: the element header
// (paper_1904_00182_amd/csrc/element.hpp) instantiated on a scalar type that counts every
// add, subtract, multiply, divide and square root it performs.  The counts are the
// algorithmic flops per element of the operator applies (an FMA counts as two), used for
// the arithmetic roofline of those kernels.  Constant folding that the device compiler
// does (products of two compile-time constants) is counted here as work, which makes the
// figures upper bounds by a handful of operations.
#include <cmath>
#include <cstdio>
#include <cstring>

namespace cnt {
struct F;
}
namespace cnt {
static long n_add = 0, n_mul = 0, n_div = 0, n_sqrt = 0;
struct F {
  double v;
  constexpr F() : v(0) {}
  constexpr F(double x) : v(x) {}
  constexpr F(int x) : v(x) {}
  explicit operator double() const { return v; }
  F& operator+=(F o) { ++n_add; v += o.v; return *this; }
  F& operator-=(F o) { ++n_add; v -= o.v; return *this; }
  F& operator*=(F o) { ++n_mul; v *= o.v; return *this; }
};
inline F operator+(F a, F b) { ++n_add; return F(a.v + b.v); }
inline F operator-(F a, F b) { ++n_add; return F(a.v - b.v); }
inline F operator*(F a, F b) { ++n_mul; return F(a.v * b.v); }
inline F operator/(F a, F b) { ++n_div; return F(a.v / b.v); }
inline F operator-(F a) { return F(-a.v); }   // a sign flip folds into the consumer
inline bool operator<(F a, F b) { return a.v < b.v; }
inline bool operator>(F a, F b) { return a.v > b.v; }
inline F sqrt(F a) { ++n_sqrt; return F(std::sqrt(a.v)); }
inline void reset() { n_add = n_mul = n_div = n_sqrt = 0; }
inline long total() { return n_add + n_mul + n_div + n_sqrt; }
}  // namespace cnt

#include "../../paper_1904_00182_amd/csrc/element.hpp"

using cnt::F;
using namespace nc;

namespace {
void fill(F* a, int n, double s) {
  for (int i = 0; i < n; ++i) a[i] = F(s * (1.0 + 0.1 * i));
}
}  // namespace

// out[0..5]: flops per element of lin_modal, elem_jv_m<5 fields>, elem_jtw_m<5 fields>,
// elem_jv_m<2 fields>, elem_jtw_m<2 fields>, elem_residual_m<5 fields>.
extern "C" void fc_counts(long* out) {
  const ElemConst<F> c = make_elem_const<F>(1.0 / 16, 1, 1, 1, 1, 1e3, 0);
  F P[8], Tn[8], p[8], t[8], wP[8], wT[8], wU[3][8];
  fill(P, 8, 0.3); fill(Tn, 8, 0.2); fill(p, 8, 0.5); fill(t, 8, 0.7);
  fill(wP, 8, 0.4); fill(wT, 8, 0.6);
  for (int d = 0; d < 3; ++d) fill(wU[d], 8, 0.1 * (d + 1));
  LinM<F> L;
  cnt::reset();
  lin_modal(P, Tn, F(1.5), F(0.002), c, L);
  out[0] = cnt::total();
  {
    F yP[8], yT[8], yU[3][8];
    cnt::reset();
    elem_jv_m<F, true>(L, p, t, c, yP, yT, yU);
    out[1] = cnt::total();
  }
  {
    F yP[8], yT[8];
    cnt::reset();
    elem_jtw_m<F, true>(L, wP, wT, wU, c, yP, yT);
    out[2] = cnt::total();
  }
  {
    F yP[8], yT[8], yU[3][8];
    cnt::reset();
    elem_jv_m<F, false>(L, p, t, c, yP, yT, yU);
    out[3] = cnt::total();
  }
  {
    F yP[8], yT[8];
    cnt::reset();
    elem_jtw_m<F, false>(L, wP, wT, wU, c, yP, yT);
    out[4] = cnt::total();
  }
  {
    F rP[8], rT[8], rU[3][8];
    cnt::reset();
    elem_residual_m<F, true>(L, c, rP, rT, rU);
    out[5] = cnt::total();
  }
}

int main() {
  long o[6];
  fc_counts(o);
  std::printf("lin_modal %ld\njv5 %ld\njtw5 %ld\njv2 %ld\njtw2 %ld\nresidual5 %ld\n", o[0], o[1], o[2], o[3], o[4],
              o[5]);
  return 0;
}
