// Oracle (measurement infrastructure only): a scalar type that counts the
// floating-point operations the scheme performs on per-cell data.
//
// Instantiating the scheme of rto_scheme.hpp with Cnt counts every addition,
// subtraction, multiplication, division and square root applied to a value
// that depends on the state, once per occurrence in the scheme as written
// (each cell's slopes, predictor, two face fluxes per face, update and
// signal speed).  Arithmetic on the run's constants alone (dt/dx, gamma - 1,
// ...) is double arithmetic and is not counted; negation and absolute value
// are sign operations, not counted.  These are the algorithmic flops of a
// step, against which the kernels' FP64 rate is compared.
#pragma once
#include <cmath>
#include <cstdint>

namespace rto {

struct FlopCount {
  uint64_t add = 0, mul = 0, div = 0, sqrt = 0;
  uint64_t total() const { return add + mul + div + sqrt; }
};

inline FlopCount& flop_count() {
  static thread_local FlopCount c;
  return c;
}

struct Cnt {
  double v;
  Cnt() : v(0.0) {}
  Cnt(double x) : v(x) {}  // NOLINT: implicit from constants
};
inline double val(const Cnt& x) { return x.v; }
inline Cnt operator+(const Cnt& a, const Cnt& b) {
  ++flop_count().add;
  return Cnt(a.v + b.v);
}
inline Cnt operator-(const Cnt& a, const Cnt& b) {
  ++flop_count().add;
  return Cnt(a.v - b.v);
}
inline Cnt operator-(const Cnt& a) { return Cnt(-a.v); }
inline Cnt operator*(const Cnt& a, const Cnt& b) {
  ++flop_count().mul;
  return Cnt(a.v * b.v);
}
inline Cnt operator/(const Cnt& a, const Cnt& b) {
  ++flop_count().div;
  return Cnt(a.v / b.v);
}
inline Cnt sqrt(const Cnt& a) {
  ++flop_count().sqrt;
  return Cnt(std::sqrt(a.v));
}
inline Cnt fabs(const Cnt& a) { return Cnt(std::fabs(a.v)); }

}  // namespace rto
