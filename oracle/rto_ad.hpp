// Oracle (test infrastructure only): scalar types for automatic differentiation.
//
// The paper obtains the exact gradient of its discretised objective by
// reverse-mode automatic differentiation through the whole time march
// (Sec. 2.3 and Sec. 3.4).  The oracle does the same, in the plainest way:
// the scheme is written once, templated on its scalar type, and run with
//   * double  - the primal,
//   * Dual    - forward mode (exact tangent-linear model, one direction),
//   * Rev     - reverse mode on an operation tape (exact adjoint).
// Branches in the scheme (limiter cases, Riemann-solver cases) are taken on
// primal values, so both AD modes differentiate the branch that the primal
// takes.  Nothing here is shared with the GPU path.
#pragma once
#include <cmath>
#include <cstddef>
#include <vector>

namespace rto {

inline double val(double x) { return x; }
inline double sqrt(double x) { return std::sqrt(x); }
inline double fabs(double x) { return std::fabs(x); }

// ---------------------------------------------------------------- forward mode
struct Dual {
  double v, d;
  Dual() : v(0.0), d(0.0) {}
  Dual(double x) : v(x), d(0.0) {}  // NOLINT: implicit from constants
  Dual(double x, double dx) : v(x), d(dx) {}
};
inline double val(const Dual& x) { return x.v; }
inline Dual operator+(const Dual& a, const Dual& b) { return Dual(a.v + b.v, a.d + b.d); }
inline Dual operator-(const Dual& a, const Dual& b) { return Dual(a.v - b.v, a.d - b.d); }
inline Dual operator-(const Dual& a) { return Dual(-a.v, -a.d); }
inline Dual operator*(const Dual& a, const Dual& b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
inline Dual operator/(const Dual& a, const Dual& b) {
  const double q = a.v / b.v;
  return Dual(q, (a.d - q * b.d) / b.v);
}
inline Dual sqrt(const Dual& a) {
  const double s = std::sqrt(a.v);
  return Dual(s, a.d / (2.0 * s));
}
inline Dual fabs(const Dual& a) { return a.v < 0.0 ? -a : a; }

// ---------------------------------------------------------------- reverse mode
// One tape node per elementary operation: up to two parents with the local
// partial derivative towards each.  A leaf (independent variable) has no
// parents; a constant is not on the tape at all (index -1).
struct Tape {
  struct Node {
    int a, b;
    double da, db;
  };
  std::vector<Node> nodes;
  std::vector<double> adj;

  void clear() {
    nodes.clear();
    adj.clear();
  }
  int push(int a, double da, int b, double db) {
    nodes.push_back(Node{a, b, da, db});
    return static_cast<int>(nodes.size()) - 1;
  }
  // Propagate adjoints from the last node back to the first.  The caller has
  // sized `adj` to nodes.size() and seeded the outputs.
  void sweep() {
    for (std::ptrdiff_t k = static_cast<std::ptrdiff_t>(nodes.size()) - 1; k >= 0; --k) {
      const double g = adj[k];
      if (g == 0.0) continue;
      const Node& n = nodes[k];
      if (n.a >= 0) adj[n.a] += n.da * g;
      if (n.b >= 0) adj[n.b] += n.db * g;
    }
  }
};

// The active tape.  The oracle is single-threaded.
Tape& tape();

struct Rev {
  double v;
  int i;
  Rev() : v(0.0), i(-1) {}
  Rev(double x) : v(x), i(-1) {}  // NOLINT: implicit from constants
  Rev(double x, int idx) : v(x), i(idx) {}
  static Rev leaf(double x) { return Rev(x, tape().push(-1, 0.0, -1, 0.0)); }
};
inline double val(const Rev& x) { return x.v; }

inline Rev rev_node(double v, const Rev& a, double da, const Rev& b, double db) {
  if (a.i < 0 && b.i < 0) return Rev(v);
  if (a.i < 0) return Rev(v, tape().push(b.i, db, -1, 0.0));
  if (b.i < 0) return Rev(v, tape().push(a.i, da, -1, 0.0));
  return Rev(v, tape().push(a.i, da, b.i, db));
}
inline Rev rev_node(double v, const Rev& a, double da) {
  if (a.i < 0) return Rev(v);
  return Rev(v, tape().push(a.i, da, -1, 0.0));
}
inline Rev operator+(const Rev& a, const Rev& b) { return rev_node(a.v + b.v, a, 1.0, b, 1.0); }
inline Rev operator-(const Rev& a, const Rev& b) { return rev_node(a.v - b.v, a, 1.0, b, -1.0); }
inline Rev operator-(const Rev& a) { return rev_node(-a.v, a, -1.0); }
inline Rev operator*(const Rev& a, const Rev& b) { return rev_node(a.v * b.v, a, b.v, b, a.v); }
inline Rev operator/(const Rev& a, const Rev& b) {
  const double q = a.v / b.v;
  return rev_node(q, a, 1.0 / b.v, b, -q / b.v);
}
inline Rev sqrt(const Rev& a) {
  const double s = std::sqrt(a.v);
  return rev_node(s, a, 0.5 / s);
}
inline Rev fabs(const Rev& a) { return a.v < 0.0 ? -a : a; }

}  // namespace rto
