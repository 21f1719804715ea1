// Scalar types for the CPU oracle (test infrastructure only).
//
// The oracle's arithmetic is written once as templates over a scalar type T.
// This header provides the non-double scalars it is instantiated with:
//
//   Dual   forward-mode number (value + one tangent): Jacobian-vector products
//          of the discrete step, and the tangents of the initial data in (mu, sigma).
//   Rev    reverse-mode number recorded on a global tape: the oracle's own
//          discrete adjoint (transpose of the Jacobian of one whole RK4 step).
//   Cnt    double that counts its arithmetic operations: the algorithmic FLOP
//          count of one right-hand-side evaluation per grid point.
//
// Every type supports +, -, *, /, sqrt, exp, sin, cos and an n-ary linear
// combination (used by the finite-difference stencils), and exposes the plain
// double through value(). Branches in the oracle (upwind direction, recovery
// clamps) always test value(), so every scalar follows the same branch as double.
#pragma once
#include <cmath>
#include <cstdint>
#include <vector>

namespace oracle {

inline double value(double x) { return x; }

// Linear combination sum_i c[i]*f[i], summed left to right.
template <class T>
inline T lincomb(const T* f, const double* c, int n) {
  T s = c[0] * f[0];
  for (int i = 1; i < n; ++i) s = s + c[i] * f[i];
  return s;
}

// ---------------------------------------------------------------- Dual
struct Dual {
  double v = 0.0, d = 0.0;
  Dual() = default;
  Dual(double x) : v(x), d(0.0) {}
  Dual(double x, double dx) : v(x), d(dx) {}
};
inline double value(const Dual& x) { return x.v; }
inline Dual operator+(const Dual& a, const Dual& b) { return {a.v + b.v, a.d + b.d}; }
inline Dual operator-(const Dual& a, const Dual& b) { return {a.v - b.v, a.d - b.d}; }
inline Dual operator-(const Dual& a) { return {-a.v, -a.d}; }
inline Dual operator*(const Dual& a, const Dual& b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
inline Dual operator/(const Dual& a, const Dual& b) {
  double q = a.v / b.v;
  return {q, (a.d - q * b.d) / b.v};
}
inline Dual sqrt(const Dual& a) {
  double s = std::sqrt(a.v);
  return {s, a.d / (2.0 * s)};
}
inline Dual exp(const Dual& a) {
  double e = std::exp(a.v);
  return {e, e * a.d};
}
inline Dual sin(const Dual& a) { return {std::sin(a.v), std::cos(a.v) * a.d}; }
inline Dual cos(const Dual& a) { return {std::cos(a.v), -std::sin(a.v) * a.d}; }

// ---------------------------------------------------------------- Rev (tape)
// A tape node holds the partial derivatives of its result with respect to its
// parents. Variables created from plain doubles are constants (id < 0) and are
// not recorded.
struct Tape {
  std::vector<int64_t> start;   // first parent of node i (CSR)
  std::vector<int64_t> parent;  // parent node ids
  std::vector<double> partial;  // d(node)/d(parent)
  std::vector<double> adj;      // adjoints, filled by sweep()
  void clear() {
    start.clear();
    parent.clear();
    partial.clear();
    adj.clear();
    start.push_back(0);
  }
  int64_t size() const { return (int64_t)start.size() - 1; }
  int64_t push() {  // closes the node whose parents were just appended
    start.push_back((int64_t)parent.size());
    return size() - 1;
  }
  void arg(int64_t id, double p) {
    if (id >= 0) {
      parent.push_back(id);
      partial.push_back(p);
    }
  }
  // Reverse sweep: adj must be seeded (size() entries) before the call.
  void sweep() {
    for (int64_t i = size() - 1; i >= 0; --i) {
      double a = adj[i];
      if (a == 0.0) continue;
      for (int64_t q = start[i]; q < start[i + 1]; ++q) adj[parent[q]] += partial[q] * a;
    }
  }
};
extern Tape g_tape;

struct Rev {
  double v = 0.0;
  int64_t id = -1;
  Rev() = default;
  Rev(double x) : v(x), id(-1) {}
  static Rev input(double x) {  // a new independent variable
    Rev r;
    r.v = x;
    r.id = g_tape.push();
    return r;
  }
};
inline double value(const Rev& x) { return x.v; }
inline Rev rev_make(double v, int64_t a, double pa, int64_t b, double pb) {
  Rev r;
  r.v = v;
  if (a < 0 && b < 0) return r;
  g_tape.arg(a, pa);
  g_tape.arg(b, pb);
  r.id = g_tape.push();
  return r;
}
inline Rev operator+(const Rev& a, const Rev& b) { return rev_make(a.v + b.v, a.id, 1.0, b.id, 1.0); }
inline Rev operator-(const Rev& a, const Rev& b) { return rev_make(a.v - b.v, a.id, 1.0, b.id, -1.0); }
inline Rev operator-(const Rev& a) { return rev_make(-a.v, a.id, -1.0, -1, 0.0); }
inline Rev operator*(const Rev& a, const Rev& b) { return rev_make(a.v * b.v, a.id, b.v, b.id, a.v); }
inline Rev operator/(const Rev& a, const Rev& b) {
  double q = a.v / b.v;
  return rev_make(q, a.id, 1.0 / b.v, b.id, -q / b.v);
}
inline Rev sqrt(const Rev& a) {
  double s = std::sqrt(a.v);
  return rev_make(s, a.id, 0.5 / s, -1, 0.0);
}
inline Rev exp(const Rev& a) {
  double e = std::exp(a.v);
  return rev_make(e, a.id, e, -1, 0.0);
}
inline Rev sin(const Rev& a) { return rev_make(std::sin(a.v), a.id, std::cos(a.v), -1, 0.0); }
inline Rev cos(const Rev& a) { return rev_make(std::cos(a.v), a.id, -std::sin(a.v), -1, 0.0); }
template <>
inline Rev lincomb<Rev>(const Rev* f, const double* c, int n) {
  double s = c[0] * f[0].v;
  for (int i = 1; i < n; ++i) s = s + c[i] * f[i].v;
  Rev r;
  r.v = s;
  bool any = false;
  for (int i = 0; i < n; ++i)
    if (f[i].id >= 0) {
      g_tape.arg(f[i].id, c[i]);
      any = true;
    }
  if (any) r.id = g_tape.push();
  return r;
}

// ---------------------------------------------------------------- Cnt
// Counts +,-,* ,/ and sqrt (each one FLOP); exp/sin/cos are counted apart.
struct OpCount {
  int64_t add = 0, mul = 0, div = 0, sqrt = 0, transc = 0;
  int64_t flops() const { return add + mul + div + sqrt; }
};
extern OpCount g_count;
struct Cnt {
  double v = 0.0;
  Cnt() = default;
  Cnt(double x) : v(x) {}
};
inline double value(const Cnt& x) { return x.v; }
inline Cnt operator+(const Cnt& a, const Cnt& b) { ++g_count.add; return {a.v + b.v}; }
inline Cnt operator-(const Cnt& a, const Cnt& b) { ++g_count.add; return {a.v - b.v}; }
inline Cnt operator-(const Cnt& a) { return {-a.v}; }  // sign flip: not a FLOP
inline Cnt operator*(const Cnt& a, const Cnt& b) { ++g_count.mul; return {a.v * b.v}; }
inline Cnt operator/(const Cnt& a, const Cnt& b) { ++g_count.div; return {a.v / b.v}; }
inline Cnt sqrt(const Cnt& a) { ++g_count.sqrt; return {std::sqrt(a.v)}; }
inline Cnt exp(const Cnt& a) { ++g_count.transc; return {std::exp(a.v)}; }
inline Cnt sin(const Cnt& a) { ++g_count.transc; return {std::sin(a.v)}; }
inline Cnt cos(const Cnt& a) { ++g_count.transc; return {std::cos(a.v)}; }

}  // namespace oracle
