// Scalar types the oracle's physics is instantiated with.
//
// TEST INFRASTRUCTURE ONLY. Part of the FP64 CPU oracle; nothing in the
// product library includes or links this.
//
//   double  - plain forward evaluation
//   Var     - operator-overloading reverse-mode AD on a per-thread tape:
//             the exact derivative of the discrete map, obtained mechanically
//             from the same code that computes the forward result
//   Cnt     - double that counts every arithmetic operation (algorithmic flops)
//
// Branch decisions (clamps, disk projection, contact activation) are taken on
// values; the tape then holds the derivative of the branch that was taken.
#pragma once
#include <cmath>
#include <cstdint>
#include <vector>

namespace orc {

// ---------------------------------------------------------------- tape
struct Tape {
  struct Node { int a, b; double da, db; };
  std::vector<Node> nodes;
  std::vector<double> adj;
  int push(int a, double da, int b, double db) {
    nodes.push_back({a, b, da, db});
    return (int)nodes.size() - 1;
  }
  int leaf() { return push(-1, 0.0, -1, 0.0); }
  void clear() { nodes.clear(); adj.clear(); }
  // Reverse sweep: adjoints of all nodes, given seeds already placed in adj.
  void sweep() {
    for (int i = (int)nodes.size() - 1; i >= 0; --i) {
      const double g = adj[i];
      if (g == 0.0) continue;
      const Node& n = nodes[i];
      if (n.a >= 0) adj[n.a] += n.da * g;
      if (n.b >= 0) adj[n.b] += n.db * g;
    }
  }
};

inline Tape*& tape() { static thread_local Tape* t = nullptr; return t; }

struct Var {
  double v;
  int id;  // -1: constant
  Var() : v(0.0), id(-1) {}
  Var(double x) : v(x), id(-1) {}
  Var(double x, int i) : v(x), id(i) {}
  static Var input(double x) { return Var(x, tape()->leaf()); }
};

inline Var mk1(double v, const Var& x, double dx) {
  if (x.id < 0) return Var(v);
  return Var(v, tape()->push(x.id, dx, -1, 0.0));
}
inline Var mk2(double v, const Var& x, double dx, const Var& y, double dy) {
  if (x.id < 0 && y.id < 0) return Var(v);
  if (x.id < 0) return Var(v, tape()->push(y.id, dy, -1, 0.0));
  if (y.id < 0) return Var(v, tape()->push(x.id, dx, -1, 0.0));
  return Var(v, tape()->push(x.id, dx, y.id, dy));
}
inline Var operator+(const Var& a, const Var& b) { return mk2(a.v + b.v, a, 1.0, b, 1.0); }
inline Var operator-(const Var& a, const Var& b) { return mk2(a.v - b.v, a, 1.0, b, -1.0); }
inline Var operator*(const Var& a, const Var& b) { return mk2(a.v * b.v, a, b.v, b, a.v); }
inline Var operator/(const Var& a, const Var& b) {
  const double q = a.v / b.v;
  return mk2(q, a, 1.0 / b.v, b, -q / b.v);
}
inline Var operator-(const Var& a) { return mk1(-a.v, a, -1.0); }
inline Var& operator+=(Var& a, const Var& b) { a = a + b; return a; }
inline Var& operator-=(Var& a, const Var& b) { a = a - b; return a; }
inline Var& operator*=(Var& a, const Var& b) { a = a * b; return a; }
inline Var sqrt(const Var& a) {
  const double s = std::sqrt(a.v);
  return mk1(s, a, s > 0.0 ? 0.5 / s : 0.0);
}
inline Var sin(const Var& a) { return mk1(std::sin(a.v), a, std::cos(a.v)); }
inline Var cos(const Var& a) { return mk1(std::cos(a.v), a, -std::sin(a.v)); }
inline Var tanh(const Var& a) { const double t = std::tanh(a.v); return mk1(t, a, 1.0 - t * t); }
inline Var atan2(const Var& y, const Var& x) {
  const double r2 = x.v * x.v + y.v * y.v;
  return mk2(std::atan2(y.v, x.v), y, r2 > 0 ? x.v / r2 : 0.0, x, r2 > 0 ? -y.v / r2 : 0.0);
}
inline double val(const Var& a) { return a.v; }

// ---------------------------------------------------------------- counted
inline uint64_t& flop_counter() { static thread_local uint64_t c = 0; return c; }
struct Cnt {
  double v;
  Cnt() : v(0.0) {}
  Cnt(double x) : v(x) {}
};
#define ORC_CNT_BIN(op)                                                  \
  inline Cnt operator op(const Cnt& a, const Cnt& b) {                   \
    ++flop_counter();                                                    \
    return Cnt(a.v op b.v);                                              \
  }
ORC_CNT_BIN(+)
ORC_CNT_BIN(-)
ORC_CNT_BIN(*)
ORC_CNT_BIN(/)
#undef ORC_CNT_BIN
inline Cnt operator-(const Cnt& a) { return Cnt(-a.v); }
inline Cnt& operator+=(Cnt& a, const Cnt& b) { a = a + b; return a; }
inline Cnt& operator-=(Cnt& a, const Cnt& b) { a = a - b; return a; }
inline Cnt& operator*=(Cnt& a, const Cnt& b) { a = a * b; return a; }
inline Cnt sqrt(const Cnt& a) { ++flop_counter(); return Cnt(std::sqrt(a.v)); }
inline Cnt sin(const Cnt& a) { ++flop_counter(); return Cnt(std::sin(a.v)); }
inline Cnt cos(const Cnt& a) { ++flop_counter(); return Cnt(std::cos(a.v)); }
inline Cnt tanh(const Cnt& a) { ++flop_counter(); return Cnt(std::tanh(a.v)); }
inline Cnt atan2(const Cnt& y, const Cnt& x) { ++flop_counter(); return Cnt(std::atan2(y.v, x.v)); }
inline double val(const Cnt& a) { return a.v; }

inline double val(double a) { return a; }
inline double sqrt(double a) { return std::sqrt(a); }
inline double sin(double a) { return std::sin(a); }
inline double cos(double a) { return std::cos(a); }
inline double tanh(double a) { return std::tanh(a); }
inline double atan2(double y, double x) { return std::atan2(y, x); }

}  // namespace orc
