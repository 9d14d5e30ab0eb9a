// Reference P3 tetrahedron tables, computed exactly in integer arithmetic.
//
// The P3 Lagrange basis on barycentric coordinates l0..l3 (section "Tetrahedral finite
// element method" of the paper uses order-3 Lagrange elements):
//   vertex a:             l_a (3 l_a - 1)(3 l_a - 2) / 2
//   edge (a,b), near a:   9/2 l_a l_b (3 l_a - 1)
//   face (a,b,c):         27 l_a l_b l_c
// Integrals of monomials over a simplex are exact:
//   (1/|T|) int_T l^al = 6 al! / (|al| + 3)!,   (1/|f|) int_f l^al = 2 al! / (|al| + 2)!
// Twice every basis coefficient is an integer, so each table entry is an integer N over a
// fixed denominator (4 * 9! for volume, 4 * 8! for faces) and is rounded to double once.
//
// Local node order: 0..3 vertices; 4..15 two nodes per edge for edges (0,1),(0,2),(0,3),
// (1,2),(1,3),(2,3), the node nearer the first vertex first; 16..19 face nodes, face f
// opposite vertex f.
#include <array>
#include <map>

#include "hz_internal.h"

namespace hz {
namespace {

using Exp = std::array<int, 4>;
using Poly = std::map<Exp, int64_t>;  // coefficients scaled by 2

const int kEdges[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};

int64_t fact(int k) {
  int64_t r = 1;
  for (int i = 2; i <= k; ++i) r *= i;
  return r;
}

Exp e1(int a, int pa, int b = -1, int pb = 0, int c = -1, int pc = 0) {
  Exp e{0, 0, 0, 0};
  e[a] += pa;
  if (b >= 0) e[b] += pb;
  if (c >= 0) e[c] += pc;
  return e;
}

std::vector<Poly> basis2() {
  std::vector<Poly> B(20);
  for (int a = 0; a < 4; ++a) {
    B[a][e1(a, 3)] += 9;
    B[a][e1(a, 2)] += -9;
    B[a][e1(a, 1)] += 2;
  }
  for (int e = 0; e < 6; ++e) {
    int a = kEdges[e][0], b = kEdges[e][1];
    Poly& p = B[4 + 2 * e];
    p[e1(a, 2, b, 1)] += 27;
    p[e1(a, 1, b, 1)] += -9;
    Poly& q = B[5 + 2 * e];
    q[e1(b, 2, a, 1)] += 27;
    q[e1(a, 1, b, 1)] += -9;
  }
  for (int f = 0; f < 4; ++f) {
    Exp e{1, 1, 1, 1};
    e[f] = 0;
    B[16 + f][e] += 54;
  }
  return B;
}

Poly deriv(const Poly& p, int a) {
  Poly d;
  for (auto& [e, c] : p)
    if (e[a] > 0) {
      Exp ne = e;
      ne[a] -= 1;
      d[ne] += c * e[a];
    }
  return d;
}

// sum over products of monomials: N = sum C_i C_j * scale * al! / (|al| + shift)!
int64_t int_prod(const Poly& p, const Poly& q, int skip_var, int shift, int64_t top, int64_t scale) {
  int64_t s = 0;
  for (auto& [ea, ca] : p)
    for (auto& [eb, cb] : q) {
      Exp e;
      int n = 0;
      bool skip = false;
      for (int k = 0; k < 4; ++k) {
        e[k] = ea[k] + eb[k];
        n += e[k];
        if (k == skip_var && e[k] > 0) skip = true;
      }
      if (skip) continue;
      int64_t num = scale;
      for (int k = 0; k < 4; ++k) num *= fact(e[k]);
      // top! / (n + shift)! is an integer since n + shift <= top
      int64_t r = 1;
      for (int k = n + shift + 1; k <= top; ++k) r *= k;
      s += ca * cb * num * r;
    }
  return s;
}

P3Tables build_tables() {
  P3Tables t{};
  auto B = basis2();
  std::vector<std::array<Poly, 4>> D(20);
  for (int i = 0; i < 20; ++i)
    for (int a = 0; a < 4; ++a) D[i][a] = deriv(B[i], a);
  const double dvol = 4.0 * (double)fact(9);
  const double dface = 4.0 * (double)fact(8);
  for (int i = 0; i < 20; ++i)
    for (int j = 0; j <= i; ++j) {
      int pk = i * (i + 1) / 2 + j;
      t.M[pk] = (double)int_prod(B[i], B[j], -1, 3, 9, 6) / dvol;
      int p = 0;
      for (int a = 0; a < 4; ++a)
        for (int b = a; b < 4; ++b, ++p) {
          int64_t N = int_prod(D[i][a], D[j][b], -1, 3, 9, 6);
          if (a != b) N += int_prod(D[i][b], D[j][a], -1, 3, 9, 6);
          t.S[p][pk] = (double)N / dvol;
        }
    }
  for (int f = 0; f < 4; ++f) {
    int m = 0;
    for (int v = 0; v < 4; ++v)
      if (v != f) t.face_nodes[f][m++] = v;
    for (int e = 0; e < 6; ++e)
      if (kEdges[e][0] != f && kEdges[e][1] != f) {
        t.face_nodes[f][m++] = 4 + 2 * e;
        t.face_nodes[f][m++] = 5 + 2 * e;
      }
    t.face_nodes[f][m++] = 16 + f;
    for (int a = 0; a < 10; ++a)
      for (int b = 0; b <= a; ++b) {
        int i = t.face_nodes[f][a], j = t.face_nodes[f][b];
        t.F[f][a * (a + 1) / 2 + b] = (double)int_prod(B[i], B[j], f, 2, 8, 2) / dface;
      }
  }
  return t;
}

}  // namespace

const P3Tables& p3_tables() {
  static const P3Tables t = build_tables();
  return t;
}

void p3_eval_basis(const double lam[4], double phi[20]) {
  for (int a = 0; a < 4; ++a) phi[a] = 0.5 * lam[a] * (3 * lam[a] - 1) * (3 * lam[a] - 2);
  for (int e = 0; e < 6; ++e) {
    int a = kEdges[e][0], b = kEdges[e][1];
    phi[4 + 2 * e] = 4.5 * lam[a] * lam[b] * (3 * lam[a] - 1);
    phi[5 + 2 * e] = 4.5 * lam[a] * lam[b] * (3 * lam[b] - 1);
  }
  for (int f = 0; f < 4; ++f) {
    double p = 27.0;
    for (int v = 0; v < 4; ++v)
      if (v != f) p *= lam[v];
    phi[16 + f] = p;
  }
}

}  // namespace hz
