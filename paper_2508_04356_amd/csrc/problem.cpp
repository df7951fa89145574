// Host-side problem construction: DOF numbering, Q2/Q1 assembly of eq. (2.1),
// the structured decomposition and the interface entities of Section 2.1,
// and the subregion bookkeeping of the three-level method (eq. 2.5).
//
// The element matrices are built from exact one-dimensional integrals of the
// Q2 (nodes 0, 1/2, 1) and Q1 Lagrange bases: on a cube of edge h the
// velocity block is mu (S x M x M + M x S x M + M x M x S) and the divergence
// block -int psi_q d(phi_a)/dx_c factors into G x G x C in the same way.
#include "problem.h"

#include <algorithm>
#include <cmath>
#include <exception>
#include <map>
#include <stdexcept>
#include <thread>
#include <utility>

namespace gdsw {
namespace {

struct ElementMatrix {
  double a[89][89];  // velocity (3*node + comp) then pressure (81 + q)
};

void element_matrix(double h, double mu, bool disc, ElementMatrix& E) {
  // int L_a L_b, int L_a' L_b', int N_q L_a, int N_q L_a' on [0, 1]
  static const double Mr[3][3] = {{4, 2, -1}, {2, 16, 2}, {-1, 2, 4}};
  static const double Sr[3][3] = {{7, -8, 1}, {-8, 16, -8}, {1, -8, 7}};
  static const double Gr[2][3] = {{1.0 / 6, 1.0 / 3, 0.0}, {0.0, 1.0 / 3, 1.0 / 6}};
  static const double Cr[2][3] = {{-5.0 / 6, 2.0 / 3, 1.0 / 6}, {-1.0 / 6, -2.0 / 3, 5.0 / 6}};
  double M[3][3], S[3][3], G[2][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      M[i][j] = Mr[i][j] * h / 30.0;
      S[i][j] = Sr[i][j] / (3.0 * h);
    }
  for (int q = 0; q < 2; ++q)
    for (int j = 0; j < 3; ++j) G[q][j] = Gr[q][j] * h;
  for (int i = 0; i < 89; ++i)
    for (int j = 0; j < 89; ++j) E.a[i][j] = 0.0;
  for (int a = 0; a < 27; ++a) {
    const int ax = a % 3, ay = (a / 3) % 3, az = a / 9;
    for (int b = 0; b < 27; ++b) {
      const int bx = b % 3, by = (b / 3) % 3, bz = b / 9;
      const double k = mu * (S[ax][bx] * M[ay][by] * M[az][bz] + M[ax][bx] * S[ay][by] * M[az][bz] +
                             M[ax][bx] * M[ay][by] * S[az][bz]);
      for (int comp = 0; comp < 3; ++comp) E.a[3 * a + comp][3 * b + comp] = k;
    }
  }
  if (disc) {
    // P1disc: psi = 1, 2x - 1, 2y - 1, 2z - 1 on the reference cube; per axis
    // int f L_a and int f L_a' for f = 1 and f = 2x - 1
    static const double I1[3] = {1.0 / 6, 2.0 / 3, 1.0 / 6}, D1[3] = {-1.0, 0.0, 1.0};
    static const double J1[3] = {-1.0 / 6, 0.0, 1.0 / 6}, JD[3] = {2.0 / 3, -4.0 / 3, 2.0 / 3};
    for (int q = 0; q < 4; ++q)
      for (int a = 0; a < 27; ++a) {
        const int ai[3] = {a % 3, (a / 3) % 3, a / 9};
        for (int comp = 0; comp < 3; ++comp) {
          double v = -h * h;
          for (int ax = 0; ax < 3; ++ax) {
            const bool lin = q == ax + 1;  // psi_q is linear along this axis
            v *= ax == comp ? (lin ? JD[ai[ax]] : D1[ai[ax]]) : (lin ? J1[ai[ax]] : I1[ai[ax]]);
          }
          E.a[81 + q][3 * a + comp] = v;
          E.a[3 * a + comp][81 + q] = v;
        }
      }
    return;
  }
  for (int q = 0; q < 8; ++q) {
    const int qx = q % 2, qy = (q / 2) % 2, qz = q / 4;
    for (int a = 0; a < 27; ++a) {
      const int ax = a % 3, ay = (a / 3) % 3, az = a / 9;
      const double d[3] = {-Cr[qx][ax] * G[qy][ay] * G[qz][az],
                           -G[qx][ax] * Cr[qy][ay] * G[qz][az],
                           -G[qx][ax] * G[qy][ay] * Cr[qz][az]};
      for (int comp = 0; comp < 3; ++comp) {
        E.a[81 + q][3 * a + comp] = d[comp];
        E.a[3 * a + comp][81 + q] = d[comp];
      }
    }
  }
}

inline void box_range(int coord, int s, int m, int& lo, int& hi) {
  const int two_s = 2 * s;
  lo = (coord % two_s == 0) ? std::max(coord / two_s - 1, 0) : coord / two_s;
  hi = std::min(coord / two_s, m - 1);
}

// f(t) for t in [0, nt), t = 0 on the calling thread; an exception thrown by
// any of them is rethrown here (the lowest t first)
template <class F>
void run_threads(int nt, F&& f) {
  std::vector<std::exception_ptr> err(nt);
  auto guarded = [&](int t) {
    try {
      f(t);
    } catch (...) {
      err[t] = std::current_exception();
    }
  };
  std::vector<std::thread> pool;
  for (int t = 1; t < nt; ++t) pool.emplace_back(guarded, t);
  guarded(0);
  for (auto& th : pool) th.join();
  for (auto& e : err)
    if (e) std::rethrow_exception(e);
}

}  // namespace

std::vector<int32_t> entity_subdomains(const Problem& P, int e) {
  const auto& k = P.ent_key[e];
  const int m = P.spec.m;
  std::vector<int32_t> out;
  for (int K = k[2]; K <= k[5]; ++K)
    for (int J = k[1]; J <= k[4]; ++J)
      for (int I = k[0]; I <= k[3]; ++I) out.push_back(I + m * (J + m * K));
  return out;
}

void build_problem(const ProblemSpec& spec, Problem& P, int threads) {
  const int n = spec.n, m = spec.m;
  if (n < 1 || m < 1 || n % m != 0) throw std::invalid_argument("need n >= 1, m >= 1 and n % m == 0");
  if (spec.overlap < 1) throw std::invalid_argument("overlap must be >= 1");
  if (spec.levels != 2 && spec.levels != 3) throw std::invalid_argument("levels must be 2 or 3");
  if (spec.levels == 3 && (spec.group < 1 || m % spec.group != 0))
    throw std::invalid_argument("three levels need m % group == 0");
  if (!(spec.mu > 0.0)) throw std::invalid_argument("viscosity must be > 0");
  if (spec.pressure != 0 && spec.pressure != 1) throw std::invalid_argument("pressure element must be 0 (Q1) or 1 (P1disc)");
  if (spec.coarse != 0 && spec.coarse != 1) throw std::invalid_argument("coarse space must be 0 (GDSW) or 1 (GDSW*)");
  const bool disc = spec.pressure == 1;
  if (disc && spec.local_dirichlet)
    throw std::invalid_argument("the P1disc pressure needs the algebraic overlap (local_algebraic = 1): with "
                                "Dirichlet velocity on the whole artificial boundary the constant pressure of an "
                                "interior local problem is a null vector");
  if (disc && spec.levels == 3) throw std::invalid_argument("three levels with the P1disc pressure are not built");
  P.spec = spec;
  P.s = n / m;
  const int N2 = 2 * n + 1, N1 = n + 1;
  const double h = 1.0 / n;

  // ---- numbering --------------------------------------------------------
  // free velocity node: a >= 1, 1 <= b <= 2n-1, 1 <= c <= 2n-1
  const int64_t fa = 2 * n, fb = 2 * n - 1;
  P.n_u = 3 * fa * fb * fb;
  P.n_p = disc ? 4 * (int64_t)n * n * n : (int64_t)N1 * N1 * N1;
  P.n_free = P.n_u + P.n_p;
  P.n_full = 3 * (int64_t)N2 * N2 * N2 + P.n_p;
  auto vel_free = [&](int a, int b, int c) { return a >= 1 && b >= 1 && b <= 2 * n - 1 && c >= 1 && c <= 2 * n - 1; };
  auto vel_dof = [&](int a, int b, int c, int comp) -> int64_t {
    return 3 * ((int64_t)(a - 1) + fa * ((int64_t)(b - 1) + fb * (c - 1))) + comp;
  };
  auto p_dof = [&](int i, int j, int k) -> int64_t { return P.n_u + i + (int64_t)N1 * (j + (int64_t)N1 * k); };
  // P1disc: element e = ex + n (ey + n ez), basis function k
  auto pe_dof = [&](int64_t e, int k) -> int64_t { return P.n_u + 4 * e + k; };
  auto inflow = [&](int a, int b, int c) -> double {  // x-velocity Dirichlet data
    if (a != 0) return 0.0;
    const double y = 0.5 * h * b, z = 0.5 * h * c;
    return spec.c * y * (1.0 - y) * z * (1.0 - z);
  };

  P.field.assign(P.n_free, 0);
  P.pnull.assign(P.n_free, 1);
  P.abc.assign(3 * P.n_free, 0);
  P.full_index.assign(P.n_free, 0);
  P.dirichlet_full.assign(P.n_full, 0.0);
  for (int c = 0; c < N2; ++c)
    for (int b = 0; b < N2; ++b)
      for (int a = 0; a < N2; ++a) {
        const int64_t node = a + (int64_t)N2 * (b + (int64_t)N2 * c);
        if (vel_free(a, b, c)) {
          for (int comp = 0; comp < 3; ++comp) {
            const int64_t d = vel_dof(a, b, c, comp);
            P.field[d] = (int8_t)comp;
            P.abc[3 * d] = a;
            P.abc[3 * d + 1] = b;
            P.abc[3 * d + 2] = c;
            P.full_index[d] = 3 * node + comp;
          }
        } else {
          P.dirichlet_full[3 * node] = inflow(a, b, c);
        }
      }
  if (disc) {
    // a P1disc pressure DOF sits at its element's centre node
    for (int ez = 0; ez < n; ++ez)
      for (int ey = 0; ey < n; ++ey)
        for (int ex = 0; ex < n; ++ex)
          for (int k = 0; k < 4; ++k) {
            const int64_t e = ex + (int64_t)n * (ey + (int64_t)n * ez), d = pe_dof(e, k);
            P.field[d] = 3;
            P.pnull[d] = k == 0;
            P.abc[3 * d] = 2 * ex + 1;
            P.abc[3 * d + 1] = 2 * ey + 1;
            P.abc[3 * d + 2] = 2 * ez + 1;
            P.full_index[d] = 3 * (int64_t)N2 * N2 * N2 + (d - P.n_u);
          }
  } else {
    for (int k = 0; k < N1; ++k)
      for (int j = 0; j < N1; ++j)
        for (int i = 0; i < N1; ++i) {
          const int64_t d = p_dof(i, j, k);
          P.field[d] = 3;
          P.abc[3 * d] = 2 * i;
          P.abc[3 * d + 1] = 2 * j;
          P.abc[3 * d + 2] = 2 * k;
          P.full_index[d] = 3 * (int64_t)N2 * N2 * N2 + (d - P.n_u);
        }
  }

  // ---- assembly, one row at a time ---------------------------------------
  ElementMatrix E;
  element_matrix(h, spec.mu, disc, E);
  const int npe = disc ? 4 : 8;  // pressure functions per element
  const double gt = std::sqrt(3.0 / 5.0);
  const double gp[3] = {0.5 - 0.5 * gt, 0.5, 0.5 + 0.5 * gt};
  const double gw[3] = {5.0 / 18.0, 8.0 / 18.0, 5.0 / 18.0};
  const double intL[3] = {1.0 / 6.0, 2.0 / 3.0, 1.0 / 6.0};
  auto L2 = [](int a, double x) {
    return a == 0 ? 2.0 * (x - 0.5) * (x - 1.0) : (a == 1 ? 4.0 * x * (1.0 - x) : 2.0 * x * (x - 0.5));
  };

  // Rows are assembled in contiguous chunks, one per thread, in two passes
  // (the first counts each row's entries, the second writes them into the
  // CSR arrays), so the threads allocate nothing.  A row's columns lie in the neighbourhood of its
  // node: per axis the nodes 2 elo .. 2 elo + 4 of the elements holding it
  // (velocity) and the pressure nodes elo .. elo + 2 (Q1) or the elements
  // elo .. elo + 1 (P1disc).  Each column has a slot there, and slot order
  // is column order (DOFs are numbered node-major, z slowest, pressure after
  // velocity), so the element contributions are summed per slot in element
  // order and the touched slots are emitted in order.
  constexpr int NVS = 5 * 5 * 5 * 3, NPS = 32;  // velocity, pressure slots (Q1 needs 27)
  const int nth = (int)std::max<int64_t>(1, std::min<int64_t>(threads, (P.n_free + 1023) / 1024));
  const int64_t chunk = (P.n_free + nth - 1) / nth;
  P.row_ptr.assign(P.n_free + 1, 0);
  P.rhs.assign(P.n_free, 0.0);
  auto assemble_rows = [&](int t, bool write) {
    const int64_t r0 = t * chunk, r1 = std::min<int64_t>(P.n_free, r0 + chunk);
    double acc[NVS + NPS];
    int32_t scol[NVS + NPS];
    int64_t mark[NVS + NPS];  // the row that last touched the slot
    std::fill(mark, mark + NVS + NPS, (int64_t)-1);
    for (int64_t r = r0; r < r1; ++r) {
      const int A = P.abc[3 * r], B = P.abc[3 * r + 1], Cc = P.abc[3 * r + 2];
      const int fr = P.field[r];
      int elo[3], ehi[3];
      const int crd[3] = {A, B, Cc};
      for (int d = 0; d < 3; ++d) {
        if (crd[d] % 2 == 0) {
          elo[d] = std::max(crd[d] / 2 - 1, 0);
          ehi[d] = std::min(crd[d] / 2, n - 1);
        } else {
          elo[d] = ehi[d] = (crd[d] - 1) / 2;
        }
      }
      auto add = [&](int slot, int32_t c, double v) {
        if (mark[slot] != r) {
          mark[slot] = r;
          scol[slot] = c;
          acc[slot] = v;
        } else {
          acc[slot] += v;
        }
      };
      double rhs = 0.0;
      for (int ez = elo[2]; ez <= ehi[2]; ++ez)
        for (int ey = elo[1]; ey <= ehi[1]; ++ey)
          for (int ex = elo[0]; ex <= ehi[0]; ++ex) {
            int li;
            if (fr < 3) {
              li = 3 * ((A - 2 * ex) + 3 * ((B - 2 * ey) + 3 * (Cc - 2 * ez))) + fr;
            } else if (disc) {
              li = 81 + (int)((r - P.n_u) % 4);
            } else {
              li = 81 + (A / 2 - ex) + 2 * ((B / 2 - ey) + 2 * (Cc / 2 - ez));
            }
            for (int lb = 0; lb < 27; ++lb) {
              const int ga = 2 * ex + lb % 3, gb = 2 * ey + (lb / 3) % 3, gc = 2 * ez + lb / 9;
              for (int comp = 0; comp < 3; ++comp) {
                const double v = E.a[li][3 * lb + comp];
                if (v == 0.0) continue;
                if (vel_free(ga, gb, gc))
                  add(3 * ((ga - 2 * elo[0]) + 5 * ((gb - 2 * elo[1]) + 5 * (gc - 2 * elo[2]))) + comp,
                      (int32_t)vel_dof(ga, gb, gc, comp), v);
                else if (comp == 0)
                  rhs -= v * inflow(ga, gb, gc);
              }
            }
            for (int q = 0; q < npe; ++q) {
              const double v = E.a[li][81 + q];
              if (v == 0.0) continue;
              if (disc)
                add(NVS + 4 * ((ex - elo[0]) + 2 * ((ey - elo[1]) + 2 * (ez - elo[2]))) + q,
                    (int32_t)pe_dof(ex + (int64_t)n * (ey + (int64_t)n * ez), q), v);
              else
                add(NVS + (ex + q % 2 - elo[0]) + 3 * ((ey + (q / 2) % 2 - elo[1]) + 3 * (ez + q / 4 - elo[2])),
                    (int32_t)p_dof(ex + q % 2, ey + (q / 2) % 2, ez + q / 4), v);
            }
            if (spec.manufactured && fr == 0) {
              // int f_x phi = h^3 int L_ax dxi * int int f(y, z) L_ay L_az (3-point Gauss, exact)
              const int ax = A - 2 * ex, ay = B - 2 * ey, az = Cc - 2 * ez;
              double s2 = 0.0;
              for (int qy = 0; qy < 3; ++qy)
                for (int qz = 0; qz < 3; ++qz) {
                  const double y = (ey + gp[qy]) * h, z = (ez + gp[qz]) * h;
                  const double f = 2.0 * spec.mu * spec.c * (y * (1.0 - y) + z * (1.0 - z));
                  s2 += gw[qy] * gw[qz] * f * L2(ay, gp[qy]) * L2(az, gp[qz]);
                }
              rhs += h * h * h * intL[ax] * s2;
            }
          }
      if (!write) {  // pass 1: the row's entry count, kept in row_ptr[r + 1]
        int32_t cnt = 0;
        for (int k = 0; k < NVS + NPS; ++k) cnt += mark[k] == r;
        P.row_ptr[r + 1] = cnt;
        continue;
      }
      int64_t o = P.row_ptr[r];
      for (int k = 0; k < NVS + NPS; ++k)
        if (mark[k] == r) {
          P.col[o] = scol[k];
          P.val[o] = acc[k];
          ++o;
        }
      P.rhs[r] = rhs;
    }
  };
  run_threads(nth, [&](int t) { assemble_rows(t, false); });
  int64_t nnz = 0;
  for (int64_t r = 0; r < P.n_free; ++r) {
    nnz += P.row_ptr[r + 1];
    if (nnz > INT32_MAX) throw std::invalid_argument("matrix too large for int32 CSR");
    P.row_ptr[r + 1] = (int32_t)nnz;
  }
  P.col.resize(nnz);
  P.val.resize(nnz);
  run_threads(nth, [&](int t) { assemble_rows(t, true); });

  // ---- decomposition ----------------------------------------------------
  const int s = P.s;
  P.n_sub = m * m * m;
  P.multiplicity.assign(P.n_free, 0);
  std::vector<std::array<int32_t, 6>> key(P.n_free);
  for (int64_t d = 0; d < P.n_free; ++d) {
    int mult = 1;
    for (int ax = 0; ax < 3; ++ax) {
      int lo, hi;
      box_range(P.abc[3 * d + ax], s, m, lo, hi);
      key[d][ax] = lo;
      key[d][3 + ax] = hi;
      mult *= hi - lo + 1;
    }
    P.multiplicity[d] = (int8_t)mult;
  }
  auto collect_box = [&](int lo_a, int hi_a, int lo_b, int hi_b, int lo_c, int hi_c, std::vector<int32_t>& out) {
    out.clear();
    for (int c = lo_c; c <= hi_c; ++c)
      for (int b = lo_b; b <= hi_b; ++b)
        for (int a = lo_a; a <= hi_a; ++a)
          if (vel_free(a, b, c))
            for (int comp = 0; comp < 3; ++comp) out.push_back((int32_t)vel_dof(a, b, c, comp));
    if (disc) {  // elements whose centre node lies in the box
      for (int ez = lo_c / 2; ez < n && 2 * ez + 1 <= hi_c; ++ez)
        for (int ey = lo_b / 2; ey < n && 2 * ey + 1 <= hi_b; ++ey)
          for (int ex = lo_a / 2; ex < n && 2 * ex + 1 <= hi_a; ++ex)
            for (int k = 0; k < 4; ++k)
              out.push_back((int32_t)pe_dof(ex + (int64_t)n * (ey + (int64_t)n * ez), k));
    } else {
      for (int k = (lo_c + 1) / 2; 2 * k <= hi_c; ++k)
        for (int j = (lo_b + 1) / 2; 2 * j <= hi_b; ++j)
          for (int i = (lo_a + 1) / 2; 2 * i <= hi_a; ++i) out.push_back((int32_t)p_dof(i, j, k));
    }
  };
  P.S.resize(P.n_sub);
  P.D.resize(P.n_sub);
  P.I.resize(P.n_sub);
  const int dl = spec.overlap;
  for (int K = 0; K < m; ++K)
    for (int J = 0; J < m; ++J)
      for (int I = 0; I < m; ++I) {
        const int i = I + m * (J + m * K);
        auto lo = [&](int X) { return std::max(0, 2 * (X * s - dl)); };
        auto hi = [&](int X) { return std::min(2 * n, 2 * ((X + 1) * s + dl)); };
        if (spec.local_dirichlet) {
          // leave out the faces of the grown box that lie inside the cube
          auto lo_d = [&](int X) { return lo(X) > 0 ? lo(X) + 1 : 0; };
          auto hi_d = [&](int X) { return hi(X) < 2 * n ? hi(X) - 1 : 2 * n; };
          collect_box(lo_d(I), hi_d(I), lo_d(J), hi_d(J), lo_d(K), hi_d(K), P.S[i]);
        } else {
          collect_box(lo(I), hi(I), lo(J), hi(J), lo(K), hi(K), P.S[i]);
        }
        collect_box(2 * I * s, 2 * (I + 1) * s, 2 * J * s, 2 * (J + 1) * s, 2 * K * s, 2 * (K + 1) * s, P.D[i]);
        P.I[i].clear();
        for (int32_t d : P.D[i])
          if (P.multiplicity[d] == 1) P.I[i].push_back(d);
      }

  // ---- interface entities -----------------------------------------------
  std::map<std::array<int32_t, 6>, int> ent_of;
  std::vector<int64_t> ent_min;
  std::vector<int32_t> ent_tmp(P.n_free, -1);
  for (int64_t d = 0; d < P.n_free; ++d) {
    if (P.multiplicity[d] < 2) continue;
    auto it = ent_of.find(key[d]);
    int e;
    if (it == ent_of.end()) {
      e = (int)ent_min.size();
      ent_of.emplace(key[d], e);
      ent_min.push_back(INT64_MAX);
    } else {
      e = it->second;
    }
    ent_tmp[d] = e;
    const int64_t q2id = P.abc[3 * d] + (int64_t)N2 * (P.abc[3 * d + 1] + (int64_t)N2 * P.abc[3 * d + 2]);
    ent_min[e] = std::min(ent_min[e], q2id);
  }
  const int n_cls = (int)ent_min.size();
  std::vector<int> order(n_cls);
  for (int e = 0; e < n_cls; ++e) order[e] = e;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return ent_min[x] < ent_min[y]; });
  std::vector<int> rank(n_cls);
  for (int r = 0; r < n_cls; ++r) rank[order[r]] = r;
  std::vector<std::array<int32_t, 6>> cls_key(n_cls);
  for (auto& kv : ent_of) cls_key[rank[kv.second]] = kv.first;
  // entity of each class (by class rank): itself, or with GDSW* the first
  // adjacent vertex class (in node order) whose subdomain box contains it
  std::vector<int> target(n_cls);
  for (int r = 0; r < n_cls; ++r) target[r] = r;
  if (spec.coarse == 1) {
    auto size_of = [](const std::array<int32_t, 6>& k) {
      return (k[3] - k[0] + 1) * (k[4] - k[1] + 1) * (k[5] - k[2] + 1);
    };
    std::vector<int> verts;
    for (int r = 0; r < n_cls; ++r)
      if (size_of(cls_key[r]) == 8) verts.push_back(r);
    for (int r = 0; r < n_cls; ++r) {
      if (size_of(cls_key[r]) != 4) continue;
      const auto& ke = cls_key[r];
      for (int v : verts) {
        const auto& kv = cls_key[v];
        if (kv[0] <= ke[0] && kv[1] <= ke[1] && kv[2] <= ke[2] && ke[3] <= kv[3] && ke[4] <= kv[4] && ke[5] <= kv[5]) {
          target[r] = v;
          break;
        }
      }
    }
  }
  // entities: the distinct targets, ordered by the smallest node id of their merged classes
  std::vector<int64_t> grp_min(n_cls, INT64_MAX);
  for (int r = 0; r < n_cls; ++r) grp_min[target[r]] = std::min(grp_min[target[r]], ent_min[order[r]]);
  std::vector<int> groups;
  for (int r = 0; r < n_cls; ++r)
    if (target[r] == r) groups.push_back(r);
  std::stable_sort(groups.begin(), groups.end(), [&](int x, int y) { return grp_min[x] < grp_min[y]; });
  std::vector<int> ent_of_grp(n_cls, -1);
  for (size_t q = 0; q < groups.size(); ++q) ent_of_grp[groups[q]] = (int)q;
  P.n_ent = (int)groups.size();
  P.ent_key.assign(P.n_ent, {});
  for (int q = 0; q < P.n_ent; ++q) P.ent_key[q] = cls_key[groups[q]];
  auto entity_of = [&](int64_t d) { return ent_of_grp[target[rank[ent_tmp[d]]]]; };
  std::vector<std::array<int, 4>> has(P.n_ent, {0, 0, 0, 0});
  for (int64_t d = 0; d < P.n_free; ++d)
    if (ent_tmp[d] >= 0) has[entity_of(d)][P.field[d]] = 1;
  std::vector<std::array<int32_t, 4>> colof(P.n_ent, {-1, -1, -1, -1});
  P.coarse_entity.clear();
  P.coarse_field.clear();
  for (int e = 0; e < P.n_ent; ++e)
    for (int f = 0; f < 4; ++f)
      if (has[e][f]) {
        colof[e][f] = (int32_t)P.coarse_entity.size();
        P.coarse_entity.push_back(e);
        P.coarse_field.push_back(f);
      }
  P.gamma_col.assign(P.n_free, -1);
  for (int64_t d = 0; d < P.n_free; ++d)
    if (ent_tmp[d] >= 0) P.gamma_col[d] = colof[entity_of(d)][P.field[d]];
  P.C.assign(P.n_sub, {});
  for (int e = 0; e < P.n_ent; ++e)
    for (int32_t i : entity_subdomains(P, e))
      for (int f = 0; f < 4; ++f)
        if (colof[e][f] >= 0) P.C[i].push_back(colof[e][f]);
  // discontinuous pressure: no pressure interface; one pressure column per
  // subdomain, constant over it, after the interface columns (Section 3)
  P.sub_pcol.clear();
  if (disc && P.n_sub > 1) {
    for (int K = 0; K < m; ++K)
      for (int J = 0; J < m; ++J)
        for (int I = 0; I < m; ++I) {
          const int i = I + m * (J + m * K);
          P.ent_key.push_back({I, J, K, I, J, K});
          P.sub_pcol.push_back((int32_t)P.coarse_entity.size());
          P.coarse_entity.push_back(P.n_ent + i);
          P.coarse_field.push_back(3);
          P.C[i].push_back(P.sub_pcol.back());
        }
  }
  P.n_coarse = (int)P.coarse_entity.size();
  for (auto& Ci : P.C) std::sort(Ci.begin(), Ci.end());

  // ---- three-level bookkeeping (eq. 2.5) ---------------------------------
  if (spec.levels == 3) {
    Level2& L = P.lv2;
    const int g = spec.group, Ms = m / g;
    L.n_sub = Ms * Ms * Ms;
    const int Nc = P.n_coarse;
    // subregion box of each coarse DOF (its entity's subdomains grouped)
    std::vector<std::array<int32_t, 6>> rkey(Nc);
    for (int c = 0; c < Nc; ++c) {
      const auto& k = P.ent_key[P.coarse_entity[c]];
      for (int ax = 0; ax < 3; ++ax) {
        rkey[c][ax] = k[ax] / g;
        rkey[c][3 + ax] = k[3 + ax] / g;
      }
    }
    auto in_box = [](const std::array<int32_t, 6>& k, int X, int Y, int Z) {
      return k[0] <= X && X <= k[3] && k[1] <= Y && Y <= k[4] && k[2] <= Z && Z <= k[5];
    };
    L.S.assign(L.n_sub, {});
    L.I.assign(L.n_sub, {});
    for (int Z = 0; Z < Ms; ++Z)
      for (int Y = 0; Y < Ms; ++Y)
        for (int X = 0; X < Ms; ++X) {
          const int j = X + Ms * (Y + Ms * Z);
          std::vector<char> touched(P.n_sub, 0);
          for (int c = 0; c < Nc; ++c)
            if (in_box(rkey[c], X, Y, Z))
              for (int32_t i : entity_subdomains(P, P.coarse_entity[c])) touched[i] = 1;
          for (int c = 0; c < Nc; ++c) {
            bool hit = false;
            if (spec.level2_layer) {
              for (int32_t i : entity_subdomains(P, P.coarse_entity[c]))
                if (touched[i]) { hit = true; break; }
            } else {
              hit = in_box(rkey[c], X, Y, Z);
            }
            if (hit) L.S[j].push_back(c);
            const auto& k = rkey[c];
            if (k[0] == X && k[3] == X && k[1] == Y && k[4] == Y && k[2] == Z && k[5] == Z) L.I[j].push_back(c);
          }
        }
    // level-3 classes: coarse DOFs in >= 2 subregions, by subregion box
    std::map<std::array<int32_t, 6>, int> cls;
    std::vector<int> cls_min;
    std::vector<int> ctmp(Nc, -1);
    for (int c = 0; c < Nc; ++c) {
      const auto& k = rkey[c];
      const int cnt = (k[3] - k[0] + 1) * (k[4] - k[1] + 1) * (k[5] - k[2] + 1);
      if (cnt < 2) continue;
      auto it = cls.find(k);
      int e;
      if (it == cls.end()) {
        e = (int)cls_min.size();
        cls.emplace(k, e);
        cls_min.push_back(c);
      } else {
        e = it->second;
      }
      ctmp[c] = e;
    }
    L.n_ent3 = (int)cls_min.size();
    std::vector<int> ord(L.n_ent3);
    for (int e = 0; e < L.n_ent3; ++e) ord[e] = e;
    std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return cls_min[x] < cls_min[y]; });
    std::vector<int> rk(L.n_ent3);
    for (int r = 0; r < L.n_ent3; ++r) rk[ord[r]] = r;
    std::vector<std::array<int, 4>> has3(L.n_ent3, {0, 0, 0, 0});
    for (int c = 0; c < Nc; ++c)
      if (ctmp[c] >= 0) has3[rk[ctmp[c]]][P.coarse_field[c]] = 1;
    std::vector<std::array<int32_t, 4>> col3(L.n_ent3, {-1, -1, -1, -1});
    std::vector<std::array<int32_t, 6>> ckey(L.n_ent3);
    for (auto& kv : cls) ckey[rk[kv.second]] = kv.first;
    int nc3 = 0;
    for (int e = 0; e < L.n_ent3; ++e)
      for (int f = 0; f < 4; ++f)
        if (has3[e][f]) col3[e][f] = nc3++;
    L.n_coarse3 = nc3;
    L.gamma_col3.assign(Nc, -1);
    for (int c = 0; c < Nc; ++c)
      if (ctmp[c] >= 0) L.gamma_col3[c] = col3[rk[ctmp[c]]][P.coarse_field[c]];
    L.C.assign(L.n_sub, {});
    for (int e = 0; e < L.n_ent3; ++e)
      for (int Z = ckey[e][2]; Z <= ckey[e][5]; ++Z)
        for (int Y = ckey[e][1]; Y <= ckey[e][4]; ++Y)
          for (int X = ckey[e][0]; X <= ckey[e][3]; ++X)
            for (int f = 0; f < 4; ++f)
              if (col3[e][f] >= 0) L.C[X + Ms * (Y + Ms * Z)].push_back(col3[e][f]);
    for (auto& Cj : L.C) std::sort(Cj.begin(), Cj.end());
  }
}

}  // namespace gdsw
