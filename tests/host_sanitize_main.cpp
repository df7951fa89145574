// Host-side set-up code (numbering, assembly, decomposition, interface
// entities, subregions, the algebraic entry point's sets) under the address
// and undefined-behaviour sanitizers: builds structured problems of every
// kind and the algebraic problem of each from its own matrix and closed
// boxes, and checks that bad input is rejected with std::invalid_argument.
// Built and run by tests/test_host_sanitizers.py.
#include <cstdio>
#include <stdexcept>
#include <vector>

#include "problem.h"

using namespace gdsw;

static int fails = 0;

static void check(bool ok, const char* what, int k) {
  if (!ok) {
    std::printf("FAIL case %d: %s\n", k, what);
    ++fails;
  }
}

int main() {
  struct Case {
    int n, m, overlap, levels, group, local_dirichlet, level2_layer, pressure, coarse;
  };
  const Case cases[] = {
      {4, 2, 1, 2, 2, 1, 0, 0, 0}, {6, 3, 2, 2, 1, 0, 0, 0, 0}, {8, 4, 1, 3, 2, 1, 1, 0, 0},
      {6, 3, 1, 2, 1, 0, 0, 1, 1}, {4, 1, 1, 2, 1, 1, 0, 0, 0}, {6, 2, 1, 2, 1, 0, 0, 1, 0},
  };
  int k = 0;
  for (const Case& c : cases) {
    ProblemSpec sp;
    sp.n = c.n;
    sp.m = c.m;
    sp.overlap = c.overlap;
    sp.levels = c.levels;
    sp.group = c.group;
    sp.local_dirichlet = c.local_dirichlet;
    sp.level2_layer = c.level2_layer;
    sp.pressure = c.pressure;
    sp.coarse = c.coarse;
    Problem P;
    build_problem(sp, P, 2);
    check((int64_t)P.field.size() == P.n_free && (int64_t)P.row_ptr.size() == P.n_free + 1, "sizes", k);
    check(P.n_sub == c.m * c.m * c.m && (int)P.S.size() == P.n_sub, "subdomains", k);
    // the algebraic problem from the same matrix and the closed boxes
    if (c.levels == 2) {
      std::vector<std::vector<int32_t>> subs(P.n_free);
      for (int i = 0; i < P.n_sub; ++i)
        for (int32_t d : P.D[i]) subs[d].push_back(i);
      std::vector<int64_t> rp(P.row_ptr.begin(), P.row_ptr.end()), sp_ptr(1, 0);
      std::vector<int32_t> fld(P.field.begin(), P.field.end()), sidx;
      std::vector<double> nul(P.n_free, 1.0);
      for (auto& s : subs) {
        sidx.insert(sidx.end(), s.begin(), s.end());
        sp_ptr.push_back((int64_t)sidx.size());
      }
      AlgebraicInput in;
      in.n = P.n_free;
      in.row_ptr = rp.data();
      in.col = P.col.data();
      in.val = P.val.data();
      in.rhs = P.rhs.data();
      in.field = fld.data();
      in.null_value = nul.data();
      in.n_sub = P.n_sub;
      in.sub_ptr = sp_ptr.data();
      in.sub_idx = sidx.data();
      ProblemSpec sa;
      sa.overlap = c.overlap;
      Problem Q;
      build_problem_algebraic(in, sa, Q);
      check(Q.n_free == P.n_free && Q.n_sub == P.n_sub && (Q.n_coarse > 0) == (P.n_coarse > 0), "algebraic sizes", k);
      // a subdomain index out of range must be rejected
      std::vector<int32_t> bad = sidx;
      bad[0] = P.n_sub;
      in.sub_idx = bad.data();
      bool threw = false;
      try {
        Problem R;
        build_problem_algebraic(in, sa, R);
      } catch (const std::invalid_argument&) {
        threw = true;
      }
      check(threw, "out-of-range subdomain rejected", k);
    }
    std::printf("case %d: n=%d m=%d n_free=%lld n_coarse=%d\n", k, c.n, c.m, (long long)P.n_free, P.n_coarse);
    ++k;
  }
  {
    ProblemSpec sp;
    sp.n = 5;
    sp.m = 2;  // n % m != 0
    bool threw = false;
    try {
      Problem P;
      build_problem(sp, P, 1);
    } catch (const std::invalid_argument&) {
      threw = true;
    }
    check(threw, "n % m rejected", -1);
  }
  std::printf("%s\n", fails ? "FAILED" : "OK");
  return fails ? 1 : 0;
}
