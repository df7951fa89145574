// Problem description from an assembled matrix and the distribution of its
// DOFs over the subdomains (Section 3: the implementation needs only which
// subdomains hold each velocity and pressure DOF).  Everything the
// structured cube derives from node coordinates is derived here from the
// subdomain sets of the DOFs and the matrix graph:
//
//   D_i   = DOFs held by subdomain i (closure of the non-overlapping part),
//   Gamma = DOFs held by at least two subdomains, I_i = D_i \ Gamma,
//   S_i   = D_i grown by `overlap` layers of the matrix graph,
//   entities = classes of Gamma DOFs with the same subdomain set, ordered by
//   their smallest DOF index, one coarse column per (entity, field present);
//   a field with DOFs but none on Gamma (a discontinuous pressure) gets one
//   column per subdomain, its null-space values on the subdomain's DOFs.
#include <algorithm>
#include <map>
#include <stdexcept>
#include <string>

#include "problem.h"

namespace gdsw {

void build_problem_algebraic(const AlgebraicInput& in, const ProblemSpec& spec_in, Problem& P) {
  const int64_t n = in.n;
  if (n < 1) throw std::invalid_argument("need n >= 1");
  if (!in.row_ptr || !in.col || !in.val || !in.field || !in.sub_ptr || !in.sub_idx)
    throw std::invalid_argument("row_ptr, col, val, field, sub_ptr and sub_idx must not be NULL");
  if (in.n_sub < 1) throw std::invalid_argument("need n_sub >= 1");
  if (spec_in.overlap < 1) throw std::invalid_argument("overlap must be >= 1");
  if (spec_in.levels != 2) throw std::invalid_argument("the algebraic entry point builds two levels");
  if (spec_in.coarse != 0) throw std::invalid_argument("the algebraic entry point builds the full GDSW space");
  const int64_t nnz = in.row_ptr[n];
  if (in.row_ptr[0] != 0 || nnz < 0 || nnz > INT32_MAX) throw std::invalid_argument("bad row_ptr (nnz must fit int32)");
  P = Problem();
  P.spec = spec_in;
  P.spec.n = 0;
  P.spec.m = 0;
  P.algebraic = true;
  P.n_free = P.n_full = n;
  P.n_sub = in.n_sub;

  // ---- matrix, fields, numbering ----------------------------------------
  P.row_ptr.resize(n + 1);
  for (int64_t r = 0; r <= n; ++r) {
    if (r > 0 && in.row_ptr[r] < in.row_ptr[r - 1]) throw std::invalid_argument("row_ptr must not decrease");
    P.row_ptr[r] = (int32_t)in.row_ptr[r];
  }
  P.col.assign(in.col, in.col + nnz);
  P.val.assign(in.val, in.val + nnz);
  for (int64_t r = 0; r < n; ++r)
    for (int64_t e = in.row_ptr[r]; e < in.row_ptr[r + 1]; ++e) {
      if (in.col[e] < 0 || in.col[e] >= n) throw std::invalid_argument("column index out of range");
      if (e > in.row_ptr[r] && in.col[e] <= in.col[e - 1])
        throw std::invalid_argument("columns must be sorted and distinct within each row");
    }
  P.rhs.assign(n, 0.0);
  if (in.rhs) P.rhs.assign(in.rhs, in.rhs + n);
  P.field.resize(n);
  P.pnull.assign(n, 1);
  P.abc.assign(3 * n, 0);
  P.full_index.resize(n);
  P.dirichlet_full.assign(n, 0.0);
  P.n_u = 0;
  for (int64_t d = 0; d < n; ++d) {
    const int32_t f = in.field[d];
    if (f < 0 || f > 3) throw std::invalid_argument("field must be 0, 1, 2 (velocity) or 3 (pressure)");
    if (d > 0 && f < 3 && P.field[d - 1] == 3)
      throw std::invalid_argument("number every velocity DOF before the pressure DOFs");
    P.field[d] = (int8_t)f;
    P.n_u += f < 3;
    P.full_index[d] = d;
    if (in.null_value) {
      const double v = in.null_value[d];
      if (v != 0.0 && v != 1.0) throw std::invalid_argument("null-space values must be 0 or 1");
      P.pnull[d] = v == 1.0;
    }
  }
  P.n_p = n - P.n_u;

  // ---- subdomain sets ----------------------------------------------------
  P.sub_ptr.assign(in.sub_ptr, in.sub_ptr + n + 1);
  P.sub_idx.assign(in.sub_idx, in.sub_idx + in.sub_ptr[n]);
  P.multiplicity.assign(n, 0);
  P.D.assign(P.n_sub, {});
  for (int64_t d = 0; d < n; ++d) {
    const int64_t b = in.sub_ptr[d], e = in.sub_ptr[d + 1];
    if (e <= b) throw std::invalid_argument("DOF " + std::to_string(d) + " belongs to no subdomain");
    for (int64_t k = b; k < e; ++k) {
      const int32_t i = in.sub_idx[k];
      if (i < 0 || i >= P.n_sub) throw std::invalid_argument("subdomain index out of range");
      if (k > b && i <= in.sub_idx[k - 1]) throw std::invalid_argument("subdomain lists must be sorted and distinct");
      P.D[i].push_back((int32_t)d);
    }
    P.multiplicity[d] = (int8_t)std::min<int64_t>(e - b, 127);
  }
  // every nonzero must couple DOFs of a common subdomain: A_0 is assembled
  // from the nonzeros each subdomain owns (the lowest one holding both DOFs)
  for (int64_t r = 0; r < n; ++r)
    for (int64_t e = in.row_ptr[r]; e < in.row_ptr[r + 1]; ++e) {
      const int32_t c = in.col[e];
      int64_t a = in.sub_ptr[r], ae = in.sub_ptr[r + 1], b = in.sub_ptr[c], be = in.sub_ptr[c + 1];
      while (a < ae && b < be && in.sub_idx[a] != in.sub_idx[b]) {
        if (in.sub_idx[a] < in.sub_idx[b]) ++a; else ++b;
      }
      if (a == ae || b == be)
        throw std::invalid_argument("matrix entry (" + std::to_string(r) + ", " + std::to_string(c) +
                                    ") couples DOFs that share no subdomain");
    }
  P.I.assign(P.n_sub, {});
  for (int i = 0; i < P.n_sub; ++i) {
    if (P.D[i].empty()) throw std::invalid_argument("subdomain " + std::to_string(i) + " holds no DOF");
    for (int32_t d : P.D[i])
      if (P.multiplicity[d] == 1) P.I[i].push_back(d);
  }
  // overlap: graph layers of the matrix around each D_i
  P.S.assign(P.n_sub, {});
  std::vector<char> mark(n, 0);
  for (int i = 0; i < P.n_sub; ++i) {
    std::vector<int32_t> cur = P.D[i];
    for (int32_t d : cur) mark[d] = 1;
    std::vector<int32_t> all = cur;
    for (int l = 0; l < spec_in.overlap; ++l) {
      std::vector<int32_t> next;
      for (int32_t r : cur)
        for (int32_t e = P.row_ptr[r]; e < P.row_ptr[r + 1]; ++e)
          if (!mark[P.col[e]]) {
            mark[P.col[e]] = 1;
            next.push_back(P.col[e]);
          }
      all.insert(all.end(), next.begin(), next.end());
      cur.swap(next);
    }
    for (int32_t d : all) mark[d] = 0;
    std::sort(all.begin(), all.end());
    P.S[i] = std::move(all);
  }

  // ---- entities and coarse columns --------------------------------------
  std::map<std::vector<int32_t>, int> cls;
  std::vector<std::vector<int32_t>> cls_sets;
  std::vector<int32_t> ent(n, -1);
  for (int64_t d = 0; d < n; ++d) {  // ascending d: classes in order of their smallest DOF
    if (P.multiplicity[d] < 2) continue;
    std::vector<int32_t> key(in.sub_idx + in.sub_ptr[d], in.sub_idx + in.sub_ptr[d + 1]);
    auto it = cls.find(key);
    if (it == cls.end()) {
      it = cls.emplace(key, (int)cls_sets.size()).first;
      cls_sets.push_back(key);
    }
    ent[d] = it->second;
  }
  P.n_ent = (int)cls_sets.size();
  std::vector<std::array<int, 4>> has(P.n_ent, {0, 0, 0, 0});
  for (int64_t d = 0; d < n; ++d)
    if (ent[d] >= 0) has[ent[d]][P.field[d]] = 1;
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
  P.gamma_col.assign(n, -1);
  for (int64_t d = 0; d < n; ++d)
    if (ent[d] >= 0) P.gamma_col[d] = colof[ent[d]][P.field[d]];
  P.C.assign(P.n_sub, {});
  for (int e = 0; e < P.n_ent; ++e)
    for (int32_t i : cls_sets[e])
      for (int f = 0; f < 4; ++f)
        if (colof[e][f] >= 0) P.C[i].push_back(colof[e][f]);
  bool p_on_gamma = false;
  for (int64_t d = 0; d < n; ++d) p_on_gamma = p_on_gamma || (P.field[d] == 3 && ent[d] >= 0);
  P.sub_pcol.clear();
  if (P.n_p > 0 && !p_on_gamma && P.n_sub > 1)
    for (int i = 0; i < P.n_sub; ++i) {
      P.sub_pcol.push_back((int32_t)P.coarse_entity.size());
      P.coarse_entity.push_back(P.n_ent + i);
      P.coarse_field.push_back(3);
      P.C[i].push_back(P.sub_pcol.back());
    }
  P.n_coarse = (int)P.coarse_entity.size();
  for (auto& Ci : P.C) std::sort(Ci.begin(), Ci.end());
  P.ent_sets = std::move(cls_sets);
}

}  // namespace gdsw
