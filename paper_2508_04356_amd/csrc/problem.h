// Host-side description of one Stokes problem and its decomposition.
//
// Everything here is integer bookkeeping plus the finite-element assembly of
// eq. (2.1); it runs once per problem (the paper's "symbolic setup", Section
// 3) and is uploaded to the device by the context.
#pragma once

#include <array>
#include <cstdint>
#include <memory>
#include <new>
#include <string>
#include <type_traits>
#include <utility>
#include <vector>

namespace gdsw {

// An allocator whose value-initialisation leaves the elements uninitialised,
// so that resize() of a large array does not touch its pages: the matrix
// assembly threads write (and first touch) every entry themselves.
template <class T>
struct NoInitAlloc : std::allocator<T> {
  template <class U>
  struct rebind {
    using other = NoInitAlloc<U>;
  };
  NoInitAlloc() = default;
  template <class U>
  NoInitAlloc(const NoInitAlloc<U>&) noexcept {}
  template <class U>
  void construct(U* p) noexcept(std::is_nothrow_default_constructible<U>::value) {
    ::new (static_cast<void*>(p)) U;
  }
  template <class U, class... Args>
  void construct(U* p, Args&&... args) {
    ::new (static_cast<void*>(p)) U(std::forward<Args>(args)...);
  }
};
template <class T>
using bulk_vector = std::vector<T, NoInitAlloc<T>>;

struct ProblemSpec {
  int n = 4;            // elements per axis
  int m = 2;            // subdomains per axis
  int overlap = 1;      // element layers
  int levels = 2;
  int group = 2;        // three levels: subdomains per subregion per axis
  double mu = 1.0;
  double c = 16.0;
  int manufactured = 0;
  int local_dirichlet = 1;  // 1: drop the artificial boundary of the grown box
  int level2_layer = 0;     // 1: level-2 local sets get one more A_0-graph layer
  int pressure = 0;         // 0: Q1 (continuous); 1: P1disc (4 DOFs per hexahedron)
  int coarse = 0;           // 0: full GDSW entities; 1: GDSW* (vertex + adjacent edges)
};

// Level-2 (coarse) structures for the three-level method (eq. 2.5).
struct Level2 {
  int n_sub = 0;                               // subregions N^(2)
  std::vector<std::vector<int32_t>> S;         // overlapping coarse index sets
  std::vector<std::vector<int32_t>> I;         // interior coarse DOFs per subregion
  int n_ent3 = 0;
  int n_coarse3 = 0;
  std::vector<int32_t> gamma_col3;             // per level-2 coarse DOF: level-3 column or -1
  std::vector<std::vector<int32_t>> C;         // level-3 columns adjacent to each subregion
};

struct Problem {
  ProblemSpec spec;
  int s = 0;                                   // elements per subdomain per axis
  int64_t n_u = 0, n_p = 0, n_free = 0, n_full = 0;

  // free-DOF CSR matrix (sorted columns) and lifted right-hand side
  std::vector<int32_t> row_ptr;
  bulk_vector<int32_t> col;
  bulk_vector<double> val;
  std::vector<double> rhs;

  // per free DOF
  std::vector<int8_t> field;                   // 0..2 velocity, 3 pressure
  std::vector<int32_t> abc;                    // Q2 node coordinates (3 per DOF)
  std::vector<int64_t> full_index;             // position in the full vector
  std::vector<double> dirichlet_full;          // full vector of Dirichlet data (0 on free)

  // decomposition
  int n_sub = 0;
  std::vector<std::vector<int32_t>> S;         // overlapping sets (sorted)
  std::vector<std::vector<int32_t>> D;         // closed boxes (sorted)
  std::vector<std::vector<int32_t>> I;         // interiors (sorted)
  std::vector<int8_t> multiplicity;            // closed boxes holding each DOF

  // interface entities and coarse columns
  int n_ent = 0;                               // interface entities
  std::vector<std::array<int32_t, 6>> ent_key; // lo_x, lo_y, lo_z, hi_x, hi_y, hi_z; with a
                                               // discontinuous pressure, n_sub more keys
                                               // (i, i): the subdomains' pressure constants
  std::vector<int32_t> sub_pcol;               // discontinuous pressure: pressure column of
                                               // each subdomain (constant over it), else empty
  std::vector<int8_t> pnull;                   // per DOF: 1 where the field's null-space
                                               // vector is 1 (0 on linear P1disc functions)
  std::vector<int32_t> gamma_col;              // per DOF: coarse column or -1
  int n_coarse = 0;
  std::vector<int32_t> coarse_entity, coarse_field;
  std::vector<std::vector<int32_t>> C;         // coarse columns adjacent to each subdomain

  Level2 lv2;

  // algebraic problems (an assembled matrix and the subdomains of each DOF)
  bool algebraic = false;
  std::vector<int64_t> sub_ptr;                // DOF d is held by sub_idx[sub_ptr[d] .. sub_ptr[d+1])
  std::vector<int32_t> sub_idx;
  std::vector<std::vector<int32_t>> ent_sets;  // subdomain set of each interface entity

  int64_t nnz() const { return (int64_t)col.size(); }
};

// Host input of the algebraic entry point (see gdsw_algebraic_problem).
struct AlgebraicInput {
  int64_t n = 0;
  const int64_t* row_ptr = nullptr;
  const int32_t* col = nullptr;
  const double* val = nullptr;
  const double* rhs = nullptr;
  const int32_t* field = nullptr;
  const double* null_value = nullptr;
  int32_t n_sub = 0;
  const int64_t* sub_ptr = nullptr;
  const int32_t* sub_idx = nullptr;
};

// Builds the problem description from an assembled matrix and the
// subdomains holding each DOF (two levels, full GDSW).  Throws
// std::invalid_argument on inconsistent input.
void build_problem_algebraic(const AlgebraicInput& in, const ProblemSpec& spec, Problem& P);

// Builds everything above.  Throws std::invalid_argument on a bad spec.
void build_problem(const ProblemSpec& spec, Problem& P, int threads);

// Subdomains (ascending) that contain coarse column c's entity.
std::vector<int32_t> entity_subdomains(const Problem& P, int e);

}  // namespace gdsw
