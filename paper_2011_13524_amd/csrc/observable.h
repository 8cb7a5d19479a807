// Observables: real combinations of Pauli strings (section 4.5), stored as
// flip masks (X/Y qubits), sign masks (Z/Y qubits) and the number of Y factors.
#pragma once

#include <vector>

#include "qsv_internal.h"

namespace qsv {
struct ExpPlan;
void free_exp_plan(ExpPlan* p);
}  // namespace qsv

struct qsv_observable {
  int n = 0;
  struct Term {
    double coef;
    uint64_t flip, zmask;
    int ny;
  };
  std::vector<Term> terms;
  // tiled evaluation plans per dtype (built on first use, dropped on change)
  qsv::ExpPlan* exp_plan[3] = {nullptr, nullptr, nullptr};

  qsv_observable() = default;
  qsv_observable(const qsv_observable& o) : n(o.n), terms(o.terms) {}
  qsv_observable& operator=(const qsv_observable& o) {
    if (this != &o) {
      drop_plans();
      n = o.n;
      terms = o.terms;
    }
    return *this;
  }
  ~qsv_observable() { drop_plans(); }
  void drop_plans() {
    for (auto*& p : exp_plan) {
      if (p) qsv::free_exp_plan(p);
      p = nullptr;
    }
  }
};

namespace qsv {

// A term as the kernels use it: alpha * i^nY as a complex number and the
// sign mask. P[x ^ flip, x] = i^nY (-1)^popcount(x & z).
struct GTerm {
  double re, im;
  uint64_t z;
};

struct Group {
  uint64_t flip;
  int begin, count;
};

// Terms grouped by flip mask (ascending flip), ready for upload.
void build_groups(const qsv_observable* o, std::vector<Group>& groups, std::vector<GTerm>& terms);

}  // namespace qsv
