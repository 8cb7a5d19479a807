// Observables: real combinations of Pauli strings (section 4.5), stored as
// flip masks (X/Y qubits), sign masks (Z/Y qubits) and the number of Y factors.
#pragma once

#include <vector>

#include "qsv_internal.h"

struct qsv_observable {
  int n = 0;
  struct Term {
    double coef;
    uint64_t flip, zmask;
    int ny;
  };
  std::vector<Term> terms;
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
