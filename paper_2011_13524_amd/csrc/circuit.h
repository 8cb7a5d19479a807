// Host-side circuit representation (section 4.4, QuantumCircuit and
// ParametricQuantumCircuit): an ordered list of basic gates, some of them
// rotations whose angle is read from a parameter vector at apply time.
#pragma once

#include <vector>

#include "qsv_internal.h"

namespace qsv {

struct Gate {
  enum Kind { MATRIX = 0, ROTATION = 1, PAULI = 2 };
  int kind = MATRIX;
  std::vector<int> targets;
  std::vector<int> controls;
  std::vector<int> ctrl_vals;
  std::vector<cd> mat;  // MATRIX: 2^k x 2^k, row-major
  // ROTATION: exp(+i angle P / 2), P = Pauli pauli (1..3) on targets[0];
  // angle = theta[slot] if slot >= 0 else fixed_angle.
  int pauli = 0;
  int slot = -1;
  double fixed_angle = 0.0;
  // PAULI: exp(+i angle P / 2) for the Pauli string paulis[j] (1..3) on
  // targets[j] (identity factors dropped); angle as for ROTATION
  std::vector<int> paulis;
};

// psi <- exp(+i t P / 2) psi for a Pauli string (ids 0..3 on distinct qubits).
int pauli_rotation_impl(qsv_state* s, const int* qubits, const int* ids, int w, double t);

// Reverse-sweep step of a parametric PAULI gate at angle t: B partials of its
// gradient -Im<lam|P|psi> into partial_row (grid of B workgroups), then psi
// and lam uncomputed.
int adjoint_pauli_step(qsv_state* psi, qsv_state* lam, const Gate& g, double t, double* partial_row, int B);

// Gate matrix of a gate for the given parameters (row-major, 2^k x 2^k).
void gate_matrix(const Gate& g, const double* theta, std::vector<cd>& out);

// Rotation matrix exp(+i t P / 2) for Pauli id p (table of named gates).
void rotation_matrix(int pauli, double t, cd* m);

}  // namespace qsv

struct qsv_circuit {
  int n = 0;
  int nparams = 0;  // 1 + largest slot used
  std::vector<qsv::Gate> gates;
};
