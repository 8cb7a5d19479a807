// Circuits (section 4.4): building, and unfused application gate by gate.
#include <cmath>

#include "circuit.h"

namespace qsv {

int validate_gate(int n, const int* targets, int k, const int* controls, const int* ctrl_vals,
                  int nc, int kmax);

void rotation_matrix(int pauli, double t, cd* m) {
  // exp(i t P/2) = cos(t/2) I + i sin(t/2) P
  const double c = std::cos(t / 2), s = std::sin(t / 2);
  switch (pauli) {
    case 1: m[0] = {c, 0}; m[1] = {0, s}; m[2] = {0, s}; m[3] = {c, 0}; break;
    case 2: m[0] = {c, 0}; m[1] = {s, 0}; m[2] = {-s, 0}; m[3] = {c, 0}; break;
    default: m[0] = {c, s}; m[1] = {0, 0}; m[2] = {0, 0}; m[3] = {c, -s}; break;
  }
}

void gate_matrix(const Gate& g, const double* theta, std::vector<cd>& out) {
  if (g.kind == Gate::ROTATION) {
    out.resize(4);
    const double t = g.slot >= 0 ? theta[g.slot] : g.fixed_angle;
    rotation_matrix(g.pauli, t, out.data());
  } else if (g.kind == Gate::PAULI) {
    // c I + i s P on the targets (matrix index bit j <-> targets[j]); one
    // nonzero of P per column: row r = col ^ F, value prod_j sigma_j[r_j][c_j]
    const int w = int(g.targets.size());
    const int D = 1 << w;
    const double t = g.slot >= 0 ? theta[g.slot] : g.fixed_angle;
    const double c = std::cos(t / 2), s = std::sin(t / 2);
    out.assign(size_t(D) * D, cd{0, 0});
    int F = 0;
    for (int j = 0; j < w; ++j)
      if (g.paulis[j] == 1 || g.paulis[j] == 2) F |= 1 << j;
    for (int col = 0; col < D; ++col) {
      const int row = col ^ F;
      cd v{1, 0};
      for (int j = 0; j < w; ++j) {
        const int rb = (row >> j) & 1;
        if (g.paulis[j] == 2) v = cmul(v, rb ? cd{0, 1} : cd{0, -1});  // Y[r][c], c = 1 - r
        else if (g.paulis[j] == 3 && rb) v = {-v.re, -v.im};           // Z[r][r]
      }
      out[size_t(row) * D + col] = cadd(out[size_t(row) * D + col], cmul(cd{0, s}, v));
      out[size_t(col) * D + col] = cadd(out[size_t(col) * D + col], cd{c, 0});
    }
  } else {
    out = g.mat;
  }
}

int circuit_apply_unfused(qsv_state* s, const qsv_circuit* c, const double* theta) {
  std::vector<cd> m;
  for (const Gate& g : c->gates) {
    if (g.kind == Gate::PAULI) {
      const double t = g.slot >= 0 ? theta[g.slot] : g.fixed_angle;
      int rc = pauli_rotation_impl(s, g.targets.data(), g.paulis.data(), int(g.targets.size()), t);
      if (rc) return rc;
      continue;
    }
    gate_matrix(g, theta, m);
    int rc = apply_gate_impl(s, m.data(), g.targets.data(), int(g.targets.size()),
                             g.controls.data(), g.ctrl_vals.data(), int(g.controls.size()));
    if (rc) return rc;
  }
  return QSV_OK;
}

}  // namespace qsv

using namespace qsv;

extern "C" {

int qsv_circuit_create(int n, qsv_circuit** out) {
  clear_error();
  if (!out) return fail(QSV_EINVAL, "null output handle");
  *out = nullptr;
  if (n < 1 || n > 34) return fail(QSV_ERANGE, "qubit count %d outside [1, 34]", n);
  qsv_circuit* c = new (std::nothrow) qsv_circuit();
  if (!c) return fail(QSV_ENOMEM, "host allocation failed");
  c->n = n;
  *out = c;
  return QSV_OK;
}

int qsv_circuit_free(qsv_circuit* c) {
  clear_error();
  delete c;
  return QSV_OK;
}

int qsv_circuit_add_gate(qsv_circuit* c, const double* mat, const int* targets, int k,
                         const int* controls, const int* ctrl_vals, int nc) {
  clear_error();
  if (!c) return fail(QSV_EINVAL, "null circuit");
  if (!mat) return fail(QSV_EINVAL, "null matrix");
  int rc = validate_gate(c->n, targets, k, controls, ctrl_vals, nc, 5);
  if (rc) return rc;
  Gate g;
  g.kind = Gate::MATRIX;
  g.targets.assign(targets, targets + k);
  if (nc) {
    g.controls.assign(controls, controls + nc);
    g.ctrl_vals.assign(ctrl_vals, ctrl_vals + nc);
  }
  const cd* m = reinterpret_cast<const cd*>(mat);
  g.mat.assign(m, m + (size_t(1) << (2 * k)));
  c->gates.push_back(std::move(g));
  return QSV_OK;
}

int qsv_circuit_add_named(qsv_circuit* c, int kind, const int* qubits, int nq, double theta) {
  clear_error();
  if (!c) return fail(QSV_EINVAL, "null circuit");
  cd m[16];
  int k = 0;
  int rc = named_matrix(kind, theta, m, &k);
  if (rc) return rc;
  if (nq != k) return fail(QSV_EINVAL, "named gate %d takes %d qubits (got %d)", kind, k, nq);
  if ((rc = validate_gate(c->n, qubits, k, nullptr, nullptr, 0, 2))) return rc;
  Gate g;
  if (kind == QSV_GATE_RX || kind == QSV_GATE_RY || kind == QSV_GATE_RZ) {
    g.kind = Gate::ROTATION;
    g.pauli = kind - QSV_GATE_RX + 1;
    g.fixed_angle = theta;
    g.targets.assign(qubits, qubits + 1);
  } else if (kind == QSV_GATE_CNOT) {
    // stored as X on the target with one control, the structure the
    // kernels apply directly
    g.kind = Gate::MATRIX;
    g.targets = {qubits[1]};
    g.controls = {qubits[0]};
    g.ctrl_vals = {1};
    g.mat = {{0, 0}, {1, 0}, {1, 0}, {0, 0}};
  } else {
    g.kind = Gate::MATRIX;
    g.targets.assign(qubits, qubits + k);
    g.mat.assign(m, m + (size_t(1) << (2 * k)));
  }
  c->gates.push_back(std::move(g));
  return QSV_OK;
}

int qsv_circuit_add_rotation(qsv_circuit* c, int pauli_id, int qubit, int param_slot) {
  clear_error();
  if (!c) return fail(QSV_EINVAL, "null circuit");
  if (pauli_id < 1 || pauli_id > 3) return fail(QSV_EINVAL, "pauli id %d not in 1..3", pauli_id);
  if (qubit < 0 || qubit >= c->n) return fail(QSV_ERANGE, "qubit %d out of range", qubit);
  if (param_slot < 0 || param_slot >= (1 << 24)) return fail(QSV_ERANGE, "bad parameter slot");
  Gate g;
  g.kind = Gate::ROTATION;
  g.pauli = pauli_id;
  g.slot = param_slot;
  g.targets = {qubit};
  c->gates.push_back(std::move(g));
  if (param_slot + 1 > c->nparams) c->nparams = param_slot + 1;
  return QSV_OK;
}

int qsv_circuit_add_pauli_rotation(qsv_circuit* c, const int* qubits, const int* pauli_ids, int w,
                                   int param_slot, double theta) {
  clear_error();
  if (!c) return fail(QSV_EINVAL, "null circuit");
  if (w < 1 || w > c->n) return fail(QSV_EINVAL, "string length %d outside [1, n]", w);
  if (!qubits || !pauli_ids) return fail(QSV_EINVAL, "null qubit or pauli list");
  if (param_slot >= (1 << 24)) return fail(QSV_ERANGE, "bad parameter slot");
  Gate g;
  g.kind = Gate::PAULI;
  uint64_t seen = 0;
  for (int j = 0; j < w; ++j) {
    if (qubits[j] < 0 || qubits[j] >= c->n) return fail(QSV_ERANGE, "qubit %d out of range", qubits[j]);
    if (pauli_ids[j] < 0 || pauli_ids[j] > 3) return fail(QSV_EINVAL, "pauli id %d not in 0..3", pauli_ids[j]);
    if (seen >> qubits[j] & 1) return fail(QSV_EDUP, "qubit %d repeated", qubits[j]);
    seen |= uint64_t(1) << qubits[j];
    if (pauli_ids[j] == 0) continue;  // identity factor
    g.targets.push_back(qubits[j]);
    g.paulis.push_back(pauli_ids[j]);
  }
  g.slot = param_slot < 0 ? -1 : param_slot;
  g.fixed_angle = theta;
  c->gates.push_back(std::move(g));
  if (param_slot >= 0 && param_slot + 1 > c->nparams) c->nparams = param_slot + 1;
  return QSV_OK;
}

int qsv_circuit_info(const qsv_circuit* c, int* n, int* gates, int* nparams) {
  clear_error();
  if (!c) return fail(QSV_EINVAL, "null circuit");
  if (n) *n = c->n;
  if (gates) *gates = int(c->gates.size());
  if (nparams) *nparams = c->nparams;
  return QSV_OK;
}

int qsv_apply_circuit(qsv_state* s, const qsv_circuit* c, const double* theta) {
  clear_error();
  int rc = check_state(s);
  if (rc) return rc;
  if (!c) return fail(QSV_EINVAL, "null circuit");
  if (c->n != s->n) return fail(QSV_ERANGE, "circuit has %d qubits, state %d", c->n, s->n);
  if (c->nparams > 0 && !theta) return fail(QSV_EINVAL, "circuit has parameters but theta is null");
  return circuit_apply_unfused(s, c, theta);
}

}  // extern "C"
