// Plain CPU oracle for the state-vector method of Qulacs (Suzuki et al., 2021).
//
// TEST INFRASTRUCTURE ONLY. This file is the slow, obviously-correct reference
// that the GPU library is checked against. Only the test suite, the smoke entry
// and the CPU-baseline leg of the benchmark load it. It shares no source with the
// GPU library: no headers, no helpers, no tables.
//
// Everything is complex128 (std::complex<double>). A state of n qubits is 2^n
// amplitudes stored interleaved (re, im) as 2*2^n doubles, basis index
// x = sum_q x_q 2^q, qubit 0 being the right-most digit of the ket (paper,
// section 4.2.1, "Initialization").
//
// Parity status of each entry point (what pins it is in the test suite):
//   orc_set_basis, orc_apply_matrix, orc_named_matrix, orc_expectation,
//   orc_norm2, orc_inner: pinned (closed forms, brute force, printed fixture).
//   orc_pauli_rotation: pinned (one-qubit case = RX/RY/RZ matrices, matrix
//   exponential of the Kronecker-product string for n <= 4, ZZ phases on basis
//   states). orc_transition: pinned (a = b gives orc_expectation's value,
//   brute-force a^dagger O b for n <= 4).
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef std::complex<double> cplx;

namespace {

inline cplx* as_c(double* p) { return reinterpret_cast<cplx*>(p); }
inline const cplx* as_c(const double* p) { return reinterpret_cast<const cplx*>(p); }

}  // namespace

extern "C" {

// Threads the parallel B0 loop uses (for reporting CPU timings).
int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

// Sets the number of threads of the parallel B0 loop (timing at one thread and
// at all cores); returns the new count. No effect on any result.
int orc_set_num_threads(int t) {
#ifdef _OPENMP
  if (t > 0) omp_set_num_threads(t);
  return omp_get_max_threads();
#else
  (void)t;
  return 1;
#endif
}

// |k> : all amplitudes zero except amplitude k, which is one (section 4.2.1).
void orc_set_basis(double* psi, int n, uint64_t k) {
  const uint64_t N = uint64_t(1) << n;
  cplx* v = as_c(psi);
  for (uint64_t x = 0; x < N; ++x) v[x] = 0.0;
  v[k] = 1.0;
}

// Basic-gate update, section 4.3.2, Eq. (update_mat):
//   for every x0 in B0 (all target bits zero), gather the temporal vector
//   t_i = psi[x0 + s(bin(i))], multiply by the gate matrix, scatter back.
// Bit j of the gate-matrix row/column index corresponds to targets[j].
// Controls (section 4.3.2, controlled gates): the update only acts on those x0
// whose control bits equal the requested control values.
// B0 is enumerated by filtering every x in [0, 2^n), which is the definition
// of the set, not an index-insertion scheme.
// mat: 2^k x 2^k complex128, row-major, interleaved. Returns 0, or -1 on bad
// arguments (duplicate or out-of-range qubits).
int orc_apply_matrix(double* psi, int n, const double* mat, const int* targets, int k,
                     const int* controls, const int* ctrl_vals, int nc) {
  if (k < 1 || n < 1 || k > n) return -1;
  uint64_t used = 0;
  for (int j = 0; j < k; ++j) {
    if (targets[j] < 0 || targets[j] >= n) return -1;
    if (used >> targets[j] & 1) return -1;
    used |= uint64_t(1) << targets[j];
  }
  uint64_t cmask = 0, cval = 0;
  for (int j = 0; j < nc; ++j) {
    if (controls[j] < 0 || controls[j] >= n) return -1;
    if (used >> controls[j] & 1) return -1;
    if (ctrl_vals[j] != 0 && ctrl_vals[j] != 1) return -1;
    used |= uint64_t(1) << controls[j];
    cmask |= uint64_t(1) << controls[j];
    if (ctrl_vals[j]) cval |= uint64_t(1) << controls[j];
  }
  uint64_t tmask = 0;
  for (int j = 0; j < k; ++j) tmask |= uint64_t(1) << targets[j];

  const uint64_t N = uint64_t(1) << n;
  const int D = 1 << k;
  // s(bin(i)): the offset of the i-th element of B1.
  std::vector<uint64_t> s(D);
  for (int i = 0; i < D; ++i) {
    uint64_t off = 0;
    for (int j = 0; j < k; ++j)
      if (i >> j & 1) off |= uint64_t(1) << targets[j];
    s[i] = off;
  }
  const cplx* K = as_c(mat);
  cplx* v = as_c(psi);
#pragma omp parallel
  {
    std::vector<cplx> t(D), u(D);
#pragma omp for schedule(static)
    for (int64_t xs = 0; xs < int64_t(N); ++xs) {
      const uint64_t x = uint64_t(xs);
      if ((x & tmask) != 0) continue;          // x is not in B0
      if ((x & cmask) != cval) continue;       // control pattern not met
      for (int i = 0; i < D; ++i) t[i] = v[x + s[i]];
      for (int r = 0; r < D; ++r) {
        cplx acc = 0.0;
        for (int c = 0; c < D; ++c) acc += K[r * D + c] * t[c];
        u[r] = acc;
      }
      for (int i = 0; i < D; ++i) v[x + s[i]] = u[i];
    }
  }
  return 0;
}

// Gate matrices of named gates (section 4.3.4, table of named gates).
// kind: 0 I, 1 X, 2 Y, 3 Z (Pauli matrices of section 4.3.2), 4 H,
//       5 RX, 6 RY, 7 RZ, rotations exp(+i theta P / 2) as the table defines them,
//       8 CNOT, 9 CZ, 10 SWAP (two-qubit, index bit 0 = first qubit argument).
// For CNOT the first qubit argument is the target and the second the control,
// so that the matrix reads as "flip bit 0 when bit 1 is set".
// out: row-major interleaved; 2x2 (8 doubles) or 4x4 (32 doubles).
// Returns the matrix dimension, or -1 for an unknown kind.
int orc_named_matrix(int kind, double theta, double* out) {
  cplx* m = as_c(out);
  const cplx I(0.0, 1.0);
  const double c = std::cos(theta / 2), s = std::sin(theta / 2);
  auto set2 = [&](cplx a, cplx b, cplx cc, cplx d) { m[0] = a; m[1] = b; m[2] = cc; m[3] = d; };
  switch (kind) {
    case 0: set2(1.0, 0.0, 0.0, 1.0); return 2;
    case 1: set2(0.0, 1.0, 1.0, 0.0); return 2;
    case 2: set2(0.0, -I, I, 0.0); return 2;
    case 3: set2(1.0, 0.0, 0.0, -1.0); return 2;
    case 4: {
      const double h = 1.0 / std::sqrt(2.0);
      set2(h, h, h, -h);
      return 2;
    }
    // exp(i t P/2) = cos(t/2) I + i sin(t/2) P, written out per Pauli.
    case 5: set2(c, I * s, I * s, c); return 2;
    case 6: set2(c, s, -s, c); return 2;
    case 7: set2(cplx(c, s), 0.0, 0.0, cplx(c, -s)); return 2;
    case 8:
    case 9:
    case 10: {
      for (int i = 0; i < 16; ++i) m[i] = 0.0;
      if (kind == 8) {        // |b1 b0> -> |b1, b0 xor b1>
        m[0 * 4 + 0] = 1.0; m[1 * 4 + 1] = 1.0; m[2 * 4 + 3] = 1.0; m[3 * 4 + 2] = 1.0;
      } else if (kind == 9) { // diag(1, 1, 1, -1)
        m[0] = 1.0; m[5] = 1.0; m[10] = 1.0; m[15] = -1.0;
      } else {                // |b1 b0> -> |b0 b1>
        m[0] = 1.0; m[1 * 4 + 2] = 1.0; m[2 * 4 + 1] = 1.0; m[15] = 1.0;
      }
      return 4;
    }
    default: return -1;
  }
}

// Squared norm <psi|psi> (section 4.2.2), Neumaier-compensated serial sum.
double orc_norm2(const double* psi, int n) {
  const uint64_t N = uint64_t(1) << n;
  const cplx* v = as_c(psi);
  double sum = 0.0, comp = 0.0;
  for (uint64_t x = 0; x < N; ++x) {
    const double a = std::norm(v[x]);
    const double t = sum + a;
    comp += (std::fabs(sum) >= std::fabs(a)) ? (sum - t) + a : (a - t) + sum;
    sum = t;
  }
  return sum + comp;
}

namespace {
struct Neumaier {
  double s = 0.0, c = 0.0;
  void add(double a) {
    const double t = s + a;
    c += (std::fabs(s) >= std::fabs(a)) ? (s - t) + a : (a - t) + s;
    s = t;
  }
  double value() const { return s + c; }
};
}  // namespace

// Inner product <a|b> = sum_x conj(a_x) b_x (section 4.2.2).
void orc_inner(const double* a, const double* b, int n, double* out_re, double* out_im) {
  const uint64_t N = uint64_t(1) << n;
  const cplx* va = as_c(a);
  const cplx* vb = as_c(b);
  Neumaier re, im;
  for (uint64_t x = 0; x < N; ++x) {
    const cplx p = std::conj(va[x]) * vb[x];
    re.add(p.real());
    im.add(p.imag());
  }
  *out_re = re.value();
  *out_im = im.value();
}

// Expectation value of an observable O = sum_k alpha_k P_k with real
// coefficients (section 4.5), <psi|O|psi> = sum_k alpha_k sum_{x,y} conj(psi_y)
// (P_k)_{y,x} psi_x. A Pauli string is a tensor product of the 2x2 Pauli
// matrices of section 4.3.2 (ids 0..3 = I, X, Y, Z); its matrix element
// (P)_{y,x} is the product over qubits of sigma_q[y_q][x_q], and it vanishes
// unless y differs from x exactly on the qubits carrying X or Y.
// Terms: term t has term_len[t] entries starting at offset sum(term_len[<t]) in
// qubits[] / paulis[]. Result returned as (re, im); im vanishes for Hermitian O.
// Returns 0, or -1 on a bad qubit / pauli id.
int orc_expectation(const double* psi, int n, int nterms, const double* coefs,
                    const int* term_len, const int* qubits, const int* paulis,
                    double* out_re, double* out_im) {
  static const cplx kPauli[4][2][2] = {
      {{1.0, 0.0}, {0.0, 1.0}},
      {{0.0, 1.0}, {1.0, 0.0}},
      {{0.0, cplx(0.0, -1.0)}, {cplx(0.0, 1.0), 0.0}},
      {{1.0, 0.0}, {0.0, -1.0}},
  };
  const uint64_t N = uint64_t(1) << n;
  const cplx* v = as_c(psi);
  Neumaier re, im;
  int off = 0;
  for (int t = 0; t < nterms; ++t) {
    const int w = term_len[t];
    std::vector<int> q(qubits + off, qubits + off + w), p(paulis + off, paulis + off + w);
    off += w;
    uint64_t flip = 0;
    for (int j = 0; j < w; ++j) {
      if (q[j] < 0 || q[j] >= n || p[j] < 0 || p[j] > 3) return -1;
      if (p[j] == 1 || p[j] == 2) flip |= uint64_t(1) << q[j];
    }
    Neumaier tre, tim;
    for (uint64_t x = 0; x < N; ++x) {
      const uint64_t y = x ^ flip;
      cplx elem = 1.0;
      for (int j = 0; j < w; ++j) elem *= kPauli[p[j]][(y >> q[j]) & 1][(x >> q[j]) & 1];
      const cplx c = std::conj(v[y]) * elem * v[x];
      tre.add(c.real());
      tim.add(c.imag());
    }
    re.add(coefs[t] * tre.value());
    im.add(coefs[t] * tim.value());
  }
  *out_re = re.value();
  *out_im = im.value();
  return 0;
}

// psi_out = O psi with O = sum_k alpha_k P_k (same term encoding as above):
// (O psi)_y = sum_k alpha_k sum_x (P_k)_{y,x} psi_x. Used by tests of the
// adjoint's lambda = H psi step.
int orc_apply_observable(const double* psi, double* out, int n, int nterms, const double* coefs,
                         const int* term_len, const int* qubits, const int* paulis) {
  static const cplx kPauli[4][2][2] = {
      {{1.0, 0.0}, {0.0, 1.0}},
      {{0.0, 1.0}, {1.0, 0.0}},
      {{0.0, cplx(0.0, -1.0)}, {cplx(0.0, 1.0), 0.0}},
      {{1.0, 0.0}, {0.0, -1.0}},
  };
  const uint64_t N = uint64_t(1) << n;
  const cplx* v = as_c(psi);
  cplx* o = as_c(out);
  for (uint64_t x = 0; x < N; ++x) o[x] = 0.0;
  int off = 0;
  for (int t = 0; t < nterms; ++t) {
    const int w = term_len[t];
    uint64_t flip = 0;
    for (int j = 0; j < w; ++j) {
      if (qubits[off + j] < 0 || qubits[off + j] >= n || paulis[off + j] < 0 || paulis[off + j] > 3)
        return -1;
      if (paulis[off + j] == 1 || paulis[off + j] == 2) flip |= uint64_t(1) << qubits[off + j];
    }
    for (uint64_t x = 0; x < N; ++x) {
      const uint64_t y = x ^ flip;
      cplx elem = 1.0;
      for (int j = 0; j < w; ++j)
        elem *= kPauli[paulis[off + j]][(y >> qubits[off + j]) & 1][(x >> qubits[off + j]) & 1];
      o[y] += coefs[t] * elem * v[x];
    }
    off += w;
  }
  return 0;
}

// Multi-qubit Pauli rotation exp(+i theta P / 2) (section 4.3.2, Pauli
// rotation; the factor 1/2 follows the one-qubit rotations of Table 1), P a
// Pauli string on w distinct qubits (ids 1..3; 0 = identity on that qubit).
// Since P^2 = I, exp(i theta P/2) = cos(theta/2) I + i sin(theta/2) P; P psi is
// formed from the matrix elements as in orc_apply_observable. Returns -1 on a
// bad qubit / pauli id or a repeated qubit.
int orc_pauli_rotation(double* psi, int n, int w, const int* qubits, const int* paulis, double theta) {
  static const cplx kPauli[4][2][2] = {
      {{1.0, 0.0}, {0.0, 1.0}},
      {{0.0, 1.0}, {1.0, 0.0}},
      {{0.0, cplx(0.0, -1.0)}, {cplx(0.0, 1.0), 0.0}},
      {{1.0, 0.0}, {0.0, -1.0}},
  };
  const uint64_t N = uint64_t(1) << n;
  uint64_t flip = 0, seen = 0;
  for (int j = 0; j < w; ++j) {
    if (qubits[j] < 0 || qubits[j] >= n || paulis[j] < 0 || paulis[j] > 3) return -1;
    if (seen >> qubits[j] & 1) return -1;
    seen |= uint64_t(1) << qubits[j];
    if (paulis[j] == 1 || paulis[j] == 2) flip |= uint64_t(1) << qubits[j];
  }
  cplx* v = as_c(psi);
  std::vector<cplx> pv(N);
  for (uint64_t x = 0; x < N; ++x) {
    const uint64_t y = x ^ flip;  // the one nonzero column of row y
    cplx elem = 1.0;
    for (int j = 0; j < w; ++j) elem *= kPauli[paulis[j]][(y >> qubits[j]) & 1][(x >> qubits[j]) & 1];
    pv[y] = elem * v[x];
  }
  const double c = std::cos(0.5 * theta), s = std::sin(0.5 * theta);
  for (uint64_t x = 0; x < N; ++x) v[x] = c * v[x] + cplx(0.0, s) * pv[x];
  return 0;
}

// Transition amplitude <a|O|b> = sum_k alpha_k sum_{x,y} conj(a_y) (P_k)_{y,x} b_x
// (section 4.5, get_transition_amplitude), complex, same term encoding as
// orc_expectation.
int orc_transition(const double* a, const double* b, int n, int nterms, const double* coefs,
                   const int* term_len, const int* qubits, const int* paulis, double* out_re,
                   double* out_im) {
  static const cplx kPauli[4][2][2] = {
      {{1.0, 0.0}, {0.0, 1.0}},
      {{0.0, 1.0}, {1.0, 0.0}},
      {{0.0, cplx(0.0, -1.0)}, {cplx(0.0, 1.0), 0.0}},
      {{1.0, 0.0}, {0.0, -1.0}},
  };
  const uint64_t N = uint64_t(1) << n;
  const cplx* va = as_c(a);
  const cplx* vb = as_c(b);
  Neumaier re, im;
  int off = 0;
  for (int t = 0; t < nterms; ++t) {
    const int w = term_len[t];
    uint64_t flip = 0;
    for (int j = 0; j < w; ++j) {
      if (qubits[off + j] < 0 || qubits[off + j] >= n || paulis[off + j] < 0 || paulis[off + j] > 3)
        return -1;
      if (paulis[off + j] == 1 || paulis[off + j] == 2) flip |= uint64_t(1) << qubits[off + j];
    }
    Neumaier tre, tim;
    for (uint64_t x = 0; x < N; ++x) {
      const uint64_t y = x ^ flip;
      cplx elem = 1.0;
      for (int j = 0; j < w; ++j)
        elem *= kPauli[paulis[off + j]][(y >> qubits[off + j]) & 1][(x >> qubits[off + j]) & 1];
      const cplx c = std::conj(va[y]) * elem * vb[x];
      tre.add(c.real());
      tim.add(c.imag());
    }
    re.add(coefs[t] * tre.value());
    im.add(coefs[t] * tim.value());
    off += w;
  }
  *out_re = re.value();
  *out_im = im.value();
  return 0;
}

}  // extern "C"
