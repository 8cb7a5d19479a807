// Adjoint gradient of E(theta) = <psi(theta)|H|psi(theta)>, psi(theta) =
// U_L ... U_1 |0...0>, for parametric rotations U = exp(+i theta P / 2)
// (table of named gates; ParametricRX/RY/RZ of section 4.4). The paper defines
// the objects (parametric circuits, observables); the sweep below is the
// standard reverse-mode identity, written for this library:
//
//   lambda = H psi_L,  E = Re <psi_L|lambda>
//   for l = L..1:   if U_l is parametric,
//                      dE/dtheta_l = 2 Re <lambda_l| (i P/2) U_l |psi_{l-1}>
//                                  = -Im <lambda_l| P |psi_l>
//                   psi <- U_l^dagger psi,  lambda <- U_l^dagger lambda
//
// One fused kernel per parametric rotation reads psi and lambda once, adds its
// share of -Im<lambda|P|psi> in FP64 and writes both uncomputed states
// (4 * 2^n amplitudes of traffic). lambda = H psi runs in tile passes that
// pack the observable's flip masks, like the expectation.
#include <algorithm>
#include <cmath>
#include <cstdlib>

#include "circuit.h"
#include "dev_common.h"
#include "observable.h"
#include "plan.h"
#include "prof.h"

namespace qsv {

constexpr int kAdjThreads = 256;
constexpr int kAdjBlocks = 1024;

__device__ __forceinline__ double block_sum(double v, double* sh) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < int(blockDim.x >> 6); ++i) r += sh[i];
  return r;
}

// Fused adjoint step of a one-qubit rotation exp(i t P/2) on qubit q:
// partial[blockIdx] = this block's share of -Im<lambda|P|psi>, then psi and
// lambda are multiplied by udag = exp(-i t P/2).
template <typename R>
__global__ void __launch_bounds__(kAdjThreads)
    k_adj_rot(R* __restrict__ psi, R* __restrict__ lam, uint64_t npairs, int q, int pauli,
              M2<R> u, double* __restrict__ partial) {
  __shared__ double sh[kAdjThreads / 64];
  double acc = 0.0;
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  const uint64_t bit = uint64_t(1) << q;
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < npairs; i += stride) {
    const uint64_t x0 = ((i >> q) << (q + 1)) | (i & (bit - 1));
    const uint64_t x1 = x0 | bit;
    const cx<R> a0 = load1(psi, x0), a1 = load1(psi, x1);
    const cx<R> l0 = load1(lam, x0), l1 = load1(lam, x1);
    // s = sum over the pair of conj(lambda_y) P[y, x] psi_x; only Im(s) is needed
    const double a0r = a0.re, a0i = a0.im, a1r = a1.re, a1i = a1.im;
    const double l0r = l0.re, l0i = l0.im, l1r = l1.re, l1i = l1.im;
    double im;
    if (pauli == 1) {  // conj(l0) a1 + conj(l1) a0
      im = (l0r * a1i - l0i * a1r) + (l1r * a0i - l1i * a0r);
    } else if (pauli == 2) {  // conj(l0) (-i a1) + conj(l1) (i a0)
      im = -(l0r * a1r + l0i * a1i) + (l1r * a0r + l1i * a0i);
    } else {  // conj(l0) a0 - conj(l1) a1
      im = (l0r * a0i - l0i * a0r) - (l1r * a1i - l1i * a1r);
    }
    acc -= im;
    store1(psi, x0, cfma(u.m00, a0, u.m01 * a1));
    store1(psi, x1, cfma(u.m10, a0, u.m11 * a1));
    store1(lam, x0, cfma(u.m00, l0, u.m01 * l1));
    store1(lam, x1, cfma(u.m10, l0, u.m11 * l1));
  }
  const double r = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = r;
}

// out[row] = sum of `cols` partials of row `row` (fixed order).
__global__ void __launch_bounds__(kAdjThreads)
    k_sum_rows(const double* __restrict__ partial, int cols, double* __restrict__ out) {
  __shared__ double sh[kAdjThreads / 64];
  double acc = 0.0;
  const double* p = partial + size_t(blockIdx.x) * cols;
  for (int i = threadIdx.x; i < cols; i += blockDim.x) acc += p[i];
  const double r = block_sum(acc, sh);
  if (threadIdx.x == 0) out[blockIdx.x] = r;
}

int expectation_impl(qsv_state* s, const qsv_observable* o, double* out);
int apply_observable_tiled(const qsv_state* in, const qsv_observable* o, qsv_state* out);
int circuit_apply_unfused(qsv_state* s, const qsv_circuit* c, const double* theta);
template <typename R>
int adjoint_backward_tiled(const qsv_circuit* c, const double* theta, qsv_state* psi, qsv_state* lam,
                           std::vector<int>& row_slot, std::vector<double>& rows);

namespace {

int adj_blocks(uint64_t work) {
  const uint64_t b = (work + kAdjThreads * 4 - 1) / (kAdjThreads * 4);
  return int(std::max<uint64_t>(1, std::min<uint64_t>(b, kAdjBlocks)));
}

int apply_obs(const qsv_state* in, const qsv_observable* o, qsv_state* out) {
  return apply_observable_tiled(in, o, out);
}

void dagger(std::vector<cd>& m) {
  const size_t D = size_t(std::lround(std::sqrt(double(m.size()))));
  std::vector<cd> t(m.size());
  for (size_t r = 0; r < D; ++r)
    for (size_t c = 0; c < D; ++c) t[c * D + r] = {m[r * D + c].re, -m[r * D + c].im};
  m.swap(t);
}

template <typename R>
int adjoint_t(const qsv_circuit* c, qsv_plan* plan, const double* theta, const qsv_observable* o,
              qsv_state* psi, qsv_state* lam, double* energy, double* grad) {
  const int n = c->n;
  const uint64_t N = dim(n);
  hipStream_t st = psi->stream;
  // forward from |0...0>
  int rc = qsv_set_basis(psi, 0);
  if (rc) return rc;
  if (plan) {
    if ((rc = qsv_apply_fused(psi, plan, theta))) return rc;
  } else {
    if ((rc = circuit_apply_unfused(psi, c, theta))) return rc;
  }
  // lambda = H psi
  if ((rc = apply_obs(psi, o, lam))) return rc;
  // E = Re <psi|lambda>
  double re = 0.0, im = 0.0;
  if ((rc = qsv_inner(psi, lam, &re, &im))) return rc;
  *energy = re;
  // backward
  int nrot = 0;
  bool wide = false;  // Pauli rotations on more than 5 qubits: per-gate sweep only
  for (const Gate& g : c->gates) {
    if ((g.kind == Gate::ROTATION || g.kind == Gate::PAULI) && g.slot >= 0) ++nrot;
    if (g.kind == Gate::PAULI && g.targets.size() > 5) wide = true;
  }
  // large states: reverse sweep by tile passes (both states streamed once per
  // pass); small states keep one launch per gate, which spreads better
  const int Ltile = sizeof(R) == 4 ? 12 : 11;
  int tiled_min = Ltile + 8;
  if (const char* e = std::getenv("QSV_ADJOINT_TILED_MIN")) tiled_min = std::atoi(e);  // testing
  if (n >= tiled_min && !wide) {
    std::vector<int> rs;
    std::vector<double> rv;
    if ((rc = adjoint_backward_tiled<R>(c, theta, psi, lam, rs, rv))) return rc;
    for (int i = 0; i < c->nparams; ++i) grad[i] = 0.0;
    for (size_t r = 0; r < rs.size(); ++r) grad[rs[r]] += rv[r];
    return QSV_OK;
  }
  const int B = adj_blocks(N / 2);
  if ((rc = ensure_reduce_scratch(psi, size_t(nrot) * B + size_t(nrot) + 1))) return rc;
  double* partial = psi->red;
  double* rows = psi->red + size_t(nrot) * B;
  int row = nrot;
  std::vector<int> row_slot(nrot);
  std::vector<cd> m;
  for (int gi = int(c->gates.size()) - 1; gi >= 0; --gi) {
    const Gate& g = c->gates[gi];
    if (g.kind == Gate::PAULI) {
      const double t = g.slot >= 0 ? theta[g.slot] : g.fixed_angle;
      if (g.slot >= 0) {
        // gradient -Im<lambda|P|psi> and the uncompute in one sweep
        --row;
        row_slot[row] = g.slot;
        if ((rc = adjoint_pauli_step(psi, lam, g, t, partial + size_t(row) * B, B))) return rc;
      } else {
        const int w = int(g.targets.size());
        if ((rc = pauli_rotation_impl(psi, g.targets.data(), g.paulis.data(), w, -t))) return rc;
        if ((rc = pauli_rotation_impl(lam, g.targets.data(), g.paulis.data(), w, -t))) return rc;
      }
      continue;
    }
    if (g.kind == Gate::ROTATION && g.slot >= 0) {
      --row;
      row_slot[row] = g.slot;
      cd u[4];
      rotation_matrix(g.pauli, -theta[g.slot], u);
      const M2<R> ud = {{R(u[0].re), R(u[0].im)}, {R(u[1].re), R(u[1].im)},
                        {R(u[2].re), R(u[2].im)}, {R(u[3].re), R(u[3].im)}};
      ProfScope ps("adjoint", 4.0 * sizeof(cx<R>) * double(N), st);
      hipLaunchKernelGGL((k_adj_rot<R>), dim3(B), dim3(kAdjThreads), 0, st,
                         static_cast<R*>(psi->ptr), static_cast<R*>(lam->ptr), N / 2,
                         g.targets[0], g.pauli, ud, partial + size_t(row) * B);
      QSV_HIP_CHECK(hipGetLastError());
      continue;
    }
    gate_matrix(g, theta, m);
    dagger(m);
    const int k = int(g.targets.size());
    if ((rc = apply_gate_impl(psi, m.data(), g.targets.data(), k, g.controls.data(),
                              g.ctrl_vals.data(), int(g.controls.size()))))
      return rc;
    if ((rc = apply_gate_impl(lam, m.data(), g.targets.data(), k, g.controls.data(),
                              g.ctrl_vals.data(), int(g.controls.size()))))
      return rc;
  }
  for (int i = 0; i < c->nparams; ++i) grad[i] = 0.0;
  if (nrot > 0) {
    hipLaunchKernelGGL(k_sum_rows, dim3(nrot), dim3(kAdjThreads), 0, st, partial, B, rows);
    QSV_HIP_CHECK(hipGetLastError());
    QSV_HIP_CHECK(hipStreamSynchronize(st));
    std::vector<double> hr(nrot);
    QSV_HIP_CHECK(hipMemcpy(hr.data(), rows, nrot * sizeof(double), hipMemcpyDeviceToHost));
    for (int r = 0; r < nrot; ++r) grad[row_slot[r]] += hr[r];
  } else {
    QSV_HIP_CHECK(hipStreamSynchronize(st));
  }
  return QSV_OK;
}

}  // namespace

}  // namespace qsv

using namespace qsv;

extern "C" {

int qsv_apply_observable(const qsv_state* in, const qsv_observable* o, qsv_state* out) {
  clear_error();
  int rc = check_state(in);
  if (rc) return rc;
  if ((rc = check_state(out))) return rc;
  if (!o) return fail(QSV_EINVAL, "null observable");
  if (in == out || in->ptr == out->ptr) return fail(QSV_EINVAL, "input and output must differ");
  if (in->n != out->n || o->n != in->n) return fail(QSV_ERANGE, "qubit counts differ");
  if (in->dtype != out->dtype) return fail(QSV_EDTYPE, "dtypes differ");
  if (in->stream != out->stream) QSV_HIP_CHECK(hipStreamSynchronize(in->stream));
  return apply_obs(in, o, out);
}

int qsv_adjoint_gradient(const qsv_circuit* c, qsv_plan* forward_plan, const double* theta,
                         const qsv_observable* o, qsv_state* psi, qsv_state* lam, double* energy,
                         double* grad) {
  clear_error();
  if (!c) return fail(QSV_EINVAL, "null circuit");
  if (!o) return fail(QSV_EINVAL, "null observable");
  int rc = check_state(psi);
  if (rc) return rc;
  if ((rc = check_state(lam))) return rc;
  if (!energy) return fail(QSV_EINVAL, "null energy output");
  if (c->nparams > 0 && (!theta || !grad)) return fail(QSV_EINVAL, "null theta or grad");
  if (psi->n != c->n || lam->n != c->n || o->n != c->n)
    return fail(QSV_ERANGE, "circuit, observable and states must have the same qubit count");
  if (psi->dtype != lam->dtype) return fail(QSV_EDTYPE, "psi and lambda dtypes differ");
  if (psi->ptr == lam->ptr) return fail(QSV_EINVAL, "psi and lambda must be distinct");
  if (psi->stream != lam->stream) return fail(QSV_EINVAL, "psi and lambda must share a stream");
  if (forward_plan) {
    if (forward_plan->n != c->n || forward_plan->dtype != psi->dtype ||
        forward_plan->circ_copy.gates.size() != c->gates.size())
      return fail(QSV_EINVAL, "forward plan does not match the circuit and dtype");
  }
  return psi->dtype == QSV_C64 ? adjoint_t<float>(c, forward_plan, theta, o, psi, lam, energy, grad)
                               : adjoint_t<double>(c, forward_plan, theta, o, psi, lam, energy, grad);
}

}  // extern "C"
