// Multi-qubit Pauli rotations exp(+i t P / 2) (section 4.3.2, Pauli rotation;
// the factor 1/2 as in the one-qubit rotations of Table 1) and transition
// amplitudes <a|O|b> (section 4.5).
//
// A Pauli string P with flip mask F (X/Y qubits), sign mask z (Z/Y qubits) and
// nY Y factors has one nonzero per column: P[x ^ F, x] = i^nY (-1)^|x & z|.
// Since P^2 = I, exp(i t P/2) = c I + i s P (c = cos t/2, s = sin t/2): on the
// pair (x, y = x ^ F), x with bit hb of F clear,
//   x <- c psi_x + g (-1)^|y & z| psi_y,  y <- c psi_y + g (-1)^|x & z| psi_x,
// with g = i s i^nY; for F = 0 (Z strings) x <- (c + i s (-1)^|x & z|) psi_x.
// <a|P|b> = i^nY sum_x (-1)^|x & z| conj(a_{x ^ F}) b_x.
#include <algorithm>
#include <cmath>

#include "circuit.h"
#include "dev_common.h"
#include "observable.h"
#include "prof.h"
#include "qsv_internal.h"

namespace qsv {

constexpr int kPauliThreads = 256;
constexpr int kPauliBlocks = 2048;

__device__ __forceinline__ uint64_t pr_ins0(uint64_t i, int hb) {
  return ((i >> hb) << (hb + 1)) | (i & ((uint64_t(1) << hb) - 1));
}

__device__ __forceinline__ bool pr_odd(uint64_t x, uint64_t z) { return __popcll(x & z) & 1; }

template <typename R>
__device__ __forceinline__ cx<R> pr_sgn(bool neg, cx<R> v) {
  return neg ? cx<R>{-v.re, -v.im} : v;
}

// complex64 with qubit 0 outside F: amplitudes x, x + 1 (x even) pair with
// x ^ F, (x ^ F) + 1, so each side of two pairs is one 16-byte vector; count
// = N / 4 (F != 0) or N / 2 (F = 0) vector steps.
__global__ void __launch_bounds__(kPauliThreads)
    k_pauli_rot_v2(float* __restrict__ psi, uint64_t count, uint64_t flip, uint64_t z, int hb, float c,
                   cx<float> g) {
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < count; i += stride) {
    cx<float> a[2], b[2];
    if (flip == 0) {
      const uint64_t x = 2 * i;
      AmpIO<float, 2>::load(psi, x, a);
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const cx<float> f = pr_sgn(pr_odd(x + k, z), g);
        a[k] = cx<float>{c + f.re, f.im} * a[k];
      }
      AmpIO<float, 2>::store(psi, x, a);
      continue;
    }
    const uint64_t x = pr_ins0(2 * i, hb), y = x ^ flip;
    AmpIO<float, 2>::load(psi, x, a);
    AmpIO<float, 2>::load(psi, y, b);
    cx<float> na[2], nb[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      na[k] = cfma(pr_sgn(pr_odd(y + k, z), g), b[k], cx<float>{c * a[k].re, c * a[k].im});
      nb[k] = cfma(pr_sgn(pr_odd(x + k, z), g), a[k], cx<float>{c * b[k].re, c * b[k].im});
    }
    AmpIO<float, 2>::store(psi, x, na);
    AmpIO<float, 2>::store(psi, y, nb);
  }
}

template <typename R>
__global__ void __launch_bounds__(kPauliThreads)
    k_pauli_rot(R* __restrict__ psi, uint64_t count, uint64_t flip, uint64_t z, int hb, R c, cx<R> g) {
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < count; i += stride) {
    if (flip == 0) {
      const cx<R> a = load1(psi, i);
      const cx<R> f = pr_sgn(pr_odd(i, z), g);  // i s (-1)^|x & z|
      store1(psi, i, cx<R>{c + f.re, f.im} * a);
      continue;
    }
    const uint64_t x = pr_ins0(i, hb), y = x ^ flip;
    const cx<R> a = load1(psi, x), b = load1(psi, y);
    store1(psi, x, cfma(pr_sgn(pr_odd(y, z), g), b, cx<R>{c * a.re, c * a.im}));
    store1(psi, y, cfma(pr_sgn(pr_odd(x, z), g), a, cx<R>{c * b.re, c * b.im}));
  }
}

__device__ __forceinline__ double pr_block_sum(double v, double* sh) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double r = 0.0;
  for (int i = 0; i < int(blockDim.x >> 6); ++i) r += sh[i];
  return r;
}

// S = sum_x (-1)^|x & z| conj(a_{x ^ F}) b_x in FP64: per-block partials
// (re, im) at partial[2 blk], partial[2 blk + 1].
template <typename R>
__global__ void __launch_bounds__(kPauliThreads)
    k_pauli_sum(const R* __restrict__ a, const R* __restrict__ b, uint64_t N, uint64_t flip, uint64_t z,
                double* __restrict__ partial) {
  __shared__ double sh[kPauliThreads / 64];
  double re = 0.0, im = 0.0;
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  for (uint64_t x = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; x < N; x += stride) {
    const cx<R> u = load1(a, x ^ flip), v = load1(b, x);
    const double pr = double(u.re) * v.re + double(u.im) * v.im;  // conj(u) v
    const double pi = double(u.re) * v.im - double(u.im) * v.re;
    if (pr_odd(x, z)) {
      re -= pr;
      im -= pi;
    } else {
      re += pr;
      im += pi;
    }
  }
  const double r = pr_block_sum(re, sh);
  const double s = pr_block_sum(im, sh);
  if (threadIdx.x == 0) {
    partial[2 * blockIdx.x] = r;
    partial[2 * blockIdx.x + 1] = s;
  }
}

// Reverse-sweep step of a parametric Pauli rotation: this block's share of
// the gradient -Im(i^nY S(lam, psi)) into partial_row[blk], then psi and lam
// uncomputed by exp(-i t P/2) (c, g of the negated angle).
template <typename R>
__global__ void __launch_bounds__(kPauliThreads)
    k_adj_pauli(R* __restrict__ psi, R* __restrict__ lam, uint64_t count, uint64_t flip, uint64_t z, int hb,
                R c, cx<R> g, double fre, double fim, double* __restrict__ partial_row) {
  __shared__ double sh[kPauliThreads / 64];
  double sre = 0.0, sim = 0.0;  // S share
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < count; i += stride) {
    if (flip == 0) {
      const cx<R> p = load1(psi, i), l = load1(lam, i);
      const double pr = double(l.re) * p.re + double(l.im) * p.im;
      const double pi = double(l.re) * p.im - double(l.im) * p.re;
      const bool neg = pr_odd(i, z);
      sre += neg ? -pr : pr;
      sim += neg ? -pi : pi;
      const cx<R> f = pr_sgn(neg, g);
      const cx<R> fc{c + f.re, f.im};
      store1(psi, i, fc * p);
      store1(lam, i, fc * l);
      continue;
    }
    const uint64_t x = pr_ins0(i, hb), y = x ^ flip;
    const cx<R> px = load1(psi, x), py = load1(psi, y), lx = load1(lam, x), ly = load1(lam, y);
    const bool nx = pr_odd(x, z), ny = pr_odd(y, z);
    // terms x and y of S: conj(lam_{x^F}) psi_x (-1)^|x&z| + conj(lam_{y^F}) psi_y (-1)^|y&z|
    const double ar = double(ly.re) * px.re + double(ly.im) * px.im, ai = double(ly.re) * px.im - double(ly.im) * px.re;
    const double br = double(lx.re) * py.re + double(lx.im) * py.im, bi = double(lx.re) * py.im - double(lx.im) * py.re;
    sre += (nx ? -ar : ar) + (ny ? -br : br);
    sim += (nx ? -ai : ai) + (ny ? -bi : bi);
    const cx<R> gx = pr_sgn(ny, g), gy = pr_sgn(nx, g);
    store1(psi, x, cfma(gx, py, cx<R>{c * px.re, c * px.im}));
    store1(psi, y, cfma(gy, px, cx<R>{c * py.re, c * py.im}));
    store1(lam, x, cfma(gx, ly, cx<R>{c * lx.re, c * lx.im}));
    store1(lam, y, cfma(gy, lx, cx<R>{c * ly.re, c * ly.im}));
  }
  // -Im((fre + i fim) (sre + i sim))
  const double v = -(fre * sim + fim * sre);
  const double r = pr_block_sum(v, sh);
  if (threadIdx.x == 0) partial_row[blockIdx.x] = r;
}

namespace {

struct PauliMasks {
  uint64_t flip = 0, z = 0;
  int ny = 0, hb = 0;
};

int pauli_masks(int n, const int* qubits, const int* ids, int w, PauliMasks* m) {
  uint64_t seen = 0;
  for (int j = 0; j < w; ++j) {
    if (qubits[j] < 0 || qubits[j] >= n) return fail(QSV_ERANGE, "qubit %d out of range", qubits[j]);
    if (ids[j] < 0 || ids[j] > 3) return fail(QSV_EINVAL, "pauli id %d not in 0..3", ids[j]);
    const uint64_t bit = uint64_t(1) << qubits[j];
    if (seen & bit) return fail(QSV_EDUP, "qubit %d repeated", qubits[j]);
    seen |= bit;
    if (ids[j] == 1 || ids[j] == 2) m->flip |= bit;
    if (ids[j] == 2 || ids[j] == 3) m->z |= bit;
    if (ids[j] == 2) ++m->ny;
  }
  m->hb = m->flip ? 63 - __builtin_clzll(m->flip) : 0;
  return QSV_OK;
}

// i^k as (re, im)
cd ipow(int k) {
  switch (k & 3) {
    case 0: return {1, 0};
    case 1: return {0, 1};
    case 2: return {-1, 0};
    default: return {0, -1};
  }
}

// reductions: a bounded number of per-block partials
int pr_blocks(uint64_t work) {
  return int(std::max<uint64_t>(1, std::min<uint64_t>((work + kPauliThreads - 1) / kPauliThreads, kPauliBlocks)));
}

// element-wise sweeps: one step per thread (a one-shot grid streams faster
// than a few thousand grid-striding workgroups), at most 2^22 workgroups
int pr_grid(uint64_t work) {
  return int(std::max<uint64_t>(1, std::min<uint64_t>((work + kPauliThreads - 1) / kPauliThreads, uint64_t(1) << 22)));
}

template <typename R>
int pauli_rotation_t(qsv_state* s, const PauliMasks& m, double t) {
  const uint64_t N = dim(s->n);
  const uint64_t count = m.flip ? N / 2 : N;
  const double c = std::cos(0.5 * t), sn = std::sin(0.5 * t);
  const cd g = cmul(cd{0, sn}, ipow(m.ny));
  ProfScope ps("pair", 2.0 * sizeof(cx<R>) * double(N), s->stream);
  if constexpr (sizeof(R) == 4) {
    if (!(m.flip & 1) && s->n >= 2) {  // 16-byte vectors: qubit 0 is not flipped
      const uint64_t vcount = count / 2;
      hipLaunchKernelGGL(k_pauli_rot_v2, dim3(pr_grid(vcount)), dim3(kPauliThreads), 0, s->stream,
                         static_cast<float*>(s->ptr), vcount, m.flip, m.z, m.hb, float(c),
                         cx<float>{float(g.re), float(g.im)});
      QSV_HIP_CHECK(hipGetLastError());
      return QSV_OK;
    }
  }
  hipLaunchKernelGGL((k_pauli_rot<R>), dim3(pr_grid(count)), dim3(kPauliThreads), 0, s->stream,
                     static_cast<R*>(s->ptr), count, m.flip, m.z, m.hb, R(c), cx<R>{R(g.re), R(g.im)});
  QSV_HIP_CHECK(hipGetLastError());
  return QSV_OK;
}

template <typename R>
int pauli_sum_t(const qsv_state* a, const qsv_state* b, qsv_state* owner, uint64_t flip, uint64_t z, cd* out) {
  const uint64_t N = dim(a->n);
  const int nb = pr_blocks(N);
  int rc = ensure_reduce_scratch(owner, size_t(2 * nb + 2));
  if (rc) return rc;
  double* partial = owner->red;
  hipLaunchKernelGGL((k_pauli_sum<R>), dim3(nb), dim3(kPauliThreads), 0, owner->stream,
                     static_cast<const R*>(a->ptr), static_cast<const R*>(b->ptr), N, flip, z, partial);
  QSV_HIP_CHECK(hipGetLastError());
  QSV_HIP_CHECK(hipStreamSynchronize(owner->stream));
  std::vector<double> h(size_t(2 * nb));
  QSV_HIP_CHECK(hipMemcpy(h.data(), partial, h.size() * sizeof(double), hipMemcpyDeviceToHost));
  double re = 0.0, im = 0.0;
  for (int i = 0; i < nb; ++i) {  // fixed order
    re += h[size_t(2 * i)];
    im += h[size_t(2 * i + 1)];
  }
  *out = {re, im};
  return QSV_OK;
}

}  // namespace

int pauli_rotation_impl(qsv_state* s, const int* qubits, const int* ids, int w, double t) {
  PauliMasks m;
  int rc = pauli_masks(s->n, qubits, ids, w, &m);
  if (rc) return rc;
  return s->dtype == QSV_C64 ? pauli_rotation_t<float>(s, m, t) : pauli_rotation_t<double>(s, m, t);
}

// Reverse-sweep step for a parametric Pauli rotation gate of the adjoint
// (per-gate sweep): writes B partials of its gradient row.
int adjoint_pauli_step(qsv_state* psi, qsv_state* lam, const Gate& g, double t, double* partial_row, int B) {
  PauliMasks m;
  int rc = pauli_masks(psi->n, g.targets.data(), g.paulis.data(), int(g.targets.size()), &m);
  if (rc) return rc;
  const uint64_t N = dim(psi->n);
  const uint64_t count = m.flip ? N / 2 : N;
  const double c = std::cos(-0.5 * t), sn = std::sin(-0.5 * t);
  const cd gg = cmul(cd{0, sn}, ipow(m.ny));
  const cd f = ipow(m.ny);
  if (psi->dtype == QSV_C64) {
    ProfScope ps("adjoint", 4.0 * sizeof(cx<float>) * double(N), psi->stream);
    hipLaunchKernelGGL((k_adj_pauli<float>), dim3(B), dim3(kPauliThreads), 0, psi->stream,
                       static_cast<float*>(psi->ptr), static_cast<float*>(lam->ptr), count, m.flip, m.z, m.hb,
                       float(c), cx<float>{float(gg.re), float(gg.im)}, f.re, f.im, partial_row);
  } else {
    ProfScope ps("adjoint", 4.0 * sizeof(cx<double>) * double(N), psi->stream);
    hipLaunchKernelGGL((k_adj_pauli<double>), dim3(B), dim3(kPauliThreads), 0, psi->stream,
                       static_cast<double*>(psi->ptr), static_cast<double*>(lam->ptr), count, m.flip, m.z, m.hb,
                       c, cx<double>{gg.re, gg.im}, f.re, f.im, partial_row);
  }
  QSV_HIP_CHECK(hipGetLastError());
  return QSV_OK;
}

}  // namespace qsv

using namespace qsv;

extern "C" {

int qsv_apply_pauli_rotation(qsv_state* s, const int* qubits, const int* pauli_ids, int w, double theta) {
  clear_error();
  int rc = check_state(s);
  if (rc) return rc;
  if (w < 0 || w > s->n) return fail(QSV_EINVAL, "string length %d outside [0, n]", w);
  if (w > 0 && (!qubits || !pauli_ids)) return fail(QSV_EINVAL, "null qubit or pauli list");
  return pauli_rotation_impl(s, qubits, pauli_ids, w, theta);
}

int qsv_transition_amplitude(const qsv_state* bra, const qsv_observable* o, const qsv_state* ket, double* re,
                             double* im) {
  clear_error();
  int rc = check_state(bra);
  if (rc) return rc;
  if ((rc = check_state(ket))) return rc;
  if (!o) return fail(QSV_EINVAL, "null observable");
  if (!re || !im) return fail(QSV_EINVAL, "null output");
  if (bra->n != ket->n || o->n != bra->n) return fail(QSV_ERANGE, "qubit counts differ");
  if (bra->dtype != ket->dtype) return fail(QSV_EDTYPE, "dtypes differ");
  if (bra->stream != ket->stream) QSV_HIP_CHECK(hipStreamSynchronize(bra->stream));
  qsv_state* owner = const_cast<qsv_state*>(ket);  // reduction scratch only
  double sr = 0.0, si = 0.0;
  for (const auto& t : o->terms) {
    cd sum{0, 0};
    rc = bra->dtype == QSV_C64 ? pauli_sum_t<float>(bra, ket, owner, t.flip, t.zmask, &sum)
                               : pauli_sum_t<double>(bra, ket, owner, t.flip, t.zmask, &sum);
    if (rc) return rc;
    const cd v = cmul(ipow(t.ny), sum);
    sr += t.coef * v.re;
    si += t.coef * v.im;
  }
  *re = sr;
  *im = si;
  return QSV_OK;
}

}  // extern "C"
