// Reductions over the state: squared norm and inner product (section 4.2.2)
// and expectation values of Pauli-string observables (section 4.5, with the
// Pauli matrices of section 4.3.2).
//
// A Pauli string P with X/Y qubits F (the flip mask), Z/Y qubits Zm and nY
// factors Y has matrix elements
//     P[x ^ F, x] = i^nY * (-1)^popcount(x & Zm),
// so <psi|P|psi> = sum_x conj(psi[x ^ F]) i^nY (-1)^|x & Zm| psi[x]. Terms are
// grouped by flip mask: one pass over the state serves every term of a group.
// For F != 0 the pass visits each pair {x, x ^ F} once (x with the highest bit
// of F clear) and, the observable being Hermitian, the two members contribute
// complex-conjugate amounts, so the pair adds 2 Re(conj(psi[x^F]) c(x) psi[x])
// with c(x) = sum_k alpha_k i^nY_k (-1)^|x & Zm_k|. For F == 0 the pass adds
// |psi[x]|^2 c(x). Every pass reads each amplitude once.
//
// Accumulation is FP64 per lane, then a wavefront butterfly, then an LDS tree
// per workgroup, then one fixed-order pass over the per-workgroup partials, so
// results are bitwise reproducible from run to run.
#include <algorithm>
#include <map>

#include "dev_common.h"
#include "observable.h"
#include "prof.h"
#include "qsv_internal.h"

namespace qsv {

int expectation_tiled(qsv_state* s, const qsv_observable* o, double* out);
int expectation_noalloc(qsv_state* s, const qsv_observable* o, double* out);
int expectation_passes(const qsv_observable* o, qsv_dtype dt);

constexpr int kRedThreads = 256;
constexpr int kMaxRedBlocks = 2048;
constexpr int kLdsTerms = 512;

__device__ __forceinline__ double block_reduce_sum(double v, double* sh) {
  // wavefront butterfly (64 lanes)
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
    for (int i = 0; i < nw; ++i) r += sh[i];
  }
  return r;
}

template <typename R>
__device__ __forceinline__ cx<double> ld(const R* psi, uint64_t x) {
  const cx<R> v = load1(psi, x);
  return {double(v.re), double(v.im)};
}

// One flip-mask group: partial[blockIdx.x] = this workgroup's share.
template <typename R>
__global__ void __launch_bounds__(kRedThreads)
    k_expect_group(const R* __restrict__ psi, uint64_t work, uint64_t flip, int hbit,
                   const GTerm* __restrict__ terms, int nterms, double* __restrict__ partial) {
  __shared__ GTerm st[kLdsTerms];
  __shared__ double sh[kRedThreads / 64];
  const int nl = min(nterms, kLdsTerms);
  for (int i = threadIdx.x; i < nl; i += blockDim.x) st[i] = terms[i];
  __syncthreads();
  double acc = 0.0;
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < work; i += stride) {
    if (flip == 0) {
      const cx<double> a = ld(psi, i);
      double c = 0.0;
      for (int k = 0; k < nterms; ++k) {
        const GTerm t = k < kLdsTerms ? st[k] : terms[k];
        c += (__popcll(i & t.z) & 1) ? -t.re : t.re;
      }
      acc += (a.re * a.re + a.im * a.im) * c;
    } else {
      const uint64_t lo = i & ((uint64_t(1) << hbit) - 1);
      const uint64_t x = ((i >> hbit) << (hbit + 1)) | lo;
      const uint64_t y = x ^ flip;
      const cx<double> a = ld(psi, x), b = ld(psi, y);
      // w = conj(b) * a
      const double wr = b.re * a.re + b.im * a.im;
      const double wi = b.re * a.im - b.im * a.re;
      double cr = 0.0, ci = 0.0;
      for (int k = 0; k < nterms; ++k) {
        const GTerm t = k < kLdsTerms ? st[k] : terms[k];
        const bool neg = __popcll(x & t.z) & 1;
        cr += neg ? -t.re : t.re;
        ci += neg ? -t.im : t.im;
      }
      acc += 2.0 * (wr * cr - wi * ci);
    }
  }
  const double r = block_reduce_sum(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = r;
}

template <typename R>
__global__ void __launch_bounds__(kRedThreads)
    k_inner(const R* __restrict__ a, const R* __restrict__ b, uint64_t N, double* __restrict__ partial) {
  __shared__ double sh[kRedThreads / 64];
  double re = 0.0, im = 0.0;
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < N; i += stride) {
    const cx<double> u = ld(a, i), v = ld(b, i);
    re += u.re * v.re + u.im * v.im;
    im += u.re * v.im - u.im * v.re;
  }
  double r = block_reduce_sum(re, sh);
  __syncthreads();
  double s = block_reduce_sum(im, sh);
  if (threadIdx.x == 0) {
    partial[2 * blockIdx.x] = r;
    partial[2 * blockIdx.x + 1] = s;
  }
}

// Fixed-order sum of `count` partials with stride `stride` into out[0].
__global__ void __launch_bounds__(kRedThreads)
    k_sum_partials(const double* __restrict__ partial, int count, int stride, double* __restrict__ out) {
  __shared__ double sh[kRedThreads / 64];
  double acc = 0.0;
  for (int i = threadIdx.x; i < count; i += blockDim.x) acc += partial[size_t(i) * stride];
  const double r = block_reduce_sum(acc, sh);
  if (threadIdx.x == 0) out[0] = r;
}

// Marginal probability (section 4.2.2): sum of |psi_x|^2 over the 2^(n - m)
// indices x whose m measured bits are fixed. Index j of the free bits becomes
// x by inserting a zero at each measured position (ascending), then OR-ing the
// requested values; partial[blockIdx.x] = this workgroup's FP64 share.
template <typename R>
__global__ void __launch_bounds__(kRedThreads)
    k_marginal(const R* __restrict__ psi, uint64_t work, InsertPos ins, uint64_t vals,
               double* __restrict__ partial) {
  __shared__ double sh[kRedThreads / 64];
  double acc = 0.0;
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  for (uint64_t j = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; j < work; j += stride) {
    uint64_t x = j;
    for (int k = 0; k < ins.m; ++k) {
      const int q = ins.pos[k];
      x = ((x >> q) << (q + 1)) | (x & ((uint64_t(1) << q) - 1));
    }
    const cx<double> a = ld(psi, x | vals);
    acc += a.re * a.re + a.im * a.im;
  }
  const double r = block_reduce_sum(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = r;
}

namespace {

int red_blocks(uint64_t work) {
  const uint64_t b = (work + kRedThreads * 4 - 1) / (kRedThreads * 4);
  return int(std::max<uint64_t>(1, std::min<uint64_t>(b, kMaxRedBlocks)));
}

}  // namespace

// Build term groups (by flip mask) as device-ready arrays.
void build_groups(const qsv_observable* o, std::vector<Group>& groups, std::vector<GTerm>& terms) {
  std::map<uint64_t, std::vector<GTerm>> by;
  for (const auto& t : o->terms) {
    // i^nY
    static const double pr[4] = {1, 0, -1, 0}, pi[4] = {0, 1, 0, -1};
    GTerm g{t.coef * pr[t.ny & 3], t.coef * pi[t.ny & 3], t.zmask};
    by[t.flip].push_back(g);
  }
  groups.clear();
  terms.clear();
  for (auto& kv : by) {
    groups.push_back({kv.first, int(terms.size()), int(kv.second.size())});
    terms.insert(terms.end(), kv.second.begin(), kv.second.end());
  }
}

namespace {

template <typename R>
int expectation_t(qsv_state* s, const qsv_observable* o, double* out) {
  std::vector<Group> groups;
  std::vector<GTerm> terms;
  build_groups(o, groups, terms);
  if (groups.empty()) {
    *out = 0.0;
    return QSV_OK;
  }
  const int n = s->n;
  // one block count for every group so the partials form a dense array
  const int B = red_blocks(dim(n) / 2);
  const size_t need = size_t(groups.size()) * B + 1 + (terms.size() * sizeof(GTerm) + 7) / 8;
  int rc = ensure_reduce_scratch(s, need);
  if (rc) return rc;
  double* partial = s->red;
  GTerm* dterms = reinterpret_cast<GTerm*>(s->red + size_t(groups.size()) * B + 1);
  QSV_HIP_CHECK(hipMemcpyAsync(dterms, terms.data(), terms.size() * sizeof(GTerm),
                               hipMemcpyHostToDevice, s->stream));
  for (size_t g = 0; g < groups.size(); ++g) {
    const uint64_t f = groups[g].flip;
    const int hbit = f ? 63 - __builtin_clzll(f) : 0;
    const uint64_t work = f ? dim(n) / 2 : dim(n);
    double* p = partial + g * B;
    ProfScope ps("expect", 2.0 * sizeof(R) * double(dim(n)), s->stream);
    hipLaunchKernelGGL((k_expect_group<R>), dim3(B), dim3(kRedThreads), 0, s->stream,
                       static_cast<const R*>(s->ptr), work, f, hbit, dterms + groups[g].begin,
                       groups[g].count, p);
    QSV_HIP_CHECK(hipGetLastError());
  }
  double* res = partial + groups.size() * B;
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kRedThreads), 0, s->stream, partial,
                     int(groups.size() * B), 1, res);
  QSV_HIP_CHECK(hipGetLastError());
  QSV_HIP_CHECK(hipMemcpyAsync(s->red_host, res, sizeof(double), hipMemcpyDeviceToHost, s->stream));
  QSV_HIP_CHECK(hipStreamSynchronize(s->stream));
  *out = s->red_host[0];
  return QSV_OK;
}

template <typename R>
int inner_t(const qsv_state* bra, const qsv_state* ket, qsv_state* scratch_owner, double* re,
            double* im) {
  const uint64_t N = dim(bra->n);
  const int nb = red_blocks(N);
  int rc = ensure_reduce_scratch(scratch_owner, size_t(2 * nb + 2));
  if (rc) return rc;
  double* partial = scratch_owner->red;
  hipStream_t st = scratch_owner->stream;
  hipLaunchKernelGGL((k_inner<R>), dim3(nb), dim3(kRedThreads), 0, st,
                     static_cast<const R*>(bra->ptr), static_cast<const R*>(ket->ptr), N, partial);
  QSV_HIP_CHECK(hipGetLastError());
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kRedThreads), 0, st, partial, nb, 2,
                     partial + 2 * nb);
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kRedThreads), 0, st, partial + 1, nb, 2,
                     partial + 2 * nb + 1);
  QSV_HIP_CHECK(hipGetLastError());
  QSV_HIP_CHECK(hipMemcpyAsync(scratch_owner->red_host, partial + 2 * nb, 2 * sizeof(double),
                               hipMemcpyDeviceToHost, st));
  QSV_HIP_CHECK(hipStreamSynchronize(st));
  *re = scratch_owner->red_host[0];
  *im = scratch_owner->red_host[1];
  return QSV_OK;
}

template <typename R>
int marginal_t(qsv_state* s, const InsertPos& ins, uint64_t vals, double* out) {
  const uint64_t work = dim(s->n - ins.m);
  const int nb = red_blocks(work);
  int rc = ensure_reduce_scratch(s, size_t(nb + 1));
  if (rc) return rc;
  double* partial = s->red;
  hipLaunchKernelGGL((k_marginal<R>), dim3(nb), dim3(kRedThreads), 0, s->stream,
                     static_cast<const R*>(s->ptr), work, ins, vals, partial);
  QSV_HIP_CHECK(hipGetLastError());
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kRedThreads), 0, s->stream, partial, nb, 1,
                     partial + nb);
  QSV_HIP_CHECK(hipGetLastError());
  QSV_HIP_CHECK(hipMemcpyAsync(s->red_host, partial + nb, sizeof(double), hipMemcpyDeviceToHost,
                               s->stream));
  QSV_HIP_CHECK(hipStreamSynchronize(s->stream));
  *out = s->red_host[0];
  return QSV_OK;
}

}  // namespace

int expectation_impl(qsv_state* s, const qsv_observable* o, double* out) {
  return s->dtype == QSV_C64 ? expectation_t<float>(s, o, out) : expectation_t<double>(s, o, out);
}

}  // namespace qsv

using namespace qsv;

extern "C" {

int qsv_norm2(const qsv_state* s_in, double* out) {
  clear_error();
  int rc = check_state(s_in);
  if (rc) return rc;
  if (!out) return fail(QSV_EINVAL, "null output");
  qsv_state* s = const_cast<qsv_state*>(s_in);  // scratch only; amplitudes untouched
  qsv_observable id;
  id.n = s->n;
  id.terms.push_back({1.0, 0, 0, 0});
  return expectation_impl(s, &id, out);
}

int qsv_marginal_probability(const qsv_state* s_in, const int* values, double* out) {
  clear_error();
  int rc = check_state(s_in);
  if (rc) return rc;
  if (!values || !out) return fail(QSV_EINVAL, "null argument");
  InsertPos ins;
  uint64_t vals = 0;
  for (int q = 0; q < s_in->n; ++q) {
    if (values[q] == 2) continue;
    if (values[q] != 0 && values[q] != 1) return fail(QSV_EINVAL, "values must be 0, 1 or 2");
    ins.pos[ins.m++] = q;  // ascending
    vals |= uint64_t(values[q]) << q;
  }
  qsv_state* s = const_cast<qsv_state*>(s_in);  // scratch only; amplitudes untouched
  return s->dtype == QSV_C64 ? marginal_t<float>(s, ins, vals, out)
                             : marginal_t<double>(s, ins, vals, out);
}

int qsv_inner(const qsv_state* bra, const qsv_state* ket, double* re, double* im) {
  clear_error();
  int rc = check_state(bra);
  if (rc) return rc;
  if ((rc = check_state(ket))) return rc;
  if (!re || !im) return fail(QSV_EINVAL, "null output");
  if (bra->n != ket->n) return fail(QSV_ERANGE, "qubit counts differ");
  if (bra->dtype != ket->dtype) return fail(QSV_EDTYPE, "dtypes differ");
  if (bra->stream != ket->stream) QSV_HIP_CHECK(hipStreamSynchronize(bra->stream));
  qsv_state* owner = const_cast<qsv_state*>(ket);
  return bra->dtype == QSV_C64 ? inner_t<float>(bra, ket, owner, re, im)
                               : inner_t<double>(bra, ket, owner, re, im);
}

int qsv_observable_create(int n, qsv_observable** out) {
  clear_error();
  if (!out) return fail(QSV_EINVAL, "null output handle");
  *out = nullptr;
  if (n < 1 || n > 34) return fail(QSV_ERANGE, "qubit count %d outside [1, 34]", n);
  qsv_observable* o = new (std::nothrow) qsv_observable();
  if (!o) return fail(QSV_ENOMEM, "host allocation failed");
  o->n = n;
  *out = o;
  return QSV_OK;
}

int qsv_observable_free(qsv_observable* o) {
  clear_error();
  delete o;
  return QSV_OK;
}

int qsv_observable_add_term(qsv_observable* o, double coef, const int* qubits, const int* pauli_ids,
                            int w) {
  clear_error();
  if (!o) return fail(QSV_EINVAL, "null observable");
  if (w < 0) return fail(QSV_EINVAL, "negative term length");
  if (w > 0 && (!qubits || !pauli_ids)) return fail(QSV_EINVAL, "null term arrays");
  qsv_observable::Term t{coef, 0, 0, 0};
  uint64_t used = 0;
  for (int j = 0; j < w; ++j) {
    const int q = qubits[j], p = pauli_ids[j];
    if (q < 0 || q >= o->n) return fail(QSV_ERANGE, "qubit %d out of range for %d qubits", q, o->n);
    if (p < 0 || p > 3) return fail(QSV_EINVAL, "pauli id %d not in 0..3", p);
    if (used >> q & 1) return fail(QSV_EDUP, "qubit %d listed twice in a term", q);
    used |= uint64_t(1) << q;
    const uint64_t b = uint64_t(1) << q;
    if (p == 1 || p == 2) t.flip |= b;
    if (p == 2 || p == 3) t.zmask |= b;
    if (p == 2) t.ny++;
  }
  o->drop_plans();
  o->terms.push_back(t);
  return QSV_OK;
}

int qsv_observable_passes(const qsv_observable* o, qsv_dtype dtype, int* passes) {
  clear_error();
  if (!o) return fail(QSV_EINVAL, "null observable");
  if (!passes) return fail(QSV_EINVAL, "null output");
  if (dtype != QSV_C64 && dtype != QSV_C128) return fail(QSV_EDTYPE, "unknown dtype");
  *passes = expectation_passes(o, dtype);
  return QSV_OK;
}

int qsv_observable_info(const qsv_observable* o, int* n, int* terms, int* groups) {
  clear_error();
  if (!o) return fail(QSV_EINVAL, "null observable");
  if (n) *n = o->n;
  if (terms) *terms = int(o->terms.size());
  if (groups) {
    std::vector<Group> g;
    std::vector<GTerm> t;
    build_groups(o, g, t);
    *groups = int(g.size());
  }
  return QSV_OK;
}

int qsv_expectation(const qsv_state* s_in, const qsv_observable* o, double* out) {
  clear_error();
  int rc = check_state(s_in);
  if (rc) return rc;
  if (!o) return fail(QSV_EINVAL, "null observable");
  if (!out) return fail(QSV_EINVAL, "null output");
  if (o->n != s_in->n) return fail(QSV_ERANGE, "observable has %d qubits, state %d", o->n, s_in->n);
  return expectation_tiled(const_cast<qsv_state*>(s_in), o, out);
}

int qsv_expectation_noalloc(const qsv_state* s_in, const qsv_observable* o, double* out) {
  clear_error();
  int rc = check_state(s_in);
  if (rc) return rc;
  if (!o) return fail(QSV_EINVAL, "null observable");
  if (!out) return fail(QSV_EINVAL, "null output");
  if (o->n != s_in->n) return fail(QSV_ERANGE, "observable has %d qubits, state %d", o->n, s_in->n);
  return expectation_noalloc(const_cast<qsv_state*>(s_in), o, out);
}

}  // extern "C"
