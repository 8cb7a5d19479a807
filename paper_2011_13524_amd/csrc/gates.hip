// Gate application kernels and their dispatch (section 4.3.2 basic gates,
// controlled gates, diagonal gates; section 4.3.4 named gates; cost model of
// section 4.3.2 and section 5.1).
//
// Every kernel enumerates B0, the indices whose gate bits are zero, from a
// dense thread counter by inserting zero bits (section 5.2), so a launch covers
// exactly the amplitudes the gate touches:
//   k_pair   two amplitudes per B0 element (one-qubit gates, X/CNOT, SWAP):
//            2 * 2^(n-m) amplitudes read and written, m = target + controls
//   k_scale  one amplitude per element of a subspace (Z, CZ, phases): only the
//            amplitudes the phase changes are touched
//   k_diag   diagonal k-qubit gates: every control-matching amplitude once
//   k_dense  dense k-qubit gates (k <= 5): 2^k amplitudes per B0 element,
//            gate matrix staged in LDS and broadcast to all lanes
// Each thread owns VEC consecutive B0 elements when the lowest inserted bit
// allows it, so loads and stores are 16-byte vectors and a wavefront covers a
// contiguous span.
#include <algorithm>

#include "dev_common.h"
#include "prof.h"
#include "qsv_internal.h"

namespace qsv {

constexpr int kMaxPos = 36;

enum PairKind { PK_DENSE = 0, PK_DIAG = 1, PK_SWAP = 2 };

template <typename R>
struct PairArgs {
  uint64_t nthreads;
  uint64_t or_mask;  // control values OR-ed into every B0 element
  uint64_t offA, offB;
  M2<R> u;
  int m;
  int pos[kMaxPos];
};

template <typename R, int VEC, int KIND>
__device__ __forceinline__ void pair_update(cx<R>* va, cx<R>* vb, const M2<R>& u) {
#pragma unroll
  for (int v = 0; v < VEC; ++v) {
    const cx<R> a = va[v], b = vb[v];
    if constexpr (KIND == PK_DENSE) {
      va[v] = cfma(u.m00, a, u.m01 * b);
      vb[v] = cfma(u.m10, a, u.m11 * b);
    } else if constexpr (KIND == PK_DIAG) {
      va[v] = u.m00 * a;
      vb[v] = u.m11 * b;
    } else {
      va[v] = b;
      vb[v] = a;
    }
  }
}

template <typename R, int VEC, int KIND>
__global__ void __launch_bounds__(256) k_pair(R* __restrict__ psi, const PairArgs<R> a) {
  // grid-stride: launches stay within 2^32 work-items for any state size
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  for (uint64_t t = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < a.nthreads; t += stride) {
    const uint64_t x0 = insert_zeros(t * VEC, a.pos, a.m) | a.or_mask;
    cx<R> va[VEC], vb[VEC];
    AmpIO<R, VEC>::load(psi, x0 + a.offA, va);
    AmpIO<R, VEC>::load(psi, x0 + a.offB, vb);
    pair_update<R, VEC, KIND>(va, vb, a.u);
    AmpIO<R, VEC>::store(psi, x0 + a.offA, va);
    AmpIO<R, VEC>::store(psi, x0 + a.offB, vb);
  }
}

// complex64 one-qubit gate on qubit 0: the pair (x0, x0 + 1) is one 16-byte vector.
template <int KIND>
__global__ void __launch_bounds__(256) k_pair_adj(float* __restrict__ psi, const PairArgs<float> a) {
  // grid-stride: launches stay within 2^32 work-items for any state size
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  for (uint64_t t = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < a.nthreads; t += stride) {
    const uint64_t x0 = insert_zeros(t, a.pos, a.m) | a.or_mask;
    cx<float> v[2];
    AmpIO<float, 2>::load(psi, x0, v);
    pair_update<float, 1, KIND>(&v[0], &v[1], a.u);
    AmpIO<float, 2>::store(psi, x0, v);
  }
}

// One-qubit gate on qubit t, streamed: wavefront w reads and writes the
// contiguous 16-byte vectors 64 w .. 64 w + 63 (one amplitude pair for
// complex64, one amplitude for complex128 per vector), so every access
// instruction covers whole cache lines. Dense / exchange gates on a low qubit
// (the pair partner within the same wavefront: lane XOR dl) take the
// partner's values by a lane shuffle; diagonal gates need no partner and run
// on any qubit. Amplitudes whose index does not match the controls
// (index & cm) == cv keep their value (both members of a pair agree: controls
// are not the target). nvec (the vector count) is a multiple of 64.
template <typename R, int KIND>
__global__ void __launch_bounds__(256) k_pair_lane(R* __restrict__ psi, const PairArgs<R> a, int t, uint64_t nvec,
                                                   uint64_t cm, uint64_t cv) {
  constexpr int V = sizeof(R) == 4 ? 2 : 1;  // amplitudes per vector
  const int dl = KIND == PK_DIAG ? 0 : (1 << t) / V;
  const bool upper = (threadIdx.x & 63) & dl;  // this lane holds the bit-t = 1 members
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  for (uint64_t v = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; v < nvec; v += stride) {
    cx<R> x[V];
    AmpIO<R, V>::load(psi, v * V, x);
#pragma unroll
    for (int k = 0; k < V; ++k) {
      const uint64_t idx = v * V + k;
      const bool on = (idx & cm) == cv;
      cx<R> r;
      if constexpr (KIND == PK_DIAG) {
        r = (((idx >> t) & 1) ? a.u.m11 : a.u.m00) * x[k];
      } else {
        const cx<R> y{__shfl_xor(x[k].re, dl, 64), __shfl_xor(x[k].im, dl, 64)};
        if constexpr (KIND == PK_DENSE) {
          r = upper ? cfma(a.u.m10, y, a.u.m11 * x[k]) : cfma(a.u.m00, x[k], a.u.m01 * y);
        } else {
          r = y;
        }
      }
      x[k] = {on ? r.re : x[k].re, on ? r.im : x[k].im};
    }
    AmpIO<R, V>::store(psi, v * V, x);
  }
}

// One-entry phase (x *= c where (x & mask) == pattern) streamed over every
// 16-byte vector: for masks with a low bit, whose strided accesses would
// touch every line anyway. nvec is a multiple of 64 (whole wavefronts).
template <typename R>
__global__ void __launch_bounds__(256) k_scale_lane(R* __restrict__ psi, cx<R> c, uint64_t mask, uint64_t pattern,
                                                    uint64_t nvec) {
  constexpr int V = sizeof(R) == 4 ? 2 : 1;
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  for (uint64_t v = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; v < nvec; v += stride) {
    cx<R> x[V];
    AmpIO<R, V>::load(psi, v * V, x);
#pragma unroll
    for (int k = 0; k < V; ++k) {
      const cx<R> r = c * x[k];
      const bool on = ((v * V + k) & mask) == pattern;
      x[k] = {on ? r.re : x[k].re, on ? r.im : x[k].im};
    }
    AmpIO<R, V>::store(psi, v * V, x);
  }
}

template <typename R>
struct ScaleArgs {
  uint64_t nthreads;
  uint64_t pattern;
  cx<R> c;
  int m;
  int pos[kMaxPos];
};

template <typename R, int VEC>
__global__ void __launch_bounds__(256) k_scale(R* __restrict__ psi, const ScaleArgs<R> a) {
  // grid-stride: launches stay within 2^32 work-items for any state size
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  for (uint64_t t = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < a.nthreads; t += stride) {
    const uint64_t x = insert_zeros(t * VEC, a.pos, a.m) | a.pattern;
    cx<R> v[VEC];
    AmpIO<R, VEC>::load(psi, x, v);
  #pragma unroll
    for (int j = 0; j < VEC; ++j) v[j] = a.c * v[j];
    AmpIO<R, VEC>::store(psi, x, v);
  }
}

template <typename R>
struct DiagArgs {
  uint64_t nthreads;
  uint64_t or_mask;
  cx<R> d[32];
  int k;
  int tq[5];
  int m;
  int pos[kMaxPos];
};

template <typename R, int VEC>
__global__ void __launch_bounds__(256) k_diag(R* __restrict__ psi, const DiagArgs<R> a) {
  // grid-stride: launches stay within 2^32 work-items for any state size
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  for (uint64_t t = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < a.nthreads; t += stride) {
    const uint64_t x = insert_zeros(t * VEC, a.pos, a.m) | a.or_mask;
    cx<R> v[VEC];
    AmpIO<R, VEC>::load(psi, x, v);
  #pragma unroll
    for (int j = 0; j < VEC; ++j) {
      const uint64_t xj = x + j;
      int idx = 0;
      for (int b = 0; b < a.k; ++b) idx |= int((xj >> a.tq[b]) & 1) << b;
      v[j] = a.d[idx] * v[j];
    }
    AmpIO<R, VEC>::store(psi, x, v);
  }
}

template <typename R, int K>
struct DenseArgs {
  uint64_t nthreads;
  uint64_t or_mask;
  uint64_t off[1 << K];  // s(bin(i)): offset of the i-th element of B1
  int m;
  int pos[kMaxPos];
};

template <typename R, int K>
__global__ void __launch_bounds__(256) k_dense(R* __restrict__ psi, const cx<R>* __restrict__ mat,
                                               const DenseArgs<R, K> a) {
  constexpr int D = 1 << K;
  __shared__ cx<R> sm[D * D];
  for (int i = threadIdx.x; i < D * D; i += blockDim.x) sm[i] = mat[i];
  __syncthreads();
  // grid-stride: launches stay within 2^32 work-items for any state size
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  for (uint64_t t = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < a.nthreads; t += stride) {
    const uint64_t x0 = insert_zeros(t, a.pos, a.m) | a.or_mask;
    cx<R> v[D];
  #pragma unroll
    for (int c = 0; c < D; ++c) v[c] = load1(psi, x0 + a.off[c]);
  #pragma unroll
    for (int r = 0; r < D; ++r) {
      cx<R> acc = {R(0), R(0)};
  #pragma unroll
      for (int c = 0; c < D; ++c) acc = cfma(sm[r * D + c], v[c], acc);
      store1(psi, x0 + a.off[r], acc);
    }
  }
}

// Dense gate on K = 6..10 targets (section 4.3.2 for any number of targets;
// the temporal vector of 2^K amplitudes sits in shared memory, as section 5.5
// does for wide gates). One workgroup per B0 element x0 (grid-stride over
// them): the 2^K amplitudes x0 + s(c) are gathered into LDS in FP64, then
// thread r forms output r = sum_c M[r][c] v[c] from the matrix stored
// transposed (mt[c * 2^K + r]: the lanes of a wavefront read consecutive
// entries) and writes it to x0 + s(r). Every read of the group comes from LDS,
// so the writes need no further ordering.
struct DenseBigArgs {
  uint64_t ngroups;
  uint64_t or_mask;
  int k;
  int tq[10];
  int m;
  int pos[kMaxPos];
};

__device__ __forceinline__ uint64_t spread_bits(uint32_t c, const int* tq, int k) {
  uint64_t o = 0;
  for (int j = 0; j < k; ++j) o |= uint64_t((c >> j) & 1) << tq[j];
  return o;
}

template <typename R>
__global__ void __launch_bounds__(256) k_dense_big(R* __restrict__ psi, const cd* __restrict__ mt,
                                                   const DenseBigArgs a) {
  extern __shared__ __align__(16) char smem[];
  cx<double>* v = reinterpret_cast<cx<double>*>(smem);
  const int D = 1 << a.k;
  for (uint64_t grp = blockIdx.x; grp < a.ngroups; grp += gridDim.x) {
    const uint64_t x0 = insert_zeros(grp, a.pos, a.m) | a.or_mask;
    __syncthreads();  // the previous group's LDS reads are done
    for (int c = threadIdx.x; c < D; c += blockDim.x) {
      const cx<R> x = load1(psi, x0 + spread_bits(uint32_t(c), a.tq, a.k));
      v[c] = {double(x.re), double(x.im)};
    }
    __syncthreads();
    for (int r = threadIdx.x; r < D; r += blockDim.x) {
      double ar = 0.0, ai = 0.0;
      for (int c = 0; c < D; ++c) {
        const cd m = mt[size_t(c) * D + r];
        const cx<double> x = v[c];
        ar = fma(m.re, x.re, fma(-m.im, x.im, ar));
        ai = fma(m.re, x.im, fma(m.im, x.re, ai));
      }
      store1(psi, x0 + spread_bits(uint32_t(r), a.tq, a.k), cx<R>{R(ar), R(ai)});
    }
  }
}

// ------------------------------------------------------------------ host side

namespace {

inline bool ceq(cd a, double re, double im = 0.0) { return a.re == re && a.im == im; }

template <typename R>
inline cx<R> to_dev(cd a) {
  return {R(a.re), R(a.im)};
}

int launch_grid(uint64_t nthreads, dim3* grid) {
  // at most 2^22 workgroups of 256 (2^30 work-items); kernels stride over the rest
  const uint64_t blocks = std::min<uint64_t>((nthreads + 255) / 256, uint64_t(1) << 22);
  *grid = dim3(unsigned(std::max<uint64_t>(blocks, 1)));
  return QSV_OK;
}

void sort_positions(uint64_t mask, InsertPos* ip) {
  ip->m = 0;
  for (int q = 0; q < 64; ++q)
    if (mask >> q & 1) ip->pos[ip->m++] = q;
}

int lowest_bit(uint64_t mask) {
  if (!mask) return 64;
  return __builtin_ctzll(mask);
}

// Pick the widest per-thread vector allowed by the lowest inserted bit and the
// number of B0 elements.
int pick_vec(qsv_dtype dt, int lowest, int free_bits) {
  int v = 1;
  // one 16-byte vector per member and thread: a wavefront's access covers
  // 1 KiB of whole lines once the pair distance reaches a line
  const int maxlog = dt == QSV_C64 ? 1 : 0;
  int lg = std::min(std::min(lowest, maxlog), free_bits);
  if (lg < 0) lg = 0;
  v = 1 << lg;
  return v;
}

template <typename R>
int launch_pair_t(qsv_state* s, uint64_t ins_mask, uint64_t or_mask, uint64_t offA, uint64_t offB,
                  const cd* u, int kind) {
  PairArgs<R> a{};
  InsertPos ip;
  sort_positions(ins_mask, &ip);
  if (ip.m > kMaxPos) return fail(QSV_ERANGE, "too many qubits");
  a.m = ip.m;
  for (int j = 0; j < ip.m; ++j) a.pos[j] = ip.pos[j];
  a.or_mask = or_mask;
  a.offA = offA;
  a.offB = offB;
  a.u = {to_dev<R>(u[0]), to_dev<R>(u[1]), to_dev<R>(u[2]), to_dev<R>(u[3])};
  const int free_bits = s->n - ip.m;
  R* psi = static_cast<R*>(s->ptr);
  dim3 grid;
  int rc;
  // no controls: streamed 16-byte vectors -- diagonal gates on any qubit,
  // dense and exchange gates on the low qubits whose pair partner sits in the
  // same wavefront (complex64: qubits 1..6, complex128: 0..5)
  // and (one control) gates on those low qubits, whose strided pair accesses
  // would waste most of each line
  {
    constexpr int V = sizeof(R) == 4 ? 2 : 1;
    const bool pairs = offA == 0 && offB != 0 && (offB & (offB - 1)) == 0 && (ins_mask & offB) &&
                       (or_mask & ~(ins_mask & ~offB)) == 0;
    const int t = pairs ? __builtin_ctzll(offB) : -1;
    const uint64_t cmask = pairs ? ins_mask & ~offB : 0;
    const int nctrl = __builtin_popcountll(cmask);
    const uint64_t nvec = (uint64_t(1) << s->n) / V;
    const bool low = sizeof(R) == 4 ? (t >= 1 && t <= 6) : (t >= 0 && t <= 5);
    if (pairs && nvec % 64 == 0 && ((nctrl == 0 && (kind == PK_DIAG || low)) || (nctrl == 1 && low))) {
      if ((rc = launch_grid(nvec, &grid))) return rc;
      ProfScope ps("pair", 4.0 * sizeof(R) * 2 * double(uint64_t(1) << free_bits), s->stream);
      if (kind == PK_DENSE)
        hipLaunchKernelGGL((k_pair_lane<R, PK_DENSE>), grid, dim3(256), 0, s->stream, psi, a, t, nvec, cmask,
                           or_mask);
      else if (kind == PK_DIAG)
        hipLaunchKernelGGL((k_pair_lane<R, PK_DIAG>), grid, dim3(256), 0, s->stream, psi, a, t, nvec, cmask,
                           or_mask);
      else
        hipLaunchKernelGGL((k_pair_lane<R, PK_SWAP>), grid, dim3(256), 0, s->stream, psi, a, t, nvec, cmask,
                           or_mask);
      QSV_HIP_CHECK(hipGetLastError());
      return QSV_OK;
    }
  }
  // complex64, gate on qubit 0 (offsets 0 and 1): one 16-byte vector per pair
  if constexpr (sizeof(R) == 4) {
    if (offA == 0 && offB == 1) {
      a.nthreads = uint64_t(1) << free_bits;
      if ((rc = launch_grid(a.nthreads, &grid))) return rc;
      ProfScope ps("pair", 4.0 * sizeof(R) * 2 * double(a.nthreads), s->stream);
      if (kind == PK_DENSE)
        hipLaunchKernelGGL(k_pair_adj<PK_DENSE>, grid, dim3(256), 0, s->stream, psi, a);
      else if (kind == PK_DIAG)
        hipLaunchKernelGGL(k_pair_adj<PK_DIAG>, grid, dim3(256), 0, s->stream, psi, a);
      else
        hipLaunchKernelGGL(k_pair_adj<PK_SWAP>, grid, dim3(256), 0, s->stream, psi, a);
      QSV_HIP_CHECK(hipGetLastError());
      return QSV_OK;
    }
  }
  const int vec = pick_vec(s->dtype, lowest_bit(ins_mask), free_bits);
  a.nthreads = (uint64_t(1) << free_bits) / vec;
  if ((rc = launch_grid(a.nthreads, &grid))) return rc;
  ProfScope ps("pair", 4.0 * sizeof(R) * 2 * double(uint64_t(1) << free_bits), s->stream);
#define QSV_PAIR_LAUNCH(V)                                                                   \
  do {                                                                                       \
    if (kind == PK_DENSE)                                                                    \
      hipLaunchKernelGGL((k_pair<R, V, PK_DENSE>), grid, dim3(256), 0, s->stream, psi, a);   \
    else if (kind == PK_DIAG)                                                                \
      hipLaunchKernelGGL((k_pair<R, V, PK_DIAG>), grid, dim3(256), 0, s->stream, psi, a);    \
    else                                                                                     \
      hipLaunchKernelGGL((k_pair<R, V, PK_SWAP>), grid, dim3(256), 0, s->stream, psi, a);    \
  } while (0)
  if (vec == 4) {
    if constexpr (sizeof(R) == 4) QSV_PAIR_LAUNCH(4);
  } else if (vec == 2) {
    QSV_PAIR_LAUNCH(2);
  } else {
    QSV_PAIR_LAUNCH(1);
  }
#undef QSV_PAIR_LAUNCH
  QSV_HIP_CHECK(hipGetLastError());
  return QSV_OK;
}

int launch_pair(qsv_state* s, uint64_t ins_mask, uint64_t or_mask, uint64_t offA, uint64_t offB,
                const cd* u, int kind) {
  return s->dtype == QSV_C64 ? launch_pair_t<float>(s, ins_mask, or_mask, offA, offB, u, kind)
                             : launch_pair_t<double>(s, ins_mask, or_mask, offA, offB, u, kind);
}

template <typename R>
int launch_scale_t(qsv_state* s, uint64_t mask, uint64_t pattern, cd c) {
  {
    // a low mask bit: stream whole lines instead of strided 8- / 16-byte accesses
    constexpr int V = sizeof(R) == 4 ? 2 : 1;
    const uint64_t nvec = (uint64_t(1) << s->n) / V;
    if (mask && __builtin_ctzll(mask) < (sizeof(R) == 4 ? 3 : 2) && nvec % 64 == 0) {
      dim3 grid;
      int rc;
      if ((rc = launch_grid(nvec, &grid))) return rc;
      const int m = __builtin_popcountll(mask);
      ProfScope ps("scale", 2.0 * sizeof(R) * 2 * double(uint64_t(1) << (s->n - m)), s->stream);
      hipLaunchKernelGGL((k_scale_lane<R>), grid, dim3(256), 0, s->stream, static_cast<R*>(s->ptr), to_dev<R>(c),
                         mask, pattern, nvec);
      QSV_HIP_CHECK(hipGetLastError());
      return QSV_OK;
    }
  }
  ScaleArgs<R> a{};
  InsertPos ip;
  sort_positions(mask, &ip);
  a.m = ip.m;
  for (int j = 0; j < ip.m; ++j) a.pos[j] = ip.pos[j];
  a.pattern = pattern;
  a.c = to_dev<R>(c);
  const int free_bits = s->n - ip.m;
  const int vec = pick_vec(s->dtype, lowest_bit(mask), free_bits);
  a.nthreads = (uint64_t(1) << free_bits) / vec;
  dim3 grid;
  int rc;
  if ((rc = launch_grid(a.nthreads, &grid))) return rc;
  R* psi = static_cast<R*>(s->ptr);
  ProfScope ps("scale", 2.0 * sizeof(R) * 2 * double(uint64_t(1) << free_bits), s->stream);
  if (vec == 4) {
    if constexpr (sizeof(R) == 4)
      hipLaunchKernelGGL((k_scale<R, 4>), grid, dim3(256), 0, s->stream, psi, a);
  } else if (vec == 2) {
    hipLaunchKernelGGL((k_scale<R, 2>), grid, dim3(256), 0, s->stream, psi, a);
  } else {
    hipLaunchKernelGGL((k_scale<R, 1>), grid, dim3(256), 0, s->stream, psi, a);
  }
  QSV_HIP_CHECK(hipGetLastError());
  return QSV_OK;
}

template <typename R>
int launch_diag_t(qsv_state* s, const cd* d, const int* targets, int k, uint64_t cmask,
                  uint64_t cval) {
  DiagArgs<R> a{};
  InsertPos ip;
  sort_positions(cmask, &ip);
  a.m = ip.m;
  for (int j = 0; j < ip.m; ++j) a.pos[j] = ip.pos[j];
  a.or_mask = cval;
  a.k = k;
  for (int j = 0; j < k; ++j) a.tq[j] = targets[j];
  for (int j = 0; j < (1 << k); ++j) a.d[j] = to_dev<R>(d[j]);
  const int free_bits = s->n - ip.m;
  const int vec = pick_vec(s->dtype, lowest_bit(cmask), free_bits);
  a.nthreads = (uint64_t(1) << free_bits) / vec;
  dim3 grid;
  int rc;
  if ((rc = launch_grid(a.nthreads, &grid))) return rc;
  R* psi = static_cast<R*>(s->ptr);
  ProfScope ps("diag", 2.0 * sizeof(R) * 2 * double(uint64_t(1) << free_bits), s->stream);
  if (vec == 4) {
    if constexpr (sizeof(R) == 4)
      hipLaunchKernelGGL((k_diag<R, 4>), grid, dim3(256), 0, s->stream, psi, a);
  } else if (vec == 2) {
    hipLaunchKernelGGL((k_diag<R, 2>), grid, dim3(256), 0, s->stream, psi, a);
  } else {
    hipLaunchKernelGGL((k_diag<R, 1>), grid, dim3(256), 0, s->stream, psi, a);
  }
  QSV_HIP_CHECK(hipGetLastError());
  return QSV_OK;
}

template <typename R, int K>
int launch_dense_k(qsv_state* s, const cd* mat, const int* targets, uint64_t cmask, uint64_t cval) {
  constexpr int D = 1 << K;
  DenseArgs<R, K> a{};
  uint64_t ins = cmask;
  for (int j = 0; j < K; ++j) ins |= uint64_t(1) << targets[j];
  InsertPos ip;
  sort_positions(ins, &ip);
  a.m = ip.m;
  for (int j = 0; j < ip.m; ++j) a.pos[j] = ip.pos[j];
  a.or_mask = cval;
  for (int i = 0; i < D; ++i) {
    uint64_t o = 0;
    for (int j = 0; j < K; ++j)
      if (i >> j & 1) o |= uint64_t(1) << targets[j];
    a.off[i] = o;
  }
  a.nthreads = uint64_t(1) << (s->n - ip.m);
  std::vector<cx<R>> hm(D * D);
  for (int i = 0; i < D * D; ++i) hm[i] = to_dev<R>(mat[i]);
  void* dmat = nullptr;
  int slot = 0;
  int rc = s->up.upload(hm.data(), hm.size() * sizeof(cx<R>), s->stream, &dmat, &slot);
  if (rc) return rc;
  dim3 grid;
  if ((rc = launch_grid(a.nthreads, &grid))) return rc;
  ProfScope ps("dense", 2.0 * sizeof(R) * 2 * D * double(a.nthreads), s->stream);
  hipLaunchKernelGGL((k_dense<R, K>), grid, dim3(256), 0, s->stream, static_cast<R*>(s->ptr),
                     static_cast<const cx<R>*>(dmat), a);
  QSV_HIP_CHECK(hipGetLastError());
  return s->up.release(slot, s->stream);
}

template <typename R>
int launch_dense_big(qsv_state* s, const cd* mat, const int* targets, int k, uint64_t cmask,
                     uint64_t cval) {
  const int D = 1 << k;
  DenseBigArgs a{};
  a.k = k;
  uint64_t ins = cmask;
  for (int j = 0; j < k; ++j) {
    a.tq[j] = targets[j];
    ins |= uint64_t(1) << targets[j];
  }
  InsertPos ip;
  sort_positions(ins, &ip);
  a.m = ip.m;
  for (int j = 0; j < ip.m; ++j) a.pos[j] = ip.pos[j];
  a.or_mask = cval;
  a.ngroups = uint64_t(1) << (s->n - ip.m);
  std::vector<cd> mt(size_t(D) * D);
  for (int r = 0; r < D; ++r)
    for (int c = 0; c < D; ++c) mt[size_t(c) * D + r] = mat[size_t(r) * D + c];
  const size_t bytes = mt.size() * sizeof(cd);
  if (s->big_cap < bytes) {
    QSV_HIP_CHECK(hipStreamSynchronize(s->stream));  // earlier gates may still read it
    if (s->big) (void)hipFree(s->big);
    s->big = nullptr;
    s->big_cap = 0;
    if (hipMalloc(&s->big, bytes) != hipSuccess) {
      s->big = nullptr;
      return fail(QSV_ENOMEM, "dense gate matrix (%zu bytes) allocation failed", bytes);
    }
    s->big_cap = bytes;
  }
  // stream-ordered after the kernels that read the previous matrix; the host
  // copy must outlive the transfer, so wait for it
  QSV_HIP_CHECK(hipMemcpyAsync(s->big, mt.data(), bytes, hipMemcpyHostToDevice, s->stream));
  QSV_HIP_CHECK(hipStreamSynchronize(s->stream));
  const unsigned grid = unsigned(std::min<uint64_t>(a.ngroups, 4096));
  ProfScope ps("dense", 2.0 * sizeof(R) * 2 * double(a.ngroups) * D, s->stream);
  hipLaunchKernelGGL(k_dense_big<R>, dim3(grid), dim3(256), size_t(D) * sizeof(cx<double>), s->stream,
                     static_cast<R*>(s->ptr), static_cast<const cd*>(s->big), a);
  QSV_HIP_CHECK(hipGetLastError());
  return QSV_OK;
}

template <typename R>
int launch_dense(qsv_state* s, const cd* mat, const int* targets, int k, uint64_t cmask,
                 uint64_t cval) {
  if (k >= 6) return launch_dense_big<R>(s, mat, targets, k, cmask, cval);
  switch (k) {
    case 2: return launch_dense_k<R, 2>(s, mat, targets, cmask, cval);
    case 3: return launch_dense_k<R, 3>(s, mat, targets, cmask, cval);
    case 4: return launch_dense_k<R, 4>(s, mat, targets, cmask, cval);
    case 5: return launch_dense_k<R, 5>(s, mat, targets, cmask, cval);
    default: return fail(QSV_EINVAL, "dense gate on %d qubits not supported", k);
  }
}

}  // namespace

// Controlled structure of section 4.3.2: if target bit j acts as a control
// with value v -- the gate matrix is the identity on (and does not couple to)
// the rows and columns whose bit j differs from v -- replace the gate by a
// (k-1)-qubit gate with one more control. Repeats until no bit qualifies.
void extract_controls(std::vector<cd>& mat, std::vector<int>& tq, uint64_t& cmask,
                      uint64_t& cval) {
  bool changed = true;
  while (changed && tq.size() > 1) {
    changed = false;
    const int k = int(tq.size());
    const int D = 1 << k;
    for (int j = 0; j < k && !changed; ++j) {
      for (int v = 0; v < 2 && !changed; ++v) {
        bool ok = true;
        for (int r = 0; r < D && ok; ++r)
          for (int c = 0; c < D && ok; ++c) {
            const bool rin = ((r >> j) & 1) == v, cin = ((c >> j) & 1) == v;
            if (rin && cin) continue;
            const cd e = mat[r * D + c];
            if (r == c) ok = ceq(e, 1.0);
            else ok = ceq(e, 0.0);
          }
        if (!ok) continue;
        // keep the block with bit j == v, drop bit j from the index
        const int D2 = D / 2;
        std::vector<cd> sub(D2 * D2);
        auto expand = [&](int i) {
          const int lo = i & ((1 << j) - 1);
          return ((i >> j) << (j + 1)) | (v << j) | lo;
        };
        for (int r = 0; r < D2; ++r)
          for (int c = 0; c < D2; ++c) sub[r * D2 + c] = mat[expand(r) * D + expand(c)];
        cmask |= uint64_t(1) << tq[j];
        if (v) cval |= uint64_t(1) << tq[j];
        tq.erase(tq.begin() + j);
        mat.swap(sub);
        changed = true;
      }
    }
  }
}

int launch_scale_subspace(qsv_state* s, uint64_t mask, uint64_t pattern, cd c) {
  return s->dtype == QSV_C64 ? launch_scale_t<float>(s, mask, pattern, c)
                             : launch_scale_t<double>(s, mask, pattern, c);
}

int apply_gate_impl(qsv_state* s, const cd* mat_in, const int* targets, int k, const int* controls,
                    const int* ctrl_vals, int nc) {
  uint64_t cmask = 0, cval = 0;
  for (int j = 0; j < nc; ++j) {
    cmask |= uint64_t(1) << controls[j];
    if (ctrl_vals[j]) cval |= uint64_t(1) << controls[j];
  }
  std::vector<cd> mat(mat_in, mat_in + (size_t(1) << (2 * k)));
  std::vector<int> tq(targets, targets + k);
  extract_controls(mat, tq, cmask, cval);
  k = int(tq.size());
  const int D = 1 << k;
  bool diag = true;
  for (int r = 0; r < D && diag; ++r)
    for (int c = 0; c < D && diag; ++c)
      if (r != c && !ceq(mat[r * D + c], 0.0)) diag = false;

  if (k == 1) {
    const uint64_t tb = uint64_t(1) << tq[0];
    const cd* u = mat.data();
    if (diag) {
      if (ceq(u[0], 1.0) && ceq(u[3], 1.0)) return QSV_OK;  // identity
      if (ceq(u[0], 1.0)) return launch_scale_subspace(s, cmask | tb, cval | tb, u[3]);
      if (ceq(u[3], 1.0)) return launch_scale_subspace(s, cmask | tb, cval, u[0]);
      if (u[0].re == u[3].re && u[0].im == u[3].im)
        return launch_scale_subspace(s, cmask, cval, u[0]);
      return launch_pair(s, cmask | tb, cval, 0, tb, u, PK_DIAG);
    }
    if (ceq(u[0], 0.0) && ceq(u[3], 0.0) && ceq(u[1], 1.0) && ceq(u[2], 1.0))
      return launch_pair(s, cmask | tb, cval, 0, tb, u, PK_SWAP);
    return launch_pair(s, cmask | tb, cval, 0, tb, u, PK_DENSE);
  }
  if (k == 2) {
    // SWAP permutation: exchange |01> and |10> on the two targets
    bool swap = true;
    for (int r = 0; r < 4 && swap; ++r)
      for (int c = 0; c < 4 && swap; ++c) {
        const int pr = (r == 1) ? 2 : (r == 2) ? 1 : r;
        swap = ceq(mat[r * 4 + c], c == pr ? 1.0 : 0.0);
      }
    if (swap) {
      const uint64_t b0 = uint64_t(1) << tq[0], b1 = uint64_t(1) << tq[1];
      const cd id[4] = {{1, 0}, {0, 0}, {0, 0}, {1, 0}};
      return launch_pair(s, cmask | b0 | b1, cval, b0, b1, id, PK_SWAP);
    }
  }
  if (diag && k <= 5) {
    std::vector<cd> d(D);
    for (int i = 0; i < D; ++i) d[i] = mat[i * D + i];
    return s->dtype == QSV_C64 ? launch_diag_t<float>(s, d.data(), tq.data(), k, cmask, cval)
                               : launch_diag_t<double>(s, d.data(), tq.data(), k, cmask, cval);
  }
  return s->dtype == QSV_C64 ? launch_dense<float>(s, mat.data(), tq.data(), k, cmask, cval)
                             : launch_dense<double>(s, mat.data(), tq.data(), k, cmask, cval);
}

// Named gate matrices (section 4.3.4, table of named gates). Two-qubit named
// gates are returned on their qubit arguments in order (bit 0 = first).
int named_matrix(int kind, double theta, cd* m, int* k) {
  const double c = std::cos(theta / 2), sn = std::sin(theta / 2);
  const double h = 0.70710678118654752440;
  *k = 1;
  switch (kind) {
    case QSV_GATE_X: m[0] = {0, 0}; m[1] = {1, 0}; m[2] = {1, 0}; m[3] = {0, 0}; return QSV_OK;
    case QSV_GATE_Y: m[0] = {0, 0}; m[1] = {0, -1}; m[2] = {0, 1}; m[3] = {0, 0}; return QSV_OK;
    case QSV_GATE_Z: m[0] = {1, 0}; m[1] = {0, 0}; m[2] = {0, 0}; m[3] = {-1, 0}; return QSV_OK;
    case QSV_GATE_H: m[0] = {h, 0}; m[1] = {h, 0}; m[2] = {h, 0}; m[3] = {-h, 0}; return QSV_OK;
    // exp(+i t P/2) = cos(t/2) I + i sin(t/2) P
    case QSV_GATE_RX: m[0] = {c, 0}; m[1] = {0, sn}; m[2] = {0, sn}; m[3] = {c, 0}; return QSV_OK;
    case QSV_GATE_RY: m[0] = {c, 0}; m[1] = {sn, 0}; m[2] = {-sn, 0}; m[3] = {c, 0}; return QSV_OK;
    case QSV_GATE_RZ: m[0] = {c, sn}; m[1] = {0, 0}; m[2] = {0, 0}; m[3] = {c, -sn}; return QSV_OK;
    case QSV_GATE_CNOT:
    case QSV_GATE_CZ:
    case QSV_GATE_SWAP:
      *k = 2;
      for (int i = 0; i < 16; ++i) m[i] = {0, 0};
      if (kind == QSV_GATE_CNOT) {
        // qubits {control, target}: bit 0 = control, bit 1 = target
        m[0] = {1, 0}; m[2 * 4 + 2] = {1, 0}; m[1 * 4 + 3] = {1, 0}; m[3 * 4 + 1] = {1, 0};
      } else if (kind == QSV_GATE_CZ) {
        m[0] = {1, 0}; m[5] = {1, 0}; m[10] = {1, 0}; m[15] = {-1, 0};
      } else {
        m[0] = {1, 0}; m[1 * 4 + 2] = {1, 0}; m[2 * 4 + 1] = {1, 0}; m[15] = {1, 0};
      }
      return QSV_OK;
    default: return fail(QSV_EINVAL, "unknown named gate %d", kind);
  }
}

// Validation shared by the gate entry points: qubits in range and distinct.
int validate_gate(int n, const int* targets, int k, const int* controls, const int* ctrl_vals,
                  int nc, int kmax) {
  if (k < 1 || k > kmax) return fail(QSV_EINVAL, "gate must act on 1..%d target qubits (got %d)", kmax, k);
  if (!targets) return fail(QSV_EINVAL, "null targets");
  if (nc < 0) return fail(QSV_EINVAL, "negative control count");
  if (nc > 0 && (!controls || !ctrl_vals)) return fail(QSV_EINVAL, "null controls");
  uint64_t used = 0;
  for (int j = 0; j < k + nc; ++j) {
    const int q = j < k ? targets[j] : controls[j - k];
    if (q < 0 || q >= n) return fail(QSV_ERANGE, "qubit %d out of range for %d qubits", q, n);
    if (used >> q & 1) return fail(QSV_EDUP, "qubit %d listed twice", q);
    used |= uint64_t(1) << q;
    if (j >= k && ctrl_vals[j - k] != 0 && ctrl_vals[j - k] != 1)
      return fail(QSV_EINVAL, "control value must be 0 or 1");
  }
  return QSV_OK;
}

}  // namespace qsv

using namespace qsv;

extern "C" {

int qsv_apply_gate(qsv_state* s, const double* mat, const int* targets, int k, const int* controls,
                   const int* ctrl_vals, int nc) {
  clear_error();
  int rc = check_state(s);
  if (rc) return rc;
  if (!mat) return fail(QSV_EINVAL, "null matrix");
  if ((rc = validate_gate(s->n, targets, k, controls, ctrl_vals, nc, 10))) return rc;
  return apply_gate_impl(s, reinterpret_cast<const cd*>(mat), targets, k, controls, ctrl_vals, nc);
}

int qsv_apply_named(qsv_state* s, int kind, const int* qubits, int nq, double theta) {
  clear_error();
  int rc = check_state(s);
  if (rc) return rc;
  cd m[16];
  int k = 0;
  if ((rc = named_matrix(kind, theta, m, &k))) return rc;
  if (nq != k) return fail(QSV_EINVAL, "named gate %d takes %d qubits (got %d)", kind, k, nq);
  if ((rc = validate_gate(s->n, qubits, k, nullptr, nullptr, 0, 2))) return rc;
  return apply_gate_impl(s, m, qubits, k, nullptr, nullptr, 0);
}

}  // extern "C"
