// Batched energies and adjoint gradients: many independent (circuit, theta,
// observable) items, possibly of different qubit counts, in ONE persistent
// kernel launch. The paper motivates this regime -- small circuits simulated
// many times, where per-call overhead dominates (section 5.1, T_over; the
// GPU per-call overhead it reports in section 6) -- but does not describe a
// batched method; this is the library's own design.
//
// Each workgroup pulls item indices from a device work queue (items ordered
// largest first for balance) and runs, for its item, entirely inside the
// workgroup: psi = |0...0>, the circuit gate by gate, lambda = H psi, E =
// Re<psi|lambda>, and the reverse sweep of qsv_adjoint_gradient with FP64
// workgroup reductions. psi and lambda live in LDS when both fit, otherwise in
// a per-item slice of device memory (served from L2 / Infinity Cache for the
// sizes this targets). Every workgroup leaves the loop once the queue is
// exhausted, so the grid always drains.
#include <algorithm>
#include <chrono>
#include <cmath>

#include "circuit.h"
#include "dev_common.h"
#include "observable.h"
#include "prof.h"
#include "wave_sum.h"

namespace qsv {

constexpr int kBatchThreads = 512;  // default workgroup size (256 also instantiated)
constexpr int kBatchMaxQ = 24;    // qubits per item
constexpr int kBatchRows = 64;    // gradient rows per reverse pass (LDS slots)
constexpr size_t kBatchStateLds = 65536;  // default LDS for psi + lambda (whole states or tiles)

enum BatchOpKind { BO_ROT = 0, BO_CZ = 1, BO_CNOT = 2, BO_DENSE1 = 3, BO_PAULI = 4 };

struct BatchOp {
  int kind;
  int q0, q1;    // ROT/DENSE1: q0 target; CZ: q0, q1; CNOT: q0 control, q1 target;
                 // PAULI: q0 flip mask (X/Y qubits), q1 sign mask (Y/Z qubits)
  int pauli;     // ROT: Pauli id; PAULI: number of Y factors
  int slot;      // ROT/PAULI: parameter slot (>= 0) or -1 for a fixed angle
  int moff;      // DENSE1 / fixed ROT: offset of the 2x2 matrix in the pool; fixed PAULI: of its angle
};

struct BatchItem {
  int n;
  int op_begin, op_count;
  int grp_begin, grp_count;
  int theta_off, grad_off, nparams;
  uint64_t psi_off, lam_off;  // amplitude offsets into the state buffer (global items)
  // items whose states live in device memory run tile passes: forward passes
  // [fp_begin, +fp_count), reverse passes [rp_begin, +rp_count); the 2x2
  // matrices of the item's ops are computed per run into mats[mat_off + op]
  int fp_begin, fp_count, rp_begin, rp_count;
  int mat_off;
};

// A tile pass of a device-memory item: L local qubits (the low b ones and
// hq[]), the others (gpos[], ascending) index the tiles.
struct BatchPass {
  int L, b, nh, ng;
  int hq[kBatchMaxQ];
  int gpos[kBatchMaxQ];
  int op_begin, op_count, row_count;
};

// An op inside a tile pass. p0/p1: local positions of q0/q1 (-1: not local,
// then the bit is read from the tile base at g0/g1). Dense targets are local.
struct BTOp {
  int kind;
  int p0, p1, g0, g1;
  int pauli, slot;  // ROT (PAULI: number of Y factors, slot)
  int bop;          // index of the op in the item's op list (its matrix)
  int row;          // reverse passes: gradient row in the pass (-1: none)
  uint32_t lf, lz, gz;  // PAULI: flip and sign masks in local index space, sign mask on non-local qubits
};

struct BatchGroup {
  uint64_t flip;
  int begin, count;
};

struct BatchArgs {
  const BatchItem* items;
  const int* order;
  int nitems;
  int* queue;
  const BatchOp* ops;
  const double* pool;  // complex128 2x2 matrices
  const BatchGroup* groups;
  const GTerm* terms;
  const double* theta;
  double* energies;
  double* grads;
  void* states;
  size_t lds_state_bytes;  // dynamic LDS available for psi + lambda
  const BatchPass* passes;
  const BTOp* tops;
  void* mats;              // M2<R> per op of the device-memory items
};

__device__ __forceinline__ double wg_sum(double v, double* red) {
  v = wave_sum_to_last(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();  // red[] may still be read from the previous reduction
  if (lane == 63) red[w] = v;
  __syncthreads();
  double r = 0.0;
  for (int i = 0; i < int(blockDim.x >> 6); ++i) r += red[i];  // same order in every thread
  return r;
}

template <typename R>
__device__ __forceinline__ M2<R> rot2(int pauli, double t) {
  // exp(i t P/2) = cos(t/2) I + i sin(t/2) P
  double s, c;
  sincos(0.5 * t, &s, &c);
  const R cr = R(c), sr = R(s);
  if (pauli == 1) return {{cr, 0}, {0, sr}, {0, sr}, {cr, 0}};
  if (pauli == 2) return {{cr, 0}, {sr, 0}, {-sr, 0}, {cr, 0}};
  return {{cr, sr}, {0, 0}, {0, 0}, {cr, -sr}};
}

template <typename R>
__device__ __forceinline__ M2<R> pool2(const double* p, bool dag) {
  const cx<R> a{R(p[0]), R(p[1])}, b{R(p[2]), R(p[3])}, c{R(p[4]), R(p[5])}, d{R(p[6]), R(p[7])};
  if (!dag) return {a, b, c, d};
  return {{a.re, -a.im}, {c.re, -c.im}, {b.re, -b.im}, {d.re, -d.im}};
}

template <typename R>
__device__ __forceinline__ void wg_apply_2x2(cx<R>* s, int n, int q, const M2<R>& u) {
  const uint32_t half = 1u << (n - 1), bit = 1u << q;
  for (uint32_t i = threadIdx.x; i < half; i += blockDim.x) {
    const uint32_t x0 = ((i >> q) << (q + 1)) | (i & (bit - 1));
    const cx<R> a = s[x0], b = s[x0 | bit];
    s[x0] = cfma(u.m00, a, u.m01 * b);
    s[x0 | bit] = cfma(u.m10, a, u.m11 * b);
  }
}

__device__ __forceinline__ uint32_t ins2(uint32_t i, int lo, int hi) {
  i = ((i >> lo) << (lo + 1)) | (i & ((1u << lo) - 1));
  i = ((i >> hi) << (hi + 1)) | (i & ((1u << hi) - 1));
  return i;
}

// Multi-qubit Pauli rotation exp(i t P/2) = cos(t/2) + i sin(t/2) P on the
// index set [0, TS) (a whole state or a tile), with
// (P v)_x = i^ny (-1)^{|(x ^ f) & z| + gs} v_{x ^ f} (gs: the tile's sign from
// Z/Y factors on non-local qubits).
__device__ __forceinline__ int par32(uint32_t x) { return __popc(x) & 1; }

template <typename R>
__device__ __forceinline__ cx<R> times_ipow(cx<R> v, int k) {  // v * i^k
  switch (k & 3) {
    case 0: return v;
    case 1: return {-v.im, v.re};
    case 2: return {-v.re, -v.im};
    default: return {v.im, -v.re};
  }
}

template <typename R>
__device__ __forceinline__ void pauli_rot_set(cx<R>* v, uint32_t TS, uint32_t f, uint32_t z, int ny, int gs,
                                              double t) {
  double sn, cs;
  sincos(0.5 * t, &sn, &cs);
  const R c = R(cs), s = R(sn);
  if (f == 0) {  // diagonal: cos + i sin (-1)^{|x & z| + gs}
    for (uint32_t x = threadIdx.x; x < TS; x += blockDim.x) {
      const cx<R> fx = {c, (par32(x & z) ^ gs) ? -s : s};
      v[x] = fx * v[x];
    }
    return;
  }
  const int h = __ffs(f) - 1;
  for (uint32_t i = threadIdx.x; i < TS / 2; i += blockDim.x) {
    const uint32_t x = ((i >> h) << (h + 1)) | (i & ((1u << h) - 1)), y = x ^ f;
    const cx<R> a = v[x], b = v[y];
    // i sin (P v)_x = sin i^(ny+1) (-1)^{|y & z| + gs} b, and symmetrically at y
    const cx<R> pb = times_ipow(b, ny + 1), pa = times_ipow(a, ny + 1);
    const R sx = (par32(y & z) ^ gs) ? -s : s, sy = (par32(x & z) ^ gs) ? -s : s;
    v[x] = {c * a.re + sx * pb.re, c * a.im + sx * pb.im};
    v[y] = {c * b.re + sy * pa.re, c * b.im + sy * pa.im};
  }
}

// This thread's share of -Im<lam|P|psi> on the index set [0, TS).
template <typename R>
__device__ __forceinline__ double pauli_grad_set(const cx<R>* ps, const cx<R>* la, uint32_t TS, uint32_t f,
                                                 uint32_t z, int ny, int gs) {
  double sr = 0.0, si = 0.0;
  for (uint32_t x = threadIdx.x; x < TS; x += blockDim.x) {
    const uint32_t y = x ^ f;
    const cx<R> a = ps[y], l = la[x];
    const double wr = double(l.re) * a.re + double(l.im) * a.im;
    const double wi = double(l.re) * a.im - double(l.im) * a.re;
    const bool neg = (par32(y & z) ^ gs) != 0;
    sr += neg ? -wr : wr;
    si += neg ? -wi : wi;
  }
  // -Im of i^ny (sr + i si)
  switch (ny & 3) {
    case 0: return -si;
    case 1: return -sr;
    case 2: return si;
    default: return sr;
  }
}

__device__ __forceinline__ double op_angle(const BatchOp& op, const double* theta, const double* pool) {
  return op.slot >= 0 ? theta[op.slot] : pool[op.moff];
}

template <typename R>
__device__ __forceinline__ void wg_apply_op(cx<R>* s, int n, const BatchOp& op, const double* theta,
                                            const double* pool, bool dag) {
  if (op.kind == BO_PAULI) {
    const double t = op_angle(op, theta, pool);
    pauli_rot_set<R>(s, 1u << n, uint32_t(op.q0), uint32_t(op.q1), op.pauli, 0, dag ? -t : t);
  } else if (op.kind == BO_ROT) {
    const double t = op.slot >= 0 ? theta[op.slot] : 0.0;
    M2<R> u = op.slot >= 0 ? rot2<R>(op.pauli, dag ? -t : t) : pool2<R>(pool + op.moff, dag);
    wg_apply_2x2(s, n, op.q0, u);
  } else if (op.kind == BO_DENSE1) {
    wg_apply_2x2(s, n, op.q0, pool2<R>(pool + op.moff, dag));
  } else {
    const int lo = min(op.q0, op.q1), hi = max(op.q0, op.q1);
    const uint32_t quarter = 1u << (n - 2);
    const uint32_t b0 = 1u << op.q0, b1 = 1u << op.q1;
    for (uint32_t i = threadIdx.x; i < quarter; i += blockDim.x) {
      const uint32_t x = ins2(i, lo, hi);
      if (op.kind == BO_CZ) {
        const cx<R> v = s[x | b0 | b1];
        s[x | b0 | b1] = {-v.re, -v.im};
      } else {  // CNOT: swap target within control = 1
        const cx<R> a = s[x | b0], b = s[x | b0 | b1];
        s[x | b0] = b;
        s[x | b0 | b1] = a;
      }
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------------- tiled items
//
// Items whose psi and lambda do not fit in LDS together run the library's
// tile-pass scheme inside their workgroup: a pass keeps L qubits local, the
// workgroup streams the item's state through an LDS tile (psi, and lambda in
// the reverse sweep) tile by tile and applies every op of the pass to it. The
// planner puts ops into passes so that dense targets are local; CZ and CNOT
// controls may be anywhere (a non-local bit is a constant of the tile). One
// pass moves the state once, instead of once per gate.

__device__ __forceinline__ uint32_t bt_bit(int p, int g, uint32_t j, uint32_t base) {
  return p >= 0 ? (j >> p) & 1u : (base >> g) & 1u;
}

// Global index of local index j in the tile at base.
__device__ __forceinline__ uint32_t bt_addr(const BatchPass& P, uint32_t base, uint32_t j) {
  uint32_t x = base | (j & ((1u << P.b) - 1));
  const uint32_t h = j >> P.b;
  for (int i = 0; i < P.nh; ++i) x |= ((h >> i) & 1u) << P.hq[i];
  return x;
}

__device__ __forceinline__ uint32_t bt_base(const BatchPass& P, uint32_t g) {
  uint32_t base = 0;
  for (int j = 0; j < P.ng; ++j) base |= ((g >> j) & 1u) << P.gpos[j];
  return base;
}

template <typename R>
__device__ __forceinline__ M2<R> m2_dag(const M2<R>& u) {
  return {{u.m00.re, -u.m00.im}, {u.m10.re, -u.m10.im}, {u.m01.re, -u.m01.im}, {u.m11.re, -u.m11.im}};
}

template <typename R>
__device__ __forceinline__ void bt_pair(cx<R>* t, int p, const M2<R>& u, uint32_t TS) {
  const uint32_t bit = 1u << p;
  for (uint32_t i = threadIdx.x; i < TS / 2; i += blockDim.x) {
    const uint32_t x0 = ((i >> p) << (p + 1)) | (i & (bit - 1));
    const cx<R> x = t[x0], y = t[x0 | bit];
    t[x0] = cfma(u.m00, x, u.m01 * y);
    t[x0 | bit] = cfma(u.m10, x, u.m11 * y);
  }
}

template <typename R>
__device__ __forceinline__ void bt_cz(cx<R>* t, const BTOp& op, uint32_t TS, uint32_t base) {
  for (uint32_t j = threadIdx.x; j < TS; j += blockDim.x)
    if (bt_bit(op.p0, op.g0, j, base) & bt_bit(op.p1, op.g1, j, base)) t[j] = {-t[j].re, -t[j].im};
}

// CNOT: control q0 (anywhere), target q1 (local).
template <typename R>
__device__ __forceinline__ void bt_cnot(cx<R>* t, const BTOp& op, uint32_t TS, uint32_t base) {
  const int p = op.p1;
  const uint32_t bit = 1u << p;
  for (uint32_t i = threadIdx.x; i < TS / 2; i += blockDim.x) {
    const uint32_t x0 = ((i >> p) << (p + 1)) | (i & (bit - 1));
    if (bt_bit(op.p0, op.g0, x0, base)) {
      const cx<R> x = t[x0];
      t[x0] = t[x0 | bit];
      t[x0 | bit] = x;
    }
  }
}

// Reverse-sweep op on both tiles; returns this thread's share of the
// gradient term -Im<lambda|P|psi> when the op is a parametric rotation.
template <typename R>
__device__ __forceinline__ double bt_rev(cx<R>* ps, cx<R>* la, const BTOp& op, const M2<R>* mats, uint32_t TS,
                                         uint32_t base, double t) {
  if (op.kind == BO_PAULI) {
    const int gs = par32(base & op.gz);
    double acc = 0.0;
    if (op.row >= 0) {
      acc = pauli_grad_set<R>(ps, la, TS, op.lf, op.lz, op.pauli, gs);
      __syncthreads();  // every read of the term before the uncompute writes
    }
    pauli_rot_set<R>(ps, TS, op.lf, op.lz, op.pauli, gs, -t);
    pauli_rot_set<R>(la, TS, op.lf, op.lz, op.pauli, gs, -t);
    return acc;
  }
  if (op.kind == BO_CZ) {
    bt_cz(ps, op, TS, base);
    bt_cz(la, op, TS, base);
    return 0.0;
  }
  if (op.kind == BO_CNOT) {
    bt_cnot(ps, op, TS, base);
    bt_cnot(la, op, TS, base);
    return 0.0;
  }
  const M2<R> u = m2_dag(mats[op.bop]);
  const int p = op.p0;
  if (op.row < 0) {
    bt_pair(ps, p, u, TS);
    bt_pair(la, p, u, TS);
    return 0.0;
  }
  double acc = 0.0;
  if (op.pauli == 3) {
    for (uint32_t j = threadIdx.x; j < TS; j += blockDim.x) {
      const cx<R> x = ps[j], l = la[j];
      const bool one = (j >> p) & 1;
      const double im = double(l.re) * x.im - double(l.im) * x.re;
      acc -= one ? -im : im;
      const cx<R> f = one ? u.m11 : u.m00;
      ps[j] = f * x;
      la[j] = f * l;
    }
    return acc;
  }
  const uint32_t bit = 1u << p;
  for (uint32_t i = threadIdx.x; i < TS / 2; i += blockDim.x) {
    const uint32_t x0 = ((i >> p) << (p + 1)) | (i & (bit - 1));
    const uint32_t x1 = x0 | bit;
    const cx<R> a0 = ps[x0], a1 = ps[x1], l0 = la[x0], l1 = la[x1];
    const double a0r = a0.re, a0i = a0.im, a1r = a1.re, a1i = a1.im;
    const double l0r = l0.re, l0i = l0.im, l1r = l1.re, l1i = l1.im;
    const double im = op.pauli == 1 ? (l0r * a1i - l0i * a1r) + (l1r * a0i - l1i * a0r)
                                    : -(l0r * a1r + l0i * a1i) + (l1r * a0r + l1i * a0i);
    acc -= im;
    ps[x0] = cfma(u.m00, a0, u.m01 * a1);
    ps[x1] = cfma(u.m10, a0, u.m11 * a1);
    la[x0] = cfma(u.m00, l0, u.m01 * l1);
    la[x1] = cfma(u.m10, l0, u.m11 * l1);
  }
  return acc;
}

// Forward passes of a device-memory item: psi = U |0...0>.
template <typename R>
__device__ void bt_forward(const BatchArgs& a, const BatchItem& I, cx<R>* psi, M2<R>* mats, char* smem) {
  const double* theta = a.theta + I.theta_off;
  for (int o = threadIdx.x; o < I.op_count; o += blockDim.x) {
    const BatchOp op = a.ops[I.op_begin + o];
    if (op.kind == BO_ROT)
      mats[o] = op.slot >= 0 ? rot2<R>(op.pauli, theta[op.slot]) : pool2<R>(a.pool + op.moff, false);
    else if (op.kind == BO_DENSE1)
      mats[o] = pool2<R>(a.pool + op.moff, false);
  }
  const uint32_t N = 1u << I.n;
  for (uint32_t x = threadIdx.x; x < N; x += blockDim.x) psi[x] = {R(x == 0 ? 1 : 0), R(0)};
  cx<R>* t = reinterpret_cast<cx<R>*>(smem);
  for (int pi = 0; pi < I.fp_count; ++pi) {
    const BatchPass& P = a.passes[I.fp_begin + pi];
    const uint32_t TS = 1u << P.L, tiles = 1u << P.ng;
    for (uint32_t g = 0; g < tiles; ++g) {
      const uint32_t base = bt_base(P, g);
      __syncthreads();  // the tile buffer is free; earlier device-memory writes are visible
      for (uint32_t j = threadIdx.x; j < TS; j += blockDim.x) t[j] = psi[bt_addr(P, base, j)];
      __syncthreads();
      for (int o = 0; o < P.op_count; ++o) {
        const BTOp op = a.tops[P.op_begin + o];
        if (op.kind == BO_CZ) bt_cz(t, op, TS, base);
        else if (op.kind == BO_CNOT) bt_cnot(t, op, TS, base);
        else if (op.kind == BO_PAULI)
          pauli_rot_set<R>(t, TS, op.lf, op.lz, op.pauli, par32(base & op.gz),
                           op_angle(a.ops[I.op_begin + op.bop], theta, a.pool));
        else bt_pair(t, op.p0, mats[op.bop], TS);
        __syncthreads();
      }
      for (uint32_t j = threadIdx.x; j < TS; j += blockDim.x) psi[bt_addr(P, base, j)] = t[j];
    }
  }
  __syncthreads();
}

// Reverse passes of a device-memory item: uncomputes psi and lambda and adds
// the gradient terms into grad[] (per-wavefront LDS slots, fixed order).
template <typename R>
__device__ void bt_reverse(const BatchArgs& a, const BatchItem& I, cx<R>* psi, cx<R>* lam, const M2<R>* mats,
                           double* grad, char* smem) {
  const double* theta = a.theta + I.theta_off;
  const int NW = int(blockDim.x >> 6);
  cx<R>* ts = reinterpret_cast<cx<R>*>(smem);
  cx<R>* tl = ts + a.lds_state_bytes / 2 / sizeof(cx<R>);
  double* slot = reinterpret_cast<double*>(smem + a.lds_state_bytes);
  const int wave = int(threadIdx.x >> 6);
  for (int pi = 0; pi < I.rp_count; ++pi) {
    const BatchPass& P = a.passes[I.rp_begin + pi];
    const uint32_t TS = 1u << P.L, tiles = 1u << P.ng;
    __syncthreads();
    for (int r = threadIdx.x; r < P.row_count * NW; r += blockDim.x) slot[r] = 0.0;
    for (uint32_t g = 0; g < tiles; ++g) {
      const uint32_t base = bt_base(P, g);
      __syncthreads();
      for (uint32_t j = threadIdx.x; j < TS; j += blockDim.x) {
        const uint32_t x = bt_addr(P, base, j);
        ts[j] = psi[x];
        tl[j] = lam[x];
      }
      __syncthreads();
      for (int o = 0; o < P.op_count; ++o) {
        const BTOp op = a.tops[P.op_begin + o];
        const double t = op.kind == BO_PAULI ? op_angle(a.ops[I.op_begin + op.bop], theta, a.pool) : 0.0;
        double acc = bt_rev(ts, tl, op, mats, TS, base, t);
        if (op.row >= 0) {
          acc = wave_sum_to_last(acc);
          if ((threadIdx.x & 63) == 63) slot[op.row * NW + wave] += acc;
        }
        __syncthreads();
      }
      for (uint32_t j = threadIdx.x; j < TS; j += blockDim.x) {
        const uint32_t x = bt_addr(P, base, j);
        psi[x] = ts[j];
        lam[x] = tl[j];
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) {  // rows in order (a parameter may own several rows)
      for (int o = 0; o < P.op_count; ++o) {
        const BTOp op = a.tops[P.op_begin + o];
        if (op.row < 0) continue;
        double sum = 0.0;
        for (int w = 0; w < NW; ++w) sum += slot[op.row * NW + w];
        grad[op.slot] += sum;
      }
    }
  }
  __syncthreads();
}

template <typename R, int NT>
__global__ void __launch_bounds__(NT) k_batch(BatchArgs a) {
  extern __shared__ __align__(16) char smem[];
  __shared__ double red[NT / 64];
  __shared__ int s_item;
  while (true) {
    __syncthreads();
    if (threadIdx.x == 0) s_item = atomicAdd(a.queue, 1);
    __syncthreads();
    const int it = s_item;
    if (it >= a.nitems) break;
    const BatchItem I = a.items[a.order[it]];
    const int n = I.n;
    const uint32_t N = 1u << n;
    cx<R>* psi;
    cx<R>* lam;
    if (size_t(2) * N * sizeof(cx<R>) <= a.lds_state_bytes) {
      psi = reinterpret_cast<cx<R>*>(smem);
      lam = psi + N;
    } else {
      psi = reinterpret_cast<cx<R>*>(a.states) + I.psi_off;
      lam = reinterpret_cast<cx<R>*>(a.states) + I.lam_off;
    }
    const double* theta = a.theta + I.theta_off;
    const bool tiled = I.fp_count > 0;
    M2<R>* mats = reinterpret_cast<M2<R>*>(a.mats) + I.mat_off;
    if (tiled) {
      bt_forward<R>(a, I, psi, mats, smem);
    } else {
      // |0...0>
      for (uint32_t x = threadIdx.x; x < N; x += blockDim.x) psi[x] = {R(x == 0 ? 1 : 0), R(0)};
      __syncthreads();
      // forward
      for (int o = 0; o < I.op_count; ++o) wg_apply_op<R>(psi, n, a.ops[I.op_begin + o], theta, a.pool, false);
    }
    // lambda = H psi
    for (uint32_t y = threadIdx.x; y < N; y += blockDim.x) {
      double ar = 0.0, ai = 0.0;
      for (int g = 0; g < I.grp_count; ++g) {
        const BatchGroup G = a.groups[I.grp_begin + g];
        const uint32_t x = y ^ uint32_t(G.flip);
        const cx<R> v = psi[x];
        double cr = 0.0, ci = 0.0;
        for (int k = G.begin; k < G.begin + G.count; ++k) {
          const GTerm t = a.terms[k];
          const bool neg = __popc(x & uint32_t(t.z)) & 1;
          cr += neg ? -t.re : t.re;
          ci += neg ? -t.im : t.im;
        }
        ar += cr * double(v.re) - ci * double(v.im);
        ai += cr * double(v.im) + ci * double(v.re);
      }
      lam[y] = {R(ar), R(ai)};
    }
    __syncthreads();
    // E = Re <psi|lambda>
    double e = 0.0;
    for (uint32_t x = threadIdx.x; x < N; x += blockDim.x)
      e += double(psi[x].re) * double(lam[x].re) + double(psi[x].im) * double(lam[x].im);
    e = wg_sum(e, red);
    if (threadIdx.x == 0) a.energies[a.order[it]] = e;
    double* grad = a.grads + I.grad_off;
    for (int i = threadIdx.x; i < I.nparams; i += blockDim.x) grad[i] = 0.0;
    __syncthreads();
    if (tiled) {
      bt_reverse<R>(a, I, psi, lam, mats, grad, smem);
      continue;
    }
    // reverse sweep
    for (int o = I.op_count - 1; o >= 0; --o) {
      const BatchOp op = a.ops[I.op_begin + o];
      if (op.kind == BO_ROT && op.slot >= 0) {
        const M2<R> ud = rot2<R>(op.pauli, -theta[op.slot]);
        const uint32_t half = N >> 1, bit = 1u << op.q0;
        double acc = 0.0;
        for (uint32_t i = threadIdx.x; i < half; i += blockDim.x) {
          const uint32_t x0 = ((i >> op.q0) << (op.q0 + 1)) | (i & (bit - 1));
          const uint32_t x1 = x0 | bit;
          const cx<R> a0 = psi[x0], a1 = psi[x1], l0 = lam[x0], l1 = lam[x1];
          const double a0r = a0.re, a0i = a0.im, a1r = a1.re, a1i = a1.im;
          const double l0r = l0.re, l0i = l0.im, l1r = l1.re, l1i = l1.im;
          double im;
          if (op.pauli == 1) im = (l0r * a1i - l0i * a1r) + (l1r * a0i - l1i * a0r);
          else if (op.pauli == 2) im = -(l0r * a1r + l0i * a1i) + (l1r * a0r + l1i * a0i);
          else im = (l0r * a0i - l0i * a0r) - (l1r * a1i - l1i * a1r);
          acc -= im;
          psi[x0] = cfma(ud.m00, a0, ud.m01 * a1);
          psi[x1] = cfma(ud.m10, a0, ud.m11 * a1);
          lam[x0] = cfma(ud.m00, l0, ud.m01 * l1);
          lam[x1] = cfma(ud.m10, l0, ud.m11 * l1);
        }
        acc = wg_sum(acc, red);
        if (threadIdx.x == 0) grad[op.slot] += acc;
        __syncthreads();
      } else if (op.kind == BO_PAULI && op.slot >= 0) {
        // -Im<lambda|P|psi>, then the uncompute of both states
        double acc = pauli_grad_set<R>(psi, lam, N, uint32_t(op.q0), uint32_t(op.q1), op.pauli, 0);
        acc = wg_sum(acc, red);  // (its barriers also order the reads before the writes)
        if (threadIdx.x == 0) grad[op.slot] += acc;
        wg_apply_op<R>(psi, n, op, theta, a.pool, true);
        wg_apply_op<R>(lam, n, op, theta, a.pool, true);
      } else {
        wg_apply_op<R>(psi, n, op, theta, a.pool, true);
        wg_apply_op<R>(lam, n, op, theta, a.pool, true);
      }
    }
  }
}

__global__ void k_zero_int(int* p) { *p = 0; }

}  // namespace qsv

// ------------------------------------------------------------------ host

struct qsv_batch {
  struct Item {
    qsv_circuit c;
    qsv_observable o;
    std::vector<double> theta;
  };
  std::vector<Item> items;
  // device cache (per dtype)
  int dev_dtype = 0;
  size_t state_elems = 0;
  void* d_states = nullptr;
  void* d_tables = nullptr;
  size_t tables_bytes = 0;
  size_t off_items = 0, off_order = 0, off_queue = 0, off_ops = 0, off_pool = 0, off_groups = 0,
         off_terms = 0, off_theta = 0, off_energy = 0, off_grads = 0, off_passes = 0, off_tops = 0,
         off_mats = 0;
  int total_params = 0;
  size_t lds_bytes = 0;
  int grid = 0;
  // launch shape (qsv_batch_autotune): LDS bytes for psi + lambda per
  // workgroup (whole states, or the tiles of device-memory items) and threads
  size_t cfg_lds = qsv::kBatchStateLds;
  int cfg_threads = qsv::kBatchThreads;
  // the launch (queue reset + persistent kernel) captured once as a HIP graph
  // and replayed by later runs
  bool use_graph = true;
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
};

namespace qsv {

namespace {

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Tile passes of one item's op list (in order, or reversed for the reverse
// sweep), greedy like the library's planners: an op joins the current pass
// when its dense target fits the pass's local set (at most L qubits, the low
// b always included) and no op deferred before it shares a qubit with it;
// reverse passes hold at most kBatchRows gradient rows.
void schedule_item(int n, int L, int b, const BatchOp* ops, int count, bool reverse,
                   std::vector<BatchPass>& passes, std::vector<BTOp>& tops, int& pbegin, int& pcount) {
  std::vector<int> rem(static_cast<size_t>(count));
  for (int i = 0; i < count; ++i) rem[size_t(i)] = reverse ? count - 1 - i : i;
  pbegin = int(passes.size());
  pcount = 0;
  const uint64_t low = (uint64_t(1) << b) - 1;
  auto qubits = [&](const BatchOp& o) {
    if (o.kind == BO_PAULI) return uint64_t(uint32_t(o.q0) | uint32_t(o.q1));
    uint64_t m = uint64_t(1) << o.q0;
    if (o.kind == BO_CZ || o.kind == BO_CNOT) m |= uint64_t(1) << o.q1;
    return m;
  };
  while (!rem.empty()) {
    uint64_t local = low, blocked = 0;
    std::vector<int> take, deferred;
    int nrow = 0;
    for (int oi : rem) {
      const BatchOp& o = ops[oi];
      const uint64_t qs = qubits(o);
      if (qs & blocked) {
        deferred.push_back(oi);
        blocked |= qs;
        continue;
      }
      const uint64_t dense =
          o.kind == BO_PAULI ? uint64_t(uint32_t(o.q0))  // the X/Y qubits: pairs x, x ^ f in one tile
          : o.kind == BO_CZ  ? 0
                             : (o.kind == BO_CNOT ? uint64_t(1) << o.q1 : uint64_t(1) << o.q0);
      const bool grad = reverse && (o.kind == BO_ROT || o.kind == BO_PAULI) && o.slot >= 0;
      const uint64_t need = dense & ~local;
      if (!(grad && nrow >= kBatchRows) && __builtin_popcountll(local | need) <= L) {
        local |= need;
        take.push_back(oi);
        if (grad) ++nrow;
      } else {
        deferred.push_back(oi);
        blocked |= qs;
      }
    }
    for (int q = 0; q < n && __builtin_popcountll(local) < L; ++q) local |= uint64_t(1) << q;
    BatchPass P{};
    P.L = L;
    P.b = b;
    P.nh = L - b;
    std::vector<int> lpos(64, -1), loc;
    for (int q = 0; q < n; ++q)
      if (local >> q & 1) {
        lpos[size_t(q)] = int(loc.size());
        loc.push_back(q);
      }
    for (int i = 0; i < P.nh; ++i) P.hq[i] = loc[size_t(b + i)];
    P.ng = 0;
    for (int q = 0; q < n; ++q)
      if (!(local >> q & 1)) P.gpos[P.ng++] = q;
    P.op_begin = int(tops.size());
    P.op_count = int(take.size());
    P.row_count = 0;
    for (int oi : take) {
      const BatchOp& o = ops[oi];
      BTOp t{};
      t.kind = o.kind;
      if (o.kind == BO_PAULI) {
        t.p0 = t.p1 = t.g0 = t.g1 = -1;
        for (int q = 0; q < n; ++q) {
          const uint32_t bit = 1u << q;
          if (uint32_t(o.q0) & bit) t.lf |= 1u << lpos[size_t(q)];  // (local)
          if (uint32_t(o.q1) & bit) {
            if (lpos[size_t(q)] >= 0) t.lz |= 1u << lpos[size_t(q)];
            else t.gz |= bit;
          }
        }
      } else {
        t.p0 = lpos[size_t(o.q0)];
        t.g0 = o.q0;
        t.p1 = (o.kind == BO_CZ || o.kind == BO_CNOT) ? lpos[size_t(o.q1)] : -1;
        t.g1 = o.q1;
      }
      t.pauli = o.pauli;
      t.slot = o.slot;
      t.bop = oi;
      t.row = (reverse && (o.kind == BO_ROT || o.kind == BO_PAULI) && o.slot >= 0) ? P.row_count++ : -1;
      tops.push_back(t);
    }
    passes.push_back(P);
    ++pcount;
    rem.swap(deferred);
  }
}

int build_device(qsv_batch* b, qsv_dtype dt) {
  const size_t S = amp_bytes(dt);
  std::vector<BatchItem> items(b->items.size());
  std::vector<BatchOp> ops;
  std::vector<double> pool;
  std::vector<BatchGroup> groups;
  std::vector<GTerm> terms;
  std::vector<double> theta;
  // LDS for psi + lambda (whole states, or tiles): 64 KiB by default (two
  // workgroups per CU); tiles of device-memory items fill it
  const size_t lds = b->cfg_lds;
  int Lt = 0;
  while ((size_t(2) << (Lt + 1)) * S <= lds) ++Lt;  // 2 * 2^Lt * S <= lds
  const int bt = std::min(Lt, dt == QSV_C64 ? 4 : 3);  // 128-byte contiguous runs
  std::vector<BatchPass> passes;
  std::vector<BTOp> tops;
  int mat_elems = 0;
  size_t state_elems = 0;
  int grad_off = 0;
  for (size_t i = 0; i < b->items.size(); ++i) {
    const auto& it = b->items[i];
    BatchItem& I = items[i];
    I.n = it.c.n;
    I.op_begin = int(ops.size());
    for (const Gate& g : it.c.gates) {
      BatchOp op{};
      if (g.kind == Gate::PAULI) {
        op.kind = BO_PAULI;
        uint32_t f = 0, z = 0;
        int ny = 0;
        for (size_t j = 0; j < g.targets.size(); ++j) {
          const uint32_t bit = 1u << g.targets[j];
          if (g.paulis[j] != 3) f |= bit;
          if (g.paulis[j] != 1) z |= bit;
          if (g.paulis[j] == 2) ++ny;
        }
        op.q0 = int(f);
        op.q1 = int(z);
        op.pauli = ny;
        op.slot = g.slot;
        if (g.slot < 0) {
          op.moff = int(pool.size());
          pool.push_back(g.fixed_angle);
        }
        ops.push_back(op);
        continue;
      }
      if (g.kind == Gate::ROTATION) {
        op.kind = BO_ROT;
        op.q0 = g.targets[0];
        op.pauli = g.pauli;
        op.slot = g.slot;
        if (g.slot < 0) {
          cd m[4];
          rotation_matrix(g.pauli, g.fixed_angle, m);
          op.moff = int(pool.size());
          for (int j = 0; j < 4; ++j) {
            pool.push_back(m[j].re);
            pool.push_back(m[j].im);
          }
        }
      } else {
        std::vector<cd> m = g.mat;
        std::vector<int> tq = g.targets;
        uint64_t cm = 0, cv = 0;
        for (size_t j = 0; j < g.controls.size(); ++j) {
          cm |= uint64_t(1) << g.controls[j];
          if (g.ctrl_vals[j]) cv |= uint64_t(1) << g.controls[j];
        }
        extract_controls(m, tq, cm, cv);
        const bool one_ctrl_on = __builtin_popcountll(cm) == 1 && cv == cm;
        auto is = [&](int r, int c, double re, double im) {
          return m[r * 2 + c].re == re && m[r * 2 + c].im == im;
        };
        if (tq.size() == 1 && cm == 0) {
          op.kind = BO_DENSE1;
          op.q0 = tq[0];
          op.moff = int(pool.size());
          for (int j = 0; j < 4; ++j) {
            pool.push_back(m[j].re);
            pool.push_back(m[j].im);
          }
        } else if (tq.size() == 1 && one_ctrl_on && is(0, 0, 1, 0) && is(0, 1, 0, 0) &&
                   is(1, 0, 0, 0) && is(1, 1, -1, 0)) {
          op.kind = BO_CZ;
          op.q0 = __builtin_ctzll(cm);
          op.q1 = tq[0];
        } else if (tq.size() == 1 && one_ctrl_on && is(0, 0, 0, 0) && is(0, 1, 1, 0) &&
                   is(1, 0, 1, 0) && is(1, 1, 0, 0)) {
          op.kind = BO_CNOT;
          op.q0 = __builtin_ctzll(cm);
          op.q1 = tq[0];
        } else {
          return fail(QSV_EINVAL, "batched items support one-qubit gates, rotations, Pauli rotations, CZ and CNOT");
        }
      }
      ops.push_back(op);
    }
    I.op_count = int(ops.size()) - I.op_begin;
    std::vector<Group> gs;
    std::vector<GTerm> ts;
    build_groups(&it.o, gs, ts);
    I.grp_begin = int(groups.size());
    I.grp_count = int(gs.size());
    const int tbase = int(terms.size());
    for (const Group& g : gs) groups.push_back({g.flip, g.begin + tbase, g.count});
    terms.insert(terms.end(), ts.begin(), ts.end());
    I.theta_off = int(theta.size());
    I.nparams = it.c.nparams;
    theta.insert(theta.end(), it.theta.begin(), it.theta.end());
    I.grad_off = grad_off;
    grad_off += it.c.nparams;
    const uint64_t N = dim(I.n);
    I.fp_begin = I.fp_count = I.rp_begin = I.rp_count = 0;
    I.mat_off = 0;
    if (2 * N * S <= lds) {
      I.psi_off = I.lam_off = 0;
    } else {
      I.psi_off = state_elems;
      I.lam_off = state_elems + N;
      state_elems += 2 * N;
      schedule_item(I.n, Lt, bt, ops.data() + I.op_begin, I.op_count, false, passes, tops, I.fp_begin, I.fp_count);
      schedule_item(I.n, Lt, bt, ops.data() + I.op_begin, I.op_count, true, passes, tops, I.rp_begin, I.rp_count);
      I.mat_off = mat_elems;
      mat_elems += I.op_count;
    }
  }
  // largest items first
  std::vector<int> order(items.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = int(i);
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return items[x].n > items[y].n; });

  size_t off = 0;
  b->off_items = off; off = align_up(off + items.size() * sizeof(BatchItem), 256);
  b->off_order = off; off = align_up(off + order.size() * sizeof(int), 256);
  b->off_queue = off; off = align_up(off + sizeof(int), 256);
  b->off_ops = off; off = align_up(off + std::max<size_t>(1, ops.size()) * sizeof(BatchOp), 256);
  b->off_pool = off; off = align_up(off + std::max<size_t>(1, pool.size()) * sizeof(double), 256);
  b->off_groups = off; off = align_up(off + std::max<size_t>(1, groups.size()) * sizeof(BatchGroup), 256);
  b->off_terms = off; off = align_up(off + std::max<size_t>(1, terms.size()) * sizeof(GTerm), 256);
  b->off_theta = off; off = align_up(off + std::max<size_t>(1, theta.size()) * sizeof(double), 256);
  b->off_energy = off; off = align_up(off + items.size() * sizeof(double), 256);
  b->off_grads = off; off = align_up(off + std::max<int>(1, grad_off) * sizeof(double), 256);
  b->off_passes = off; off = align_up(off + std::max<size_t>(1, passes.size()) * sizeof(BatchPass), 256);
  b->off_tops = off; off = align_up(off + std::max<size_t>(1, tops.size()) * sizeof(BTOp), 256);
  b->off_mats = off; off = align_up(off + std::max<size_t>(1, size_t(mat_elems)) * sizeof(M2<double>), 256);
  if (hipMalloc(&b->d_tables, off) != hipSuccess) return fail(QSV_ENOMEM, "batch table allocation failed");
  b->tables_bytes = off;
  if (state_elems && hipMalloc(&b->d_states, state_elems * S) != hipSuccess)
    return fail(QSV_ENOMEM, "batch state allocation failed (%zu bytes)", state_elems * S);
  char* d = static_cast<char*>(b->d_tables);
  auto put = [&](size_t o, const void* src, size_t bytes) -> int {
    if (bytes) QSV_HIP_CHECK(hipMemcpy(d + o, src, bytes, hipMemcpyHostToDevice));
    return QSV_OK;
  };
  int rc;
  if ((rc = put(b->off_items, items.data(), items.size() * sizeof(BatchItem)))) return rc;
  if ((rc = put(b->off_order, order.data(), order.size() * sizeof(int)))) return rc;
  if ((rc = put(b->off_ops, ops.data(), ops.size() * sizeof(BatchOp)))) return rc;
  if ((rc = put(b->off_pool, pool.data(), pool.size() * sizeof(double)))) return rc;
  if ((rc = put(b->off_groups, groups.data(), groups.size() * sizeof(BatchGroup)))) return rc;
  if ((rc = put(b->off_terms, terms.data(), terms.size() * sizeof(GTerm)))) return rc;
  if ((rc = put(b->off_passes, passes.data(), passes.size() * sizeof(BatchPass)))) return rc;
  if ((rc = put(b->off_tops, tops.data(), tops.size() * sizeof(BTOp)))) return rc;
  b->state_elems = state_elems;
  b->total_params = grad_off;
  b->lds_bytes = lds + size_t(kBatchRows) * (b->cfg_threads / 64) * sizeof(double);  // + gradient slots
  b->dev_dtype = int(dt);
  return QSV_OK;
}

template <typename R>
int run_t(qsv_batch* b, hipStream_t st, double* energies, double* grads) {
  char* d = static_cast<char*>(b->d_tables);
  std::vector<double> theta;
  for (const auto& it : b->items) theta.insert(theta.end(), it.theta.begin(), it.theta.end());
  if (!theta.empty())
    QSV_HIP_CHECK(hipMemcpyAsync(d + b->off_theta, theta.data(), theta.size() * sizeof(double),
                                 hipMemcpyHostToDevice, st));
  const int NT = b->cfg_threads;
  auto kfn = NT == 256 ? &k_batch<R, 256> : &k_batch<R, 512>;
  if (b->grid == 0) {
    int dev = 0, cus = 0, per = 0;
    QSV_HIP_CHECK(hipGetDevice(&dev));
    QSV_HIP_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    QSV_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(kfn),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, int(b->lds_bytes)));
    QSV_HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kfn, NT, b->lds_bytes));
    b->grid = std::max(1, cus * std::max(1, per));
  }
  BatchArgs a;
  a.items = reinterpret_cast<const BatchItem*>(d + b->off_items);
  a.order = reinterpret_cast<const int*>(d + b->off_order);
  a.nitems = int(b->items.size());
  a.queue = reinterpret_cast<int*>(d + b->off_queue);
  a.ops = reinterpret_cast<const BatchOp*>(d + b->off_ops);
  a.pool = reinterpret_cast<const double*>(d + b->off_pool);
  a.groups = reinterpret_cast<const BatchGroup*>(d + b->off_groups);
  a.terms = reinterpret_cast<const GTerm*>(d + b->off_terms);
  a.theta = reinterpret_cast<const double*>(d + b->off_theta);
  a.energies = reinterpret_cast<double*>(d + b->off_energy);
  a.grads = reinterpret_cast<double*>(d + b->off_grads);
  a.states = b->d_states;
  a.lds_state_bytes = b->cfg_lds;
  a.passes = reinterpret_cast<const BatchPass*>(d + b->off_passes);
  a.tops = reinterpret_cast<const BTOp*>(d + b->off_tops);
  a.mats = d + b->off_mats;
  if (b->use_graph && !b->graph_exec) {
    // capture on a private stream (the caller's may be the legacy default
    // stream, which cannot be captured); the queue reset is a kernel, not a
    // memset node
    hipStream_t cs = nullptr;
    QSV_HIP_CHECK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(1), 0, cs, a.queue);
      hipLaunchKernelGGL(kfn, dim3(b->grid), dim3(NT), b->lds_bytes, cs, a);
      e = hipStreamEndCapture(cs, &b->graph);
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&b->graph_exec, b->graph, nullptr, nullptr, 0);
    (void)hipStreamDestroy(cs);
    if (e != hipSuccess) return fail(QSV_EHIP, "batch graph capture failed: %s", hipGetErrorString(e));
  }
  if (b->use_graph) {
    ProfScope ps("batch", 0.0, st);
    QSV_HIP_CHECK(hipGraphLaunch(b->graph_exec, st));
  } else {
    hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(1), 0, st, a.queue);
    {
      ProfScope ps("batch", 0.0, st);
      hipLaunchKernelGGL(kfn, dim3(b->grid), dim3(NT), b->lds_bytes, st, a);
    }
    QSV_HIP_CHECK(hipGetLastError());
  }
  QSV_HIP_CHECK(hipMemcpyAsync(energies, a.energies, b->items.size() * sizeof(double),
                               hipMemcpyDeviceToHost, st));
  if (grads && b->total_params)
    QSV_HIP_CHECK(hipMemcpyAsync(grads, a.grads, size_t(b->total_params) * sizeof(double),
                                 hipMemcpyDeviceToHost, st));
  QSV_HIP_CHECK(hipStreamSynchronize(st));
  return QSV_OK;
}

void release_graph(qsv_batch* b) {
  if (b->graph_exec) (void)hipGraphExecDestroy(b->graph_exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->graph_exec = nullptr;
  b->graph = nullptr;
}

void release_device(qsv_batch* b) {
  release_graph(b);
  if (b->d_tables) (void)hipFree(b->d_tables);
  if (b->d_states) (void)hipFree(b->d_states);
  b->d_tables = b->d_states = nullptr;
  b->dev_dtype = 0;
  b->grid = 0;
}

}  // namespace

}  // namespace qsv

using namespace qsv;

extern "C" {

int qsv_batch_create(qsv_batch** out) {
  clear_error();
  if (!out) return fail(QSV_EINVAL, "null output handle");
  *out = new (std::nothrow) qsv_batch();
  return *out ? QSV_OK : fail(QSV_ENOMEM, "host allocation failed");
}

int qsv_batch_free(qsv_batch* b) {
  clear_error();
  if (!b) return QSV_OK;
  release_device(b);
  delete b;
  return QSV_OK;
}

int qsv_batch_add(qsv_batch* b, const qsv_circuit* c, const qsv_observable* o, const double* theta) {
  clear_error();
  if (!b || !c || !o) return fail(QSV_EINVAL, "null argument");
  if (c->n != o->n) return fail(QSV_ERANGE, "circuit and observable qubit counts differ");
  if (c->n < 2 || c->n > 24) return fail(QSV_ERANGE, "batched items take 2..24 qubits");
  if (c->nparams > 0 && !theta) return fail(QSV_EINVAL, "null theta");
  qsv_batch::Item it;
  it.c = *c;
  it.o = *o;
  if (c->nparams) it.theta.assign(theta, theta + c->nparams);
  b->items.push_back(std::move(it));
  release_device(b);
  return QSV_OK;
}

int qsv_batch_set_theta(qsv_batch* b, int item, const double* theta) {
  clear_error();
  if (!b) return fail(QSV_EINVAL, "null batch");
  if (item < 0 || item >= int(b->items.size())) return fail(QSV_ERANGE, "item out of range");
  auto& it = b->items[item];
  if (it.c.nparams && !theta) return fail(QSV_EINVAL, "null theta");
  std::copy(theta, theta + it.c.nparams, it.theta.begin());
  return QSV_OK;
}

int qsv_batch_info(const qsv_batch* b, int* items, int* total_params) {
  clear_error();
  if (!b) return fail(QSV_EINVAL, "null batch");
  int tp = 0;
  for (const auto& it : b->items) tp += it.c.nparams;
  if (items) *items = int(b->items.size());
  if (total_params) *total_params = tp;
  return QSV_OK;
}

int qsv_batch_autotune(qsv_batch* b, qsv_dtype dtype, void* stream, int reps, int* choice) {
  clear_error();
  if (!b) return fail(QSV_EINVAL, "null batch");
  if (dtype != QSV_C64 && dtype != QSV_C128) return fail(QSV_EDTYPE, "unknown dtype");
  if (reps < 1 || reps > 100) return fail(QSV_EINVAL, "reps must be in 1..100");
  if (b->items.empty()) return fail(QSV_EINVAL, "empty batch");
  hipStream_t st = static_cast<hipStream_t>(stream);
  int tp = 0;
  for (const auto& it : b->items) tp += it.c.nparams;
  std::vector<double> en(b->items.size()), gr(size_t(std::max(tp, 1)));
  // candidates: LDS bytes for psi + lambda (64 KiB: 12-qubit complex64 items
  // in LDS, 2^12 tiles; 32 KiB: more workgroups per CU), threads per workgroup
  const size_t ldsc[2] = {65536, 32768};
  const int thr[2] = {512, 256};
  double best_s = 0.0;
  size_t best_lds = 0;
  int best_thr = 0;
  for (size_t li = 0; li < 2; ++li) {
    for (int ti = 0; ti < 2; ++ti) {
      release_device(b);
      b->cfg_lds = ldsc[li];
      b->cfg_threads = thr[ti];
      int rc = build_device(b, dtype);
      auto run = [&]() {
        return dtype == QSV_C64 ? run_t<float>(b, st, en.data(), gr.data())
                                : run_t<double>(b, st, en.data(), gr.data());
      };
      if (!rc) rc = run();  // warm-up (and graph capture)
      if (rc) {
        release_device(b);
        if (rc == QSV_ENOMEM) {  // a shape that does not fit is skipped
          clear_error();
          continue;
        }
        return rc;
      }
      const auto t0 = std::chrono::steady_clock::now();
      for (int r = 0; r < reps && !rc; ++r) rc = run();
      const double sec = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      if (rc) {
        release_device(b);
        return rc;
      }
      if (best_thr == 0 || sec < best_s) {
        best_s = sec;
        best_lds = ldsc[li];
        best_thr = thr[ti];
      }
    }
  }
  release_device(b);
  if (best_thr == 0) return fail(QSV_ENOMEM, "autotune: no launch shape fits");
  b->cfg_lds = best_lds;
  b->cfg_threads = best_thr;
  if (choice) {
    choice[0] = int(best_lds / 1024);
    choice[1] = best_thr;
  }
  return QSV_OK;
}

int qsv_batch_set_graph(qsv_batch* b, int enable) {
  clear_error();
  if (!b) return fail(QSV_EINVAL, "null batch");
  b->use_graph = enable != 0;
  if (!b->use_graph) release_graph(b);
  return QSV_OK;
}

int qsv_batch_run(qsv_batch* b, qsv_dtype dtype, void* stream, double* energies, double* grads) {
  clear_error();
  if (!b) return fail(QSV_EINVAL, "null batch");
  if (!energies) return fail(QSV_EINVAL, "null energies");
  if (dtype != QSV_C64 && dtype != QSV_C128) return fail(QSV_EDTYPE, "unknown dtype");
  if (b->items.empty()) return QSV_OK;
  if (b->dev_dtype != int(dtype)) {
    release_device(b);
    int rc = build_device(b, dtype);
    if (rc) {
      release_device(b);
      return rc;
    }
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  return dtype == QSV_C64 ? run_t<float>(b, st, energies, grads) : run_t<double>(b, st, energies, grads);
}

}  // extern "C"
