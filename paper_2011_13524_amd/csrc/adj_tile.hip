// Tiled reverse sweep of the adjoint gradient.
//
// The per-gate reverse sweep (psi <- U^dagger psi, lambda <- U^dagger lambda,
// and -Im<lambda|P|psi> before each parametric rotation) reads and writes both
// states once per gate. Here the reversed, daggered gate list is scheduled into
// tile passes exactly like a forward fused plan: a pass keeps L qubits local,
// a workgroup holds the psi and lambda tiles in LDS, applies every op of the
// pass to both and evaluates each gradient term on the tile. Gradient terms go
// into per-workgroup FP64 partials (each workgroup owns a fixed set of tiles
// and adds them in a fixed order), reduced per parameter at the end. Two
// states are streamed once per pass instead of once per gate.
#include <algorithm>
#include <cmath>

#include "circuit.h"
#include "dev_common.h"
#include "plan.h"
#include "prof.h"
#include "tile_reg.h"

namespace qsv {

constexpr int kAdjTileThreads = 256;
constexpr int kAdjTileGrid = 2048;

// TileOpDev with kind 2 = parametric rotation exp(i t P/2) seen by the reverse
// sweep: k = Pauli id, lt[0] = local target or -1, gq[0] = global qubit (Z on
// a non-local qubit), moff = pool offset of exp(-i t P/2) (2x2), ins[0] =
// partial row. One LDS sweep adds -Im<lambda|P|psi> of the tile and multiplies
// both states by exp(-i t P/2).

// Dense one-qubit op on both states in one sweep (matrix in registers).
template <typename R>
__device__ __forceinline__ void adj_dense1(cx<R>* __restrict__ ts, cx<R>* __restrict__ tl,
                                           const TileOpDev& op, const cx<R>* __restrict__ mat, int L) {
  const cx<R> m00 = mat[0], m01 = mat[1], m10 = mat[2], m11 = mat[3];
  const int cnt = 1 << (L - op.m);
  const uint32_t o1 = op.off[1];
  for (int i = threadIdx.x; i < cnt; i += blockDim.x) {
    const uint32_t j0 = insert_zeros32(i, op.ins, op.m) | op.lcv;
    const cx<R> a = ts[j0], b = ts[j0 + o1], c = tl[j0], d = tl[j0 + o1];
    ts[j0] = cfma(m00, a, m01 * b);
    ts[j0 + o1] = cfma(m10, a, m11 * b);
    tl[j0] = cfma(m00, c, m01 * d);
    tl[j0 + o1] = cfma(m10, c, m11 * d);
  }
}

// Diagonal op on both states in one sweep.
template <typename R>
__device__ __forceinline__ void adj_diag(cx<R>* __restrict__ ts, cx<R>* __restrict__ tl,
                                         const TileOpDev& op, const cx<R>* __restrict__ d, int L,
                                         uint64_t base) {
  int gidx = 0;
  for (int b = 0; b < op.k; ++b)
    if (op.gq[b] >= 0) gidx |= int((base >> op.gq[b]) & 1) << b;
  const int TS = 1 << L;
  for (int j = threadIdx.x; j < TS; j += blockDim.x) {
    if ((uint32_t(j) & op.lcm) != op.lcv) continue;
    int idx = gidx;
    for (int b = 0; b < op.k; ++b)
      if (op.lt[b] >= 0) idx |= ((j >> op.lt[b]) & 1) << b;
    const cx<R> f = d[idx];
    ts[j] = f * ts[j];
    tl[j] = f * tl[j];
  }
}

// Gradient term of a rotation fused with its uncompute; returns this thread's
// share of -Im<lambda|P|psi> (taken before the uncompute).
template <typename R>
__device__ __forceinline__ double adj_rot(cx<R>* __restrict__ ps, cx<R>* __restrict__ la,
                                          const TileOpDev& op, const cx<R>* __restrict__ u, int L,
                                          uint64_t base) {
  double acc = 0.0;
  const int pauli = op.k;
  const int TS = 1 << L;
  const cx<R> u00 = u[0], u01 = u[1], u10 = u[2], u11 = u[3];
  if (pauli == 3) {
    // Z: sum_x (-1)^{x_q} Im(conj(lambda_x) psi_x); exp(-i t Z/2) is diagonal
    const int p = op.lt[0];
    if (p < 0) {
      const bool one = (base >> op.gq[0]) & 1;
      const double sg = one ? -1.0 : 1.0;
      const cx<R> f = one ? u11 : u00;
      for (int j = threadIdx.x; j < TS; j += blockDim.x) {
        const cx<R> a = ps[j], l = la[j];
        acc -= sg * (double(l.re) * a.im - double(l.im) * a.re);
        ps[j] = f * a;
        la[j] = f * l;
      }
    } else {
      for (int j = threadIdx.x; j < TS; j += blockDim.x) {
        const cx<R> a = ps[j], l = la[j];
        const bool one = (j >> p) & 1;
        const double im = double(l.re) * a.im - double(l.im) * a.re;
        acc -= one ? -im : im;
        const cx<R> f = one ? u11 : u00;
        ps[j] = f * a;
        la[j] = f * l;
      }
    }
  } else {
    const int p = op.lt[0];
    const uint32_t bit = 1u << p;
    for (int i = threadIdx.x; i < TS / 2; i += blockDim.x) {
      const uint32_t x0 = ((uint32_t(i) >> p) << (p + 1)) | (uint32_t(i) & (bit - 1));
      const uint32_t x1 = x0 | bit;
      const cx<R> a0 = ps[x0], a1 = ps[x1], l0 = la[x0], l1 = la[x1];
      const double a0r = a0.re, a0i = a0.im, a1r = a1.re, a1i = a1.im;
      const double l0r = l0.re, l0i = l0.im, l1r = l1.re, l1i = l1.im;
      double im;
      if (pauli == 1) im = (l0r * a1i - l0i * a1r) + (l1r * a0i - l1i * a0r);
      else im = -(l0r * a1r + l0i * a1i) + (l1r * a0r + l1i * a0i);
      acc -= im;
      ps[x0] = cfma(u00, a0, u01 * a1);
      ps[x1] = cfma(u10, a0, u11 * a1);
      la[x0] = cfma(u00, l0, u01 * l1);
      la[x1] = cfma(u10, l0, u11 * l1);
    }
  }
  return acc;
}

template <typename R, int KMAX>
__global__ void __launch_bounds__(kAdjTileThreads)
    k_tile_adj(R* __restrict__ psi, R* __restrict__ lam, const TilePassDev* __restrict__ passes,
               int pass_idx, const TileOpDev* __restrict__ ops, const cx<R>* __restrict__ pool,
               double* __restrict__ partial, uint64_t tiles) {
  extern __shared__ __align__(16) char smem[];
  __shared__ double red[kAdjTileThreads / 64];
  const TilePassDev& P = passes[pass_idx];
  const int L = P.L, b = P.b, nh = P.nh;
  const int TS = 1 << L;
  cx<R>* ts = reinterpret_cast<cx<R>*>(smem);
  cx<R>* tl = ts + TS;
  constexpr int V = sizeof(R) == 4 ? 2 : 1;
  const uint32_t lowmask = (1u << b) - 1;
  for (uint64_t g = blockIdx.x; g < tiles; g += gridDim.x) {
    uint64_t base = 0;
    for (int j = 0; j < P.ng; ++j) base |= ((g >> j) & 1) << P.gpos[j];
    __syncthreads();  // previous tile's stores have read the LDS tiles
    for (int e = threadIdx.x; e < TS / V; e += blockDim.x) {
      const uint32_t j = uint32_t(e) * V;
      const uint32_t h = j >> b;
      uint64_t x = base + (j & lowmask);
      for (int i = 0; i < nh; ++i) x |= uint64_t((h >> i) & 1) << P.hq[i];
      AmpIO<R, V>::load(psi, x, &ts[j]);
      AmpIO<R, V>::load(lam, x, &tl[j]);
    }
    __syncthreads();
    for (int o = 0; o < P.op_count; ++o) {
      const TileOpDev& op = ops[P.op_begin + o];
      if ((base & op.gcm) != op.gcv) continue;
      if (op.kind == 2) {
        double acc = adj_rot<R>(ts, tl, op, pool + op.moff, L, base);
#pragma unroll
        for (int s = 32; s > 0; s >>= 1) acc += __shfl_xor(acc, s, 64);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
        __syncthreads();
        if (threadIdx.x == 0) {
          double r = 0.0;
          for (int w = 0; w < kAdjTileThreads / 64; ++w) r += red[w];
          partial[size_t(op.ins[0]) * gridDim.x + blockIdx.x] += r;
        }
      } else if (op.kind == 1) {
        adj_diag<R>(ts, tl, op, pool + op.moff, L, base);
      } else if (op.k == 1) {
        adj_dense1<R>(ts, tl, op, pool + op.moff, L);
      } else {
        lds_op<R, KMAX>(ts, op, pool, L, base, NoSwz());
        lds_op<R, KMAX>(tl, op, pool, L, base, NoSwz());
      }
      __syncthreads();
    }
    for (int e = threadIdx.x; e < TS / V; e += blockDim.x) {
      const uint32_t j = uint32_t(e) * V;
      const uint32_t h = j >> b;
      uint64_t x = base + (j & lowmask);
      for (int i = 0; i < nh; ++i) x |= uint64_t((h >> i) & 1) << P.hq[i];
      AmpIO<R, V>::store(psi, x, &ts[j]);
      AmpIO<R, V>::store(lam, x, &tl[j]);
    }
  }
}


// rows[r] = sum of the cols partials of row r (fixed order)
__global__ void __launch_bounds__(kAdjTileThreads)
    k_rows_sum(const double* __restrict__ partial, int cols, double* __restrict__ rows) {
  __shared__ double red[kAdjTileThreads / 64];
  double acc = 0.0;
  const double* p = partial + size_t(blockIdx.x) * cols;
  for (int i = threadIdx.x; i < cols; i += blockDim.x) acc += p[i];
#pragma unroll
  for (int s = 32; s > 0; s >>= 1) acc += __shfl_xor(acc, s, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = 0.0;
    for (int w = 0; w < kAdjTileThreads / 64; ++w) r += red[w];
    rows[blockIdx.x] = r;
  }
}

__global__ void k_zero_doubles(double* __restrict__ p, uint64_t n) {
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = 0.0;
}

// ------------------------------------------------------------------ host

namespace {

struct BOp {
  int kind;  // 0 dense, 1 diagonal, 2 gradient
  std::vector<int> targets, controls, ctrl_vals;
  std::vector<cd> val;  // dense: matrix; diagonal: diagonal entries
  int pauli = 0, row = -1;
};

void dagger_inplace(std::vector<cd>& m, int D) {
  std::vector<cd> t(m.size());
  for (int r = 0; r < D; ++r)
    for (int c = 0; c < D; ++c) t[size_t(c) * D + r] = {m[size_t(r) * D + c].re, -m[size_t(r) * D + c].im};
  m.swap(t);
}

uint64_t qmask_of(const std::vector<int>& qs) {
  uint64_t m = 0;
  for (int q : qs) m |= uint64_t(1) << q;
  return m;
}

}  // namespace

// Reverse sweep by tile passes. On entry psi = psi_L and lam = H psi_L; on
// return both are uncomputed and rows[r] holds the gradient term of the r-th
// parametric rotation counted from the end (row_slot maps rows to slots).
template <typename R>
int adjoint_backward_tiled(const qsv_circuit* c, const double* theta, qsv_state* psi, qsv_state* lam,
                           std::vector<int>& row_slot, std::vector<double>& rows) {
  const int n = c->n;
  // reversed, daggered op list with gradient terms
  std::vector<BOp> ops;
  row_slot.clear();
  std::vector<cd> m;
  for (int gi = int(c->gates.size()) - 1; gi >= 0; --gi) {
    const Gate& g = c->gates[gi];
    if (g.kind == Gate::ROTATION && g.slot >= 0) {
      // gradient term fused with the uncompute exp(-i t P/2)
      BOp gr;
      gr.kind = 2;
      gr.pauli = g.pauli;
      gr.targets = g.targets;
      gr.row = int(row_slot.size());
      row_slot.push_back(g.slot);
      gr.val.resize(4);
      rotation_matrix(g.pauli, -theta[g.slot], gr.val.data());
      ops.push_back(gr);
      continue;
    }
    gate_matrix(g, theta, m);
    std::vector<int> tq = g.targets;
    dagger_inplace(m, 1 << tq.size());
    uint64_t cm = 0, cv = 0;
    for (size_t j = 0; j < g.controls.size(); ++j) {
      cm |= uint64_t(1) << g.controls[j];
      if (g.ctrl_vals[j]) cv |= uint64_t(1) << g.controls[j];
    }
    extract_controls(m, tq, cm, cv);
    const int D = 1 << tq.size();
    bool diag = true;
    for (int r = 0; r < D && diag; ++r)
      for (int cc = 0; cc < D && diag; ++cc)
        if (r != cc && !(m[size_t(r) * D + cc].re == 0 && m[size_t(r) * D + cc].im == 0)) diag = false;
    BOp op;
    op.kind = diag ? 1 : 0;
    op.targets = tq;
    for (int q = 0; q < 64; ++q)
      if (cm >> q & 1) {
        op.controls.push_back(q);
        op.ctrl_vals.push_back(int(cv >> q & 1));
      }
    if (diag) {
      if (tq.size() > 5) return fail(QSV_EINVAL, "diagonal gate too wide for the tiled sweep");
      for (int i = 0; i < D; ++i) op.val.push_back(m[size_t(i) * D + i]);
    } else {
      op.val = m;
    }
    ops.push_back(op);
  }
  // passes (as in the forward planner): dense targets must be local
  const int Lc = sizeof(R) == 4 ? 12 : 11;
  const int L = std::min(n, Lc);
  const int b = std::min(L, sizeof(R) == 4 ? 4 : 3);  // 128-byte contiguous runs
  const uint64_t low = (uint64_t(1) << b) - 1;
  std::vector<std::vector<int>> pass_ops;
  std::vector<uint64_t> pass_local;
  std::vector<int> rem(ops.size());
  for (size_t i = 0; i < ops.size(); ++i) rem[i] = int(i);
  while (!rem.empty()) {
    uint64_t local = low, blocked = 0;
    std::vector<int> take, deferred;
    for (int oi : rem) {
      const BOp& o = ops[oi];
      const uint64_t all = qmask_of(o.targets) | qmask_of(o.controls);
      if (all & blocked) {
        deferred.push_back(oi);
        blocked |= all;
        continue;
      }
      uint64_t dense = 0;
      if (o.kind == 0 || (o.kind == 2 && o.pauli != 3)) dense = qmask_of(o.targets);
      const uint64_t need = dense & ~local;
      if (__builtin_popcountll(local | need) <= L) {
        local |= need;
        take.push_back(oi);
      } else {
        deferred.push_back(oi);
        blocked |= all;
      }
    }
    if (take.empty()) return fail(QSV_EINVAL, "internal: tiled sweep made no progress");
    for (int q = 0; q < n && __builtin_popcountll(local) < L; ++q) local |= uint64_t(1) << q;
    pass_ops.push_back(take);
    pass_local.push_back(local);
    rem.swap(deferred);
  }
  // device tables
  std::vector<TilePassDev> hp;
  std::vector<TileOpDev> ho;
  std::vector<cx<R>> pool;
  int kmax = 1;
  for (size_t pi = 0; pi < pass_ops.size(); ++pi) {
    const uint64_t local = pass_local[pi];
    std::vector<int> lpos(64, -1), loc;
    for (int q = 0; q < n; ++q)
      if (local >> q & 1) {
        lpos[q] = int(loc.size());
        loc.push_back(q);
      }
    TilePassDev d{};
    d.L = L;
    d.b = b;
    d.nh = L - b;
    for (int i = 0; i < d.nh; ++i) d.hq[i] = loc[b + i];
    d.ng = 0;
    for (int q = 0; q < n; ++q)
      if (!(local >> q & 1)) d.gpos[d.ng++] = q;
    d.op_begin = int(ho.size());
    d.op_count = int(pass_ops[pi].size());
    for (int oi : pass_ops[pi]) {
      const BOp& o = ops[oi];
      TileOpDev t{};
      for (int j = 0; j < 5; ++j) t.lt[j] = t.gq[j] = -1;
      if (o.kind == 2) {
        t.kind = 2;
        t.k = o.pauli;
        t.ins[0] = o.row;
        t.moff = int(pool.size());
        for (const cd& v : o.val) pool.push_back({R(v.re), R(v.im)});
        const int q = o.targets[0];
        if (lpos[q] >= 0) t.lt[0] = lpos[q];
        else t.gq[0] = q;
        ho.push_back(t);
        continue;
      }
      t.kind = o.kind;
      t.k = int(o.targets.size());
      t.moff = int(pool.size());
      for (const cd& v : o.val) pool.push_back({R(v.re), R(v.im)});
      for (size_t j = 0; j < o.controls.size(); ++j) {
        const int q = o.controls[j];
        if (lpos[q] >= 0) {
          t.lcm |= 1u << lpos[q];
          if (o.ctrl_vals[j]) t.lcv |= 1u << lpos[q];
        } else {
          t.gcm |= uint64_t(1) << q;
          if (o.ctrl_vals[j]) t.gcv |= uint64_t(1) << q;
        }
      }
      for (int j = 0; j < t.k; ++j) {
        const int q = o.targets[j];
        if (lpos[q] >= 0) t.lt[j] = lpos[q];
        else t.gq[j] = q;
      }
      if (t.kind == 0) {
        kmax = std::max(kmax, t.k);
        uint32_t ins = t.lcm;
        for (int j = 0; j < t.k; ++j) ins |= 1u << t.lt[j];
        if (__builtin_popcount(ins) > 10) return fail(QSV_EINVAL, "too many local controls on one gate");
        t.m = 0;
        for (int q = 0; q < 32; ++q)
          if (ins >> q & 1) t.ins[t.m++] = q;
        for (int i = 0; i < (1 << t.k); ++i) {
          uint32_t off = 0;
          for (int j = 0; j < t.k; ++j)
            if (i >> j & 1) off |= 1u << t.lt[j];
          t.off[i] = off;
        }
      }
      ho.push_back(t);
    }
    hp.push_back(d);
  }
  const int nrows = int(row_slot.size());
  const uint64_t tiles = dim(n - L);
  const int G = int(std::min<uint64_t>(tiles, kAdjTileGrid));
  // one device allocation: passes | ops | pool | partial[nrows x G] | rows[nrows]
  auto al = [](size_t x) { return (x + 255) / 256 * 256; };
  const size_t o_ops = al(hp.size() * sizeof(TilePassDev));
  const size_t o_pool = o_ops + al(std::max<size_t>(1, ho.size()) * sizeof(TileOpDev));
  const size_t o_part = o_pool + al(std::max<size_t>(1, pool.size()) * sizeof(cx<R>));
  const size_t o_rows = o_part + al(std::max<size_t>(1, size_t(nrows) * G) * sizeof(double));
  const size_t total = o_rows + al(std::max(1, nrows) * sizeof(double));
  char* d = nullptr;
  if (hipMalloc(reinterpret_cast<void**>(&d), total) != hipSuccess)
    return fail(QSV_ENOMEM, "tiled sweep tables allocation failed");
  hipStream_t st = psi->stream;
  int rc = QSV_OK;
  auto fin = [&](int r) {
    (void)hipStreamSynchronize(st);
    (void)hipFree(d);
    return r;
  };
  if (hipMemcpyAsync(d, hp.data(), hp.size() * sizeof(TilePassDev), hipMemcpyHostToDevice, st) != hipSuccess ||
      (!ho.empty() && hipMemcpyAsync(d + o_ops, ho.data(), ho.size() * sizeof(TileOpDev),
                                     hipMemcpyHostToDevice, st) != hipSuccess) ||
      (!pool.empty() && hipMemcpyAsync(d + o_pool, pool.data(), pool.size() * sizeof(cx<R>),
                                       hipMemcpyHostToDevice, st) != hipSuccess))
    return fin(fail(QSV_EHIP, "tiled sweep table upload failed"));
  double* part = reinterpret_cast<double*>(d + o_part);
  hipLaunchKernelGGL(k_zero_doubles, dim3(256), dim3(256), 0, st, part, uint64_t(nrows) * G);
  const size_t lds = 2 * (size_t(1) << L) * sizeof(cx<R>);
  for (const void* k : {reinterpret_cast<const void*>(&k_tile_adj<R, 2>),
                        reinterpret_cast<const void*>(&k_tile_adj<R, 3>),
                        reinterpret_cast<const void*>(&k_tile_adj<R, 5>)})
    if (hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)) != hipSuccess)
      return fin(fail(QSV_EHIP, "cannot raise LDS limit of the tiled sweep"));
  for (size_t pi = 0; pi < hp.size(); ++pi) {
    ProfScope ps("adjoint", 4.0 * sizeof(cx<R>) * double(dim(n)), st);
#define QSV_ADJ_LAUNCH(KM)                                                                       \
  hipLaunchKernelGGL((k_tile_adj<R, KM>), dim3(G), dim3(kAdjTileThreads), lds, st,               \
                     static_cast<R*>(psi->ptr), static_cast<R*>(lam->ptr),                      \
                     reinterpret_cast<const TilePassDev*>(d), int(pi),                          \
                     reinterpret_cast<const TileOpDev*>(d + o_ops),                             \
                     reinterpret_cast<const cx<R>*>(d + o_pool), part, tiles)
    if (kmax <= 2) QSV_ADJ_LAUNCH(2);
    else if (kmax <= 3) QSV_ADJ_LAUNCH(3);
    else QSV_ADJ_LAUNCH(5);
#undef QSV_ADJ_LAUNCH
    if (hipGetLastError() != hipSuccess) return fin(fail(QSV_EHIP, "tiled sweep launch failed"));
  }
  rows.assign(nrows, 0.0);
  if (nrows > 0) {
    hipLaunchKernelGGL(k_rows_sum, dim3(nrows), dim3(kAdjTileThreads), 0, st, part, G,
                       reinterpret_cast<double*>(d + o_rows));
    if (hipMemcpyAsync(rows.data(), d + o_rows, nrows * sizeof(double), hipMemcpyDeviceToHost, st) !=
        hipSuccess)
      return fin(fail(QSV_EHIP, "gradient download failed"));
  }
  return fin(rc);
}

template int adjoint_backward_tiled<float>(const qsv_circuit*, const double*, qsv_state*, qsv_state*,
                                           std::vector<int>&, std::vector<double>&);
template int adjoint_backward_tiled<double>(const qsv_circuit*, const double*, qsv_state*, qsv_state*,
                                            std::vector<int>&, std::vector<double>&);

}  // namespace qsv
