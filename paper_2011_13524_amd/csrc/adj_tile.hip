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
#include <cstdlib>

#include "circuit.h"
#include "dev_common.h"
#include "plan.h"
#include "prof.h"
#include "tile_reg.h"
#include "wave_sum.h"

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

// -Im of i^ph (sr + i si).
__device__ __forceinline__ double neg_im_phase(double sr, double si, int ph) {
  switch (ph & 3) {
    case 0: return -si;
    case 1: return -sr;
    case 2: return si;
    default: return sr;
  }
}

// Gradient term of a multi-qubit Pauli rotation exp(i t P/2) (TileOpDev kind
// 3): this thread's share of -Im<lambda|P|psi> over the tile, with
// (P psi)_x = i^ph (-1)^{|x & zy|} psi_{x ^ f} (the constant part of the sign
// folded into ph on the host; Z/Y factors on non-local qubits give the tile's
// sign). The states are not changed.
template <typename R>
__device__ __forceinline__ double adj_pauli_grad(const cx<R>* __restrict__ ps, const cx<R>* __restrict__ la,
                                                 const TileOpDev& op, int L, uint64_t base) {
  const uint32_t lf = op.off[0], zl = op.off[1];
  const uint64_t zg = uint64_t(op.off[3]) | (uint64_t(op.off[4]) << 32);
  const uint32_t gs = uint32_t(__popcll(base & zg) & 1);
  const int TS = 1 << L;
  double sr = 0.0, si = 0.0;
  for (int j = threadIdx.x; j < TS; j += blockDim.x) {
    const cx<R> a = ps[uint32_t(j) ^ lf], l = la[j];
    const double wr = double(l.re) * a.re + double(l.im) * a.im;
    const double wi = double(l.re) * a.im - double(l.im) * a.re;
    const bool neg = ((__popc(uint32_t(j) & zl) & 1) ^ gs) != 0;
    sr += neg ? -wr : wr;
    si += neg ? -wi : wi;
  }
  return neg_im_phase(sr, si, int(op.off[2]));
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
      if (op.kind == 2 || op.kind == 3) {
        double acc = op.kind == 2 ? adj_rot<R>(ts, tl, op, pool + op.moff, L, base)
                                  : adj_pauli_grad<R>(ts, tl, op, L, base);
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


// ------------------------------------------------------------------ register-resident sweep
//
// The reverse sweep with both tiles (psi and lambda) register-resident, using
// the segment layouts of the forward tile passes: ops on register bits run on
// both states from registers, X / CNOT ops fold into the LDS re-maps (a
// permutation of indices, applied to both states), and a rotation's gradient
// term -Im<lambda|P|psi> is evaluated on the register pairs just before its
// uncompute. Per gradient op, each wavefront sums its share (fixed order) into
// its own LDS slot; workgroups are persistent over a contiguous range of tiles
// and write one FP64 partial per (row, workgroup) at the end of the pass.
constexpr int kAdjMaxRows = 64;  // gradient rows per pass (LDS slots)

// X/Y rotation on register bit P: share of -Im<lambda|P|psi>, then
// psi, lambda <- u psi, u lambda (u = exp(-i t P/2)); writes every slot of os, ol.
// u = c I - i s' P has a real diagonal c and off-diagonals s' (Y: real, -s'
// below the diagonal) or i s' (X), so each output takes two real products
// per component instead of a complex 2x2 product. The gradient share is
// summed in the amplitude precision over the thread's pairs (complex64:
// FP32 products and 8-term sums, relative error <= 11 x 2^-24 of
// sum |lambda_x||psi_y| <= |lambda||psi|; the caller sums in FP64).
template <typename R, int NR, int P>
__device__ __forceinline__ double grad_xy(const cx<R>* s, const cx<R>* l, cx<R>* os, cx<R>* ol, bool ypauli,
                                          const cx<R>* __restrict__ u) {
  if constexpr ((1 << P) >= NR) {  // no such register bit (never selected)
    reg_copy<R, NR>(s, os);
    reg_copy<R, NR>(l, ol);
    return 0.0;
  }
  const R c = u[0].re, sn = ypauli ? u[1].re : u[1].im;
  R acc = R(0);
#pragma unroll
  for (int g = 0; g < NR / 2; ++g) {
    const int i = ins1<P>(g), j = i | (1 << P);
    const cx<R> a0 = s[i], a1 = s[j], l0 = l[i], l1 = l[j];
    const R im = ypauli ? fma(l1.re, a0.re, l1.im * a0.im) - fma(l0.re, a1.re, l0.im * a1.im)
                        : fma(l0.re, a1.im, -(l0.im * a1.re)) + fma(l1.re, a0.im, -(l1.im * a0.re));
    acc -= im;
    if (ypauli) {  // u = [[c, s'], [-s', c]]
      os[i] = {fma(c, a0.re, sn * a1.re), fma(c, a0.im, sn * a1.im)};
      os[j] = {fma(c, a1.re, -(sn * a0.re)), fma(c, a1.im, -(sn * a0.im))};
      ol[i] = {fma(c, l0.re, sn * l1.re), fma(c, l0.im, sn * l1.im)};
      ol[j] = {fma(c, l1.re, -(sn * l0.re)), fma(c, l1.im, -(sn * l0.im))};
    } else {  // u = [[c, i s'], [i s', c]]
      os[i] = {fma(c, a0.re, -(sn * a1.im)), fma(c, a0.im, sn * a1.re)};
      os[j] = {fma(c, a1.re, -(sn * a0.im)), fma(c, a1.im, sn * a0.re)};
      ol[i] = {fma(c, l0.re, -(sn * l1.im)), fma(c, l0.im, sn * l1.re)};
      ol[j] = {fma(c, l1.re, -(sn * l0.im)), fma(c, l1.im, sn * l0.re)};
    }
  }
  return double(acc);
}

// Z rotation: the bit of the target is register bit P (P >= 0) or `fixed`;
// share of -Im<lambda|Z|psi> (summed in the amplitude precision over the
// thread's elements, as for grad_xy), then the diagonal u on both states.
template <typename R, int NR, int P>
__device__ __forceinline__ double grad_z(const cx<R>* s, const cx<R>* l, cx<R>* os, cx<R>* ol, int fixed,
                                         const cx<R>* __restrict__ u) {
  if constexpr (P >= 0 && (1 << P) >= NR) {  // no such register bit (never selected)
    reg_copy<R, NR>(s, os);
    reg_copy<R, NR>(l, ol);
    return 0.0;
  }
  const cx<R> f0 = u[0], f1 = u[3];
  R acc = R(0);
#pragma unroll
  for (int i = 0; i < NR; ++i) {
    const int bit = P >= 0 ? (i >> P) & 1 : fixed;
    const cx<R> a = s[i], c = l[i];
    const R im = fma(c.re, a.im, -(c.im * a.re));
    acc -= bit ? -im : im;
    const cx<R> f = csel(bit != 0, f1, f0);
    os[i] = f * a;
    ol[i] = f * c;
  }
  return double(acc);
}

// Gradient op: share of the gradient from (s, l), the rotation applied into
// (os, ol) (every element written).
template <typename R, int NR>
__device__ __forceinline__ double grad_apply(const cx<R>* s, const cx<R>* l, cx<R>* os, cx<R>* ol,
                                             const RegOpDev& op, uint32_t tau, uint64_t base,
                                             const cx<R>* __restrict__ u) {
  double acc = 0.0;
  if (op.kind == 5) {
    const bool y = op.k == 2;
    switch (op.p1) {
      case 0: acc = grad_xy<R, NR, 0>(s, l, os, ol, y, u); break;
      case 1: acc = grad_xy<R, NR, 1>(s, l, os, ol, y, u); break;
      case 2: acc = grad_xy<R, NR, 2>(s, l, os, ol, y, u); break;
      default: acc = grad_xy<R, NR, 3>(s, l, os, ol, y, u); break;
    }
  } else {
    int fixed = 0, p = -1;
    if (op.dsrc[0] == 0) p = op.dbit[0];
    else if (op.dsrc[0] == 1) fixed = int((tau >> op.dbit[0]) & 1);
    else fixed = int((base >> op.dbit[0]) & 1);
    switch (p) {
      case 0: acc = grad_z<R, NR, 0>(s, l, os, ol, 0, u); break;
      case 1: acc = grad_z<R, NR, 1>(s, l, os, ol, 0, u); break;
      case 2: acc = grad_z<R, NR, 2>(s, l, os, ol, 0, u); break;
      case 3: acc = grad_z<R, NR, 3>(s, l, os, ol, 0, u); break;
      default: acc = grad_z<R, NR, -1>(s, l, os, ol, fixed, u); break;
    }
  }
  return acc;
}

// Re-map of one state's registers through LDS (write in the old layout with
// the folded map, read in the new one).
// close: a cross-wave re-map ends with a workgroup barrier (another state's
// re-map writes next); otherwise that barrier is left to the next LDS write.
template <typename R, int RB, int TB>
__device__ __forceinline__ void adj_remap(cx<R> (&v)[1 << RB], const LdsMap<R, RB, TB>& mo,
                                          const LdsMap<R, RB, TB>& mn, bool xw, bool close, char* smem) {
#pragma unroll
  for (int i = 0; i < (1 << RB); ++i) mo.put(smem, i, v[i]);
  if (xw) __syncthreads();
  else wave_sync();
#pragma unroll
  for (int i = 0; i < (1 << RB); ++i) v[i] = mn.get(smem, i);
  if (!xw) wave_sync();
  else if (close) __syncthreads();
}

// A block applied through LDS to one state held in registers (v in, o out).
template <typename R, int RB, int TB, int KMAX, typename SW>
__device__ __forceinline__ void adj_lds_op(const cx<R>* v, cx<R>* o, const LdsMap<R, RB, TB>& ms,
                                           char* smem, const TileOpDev& op, const cx<R>* pool, int L,
                                           uint64_t base, SW sw) {
#pragma unroll
  for (int i = 0; i < (1 << RB); ++i) ms.put(smem, i, v[i]);
  __syncthreads();
  lds_op<R, KMAX>(reinterpret_cast<cx<R>*>(smem), op, pool, L, base, sw);
  __syncthreads();
#pragma unroll
  for (int i = 0; i < (1 << RB); ++i) o[i] = ms.get(smem, i);
  __syncthreads();
}

// One op of the reverse sweep on both states: reads (s, l) and writes every
// element of (os, ol); gradient ops add this wavefront's share to its slot.
template <typename R, int RB, int KMAX, int TB>
__device__ __forceinline__ void adj_step(const RegOpDev& opr, const cx<R>* s, const cx<R>* l, cx<R>* os,
                                         cx<R>* ol, const RegSegDev& S, uint32_t tau, uint64_t base,
                                         Swz<sizeof(R) == 4 ? 5 : 4> sw, char* smem,
                                         const TileOpDev* __restrict__ lops, const cx<R>* __restrict__ pool,
                                         int L, double* wslot) {
  constexpr int NR = 1 << RB;
  const RegOpDev op = opr;  // (one burst of scalar loads)
  if ((base & op.gcm) != op.gcv) {  // non-local controls: uniform per tile
    reg_copy<R, NR>(s, os);
    reg_copy<R, NR>(l, ol);
    return;
  }
  const cx<R>* m = pool + op.moff;
  if (op.kind == 8) {
    // Pauli-string gradient: psi staged in LDS in this segment's layout; the
    // partner x ^ f of element i is at its address XOR pf_lds (the swizzle is
    // linear over XOR and the tile starts at LDS address 0)
    const LdsMap<R, RB, TB> ms(S.get_reg, S.get_tcol, 0u, tau);
    __syncthreads();  // (a preceding cross-wave re-map's reads are done)
#pragma unroll
    for (int i = 0; i < NR; ++i) ms.put(smem, i, s[i]);
    __syncthreads();
    typedef R R2 __attribute__((ext_vector_type(2)));
    typedef __attribute__((address_space(3))) R2 lds_r2;
    const uint32_t tpar = uint32_t(__popc(tau & op.pz_thr) + __popcll(base & op.pz_glob)) & 1u;
    double sr = 0.0, si = 0.0;
#pragma unroll
    for (int i = 0; i < NR; ++i) {
      const R2 av = *reinterpret_cast<lds_r2*>(uintptr_t(reinterpret_cast<uintptr_t>(ms.at(smem, i)) ^ op.pf_lds));
      const cx<R> c = l[i];
      const double wr = double(c.re) * av.x + double(c.im) * av.y;
      const double wi = double(c.re) * av.y - double(c.im) * av.x;
      const bool neg = ((uint32_t(__popc(uint32_t(i) & op.pz_reg)) ^ tpar) & 1u) != 0;
      sr += neg ? -wr : wr;
      si += neg ? -wi : wi;
      os[i] = s[i];
      ol[i] = c;
    }
    __syncthreads();  // every read done before the LDS tile is written again
    const double acc = wave_sum_to_last(neg_im_phase(sr, si, op.pph));
    if ((tau & 63) == 63) wslot[op.aux * (1 << (TB - 6))] += acc;
    return;
  }
  if (op.kind == 5 || op.kind == 6) {
    const double acc = wave_sum_to_last(grad_apply<R, NR>(s, l, os, ol, op, tau, base, m));
    if ((tau & 63) == 63) wslot[op.aux * (1 << (TB - 6))] += acc;
    return;
  }
  if (op.kind == 3) {
    const LdsMap<R, RB, TB> ms(S.get_reg, S.get_tcol, 0u, tau);
    __syncthreads();  // (a preceding cross-wave re-map's reads are done)
    adj_lds_op<R, RB, TB, KMAX>(s, os, ms, smem, lops[op.lop], pool, L, base, sw);
    adj_lds_op<R, RB, TB, KMAX>(l, ol, ms, smem, lops[op.lop], pool, L, base, sw);
    return;
  }
  cx<R> gtab[4];
  int a = op.p1, bb = op.p2;
  if (op.kind == 2) diag_table<R>(op, m, tau, base, gtab, a, bb);
  const bool lane = (tau & op.ti_cm) == op.ti_cv;
  reg_apply<R, NR, false>(s, os, op.key, m, gtab, op.ri_cm, op.ri_cv, lane, pool, op.lm);
  reg_apply<R, NR, false>(l, ol, op.key, m, gtab, op.ri_cm, op.ri_cv, lane, pool, op.lm);
}

template <typename R, int RB, int KMAX, int TB>
__global__ void __launch_bounds__(1 << TB)
    k_adj_reg(R* __restrict__ psi, R* __restrict__ lam, const TilePassDev* __restrict__ passes, int pass_idx,
              const RegSegDev* __restrict__ segs, const RegOpDev* __restrict__ rops,
              const TileOpDev* __restrict__ lops, const cx<R>* __restrict__ pool,
              const int* __restrict__ prow, double* __restrict__ partial, uint64_t ntiles) {
  constexpr int NR = 1 << RB;
  constexpr int NW = 1 << (TB - 6);  // wavefronts per workgroup
  constexpr int SB = sizeof(R) == 4 ? 5 : 4;
  const Swz<SB> sw;
  // one dynamic LDS block: the tile (first, at LDS address 0, as the re-map
  // addressing requires) then the gradient slots [row][wave]
  extern __shared__ __align__(16) char smem[];
  const TilePassDev& P = passes[pass_idx];
  const int L = P.L;
  double(*slot)[NW] = reinterpret_cast<double(*)[NW]>(smem + (size_t(1) << L) * sizeof(cx<R>));
  const uint32_t tau = threadIdx.x;
  const int wave = int(tau >> 6);
  for (int i = int(tau); i < kAdjMaxRows * NW; i += blockDim.x) slot[i / NW][i % NW] = 0.0;
  // tiles of this workgroup: a contiguous range (fixed order of its partial sums)
  uint64_t gmask = 0;
  for (int r = 0; r < P.nrun; ++r) gmask |= ((uint64_t(1) << P.rlen[r]) - 1) << P.rdst[r];
  const uint64_t per = (ntiles + gridDim.x - 1) / gridDim.x;
  const uint64_t g0 = uint64_t(blockIdx.x) * per;
  const uint64_t gend = g0 + per < ntiles ? g0 + per : ntiles;
  uint64_t base = 0;
  for (int r = 0; r < P.nrun; ++r) base |= ((g0 >> P.rsrc[r]) & ((uint64_t(1) << P.rlen[r]) - 1)) << P.rdst[r];
  const RegSegDev* S0 = &segs[P.seg_begin];
  const RegSegDev* SL = &segs[P.seg_begin + P.seg_count - 1];
  // HBM address parts of the first and last layouts: per thread (fixed for
  // the kernel) and per register element (uniform columns)
  uint64_t th0 = 0, thL = 0;
#pragma unroll
  for (int k = 0; k < TB; ++k) {
    const uint64_t on = uint64_t(0) - ((tau >> k) & 1);
    th0 |= S0->gcol_t[k] & on;
    thL |= SL->gcol_t[k] & on;
  }
  auto addr = [&](const RegSegDev& s, uint64_t th, uint64_t bs, int i) -> uint64_t {
    uint64_t x = bs | th;
#pragma unroll
    for (int k = 0; k < RB; ++k)
      if ((i >> k) & 1) x |= s.gcol_r[k];
    return x;
  };
  cx<R> vs[NR], vl[NR], ws[NR], wl[NR];
  for (uint64_t g = g0; g < gend; ++g) {
    if (g > g0) base = ((base | ~gmask) + 1) & gmask;
    // HBM -> registers in the first segment's layout
    if (sizeof(R) == 4 && S0->reg[0] == 0) {
#pragma unroll
      for (int i = 0; i < NR; i += 2) {
        const uint64_t x = addr(*S0, th0, base, i);
        AmpIO<R, 2>::load(psi, x, &vs[i]);
        AmpIO<R, 2>::load(lam, x, &vl[i]);
      }
    } else {
#pragma unroll
      for (int i = 0; i < NR; ++i) {
        const uint64_t x = addr(*S0, th0, base, i);
        AmpIO<R, 1>::load(psi, x, &vs[i]);
        AmpIO<R, 1>::load(lam, x, &vl[i]);
      }
    }
    __syncthreads();  // the previous tile's last LDS reads are done (and the slots cleared)
    const RegSegDev* S = S0;
    for (int sgi = 0; sgi < P.seg_count; ++sgi) {
      const RegSegDev* Sn = &segs[P.seg_begin + sgi];
      if (sgi > 0) {
        // re-map both states through LDS (folded X / CNOT ops applied to both)
        const bool xw = (Sn->xwave & 1) != 0;
        if (Sn->xwave & 2) __syncthreads();
        const LdsMap<R, RB, TB> mo(Sn->put_reg, Sn->put_tcol, Sn->put_tcst, tau);
        const LdsMap<R, RB, TB> mn(Sn->get_reg, Sn->get_tcol, 0u, tau);
        adj_remap<R, RB, TB>(vs, mo, mn, xw, true, smem);
        adj_remap<R, RB, TB>(vl, mo, mn, xw, false, smem);
      }
      S = Sn;
      // ops alternate between the register arrays (vs, vl) and (ws, wl)
      const int oc = S->op_count, ob = S->op_begin;
      for (int o = 0; o < oc; o += 2) {
        adj_step<R, RB, KMAX, TB>(rops[ob + o], vs, vl, ws, wl, *S, tau, base, sw, smem, lops, pool, L,
                                  &slot[0][wave]);
        if (o + 1 < oc) {
          adj_step<R, RB, KMAX, TB>(rops[ob + o + 1], ws, wl, vs, vl, *S, tau, base, sw, smem, lops, pool, L,
                                    &slot[0][wave]);
        } else {
          reg_copy<R, NR>(ws, vs);
          reg_copy<R, NR>(wl, vl);
        }
      }
    }
    // registers -> HBM in the last segment's layout
    if (sizeof(R) == 4 && SL->reg[0] == 0) {
#pragma unroll
      for (int i = 0; i < NR; i += 2) {
        const uint64_t x = addr(*SL, thL, base, i);
        AmpIO<R, 2>::store(psi, x, &vs[i]);
        AmpIO<R, 2>::store(lam, x, &vl[i]);
      }
    } else {
#pragma unroll
      for (int i = 0; i < NR; ++i) {
        const uint64_t x = addr(*SL, thL, base, i);
        AmpIO<R, 1>::store(psi, x, &vs[i]);
        AmpIO<R, 1>::store(lam, x, &vl[i]);
      }
    }
  }
  __syncthreads();
  for (int r = int(tau); r < P.row_count; r += blockDim.x) {
    double sum = 0.0;
    for (int w = 0; w < NW; ++w) sum += slot[r][w];
    partial[size_t(prow[P.row_begin + r]) * gridDim.x + blockIdx.x] = sum;
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
  std::vector<int> paulis;  // kind 3: Pauli ids (1..3) of the string on targets
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
    if (g.kind == Gate::PAULI && g.slot >= 0) {
      // gradient term -Im<lambda|P|psi> of exp(i t P/2) (its own op), then the
      // uncompute exp(-i t P/2) as an ordinary gate below
      BOp gr;
      gr.kind = 3;
      gr.targets = g.targets;
      gr.paulis = g.paulis;
      gr.row = int(row_slot.size());
      row_slot.push_back(g.slot);
      ops.push_back(gr);
    }
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
  // passes (as in the forward planner): dense targets must be local. complex64
  // states of at least one 2^12 tile run register-resident (256 threads x 16
  // amplitudes per state), at most kAdjMaxRows gradient rows per pass
  const int Lc = sizeof(R) == 4 ? 12 : 11;
  const int L = std::min(n, Lc);
  // complex64: 256 threads x 16 amplitudes per state; complex128: 256 x 8
  const bool reg = n >= Lc;
  SegCfg cfg{sizeof(R) == 4 ? 4 : 3, 8, sizeof(R) == 4, sizeof(R) == 4 && tile_mfma_default()};
  cfg.layers = false;  // (k_adj_reg has no layer variants)
  const int b = std::min(L, sizeof(R) == 4 ? 4 : 3);  // 128-byte contiguous runs
  const uint64_t low = (uint64_t(1) << b) - 1;
  std::vector<std::vector<int>> pass_ops;
  std::vector<uint64_t> pass_local;
  std::vector<int> rem(ops.size());
  for (size_t i = 0; i < ops.size(); ++i) rem[i] = int(i);
  while (!rem.empty()) {
    uint64_t local = low, blocked = 0;
    std::vector<int> take, deferred;
    int nrow = 0;
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
      if (o.kind == 3)  // the X/Y qubits of the string: pairs x, x ^ f in one tile
        for (size_t j = 0; j < o.targets.size(); ++j)
          if (o.paulis[j] != 3) dense |= uint64_t(1) << o.targets[j];
      const uint64_t need = dense & ~local;
      const bool grad = o.kind == 2 || o.kind == 3;
      const bool rows_full = reg && grad && nrow >= kAdjMaxRows;
      if (!rows_full && __builtin_popcountll(local | need) <= L) {
        if (grad) ++nrow;
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
  std::vector<int> prow;  // gradient rows of each pass, in slot order
  std::vector<RegSegDev> segs;
  std::vector<RegOpDev> rops;
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
    pass_runs(d);
    d.op_begin = int(ho.size());
    d.op_count = int(pass_ops[pi].size());
    d.row_begin = int(prow.size());
    d.row_count = 0;
    for (int oi : pass_ops[pi]) {
      const BOp& o = ops[oi];
      TileOpDev t{};
      for (int j = 0; j < 5; ++j) t.lt[j] = t.gq[j] = -1;
      if (o.kind == 3) {
        t.kind = 3;
        t.k = int(o.targets.size());
        t.ins[0] = o.row;
        t.ins[1] = d.row_count++;
        prow.push_back(o.row);
        uint32_t lf = 0, zl = 0;
        uint64_t zg = 0;
        int ny = 0;
        for (size_t j = 0; j < o.targets.size(); ++j) {
          const int q = o.targets[j], pid = o.paulis[j];
          if (pid == 2) ++ny;
          if (pid != 3) lf |= 1u << lpos[q];  // (X/Y qubits are local)
          if (pid != 1) {
            if (lpos[q] >= 0) zl |= 1u << lpos[q];
            else zg |= uint64_t(1) << q;
          }
        }
        t.off[0] = lf;
        t.off[1] = zl;
        // (P psi)_x = i^nY (-1)^{|(x ^ f) & zy|} psi_{x ^ f}; the part of the
        // sign from f & zy is a constant: two more quarter turns when odd
        t.off[2] = uint32_t((ny + 2 * (__builtin_popcount(lf & zl) & 1)) & 3);
        t.off[3] = uint32_t(zg);
        t.off[4] = uint32_t(zg >> 32);
        ho.push_back(t);
        continue;
      }
      if (o.kind == 2) {
        t.kind = 2;
        t.k = o.pauli;
        t.ins[0] = o.row;
        t.ins[1] = d.row_count++;
        prow.push_back(o.row);
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
    if (reg) {
      d.seg_begin = int(segs.size());
      d.seg_count = 0;
      const int rc = build_reg_segments(cfg, ho, d, segs, rops);
      if (rc) return rc;
    }
    hp.push_back(d);
  }
  const int nrows = int(row_slot.size());
  const uint64_t tiles = dim(n - L);
  // register-resident passes: tile + gradient slots in LDS
  const size_t reg_lds = (size_t(1) << L) * sizeof(cx<R>) + size_t(kAdjMaxRows) * (256 / 64) * sizeof(double);
  constexpr int RBs = sizeof(R) == 4 ? 4 : 3;
  const void* reg_fn = kmax <= 2   ? reinterpret_cast<const void*>(&k_adj_reg<R, RBs, 2, 8>)
                       : kmax <= 3 ? reinterpret_cast<const void*>(&k_adj_reg<R, RBs, 3, 8>)
                                   : reinterpret_cast<const void*>(&k_adj_reg<R, RBs, 5, 8>);
  // persistent grid: for the register sweep, eight rounds of the workgroups
  // the device holds at once (the variant's occupancy times the compute
  // units), so no round runs part-full and the last one is short (measured:
  // 24 qubits complex64 27.7 ms with a fixed 1024, 25.1 ms with 4 x 768, 24.7
  // ms with 8 x 768; 32 qubits 8.10, 7.14 and 6.98 s); QSV_ADJOINT_GRID
  // overrides it (tuning, and tests that give every workgroup a ragged range
  // of several tiles at small sizes)
  uint64_t gmax = kAdjTileGrid;
  if (reg) {
    int per_cu = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reg_fn, 256, reg_lds) != hipSuccess || per_cu < 1)
      per_cu = 1;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, psi->device) != hipSuccess || cus < 1)
      cus = 256;
    gmax = uint64_t(per_cu) * uint64_t(cus) * 8;
  }
  if (const char* e = std::getenv("QSV_ADJOINT_GRID")) gmax = uint64_t(std::max(1, std::atoi(e)));
  const int G = int(std::min<uint64_t>(tiles, gmax));
  // one device allocation: passes | ops | pool | segs | rops | prow | partial[nrows x G] | rows[nrows]
  auto al = [](size_t x) { return (x + 255) / 256 * 256; };
  const size_t o_ops = al(hp.size() * sizeof(TilePassDev));
  const size_t o_pool = o_ops + al(std::max<size_t>(1, ho.size()) * sizeof(TileOpDev));
  const size_t o_segs = o_pool + al(std::max<size_t>(1, pool.size()) * sizeof(cx<R>));
  const size_t o_rops = o_segs + al(std::max<size_t>(1, segs.size()) * sizeof(RegSegDev));
  const size_t o_prow = o_rops + al(std::max<size_t>(1, rops.size()) * sizeof(RegOpDev));
  const size_t o_part = o_prow + al(std::max<size_t>(1, prow.size()) * sizeof(int));
  const size_t o_rows = o_part + al(std::max<size_t>(1, size_t(nrows) * G) * sizeof(double));
  const size_t total = o_rows + al(std::max(1, nrows) * sizeof(double));
  // the tables live in psi's work buffer (kept for the next gradient; the
  // sweep synchronises before returning)
  void* wb = nullptr;
  if (int e = state_work(psi, total, &wb)) return e;
  char* d = static_cast<char*>(wb);
  hipStream_t st = psi->stream;
  int rc = QSV_OK;
  auto fin = [&](int r) {
    (void)hipStreamSynchronize(st);
    return r;
  };
  if (hipMemcpyAsync(d, hp.data(), hp.size() * sizeof(TilePassDev), hipMemcpyHostToDevice, st) != hipSuccess ||
      (!ho.empty() && hipMemcpyAsync(d + o_ops, ho.data(), ho.size() * sizeof(TileOpDev),
                                     hipMemcpyHostToDevice, st) != hipSuccess) ||
      (!pool.empty() && hipMemcpyAsync(d + o_pool, pool.data(), pool.size() * sizeof(cx<R>),
                                       hipMemcpyHostToDevice, st) != hipSuccess) ||
      (!segs.empty() && hipMemcpyAsync(d + o_segs, segs.data(), segs.size() * sizeof(RegSegDev),
                                       hipMemcpyHostToDevice, st) != hipSuccess) ||
      (!rops.empty() && hipMemcpyAsync(d + o_rops, rops.data(), rops.size() * sizeof(RegOpDev),
                                       hipMemcpyHostToDevice, st) != hipSuccess) ||
      (!prow.empty() && hipMemcpyAsync(d + o_prow, prow.data(), prow.size() * sizeof(int),
                                       hipMemcpyHostToDevice, st) != hipSuccess))
    return fin(fail(QSV_EHIP, "tiled sweep table upload failed"));
  double* part = reinterpret_cast<double*>(d + o_part);
  hipLaunchKernelGGL(k_zero_doubles, dim3(256), dim3(256), 0, st, part, uint64_t(nrows) * G);
  {
    if (reg) {
      const size_t lds = reg_lds;
      for (size_t pi = 0; pi < hp.size(); ++pi) {
        ProfScope ps("adjoint", 4.0 * sizeof(cx<R>) * double(dim(n)), st);
#define QSV_ADJR_LAUNCH(KM)                                                                      \
    hipLaunchKernelGGL((k_adj_reg<R, sizeof(R) == 4 ? 4 : 3, KM, 8>), dim3(G), dim3(256), lds, st, \
                       static_cast<R*>(psi->ptr), static_cast<R*>(lam->ptr),                      \
                       reinterpret_cast<const TilePassDev*>(d), int(pi),                          \
                       reinterpret_cast<const RegSegDev*>(d + o_segs),                            \
                       reinterpret_cast<const RegOpDev*>(d + o_rops),                             \
                       reinterpret_cast<const TileOpDev*>(d + o_ops),                             \
                       reinterpret_cast<const cx<R>*>(d + o_pool),                                \
                       reinterpret_cast<const int*>(d + o_prow), part, tiles)
        if (kmax <= 2) QSV_ADJR_LAUNCH(2);
        else if (kmax <= 3) QSV_ADJR_LAUNCH(3);
        else QSV_ADJR_LAUNCH(5);
#undef QSV_ADJR_LAUNCH
        if (hipGetLastError() != hipSuccess) return fin(fail(QSV_EHIP, "register sweep launch failed"));
      }
    }
  }
  if (!reg) {
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
