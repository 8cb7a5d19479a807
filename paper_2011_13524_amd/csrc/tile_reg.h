// Register-resident tile pass (device code, included by plan.hip).
//
// The 2^L amplitudes of a tile are spread over 2^TB threads, 2^RB per thread
// in VGPRs (RB = L - TB). A segment's layout says which local bits index a
// thread's registers (reg[0..RB-1]) and which index the thread (thr[0..TB-1]).
// Ops of a segment act on register bits: a one- or two-qubit dense block is a
// fully unrolled loop over register pairs / quads with the matrix in scalar
// registers; diagonal blocks and controls may sit on register bits, thread
// bits or non-local qubits. Between segments the tile is re-mapped through LDS
// (write in the old layout, barrier, read in the new one). LDS addresses are
// XOR-swizzled so that lanes whose local indices differ only in high bits do
// not collide on a bank. The first and last segments keep local bit 0 in
// registers (complex64), so HBM is read and written with 16-byte vectors and
// the low local bits index consecutive lanes (contiguous runs).
#pragma once

#include "dev_common.h"
#include "plan.h"

namespace qsv {

// LDS index swizzle: XOR the low SB bits with two higher SB-bit fields.
template <int SB>
struct Swz {
  __device__ __forceinline__ uint32_t operator()(uint32_t j) const {
    constexpr uint32_t m = (1u << SB) - 1;
    return j ^ ((j >> SB) & m) ^ ((j >> (2 * SB)) & m);
  }
};

struct NoSwz {
  __device__ __forceinline__ uint32_t operator()(uint32_t j) const { return j; }
};

__device__ __forceinline__ uint32_t insert_zeros32(uint32_t i, const int* pos, int m) {
  for (int j = 0; j < m; ++j) {
    const uint32_t lo = i & ((1u << pos[j]) - 1);
    i = ((i >> pos[j]) << (pos[j] + 1)) | lo;
  }
  return i;
}

// Dense block on local targets, whole tile in LDS (addresses through sw).
template <typename R, int K, typename SW>
__device__ __forceinline__ void lds_dense(cx<R>* __restrict__ t, const TileOpDev& op,
                                          const cx<R>* __restrict__ mat, int L, SW sw) {
  constexpr int D = 1 << K;
  const int cnt = 1 << (L - op.m);
  for (int i = threadIdx.x; i < cnt; i += blockDim.x) {
    const uint32_t j0 = insert_zeros32(i, op.ins, op.m) | op.lcv;
    cx<R> v[D];
#pragma unroll
    for (int c = 0; c < D; ++c) v[c] = t[sw(j0 + op.off[c])];
#pragma unroll
    for (int r = 0; r < D; ++r) {
      cx<R> acc = {R(0), R(0)};
#pragma unroll
      for (int c = 0; c < D; ++c) acc = cfma(mat[r * D + c], v[c], acc);
      t[sw(j0 + op.off[r])] = acc;
    }
  }
}

template <typename R, typename SW>
__device__ __forceinline__ void lds_diag(cx<R>* __restrict__ t, const TileOpDev& op,
                                         const cx<R>* __restrict__ d, int L, uint64_t base, SW sw) {
  int gidx = 0;
  for (int b = 0; b < op.k; ++b)
    if (op.gq[b] >= 0) gidx |= int((base >> op.gq[b]) & 1) << b;
  const int TS = 1 << L;
  for (int j = threadIdx.x; j < TS; j += blockDim.x) {
    if ((uint32_t(j) & op.lcm) != op.lcv) continue;
    int idx = gidx;
    for (int b = 0; b < op.k; ++b)
      if (op.lt[b] >= 0) idx |= ((j >> op.lt[b]) & 1) << b;
    const uint32_t a = sw(uint32_t(j));
    t[a] = d[idx] * t[a];
  }
}

// KMAX bounds the widest dense block compiled in: a kernel instantiated for
// small blocks does not pay the register cost of 32-amplitude temporaries.
template <typename R, int KMAX, typename SW>
__device__ __forceinline__ void lds_op(cx<R>* t, const TileOpDev& op, const cx<R>* pool, int L,
                                       uint64_t base, SW sw) {
  const cx<R>* mat = pool + op.moff;
  if (op.kind == 1) {
    lds_diag<R>(t, op, mat, L, base, sw);
  } else {
    switch (op.k) {
      case 1: lds_dense<R, 1>(t, op, mat, L, sw); break;
      case 2: if constexpr (KMAX >= 2) lds_dense<R, 2>(t, op, mat, L, sw); break;
      case 3: if constexpr (KMAX >= 3) lds_dense<R, 3>(t, op, mat, L, sw); break;
      case 4: if constexpr (KMAX >= 4) lds_dense<R, 4>(t, op, mat, L, sw); break;
      default: if constexpr (KMAX >= 5) lds_dense<R, 5>(t, op, mat, L, sw); break;
    }
  }
}

// ------------------------------------------------------------------ register ops
//
// Register element indices are compile-time constants in every loop below
// (loops run over the compressed index g and insert the target bits), so the
// per-thread amplitude array stays in VGPRs.

// Register bits that do not exist for NR elements (a variant compiled for a
// larger register file): the variant copies v to o unchanged; the planner
// never selects it.
template <typename R, int NR>
__device__ __forceinline__ void reg_copy(const cx<R>* v, cx<R>* o) {
#pragma unroll
  for (int i = 0; i < NR; ++i) o[i] = v[i];
}

// Component-wise select: a conditional choice between two complex values
// written on the scalars keeps both in registers (a select of whole structs
// can become a select of their addresses, which pins the arrays in memory).
template <typename R>
__device__ __forceinline__ cx<R> csel(bool c, const cx<R>& a, const cx<R>& b) {
  return {c ? a.re : b.re, c ? a.im : b.im};
}

template <int P>
__device__ __forceinline__ constexpr int ins1(int g) {
  return ((g >> P) << (P + 1)) | (g & ((1 << P) - 1));
}

template <int A, int B>
__device__ __forceinline__ constexpr int ins2(int g) {
  constexpr int lo = A < B ? A : B, hi = A < B ? B : A;
  return ins1<hi>(ins1<lo>(g));
}

// Each variant reads v and writes EVERY element of o (updated or copied). The
// kernels alternate two register arrays from op to op (v -> o, then o -> v),
// so the values a variant produces already sit in the registers the next op
// reads: no copies at the join after the switch over variants. A variant for
// a register bit that does not exist for NR elements (compiled for a larger
// register file, never selected) copies. Controlled variants (HASC) take the
// per-element register-bit control (i & cm) == cv and the per-lane thread-bit
// control `lane`.
template <typename R, int NR, int P, bool HASC>
__device__ __forceinline__ void reg_dense1(const cx<R>* v, cx<R>* o, const cx<R>* __restrict__ m,
                                           uint32_t cm, uint32_t cv, bool lane) {
  if constexpr ((1 << P) >= NR) {
    reg_copy<R, NR>(v, o);
  } else {
    const cx<R> m00 = m[0], m01 = m[1], m10 = m[2], m11 = m[3];
#pragma unroll
    for (int g = 0; g < NR / 2; ++g) {
      const int i = ins1<P>(g), j = i | (1 << P);
      const cx<R> a = v[i], b = v[j];
      const cx<R> na = cfma(m00, a, m01 * b), nb = cfma(m10, a, m11 * b);
      if constexpr (HASC) {
        const bool on = lane && (uint32_t(i) & cm) == cv;
        o[i] = csel(on, na, a);
        o[j] = csel(on, nb, b);
      } else {
        o[i] = na;
        o[j] = nb;
      }
    }
  }
}

// Dense one-qubit op on the matrix cores (complex64, no controls). For the
// register pair (a, b) of a lane, the output (a', b') is the real 4x4 matrix
// [[Re m00, -Im m00, Re m01, -Im m01], [Im m00, Re m00, Im m01, Re m01],
//  [Re m10, -Im m10, Re m11, -Im m11], [Im m10, Re m10, Im m11, Re m11]]
// times (Re a, Im a, Re b, Im b). v_mfma_f32_4x4x1_16b_f32 forms, per block of
// four lanes, the outer product of a 4-vector held one element per lane (A)
// and each lane's own scalar (B), accumulated into four registers per lane:
// register r of lane l gains A(lane 4*(l/4) + r) * B(l). With A = column c of
// the matrix (row = lane % 4) and B = input component c of the lane's own
// pair, four accumulating instructions give each lane its own (a', b') in the
// register order (Re a', Im a', Re b', Im b'): the layout the vector ALU code
// uses, at twice the non-packed FP32 FMA rate, off the vector ALU.
template <int NR, int P>
__device__ __forceinline__ void reg_dense1_mfma(const cx<float>* v, cx<float>* o,
                                                const cx<float>* __restrict__ m) {
  if constexpr ((1 << P) >= NR) {
    reg_copy<float, NR>(v, o);
  } else {
    typedef float v4f __attribute__((ext_vector_type(4)));
    const uint32_t lane = threadIdx.x & 63u;
    const bool hi = (lane & 2u) != 0, odd = (lane & 1u) != 0;
    const cx<float> m00 = m[0], m01 = m[1], m10 = m[2], m11 = m[3];
    const float c0r = hi ? m10.re : m00.re, c0i = hi ? m10.im : m00.im;
    const float c1r = hi ? m11.re : m01.re, c1i = hi ? m11.im : m01.im;
    const float a0 = odd ? c0i : c0r, a1 = odd ? c0r : -c0i;
    const float a2 = odd ? c1i : c1r, a3 = odd ? c1r : -c1i;
#pragma unroll
    for (int g = 0; g < NR / 2; ++g) {
      const int i = ins1<P>(g), j = i | (1 << P);
      v4f d = {0.f, 0.f, 0.f, 0.f};
      d = __builtin_amdgcn_mfma_f32_4x4x1f32(a0, v[i].re, d, 0, 0, 0);
      d = __builtin_amdgcn_mfma_f32_4x4x1f32(a1, v[i].im, d, 0, 0, 0);
      d = __builtin_amdgcn_mfma_f32_4x4x1f32(a2, v[j].re, d, 0, 0, 0);
      d = __builtin_amdgcn_mfma_f32_4x4x1f32(a3, v[j].im, d, 0, 0, 0);
      o[i] = {d[0], d[1]};
      o[j] = {d[2], d[3]};
    }
  }
}

// A layer of uncontrolled dense one-qubit ops on distinct register bits (the
// bits of MASK, applied in bit order: ops on distinct qubits commute), in one
// dispatch: the per-op scalar work of the op loop (descriptor loads, control
// checks, the branch tree over the variants) is shared by the whole layer.
// The first step reads v and writes every element of o; later steps update o
// in place (no temporary copy of the tile: the register budget keeps four
// workgroups per compute unit). The matrix of bit p is at pool + lm[p].
template <typename R, int NR, int P>
__device__ __forceinline__ void lay_dense1(const cx<R>* src, cx<R>* dst, const cx<R>* __restrict__ m) {
  const cx<R> m00 = m[0], m01 = m[1], m10 = m[2], m11 = m[3];
#pragma unroll
  for (int g = 0; g < NR / 2; ++g) {
    const int i = ins1<P>(g), j = i | (1 << P);
    const cx<R> a = src[i], b = src[j];
    dst[i] = cfma(m00, a, m01 * b);
    dst[j] = cfma(m10, a, m11 * b);
  }
}

// The same on the matrix cores (complex64; see reg_dense1_mfma), four pairs'
// accumulation chains interleaved at a time.
template <int NR, int P>
__device__ __forceinline__ void lay_dense1_mfma(const cx<float>* src, cx<float>* dst,
                                                const cx<float>* __restrict__ m) {
  typedef float v4f __attribute__((ext_vector_type(4)));
  const uint32_t lane = threadIdx.x & 63u;
  const bool hi = (lane & 2u) != 0, odd = (lane & 1u) != 0;
  const cx<float> m00 = m[0], m01 = m[1], m10 = m[2], m11 = m[3];
  const float c0r = hi ? m10.re : m00.re, c0i = hi ? m10.im : m00.im;
  const float c1r = hi ? m11.re : m01.re, c1i = hi ? m11.im : m01.im;
  const float a0 = odd ? c0i : c0r, a1 = odd ? c0r : -c0i;
  const float a2 = odd ? c1i : c1r, a3 = odd ? c1r : -c1i;
  constexpr int C = NR / 2 < 4 ? NR / 2 : 4;
#pragma unroll
  for (int g0 = 0; g0 < NR / 2; g0 += C) {
    v4f d[C];
#pragma unroll
    for (int c = 0; c < C; ++c)
      d[c] = __builtin_amdgcn_mfma_f32_4x4x1f32(a0, src[ins1<P>(g0 + c)].re, v4f{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
#pragma unroll
    for (int c = 0; c < C; ++c) d[c] = __builtin_amdgcn_mfma_f32_4x4x1f32(a1, src[ins1<P>(g0 + c)].im, d[c], 0, 0, 0);
#pragma unroll
    for (int c = 0; c < C; ++c)
      d[c] = __builtin_amdgcn_mfma_f32_4x4x1f32(a2, src[ins1<P>(g0 + c) | (1 << P)].re, d[c], 0, 0, 0);
#pragma unroll
    for (int c = 0; c < C; ++c)
      d[c] = __builtin_amdgcn_mfma_f32_4x4x1f32(a3, src[ins1<P>(g0 + c) | (1 << P)].im, d[c], 0, 0, 0);
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int i = ins1<P>(g0 + c), j = i | (1 << P);
      dst[i] = {d[c][0], d[c][1]};
      dst[j] = {d[c][2], d[c][3]};
    }
  }
}

template <typename R, int NR, int P, bool MF>
__device__ __forceinline__ void lay_step(const cx<R>* src, cx<R>* dst, const cx<R>* __restrict__ m) {
  if constexpr ((1 << P) >= NR) {  // no such register bit (never selected)
    if (src != dst) reg_copy<R, NR>(src, dst);
  } else if constexpr (MF && sizeof(R) == 4) {
    lay_dense1_mfma<NR, P>(src, dst, m);
  } else {
    lay_dense1<R, NR, P>(src, dst, m);
  }
}

template <typename R, int NR, int MASK, bool MF>
__device__ __forceinline__ void reg_layer(const cx<R>* v, cx<R>* o, const cx<R>* __restrict__ pool,
                                          const int* lm) {
  constexpr int F = (MASK & 1) ? 0 : (MASK & 2) ? 1 : (MASK & 4) ? 2 : 3;
  lay_step<R, NR, F, MF>(v, o, pool + lm[F]);
  if constexpr (F < 1 && (MASK & 2)) lay_step<R, NR, 1, MF>(o, o, pool + lm[1]);
  if constexpr (F < 2 && (MASK & 4)) lay_step<R, NR, 2, MF>(o, o, pool + lm[2]);
  if constexpr (F < 3 && (MASK & 8)) lay_step<R, NR, 3, MF>(o, o, pool + lm[3]);
}

// Pauli-X exchange (X, CNOT on register bits): moves only.
template <typename R, int NR, int P, bool HASC>
__device__ __forceinline__ void reg_swap1(const cx<R>* v, cx<R>* o, uint32_t cm, uint32_t cv, bool lane) {
  if constexpr ((1 << P) >= NR) {
    reg_copy<R, NR>(v, o);
  } else {
#pragma unroll
    for (int g = 0; g < NR / 2; ++g) {
      const int i = ins1<P>(g), j = i | (1 << P);
      const bool on = !HASC || (lane && (uint32_t(i) & cm) == cv);
      o[i] = csel(on, v[j], v[i]);
      o[j] = csel(on, v[i], v[j]);
    }
  }
}

// Matrix index bit 0 <-> register bit A, bit 1 <-> register bit B.
template <typename R, int NR, int A, int B, bool HASC>
__device__ __forceinline__ void reg_dense2(const cx<R>* v, cx<R>* o, const cx<R>* __restrict__ m,
                                           uint32_t cm, uint32_t cv, bool lane) {
  if constexpr ((1 << A) >= NR || (1 << B) >= NR) {
    reg_copy<R, NR>(v, o);
  } else {
    const cx<R> k0 = m[0], k1 = m[1], k2 = m[2], k3 = m[3], k4 = m[4], k5 = m[5], k6 = m[6],
                k7 = m[7], k8 = m[8], k9 = m[9], k10 = m[10], k11 = m[11], k12 = m[12],
                k13 = m[13], k14 = m[14], k15 = m[15];
#pragma unroll
    for (int g = 0; g < NR / 4; ++g) {
      const int i0 = ins2<A, B>(g);
      const int i1 = i0 | (1 << A), i2 = i0 | (1 << B), i3 = i0 | (1 << A) | (1 << B);
      const bool on = !HASC || (lane && (uint32_t(i0) & cm) == cv);
      const cx<R> x0 = v[i0], x1 = v[i1], x2 = v[i2], x3 = v[i3];
      const cx<R> y0 = cfma(k3, x3, cfma(k2, x2, cfma(k1, x1, k0 * x0)));
      const cx<R> y1 = cfma(k7, x3, cfma(k6, x2, cfma(k5, x1, k4 * x0)));
      const cx<R> y2 = cfma(k11, x3, cfma(k10, x2, cfma(k9, x1, k8 * x0)));
      const cx<R> y3 = cfma(k15, x3, cfma(k14, x2, cfma(k13, x1, k12 * x0)));
      o[i0] = csel(on, y0, x0);
      o[i1] = csel(on, y1, x1);
      o[i2] = csel(on, y2, x2);
      o[i3] = csel(on, y3, x3);
    }
  }
}

// Diagonal factor on up to two register bits (A < B; -1: absent): the factor
// of element i is g[(bit A of i) | (bit B of i) << 1], picked at compile time.
template <typename R, int NR, int A, int B, bool HASC>
__device__ __forceinline__ void reg_diag(const cx<R>* v, cx<R>* o, const cx<R>* g, uint32_t cm, uint32_t cv,
                                         bool lane) {
  if constexpr ((A >= 0 && (1 << A) >= NR) || (B >= 0 && (1 << B) >= NR)) {
    reg_copy<R, NR>(v, o);
  } else {
#pragma unroll
    for (int i = 0; i < NR; ++i) {
      const int idx = (A >= 0 ? (i >> A) & 1 : 0) | (B >= 0 ? ((i >> B) & 1) << 1 : 0);
      const bool on = !HASC || (lane && (uint32_t(i) & cm) == cv);
      o[i] = csel(on, g[idx] * v[i], v[i]);
    }
  }
}

// One flat switch over (op type, control presence, register bits). Keys:
// reg_key().
#define QSV_C1(SW, HC, P)                                                        \
  case ((SW) * 2 + (HC)) * 8 + (P):                                              \
    if constexpr (SW) reg_swap1<R, NR, P, HC>(v, o, cm, cv, lane);               \
    else reg_dense1<R, NR, P, HC>(v, o, m, cm, cv, lane);                        \
    break;
#define QSV_C1P(SW, HC) QSV_C1(SW, HC, 0) QSV_C1(SW, HC, 1) QSV_C1(SW, HC, 2) QSV_C1(SW, HC, 3)
#define QSV_C2(HC, A, B)                                                         \
  case 32 + (HC) * 64 + (A) * 8 + (B):                                           \
    reg_dense2<R, NR, A, B, HC>(v, o, m, cm, cv, lane);                          \
    break;
#define QSV_C2P4(HC)                                                             \
  QSV_C2(HC, 0, 1) QSV_C2(HC, 0, 2) QSV_C2(HC, 0, 3) QSV_C2(HC, 1, 0) QSV_C2(HC, 1, 2) \
  QSV_C2(HC, 1, 3) QSV_C2(HC, 2, 0) QSV_C2(HC, 2, 1) QSV_C2(HC, 2, 3) QSV_C2(HC, 3, 0) \
  QSV_C2(HC, 3, 1) QSV_C2(HC, 3, 2)
#define QSV_C2P5(HC)                                                             \
  QSV_C2(HC, 0, 4) QSV_C2(HC, 1, 4) QSV_C2(HC, 2, 4) QSV_C2(HC, 3, 4) QSV_C2(HC, 4, 0) \
  QSV_C2(HC, 4, 1) QSV_C2(HC, 4, 2) QSV_C2(HC, 4, 3)
#define QSV_CD(HC, A, B)                                                         \
  case 160 + (HC) * 64 + ((A) + 1) * 8 + ((B) + 1):                              \
    reg_diag<R, NR, A, B, HC>(v, o, g, cm, cv, lane);                            \
    break;
#define QSV_CDP4(HC)                                                             \
  QSV_CD(HC, -1, -1) QSV_CD(HC, 0, -1) QSV_CD(HC, 1, -1) QSV_CD(HC, 2, -1)         \
  QSV_CD(HC, 3, -1) QSV_CD(HC, 0, 1) QSV_CD(HC, 0, 2) QSV_CD(HC, 0, 3)             \
  QSV_CD(HC, 1, 2) QSV_CD(HC, 1, 3) QSV_CD(HC, 2, 3)
#define QSV_CDP5(HC)                                                             \
  QSV_CD(HC, 4, -1) QSV_CD(HC, 0, 4) QSV_CD(HC, 1, 4) QSV_CD(HC, 2, 4) QSV_CD(HC, 3, 4)

#define QSV_CM(P)                                                                \
  case 288 + (P):                                                                \
    if constexpr (sizeof(R) == 4) reg_dense1_mfma<NR, P>(v, o, m);               \
    else __builtin_unreachable();                                                \
    break;

#define QSV_CL(MASK)                                                             \
  case 320 + (MASK):                                                             \
    reg_layer<R, NR, MASK, false>(v, o, pool, lm);                               \
    break;                                                                       \
  case 336 + (MASK):                                                             \
    if constexpr (sizeof(R) == 4) reg_layer<R, NR, MASK, true>(v, o, pool, lm);  \
    else __builtin_unreachable();                                                \
    break;
#define QSV_CLP                                                                  \
  QSV_CL(3) QSV_CL(5) QSV_CL(6) QSV_CL(7) QSV_CL(9) QSV_CL(10) QSV_CL(11)        \
  QSV_CL(12) QSV_CL(13) QSV_CL(14) QSV_CL(15)

// kind 0 dense one-qubit, 1 dense two-qubit, 2 diagonal, 4 Pauli-X exchange,
// 7 dense one-qubit on the matrix cores (complex64, no controls), 10 layer of
// dense one-qubit ops on the register bits of mask a (at least two; b = 1:
// on the matrix cores); a, b: register bits (diagonal: -1 when absent, a < b)
__host__ __device__ __forceinline__ int reg_key(int kind, int a, int b, bool hc) {
  const int h = hc ? 1 : 0;
  if (kind == 7) return 288 + a;
  if (kind == 10) return (b ? 336 : 320) + a;
  if (kind == 1) return 32 + h * 64 + a * 8 + b;
  if (kind == 2) return 160 + h * 64 + (a + 1) * 8 + (b + 1);
  return ((kind == 4) * 2 + h) * 8 + a;
}

// LAY: the layer variants are compiled in (the forward tile kernel; the
// reverse sweep, whose two register-resident states leave no room for them,
// leaves them out and its planner emits none).
template <typename R, int NR, bool LAY = true>
__device__ __forceinline__ void reg_apply(const cx<R>* v, cx<R>* o, int key, const cx<R>* m, const cx<R>* g,
                                          uint32_t cm, uint32_t cv, bool lane, const cx<R>* __restrict__ pool,
                                          const int* lm) {
  if constexpr (LAY) {
    if (key >= 320) {
      switch (key) {
        QSV_CLP
        default:
          __builtin_unreachable();
      }
      return;
    }
  }
  switch (key) {
    QSV_C1P(0, 0) QSV_C1P(0, 1) QSV_C1P(1, 0) QSV_C1P(1, 1)
    QSV_C2P4(0) QSV_C2P4(1)
    QSV_CDP4(0) QSV_CDP4(1)
    QSV_CM(0) QSV_CM(1) QSV_CM(2) QSV_CM(3)
    default:
      if constexpr (NR > 16) {
        switch (key) {
          QSV_CM(4)
          QSV_C1(0, 0, 4) QSV_C1(0, 1, 4) QSV_C1(1, 0, 4) QSV_C1(1, 1, 4)
          QSV_C2P5(0) QSV_C2P5(1)
          QSV_CDP5(0) QSV_CDP5(1)
          default:
            __builtin_unreachable();  // the planner emits only the keys above
        }
      } else {
        __builtin_unreachable();
      }
      break;
  }
}
#undef QSV_C1
#undef QSV_C1P
#undef QSV_C2
#undef QSV_C2P4
#undef QSV_C2P5
#undef QSV_CD
#undef QSV_CDP4
#undef QSV_CDP5
#undef QSV_CM
#undef QSV_CL
#undef QSV_CLP

// Factor table of a diagonal op (k <= 2) for this thread: index bits from
// thread and non-local targets are fixed; register targets become the bits
// a < b of the table index.
template <typename R>
__device__ __forceinline__ void diag_table(const RegOpDev& op, const cx<R>* __restrict__ d, uint32_t tau,
                                           uint64_t base, cx<R>* g, int& a, int& b) {
  int fixed = 0, ja = 0, jb = 0;
  a = -1;
  b = -1;
#pragma unroll
  for (int j = 0; j < 2; ++j) {  // (k <= 2)
    if (j >= op.k) break;
    if (op.dsrc[j] == 1) fixed |= int((tau >> op.dbit[j]) & 1) << j;
    else if (op.dsrc[j] == 2) fixed |= int((base >> op.dbit[j]) & 1) << j;
    else if (a < 0) {
      a = op.dbit[j];
      ja = j;
    } else {
      b = op.dbit[j];
      jb = j;
    }
  }
  if (b >= 0 && b < a) {
    const int t = a, tj = ja;
    a = b;
    ja = jb;
    b = t;
    jb = tj;
  }
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    int idx = fixed;
    if (a >= 0 && (e & 1)) idx |= 1 << ja;
    if (b >= 0 && (e & 2)) idx |= 1 << jb;
    g[e] = d[idx];
  }
}

// Orders this wavefront's LDS accesses (a compiler barrier: the hardware
// performs one wavefront's LDS operations in issue order).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// LDS addresses of a layout. The swizzle is linear over XOR and a local index
// is the XOR of its register part and its thread part, so the byte offset of
// element i is the per-thread part XOR a part that depends only on i and the
// layout (uniform across the workgroup: a table the planner fills, read
// through the scalar cache). Kernels using it declare no static LDS and put
// the tile first in their dynamic LDS, so it starts at LDS address 0 and the
// base folds into the per-thread part: one vector XOR per element remains.
template <typename R, int RB, int TB>
struct LdsMap {
  uint32_t thr;        // per-thread part, in bytes
  const uint32_t* reg;  // per-element parts, in bytes (uniform)
  __device__ __forceinline__ LdsMap(const uint32_t* regt, const uint32_t* tcol, uint32_t tcst, uint32_t tau)
      : reg(regt) {
    uint32_t j = tcst;
#pragma unroll
    for (int b = 0; b < TB; ++b) j ^= tcol[b] & (0u - ((tau >> b) & 1));  // (branch-free)
    thr = j;
  }
  typedef R R2 __attribute__((ext_vector_type(2)));
  typedef __attribute__((address_space(3))) R2 lds_r2;
  __device__ __forceinline__ lds_r2* at(char* lds, int i) const {
    const uint32_t base = uint32_t(reinterpret_cast<uintptr_t>(lds));
    return reinterpret_cast<lds_r2*>(uintptr_t((base + thr) ^ reg[i]));
  }
  __device__ __forceinline__ void put(char* lds, int i, const cx<R>& x) const {
    R2 w;
    w.x = x.re;
    w.y = x.im;
    *at(lds, i) = w;
  }
  __device__ __forceinline__ cx<R> get(char* lds, int i) const {
    const R2 w = *at(lds, i);
    return {w.x, w.y};
  }
};

// One register-segment op: reads the register array v and writes every
// element of o. Ops with non-local controls that do not match this tile copy;
// ops on LDS (kind 3) go through the tile in LDS; controls on thread bits are
// per lane.
template <typename R, int RB, int KMAX, int TB>
__device__ __forceinline__ void reg_step(const RegOpDev& opr, const cx<R>* v, cx<R>* o, const RegSegDev& S,
                                         uint32_t tau, uint64_t base, Swz<sizeof(R) == 4 ? 5 : 4> sw,
                                         char* smem, const TileOpDev* __restrict__ lops,
                                         const cx<R>* __restrict__ pool, int L) {
  constexpr int NR = 1 << RB;
  const RegOpDev op = opr;  // (one burst of scalar loads)
  if ((base & op.gcm) != op.gcv) {  // non-local controls: uniform per tile
    reg_copy<R, NR>(v, o);
    return;
  }
  const cx<R>* m = pool + op.moff;
  if (op.kind == 3) {
    const LdsMap<R, RB, TB> ms(S.get_reg, S.get_tcol, 0u, tau);
    __syncthreads();  // (a preceding cross-wave re-map's reads are done)
#pragma unroll
    for (int i = 0; i < NR; ++i) ms.put(smem, i, v[i]);
    __syncthreads();
    lds_op<R, KMAX>(reinterpret_cast<cx<R>*>(smem), lops[op.lop], pool, L, base, sw);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NR; ++i) o[i] = ms.get(smem, i);
    __syncthreads();
    return;
  }
  cx<R> g[4];
  int a = op.p1, bb = op.p2;
  if (op.kind == 2) diag_table<R>(op, m, tau, base, g, a, bb);
  const bool lane = (tau & op.ti_cm) == op.ti_cv;
  reg_apply<R, NR>(v, o, op.key, m, g, op.ri_cm, op.ri_cv, lane, pool, op.lm);
}

// Register budget (the launch bound's second argument: wavefronts per SIMD):
// complex64 tiles of 16 amplitudes per thread keep four (128 VGPRs; with 32
// KiB of LDS per 256 threads, four workgroups of 256 or two of 512 per compute
// unit); wider tiles and complex128 take what they need.
template <typename R, int RB>
constexpr int tile_waves_per_simd() {
  return (sizeof(R) == 4 && RB == 4) ? 4 : 1;
}

template <typename R, int RB, int KMAX, int TB>
__global__ void __launch_bounds__(1 << TB, (tile_waves_per_simd<R, RB>()))
    k_tile_reg(R* __restrict__ psi, const TilePassDev* __restrict__ passes, int pass_idx,
               const RegSegDev* __restrict__ segs, const RegOpDev* __restrict__ rops,
               const TileOpDev* __restrict__ lops, const cx<R>* __restrict__ pool) {
  constexpr int NR = 1 << RB;
  constexpr int SB = sizeof(R) == 4 ? 5 : 4;
  const Swz<SB> sw;
  extern __shared__ __align__(16) char smem[];
  const TilePassDev& P = passes[pass_idx];
  const int L = P.L;
  const uint64_t g = blockIdx.x;
  uint64_t base = 0;
  for (int r = 0; r < P.nrun; ++r) base |= ((g >> P.rsrc[r]) & ((uint64_t(1) << P.rlen[r]) - 1)) << P.rdst[r];
  const uint32_t tau = threadIdx.x;

  cx<R> v[NR], w[NR];
  // HBM -> registers in the first segment's layout
  const RegSegDev* S = &segs[P.seg_begin];
  uint64_t gthr = base;
#pragma unroll
  for (int k = 0; k < TB; ++k) gthr |= S->gcol_t[k] & (uint64_t(0) - ((tau >> k) & 1));  // (branch-free)
  uint64_t greg[RB];
#pragma unroll
  for (int k = 0; k < RB; ++k) greg[k] = S->gcol_r[k];
  const bool vec = sizeof(R) == 4 && S->reg[0] == 0;
  if (vec) {
#pragma unroll
    for (int i = 0; i < NR; i += 2) {
      uint64_t x = gthr;
#pragma unroll
      for (int k = 1; k < RB; ++k)
        if ((i >> k) & 1) x |= greg[k];
      AmpIO<R, 2>::load(psi, x, &v[i]);
    }
  } else {
#pragma unroll
    for (int i = 0; i < NR; ++i) {
      uint64_t x = gthr;
#pragma unroll
      for (int k = 0; k < RB; ++k)
        if ((i >> k) & 1) x |= greg[k];
      AmpIO<R, 1>::load(psi, x, &v[i]);
    }
  }

  for (int sgi = 0; sgi < P.seg_count; ++sgi) {
    const RegSegDev* Sn = &segs[P.seg_begin + sgi];
    if (sgi > 0) {
      // re-map through LDS, applying the ops folded into it on the way; when
      // both layouts share the wave bits (and no folded op targets one), every
      // wavefront reads back only what it wrote, and LDS operations of one
      // wavefront complete in order: no workgroup barrier is needed
      const bool xw = (Sn->xwave & 1) != 0;
      if (Sn->xwave & 2) __syncthreads();
      {
        const LdsMap<R, RB, TB> mo(Sn->put_reg, Sn->put_tcol, Sn->put_tcst, tau);
#pragma unroll
        for (int i = 0; i < NR; ++i) mo.put(smem, i, v[i]);
      }
      if (xw) __syncthreads();
      else wave_sync();
      {
        const LdsMap<R, RB, TB> mn(Sn->get_reg, Sn->get_tcol, 0u, tau);
#pragma unroll
        for (int i = 0; i < NR; ++i) v[i] = mn.get(smem, i);
      }
      // a cross-wave re-map's closing barrier waits for the next LDS write
      // (marked on the next re-map; ops through LDS always wait first), so
      // the segment's register ops overlap the wavefronts' skew
      if (!xw) wave_sync();
    }
    S = Sn;
    // ops alternate between the register arrays v and w (one op reads one and
    // writes all of the other)
    const int oc = S->op_count, ob = S->op_begin;
    for (int o = 0; o < oc; o += 2) {
      reg_step<R, RB, KMAX, TB>(rops[ob + o], v, w, *S, tau, base, sw, smem, lops, pool, L);
      if (o + 1 < oc) reg_step<R, RB, KMAX, TB>(rops[ob + o + 1], w, v, *S, tau, base, sw, smem, lops, pool, L);
      else reg_copy<R, 1 << RB>(w, v);
    }
  }

  // registers -> HBM in the last segment's layout
  gthr = base;
#pragma unroll
  for (int k = 0; k < TB; ++k) gthr |= S->gcol_t[k] & (uint64_t(0) - ((tau >> k) & 1));
#pragma unroll
  for (int k = 0; k < RB; ++k) greg[k] = S->gcol_r[k];
  if (sizeof(R) == 4 && S->reg[0] == 0) {
#pragma unroll
    for (int i = 0; i < NR; i += 2) {
      uint64_t x = gthr;
#pragma unroll
      for (int k = 1; k < RB; ++k)
        if ((i >> k) & 1) x |= greg[k];
      AmpIO<R, 2>::store(psi, x, &v[i]);
    }
  } else {
#pragma unroll
    for (int i = 0; i < NR; ++i) {
      uint64_t x = gthr;
#pragma unroll
      for (int k = 0; k < RB; ++k)
        if ((i >> k) & 1) x |= greg[k];
      AmpIO<R, 1>::store(psi, x, &v[i]);
    }
  }
}

}  // namespace qsv
