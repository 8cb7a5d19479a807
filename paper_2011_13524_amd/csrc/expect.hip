// Tiled evaluation of <psi|O|psi> for a Pauli-string observable (section 4.5).
//
// A term with flip mask F pairs amplitude x with x ^ F, so it can be evaluated
// from any tile of the state whose local qubits include every qubit of F: both
// members of each pair are then in the same tile. The host groups the
// observable's flip masks into passes: a pass fixes L local qubits (always the
// low b ones, for contiguous HBM runs) chosen to hold as many flip masks as it
// can (pick_pass_local below); a mask with more flip qubits than a tile holds
// is evaluated on its own, its pairs read straight from the state. Each pass reads the
// state once into LDS, tile by tile, and evaluates every group of the pass on
// it. Workgroups are persistent and prefetch their next tile while computing
// on the current one; each sums its tiles in a fixed order into one FP64
// partial (passes run in order on one stream, so each partial has a single
// writer in a fixed order), and one final fixed-order reduction gives the
// value: bitwise reproducible. Compared with one pass per flip mask, HBM
// traffic drops by the number of masks per pass. Z/Y signs on non-local qubits
// are constants per tile. The same passes give lambda = O psi (adjoint).
#include <algorithm>
#include <cstdlib>
#include <mutex>

#include "dev_common.h"
#include "observable.h"
#include "prof.h"
#include "qsv_internal.h"

namespace qsv {

constexpr int kExpThreads = 512;
// largest tiles (expectation and lambda passes): 2^13 amplitudes, 64 KiB of
// complex64
constexpr int kExpTileMax = 8192;
// expectation workgroups: 512 threads over a 2^13-amplitude tile, so a
// single-term group gives each thread 8 pairs per tile (the group's scalar
// setup repeats per wave) and two workgroups (64 KiB of LDS each) keep 16
// waves on a compute unit; measured at 30 qubits complex64 against 256
// threads over 2^12 tiles (21 passes: 52.7 ms) and 256 over 2^13 (18
// passes but 8 waves per compute unit: 62.4 ms): 18 passes, 50.9 ms
constexpr int kExpThreadsE = 512;
constexpr int kExpMaxHigh = 16;
constexpr int kExpMaxGlobal = 40;

struct ExpPassDev {
  int L, b, nh, ng;
  int grp_begin, grp_count;
  int hq[kExpMaxHigh];
  int gpos[kExpMaxGlobal];
};

constexpr int kExpSteps = kExpTileMax / kExpThreadsE;  // per-thread steps over the largest tile

// A flip-mask group of a pass, with its first term folded in and, for
// expectation workgroups of kExpThreadsE threads, the workgroup-uniform parts
// of each step's indices and signs (the same for every tile of the pass).
struct ExpGroupDev {
  double re, im;   // first term: alpha * i^nY
  uint64_t zg;     // first term: sign mask on non-local qubits (global index space)
  uint32_t lf;     // flip mask in the tile's local index space
  uint32_t zl;     // first term: sign mask on local qubits
  int hbit;        // a set bit of lf (pairs are enumerated with it clear)
  int term_begin, term_count;
  uint32_t kind;  // ExpKind: which loop evaluates the record
  // lf != 0, kExpThreadsE-thread workgroups: bits below hbit, and the flip
  // bits inside the thread part of x = ins0(pair index, hbit)
  uint32_t hmask, lft;
  // lf != 0, step k (pair index k * kExpThreadsE + thread): the step part of
  // x = ins0(pair index, hbit) and of y = x ^ lf outside the thread's bits
  uint32_t offx[kExpSteps / 2], offy[kExpSteps / 2];
  // bit 31: parity of (step part of x) & zl (complex64 plans, lf != 0: as
  // the float +-1.0); for lf == 0 the step part of x is k * kExpThreadsE
  uint32_t sgn[kExpSteps];
};

// Record kinds (set by the planner): one term with flip mask 0; several
// terms with flip mask 0; one term with a flip mask and a real (REAL) or
// imaginary (IMAG) coefficient alpha i^nY; several terms with a flip mask.
enum ExpKind : uint32_t { kExpZ1 = 0, kExpZN = 1, kExpFlipRe = 2, kExpFlipIm = 3, kExpFlipN = 4 };

struct ExpTermDev {
  double re, im;  // alpha * i^nY
  uint64_t zg;    // sign mask on non-local qubits (global index space)
  uint32_t zl;    // sign mask on local qubits (local index space)
  uint32_t pad;
};

// A term as staged in LDS for one tile: coefficient with the tile's sign on
// non-local qubits folded in, and the local sign mask.
struct ExpTermLds {
  double re, im;
  uint32_t zl;
};
constexpr int kExpLdsTerms = 128;
// Flip-mask groups of at most this many terms are split into single-term
// records: a shared multi-term record (FP64 sign sums per pair, terms staged
// in LDS) costs about six single-term ones or more; splitting masks of up to
// eight terms (not only up to four) took the 24-qubit 500-term lambda pass
// from 0.279 to 0.254 ms (complex64). Larger groups share the pair products.
constexpr int kExpSplitTerms = 8;
// persistent workgroups per observable pass: 8 per compute unit (2 resident
// at a time for the 512-thread expectation workgroups over 64 KiB tiles, 1
// for the lambda workgroups, which their registers limit); measured at 30
// qubits complex64: 2048 beats 1024 (shorter ranges even out the tail);
// QSV_EXPECT_GRID overrides
constexpr int kExpGrid = 2048;

// Persistent grid of the expectation and lambda passes: kExpGrid, or the
// QSV_EXPECT_GRID override (tuning, and tests that give every workgroup a
// ragged range of several tiles at small sizes).
uint64_t exp_grid_max() {
  if (const char* e = std::getenv("QSV_EXPECT_GRID")) return uint64_t(std::max(1, std::atoi(e)));
  return kExpGrid;
}

// A group whose flip mask has more qubits than a tile holds (with the low
// ones): its terms are wide_terms[term_begin, term_begin + term_count), with
// zg the whole sign mask.
struct ExpWide {
  uint64_t flip;
  int hbit;  // highest bit of flip
  int term_begin, term_count;
};

struct ExpPlan {
  int n = 0, L = 0, b = 0;
  std::vector<ExpPassDev> passes;
  std::vector<ExpGroupDev> groups;
  std::vector<ExpTermDev> terms;
  std::vector<ExpWide> wide;
  std::vector<ExpTermDev> wide_terms;
  void* dev = nullptr;  // passes | groups | terms | wide_terms
  size_t off_groups = 0, off_terms = 0, off_wide = 0;
  int device = -1;
};

void free_exp_plan(ExpPlan* p) {
  if (!p) return;
  if (p->dev) (void)hipFree(p->dev);
  delete p;
}

// Local index -> global index bits of a pass (bit placement: linear over OR
// for local indices with disjoint bits, so per-thread and per-iteration parts
// are placed once and combined with one OR).
__device__ __forceinline__ uint64_t exp_place(const ExpPassDev& P, uint32_t j) {
  uint64_t x = j & ((1u << P.b) - 1);
  for (int i = 0; i < P.nh; ++i) x |= uint64_t((j >> (P.b + i)) & 1) << P.hq[i];
  return x;
}

__device__ __forceinline__ uint64_t exp_tile_base(const ExpPassDev& P, uint64_t g) {
  uint64_t base = 0;
  for (int j = 0; j < P.ng; ++j) base |= ((g >> j) & 1) << P.gpos[j];
  return base;
}

// -v when s is 1, v when 0 (one XOR into the sign bit).
__device__ __forceinline__ double flip_sign(double v, uint32_t s) {
  return __hiloint2double(__double2hiint(v) ^ int(s << 31), __double2loint(v));
}

// v with its sign bit XOR-ed with bit 31 of m.
__device__ __forceinline__ double xor_sign(double v, uint32_t m) {
  return __hiloint2double(__double2hiint(v) ^ int(m), __double2loint(v));
}
__device__ __forceinline__ float xor_sign(float v, uint32_t m) {
  return __uint_as_float(__float_as_uint(v) ^ m);
}

__device__ __forceinline__ uint32_t ins0(uint32_t i, int hb) {
  return ((i >> hb) << (hb + 1)) | (i & ((1u << hb) - 1));
}

__device__ __forceinline__ uint32_t uni(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ double uni(double v) {
  return __hiloint2double(__builtin_amdgcn_readfirstlane(__double2hiint(v)),
                          __builtin_amdgcn_readfirstlane(__double2loint(v)));
}
__device__ __forceinline__ uint64_t uni(uint64_t v) {
  // (readfirstlane yields a signed int: widen through uint32_t, no sign extension)
  const uint32_t hi = uint32_t(__builtin_amdgcn_readfirstlane(uint32_t(v >> 32)));
  const uint32_t lo = uint32_t(__builtin_amdgcn_readfirstlane(uint32_t(v)));
  return (uint64_t(hi) << 32) | lo;
}

// Streaming of tiles through registers into LDS. Workgroups are persistent:
// workgroup b takes the contiguous range of tile indices [b per, (b + 1) per),
// per = ceil(tiles / grid), in increasing order (ExpTileRange below: the next
// tile's base is the current one carried within the non-local qubit mask), so
// its partial sum has a fixed order; the loads of its next tile are issued
// before it computes on the current one.
template <typename R, int NT, int LT = 0, int TMAX = kExpTileMax>
struct ExpTileStream {
  static constexpr int V = sizeof(R) == 4 ? 2 : 1;
  // loads per thread (16-byte pairs or complex128); TMAX: the largest tile in
  // 8-byte units (complex64 amplitudes)
  static constexpr int NL = TMAX / 2 / NT;
  uint64_t xt;          // per-thread part of the element addresses
  uint64_t xk[NL];      // workgroup-uniform parts
  cx<R> buf[NL * V];
  uint32_t TS;          // tile size (a constant when LT > 0: LT tile qubits)
  __device__ __forceinline__ ExpTileStream(const ExpPassDev& P) {
    TS = LT > 0 ? (1u << LT) : (1u << P.L);
    xt = exp_place(P, threadIdx.x * V);
#pragma unroll
    for (int k = 0; k < NL; ++k) xk[k] = exp_place(P, uint32_t(k) * NT * V);
  }
  __device__ __forceinline__ void fetch(const R* __restrict__ psi, uint64_t base) {
#pragma unroll
    for (int k = 0; k < NL; ++k) {
      const uint32_t e = threadIdx.x + uint32_t(k) * NT;
      if (e < TS / V) AmpIO<R, V>::load(psi, base | xt | xk[k], &buf[k * V]);
    }
  }
  __device__ __forceinline__ void to_lds(cx<R>* t) const {
#pragma unroll
    for (int k = 0; k < NL; ++k) {
      const uint32_t e = threadIdx.x + uint32_t(k) * NT;
      if (e < TS / V)
#pragma unroll
        for (int v = 0; v < V; ++v) t[e * V + v] = buf[k * V + v];
    }
  }
};

// Tiles of a workgroup: a contiguous range of tile indices (fixed order); the
// base of the next tile is the current one incremented within the mask of
// non-local qubits (a carry that skips local bit positions).
struct ExpTileRange {
  uint64_t g, end, base, gmask;
  __device__ __forceinline__ ExpTileRange(const ExpPassDev& P, uint64_t ntiles) {
    const uint64_t per = (ntiles + gridDim.x - 1) / gridDim.x;
    g = uint64_t(blockIdx.x) * per;
    end = g + per < ntiles ? g + per : ntiles;
    gmask = 0;
    for (int j = 0; j < P.ng; ++j) gmask |= uint64_t(1) << P.gpos[j];
    base = g < end ? exp_tile_base(P, g) : 0;
  }
  __device__ __forceinline__ uint64_t next_base() const { return ((base | ~gmask) + 1) & gmask; }
};

// Group gi of the pass with its first term's sign for the tile at base
// folded in (workgroup-uniform values, read through the scalar cache).
struct ExpGroup {
  double re, im;
  uint32_t lf, zl;
  int hbit, term_begin, term_count;
  uint32_t hmask, lft;
  const ExpGroupDev* d;
};

// The leading fields of a group record, read one group ahead so that their
// scalar loads overlap the current group's work; fold() gives the group with
// its first term's sign for the tile at base folded in.
struct ExpGroupHead {
  double re, im;
  uint64_t zg;
  uint32_t lf, zl;
  int hbit, term_begin, term_count;
  uint32_t kind, hmask, lft;
  __device__ __forceinline__ explicit ExpGroupHead(const ExpGroupDev& G)
      : re(G.re), im(G.im), zg(G.zg), lf(G.lf), zl(G.zl), hbit(G.hbit), term_begin(G.term_begin),
        term_count(G.term_count), kind(G.kind), hmask(G.hmask), lft(G.lft) {}
  __device__ __forceinline__ ExpGroup fold(uint64_t base, const ExpGroupDev* d) const {
    const uint32_t sg = uint32_t(__popcll(base & zg) & 1) << 31;
    return ExpGroup{xor_sign(re, sg), xor_sign(im, sg), lf, zl, hbit, term_begin, term_count, hmask, lft, d};
  }
};

// Stages the terms of a multi-term group for the tile at base (sign folded in).
__device__ __forceinline__ void exp_stage_terms(const ExpTermDev* __restrict__ terms, const ExpGroup& G,
                                                uint64_t base, ExpTermLds* et) {
  const int ns = min(G.term_count, kExpLdsTerms);
  for (int k = threadIdx.x; k < ns; k += blockDim.x) {
    const ExpTermDev T = terms[G.term_begin + k];
    const bool gneg = __popcll(base & T.zg) & 1;
    et[k] = {gneg ? -T.re : T.re, gneg ? -T.im : T.im, T.zl};
  }
}

__device__ __forceinline__ void exp_term(const ExpTermDev* __restrict__ terms, const ExpTermLds* et,
                                         const ExpGroup& G, uint64_t base, int k, double& re, double& im,
                                         uint32_t& zl) {
  if (k < kExpLdsTerms) {
    re = et[k].re;
    im = et[k].im;
    zl = et[k].zl;
  } else {
    const ExpTermDev T = terms[G.term_begin + k];
    const bool gneg = __popcll(base & T.zg) & 1;
    re = gneg ? -T.re : T.re;
    im = gneg ? -T.im : T.im;
    zl = T.zl;
  }
}

// Tile qubits of the fixed-size expectation and lambda kernel variants (64
// KiB tiles), and the lambda workgroup size and outputs per thread (1024
// threads: 8 complex64 or 4 complex128 outputs each; 512 threads with 8
// complex128 outputs took 181 VGPRs, two wavefronts per SIMD).
template <typename R>
__host__ __device__ constexpr int exp_tile_bits() {
  return sizeof(R) == 4 ? 13 : 12;
}
template <typename R>
__host__ __device__ constexpr int obs_tile_bits() {
  return sizeof(R) == 4 ? 13 : 12;
}
template <typename R>
__host__ __device__ constexpr int obs_threads() {
  return 1024;
}
template <typename R>
__host__ __device__ constexpr int obs_out() {
  return (1 << obs_tile_bits<R>()) / obs_threads<R>();
}

// Re (REAL) or Im of conj(b) a. complex64: formed in FP32 (relative error
// <= 2^-23 of |a||b|; see exp_pairs for the sums), which
// halves the vector instructions per pair against converting all four
// components first; complex128: FP64.
template <typename R, bool REAL>
__device__ __forceinline__ R pair_product(const cx<R>& a, const cx<R>& b) {
  return REAL ? fma(b.re, a.re, b.im * a.im) : fma(b.re, a.im, -(b.im * a.re));
}

// One single-term group with flip mask lf != 0 over a tile: the sum over the
// pairs (x, x ^ lf), x with bit hb clear, of Re (REAL) or Im of
// conj(psi_y) psi_x with the term's local Z/Y sign. A thread's pair products
// are summed in the amplitude precision in chunks of at most 8 (complex64:
// FP32, one conversion to FP64 per chunk instead of one per pair; with the
// products' own rounding the error is at most 9 x 2^-24 of the sum of
// |psi_x||psi_y| over the pairs, i.e. of <psi|psi>/2) and the chunks, threads
// and tiles in FP64. x is the thread
// part xt (tx = t + xt) OR-ed with a workgroup-uniform step part xs (disjoint
// bits); likewise y = (xt ^ (lf & thread bits)) | (xs ^ (lf outside them)),
// so each step adds a uniform offset to two per-thread LDS pointers. The sign
// splits the same way: pt (per thread, in bit 31) XOR the uniform parity of
// xs & zl. The uniform parts come precomputed with the group.
template <typename R, bool REAL, bool FULL, int NP, int NT>
__device__ __forceinline__ double exp_pairs(const cx<R>* tx, const cx<R>* ty, const ExpGroupDev& D, uint32_t pt,
                                            uint32_t TS, uint32_t tid) {
  // every LDS read of the group is issued before its arithmetic (one wait
  // instead of one per few pairs)
  cx<R> a[NP], b[NP];
#pragma unroll
  for (int k = 0; k < NP; ++k) {
    const uint32_t i0 = uint32_t(k) * NT;
    if (i0 < TS / 2 && (FULL || i0 + tid < TS / 2)) {
      a[k] = tx[D.offx[k]];
      b[k] = ty[D.offy[k]];
    } else {
      a[k] = b[k] = cx<R>{R(0), R(0)};  // zero product
    }
  }
  double sd = 0.0;
  R sw = R(0);
#pragma unroll
  for (int k = 0; k < NP; ++k) {
    if (uint32_t(k) * NT >= TS / 2) break;
    if constexpr (sizeof(R) == 4)  // complex64 plans store the step sign as +-1.0f
      sw = fmaf(__uint_as_float(D.sgn[k]), pair_product<R, REAL>(a[k], b[k]), sw);
    else
      sw += xor_sign(pair_product<R, REAL>(a[k], b[k]), D.sgn[k]);
    if ((k & 7) == 7) {  // sums of at most 8 products in the amplitude precision
      sd += double(sw);
      sw = R(0);
    }
  }
  sd += double(sw);  // (the loop may end early on small tiles)
  return xor_sign(sd, pt);  // the thread's part of the sign, common to every step
}

// <psi|O|psi> over the tiles of one pass. Sums over threads and tiles are
// FP64; single-term groups form their products in the amplitude precision,
// and a flip group also sums each thread's 8 pairs per tile in it
// (complex64: |dE| <= 9 x 2^-24 sum |alpha| <psi|psi> beyond the stored
// amplitudes, see exp_pairs); multi-term groups work in FP64. Each workgroup sums its
// tiles in a fixed order into partial[blockIdx.x] (added to the value of
// earlier passes when accumulate is set). MODE 0: any tile size (per-lane
// guards); 1: the tile has at least two amplitudes per thread, so every loop
// below has a workgroup-uniform trip count; 2: the tile has exp_tile_bits<R>()
// qubits (trip counts known at compile time).
template <typename R, int MODE>
__global__ void __launch_bounds__(kExpThreadsE)
    k_expect_tile(const R* __restrict__ psi, const ExpPassDev* __restrict__ passes, int pass_idx,
                  const ExpGroupDev* __restrict__ groups, const ExpTermDev* __restrict__ terms,
                  double* __restrict__ partial, int accumulate, uint64_t ntiles) {
  constexpr int NT = kExpThreadsE;
  constexpr int NA = kExpTileMax / NT;  // amplitudes per thread, at most
  constexpr bool FULL = MODE >= 1;
  constexpr int LT = MODE == 2 ? exp_tile_bits<R>() : 0;
  extern __shared__ __align__(16) char smem[];
  __shared__ double red[NT / 64];
  __shared__ ExpTermLds et[kExpLdsTerms];
  cx<R>* t = reinterpret_cast<cx<R>*>(smem);
  const ExpPassDev& P = passes[pass_idx];
  const uint32_t TS = LT > 0 ? (1u << LT) : (1u << P.L);
  const uint32_t tid = threadIdx.x;
  ExpTileStream<R, NT, LT> io(P);
  ExpTileRange tr(P, ntiles);
  double acc = 0.0;
  if (tr.g < tr.end) io.fetch(psi, tr.base);
  for (; tr.g < tr.end; ++tr.g) {
    const uint64_t base = tr.base;
    __syncthreads();  // previous tile consumed
    io.to_lds(t);
    if (tr.g + 1 < tr.end) {
      tr.base = tr.next_base();
      io.fetch(psi, tr.base);
    }
    const ExpGroupDev* gd = groups + P.grp_begin;
    ExpGroupHead head(gd[0]);
    __syncthreads();  // tile (and, first time, the group table) in LDS
    for (int left = P.grp_count; left > 0; --left, ++gd) {
      const ExpGroup G = head.fold(base, gd);
      const uint32_t kind = head.kind;
      head = ExpGroupHead(gd[1]);  // (after a pass's last record: the next pass's first, or the spare)
      const int nt = G.term_count;
      if (kind == kExpFlipRe || kind == kExpFlipIm) {
        // one term (the common case for random strings). A Hermitian term's
        // coefficient alpha i^nY is real (nY even) or imaginary (nY odd):
        // only Re or Im of w = conj(psi[y]) psi[x] counts
        const uint32_t xt = ((tid & ~G.hmask) << 1) | (tid & G.hmask);  // ins0(tid, hbit)
        const cx<R>* tx = t + xt;
        const cx<R>* ty = t + (xt ^ G.lft);
        uint32_t pt = uint32_t(__popc(xt & G.zl) & 1) << 31;
        if (kind == kExpFlipRe)
          acc += 2.0 * G.re * exp_pairs<R, true, FULL, NA / 2, NT>(tx, ty, *G.d, pt, TS, tid);
        else
          acc -= 2.0 * G.im * exp_pairs<R, false, FULL, NA / 2, NT>(tx, ty, *G.d, pt, TS, tid);
        continue;
      }
      if (nt > 1) {
        __syncthreads();
        exp_stage_terms(terms, G, base, et);
        __syncthreads();
      }
      if (kind == kExpZ1) {
        // sum of +-|psi_x|^2: thread part of the sign once, uniform part per step
        uint32_t pt = uint32_t(__popc(tid & G.zl) & 1) << 31;
        double sum = 0.0;
#pragma unroll
        for (int k = 0; k < NA; ++k) {
          const uint32_t j0 = uint32_t(k) * NT;
          if (j0 >= TS) break;
          if (FULL || j0 + tid < TS) {
            const cx<R> a = t[j0 + tid];
            sum += xor_sign(double(pair_product<R, true>(a, a)), G.d->sgn[k]);
          }
        }
        acc += G.re * xor_sign(sum, pt);
      } else if (kind == kExpZN) {
        for (uint32_t j = tid; j < TS; j += NT) {
          const cx<R> a = t[j];
          double c = 0.0;
          for (int k = 0; k < nt; ++k) {
            double re, im;
            uint32_t zl;
            exp_term(terms, et, G, base, k, re, im, zl);
            c += (__popc(j & zl) & 1) ? -re : re;
          }
          acc += (double(a.re) * a.re + double(a.im) * a.im) * c;
        }
      } else {  // kExpFlipN
        const int hb = G.hbit;
        const uint32_t lf = G.lf;
        for (uint32_t i = tid; i < TS / 2; i += NT) {
          const uint32_t x = ins0(i, hb);
          const cx<R> a = t[x], bb = t[x ^ lf];
          // w = conj(psi[y]) psi[x]
          const double wr = double(bb.re) * a.re + double(bb.im) * a.im;
          const double wi = double(bb.re) * a.im - double(bb.im) * a.re;
          double cr = 0.0, ci = 0.0;
          for (int k = 0; k < nt; ++k) {
            double re, im;
            uint32_t zl;
            exp_term(terms, et, G, base, k, re, im, zl);
            const bool neg = __popc(x & zl) & 1;
            cr += neg ? -re : re;
            ci += neg ? -im : im;
          }
          acc += 2.0 * (wr * cr - wi * ci);
        }
      }
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  __syncthreads();
  if ((tid & 63) == 0) red[tid >> 6] = acc;
  __syncthreads();
  if (tid == 0) {
    double r = 0.0;
    for (int w = 0; w < NT / 64; ++w) r += red[w];
    partial[blockIdx.x] = accumulate ? partial[blockIdx.x] + r : r;
  }
}

template <typename R>
__global__ void __launch_bounds__(kExpThreads) k_zero_amps(R* __restrict__ a, uint64_t n) {
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride)
    store1(a, i, cx<R>{R(0), R(0)});
}

// lambda = O psi over the tiles of one pass (the pass's flip masks only): every
// output y of a tile gathers psi[y ^ F] from LDS for each group F of the pass,
// with c(x) = sum over the group's terms of alpha i^nY (-1)^|x & z| (in FP64),
// summed per pass in the amplitude precision (that of lambda itself); the
// first pass writes lambda, later passes add to it.

// One single-term group's contribution to this thread's outputs: lambda_y +=
// c psi_{y ^ F} (REAL) or i c psi_{y ^ F} with c = +-coefficient, the sign of
// (-1)^|x & z| split into a per-thread bit (pt) and a per-step bit.
template <typename R, bool REAL, bool FIXED, int NT>
__device__ __forceinline__ void obs_single(const cx<R>* t, uint32_t tid, uint32_t lf, uint32_t zl, uint32_t pt,
                                           R cm, uint32_t TS, R* ar, R* ai) {
  constexpr int KO = obs_out<R>();
#pragma unroll
  for (int k = 0; k < KO; ++k) {
    const uint32_t y = tid + uint32_t(k) * NT;
    if (FIXED || y < TS) {
      const cx<R> v = t[y ^ lf];
      const R c = (pt ^ (__popc((uint32_t(k) * NT) & zl) & 1)) ? -cm : cm;
      if constexpr (REAL) {
        ar[k] += c * v.re;
        ai[k] += c * v.im;
      } else {
        ar[k] += -c * v.im;
        ai[k] += c * v.re;
      }
    }
  }
}

// FIXED: the tile has obs_tile_bits<R>() qubits and every thread's outputs
// exist (complex64: 2^13 = 8 x 1024, complex128: 2^12 = 4 x 1024). Tiles of
// at most obs_out<R>() x NT amplitudes.
template <typename R, bool FIXED, int NT>
__global__ void __launch_bounds__(NT)
    k_apply_obs_tile(const R* __restrict__ psi, R* __restrict__ lam, const ExpPassDev* __restrict__ passes,
                     int pass_idx, const ExpGroupDev* __restrict__ groups,
                     const ExpTermDev* __restrict__ terms, int accumulate, uint64_t ntiles) {
  constexpr int KO = obs_out<R>();
  extern __shared__ __align__(16) char smem[];
  __shared__ ExpTermLds et[kExpLdsTerms];
  cx<R>* t = reinterpret_cast<cx<R>*>(smem);
  const ExpPassDev& P = passes[pass_idx];
  const uint32_t TS = FIXED ? (1u << obs_tile_bits<R>()) : (1u << P.L);
  const uint32_t tid = threadIdx.x;
  // (the stream's maximum counts 8-byte units: a complex128 tile of 4 x NT
  // amplitudes is 8 x NT of them)
  ExpTileStream<R, NT, 0, obs_out<R>() * NT * int(sizeof(R) / 4)> io(P);
  const uint64_t yt = exp_place(P, tid);
  uint64_t yk[KO];
#pragma unroll
  for (int k = 0; k < KO; ++k) yk[k] = exp_place(P, uint32_t(k) * NT);
  ExpTileRange tr(P, ntiles);
  if (tr.g < tr.end) io.fetch(psi, tr.base);
  for (; tr.g < tr.end; ++tr.g) {
    const uint64_t base = tr.base;
    __syncthreads();  // previous tile consumed
    io.to_lds(t);
    if (tr.g + 1 < tr.end) {
      tr.base = tr.next_base();
      io.fetch(psi, tr.base);
    }
    // per-pass sums in the amplitude precision (lambda is stored in it)
    R ar[KO], ai[KO];
#pragma unroll
    for (int k = 0; k < KO; ++k) ar[k] = ai[k] = R(0);
    const ExpGroupDev* gd = groups + P.grp_begin;
    ExpGroupHead head(gd[0]);
    __syncthreads();  // tile (and, first time, the group table) in LDS
    for (int left = P.grp_count; left > 0; --left, ++gd) {
      const ExpGroup G = head.fold(base, gd);
      const uint32_t kind = head.kind;
      head = ExpGroupHead(gd[1]);  // (see k_expect_tile)
      const uint32_t lf = G.lf;
      if (kind == kExpZ1 || kind == kExpFlipRe || kind == kExpFlipIm) {
        // alpha i^nY is real or imaginary (a Z-only string's is real):
        // lambda += c psi or i c psi
        const uint32_t pt = (__popc((tid ^ lf) & G.zl) & 1);
        if (kind != kExpFlipIm)
          obs_single<R, true, FIXED, NT>(t, tid, lf, G.zl, pt, R(G.re), TS, ar, ai);
        else
          obs_single<R, false, FIXED, NT>(t, tid, lf, G.zl, pt, R(G.im), TS, ar, ai);
        continue;
      }
      const int nt = G.term_count;
      __syncthreads();
      exp_stage_terms(terms, G, base, et);
      __syncthreads();
      {
#pragma unroll
        for (int k = 0; k < KO; ++k) {
          const uint32_t y = tid + uint32_t(k) * NT;
          if (y < TS) {
            const uint32_t x = y ^ lf;
            const cx<R> v = t[x];
            double cr = 0.0, ci = 0.0;
            for (int q = 0; q < nt; ++q) {
              double re, im;
              uint32_t zl;
              exp_term(terms, et, G, base, q, re, im, zl);
              const bool neg = __popc(x & zl) & 1;
              cr += neg ? -re : re;
              ci += neg ? -im : im;
            }
            ar[k] += R(cr * double(v.re) - ci * double(v.im));
            ai[k] += R(cr * double(v.im) + ci * double(v.re));
          }
        }
      }
    }
#pragma unroll
    for (int k = 0; k < KO; ++k) {
      if (!FIXED && tid + uint32_t(k) * NT >= TS) continue;
      cx<R> r;
      if (accumulate) {
        const cx<R> old = load1(lam, base | yt | yk[k]);
        r = {old.re + ar[k], old.im + ai[k]};
      } else {
        r = {ar[k], ai[k]};
      }
      store1(lam, base | yt | yk[k], r);
    }
  }
}

// Groups whose flip mask F has more qubits than a tile holds: the pairs
// (x, x ^ F), x with the highest bit h of F clear, are read straight from the
// state (both members of a pair in one thread; consecutive threads read
// consecutive x). Each workgroup walks the pair indices in a fixed
// grid-stride order and adds its FP64 sum to partial[blockIdx.x], the
// partials of the tiled passes (same grid), so the value stays bitwise
// reproducible.
template <typename R>
__global__ void __launch_bounds__(kExpThreadsE)
    k_expect_wide(const R* __restrict__ psi, uint64_t flip, int hbit, const ExpTermDev* __restrict__ terms,
                  int nt, uint64_t pairs, double* __restrict__ partial, int accumulate) {
  __shared__ double red[kExpThreadsE / 64];
  const uint64_t stride = uint64_t(gridDim.x) * kExpThreadsE;
  const uint64_t lowm = (uint64_t(1) << hbit) - 1;
  double acc = 0.0;
  for (uint64_t i = uint64_t(blockIdx.x) * kExpThreadsE + threadIdx.x; i < pairs; i += stride) {
    const uint64_t x = ((i & ~lowm) << 1) | (i & lowm);
    const cx<R> a = load1(psi, x), bb = load1(psi, x ^ flip);
    // w = conj(psi[y]) psi[x]
    const double wr = double(bb.re) * a.re + double(bb.im) * a.im;
    const double wi = double(bb.re) * a.im - double(bb.im) * a.re;
    double cr = 0.0, ci = 0.0;
    for (int k = 0; k < nt; ++k) {
      const ExpTermDev T = terms[k];
      const bool neg = __popcll(x & T.zg) & 1;
      cr += neg ? -T.re : T.re;
      ci += neg ? -T.im : T.im;
    }
    acc += 2.0 * (wr * cr - wi * ci);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = 0.0;
    for (int w = 0; w < kExpThreadsE / 64; ++w) r += red[w];
    partial[blockIdx.x] = accumulate ? partial[blockIdx.x] + r : r;
  }
}

// lambda_y (+)= c(x) psi_x, x = y ^ F, for one group whose flip mask F has
// more qubits than a tile holds (c(x) as in the tiled passes, in FP64; the
// sum is stored in the amplitude precision).
template <typename R>
__global__ void __launch_bounds__(kExpThreads)
    k_apply_obs_wide(const R* __restrict__ psi, R* __restrict__ lam, uint64_t flip,
                     const ExpTermDev* __restrict__ terms, int nt, uint64_t N, int accumulate) {
  const uint64_t stride = uint64_t(gridDim.x) * kExpThreads;
  for (uint64_t y = uint64_t(blockIdx.x) * kExpThreads + threadIdx.x; y < N; y += stride) {
    const uint64_t x = y ^ flip;
    const cx<R> v = load1(psi, x);
    double cr = 0.0, ci = 0.0;
    for (int k = 0; k < nt; ++k) {
      const ExpTermDev T = terms[k];
      const bool neg = __popcll(x & T.zg) & 1;
      cr += neg ? -T.re : T.re;
      ci += neg ? -T.im : T.im;
    }
    cx<R> r{R(cr * double(v.re) - ci * double(v.im)), R(cr * double(v.im) + ci * double(v.re))};
    if (accumulate) {
      const cx<R> old = load1(lam, y);
      r = {old.re + r.re, old.im + r.im};
    }
    store1(lam, y, r);
  }
}

__global__ void __launch_bounds__(kExpThreads)
    k_exp_sum(const double* __restrict__ partial, uint64_t count, double* __restrict__ out) {
  __shared__ double red[kExpThreads / 64];
  double acc = 0.0;
  for (uint64_t i = threadIdx.x; i < count; i += blockDim.x) acc += partial[i];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = 0.0;
    for (int w = 0; w < kExpThreads / 64; ++w) r += red[w];
    out[0] = r;
  }
}

namespace {

int popc64(uint64_t x) { return __builtin_popcountll(x); }

// Local qubit set of the next pass, given the flip masks hi (low qubits
// removed) of the groups not yet evaluated; low: the always-local low qubits.
// The set is grown from a seed mask by adding, one at a time, the mask that
// needs the fewest new local qubits (ties: the one after which most masks lie
// inside the set), up to L qubits; of the sets grown from up to kPackSeeds
// seeds (spread over the list), the one holding the most masks is kept. On
// random weight-4 strings at 30 qubits this takes 21 passes where adding
// masks to one set in list order takes 26.
constexpr int kPackSeeds = 64, kPackTies = 8;

uint64_t pick_pass_local(const std::vector<uint64_t>& hi, uint64_t low, int L) {
  const size_t nm = hi.size();
  auto inside = [&](uint64_t loc) {
    int c = 0;
    for (uint64_t g : hi) c += (g & ~loc) == 0;
    return c;
  };
  uint64_t best = low;
  int best_cov = -1;
  const size_t ns = std::min<size_t>(nm, kPackSeeds);
  std::vector<uint64_t> ties;
  for (size_t si = 0; si < ns; ++si) {
    uint64_t local = low | hi[si * nm / ns];
    while (true) {
      int mn = 65;
      ties.clear();
      for (uint64_t f : hi) {
        const uint64_t nf = f & ~local;
        if (!nf || popc64(local | f) > L) continue;
        const int need = popc64(nf);
        if (need < mn) {
          mn = need;
          ties.assign(1, f);
        } else if (need == mn && int(ties.size()) < kPackTies) {
          ties.push_back(f);
        }
      }
      if (ties.empty()) break;
      uint64_t pick = ties[0];
      if (ties.size() > 1) {
        int pc = -1;
        for (uint64_t f : ties) {
          const int c = inside(local | f);
          if (c > pc) {
            pc = c;
            pick = f;
          }
        }
      }
      local |= pick;
    }
    const int c = inside(local);
    if (c > best_cov) {
      best_cov = c;
      best = local;
    }
  }
  return best;
}

// Moves flip-mask groups from heavily loaded passes to lighter ones whose
// local set also holds their mask (the packing above fills the first passes
// and leaves the last ones light). Cost of a pass in units of one
// single-term record's work (complex64, 30 qubits: 0.12 ms each), measured:
// max(10.9, 4.9 + records) -- at least its read of the state, and a fixed
// part per tile on top of its records; a shared record of more than
// kExpSplitTerms terms costs about six. A group moves when the modelled sum
// drops; deterministic (passes by load, groups in order).
void rebalance_passes(const std::vector<Group>& groups, const std::vector<uint64_t>& plocal,
                      std::vector<std::vector<int>>& pchosen) {
  const size_t np = plocal.size();
  auto weight = [&](int gi) { return groups[gi].count <= kExpSplitTerms ? double(groups[gi].count) : 6.0; };
  auto cost = [](double g) { return std::max(10.9, 4.9 + g); };
  std::vector<double> load(np, 0.0);
  for (size_t pi = 0; pi < np; ++pi)
    for (int gi : pchosen[pi]) load[pi] += weight(gi);
  for (int round = 0; round < 64; ++round) {
    bool moved = false;
    std::vector<size_t> order(np);
    for (size_t pi = 0; pi < np; ++pi) order[pi] = pi;
    std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) { return load[a] > load[b]; });
    for (size_t pa : order) {
      for (size_t k = 0; k < pchosen[pa].size();) {
        const int gi = pchosen[pa][k];
        const double w = weight(gi);
        size_t best = np;
        double bd = -1e-9;
        for (size_t pb = 0; pb < np; ++pb) {
          if (pb == pa || (groups[gi].flip & ~plocal[pb])) continue;
          const double d = cost(load[pa] - w) + cost(load[pb] + w) - cost(load[pa]) - cost(load[pb]);
          if (d < bd) {
            bd = d;
            best = pb;
          }
        }
        if (best == np) {
          ++k;
          continue;
        }
        pchosen[pa].erase(pchosen[pa].begin() + long(k));
        pchosen[best].push_back(gi);
        load[pa] -= w;
        load[best] += w;
        moved = true;
      }
    }
    if (!moved) break;
  }
}

ExpPlan* build_exp_plan(const qsv_observable* o, qsv_dtype dt) {
  std::vector<Group> groups;
  std::vector<GTerm> terms;
  build_groups(o, groups, terms);
  ExpPlan* p = new ExpPlan();
  const int n = o->n;
  p->n = n;
  // tile: 2^L amplitudes, 64 KiB (2^13 complex64, 2^12 complex128): more
  // flip masks fit a pass (18 expectation passes instead of 21 for the
  // 200-term 30-qubit observable); QSV_EXPECT_TILE lowers L, for tuning
  int Ldef = dt == QSV_C64 ? 13 : 12;
  if (const char* e = std::getenv("QSV_EXPECT_TILE")) Ldef = std::max(6, std::min(Ldef, std::atoi(e)));
  p->L = std::min(n, Ldef);
  int bdef = dt == QSV_C64 ? 4 : 3;  // 128-byte contiguous runs
  if (const char* e = std::getenv("QSV_EXPECT_LOW")) bdef = std::max(1, std::min(8, std::atoi(e)));
  p->b = std::min(p->L, bdef);
  const int L = p->L, b = p->b;
  const uint64_t low = (uint64_t(1) << b) - 1;
  std::vector<int> rem;
  for (size_t i = 0; i < groups.size(); ++i) {
    if (popc64(groups[i].flip | low) <= L) {
      rem.push_back(int(i));
      continue;
    }
    // more flip qubits than a tile holds: evaluated on its own, pairs read
    // straight from the state
    const Group& G = groups[i];
    ExpWide w{G.flip, 63 - __builtin_clzll(G.flip), int(p->wide_terms.size()), G.count};
    for (int k = G.begin; k < G.begin + G.count; ++k)
      p->wide_terms.push_back(ExpTermDev{terms[k].re, terms[k].im, terms[k].z, 0u, 0u});
    p->wide.push_back(w);
  }
  std::vector<uint64_t> plocal;
  std::vector<std::vector<int>> pchosen;
  while (!rem.empty()) {
    std::vector<uint64_t> hi;
    for (int r : rem) hi.push_back(groups[r].flip & ~low);
    const uint64_t local0 = pick_pass_local(hi, low, L);
    std::vector<int> chosen, rest;
    for (int r : rem) ((groups[r].flip & ~local0) == 0 ? chosen : rest).push_back(r);
    rem.swap(rest);
    uint64_t local = local0;
    for (int q = 0; q < n && popc64(local) < L; ++q) local |= uint64_t(1) << q;
    plocal.push_back(local);
    pchosen.push_back(chosen);
  }
  rebalance_passes(groups, plocal, pchosen);
  for (size_t pi = 0; pi < plocal.size(); ++pi) {
    const uint64_t local = plocal[pi];
    const std::vector<int>& chosen = pchosen[pi];
    if (chosen.empty()) continue;  // (every group moved elsewhere)
    std::vector<int> lpos(64, -1), loc;
    for (int q = 0; q < 64; ++q)
      if (local >> q & 1) {
        lpos[q] = int(loc.size());
        loc.push_back(q);
      }
    ExpPassDev d{};
    d.L = L;
    d.b = b;
    d.nh = L - b;
    for (int i = 0; i < d.nh; ++i) d.hq[i] = loc[b + i];
    d.ng = 0;
    for (int q = 0; q < n; ++q)
      if (!(local >> q & 1)) d.gpos[d.ng++] = q;
    d.grp_begin = int(p->groups.size());
    for (int gi : chosen) {
      const Group& G = groups[gi];
      uint32_t lf = 0;
      for (int q = 0; q < n; ++q)
        if (G.flip >> q & 1) lf |= 1u << lpos[q];
      // a few terms on one flip mask run as that many single-term records
      // (the single-term loop, once per term); more share one record
      const int nrec = G.count <= kExpSplitTerms ? G.count : 1;
      for (int r = 0; r < nrec; ++r) {
        ExpGroupDev gd{};
        gd.lf = lf;
        gd.hbit = lf ? 31 - __builtin_clz(lf) : 0;
        gd.term_begin = int(p->terms.size());
        gd.term_count = nrec > 1 ? 1 : G.count;
        const double im0 = terms[G.begin + (nrec > 1 ? r : 0)].im;
        gd.kind = lf == 0 ? (gd.term_count == 1 ? kExpZ1 : kExpZN)
                          : (gd.term_count > 1 ? kExpFlipN : (im0 == 0.0 ? kExpFlipRe : kExpFlipIm));
        const int k0 = G.begin + (nrec > 1 ? r : 0);
        for (int k = k0; k < k0 + gd.term_count; ++k) {
          ExpTermDev td{};
          td.re = terms[k].re;
          td.im = terms[k].im;
          for (int q = 0; q < n; ++q) {
            if (!(terms[k].z >> q & 1)) continue;
            if (lpos[q] >= 0) td.zl |= 1u << lpos[q];
            else td.zg |= uint64_t(1) << q;
          }
          if (k == k0) {
            gd.re = td.re;
            gd.im = td.im;
            gd.zg = td.zg;
            gd.zl = td.zl;
          }
          p->terms.push_back(td);
        }
        // uniform step parts for kExpThreadsE-thread workgroups
        auto ins0h = [](uint32_t i, int hb) { return ((i >> hb) << (hb + 1)) | (i & ((1u << hb) - 1)); };
        const uint32_t mt = ins0h(kExpThreadsE - 1, gd.hbit);
        gd.hmask = (1u << gd.hbit) - 1;
        gd.lft = lf & mt;
        for (int k = 0; k < kExpSteps; ++k) {
          const uint32_t xs = lf ? ins0h(uint32_t(k) * kExpThreadsE, gd.hbit) : uint32_t(k) * kExpThreadsE;
          if (lf && k < kExpSteps / 2) {
            gd.offx[k] = xs;
            gd.offy[k] = xs ^ (lf & ~mt);
          }
          if (!lf || k < kExpSteps / 2) gd.sgn[k] = uint32_t(__builtin_popcount(xs & gd.zl) & 1) << 31;
          // flip records of complex64 plans: the sign as +-1.0f, applied by
          // one FMA into the running sum (exact: the same result as a sign
          // flip and an add)
          if (lf && k < kExpSteps / 2 && dt == QSV_C64) gd.sgn[k] |= 0x3f800000u;
        }
        p->groups.push_back(gd);
      }
    }
    d.grp_count = int(p->groups.size()) - d.grp_begin;
    p->passes.push_back(d);
  }
  // the kernels read each record's successor ahead of use: one spare record
  // after the last pass keeps that read inside the table
  if (!p->passes.empty()) p->groups.push_back(ExpGroupDev{});
  return p;
}

int upload_exp_plan(ExpPlan* p, int device) {
  if (p->dev && p->device == device) return QSV_OK;
  if (p->dev) (void)hipFree(p->dev);
  p->dev = nullptr;
  const size_t a = p->passes.size() * sizeof(ExpPassDev);
  p->off_groups = (a + 255) / 256 * 256;
  const size_t bsz = p->groups.size() * sizeof(ExpGroupDev);
  p->off_terms = (p->off_groups + bsz + 255) / 256 * 256;
  p->off_wide = (p->off_terms + p->terms.size() * sizeof(ExpTermDev) + 255) / 256 * 256;
  const size_t total = p->off_wide + std::max<size_t>(1, p->wide_terms.size()) * sizeof(ExpTermDev);
  if (hipMalloc(&p->dev, total) != hipSuccess) return fail(QSV_ENOMEM, "observable plan allocation failed");
  char* d = static_cast<char*>(p->dev);
  if (a) QSV_HIP_CHECK(hipMemcpy(d, p->passes.data(), a, hipMemcpyHostToDevice));
  if (bsz) QSV_HIP_CHECK(hipMemcpy(d + p->off_groups, p->groups.data(), bsz, hipMemcpyHostToDevice));
  if (!p->terms.empty())
    QSV_HIP_CHECK(hipMemcpy(d + p->off_terms, p->terms.data(), p->terms.size() * sizeof(ExpTermDev),
                            hipMemcpyHostToDevice));
  if (!p->wide_terms.empty())
    QSV_HIP_CHECK(hipMemcpy(d + p->off_wide, p->wide_terms.data(), p->wide_terms.size() * sizeof(ExpTermDev),
                            hipMemcpyHostToDevice));
  p->device = device;
  return QSV_OK;
}

template <typename R>
int expect_tiled_t(qsv_state* s, qsv_observable* o, double* out) {
  ExpPlan*& pl = o->exp_plan[s->dtype];
  if (!pl) pl = build_exp_plan(o, s->dtype);
  if (pl->passes.empty() && pl->wide.empty()) {
    *out = 0.0;
    return QSV_OK;
  }
  int rc = upload_exp_plan(pl, s->device);
  if (rc) return rc;
  const uint64_t tiles = dim(s->n - pl->L);
  const uint64_t grid = std::min<uint64_t>(tiles, exp_grid_max());
  if ((rc = ensure_reduce_scratch(s, size_t(grid) + 1))) return rc;
  const size_t lds = (size_t(1) << pl->L) * sizeof(cx<R>);
  // kernel variant: tile of the default size (compile-time trip counts), at
  // least two amplitudes per thread, or any size
  const int mode = pl->L == exp_tile_bits<R>() ? 2 : ((size_t(1) << pl->L) >= size_t(2 * kExpThreadsE) ? 1 : 0);
  const void* kfn = mode == 2   ? reinterpret_cast<const void*>(&k_expect_tile<R, 2>)
                    : mode == 1 ? reinterpret_cast<const void*>(&k_expect_tile<R, 1>)
                                : reinterpret_cast<const void*>(&k_expect_tile<R, 0>);
  QSV_HIP_CHECK(hipFuncSetAttribute(kfn, hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)));
  char* d = static_cast<char*>(pl->dev);
  for (size_t pi = 0; pi < pl->passes.size(); ++pi) {
    ProfScope ps("expect", double(sizeof(cx<R>)) * double(dim(s->n)), s->stream);
    const auto* pd = reinterpret_cast<const ExpPassDev*>(d);
    const auto* gd = reinterpret_cast<const ExpGroupDev*>(d + pl->off_groups);
    const auto* td = reinterpret_cast<const ExpTermDev*>(d + pl->off_terms);
    const R* psi = static_cast<const R*>(s->ptr);
    if (mode == 2)
      hipLaunchKernelGGL((k_expect_tile<R, 2>), dim3(unsigned(grid)), dim3(kExpThreadsE), lds, s->stream, psi,
                         pd, int(pi), gd, td, s->red, pi > 0 ? 1 : 0, tiles);
    else if (mode == 1)
      hipLaunchKernelGGL((k_expect_tile<R, 1>), dim3(unsigned(grid)), dim3(kExpThreadsE), lds, s->stream, psi,
                         pd, int(pi), gd, td, s->red, pi > 0 ? 1 : 0, tiles);
    else
      hipLaunchKernelGGL((k_expect_tile<R, 0>), dim3(unsigned(grid)), dim3(kExpThreadsE), lds, s->stream, psi,
                         pd, int(pi), gd, td, s->red, pi > 0 ? 1 : 0, tiles);
    QSV_HIP_CHECK(hipGetLastError());
  }
  const auto* wt = reinterpret_cast<const ExpTermDev*>(d + pl->off_wide);
  for (size_t wi = 0; wi < pl->wide.size(); ++wi) {
    ProfScope ps("expect_wide", double(sizeof(cx<R>)) * double(dim(s->n)), s->stream);
    const ExpWide& w = pl->wide[wi];
    hipLaunchKernelGGL((k_expect_wide<R>), dim3(unsigned(grid)), dim3(kExpThreadsE), 0, s->stream,
                       static_cast<const R*>(s->ptr), w.flip, w.hbit, wt + w.term_begin, w.term_count,
                       dim(s->n - 1), s->red, pl->passes.empty() && wi == 0 ? 0 : 1);
    QSV_HIP_CHECK(hipGetLastError());
  }
  hipLaunchKernelGGL(k_exp_sum, dim3(1), dim3(kExpThreads), 0, s->stream, s->red, grid, s->red + grid);
  QSV_HIP_CHECK(hipGetLastError());
  QSV_HIP_CHECK(hipMemcpyAsync(s->red_host, s->red + grid, sizeof(double), hipMemcpyDeviceToHost,
                               s->stream));
  QSV_HIP_CHECK(hipStreamSynchronize(s->stream));
  *out = s->red_host[0];
  return QSV_OK;
}

template <typename R>
int apply_obs_tiled_t(const qsv_state* in, qsv_observable* o, qsv_state* out) {
  ExpPlan*& pl = o->exp_plan[in->dtype];
  if (!pl) pl = build_exp_plan(o, in->dtype);
  const uint64_t N = dim(in->n);
  if (pl->passes.empty() && pl->wide.empty()) {  // no terms: lambda = 0
    const uint64_t blocks = std::min<uint64_t>((N + kExpThreads - 1) / kExpThreads, 65536);
    hipLaunchKernelGGL((k_zero_amps<R>), dim3(unsigned(blocks)), dim3(kExpThreads), 0, in->stream,
                       static_cast<R*>(out->ptr), N);
    QSV_HIP_CHECK(hipGetLastError());
    return QSV_OK;
  }
  int rc = upload_exp_plan(pl, in->device);
  if (rc) return rc;
  const uint64_t tiles = dim(in->n - pl->L);
  const size_t lds = (size_t(1) << pl->L) * sizeof(cx<R>);
  // compile-time output count when every thread has obs_out<R>() outputs
  constexpr int NTo = obs_threads<R>();
  const bool fixed = pl->L == obs_tile_bits<R>() && (size_t(1) << pl->L) == size_t(obs_out<R>()) * NTo;
  QSV_HIP_CHECK(hipFuncSetAttribute(fixed ? reinterpret_cast<const void*>(&k_apply_obs_tile<R, true, NTo>)
                                          : reinterpret_cast<const void*>(&k_apply_obs_tile<R, false, NTo>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)));
  char* d = static_cast<char*>(pl->dev);
  for (size_t pi = 0; pi < pl->passes.size(); ++pi) {
    ProfScope ps("apply_obs", double(sizeof(cx<R>)) * double(N) * (pi > 0 ? 3.0 : 2.0), in->stream);
    const dim3 grid(unsigned(std::min<uint64_t>(tiles, exp_grid_max())));
    const auto* pd = reinterpret_cast<const ExpPassDev*>(d);
    const auto* gd = reinterpret_cast<const ExpGroupDev*>(d + pl->off_groups);
    const auto* td = reinterpret_cast<const ExpTermDev*>(d + pl->off_terms);
    if (fixed)
      hipLaunchKernelGGL((k_apply_obs_tile<R, true, NTo>), grid, dim3(NTo), lds, in->stream,
                         static_cast<const R*>(in->ptr), static_cast<R*>(out->ptr), pd, int(pi), gd, td,
                         pi > 0 ? 1 : 0, tiles);
    else
      hipLaunchKernelGGL((k_apply_obs_tile<R, false, NTo>), grid, dim3(NTo), lds, in->stream,
                         static_cast<const R*>(in->ptr), static_cast<R*>(out->ptr), pd, int(pi), gd, td,
                         pi > 0 ? 1 : 0, tiles);
    QSV_HIP_CHECK(hipGetLastError());
  }
  const auto* wt = reinterpret_cast<const ExpTermDev*>(d + pl->off_wide);
  for (size_t wi = 0; wi < pl->wide.size(); ++wi) {
    const bool acc = !pl->passes.empty() || wi > 0;
    ProfScope ps("apply_obs_wide", double(sizeof(cx<R>)) * double(N) * (acc ? 3.0 : 2.0), in->stream);
    const ExpWide& w = pl->wide[wi];
    const unsigned blocks = unsigned(std::min<uint64_t>((N + kExpThreads - 1) / kExpThreads, 8192));
    hipLaunchKernelGGL((k_apply_obs_wide<R>), dim3(blocks), dim3(kExpThreads), 0, in->stream,
                       static_cast<const R*>(in->ptr), static_cast<R*>(out->ptr), w.flip, wt + w.term_begin,
                       w.term_count, N, acc ? 1 : 0);
    QSV_HIP_CHECK(hipGetLastError());
  }
  return QSV_OK;
}

// ------------------------------------------------------------------ no-allocation variant
//
// qsv_expectation_noalloc runs the same passes with every device buffer they
// need -- the observable's pass / group / term tables and the per-workgroup
// FP64 partials -- in one file-scope device array of kNoAllocBytes, so the
// call allocates no device or pinned memory (for callers that cannot: code
// under stream capture, serving loops). Each device holds its own copy of the
// array; its address on a device is taken once (hipGetSymbolAddress, with
// that device current) and only that address is used from the host. Calls on
// one device share the array: calls that overlap on one device race.
constexpr size_t kNoAllocBytes = size_t(1) << 20;
static __device__ __align__(256) char scratch[kNoAllocBytes];

constexpr int kNoAllocMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[kNoAllocMaxDevices] = {};

// Device address of `scratch` on `device` (taken on first use).
int noalloc_scratch(int device, char** out) {
  if (device < 0 || device >= kNoAllocMaxDevices) return fail(QSV_EINVAL, "device index %d out of range", device);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    int cur = -1;
    QSV_HIP_CHECK(hipGetDevice(&cur));
    if (cur != device) QSV_HIP_CHECK(hipSetDevice(device));
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (cur != device) (void)hipSetDevice(cur);
    if (e != hipSuccess || !ptr)
      return fail(QSV_EHIP, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
    g_scratch_ptr[device] = static_cast<char*>(ptr);
  }
  *out = g_scratch_ptr[device];
  return QSV_OK;
}

template <typename R>
int expect_noalloc_t(qsv_state* s, qsv_observable* o, double* out) {
  ExpPlan*& pl = o->exp_plan[s->dtype];
  if (!pl) pl = build_exp_plan(o, s->dtype);  // host tables only
  if (pl->passes.empty() && pl->wide.empty()) {
    *out = 0.0;
    return QSV_OK;
  }
  const uint64_t tiles = dim(s->n - pl->L);
  const uint64_t grid = std::min<uint64_t>(tiles, exp_grid_max());
  // scratch layout: partials[grid + 1] | passes | groups | terms (256-byte aligned)
  auto al = [](size_t x) { return (x + 255) / 256 * 256; };
  const size_t o_pass = al((size_t(grid) + 1) * sizeof(double));
  const size_t o_grp = o_pass + al(pl->passes.size() * sizeof(ExpPassDev));
  const size_t o_term = o_grp + al(pl->groups.size() * sizeof(ExpGroupDev));
  const size_t o_wide = o_term + al(pl->terms.size() * sizeof(ExpTermDev));
  const size_t need = o_wide + al(pl->wide_terms.size() * sizeof(ExpTermDev));
  if (need > kNoAllocBytes)
    return fail(QSV_ERANGE, "observable needs %zu bytes of device scratch; the no-allocation limit is %zu",
                need, kNoAllocBytes);
  char* d = nullptr;
  int rc = noalloc_scratch(s->device, &d);
  if (rc) return rc;
  hipStream_t st = s->stream;
  if (!pl->passes.empty())
    QSV_HIP_CHECK(hipMemcpyAsync(d + o_pass, pl->passes.data(), pl->passes.size() * sizeof(ExpPassDev),
                                 hipMemcpyHostToDevice, st));
  if (!pl->groups.empty())
    QSV_HIP_CHECK(hipMemcpyAsync(d + o_grp, pl->groups.data(), pl->groups.size() * sizeof(ExpGroupDev),
                                 hipMemcpyHostToDevice, st));
  if (!pl->terms.empty())
    QSV_HIP_CHECK(hipMemcpyAsync(d + o_term, pl->terms.data(), pl->terms.size() * sizeof(ExpTermDev),
                                 hipMemcpyHostToDevice, st));
  if (!pl->wide_terms.empty())
    QSV_HIP_CHECK(hipMemcpyAsync(d + o_wide, pl->wide_terms.data(), pl->wide_terms.size() * sizeof(ExpTermDev),
                                 hipMemcpyHostToDevice, st));
  double* part = reinterpret_cast<double*>(d);
  const auto* pd = reinterpret_cast<const ExpPassDev*>(d + o_pass);
  const auto* gd = reinterpret_cast<const ExpGroupDev*>(d + o_grp);
  const auto* td = reinterpret_cast<const ExpTermDev*>(d + o_term);
  const size_t lds = (size_t(1) << pl->L) * sizeof(cx<R>);
  const int mode = pl->L == exp_tile_bits<R>() ? 2 : ((size_t(1) << pl->L) >= size_t(2 * kExpThreadsE) ? 1 : 0);
  const void* kfn = mode == 2   ? reinterpret_cast<const void*>(&k_expect_tile<R, 2>)
                    : mode == 1 ? reinterpret_cast<const void*>(&k_expect_tile<R, 1>)
                                : reinterpret_cast<const void*>(&k_expect_tile<R, 0>);
  QSV_HIP_CHECK(hipFuncSetAttribute(kfn, hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)));
  const R* psi = static_cast<const R*>(s->ptr);
  // the first pass writes every partial (accumulate = 0): nothing left from an
  // earlier call is read
  for (size_t pi = 0; pi < pl->passes.size(); ++pi) {
    if (mode == 2)
      hipLaunchKernelGGL((k_expect_tile<R, 2>), dim3(unsigned(grid)), dim3(kExpThreadsE), lds, st, psi, pd,
                         int(pi), gd, td, part, pi > 0 ? 1 : 0, tiles);
    else if (mode == 1)
      hipLaunchKernelGGL((k_expect_tile<R, 1>), dim3(unsigned(grid)), dim3(kExpThreadsE), lds, st, psi, pd,
                         int(pi), gd, td, part, pi > 0 ? 1 : 0, tiles);
    else
      hipLaunchKernelGGL((k_expect_tile<R, 0>), dim3(unsigned(grid)), dim3(kExpThreadsE), lds, st, psi, pd,
                         int(pi), gd, td, part, pi > 0 ? 1 : 0, tiles);
    QSV_HIP_CHECK(hipGetLastError());
  }
  const auto* wt = reinterpret_cast<const ExpTermDev*>(d + o_wide);
  for (size_t wi = 0; wi < pl->wide.size(); ++wi) {
    const ExpWide& w = pl->wide[wi];
    hipLaunchKernelGGL((k_expect_wide<R>), dim3(unsigned(grid)), dim3(kExpThreadsE), 0, st, psi, w.flip, w.hbit,
                       wt + w.term_begin, w.term_count, dim(s->n - 1), part,
                       pl->passes.empty() && wi == 0 ? 0 : 1);
    QSV_HIP_CHECK(hipGetLastError());
  }
  hipLaunchKernelGGL(k_exp_sum, dim3(1), dim3(kExpThreads), 0, st, part, grid, part + grid);
  QSV_HIP_CHECK(hipGetLastError());
  double v = 0.0;
  QSV_HIP_CHECK(hipMemcpyAsync(&v, part + grid, sizeof(double), hipMemcpyDeviceToHost, st));
  QSV_HIP_CHECK(hipStreamSynchronize(st));
  *out = v;
  return QSV_OK;
}

}  // namespace

int expectation_noalloc(qsv_state* s, const qsv_observable* o, double* out) {
  qsv_observable* mo = const_cast<qsv_observable*>(o);  // host plan cache only
  return s->dtype == QSV_C64 ? expect_noalloc_t<float>(s, mo, out) : expect_noalloc_t<double>(s, mo, out);
}

int expectation_tiled(qsv_state* s, const qsv_observable* o, double* out) {
  qsv_observable* mo = const_cast<qsv_observable*>(o);  // plan cache only
  return s->dtype == QSV_C64 ? expect_tiled_t<float>(s, mo, out) : expect_tiled_t<double>(s, mo, out);
}

// lambda = O psi (out must not alias in; both on in's stream).
int apply_observable_tiled(const qsv_state* in, const qsv_observable* o, qsv_state* out) {
  qsv_observable* mo = const_cast<qsv_observable*>(o);  // plan cache only
  return in->dtype == QSV_C64 ? apply_obs_tiled_t<float>(in, mo, out) : apply_obs_tiled_t<double>(in, mo, out);
}

int expectation_passes(const qsv_observable* o, qsv_dtype dt) {
  qsv_observable* mo = const_cast<qsv_observable*>(o);
  ExpPlan*& pl = mo->exp_plan[dt];
  if (!pl) pl = build_exp_plan(mo, dt);
  return int(pl->passes.size() + pl->wide.size());
}

}  // namespace qsv
