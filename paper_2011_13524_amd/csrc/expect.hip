// Tiled evaluation of <psi|O|psi> for a Pauli-string observable (section 4.5).
//
// A term with flip mask F pairs amplitude x with x ^ F, so it can be evaluated
// from any tile of the state whose local qubits include every qubit of F: both
// members of each pair are then in the same tile. The host groups the
// observable's flip masks into passes: a pass fixes L local qubits (always the
// low b ones, for contiguous HBM runs) and greedily packs the flip masks that
// need the fewest extra local qubits until the set is full. Each pass reads the
// state once into LDS, tile by tile, and evaluates every group of the pass on
// it; a tile's contribution accumulates in FP64 into one partial per tile
// (passes run in order on one stream, so each partial has a single writer in a
// fixed order), and one final fixed-order reduction gives the value. Compared
// with one pass per flip mask, HBM traffic drops by the number of masks per
// pass. Z/Y signs on non-local qubits are constants per tile.
#include <algorithm>
#include <cstdlib>

#include "dev_common.h"
#include "observable.h"
#include "prof.h"
#include "qsv_internal.h"

namespace qsv {

constexpr int kExpThreads = 512;
constexpr int kExpMaxHigh = 16;
constexpr int kExpMaxGlobal = 40;

struct ExpPassDev {
  int L, b, nh, ng;
  int grp_begin, grp_count;
  int hq[kExpMaxHigh];
  int gpos[kExpMaxGlobal];
};

struct ExpGroupDev {
  uint32_t lf;  // flip mask in the tile's local index space
  int hbit;     // a set bit of lf (pairs are enumerated with it clear)
  int term_begin, term_count;
};

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
constexpr int kExpLdsTerms = 256;

struct ExpPlan {
  int n = 0, L = 0, b = 0;
  std::vector<ExpPassDev> passes;
  std::vector<ExpGroupDev> groups;
  std::vector<ExpTermDev> terms;
  void* dev = nullptr;  // passes | groups | terms
  size_t off_groups = 0, off_terms = 0;
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

__device__ __forceinline__ uint32_t ins0(uint32_t i, int hb) {
  return ((i >> hb) << (hb + 1)) | (i & ((1u << hb) - 1));
}

// One tile of one pass: the tile is read into LDS once, then every flip-mask
// group of the pass is evaluated on it. Pair products conj(psi_y) psi_x and
// the thread's few partial sums use the amplitude precision; every sum over
// threads, tiles and passes is FP64.
template <typename R>
__global__ void __launch_bounds__(kExpThreads)
    k_expect_tile(const R* __restrict__ psi, const ExpPassDev* __restrict__ passes, int pass_idx,
                  const ExpGroupDev* __restrict__ groups, const ExpTermDev* __restrict__ terms,
                  double* __restrict__ partial, int accumulate) {
  extern __shared__ __align__(16) char smem[];
  __shared__ double red[kExpThreads / 64];
  __shared__ ExpTermLds et[kExpLdsTerms];
  cx<R>* t = reinterpret_cast<cx<R>*>(smem);
  const ExpPassDev& P = passes[pass_idx];
  const int L = P.L;
  const uint64_t g = blockIdx.x;
  uint64_t base = 0;
  for (int j = 0; j < P.ng; ++j) base |= ((g >> j) & 1) << P.gpos[j];
  constexpr int V = sizeof(R) == 4 ? 2 : 1;
  const uint32_t TS = 1u << L;
  const uint32_t tid = threadIdx.x;
  {
    const uint64_t xt = base | exp_place(P, tid * V);
    for (uint32_t e0 = 0; e0 < TS / V; e0 += kExpThreads) {
      if (e0 + tid >= TS / V) break;
      const uint64_t x = xt | exp_place(P, e0 * V);
      AmpIO<R, V>::load(psi, x, &t[(e0 + tid) * V]);
    }
  }
  double acc = 0.0;
  for (int gi = 0; gi < P.grp_count; ++gi) {
    const ExpGroupDev G = groups[P.grp_begin + gi];
    const int nt = G.term_count;
    if (gi == 0) __syncthreads();  // tile loaded
    if (nt > 1) {
      // stage the group's terms with their sign on non-local qubits folded in
      // (a constant for this tile)
      __syncthreads();
      const int ns = min(nt, kExpLdsTerms);
      for (int k = tid; k < ns; k += blockDim.x) {
        const ExpTermDev T = terms[G.term_begin + k];
        const bool gneg = __popcll(base & T.zg) & 1;
        et[k] = {gneg ? -T.re : T.re, gneg ? -T.im : T.im, T.zl};
      }
      __syncthreads();
    }
    if (G.lf == 0 && nt == 1) {
      // sum of +-|psi_x|^2: thread part of the sign once, uniform part per step
      const ExpTermDev T = terms[G.term_begin];
      const double re = (__popcll(base & T.zg) & 1) ? -T.re : T.re;
      const uint32_t pt = __popc(tid & T.zl) & 1;
      R sum = R(0);
      for (uint32_t j0 = 0; j0 < TS; j0 += kExpThreads) {
        if (j0 + tid >= TS) break;
        const cx<R> a = t[j0 + tid];
        const R p = a.re * a.re + a.im * a.im;
        sum += (pt ^ (__popc(j0 & T.zl) & 1)) ? -p : p;
      }
      acc += re * double(sum);
    } else if (G.lf == 0) {
      for (uint32_t j = tid; j < TS; j += blockDim.x) {
        const cx<R> a = t[j];
        double c = 0.0;
        for (int k = 0; k < nt; ++k) {
          double re;
          uint32_t zl;
          if (k < kExpLdsTerms) {
            re = et[k].re;
            zl = et[k].zl;
          } else {
            const ExpTermDev T = terms[G.term_begin + k];
            re = (__popcll(base & T.zg) & 1) ? -T.re : T.re;
            zl = T.zl;
          }
          c += (__popc(j & zl) & 1) ? -re : re;
        }
        acc += double(a.re * a.re + a.im * a.im) * c;
      }
    } else {
      const int hb = G.hbit;
      const uint32_t lf = G.lf;
      // pairs (x, x ^ lf) with bit hb of x clear: x = ins0(i) for i < TS/2,
      // i = tid + step; ins0 places bits, so x = ins0(tid) | ins0(step)
      const uint32_t xt = ins0(tid, hb);
      if (nt == 1) {
        // one term (the common case for random strings): c(x) = +-(re + i im)
        const ExpTermDev T = terms[G.term_begin];
        const bool gneg = __popcll(base & T.zg) & 1;
        const double re = gneg ? -T.re : T.re, im = gneg ? -T.im : T.im;
        const uint32_t zl = T.zl;
        const uint32_t pt = __popc(xt & zl) & 1;
        R sr = R(0), si = R(0);
        for (uint32_t i0 = 0; i0 < TS / 2; i0 += kExpThreads) {
          if (i0 + tid >= TS / 2) break;
          const uint32_t xs = ins0(i0, hb);
          const uint32_t x = xt | xs;
          const cx<R> a = t[x], bb = t[x ^ lf];
          // w = conj(psi[y]) psi[x]
          const R wr = bb.re * a.re + bb.im * a.im;
          const R wi = bb.re * a.im - bb.im * a.re;
          const bool neg = pt ^ (__popc(xs & zl) & 1);
          sr += neg ? -wr : wr;
          si += neg ? -wi : wi;
        }
        acc += 2.0 * (double(sr) * re - double(si) * im);
      } else {
        for (uint32_t i = tid; i < TS / 2; i += blockDim.x) {
          const uint32_t x = ins0(i, hb);
          const cx<R> a = t[x], bb = t[x ^ lf];
          const double wr = double(bb.re * a.re + bb.im * a.im);
          const double wi = double(bb.re * a.im - bb.im * a.re);
          double cr = 0.0, ci = 0.0;
          for (int k = 0; k < nt; ++k) {
            double re, im;
            uint32_t zl;
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
  if ((tid & 63) == 0) red[tid >> 6] = acc;
  __syncthreads();
  if (tid == 0) {
    double r = 0.0;
    for (int w = 0; w < kExpThreads / 64; ++w) r += red[w];
    partial[blockIdx.x] = accumulate ? partial[blockIdx.x] + r : r;
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

// Pack flip masks into passes (greedy: repeatedly add the mask needing the
// fewest extra local qubits while the local set stays within L).
ExpPlan* build_exp_plan(const qsv_observable* o, qsv_dtype dt) {
  std::vector<Group> groups;
  std::vector<GTerm> terms;
  build_groups(o, groups, terms);
  ExpPlan* p = new ExpPlan();
  const int n = o->n;
  p->n = n;
  // tile: 2^L amplitudes, 32 KiB (measured on MI355X at 30 qubits: 32 KiB
  // tiles under 512-thread workgroups beat 64 KiB and 16 KiB ones);
  // QSV_EXPECT_TILE overrides L, for tuning
  int Ldef = dt == QSV_C64 ? 12 : 11;
  if (const char* e = std::getenv("QSV_EXPECT_TILE")) Ldef = std::max(6, std::min(Ldef, std::atoi(e)));
  p->L = std::min(n, Ldef);
  p->b = std::min(p->L, dt == QSV_C64 ? 6 : 5);
  const int L = p->L, b = p->b;
  const uint64_t low = (uint64_t(1) << b) - 1;
  std::vector<int> rem(groups.size());
  for (size_t i = 0; i < groups.size(); ++i) rem[i] = int(i);
  while (!rem.empty()) {
    uint64_t local = low;
    std::vector<int> chosen;
    while (true) {
      int best = -1, bc = 1 << 30;
      for (size_t r = 0; r < rem.size(); ++r) {
        const uint64_t f = groups[rem[r]].flip;
        if (popc64(local | f) > L) continue;
        const int need = popc64(f & ~local);
        if (need < bc) {
          bc = need;
          best = int(r);
        }
      }
      if (best < 0) break;
      local |= groups[rem[best]].flip;
      chosen.push_back(rem[best]);
      rem.erase(rem.begin() + best);
    }
    for (int q = 0; q < n && popc64(local) < L; ++q) local |= uint64_t(1) << q;
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
    d.grp_count = int(chosen.size());
    for (int gi : chosen) {
      const Group& G = groups[gi];
      ExpGroupDev gd{};
      uint32_t lf = 0;
      for (int q = 0; q < n; ++q)
        if (G.flip >> q & 1) lf |= 1u << lpos[q];
      gd.lf = lf;
      gd.hbit = lf ? 31 - __builtin_clz(lf) : 0;
      gd.term_begin = int(p->terms.size());
      gd.term_count = G.count;
      for (int k = G.begin; k < G.begin + G.count; ++k) {
        ExpTermDev td{};
        td.re = terms[k].re;
        td.im = terms[k].im;
        for (int q = 0; q < n; ++q) {
          if (!(terms[k].z >> q & 1)) continue;
          if (lpos[q] >= 0) td.zl |= 1u << lpos[q];
          else td.zg |= uint64_t(1) << q;
        }
        p->terms.push_back(td);
      }
      p->groups.push_back(gd);
    }
    p->passes.push_back(d);
  }
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
  const size_t total = p->off_terms + std::max<size_t>(1, p->terms.size()) * sizeof(ExpTermDev);
  if (hipMalloc(&p->dev, total) != hipSuccess) return fail(QSV_ENOMEM, "observable plan allocation failed");
  char* d = static_cast<char*>(p->dev);
  QSV_HIP_CHECK(hipMemcpy(d, p->passes.data(), a, hipMemcpyHostToDevice));
  if (bsz) QSV_HIP_CHECK(hipMemcpy(d + p->off_groups, p->groups.data(), bsz, hipMemcpyHostToDevice));
  if (!p->terms.empty())
    QSV_HIP_CHECK(hipMemcpy(d + p->off_terms, p->terms.data(), p->terms.size() * sizeof(ExpTermDev),
                            hipMemcpyHostToDevice));
  p->device = device;
  return QSV_OK;
}

template <typename R>
int expect_tiled_t(qsv_state* s, qsv_observable* o, double* out) {
  ExpPlan*& pl = o->exp_plan[s->dtype];
  if (!pl) pl = build_exp_plan(o, s->dtype);
  if (pl->passes.empty()) {
    *out = 0.0;
    return QSV_OK;
  }
  int rc = upload_exp_plan(pl, s->device);
  if (rc) return rc;
  const uint64_t tiles = dim(s->n - pl->L);
  if ((rc = ensure_reduce_scratch(s, size_t(tiles) + 1))) return rc;
  const size_t lds = (size_t(1) << pl->L) * sizeof(cx<R>);
  QSV_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_expect_tile<R>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)));
  char* d = static_cast<char*>(pl->dev);
  for (size_t pi = 0; pi < pl->passes.size(); ++pi) {
    ProfScope ps("expect", double(sizeof(cx<R>)) * double(dim(s->n)), s->stream);
    hipLaunchKernelGGL((k_expect_tile<R>), dim3(unsigned(tiles)), dim3(kExpThreads), lds, s->stream,
                       static_cast<const R*>(s->ptr), reinterpret_cast<const ExpPassDev*>(d), int(pi),
                       reinterpret_cast<const ExpGroupDev*>(d + pl->off_groups),
                       reinterpret_cast<const ExpTermDev*>(d + pl->off_terms), s->red, pi > 0 ? 1 : 0);
    QSV_HIP_CHECK(hipGetLastError());
  }
  hipLaunchKernelGGL(k_exp_sum, dim3(1), dim3(kExpThreads), 0, s->stream, s->red, tiles, s->red + tiles);
  QSV_HIP_CHECK(hipGetLastError());
  QSV_HIP_CHECK(hipMemcpyAsync(s->red_host, s->red + tiles, sizeof(double), hipMemcpyDeviceToHost,
                               s->stream));
  QSV_HIP_CHECK(hipStreamSynchronize(s->stream));
  *out = s->red_host[0];
  return QSV_OK;
}

}  // namespace

int expectation_tiled(qsv_state* s, const qsv_observable* o, double* out) {
  qsv_observable* mo = const_cast<qsv_observable*>(o);  // plan cache only
  return s->dtype == QSV_C64 ? expect_tiled_t<float>(s, mo, out) : expect_tiled_t<double>(s, mo, out);
}

int expectation_passes(const qsv_observable* o, qsv_dtype dt) {
  qsv_observable* mo = const_cast<qsv_observable*>(o);
  ExpPlan*& pl = mo->exp_plan[dt];
  if (!pl) pl = build_exp_plan(mo, dt);
  return int(pl->passes.size());
}

}  // namespace qsv
