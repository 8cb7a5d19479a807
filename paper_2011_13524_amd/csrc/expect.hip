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

#include "dev_common.h"
#include "observable.h"
#include "prof.h"
#include "qsv_internal.h"

namespace qsv {

constexpr int kExpThreads = 256;
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

template <typename R>
__global__ void __launch_bounds__(kExpThreads)
    k_expect_tile(const R* __restrict__ psi, const ExpPassDev* __restrict__ passes, int pass_idx,
                  const ExpGroupDev* __restrict__ groups, const ExpTermDev* __restrict__ terms,
                  double* __restrict__ partial, int accumulate) {
  extern __shared__ __align__(16) char smem[];
  __shared__ double red[kExpThreads / 64];
  cx<R>* t = reinterpret_cast<cx<R>*>(smem);
  const ExpPassDev& P = passes[pass_idx];
  const int L = P.L, b = P.b, nh = P.nh;
  const uint64_t g = blockIdx.x;
  uint64_t base = 0;
  for (int j = 0; j < P.ng; ++j) base |= ((g >> j) & 1) << P.gpos[j];
  constexpr int V = sizeof(R) == 4 ? 2 : 1;
  const int TS = 1 << L;
  const uint32_t lowmask = (1u << b) - 1;
  for (int e = threadIdx.x; e < TS / V; e += blockDim.x) {
    const uint32_t j = uint32_t(e) * V;
    const uint32_t h = j >> b;
    uint64_t x = base + (j & lowmask);
    for (int i = 0; i < nh; ++i) x |= uint64_t((h >> i) & 1) << P.hq[i];
    AmpIO<R, V>::load(psi, x, &t[j]);
  }
  __syncthreads();
  double acc = 0.0;
  for (int gi = 0; gi < P.grp_count; ++gi) {
    const ExpGroupDev G = groups[P.grp_begin + gi];
    if (G.lf == 0) {
      for (int j = threadIdx.x; j < TS; j += blockDim.x) {
        const cx<R> a = t[j];
        double c = 0.0;
        for (int k = G.term_begin; k < G.term_begin + G.term_count; ++k) {
          const ExpTermDev T = terms[k];
          const int s = (__popc(uint32_t(j) & T.zl) + __popcll(base & T.zg)) & 1;
          c += s ? -T.re : T.re;
        }
        acc += (double(a.re) * a.re + double(a.im) * a.im) * c;
      }
    } else {
      const int hb = G.hbit;
      for (int i = threadIdx.x; i < TS / 2; i += blockDim.x) {
        const uint32_t x = ((uint32_t(i) >> hb) << (hb + 1)) | (uint32_t(i) & ((1u << hb) - 1));
        const uint32_t y = x ^ G.lf;
        const cx<R> a = t[x], bb = t[y];
        // w = conj(psi[y]) psi[x]
        const double wr = double(bb.re) * a.re + double(bb.im) * a.im;
        const double wi = double(bb.re) * a.im - double(bb.im) * a.re;
        double cr = 0.0, ci = 0.0;
        for (int k = G.term_begin; k < G.term_begin + G.term_count; ++k) {
          const ExpTermDev T = terms[k];
          const int s = (__popc(x & T.zl) + __popcll(base & T.zg)) & 1;
          cr += s ? -T.re : T.re;
          ci += s ? -T.im : T.im;
        }
        acc += 2.0 * (wr * cr - wi * ci);
      }
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
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
  p->L = std::min(n, dt == QSV_C64 ? 13 : 12);
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
