// Circuit fusion (section 5.4) and tile passes.
//
// Planning, on the host, in three stages:
//  1. Structure: every gate is reduced to its controlled form (section 4.3.2)
//     and marked diagonal or not.
//  2. Merge (section 5.4, merge of two successive gates): a gate joins the
//     block it depends on when that block is the only earlier block sharing
//     its qubits -- so it commutes with every block created in between -- and
//     the merged block stays within max_k qubits. Merges never raise the
//     arithmetic per amplitude: a dense k-qubit block costs 2^k complex
//     multiply-adds per amplitude, a diagonal block one multiply and an
//     exchange (X or controlled X) none. So diagonal gates join diagonal
//     blocks (the product stays diagonal); diagonal and exchange gates join a
//     dense block only on a subset of its qubits, and a dense gate absorbs a
//     diagonal or exchange block only on a subset of its own qubits. Block
//     matrices are products K_later K_earlier on the ascending union of
//     qubits.
//     Heavy mode (section 5.4, the heavy optimization): every gate carries,
//     per qubit it touches, the set of Paulis it commutes with there (a CNOT
//     commutes with Z on its control and X on its target; a diagonal gate
//     with Z on every qubit; RX/RY/RZ with X/Y/Z). A gate may then join an
//     earlier block that is not its immediate predecessor: walking back from
//     the newest block, it moves past every block with which it shares, on
//     each common qubit, a commuting Pauli (such a block and the gate are
//     then both block-diagonal in that Pauli's eigenbasis on every shared
//     qubit, so they commute), and joins the first block sharing a qubit
//     where the merge rules above allow it. On circuits whose gates all
//     commute (diagonal layers) this compresses the depth to a constant.
//  3. Passes: a pass fixes a set of L local qubits (always including the low b
//     qubits, so that each run of 2^b amplitudes is contiguous in HBM) and
//     greedily takes, in order, every block whose non-diagonal targets are
//     local or can still be made local, skipping blocks that share a qubit
//     with one already deferred. Diagonal blocks and controls may sit on any
//     qubit: for one tile their non-local bits are constants.
//
// Execution: one kernel launch per pass; workgroup g owns tile g, the 2^L
// amplitudes whose non-local bits spell g. It streams the tile from HBM into
// LDS (non-temporal 16-byte vectors), applies the pass's blocks in order with a
// barrier between them, and streams the tile back. Each pass therefore reads
// and writes the state once however many gates it applies.
#include <algorithm>
#include <cmath>
#include <cstdlib>

#include "dev_common.h"
#include "plan.h"
#include "prof.h"
#include "tile_reg.h"

namespace qsv {

// LDS-resident tile pass: the whole tile in LDS, every block an LDS sweep.
// Used when the tile does not match the register-resident shape (small
// states, non-default tile sizes).
template <typename R, int KMAX>
__global__ void __launch_bounds__(256)
    k_tile(R* __restrict__ psi, const TilePassDev* __restrict__ passes, int pass_idx,
           const TileOpDev* __restrict__ ops, const cx<R>* __restrict__ pool) {
  extern __shared__ __align__(16) char smem[];
  cx<R>* t = reinterpret_cast<cx<R>*>(smem);
  const TilePassDev& P = passes[pass_idx];
  const int L = P.L, b = P.b, nh = P.nh, ng = P.ng;
  const uint64_t g = blockIdx.x;
  uint64_t base = 0;
  for (int j = 0; j < ng; ++j) base |= ((g >> j) & 1) << P.gpos[j];
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
  for (int o = 0; o < P.op_count; ++o) {
    const TileOpDev& op = ops[P.op_begin + o];
    if ((base & op.gcm) != op.gcv) continue;  // non-local controls not met: skip for this tile
    lds_op<R, KMAX>(t, op, pool, L, base, NoSwz());
    __syncthreads();
  }
  for (int e = threadIdx.x; e < TS / V; e += blockDim.x) {
    const uint32_t j = uint32_t(e) * V;
    const uint32_t h = j >> b;
    uint64_t x = base + (j & lowmask);
    for (int i = 0; i < nh; ++i) x |= uint64_t((h >> i) & 1) << P.hq[i];
    AmpIO<R, V>::store(psi, x, &t[j]);
  }
}

// ------------------------------------------------------------------ host: matrices

namespace {

uint64_t qmask(const std::vector<int>& qs) {
  uint64_t m = 0;
  for (int q : qs) m |= uint64_t(1) << q;
  return m;
}

std::vector<int> mask_list(uint64_t m) {
  std::vector<int> v;
  for (int q = 0; q < 64; ++q)
    if (m >> q & 1) v.push_back(q);
  return v;
}

// Structure of one gate: targets/controls after control extraction and
// whether the remaining target matrix is diagonal (value-independent for
// rotations: Z rotations are diagonal for every angle).
struct GateInfo {
  std::vector<int> targets, controls, ctrl_vals;
  std::vector<cd> mat;  // extracted matrix (MATRIX gates only)
  bool diagonal = false;
  bool exchange = false;  // extracted matrix is Pauli X on one target
  uint64_t qubits = 0;
};

GateInfo analyse(const Gate& g) {
  GateInfo gi;
  if (g.kind == Gate::ROTATION) {
    gi.targets = g.targets;
    gi.diagonal = (g.pauli == 3);
  } else if (g.kind == Gate::PAULI) {
    gi.targets = g.targets;
    gi.diagonal = std::all_of(g.paulis.begin(), g.paulis.end(), [](int p) { return p == 3; });
  } else {
    std::vector<cd> m = g.mat;
    std::vector<int> tq = g.targets;
    uint64_t cm = 0, cv = 0;
    for (size_t j = 0; j < g.controls.size(); ++j) {
      cm |= uint64_t(1) << g.controls[j];
      if (g.ctrl_vals[j]) cv |= uint64_t(1) << g.controls[j];
    }
    extract_controls(m, tq, cm, cv);
    gi.targets = tq;
    for (int q : mask_list(cm)) {
      gi.controls.push_back(q);
      gi.ctrl_vals.push_back(int(cv >> q & 1));
    }
    const int D = 1 << tq.size();
    bool dg = true;
    for (int r = 0; r < D && dg; ++r)
      for (int c = 0; c < D && dg; ++c)
        if (r != c && !(m[r * D + c].re == 0.0 && m[r * D + c].im == 0.0)) dg = false;
    gi.diagonal = dg;
    gi.exchange = tq.size() == 1 && m[0].re == 0 && m[0].im == 0 && m[1].re == 1 && m[1].im == 0 &&
                  m[2].re == 1 && m[2].im == 0 && m[3].re == 0 && m[3].im == 0;
    gi.mat = m;
  }
  gi.qubits = qmask(gi.targets) | qmask(gi.controls);
  return gi;
}

// Target matrix of a gate in its extracted form, for the given parameters.
void extracted_matrix(const Gate& g, const GateInfo& gi, const double* theta, std::vector<cd>& m) {
  if (g.kind == Gate::ROTATION || g.kind == Gate::PAULI) {
    gate_matrix(g, theta, m);
  } else {
    m = gi.mat;
  }
}

// Full matrix of a gate (targets + controls) embedded in the index space of
// `qs` (bit j <-> qs[j]); result is 2^|qs| square, row-major.
void embed(const std::vector<cd>& gm, const GateInfo& gi, const std::vector<int>& qs,
           std::vector<cd>& out) {
  const int k = int(qs.size());
  const int D = 1 << k;
  out.assign(size_t(D) * D, cd{0, 0});
  std::vector<int> tpos(gi.targets.size()), cpos(gi.controls.size());
  for (size_t j = 0; j < gi.targets.size(); ++j)
    tpos[j] = int(std::find(qs.begin(), qs.end(), gi.targets[j]) - qs.begin());
  for (size_t j = 0; j < gi.controls.size(); ++j)
    cpos[j] = int(std::find(qs.begin(), qs.end(), gi.controls[j]) - qs.begin());
  const int kt = int(tpos.size());
  const int Dt = 1 << kt;
  for (int c = 0; c < D; ++c) {
    bool on = true;
    for (size_t j = 0; j < cpos.size(); ++j)
      if (((c >> cpos[j]) & 1) != gi.ctrl_vals[j]) on = false;
    if (!on) {
      out[size_t(c) * D + c] = {1, 0};
      continue;
    }
    int cc = 0, rest = c;
    for (int j = 0; j < kt; ++j) {
      cc |= ((c >> tpos[j]) & 1) << j;
      rest &= ~(1 << tpos[j]);
    }
    for (int rr = 0; rr < Dt; ++rr) {
      int r = rest;
      for (int j = 0; j < kt; ++j) r |= ((rr >> j) & 1) << tpos[j];
      out[size_t(r) * D + c] = gm[size_t(rr) * Dt + cc];
    }
  }
}

void matmul(const std::vector<cd>& a, const std::vector<cd>& b, int D, std::vector<cd>& out) {
  out.assign(size_t(D) * D, cd{0, 0});
  for (int r = 0; r < D; ++r)
    for (int k = 0; k < D; ++k) {
      const cd x = a[size_t(r) * D + k];
      if (x.re == 0.0 && x.im == 0.0) continue;
      for (int c = 0; c < D; ++c) out[size_t(r) * D + c] = cadd(out[size_t(r) * D + c], cmul(x, b[size_t(k) * D + c]));
    }
}

// Paulis (bit 0: X, bit 1: Y, bit 2: Z) commuting with the gate on each of
// its qubits; 7 on qubits it does not touch. Rotations exp(i t P / 2) commute
// with P on their target(s) for every angle; fixed matrices are tested on
// their full matrix over targets and controls.
std::vector<uint8_t> commute_masks(const Gate& g, const GateInfo& gi, int n) {
  std::vector<uint8_t> m(size_t(n), 7);
  if (g.kind == Gate::ROTATION) {
    m[size_t(g.targets[0])] = uint8_t(1u << (g.pauli - 1));
    return m;
  }
  if (g.kind == Gate::PAULI) {
    for (size_t j = 0; j < g.targets.size(); ++j) m[size_t(g.targets[j])] = uint8_t(1u << (g.paulis[j] - 1));
    return m;
  }
  const std::vector<int> qs = mask_list(gi.qubits);
  std::vector<cd> M;
  embed(gi.mat, gi, qs, M);
  const int D = 1 << qs.size();
  double big = 0.0;
  for (const cd& z : M) big = std::max(big, std::fabs(z.re) + std::fabs(z.im));
  const double tol = 1e-12 * std::max(big, 1.0);
  auto close = [tol](cd a, cd b) { return std::fabs(a.re - b.re) + std::fabs(a.im - b.im) <= tol; };
  for (size_t j = 0; j < qs.size(); ++j) {
    const int bit = 1 << j;
    bool cx = true, cy = true, cz = true;
    for (int r = 0; r < D; ++r)
      for (int c = 0; c < D; ++c) {
        const cd v = M[size_t(r) * D + c];
        // Z_j M = M Z_j: no element between rows and columns whose bit j differs
        if (((r ^ c) & bit) && !close(v, cd{0, 0})) cz = false;
        // X_j M = M X_j: M[r ^ bit][c] = M[r][c ^ bit]
        if (!close(M[size_t(r ^ bit) * D + c], M[size_t(r) * D + (c ^ bit)])) cx = false;
        // Y_j M = M Y_j with Y|0> = i|1>, Y|1> = -i|0>:
        //   (Y M)[r][c] = (bit of r ? i : -i) M[r ^ bit][c]
        //   (M Y)[r][c] = (bit of c ? -i : i) M[r][c ^ bit]
        const cd a = M[size_t(r ^ bit) * D + c], b = M[size_t(r) * D + (c ^ bit)];
        const cd ya = (r & bit) ? cd{-a.im, a.re} : cd{a.im, -a.re};
        const cd yb = (c & bit) ? cd{b.im, -b.re} : cd{-b.im, b.re};
        if (!close(ya, yb)) cy = false;
      }
    m[size_t(qs[j])] = uint8_t((cx ? 1 : 0) | (cy ? 2 : 0) | (cz ? 4 : 0));
  }
  return m;
}

}  // namespace

// ------------------------------------------------------------------ host: planning

static int build_plan(qsv_plan* p) {
  const qsv_circuit& C = p->circ_copy;
  const int n = C.n;
  std::vector<GateInfo> info(C.gates.size());
  for (size_t i = 0; i < C.gates.size(); ++i) info[i] = analyse(C.gates[i]);

  // stage 2: merge
  std::vector<Block>& blocks = p->blocks;
  blocks.clear();
  std::vector<uint64_t> bq;  // qubit masks of blocks
  std::vector<char> bx;      // block is a single exchange gate
  std::vector<int> last(n, -1);
  std::vector<std::vector<uint8_t>> bcm;  // heavy: per block, commuting Paulis per qubit
  // merge rule for gate I joining block j (arithmetic per amplitude never rises)
  auto merge_ok = [&](int j, const GateInfo& I) {
    const Block& B = blocks[size_t(j)];
    const uint64_t uni = bq[size_t(j)] | I.qubits;
    const int ku = __builtin_popcountll(uni);
    const bool cheap_b = B.diagonal || bx[size_t(j)], cheap_i = I.diagonal || I.exchange;
    if (B.diagonal && I.diagonal) return ku <= 2;  // diagonal blocks stay register-friendly
    if (cheap_b && cheap_i) return false;          // the product would be dense: costlier
    if (cheap_i) return (I.qubits & ~bq[size_t(j)]) == 0;
    if (cheap_b) return (bq[size_t(j)] & ~I.qubits) == 0 && ku <= std::max(p->max_k, 1);
    return ku <= p->max_k;
  };
  for (size_t gi = 0; gi < C.gates.size(); ++gi) {
    const GateInfo& I = info[gi];
    std::vector<uint8_t> gcm;
    int target = -1;
    if (p->heavy) {
      gcm = commute_masks(C.gates[gi], I, n);
      for (int j = int(blocks.size()) - 1; j >= 0; --j) {
        const uint64_t shared = bq[size_t(j)] & I.qubits;
        if (!shared) continue;
        if (merge_ok(j, I)) {
          target = j;
          break;
        }
        bool passes = true;  // the gate commutes with block j: move it further back
        for (int q : mask_list(shared))
          if (!(bcm[size_t(j)][size_t(q)] & gcm[size_t(q)])) passes = false;
        if (!passes) break;
      }
    } else {
      int cand = -2;
      for (int q : mask_list(I.qubits)) {
        if (last[q] < 0) continue;
        if (cand == -2) cand = last[q];
        else if (cand != last[q]) cand = -1;
      }
      if (cand >= 0 && merge_ok(cand, I)) target = cand;
    }
    if (target >= 0) {
      Block& B = blocks[size_t(target)];
      B.gates.push_back(int(gi));
      bq[size_t(target)] |= I.qubits;
      bx[size_t(target)] = 0;
      B.diagonal = B.diagonal && I.diagonal;
      for (int q : mask_list(I.qubits)) {
        last[q] = std::max(last[q], target);
        if (p->heavy) bcm[size_t(target)][size_t(q)] &= gcm[size_t(q)];
      }
    } else {
      Block B;
      B.gates = {int(gi)};
      B.diagonal = I.diagonal;
      blocks.push_back(B);
      bq.push_back(I.qubits);
      bx.push_back(I.exchange ? 1 : 0);
      if (p->heavy) bcm.push_back(gcm);
      for (int q : mask_list(I.qubits)) last[q] = int(blocks.size()) - 1;
    }
  }
  for (size_t i = 0; i < blocks.size(); ++i) {
    Block& B = blocks[i];
    B.qubits = mask_list(bq[i]);
    if (B.gates.size() == 1) {
      const GateInfo& I = info[B.gates[0]];
      B.targets = I.targets;
      B.controls = I.controls;
      B.ctrl_vals = I.ctrl_vals;
      B.xswap = I.exchange;
    } else {
      B.targets = B.qubits;
      B.controls.clear();
      B.ctrl_vals.clear();
    }
    if (B.targets.size() > size_t(5)) return fail(QSV_EINVAL, "block wider than 5 qubits");
  }

  // stage 3: passes
  const int L = p->L, b = p->b;
  p->passes.clear();
  std::vector<int> rem(blocks.size());
  for (size_t i = 0; i < blocks.size(); ++i) rem[i] = int(i);
  const uint64_t low = (b >= 64) ? ~0ull : ((uint64_t(1) << b) - 1);
  while (!rem.empty()) {
    qsv_plan::Pass P;
    uint64_t local = low;
    // qubits of the blocks deferred so far, and of the non-diagonal ones: a
    // block may run ahead of deferred blocks it commutes with -- those on
    // other qubits, and for a diagonal block also diagonal ones on its qubits
    uint64_t blocked = 0, blocked_dense = 0;
    std::vector<int> deferred;
    auto defer = [&](int bi) {
      deferred.push_back(bi);
      blocked |= bq[bi];
      if (!blocks[bi].diagonal) blocked_dense |= bq[bi];
    };
    for (int bi : rem) {
      const Block& B = blocks[bi];
      const uint64_t all = bq[bi];
      if (all & (B.diagonal ? blocked_dense : blocked)) {
        defer(bi);
        continue;
      }
      const uint64_t dense = B.diagonal ? 0 : qmask(B.targets);
      const uint64_t need = dense & ~local;
      if (__builtin_popcountll(local | need) <= L) {
        local |= need;
        P.blocks.push_back(bi);
      } else {
        defer(bi);
      }
    }
    if (P.blocks.empty()) return fail(QSV_EINVAL, "planner made no progress (tile too small)");
    // fill the local set up to L qubits with the lowest unused qubits
    for (int q = 0; q < n && __builtin_popcountll(local) < L; ++q) local |= uint64_t(1) << q;
    P.local = mask_list(local);
    p->passes.push_back(P);
    rem.swap(deferred);
  }
  return QSV_OK;
}

// Split a pass's ops into register-resident segments.
//
// Scheduling: ops that commute may run in any order. Two ops commute when
// every local qubit they share is acted on diagonally by both (a control, or a
// diagonal target); otherwise the later op depends on the earlier one. A
// segment fixes reg_bits register bits and takes, by list scheduling over
// this dependency order, every ready op whose register needs (the targets of
// one- and two-qubit dense ops; diagonal and LDS ops need none) still fit;
// when no ready op fits, the next segment starts.
//
// Folding: an X gate, or an X with one local control, permutes the tile's
// local indices by an affine map over GF(2) (x_t ^= x_c, or ^= 1). Such an op
// moves no data: it is folded into the next re-map through LDS, whose write
// addresses go through the composed map. Ops that depend on a folded op wait
// for the next segment; ops that commute with it are unaffected.
//
// Layouts: the first segment is the layout the tile is read in and the last
// the one it is written in, so both put the low local bits that form
// contiguous 128-byte runs on lanes 0..2 (and, for complex64, local bit 0 in
// registers: amplitude pairs are 16-byte vectors). A segment's wave bits
// (thread-index bits above the 64 lanes) are chosen so that consecutive
// segments share them where possible: a re-map between two such layouts
// moves data only within each wavefront and needs no workgroup barrier.
void pass_runs(TilePassDev& d) {
  d.nrun = 0;
  for (int j = 0; j < d.ng; ++j) {
    if (j > 0 && d.gpos[j] == d.gpos[j - 1] + 1) {
      ++d.rlen[d.nrun - 1];
      continue;
    }
    d.rsrc[d.nrun] = j;
    d.rdst[d.nrun] = d.gpos[j];
    d.rlen[d.nrun] = 1;
    ++d.nrun;
  }
}

bool tile_mfma_default() {
  const char* e = std::getenv("QSV_TILE_MFMA");
  return !(e && e[0] == '0');
}

int build_reg_segments(const SegCfg& cfg, const std::vector<TileOpDev>& ho, TilePassDev& d,
                       std::vector<RegSegDev>& out_segs, std::vector<RegOpDev>& out_rops) {
  const int RB = cfg.reg_bits, TB = cfg.thread_bits, L = d.L;
  const int NW = TB - 6;
  const bool c64 = cfg.c64;
  const uint32_t full = (1u << L) - 1;
  const uint32_t io_reg = c64 ? 1u : 0u;
  const uint32_t io_lane = c64 ? 0xEu : 0x7u;
  const int nops = d.op_count;

  // dependency order
  std::vector<uint32_t> need(nops), nd(nops), dg(nops);
  for (int i = 0; i < nops; ++i) {
    const TileOpDev& o = ho[d.op_begin + i];
    uint32_t tg = 0;
    if (o.kind != 2)
      for (int j = 0; j < o.k && j < 5; ++j)
        if (o.lt[j] >= 0) tg |= 1u << o.lt[j];
    if (o.kind == 2) {  // gradient rotation of the reverse sweep: k = Pauli id, target lt[0]/gq[0]
      const uint32_t t1 = o.lt[0] >= 0 ? (1u << o.lt[0]) : 0u;
      nd[i] = o.k == 3 ? 0u : t1;
      dg[i] = o.k == 3 ? t1 : 0u;
      need[i] = o.k == 3 ? 0u : t1;
    } else if (o.kind == 3) {  // Pauli-string gradient: X/Y qubits non-diagonal, Z diagonal
      nd[i] = o.off[0];
      dg[i] = o.off[1] & ~o.off[0];
      need[i] = 0;
    } else if (o.kind == 0) {
      nd[i] = tg;
      dg[i] = o.lcm;
      need[i] = o.k <= 2 ? tg : 0u;
    } else {
      nd[i] = 0;
      dg[i] = tg | o.lcm;
      need[i] = 0;
    }
  }
  std::vector<std::vector<int>> preds(nops);
  for (int j = 0; j < nops; ++j)
    for (int i = 0; i < j; ++i)
      if ((nd[i] & (nd[j] | dg[j])) | (dg[i] & nd[j])) preds[j].push_back(i);
  std::vector<char> foldable(nops, 0);
  for (int i = 0; i < nops; ++i) {
    const TileOpDev& o = ho[d.op_begin + i];
    foldable[i] = o.kind == 0 && o.k == 1 && o.xswap && o.gcm == 0 && __builtin_popcount(o.lcm) <= 1;
  }

  // list scheduling into segments; state 1: executed or folded into an
  // earlier re-map, 2: folded into the re-map after the current segment
  struct Seg {
    uint32_t regs = 0;  // register positions the ops need (+ IO constraints)
    bool io = false;
    std::vector<int> ops;
    std::vector<int> fold;  // ops folded into the re-map after this segment
    uint32_t w = 0;         // wave positions
    bool xwave = false;
  };
  std::vector<Seg> segs;
  std::vector<char> st(nops, 0);
  int left = nops;
  do {
    Seg s;
    const bool first = segs.empty();
    s.io = first;
    s.regs = first ? io_reg : 0u;
    const uint32_t forbid = first ? io_lane : 0u;
    for (bool progress = true; progress;) {
      progress = false;
      for (int i = 0; i < nops; ++i) {
        if (st[i]) continue;
        bool exec_ready = true, fold_ready = true;
        for (int q : preds[i]) {
          exec_ready = exec_ready && st[q] == 1;
          fold_ready = fold_ready && st[q] != 0;
        }
        if (foldable[i] && fold_ready) {
          st[i] = 2;
          s.fold.push_back(i);
        } else {
          const uint32_t u = s.regs | need[i];
          if (!exec_ready || (need[i] & forbid) || __builtin_popcount(u) > RB) continue;
          s.regs = u;
          s.ops.push_back(i);
          st[i] = 1;
        }
        --left;
        progress = true;
      }
    }
    if (s.ops.empty() && s.fold.empty() && !first) return fail(QSV_EINVAL, "internal: segment scheduling stalled");
    for (int i : s.fold) st[i] = 1;
    segs.push_back(std::move(s));
  } while (left > 0);
  {
    Seg& last = segs.back();
    // ops folded after the last segment need a re-map; when it would be the
    // only reason for one, run them as register exchanges instead
    if (!last.fold.empty() && (last.io || ((last.regs & io_lane) == 0 &&
                                           __builtin_popcount(last.regs | io_reg) <= RB))) {
      uint32_t u = last.regs | io_reg;
      for (int i : last.fold) u |= need[i] | (1u << ho[d.op_begin + i].lt[0]);
      if ((u & io_lane) == 0 && __builtin_popcount(u) <= RB) {
        last.regs = u;
        for (int i : last.fold) last.ops.push_back(i);
        last.fold.clear();
      }
    }
    if (!last.io || !last.fold.empty()) {
      if (last.fold.empty() && (last.regs & io_lane) == 0 && __builtin_popcount(last.regs | io_reg) <= RB) {
        last.regs |= io_reg;
        last.io = true;
      } else {
        Seg s;
        s.regs = io_reg;
        s.io = true;
        segs.push_back(std::move(s));
      }
    }
  }
  // affine map of each re-map (into segment k: the folds of segment k-1):
  // image of local basis vector p, and the constant
  const int K = int(segs.size());
  std::vector<std::vector<uint32_t>> mcol(K, std::vector<uint32_t>(L));
  std::vector<uint32_t> mcst(K, 0), ftarget(K, 0);
  for (int k = 0; k < K; ++k) {
    for (int q = 0; q < L; ++q) mcol[k][q] = 1u << q;
    if (k == 0) continue;
    for (int i : segs[k - 1].fold) {
      const TileOpDev& o = ho[d.op_begin + i];
      const uint32_t t = 1u << o.lt[0];
      ftarget[k] |= t;
      // x_t ^= x_c (control value 1) or x_t ^= x_c ^ 1 (value 0); no control: x_t ^= 1
      auto apply = [&](uint32_t y) -> uint32_t {
        if (o.lcm == 0) return y;
        return (y & o.lcm) ? (y ^ t) : y;
      };
      for (int q = 0; q < L; ++q) mcol[k][q] = apply(mcol[k][q]);
      mcst[k] = apply(mcst[k]);
      if (o.lcm == 0 || (o.lcv & o.lcm) == 0) mcst[k] ^= t;
    }
  }

  // wave bits: maximal runs of segments sharing NW available positions;
  // prefer positions off the low lanes (longer contiguous HBM runs)
  // (a run continues into segment k only if no op folded into the re-map
  // before k targets a wave bit: that re-map would move data across waves)
  std::vector<uint32_t> avail(K);
  for (int k = 0; k < K; ++k) avail[k] = full & ~segs[k].regs & ~(segs[k].io ? (io_lane | io_reg) : 0u);
  for (int k = 0; k < K;) {
    uint32_t I = avail[k];
    int m = k + 1;
    while (m < K && __builtin_popcount(I & avail[m] & ~ftarget[m]) >= NW) {
      I &= avail[m] & ~ftarget[m];
      ++m;
    }
    uint32_t w = 0;
    for (int pass = 0; pass < 2 && __builtin_popcount(w) < NW; ++pass)
      for (int pos = L - 1; pos >= 0 && __builtin_popcount(w) < NW; --pos) {
        const bool low = pos >= 1 && pos <= 6;
        if ((I >> pos & 1) && (pass == 1 || !low)) w |= 1u << pos;
      }
    if (__builtin_popcount(w) != NW) return fail(QSV_EINVAL, "internal: no wave bits");
    for (int t = k; t < m; ++t) {
      segs[t].w = w;
      segs[t].xwave = (t == k && k > 0);
    }
    k = m;
  }
  // A cross-wave re-map writes with the folded map, which may move elements
  // into other wavefronts' regions of the old layout; after a wave-local re-map
  // (no trailing barrier) those wavefronts may still be reading there, so such
  // a re-map also waits for the workgroup before writing.
  // A cross-wave re-map does not close with a barrier: waves go on with the
  // segment's register ops, and the barrier moves to the next LDS write (the
  // next re-map's, or an op through LDS, which always waits first). Until then
  // other waves may still read any region, so the next re-map waits first.
  std::vector<char> pre(K, 0);
  for (int k = 2; k < K; ++k) {
    if (segs[k].xwave && !segs[k - 1].xwave && (ftarget[k] & segs[k - 1].w)) pre[k] = 1;
    if (segs[k - 1].xwave) pre[k] = 1;
  }

  for (Seg& s : segs) {
    RegSegDev sd{};
    uint32_t regs = s.regs;
    const uint32_t keep_off = s.w | (s.io ? io_lane : 0u);
    for (int pos = L - 1; pos >= 0 && __builtin_popcount(regs) < RB; --pos)
      if (!(keep_off >> pos & 1)) regs |= 1u << pos;
    if (__builtin_popcount(regs) != RB) return fail(QSV_EINVAL, "internal: bad segment layout");
    int nr = 0, nt = 0;
    int regidx[32], thridx[32];
    for (int pos = 0; pos < L; ++pos) {
      regidx[pos] = -1;
      thridx[pos] = -1;
    }
    for (int pos = 0; pos < L; ++pos)
      if (regs >> pos & 1) {
        regidx[pos] = nr;
        sd.reg[nr++] = pos;
      }
    // lanes: the IO lane positions first, then the remaining ascending; then waves
    const uint32_t lanes = full & ~regs & ~s.w;
    if (s.io)
      for (int pos = 0; pos < L; ++pos)
        if (io_lane >> pos & 1) {
          thridx[pos] = nt;
          sd.thr[nt++] = pos;
        }
    for (int pos = 0; pos < L; ++pos)
      if ((lanes >> pos & 1) && thridx[pos] < 0) {
        thridx[pos] = nt;
        sd.thr[nt++] = pos;
      }
    if (nt != 6) return fail(QSV_EINVAL, "internal: bad lane layout");
    for (int pos = 0; pos < L; ++pos)
      if (s.w >> pos & 1) {
        thridx[pos] = nt;
        sd.thr[nt++] = pos;
      }
    if (nr != RB || nt != TB) return fail(QSV_EINVAL, "internal: bad segment layout");
    sd.xwave = (s.xwave ? 1 : 0) | (pre[&s - segs.data()] ? 2 : 0);
    {
      const int k = int(&s - segs.data());
      for (int q = 0; q < L; ++q) sd.mcol[q] = mcol[k][q];
      sd.mcst = mcst[k];
    }
    sd.op_begin = int(out_rops.size());
    // runs of uncontrolled dense one-qubit ops on distinct register bits 0..3
    // become one layer op (one dispatch: the op loop's scalar work per op --
    // descriptor loads, control checks, the branch tree over the variants --
    // costs as much as a one-qubit op's arithmetic)
    const char* lay_env = std::getenv("QSV_TILE_LAYERS");  // "0": one dispatch per op (comparison)
    const bool use_layers = cfg.layers && !(lay_env && lay_env[0] == '0');
    int lay_mask = 0;
    int lay_moff[4] = {0, 0, 0, 0};
    RegOpDev lay_first{};
    auto flush_layer = [&]() {
      if (lay_mask == 0) return;
      if (__builtin_popcount(lay_mask) == 1) {
        out_rops.push_back(lay_first);
      } else {
        RegOpDev lr{};
        lr.kind = 10;
        lr.moff = lay_first.moff;
        lr.lop = lay_first.lop;
        for (int p = 0; p < 4; ++p) lr.lm[p] = (lay_mask >> p & 1) ? lay_moff[p] : 0;
        lr.key = reg_key(10, lay_mask, cfg.c64 && cfg.mfma ? 1 : 0, false);
        out_rops.push_back(lr);
      }
      lay_mask = 0;
    };
    for (int li : s.ops) {
      const int oi = d.op_begin + li;
      const TileOpDev& o = ho[oi];
      RegOpDev r{};
      r.lop = oi;
      r.moff = o.moff;
      r.k = o.k;
      r.gcm = o.gcm;
      r.gcv = o.gcv;
      for (int pos = 0; pos < L; ++pos) {
        if (!(o.lcm >> pos & 1)) continue;
        const uint32_t val = (o.lcv >> pos) & 1;
        if (regidx[pos] >= 0) {
          r.ri_cm |= 1u << regidx[pos];
          r.ri_cv |= val << regidx[pos];
        } else {
          r.ti_cm |= 1u << thridx[pos];
          r.ti_cv |= val << thridx[pos];
        }
      }
      r.aux = (o.kind == 2 || o.kind == 3) ? o.ins[1] : 0;  // gradient: slot of the row in the pass
      if (o.kind == 3) {
        // Pauli-string gradient through LDS in this segment's layout
        r.kind = 8;
        const int SBp = c64 ? 5 : 4;
        const uint32_t msk = (1u << SBp) - 1, fl = o.off[0];
        r.pf_lds = (fl ^ ((fl >> SBp) & msk) ^ ((fl >> (2 * SBp)) & msk)) * (c64 ? 8u : 16u);
        r.pz_reg = r.pz_thr = 0;
        for (int pos = 0; pos < L; ++pos) {
          if (!(o.off[1] >> pos & 1)) continue;
          if (regidx[pos] >= 0) r.pz_reg |= 1u << regidx[pos];
          else r.pz_thr |= 1u << thridx[pos];
        }
        r.pph = int(o.off[2]);
        r.pz_glob = uint64_t(o.off[3]) | (uint64_t(o.off[4]) << 32);
      } else if (o.kind == 2 && o.k != 3) {
        r.kind = 5;
        r.p1 = regidx[o.lt[0]];
        if (r.p1 < 0) return fail(QSV_EINVAL, "internal: gradient target not in registers");
      } else if (o.kind == 2) {
        r.kind = 6;
        if (o.lt[0] >= 0) {
          if (regidx[o.lt[0]] >= 0) {
            r.dsrc[0] = 0;
            r.dbit[0] = regidx[o.lt[0]];
          } else {
            r.dsrc[0] = 1;
            r.dbit[0] = thridx[o.lt[0]];
          }
        } else {
          r.dsrc[0] = 2;
          r.dbit[0] = o.gq[0];
        }
      } else if (o.kind == 0 && o.k <= 2) {
        r.kind = o.k == 1 ? (o.xswap ? 4 : 0) : 1;
        r.p1 = regidx[o.lt[0]];
        r.p2 = o.k == 2 ? regidx[o.lt[1]] : 0;
        if (r.p1 < 0 || (o.k == 2 && r.p2 < 0)) return fail(QSV_EINVAL, "internal: target not in registers");
      } else if (o.kind == 1 && o.k <= 2) {
        r.kind = 2;
        for (int j = 0; j < o.k; ++j) {
          if (o.lt[j] >= 0) {
            if (regidx[o.lt[j]] >= 0) {
              r.dsrc[j] = 0;
              r.dbit[j] = regidx[o.lt[j]];
            } else {
              r.dsrc[j] = 1;
              r.dbit[j] = thridx[o.lt[j]];
            }
          } else {
            r.dsrc[j] = 2;
            r.dbit[j] = o.gq[j];
          }
        }
      } else {
        r.kind = 3;
      }
      if (r.kind == 0 && cfg.c64 && cfg.mfma && r.ri_cm == 0 && r.ti_cm == 0) {
        r.key = reg_key(7, r.p1, 0, false);
      } else if (r.kind == 0 || r.kind == 1 || r.kind == 4) {
        r.key = reg_key(r.kind, r.p1, r.p2, r.ri_cm != 0 || r.ti_cm != 0);
      } else if (r.kind == 2) {
        // register-bit targets of the diagonal, ascending (-1: absent)
        int a = -1, b = -1;
        for (int j = 0; j < o.k; ++j) {
          if (r.dsrc[j] != 0) continue;
          if (a < 0) a = r.dbit[j];
          else b = r.dbit[j];
        }
        if (b >= 0 && b < a) std::swap(a, b);
        r.key = reg_key(2, a, b, r.ri_cm != 0 || r.ti_cm != 0);
      }
      const bool layerable = use_layers && r.kind == 0 && o.kind == 0 && o.k == 1 && !o.xswap && r.ri_cm == 0 &&
                             r.ti_cm == 0 && r.gcm == 0 && r.p1 >= 0 && r.p1 < 4;
      if (layerable) {
        if (lay_mask >> r.p1 & 1) flush_layer();  // (same qubit: keep the order)
        if (lay_mask == 0) lay_first = r;
        lay_mask |= 1 << r.p1;
        lay_moff[r.p1] = r.moff;
        continue;
      }
      flush_layer();
      out_rops.push_back(r);
    }
    flush_layer();
    sd.op_count = int(out_rops.size()) - sd.op_begin;
    out_segs.push_back(sd);
    d.seg_count++;
  }
  // LDS address tables of the pass's segments: the tile's LDS index is
  // swizzled by j ^ (j >> SB) ^ (j >> 2 SB) (low SB bits of each), linear over
  // XOR, so the byte offset splits into a per-thread part (XOR of per-bit
  // columns) and a per-element part
  const int SB = c64 ? 5 : 4;
  const uint32_t esz = c64 ? 8u : 16u;
  auto swz = [SB](uint32_t j) {
    const uint32_t m = (1u << SB) - 1;
    return j ^ ((j >> SB) & m) ^ ((j >> (2 * SB)) & m);
  };
  auto gbit = [&](int p) { return uint64_t(1) << (p < d.b ? p : d.hq[p - d.b]); };
  for (int si = d.seg_begin; si < d.seg_begin + d.seg_count; ++si) {
    RegSegDev& S = out_segs[size_t(si)];
    for (int k = 0; k < TB; ++k) S.gcol_t[k] = gbit(S.thr[k]);
    for (int k = 0; k < RB; ++k) S.gcol_r[k] = gbit(S.reg[k]);
    for (int k = 0; k < TB; ++k) S.get_tcol[k] = swz(1u << S.thr[k]) * esz;
    for (int i = 0; i < (1 << RB); ++i) {
      uint32_t x = 0;
      for (int k = 0; k < RB; ++k)
        if (i >> k & 1) x |= 1u << S.reg[k];
      S.get_reg[i] = swz(x) * esz;
    }
    if (si == d.seg_begin) continue;
    const RegSegDev& O = out_segs[size_t(si) - 1];  // written through S's map
    S.put_tcst = swz(S.mcst) * esz;
    for (int k = 0; k < TB; ++k) S.put_tcol[k] = swz(S.mcol[O.thr[k]]) * esz;
    for (int i = 0; i < (1 << RB); ++i) {
      uint32_t x = 0;
      for (int k = 0; k < RB; ++k)
        if (i >> k & 1) x ^= S.mcol[O.reg[k]];
      S.put_reg[i] = swz(x) * esz;
    }
  }
  return QSV_OK;
}

// Device tables for the passes and ops (matrix offsets fixed here; matrix
// values are uploaded at apply time).
static int upload_tables(qsv_plan* p, std::vector<int>& moffs, size_t& pool_elems) {
  const int n = p->n;
  std::vector<TilePassDev> hp;
  std::vector<TileOpDev> ho;
  moffs.assign(p->blocks.size(), 0);
  pool_elems = 0;
  for (size_t bi = 0; bi < p->blocks.size(); ++bi) {
    const Block& B = p->blocks[bi];
    moffs[bi] = int(pool_elems);
    const size_t k = B.targets.size();
    pool_elems += B.diagonal ? (size_t(1) << k) : (size_t(1) << (2 * k));
  }
  for (const auto& P : p->passes) {
    TilePassDev d{};
    d.L = int(P.local.size());
    d.b = std::min(p->b, d.L);
    d.nh = d.L - d.b;
    if (d.nh > kTileMaxHigh) return fail(QSV_EINVAL, "too many high local qubits");
    for (int i = 0; i < d.nh; ++i) d.hq[i] = P.local[d.b + i];
    uint64_t lm = qmask(P.local);
    d.ng = 0;
    for (int q = 0; q < n; ++q)
      if (!(lm >> q & 1)) d.gpos[d.ng++] = q;
    pass_runs(d);
    d.op_begin = int(ho.size());
    d.op_count = int(P.blocks.size());
    std::vector<int> lpos(64, -1);
    for (size_t i = 0; i < P.local.size(); ++i) lpos[P.local[i]] = int(i);
    for (int bi : P.blocks) {
      const Block& B = p->blocks[bi];
      TileOpDev o{};
      o.kind = B.diagonal ? 1 : 0;
      o.xswap = B.xswap ? 1 : 0;
      o.k = int(B.targets.size());
      o.moff = moffs[bi];
      for (size_t j = 0; j < B.controls.size(); ++j) {
        const int q = B.controls[j];
        if (lpos[q] >= 0) {
          o.lcm |= 1u << lpos[q];
          if (B.ctrl_vals[j]) o.lcv |= 1u << lpos[q];
        } else {
          o.gcm |= uint64_t(1) << q;
          if (B.ctrl_vals[j]) o.gcv |= uint64_t(1) << q;
        }
      }
      for (int j = 0; j < 5; ++j) {
        o.lt[j] = -1;
        o.gq[j] = -1;
      }
      for (int j = 0; j < o.k; ++j) {
        const int q = B.targets[j];
        if (lpos[q] >= 0) o.lt[j] = lpos[q];
        else o.gq[j] = q;
      }
      if (o.kind == 0) {
        uint32_t ins = o.lcm;
        for (int j = 0; j < o.k; ++j) {
          if (o.lt[j] < 0) return fail(QSV_EINVAL, "internal: dense target not local");
          ins |= 1u << o.lt[j];
        }
        if (__builtin_popcount(ins) > 10) return fail(QSV_EINVAL, "too many local controls on one gate");
        o.m = 0;
        for (int q = 0; q < 32; ++q)
          if (ins >> q & 1) o.ins[o.m++] = q;
        for (int i = 0; i < (1 << o.k); ++i) {
          uint32_t off = 0;
          for (int j = 0; j < o.k; ++j)
            if (i >> j & 1) off |= 1u << o.lt[j];
          o.off[i] = off;
        }
      }
      if (o.kind == 0) p->kmax_dense = std::max(p->kmax_dense, o.k);
      ho.push_back(o);
    }
    d.seg_begin = int(p->h_segs.size());
    d.seg_count = 0;
    if (p->reg_bits > 0 && d.L == p->reg_bits + p->thread_bits) {
      const SegCfg cfg{p->reg_bits, p->thread_bits, p->dtype == QSV_C64,
                       p->dtype == QSV_C64 && tile_mfma_default()};
      int rc = build_reg_segments(cfg, ho, d, p->h_segs, p->h_rops);
      if (rc) return rc;
    }
    hp.push_back(d);
  }
  p->h_pass.swap(hp);
  p->h_ops.swap(ho);
  return QSV_OK;
}

// Device copies of the pass and op tables, made on the first apply so that
// planning itself needs no device.
static int ensure_tables(qsv_plan* p, hipStream_t stream) {
  if (p->d_pass) return QSV_OK;
  if (hipMalloc(reinterpret_cast<void**>(&p->d_pass), p->h_pass.size() * sizeof(TilePassDev)) != hipSuccess)
    return fail(QSV_ENOMEM, "plan table allocation failed");
  if (hipMalloc(reinterpret_cast<void**>(&p->d_ops),
                std::max<size_t>(1, p->h_ops.size()) * sizeof(TileOpDev)) != hipSuccess) {
    (void)hipFree(p->d_pass);
    p->d_pass = nullptr;
    return fail(QSV_ENOMEM, "plan table allocation failed");
  }
  if (hipMalloc(reinterpret_cast<void**>(&p->d_segs),
                std::max<size_t>(1, p->h_segs.size()) * sizeof(RegSegDev)) != hipSuccess ||
      hipMalloc(reinterpret_cast<void**>(&p->d_rops),
                std::max<size_t>(1, p->h_rops.size()) * sizeof(RegOpDev)) != hipSuccess)
    return fail(QSV_ENOMEM, "plan table allocation failed");
  QSV_HIP_CHECK(hipMemcpyAsync(p->d_pass, p->h_pass.data(), p->h_pass.size() * sizeof(TilePassDev),
                               hipMemcpyHostToDevice, stream));
  if (!p->h_ops.empty())
    QSV_HIP_CHECK(hipMemcpyAsync(p->d_ops, p->h_ops.data(), p->h_ops.size() * sizeof(TileOpDev),
                                 hipMemcpyHostToDevice, stream));
  if (!p->h_segs.empty())
    QSV_HIP_CHECK(hipMemcpyAsync(p->d_segs, p->h_segs.data(), p->h_segs.size() * sizeof(RegSegDev),
                                 hipMemcpyHostToDevice, stream));
  if (!p->h_rops.empty())
    QSV_HIP_CHECK(hipMemcpyAsync(p->d_rops, p->h_rops.data(), p->h_rops.size() * sizeof(RegOpDev),
                                 hipMemcpyHostToDevice, stream));
  QSV_HIP_CHECK(hipStreamSynchronize(stream));
  return QSV_OK;
}

// Block matrices (or diagonals) for parameters theta, written as complex
// doubles in block order.
void plan_block_values(const qsv_plan* p, const double* theta, std::vector<cd>& pool) {
  const qsv_circuit& C = p->circ_copy;
  pool.clear();
  std::vector<cd> gm, full, acc, tmp;
  for (const Block& B : p->blocks) {
    const int k = int(B.targets.size());
    const int D = 1 << k;
    if (B.gates.size() == 1) {
      const Gate& g = C.gates[B.gates[0]];
      GateInfo gi = analyse(g);
      extracted_matrix(g, gi, theta, gm);
      if (B.diagonal) {
        for (int i = 0; i < D; ++i) pool.push_back(gm[size_t(i) * D + i]);
      } else {
        pool.insert(pool.end(), gm.begin(), gm.end());
      }
      continue;
    }
    acc.assign(size_t(D) * D, cd{0, 0});
    for (int i = 0; i < D; ++i) acc[size_t(i) * D + i] = {1, 0};
    for (int gidx : B.gates) {
      const Gate& g = C.gates[gidx];
      GateInfo gi = analyse(g);
      extracted_matrix(g, gi, theta, gm);
      embed(gm, gi, B.targets, full);
      matmul(full, acc, D, tmp);  // later gate on the left
      acc.swap(tmp);
    }
    if (B.diagonal) {
      for (int i = 0; i < D; ++i) pool.push_back(acc[size_t(i) * D + i]);
    } else {
      pool.insert(pool.end(), acc.begin(), acc.end());
    }
  }
}

// Register-resident pass launch for the instantiated shapes (register bits,
// thread bits): complex64 (4, 9), (4, 8), (5, 8), (4, 7); complex128 (4, 8), (4, 7).
template <typename R, int RB, int TB>
static void launch_tile_reg_km(int km, dim3 grid, size_t lds, hipStream_t st, R* psi, const qsv_plan* p,
                               int pi, const cx<R>* pool) {
  const dim3 block(1u << TB);
  const TilePassDev* pd = p->d_pass;
  if (km == 2)
    hipLaunchKernelGGL((k_tile_reg<R, RB, 2, TB>), grid, block, lds, st, psi, pd, pi, p->d_segs, p->d_rops, p->d_ops, pool);
  else if (km == 3)
    hipLaunchKernelGGL((k_tile_reg<R, RB, 3, TB>), grid, block, lds, st, psi, pd, pi, p->d_segs, p->d_rops, p->d_ops, pool);
  else
    hipLaunchKernelGGL((k_tile_reg<R, RB, 5, TB>), grid, block, lds, st, psi, pd, pi, p->d_segs, p->d_rops, p->d_ops, pool);
}

template <typename R>
static void launch_tile_reg(int rb, int tb, int km, dim3 grid, size_t lds, hipStream_t st, R* psi,
                            const qsv_plan* p, int pi, const cx<R>* pool) {
  if constexpr (sizeof(R) == 4) {
    if (tb == 9) return launch_tile_reg_km<R, 4, 9>(km, grid, lds, st, psi, p, pi, pool);
    if (tb == 8 && rb == 5) return launch_tile_reg_km<R, 5, 8>(km, grid, lds, st, psi, p, pi, pool);
  }
  if (tb == 7) return launch_tile_reg_km<R, 4, 7>(km, grid, lds, st, psi, p, pi, pool);
  launch_tile_reg_km<R, 4, 8>(km, grid, lds, st, psi, p, pi, pool);
}

template <typename R>
static int apply_fused_t(qsv_state* s, qsv_plan* p, const double* theta) {
  int trc = ensure_tables(p, s->stream);
  if (trc) return trc;
  std::vector<cd> vals;
  plan_block_values(p, theta, vals);
  const size_t bytes = vals.size() * sizeof(cx<R>);
  if (p->pool_cap < vals.size()) {
    if (p->d_pool) {
      QSV_HIP_CHECK(hipStreamSynchronize(s->stream));
      (void)hipFree(p->d_pool);
      p->d_pool = nullptr;
    }
    if (hipMalloc(&p->d_pool, std::max<size_t>(bytes, 16)) != hipSuccess)
      return fail(QSV_ENOMEM, "plan pool allocation failed");
    p->pool_cap = vals.size();
  }
  if (p->stage_bytes < bytes) {
    if (p->h_stage) {
      if (p->stage_used) QSV_HIP_CHECK(hipEventSynchronize(p->stage_ev));
      (void)hipHostFree(p->h_stage);
      p->h_stage = nullptr;
    }
    if (hipHostMalloc(&p->h_stage, std::max<size_t>(bytes, 16), hipHostMallocDefault) != hipSuccess)
      return fail(QSV_ENOMEM, "plan staging allocation failed");
    p->stage_bytes = bytes;
  }
  if (!p->stage_ev) QSV_HIP_CHECK(hipEventCreateWithFlags(&p->stage_ev, hipEventDisableTiming));
  if (p->stage_used) QSV_HIP_CHECK(hipEventSynchronize(p->stage_ev));
  cx<R>* st = static_cast<cx<R>*>(p->h_stage);
  for (size_t i = 0; i < vals.size(); ++i) st[i] = {R(vals[i].re), R(vals[i].im)};
  if (bytes)
    QSV_HIP_CHECK(hipMemcpyAsync(p->d_pool, p->h_stage, bytes, hipMemcpyHostToDevice, s->stream));
  const int n = s->n;
  for (size_t pi = 0; pi < p->passes.size(); ++pi) {
    const int L = int(p->passes[pi].local.size());
    const uint64_t tiles = dim(n - L);
    size_t lds = (size_t(1) << L) * sizeof(cx<R>);
    const TilePassDev& hp = p->h_pass[pi];
    if (hp.seg_count == 1) {
      // a single register-resident segment never touches LDS unless one of
      // its blocks runs through LDS: launch without it (higher occupancy)
      const RegSegDev& sg = p->h_segs[hp.seg_begin];
      bool needs = false;
      for (int o = sg.op_begin; o < sg.op_begin + sg.op_count; ++o) needs |= p->h_rops[o].kind == 3;
      if (!needs) lds = 0;
    }
    if (lds > 65536) {
      QSV_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_tile<R, 2>),
                                        hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)));
      QSV_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_tile<R, 3>),
                                        hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)));
      QSV_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_tile<R, 5>),
                                        hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)));
    }
    ProfScope ps("tile", 2.0 * sizeof(cx<R>) * double(dim(n)), s->stream);
    R* psi = static_cast<R*>(s->ptr);
    const cx<R>* pool = static_cast<const cx<R>*>(p->d_pool);
    const dim3 grid(static_cast<unsigned>(tiles));
    const int km = p->kmax_dense <= 2 ? 2 : (p->kmax_dense <= 3 ? 3 : 5);
    if (p->h_pass[pi].seg_count > 0)
      launch_tile_reg<R>(p->reg_bits, p->thread_bits, km, grid, lds, s->stream, psi, p, int(pi), pool);
    else if (km == 2)
      hipLaunchKernelGGL((k_tile<R, 2>), grid, dim3(256), lds, s->stream, psi, p->d_pass, int(pi), p->d_ops, pool);
    else if (km == 3)
      hipLaunchKernelGGL((k_tile<R, 3>), grid, dim3(256), lds, s->stream, psi, p->d_pass, int(pi), p->d_ops, pool);
    else
      hipLaunchKernelGGL((k_tile<R, 5>), grid, dim3(256), lds, s->stream, psi, p->d_pass, int(pi), p->d_ops, pool);
    QSV_HIP_CHECK(hipGetLastError());
  }
  QSV_HIP_CHECK(hipEventRecord(p->stage_ev, s->stream));
  p->stage_used = true;
  return QSV_OK;
}

// Releases a plan and its device tables (keeps the error message).
static void plan_release(qsv_plan* p) {
  if (!p) return;
  if (p->stage_used) (void)hipEventSynchronize(p->stage_ev);
  if (p->stage_ev) (void)hipEventDestroy(p->stage_ev);
  if (p->h_stage) (void)hipHostFree(p->h_stage);
  if (p->d_pool) (void)hipFree(p->d_pool);
  if (p->d_pass) (void)hipFree(p->d_pass);
  if (p->d_ops) (void)hipFree(p->d_ops);
  if (p->d_segs) (void)hipFree(p->d_segs);
  if (p->d_rops) (void)hipFree(p->d_rops);
  delete p;
}

// Plan with an explicit register tile shape (thread bits TB); tile_qubits /
// low_qubits 0 select the defaults.
static int plan_create(const qsv_circuit* c, qsv_dtype dtype, int max_k, int tile_qubits, int low_qubits,
                       int TB, qsv_plan** out, bool heavy = false) {
  *out = nullptr;
  const int n = c->n;
  int L = tile_qubits > 0 ? tile_qubits : 12;
  // low qubits always local: 2^b amplitudes form one contiguous run, 128 bytes
  // (one cache line) at the default; fewer fixed low qubits leave more local
  // qubits free for the circuit, so fewer passes
  int b = low_qubits > 0 ? low_qubits : (dtype == QSV_C64 ? 4 : 3);
  if (L > 14 || (dtype == QSV_C128 && L > 13)) return fail(QSV_EINVAL, "tile of %d qubits exceeds LDS", L);
  L = std::min(L, n);
  b = std::min(b, L);
  if (dtype == QSV_C64 && b < 1) b = 1;
  if (L - b < max_k && L < n) return fail(QSV_EINVAL, "tile leaves fewer than max_k free qubits");
  if (L - b > kTileMaxHigh) return fail(QSV_EINVAL, "too many high local qubits");
  qsv_plan* p = new (std::nothrow) qsv_plan();
  if (!p) return fail(QSV_ENOMEM, "host allocation failed");
  p->n = n;
  p->dtype = dtype;
  p->max_k = max_k;
  p->heavy = heavy;
  p->L = L;
  p->b = b;
  // (blocks of 4-5 qubits run through LDS with 32-amplitude temporaries: the
  // 512-thread kernel would spill, and complex128 has no 512-thread shape)
  if ((dtype == QSV_C128 || max_k > 3) && TB == 9) TB = kRegThreadBits;
  // register bits: the rest of the tile; instantiated shapes (register bits,
  // thread bits): complex64 (4, 9), (4, 8), (5, 8), (4, 7); complex128 (4, 8), (4, 7)
  const int RB = L - TB;
  const bool rb_ok = RB == 4 || (dtype == QSV_C64 && RB == 5 && TB == 8);
  p->thread_bits = TB;
  p->reg_bits = (rb_ok && n >= L) ? RB : 0;
  p->circ_copy = *c;
  int rc = build_plan(p);
  std::vector<int> moffs;
  size_t pool_elems = 0;
  if (!rc) rc = upload_tables(p, moffs, pool_elems);
  if (rc) {
    plan_release(p);
    return rc;
  }
  *out = p;
  return QSV_OK;
}

}  // namespace qsv

using namespace qsv;

extern "C" {

int qsv_plan_fused(const qsv_circuit* c, qsv_dtype dtype, int max_k, int tile_qubits, int low_qubits,
                   qsv_plan** out) {
  return qsv_plan_fused_ex(c, dtype, max_k, tile_qubits, low_qubits, 0, out);
}

int qsv_plan_fused_ex(const qsv_circuit* c, qsv_dtype dtype, int max_k, int tile_qubits, int low_qubits,
                      int flags, qsv_plan** out) {
  clear_error();
  if (!out) return fail(QSV_EINVAL, "null output handle");
  *out = nullptr;
  if (!c) return fail(QSV_EINVAL, "null circuit");
  if (dtype != QSV_C64 && dtype != QSV_C128) return fail(QSV_EDTYPE, "unknown dtype");
  if (max_k < 1 || max_k > 5) return fail(QSV_EINVAL, "max_k must be in 1..5");
  if (flags & ~QSV_PLAN_HEAVY) return fail(QSV_EINVAL, "unknown plan flags 0x%x", unsigned(flags));
  // default tile: 2^12 amplitudes over 256 threads (TB = 8) x 16 in registers:
  // measured on MI355X, 2^12-amplitude tiles with 256 threads beat 2^13 with
  // 512 threads (6% at 30 qubits complex64, more workgroups in flight per
  // compute unit) despite more passes. QSV_TILE_QUBITS and
  // QSV_TILE_THREAD_BITS (7, 8, 9) override the defaults; qsv_plan_autotune
  // picks by measurement.
  int L = tile_qubits;
  if (const char* e = std::getenv("QSV_TILE_QUBITS"); e && tile_qubits <= 0) L = std::atoi(e);
  int TB = kRegThreadBits;
  if (const char* e = std::getenv("QSV_TILE_THREAD_BITS")) {
    const int v = std::atoi(e);
    TB = v == 9 ? 9 : (v == 7 ? 7 : 8);
  }
  return plan_create(c, dtype, max_k, L, low_qubits, TB, out, (flags & QSV_PLAN_HEAVY) != 0);
}

int qsv_plan_autotune(const qsv_circuit* c, qsv_state* scratch, const double* theta, int reps,
                      qsv_plan** out, int* choice) {
  clear_error();
  if (!out) return fail(QSV_EINVAL, "null output handle");
  *out = nullptr;
  if (!c) return fail(QSV_EINVAL, "null circuit");
  int rc = check_state(scratch);
  if (rc) return rc;
  if (scratch->n != c->n) return fail(QSV_ERANGE, "circuit has %d qubits, state %d", c->n, scratch->n);
  if (c->nparams > 0 && !theta) return fail(QSV_EINVAL, "circuit has parameters but theta is null");
  if (reps < 1 || reps > 100) return fail(QSV_EINVAL, "reps must be in 1..100");
  const qsv_dtype dt = scratch->dtype;
  // candidates: (max_k, tile qubits, thread bits)
  struct Cand { int k, L, TB; };
  std::vector<Cand> cands;
  for (int k : {1, 2, 3}) {
    cands.push_back({k, 12, 8});
    cands.push_back({k, 11, 7});
    if (dt == QSV_C64) {
      cands.push_back({k, 13, 9});
      cands.push_back({k, 13, 8});
    }
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  QSV_HIP_CHECK(hipEventCreate(&e0));
  QSV_HIP_CHECK(hipEventCreate(&e1));
  qsv_plan* best = nullptr;
  float best_ms = 0.f;
  int best_i = -1;
  for (size_t i = 0; i < cands.size(); ++i) {
    qsv_plan* p = nullptr;
    if (plan_create(c, dt, cands[i].k, cands[i].L, 0, cands[i].TB, &p) != QSV_OK) {
      clear_error();  // a shape that does not fit this circuit is skipped
      continue;
    }
    int r = qsv_apply_fused(scratch, p, theta);  // warm-up (uploads tables)
    if (!r) r = hipEventRecord(e0, scratch->stream) == hipSuccess ? QSV_OK : QSV_EHIP;
    for (int k = 0; k < reps && !r; ++k) r = qsv_apply_fused(scratch, p, theta);
    float ms = 0.f;
    if (!r) r = hipEventRecord(e1, scratch->stream) == hipSuccess ? QSV_OK : QSV_EHIP;
    if (!r) r = hipEventSynchronize(e1) == hipSuccess ? QSV_OK : QSV_EHIP;
    if (!r) r = hipEventElapsedTime(&ms, e0, e1) == hipSuccess ? QSV_OK : QSV_EHIP;
    if (r) {
      plan_release(p);
      plan_release(best);
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      return fail(r, "autotune: timing a candidate failed");
    }
    if (!best || ms < best_ms) {
      plan_release(best);
      best = p;
      best_ms = ms;
      best_i = int(i);
    } else {
      plan_release(p);
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (!best) return fail(QSV_EINVAL, "autotune: no candidate plan fits this circuit");
  if (choice) {
    choice[0] = cands[best_i].k;
    choice[1] = best->L;
    choice[2] = best->thread_bits;
    choice[3] = best->reg_bits;
  }
  *out = best;
  return QSV_OK;
}

int qsv_circuit_commute(const qsv_circuit* c, int gate, int qubit, int* paulis) {
  clear_error();
  if (!c || !paulis) return fail(QSV_EINVAL, "null argument");
  if (gate < 0 || gate >= int(c->gates.size())) return fail(QSV_ERANGE, "gate index %d out of range", gate);
  if (qubit < 0 || qubit >= c->n) return fail(QSV_ERANGE, "qubit %d out of range", qubit);
  const Gate& g = c->gates[size_t(gate)];
  *paulis = commute_masks(g, analyse(g), c->n)[size_t(qubit)];
  return QSV_OK;
}

int qsv_plan_info(const qsv_plan* p, int* passes, int* blocks, int* gates) {
  clear_error();
  if (!p) return fail(QSV_EINVAL, "null plan");
  if (passes) *passes = int(p->passes.size());
  if (blocks) *blocks = int(p->blocks.size());
  if (gates) *gates = int(p->circ_copy.gates.size());
  return QSV_OK;
}

int qsv_plan_stats(const qsv_plan* p, int* segments, int* lds_ops, int* kmax) {
  clear_error();
  if (!p) return fail(QSV_EINVAL, "null plan");
  int lo = 0;
  for (const RegOpDev& r : p->h_rops)
    if (r.kind == 3) ++lo;
  if (segments) *segments = int(p->h_segs.size());
  if (lds_ops) *lds_ops = lo;
  if (kmax) *kmax = p->kmax_dense;
  return QSV_OK;
}

int qsv_plan_free(qsv_plan* p) {
  clear_error();
  plan_release(p);
  return QSV_OK;
}

int qsv_apply_fused(qsv_state* s, qsv_plan* p, const double* theta) {
  clear_error();
  int rc = check_state(s);
  if (rc) return rc;
  if (!p) return fail(QSV_EINVAL, "null plan");
  if (p->n != s->n) return fail(QSV_ERANGE, "plan has %d qubits, state %d", p->n, s->n);
  if (p->dtype != s->dtype) return fail(QSV_EDTYPE, "plan and state dtypes differ");
  if (p->circ_copy.nparams > 0 && !theta) return fail(QSV_EINVAL, "plan has parameters but theta is null");
  return s->dtype == QSV_C64 ? apply_fused_t<float>(s, p, theta) : apply_fused_t<double>(s, p, theta);
}

}  // extern "C"
