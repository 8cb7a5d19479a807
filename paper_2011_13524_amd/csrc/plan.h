// Fusion plans: gates merged into dense blocks (section 5.4) and blocks
// scheduled into tile passes, each pass applying many blocks per read and
// write of the state.
#pragma once

#include <vector>

#include "circuit.h"

namespace qsv {

constexpr int kTileMaxOps = 4096;
constexpr int kTileMaxHigh = 16;
constexpr int kTileMaxGlobal = 40;

// One operation inside a tile pass, in the tile's local index space (local
// bit p <-> qubit local[p]).
struct TileOpDev {
  int kind;        // 0 dense on local targets, 1 diagonal (targets local or not),
                   // 2 gradient rotation of the reverse sweep (k = Pauli id),
                   // 3 gradient term of a multi-qubit Pauli rotation (reverse sweep;
                   //   no update): off[0] local flip mask, off[1] local Z/Y mask,
                   //   off[2] phase exponent (P x = i^off[2] (-1)^|x & zy| (x ^ f)
                   //   up to the tile's sign), off[3..4] Z/Y mask on non-local
                   //   qubits (low, high word), ins[0] row, ins[1] slot in the pass
  int k;           // number of targets
  int m;           // number of inserted zero positions (dense: targets + local controls)
  int moff;        // offset of the matrix / diagonal in the pool (complex elements)
  int lt[5];       // dense: local target positions; diag: local position or -1
  int gq[5];       // diag: global qubit of a non-local target, or -1
  int ins[10];     // dense: sorted local positions with zero bits (targets + local controls);
                   // gradient: ins[0] = row of the gradient, ins[1] = its slot in the pass
  int xswap;       // 1: the one-qubit matrix is Pauli X (a pure exchange)
  uint32_t lcm, lcv;  // local control mask / values (local index space)
  uint64_t gcm, gcv;  // non-local control mask / values (global index space)
  uint32_t off[32];   // dense: local offset of the i-th element of B1
};

struct TilePassDev {
  int L, b, nh, ng;
  int op_begin, op_count;
  int seg_begin, seg_count;  // register-resident execution (seg_count > 0)
  int row_begin, row_count;  // reverse sweep: gradient rows of the pass (slot s -> rows[row_begin + s])
  int hq[kTileMaxHigh];      // qubits of local bits b..L-1
  int gpos[kTileMaxGlobal];  // non-local qubits, ascending
  // the same map from tile index to tile base as runs of consecutive
  // non-local qubits: base = OR over r of ((g >> rsrc[r]) & (2^rlen[r] - 1)) << rdst[r]
  int nrun;
  int rsrc[kTileMaxHigh + 1], rdst[kTileMaxHigh + 1], rlen[kTileMaxHigh + 1];
};

// Register-resident tiles: the 2^L tile is spread over 2^TB threads holding
// 2^RB amplitudes each. A segment fixes which local bits index a thread's
// registers (reg) and which index the thread (thr: lanes first, then the
// wavefront index); ops of the segment whose dense targets are register bits
// run without touching LDS.
constexpr int kRegMaxBits = 6;
constexpr int kRegThreadBits = 8;      // default: 256-thread workgroups
constexpr int kRegMaxThreadBits = 9;   // up to 512-thread workgroups

struct RegSegDev {
  int reg[kRegMaxBits];        // local positions of register-index bits, ascending
  int thr[kRegMaxThreadBits];  // local position of thread-index bit k
  int xwave;                   // re-map into this layout: bit 0 across wavefronts (a
                               // barrier between writes and reads; none after the
                               // reads), bit 1 a workgroup barrier before the writes
  int op_begin, op_count;
  // the re-map into this layout writes local index x of the previous layout
  // to position M x ^ mcst (folded X / controlled-X ops); mcol[p] = M e_p
  uint32_t mcol[kTileMaxHigh + 8];
  uint32_t mcst;
  // LDS byte offsets, XOR-swizzled (filled by the planner for the plan's
  // dtype): element i of the thread with index tau sits at
  //   (tcst ^ XOR of tcol[k] over the set bits k of tau) ^ reg[i]
  // put_*: the previous layout written through the map above (the re-map
  // into this layout); get_*: this layout (tcst = 0).
  uint32_t put_reg[1 << (kRegMaxBits - 1)], put_tcol[kRegMaxThreadBits], put_tcst;
  uint32_t get_reg[1 << (kRegMaxBits - 1)], get_tcol[kRegMaxThreadBits];
  // global index bit of thread-index bit k and of register-index bit k in this
  // layout (HBM addresses of the first and last segments of a pass)
  uint64_t gcol_t[kRegMaxThreadBits], gcol_r[kRegMaxBits];
};

struct RegOpDev {
  int kind;             // 0 dense one-qubit, 1 dense two-qubit, 2 diagonal (k <= 2), 3 via LDS,
                        // 4 Pauli-X exchange on one register bit; reverse sweep: 5 gradient of an
                        // X/Y rotation on register bit p1, 6 gradient of a Z rotation (dsrc/dbit[0]),
                        // 8 gradient of a Pauli string; 10 layer of one-qubit ops (lm)
  int p1, p2;           // register bits of matrix index bits 0 and 1
  int k;
  int dsrc[2], dbit[2]; // diagonal targets: source 0 register bit, 1 thread bit, 2 global qubit
  uint32_t ri_cm, ri_cv;  // controls on register bits (register-index space)
  uint32_t ti_cm, ti_cv;  // controls on thread bits (thread-index space)
  uint64_t gcm, gcv;      // controls on non-local qubits
  int moff;
  int lop;              // index of the equivalent TileOpDev (LDS execution)
  int aux;              // gradient: slot of its row in the pass
  int key;              // kinds 0, 1, 2, 4, 10: variant of the register op (reg_key)
  // kind 10: a layer of uncontrolled dense one-qubit ops on distinct register
  // bits 0..3 in one dispatch; lm[p]: pool offset of the matrix on bit p
  int lm[4];
  // kind 8 (reverse sweep): gradient term of a multi-qubit Pauli rotation,
  // evaluated with psi staged in LDS: the partner of element i sits at its LDS
  // address XOR pf_lds; the sign parity is that of (i & pz_reg), (thread index
  // & pz_thr) and (tile base & pz_glob); phase exponent pph (0..3)
  uint32_t pf_lds, pz_reg, pz_thr;
  int pph;
  uint64_t pz_glob;
};

// Register-resident layout of a tile: 2^reg_bits amplitudes per thread,
// 2^thread_bits threads.
struct SegCfg {
  int reg_bits, thread_bits;
  bool c64;  // complex64: the HBM layouts keep local bit 0 in registers (16-byte pairs)
  bool mfma = false;  // complex64: uncontrolled dense one-qubit ops on the matrix cores
  bool layers = true;  // group one-qubit ops on distinct register bits into layer ops
};

// Whether complex64 register segments put uncontrolled dense one-qubit ops on
// the matrix cores (default on; QSV_TILE_MFMA=0 keeps them on the vector ALUs,
// for comparison).
bool tile_mfma_default();

// Splits the ops of pass d (ho[d.op_begin ..]) into register segments,
// appending them to segs / rops; d.seg_count is incremented per segment (the
// caller sets d.seg_begin = segs.size() and d.seg_count = 0 first).
// Fills the run-length form of d.gpos (d.nrun, rsrc, rdst, rlen).
void pass_runs(TilePassDev& d);

int build_reg_segments(const SegCfg& cfg, const std::vector<TileOpDev>& ho, TilePassDev& d,
                       std::vector<RegSegDev>& segs, std::vector<RegOpDev>& rops);

// A fused block: gates (indices into the circuit) applied in order, acting on
// `qubits` (ascending). Single-gate blocks keep the gate's control structure.
struct Block {
  std::vector<int> gates;
  std::vector<int> qubits;  // all qubits the block touches
  bool diagonal = false;
  bool xswap = false;  // single gate whose extracted matrix is Pauli X (CNOT, X)
  // structure used on the device (targets + controls after extraction)
  std::vector<int> targets;
  std::vector<int> controls, ctrl_vals;
};

}  // namespace qsv

struct qsv_plan;

namespace qsv {
// Block matrices (dense: 2^k x 2^k row-major; diagonal: 2^k entries) for
// parameters theta, concatenated in block order (the device pool layout).
void plan_block_values(const qsv_plan* p, const double* theta, std::vector<cd>& pool);
}  // namespace qsv

struct qsv_plan {
  int n = 0;
  qsv_dtype dtype = QSV_C128;
  int max_k = 2;
  bool heavy = false;  // commutation-aware merging (QSV_PLAN_HEAVY)
  int L = 12, b = 5;
  const qsv_circuit* circ = nullptr;  // borrowed structure snapshot below
  qsv_circuit circ_copy;
  std::vector<qsv::Block> blocks;
  struct Pass {
    std::vector<int> local;   // ascending local qubits (first b are 0..b-1)
    std::vector<int> blocks;  // block indices in execution order
  };
  std::vector<Pass> passes;
  // host copies of the device tables (uploaded on first apply)
  std::vector<qsv::TilePassDev> h_pass;
  std::vector<qsv::TileOpDev> h_ops;
  std::vector<qsv::RegSegDev> h_segs;
  std::vector<qsv::RegOpDev> h_rops;
  int reg_bits = 0;  // > 0: passes run register-resident
  int thread_bits = qsv::kRegThreadBits;  // workgroup = 2^thread_bits threads
  int kmax_dense = 1;  // widest dense op (selects the kernel instantiation)
  // device buffers
  qsv::TilePassDev* d_pass = nullptr;
  qsv::TileOpDev* d_ops = nullptr;
  qsv::RegSegDev* d_segs = nullptr;
  qsv::RegOpDev* d_rops = nullptr;
  void* d_pool = nullptr;
  size_t pool_cap = 0;  // complex elements
  // pinned staging for per-apply uploads
  void* h_stage = nullptr;
  size_t stage_bytes = 0;
  hipEvent_t stage_ev = nullptr;
  bool stage_used = false;
};
