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
  int kind;        // 0 dense on local targets, 1 diagonal (targets local or not)
  int k;           // number of targets
  int m;           // number of inserted zero positions (dense: targets + local controls)
  int moff;        // offset of the matrix / diagonal in the pool (complex elements)
  int lt[5];       // dense: local target positions; diag: local position or -1
  int gq[5];       // diag: global qubit of a non-local target, or -1
  int ins[10];     // dense: sorted local positions with zero bits (targets + local controls)
  uint32_t lcm, lcv;  // local control mask / values (local index space)
  uint64_t gcm, gcv;  // non-local control mask / values (global index space)
  uint32_t off[32];   // dense: local offset of the i-th element of B1
};

struct TilePassDev {
  int L, b, nh, ng;
  int op_begin, op_count;
  int hq[kTileMaxHigh];     // qubits of local bits b..L-1
  int gpos[kTileMaxGlobal]; // non-local qubits, ascending
};

// A fused block: gates (indices into the circuit) applied in order, acting on
// `qubits` (ascending). Single-gate blocks keep the gate's control structure.
struct Block {
  std::vector<int> gates;
  std::vector<int> qubits;  // all qubits the block touches
  bool diagonal = false;
  // structure used on the device (targets + controls after extraction)
  std::vector<int> targets;
  std::vector<int> controls, ctrl_vals;
};

}  // namespace qsv

struct qsv_plan {
  int n = 0;
  qsv_dtype dtype = QSV_C128;
  int max_k = 2;
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
  // device buffers
  qsv::TilePassDev* d_pass = nullptr;
  qsv::TileOpDev* d_ops = nullptr;
  void* d_pool = nullptr;
  size_t pool_cap = 0;  // complex elements
  // pinned staging for per-apply uploads
  void* h_stage = nullptr;
  size_t stage_bytes = 0;
  hipEvent_t stage_ev = nullptr;
  bool stage_used = false;
};
