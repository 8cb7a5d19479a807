// Internal declarations shared by the libqsv translation units (host + device).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/qsv.h"

namespace qsv {

// ------------------------------------------------------------------ errors

void set_error(const char* fmt, ...);
int fail(int code, const char* fmt, ...);
void clear_error();

#define QSV_HIP_CHECK(expr)                                                        \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess)                                                          \
      return ::qsv::fail(QSV_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

// ------------------------------------------------------------------ host-side complex (FP64)

struct cd {
  double re, im;
};
inline cd cmul(cd a, cd b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
inline cd cadd(cd a, cd b) { return {a.re + b.re, a.im + b.im}; }

// ------------------------------------------------------------------ small device buffer uploads

// A ring of pinned host slots mirrored by device slots. A slot is reused only
// after the event recorded behind the last kernel that read it has completed,
// so host writes never race with in-flight copies or kernels.
class Uploader {
 public:
  static constexpr size_t kSlotBytes = 64 * 1024;
  static constexpr int kSlots = 32;
  ~Uploader();
  // Copies `bytes` (<= kSlotBytes) from src into the next slot and enqueues the
  // host-to-device copy on `stream`. Returns the device address via *dev.
  int upload(const void* src, size_t bytes, hipStream_t stream, void** dev, int* slot);
  // Records the completion event of `slot` on `stream` (call after the kernels
  // that read the slot have been enqueued).
  int release(int slot, hipStream_t stream);

 private:
  int init();
  bool ready_ = false;
  char* host_ = nullptr;
  char* dev_ = nullptr;
  hipEvent_t ev_[kSlots] = {};
  bool used_[kSlots] = {};
  int next_ = 0;
};

// ------------------------------------------------------------------ handles

}  // namespace qsv

struct qsv_state {
  void* ptr = nullptr;
  int n = 0;
  qsv_dtype dtype = QSV_C128;
  hipStream_t stream = nullptr;
  bool owned = false;
  int device = 0;
  qsv::Uploader up;
  // FP64 reduction scratch (partials), allocated on first use.
  double* red = nullptr;
  double* red_host = nullptr;  // pinned
  size_t red_cap = 0;
  // matrix of a dense gate on 6..10 targets (FP64, transposed), grown on use
  void* big = nullptr;
  size_t big_cap = 0;
  // work buffer of calls that synchronise the stream before returning
  // (sampling tables, reverse-sweep tables): grown on demand, kept for the
  // next call, freed with the state
  mutable void* work = nullptr;
  mutable size_t work_cap = 0;
};

namespace qsv {
// *out = at least `bytes` of the state's work buffer (grown after a stream
// sync when too small); QSV_OK, or QSV_ENOMEM / QSV_EHIP with the error set.
int state_work(const qsv_state* s, size_t bytes, void** out);
}  // namespace qsv

namespace qsv {

inline size_t amp_bytes(qsv_dtype d) { return d == QSV_C64 ? 8 : 16; }
inline uint64_t dim(int n) { return uint64_t(1) << n; }

// Insert-zero index positions for a gate: the sorted qubit positions whose
// bits are zero in every B0 element (section 4.3.2, B0 and the on-the-fly index
// computation of section 5.2).
struct InsertPos {
  int m = 0;
  int pos[40];
};

int check_state(const qsv_state* s);
int ensure_reduce_scratch(qsv_state* s, size_t doubles);

// Gate application, dispatched by matrix structure (gates.hip).
int apply_gate_impl(qsv_state* s, const cd* mat, const int* targets, int k, const int* controls,
                    const int* ctrl_vals, int nc);
int named_matrix(int kind, double theta, cd* out, int* k);

// Controlled structure of a gate matrix (gates.hip): peel off target bits that
// act as controls, shrinking the matrix and extending (cmask, cval).
void extract_controls(std::vector<cd>& mat, std::vector<int>& tq, uint64_t& cmask, uint64_t& cval);
int validate_gate(int n, const int* targets, int k, const int* controls, const int* ctrl_vals,
                  int nc, int kmax);

// Launch helpers (gates.hip).
int launch_scale_subspace(qsv_state* s, uint64_t mask, uint64_t pattern, cd c);

}  // namespace qsv
