// Per-launch timing scope (see qsv_prof_enable in qsv.h).
#pragma once

#include "qsv_internal.h"

namespace qsv {

bool prof_on();

// Records an event on `stream` at construction and at destruction when
// profiling is on; wrap exactly one kernel launch.
class ProfScope {
 public:
  ProfScope(const char* name, double bytes, hipStream_t stream);
  ~ProfScope();

 private:
  const char* name_;
  double bytes_;
  hipStream_t stream_;
  int a_ = -1;
};

}  // namespace qsv
