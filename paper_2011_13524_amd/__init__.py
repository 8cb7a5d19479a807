"""MI355X (gfx950) state-vector simulation core for the method of Qulacs
(Suzuki et al., 2021): HIP kernels behind a C ABI (include/qsv.h), with this
package as a thin ctypes binding."""
from .binding import (LIB_PATH, Observable, QsvError, State, apply_record, expectation,  # noqa: F401
                      lib)
