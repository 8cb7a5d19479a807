"""MI355X (gfx950) state-vector simulation core for the method of Qulacs
(Suzuki et al., 2021): HIP kernels behind a C ABI (include/qsv.h), with this
package as a thin ctypes binding."""
from .binding import (LIB_PATH, Batch, Circuit, Observable, Plan, QsvError, State,  # noqa: F401
                      adjoint_gradient, apply_circuit, apply_fused, apply_observable,
                      apply_pauli_rotation, apply_record, expectation, lib, prof_enable, prof_read,
                      transition_amplitude)
