/*
 * qsv.h -- C ABI of libqsv, an MI355X (gfx950) state-vector simulator core.
 *
 * Method: Suzuki et al., "Qulacs: a fast and versatile quantum circuit
 * simulator for research purpose" (Quantum, 2021). Section references below
 * are to that paper.
 *
 * Conventions shared by every entry point
 * ----------------------------------------
 * - A state of n qubits is 2^n complex amplitudes in device memory, stored
 *   interleaved (re, im): complex64 = 2 x float, complex128 = 2 x double. This
 *   is the layout of torch.complex64 / torch.complex128 tensors.
 * - Basis index x = sum_q x_q 2^q: qubit 0 is the right-most digit of the ket
 *   (section 4.2.1).
 * - Gate matrices are passed from the host as complex128, row-major,
 *   interleaved, 2^k x 2^k doubles pairs. Bit j of the row / column index
 *   corresponds to targets[j] (qubit targets[0] is the least significant bit
 *   of the matrix index), so DenseMatrix({t, c}, CNOT-as-printed) in
 *   Appendix A flips t when c is set. Complex64 states round the matrix to
 *   float on the host.
 * - Rotations are R_P(theta) = exp(+i theta P / 2) as in the table of named
 *   gates (section 4.3.4).
 * - Host arrays passed in (matrices, qubit lists, coefficients) are copied
 *   before the call returns; the caller keeps ownership.
 * - Every function returns 0 (QSV_OK) or a negative error code. On error
 *   nothing has been enqueued and no state has been modified; the message is
 *   available from qsv_last_error() (thread-local). No C++ exception crosses
 *   this boundary and the library never aborts the process.
 * - Work is enqueued asynchronously on the stream the state was created with.
 *   Calls that return values to the host (qsv_store, qsv_norm2, qsv_inner,
 *   qsv_expectation, qsv_adjoint_gradient) synchronise that stream.
 */
#ifndef QSV_H_
#define QSV_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct qsv_state qsv_state;
typedef struct qsv_circuit qsv_circuit;
typedef struct qsv_plan qsv_plan;
typedef struct qsv_observable qsv_observable;
typedef struct qsv_batch qsv_batch;

typedef enum { QSV_C64 = 1, QSV_C128 = 2 } qsv_dtype;

enum {
  QSV_OK = 0,
  QSV_EINVAL = -1, /* malformed argument (null pointer, bad kind, bad size)  */
  QSV_ERANGE = -2, /* qubit index, basis index or count out of range        */
  QSV_EDUP = -3,   /* a qubit listed twice among targets and controls       */
  QSV_ENOMEM = -4, /* device or host allocation failed                      */
  QSV_EHIP = -5,   /* a HIP runtime call failed                             */
  QSV_EDTYPE = -6, /* dtype mismatch between states                         */
  QSV_ENODEV = -7  /* no usable gfx950 device                               */
};

/* Named gates of the table of named gates (section 4.3.4). */
enum {
  QSV_GATE_X = 1,    /* Pauli X, qubits {q}                                    */
  QSV_GATE_Y = 2,    /* Pauli Y, qubits {q}                                    */
  QSV_GATE_Z = 3,    /* Pauli Z, qubits {q}                                    */
  QSV_GATE_H = 4,    /* Hadamard, qubits {q}                                   */
  QSV_GATE_RX = 5,   /* exp(+i theta X/2), qubits {q}                          */
  QSV_GATE_RY = 6,   /* exp(+i theta Y/2), qubits {q}                          */
  QSV_GATE_RZ = 7,   /* exp(+i theta Z/2), qubits {q}                          */
  QSV_GATE_CNOT = 8, /* qubits {control, target}                              */
  QSV_GATE_CZ = 9,   /* qubits {a, b}                                          */
  QSV_GATE_SWAP = 10 /* qubits {a, b}                                          */
};

/* Message of the last failed call on this thread ("" if none). */
const char* qsv_last_error(void);

/* ABI version (major * 100 + minor). */
int qsv_version(void);

/* ---------------------------------------------------------------- states */

/* Allocate a 2^n-amplitude state on the current HIP device, initialised to
 * |0...0> (section 4.2.1). 1 <= n <= 34. stream: a hipStream_t (NULL = the
 * default stream). The library owns the memory; free with qsv_state_free.
 * QSV_ENOMEM if the device cannot hold it. */
int qsv_state_alloc(int n, qsv_dtype dtype, void* stream, qsv_state** out);

/* Wrap caller-owned device memory of 2^n amplitudes (e.g. a torch tensor's
 * storage, 256-byte aligned). Contents are left untouched. The caller keeps
 * the memory alive until qsv_state_free. */
int qsv_state_wrap(void* dev_ptr, int n, qsv_dtype dtype, void* stream, qsv_state** out);

/* Release a state (frees the memory only if the library allocated it). NULL is
 * accepted. The state's stream is synchronised first. */
int qsv_state_free(qsv_state* s);

/* Report qubit count, dtype and device pointer (any out pointer may be NULL). */
int qsv_state_info(const qsv_state* s, int* n, int* dtype, void** dev_ptr);

/* Wait for all work enqueued on the state's stream (QSV_EHIP if it failed). */
int qsv_state_sync(const qsv_state* s);

/* Set the state to the computational basis state |k> (section 4.2.1). */
int qsv_set_basis(qsv_state* s, uint64_t k);

/* Upload 2^n complex128 amplitudes (2 * 2^n doubles, interleaved) from host
 * memory (section 4.2.1, load). */
int qsv_load(qsv_state* s, const double* host_interleaved);

/* Download the amplitudes as complex128 into host memory (complex64 states are
 * widened exactly). Synchronises the state's stream (section 4.2.2,
 * get_vector). */
int qsv_store(const qsv_state* s, double* host_interleaved);

/* dst <- src (same n and dtype), enqueued on dst's stream (section 4.2.1, copy). */
int qsv_copy(qsv_state* dst, const qsv_state* src);

/* ---------------------------------------------------------------- gates */

/* Apply a basic gate psi <- K psi (section 4.3.2, Eq. update_mat) with gate
 * matrix mat (2^k x 2^k, see conventions) on targets[0..k-1], acting only on
 * the amplitudes whose control qubits controls[i] hold ctrl_vals[i] in {0, 1}
 * (controlled gates, section 4.3.2). 1 <= k <= 10; targets and controls
 * distinct and in [0, n). K need not be unitary. The library recognises the
 * structured matrices the paper lists (diagonal, Pauli-X / CNOT / SWAP
 * permutations, one-entry phases such as Z or CZ) and applies them with fewer
 * memory operations. k <= 5 runs on register-resident kernels; 6 <= k <= 10
 * on the generic path (the 2^k-amplitude temporal vector of one B0 element in
 * LDS, as section 5.5 does for wide gates; the matrix is kept in FP64 in a
 * per-state device buffer, grown on first use, so such a call may allocate
 * and synchronises the state's stream once to stage the matrix). Circuits and
 * fused plans take gates of at most 5 targets. controls / ctrl_vals may be
 * NULL when nc == 0. Errors: QSV_EINVAL (k outside 1..10, bad control
 * values), QSV_ERANGE / QSV_EDUP (qubits), QSV_ENOMEM (matrix buffer). */
int qsv_apply_gate(qsv_state* s, const double* mat, const int* targets, int k,
                   const int* controls, const int* ctrl_vals, int nc);

/* Apply a named gate (QSV_GATE_*) on qubits[0..nq-1]; theta is used by the
 * rotations only. */
int qsv_apply_named(qsv_state* s, int kind, const int* qubits, int nq, double theta);

/* ---------------------------------------------------------------- reductions */

/* Squared norm <psi|psi> accumulated in double (section 4.2.2). */
int qsv_norm2(const qsv_state* s, double* out);

/* Inner product <bra|ket> accumulated in double (section 4.2.2). Same n and
 * dtype. */
int qsv_inner(const qsv_state* bra, const qsv_state* ket, double* re, double* im);

/* Marginal probability of a Z-basis outcome (section 4.2.2, the marginal-
 * probability utility). values: host array of n ints, values[q] for qubit q:
 * 0 or 1 for a measured qubit, 2 for one left unmeasured. *out = sum of
 * |psi_x|^2 over the basis indices x whose measured bits equal the values,
 * visiting only those 2^(n - m) amplitudes (m measured), FP64 accumulation
 * with per-block partials summed in a fixed order. The state is not
 * normalised first. Synchronises.
 * Errors: QSV_EINVAL (null arguments, a value outside {0, 1, 2}). */
int qsv_marginal_probability(const qsv_state* s, const int* values, double* out);

/* Z-basis sampling (section 4.2.2: sampling through a cumulative distribution
 * built first, which needs an extra 2^n-long array). u: host array of `count`
 * uniforms in [0, 1), drawn by the caller; out: host array of `count` basis
 * indices, out[i] = the smallest x with C(x) > u[i] * C(2^n - 1), C the
 * inclusive cumulative sum of |psi|^2 in FP64 (unnormalised states are
 * sampled from |psi|^2 / <psi|psi>). An index of probability zero is never
 * returned. The table takes 2^n FP64 entries (8 bytes per amplitude) plus
 * 2^(n-12) chunk totals and 16 bytes per sample, carved from the state's work
 * buffer: allocated on the first call (or grown), kept for later calls and
 * freed with the state. The call synchronises. count == 0 only builds the
 * table.
 * Errors: QSV_EINVAL (null arguments, count < 0, a state of zero norm),
 * QSV_ERANGE (a uniform outside [0, 1) or NaN, count > 2^31), QSV_ENOMEM. */
int qsv_sample(const qsv_state* s, const double* u, int64_t count, int64_t* out);

/* ---------------------------------------------------------------- circuits */

/* A circuit is an ordered host-side list of basic gates (section 4.4,
 * QuantumCircuit), some of them parametric rotations whose angles are read
 * from a parameter vector at apply time (ParametricQuantumCircuit). */
int qsv_circuit_create(int n, qsv_circuit** out);
int qsv_circuit_free(qsv_circuit* c);

/* Append a basic gate: same arguments and limits as qsv_apply_gate. */
int qsv_circuit_add_gate(qsv_circuit* c, const double* mat, const int* targets, int k,
                         const int* controls, const int* ctrl_vals, int nc);

/* Append a named gate (QSV_GATE_*); RX/RY/RZ with the fixed angle theta. */
int qsv_circuit_add_named(qsv_circuit* c, int kind, const int* qubits, int nq, double theta);

/* Append a parametric rotation exp(+i theta[param_slot] P / 2) on one qubit,
 * P = X, Y, Z for pauli_id = 1, 2, 3 (ParametricRX/RY/RZ, section 4.4). The
 * circuit's parameter count becomes at least param_slot + 1. */
int qsv_circuit_add_rotation(qsv_circuit* c, int pauli_id, int qubit, int param_slot);

/* Append a multi-qubit Pauli rotation exp(+i theta P / 2) (section 4.3.2,
 * Pauli rotation; the factor 1/2 as in Table 1's one-qubit rotations, so a
 * one-qubit string is RX/RY/RZ), P = prod_j sigma_{pauli_ids[j]} on qubits[j]
 * (ids 0..3 = I, X, Y, Z; distinct qubits, 1 <= w <= n). param_slot >= 0:
 * theta = theta[param_slot] at apply time (the circuit's parameter count grows
 * to param_slot + 1); param_slot < 0: the fixed angle `theta`. Fused plans take
 * strings of up to 5 non-identity factors (a dense block; pure-Z strings are
 * diagonal); qsv_adjoint_gradient takes them with the per-gate reverse sweep;
 * batches reject them (QSV_EINVAL). Errors: QSV_EINVAL, QSV_ERANGE, QSV_EDUP. */
int qsv_circuit_add_pauli_rotation(qsv_circuit* c, const int* qubits, const int* pauli_ids, int w,
                                   int param_slot, double theta);

/* Qubit count, gate count and parameter count (any out pointer may be NULL). */
int qsv_circuit_info(const qsv_circuit* c, int* n, int* gates, int* nparams);

/* psi <- exp(+i theta P / 2) psi for the Pauli string P = prod_j
 * sigma_{pauli_ids[j]} on qubits[j] (section 4.3.2; ids 0..3, distinct qubits,
 * 0 <= w <= n): one sweep over the amplitude pairs (x, x ^ F), F the X/Y
 * qubits (P's one nonzero per column is i^nY (-1)^|x & z|, z the Z/Y qubits).
 * Asynchronous on the state's stream. Errors: QSV_EINVAL (bad id or length,
 * null lists), QSV_ERANGE (qubit out of range), QSV_EDUP (repeated qubit). */
int qsv_apply_pauli_rotation(qsv_state* s, const int* qubits, const int* pauli_ids, int w, double theta);

/* Apply every gate in order, one kernel launch per gate (section 4.4,
 * update_quantum_state). theta: the parameter vector (may be NULL when the
 * circuit has no parameters). */
int qsv_apply_circuit(qsv_state* s, const qsv_circuit* c, const double* theta);

/* ---------------------------------------------------------------- fusion */

/* Plan the fused execution of a circuit (section 5.4, circuit optimization)
 * for states of dtype `dtype`:
 *  - gates are merged into dense blocks of at most max_k qubits (1..5) where a
 *    gate depends on a single earlier block (merge of two successive gates);
 *    diagonal gates only merge with blocks whose qubits they do not widen;
 *  - blocks are grouped into tile passes: each pass keeps tile_qubits qubits
 *    local (0 = default: 12), always including
 *    the low_qubits lowest qubits (0 = default: 4 / 3) so that HBM runs are
 *    contiguous, and applies every block whose non-diagonal targets are local.
 *    One pass reads and writes the state once.
 * The plan copies the circuit's structure; later edits of the circuit do not
 * affect it. Parameters are read at apply time. */
int qsv_plan_fused(const qsv_circuit* c, qsv_dtype dtype, int max_k, int tile_qubits,
                   int low_qubits, qsv_plan** out);

/* qsv_plan_fused with options. flags: 0, or QSV_PLAN_HEAVY for the heavy
 * optimization of section 5.4: every gate carries, per qubit it touches, the
 * Paulis it commutes with there (CNOT: Z on the control, X on the target;
 * diagonal gates: Z; RX/RY/RZ and Pauli rotations: their Pauli; fixed
 * matrices: tested on the matrix), and a gate joins an earlier block that it
 * can be moved next to by passing blocks it commutes with (a shared commuting
 * Pauli on every common qubit), within the same size and arithmetic rules.
 * Planning takes longer (each gate may scan back over all blocks); circuits
 * of commuting gates compress to constant depth. Errors as qsv_plan_fused,
 * plus QSV_EINVAL for unknown flags. */
#define QSV_PLAN_HEAVY 1

/* Commutation information of gate `gate` of a circuit on `qubit` (section 5.4:
 * each gate keeps, per qubit, the Pauli bases it commutes with): *paulis
 * receives bit 0 if the gate commutes with X on that qubit, bit 1 for Y, bit 2
 * for Z (7 on qubits the gate does not touch). Errors: QSV_EINVAL (null
 * argument), QSV_ERANGE (gate or qubit out of range). */
int qsv_circuit_commute(const qsv_circuit* c, int gate, int qubit, int* paulis);
int qsv_plan_fused_ex(const qsv_circuit* c, qsv_dtype dtype, int max_k, int tile_qubits,
                      int low_qubits, int flags, qsv_plan** out);

/* Autotuned plan (section 5.4: the fusion width is a tuning choice): builds
 * candidate plans over fusion widths max_k = 1, 2, 3 and tile shapes
 * (tile qubits, thread bits) = (12, 8), (11, 7) and, for complex64, (13, 9)
 * and (13, 8), times `reps` (1..100) fused applications of each on `scratch`
 * (a state of the circuit's width and the plan's dtype, on its stream, after
 * one untimed warm-up application) with HIP events, and returns the fastest
 * in *out (caller frees with qsv_plan_free). choice (may be NULL) receives
 * int[4]: max_k, tile qubits, thread bits, register bits (0 = LDS kernel).
 * The contents of `scratch` are overwritten with the circuit applied
 * (1 + reps) times per candidate. Blocks the calling thread. Errors:
 * QSV_EINVAL (null arguments, reps out of range, null theta for a
 * parametric circuit, no candidate fits), QSV_ERANGE (width mismatch),
 * QSV_EHIP (a launch or event failed; no plan is returned). */
int qsv_plan_autotune(const qsv_circuit* c, qsv_state* scratch, const double* theta, int reps,
                      qsv_plan** out, int* choice);

/* Number of passes, fused blocks and original gates (any out pointer may be NULL). */
int qsv_plan_info(const qsv_plan* p, int* passes, int* blocks, int* gates);

/* Execution shape of a plan: register-resident segments summed over passes
 * (0 when passes run LDS-resident), blocks applied through LDS inside
 * register-resident passes, and the widest dense block. */
int qsv_plan_stats(const qsv_plan* p, int* segments, int* lds_ops, int* kmax);
int qsv_plan_free(qsv_plan* p);

/* Apply a plan to a state of the plan's qubit count and dtype: block matrices
 * are formed on the host in double precision for theta (products of the gate
 * matrices, later gate on the left), uploaded, and one tile kernel per pass is
 * enqueued on the state's stream. A plan must not be applied concurrently from
 * two streams. */
int qsv_apply_fused(qsv_state* s, qsv_plan* p, const double* theta);

/* ---------------------------------------------------------------- profiling */

/* Opt-in per-kernel timing with HIP events recorded on the launching stream
 * around every kernel launch, and the algorithmic bytes each launch must move
 * (the cost model of section 4.3.2: every amplitude a gate touches is read and
 * written once). qsv_prof_enable(1) clears the records and starts recording;
 * qsv_prof_enable(0) stops. qsv_prof_read synchronises the recorded events and
 * reports, for kernel family `name` (e.g. "pair", "tile"), the number of
 * launches, their summed duration in milliseconds and summed algorithmic
 * bytes. Not thread-safe; meant for benchmarks. */
int qsv_prof_enable(int on);
int qsv_prof_read(const char* name, int* launches, double* total_ms, double* bytes);

/* ---------------------------------------------------------------- observables */

/* An observable O = sum_k alpha_k P_k, a real linear combination of Pauli
 * strings (section 4.5). Host-side object; freed with qsv_observable_free. */
int qsv_observable_create(int n, qsv_observable** out);
int qsv_observable_free(qsv_observable* o);

/* Add alpha * P with P = prod_j sigma_{pauli_ids[j]}(qubits[j]); pauli ids
 * 0..3 = I, X, Y, Z (section 4.3.2, Pauli gate). w = 0 adds alpha * identity.
 * Qubits distinct and < n. */
int qsv_observable_add_term(qsv_observable* o, double coef, const int* qubits,
                            const int* pauli_ids, int w);

/* Number of qubits, terms and distinct flip masks (X/Y positions); any out
 * pointer may be NULL. Terms sharing a flip mask share one pass over the state. */
int qsv_observable_info(const qsv_observable* o, int* n, int* terms, int* groups);

/* Transition amplitude <bra|O|ket> = sum_k alpha_k <bra|P_k|ket> (section
 * 4.5, get_transition_amplitude), complex, accumulated in FP64 (one sweep of
 * both states per term; per-block partials summed in a fixed order). Both
 * states have the observable's qubit count and one dtype. Synchronises.
 * Errors: QSV_EINVAL (null arguments), QSV_ERANGE, QSV_EDTYPE. */
int qsv_transition_amplitude(const qsv_state* bra, const qsv_observable* o, const qsv_state* ket,
                             double* re, double* im);

/* Number of state passes an expectation (or qsv_apply_observable) of this
 * observable takes for states of dtype `dtype`: its flip masks packed into
 * tiles of 2^13 (complex64) or 2^12 (complex128) amplitudes, plus one pass per
 * flip mask wider than a tile. Host-only. */
int qsv_observable_passes(const qsv_observable* o, qsv_dtype dtype, int* passes);

/* <psi|O|psi> accumulated in double (section 4.5, get_expectation_value). The
 * state is not normalised first (basic gates need not be unitary). Flip masks
 * are packed into passes that each read the state once (a mask with more flip
 * qubits than a tile holds gets a pass of its own); the terms of a flip mask
 * shared by at most eight strings are evaluated one by one, larger sets
 * together. complex64: a single-term evaluation's pair products, and each
 * thread's sum of 8 of them per tile, are formed in FP32 (|error| <= 9 x
 * 2^-24 x sum|alpha| x <psi|psi> beyond the stored amplitudes), every other
 * sum in double. Synchronises the state's stream. */
int qsv_expectation(const qsv_state* s, const qsv_observable* o, double* out);

/* qsv_expectation for callers that cannot allocate device memory (code under
 * stream capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same passes, kernels and result (bitwise, at the same launch shape), with
 * every device buffer the call needs -- the observable's pass / group / term
 * tables and the per-workgroup FP64 partials -- in one file-scope device
 * array of 1 MiB that each GPU holds from the library's first use of it
 * until the process ends; the call makes no hipMalloc, hipFree or pinned-
 * memory allocation (host-side plan tables are built and cached on the
 * observable as for qsv_expectation). The tables of one pass cost about
 * 250 bytes, of one flip-mask record about 184 (one per term for a mask
 * shared by at most eight strings, else one per mask) and of one term 32, plus
 * 16 KiB of partials: some 4700 strings with distinct flip masks fit. Calls that overlap on one
 * GPU share the array and race; calls in order on one stream do not (the
 * array keeps the last call's contents, and each call rewrites what it
 * reads). Synchronises the state's stream.
 * Errors: QSV_EINVAL (null arguments), QSV_ERANGE (qubit-count mismatch, or
 * the observable's tables exceed the array: nothing is enqueued), QSV_EHIP. */
int qsv_expectation_noalloc(const qsv_state* s, const qsv_observable* o, double* out);

/* out <- O in (out must be a different state of the same n and dtype): the
 * Pauli-string sum of section 4.5 applied to a state. Flip masks are packed
 * into tile passes as for qsv_expectation; each pass reads `in` once and adds
 * its masks' contributions to `out` (the first pass writes it). Asynchronous
 * on in's stream (out's stream is synchronised first if it differs). */
int qsv_apply_observable(const qsv_state* in, const qsv_observable* o, qsv_state* out);

/* ---------------------------------------------------------------- gradients */

/* Energy E = <psi|O|psi> of psi = U(theta)|0...0> and its gradient dE/dtheta
 * for every parameter slot of the circuit (ParametricRX/RY/RZ of section 4.4,
 * rotations exp(+i theta P/2)), by one forward pass and one reverse sweep that
 * uncomputes psi and lambda = O psi gate by gate (adjoint differentiation; the
 * paper defines the parametric circuits and observables, not this method).
 * psi, lam: caller-provided workspace states (same n as the circuit, same
 * dtype, distinct, same stream); on return psi holds |0...0> up to rounding.
 * forward_plan: optional fused plan of the same circuit and dtype for the
 * forward pass (NULL = one launch per gate). grad: circuit nparams doubles,
 * overwritten; a slot used by several gates receives the sum of their
 * contributions. Gradients accumulate in double. Parametric multi-qubit Pauli
 * rotations (qsv_circuit_add_pauli_rotation) are differentiated too. From 20
 * (complex64) / 19 (complex128) qubits the reverse sweep runs in tile passes
 * whose tables live in psi's work buffer (allocated on first use, kept,
 * freed with the state); Pauli strings on more than 5 qubits keep the
 * per-gate sweep. Synchronises the stream. */
int qsv_adjoint_gradient(const qsv_circuit* c, qsv_plan* forward_plan, const double* theta,
                         const qsv_observable* o, qsv_state* psi, qsv_state* lam,
                         double* energy, double* grad);

/* ---------------------------------------------------------------- batches */

/* A batch of independent items (circuit, observable, parameters) whose
 * energies and adjoint gradients are computed by ONE persistent kernel launch:
 * each workgroup takes items from a device work queue (largest first) and runs
 * forward pass, lambda = O psi, energy and reverse sweep for its item with the
 * item's states in LDS when psi and lambda fit in 64 KiB, else in device
 * memory streamed through LDS tiles in passes (several gates per pass, as in
 * qsv_plan_fused). The launch is captured once as a HIP graph and replayed
 * by later runs (qsv_batch_set_graph). This serves the regime the paper motivates -- small circuits
 * evaluated many times, where per-call overhead dominates (section 5.1) --
 * with a design of this library's own. Items take 2..24 qubits; their gates
 * must be one-qubit gates, rotations, CZ or CNOT (other gates: QSV_EINVAL at
 * run). The batch copies circuits, observables and parameters when added. */
int qsv_batch_create(qsv_batch** out);
int qsv_batch_free(qsv_batch* b);
int qsv_batch_add(qsv_batch* b, const qsv_circuit* c, const qsv_observable* o, const double* theta);

/* Replace the parameters of item `item` (the circuit's nparams doubles). */
int qsv_batch_set_theta(qsv_batch* b, int item, const double* theta);

/* Item count and the total parameter count (the length of the grads output). */
int qsv_batch_info(const qsv_batch* b, int* items, int* total_params);

/* Run every item in dtype `dtype` on `stream` (a hipStream_t, NULL = default).
 * energies: one double per item (in the order added). grads (nullable): the
 * items' gradients concatenated in the order added (item i occupies its
 * circuit's nparams entries). Device buffers are built on the first run for a
 * dtype and reused. Synchronises the stream. */
int qsv_batch_run(qsv_batch* b, qsv_dtype dtype, void* stream, double* energies, double* grads);

/* Launch-shape autotuner for the batch: times `reps` (1..100) runs of the
 * batch on `stream` for each candidate -- LDS for psi + lambda per workgroup
 * of 64 KiB (complex64 items up to 12 qubits held in LDS, 2^12-amplitude
 * tiles otherwise) or 32 KiB (2^11 tiles, more workgroups per CU) times 512 or
 * 256 threads per workgroup -- after one untimed run each, and keeps the
 * fastest for later runs. choice (may be NULL) receives int[2]: LDS KiB and
 * threads. Results do not depend on the shape beyond rounding order. Errors:
 * QSV_EINVAL (null or empty batch, reps out of range), QSV_EDTYPE, and those of
 * qsv_batch_run. */
int qsv_batch_autotune(qsv_batch* b, qsv_dtype dtype, void* stream, int reps, int* choice);

/* enable != 0 (the default): qsv_batch_run captures its launch (work-queue
 * reset kernel + persistent kernel) into a HIP graph on its first run for a
 * dtype and replays that graph afterwards; 0: plain launches every run (and
 * the captured graph is released). Parameter uploads and result copies stay
 * outside the graph. Results are identical either way. */
int qsv_batch_set_graph(qsv_batch* b, int enable);

#ifdef __cplusplus
}
#endif

#endif /* QSV_H_ */
