/*
 * qsim.h -- C ABI of the MI355X (gfx950) dense state-vector simulator.
 *
 * The library implements the hot path of the Qibo simulator (Efthymiou et al.,
 * arXiv:2009.01845): a dense vector of 2^n complex amplitudes updated in place
 * by gate matrices (Sec. 2.3, Eq. (1)), controlled gates (Sec. 2.4.1), gate
 * fusion (Sec. 2.4.5), Hamiltonian expectation values (Sec. 2.4.4),
 * measurement sampling (Sec. 2.4.2) and Trotterised adiabatic evolution
 * (Sec. 2.6, Eqs. (2)-(4)).  Beyond the paper it adds an adjoint gradient, a
 * batched persistent launch and a per-circuit tuner.
 *
 * Conventions shared by every call
 *  - Qubit q of an n-qubit state is index bit n-1-q: qubit 0 is the most
 *    significant bit of the flat index (the rank-N tensor psi(sigma_1..sigma_N)
 *    of Sec. 2.3 flattened in C order).
 *  - A state is 2^n contiguous interleaved (re, im) pairs of float (QS_C64) or
 *    double (QS_C128), i.e. the layout of torch.complex64 / complex128.
 *  - A k-qubit matrix is 2^k x 2^k complex128, row-major, interleaved
 *    (re, im), host memory, row index = output.  targets[0] is the most
 *    significant bit of the matrix index (G(tau, tau') of Eq. (1)).
 *  - A gate with controls acts only where every control qubit is 1.
 *  - Every host array argument is read during the call and not kept.
 *  - Calls that return host values (expectation, norm2, sample, download,
 *    adiabatic_run, adjoint, batch_run) synchronise the state's stream; the
 *    others only enqueue work on it.  Handles are not thread safe.
 *  - Every call returns a qs_status; on failure qs_last_error() holds a
 *    message for the calling thread.  No C++ exception crosses this ABI.
 *    Arguments are validated on the host before anything is enqueued.
 *    Asynchronous device errors surface as QS_E_DEVICE at the next
 *    synchronising call.
 */
#ifndef QSIM_H
#define QSIM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t qs_status;
#define QS_OK 0
#define QS_E_INVALID (-1)     /* bad argument: range, duplicates, null, dtype */
#define QS_E_NOMEM (-2)       /* device allocation failed or cap exceeded      */
#define QS_E_DEVICE (-3)      /* HIP runtime error                             */
#define QS_E_UNSUPPORTED (-4) /* not gfx950, or an operation it cannot do      */
#define QS_E_STATE (-5)       /* handle misuse (e.g. mismatched sizes)         */

typedef int32_t qs_dtype;
#define QS_C64 1
#define QS_C128 2

#define QS_MAX_QUBITS_C64 35
#define QS_MAX_QUBITS_C128 34
#define QS_MAX_GATE_QUBITS 5 /* k of a dense matrix */

typedef struct qs_state qs_state;
typedef struct qs_circuit qs_circuit;
typedef struct qs_obs qs_obs;
typedef struct qs_batch qs_batch;

/* Compilation options of a circuit (Sec. 2.4.5 gate fusion, extended).
 *   tile_bits  m: qubits held on chip by one tiled pass (0 = auto; 6..13).
 *   fuse_k     width of dense fused blocks (0 = auto, 1 = no dense fusion,
 *              2..5 = merge runs of gates into k-qubit matrices).
 *   use_mfma   -1 auto, 0 never, 1 apply 4- and 5-qubit fused blocks with
 *              matrix-core (MFMA) instructions.
 *   low_bits   L: lowest index bits always inside a tile (0 = auto).
 *   lane_ops   1: register stages also take uncontrolled one-qubit gates on
 *              the four lowest tile bits outside their registers, applied
 *              across lanes with DPP moves (fewer stages, more arithmetic);
 *              0 (default): register stages only. */
typedef struct qs_tune {
  int32_t tile_bits;
  int32_t fuse_k;
  int32_t use_mfma;
  int32_t low_bits;
  int32_t lane_ops;
  int32_t reserved[3];
} qs_tune;

const char* qs_version(void);
/* Message of the last failed call on this thread ("" if none). */
const char* qs_last_error(void);

/* ------------------------------------------------------------------ states
 * Sec. 2.3: the state is stored as a vector of 2^N components and updated in
 * place, so memory is the minimum 2^N complex numbers. */

/* Allocate a library-owned device state of 2^n amplitudes on the current HIP
 * device, set to |0..0>.  n in [1, 35] (C64) or [1, 34] (C128).  stream: a
 * hipStream_t (NULL = default stream) on which all work for this state is
 * enqueued.  QS_E_NOMEM if 2^n amplitudes do not fit (or exceed the byte cap
 * in the environment variable QS_MEM_LIMIT_BYTES). */
qs_status qs_state_create(int32_t n, qs_dtype dt, void* stream, qs_state** out);
/* Borrow caller device memory (e.g. a torch tensor): dev_ptr must hold 2^n
 * contiguous elements of dt, 16-byte aligned, and outlive the handle. */
qs_status qs_state_wrap(void* dev_ptr, int32_t n, qs_dtype dt, void* stream, qs_state** out);
/* Free the handle (and the buffer if the library owns it).  NULL is a no-op. */
qs_status qs_state_destroy(qs_state* s);
qs_status qs_state_info(const qs_state* s, int32_t* n, qs_dtype* dt, void** dev_ptr);
/* Basis state |x>, x < 2^n (x's bit n-1-q is qubit q). */
qs_status qs_state_set_basis(qs_state* s, uint64_t x);
/* Uniform superposition 2^(-n/2) sum_x |x>: the ground state of
 * H0 = -sum X_i (Sec. 2.6, Eq. (4)). */
qs_status qs_state_set_plus(qs_state* s);
/* Synchronous copies of the whole state between host and device. */
qs_status qs_state_upload(qs_state* s, const void* host_src);
qs_status qs_state_download(const qs_state* s, void* host_dst);
/* dst <- src (same n and dtype), enqueued on dst's stream. */
qs_status qs_state_copy(qs_state* dst, const qs_state* src);
/* Wait for all work enqueued on the state's stream. */
qs_status qs_state_sync(const qs_state* s);

/* Write the matrix of a named gate into out (room for 32x32 complex) and its
 * qubit count into k_out.  Names: H X Y Z S T RX RY RZ U1 SWAP (SWAP: k=2).
 * Rotations are exp(-i theta P/2); U1(theta) = diag(1, e^{i theta}).  The
 * paper's CZPow(t) (Sec. 3.1) is U1(pi t) with one control. */
qs_status qs_gate_matrix(const char* name, double theta, double* out, int32_t* k_out);

/* ------------------------------------------------------------ single gate
 * Eq. (1) with k = 1..5 targets and nctrl >= 0 controls, in place.
 * Invalid: qubit out of range, duplicates among targets+controls, k+nctrl > n,
 * null pointers.  The matrix is classified from exact zeros (diagonal,
 * generalised permutation, dense) and cast to the state precision. */
qs_status qs_apply(qs_state* s, const double* mat, int32_t k, const int32_t* targets,
                   int32_t nctrl, const int32_t* controls);

/* ---------------------------------------------------------------- circuits
 * Sec. 2.3: a circuit is a queue of gates executed in order on a state. */
qs_status qs_circuit_create(int32_t n, qs_circuit** out);
qs_status qs_circuit_add_gate(qs_circuit* c, const double* mat, int32_t k, const int32_t* targets,
                              int32_t nctrl, const int32_t* controls);
/* A trainable rotation exp(-i theta P / 2), P in {'X','Y','Z'}, with
 * theta = params[param_index] supplied at run time. */
qs_status qs_circuit_add_rot(qs_circuit* c, char pauli, int32_t target, int32_t param_index,
                             int32_t nctrl, const int32_t* controls);
/* Plan the circuit: fusion, tiled passes and (optionally) MFMA blocks
 * (Sec. 2.4.5).  opts may be NULL (automatic).  Host-only work; device
 * buffers are created at the first run.  Adding a gate after compile
 * invalidates the plan (the next run recompiles with the same options). */
qs_status qs_circuit_compile(qs_circuit* c, const qs_tune* opts);
/* Execute on s (same n).  params: nparams doubles, host memory unless
 * params_on_device != 0 (then a device pointer read by the kernels).
 * Asynchronous on s's stream. */
qs_status qs_circuit_run(qs_circuit* c, qs_state* s, const double* params, int32_t params_on_device);
/* Counts: user gates, planned passes over the state, parameter slots. */
qs_status qs_circuit_info(const qs_circuit* c, int32_t* ngates, int32_t* npasses, int32_t* nparams);
/* Describe pass i: kind (1 tile, 2 phase, 3 permutation, 4 mfma, 5 dense),
 * bits held on chip, ops applied. */
qs_status qs_circuit_pass_info(const qs_circuit* c, int32_t i, int32_t* kind, int32_t* tile_bits, int32_t* nops);
/* Which choice of high tile bits produced the current plan (Sec. 2.4.5
 * fusion taken to whole tiles; the planner builds up to three plans and keeps
 * the one with the fewest passes): 0 = the bits the next gates in list order
 * need, 1 = greedy lookahead by gates unlocked per added bit, 2 = one-step
 * rollout over every first choice.  QS_E_STATE if the circuit is not
 * compiled. */
qs_status qs_circuit_schedule(const qs_circuit* c, int32_t* schedule);
qs_status qs_circuit_destroy(qs_circuit* c);

/* -------------------------------------------------------- density matrices
 * Sec. 2.4.3: circuits that hold noise channels evolve a density matrix
 * instead of a state vector.  An n-qubit density matrix rho is an ordinary
 * qs_state of 2n qubits (4^n amplitudes, n <= 17 for QS_C64 and QS_C128 alike
 * within the 35/34 caps): rho[r][c] sits at flat index r * 2^n + c, so its
 * row index is held by state qubits 0..n-1 and its column index by state
 * qubits n..2n-1.  |x><x| is qs_state_set_basis(rho, x * 2^n + x).
 *
 * A density-matrix circuit takes qubit numbers of the n-qubit system.  Its
 * qs_circuit_add_gate(U) applies rho -> U rho U^dagger (U on the row qubits,
 * conj(U) on the column qubits), qs_circuit_add_rot the same for
 * exp(-i theta P/2), and qs_circuit_add_channel the map
 * rho -> sum_i K_i rho K_i^dagger.  qs_circuit_run / compile / info work as
 * for state vectors on the 2n-qubit rho; qs_adjoint and qs_batch_create
 * reject density-matrix circuits (QS_E_UNSUPPORTED). */
qs_status qs_circuit_create_density(int32_t n, qs_circuit** out);
/* Kraus operators K_0..K_{nkraus-1}: nkraus consecutive 2^k x 2^k complex128
 * matrices (row-major, interleaved, host), k in {1, 2}, nkraus in [1, 16],
 * targets[0] the most significant bit of each matrix index.  The map is
 * applied as given (trace preservation, sum_i K_i^dagger K_i = I, is the
 * caller's to ensure).  QS_E_STATE on a state-vector circuit. */
qs_status qs_circuit_add_channel(qs_circuit* c, int32_t nkraus, const double* kraus, int32_t k,
                                 const int32_t* targets);
/* Kraus operators of a named one-qubit channel (Nielsen & Chuang, Sec. 8.3),
 * written as *nkraus_out 2x2 complex128 matrices into out (room for 4):
 *   "depolarizing"       rho -> (1 - p) rho + p I/2
 *   "amplitude_damping"  |1> decays to |0> with probability p
 *   "phase_damping"      off-diagonal terms scaled by sqrt(1 - p)
 *   "bit_flip", "phase_flip"  X or Z with probability p
 * p in [0, 1]; *k_out (may be NULL) = 1. */
qs_status qs_channel_kraus(const char* name, double p, double* out, int32_t* nkraus_out, int32_t* k_out);
/* rho <- |psi><psi| (rho has 2n qubits of psi's n, same dtype); enqueued on
 * rho's stream after psi's stream has finished. */
qs_status qs_density_set_pure(qs_state* rho, const qs_state* psi);
/* Re Tr(H rho) in float64 for an observable H on the n-qubit system (Pauli
 * sum or Ising form); synchronises rho's stream. */
qs_status qs_density_expectation(const qs_state* rho, const qs_obs* H, double* out);
/* Re Tr(rho) in float64; synchronises rho's stream. */
qs_status qs_density_trace(const qs_state* rho, double* out);

/* ------------------------------------------------------------- observables
 * Sec. 2.4.4: energy = <psi|H|psi>.  H = sum_t coeffs[t] * P_t with each
 * strings[t] a NUL-terminated length-n word over {I,X,Y,Z}; character j acts
 * on qubit j.  Coefficients are real, so H is Hermitian. */
qs_status qs_pauli_sum_create(int32_t n, int32_t nterms, const double* coeffs,
                              const char* const* strings, qs_obs** out);
/* Diagonal Ising Hamiltonian E(z) = sum_{i<j} J[i*n+j] z_i z_j + sum_i h[i] z_i,
 * z_q = +1 for qubit q in |0> and -1 in |1> (only i<j entries of J are read). */
qs_status qs_ising_create(int32_t n, const double* J, const double* h, qs_obs** out);
qs_status qs_obs_destroy(qs_obs* o);
/* Real part of <psi|H|psi>, accumulated in float64, not divided by the norm. */
qs_status qs_expectation(const qs_state* s, const qs_obs* o, double* out);
/* Same, written to a device double; stays on the stream (no host sync). */
qs_status qs_expectation_async(const qs_state* s, const qs_obs* o, double* dev_out);
/* Same result as qs_expectation_async, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): this call performs no hipMalloc, hipFree or other
 * allocation.  Its partial sums go to a fixed workspace of the library, one
 * per GPU (about 1 MiB, held until the process ends), which fits an
 * observable with at most 64 reduction slots (one for all diagonal terms, one
 * per tile set and one per far flip group); a larger observable returns
 * QS_E_INVALID.  The observable's own tables must already be on the device:
 * one qs_expectation or qs_expectation_async call with it uploads them;
 * otherwise QS_E_STATE.  dev_out is a device double written on s's stream
 * (no host sync).  Every call on one GPU shares that workspace, and the
 * kernels clear what they accumulate into at the start of each call: calls
 * that overlap on one GPU (other streams, other threads) race and may return
 * wrong values; serialise them. */
qs_status qs_expectation_noalloc(const qs_state* s, const qs_obs* o, double* dev_out);
/* <psi|psi> in float64. */
qs_status qs_norm2(const qs_state* s, double* out);

/* ---------------------------------------------------------------- sampling
 * Sec. 2.4.2: sample the outcome distribution of the measured qubits (the
 * trace-out of |psi|^2 over the others).  Shot j draws
 *   x_j = min{ x : CDF(x) > u_j * CDF(2^n - 1) }   (natural index order, f64)
 * and out[j] holds the measured bits of x_j, qubits[0] as the most
 * significant bit.  uniforms (host, shots values in [0,1)) may be NULL: then
 * u_j comes from Philox4x32-10 (Salmon et al., SC'11) with counter
 * (j mod 2^32, j div 2^32, 0, 0), key (seed mod 2^32, seed div 2^32),
 * u_j = ((w0 << 32 | w1) >> 11) * 2^-53.  m in [1, min(n, 63)]. */
qs_status qs_sample(const qs_state* s, int32_t m, const int32_t* qubits, int64_t shots, uint64_t seed,
                    const double* uniforms, int64_t* out);

/* ----------------------------------------------------- adiabatic evolution
 * Sec. 2.6, Eq. (3): H(s) = (1 - s) H0 + s H1, H0 = -sum X_i, s = t/T.
 * h1 must be an Ising observable.  order = 2: per step k, with
 * s_k = (k + 1/2) dt / T: RX(-(1 - s_k) dt) on every qubit, the phase
 * exp(-i s_k dt E(x)), RX(-(1 - s_k) dt) again (adjacent RX halves merged).
 * The state is evolved in place from whatever it holds (use set_plus for
 * the ground state of H0).  energy_out (may be NULL) receives <H1> at the end.
 * The pass plans of the Trotter blocks are built at the first run with h1 in
 * a precision and kept in h1 for later runs (freed by qs_obs_destroy): runs
 * that share h1 must not overlap (one host thread at a time). */
qs_status qs_adiabatic_run(qs_state* s, const qs_obs* h1, double T, double dt, int32_t order,
                           double* energy_out);

/* ------------------------------------------------------------- callbacks
 * Sec. 2.4.4: quantities computed on intermediate states during an
 * evolution.  After every `every` time steps (steps every, 2 every, ...,
 * K = T/dt of them in all) the run records, into entry i of the host arrays:
 *   energies[i]  = Re <psi|energy|psi> (float64), if energy is not NULL;
 *   entropies[i] = the entanglement entropy of qubits 0..entropy_qubits-1
 *                  against the rest (see qs_entanglement_entropy), if
 *                  entropy_qubits > 0.
 * Each array needs room for K / every values (integer division). */
typedef struct qs_callbacks {
  int32_t every;
  int32_t entropy_qubits;
  const qs_obs* energy;
  double* energies;
  double* entropies;
} qs_callbacks;

/* Entanglement entropy -Tr(rho_A ln rho_A) of the first a qubits (qubits
 * 0..a-1), rho_A = M M^dagger with M = psi viewed as a 2^a x 2^(n-a) matrix
 * (rho_A is not renormalised; eigenvalues below 1e-15 contribute nothing).
 * The Gram matrix of the smaller side is formed on the GPU (complex128
 * matrix-core products) and its eigenvalues on the host, so
 * min(a, n - a) <= 10.  a in [1, n-1].  Synchronises the state's stream. */
qs_status qs_entanglement_entropy(const qs_state* s, int32_t a, double* out);

/* Same as qs_adiabatic_run, recording the callbacks (cb may be NULL).  The
 * run is split at the callback steps: each segment closes its last half
 * rotation layer, so the recorded states are the Trotter states after those
 * steps. */
qs_status qs_adiabatic_run_callbacks(qs_state* s, const qs_obs* h1, double T, double dt, int32_t order,
                                     const qs_callbacks* cb, double* energy_out);

/* ---------------------------------------------------------- ODE evolution
 * Sec. 2.6: integrate i dpsi/dt = H(t) psi with H(t) = (1 - t/T) h0 + (t/T) h1
 * (h0, h1 any observables of the state's n) over K = T/dt steps, in place.
 *   QS_SOLVER_EXP   each step multiplies psi by exp(-i H(s_k) dt), H at the
 *                   step midpoint s_k = (k + 1/2) dt / T, built as a dense
 *                   2^n x 2^n complex128 matrix; the exponential by scaling
 *                   and squaring of its Taylor series (terms until the
 *                   remainder bound is below 1e-18), every product on FP64
 *                   matrix cores.  n <= 12.
 *   QS_SOLVER_RK4   classical four-stage Runge-Kutta on the continuous
 *                   schedule, H psi applied term by term from the Pauli sums.
 *   QS_SOLVER_RK45  Dormand-Prince 5(4) tableau with the fixed step dt,
 *                   advancing the fifth-order solution.
 * The Runge-Kutta solvers keep 2 + (4 or 7) state-sized buffers.  cb may be
 * NULL.  Synchronises the state's stream. */
#define QS_SOLVER_EXP 1
#define QS_SOLVER_RK4 2
#define QS_SOLVER_RK45 3
qs_status qs_evolve(qs_state* s, const qs_obs* h0, const qs_obs* h1, double T, double dt, int32_t solver,
                    const qs_callbacks* cb);

/* ---------------------------------------------------------------- gradient
 * Adjoint differentiation (Jones & Gacon 2020; not in the paper): on entry
 * psi holds the output of qs_circuit_run(c, psi, params); lambda is a second
 * state of the same n and dtype used as scratch.  Writes dE/dparams (nparams
 * doubles, host) for E = <psi|H|psi> and the energy E itself.  On exit psi
 * holds the circuit's input state up to rounding.  Every gate must be
 * unitary. */
qs_status qs_adjoint(qs_circuit* c, const double* params, const qs_obs* H, qs_state* psi,
                     qs_state* lambda, double* grad_out, double* energy_out);

/* ------------------------------------------------------------------- batch
 * Many small circuits (each with its own n <= 24, parameters and diagonal
 * observable) evaluated together; each instance starts from |0..0>.  The
 * work runs level by level: one launch applies pass k of every instance that
 * has it, one workgroup per tile of each instance, so a large instance is
 * spread over as many workgroups as it has tiles; then the energies and
 * lambda = H psi, then the adjoint levels in reverse.  The first run of each
 * kind (with or without gradients) captures that launch sequence as a HIP
 * graph; later runs replay it after uploading new parameters.
 * stream: the HIP stream to run on, or NULL for a stream the batch creates
 * and owns.  The batch borrows the circuit and observable handles: they must
 * outlive it.  params_packed holds every instance's parameters back to back in
 * instance order; energies gets count doubles; grads (may be NULL: then the
 * adjoint levels are skipped) gets the gradients packed like params.  Runs
 * synchronise the batch's stream. */
qs_status qs_batch_create(int32_t count, qs_circuit* const* circs, const qs_obs* const* obs, qs_dtype dt,
                          void* stream, qs_batch** out);
qs_status qs_batch_run(qs_batch* b, const double* params_packed, double* energies, double* grads);
qs_status qs_batch_destroy(qs_batch* b);
/* Tune a batch per size class (the instances with one qubit count): each
 * candidate (the circuits' own options, lane ops, low runs of 2^5
 * amplitudes, 10- and 11-bit tiles, two-qubit fusion) is run on a batch of
 * that class alone, its launch sequence replayed as a graph and timed; the
 * fastest whose energies and gradients agree with the first candidate's
 * (1e-4 complex64, 1e-9 complex128) is kept, and the batch is rebuilt with
 * each instance's choice.  params_packed as for qs_batch_run.  cache_path
 * (may be NULL): a text file of earlier choices, one line per class key
 * (qubit count, instance count, dtype, device, circuit hash), read first and
 * appended to.  The batch's circuits and observables must still exist. */
qs_status qs_batch_autotune(qs_batch* b, const double* params_packed, const char* cache_path);
/* The options instance i of the batch runs with (after qs_batch_autotune, its
 * class's choice; before, its circuit's own). */
qs_status qs_batch_choice(const qs_batch* b, int32_t i, qs_tune* out);

/* ------------------------------------------------------------------- tuner
 * Time the candidate plans (fusion width 0, 2..5, MFMA on/off) of c on
 * state s, keep the fastest whose result from |+...+> agrees with the
 * default plan's (2-norm distance below 1e-4 for complex64, 1e-9 for
 * complex128), and compile c with it.  cache_path (may be NULL) is a text
 * file of previous choices, one line per key (n, gate count, dtype, device
 * architecture, 64-bit hash of the gate list); a hit skips the timing, a miss
 * appends a line.  Needs one extra state-sized device buffer while it runs.
 * The state's contents are destroyed. */
qs_status qs_autotune(qs_circuit* c, qs_state* s, const double* params, const char* cache_path);

/* --------------------------------------------------------------- profiling
 * When enabled, every kernel launch is bracketed by HIP events on its own
 * stream; qs_profile_read returns, per kernel family, the launch count and
 * the summed device milliseconds since the last reset (it synchronises).
 * Families: 0 tile, 1 phase, 2 permutation, 3 mfma, 4 dense, 5 reduce,
 * 6 sample, 7 adjoint, 8 batch, 9 other. */
qs_status qs_profile_enable(int32_t on);
qs_status qs_profile_reset(void);
qs_status qs_profile_read(int32_t family, int64_t* launches, double* total_ms);

#ifdef __cplusplus
}
#endif
#endif /* QSIM_H */
