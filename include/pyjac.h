/*
 * pyjac.h -- C ABI of libpyjac_mi355x.so, an MI355X (gfx950) library for the
 * data-parallel hot path of the analytical chemical-kinetics Jacobian of
 * Niemeyer, Curtis & Sung, "pyJac: analytical Jacobian generator for chemical
 * kinetics" (arXiv:1605.03262): reaction rates, species production rates, the
 * constant-pressure ideal-gas source terms and their dense analytical Jacobian,
 * evaluated for very many independent thermochemical states, plus a batched
 * solve of the Newton matrix I - h*gamma*J.
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Units are SI with kmol: T [K], p [Pa], Y [-], t [s], concentrations
 *    [kmol/m^3], rates of progress [kmol/(m^3 s)].  All floating point is FP64
 *    unless stated.
 *  - State vector (Sec. 2.1, Eq. vars): Phi = {T, Y_1, ..., Y_{N-1}}; the last
 *    species' mass fraction is Y_N = 1 - sum Y_k (Eq. y_nsp) and is not stored.
 *  - Layout: every per-state array is element-major with the state index
 *    fastest: element e of state s lives at ptr[e*ld + s], ld >= n_states.
 *      phi  [N][ld]        e = 0 is T, e = j (1..N-1) is Y_j
 *      p    [ld]           pressure, held constant (Sec. 2.1 footnote)
 *      jac  [N*N][ld]      e = i*N + j holds J_ij = d f_i / d Phi_j (Sec. 3.1)
 *  - Array arguments of the evaluation calls are DEVICE pointers owned by the
 *    caller (e.g. a torch tensor's data_ptr()).  Every double pointer must be
 *    8-byte aligned.
 *  - stream is a hipStream_t passed as void*; NULL means the default stream.
 *    Evaluation calls only enqueue work and return; results are ready when the
 *    stream reaches that point.  Argument errors are reported synchronously
 *    and nothing is enqueued; a failed launch returns PYJAC_E_DEVICE.
 *  - Numerical trouble in a state (non-finite inputs, T outside the thermo
 *    fits, a singular Newton matrix) never fails a call: it shows up as
 *    non-finite outputs or in the per-state info array.
 *  - The result for a state depends only on that state's inputs and the
 *    mechanism: never on n_states, ld, the stream or other states in the
 *    batch (no atomics, fixed reduction order).
 *  - A const pyjac_mech* may be used concurrently from many host threads and
 *    streams; pyjac_mech_free must not race with calls using the handle.
 *  - pyjac_last_error() returns a thread-local message for the most recent
 *    failing call on the calling thread.
 */
#ifndef PYJAC_MI355X_H
#define PYJAC_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pyjac_mech pyjac_mech;   /* opaque; owns device-resident tables */
typedef int32_t pyjac_status;

#define PYJAC_OK              0
#define PYJAC_E_INVALID      -1   /* bad argument (NULL, negative size, ld < n, misaligned) */
#define PYJAC_E_PARSE        -2   /* malformed mechanism text */
#define PYJAC_E_UNSUPPORTED  -3   /* feature outside the supported set */
#define PYJAC_E_DEVICE       -4   /* HIP runtime or launch failure */
#define PYJAC_E_NOMEM        -5   /* device or host allocation failed */
#define PYJAC_E_IO           -6   /* file could not be read */
#define PYJAC_E_UNBALANCED   -7   /* a reaction does not conserve elements */
#define PYJAC_E_WORKSPACE    -8   /* Newton workspace too small */

/* Load a mechanism from the project's whitespace-separated token format
 * ("pyjac-mech 1", then elements with atomic weights, species with
 * composition, T_mid and 2x7 NASA-7 coefficients, and reactions of the
 * classes of Sec. 2.3: elementary, third-body, Lindemann/Troe/SRI falloff and
 * chemically activated, PLOG, Chebyshev; reverse rates via K_c, explicit
 * Arrhenius or irreversible; SI-kmol units, activation as T_a in K).  Validates element balance and supported
 * features, packs device tables on HIP device `hip_device` and returns an
 * owned handle in *out.  Errors: PYJAC_E_IO, _PARSE, _UNSUPPORTED,
 * _UNBALANCED, _NOMEM, _DEVICE; *out is left NULL on error. */
pyjac_status pyjac_mech_load(const char* path, int32_t hip_device, pyjac_mech** out);

/* Same as pyjac_mech_load, from a NUL-terminated text buffer. */
pyjac_status pyjac_mech_load_string(const char* text, int32_t hip_device, pyjac_mech** out);

/* Chemkin-format mechanisms (host only).  Converts Chemkin-II text (ELEMENTS,
 * SPECIES, REACTIONS and an optional THERMO block) into the token format
 * above.  `thermo_text` holds the NASA-7 records when they are not in
 * mech_text (NULL otherwise).  Covered: the reaction classes of Sec. 2.3 as
 * "+M" third-body, "(+M)"/"(+X)" falloff with LOW (or chemically activated
 * with HIGH) and TROE/SRI, PLOG and CHEB/TCHEB/PCHEB, REV, efficiencies and
 * DUPLICATE; units CAL/MOLE (default), KCAL/MOLE, JOULES/MOLE, KJOULES/MOLE,
 * KELVINS, EVOLTS with MOLES.  A in cm-mol-s is scaled to SI-kmol by
 * 1e-3^(order-1) (order = molecularity of that coefficient, counting [M]),
 * pressures from atm to Pa.  Elements without an explicit "/weight/" take
 * the IUPAC abridged standard atomic weight.
 * Output: when `out` is NULL only *out_len is set (bytes including the
 * terminating NUL); otherwise the text is written if out_capacity >= *out_len.
 * Errors: PYJAC_E_INVALID (NULL mech_text/out_len, buffer too small),
 * PYJAC_E_PARSE (with the line number in pyjac_last_error), PYJAC_E_UNSUPPORTED
 * (e.g. MOLECULES units, FORD/RORD, fractional element counts). */
pyjac_status pyjac_chemkin_to_text(const char* mech_text, const char* thermo_text, char* out,
                                   size_t out_capacity, size_t* out_len);

/* Reads a Chemkin-format mechanism file (and a separate thermo file, or NULL),
 * converts it as pyjac_chemkin_to_text does and loads it as pyjac_mech_load. */
pyjac_status pyjac_mech_load_chemkin(const char* mech_path, const char* thermo_path, int32_t hip_device,
                                     pyjac_mech** out);

/* Sizes and a 64-bit content hash of the parsed mechanism (any out may be
 * NULL): N species and N_R reactions as in Sec. 2 (the state has N entries,
 * Eq. vars, and the Jacobian N x N). */
pyjac_status pyjac_mech_info(const pyjac_mech* mech, int32_t* n_species, int32_t* n_reactions,
                             uint64_t* content_hash);

/* Synchronizes the mechanism's device, then frees its tables (the per-mechanism
 * data of Sec. 2.2-2.3 held on the device) and the handle.  NULL is accepted
 * and ignored. */
pyjac_status pyjac_mech_free(pyjac_mech* mech);

/* Reaction rates, production rates and the RHS (Sec. 2.1 Eqs. ode/dTdt,
 * Sec. 2.3).  For each of n_states states reads phi[N][ld], p[ld] and writes
 * whichever outputs are non-NULL:
 *   rop_f    [N_R][ld]  forward rate of progress  R_f,i = k_f,i prod [X_j]^nu'_ji
 *   rop_r    [N_R][ld]  reverse rate of progress  R_r,i = k_r,i prod [X_j]^nu''_ji
 *   pres_mod [N_R][ld]  pressure modification c_i (Eq. rxn_pressure; 1 for
 *                       elementary, PLOG and Chebyshev reactions)
 *   wdot     [N][ld]    species production rates wdot_k = sum_i nu_ki c_i (R_f,i - R_r,i)
 *   dphi     [N][ld]    f = dPhi/dt: dT/dt and dY_k/dt for k = 1..N-1
 * Reaction index i is the order of the mechanism file.  n_states == 0 is a
 * no-op.  Errors: PYJAC_E_INVALID (NULL mech/phi/p, n_states < 0, ld < n_states,
 * misaligned pointer, wrong device), PYJAC_E_DEVICE. */
pyjac_status pyjac_eval_rates(const pyjac_mech* mech, int64_t n_states, int64_t ld,
                              const double* phi, const double* p, double* rop_f, double* rop_r,
                              double* pres_mod, double* wdot, double* dphi, void* stream);

/* Dense analytical Jacobian J = df/dPhi of the constant-pressure RHS
 * (Sec. 3.1 elements, Sec. 3.2 evaluation order with the last-species
 * placeholder row, Sec. 3.3: the matrix is dense).  Writes jac[N*N][ld]
 * (row i = equation, column j = state variable; row/column 0 is temperature).
 * Errors as pyjac_eval_rates; jac must be non-NULL. */
pyjac_status pyjac_eval_jacobian(const pyjac_mech* mech, int64_t n_states, int64_t ld,
                                 const double* phi, const double* p, double* jac, void* stream);

/* One batch of a multi-mechanism Jacobian launch. */
typedef struct pyjac_work_item {
  const pyjac_mech* mech;
  int64_t n_states, ld;
  const double* phi;   /* [N][ld] device */
  const double* p;     /* [ld] device */
  double* jac;         /* [N*N][ld] device */
} pyjac_work_item;

/* The Jacobians of several batches, possibly of different mechanisms, in one
 * kernel launch (per state the same values, bitwise, as pyjac_eval_jacobian):
 * the grid is a work list whose blocks map to (item, tile) pairs, each block
 * reading its item's mechanism tables.  Every mechanism must currently use
 * the same Jacobian launch shape (pyjac_mech_get_variant / set_variant) and
 * column-stream form; the items go out in launches of at most 8.  The item
 * array is read during the call (host memory, caller-owned); nothing is
 * allocated or copied, so the launch can be captured into a HIP graph.
 * Errors: as pyjac_eval_jacobian per item, PYJAC_E_UNSUPPORTED when the items
 * do not share a launch shape; nothing is enqueued on an error. */
pyjac_status pyjac_eval_jacobian_multi(int32_t n_items, const pyjac_work_item* items, void* stream);

/* Sparse Jacobian of the concentration-based, constant-volume formulation
 * that Sec. 3.3 names as the route to Jacobian sparsity (concentrations as
 * state variables remove the density from the cross-species elements) and
 * Sec. 6 plans.  State per state s: phi_c[(N+1)][ld] = {T, [X_1], ..., [X_N]}
 * (K, kmol/m^3), constant volume, p = R T sum [X_k] (Eq. state) in the PLOG
 * and Chebyshev rates; the ODE is d[X_k]/dt = wdot_k (Sec. 2.3 rate laws) and
 * dT/dt = -sum_k U_k wdot_k / sum_k [X_k] C_v,k with molar U_k = H_k - R T,
 * C_v,k = C_p,k - R (Sec. 2.2 polynomials).  The species block is stored as a
 * dense vector u plus a sparse matrix S with the fixed compressed-column
 * pattern of pyjac_conc_pattern: J_{k,j} = u_k + S_{k,j} (u collects the
 * all-species third-body baseline and the pressure dependence; S the
 * mass-action and non-unit-efficiency terms).  jac[(3N+1+nnz)][ld]:
 *   e = 0            d(dT/dt)/dT
 *   e = 1 .. N       d wdot_k/dT,            k = e - 1
 *   e = N+1 .. 2N    d(dT/dt)/d[X_j],        j = e - N - 1
 *   e = 2N+1 .. 3N   u_k,                     k = e - 2N - 1
 *   e = 3N+1 + q     S value q: column j holds q in [colptr[j], colptr[j+1]),
 *                    row rowidx[q] (ascending within a column)
 * Errors: PYJAC_E_INVALID (NULL arrays, n < 0, ld < n, misaligned, wrong
 * device), PYJAC_E_UNSUPPORTED (mechanism too large for the tile),
 * PYJAC_E_DEVICE.  n_states == 0 is a no-op. */
pyjac_status pyjac_eval_jacobian_conc(const pyjac_mech* mech, int64_t n_states, int64_t ld,
                                      const double* phi_c, double* jac, void* stream);

/* Host copy of the compressed-column pattern of S above: colptr[N+1] and
 * rowidx[nnz] (either may be NULL; *nnz, if given, receives nnz).  Caller-owned
 * host arrays. */
pyjac_status pyjac_conc_pattern(const pyjac_mech* mech, int32_t* colptr, int32_t* rowidx, int64_t* nnz);

/* Finite-difference Jacobian: the first-order forward-difference
 * approximation the paper measures the analytical Jacobian against (Sec. 5,
 * finite differences as in CVODE).  Column j of state s is
 * (f(Phi + d_j e_j) - f(Phi)) / d_j with f the RHS of pyjac_eval_rates and
 * d_j = (Phi_j + inc_j) - Phi_j, inc_j = 2^-26 max(|Phi_j|, floor_j) (floor
 * 1 K for T, 1e-10 for mass fractions).  Same layout as pyjac_eval_jacobian.
 * States are processed in chunks as large as the workspace allows
 * (pyjac_fd_workspace_bytes(mech, c) holds a chunk of c states); each chunk
 * evaluates the RHS kernel on c*(N+1) states.  Errors: as
 * pyjac_eval_jacobian, PYJAC_E_WORKSPACE if not even one state fits. */
size_t pyjac_fd_workspace_bytes(const pyjac_mech* mech, int64_t chunk_states);
pyjac_status pyjac_eval_jacobian_fd(const pyjac_mech* mech, int64_t n_states, int64_t ld, const double* phi,
                                    const double* p, double* jac, void* workspace, size_t workspace_bytes,
                                    void* stream);

/* One implicit integrator step per state (the consumer of J + Newton that
 * motivates fast Jacobians, Sec. 1): the three-stage, L-stable, stiffly
 * accurate SDIRK method of order 3 (Alexander, 1977) with diagonal
 * coefficient gamma = 0.43586652150845899942, a_21 = (1 - gamma)/2,
 * a_31 = -(6 gamma^2 - 16 gamma + 1)/4, a_32 = (6 gamma^2 - 20 gamma + 5)/4,
 * a_33 = gamma, y_next = y + z_3.  Stage i solves
 * z_i = h sum_{j<i} a_ij f(y + z_j) + h gamma f(y + z_i) by simplified Newton
 * with the matrix I - h gamma J(y) (one Jacobian per step), starting from
 * z_i = 0, for exactly newton_iters iterations; each iteration evaluates the
 * RHS and calls pyjac_newton_factor_solve (mode 0 FP64, 1 FP32 LU + FP64
 * refinement with max_refine 4, rtol 1e-14); every solve after the step's
 * first passes PYJAC_NEWTON_REUSE_FACTOR (the first, KEEP), so in mode 0
 * the matrix is factored once per step (mode 1 with N <= 64: once per solve).
 * phi [N][ld] at constant pressure p [ld] with step h [ld] (seconds) ->
 * phi_out [N][ld] (may alias phi).  dnorm [3][ld] (or NULL) receives each
 * stage's last Newton increment max_e |dz_e|, a convergence indicator.
 * workspace: device memory of pyjac_sdirk3_workspace_bytes(mech, n, ld, mode).
 * n_states == 0 is a no-op (the arrays may then be NULL).  Errors:
 * PYJAC_E_INVALID (NULL arrays, n < 0, ld < n, newton_iters outside [1, 16],
 * bad mode), PYJAC_E_WORKSPACE, and those of the calls it makes. */
size_t pyjac_sdirk3_workspace_bytes(const pyjac_mech* mech, int64_t n_states, int64_t ld, int32_t mode);
pyjac_status pyjac_sdirk3_step(const pyjac_mech* mech, int64_t n_states, int64_t ld, const double* phi,
                               const double* p, const double* h, int32_t newton_iters, int32_t mode,
                               double* phi_out, double* dnorm, void* workspace, size_t workspace_bytes,
                               void* stream);

/* Complex-step Jacobian of the same constant-pressure RHS: column j of state
 * s is Im f(Phi + i step e_j) / step, with every operation of the RHS
 * (Sec. 2.1, Sec. 2.3 rate laws) in complex arithmetic and branch decisions
 * on real parts.  Exact to rounding for any small step (no difference of
 * nearby values), it is an accuracy reference of the kind Sec. 5.1 discusses,
 * next to finite differences; it costs N complex RHS evaluations per state.
 * Same arguments and layout as pyjac_eval_jacobian, plus step in (0, 1e-6]
 * (1e-30 is typical).  Errors: as pyjac_eval_jacobian, PYJAC_E_UNSUPPORTED
 * for more than 384 species. */
pyjac_status pyjac_eval_jacobian_cs(const pyjac_mech* mech, int64_t n_states, int64_t ld, const double* phi,
                                    const double* p, double step, double* jac, void* stream);

/* Mixing fractional step of a partially stirred reactor (App. C): for every
 * particle s with partner q = partner[s] (0 <= q < n_states; a negative value
 * leaves s unchanged), the mixture enthalpy h and the mass fractions relax
 * towards the partner's, x_s <- x_s - weight (x_s - x_q) with weight =
 * (1 - exp(-2 dt_sub / tau_mix)) / 2 in [0, 1/2], and the temperature is
 * recovered from the mixed enthalpy (Newton on h(T) = sum_k Y_k h_k(T),
 * Sec. 2.2).  phi, phi_out [N][ld] as pyjac_eval_rates' phi (phi_out must not
 * alias phi: both members of a pair read the old states); partner [ld] int32
 * device array.  Pairs are symmetric in the PaSR driver, so the pair's
 * enthalpy and mass are conserved.  Errors: PYJAC_E_INVALID,
 * PYJAC_E_UNSUPPORTED (more than 1024 species), PYJAC_E_DEVICE. */
pyjac_status pyjac_mix_pairs(const pyjac_mech* mech, int64_t n_states, int64_t ld, const double* phi,
                             const int32_t* partner, double weight, double* phi_out, void* stream);

/* Bytes of device workspace pyjac_newton_factor_solve needs for n_states
 * states in `mode` (0 or 1; with PYJAC_NEWTON_KEEP_FACTOR including the kept
 * factor's storage; PYJAC_NEWTON_REUSE_FACTOR is ignored here).
 * Returns 0 for a bad handle or mode. */
size_t pyjac_newton_workspace_bytes(const pyjac_mech* mech, int64_t n_states, int32_t mode);

/* Batched solve of the Newton system of an implicit integrator step (the
 * consumer of the Jacobian that Sec. 1 gives as the method's motivation:
 * implicit integration of stiff chemistry needs J for its Newton iterations),
 * A x = rhs with A = I - h_s * gamma * J_s for every state s (N x N, FP64
 * Jacobian as written by pyjac_eval_jacobian, same layout and ld).
 *   h      [ld]      per-state step size
 *   rhs    [N][ld]   right-hand side b
 *   x      [N][ld]   solution (may not alias rhs or jac)
 *   mode 0: LU with partial pivoting in FP64.
 *   mode 1: LU with partial pivoting in FP32 (on the matrix cores for
 *           N > 64; for N <= 64 in registers, several states per wavefront),
 *           FP64 residual r = b - A x and up to max_refine refinement sweeps,
 *           until ||dx||_inf <= rtol * ||x||_inf, or, from the second sweep,
 *           until the contraction rho = ||dx_k|| / ||dx_k-1|| < 1/2 predicts
 *           the remaining error rho / (1 - rho) ||dx_k||_inf <= rtol *
 *           ||x||_inf; a state that does not converge is re-solved in FP64
 *           (counted in info).
 *   info   [ld]      >= 0: refinement sweeps used (mode 1; 0 for mode 0);
 *                    -1: zero pivot (singular A); -2: mode-1 state fell back to
 *                    FP64 and converged there; -3: non-finite input.
 * workspace must hold pyjac_newton_workspace_bytes(mech, n_states, mode)
 * device bytes (it may be NULL when that is 0).
 * mode | PYJAC_NEWTON_REUSE_FACTOR: solve with the factor that the previous
 * call with the same jac, h, gamma, n_states, ld and mode left in this
 * workspace, skipping the formation and factorization of A (for the several
 * solves of one implicit step).  The caller guarantees that nothing else
 * used the workspace in between and orders the calls on one stream.  Only
 * the blocked path (N > 64) keeps its factor in the workspace on its own;
 * for N <= 64 (mode 0) the factoring call must have passed
 * PYJAC_NEWTON_KEEP_FACTOR (mode 1: the flag is accepted and the system is
 * factored again).  States that fall back to FP64 in mode 1 are always
 * factored again.  Errors: PYJAC_E_INVALID, PYJAC_E_WORKSPACE, PYJAC_E_DEVICE. */
#define PYJAC_NEWTON_REUSE_FACTOR 16
/* mode | PYJAC_NEWTON_KEEP_FACTOR: keep the FP64 factor of the register
 * path (N <= 64, mode 0) in the workspace for later REUSE calls; the
 * workspace must then hold pyjac_newton_workspace_bytes(mech, n, mode |
 * PYJAC_NEWTON_KEEP_FACTOR) bytes (N^2-sized per state).  The blocked path
 * always keeps its factor; on the register path in mode 1 the flag is
 * accepted and the system factored on every call. */
#define PYJAC_NEWTON_KEEP_FACTOR 32
pyjac_status pyjac_newton_factor_solve(const pyjac_mech* mech, int64_t n_states, int64_t ld,
                                       const double* jac, const double* h, double gamma,
                                       const double* rhs, double* x, int32_t mode,
                                       int32_t max_refine, double rtol, int32_t* info,
                                       void* workspace, size_t workspace_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * solve as pyjac_newton_factor_solve (same kernels, same results bit for bit)
 * with its workspace taken from a static device array of
 * PYJAC_NEWTON_STATIC_SCRATCH_BYTES held by each GPU the library runs on until
 * the process ends.  No allocation of any kind happens in the call.
 * mode is 0 or 1 only (the factor-keeping flags are refused, since every call
 * on a GPU shares that GPU's array).  Calls that overlap on one GPU (other
 * streams or host threads) race on the array: order them.  Errors:
 * PYJAC_E_WORKSPACE when n_states needs more than the array holds
 * (pyjac_newton_workspace_bytes(mech, n_states, mode) >
 * PYJAC_NEWTON_STATIC_SCRATCH_BYTES), otherwise as pyjac_newton_factor_solve. */
#define PYJAC_NEWTON_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
pyjac_status pyjac_newton_factor_solve_noalloc(const pyjac_mech* mech, int64_t n_states, int64_t ld,
                                               const double* jac, const double* h, double gamma,
                                               const double* rhs, double* x, int32_t mode,
                                               int32_t max_refine, double rtol, int32_t* info,
                                               void* stream);

/* Tuning: force the launch shape of one kernel family of this handle
 * (which = 0: rates kernel, 1: Jacobian kernel, 2: concentration-form
 * Jacobian) to tile_states states per
 * workgroup and `threads` threads per workgroup; tile_states = 0 restores the
 * automatic choice (largest tile whose LDS working set fits the device).
 * Results per state do not depend on the shape (all per-state sums run in
 * species order).  Not thread-safe against
 * concurrent evaluation calls on the same handle.  Errors: PYJAC_E_INVALID,
 * PYJAC_E_UNSUPPORTED (shape not compiled or does not fit). */
pyjac_status pyjac_mech_set_variant(pyjac_mech* mech, int32_t which, int32_t tile_states,
                                    int32_t threads);

/* Autotuner: times every compiled launch shape of one kernel family
 * (which = 0: rates kernel writing the RHS only, 1: Jacobian kernel, 2:
 * concentration-form Jacobian) that fits the device and the mechanism, on the
 * caller's own batch (n_states states of phi[N][ld], p[ld], output written to
 * out: [N][ld] doubles for which = 0, [N*N][ld] for which = 1; for which = 2
 * phi is phi_c[(N+1)][ld], p is ignored (may be NULL) and out holds
 * [(3N+1+nnz)][ld]), `reps` timed launches each after one warm-up,
 * and keeps the fastest median for this handle (a shape later in the
 * preference order must be at least 2 % faster to win).  Every launch is ordered on
 * `stream` and the call returns after the last one has finished.  Optional
 * report: up to max_entries (tile_states, threads) pairs in shapes[2*e],
 * their median milliseconds in ms[e], and the count in *n_entries.  Since
 * results per state do not depend on the shape, tuning never changes
 * answers.  Not thread-safe against concurrent calls on the same handle.
 * Errors: as pyjac_eval_jacobian / pyjac_eval_rates, PYJAC_E_INVALID for
 * reps < 1 or n_states < 1, PYJAC_E_DEVICE if timing fails. */
pyjac_status pyjac_mech_autotune(pyjac_mech* mech, int32_t which, int64_t n_states, int64_t ld,
                                 const double* phi, const double* p, double* out, int32_t reps,
                                 int32_t* shapes, float* ms, int32_t max_entries,
                                 int32_t* n_entries, void* stream);

/* Current launch shape of a kernel family and its dynamic LDS bytes. */
pyjac_status pyjac_mech_get_variant(const pyjac_mech* mech, int32_t which, int32_t* tile_states,
                                    int32_t* threads, size_t* lds_bytes);

/* ------------------------------------------------------------------------
 * Serving: continuous batching of Jacobian + Newton requests (the consumer of
 * Sec. 1: many independent implicit steps asking for J and a Newton solve).
 * A server owns n_streams streams on `device`; each stream holds resident
 * slot pools per mechanism (states, Jacobians, Newton workspace) created at
 * the mechanism's first request with capacity min(max_batch_states, what
 * 90 % of the remaining hbm_budget_bytes holds across the streams).  Requests
 * (host arrays, element-major with the request's own state count as leading
 * dimension: phi [N][n], p/h [n], rhs [N][n]; outputs x [N][n], info [n])
 * are taken in arrival order into rounds: the head request fixes the round's
 * mode and gamma, later requests of any mechanism with the same mode and gamma
 * join while each mechanism's share fits its pool.  A round copies its inputs
 * into a free stream's pools, evaluates the Jacobians of all its mechanisms in
 * one work-list launch per launch shape (pyjac_eval_jacobian_multi), solves
 * each mechanism's Newton systems (pyjac_newton_factor_solve with
 * max_refine/rtol) and copies the results out, while other rounds run on
 * other streams.  Per mechanism a round computes its state count rounded up to
 * 256 columns; the second round with the same kernel sequence on a stream is
 * captured into a HIP graph, later ones replay it.  A state's result does not
 * depend on the round it lands in.  Inputs are copied into pinned host
 * staging memory (min(budget / 4, 2 GiB), at least 64 MiB) during submit,
 * which blocks while that memory is full; outputs are written to the caller's
 * x / info when the request completes, so those two arrays must stay valid
 * until pyjac_serve_wait has returned.
 * ------------------------------------------------------------------------ */
typedef struct pyjac_server pyjac_server;

/* Errors: PYJAC_E_INVALID (bad parameters), PYJAC_E_NOMEM (budget or pinned
 * staging memory cannot be reserved), PYJAC_E_DEVICE. */
pyjac_status pyjac_serve_create(int32_t device, size_t hbm_budget_bytes, int64_t max_batch_states,
                                int32_t n_streams, int32_t max_refine, double rtol,
                                pyjac_server** out);

/* Queues one request and returns its id at once.  Errors: PYJAC_E_INVALID
 * (n_states above max_batch_states, bad arguments, shutting down),
 * PYJAC_E_NOMEM (the mechanism's pools cannot hold the request). */
pyjac_status pyjac_serve_submit(pyjac_server* server, const pyjac_mech* mech, int64_t n_states,
                                const double* phi, const double* p, const double* h,
                                const double* rhs, double gamma, int32_t mode, double* x,
                                int32_t* info, uint64_t* request_id);

/* Blocks until the request completes (timeout_s < 0: no limit) and returns
 * its latency (completion - submission) in seconds; the id is then released. */
pyjac_status pyjac_serve_wait(pyjac_server* server, uint64_t request_id, double timeout_s,
                              double* latency_s);

/* Counters since creation and the p50/p99 latency of all completed requests;
 * batches_done counts rounds, hbm_in_use the bytes of the resident pools. */
pyjac_status pyjac_serve_stats(pyjac_server* server, int64_t* requests_done, int64_t* states_done,
                               int64_t* batches_done, double* p50_s, double* p99_s,
                               size_t* hbm_in_use);

/* Rounds run eagerly (first sighting of their kernel sequence, or capture
 * refused), captured into a graph, and replayed from one; Jacobian launches
 * and how many of them served more than one mechanism.  Any out may be NULL. */
pyjac_status pyjac_serve_graph_stats(pyjac_server* server, int64_t* eager_rounds, int64_t* captured_rounds,
                                     int64_t* replayed_rounds, int64_t* jacobian_launches,
                                     int64_t* multi_mechanism_launches);

/* Completes every submitted request, then frees graphs, pools and streams. */
pyjac_status pyjac_serve_destroy(pyjac_server* server);

/* Static description of a status code. */
const char* pyjac_status_string(pyjac_status status);

/* Thread-local detail for the last failing call on this thread ("" if none). */
const char* pyjac_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PYJAC_MI355X_H */
