/*
 * hotrg.h — C ABI of the MI355X (gfx950) HOTRG coarse-graining library.
 *
 * The library evaluates the partition function of a 2D square-lattice
 * classical model written as the contraction of a network of identical
 * rank-4 tensors, Z = Tr T^N (Sec. II.A, Eq. (2)), by the higher-order tensor
 * renormalization group: at each step two neighbouring tensors are merged
 * along one lattice direction, the two parallel bonds are fused, and the fused
 * bond is truncated to at most D states by the leading eigenvectors of the
 * environment matrix, to which the higher-order SVD reduces (Sec. II.A).  The
 * contractions run as hand-written MFMA kernels; the truncation eigensolve,
 * the per-step normalisation and the ln Z accumulation are always FP64.
 *
 * Conventions used by every entry point
 *   - A local tensor is T[l, r, d, u] with dims [Dx, Dx, Dy, Dy], row-major,
 *     u fastest (l, r: the x bond; d, u: the y bond).
 *   - A step stacks two copies along y, fuses the two x legs (bottom first),
 *     keeps D' = min(D, Dx^2) states, normalises by c_n = max|T'| and then
 *     exchanges x and y, so the next step merges the other direction.  The
 *     dims go (Dx, Dy) -> (Dy, D').
 *   - After n steps the tensor stands for a periodic torus of 2^n sites,
 *     2^floor(n/2) sites along x by 2^ceil(n/2) along y.
 *
 * Memory and streams: the caller owns the device workspace (one allocation
 * of hotrg_workspace_bytes(), e.g. a torch uint8 tensor) and the HIP stream;
 * every kernel of a solve is enqueued on that stream and nothing is
 * allocated on the device per step.  The library owns only the host handle
 * and its timing events.
 *
 * The truncation eigensolve (FP64) runs on the device: environments up to
 * 96 x 96 are diagonalised completely by a parallel two-sided Jacobi method
 * (the 2x2-block rotation scheme of Sec. II.B, Eqs. (5)-(6)); larger ones by
 * a block subspace iteration with Rayleigh-Ritz projection (the small
 * projected problem again by that Jacobi method), warm-started from the
 * isometry of the step two earlier (the previous step's for steps without
 * the axis exchange), until the kept Ritz pairs have relative residual
 * <= 1e-12, at most 30 passes, or until the residual stagnates (three
 * convergence checks in a row without getting below 0.9x the best so far,
 * as when kept pairs lie in the rounding noise of a nearly rank-deficient
 * environment; hotrg_eig_info then reports the residual reached and
 * HOTRG_EIG_STAGNATED).  A solve that stops short of the 1e-12 bound with a
 * residual above the failure bound (5e-2 of the largest eigenvalue by
 * default, see hotrg_set_eig_limits: the block has not found the dominant
 * subspace), or whose eigenvalues are not finite, or a dense Jacobi
 * diagonalisation that ends at its sweep cap, is a failed eigensolve:
 * HOTRG_EEIG is latched on the device.  Slow convergence where the spectrum
 * is flat at the cut is not a failure (residuals up to ~5e-3 at the pass cap
 * are measured for the Heisenberg chain at beta ~ 800).
 *
 * Errors: every int-returning call returns HOTRG_OK (0) or a negative
 * status.  Errors detected on the device (HOTRG_ENONFINITE: a non-finite or
 * non-positive c_n; HOTRG_EEIG: a failed eigensolve) are latched in a device
 * status word; the first one sticks and is returned by the next
 * synchronising call (hotrg_log_z, hotrg_log_z_chain, hotrg_step_info,
 * hotrg_step_sides, hotrg_eig_info, hotrg_observables, hotrg_copy_tensor).
 * The kernels of later steps still run (and exit normally) on whatever the
 * failed step left; only the status is reported.  No C++ exception crosses
 * this ABI.
 * Distinct handles are independent and may be driven from different host
 * threads; one handle must not be used from two threads at once.
 */
#ifndef HOTRG_H
#define HOTRG_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define HOTRG_OK          0
#define HOTRG_EINVAL     -1  /* invalid argument or parameter set           */
#define HOTRG_ENOMEM     -2  /* workspace smaller than hotrg_workspace_bytes */
#define HOTRG_EHIP       -3  /* a HIP runtime call failed                    */
#define HOTRG_EEIG       -4  /* eigensolve failed (latched on the device)     */
#define HOTRG_ENONFINITE -5  /* c_n or the final trace not finite or <= 0    */
#define HOTRG_ESTATE     -6  /* call not valid in the handle's state         */
#define HOTRG_ENODEV     -7  /* no HIP device                                */

/* ---- models and contraction precisions -------------------------------- */
#define HOTRG_ISING   0  /* q = 2, H = -J sum s s'                              */
#define HOTRG_POTTS   1  /* q states, H = -J sum delta(s, s')                  */
#define HOTRG_CUSTOM  2  /* caller-supplied initial tensor (FP64, host memory) */
#define HOTRG_QCHAIN  3  /* spin-1/2 chain, bond term bond_h, Trotter step tau:
                            one tensor per two-site block and step (x = space,
                            y = imaginary time), see hotrg_log_z_chain      */

#define HOTRG_FP64    0  /* contractions in FP64 MFMA                          */
#define HOTRG_FP32    1  /* contractions in FP32 MFMA, FP32 accumulation       */
#define HOTRG_BF16X3  2  /* operands split in 2 BF16 terms, 3 products, FP32 acc */
#define HOTRG_BF16X6  3  /* operands split in 3 BF16 terms, 6 products, FP32 acc */
#define HOTRG_FP16X3  4  /* as HOTRG_BF16X6, except the D^7 product at full size
                            (Y = X . T, Sec. II.B) and the environment
                            products in the panel layout: their operands
                            split in 2 FP16 terms of the value times a fixed
                            power of two (2^11 for X, 2^14 for T, s_H with
                            s_H Dx Dy <= 2^15 for the half environments, all
                            bounded because max|T| = 1 and U is an isometry,
                            so that the terms stay in FP16's range), 3
                            products, FP32 accumulation; no observables     */

#define HOTRG_MAX_STEPS 60  /* total steps per handle (2^60 sites)            */
#define HOTRG_MAX_DIM   96  /* largest bond dimension accepted                */

/* Stage indices of hotrg_stage_times(). */
#define HOTRG_STAGE_PERMUTE 0  /* operand re-layouts of T (D^4)               */
#define HOTRG_STAGE_ENV     1  /* half environments and E (GEMMs)             */
#define HOTRG_STAGE_EIG     2  /* FP64 eigensolve of E, isometry selection    */
#define HOTRG_STAGE_X       3  /* X = U . T (GEMM)                            */
#define HOTRG_STAGE_Y       4  /* Y = X . T (GEMM, the D^7 term)              */
#define HOTRG_STAGE_TP      5  /* T' = Y . U (GEMM)                           */
#define HOTRG_STAGE_NORM    6  /* max|T'|, scaling, ln Z accumulation         */
#define HOTRG_STAGE_OBS     7  /* impurity-tensor contractions (observables)  */
#define HOTRG_NUM_STAGES    8

/* Observables carried as impurity tensors (bits of hotrg_params.observables;
 * slot 0 and slot 1 of hotrg_observables()). */
#define HOTRG_OBS_MAGNETIZATION 1  /* slot 0: order parameter per site        */
#define HOTRG_OBS_BOND_ENERGY   2  /* slot 1: energy of one y bond            */

typedef struct hotrg_solve hotrg_solve;  /* opaque host handle */

typedef struct hotrg_params {
    int model;           /* HOTRG_ISING, HOTRG_POTTS or HOTRG_CUSTOM           */
    int q;               /* spin states: 2 for Ising, 2..16 for Potts         */
    double coupling;     /* J > 0 (ferromagnetic), k_B = 1                    */
    double temperature;  /* T > 0                                             */
    int dmax;            /* bond dimension D, 1..HOTRG_MAX_DIM                */
    int precision;       /* HOTRG_FP64, HOTRG_FP32, HOTRG_BF16X3, HOTRG_BF16X6,
                            HOTRG_FP16X3 (then observables must be 0)       */
    const double* custom_tensor; /* HOTRG_CUSTOM: host T[l,r,d,u], row-major,
                                    dims [Dx, Dx, Dy, Dy]; read during init only */
    int custom_dx;       /* HOTRG_CUSTOM: Dx (1..HOTRG_MAX_DIM)               */
    int custom_dy;       /* HOTRG_CUSTOM: Dy (1..HOTRG_MAX_DIM)               */
    int max_steps;       /* steps the handle may take in total; sizes the
                            workspace (0 = HOTRG_MAX_STEPS)                   */
    double field;        /* h: H gains -h sum_i f(s_i), f(s) = s (Ising, s = +-1)
                            or delta(s, 0) (Potts); must be 0 for HOTRG_CUSTOM */
    int two_sided;       /* 0: isometry from the left environment; 1: both
                            environments, the smaller truncation error wins  */
    int observables;     /* bitmask of HOTRG_OBS_*: impurity tensors carried  */
    const double* custom_impurity[2]; /* HOTRG_CUSTOM: the impurity tensors of
                            slots 0 and 1 (host, dims of custom_tensor), read
                            during init only, for the bits set in observables */
    const double* bond_h; /* HOTRG_QCHAIN: two-site term h, real symmetric 4 x 4,
                            row-major, basis |s t> = 2 s + t (read at init)   */
    double tau;          /* HOTRG_QCHAIN: Trotter step (> 0)                   */
} hotrg_params;

/* Bytes of device workspace one solve with these parameters needs, for any
 * number of steps up to p->max_steps.  Dominated by the two D^5
 * intermediates X and Y (Sec. II.B: the coarse-grained matrices are D^2 on
 * a side).  Pure host arithmetic; returns 0 for an invalid parameter set. */
size_t hotrg_workspace_bytes(const hotrg_params* p);

/* Builds the initial local tensor of Eq. (2) and readies a solve.
 *   p          parameters (copied; custom_tensor is read before returning)
 *   workspace  device pointer, 256-byte aligned, >= hotrg_workspace_bytes(p)
 *              bytes; owned by the caller, must outlive the handle
 *   ws_bytes   size of that allocation
 *   stream     hipStream_t on which all work of this solve is enqueued
 *              (NULL = the legacy default stream)
 *   out        receives the new handle
 * For Ising/Potts, T0[x,x',y,y'] = sum_s g(s) Q[s,x]Q[s,x']Q[s,y]Q[s,y'] with
 * Q the symmetric square root of the bond Boltzmann weight matrix and g(s) =
 * exp(h f(s) / temperature) the field's site factor; T0 (and any impurity
 * tensor, see hotrg_observables) is normalised by c_0 = max|T0| and ln c_0
 * starts the ln Z accumulator.  The tensors and the device state are copied
 * on the stream, which init synchronises.
 * Errors: EINVAL (parameters, NULL pointers, misaligned workspace, a
 * non-zero field or a missing impurity tensor with HOTRG_CUSTOM, or a bond
 * dimension too large for the eigensolver's Ritz block: every step with
 * Dx^2 > 96 needs D' < 96), ENOMEM (ws_bytes too small), ENODEV, EHIP. */
int hotrg_init_tensor(const hotrg_params* p, void* workspace, size_t ws_bytes,
                      void* stream, hotrg_solve** out);

/* Restarts an existing handle on a new parameter set (a new temperature,
 * model or bond dimension) without creating a new one: the initial tensor is
 * rebuilt exactly as in hotrg_init_tensor, the step count and the device
 * status are cleared, and the handle's workspace and timing events are kept.  Synchronises the handle's stream first.
 * Errors: EINVAL (parameters), ENOMEM (the handle's workspace is too small
 * for p: create a new handle instead), EHIP. */
int hotrg_reset(hotrg_solve* s, const hotrg_params* p);

/* Enqueues nsteps >= 0 coarse-graining steps (Sec. II.A: coarse-grain the
 * bonds of one direction and truncate them), continuing the x/y alternation
 * of earlier calls.  Asynchronous: returns once the work is enqueued.
 * Errors: EINVAL (nsteps < 0 or the total would exceed max_steps),
 * ESTATE (handle already failed), EHIP. */
int hotrg_coarse_grain(hotrg_solve* s, int nsteps);

/* hotrg_coarse_grain with a choice of axis: exchange = 1 is the usual step
 * (merge along y, then exchange x and y); exchange = 0 keeps the axes, so the
 * next step merges along y again (dims (Dx, Dy) -> (D', Dy)).  For a quantum
 * chain (HOTRG_QCHAIN, y = imaginary time) k steps with exchange = 0 are
 * operator evolution to beta = 2^k tau: only the space bonds are truncated.
 * Before each step the library checks that its dims fit the workspace (sized
 * for the alternating schedule up to max_steps); a schedule that reaches
 * larger dims gets ENOMEM with nothing enqueued for that step.
 * Errors: EINVAL (nsteps < 0, exchange not 0/1, step cap), ENOMEM, ESTATE,
 * EHIP. */
int hotrg_coarse_grain_axis(hotrg_solve* s, int nsteps, int exchange);

/* Serving form of hotrg_coarse_grain for a group of independent solves:
 * enqueues nsteps steps on each of the count handles in solves[], step by
 * step across the group (step 1 of every handle, then step 2, ...), each on
 * its own handle's stream, so that solves on different streams overlap on
 * the device.  Each handle continues its own alternation; the result of
 * every solve is the same as from hotrg_coarse_grain alone.  The array is
 * read, not kept.  A handle listed twice advances twice.
 * Errors: EINVAL (solves NULL with count > 0, a NULL entry, count < 0,
 * nsteps < 0, or a handle whose total would exceed its max_steps; nothing
 * is enqueued then), ESTATE (a listed handle has already failed; nothing is
 * enqueued), EHIP (enqueueing failed part-way: the handles already advanced
 * keep their steps, see hotrg_log_z of each). */
int hotrg_coarse_grain_batch(hotrg_solve* const* solves, int count, int nsteps);

/* Host-polled stepping (serving).  hotrg_coarse_grain enqueues every pass
 * the eigensolve of a step may need (up to the pass cap), and the passes
 * after convergence exit at once; with many solves on one device those
 * launches still take dispatch slots from the others.  In this form one step
 * is enqueued in parts and the host decides, from the eigensolver's stop
 * state written to pinned host memory (allocated by the library, one word
 * per handle, freed by hotrg_destroy), whether more passes are needed
 * before the step's products are enqueued:
 *   hotrg_step_begin  enqueues the step's environment, the start of its
 *                     eigensolve and as many subspace passes as the handle's
 *                     last eigensolve of the same parity needed (8 for the
 *                     first) plus `extra` >= 0 (fewer host round trips for
 *                     more passes that may run after convergence; the group
 *                     is rounded up to an even count, since convergence is
 *                     tested every second pass, and capped at the pass
 *                     limit), then the store of the stop state;
 *                     *pending (may be NULL) = 1.  A step whose environment
 *                     is diagonalised densely (Dx^2 <= 96) is enqueued whole
 *                     at once and *pending = 0.  On a two-sided handle the
 *                     left eigensolve goes first; once it has stopped, a poll
 *                     enqueues its end and the right one's start and first
 *                     passes (HOTRG_POLL_PASSES), and the step's products
 *                     follow the right one.  exchange as in
 *                     hotrg_coarse_grain_axis.
 *   hotrg_step_poll   never waits.  *state = HOTRG_POLL_IDLE (no step
 *                     pending), HOTRG_POLL_RUNNING (the last store has not
 *                     arrived; nothing enqueued), HOTRG_POLL_PASSES (not
 *                     converged: 4 more passes and a new store enqueued) or
 *                     HOTRG_POLL_STEPPED (the eigensolve has stopped: its end,
 *                     the products and the normalisation are enqueued and the
 *                     step counts among the steps taken).
 * The passes, their order and their arguments are those of the whole-step
 * form, so the results are bitwise the same.  Each step then waits for the
 * host between its eigensolve and its products: with several solves in
 * one process this form measures a few percent slower than whole steps; it
 * is for devices whose dispatch is shared with other launchers.  While a
 * step is pending, the
 * whole-step calls return EINVAL.  Errors: EINVAL (begin: exchange not
 * 0/1, extra < 0, a step already pending, step cap; poll: NULL state),
 * ESTATE, ENOMEM, EHIP (pinned memory or enqueueing). */
#define HOTRG_POLL_IDLE     0
#define HOTRG_POLL_RUNNING  1
#define HOTRG_POLL_PASSES   2
#define HOTRG_POLL_STEPPED  3
int hotrg_step_begin(hotrg_solve* s, int exchange, int extra, int* pending);
int hotrg_step_poll(hotrg_solve* s, int* state);

/* The host-polled form driven by the library itself: returns at once, and
 * a thread of the library (one per process, started by the first call)
 * begins the handle's nsteps steps one after another with
 * hotrg_step_begin(s, exchange, extra) and polls each with hotrg_step_poll
 * as soon as its eigensolve's stop state arrives, so that a step's
 * products are enqueued microseconds after its eigensolve ends and no pass
 * after convergence is launched.  The results are bitwise those of
 * hotrg_coarse_grain_axis(s, nsteps, exchange).  The thread spins (yielding
 * the CPU between rounds) while any handle is in flight and sleeps
 * otherwise.  Every other call on the handle first waits until the thread
 * has enqueued all of its steps (hotrg_async_busy tells without waiting);
 * hotrg_destroy waits too.  An error met by the thread (ENOMEM for a step
 * that does not fit, EHIP) puts the handle in the failed state: the next
 * hotrg_log_z returns it.  Errors: EINVAL (nsteps < 0, exchange not 0/1,
 * extra < 0, a polled step pending, step cap), ESTATE, EHIP (the thread
 * could not be started; nothing is enqueued). */
int hotrg_coarse_grain_async(hotrg_solve* s, int nsteps, int exchange, int extra);

/* *busy = 1 while the library's thread still has steps of the handle to
 * enqueue (hotrg_coarse_grain_async), else 0; never waits.  The enqueued
 * work itself completes on the handle's stream.  Errors: EINVAL. */
int hotrg_async_busy(hotrg_solve* s, int* busy);

/* Synchronises the stream and returns ln Z / N of the torus reached so far:
 *   ln Z/N = ln c_0 + sum_n ln(c_n) / 2^n + ln(sum_{x,y} T[x,x,y,y]) / 2^n_steps
 * lnz_per_site receives that value, log2_sites (may be NULL) the number of
 * steps taken (N = 2^log2_sites).  The free energy per site is
 * -temperature * lnz_per_site.
 * Errors: any latched device error; ENONFINITE if the final trace is <= 0. */
int hotrg_log_z(hotrg_solve* s, double* lnz_per_site, int* log2_sites);

/* ln Z per tensor of the network that is infinite along x and periodic
 * along y with the current tensor's extent (2^steps original tensors in
 * each column, for HOTRG_QCHAIN after y-only steps: beta = 2^steps tau):
 * y is closed by the trace t[l, r] = sum_s T[l, r, s, s], and the infinite
 * chain of columns contributes the dominant eigenvalue of t,
 *   ln Z/N = ln c_0 + sum_n ln(c_n) / 2^n + ln(lambda_max(t)) / 2^steps,
 * lambda_max from 64 normalised squarings of t on the device (FP64; a
 * modulus-degenerate pair +-lambda gives ln |lambda|).  For HOTRG_QCHAIN the
 * free energy per site is -(ln Z/N) / (2 tau).  Synchronises.  Errors:
 * latched device errors; ENONFINITE if the trace of the last square is not
 * positive; EINVAL (Dx > 96). */
int hotrg_log_z_chain(hotrg_solve* s, double* lnz_per_tensor);

/* Synchronises and reports diagnostics of step n (1..steps taken): the
 * normalisation c_n = max|T'|, the truncation error (discarded eigenvalue
 * weight over total weight of E) and the relative gap at the cut
 * (lam[D'-1] - lam[D']) / lam[0] (+inf when nothing is cut).  When E is
 * diagonalised in full (n <= 96) these are its eigenvalues; above that the
 * subspace iteration tests only the D' kept Ritz pairs for convergence, so
 * lam[D'] there is the next Ritz value of the block, which is not tested
 * and lies at or below the eigenvalue it approximates, so that gap is an
 * estimate from above; the discarded weight is the trace of E minus the
 * kept Ritz values.  n = 0 gives c_0 and
 * zeros.  Any output pointer may be NULL.  Errors: EINVAL, latched. */
int hotrg_step_info(hotrg_solve* s, int n, double* c_n, double* trunc_err,
                    double* cut_gap);

/* Two-sided truncation (Xie et al., PRB 86, 045139 (2012), the HOTRG the
 * paper's Sec. II.A builds on): with p->two_sided the right environment of
 * the merged pair (rows = the fused right leg) is diagonalised as well, and
 * the step applies, to both fused legs, the isometry of the side with the
 * smaller discarded weight (ties keep the left).  Synchronises and reports
 * step n (1..steps taken): both sides' discarded weight over total weight
 * (eps_right = NaN for one-sided handles) and the side applied (0 left,
 * 1 right).  hotrg_step_info and hotrg_eig_info report the applied side.
 * Any output pointer may be NULL.  Errors: EINVAL, latched. */
int hotrg_step_sides(hotrg_solve* s, int n, double* eps_left, double* eps_right, int* side);

/* Impurity-tensor observables.  An observable enters as one modified copy I
 * of the local tensor; every step replaces I by U^T (I (x) T + T (x) I) U,
 * the average of its two placements in the merged pair, divided by the same
 * c_n as T, so that after n steps Tr I / Tr T is the observable averaged
 * over the 2^n-site torus (exact when nothing is truncated).  For Ising /
 * Potts the library builds
 *   slot 0: sum_s m(s) g(s) Q[s,.]^4 with m = s (Ising), (q delta(s,0) - 1) /
 *           (q - 1) (Potts): the order parameter per site <m>;
 *   slot 1: T0 with its d leg carrying e(s,s') W(s,s') instead of W(s,s')
 *           (e = -J s s' or -J delta(s,s')): the mean energy <e_b> of one y
 *           bond.  The internal energy per site of these isotropic models is
 *           2 <e_b> - h <f>.
 * For HOTRG_CUSTOM the slots hold Tr I / Tr T of the caller's tensors.
 * Each carried tensor costs one more D^6 product and one D^7 product over
 * twice the contraction length per step.  Synchronises; values[slot] gets
 * the estimate, NaN for a slot not carried.  Errors: EINVAL, latched,
 * ENONFINITE (Tr T = 0). */
int hotrg_observables(hotrg_solve* s, double values[2]);

/* How the eigensolve of a step ended (hotrg_eig_info's `stop`). */
#define HOTRG_EIG_CONVERGED  0  /* every kept Ritz pair met the 1e-12 bound, or
                                   E was diagonalised densely to the Jacobi
                                   rotation threshold                         */
#define HOTRG_EIG_STAGNATED  1  /* stopped when the residual stopped falling   */
#define HOTRG_EIG_PASS_CAP   2  /* stopped at the pass cap (dense: sweep cap)   */

/* Synchronises and reports the eigensolve of step n (1..steps taken):
 * iterations = subspace passes used (0 when E was diagonalised densely),
 * sweeps = Jacobi sweeps of the last projected problem (of E itself when
 * dense), residual = max_j |E u_j - theta_j u_j| / theta_0 over the kept
 * pairs (0 when dense), stop = HOTRG_EIG_* above.  A step whose stop is not
 * HOTRG_EIG_CONVERGED and whose residual exceeds the failure bound has
 * latched HOTRG_EEIG, which this call then returns (the outputs are left
 * unset).  Any output pointer may be NULL.  Errors: EINVAL, latched. */
int hotrg_eig_info(hotrg_solve* s, int n, int* iterations, int* sweeps, double* residual, int* stop);

/* Eigensolver limits for the steps enqueued after this call (the defaults
 * are restored by hotrg_reset):
 *   max_passes    subspace passes per eigensolve, 1..HOTRG_EIG_MAX_PASSES
 *                 (default 30)
 *   fail_residual a solve that stops short of convergence with a residual
 *                 above fail_residual (relative to the largest eigenvalue)
 *                 latches HOTRG_EEIG; > 0, default 5e-2.
 * A small pass cap makes the failure reachable on purpose without any
 * invalid input (tests of the error path): every kernel still exits
 * normally.  Errors: EINVAL. */
#define HOTRG_EIG_MAX_PASSES 60
int hotrg_set_eig_limits(hotrg_solve* s, int max_passes, double fail_residual);

/* Synchronises and copies the current normalised tensor (FP64) to host
 * memory `host` of `capacity` doubles; dims receives {Dx, Dy} (the tensor
 * has Dx*Dx*Dy*Dy entries, layout as above).  Errors: EINVAL (capacity too
 * small: dims are still filled in), latched errors. */
int hotrg_copy_tensor(hotrg_solve* s, double* host, size_t capacity, int dims[2]);

/* Synchronises and copies the environment of the last step taken (left
 * environment E = M M^T, symmetrised, FP64 as the eigensolver received it;
 * Sec. II.A) to host memory `host` of `capacity` doubles, row-major n x n
 * with rows and columns the fused leg (a1 a2), a1 the bottom copy's; *n
 * receives n = Dx^2 of that step.  For tests and diagnostics: the buffer is
 * overwritten by the next step.  Errors: EINVAL (no step taken, capacity
 * too small: *n is still filled in), latched errors. */
int hotrg_copy_environment(hotrg_solve* s, double* host, size_t capacity, int* n);

/* Synchronises and copies the isometry the last step applied to host memory
 * `host` of `capacity` doubles, row-major n x D' (column l = kept vector l,
 * rows the fused leg (a1 a2)), as the contractions used it: FP64 values
 * for HOTRG_FP64, the FP32 value or the sum of the BF16 planes otherwise.
 * dims receives {n, D'}.  For tests and diagnostics.  Errors: as
 * hotrg_copy_environment. */
int hotrg_copy_isometry(hotrg_solve* s, double* host, size_t capacity, int dims[2]);

/* Per-stage timing with HIP events recorded on the solve's stream.
 * hotrg_set_timing(s, 1) starts recording for the steps enqueued afterwards
 * (it allocates the events, so call it before the timed region);
 * hotrg_stage_times synchronises and writes the summed GPU milliseconds of
 * each stage (HOTRG_NUM_STAGES values, indices HOTRG_STAGE_*) over the steps
 * recorded since timing was enabled, and the number of such steps. */
int hotrg_set_timing(hotrg_solve* s, int enable);
int hotrg_stage_times(hotrg_solve* s, double* ms, int* steps_timed);
/* The same for one recorded step: ms[HOTRG_NUM_STAGES] of the k-th step
 * enqueued since timing was enabled (0-based), and that step's input dims
 * {Dx, Dy, D'} in dims (may be NULL).  Synchronises.  Errors: EINVAL (timing
 * off or k out of range). */
int hotrg_step_stage_times(hotrg_solve* s, int k, double* ms, int dims[3]);

/* Per-kernel timing of the Y contraction (the D^7 GEMM): summed GPU ms and
 * launch count over the recorded steps, from events around that launch. */
int hotrg_gemm_y_time(hotrg_solve* s, double* ms, int* launches);

/* Releases the host handle and its events.  Waits for the solve's enqueued
 * work to finish first.  The caller then frees the workspace.  NULL is a
 * no-op. */
void hotrg_destroy(hotrg_solve* s);

/* Short description of a status code (static string). */
const char* hotrg_strerror(int status);

/* ---- device/runtime queries ------------------------------------------- */
/* Number of visible HIP devices (0 without a GPU).  Returns HOTRG_OK. */
int hotrg_device_count(int* count);
/* Version of the HIP runtime this library is bound to (hipRuntimeGetVersion). */
int hotrg_runtime_version(int* version);

/* ---- contraction building block (kernel unit tests) -------------------- */
/* Index-mapped matrix product, the one contraction kernel every step uses:
 *   C[map(m, n)] = alpha * sum_k A[m*lda + k] * B[n*ldb + k]
 * for 0 <= m < M, 0 <= n < N, 0 <= k < K (both operands K-contiguous).  The
 * output map writes the fused-index target layout directly, with no
 * separate permute (the permute-free layout of Sec. II.B, Eq. (3)):
 *   map(m, n) = (m / sm) * rs_hi + (m % sm) * rs_lo
 *             + (n / sn) * cs_hi + (n % sn) * cs_lo.
 * precision selects the MFMA path (HOTRG_FP64 / HOTRG_FP32 / HOTRG_BF16X3 /
 * HOTRG_BF16X6).  A, B and C are device pointers in FP64; for the reduced
 * precisions the library rounds/splits the operands into an internal copy
 * inside `scratch` (device memory of hotrg_gemm_scratch_bytes() bytes, may be
 * NULL for HOTRG_FP64) and writes C in FP64.  Enqueued on `stream`.
 * Errors: EINVAL (sizes < 0, NULL, sm or sn < 1), EHIP. */
size_t hotrg_gemm_scratch_bytes(int precision, int M, int N, int K);
int hotrg_gemm_nt(int precision, int M, int N, int K,
                  const double* A, long lda, const double* B, long ldb,
                  double* C, double alpha,
                  long sm, long rs_hi, long rs_lo, long sn, long cs_hi, long cs_lo,
                  void* scratch, void* stream);

/* hotrg_gemm_nt with the tile choice of one contraction of a step, so that a
 * test reaches the very kernel a solve launches for it:
 *   role   HOTRG_ROLE_GENERIC (half environments and E), HOTRG_ROLE_X,
 *          HOTRG_ROLE_Y (the D^7 product) or HOTRG_ROLE_TP
 *   panel  1: both converted operands are stored in the 32 x 16 panel layout
 *          a solve's producers write for the environment and Y products
 *          (split precisions only; M and N multiples of 32, K of 16)
 * HOTRG_FP16X3 runs as the full-size Y product (role HOTRG_ROLE_Y, panel 1,
 * at least 512 tiles of 256 x 256) and as the environment product (role
 * HOTRG_ROLE_GENERIC, panel 1, N > 64); each operand is converted as
 * 2^11 times its value into two FP16 planes, so |A| and |B| must stay below
 * 31 (larger entries overflow FP16 and give non-finite results).
 * The output is FP64 through the map, as for hotrg_gemm_nt (a solve's Y
 * writes FP32 in the split modes; the products themselves are the same).
 * Errors: EINVAL (as hotrg_gemm_nt, role out of range, panel with FP64 or
 * with shapes the layout cannot hold), EHIP (also when the role's kernel
 * does not accept the shape). */
#define HOTRG_ROLE_GENERIC 0
#define HOTRG_ROLE_X       1
#define HOTRG_ROLE_Y       2
#define HOTRG_ROLE_TP      3
int hotrg_gemm_nt_role(int precision, int role, int panel, int M, int N, int K,
                       const double* A, long lda, const double* B, long ldb,
                       double* C, double alpha,
                       long sm, long rs_hi, long rs_lo, long sn, long cs_hi, long cs_lo,
                       void* scratch, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* HOTRG_H */
