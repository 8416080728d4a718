/*
 * itebd.h — C ABI of the MI355X (gfx950) iTEBD library part: imaginary-time
 * evolution of many independent infinite spin-1/2 chains at once.
 *
 * Each chain is a two-site periodic matrix product state (Sec. II.A,
 * Eq. (1)): ... lambda_2 A lambda_1 B lambda_2 ..., stored as B1 = A lambda_1,
 * B2 = B lambda_2 (arrays [s][a][b], s the physical index, a and b the
 * virtual ones, D_b = chi states each) and the weights lambda_1, lambda_2.
 * The ground state is approached by repeated imaginary-time evolution with
 * U = exp(-tau h) on alternating bonds (Sec. II.A); each bond update is the
 * tensor contraction followed by the SVD that the paper identifies as the
 * two costs (Sec. II.A, Sec. II.B), in the update form that needs no
 * division by the weights (Hastings 2009, on the iTEBD of Vidal 2007):
 *   psi  = B1 B2 contracted over the shared bond, psi' = G psi, G = exp(-tau h)
 *   M[(a s),(t b)] = lambda_2[a] psi'[a,s,t,b];  M = X S Y^T
 *   B2' = rows of Y^T kept, B1' = psi' Y / |S_kept|, lambda_1' = S_kept / |S_kept|
 * after which the two sites exchange roles, so the next update acts on the
 * other bond.  The SVD, in FP64, is a Householder QR with column pivoting,
 * M Pi = Q R, followed by a one-sided (column) Jacobi method with a
 * round-robin pair ordering on R^T: its converged columns, normalised and
 * permuted back by Pi, are the right singular vectors of M and their norms
 * the singular values (Q and the left vectors are never formed).  The kept
 * right vectors have their largest-magnitude entry made positive.
 *
 * Device mapping: one workgroup per chain keeps the decomposition's work
 * matrix in LDS (chi <= 32, 37 KB); the unit cell and the evolved pair go
 * through the chain's slice of the workspace, which stays in L2, and a
 * launch runs many updates of a chain.  Up to four chains share a CU.
 *
 * Status codes are those of hotrg.h.  The caller owns the device workspace
 * (itebd_workspace_bytes: state rows, the evolved pair per chain, status
 * words, counters) and the stream; nothing is allocated on the device by
 * the library.  All arithmetic is FP64.
 *
 * Failures are recorded per chain in a device status word (bits below) and
 * reported by the synchronising calls itebd_energy and itebd_info:
 * HOTRG_ENONFINITE when a chain's kept singular values had a zero or
 * non-finite norm (that update is not applied and the chain is not updated
 * again: its state row keeps the last good update), else HOTRG_EEIG when a
 * decomposition was still rotating at the sweep limit (that update is
 * applied as it stands).  The other chains of the batch are unaffected.
 */
#ifndef ITEBD_H
#define ITEBD_H

#include <stddef.h>

#include "hotrg.h"

#ifdef __cplusplus
extern "C" {
#endif

#define ITEBD_MAX_CHI 32  /* largest bond dimension (the state lives in LDS) */
#define ITEBD_PHYS    2   /* physical dimension (spin 1/2)                   */
#define ITEBD_MAX_SWEEPS 40  /* default and largest Jacobi sweep limit       */

/* Bits of a chain's status word (itebd_status). */
#define ITEBD_CHAIN_SWEEP_CAP 1  /* a decomposition reached the sweep limit    */
#define ITEBD_CHAIN_NONFINITE 2  /* kept singular values' norm zero or not
                                    finite: the chain is frozen                 */

typedef struct itebd_batch itebd_batch;  /* opaque host handle */

/* Doubles in one chain's state row: B1 (2 chi^2), B2 (2 chi^2), lambda_1
 * (chi), lambda_2 (chi), in that order, row-major. */
size_t itebd_state_len(int chi);

/* Device bytes for `batch` chains of bond dimension chi (0 if invalid). */
size_t itebd_workspace_bytes(int batch, int chi);

/* Uploads the initial states and readies the batch.
 *   batch      number of chains (>= 1)
 *   chi        bond dimension D_b (1..ITEBD_MAX_CHI)
 *   h          the two-site Hamiltonian term, real symmetric 4 x 4, row-major,
 *              basis |s t> with index 2 s + t (host memory, copied)
 *   states     batch rows of itebd_state_len(chi) doubles (host, copied)
 *   workspace  device memory of itebd_workspace_bytes(batch, chi) bytes,
 *              256-byte aligned, owned by the caller
 *   stream     hipStream_t for all work of this batch (NULL = default)
 * Errors: EINVAL (sizes, NULL pointers, misalignment, h not symmetric or
 * not finite), ENOMEM (ws_bytes too small), ENODEV, EHIP. */
int itebd_init(int batch, int chi, const double* h, const double* states, void* workspace,
               size_t ws_bytes, void* stream, itebd_batch** out);

/* Enqueues nupdates bond updates (alternating bonds) of every chain with
 * the gate exp(-tau h), tau > 0.  Asynchronous.  Errors: EINVAL, EHIP. */
int itebd_evolve(itebd_batch* b, double tau, int nupdates);

/* Synchronises and writes each chain's energy per site, the mean of <h>
 * on its two bonds, <h> = theta.(h theta) / theta.theta with theta the
 * weighted two-site wave function of the bond.  energies: batch doubles,
 * written for every chain (a frozen chain's from its last good state).
 * Errors: EINVAL, EHIP; ENONFINITE or EEIG when a chain's status word is
 * set (see above; itebd_status tells which chains). */
int itebd_energy(itebd_batch* b, double* energies);

/* Synchronises and copies the states (batch rows, layout as for init; B1 is
 * the left site of the bond the next update acts on).  Errors: EINVAL, EHIP. */
int itebd_copy_states(itebd_batch* b, double* host, size_t capacity);

/* Bond updates enqueued so far (a frozen chain applied fewer) and the
 * largest Jacobi sweep count any chain needed in the last launch
 * (synchronises).  Either pointer may be NULL.  Returns ENONFINITE or EEIG
 * as itebd_energy does, after writing the outputs. */
int itebd_info(itebd_batch* b, long* updates, int* max_sweeps);

/* Synchronises and copies every chain's status word (ITEBD_CHAIN_* bits,
 * 0 = no failure) to status (batch ints, host).  Errors: EINVAL, EHIP. */
int itebd_status(itebd_batch* b, int* status);

/* Sets the Jacobi sweep limit of later updates, 1..ITEBD_MAX_SWEEPS
 * (default ITEBD_MAX_SWEEPS).  A converged decomposition takes one sweep
 * without rotations to be recognised, so a limit of 1 marks every update
 * with a rotation as ITEBD_CHAIN_SWEEP_CAP.  Errors: EINVAL. */
int itebd_set_max_sweeps(itebd_batch* b, int max_sweeps);

/* Work done so far, summed over the chains (synchronises): Jacobi sweeps
 * and pair rotations applied.  One sweep over n = 2 chi columns forms the
 * three dot products of every pair (n (n - 1) / 2 pairs, 6 n FLOPs each);
 * a rotation updates two columns of R^T (6 n FLOPs).  Either pointer may
 * be NULL. */
int itebd_work(itebd_batch* b, double* sweeps, double* rotations);

/* Releases the host handle (waits for the stream first).  NULL is a no-op. */
void itebd_destroy(itebd_batch* b);

#ifdef __cplusplus
}
#endif
#endif /* ITEBD_H */
