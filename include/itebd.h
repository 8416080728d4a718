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
 * other bond.  The SVD is a one-sided (column) Jacobi method in FP64 with a
 * round-robin pair ordering, warm-started from the right singular vectors
 * of the same bond's previous update; the kept right vectors have their
 * largest-magnitude entry made positive.
 *
 * Device mapping: one workgroup per chain keeps the Jacobi matrices (W, V)
 * in LDS (chi <= 32); the unit cell and the evolved pair go through the
 * chain's slice of the workspace, which stays in L2, and a launch runs many
 * updates of a chain.  Two chains share a CU, so a batch of twice the CU
 * count fills the chip.
 *
 * Status codes are those of hotrg.h.  The caller owns the device workspace
 * (itebd_workspace_bytes: state rows, the evolved pair and two bonds' right
 * vectors per chain, counters) and the stream; nothing is allocated on the
 * device by the library.  All arithmetic is FP64.
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
 * weighted two-site wave function of the bond.  energies: batch doubles.
 * Errors: EINVAL, EHIP. */
int itebd_energy(itebd_batch* b, double* energies);

/* Synchronises and copies the states (batch rows, layout as for init; B1 is
 * the left site of the bond the next update acts on).  Errors: EINVAL, EHIP. */
int itebd_copy_states(itebd_batch* b, double* host, size_t capacity);

/* Bond updates applied so far and the largest Jacobi sweep count any chain
 * needed in the last launch (synchronises).  Either pointer may be NULL. */
int itebd_info(itebd_batch* b, long* updates, int* max_sweeps);

/* Work done so far, summed over the chains (synchronises): Jacobi sweeps
 * and pair rotations applied.  One sweep over n = 2 chi columns forms the
 * three dot products of every pair (n (n - 1) / 2 pairs, 6 n FLOPs each);
 * a rotation updates two columns of M and of V (12 n FLOPs).  Either
 * pointer may be NULL. */
int itebd_work(itebd_batch* b, double* sweeps, double* rotations);

/* Releases the host handle (waits for the stream first).  NULL is a no-op. */
void itebd_destroy(itebd_batch* b);

#ifdef __cplusplus
}
#endif
#endif /* ITEBD_H */
