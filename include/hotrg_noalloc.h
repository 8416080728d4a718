/*
 * hotrg_noalloc.h — allocation-free entry point of the HOTRG library.
 *
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation.  The
 * stand-alone contraction hotrg_gemm_nt_role (include/hotrg.h) needs a
 * caller-provided scratch buffer for the split operands of the reduced
 * precisions; this form keeps them in a library-owned device array instead.
 */
#ifndef HOTRG_NOALLOC_H
#define HOTRG_NOALLOC_H

#include "hotrg.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Size of the library-owned device array (per GPU). */
#define HOTRG_NOALLOC_SCRATCH_BYTES (64u << 20)

/* hotrg_gemm_nt_role without the scratch argument: same arguments, meaning,
 * layouts, output and errors otherwise.  The converted operands live in a
 * file-scope device array of HOTRG_NOALLOC_SCRATCH_BYTES bytes that every GPU
 * the library runs on holds until the process ends; the call makes no
 * hipMalloc, hipFree or other allocating call (its first call on a device
 * only looks up that device's address of the array).
 *   - A product needing more than HOTRG_NOALLOC_SCRATCH_BYTES of converted
 *     operands (hotrg_gemm_scratch_bytes) is rejected with HOTRG_ENOMEM and
 *     nothing is enqueued.  HOTRG_FP64 needs none.
 *   - Every call on one GPU uses the same array, which keeps the last call's
 *     contents: calls that overlap on that GPU (other streams, other host
 *     threads) race on it and must be ordered by the caller (one stream, or
 *     events between streams).  Every call fully rewrites the part it reads,
 *     so nothing needs to start at zero.
 * Errors: as hotrg_gemm_nt_role, and HOTRG_ENOMEM as above. */
int hotrg_gemm_nt_noalloc(int precision, int role, int panel, int M, int N, int K,
                          const double* A, long lda, const double* B, long ldb,
                          double* C, double alpha,
                          long sm, long rs_hi, long rs_lo, long sn, long cs_hi, long cs_lo,
                          void* stream);

#ifdef __cplusplus
}
#endif
#endif /* HOTRG_NOALLOC_H */
