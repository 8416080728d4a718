// Internal declarations shared by the HOTRG library's HIP sources.
// Nothing here is part of the C ABI (include/hotrg.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

namespace hotrg {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

// Storage format of contraction operands and intermediates.
enum class Fmt : int {
    F64 = 0,      // double
    F32 = 1,      // float
    BF16x2 = 2,   // two bf16 planes: hi, lo (value ~ hi + lo)
    BF16x3 = 3,   // three bf16 planes: hi, mid, lo
    F16x2 = 4,    // two fp16 planes: hi, lo of the value times a power-of-two scale
};

inline int fmt_planes(Fmt f) {
    return f == Fmt::BF16x2 || f == Fmt::F16x2 ? 2 : (f == Fmt::BF16x3 ? 3 : 1);
}
inline size_t fmt_plane_elem_bytes(Fmt f) { return f == Fmt::F64 ? 8 : (f == Fmt::F32 ? 4 : 2); }
inline size_t fmt_elem_bytes(Fmt f) { return fmt_plane_elem_bytes(f) * fmt_planes(f); }

// A buffer of `count` logical elements in format `fmt`.  Planes of the
// split formats are stored one after the other, `plane` elements apart.
//
// panel_k != 0 marks a matrix of rows x panel_k elements stored as 32 x 16
// panels (BF16 formats only): element (r, c) at
//   ((r / 32) * (panel_k / 16) + c / 16) * 512 + (r % 32) * 16 + c % 16,
// so that the 32 rows x 16 columns a product kernel stages per K step are
// one contiguous KiB.  Rows must be a multiple of 32, panel_k of 16.  As a
// product operand, ptr may point at column c0 (a multiple of 16) of a wider
// panel matrix: the operand is then columns c0 .. c0 + K - 1 and lda equals
// panel_k.
//
// cols != 0 makes ptr a block of `cols` columns inside a wider matrix for the
// element-wise writers: logical element i is (i / cols, i % cols), stored at
// row stride ld (row-major) or at panel_index() of the panel_k-wide layout.
struct Buf {
    void* ptr;
    Fmt fmt;
    size_t plane;      // elements between planes (>= count, rounded up)
    long panel_k = 0;  // 0: row-major; else the row length of the panel layout
    long cols = 0;     // 0: dense; else the column count of a sub-block
    long ld = 0;       // row stride of a row-major sub-block (cols != 0, panel_k == 0)
    float scale = 1.f; // F16x2 writers store the planes of value * scale (a power of two)
};

// FP16 two-plane split of f (already scaled): hi = fp16(f), lo = fp16(f - hi),
// both by round-to-nearest-even; f - hi is exact in FP32.
__device__ __forceinline__ void f16_split(float f, _Float16* hi, _Float16* lo) {
    const _Float16 h = (_Float16)f;
    *hi = h;
    *lo = (_Float16)(f - (float)h);
}

__host__ __device__ inline long panel_index(long r, long c, long panel_k) {
    return ((r >> 5) * (panel_k >> 4) + (c >> 4)) * 512 + (r & 31) * 16 + (c & 15);
}

// Output map of the index-mapped product (see hotrg_gemm_nt in hotrg.h):
//   R(m, n) = (m / sm) * rs_hi + (m % sm) * rs_lo + (n / sn) * cs_hi + (n % sn) * cs_lo
// is the output offset when panel_k == 0.  With panel_k != 0 the output is
// a panel-layout matrix (see Buf): R is its row and
//   C(m, n) = (m / sm) * rc_hi + (m % sm) * rc_lo + (n / sn) * cc_hi + (n % sn) * cc_lo
// its column, and the offset is panel_index(R, C, panel_k).
struct OutMap {
    long sm, rs_hi, rs_lo;
    long sn, cs_hi, cs_lo;
    long rc_hi = 0, rc_lo = 0, cc_hi = 0, cc_lo = 0;
    long panel_k = 0;
    // Tile-order hint for the BF16 product at full size: when the columns
    // are n = g * ngroup + h (ngroup a multiple of 16, N / ngroup too), a
    // 256-wide tile may take 16 g x 16 h instead of 256 consecutive n (0: off).
    long ngroup = 0;
};

// Which contraction of a step a product is (selects tiles; distinct symbols).
enum class GemmRole : int { Generic = 0, X = 1, Y = 2, TP = 3 };

// C[map(m,n)] = alpha * sum_k A[m*lda + k] * B[n*ldb + k].
// A, B: operand buffers (same format); C: output buffer (any format).
// `products` selects the split-product count for the bf16 formats (3 or 6).
hipError_t launch_gemm_nt(const Buf& A, long lda, const Buf& B, long ldb, const Buf& C,
                          int M, int N, int K, double alpha, const OutMap& map,
                          int products, GemmRole role, hipStream_t stream);

// out[j0,j1,j2,j3] = in[...] with out axis a taken from input axis perm[a];
// in has dims (n0,n1,n2,n3) row-major, FP64.  Output in any format.
hipError_t launch_permute4(const double* in, const int dims[4], const int perm[4],
                           const Buf& out, hipStream_t stream);

// Device-side bookkeeping of one solve.
struct DevState {
    double lnz_acc;       // ln c_0 + sum ln(c_n) / 2^n
    double trace;         // sum_{x,y} T[x,x,y,y] of the current tensor
    double c_cur;         // c_n of the last normalisation
    int status;           // first latched error (0 = none)
    int pad;
    double c[64];
    double trunc_err[64];
    double cut_gap[64];
    int info[64];         // eigensolver iterations per step (0: dense Jacobi of E)
    int eig_sweeps[64];   // Jacobi sweeps of the last Rayleigh-Ritz problem per step
    double eig_resid[64]; // max residual / theta_0 of the kept Ritz pairs per step
    // two-sided truncation: both sides' discarded weights, the side applied
    // (0 left, 1 right) and the right eigensolve's diagnostics per step
    double eps_left[64];
    double eps_right[64];
    int side[64];
    double r_cut_gap[64];
    int r_info[64];
    int r_sweeps[64];
    double r_resid[64];
    int eig_stop[64];     // how each step's eigensolve ended (HOTRG_EIG_*)
    int r_eig_stop[64];   // the same for the right environment
    double imp_trace[2];  // sum_{x,y} I[x,x,y,y] of the impurity tensors
    double chain_lnz;     // ln lambda_max of the y-traced tensor (hotrg_log_z_chain)
    int chain_ok;         // 1 if the last normalised square had a positive trace
    double partial[1024]; // partial maxima of the normalisation reduction
};

// Device control block of one eigensolve.
struct EigCtl {
    int done;        // set once the kept Ritz pairs have converged (or the last pass ran)
    int iters;       // subspace passes used
    int converged;   // 1 if the residual test passed
    int sweeps;      // Jacobi sweeps of the last small eigenproblem
    double resid;    // max_j |E u_j - theta_j u_j| / theta_0 over the kept pairs
    double trace;    // Tr E
    double best;     // smallest residual seen at a convergence check
    int stall;       // consecutive checks that did not bring it below 0.9 best
    int jac_capped;  // the last Jacobi diagonalisation ended at its sweep cap
};

// Host-visible stop state of an eigensolve (pinned, fine-grained host
// memory), written by one device thread after a group of subspace passes as
// one 64-bit word: seq << 32 | iters << 1 | done.  A single store needs no
// fence (a release at system scope would write back the whole L2), and the
// host that reads the seq it expects has the matching done and iters.
struct EigMail {
    unsigned long long word;
};
hipError_t launch_eig_mail(const EigCtl* ctl, EigMail* mail, int seq, hipStream_t stream);

constexpr int kEigPMax = 96;   // largest Ritz block / largest fully diagonalised E

// Device buffers of the eigensolver (FP64), carved from the workspace.
struct EigWork {
    double* V[2];    // Ritz blocks, n x p row-major, one per step parity (warm starts)
    double* W;       // n x p
    double* part;    // partial Gram blocks, ceil(n/32) x (kEigPMax^2 + kEigPMax)
    double* G;       // reduced Gram (+ residuals), kEigPMax^2 + kEigPMax
    double* S;       // Jacobi eigenvectors, kEigPMax^2
    double* theta;   // Ritz values, kEigPMax
    double* L;       // Cholesky factor, kEigPMax^2
    double* dsc;     // column scales, kEigPMax
    EigCtl* ctl;
};

// Ritz block width for an n x n environment keeping k vectors (n > kEigPMax).
// p = min(2k, k + 32), at least k + 16, rounded up to 16.  The Rayleigh-
// Ritz problem (one-workgroup Jacobi, ~p^3 per sweep) dominates a pass, so
// the block is kept as narrow as convergence allows: at k = 48 (D = 48),
// p = 80 takes 0.65x the eigensolve time of p = 96 for the same residual
// bound, while p = 64 misses the bound at Tc within 30 passes.
inline int eig_block(int n, int k) {
    int p = 2 * k < k + 32 ? 2 * k : k + 32;
    if (p < k + 16) p = k + 16;
    p = (p + 15) / 16 * 16;
    if (p > kEigPMax) p = kEigPMax;
    if (p > n) p = n;
    return p;
}

// Leading k eigenpairs of the symmetric n x n matrix E (FP64), written as the
// isometry Ut / Ux (see launch_select_isometry) with the sign gauge; step
// diagnostics into st.  warm: V[parity] already holds the Ritz block of the
// step two earlier with the same (n, p).
// slot 0 records the diagnostics as the step's own (and eps_left), slot 1 as
// the right environment's (eps_right, r_*).
// A solve that stops unconverged with a residual above fail_tol (relative to
// theta_0), with non-finite eigenvalues, or a dense Jacobi at its sweep cap,
// latches HOTRG_EEIG in st->status (first error sticks).
//
// The subspace iteration can be enqueued in parts (host-polled stepping):
// `range` selects the start (initial block and its orthonormalisation),
// passes [first, last) of the maxit passes, and the end (selection of the
// kept vectors and the statistics).  A pass enqueued after the solve has
// converged exits at once, so any split of [0, maxit) that stops at a pass
// after which the convergence word reads done gives the result of the whole
// range.  A dense solve (n <= kEigPMax) runs entirely with the start.
struct EigRange {
    int first = 0, last = -1;   // passes [first, last); last < 0: up to maxit
    bool start = true, end = true;
};
hipError_t launch_eig_topk(const double* E, int n, int k, int dx, const EigWork& w, int parity, bool warm,
                           unsigned long long seed, int maxit, double tol, double fail_tol, const Buf& Ut,
                           const Buf& Ux, DevState* st, int step, hipStream_t stream, int slot = 0,
                           const EigRange& range = EigRange());

// Two-sided truncation: when eps_right[step] < eps_left[step], copies the
// right isometry (UtR, UxR: `bytes` bytes each, 16-byte multiple) over the
// left one and makes the right side's diagnostics the step's own; records
// the side either way.
hipError_t launch_choose_side(DevState* st, int step, void* Ut, void* Ux, const void* UtR, const void* UxR,
                              size_t bytes, hipStream_t stream);

// Normalisation of step n: c_n = max|T|, T /= c_n, lnz_acc += ln(c_n) / 2^n.
hipError_t launch_normalize(double* T, size_t count, DevState* st, int n, hipStream_t stream);
// trace = sum_{x,y} T[x,x,y,y] for T of dims [Dx,Dx,Dy,Dy] (into *out, a
// device address, default st->trace).
hipError_t launch_trace(const double* T, int Dx, int Dy, DevState* st, hipStream_t stream, double* out = nullptr);
// ln lambda_max of t[l, r] = sum_s T[l, r, s, s] (T of dims [Dx, Dx, Dy, Dy],
// Dx <= 96) by `squarings` normalised squarings in one workgroup, into
// st->chain_lnz and st->chain_ok.
hipError_t launch_chain_lnz(const double* T, int Dx, int Dy, int squarings, DevState* st, hipStream_t stream);
// I <- I * factor / c_n (c_n of the last normalisation, read on the device).
hipError_t launch_scale_by_norm(double* I, size_t count, const DevState* st, double factor, hipStream_t stream);
// E <- (E + E^T) / 2 for an n x n matrix.
hipError_t launch_symmetrize(double* E, int n, hipStream_t stream);

}  // namespace hotrg

namespace hotrg {
// The stand-alone product of the C ABI (hotrg_gemm_nt_role) with its operand
// conversion into `scratch` (scratch_bytes available; ENOMEM when the
// conversion needs more), and the bytes that conversion needs.
size_t gemm_scratch_bytes(int precision, int M, int N, int K);
int gemm_nt_with_scratch(int precision, int role, int panel, int M, int N, int K, const double* A, long lda,
                         const double* B, long ldb, double* C, double alpha, long sm, long rs_hi, long rs_lo, long sn,
                         long cs_hi, long cs_lo, void* scratch, size_t scratch_bytes, void* stream);

// out[r, c] = in[r * ld + c] for r < rows, c < cols, converted to out's format
// (dense, row length cols).
hipError_t launch_convert2d(const double* in, long ld, int rows, int cols, const Buf& out,
                            hipStream_t stream);
}  // namespace hotrg
