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

// Storage format of contraction operands and intermediates.
enum class Fmt : int {
    F64 = 0,      // double
    F32 = 1,      // float
    BF16x2 = 2,   // two bf16 planes: hi, lo (value ~ hi + lo)
    BF16x3 = 3,   // three bf16 planes: hi, mid, lo
};

inline int fmt_planes(Fmt f) { return f == Fmt::BF16x2 ? 2 : (f == Fmt::BF16x3 ? 3 : 1); }
inline size_t fmt_plane_elem_bytes(Fmt f) { return f == Fmt::F64 ? 8 : (f == Fmt::F32 ? 4 : 2); }
inline size_t fmt_elem_bytes(Fmt f) { return fmt_plane_elem_bytes(f) * fmt_planes(f); }

// A buffer of `count` logical elements in format `fmt`.  Planes of the
// split formats are stored one after the other, `plane` elements apart.
struct Buf {
    void* ptr;
    Fmt fmt;
    size_t plane;  // elements between planes (>= count, rounded up)
};

// Output map of the index-mapped product (see hotrg_gemm_nt in hotrg.h):
//   off(m, n) = (m / sm) * rs_hi + (m % sm) * rs_lo + (n / sn) * cs_hi + (n % sn) * cs_lo
struct OutMap {
    long sm, rs_hi, rs_lo;
    long sn, cs_hi, cs_lo;
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
    int info[64];         // eigensolver info per step
    double partial[1024]; // partial maxima of the normalisation reduction
};

// Normalisation of step n: c_n = max|T|, T /= c_n, lnz_acc += ln(c_n) / 2^n.
hipError_t launch_normalize(double* T, size_t count, DevState* st, int n, hipStream_t stream);
// trace = sum_{x,y} T[x,x,y,y] for T of dims [Dx,Dx,Dy,Dy].
hipError_t launch_trace(const double* T, int Dx, int Dy, DevState* st, hipStream_t stream);
// E <- (E + E^T) / 2 for an n x n matrix.
hipError_t launch_symmetrize(double* E, int n, hipStream_t stream);
// From the eigensolver output (eigenvalues ascending in w; eigenvector j in
// column j of the column-major V, leading dimension n) take the leading kept
// eigenvectors in descending order, fix each sign so its largest-magnitude
// entry (lowest index on ties) is positive, and write
//   Ut[l, i]             = u_l[i]                (kept x n, isometry rows)
//   Ux[l, a2, a1]        = u_l[a1 * dx + a2]     (kept x dx x dx)
// Records truncation error, cut gap and eigensolver status of step n.
hipError_t launch_select_isometry(const double* V, const double* w, const int* info, int n, int dx,
                                  int kept, const Buf& Ut, const Buf& Ux, DevState* st, int step,
                                  hipStream_t stream);

}  // namespace hotrg

namespace hotrg {
// out[r, c] = in[r * ld + c] for r < rows, c < cols, converted to out's format
// (dense, row length cols).
hipError_t launch_convert2d(const double* in, long ld, int rows, int cols, const Buf& out,
                            hipStream_t stream);
}  // namespace hotrg
