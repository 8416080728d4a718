// FP64 top-k eigensolver of the symmetric environment E (n x n) on the device.
//
// The truncation of a HOTRG step keeps the leading k eigenvectors of
// E = M M^T, to which the higher-order SVD of the merged tensor reduces
// (Sec. II.A).  Only k << n of them are needed, so for n > P_MAX the solver
// is a block subspace iteration with a Rayleigh-Ritz projection on every
// second pass:
//
//   V (n x p, orthonormal)  ->  W = E V           (MFMA FP64, eig_ev_kernel)
//   H = V^T W (p x p)       ->  H = S diag(theta) S^T   (Jacobi, one workgroup)
//   V <- V S, W <- W S      (Ritz vectors; residual |W_j - theta_j V_j|)
//   converged?  else  V <- orth(W diag(1/|W_j|))  (CholeskyQR)
//
// and on the passes between only W = E V and V <- orth(W diag(1/|W_j|)).
//
// warm-started from the Ritz block of the step two earlier (same fused leg
// basis once the dims are steady), else from a counter-based random block.
// For n <= P_MAX the Jacobi kernel diagonalises E itself.
//
// The small symmetric eigenproblem is solved with the paper's two-sided
// Jacobi scheme (Sec. II.B, Eqs. (5)-(6), Fig. 3): the matrix is cut into
// 2x2 blocks; each diagonal block M_II is diagonalised by a plane rotation
// J_I (left = right rotation, the matrix being symmetric); every block
// M_IJ is then updated as J_I^T M_IJ J_J and the rotations are accumulated;
// the index pairs then move by the round-robin (systolic) exchange, so that
// after p-1 rounds every pair has met once (one sweep).  Here one workgroup
// holds the matrix in LDS and a thread updates whole 2x2 blocks; the
// "exchange" is a relabelling of which indices form each pair.
//
// All reductions are in a fixed order (no atomics), so a solve is bitwise
// reproducible.
#include <math.h>
#include "common.h"
#include "../../include/hotrg.h"

namespace hotrg {

constexpr int EIG_PMAX = kEigPMax; // largest Ritz block / fully diagonalised matrix
constexpr int EIG_LDP = EIG_PMAX + 1;
constexpr int EIG_GRAM_ROWS = 32;  // rows per partial Gram block
constexpr int EIG_MAX_SWEEPS = 40;
// Rayleigh-Ritz (and the convergence test) on every second pass; the pass
// between is a plain power step V <- orth(E V).  The span of the block, on
// which convergence depends, is the same either way, and the Jacobi of the
// Rayleigh quotient dominates a pass: measured at D = 48, 0.66-0.76x the
// eigensolve time at the same residual bound (every third pass misses the
// bound in 30 passes).
constexpr int EIG_RR_EVERY = 2;
constexpr int EIG_JT = 1024;   // threads of the one-workgroup Jacobi kernel

// ---------------------------------------------------------------- helpers

__device__ __forceinline__ bool eig_done(const EigCtl* c) { return c->done != 0; }

// splitmix64 hash of a counter -> uniform double in [-1, 1)
__device__ __forceinline__ double hash_uniform(unsigned long long x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    x = x ^ (x >> 31);
    return (double)(x >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

// ---------------------------------------------------------------- init

// Trace of E, control reset; fills V with random columns unless warm.
__global__ __launch_bounds__(256) void eig_init_kernel(const double* __restrict__ E, int n, double* __restrict__ V,
                                                       int p, int warm, unsigned long long seed, EigCtl* ctl) {
    __shared__ double sh[256];
    if (blockIdx.x == 0) {
        double t = 0.0;
        for (int i = threadIdx.x; i < n; i += 256) t += E[(long)i * n + i];
        sh[threadIdx.x] = t;
        __syncthreads();
        for (int s = 128; s > 0; s >>= 1) {
            if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            ctl->trace = sh[0];
            ctl->done = 0;
            ctl->iters = 0;
            ctl->converged = 0;
            ctl->resid = 0.0;
            ctl->best = 1e300;
            ctl->stall = 0;
            ctl->jac_capped = 0;
        }
    }
    if (!warm) {
        const long total = (long)n * p;
        for (long e = blockIdx.x * 256L + threadIdx.x; e < total; e += (long)gridDim.x * 256)
            V[e] = hash_uniform(seed * 0x100000001B3ull + (unsigned long long)e);
    }
}

// ---------------------------------------------------------------- W = E V

// Workgroup: 16 rows of W, all p columns; the 4 waves split K and reduce in LDS.
__global__ __launch_bounds__(256) void eig_ev_kernel(const double* __restrict__ E, int n,
                                                     const double* __restrict__ V, double* __restrict__ W, int p,
                                                     const EigCtl* ctl) {
    if (eig_done(ctl)) return;
    __shared__ double red[3][16][EIG_PMAX + 1];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r0 = blockIdx.x * 16;
    const int fr = lane & 15, fk = lane >> 4;
    const int nf = p / 16;  // p is a multiple of 16, <= 96
    d4 acc[6];
#pragma unroll
    for (int f = 0; f < 6; ++f) acc[f] = d4{0, 0, 0, 0};
    const int kchunk = ((n + 63) / 64) * 16;  // multiple of 16 per wave
    const int kb = wave * kchunk, ke = min(n, kb + kchunk);
    const int row = r0 + fr;
    const double* erow = E + (long)min(row, n - 1) * n;
    // four 4-wide k steps per batch: all loads issued before the MFMAs
    for (int k = kb; k < ke; k += 16) {
        double a[4], b[4][6];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int kk = k + 4 * u + fk;
            const bool kin = kk < ke;
            a[u] = (row < n && kin) ? erow[kk] : 0.0;
#pragma unroll
            for (int f = 0; f < 6; ++f) b[u][f] = (kin && f < nf) ? V[(long)kk * p + f * 16 + fr] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int f = 0; f < 6; ++f)
                if (f < nf) acc[f] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], b[u][f], acc[f], 0, 0, 0);
    }
    // component r of lane l holds row (l/16) + 4r, column l%16 of each fragment
    if (wave > 0) {
#pragma unroll
        for (int f = 0; f < 6; ++f)
            if (f < nf)
#pragma unroll
                for (int r = 0; r < 4; ++r) red[wave - 1][fk + 4 * r][f * 16 + fr] = acc[f][r];
    }
    __syncthreads();
    if (wave == 0) {
#pragma unroll
        for (int f = 0; f < 6; ++f) {
            if (f < nf) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int rr = fk + 4 * r;
                    const double v = acc[f][r] + red[0][rr][f * 16 + fr] + red[1][rr][f * 16 + fr] +
                                     red[2][rr][f * 16 + fr];
                    if (r0 + rr < n) W[(long)(r0 + rr) * p + f * 16 + fr] = v;
                }
            }
        }
    }
}

// ---------------------------------------------------------------- Gram partials

// part[b] = X_b^T Y_b over rows [32 b, 32 b + 32) (p x p, row-major).
__global__ __launch_bounds__(256) void eig_gram_kernel(const double* __restrict__ X, const double* __restrict__ Y,
                                                       int n, int p, double* __restrict__ part, int part_stride,
                                                       const EigCtl* ctl) {
    if (eig_done(ctl)) return;
    __shared__ double xs[EIG_GRAM_ROWS][EIG_PMAX + 1];
    __shared__ double ys[EIG_GRAM_ROWS][EIG_PMAX + 1];
    const int r0 = blockIdx.x * EIG_GRAM_ROWS;
    for (int e = threadIdx.x; e < EIG_GRAM_ROWS * p; e += 256) {
        const int r = e / p, c = e - (e / p) * p;
        const bool in = r0 + r < n;
        xs[r][c] = in ? X[(long)(r0 + r) * p + c] : 0.0;
        ys[r][c] = in ? Y[(long)(r0 + r) * p + c] : 0.0;
    }
    __syncthreads();
    double* out = part + (long)blockIdx.x * part_stride;
    for (int e = threadIdx.x; e < p * p; e += 256) {
        const int i = e / p, j = e - (e / p) * p;
        double s = 0.0;
        for (int r = 0; r < EIG_GRAM_ROWS; ++r) s += xs[r][i] * ys[r][j];
        out[e] = s;
    }
}

// out[e] = sum_b part[b][e], fixed order.
__global__ __launch_bounds__(256) void eig_reduce_kernel(const double* __restrict__ part, int nb, int part_stride,
                                                         int count, double* __restrict__ out, const EigCtl* ctl) {
    if (eig_done(ctl)) return;
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= count) return;
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += part[(long)b * part_stride + e];
    out[e] = s;
}

// ---------------------------------------------------------------- Jacobi

// Diagonalises the symmetric p x p matrix Hin (p <= EIG_PMAX; read with
// leading dimension ldh): theta[j] descending, S column j the matching
// eigenvector (S row-major p x p, S[i*p + j]).  sym: use (H + H^T)/2.
__global__ __launch_bounds__(EIG_JT) void eig_jacobi_kernel(const double* __restrict__ Hin, int ldh, int p,
                                                          double* __restrict__ theta, double* __restrict__ S,
                                                          EigCtl* ctl, int check_done) {
    if (check_done && eig_done(ctl)) return;
    __shared__ double H[EIG_PMAX * EIG_LDP];
    __shared__ double V[EIG_PMAX * EIG_LDP];
    __shared__ double cs[EIG_PMAX / 2], sn[EIG_PMAX / 2], tt[EIG_PMAX / 2];
    __shared__ int pi[EIG_PMAX / 2], pj[EIG_PMAX / 2];
    __shared__ int any_rot;
    __shared__ double sfloor;
    __shared__ int rank[EIG_PMAX];
    const int tid = threadIdx.x;
    const int pp = p + (p & 1);   // even number of players; index p (if any) is a zero dummy
    const int half = pp / 2;
    const int bstride = EIG_JT / half;      // threads per block column
    // threads 0 .. half*bstride-1 own block column bq and rows bp0, bp0+bstride, ...
    const int bq = tid < half * bstride ? tid % half : half;
    const int bp0 = tid / half;
    for (int e = tid; e < pp * pp; e += EIG_JT) {
        const int i = e / pp, j = e - (e / pp) * pp;
        double h = 0.0;
        if (i < p && j < p) h = 0.5 * (Hin[(long)i * ldh + j] + Hin[(long)j * ldh + i]);
        H[i * EIG_LDP + j] = h;
        V[i * EIG_LDP + j] = (i == j) ? 1.0 : 0.0;
    }
    if (tid == 0) {
        double m = 0.0;
        for (int i = 0; i < p; ++i) m = fmax(m, fabs(Hin[(long)i * ldh + i]));
        sfloor = fmax(1e-300, 1e-18 * m);
    }
    __syncthreads();
    // Rotation test: an off-diagonal element is zeroed while it is large
    // relative to its own diagonal pair, |hij| > 1e-14 sqrt|hii hjj| (taken
    // squared: no square root on the round's critical path), and above
    // 1e-18 of the largest diagonal element: smaller elements lie under the
    // rounding of the matrix itself (a rank-deficient tail would otherwise be
    // rotated until its elements are tiny next to its own tiny diagonal).
    const double floor_abs = sfloor;
    auto passes = [&](double hij, double hii, double hjj) {
        return hij * hij > 1e-28 * fabs(hii * hjj) && fabs(hij) > floor_abs;
    };
    int sweeps = 0, capped = 0;
    for (int sweep = 0;; ++sweep) {
        // A sweep in which no off-diagonal element passes the rotation test
        // below changes nothing; find that out directly (one pass over the
        // upper triangle) instead of by running the sweep's pp - 1 rounds.
        if (tid == 0) any_rot = 0;
        __syncthreads();
        for (int e = tid; e < p * p; e += EIG_JT) {
            const int i = e / p, j = e - (e / p) * p;
            if (j > i) {
                if (passes(H[i * EIG_LDP + j], H[i * EIG_LDP + i], H[j * EIG_LDP + j])) any_rot = 1;
            }
        }
        __syncthreads();
        if (!any_rot) break;
        if (sweep == EIG_MAX_SWEEPS) {   // rotations still pending after the cap
            capped = 1;
            break;
        }
        for (int r = 0; r < pp - 1; ++r) {
            // round-robin pairing: position 0 fixed, positions 1..pp-1 rotate by r
            if (tid < half) {
                const int qa = tid, qb = pp - 1 - tid;
                // (q - 1 + r) modulo pp - 1 (both terms below pp - 1), plus 1
                int a = qa - 1 + r, b = qb - 1 + r;
                a -= a >= pp - 1 ? pp - 1 : 0;
                b -= b >= pp - 1 ? pp - 1 : 0;
                a = qa == 0 ? 0 : a + 1;
                b += 1;
                const int i = min(a, b), j = max(a, b);
                pi[tid] = i;
                pj[tid] = j;
                const double hii = H[i * EIG_LDP + i], hjj = H[j * EIG_LDP + j], hij = H[i * EIG_LDP + j];
                double c = 1.0, s = 0.0, t = 0.0;
                if (passes(hij, hii, hjj)) {
                    // the smaller root of t^2 + 2 tau t - 1 = 0, tau = (hjj - hii) / (2 hij),
                    // written without forming tau: t = sign(d) 2hij / (|d| + sqrt(d^2 + 4 hij^2))
                    const double d = hjj - hii, h2 = 2.0 * hij;
                    t = (d >= 0.0 ? h2 : -h2) / (fabs(d) + sqrt(fma(d, d, h2 * h2)));
                    c = rsqrt(fma(t, t, 1.0));
                    s = t * c;
                }
                cs[tid] = c;
                sn[tid] = s;
                tt[tid] = t;
            }
            __syncthreads();
            // two-sided update of every 2x2 block: B' = J_P^T B J_Q; thread
            // (bq, bp0) handles blocks (P, Q = bq) for P = bp0, bp0 + bstride, ...
            if (bq < half) {
                const int k = pi[bq], l = pj[bq];
                const double cq = cs[bq], sq = sn[bq];
                for (int P = bp0; P < half; P += bstride) {
                    const int i = pi[P], j = pj[P];
                    if (P == bq) {
                        const double t = tt[P];
                        if (t != 0.0) {
                            const double hij = H[i * EIG_LDP + j];
                            H[i * EIG_LDP + i] -= t * hij;
                            H[j * EIG_LDP + j] += t * hij;
                            H[i * EIG_LDP + j] = 0.0;
                            H[j * EIG_LDP + i] = 0.0;
                        }
                        continue;
                    }
                    const double cp = cs[P], sp = sn[P];
                    if (sp == 0.0 && sq == 0.0) continue;   // both rotations are the identity
                    const double bik = H[i * EIG_LDP + k], bil = H[i * EIG_LDP + l];
                    const double bjk = H[j * EIG_LDP + k], bjl = H[j * EIG_LDP + l];
                    // rows: J_P^T
                    const double rik = cp * bik - sp * bjk, ril = cp * bil - sp * bjl;
                    const double rjk = sp * bik + cp * bjk, rjl = sp * bil + cp * bjl;
                    // columns: J_Q
                    H[i * EIG_LDP + k] = cq * rik - sq * ril;
                    H[i * EIG_LDP + l] = sq * rik + cq * ril;
                    H[j * EIG_LDP + k] = cq * rjk - sq * rjl;
                    H[j * EIG_LDP + l] = sq * rjk + cq * rjl;
                }
            }
            // accumulate: V <- V J (columns k, l of rows bp0, bp0 + bstride, ...)
            if (bq < half) {
                const double c = cs[bq], sv = sn[bq];
                if (sv != 0.0) {
                    const int k = pi[bq], l = pj[bq];
                    for (int row = bp0; row < pp; row += bstride) {
                        const double a = V[row * EIG_LDP + k], b = V[row * EIG_LDP + l];
                        V[row * EIG_LDP + k] = c * a - sv * b;
                        V[row * EIG_LDP + l] = sv * a + c * b;
                    }
                }
            }
            __syncthreads();
        }
        sweeps = sweep + 1;
        __syncthreads();
    }
    // descending order, ties by index
    for (int i = tid; i < p; i += EIG_JT) {
        const double ti = H[i * EIG_LDP + i];
        int rk = 0;
        for (int j = 0; j < p; ++j) {
            const double tj = H[j * EIG_LDP + j];
            rk += (tj > ti) || (tj == ti && j < i);
        }
        rank[i] = rk;
    }
    __syncthreads();
    for (int i = tid; i < p; i += EIG_JT) theta[rank[i]] = H[i * EIG_LDP + i];
    for (int e = tid; e < p * p; e += EIG_JT) {
        const int row = e / p, col = e - (e / p) * p;
        S[(long)row * p + rank[col]] = V[row * EIG_LDP + col];
    }
    if (tid == 0) {
        ctl->sweeps = sweeps;
        ctl->jac_capped = capped;
    }
}

// ---------------------------------------------------------------- Ritz rotation

// V_b <- V_b S, W_b <- W_b S for the 32-row block b; then the partial Gram
// W_b^T W_b and the partial squared residuals |W_j - theta_j V_j|^2 (j < p)
// into part[b] = [p*p Gram | p residuals].
__global__ __launch_bounds__(256) void eig_rotate_kernel(double* __restrict__ V, double* __restrict__ W, int n, int p,
                                                         const double* __restrict__ S, const double* __restrict__ theta,
                                                         double* __restrict__ part, int part_stride,
                                                         const EigCtl* ctl) {
    if (eig_done(ctl)) return;
    __shared__ double ss[EIG_PMAX * EIG_LDP];
    __shared__ double vs[EIG_GRAM_ROWS][EIG_PMAX + 1];
    __shared__ double ws[EIG_GRAM_ROWS][EIG_PMAX + 1];
    const int r0 = blockIdx.x * EIG_GRAM_ROWS;
    for (int e = threadIdx.x; e < p * p; e += 256) {
        const int i = e / p, j = e - (e / p) * p;
        ss[i * EIG_LDP + j] = S[e];
    }
    for (int e = threadIdx.x; e < EIG_GRAM_ROWS * p; e += 256) {
        const int r = e / p, c = e - (e / p) * p;
        const bool in = r0 + r < n;
        vs[r][c] = in ? V[(long)(r0 + r) * p + c] : 0.0;
        ws[r][c] = in ? W[(long)(r0 + r) * p + c] : 0.0;
    }
    __syncthreads();
    // each thread: outputs (r, c) of both products
    double vo[12], wo[12];   // EIG_GRAM_ROWS * EIG_PMAX / 256 = 12
    int cnt = 0;
    for (int e = threadIdx.x; e < EIG_GRAM_ROWS * p; e += 256, ++cnt) {
        const int r = e / p, c = e - (e / p) * p;
        double a = 0.0, b = 0.0;
        for (int m = 0; m < p; ++m) {
            const double sm = ss[m * EIG_LDP + c];
            a += vs[r][m] * sm;
            b += ws[r][m] * sm;
        }
        vo[cnt] = a;
        wo[cnt] = b;
    }
    __syncthreads();
    cnt = 0;
    for (int e = threadIdx.x; e < EIG_GRAM_ROWS * p; e += 256, ++cnt) {
        const int r = e / p, c = e - (e / p) * p;
        vs[r][c] = vo[cnt];
        ws[r][c] = wo[cnt];
        if (r0 + r < n) {
            V[(long)(r0 + r) * p + c] = vo[cnt];
            W[(long)(r0 + r) * p + c] = wo[cnt];
        }
    }
    __syncthreads();
    double* out = part + (long)blockIdx.x * part_stride;
    for (int e = threadIdx.x; e < p * p; e += 256) {
        const int i = e / p, j = e - (e / p) * p;
        double s = 0.0;
        for (int r = 0; r < EIG_GRAM_ROWS; ++r) s += ws[r][i] * ws[r][j];
        out[e] = s;
    }
    for (int j = threadIdx.x; j < p; j += 256) {
        const double th = theta[j];
        double s = 0.0;
        for (int r = 0; r < EIG_GRAM_ROWS; ++r) {
            const double d = ws[r][j] - th * vs[r][j];
            s += d * d;
        }
        out[p * p + j] = s;
    }
}

// ---------------------------------------------------------------- Cholesky


// One workgroup.  G (p x p) is the Gram matrix of the block X to be
// orthonormalised.  check >= 0: first decide convergence from the reduced
// residuals (stored after G) of the leading k Ritz pairs; on convergence, or
// when check == last iteration, mark the solve done and stop.  Then
// d_j = 1/sqrt(G_jj) (0 for a vanishing column), Gs = D G D (+ shift*I), and
// Gs = L L^T; Lout receives Q = D L^{-T} (row-major, upper triangular), so
// that X Q has orthonormal columns, and dout receives d.
__global__ __launch_bounds__(1024) void eig_chol_kernel(const double* __restrict__ G, int n, int p, int k,
                                                        const double* __restrict__ theta, double tol, int check,
                                                        int last_iter, double shift, double* __restrict__ Lout,
                                                        double* __restrict__ dout, EigCtl* ctl) {
    if (eig_done(ctl)) return;
    __shared__ double A[EIG_PMAX * EIG_LDP];
    __shared__ double d[EIG_PMAX];
    __shared__ int stop;
    const int tid = threadIdx.x;
    if (check >= 0) {
        if (tid == 0) {
            double worst = 0.0;
            for (int j = 0; j < k; ++j) worst = fmax(worst, sqrt(fmax(G[p * p + j], 0.0)));
            const double scale = fmax(fabs(theta[0]), 1e-300);
            const int conv = worst <= tol * scale;
            const double r = worst / scale;
            ctl->iters = check + 1;
            ctl->resid = r;
            ctl->converged = conv;
            // stagnation: three checks in a row without getting below 0.9x
            // the best residual so far mean the block has reached its
            // rounding floor (kept pairs in the noise of a nearly rank-
            // deficient E); further passes would end at the same residual at
            // the pass cap, so stop here (converged stays 0, as at the cap)
            if (r < 0.9 * ctl->best) {
                ctl->best = r;
                ctl->stall = 0;
            } else {
                ctl->stall += 1;
            }
            stop = conv || check == last_iter || ctl->stall >= 3;
            if (stop) ctl->done = 1;
        }
        __syncthreads();
        if (stop) return;
    }
    for (int j = tid; j < p; j += 1024) {
        const double g = G[(long)j * p + j];
        d[j] = g > 1e-280 ? 1.0 / sqrt(g) : 0.0;
    }
    __syncthreads();
    for (int e = tid; e < p * p; e += 1024) {
        const int i = e / p, j = e - (e / p) * p;
        double v = 0.5 * (G[(long)i * p + j] + G[(long)j * p + i]) * d[i] * d[j];
        if (i == j) v = (d[i] == 0.0 ? 1.0 : v) + shift;
        if (i != j && (d[i] == 0.0 || d[j] == 0.0)) v = 0.0;
        A[i * EIG_LDP + j] = v;
    }
    __syncthreads();
    // Right-looking Cholesky of the lower triangle with the elimination
    // applied to the identity beside it, one barrier per column: every thread
    // takes the pivot L_jj = sqrt(A_jj) itself (A_jj is final at column j);
    // the trailing update of A scales the column-j entries it needs on the
    // fly (column j is only read in this phase), and the same row operations
    // on R (= I at the start) leave R = L^{-1} (rows unscaled until the end:
    // row j of R is read only at column j, scaled on the fly as well).
    __shared__ double R[EIG_PMAX * EIG_LDP];
    __shared__ double ldiag[EIG_PMAX];
    for (int e = tid; e < p * p; e += 1024) {
        const int i = e / p, c = e - (e / p) * p;
        if (c <= i) R[i * EIG_LDP + c] = i == c ? 1.0 : 0.0;
    }
    __syncthreads();
    const int ty = tid >> 5, tx = tid & 31;
    for (int j = 0; j < p; ++j) {
        const double a = A[j * EIG_LDP + j];
        const double ljj = a > 1e-300 ? sqrt(a) : 1.0;
        const double inv = 1.0 / ljj;
        if (tid == 0) ldiag[j] = ljj;
        // thread (ty, tx) of a 32 x 32 grid: rows i = j + 1 + ty, ...; columns
        // l = j + 1 + tx, ... <= i of A and c = tx, ... <= j of R
        for (int i = j + 1 + ty; i < p; i += 32) {
            const double lij = A[i * EIG_LDP + j] * inv;
            for (int l = j + 1 + tx; l <= i; l += 32) A[i * EIG_LDP + l] -= lij * (A[l * EIG_LDP + j] * inv);
            for (int c = tx; c <= j; c += 32) R[i * EIG_LDP + c] -= lij * (R[j * EIG_LDP + c] * inv);
        }
        __syncthreads();
    }
    // Q[r][c] = d_r * M[c][r] (X_new = X D L^{-T}), M = L^{-1} = R with row c
    // scaled by 1 / L_cc; M[c][r] = 0 for r > c
    for (int e = tid; e < p * p; e += 1024) {
        const int r = e / p, c = e - (e / p) * p;
        const double m = r <= c ? R[c * EIG_LDP + r] * (1.0 / ldiag[c]) : 0.0;
        // a vanishing column is replaced by uniform(-1,1) entries of norm ~ sqrt(n/3)
        const double dr = d[r] != 0.0 ? d[r] : 1.0 / sqrt(n / 3.0);
        Lout[e] = dr * m;
    }
    for (int j = tid; j < p; j += 1024) dout[j] = d[j];
}

// X_b <- X_b Q for 32-row blocks, Q = D L^{-T} from eig_chol_kernel (a
// column with d_j = 0 is first replaced by random entries).  in and out may
// alias (each block is loaded before it is written).
__global__ __launch_bounds__(256) void eig_orth_apply_kernel(const double* in, double* out, int n, int p,
                                                             const double* __restrict__ Q,
                                                             const double* __restrict__ dsc,
                                                             unsigned long long seed, const EigCtl* ctl) {
    if (eig_done(ctl)) return;
    __shared__ double qs[EIG_PMAX * EIG_LDP];
    __shared__ double xs[EIG_GRAM_ROWS][EIG_PMAX + 1];
    const int r0 = blockIdx.x * EIG_GRAM_ROWS;
    for (int e = threadIdx.x; e < p * p; e += 256) {
        const int i = e / p, j = e - (e / p) * p;
        qs[i * EIG_LDP + j] = Q[e];
    }
    for (int e = threadIdx.x; e < EIG_GRAM_ROWS * p; e += 256) {
        const int r = e / p, c = e - (e / p) * p;
        const long gr = r0 + r;
        double v = 0.0;
        if (gr < n)
            v = dsc[c] != 0.0 ? in[gr * p + c]
                              : hash_uniform(seed ^ (0xD1B54A32D192ED03ull * (unsigned long long)(gr * p + c + 1)));
        xs[r][c] = v;
    }
    __syncthreads();
    double o[12];
    int cnt = 0;
    for (int e = threadIdx.x; e < EIG_GRAM_ROWS * p; e += 256, ++cnt) {
        const int r = e / p, c = e - (e / p) * p;
        double a = 0.0;
        for (int m = 0; m <= c; ++m) a += xs[r][m] * qs[m * EIG_LDP + c];   // Q is upper triangular
        o[cnt] = a;
    }
    cnt = 0;
    for (int e = threadIdx.x; e < EIG_GRAM_ROWS * p; e += 256, ++cnt) {
        const int r = e / p, c = e - (e / p) * p;
        if (r0 + r < n) out[(long)(r0 + r) * p + c] = o[cnt];
    }
}

// ---------------------------------------------------------------- output

// Leading k columns of the row-major n x ldv block Vr (descending order):
// largest-magnitude entry made positive (lowest index on ties), written as
// Ut[l, i] = u_l[i] and Ux[l, a2, a1] = u_l[a1 * dx + a2].
__device__ __forceinline__ void put_val(const Buf& o, size_t idx, double v) {
    switch (o.fmt) {
        case Fmt::F64: static_cast<double*>(o.ptr)[idx] = v; break;
        case Fmt::F32: static_cast<float*>(o.ptr)[idx] = (float)v; break;
        default: {
            __bf16* q = static_cast<__bf16*>(o.ptr);
            const float f = (float)v;
            const __bf16 h = (__bf16)f;
            q[idx] = h;
            const float r = f - (float)h;
            const __bf16 m = (__bf16)r;
            q[idx + o.plane] = m;
            if (o.fmt == Fmt::BF16x3) q[idx + 2 * o.plane] = (__bf16)(r - (float)m);
        }
    }
}

// One block per kept column l.
__global__ __launch_bounds__(256) void eig_select_kernel(const double* __restrict__ Vr, int ldv, int n, int dx, int k,
                                                         Buf Ut, Buf Ux) {
    __shared__ double sv[256];
    __shared__ int si[256];
    const int l = blockIdx.x;
    double best = -1.0;
    int bi = 0x7fffffff;
    for (int i = threadIdx.x; i < n; i += 256) {
        const double a = fabs(Vr[(long)i * ldv + l]);
        if (a > best) { best = a; bi = i; }
    }
    sv[threadIdx.x] = best;
    si[threadIdx.x] = bi;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            const double a = sv[threadIdx.x + s];
            const int ia = si[threadIdx.x + s];
            if (a > sv[threadIdx.x] || (a == sv[threadIdx.x] && ia < si[threadIdx.x])) {
                sv[threadIdx.x] = a;
                si[threadIdx.x] = ia;
            }
        }
        __syncthreads();
    }
    const double sgn = Vr[(long)si[0] * ldv + l] < 0.0 ? -1.0 : 1.0;
    for (int i = threadIdx.x; i < n; i += 256) {
        const double u = sgn * Vr[(long)i * ldv + l];
        put_val(Ut, (size_t)l * n + i, u);
        const int a1 = i / dx, a2 = i - (i / dx) * dx;
        put_val(Ux, ((size_t)l * dx + a2) * dx + a1, u);
    }
}

__global__ __launch_bounds__(64) void eig_stats_kernel(const double* __restrict__ theta, int p, int n, int k,
                                                       const EigCtl* ctl, DevState* st, int step, int slot,
                                                       double fail_tol) {
    if (threadIdx.x != 0 || step >= 64) return;
    // how the solve ended, and whether it failed: a dense diagonalisation
    // (p == n) fails only at its sweep cap; a subspace solve that stopped
    // short of the convergence bound fails when its residual is above
    // fail_tol (NaN included); non-finite eigenvalues fail either way
    int stop;
    bool failed;
    if (p == n) {
        stop = ctl->jac_capped ? HOTRG_EIG_PASS_CAP : HOTRG_EIG_CONVERGED;
        failed = ctl->jac_capped != 0;
    } else {
        stop = ctl->converged ? HOTRG_EIG_CONVERGED : (ctl->stall >= 3 ? HOTRG_EIG_STAGNATED : HOTRG_EIG_PASS_CAP);
        failed = !ctl->converged && !(ctl->resid <= fail_tol);
    }
    if (!isfinite(theta[0])) failed = true;
    if (failed && st->status == 0) st->status = HOTRG_EEIG;
    double err;
    if (p == n) {   // every eigenvalue known: discarded weight summed directly
        double tot = 0.0, dis = 0.0;
        for (int j = 0; j < n; ++j) {
            tot += theta[j];
            if (j >= k) dis += theta[j];
        }
        err = tot != 0.0 ? dis / tot : 0.0;
    } else {
        double kept = 0.0;
        for (int j = 0; j < k; ++j) kept += theta[j];
        const double tr = ctl->trace;
        err = tr != 0.0 ? (tr - kept) / tr : 0.0;
    }
    const double gap = k < n ? (k < p ? (theta[k - 1] - theta[k]) / theta[0] : NAN) : INFINITY;
    if (slot == 0) {
        st->trunc_err[step] = err;
        st->eps_left[step] = err;
        st->cut_gap[step] = gap;
        st->info[step] = ctl->iters;
        st->eig_resid[step] = ctl->resid;
        st->eig_sweeps[step] = ctl->sweeps;
        st->eig_stop[step] = stop;
        st->side[step] = 0;
    } else {
        st->eps_right[step] = err;
        st->r_cut_gap[step] = gap;
        st->r_info[step] = ctl->iters;
        st->r_resid[step] = ctl->resid;
        st->r_sweeps[step] = ctl->sweeps;
        st->r_eig_stop[step] = stop;
    }
}

// Two-sided truncation (the side with the smaller discarded weight wins,
// ties keep the left one).  Every block reads the same two numbers, so all
// take the same branch; block 0 records the outcome.
__global__ __launch_bounds__(256) void choose_side_kernel(DevState* st, int step, uint4* __restrict__ Ut,
                                                          uint4* __restrict__ Ux, const uint4* __restrict__ UtR,
                                                          const uint4* __restrict__ UxR, size_t words) {
    if (step >= 64) return;
    const bool right = st->eps_right[step] < st->eps_left[step];
    if (right) {
        for (size_t i = blockIdx.x * (size_t)256 + threadIdx.x; i < words; i += (size_t)gridDim.x * 256) {
            Ut[i] = UtR[i];
            Ux[i] = UxR[i];
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->side[step] = right ? 1 : 0;
        if (right) {
            st->trunc_err[step] = st->eps_right[step];
            st->cut_gap[step] = st->r_cut_gap[step];
            st->info[step] = st->r_info[step];
            st->eig_resid[step] = st->r_resid[step];
            st->eig_sweeps[step] = st->r_sweeps[step];
            st->eig_stop[step] = st->r_eig_stop[step];
        }
    }
}

// ---------------------------------------------------------------- host side

static unsigned grid_for(long count, int per) { return (unsigned)((count + per - 1) / per); }

// One thread copies the eigensolve's stop state to host memory as one
// system-scope store, so that the host sees it without a copy engine or an
// event.
__global__ __launch_bounds__(64) void eig_mail_kernel(const EigCtl* __restrict__ ctl, EigMail* mail, int seq) {
    if (threadIdx.x != 0) return;
    const unsigned long long word = ((unsigned long long)(unsigned)seq << 32) |
                                    ((unsigned long long)(unsigned)ctl->iters << 1) | (ctl->done ? 1ull : 0ull);
    __hip_atomic_store(&mail->word, word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

hipError_t launch_eig_mail(const EigCtl* ctl, EigMail* mail, int seq, hipStream_t stream) {
    hipLaunchKernelGGL(eig_mail_kernel, dim3(1), dim3(64), 0, stream, ctl, mail, seq);
    return hipGetLastError();
}

hipError_t launch_choose_side(DevState* st, int step, void* Ut, void* Ux, const void* UtR, const void* UxR,
                              size_t bytes, hipStream_t stream) {
    if (bytes % 16) return hipErrorInvalidValue;
    const size_t words = bytes / 16;
    unsigned blocks = grid_for((long)words, 256);
    if (blocks > 1024) blocks = 1024;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(choose_side_kernel, dim3(blocks), dim3(256), 0, stream, st, step, static_cast<uint4*>(Ut),
                       static_cast<uint4*>(Ux), static_cast<const uint4*>(UtR), static_cast<const uint4*>(UxR), words);
    return hipGetLastError();
}

hipError_t launch_eig_topk(const double* E, int n, int k, int dx, const EigWork& w, int parity, bool warm,
                           unsigned long long seed, int maxit, double tol, double fail_tol, const Buf& Ut,
                           const Buf& Ux, DevState* st, int step, hipStream_t stream, int slot,
                           const EigRange& range) {
    if (n < 1 || k < 1 || k > n || maxit < 1) return hipErrorInvalidValue;
    const int it_first = range.first < 0 ? 0 : range.first;
    const int it_last = range.last < 0 || range.last > maxit ? maxit : range.last;
    if (n <= EIG_PMAX) {
        if (!range.start) return hipSuccess;
        hipLaunchKernelGGL(eig_init_kernel, dim3(1), dim3(256), 0, stream, E, n, (double*)nullptr, 0, 1, seed, w.ctl);
        hipLaunchKernelGGL(eig_jacobi_kernel, dim3(1), dim3(EIG_JT), 0, stream, E, n, n, w.theta, w.S, w.ctl, 0);
        hipLaunchKernelGGL(eig_select_kernel, dim3(k), dim3(256), 0, stream, w.S, n, n, dx, k, Ut, Ux);
        hipLaunchKernelGGL(eig_stats_kernel, dim3(1), dim3(64), 0, stream, w.theta, n, n, k, w.ctl, st, step, slot,
                           fail_tol);
        return hipGetLastError();
    }
    const int p = eig_block(n, k);
    if (p <= k || p % 16) return hipErrorInvalidValue;
    double* V = w.V[parity];
    const int pstride = EIG_PMAX * EIG_PMAX + EIG_PMAX;
    const int nb = (n + EIG_GRAM_ROWS - 1) / EIG_GRAM_ROWS;
    const unsigned g_init = grid_for((long)n * p, 256) > 1024 ? 1024 : grid_for((long)n * p, 256);
    if (range.start)
        hipLaunchKernelGGL(eig_init_kernel, dim3(g_init), dim3(256), 0, stream, E, n, V, p, warm ? 1 : 0, seed,
                           w.ctl);

    auto orth = [&](const double* src, double shift1, unsigned long long s2) {
        // pass 1 (column-scaled, shifted) from src into V, pass 2 in place
        hipLaunchKernelGGL(eig_gram_kernel, dim3(nb), dim3(256), 0, stream, src, src, n, p, w.part, pstride, w.ctl);
        hipLaunchKernelGGL(eig_reduce_kernel, dim3(grid_for(p * p, 256)), dim3(256), 0, stream, w.part, nb, pstride,
                           p * p, w.G, w.ctl);
        hipLaunchKernelGGL(eig_chol_kernel, dim3(1), dim3(1024), 0, stream, w.G, n, p, k, w.theta, tol, -1, maxit - 1,
                           shift1, w.L, w.dsc, w.ctl);
        hipLaunchKernelGGL(eig_orth_apply_kernel, dim3(nb), dim3(256), 0, stream, src, V, n, p, w.L, w.dsc, s2,
                           w.ctl);
        hipLaunchKernelGGL(eig_gram_kernel, dim3(nb), dim3(256), 0, stream, V, V, n, p, w.part, pstride, w.ctl);
        hipLaunchKernelGGL(eig_reduce_kernel, dim3(grid_for(p * p, 256)), dim3(256), 0, stream, w.part, nb, pstride,
                           p * p, w.G, w.ctl);
        hipLaunchKernelGGL(eig_chol_kernel, dim3(1), dim3(1024), 0, stream, w.G, n, p, k, w.theta, tol, -1, maxit - 1,
                           0.0, w.L, w.dsc, w.ctl);
        hipLaunchKernelGGL(eig_orth_apply_kernel, dim3(nb), dim3(256), 0, stream, V, V, n, p, w.L, w.dsc, s2 + 1,
                           w.ctl);
    };
    const double shift = 1e-13;
    if (range.start) orth(V, shift, seed * 31 + 7);
    for (int it = it_first; it < it_last; ++it) {
        hipLaunchKernelGGL(eig_ev_kernel, dim3(grid_for(n, 16)), dim3(256), 0, stream, E, n, V, w.W, p, w.ctl);
        if (it % EIG_RR_EVERY != EIG_RR_EVERY - 1 && it != maxit - 1) {
            // power step without Rayleigh-Ritz: V <- orth(E V)
            hipLaunchKernelGGL(eig_gram_kernel, dim3(nb), dim3(256), 0, stream, w.W, w.W, n, p, w.part, pstride,
                               w.ctl);
            hipLaunchKernelGGL(eig_reduce_kernel, dim3(grid_for(p * p, 256)), dim3(256), 0, stream, w.part, nb,
                               pstride, p * p, w.G, w.ctl);
            hipLaunchKernelGGL(eig_chol_kernel, dim3(1), dim3(1024), 0, stream, w.G, n, p, k, w.theta, tol, -1,
                               maxit - 1, shift, w.L, w.dsc, w.ctl);
            hipLaunchKernelGGL(eig_orth_apply_kernel, dim3(nb), dim3(256), 0, stream, w.W, V, n, p, w.L, w.dsc,
                               seed * 131 + it, w.ctl);
            continue;
        }
        hipLaunchKernelGGL(eig_gram_kernel, dim3(nb), dim3(256), 0, stream, V, w.W, n, p, w.part, pstride, w.ctl);
        hipLaunchKernelGGL(eig_reduce_kernel, dim3(grid_for(p * p, 256)), dim3(256), 0, stream, w.part, nb, pstride,
                           p * p, w.G, w.ctl);
        hipLaunchKernelGGL(eig_jacobi_kernel, dim3(1), dim3(EIG_JT), 0, stream, w.G, p, p, w.theta, w.S, w.ctl, 1);
        hipLaunchKernelGGL(eig_rotate_kernel, dim3(nb), dim3(256), 0, stream, V, w.W, n, p, w.S, w.theta, w.part,
                           pstride, w.ctl);
        hipLaunchKernelGGL(eig_reduce_kernel, dim3(grid_for(p * p + p, 256)), dim3(256), 0, stream, w.part, nb,
                           pstride, p * p + p, w.G, w.ctl);
        hipLaunchKernelGGL(eig_chol_kernel, dim3(1), dim3(1024), 0, stream, w.G, n, p, k, w.theta, tol, it, maxit - 1,
                           shift, w.L, w.dsc, w.ctl);
        // one CholeskyQR pass: the column-scaled Ritz block W is close to
        // orthonormal, so a second pass is not needed inside the iteration
        hipLaunchKernelGGL(eig_orth_apply_kernel, dim3(nb), dim3(256), 0, stream, w.W, V, n, p, w.L, w.dsc,
                           seed * 131 + it, w.ctl);
    }
    if (!range.end) return hipGetLastError();
    hipLaunchKernelGGL(eig_select_kernel, dim3(k), dim3(256), 0, stream, V, p, n, dx, k, Ut, Ux);
    hipLaunchKernelGGL(eig_stats_kernel, dim3(1), dim3(64), 0, stream, w.theta, p, n, k, w.ctl, st, step, slot,
                       fail_tol);
    return hipGetLastError();
}

}  // namespace hotrg
