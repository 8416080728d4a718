// iTEBD on the device: many independent infinite chains, one workgroup per
// chain, all FP64.  The decomposition's work matrix lives in LDS (37 KB, so
// up to four chains share a CU); B1 and B2 are staged into it from the
// chain's state row at the start of each update and written back at its
// end, and the evolved pair P goes to the chain's workspace slice
// (column-major, read row-parallel by the product B1' = P Y_kept, and small
// enough to stay in L2).  The C ABI is declared in include/itebd.h.
//
// One bond update (Sec. II.A, Eq. (1); the inverse-free form of the iTEBD
// update), n = 2 chi:
//   P[(a s),(t b)] = sum_c B1[s][a][c] B2[t][c][b]          (contraction)
//   P <- G P on the physical pair (s, t) of every (a, b)     (gate)
//   W = diag(lambda_2 (x) 1) P
//   W Pi = Q R: Householder QR with column pivoting (Pi the permutation)
//   one-sided Jacobi on the columns of A = R^T:  A J = U S
//     then W = Q J S U^T Pi^T, so the right singular vectors of W are
//     Y = Pi U: the normalised final columns of A, rows permuted back; no
//     rotation is accumulated and the left vectors are never formed
//   keep the chi largest; sign gauge on the kept columns of Y
//   B2' = Y_kept^T, B1' = P Y_kept / |S_kept|, lambda_1' = S_kept / |S_kept|
//   exchange the sites' roles
// Pivoting makes R graded, with columns of A = R^T close to orthogonal, so
// the Jacobi method needs about half the sweeps of a cold start on W (the
// preconditioning of Drmac and Veselic, SIAM J. Matrix Anal. Appl. 29
// (2008)), and each sweep rotates one matrix instead of two.
//
// Lanes: groups of eight lanes, one group per column pair in a Jacobi round
// and per trailing column (two of them) in a QR step; a lane holds rows
// l, l + 8, ..., l + 56 of its columns in registers.  A pair's three dot
// products and a column's reflector product are reduced over the eight lanes
// with DPP moves (every lane gets the same bits: each stage adds two equal
// partial sums in either order).  The Jacobi sweep visits all column pairs
// in n - 1 rounds of n/2 disjoint pairs (round-robin ordering, the systolic
// schedule of Sec. II.B used for one-sided rotations).  A QR step is one
// barrier: every wave finds the pivot (the largest remaining column norm,
// lowest index on ties) and the reflector itself from the norms the previous
// step left in LDS, keeps the column permutation in registers (lane j holds
// the storage column of logical column j), and the groups then update the
// trailing columns and write their new norms for the next step.  The work
// matrix is column-major with a column stride ld = 8 (mod 32) doubles: the
// eight groups of a wave read eight consecutive doubles each from columns
// ld apart, which spreads a wave's read evenly over the banks.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <new>

#include "../../include/itebd.h"

namespace {

constexpr int kMaxChi = ITEBD_MAX_CHI;
constexpr int kMaxN = 2 * kMaxChi;
// column stride of the work matrix, 8 (mod 32) doubles; every column has
// kMaxN rows, those at and beyond n held at zero, so the row loops need no
// bounds
constexpr int kLd = 72;
static_assert(kLd >= kMaxN && kLd % 32 == 8, "column stride");
static_assert(4 * kMaxChi * kMaxChi <= kMaxN * kLd, "B1 and B2 are staged in the work matrix");
constexpr int kLanes = 8;                       // lanes per Jacobi pair / QR column
constexpr int kRows = kMaxN / kLanes;           // rows per lane
constexpr int kGroups = kMaxN / 2;              // lane groups (one per pair of a round)
constexpr int kUpdThreads = kLanes * kGroups;   // update kernel
constexpr int kThreads = 256;                   // energy kernel
static_assert(kMaxN <= 64, "a QR step holds one remaining row or column per lane of a wave");
static_assert(2 * kGroups >= kMaxN - 1, "two trailing columns per group cover a QR step");
// the contraction: one 2 x 2 block of (a, b) per thread
static_assert(((kMaxChi + 1) / 2) * ((kMaxChi + 1) / 2) <= kUpdThreads, "contraction blocks");
// the transposition R -> A through registers
constexpr int kPerThread = (kMaxN * kMaxN + kUpdThreads - 1) / kUpdThreads;
// the product B1' = P Y_kept: kUpdThreads / n >= 4 groups of n lanes, each
// lane one row and at most this many kept columns
constexpr int kMaxColsPerLane = (kMaxChi + 3) / 4;
static_assert(kUpdThreads / kMaxN >= 4, "row-parallel product assumes at least 4 lane groups");
constexpr int kUpdatesPerLaunch = 32;
// rotate a pair while |a_p.a_q| > kTol |a_p| |a_q| (relative test)
constexpr double kTol = 1e-14;

struct Gate {
    double g[16];   // exp(-tau h), row-major [(s' t'), (s t)]
};

// a double from another lane of the same row through a DPP move of each half
template <int Ctrl>
__device__ __forceinline__ double dpp_d(double v) {
    const unsigned long long u = (unsigned long long)__double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)u, Ctrl, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(u >> 32), Ctrl, 0xF, 0xF, false);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// sum over an aligned group of eight lanes: partner lane ^1 (quad_perm
// [1,0,3,2]), ^2 (quad_perm [2,3,0,1]), then the mirror lane 7 - l inside
// the half-row (the other quad)
__device__ __forceinline__ double sum8(double v) {
    v += dpp_d<0xB1>(v);
    v += dpp_d<0x4E>(v);
    v += dpp_d<0x141>(v);
    return v;
}

// sum over a row of sixteen lanes: sum8, then the mirror lane 15 - l inside
// the row (the other half-row)
__device__ __forceinline__ double sum16(double v) {
    v = sum8(v);
    v += dpp_d<0x140>(v);
    return v;
}

template <int Ctrl>
__device__ __forceinline__ int dpp_i(int v) {
    return __builtin_amdgcn_update_dpp(0, v, Ctrl, 0xF, 0xF, false);
}

// a double of lane l (uniform l) in every lane
__device__ __forceinline__ double readlane_d(double v, int l) {
    const unsigned long long u = (unsigned long long)__double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(unsigned)u, l);
    const int hi = __builtin_amdgcn_readlane((int)(unsigned)(u >> 32), l);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// sum over the 64 lanes of a wave: the four row sums (sum16), read from one
// lane of each row and added in a fixed order, so every lane, and every wave
// holding the same data, gets the same bits
__device__ __forceinline__ double wave_sum(double v) {
    v = sum16(v);
    return (readlane_d(v, 0) + readlane_d(v, 16)) + (readlane_d(v, 32) + readlane_d(v, 48));
}

// (v, i) beats (w, j): larger value, lower index on ties
__device__ __forceinline__ bool beats(double v, int i, double w, int j) { return v > w || (v == w && i < j); }

template <int Ctrl>
__device__ __forceinline__ void argmax_step(double& v, int& i) {
    const double ov = dpp_d<Ctrl>(v);
    const int oi = dpp_i<Ctrl>(i);
    if (beats(ov, oi, v, i)) {
        v = ov;
        i = oi;
    }
}

// index of the largest value over the wave (lowest index on ties): the same
// pairings as sum16 inside each row, then the four row winners in order
__device__ __forceinline__ int wave_argmax(double v, int i) {
    argmax_step<0xB1>(v, i);
    argmax_step<0x4E>(v, i);
    argmax_step<0x141>(v, i);
    argmax_step<0x140>(v, i);
    double bv = readlane_d(v, 0);
    int bi = __builtin_amdgcn_readlane(i, 0);
#pragma unroll
    for (int w = 1; w < 4; ++w) {
        const double ov = readlane_d(v, 16 * w);
        const int oi = __builtin_amdgcn_readlane(i, 16 * w);
        if (beats(ov, oi, bv, bi)) {
            bv = ov;
            bi = oi;
        }
    }
    return bi;
}

__global__ __launch_bounds__(kUpdThreads) __attribute__((amdgpu_waves_per_eu(2)))
void itebd_update_kernel(double* __restrict__ states, double* __restrict__ pair, int* __restrict__ status,
                         int* __restrict__ sweeps_out, unsigned long long* __restrict__ work, int chi, Gate G,
                         int nupd, int max_sweeps)
{
    __shared__ double sA[kMaxN * kLd];      // work matrix, column-major, stride kLd; stages B1 and B2
    __shared__ double sl1[kMaxChi], sl2[kMaxChi];
    __shared__ double sG[16];                // the gate (read from LDS: no long-lived scalar copies)
    __shared__ double scn[2][kMaxN];         // squared norms of the remaining columns, by QR step parity
    __shared__ double sdiag[kMaxN];          // diagonal of R
    __shared__ double ssig[kMaxN], ssgn[kMaxChi], sscale[kMaxChi];
    __shared__ int scol[kMaxN], sinv[kMaxN], sord[kMaxChi];
    __shared__ int srot;
    __shared__ unsigned long long srotc;
    __shared__ double snrm;

    const int tid = threadIdx.x;
    if (status[blockIdx.x] & ITEBD_CHAIN_NONFINITE) return;   // a failed chain stays as it was
    const int n = 2 * chi;
    constexpr int ld = kLd;
    const int nb = 2 * chi * chi;
    const long len = 2L * nb + 2 * chi;
    double* st = states + (long)blockIdx.x * len;        // B1 and B2 are rewritten every update
    double* gP = pair + (long)blockIdx.x * n * n;        // P, column-major: P[(a s),(t b)] at (t b) n + (a s)
    const int lane = tid & 63;
    const int g = tid / kLanes, r = tid % kLanes;
    const int ng = kUpdThreads / n;                      // lane groups of the row-parallel product (>= 4)
    const int prow = tid % n, pgrp = tid / n;

    for (int i = tid; i < chi; i += kUpdThreads) {
        sl1[i] = st[2 * nb + i];
        sl2[i] = st[2 * nb + chi + i];
    }
    if (tid < 16) sG[tid] = G.g[tid];
    if (tid == 0) srotc = 0;
    __syncthreads();

    int max_sw = 0, fail = 0;
    unsigned long long tot_sweeps = 0;
    unsigned nrot = 0;   // rotations of this lane's group (counted by its lane 0)
    for (int u = 0; u < nupd; ++u) {
        // stage B1 and B2 in the work matrix
        double* sB1 = sA;
        double* sB2 = sA + nb;
        for (int i = tid; i < nb; i += kUpdThreads) {
            sB1[i] = st[i];
            sB2[i] = st[nb + i];
        }
        __syncthreads();
        // contraction P[(a s),(t b)] = sum_c B1[s][a][c] B2[t][c][b] and the gate on
        // the physical pair: a 2 x 2 block of (a, b) per thread, its sixteen (s, t)
        const int nbk = (chi + 1) / 2;
        double pw[16];
        const bool blk = tid < nbk * nbk;
        const int a0 = 2 * (tid / nbk), b0 = 2 * (tid % nbk);
        if (blk) {
            double acc[16];
#pragma unroll
            for (int e = 0; e < 16; ++e) acc[e] = 0.0;
            const bool a1 = a0 + 1 < chi, b1 = b0 + 1 < chi;
            for (int c = 0; c < chi; ++c) {
                double x[2][2], y[2][2];   // x[a'][s], y[t][b']
#pragma unroll
                for (int s = 0; s < 2; ++s) {
                    x[0][s] = sB1[(s * chi + a0) * chi + c];
                    x[1][s] = a1 ? sB1[(s * chi + a0 + 1) * chi + c] : 0.0;
                    y[s][0] = sB2[(s * chi + c) * chi + b0];
                    y[s][1] = b1 ? sB2[(s * chi + c) * chi + b0 + 1] : 0.0;
                }
#pragma unroll
                for (int ap = 0; ap < 2; ++ap)
#pragma unroll
                    for (int s = 0; s < 2; ++s)
#pragma unroll
                        for (int t = 0; t < 2; ++t)
#pragma unroll
                            for (int bp = 0; bp < 2; ++bp) {
                                const int e = ((ap * 2 + s) * 2 + t) * 2 + bp;
                                acc[e] = fma(x[ap][s], y[t][bp], acc[e]);
                            }
            }
#pragma unroll
            for (int ap = 0; ap < 2; ++ap)
#pragma unroll
                for (int bp = 0; bp < 2; ++bp) {
                    double v[4];
#pragma unroll
                    for (int i = 0; i < 4; ++i) v[i] = acc[((ap * 2 + (i >> 1)) * 2 + (i & 1)) * 2 + bp];
#pragma unroll
                    for (int o = 0; o < 4; ++o) {
                        double q = 0.0;
#pragma unroll
                        for (int i = 0; i < 4; ++i) q = fma(sG[4 * o + i], v[i], q);
                        pw[(ap * 2 + bp) * 4 + o] = q;
                        const int a = a0 + ap, b = b0 + bp;
                        if (a < chi && b < chi) gP[((o & 1) * chi + b) * n + 2 * a + (o >> 1)] = q;
                    }
                }
        }
        __syncthreads();   // the staged B1, B2 are no longer needed
        // W = diag(lambda_2 (x) 1) P into the work matrix, rows n.. of its
        // columns zero
        for (int idx = tid; idx < n * (kMaxN - n); idx += kUpdThreads) {
            const int j = idx / (kMaxN - n), i = n + idx - j * (kMaxN - n);
            sA[j * ld + i] = 0.0;
        }
        if (blk) {
#pragma unroll
            for (int ap = 0; ap < 2; ++ap)
#pragma unroll
                for (int bp = 0; bp < 2; ++bp) {
                    const int a = a0 + ap, b = b0 + bp;
                    if (a < chi && b < chi) {
                        const double lam = sl2[a];
#pragma unroll
                        for (int o = 0; o < 4; ++o)
                            sA[((o & 1) * chi + b) * ld + 2 * a + (o >> 1)] = lam * pw[(ap * 2 + bp) * 4 + o];
                    }
                }
        }
        __syncthreads();
        // squared column norms for the first pivot (column j stored at j)
        for (int h = 0; h < 2; ++h) {
            const int l = g + kGroups * h;
            if (l < n) {
                double s2 = 0.0;
#pragma unroll
                for (int m = 0; m < kRows; ++m) {
                    const double a = sA[l * ld + r + kLanes * m];
                    s2 = fma(a, a, s2);
                }
                s2 = sum8(s2);
                if (r == 0) scn[0][l] = s2;
            }
        }
        __syncthreads();

        // Householder QR with column pivoting, one barrier per step
        int col = lane;   // storage column of logical column `lane` (the same in every wave)
        for (int k = 0; k < n - 1; ++k) {
            const int cur = k & 1, nxt = cur ^ 1;
            // storage columns of this group's trailing logical columns k + 1 + g and
            // k + 1 + g + kGroups before this step's swap (fetched while the pivot is found)
            const int l0 = k + 1 + g, l1 = l0 + kGroups;
            const int cb0 = __shfl(col, min(l0, n - 1), 64), cb1 = __shfl(col, min(l1, n - 1), 64);
            // pivot: the largest remaining norm, lowest logical index on ties
            int jm = wave_argmax((lane >= k && lane < n) ? scn[cur][lane] : -1.0, lane);
            if (jm < k || jm >= n) jm = k;   // only with non-finite norms
            const int colk = __builtin_amdgcn_readlane(col, k), coljm = __builtin_amdgcn_readlane(col, jm);
            col = lane == k ? coljm : (lane == jm ? colk : col);
            // the reflector H = I - beta v v^T mapping rows k.. of the pivot column to (alpha, 0, ...)
            const double* Wc = sA + coljm * ld;
            const double x = k + lane < kMaxN ? Wc[k + lane] : 0.0;
            const double sig = wave_sum(x * x);
            const double x0 = readlane_d(x, 0);
            // a remaining column below 1e-140 in norm (zero, in practice) is
            // left as it is: R[k][k] = x0 and the entries below it, which the
            // transposition never reads, are dropped; beta then stays finite
            double al = x0, be = 0.0;
            if (sig > 1e-280) {
                al = -copysign(sqrt(sig), x0);
                be = 1.0 / (sig - x0 * al);
            }
            const double v0 = x0 - al;
            if (tid == 0) sdiag[k] = al;
            if (k == n - 2 && tid < n) scol[tid] = col;   // the final order (wave 0)
            // the swap moved logical column jm's storage to k and k's to jm
            const int c0 = l0 == jm ? colk : cb0, c1 = l1 == jm ? colk : cb1;
            double vv[kRows];
#pragma unroll
            for (int m = 0; m < kRows; ++m) {
                const int i = r + kLanes * m;
                const double wi = Wc[i];
                vv[m] = i > k ? wi : (i == k ? v0 : 0.0);
            }
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int l = h ? l1 : l0;
                if (l < n) {
                    double* Wp = sA + (h ? c1 : c0) * ld;
                    double xr[kRows];
                    double w = 0.0;
#pragma unroll
                    for (int m = 0; m < kRows; ++m) {
                        xr[m] = Wp[r + kLanes * m];
                        w = fma(vv[m], xr[m], w);   // v is zero above row k
                    }
                    w = sum8(w);
                    const double bw = be * w;
                    double s2 = 0.0;
#pragma unroll
                    for (int m = 0; m < kRows; ++m) {
                        const int i = r + kLanes * m;
                        xr[m] = fma(-bw, vv[m], xr[m]);   // rows above k unchanged
                        Wp[i] = xr[m];
                        s2 = fma(i > k ? xr[m] : 0.0, xr[m], s2);
                    }
                    s2 = sum8(s2);
                    if (r == 0) scn[nxt][l] = s2;
                }
            }
            __syncthreads();
        }
        // A = R^T, column-major: A[l][j] = R[j][l] (l >= j); R[j][l] is row j of
        // the storage column of logical column l, R[j][j] the reflector's alpha
        // (row n - 1 has no reflector)
        {
            double tv[kPerThread];
#pragma unroll
            for (int q = 0; q < kPerThread; ++q) {
                const int e = tid + kUpdThreads * q;
                tv[q] = 0.0;
                if (e < n * n) {
                    const int j = e / n, l = e - (e / n) * n;
                    if (l > j || (l == j && j == n - 1)) tv[q] = sA[scol[l] * ld + j];
                    else if (l == j) tv[q] = sdiag[j];
                }
            }
            __syncthreads();
#pragma unroll
            for (int q = 0; q < kPerThread; ++q) {
                const int e = tid + kUpdThreads * q;
                if (e < n * n) {
                    const int j = e / n, l = e - (e / n) * n;
                    sA[j * ld + l] = tv[q];
                }
            }
            if (tid < n) sinv[scol[tid]] = tid;
            __syncthreads();
        }

        // one-sided Jacobi on the columns of A
        const int npair = n >> 1;
        int sweeps = max_sweeps + 1;   // not converged
        for (int sw = 0; sw < max_sweeps; ++sw) {
            if (tid == 0) srot = 0;
            __syncthreads();
            for (int rd = 0; rd < n - 1; ++rd) {
                if (g < npair) {
                    int p, q;
                    if (g == 0) {
                        p = rd;
                        q = n - 1;
                    } else {   // (rd + g) and (rd - g) modulo n - 1, with 1 <= g < n - 1
                        p = rd + g;
                        p -= p >= n - 1 ? n - 1 : 0;
                        q = rd - g;
                        q += q < 0 ? n - 1 : 0;
                    }
                    double* Ap = sA + p * ld;
                    double* Aq = sA + q * ld;
                    double wp[kRows], wq[kRows];
                    double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
                    for (int m = 0; m < kRows; ++m) {
                        wp[m] = Ap[r + kLanes * m];
                        wq[m] = Aq[r + kLanes * m];
                    }
#pragma unroll
                    for (int m = 0; m < kRows; ++m) {
                        al = fma(wp[m], wp[m], al);
                        be = fma(wq[m], wq[m], be);
                        ga = fma(wp[m], wq[m], ga);
                    }
                    al = sum8(al);
                    be = sum8(be);
                    ga = sum8(ga);
                    // rotate while ga^2 > kTol^2 al be (the relative test, squared)
                    if (ga * ga > (kTol * kTol) * (al * be)) {
                        // the smaller root of t^2 + 2 zeta t - 1 = 0, zeta = (be - al) / (2 ga):
                        // t = sign(d) 2ga / (|d| + sqrt(d^2 + 4 ga^2)), d = be - al
                        const double d = be - al, g2 = 2.0 * ga;
                        const double t = (d >= 0.0 ? g2 : -g2) / (fabs(d) + sqrt(fma(d, d, g2 * g2)));
                        const double c = rsqrt(fma(t, t, 1.0)), s = c * t;
#pragma unroll
                        for (int m = 0; m < kRows; ++m) {
                            Ap[r + kLanes * m] = c * wp[m] - s * wq[m];
                            Aq[r + kLanes * m] = s * wp[m] + c * wq[m];
                        }
                        if (r == 0) {
                            srot = 1;
                            ++nrot;
                        }
                    }
                }
                __syncthreads();
            }
            const int any = srot;
            __syncthreads();
            if (!any) {
                sweeps = sw + 1;
                break;
            }
        }
        if (sweeps > max_sweeps) {
            fail |= ITEBD_CHAIN_SWEEP_CAP;   // the last sweep still rotated: used as it stands
            sweeps = max_sweeps;
        }
        max_sw = max(max_sw, sweeps);
        tot_sweeps += (unsigned long long)sweeps;

        // singular values (column norms), the chi largest (ties: lower column first)
        for (int h = 0; h < 2; ++h) {
            const int l = g + kGroups * h;
            if (l < n) {
                double s2 = 0.0;
#pragma unroll
                for (int m = 0; m < kRows; ++m) {
                    const double a = sA[l * ld + r + kLanes * m];
                    s2 = fma(a, a, s2);
                }
                s2 = sum8(s2);
                if (r == 0) ssig[l] = sqrt(s2);
            }
        }
        __syncthreads();
        for (int j = tid; j < n; j += kUpdThreads) {
            int rank = 0;
            for (int i = 0; i < n; ++i) rank += (ssig[i] > ssig[j]) || (ssig[i] == ssig[j] && i < j);
            if (rank < chi) sord[rank] = j;
        }
        __syncthreads();
        // kept right vectors y_c[m] = A[sinv[m]][sord[c]] / sigma: sign gauge (largest
        // magnitude entry positive, the lowest m on ties) and scale; norm of the kept values
        for (int c = tid; c < chi; c += kUpdThreads) {
            const int j = sord[c];
            double best = -1.0;
            int bm = 0;
            for (int m = 0; m < n; ++m) {
                const double a = fabs(sA[j * ld + sinv[m]]);
                if (a > best) {
                    best = a;
                    bm = m;
                }
            }
            const double sgn = sA[j * ld + sinv[bm]] < 0.0 ? -1.0 : 1.0;
            ssgn[c] = sgn;
            sscale[c] = ssig[j] > 0.0 ? sgn / ssig[j] : 0.0;   // a zero value keeps a zero vector
        }
        if (tid == 0) {
            double acc = 0.0;
            for (int c = 0; c < chi; ++c) acc = fma(ssig[sord[c]], ssig[sord[c]], acc);
            snrm = sqrt(acc);
        }
        __syncthreads();
        const double nrm = snrm;
        if (!(nrm > 0.0) || !isfinite(nrm)) {   // the same in every thread
            fail |= ITEBD_CHAIN_NONFINITE;      // this update is not applied, and no later one
            break;
        }
        // new tensors, roles exchanged, into the state row:
        //   B1 <- B2' = Y_kept^T, B2 <- B1' = P Y_kept / nrm
        const double inv = 1.0 / nrm;
        for (int idx = tid; idx < nb; idx += kUpdThreads) {
            const int t = idx / (chi * chi), rem = idx - t * chi * chi;
            const int c = rem / chi, b = rem - (rem / chi) * chi;
            st[idx] = sscale[c] * sA[sord[c] * ld + sinv[t * chi + b]];
        }
        if (pgrp < ng) {   // row (a s) = prow, kept columns c = pgrp, pgrp + ng, ...
            double acc[kMaxColsPerLane];
#pragma unroll
            for (int q = 0; q < kMaxColsPerLane; ++q) acc[q] = 0.0;
            for (int i = 0; i < n; ++i) {
                const double pk = gP[scol[i] * n + prow];
#pragma unroll
                for (int q = 0; q < kMaxColsPerLane; ++q) {
                    const int c = pgrp + q * ng;
                    if (c < chi) acc[q] = fma(pk, sA[sord[c] * ld + i], acc[q]);
                }
            }
            const int a = prow >> 1, sp = prow & 1;
#pragma unroll
            for (int q = 0; q < kMaxColsPerLane; ++q) {
                const int c = pgrp + q * ng;
                if (c < chi) st[nb + (sp * chi + a) * chi + c] = sscale[c] * inv * acc[q];
            }
        }
        for (int c = tid; c < chi; c += kUpdThreads) {
            const double old = sl2[c];
            sl2[c] = ssig[sord[c]] * inv;
            sl1[c] = old;
        }
        __syncthreads();
    }

    // the weights of the last applied update (after a failed one, the state
    // row still holds that update's tensors)
    for (int i = tid; i < chi; i += kUpdThreads) {
        st[2 * nb + i] = sl1[i];
        st[2 * nb + chi + i] = sl2[i];
    }
    if (r == 0 && nrot) atomicAdd(&srotc, (unsigned long long)nrot);
    __syncthreads();
    if (tid == 0) {
        sweeps_out[blockIdx.x] = max_sw;
        work[2 * blockIdx.x] += tot_sweeps;
        work[2 * blockIdx.x + 1] += srotc;
        status[blockIdx.x] |= fail;
    }
}

// Energy per site of every chain: <h> on bond (B1, B2) weighted by lambda_2
// and on bond (B2, B1) weighted by lambda_1, averaged.  Fixed-order sums.
__global__ __launch_bounds__(kThreads) void itebd_energy_kernel(const double* __restrict__ states, int chi,
                                                                Gate H, double* __restrict__ energies)
{
    __shared__ double sP[kMaxN * kMaxN];
    __shared__ double red[2][kThreads];
    const int tid = threadIdx.x;
    const int n = 2 * chi;
    const int nb = 2 * chi * chi;
    const long len = 2L * nb + 2 * chi;
    const double* st = states + (long)blockIdx.x * len;
    double e[2];
    for (int bond = 0; bond < 2; ++bond) {
        const double* X = st + (bond == 0 ? 0 : nb);
        const double* Y = st + (bond == 0 ? nb : 0);
        const double* lw = st + 2 * nb + (bond == 0 ? chi : 0);
        for (int idx = tid; idx < n * n; idx += kThreads) {
            const int r = idx / n, k = idx - (idx / n) * n;
            const int a = r >> 1, s = r & 1, t = k / chi, b = k - (k / chi) * chi;
            double acc = 0.0;
            for (int c = 0; c < chi; ++c) acc = fma(X[(s * chi + a) * chi + c], Y[(t * chi + c) * chi + b], acc);
            sP[idx] = lw[a] * acc;
        }
        __syncthreads();
        double num = 0.0, den = 0.0;
        for (int idx = tid; idx < chi * chi; idx += kThreads) {
            const int a = idx / chi, b = idx - (idx / chi) * chi;
            double v[4];
            for (int s = 0; s < 2; ++s)
                for (int t = 0; t < 2; ++t) v[2 * s + t] = sP[(2 * a + s) * n + t * chi + b];
            for (int o = 0; o < 4; ++o) {
                double hv = 0.0;
                for (int i = 0; i < 4; ++i) hv = fma(H.g[4 * o + i], v[i], hv);
                num = fma(v[o], hv, num);
                den = fma(v[o], v[o], den);
            }
        }
        red[0][tid] = num;
        red[1][tid] = den;
        __syncthreads();
        for (int s = kThreads / 2; s > 0; s >>= 1) {
            if (tid < s) {
                red[0][tid] += red[0][tid + s];
                red[1][tid] += red[1][tid + s];
            }
            __syncthreads();
        }
        e[bond] = red[0][0] / red[1][0];
        __syncthreads();
    }
    if (tid == 0) energies[blockIdx.x] = 0.5 * (e[0] + e[1]);
}

size_t round_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

struct Layout {
    size_t states, pair, status, sweeps, work, energies, total;
};

Layout plan(int batch, int chi) {
    const size_t len = 4 * (size_t)chi * chi + 2 * (size_t)chi;
    const size_t n = 2 * (size_t)chi;
    Layout L;
    size_t o = 0;
    L.states = o;
    o = round_up(o + 8 * len * batch, 256);
    L.pair = o;
    o = round_up(o + 8 * n * n * batch, 256);
    L.status = o;
    o = round_up(o + 4 * (size_t)batch, 256);
    L.sweeps = o;
    o = round_up(o + 4 * (size_t)batch, 256);
    L.work = o;
    o = round_up(o + 16 * (size_t)batch, 256);
    L.energies = o;
    o = round_up(o + 8 * (size_t)batch, 256);
    L.total = o;
    return L;
}

// G = exp(-tau h) for a real symmetric 4 x 4 h: cyclic Jacobi eigen-
// decomposition h = Q diag(w) Q^T on the host, then Q diag(exp(-tau w)) Q^T.
Gate gate_of(const double* h, double tau) {
    double A[16], Q[16];
    memcpy(A, h, sizeof A);
    for (int i = 0; i < 16; ++i) Q[i] = (i % 5 == 0) ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 50; ++sweep) {
        double off = 0.0;
        for (int p = 0; p < 4; ++p)
            for (int q = p + 1; q < 4; ++q) off += A[4 * p + q] * A[4 * p + q];
        if (off < 1e-300) break;
        for (int p = 0; p < 4; ++p)
            for (int q = p + 1; q < 4; ++q) {
                const double apq = A[4 * p + q];
                if (apq == 0.0) continue;
                const double z = (A[4 * q + q] - A[4 * p + p]) / (2.0 * apq);
                const double t = (z >= 0.0 ? 1.0 : -1.0) / (fabs(z) + sqrt(1.0 + z * z));
                const double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
                for (int k = 0; k < 4; ++k) {   // A <- J^T A J, columns then rows
                    const double akp = A[4 * k + p], akq = A[4 * k + q];
                    A[4 * k + p] = c * akp - s * akq;
                    A[4 * k + q] = s * akp + c * akq;
                }
                for (int k = 0; k < 4; ++k) {
                    const double apk = A[4 * p + k], aqk = A[4 * q + k];
                    A[4 * p + k] = c * apk - s * aqk;
                    A[4 * q + k] = s * apk + c * aqk;
                }
                for (int k = 0; k < 4; ++k) {
                    const double qkp = Q[4 * k + p], qkq = Q[4 * k + q];
                    Q[4 * k + p] = c * qkp - s * qkq;
                    Q[4 * k + q] = s * qkp + c * qkq;
                }
            }
    }
    Gate G;
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            double acc = 0.0;
            for (int k = 0; k < 4; ++k) acc += Q[4 * i + k] * exp(-tau * A[4 * k + k]) * Q[4 * j + k];
            G.g[4 * i + j] = acc;
        }
    return G;
}

}  // namespace

struct itebd_batch;
static int chain_status(itebd_batch* b, int* per_chain);

struct itebd_batch {
    int batch = 0, chi = 0;
    double h[16];
    hipStream_t stream = nullptr;
    char* ws = nullptr;
    Layout L;
    long updates = 0;
    int max_sweeps = ITEBD_MAX_SWEEPS;
    int host_status = HOTRG_OK;
    double* states() const { return reinterpret_cast<double*>(ws + L.states); }
};

extern "C" {

size_t itebd_state_len(int chi) {
    if (chi < 1 || chi > ITEBD_MAX_CHI) return 0;
    return 4 * (size_t)chi * chi + 2 * (size_t)chi;
}

size_t itebd_workspace_bytes(int batch, int chi) {
    if (batch < 1 || batch > (1 << 20) || chi < 1 || chi > ITEBD_MAX_CHI) return 0;
    return plan(batch, chi).total;
}

int itebd_init(int batch, int chi, const double* h, const double* states, void* workspace, size_t ws_bytes,
               void* stream, itebd_batch** out) {
    if (!out) return HOTRG_EINVAL;
    *out = nullptr;
    if (batch < 1 || batch > (1 << 20) || chi < 1 || chi > ITEBD_MAX_CHI || !h || !states || !workspace ||
        ((uintptr_t)workspace & 255u))
        return HOTRG_EINVAL;
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j)
            if (!isfinite(h[4 * i + j]) || h[4 * i + j] != h[4 * j + i]) return HOTRG_EINVAL;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return HOTRG_ENODEV;
    const Layout L = plan(batch, chi);
    if (ws_bytes < L.total) return HOTRG_ENOMEM;
    itebd_batch* b = new (std::nothrow) itebd_batch();
    if (!b) return HOTRG_EINVAL;
    b->batch = batch;
    b->chi = chi;
    memcpy(b->h, h, sizeof b->h);
    b->stream = static_cast<hipStream_t>(stream);
    b->ws = static_cast<char*>(workspace);
    b->L = L;
    const size_t bytes = 8 * itebd_state_len(chi) * (size_t)batch;
    if (hipMemcpyAsync(b->states(), states, bytes, hipMemcpyHostToDevice, b->stream) != hipSuccess ||
        hipMemsetAsync(b->ws + L.status, 0, 4 * (size_t)batch, b->stream) != hipSuccess ||
        hipMemsetAsync(b->ws + L.sweeps, 0, 4 * (size_t)batch, b->stream) != hipSuccess ||
        hipMemsetAsync(b->ws + L.work, 0, 16 * (size_t)batch, b->stream) != hipSuccess ||
        hipStreamSynchronize(b->stream) != hipSuccess) {
        delete b;
        return HOTRG_EHIP;
    }
    *out = b;
    return HOTRG_OK;
}

int itebd_evolve(itebd_batch* b, double tau, int nupdates) {
    if (!b || nupdates < 0 || !(tau > 0.0) || !isfinite(tau)) return HOTRG_EINVAL;
    if (b->host_status) return HOTRG_ESTATE;
    const Gate G = gate_of(b->h, tau);
    double* pair = reinterpret_cast<double*>(b->ws + b->L.pair);
    int* status = reinterpret_cast<int*>(b->ws + b->L.status);
    int* sweeps = reinterpret_cast<int*>(b->ws + b->L.sweeps);
    unsigned long long* work = reinterpret_cast<unsigned long long*>(b->ws + b->L.work);
    for (int done = 0; done < nupdates;) {
        const int k = std::min(kUpdatesPerLaunch, nupdates - done);
        hipLaunchKernelGGL(itebd_update_kernel, dim3((unsigned)b->batch), dim3(kUpdThreads), 0, b->stream, b->states(),
                           pair, status, sweeps, work, b->chi, G, k, b->max_sweeps);
        if (hipGetLastError() != hipSuccess) {
            b->host_status = HOTRG_EHIP;
            return HOTRG_EHIP;
        }
        b->updates += k;
        done += k;
    }
    return HOTRG_OK;
}

int itebd_energy(itebd_batch* b, double* energies) {
    if (!b || !energies) return HOTRG_EINVAL;
    if (b->host_status) return b->host_status;
    Gate H;
    memcpy(H.g, b->h, sizeof H.g);
    double* dev = reinterpret_cast<double*>(b->ws + b->L.energies);
    hipLaunchKernelGGL(itebd_energy_kernel, dim3((unsigned)b->batch), dim3(kThreads), 0, b->stream, b->states(),
                       b->chi, H, dev);
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(energies, dev, 8 * (size_t)b->batch, hipMemcpyDeviceToHost, b->stream) != hipSuccess ||
        hipStreamSynchronize(b->stream) != hipSuccess)
        return HOTRG_EHIP;
    return chain_status(b, nullptr);
}

int itebd_copy_states(itebd_batch* b, double* host, size_t capacity) {
    if (!b || !host) return HOTRG_EINVAL;
    const size_t count = itebd_state_len(b->chi) * (size_t)b->batch;
    if (capacity < count) return HOTRG_EINVAL;
    if (hipMemcpyAsync(host, b->states(), 8 * count, hipMemcpyDeviceToHost, b->stream) != hipSuccess ||
        hipStreamSynchronize(b->stream) != hipSuccess)
        return HOTRG_EHIP;
    return HOTRG_OK;
}

int itebd_work(itebd_batch* b, double* sweeps, double* rotations) {
    if (!b) return HOTRG_EINVAL;
    unsigned long long* host = new (std::nothrow) unsigned long long[2 * (size_t)b->batch];
    if (!host) return HOTRG_EINVAL;
    const bool ok = hipMemcpyAsync(host, b->ws + b->L.work, 16 * (size_t)b->batch, hipMemcpyDeviceToHost,
                                   b->stream) == hipSuccess &&
                    hipStreamSynchronize(b->stream) == hipSuccess;
    double sw = 0.0, rot = 0.0;
    for (int i = 0; ok && i < b->batch; ++i) {
        sw += (double)host[2 * i];
        rot += (double)host[2 * i + 1];
    }
    delete[] host;
    if (!ok) return HOTRG_EHIP;
    if (sweeps) *sweeps = sw;
    if (rotations) *rotations = rot;
    return HOTRG_OK;
}

int itebd_info(itebd_batch* b, long* updates, int* max_sweeps) {
    if (!b) return HOTRG_EINVAL;
    if (updates) *updates = b->updates;
    if (max_sweeps) {
        int* host = new (std::nothrow) int[b->batch];
        if (!host) return HOTRG_EINVAL;
        const bool ok = hipMemcpyAsync(host, b->ws + b->L.sweeps, 4 * (size_t)b->batch, hipMemcpyDeviceToHost,
                                       b->stream) == hipSuccess &&
                        hipStreamSynchronize(b->stream) == hipSuccess;
        int m = 0;
        for (int i = 0; ok && i < b->batch; ++i) m = std::max(m, host[i]);
        delete[] host;
        if (!ok) return HOTRG_EHIP;
        *max_sweeps = m;
    }
    return chain_status(b, nullptr);
}

int itebd_status(itebd_batch* b, int* status) {
    if (!b || !status) return HOTRG_EINVAL;
    const int rc = chain_status(b, status);
    return rc == HOTRG_EHIP ? rc : HOTRG_OK;
}

int itebd_set_max_sweeps(itebd_batch* b, int max_sweeps) {
    if (!b || max_sweeps < 1 || max_sweeps > ITEBD_MAX_SWEEPS) return HOTRG_EINVAL;
    b->max_sweeps = max_sweeps;
    return HOTRG_OK;
}

}  // extern "C"

// Synchronises, copies the per-chain status words (into per_chain when
// given) and maps them to one code: ENONFINITE if a chain stopped on a
// vanishing or non-finite norm, else EEIG if a decomposition reached the
// sweep limit, else OK.
static int chain_status(itebd_batch* b, int* per_chain) {
    int* host = new (std::nothrow) int[b->batch];
    if (!host) return HOTRG_EINVAL;
    const bool ok = hipMemcpyAsync(host, b->ws + b->L.status, 4 * (size_t)b->batch, hipMemcpyDeviceToHost,
                                   b->stream) == hipSuccess &&
                    hipStreamSynchronize(b->stream) == hipSuccess;
    int any = 0;
    for (int i = 0; ok && i < b->batch; ++i) {
        any |= host[i];
        if (per_chain) per_chain[i] = host[i];
    }
    delete[] host;
    if (!ok) return HOTRG_EHIP;
    if (any & ITEBD_CHAIN_NONFINITE) return HOTRG_ENONFINITE;
    if (any & ITEBD_CHAIN_SWEEP_CAP) return HOTRG_EEIG;
    return HOTRG_OK;
}

extern "C" {

void itebd_destroy(itebd_batch* b) {
    if (!b) return;
    (void)hipStreamSynchronize(b->stream);
    delete b;
}

}  // extern "C"
