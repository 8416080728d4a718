// iTEBD on the device: many independent infinite chains, one workgroup per
// chain, all FP64.  The SVD work matrices (W, V) live in LDS (75 KB, so two
// chains share a CU); B1 and B2 are staged into LDS from the chain's state
// row at the start of each update and written back at its end, and the
// evolved pair P goes to the chain's workspace slice (column-major, read
// row-parallel by the products W = P V and B1' = P V_kept, and small enough
// to stay in L2).  The C ABI is declared in include/itebd.h.
//
// One bond update (Sec. II.A, Eq. (1); the inverse-free form of the iTEBD
// update), n = 2 chi:
//   P[(a s),(t b)] = sum_c B1[s][a][c] B2[t][c][b]          (contraction)
//   P <- G P on the physical pair (s, t) of every (a, b)     (gate)
//   W = diag(lambda_2 (x) 1) P V0                             (V0: warm start or 1)
//   one-sided Jacobi on the columns of W, rotations also applied to V
//     -> W = X S, V = right singular vectors (unordered)
//   keep the chi largest; sign gauge on the kept columns of V
//   B2' = V_kept^T, B1' = P V_kept / |S_kept|, lambda_1' = S_kept / |S_kept|
//   exchange the sites' roles
// The Jacobi sweep visits all column pairs in n - 1 rounds of n/2 disjoint
// pairs (round-robin ordering, the systolic schedule of Sec. II.B used for
// one-sided rotations); sixteen lanes own a pair: they hold the pair's two
// columns of W and of V in registers (rows l, l + 16, ...), form the three
// dot products, reduce them over the sixteen lanes with DPP moves (every
// lane gets the same bits: each stage adds two equal partial sums in either
// order), and rotate their rows of W and V.  With 512 threads two waves share
// each SIMD, so one wave's dependent FP64 chain (square roots, division)
// overlaps the other's.  W and V are kept column-major with a column stride
// ld = 8 (mod 32) doubles: the four pairs of a wave (consecutive column
// indices) read 16 consecutive doubles each, starting 8 doubles apart in the
// 32 double-wide banks, which covers every bank exactly twice (the least a
// 64-lane 8-byte read can take).
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
// column stride of W and V: the smallest ld >= n with ld = 8 (mod 32)
__host__ __device__ constexpr int col_stride(int n) { return ((n + 23) / 32) * 32 + 8; }
constexpr int kMaxLd = col_stride(kMaxN);
static_assert(4 * kMaxChi * kMaxChi <= kMaxN * kMaxLd, "B1 and B2 are staged in the V buffer");
constexpr int kLanesPerPair = 16;
constexpr int kRowsPerLane = kMaxN / kLanesPerPair;
constexpr int kThreads = 256;                       // energy kernel
constexpr int kUpdThreads = kLanesPerPair * kMaxN / 2;   // update kernel: one lane group per pair
// row-parallel products (W = P V, B1' = P V_kept): kUpdThreads / n >= 8 groups
// of n lanes, each lane one row and at most this many columns
constexpr int kMaxColsPerLane = (kMaxN + 7) / 8;
static_assert(kUpdThreads / kMaxN >= 8, "row-parallel products assume at least 8 lane groups");
constexpr int kUpdatesPerLaunch = 32;
constexpr int kMaxSweeps = 40;
// rotate a pair while |w_p.w_q| > kTol |w_p| |w_q| (relative test)
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

// sum over an aligned row of sixteen lanes: partner lane ^1 (quad_perm
// [1,0,3,2]), ^2 (quad_perm [2,3,0,1]), the mirror lane 7 - l inside the
// half-row (the other quad), then the mirror lane 15 - l inside the row (the
// other half-row)
__device__ __forceinline__ double sum16(double v) {
    v += dpp_d<0xB1>(v);
    v += dpp_d<0x4E>(v);
    v += dpp_d<0x141>(v);
    v += dpp_d<0x140>(v);
    return v;
}

// four waves per SIMD (at most 128 VGPRs): with 75 KB of LDS two workgroups
// of eight waves then share a CU
__global__ __launch_bounds__(kUpdThreads) __attribute__((amdgpu_waves_per_eu(4)))
void itebd_update_kernel(double* __restrict__ states, double* __restrict__ vprev, double* __restrict__ pair,
                         int* __restrict__ sweeps_out, unsigned long long* __restrict__ work, int chi, Gate G,
                         long base, int nupd)
{
    // 75 KB in all, so two chains share a CU
    __shared__ double sW[kMaxN * kMaxLd];   // column-major, stride ld
    __shared__ double sV[kMaxN * kMaxLd];   // also stages B1 and B2 at the start of an update
    __shared__ double sl1[kMaxChi], sl2[kMaxChi];
    __shared__ double ssig[kMaxN], ssgn[kMaxChi];
    __shared__ int sord[kMaxChi];
    __shared__ int srot;
    __shared__ unsigned int srotc;   // rotations applied in this update
    __shared__ double snrm;

    const int tid = threadIdx.x;
    const int n = 2 * chi;
    const int ld = col_stride(n);
    const int nb = 2 * chi * chi;
    const long len = 2L * nb + 2 * chi;
    double* st = states + (long)blockIdx.x * len;        // B1 and B2 are rewritten every update
    double* vp = vprev + (long)blockIdx.x * 2 * n * n;
    double* gP = pair + (long)blockIdx.x * n * n;        // P, column-major: P[(a s),(t b)] at (t b) n + (a s)
    const int ng = kUpdThreads / n;                      // lane groups of the row-parallel products (>= 8)
    const int prow = tid % n, pgrp = tid / n;

    for (int i = tid; i < chi; i += kUpdThreads) {
        sl1[i] = st[2 * nb + i];
        sl2[i] = st[2 * nb + chi + i];
    }
    __syncthreads();

    int max_sweeps = 0;
    unsigned long long tot_sweeps = 0, tot_rot = 0;
    for (int u = 0; u < nupd; ++u) {
        if (tid == 0) srotc = 0;
        const long count = base + u;
        const int par = (int)(count & 1);
        const bool warm = count >= 2;

        // stage B1 and B2 in the V buffer
        double* sB1 = sV;
        double* sB2 = sV + nb;
        for (int i = tid; i < nb; i += kUpdThreads) {
            sB1[i] = st[i];
            sB2[i] = st[nb + i];
        }
        __syncthreads();
        // contraction P[(a s),(t b)] = sum_c B1[s][a][c] B2[t][c][b] and the gate on the
        // physical pair: one (a, b) per thread, its four (s, t)
        for (int idx = tid; idx < chi * chi; idx += kUpdThreads) {
            const int a = idx / chi, b = idx - (idx / chi) * chi;
            double v[4];
            for (int s = 0; s < 2; ++s)
                for (int t = 0; t < 2; ++t) {
                    const double* x = sB1 + (s * chi + a) * chi;
                    const double* y = sB2 + t * chi * chi + b;
                    double acc = 0.0;
                    for (int c = 0; c < chi; ++c) acc = fma(x[c], y[c * chi], acc);
                    v[2 * s + t] = acc;
                }
            for (int s = 0; s < 2; ++s)
                for (int t = 0; t < 2; ++t) {
                    const int o = 2 * s + t;
                    double acc = 0.0;
                    for (int i = 0; i < 4; ++i) acc = fma(G.g[4 * o + i], v[i], acc);
                    gP[(t * chi + b) * n + 2 * a + s] = acc;
                }
        }
        __syncthreads();   // P complete; the staged B1, B2 are no longer needed
        // starting right basis: the same bond's vectors of two updates ago, or 1
        // (stored column-major, n x n)
        double* vpar = vp + (long)par * n * n;
        for (int idx = tid; idx < n * n; idx += kUpdThreads) {
            const int j = idx / n, i = idx - (idx / n) * n;
            sV[j * ld + i] = warm ? vpar[idx] : (i == j ? 1.0 : 0.0);
        }
        __syncthreads();
        // W = diag(lambda_2 (x) 1) P V: thread (row r, group g) forms columns g, g + ng, ...
        if (pgrp < ng) {
            double acc[kMaxColsPerLane];
#pragma unroll
            for (int q = 0; q < kMaxColsPerLane; ++q) acc[q] = 0.0;
            if (warm) {
                for (int k = 0; k < n; ++k) {
                    const double pk = gP[k * n + prow];
#pragma unroll
                    for (int q = 0; q < kMaxColsPerLane; ++q) {
                        const int j = pgrp + q * ng;
                        if (j < n) acc[q] = fma(pk, sV[j * ld + k], acc[q]);
                    }
                }
            } else {
#pragma unroll
                for (int q = 0; q < kMaxColsPerLane; ++q) {
                    const int j = pgrp + q * ng;
                    if (j < n) acc[q] = gP[j * n + prow];
                }
            }
            const double lam = sl2[prow >> 1];
#pragma unroll
            for (int q = 0; q < kMaxColsPerLane; ++q) {
                const int j = pgrp + q * ng;
                if (j < n) sW[j * ld + prow] = lam * acc[q];
            }
        }
        __syncthreads();

        // one-sided Jacobi
        const int g = tid / kLanesPerPair, lane = tid % kLanesPerPair;
        const int npair = n >> 1;
        int sweeps = kMaxSweeps;
        for (int sw = 0; sw < kMaxSweeps; ++sw) {
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
                    double* Wp = sW + p * ld;
                    double* Wq = sW + q * ld;
                    double* Vp = sV + p * ld;
                    double* Vq = sV + q * ld;
                    // both columns of W and of V in registers: the V loads are in
                    // flight while the dot products and the rotation are formed
                    double wp[kRowsPerLane], wq[kRowsPerLane], vpr[kRowsPerLane], vqr[kRowsPerLane];
                    double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
                    for (int r = 0; r < kRowsPerLane; ++r) {
                        const int i = lane + kLanesPerPair * r;
                        wp[r] = i < n ? Wp[i] : 0.0;
                        wq[r] = i < n ? Wq[i] : 0.0;
                    }
#pragma unroll
                    for (int r = 0; r < kRowsPerLane; ++r) {
                        const int i = lane + kLanesPerPair * r;
                        vpr[r] = i < n ? Vp[i] : 0.0;
                        vqr[r] = i < n ? Vq[i] : 0.0;
                    }
#pragma unroll
                    for (int r = 0; r < kRowsPerLane; ++r) {
                        al = fma(wp[r], wp[r], al);
                        be = fma(wq[r], wq[r], be);
                        ga = fma(wp[r], wq[r], ga);
                    }
                    al = sum16(al);
                    be = sum16(be);
                    ga = sum16(ga);
                    // rotate while ga^2 > kTol^2 al be (the relative test, squared)
                    if (ga * ga > (kTol * kTol) * (al * be)) {
                        // the smaller root of t^2 + 2 zeta t - 1 = 0, zeta = (be - al) / (2 ga):
                        // t = sign(d) 2ga / (|d| + sqrt(d^2 + 4 ga^2)), d = be - al
                        const double d = be - al, g2 = 2.0 * ga;
                        const double t = (d >= 0.0 ? g2 : -g2) / (fabs(d) + sqrt(fma(d, d, g2 * g2)));
                        const double c = rsqrt(fma(t, t, 1.0)), s = c * t;
#pragma unroll
                        for (int r = 0; r < kRowsPerLane; ++r) {
                            const int i = lane + kLanesPerPair * r;
                            if (i < n) {
                                Wp[i] = c * wp[r] - s * wq[r];
                                Wq[i] = s * wp[r] + c * wq[r];
                                Vp[i] = c * vpr[r] - s * vqr[r];
                                Vq[i] = s * vpr[r] + c * vqr[r];
                            }
                        }
                        if (lane == 0) {
                            srot = 1;
                            atomicAdd(&srotc, 1u);
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
        max_sweeps = max(max_sweeps, sweeps);
        tot_sweeps += (unsigned long long)sweeps;
        tot_rot += (unsigned long long)srotc;   // read after the sweeps' barriers

        // singular values, the chi largest (ties: lower column first)
        for (int j = tid; j < n; j += kUpdThreads) {
            double acc = 0.0;
            for (int i = 0; i < n; ++i) acc = fma(sW[j * ld + i], sW[j * ld + i], acc);
            ssig[j] = sqrt(acc);
        }
        __syncthreads();
        for (int j = tid; j < n; j += kUpdThreads) {
            int rank = 0;
            for (int i = 0; i < n; ++i) rank += (ssig[i] > ssig[j]) || (ssig[i] == ssig[j] && i < j);
            if (rank < chi) sord[rank] = j;
        }
        __syncthreads();
        // sign gauge of the kept right vectors; norm of the kept values
        for (int c = tid; c < chi; c += kUpdThreads) {
            const int j = sord[c];
            double best = -1.0;
            int bi = 0;
            for (int i = 0; i < n; ++i) {
                const double a = fabs(sV[j * ld + i]);
                if (a > best) {
                    best = a;
                    bi = i;
                }
            }
            ssgn[c] = sV[j * ld + bi] < 0.0 ? -1.0 : 1.0;
        }
        if (tid == 0) {
            double acc = 0.0;
            for (int c = 0; c < chi; ++c) acc = fma(ssig[sord[c]], ssig[sord[c]], acc);
            snrm = sqrt(acc);
        }
        // the bond's right vectors for the next warm start
        for (int idx = tid; idx < n * n; idx += kUpdThreads) {
            const int j = idx / n, i = idx - (idx / n) * n;
            vpar[idx] = sV[j * ld + i];
        }
        __syncthreads();
        // new tensors, roles exchanged, into the state row:
        //   B1 <- B2' = V_kept^T, B2 <- B1' = P V_kept / nrm
        const double inv = 1.0 / snrm;
        for (int idx = tid; idx < nb; idx += kUpdThreads) {
            const int t = idx / (chi * chi), rem = idx - t * chi * chi;
            const int c = rem / chi, b = rem - (rem / chi) * chi;
            st[idx] = ssgn[c] * sV[sord[c] * ld + t * chi + b];
        }
        if (pgrp < ng) {   // row (a s) = prow, kept columns c = g, g + ng, ...
            double acc[kMaxColsPerLane];
#pragma unroll
            for (int q = 0; q < kMaxColsPerLane; ++q) acc[q] = 0.0;
            for (int k = 0; k < n; ++k) {
                const double pk = gP[k * n + prow];
#pragma unroll
                for (int q = 0; q < kMaxColsPerLane; ++q) {
                    const int c = pgrp + q * ng;
                    if (c < chi) acc[q] = fma(pk, sV[sord[c] * ld + k], acc[q]);
                }
            }
            const int a = prow >> 1, sp = prow & 1;
#pragma unroll
            for (int q = 0; q < kMaxColsPerLane; ++q) {
                const int c = pgrp + q * ng;
                if (c < chi) st[nb + (sp * chi + a) * chi + c] = ssgn[c] * inv * acc[q];
            }
        }
        for (int c = tid; c < chi; c += kUpdThreads) {
            const double old = sl2[c];
            sl2[c] = ssig[sord[c]] * inv;
            sl1[c] = old;
        }
        __syncthreads();
    }

    for (int i = tid; i < chi; i += kUpdThreads) {
        st[2 * nb + i] = sl1[i];
        st[2 * nb + chi + i] = sl2[i];
    }
    if (tid == 0) {
        sweeps_out[blockIdx.x] = max_sweeps;
        work[2 * blockIdx.x] += tot_sweeps;
        work[2 * blockIdx.x + 1] += tot_rot;
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
    size_t states, vprev, pair, sweeps, work, energies, total;
};

Layout plan(int batch, int chi) {
    const size_t len = 4 * (size_t)chi * chi + 2 * (size_t)chi;
    const size_t n = 2 * (size_t)chi;
    Layout L;
    size_t o = 0;
    L.states = o;
    o = round_up(o + 8 * len * batch, 256);
    L.vprev = o;
    o = round_up(o + 8 * 2 * n * n * batch, 256);
    L.pair = o;
    o = round_up(o + 8 * n * n * batch, 256);
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

struct itebd_batch {
    int batch = 0, chi = 0;
    double h[16];
    hipStream_t stream = nullptr;
    char* ws = nullptr;
    Layout L;
    long updates = 0;
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
    double* vprev = reinterpret_cast<double*>(b->ws + b->L.vprev);
    double* pair = reinterpret_cast<double*>(b->ws + b->L.pair);
    int* sweeps = reinterpret_cast<int*>(b->ws + b->L.sweeps);
    unsigned long long* work = reinterpret_cast<unsigned long long*>(b->ws + b->L.work);
    for (int done = 0; done < nupdates;) {
        const int k = std::min(kUpdatesPerLaunch, nupdates - done);
        hipLaunchKernelGGL(itebd_update_kernel, dim3((unsigned)b->batch), dim3(kUpdThreads), 0, b->stream, b->states(),
                           vprev, pair, sweeps, work, b->chi, G, b->updates, k);
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
    return HOTRG_OK;
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
    return HOTRG_OK;
}

void itebd_destroy(itebd_batch* b) {
    if (!b) return;
    (void)hipStreamSynchronize(b->stream);
    delete b;
}

}  // extern "C"
