// Host engine of the HOTRG library: parameter checking, workspace carving,
// the per-step launch schedule on the caller's stream, the FP64 eigensolve,
// and the C ABI declared in include/hotrg.h.
//
// One step on T[l,r,d,u] with dims [Dx,Dx,Dy,Dy], D' = min(D, Dx^2)
// (Sec. II.A: merge two tensors along one direction, truncate the fused bond
// by the decomposition the higher-order SVD reduces to):
//   P1 = T as [(l,u),(r,d)]           (re-layout, D^4)
//   P2 = T as [(l,d),(r,u)]           (re-layout, D^4)
//   Ah[a1,b1,k,k'] = P1 P1^T          (half environment of the bottom copy)
//   Bh[a2,b2,k,k'] = P2 P2^T          (half environment of the top copy)
//   E[(a1a2),(b1b2)] = Ah Bh^T        (= M M^T, M never formed), symmetrised
//   E u_j = lambda_j u_j (FP64, eig.hip) -> U = leading D' eigenvectors, sign-fixed
//   P3 = T as [(d,r,u), l]; X[l,d,r1,a2,k] = Ux P3^T            (K = Dx)
//   P4 = T as [(u,r), (l,d)]; Y[l,d,u,r1,r2] = X P4^T            (K = Dx Dy, the D^7 term)
//   T'[d,u,l,r] = Y Ut^T  (written already x<->y exchanged)      (K = Dx^2)
//   c_n = max|T'|, T' /= c_n, ln Z accumulator += ln(c_n) / 2^n
// Two-sided truncation (HOTRG's choice between the two fused legs) also
// builds the right environment from P1, P2 of the mirrored tensor, solves it
// and keeps the isometry with the smaller discarded weight, on the device.
// Impurity tensors I (observables) follow T with the same isometry:
//   X_I = U P3(I)^T;  Y_I = [X_I | X] [P4(T) | P4(I)]^T  (one product, K = 2 Dx Dy)
//   I' = Y_I Ut^T / (2 c_n)
// X, X_I and P4(T), P4(I) are column blocks of two wide operand buffers, so
// each Y_I is a single launch over the doubled K.
// All products are the one index-mapped MFMA kernel (gemm.hip).
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "../../include/hotrg.h"
#include "common.h"

using namespace hotrg;

namespace {

constexpr int kMaxQ = 16;
constexpr int kEventsPerStep = 11;

struct StepDims {
    int dx, dy, dp;
};

std::vector<StepDims> trajectory(int dx, int dy, int dmax, int nsteps) {
    std::vector<StepDims> t;
    t.reserve(nsteps);
    for (int i = 0; i < nsteps; ++i) {
        const int dp = std::min<long>(dmax, (long)dx * dx);
        t.push_back({dx, dy, dp});
        const int nx = dy;
        dy = dp;
        dx = nx;
    }
    return t;
}

// Storage of contraction operands: FP64, FP32, or the BF16 planes of the
// split modes (written once by each producer, read by the split products).
Fmt fmt_of(int prec) {
    switch (prec) {
        case HOTRG_FP32: return Fmt::F32;
        case HOTRG_BF16X3: return Fmt::BF16x2;
        case HOTRG_BF16X6: return Fmt::BF16x3;
        case HOTRG_FP16X3: return Fmt::BF16x3;   // all but the full-size Y operands
        default: return Fmt::F64;
    }
}

int products_of(int prec) {
    return prec == HOTRG_BF16X3 ? 3 : (prec == HOTRG_BF16X6 || prec == HOTRG_FP16X3 ? 6 : 1);
}

// HOTRG_FP16X3: scales of the FP16 planes of Y's operands.  max|T| = 1 after
// every normalisation (T0 is divided by c_0), and the columns of U are
// orthonormal, so |X| <= sqrt(Dx) <= sqrt(HOTRG_MAX_DIM) < 10: the scaled
// values stay below 2^14 * 1 and 2^11 * 10, under FP16's largest finite
// number (65504), while everything above 2^-25 of the largest value keeps
// normal (11-bit) FP16 terms.
constexpr float kF16ScaleT = 16384.f;   // 2^14
constexpr float kF16ScaleX = 2048.f;    // 2^11

// HOTRG_FP16X3, environment products: P1 and P2 (re-layouts of T, |.| <= 1)
// are planes of 2^14 x T as for Y; a half environment sums Dx Dy products of
// two such entries, so |Ah|, |Bh| <= Dx Dy, and they are stored as planes of
// s_H x value with s_H the largest power of two for which s_H Dx Dy <= 2^15
// (under 65504 after rounding); E's product undoes s_H^2.
double f16_half_scale(long k) {
    double sc = 1.0;
    while (sc * 2.0 * (double)k <= 32768.0) sc *= 2.0;
    while (sc * (double)k > 32768.0) sc *= 0.5;
    return sc;
}

size_t round_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// bytes of a buffer of `count` elements in format f (planes 64-element aligned)
size_t buf_bytes(Fmt f, size_t count) {
    return (size_t)fmt_planes(f) * round_up(std::max<size_t>(count, 1), 64) * fmt_plane_elem_bytes(f);
}

int popcount2(int m) { return (m & 1) + ((m >> 1) & 1); }

// Y is kept in FP32 in the split modes: T' splits it into planes as it loads
// its tiles, so Y is written and read at 4 bytes an element instead of 6
// (BF16x3 planes), with the same planes reaching the products.
Fmt y_fmt(Fmt f) { return f == Fmt::BF16x2 || f == Fmt::BF16x3 ? Fmt::F32 : f; }

struct Layout {
    size_t nT = 0, nP = 0, nAB = 0, nE = 0, nU = 0, nX = 0, nEig = 0;
    int nimp = 0;   // impurity tensors carried (one per observable slot set)
    size_t oState, oT, oPa, oPb, oAh, oBh, oE, oEigV0, oEigV1, oEigW, oEigPart, oEigG, oEigS, oEigTheta, oEigL,
        oEigD, oEigCtl, oUt, oUx, oX, oY, total;
    size_t oI[2] = {0, 0};                                   // impurity tensors (FP64)
    size_t oER = 0, oEigVR0 = 0, oEigVR1 = 0, oUtR = 0, oUxR = 0;  // two-sided
};

constexpr double kEigTol = 1e-12;
constexpr int kEigMaxIt = 30;
// An eigensolve that stops unconverged with a residual above this (relative
// to the largest eigenvalue) has not found the dominant subspace and latches
// HOTRG_EEIG.  Slow convergence is not failure: where the spectrum is flat
// at the cut (the Heisenberg chain at beta ~ 800 discards 87-95% of the
// weight per step) solves reach the pass cap with residuals up to 5.5e-3
// and still give f within 1e-5 of the exact diagonalisation.
constexpr double kEigFailTol = 5e-2;

int step_cap(const hotrg_params* p) { return p->max_steps > 0 ? p->max_steps : HOTRG_MAX_STEPS; }

bool valid_params(const hotrg_params* p) {
    if (!p) return false;
    if (p->max_steps < 0 || p->max_steps > HOTRG_MAX_STEPS) return false;
    if (p->two_sided != 0 && p->two_sided != 1) return false;
    if (p->observables & ~(HOTRG_OBS_MAGNETIZATION | HOTRG_OBS_BOND_ENERGY)) return false;
    if (!isfinite(p->field)) return false;
    if (p->dmax < 1 || p->dmax > HOTRG_MAX_DIM) return false;
    if (p->precision < HOTRG_FP64 || p->precision > HOTRG_FP16X3) return false;
    if (p->precision == HOTRG_FP16X3 && p->observables) return false;
    if (p->model == HOTRG_ISING) {
        if (p->q != 2) return false;
    } else if (p->model == HOTRG_POTTS) {
        if (p->q < 2 || p->q > kMaxQ) return false;
    } else if (p->model == HOTRG_QCHAIN) {
        if (!p->bond_h || !(p->tau > 0.0) || !isfinite(p->tau)) return false;
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 4; ++j)
                if (!isfinite(p->bond_h[4 * i + j]) || p->bond_h[4 * i + j] != p->bond_h[4 * j + i]) return false;
        if (p->field != 0.0 || p->observables) return false;
        return true;
    } else if (p->model == HOTRG_CUSTOM) {
        if (!p->custom_tensor) return false;
        if (p->custom_dx < 1 || p->custom_dx > HOTRG_MAX_DIM) return false;
        if (p->custom_dy < 1 || p->custom_dy > HOTRG_MAX_DIM) return false;
        if (p->field != 0.0) return false;
        for (int j = 0; j < 2; ++j)
            if ((p->observables >> j & 1) && !p->custom_impurity[j]) return false;
        return true;
    } else {
        return false;
    }
    if (!(p->temperature > 0.0) || !isfinite(p->temperature)) return false;
    if (!(p->coupling > 0.0) || !isfinite(p->coupling)) return false;
    return true;
}

void initial_dims(const hotrg_params* p, int* dx, int* dy);

// Every step whose environment is too large to diagonalise densely needs a
// Ritz block wider than the kept count.
bool eig_feasible(const hotrg_params* p);

void initial_dims(const hotrg_params* p, int* dx, int* dy) {
    if (p->model == HOTRG_QCHAIN) {
        *dx = *dy = 4;   // split bond of the gate, two spins of a block
    } else if (p->model == HOTRG_CUSTOM) {
        *dx = p->custom_dx;
        *dy = p->custom_dy;
    } else {
        *dx = *dy = p->q;
    }
}

bool eig_feasible(const hotrg_params* p) {
    int dx, dy;
    initial_dims(p, &dx, &dy);
    for (const StepDims& s : trajectory(dx, dy, p->dmax, step_cap(p))) {
        const int n = s.dx * s.dx;
        if (n > kEigPMax && eig_block(n, s.dp) <= s.dp) return false;
    }
    return true;
}

Layout plan(const hotrg_params* p) {
    Layout L;
    int dx, dy;
    initial_dims(p, &dx, &dy);
    L.nT = (size_t)dx * dx * dy * dy;
    for (const StepDims& s : trajectory(dx, dy, p->dmax, step_cap(p))) {
        const size_t x = s.dx, y = s.dy, dp = s.dp;
        L.nT = std::max(L.nT, std::max(x * x * y * y, y * y * dp * dp));
        L.nP = std::max(L.nP, x * x * y * y);
        L.nAB = std::max(L.nAB, x * x * y * y);
        L.nE = std::max(L.nE, x * x * x * x);
        if (x * x > (size_t)kEigPMax) L.nEig = std::max(L.nEig, x * x);
        L.nU = std::max(L.nU, dp * x * x);
        L.nX = std::max(L.nX, dp * x * x * y * y);
    }
    const Fmt f = fmt_of(p->precision);
    L.nimp = popcount2(p->observables);
    const size_t wide = 1 + (size_t)L.nimp;   // column blocks of the X and P4 operands
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = round_up(o + bytes, 256);
        return at;
    };
    L.oState = take(sizeof(DevState));
    L.oT = take(buf_bytes(Fmt::F64, L.nT));
    for (int j = 0; j < L.nimp; ++j) L.oI[j] = take(buf_bytes(Fmt::F64, L.nT));
    L.oPa = take(buf_bytes(f, L.nP));
    L.oPb = take(buf_bytes(f, L.nP * wide));
    L.oAh = take(buf_bytes(f, L.nAB));
    L.oBh = take(buf_bytes(f, L.nAB));
    L.oE = take(buf_bytes(Fmt::F64, L.nE));
    const size_t pb = (size_t)kEigPMax;
    L.oEigV0 = take(8 * L.nEig * pb);
    L.oEigV1 = take(8 * L.nEig * pb);
    L.oEigW = take(8 * L.nEig * pb);
    L.oEigPart = take(8 * ((L.nEig + 31) / 32) * (pb * pb + pb));
    L.oEigG = take(8 * (pb * pb + pb));
    L.oEigS = take(8 * pb * pb);
    L.oEigTheta = take(8 * pb);
    L.oEigL = take(8 * pb * pb);
    L.oEigD = take(8 * pb);
    L.oEigCtl = take(sizeof(EigCtl));
    L.oUt = take(buf_bytes(f, L.nU));
    L.oUx = take(buf_bytes(f, L.nU));
    if (p->two_sided) {
        L.oER = take(buf_bytes(Fmt::F64, L.nE));
        L.oEigVR0 = take(8 * L.nEig * pb);
        L.oEigVR1 = take(8 * L.nEig * pb);
        L.oUtR = take(buf_bytes(f, L.nU));
        L.oUxR = take(buf_bytes(f, L.nU));
    }
    L.oX = take(buf_bytes(f, L.nX * wide));
    L.oY = take(buf_bytes(y_fmt(f), L.nX));
    L.total = o;
    return L;
}

Buf make_buf(char* base, size_t off, Fmt f, size_t count) {
    return Buf{base + off, f, round_up(std::max<size_t>(count, 1), 64)};
}

// T0[x,x',y,y'] = sum_s g(s) Q[s,x]Q[s,x']Q[s,y]Q[s,y'], Q = W^(1/2), g(s) =
// exp(beta h f(s)) the field's site factor (f = sigma for Ising with s = 0
// the +1 state, f = delta(s, 0) for Potts).  W = a I + b 1 1^T for both
// models (Ising: a = 2 sinh(beta J), b = exp(-beta J); Potts:
// a = exp(beta J) - 1, b = 1), so Q = sqrt(a) I + c 1 1^T with
// c = (sqrt(a + q b) - sqrt(a)) / q, and Q^-1 = (I - c / (sqrt(a) + q c) 1 1^T) / sqrt(a).
// Impurity tensors of the observables:
//   slot 0 (order parameter m(s) = sigma, or (q delta(s,0) - 1)/(q - 1)):
//     S = sum_s m(s) g(s) Q[s,.]^4, one copy giving Z <m>;
//   slot 1 (bond energy e(s,s') = -J sigma sigma', or -J delta(s,s')): T0
//     with its d leg contracted with G = Q^-1 (e o W) Q^-1, so the y bond
//     below the site carries e(s,s') W(s,s'); one copy gives Z <e_b>.
struct ModelTensors {
    std::vector<double> T, I[2];
};

ModelTensors model_tensors(const hotrg_params* p) {
    const int q = p->q;
    const double beta = 1.0 / p->temperature;
    const double bj = p->coupling * beta;
    const bool ising = p->model == HOTRG_ISING;
    double a, b;
    if (ising) {
        a = 2.0 * sinh(bj);
        b = exp(-bj);
    } else {
        a = expm1(bj);
        b = 1.0;
    }
    const double sa = sqrt(a);
    const double off = (sqrt(a + q * b) - sa) / q;
    std::vector<double> Q((size_t)q * q), Qi((size_t)q * q), We((size_t)q * q);
    const double ioff = -off / (sa * (sa + q * off));
    for (int i = 0; i < q; ++i)
        for (int j = 0; j < q; ++j) {
            Q[(size_t)i * q + j] = off + (i == j ? sa : 0.0);
            Qi[(size_t)i * q + j] = ioff + (i == j ? 1.0 / sa : 0.0);
            const double w = (i == j ? a : 0.0) + b;
            const double e = ising ? -p->coupling * (i == j ? 1.0 : -1.0) : (i == j ? -p->coupling : 0.0);
            We[(size_t)i * q + j] = e * w;
        }
    std::vector<double> g(q), m(q);
    for (int k = 0; k < q; ++k) {
        const double fs = ising ? (k == 0 ? 1.0 : -1.0) : (k == 0 ? 1.0 : 0.0);
        g[k] = exp(beta * p->field * fs);
        m[k] = ising ? (k == 0 ? 1.0 : -1.0) : (k == 0 ? 1.0 : -1.0 / (q - 1.0));
    }
    auto site = [&](const std::vector<double>& wts) {
        std::vector<double> T((size_t)q * q * q * q, 0.0);
        for (int x = 0; x < q; ++x)
            for (int xp = 0; xp < q; ++xp)
                for (int y = 0; y < q; ++y)
                    for (int yp = 0; yp < q; ++yp) {
                        double s = 0.0;
                        for (int k = 0; k < q; ++k)
                            s += wts[k] * Q[(size_t)k * q + x] * Q[(size_t)k * q + xp] * Q[(size_t)k * q + y] *
                                 Q[(size_t)k * q + yp];
                        T[(((size_t)x * q + xp) * q + y) * q + yp] = s;
                    }
        return T;
    };
    ModelTensors mt;
    mt.T = site(g);
    if (p->observables & HOTRG_OBS_MAGNETIZATION) {
        std::vector<double> mg(q);
        for (int k = 0; k < q; ++k) mg[k] = m[k] * g[k];
        mt.I[0] = site(mg);
    }
    if (p->observables & HOTRG_OBS_BOND_ENERGY) {
        // G = Qi We Qi
        std::vector<double> t((size_t)q * q, 0.0), G((size_t)q * q, 0.0);
        for (int i = 0; i < q; ++i)
            for (int j = 0; j < q; ++j)
                for (int k = 0; k < q; ++k) t[(size_t)i * q + j] += Qi[(size_t)i * q + k] * We[(size_t)k * q + j];
        for (int i = 0; i < q; ++i)
            for (int j = 0; j < q; ++j)
                for (int k = 0; k < q; ++k) G[(size_t)i * q + j] += t[(size_t)i * q + k] * Qi[(size_t)k * q + j];
        std::vector<double> TG((size_t)q * q * q * q, 0.0);
        for (int x = 0; x < q; ++x)
            for (int xp = 0; xp < q; ++xp)
                for (int y = 0; y < q; ++y)
                    for (int yp = 0; yp < q; ++yp) {
                        double s = 0.0;
                        for (int k = 0; k < q; ++k)
                            s += G[(size_t)y * q + k] * mt.T[(((size_t)x * q + xp) * q + k) * q + yp];
                        TG[(((size_t)x * q + xp) * q + y) * q + yp] = s;
                    }
        mt.I[1] = TG;
    }
    return mt;
}

// Eigendecomposition a = Q diag(w) Q^T of a real symmetric 4 x 4 matrix by
// cyclic Jacobi rotations (host, FP64).
void sym_eig4(const double* a, double* w, double* Q) {
    double A[16];
    memcpy(A, a, sizeof A);
    for (int i = 0; i < 16; ++i) Q[i] = (i % 5 == 0) ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 60; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int p = 0; p < 4; ++p)
            for (int q = 0; q < 4; ++q) {
                tot += A[4 * p + q] * A[4 * p + q];
                if (p != q) off += A[4 * p + q] * A[4 * p + q];
            }
        if (off <= 1e-32 * tot || off < 1e-300) break;
        for (int p = 0; p < 4; ++p)
            for (int q = p + 1; q < 4; ++q) {
                const double apq = A[4 * p + q];
                if (apq == 0.0) continue;
                const double z = (A[4 * q + q] - A[4 * p + p]) / (2.0 * apq);
                const double t = (z >= 0.0 ? 1.0 : -1.0) / (fabs(z) + sqrt(1.0 + z * z));
                const double c = 1.0 / sqrt(1.0 + t * t), sn = c * t;
                for (int k = 0; k < 4; ++k) {
                    const double akp = A[4 * k + p], akq = A[4 * k + q];
                    A[4 * k + p] = c * akp - sn * akq;
                    A[4 * k + q] = sn * akp + c * akq;
                }
                for (int k = 0; k < 4; ++k) {
                    const double apk = A[4 * p + k], aqk = A[4 * q + k];
                    A[4 * p + k] = c * apk - sn * aqk;
                    A[4 * q + k] = sn * apk + c * aqk;
                }
                for (int k = 0; k < 4; ++k) {
                    const double qkp = Q[4 * k + p], qkq = Q[4 * k + q];
                    Q[4 * k + p] = c * qkp - sn * qkq;
                    Q[4 * k + q] = sn * qkp + c * qkq;
                }
            }
    }
    for (int i = 0; i < 4; ++i) w[i] = A[4 * i + i];
}

// Block tensor of a spin-1/2 chain (one tensor = two sites x one Trotter
// step of U = G_odd G_even, G = exp(-tau h)):
//   G[(s1' s2'),(s1 s2)] = sum_k A_k[s1', s1] B_k[s2', s2] from the SVD of the
//   rearranged R[(s1' s1), (s2' s2)] (through the eigenvectors of R^T R);
//   T[l, r, (s0 s1), (s0' s1')] = sum_{x,y} B_l[s0', x] A_r[s1', y] G[(x y), (s0 s1)]
// x = the split bonds (space), y = the block's spins below/above (time).
std::vector<double> qchain_tensor(const double* h, double tau) {
    double w[4], Q[16], G[16];
    sym_eig4(h, w, Q);
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            double acc = 0.0;
            for (int k = 0; k < 4; ++k) acc += Q[4 * i + k] * exp(-tau * w[k]) * Q[4 * j + k];
            G[4 * i + j] = acc;
        }
    double R[16], RtR[16], sv[4], V[16];
    for (int a = 0; a < 2; ++a)          // s1'
        for (int b = 0; b < 2; ++b)      // s2'
            for (int c = 0; c < 2; ++c)  // s1
                for (int d = 0; d < 2; ++d) R[4 * (2 * a + c) + (2 * b + d)] = G[4 * (2 * a + b) + (2 * c + d)];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            double acc = 0.0;
            for (int k = 0; k < 4; ++k) acc += R[4 * k + i] * R[4 * k + j];
            RtR[4 * i + j] = acc;
        }
    sym_eig4(RtR, sv, V);
    double A[4][4], B[4][4];   // A[k][(s1' s1)], B[k][(s2' s2)]
    for (int k = 0; k < 4; ++k) {
        const double sig = sqrt(fmax(sv[k], 0.0));
        const double rs = sqrt(sig);
        for (int i = 0; i < 4; ++i) {
            B[k][i] = rs * V[4 * i + k];
            double u = 0.0;
            for (int j = 0; j < 4; ++j) u += R[4 * i + j] * V[4 * j + k];
            A[k][i] = sig > 1e-300 ? u / rs : 0.0;
        }
    }
    std::vector<double> T(256, 0.0);
    for (int l = 0; l < 4; ++l)
        for (int r = 0; r < 4; ++r)
            for (int s0 = 0; s0 < 2; ++s0)
                for (int s1 = 0; s1 < 2; ++s1)
                    for (int p0 = 0; p0 < 2; ++p0)
                        for (int p1 = 0; p1 < 2; ++p1) {
                            double acc = 0.0;
                            for (int x = 0; x < 2; ++x)
                                for (int y = 0; y < 2; ++y)
                                    acc += B[l][2 * p0 + x] * A[r][2 * p1 + y] * G[4 * (2 * x + y) + (2 * s0 + s1)];
                            T[((l * 4 + r) * 4 + (2 * s0 + s1)) * 4 + (2 * p0 + p1)] = acc;
                        }
    return T;
}

}  // namespace

struct hotrg_solve {
    hotrg_params p;
    hipStream_t stream = nullptr;
    char* ws = nullptr;
    size_t ws_bytes = 0;
    Layout L;
    Fmt fmt = Fmt::F64;
    int products = 1;
    int dx = 0, dy = 0, steps = 0;
    int host_status = HOTRG_OK;
    int warm_n[2] = {0, 0};   // (n, p) of the Ritz block kept per step parity
    int warm_p[2] = {0, 0};
    int warm_nr[2] = {0, 0};  // the same for the right environment (two-sided)
    int warm_pr[2] = {0, 0};
    int imp_slot[2] = {0, 0}; // observable slot of each carried impurity tensor
    int last_n = 0, last_dp = 0;    // fused-leg size and kept count of the last step
    int eig_maxit = kEigMaxIt;      // subspace passes per eigensolve
    double eig_fail = kEigFailTol;  // residual above which an unconverged solve fails
    // host-polled stepping: the stop state of the eigensolve in flight is
    // written to pinned host memory after each group of passes, so the host
    // enqueues only the passes a solve needs
    EigMail* mail = nullptr;        // pinned, fine-grained (hipHostMalloc)
    int mail_seq = 0;               // seq of the last write enqueued
    bool pend = false;              // a begun step waits for its eigensolve
    bool pend_exchange = true;
    int pend_next = 0;              // next subspace pass to enqueue
    int pend_par = 0;
    int pend_side = 0;              // two-sided: 0 left eigensolve in flight, 1 right
    bool pend_warm_r = false;       // warm start of the right eigensolve
    int hist[2] = {0, 0};           // passes the last polled eigensolve of each parity used
    // steps driven by the library's progress thread (hotrg_coarse_grain_async);
    // while async_active is set only that thread touches the handle
    std::atomic<int> async_active{0};
    int async_left = 0;
    bool async_exchange = true;
    int async_extra = 0;
    bool timing = false;
    int timed_from = 0;  // first step recorded with events
    std::vector<hipEvent_t> ev;
    std::vector<StepDims> timed_dims;  // input dims of each recorded step

    DevState* state() const { return reinterpret_cast<DevState*>(ws + L.oState); }
    EigWork eig() const {
        EigWork w;
        w.V[0] = reinterpret_cast<double*>(ws + L.oEigV0);
        w.V[1] = reinterpret_cast<double*>(ws + L.oEigV1);
        w.W = reinterpret_cast<double*>(ws + L.oEigW);
        w.part = reinterpret_cast<double*>(ws + L.oEigPart);
        w.G = reinterpret_cast<double*>(ws + L.oEigG);
        w.S = reinterpret_cast<double*>(ws + L.oEigS);
        w.theta = reinterpret_cast<double*>(ws + L.oEigTheta);
        w.L = reinterpret_cast<double*>(ws + L.oEigL);
        w.dsc = reinterpret_cast<double*>(ws + L.oEigD);
        w.ctl = reinterpret_cast<EigCtl*>(ws + L.oEigCtl);
        return w;
    }
    EigWork eig_right() const {
        EigWork w = eig();
        w.V[0] = reinterpret_cast<double*>(ws + L.oEigVR0);
        w.V[1] = reinterpret_cast<double*>(ws + L.oEigVR1);
        return w;
    }
    double* T() const { return reinterpret_cast<double*>(ws + L.oT); }
    double* I(int j) const { return reinterpret_cast<double*>(ws + L.oI[j]); }
};

#define HIP_TRY(s, x)                                  \
    do {                                               \
        if ((x) != hipSuccess) {                       \
            if ((s)) (s)->host_status = HOTRG_EHIP;    \
            return HOTRG_EHIP;                         \
        }                                              \
    } while (0)

namespace {

int read_state(hotrg_solve* s, DevState* out) {
    HIP_TRY(s, hipMemcpyAsync(out, s->state(), sizeof(DevState), hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(s, hipStreamSynchronize(s->stream));
    return HOTRG_OK;
}

void record(hotrg_solve* s, int step_index, int slot) {
    if (!s->timing) return;
    const int i = step_index - s->timed_from;
    if (i < 0 || (size_t)((i + 1) * kEventsPerStep) > s->ev.size()) return;
    (void)hipEventRecord(s->ev[(size_t)i * kEventsPerStep + slot], s->stream);
}

int gemm(hotrg_solve* s, const Buf& A, long lda, const Buf& B, long ldb, const Buf& C, int M, int N, int K,
         const OutMap& mp, GemmRole role = GemmRole::Generic, double alpha = 1.0) {
    HIP_TRY(s, launch_gemm_nt(A, lda, B, ldb, C, M, N, K, alpha, mp, s->products, role, s->stream));
    return HOTRG_OK;
}

// Column block `blk` (of width w columns) of a wide operand buffer: panel
// layout of row length ld, or row-major with row stride ld.
Buf column_block(const Buf& B, int blk, long w, long ld, bool panel) {
    Buf o = B;
    const size_t el = fmt_plane_elem_bytes(B.fmt);
    const long off = panel ? (long)blk * (w / 16) * 512 : (long)blk * w;
    o.ptr = static_cast<char*>(B.ptr) + (size_t)off * el;
    o.panel_k = panel ? ld : 0;
    return o;
}

// Whether a step from dims (Dx, Dy) fits the workspace carved for the handle.
bool step_fits(const Layout& L, int Dx, int Dy, int Dp) {
    const size_t x = Dx, y = Dy, dp = Dp;
    if (std::max(x * x * y * y, y * y * dp * dp) > L.nT || dp * dp * y * y > L.nT) return false;
    if (x * x * y * y > L.nP || x * x * y * y > L.nAB || x * x * x * x > L.nE) return false;
    if (dp * x * x > L.nU || dp * x * x * y * y > L.nX) return false;
    const int n = Dx * Dx;
    if (n > kEigPMax && ((size_t)n > L.nEig || eig_block(n, Dp) <= Dp)) return false;
    return true;
}

// Which parts of a step enqueue_step enqueues: the environment(s), a range
// of the eigensolve, and the products with the normalisation and the step
// bookkeeping.  The default is the whole step.
struct StepPart {
    bool env = true;
    bool left = true, right = true;   // launch the range of the left / right eigensolve
    EigRange eig;                     // of the left one
    EigRange eigR;                    // of the right one (two-sided handles)
    bool rest = true;
};

int enqueue_step(hotrg_solve* s, bool exchange = true, const StepPart& part = StepPart()) {
    const int n = s->steps + 1;       // 1-based step number
    const int Dx = s->dx, Dy = s->dy;
    const int Dp = (int)std::min<long>(s->p.dmax, (long)Dx * Dx);
    const int nE = Dx * Dx;
    if (!step_fits(s->L, Dx, Dy, Dp)) return HOTRG_ENOMEM;
    const Fmt f = s->fmt;
    const Layout& L = s->L;
    const int nimp = L.nimp;
    const bool two = s->p.two_sided != 0;
    char* w = s->ws;
    const Buf Pa = make_buf(w, L.oPa, f, L.nP), Pb = make_buf(w, L.oPb, f, L.nP * (1 + nimp));
    const Buf Ah = make_buf(w, L.oAh, f, L.nAB), Bh = make_buf(w, L.oBh, f, L.nAB);
    const Buf Ut = make_buf(w, L.oUt, f, L.nU), Ux = make_buf(w, L.oUx, f, L.nU);
    const Buf X = make_buf(w, L.oX, f, L.nX * (1 + nimp)), Y = make_buf(w, L.oY, y_fmt(f), L.nX);
    double* E = reinterpret_cast<double*>(w + L.oE);
    const Buf Ebuf{E, Fmt::F64, 0};
    const Buf Tbuf{s->T(), Fmt::F64, 0};
    const int dims[4] = {Dx, Dx, Dy, Dy};
    const int step_index = s->steps;
    int rc;
    if (part.env && s->timing && step_index >= s->timed_from) s->timed_dims.push_back({Dx, Dy, Dp});

    // -- half environments and E
    // With the split formats and whole 32-row panels, the half-environment
    // operands P1, P2 [(a,k) x (r,d)] and the half environments themselves,
    // as E's operands [(a,b) x (k,k')], are stored in the 32 x 16 panel
    // layout (as X and T are for Y), so the three products load contiguous
    // KiBs.
    const bool split = f == Fmt::BF16x2 || f == Fmt::BF16x3;
    const long mxy = (long)Dx * Dy, mxx = (long)Dx * Dx, myy = (long)Dy * Dy;
    const bool panel_env = split && mxy % 32 == 0 && mxy > 64 && mxx % 32 == 0 && mxx > 64 && myy % 16 == 0;
    // HOTRG_FP16X3: with the panel layout the three products take two scaled
    // FP16 planes per operand (three split products instead of six), views of
    // the same buffers
    const bool f16env = s->p.precision == HOTRG_FP16X3 && panel_env && nimp == 0;
    const double sH = f16env ? f16_half_scale(mxy) : 1.0;
    Buf P1b = f16env ? make_buf(w, L.oPa, Fmt::F16x2, L.nP) : Pa;
    Buf P2b = f16env ? make_buf(w, L.oPb, Fmt::F16x2, L.nP) : Pb;
    Buf Aho = f16env ? make_buf(w, L.oAh, Fmt::F16x2, L.nAB) : Ah;
    Buf Bho = f16env ? make_buf(w, L.oBh, Fmt::F16x2, L.nAB) : Bh;
    if (f16env) {
        P1b.scale = P2b.scale = kF16ScaleT;
        Aho.scale = Bho.scale = (float)sH;
    }
    Buf Ahb = Aho, Bhb = Bho;
    if (panel_env) {
        P1b.panel_k = P2b.panel_k = mxy;
        Ahb.panel_k = Bhb.panel_k = myy;
    }
    const int m = Dx * Dy;
    // rows (a, k), columns (b, k') -> [a,b,k,k'], i.e. row a Dx + b and
    // column k Dy + k' of E's [Dx^2 x Dy^2] operand
    const OutMap half = panel_env ? OutMap{Dy, Dx, 0, Dy, 1, 0, 0, Dy, 0, 1, myy}
                                  : OutMap{Dy, (long)Dx * Dy * Dy, Dy, Dy, (long)Dy * Dy, 1};
    const OutMap env{Dx, (long)Dx * Dx * Dx, Dx, Dx, (long)Dx * Dx, 1};  // -> E[(a1a2),(b1b2)]
    // The left environment takes P1 = T as [(l,u),(r,d)], P2 = T as
    // [(l,d),(r,u)]; the right one the same re-layouts of the mirrored
    // tensor T[r,l,d,u]: [(r,u),(l,d)] and [(r,d),(l,u)].
    auto environment = [&](const int* p1, const int* p2, double* Eout) -> int {
        int r;
        HIP_TRY(s, launch_permute4(s->T(), dims, p1, P1b, s->stream));
        HIP_TRY(s, launch_permute4(s->T(), dims, p2, P2b, s->stream));
        if (Eout == E) record(s, step_index, 1);
        const double a_half = f16env ? sH / ((double)kF16ScaleT * (double)kF16ScaleT) : 1.0;
        if ((r = gemm(s, P1b, m, P1b, m, Aho, m, m, m, half, GemmRole::Generic, a_half))) return r;
        if ((r = gemm(s, P2b, m, P2b, m, Bho, m, m, m, half, GemmRole::Generic, a_half))) return r;
        const Buf Eo{Eout, Fmt::F64, 0};
        if ((r = gemm(s, Ahb, (long)Dy * Dy, Bhb, (long)Dy * Dy, Eo, nE, nE, Dy * Dy, env, GemmRole::Generic,
                      f16env ? 1.0 / (sH * sH) : 1.0)))
            return r;
        HIP_TRY(s, launch_symmetrize(Eout, nE, s->stream));
        return HOTRG_OK;
    };
    double* ER = two ? reinterpret_cast<double*>(w + L.oER) : nullptr;
    if (part.env) {
        record(s, step_index, 0);
        {
            const int p1[4] = {0, 3, 1, 2}, p2[4] = {0, 2, 1, 3};
            if ((rc = environment(p1, p2, E))) return rc;
        }
        if (two) {
            const int p1[4] = {1, 3, 0, 2}, p2[4] = {1, 2, 0, 3};
            if ((rc = environment(p1, p2, ER))) return rc;
        }
        record(s, step_index, 2);
    }
    // -- FP64 eigensolve(s) and isometry
    {
        // Ritz block kept per fused axis: with the exchange the axes alternate,
        // so the last block of this axis is the step two earlier; without it
        // every step fuses the same legs and the previous step's block is used
        const int par = exchange ? (step_index & 1) : 0;
        const int pblk = nE > kEigPMax ? eig_block(nE, Dp) : nE;
        const unsigned long long seed = 0x5EEDull + 7919ull * (unsigned long long)n;
        const bool warm = nE > kEigPMax && s->warm_n[par] == nE && s->warm_p[par] == pblk;
        if (part.left)
            HIP_TRY(s, launch_eig_topk(E, nE, Dp, Dx, s->eig(), par, warm, seed, s->eig_maxit, kEigTol,
                                       s->eig_fail, Ut, Ux, s->state(), n, s->stream, 0, part.eig));
        if (two) {
            // the right eigensolve follows the left one on the same control
            // block; in the host-polled form it starts in a later part, with
            // the warm-start choice taken when the left one started
            const Buf UtR = make_buf(w, L.oUtR, f, L.nU), UxR = make_buf(w, L.oUxR, f, L.nU);
            const bool warm_r = part.left && part.eig.start
                                    ? nE > kEigPMax && s->warm_nr[par] == nE && s->warm_pr[par] == pblk
                                    : s->pend_warm_r;
            if (part.right)
                HIP_TRY(s, launch_eig_topk(ER, nE, Dp, Dx, s->eig_right(), par, warm_r, seed, s->eig_maxit,
                                           kEigTol, s->eig_fail, UtR, UxR, s->state(), n, s->stream, 1,
                                           part.eigR));
            if (part.rest)
                HIP_TRY(s, launch_choose_side(s->state(), n, Ut.ptr, Ux.ptr, UtR.ptr, UxR.ptr,
                                              buf_bytes(f, L.nU), s->stream));
            if (part.left && part.eig.start) s->pend_warm_r = warm_r;
        }
        if (nE > kEigPMax && part.left && part.eig.start) {
            s->warm_n[par] = s->warm_nr[par] = nE;
            s->warm_p[par] = s->warm_pr[par] = pblk;
        }
    }
    if (!part.rest) return HOTRG_OK;
    record(s, step_index, 3);
    // The Y product's operands, X [(l,d,r1) x (a2,k)] and P4 [(u,r) x (l,d)],
    // both with rows of Kp = Dx Dy elements, are written in the 32 x 16 panel
    // layout when the split formats are used and the shapes allow it (Kp a
    // multiple of 32, more than 64 columns of Y), so that every tile load of
    // the D^7 product is one contiguous KiB.  With impurity tensors both are
    // column blocks of wider buffers (row length Kx):
    //   X buffer:  [X_0 | X | X_1]        P4 buffer: [P4(I_1) | P4(T) | P4(I_0)]
    // (one impurity: [X_0 | X] and [P4(T) | P4(I_0)]), so that
    //   Y_0 = [X_0 | X] [P4(T) | P4(I_0)]^T and Y_1 = [X | X_1] [P4(I_1) | P4(T)]^T
    // are single products over K = 2 Kp.
    const long Kp = (long)Dx * Dy;
    const long Kx = Kp * (1 + nimp);
    const bool panel = split && Kp % 32 == 0 && Kp > 64;
    // HOTRG_FP16X3: Y's operands X and P4 as scaled FP16 planes when Y runs
    // on the full-size tiles (views of the same buffers: 4 bytes an element
    // instead of 6); the early, smaller steps keep the BF16 planes
    const long ym_rows = (long)Dp * Dy * Dx;
    const bool f16y = s->p.precision == HOTRG_FP16X3 && panel && nimp == 0 && ym_rows % 32 == 0 &&
                      ((ym_rows + 255) / 256) * ((Kp + 255) / 256) >= 512;
    const Buf Xy = f16y ? make_buf(w, L.oX, Fmt::F16x2, L.nX * (1 + nimp)) : X;
    Buf Py = f16y ? make_buf(w, L.oPb, Fmt::F16x2, L.nP * (1 + nimp)) : Pb;
    if (f16y) Py.scale = kF16ScaleT;
    const int xblk_T = nimp >= 1 ? 1 : 0;                 // X's block
    const int bblk_T = nimp == 2 ? 1 : 0;                 // P4(T)'s block
    auto xblk_imp = [&](int j) { return j == 0 ? 0 : 2; };
    auto bblk_imp = [&](int j) { return nimp == 2 ? (j == 0 ? 2 : 0) : 1; };
    // rows (l, a2), columns (d r1, k): offset l Dy Dx Kx + a2 Dy + (d r1) Kx + k,
    // i.e. row l Dy Dx + (d r1) and column a2 Dy + k of the [Dp Dy Dx x Kp] block
    // With Dy and Dx Dy multiples of 16, a tile takes 16 (d r1) x 16 k
    // columns, so its rows of X are whole runs of 16 panel rows.
    OutMap xm = panel ? OutMap{Dx, (long)Dy * Dx, 0, Dy, 1, 0, 0, Dy, 0, 1, Kx}
                      : OutMap{Dx, (long)Dy * Dx * Kx, Dy, Dy, Kx, 1};
    if (panel && Dy % 16 == 0 && Kp % 16 == 0) xm.ngroup = Dy;
    auto x_product = [&](const double* src, int blk) -> int {
        const int p3[4] = {2, 1, 3, 0};  // P3[d,r,u,l]
        HIP_TRY(s, launch_permute4(src, dims, p3, Pa, s->stream));
        if (src == s->T()) record(s, step_index, 4);
        Buf Xo = Xy;
        Xo.ptr = column_block(Xy, blk, Kp, Kx, panel).ptr;
        return gemm(s, Ux, Dx, Pa, Dx, Xo, Dp * Dx, Dy * Dx * Dy, Dx, xm, GemmRole::X, f16y ? kF16ScaleX : 1.0);
    };
    auto p4_into = [&](const double* src, int blk) -> int {
        const int p4[4] = {3, 1, 0, 2};  // P4[u,r,l,d]
        Buf Po = column_block(Py, blk, Kp, Kx, panel);
        if (nimp) {
            Po.cols = Kp;
            Po.ld = Kx;
        }
        HIP_TRY(s, launch_permute4(src, dims, p4, Po, s->stream));
        return HOTRG_OK;
    };
    const OutMap ym{Dx, (long)Dy * Dx * Dx, Dx, Dx, (long)Dx * Dx, 1};   // -> Y[l,d,u,r1,r2]
    // -> next T[d,u,l,r] (x <-> y exchanged), or T[l,r,d,u] kept
    const OutMap tm = exchange ? OutMap{(long)Dy * Dy, Dp, (long)Dp * Dp, Dp, 0, 1}
                               : OutMap{(long)Dy * Dy, (long)Dp * Dy * Dy, 1, Dp, 0, (long)Dy * Dy};
    // -- X = U . T  -> X[l,d,r1,a2,k]
    if ((rc = x_product(s->T(), xblk_T))) return rc;
    record(s, step_index, 5);
    // -- Y = X . T  -> Y[l,d,u,r1,r2]
    if ((rc = p4_into(s->T(), bblk_T))) return rc;
    record(s, step_index, 6);
    if ((rc = gemm(s, column_block(Xy, xblk_T, Kp, Kx, panel), Kx, column_block(Py, bblk_T, Kp, Kx, panel), Kx, Y,
                   Dp * Dy * Dx, Dy * Dx, (int)Kp, ym, GemmRole::Y,
                   f16y ? 1.0 / ((double)kF16ScaleX * (double)kF16ScaleT) : 1.0)))
        return rc;
    record(s, step_index, 7);
    // -- T' = Y . U  -> next T[d,u,l,r] (x <-> y exchanged), FP64
    if ((rc = gemm(s, Y, (long)Dx * Dx, Ut, (long)Dx * Dx, Tbuf, Dp * Dy * Dy, Dp, Dx * Dx, tm, GemmRole::TP)))
        return rc;
    record(s, step_index, 8);
    const size_t nnext = (size_t)Dy * Dy * Dp * Dp;
    HIP_TRY(s, launch_normalize(s->T(), nnext, s->state(), n, s->stream));
    record(s, step_index, 9);
    // -- impurity tensors: I' = U^T (I (x) T + T (x) I) U / (2 c_n)
    if (nimp) {
        for (int j = 0; j < nimp; ++j) {
            if ((rc = x_product(s->I(j), xblk_imp(j)))) return rc;
            if ((rc = p4_into(s->I(j), bblk_imp(j)))) return rc;
        }
        for (int j = 0; j < nimp; ++j) {
            const int ax = j == 0 ? 0 : 1;                       // [X_0 | X] or [X | X_1]
            const int bx = j == 0 ? bblk_T : 0;                  // [P4(T) | P4(I_0)] or [P4(I_1) | P4(T)]
            if ((rc = gemm(s, column_block(X, ax, Kp, Kx, panel), Kx, column_block(Pb, bx, Kp, Kx, panel), Kx, Y,
                           Dp * Dy * Dx, Dy * Dx, (int)(2 * Kp), ym, GemmRole::Y)))
                return rc;
            const Buf Io{s->I(j), Fmt::F64, 0};
            if ((rc = gemm(s, Y, (long)Dx * Dx, Ut, (long)Dx * Dx, Io, Dp * Dy * Dy, Dp, Dx * Dx, tm, GemmRole::TP)))
                return rc;
            HIP_TRY(s, launch_scale_by_norm(s->I(j), nnext, s->state(), 0.5, s->stream));
        }
    }
    record(s, step_index, 10);
    s->last_n = nE;
    s->last_dp = Dp;
    if (exchange) {
        s->dx = Dy;
        s->dy = Dp;
    } else {
        s->dx = Dp;
    }
    s->steps = n;
    return HOTRG_OK;
}

// Host-polled stepping: the first group of subspace passes is as many as the
// handle's last eigensolve of the same parity needed (kPollFirst before any
// is known); later groups are kPollChunk passes.  Groups end on a pass with
// a convergence check (every EIG_RR_EVERY = 2 passes).
constexpr int kPollFirst = 8;
constexpr int kPollChunk = 4;

int mail_copy(hotrg_solve* s) {
    s->mail_seq += 1;
    HIP_TRY(s, launch_eig_mail(s->eig().ctl, s->mail, s->mail_seq, s->stream));
    return HOTRG_OK;
}

// Builds T0 (and the impurity tensors) for p on the host, normalises them by
// c_0 = max|T0|, uploads them and a fresh device state (ln Z accumulator =
// ln c_0), and resets the step count.
int upload_initial(hotrg_solve* s, const hotrg_params* p) {
    initial_dims(p, &s->dx, &s->dy);
    s->steps = 0;
    s->pend = false;
    s->hist[0] = s->hist[1] = 0;
    s->timed_from = 0;
    s->timed_dims.clear();
    for (int i = 0; i < 2; ++i) s->warm_n[i] = s->warm_p[i] = s->warm_nr[i] = s->warm_pr[i] = 0;
    const size_t count = (size_t)s->dx * s->dx * s->dy * s->dy;
    ModelTensors mt;
    if (p->model == HOTRG_QCHAIN) {
        mt.T = qchain_tensor(p->bond_h, p->tau);
    } else if (p->model == HOTRG_CUSTOM) {
        mt.T.assign(p->custom_tensor, p->custom_tensor + count);
        for (int j = 0; j < 2; ++j)
            if (p->observables >> j & 1) mt.I[j].assign(p->custom_impurity[j], p->custom_impurity[j] + count);
    } else {
        mt = model_tensors(p);
    }
    double c0 = 0.0;
    for (double v : mt.T) c0 = std::max(c0, fabs(v));
    if (!(c0 > 0.0) || !isfinite(c0)) return HOTRG_ENONFINITE;
    for (double& v : mt.T) v /= c0;
    int j = 0;
    for (int slot = 0; slot < 2; ++slot) {
        if (!(p->observables >> slot & 1)) continue;
        for (double& v : mt.I[slot]) {
            v /= c0;
            if (!isfinite(v)) return HOTRG_ENONFINITE;
        }
        s->imp_slot[j++] = slot;
    }
    std::vector<char> hs(sizeof(DevState), 0);
    DevState* h = reinterpret_cast<DevState*>(hs.data());
    h->lnz_acc = log(c0);
    h->c[0] = c0;
    h->c_cur = c0;
    if (hipMemcpyAsync(s->state(), h, sizeof(DevState), hipMemcpyHostToDevice, s->stream) != hipSuccess ||
        hipMemcpyAsync(s->T(), mt.T.data(), count * sizeof(double), hipMemcpyHostToDevice, s->stream) != hipSuccess)
        return HOTRG_EHIP;
    for (int i = 0; i < j; ++i)
        if (hipMemcpyAsync(s->I(i), mt.I[s->imp_slot[i]].data(), count * sizeof(double), hipMemcpyHostToDevice,
                           s->stream) != hipSuccess)
            return HOTRG_EHIP;
    if (hipStreamSynchronize(s->stream) != hipSuccess) return HOTRG_EHIP;
    return HOTRG_OK;
}

int begin_step(hotrg_solve* s, int exchange, int extra, int* pending) {
    if (pending) *pending = 0;
    if (!s || (exchange != 0 && exchange != 1) || extra < 0 || s->pend) return HOTRG_EINVAL;
    if (s->host_status) return HOTRG_ESTATE;
    if (s->steps + 1 > step_cap(&s->p)) return HOTRG_EINVAL;
    // steps whose environment is diagonalised densely are enqueued whole
    if (s->dx * s->dx <= kEigPMax) return enqueue_step(s, exchange != 0);
    if (!s->mail) {
        void* h = nullptr;
        if (hipHostMalloc(&h, sizeof(EigMail), hipHostMallocCoherent) != hipSuccess) return HOTRG_EHIP;
        s->mail = static_cast<EigMail*>(h);
        memset(s->mail, 0, sizeof(EigMail));
        s->mail_seq = 0;
    }
    const int par = exchange ? (s->steps & 1) : 0;
    int first = (s->hist[par] > 0 ? s->hist[par] : kPollFirst) + std::min(extra, HOTRG_EIG_MAX_PASSES);
    first = std::min((first + 1) / 2 * 2, s->eig_maxit);
    StepPart part;
    part.right = false;            // a two-sided step starts with the left eigensolve
    part.eig.last = first;
    part.eig.end = false;
    part.rest = false;
    int rc = enqueue_step(s, exchange != 0, part);
    if (rc) return rc;
    if ((rc = mail_copy(s))) return rc;
    s->pend = true;
    s->pend_exchange = exchange != 0;
    s->pend_next = first;
    s->pend_par = par;
    s->pend_side = 0;
    if (pending) *pending = 1;
    return HOTRG_OK;
}

int poll_step(hotrg_solve* s, int* state) {
    if (!s || !state) return HOTRG_EINVAL;
    *state = HOTRG_POLL_IDLE;
    if (!s->pend) return HOTRG_OK;
    if (s->host_status) return HOTRG_ESTATE;
    const unsigned long long word = __atomic_load_n(&s->mail->word, __ATOMIC_ACQUIRE);
    if ((int)(word >> 32) != s->mail_seq) {
        *state = HOTRG_POLL_RUNNING;
        return HOTRG_OK;
    }
    struct {
        int done, iters;
    } c{(int)(word & 1u), (int)((word >> 1) & 0x7fffffffu)};
    // the eigensolve in flight: the left one, or the right one of a
    // two-sided step once the left one has ended
    const bool on_right = s->pend_side == 1;
    StepPart part;
    part.env = false;
    part.left = !on_right;
    part.right = on_right;
    EigRange& cur = on_right ? part.eigR : part.eig;
    cur.start = false;
    cur.first = s->pend_next;
    int rc;
    if (c.done || s->pend_next >= s->eig_maxit) {
        // converged, stagnated or at the pass cap: the end of this
        // eigensolve, then the right one's start or the rest of the step
        cur.last = s->pend_next;
        s->hist[s->pend_par] = c.iters > 0 ? c.iters : s->pend_next;
        if (s->p.two_sided && !on_right) {
            const int first = std::min((s->hist[s->pend_par] + 1) / 2 * 2, s->eig_maxit);
            part.right = true;
            part.eigR.last = first;
            part.eigR.end = false;
            part.rest = false;
            if ((rc = enqueue_step(s, s->pend_exchange, part))) return rc;
            if ((rc = mail_copy(s))) return rc;
            s->pend_side = 1;
            s->pend_next = first;
            *state = HOTRG_POLL_PASSES;
            return HOTRG_OK;
        }
        s->pend = false;
        if ((rc = enqueue_step(s, s->pend_exchange, part))) return rc;
        *state = HOTRG_POLL_STEPPED;
        return HOTRG_OK;
    }
    cur.last = std::min(s->pend_next + kPollChunk, s->eig_maxit);
    cur.end = false;
    part.rest = false;
    if ((rc = enqueue_step(s, s->pend_exchange, part))) return rc;
    if ((rc = mail_copy(s))) return rc;
    s->pend_next = cur.last;
    *state = HOTRG_POLL_PASSES;
    return HOTRG_OK;
}

// ---------------------------------------------------------------- progress thread
//
// Host-polled steps without a host scheduling loop: the library's own thread
// keeps every handle given to hotrg_coarse_grain_async moving, enqueueing its
// next group of passes or the rest of its step as soon as the stop state of
// its eigensolve arrives (a read of host memory), and beginning its next
// step right after.  It spins (yielding) while any handle is in flight and
// sleeps on a condition variable otherwise.  The thread and its registry
// live until the process ends.

// One round for one handle; true when it has nothing left to enqueue.
bool advance_async(hotrg_solve* s, bool* progress) {
    if (s->host_status) return true;
    if (s->pend) {
        int st = HOTRG_POLL_IDLE;
        const int rc = poll_step(s, &st);
        if (rc) {
            if (!s->host_status) s->host_status = rc;
            return true;
        }
        if (st == HOTRG_POLL_RUNNING) return false;
        *progress = true;
        if (st == HOTRG_POLL_PASSES) return false;
    }
    while (s->async_left > 0) {
        int pending = 0;
        s->async_left -= 1;
        const int rc = begin_step(s, s->async_exchange ? 1 : 0, s->async_extra, &pending);
        *progress = true;
        if (rc) {
            if (!s->host_status) s->host_status = rc;
            s->async_left = 0;
            return true;
        }
        if (pending) return false;
    }
    return true;
}

class Engine {
public:
    static Engine& get() {
        static Engine* e = new Engine();   // never destroyed: its thread may outlive static destructors
        return *e;
    }
    // Throws if the thread cannot be started or the registry cannot grow;
    // the handle is then not registered.
    void add(hotrg_solve* s) {
        std::lock_guard<std::mutex> lock(mu_);
        if (!started_) {
            std::thread(&Engine::run, this).detach();
            started_ = true;
        }
        incoming_.push_back(s);
        has_incoming_.store(true, std::memory_order_release);
        cv_.notify_one();
    }

private:
    void run() {
        std::vector<hotrg_solve*> mine;
        for (;;) {
            if (mine.empty() || has_incoming_.load(std::memory_order_acquire)) {
                std::unique_lock<std::mutex> lock(mu_);
                if (mine.empty()) cv_.wait(lock, [&] { return !incoming_.empty(); });
                mine.insert(mine.end(), incoming_.begin(), incoming_.end());
                incoming_.clear();
                has_incoming_.store(false, std::memory_order_release);
            }
            bool progress = false;
            for (size_t i = 0; i < mine.size();) {
                hotrg_solve* s = mine[i];
                bool finished;
                try {
                    finished = advance_async(s, &progress);
                } catch (...) {   // host allocation failure: the handle fails, the thread goes on
                    if (!s->host_status) s->host_status = HOTRG_EHIP;
                    finished = true;
                }
                if (finished) {
                    mine[i] = mine.back();
                    mine.pop_back();
                    s->async_active.store(0, std::memory_order_release);
                } else {
                    ++i;
                }
            }
            if (!progress) std::this_thread::yield();
        }
    }
    std::mutex mu_;
    std::condition_variable cv_;
    std::vector<hotrg_solve*> incoming_;
    std::atomic<bool> has_incoming_{false};
    bool started_ = false;
};

// Every entry point that takes a handle first waits until the progress
// thread has released it (all of its asynchronous steps enqueued).
void quiesce(hotrg_solve* s) {
    while (s->async_active.load(std::memory_order_acquire)) std::this_thread::yield();
}

int latched(const DevState& d) { return d.status; }

}  // namespace

namespace hotrg {

// Format of the stand-alone product's converted operands.
Fmt gemm_operand_fmt(int precision) { return precision == HOTRG_FP16X3 ? Fmt::F16x2 : fmt_of(precision); }

size_t gemm_scratch_bytes(int precision, int M, int N, int K) {
    if (M < 0 || N < 0 || K < 0) return 0;
    if (precision == HOTRG_FP64) return 0;
    const Fmt f = gemm_operand_fmt(precision);
    return round_up(buf_bytes(f, (size_t)M * K), 256) + buf_bytes(f, (size_t)N * K);
}

int gemm_nt_with_scratch(int precision, int role, int panel, int M, int N, int K, const double* A, long lda,
                         const double* B, long ldb, double* C, double alpha, long sm, long rs_hi, long rs_lo, long sn,
                         long cs_hi, long cs_lo, void* scratch, size_t scratch_bytes, void* stream) {
    if (M < 0 || N < 0 || K < 0 || sm < 1 || sn < 1 || !C) return HOTRG_EINVAL;
    if (precision < HOTRG_FP64 || precision > HOTRG_FP16X3) return HOTRG_EINVAL;
    if (role < HOTRG_ROLE_GENERIC || role > HOTRG_ROLE_TP || (panel != 0 && panel != 1)) return HOTRG_EINVAL;
    if (K > 0 && (!A || !B || lda < K || ldb < K)) return HOTRG_EINVAL;
    const bool split = precision == HOTRG_BF16X3 || precision == HOTRG_BF16X6 || precision == HOTRG_FP16X3;
    if (panel && (!split || M % 32 || N % 32 || K % 16 || K == 0)) return HOTRG_EINVAL;
    if (gemm_scratch_bytes(precision, M, N, K) > scratch_bytes) return HOTRG_ENOMEM;
    const GemmRole gr = static_cast<GemmRole>(role);
    hipStream_t st = static_cast<hipStream_t>(stream);
    const OutMap mp{sm, rs_hi, rs_lo, sn, cs_hi, cs_lo};
    const Buf Cb{C, Fmt::F64, 0};
    if (precision == HOTRG_FP64) {
        const Buf Ab{const_cast<double*>(A), Fmt::F64, 0}, Bb{const_cast<double*>(B), Fmt::F64, 0};
        return launch_gemm_nt(Ab, lda, Bb, ldb, Cb, M, N, K, alpha, mp, 1, gr, st) == hipSuccess ? HOTRG_OK
                                                                                              : HOTRG_EHIP;
    }
    if (!scratch || ((uintptr_t)scratch & 255u)) return HOTRG_EINVAL;
    const Fmt f = gemm_operand_fmt(precision);
    char* base = static_cast<char*>(scratch);
    Buf Ab = make_buf(base, 0, f, (size_t)M * K);
    Buf Bb = make_buf(base, round_up(buf_bytes(f, (size_t)M * K), 256), f, (size_t)N * K);
    if (panel) {
        Ab.panel_k = K;
        Bb.panel_k = K;
    }
    double a_eff = alpha;
    if (f == Fmt::F16x2) {   // both operands as 2^11 x value, undone on the output
        Ab.scale = Bb.scale = kF16ScaleX;
        a_eff = alpha / ((double)kF16ScaleX * (double)kF16ScaleX);
    }
    if (launch_convert2d(A, lda, M, K, Ab, st) != hipSuccess) return HOTRG_EHIP;
    if (launch_convert2d(B, ldb, N, K, Bb, st) != hipSuccess) return HOTRG_EHIP;
    return launch_gemm_nt(Ab, K, Bb, K, Cb, M, N, K, a_eff, mp, products_of(precision), gr, st) == hipSuccess
               ? HOTRG_OK
               : HOTRG_EHIP;
}

}  // namespace hotrg

extern "C" {

size_t hotrg_workspace_bytes(const hotrg_params* p) {
    if (!valid_params(p) || !eig_feasible(p)) return 0;
    return plan(p).total;
}

int hotrg_init_tensor(const hotrg_params* p, void* workspace, size_t ws_bytes, void* stream, hotrg_solve** out) {
    if (!out) return HOTRG_EINVAL;
    *out = nullptr;
    if (!valid_params(p) || !eig_feasible(p) || !workspace || ((uintptr_t)workspace & 255u)) return HOTRG_EINVAL;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return HOTRG_ENODEV;
    const Layout L = plan(p);
    if (ws_bytes < L.total) return HOTRG_ENOMEM;

    hotrg_solve* s = new (std::nothrow) hotrg_solve();
    if (!s) return HOTRG_EINVAL;
    s->p = *p;
    s->p.custom_tensor = nullptr;
    s->p.custom_impurity[0] = s->p.custom_impurity[1] = nullptr;
    s->p.bond_h = nullptr;
    s->stream = static_cast<hipStream_t>(stream);
    s->ws = static_cast<char*>(workspace);
    s->ws_bytes = ws_bytes;
    s->L = L;
    s->fmt = fmt_of(p->precision);
    s->products = products_of(p->precision);
    initial_dims(p, &s->dx, &s->dy);

    int rc = upload_initial(s, p);
    if (rc) {
        delete s;
        return rc;
    }

    *out = s;
    return HOTRG_OK;
}

int hotrg_reset(hotrg_solve* s, const hotrg_params* p) {
    if (s) quiesce(s);
    if (!s || !valid_params(p) || !eig_feasible(p)) return HOTRG_EINVAL;
    if (hipStreamSynchronize(s->stream) != hipSuccess) return HOTRG_EHIP;
    const Layout L = plan(p);
    if (L.total > s->ws_bytes) return HOTRG_ENOMEM;
    s->L = L;
    s->p = *p;
    s->p.custom_tensor = nullptr;
    s->p.custom_impurity[0] = s->p.custom_impurity[1] = nullptr;
    s->p.bond_h = nullptr;
    s->fmt = fmt_of(p->precision);
    s->products = products_of(p->precision);
    s->host_status = HOTRG_OK;
    s->eig_maxit = kEigMaxIt;
    s->eig_fail = kEigFailTol;
    return upload_initial(s, p);
}

int hotrg_coarse_grain(hotrg_solve* s, int nsteps) {
    if (s) quiesce(s);
    if (!s || nsteps < 0 || s->pend) return HOTRG_EINVAL;
    if (s->host_status) return HOTRG_ESTATE;
    if (s->steps + nsteps > step_cap(&s->p)) return HOTRG_EINVAL;
    for (int i = 0; i < nsteps; ++i) {
        const int rc = enqueue_step(s);
        if (rc) return rc;
    }
    return HOTRG_OK;
}

int hotrg_coarse_grain_axis(hotrg_solve* s, int nsteps, int exchange) {
    if (s) quiesce(s);
    if (!s || nsteps < 0 || (exchange != 0 && exchange != 1) || s->pend) return HOTRG_EINVAL;
    if (s->host_status) return HOTRG_ESTATE;
    if (s->steps + nsteps > step_cap(&s->p)) return HOTRG_EINVAL;
    for (int i = 0; i < nsteps; ++i) {
        const int rc = enqueue_step(s, exchange != 0);
        if (rc) return rc;
    }
    return HOTRG_OK;
}

int hotrg_log_z_chain(hotrg_solve* s, double* lnz_per_tensor) {
    if (s) quiesce(s);
    if (!s || !lnz_per_tensor) return HOTRG_EINVAL;
    if (s->host_status) return s->host_status;
    if (s->dx > 96) return HOTRG_EINVAL;
    HIP_TRY(s, launch_chain_lnz(s->T(), s->dx, s->dy, 64, s->state(), s->stream));
    DevState d;
    int rc = read_state(s, &d);
    if (rc) return rc;
    if (latched(d)) return latched(d);
    if (!d.chain_ok) return HOTRG_ENONFINITE;
    *lnz_per_tensor = d.lnz_acc + d.chain_lnz * ldexp(1.0, -s->steps);
    return HOTRG_OK;
}

int hotrg_coarse_grain_batch(hotrg_solve* const* solves, int count, int nsteps) {
    if (count < 0 || nsteps < 0 || (count > 0 && !solves)) return HOTRG_EINVAL;
    // validate the whole group before enqueueing anything; a handle listed
    // k times needs room for k * nsteps more steps
    for (int i = 0; i < count; ++i) {
        hotrg_solve* s = solves[i];
        if (s) quiesce(s);
        if (!s || s->pend) return HOTRG_EINVAL;
        int times = 0;
        for (int j = 0; j < count; ++j) times += solves[j] == s;
        if (s->steps + (long)times * nsteps > step_cap(&s->p)) return HOTRG_EINVAL;
    }
    for (int i = 0; i < count; ++i)
        if (solves[i]->host_status) return HOTRG_ESTATE;
    for (int n = 0; n < nsteps; ++n)
        for (int i = 0; i < count; ++i) {
            const int rc = enqueue_step(solves[i]);
            if (rc) return rc;
        }
    return HOTRG_OK;
}

int hotrg_step_begin(hotrg_solve* s, int exchange, int extra, int* pending) {
    if (pending) *pending = 0;
    if (!s) return HOTRG_EINVAL;
    quiesce(s);
    return begin_step(s, exchange, extra, pending);
}

int hotrg_step_poll(hotrg_solve* s, int* state) {
    if (state) *state = HOTRG_POLL_IDLE;
    if (!s || !state) return HOTRG_EINVAL;
    quiesce(s);
    return poll_step(s, state);
}

int hotrg_coarse_grain_async(hotrg_solve* s, int nsteps, int exchange, int extra) {
    if (!s || nsteps < 0 || (exchange != 0 && exchange != 1) || extra < 0) return HOTRG_EINVAL;
    quiesce(s);
    if (s->pend) return HOTRG_EINVAL;
    if (s->host_status) return HOTRG_ESTATE;
    if (s->steps + nsteps > step_cap(&s->p)) return HOTRG_EINVAL;
    if (nsteps == 0) return HOTRG_OK;
    s->async_left = nsteps;
    s->async_exchange = exchange != 0;
    s->async_extra = extra;
    s->async_active.store(1, std::memory_order_release);
    try {
        Engine::get().add(s);   // may start the thread: no exception leaves this ABI
    } catch (...) {
        s->async_left = 0;
        s->async_active.store(0, std::memory_order_release);
        return HOTRG_EHIP;
    }
    return HOTRG_OK;
}

int hotrg_async_busy(hotrg_solve* s, int* busy) {
    if (busy) *busy = 0;
    if (!s || !busy) return HOTRG_EINVAL;
    *busy = s->async_active.load(std::memory_order_acquire);
    return HOTRG_OK;
}

int hotrg_log_z(hotrg_solve* s, double* lnz_per_site, int* log2_sites) {
    if (s) quiesce(s);
    if (!s || !lnz_per_site) return HOTRG_EINVAL;
    if (s->host_status) return s->host_status;
    HIP_TRY(s, launch_trace(s->T(), s->dx, s->dy, s->state(), s->stream));
    DevState d;
    int rc = read_state(s, &d);
    if (rc) return rc;
    if (latched(d)) return latched(d);
    if (!(d.trace > 0.0) || !isfinite(d.trace)) return HOTRG_ENONFINITE;
    *lnz_per_site = d.lnz_acc + log(d.trace) * ldexp(1.0, -s->steps);
    if (log2_sites) *log2_sites = s->steps;
    return HOTRG_OK;
}

int hotrg_step_info(hotrg_solve* s, int n, double* c_n, double* trunc_err, double* cut_gap) {
    if (s) quiesce(s);
    if (!s || n < 0 || n > s->steps) return HOTRG_EINVAL;
    if (s->host_status) return s->host_status;
    DevState d;
    int rc = read_state(s, &d);
    if (rc) return rc;
    if (latched(d)) return latched(d);
    if (c_n) *c_n = d.c[n];
    if (trunc_err) *trunc_err = n ? d.trunc_err[n] : 0.0;
    if (cut_gap) *cut_gap = n ? d.cut_gap[n] : 0.0;
    return HOTRG_OK;
}

int hotrg_eig_info(hotrg_solve* s, int n, int* iterations, int* sweeps, double* residual, int* stop) {
    if (s) quiesce(s);
    if (!s || n < 1 || n > s->steps) return HOTRG_EINVAL;
    if (s->host_status) return s->host_status;
    DevState d;
    int rc = read_state(s, &d);
    if (rc) return rc;
    if (latched(d)) return latched(d);
    if (iterations) *iterations = d.info[n];
    if (sweeps) *sweeps = d.eig_sweeps[n];
    if (residual) *residual = d.eig_resid[n];
    if (stop) *stop = d.eig_stop[n];
    return HOTRG_OK;
}

int hotrg_set_eig_limits(hotrg_solve* s, int max_passes, double fail_residual) {
    if (s) quiesce(s);
    if (!s || max_passes < 1 || max_passes > HOTRG_EIG_MAX_PASSES) return HOTRG_EINVAL;
    if (!(fail_residual > 0.0) || !isfinite(fail_residual)) return HOTRG_EINVAL;
    s->eig_maxit = max_passes;
    s->eig_fail = fail_residual;
    return HOTRG_OK;
}

int hotrg_step_sides(hotrg_solve* s, int n, double* eps_left, double* eps_right, int* side) {
    if (s) quiesce(s);
    if (!s || n < 1 || n > s->steps) return HOTRG_EINVAL;
    if (s->host_status) return s->host_status;
    DevState d;
    int rc = read_state(s, &d);
    if (rc) return rc;
    if (latched(d)) return latched(d);
    if (eps_left) *eps_left = d.eps_left[n];
    if (eps_right) *eps_right = s->p.two_sided ? d.eps_right[n] : NAN;
    if (side) *side = d.side[n];
    return HOTRG_OK;
}

int hotrg_observables(hotrg_solve* s, double values[2]) {
    if (s) quiesce(s);
    if (!s || !values) return HOTRG_EINVAL;
    if (s->host_status) return s->host_status;
    HIP_TRY(s, launch_trace(s->T(), s->dx, s->dy, s->state(), s->stream));
    for (int j = 0; j < s->L.nimp; ++j)
        HIP_TRY(s, launch_trace(s->I(j), s->dx, s->dy, s->state(), s->stream, &s->state()->imp_trace[j]));
    DevState d;
    int rc = read_state(s, &d);
    if (rc) return rc;
    if (latched(d)) return latched(d);
    if (!(d.trace != 0.0) || !isfinite(d.trace)) return HOTRG_ENONFINITE;
    values[0] = values[1] = NAN;
    for (int j = 0; j < s->L.nimp; ++j) values[s->imp_slot[j]] = d.imp_trace[j] / d.trace;
    return HOTRG_OK;
}

int hotrg_copy_tensor(hotrg_solve* s, double* host, size_t capacity, int dims[2]) {
    if (s) quiesce(s);
    if (!s || !dims) return HOTRG_EINVAL;
    if (s->host_status) return s->host_status;
    dims[0] = s->dx;
    dims[1] = s->dy;
    const size_t count = (size_t)s->dx * s->dx * s->dy * s->dy;
    if (!host || capacity < count) return HOTRG_EINVAL;
    DevState d;
    int rc = read_state(s, &d);
    if (rc) return rc;
    if (latched(d)) return latched(d);
    HIP_TRY(s, hipMemcpyAsync(host, s->T(), count * sizeof(double), hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(s, hipStreamSynchronize(s->stream));
    return HOTRG_OK;
}

int hotrg_copy_environment(hotrg_solve* s, double* host, size_t capacity, int* n) {
    if (s) quiesce(s);
    if (!s || !n) return HOTRG_EINVAL;
    if (s->host_status) return s->host_status;
    *n = s->last_n;
    const size_t count = (size_t)s->last_n * s->last_n;
    if (s->steps < 1 || !host || capacity < count) return HOTRG_EINVAL;
    DevState d;
    int rc = read_state(s, &d);
    if (rc) return rc;
    if (latched(d)) return latched(d);
    HIP_TRY(s, hipMemcpyAsync(host, s->ws + s->L.oE, count * sizeof(double), hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(s, hipStreamSynchronize(s->stream));
    return HOTRG_OK;
}

int hotrg_copy_isometry(hotrg_solve* s, double* host, size_t capacity, int dims[2]) {
    if (s) quiesce(s);
    if (!s || !dims) return HOTRG_EINVAL;
    if (s->host_status) return s->host_status;
    const int n = s->last_n, dp = s->last_dp;
    dims[0] = n;
    dims[1] = dp;
    const size_t count = (size_t)n * dp;
    if (s->steps < 1 || !host || capacity < count) return HOTRG_EINVAL;
    DevState d;
    int rc = read_state(s, &d);
    if (rc) return rc;
    if (latched(d)) return latched(d);
    // Ut[l, i] = u_l[i] in the contraction format: planes of round_up(nU, 64)
    // elements one after the other
    const Fmt f = s->fmt;
    const size_t plane = round_up(std::max<size_t>(s->L.nU, 1), 64);
    const int planes = fmt_planes(f);
    const size_t eb = fmt_plane_elem_bytes(f);
    std::vector<char> raw((size_t)planes * plane * eb);
    HIP_TRY(s, hipMemcpyAsync(raw.data(), s->ws + s->L.oUt, raw.size(), hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(s, hipStreamSynchronize(s->stream));
    for (int l = 0; l < dp; ++l)
        for (int i = 0; i < n; ++i) {
            const size_t e = (size_t)l * n + i;
            double v = 0.0;
            if (f == Fmt::F64) {
                v = reinterpret_cast<const double*>(raw.data())[e];
            } else if (f == Fmt::F32) {
                v = reinterpret_cast<const float*>(raw.data())[e];
            } else {
                for (int pl = 0; pl < planes; ++pl) {
                    uint16_t b;
                    memcpy(&b, raw.data() + ((size_t)pl * plane + e) * 2, 2);
                    const uint32_t bits = (uint32_t)b << 16;
                    float x;
                    memcpy(&x, &bits, 4);
                    v += x;
                }
            }
            host[(size_t)i * dp + l] = v;
        }
    return HOTRG_OK;
}

int hotrg_set_timing(hotrg_solve* s, int enable) {
    if (s) quiesce(s);
    if (!s) return HOTRG_EINVAL;
    HIP_TRY(s, hipStreamSynchronize(s->stream));
    for (hipEvent_t e : s->ev) (void)hipEventDestroy(e);
    s->ev.clear();
    s->timed_dims.clear();
    s->timing = enable != 0;
    s->timed_from = s->steps;
    if (s->timing) {
        const int n = (HOTRG_MAX_STEPS - s->steps) * kEventsPerStep;
        s->ev.resize(n);
        for (int i = 0; i < n; ++i) HIP_TRY(s, hipEventCreate(&s->ev[i]));
    }
    return HOTRG_OK;
}

static float elapsed(hotrg_solve* s, int step, int a, int b) {
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, s->ev[(size_t)step * kEventsPerStep + a], s->ev[(size_t)step * kEventsPerStep + b]);
    return ms;
}

int hotrg_stage_times(hotrg_solve* s, double* ms, int* steps_timed) {
    if (s) quiesce(s);
    if (!s || !ms) return HOTRG_EINVAL;
    for (int i = 0; i < HOTRG_NUM_STAGES; ++i) ms[i] = 0.0;
    const int nt = s->timing ? s->steps - s->timed_from : 0;
    if (steps_timed) *steps_timed = nt;
    if (!nt) return HOTRG_OK;
    HIP_TRY(s, hipStreamSynchronize(s->stream));
    for (int i = 0; i < nt; ++i) {
        ms[HOTRG_STAGE_PERMUTE] += elapsed(s, i, 0, 1) + elapsed(s, i, 3, 4) + elapsed(s, i, 5, 6);
        ms[HOTRG_STAGE_ENV] += elapsed(s, i, 1, 2);
        ms[HOTRG_STAGE_EIG] += elapsed(s, i, 2, 3);
        ms[HOTRG_STAGE_X] += elapsed(s, i, 4, 5);
        ms[HOTRG_STAGE_Y] += elapsed(s, i, 6, 7);
        ms[HOTRG_STAGE_TP] += elapsed(s, i, 7, 8);
        ms[HOTRG_STAGE_NORM] += elapsed(s, i, 8, 9);
        ms[HOTRG_STAGE_OBS] += elapsed(s, i, 9, 10);
    }
    return HOTRG_OK;
}

int hotrg_step_stage_times(hotrg_solve* s, int k, double* ms, int dims[3]) {
    if (s) quiesce(s);
    if (!s || !ms || !s->timing || k < 0 || k >= s->steps - s->timed_from || (size_t)k >= s->timed_dims.size())
        return HOTRG_EINVAL;
    HIP_TRY(s, hipStreamSynchronize(s->stream));
    for (int i = 0; i < HOTRG_NUM_STAGES; ++i) ms[i] = 0.0;
    ms[HOTRG_STAGE_PERMUTE] = elapsed(s, k, 0, 1) + elapsed(s, k, 3, 4) + elapsed(s, k, 5, 6);
    ms[HOTRG_STAGE_ENV] = elapsed(s, k, 1, 2);
    ms[HOTRG_STAGE_EIG] = elapsed(s, k, 2, 3);
    ms[HOTRG_STAGE_X] = elapsed(s, k, 4, 5);
    ms[HOTRG_STAGE_Y] = elapsed(s, k, 6, 7);
    ms[HOTRG_STAGE_TP] = elapsed(s, k, 7, 8);
    ms[HOTRG_STAGE_NORM] = elapsed(s, k, 8, 9);
    ms[HOTRG_STAGE_OBS] = elapsed(s, k, 9, 10);
    if (dims) {
        dims[0] = s->timed_dims[(size_t)k].dx;
        dims[1] = s->timed_dims[(size_t)k].dy;
        dims[2] = s->timed_dims[(size_t)k].dp;
    }
    return HOTRG_OK;
}

int hotrg_gemm_y_time(hotrg_solve* s, double* ms, int* launches) {
    if (s) quiesce(s);
    if (!s || !ms) return HOTRG_EINVAL;
    double st[HOTRG_NUM_STAGES];
    int nt = 0;
    const int rc = hotrg_stage_times(s, st, &nt);
    if (rc) return rc;
    *ms = st[HOTRG_STAGE_Y];
    if (launches) *launches = nt;
    return HOTRG_OK;
}

void hotrg_destroy(hotrg_solve* s) {
    if (!s) return;
    quiesce(s);
    (void)hipStreamSynchronize(s->stream);
    for (hipEvent_t e : s->ev) (void)hipEventDestroy(e);
    if (s->mail) (void)hipHostFree(s->mail);
    delete s;
}

const char* hotrg_strerror(int status) {
    switch (status) {
        case HOTRG_OK: return "ok";
        case HOTRG_EINVAL: return "invalid argument";
        case HOTRG_ENOMEM: return "workspace too small";
        case HOTRG_EHIP: return "HIP runtime error";
        case HOTRG_EEIG: return "eigensolver failure";
        case HOTRG_ENONFINITE: return "non-finite or non-positive normalisation";
        case HOTRG_ESTATE: return "handle in failed state";
        case HOTRG_ENODEV: return "no HIP device";
        default: return "unknown status";
    }
}

int hotrg_device_count(int* count) {
    if (!count) return HOTRG_EINVAL;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess) n = 0;
    *count = n;
    return HOTRG_OK;
}

int hotrg_runtime_version(int* version) {
    if (!version) return HOTRG_EINVAL;
    return hipRuntimeGetVersion(version) == hipSuccess ? HOTRG_OK : HOTRG_EHIP;
}

size_t hotrg_gemm_scratch_bytes(int precision, int M, int N, int K) {
    return hotrg::gemm_scratch_bytes(precision, M, N, K);
}

int hotrg_gemm_nt_role(int precision, int role, int panel, int M, int N, int K, const double* A, long lda,
                       const double* B, long ldb, double* C, double alpha, long sm, long rs_hi, long rs_lo, long sn,
                       long cs_hi, long cs_lo, void* scratch, void* stream) {
    return hotrg::gemm_nt_with_scratch(precision, role, panel, M, N, K, A, lda, B, ldb, C, alpha, sm, rs_hi, rs_lo,
                                       sn, cs_hi, cs_lo, scratch, SIZE_MAX, stream);
}

int hotrg_gemm_nt(int precision, int M, int N, int K, const double* A, long lda, const double* B, long ldb,
                  double* C, double alpha, long sm, long rs_hi, long rs_lo, long sn, long cs_hi, long cs_lo,
                  void* scratch, void* stream) {
    return hotrg_gemm_nt_role(precision, HOTRG_ROLE_GENERIC, 0, M, N, K, A, lda, B, ldb, C, alpha, sm, rs_hi, rs_lo,
                              sn, cs_hi, cs_lo, scratch, stream);
}

}  // extern "C"
