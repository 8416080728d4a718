// Index-mapped "NT" matrix product on gfx950 matrix cores:
//   C[map(m, n)] = alpha * sum_k A[m*lda + k] * B[n*ldb + k]
//
// Every contraction of a HOTRG step (half environments, E, X = U.T,
// Y = X.T, T' = Y.U) is this one kernel with different operand strides and
// output maps.  The output map writes each result straight into the fused-
// index layout the next stage reads, so no contraction result is ever
// permuted afterwards (the permute-free mapping of Sec. II.B, Eq. (3)).
//
// The paper's quad-tile scheme splits every index into a small in-block part
// and a block index, multiplies all 2x2 blocks at once and then sums over the
// K blocks (Sec. II.B, Eq. (4)).  On a CDNA4 compute unit the same split is
// a 16x16xk MFMA fragment product per wavefront (the in-block part) and an
// LDS-staged loop over K tiles (the block sum); workgroup tiles are spread
// over all 256 CUs instead of over FPGA DSP slices.
//
// Layout: a workgroup of WAVES_M x WAVES_N wavefronts owns a BM x BN tile of
// C; each wave owns (BM/WAVES_M) x (BN/WAVES_N) as 16x16 MFMA fragments.
// K is consumed in BK-wide tiles, double-buffered in LDS (rows padded so the
// 16-row fragment reads hit distinct banks), with the next tile's global
// loads in flight while the current one is multiplied.  Tiles are assigned
// so that the workgroups one XCD runs together share the same A rows
// (workgroup i runs on XCD i mod 8), keeping the big operand's re-reads in
// that XCD's L2.
#include <type_traits>

#include "common.h"

namespace hotrg {

// ---------------------------------------------------------------- tile choices

// Register-staged BF16-split product (K not a multiple of 16): workgroup
// BM x BN over WM x WN waves, PF K stages of global loads in flight.
// 256 x 256 on 8 waves measured fastest for the D = 48 Y product in this
// form (6.9 ms vs 8.5 ms for 256 x 128, 11.5 ms for 128 x 128): the split
// operands make the product L2-bandwidth-bound, and the larger tile reads
// each operand byte fewer times.
constexpr int kP32BM = 256, kP32BN = 256, kP32WM = 4, kP32WN = 2, kP32PF = 1;
// direct-to-LDS 256 x 256 tiles on row-major operands: waves
constexpr int kDmaWM = 4, kDmaWN = 2;
// narrow outputs (T', N = D'): three stages (two measured slower for T':
// 12.1 -> 16.1 ms per D = 48 solve), one workgroup per CU
constexpr int kNarrowNst = 3, kNarrowMinw = 1;
// T' reading Y in FP32 (split on load): register-staged 128 x 64 tiles,
// four waves, one prefetch stage and one LDS tile (two barriers per K step)
// so that five workgroups fit a CU: the product is bound by the latency of
// its A loads, and more workgroups keep more of them in flight (per D = 48
// solve: 10.4 ms, against 14.4 with two LDS tiles of 64 rows, 11.0 with one
// of 64 rows, 17.4 with one of 32)
constexpr int kTpBM = 128, kTpWM = 4, kTpPF = 1, kTpNbuf = 1;
// mid-size products (half environments, E): two stages, up to three
// workgroups per CU (env 19.2 -> 18.3 ms per D = 48 solve)
constexpr int kMidNst = 2, kMidMinw = 2;
// the Y product (panel operands) at full size
constexpr int kYBM = 256, kYBN = 256, kYWM = 4, kYWN = 2, kYNst = 3, kYMinw = 1;


// ---------------------------------------------------------------- MFMA ops

template <typename T> struct Mma;

template <> struct Mma<double> {
    using acc_t = d4;
    // v_mfma_f64_16x16x4_f64: lane l supplies A[l%16][l/16] and B[l/16][l%16];
    // the result rows interleave: D[(l/16) + 4r][l%16] is component r of lane l
    // (measured on gfx950).
    __device__ static acc_t run(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    __device__ static int row(int group, int r) { return group + 4 * r; }
};

template <> struct Mma<float> {
    using acc_t = f4;
    // v_mfma_f32_16x16x4_f32: same A/B lane layout as the f64 form; the
    // result is blocked: D[4*(l/16) + r][l%16] is component r of lane l.
    __device__ static acc_t run(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    __device__ static int row(int group, int r) { return 4 * group + r; }
};

// ---------------------------------------------------------------- stores

__device__ __forceinline__ void split_store(__bf16* base, size_t plane, int nplanes, long off, float v) {
    // v = hi + mid + lo, each rounded to nearest-even bf16 in fp32 arithmetic
    __bf16 h = (__bf16)v;
    base[off] = h;
    float r = v - (float)h;
    __bf16 m = (__bf16)r;
    base[off + plane] = m;
    if (nplanes == 3) {
        float r2 = r - (float)m;
        base[off + 2 * plane] = (__bf16)r2;
    }
}

struct Store {
    void* ptr;
    size_t plane;
    int fmt;  // Fmt
    double alpha;
    template <typename V>
    __device__ __forceinline__ void operator()(long off, V v) const {
        switch (fmt) {
            case (int)Fmt::F64: static_cast<double*>(ptr)[off] = alpha * (double)v; break;
            case (int)Fmt::F32: static_cast<float*>(ptr)[off] = (float)(alpha * (double)v); break;
            case (int)Fmt::BF16x2: split_store(static_cast<__bf16*>(ptr), plane, 2, off, (float)(alpha * (double)v)); break;
            case (int)Fmt::F16x2: {
                _Float16* p = static_cast<_Float16*>(ptr);
                f16_split((float)(alpha * (double)v), p + off, p + off + plane);
                break;
            }
            default: split_store(static_cast<__bf16*>(ptr), plane, 3, off, (float)(alpha * (double)v)); break;
        }
    }
};

// Row and column parts of the output map: r sums to the offset (or the
// panel row), c to the panel column (zero for row-major maps).
struct MapPart {
    long r, c;
};
__device__ __forceinline__ MapPart map_row(const OutMap& mp, unsigned m) {
    const unsigned sm = (unsigned)mp.sm;
    const unsigned hi = m / sm;
    const long lo = (long)(m - hi * sm);
    return {(long)hi * mp.rs_hi + lo * mp.rs_lo, (long)hi * mp.rc_hi + lo * mp.rc_lo};
}
__device__ __forceinline__ MapPart map_col(const OutMap& mp, unsigned n) {
    const unsigned sn = (unsigned)mp.sn;
    const unsigned hi = n / sn;
    const long lo = (long)(n - hi * sn);
    return {(long)hi * mp.cs_hi + lo * mp.cs_lo, (long)hi * mp.cc_hi + lo * mp.cc_lo};
}
__device__ __forceinline__ long map_off(const OutMap& mp, const MapPart& row, const MapPart& col) {
    return mp.panel_k ? panel_index(row.r + col.r, row.c + col.c, mp.panel_k) : row.r + col.r;
}

// ---------------------------------------------------------------- kernel

// ROLE only gives each contraction of a step its own kernel symbol (so a
// profiler separates them); the code is the same.
template <typename T, int BM, int BN, int BK, int WAVES_M, int WAVES_N, int ROLE>
__global__ __launch_bounds__(64 * WAVES_M * WAVES_N)
void gemm_nt_kernel(const T* __restrict__ A, long lda, const T* __restrict__ B, long ldb,
                    int M, int N, int K, Store store, OutMap mp,
                    int tiles_m, int tiles_n, int per_xcd)
{
    using Op = Mma<T>;
    using acc_t = typename Op::acc_t;
    constexpr int NT = 64 * WAVES_M * WAVES_N;
    constexpr int WM = BM / WAVES_M;
    constexpr int WN = BN / WAVES_N;
    constexpr int FM = WM / 16;
    constexpr int FN = WN / 16;
    constexpr int PAD = sizeof(T) == 8 ? 2 : 4;
    constexpr int LDK = BK + PAD;
    constexpr int A_PER_T = BM * BK / NT;
    constexpr int B_PER_T = BN * BK / NT;
    static_assert(BM * BK % NT == 0 && BN * BK % NT == 0, "tile/threads mismatch");
    static_assert(NT % BK == 0, "a row of the K tile must be loaded by whole thread groups");

    __shared__ T As[2][BM * LDK];
    __shared__ T Bs[2][BN * LDK];

    // XCD-aware tile order: consecutive tiles (same A rows, N fastest) go to
    // workgroups that the dispatcher places on the same XCD.
    const int bid = blockIdx.x;
    const int tile = (bid & 7) * per_xcd + (bid >> 3);
    if (tile >= tiles_m * tiles_n) return;
    const int tm = tile / tiles_n;
    const int tn = tile - tm * tiles_n;
    const int m0 = tm * BM;
    const int n0 = tn * BN;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm = wave / WAVES_N;
    const int wn = wave - wm * WAVES_N;

    // global -> register staging: element e = tid + NT*i of the tile,
    // row e / BK, column e % BK (BK consecutive threads read one row segment)
    const int lrow = tid / BK;
    const int lcol = tid - lrow * BK;
    constexpr int ROWS_PER_PASS = NT / BK;

    T ra[A_PER_T], rb[B_PER_T];

    auto load_tile = [&](int k0) {
        const int k = k0 + lcol;
        const bool kin = k < K;
#pragma unroll
        for (int i = 0; i < A_PER_T; ++i) {
            const int r = m0 + lrow + i * ROWS_PER_PASS;
            ra[i] = (kin && r < M) ? A[(long)r * lda + k] : T(0);
        }
#pragma unroll
        for (int i = 0; i < B_PER_T; ++i) {
            const int r = n0 + lrow + i * ROWS_PER_PASS;
            rb[i] = (kin && r < N) ? B[(long)r * ldb + k] : T(0);
        }
    };
    auto store_tile = [&](int buf) {
#pragma unroll
        for (int i = 0; i < A_PER_T; ++i) As[buf][(lrow + i * ROWS_PER_PASS) * LDK + lcol] = ra[i];
#pragma unroll
        for (int i = 0; i < B_PER_T; ++i) Bs[buf][(lrow + i * ROWS_PER_PASS) * LDK + lcol] = rb[i];
    };

    acc_t acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[i][j] = acc_t{0, 0, 0, 0};

    const int nk = (K + BK - 1) / BK;
    load_tile(0);
    store_tile(0);
    __syncthreads();

    const int frow = lane & 15;   // fragment row (A) / column (B) of this lane
    const int fk = lane >> 4;     // k offset within a 4-wide MFMA step

    for (int kt = 0; kt < nk; ++kt) {
        const int buf = kt & 1;
        if (kt + 1 < nk) load_tile((kt + 1) * BK);
        const T* as = &As[buf][(wm * WM + frow) * LDK + fk];
        const T* bs = &Bs[buf][(wn * WN + frow) * LDK + fk];
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
            T a[FM], b[FN];
#pragma unroll
            for (int i = 0; i < FM; ++i) a[i] = as[i * 16 * LDK + kk];
#pragma unroll
            for (int j = 0; j < FN; ++j) b[j] = bs[j * 16 * LDK + kk];
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j) acc[i][j] = Op::run(a[i], b[j], acc[i][j]);
        }
        if (kt + 1 < nk) store_tile(buf ^ 1);
        __syncthreads();
    }

    // epilogue: component r of each fragment holds row Op::row(lane/16, r), column lane%16
    MapPart coff[FN];
    bool cin[FN];
#pragma unroll
    for (int j = 0; j < FN; ++j) {
        const int n = n0 + wn * WN + j * 16 + frow;
        cin[j] = n < N;
        coff[j] = cin[j] ? map_col(mp, (unsigned)n) : MapPart{0, 0};
    }
#pragma unroll
    for (int i = 0; i < FM; ++i) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int m = m0 + wm * WM + i * 16 + Op::row(fk, r);
            if (m >= M) continue;
            const MapPart roff = map_row(mp, (unsigned)m);
#pragma unroll
            for (int j = 0; j < FN; ++j)
                if (cin[j]) store(map_off(mp, roff, coff[j]), acc[i][j][r]);
        }
    }
}


// ---------------------------------------------------------------- BF16-split kernel

// Split products: plane pairs (a, b) multiplied for each precision mode.
//   2 terms, 3 products:  hi*hi + hi*lo + lo*hi
//   3 terms, 6 products:  hi*hi + hi*mid + mid*hi + hi*lo + lo*hi + mid*mid
template <int NPROD> struct SplitProducts;
template <> struct SplitProducts<3> {
    static constexpr int planes = 2;
    __device__ static constexpr int a(int i) { return i == 2 ? 1 : 0; }
    __device__ static constexpr int b(int i) { return i == 1 ? 1 : 0; }
};
template <> struct SplitProducts<6> {
    static constexpr int planes = 3;
    // order: hi*hi, hi*mid, mid*hi, hi*lo, lo*hi, mid*mid
    __device__ static constexpr int a(int i) { return i == 2 ? 1 : (i == 4 ? 2 : (i == 5 ? 1 : 0)); }
    __device__ static constexpr int b(int i) { return i == 1 ? 1 : (i == 3 ? 2 : (i == 5 ? 1 : 0)); }
};

// Operands stored as bf16 planes (plane p of A at A + p * a_plane, rows of
// length lda), the planes of one value summing to it (hi + lo or
// hi + mid + lo, written by the producing kernels); products on
// v_mfma_f32_32x32x16_bf16 with FP32 accumulation (measured on gfx950: lane l supplies A[l%32][8(l/32)..8(l/32)+7] and
// B[8(l/32)..+7][l%32]; component r of lane l is result row
// 8(r/4) + 4(l/32) + r%4, column l%32).  K is staged 16 at a time (one MFMA
// k-step per LDS stage), which lets a 256-row tile double-buffer three planes
// of both operands in LDS.
//
// AF32: A is one FP32 array instead (the Y product's output, read by T'):
// its rows are fetched as FP32 and split into the BF16 planes (hi, mid, lo
// by round-to-nearest-even, the split the producers' epilogues use) as the
// tile is written to LDS, so each element is split once.
template <int NPROD, int BM, int BN, int WAVES_M, int WAVES_N, int PF, int ROLE, bool AF32 = false, int NBUF = 2>
__global__ __launch_bounds__(64 * WAVES_M * WAVES_N)
void gemm_nt_bf16p32_kernel(const __bf16* __restrict__ A, long lda, long a_plane,
                            const __bf16* __restrict__ B, long ldb, long b_plane,
                            int M, int N, int K, Store store, OutMap mp,
                            int tiles_m, int tiles_n, int per_xcd, int vec)
{
    using SP = SplitProducts<NPROD>;
    typedef float f16v __attribute__((ext_vector_type(16)));
    typedef unsigned int u4 __attribute__((ext_vector_type(4)));
    constexpr int NPL = SP::planes;
    constexpr int BK = 16;
    constexpr int NT = 64 * WAVES_M * WAVES_N;
    constexpr int WM = BM / WAVES_M;
    constexpr int WN = BN / WAVES_N;
    constexpr int FM = WM / 32;
    constexpr int FN = WN / 32;
    constexpr int LDK = BK + 8;           // 48-byte LDS rows: 16-byte aligned, conflict-free 16-byte reads
    constexpr int CPR = BK / 8;           // 16-byte chunks per tile row
    constexpr int A_CH = (BM * CPR + NT - 1) / NT;   // chunks per thread (the last pass may be partial)
    constexpr int B_CH = (BN * CPR + NT - 1) / NT;
    static_assert(WM % 32 == 0 && WN % 32 == 0, "wave tile must be whole 32x32 fragments");

    // NBUF = 1: one LDS tile (two barriers per K step), so that twice as many
    // workgroups, and twice as many loads, fit a CU
    static_assert(NBUF == 2 || (NBUF == 1 && PF == 1), "one LDS buffer only with one prefetch stage");
    __shared__ __attribute__((aligned(16))) __bf16 As[NBUF][NPL][BM * LDK];
    __shared__ __attribute__((aligned(16))) __bf16 Bs[NBUF][NPL][BN * LDK];

    const int bid = blockIdx.x;
    const int tile = (bid & 7) * per_xcd + (bid >> 3);
    if (tile >= tiles_m * tiles_n) return;
    const int tm = tile / tiles_n;
    const int tn = tile - tm * tiles_n;
    const int m0 = tm * BM;
    const int n0 = tn * BN;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm = wave / WAVES_N;
    const int wn = wave - wm * WAVES_N;

    static_assert(PF == 1 || PF == 2, "prefetch depth 1 or 2");
    constexpr int ARP = AF32 ? 2 : NPL;   // registers (u4) per A chunk: 8 floats, or the planes
    u4 ra[PF][ARP][A_CH], rb[PF][NPL][B_CH];

    // 8 FP32 values of row `row` from column k (zeros outside), kept raw
    auto fetch_a32 = [&](int nrows, int row, int k, u4 (&dst)[ARP]) {
        const float* base = reinterpret_cast<const float*>(A);
        if (row < nrows && vec && k + 8 <= K) {
            const u4* src = reinterpret_cast<const u4*>(base + (long)row * lda + k);
            dst[0] = src[0];
            dst[1] = src[1];
        } else {
            float e[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) e[q] = (row < nrows && k + q < K) ? base[(long)row * lda + k + q] : 0.f;
            dst[0] = u4{__builtin_bit_cast(unsigned, e[0]), __builtin_bit_cast(unsigned, e[1]),
                        __builtin_bit_cast(unsigned, e[2]), __builtin_bit_cast(unsigned, e[3])};
            dst[1] = u4{__builtin_bit_cast(unsigned, e[4]), __builtin_bit_cast(unsigned, e[5]),
                        __builtin_bit_cast(unsigned, e[6]), __builtin_bit_cast(unsigned, e[7])};
        }
    };
    // the NPL planes of 8 raw FP32 values
    auto split8 = [&](const u4 (&raw)[ARP], u4 (&pl)[NPL]) {
        unsigned short e[NPL][8];
        // components copied out by name first: __builtin_bit_cast of an
        // indexed vector component was measured to read component 0
        const unsigned w[8] = {raw[0].x, raw[0].y, raw[0].z, raw[0].w, raw[1].x, raw[1].y, raw[1].z, raw[1].w};
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const float f = __builtin_bit_cast(float, w[q]);
            const __bf16 hi = (__bf16)f;
            const float rem = f - (float)hi;
            const __bf16 md = (__bf16)rem;
            e[0][q] = __builtin_bit_cast(unsigned short, hi);
            e[1][q] = __builtin_bit_cast(unsigned short, md);
            if constexpr (NPL == 3) e[2][q] = __builtin_bit_cast(unsigned short, (__bf16)(rem - (float)md));
        }
#pragma unroll
        for (int p = 0; p < NPL; ++p)
            pl[p] = u4{e[p][0] | (unsigned)e[p][1] << 16, e[p][2] | (unsigned)e[p][3] << 16,
                       e[p][4] | (unsigned)e[p][5] << 16, e[p][6] | (unsigned)e[p][7] << 16};
    };

    auto fetch = [&](const __bf16* base, long ld, long pstride, int nrows, int row, int k, u4 (&dst)[NPL]) {
        if (row < nrows && vec && k + 8 <= K) {
#pragma unroll
            for (int pl = 0; pl < NPL; ++pl)
                dst[pl] = *reinterpret_cast<const u4*>(base + pl * pstride + (long)row * ld + k);
        } else {
#pragma unroll
            for (int pl = 0; pl < NPL; ++pl) {
                unsigned short e[8];
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    __bf16 v = (__bf16)0.0f;
                    if (row < nrows && k + q < K) v = base[pl * pstride + (long)row * ld + k + q];
                    e[q] = __builtin_bit_cast(unsigned short, v);
                }
                dst[pl] = u4{e[0] | (unsigned)e[1] << 16, e[2] | (unsigned)e[3] << 16,
                             e[4] | (unsigned)e[5] << 16, e[6] | (unsigned)e[7] << 16};
            }
        }
    };
    auto load_tile = [&](int k0, auto set) {
        constexpr int S = decltype(set)::value;
#pragma unroll
        for (int i = 0; i < A_CH; ++i) {
            const int c = tid + i * NT, row = c / CPR, kc = c - (c / CPR) * CPR;
            u4 t[ARP];
            if constexpr (AF32)
                fetch_a32(c < BM * CPR ? M : 0, m0 + row, k0 + 8 * kc, t);
            else
                fetch(A, lda, a_plane, c < BM * CPR ? M : 0, m0 + row, k0 + 8 * kc, t);
#pragma unroll
            for (int pl = 0; pl < ARP; ++pl) ra[S][pl][i] = t[pl];
        }
#pragma unroll
        for (int i = 0; i < B_CH; ++i) {
            const int c = tid + i * NT, row = c / CPR, kc = c - (c / CPR) * CPR;
            u4 t[NPL];
            fetch(B, ldb, b_plane, c < BN * CPR ? N : 0, n0 + row, k0 + 8 * kc, t);
#pragma unroll
            for (int pl = 0; pl < NPL; ++pl) rb[S][pl][i] = t[pl];
        }
    };
    auto store_tile = [&](int buf, auto set) {
        constexpr int S = decltype(set)::value;
#pragma unroll
        for (int i = 0; i < A_CH; ++i) {
            const int c = tid + i * NT, row = c / CPR, kc = c - (c / CPR) * CPR;
            if (c < BM * CPR) {
                u4 t[NPL];
                if constexpr (AF32) {
                    u4 raw[ARP];
#pragma unroll
                    for (int q = 0; q < ARP; ++q) raw[q] = ra[S][q][i];
                    split8(raw, t);
                } else {
#pragma unroll
                    for (int pl = 0; pl < NPL; ++pl) t[pl] = ra[S][pl][i];
                }
#pragma unroll
                for (int pl = 0; pl < NPL; ++pl) *reinterpret_cast<u4*>(&As[buf][pl][row * LDK + 8 * kc]) = t[pl];
            }
        }
#pragma unroll
        for (int i = 0; i < B_CH; ++i) {
            const int c = tid + i * NT, row = c / CPR, kc = c - (c / CPR) * CPR;
            if (c < BN * CPR)
#pragma unroll
                for (int pl = 0; pl < NPL; ++pl) *reinterpret_cast<u4*>(&Bs[buf][pl][row * LDK + 8 * kc]) = rb[S][pl][i];
        }
    };
    using S0 = std::integral_constant<int, 0>;
    using S1 = std::integral_constant<int, PF - 1>;

    f16v acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

    const int frow = lane & 31;
    const int fk = lane >> 5;   // which 8-element half of the 16-wide k step

    auto compute = [&](int buf) {
        bf16x8 a[NPL][FM], b[NPL][FN];
#pragma unroll
        for (int pl = 0; pl < NPL; ++pl) {
#pragma unroll
            for (int i = 0; i < FM; ++i)
                a[pl][i] = *reinterpret_cast<const bf16x8*>(&As[buf][pl][(wm * WM + i * 32 + frow) * LDK + 8 * fk]);
#pragma unroll
            for (int j = 0; j < FN; ++j)
                b[pl][j] = *reinterpret_cast<const bf16x8*>(&Bs[buf][pl][(wn * WN + j * 32 + frow) * LDK + 8 * fk]);
        }
#pragma unroll
        for (int pr = NPROD - 1; pr >= 0; --pr)   // smallest products first
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[SP::a(pr)][i], b[SP::b(pr)][j], acc[i][j],
                                                                        0, 0, 0);
    };

    const int nk = (K + BK - 1) / BK;
    load_tile(0, S0{});
    store_tile(0, S0{});
    if constexpr (NBUF == 1) {
        __syncthreads();
        for (int kt = 0; kt < nk; ++kt) {
            if (kt + 1 < nk) load_tile((kt + 1) * BK, S0{});
            compute(0);
            __syncthreads();
            if (kt + 1 < nk) store_tile(0, S0{});
            __syncthreads();
        }
    } else if constexpr (PF == 1) {
        __syncthreads();
        for (int kt = 0; kt < nk; ++kt) {
            const int buf = kt & 1;
            if (kt + 1 < nk) load_tile((kt + 1) * BK, S0{});
            compute(buf);
            if (kt + 1 < nk) store_tile(buf ^ 1, S0{});
            __syncthreads();
        }
    } else {
        // two stages in flight: stage kt+1 waits in register set (kt+1)&1 while
        // stage kt+2 is being fetched into the other set
        if (nk > 1) load_tile(BK, S1{});
        __syncthreads();
        for (int kt = 0; kt < nk; kt += 2) {
            if (kt + 2 < nk) load_tile((kt + 2) * BK, S0{});
            compute(0);
            if (kt + 1 < nk) store_tile(1, S1{});
            __syncthreads();
            if (kt + 1 >= nk) break;
            if (kt + 3 < nk) load_tile((kt + 3) * BK, S1{});
            compute(1);
            if (kt + 2 < nk) store_tile(0, S0{});
            __syncthreads();
        }
    }

    // Wave tiles of more than four 32 x 32 fragments: the output goes
    // through 16-row FP32 slabs in LDS (the A and B tiles are free now), so
    // the accumulators are only ever indexed with constants; indexing them
    // by a loop counter the compiler keeps as a loop would put the whole
    // accumulator array in scratch memory in every launch.  A lane stores
    // columns lane, lane + 64, ... of each slab row.
    constexpr int RW4 = WN + 4;
    constexpr int SLAB4 = 16 * RW4;
    constexpr int A_SLABS = (int)(sizeof(As) / sizeof(float)) / SLAB4;
    constexpr int B_SLABS = (int)(sizeof(Bs) / sizeof(float)) / SLAB4;
    constexpr int NW = WAVES_M * WAVES_N;
    if constexpr (FM * FN > 4 && A_SLABS + B_SLABS >= NW) {
        constexpr int CPLG = (WN + 63) / 64;
        float* reg = wave < A_SLABS ? reinterpret_cast<float*>(&As[0][0][0]) + wave * SLAB4
                                    : reinterpret_cast<float*>(&Bs[0][0][0]) + (wave - A_SLABS) * SLAB4;
        MapPart gcol[CPLG];
        bool gok[CPLG];
#pragma unroll
        for (int t = 0; t < CPLG; ++t) {
            const int c = lane + 64 * t;
            const int n = c < WN ? n0 + wn * WN + c : N;
            gok[t] = n < N;
            gcol[t] = gok[t] ? map_col(mp, (unsigned)n) : MapPart{0, 0};
        }
#pragma unroll
        for (int i = 0; i < FM; ++i) {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
#pragma unroll
                for (int j = 0; j < FN; ++j)
#pragma unroll
                    for (int rr = 0; rr < 8; ++rr) {
                        const int row = 8 * (rr >> 2) + 4 * fk + (rr & 3);
                        reg[row * RW4 + j * 32 + frow] = acc[i][j][8 * h + rr];
                    }
                __builtin_amdgcn_s_waitcnt(0xC07F);   // lgkmcnt(0): this wave's staging writes are done
                for (int row = 0; row < 16; ++row) {
                    const int m = m0 + wm * WM + i * 32 + 16 * h + row;
                    if (m >= M) break;
                    const MapPart roff = map_row(mp, (unsigned)m);
#pragma unroll
                    for (int t = 0; t < CPLG; ++t)
                        if (gok[t]) store(map_off(mp, roff, gcol[t]), reg[row * RW4 + lane + 64 * t]);
                }
                __builtin_amdgcn_s_waitcnt(0xC07F);   // staging reads are done before the region is rewritten
            }
        }
        return;
    }

    MapPart coff[FN];
    bool cin[FN];
#pragma unroll
    for (int j = 0; j < FN; ++j) {
        const int n = n0 + wn * WN + j * 32 + frow;
        cin[j] = n < N;
        coff[j] = cin[j] ? map_col(mp, (unsigned)n) : MapPart{0, 0};
    }
#pragma unroll
    for (int i = 0; i < FM; ++i) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int m = m0 + wm * WM + i * 32 + 8 * (r >> 2) + 4 * fk + (r & 3);
            if (m >= M) continue;
            const MapPart roff = map_row(mp, (unsigned)m);
#pragma unroll
            for (int j = 0; j < FN; ++j)
                if (cin[j]) store(map_off(mp, roff, coff[j]), acc[i][j][r]);
        }
    }
}

template <int NPROD, int BM, int BN, int WAVES_M, int WAVES_N, int PF, int ROLE, bool AF32 = false, int NBUF = 2>
static hipError_t run_gemm_p32(const Buf& A, long lda, const Buf& B, long ldb, int M, int N, int K,
                               const Store& st, const OutMap& mp, hipStream_t stream)
{
    const int tiles_m = (M + BM - 1) / BM;
    const int tiles_n = (N + BN - 1) / BN;
    const long tiles = (long)tiles_m * tiles_n;
    const int per_xcd = (int)((tiles + 7) / 8);
    const long grid = 8L * per_xcd;
    if (grid > 0x7fffffffL) return hipErrorInvalidValue;
    const bool vec = (AF32 ? lda % 4 == 0 : lda % 8 == 0 && (long)A.plane % 8 == 0) && ldb % 8 == 0 &&
                     (long)B.plane % 8 == 0 && ((uintptr_t)A.ptr & 15) == 0 && ((uintptr_t)B.ptr & 15) == 0;
    hipLaunchKernelGGL((gemm_nt_bf16p32_kernel<NPROD, BM, BN, WAVES_M, WAVES_N, PF, ROLE, AF32, NBUF>), dim3((unsigned)grid),
                       dim3(64 * WAVES_M * WAVES_N), 0, stream, static_cast<const __bf16*>(A.ptr), lda, (long)A.plane,
                       static_cast<const __bf16*>(B.ptr), ldb, (long)B.plane, M, N, K, st, mp, tiles_m, tiles_n,
                       per_xcd, vec ? 1 : 0);
    return hipGetLastError();
}

// Same product with the operand tiles moved by the load unit straight into
// LDS (global_load_lds_dwordx4: no staging registers, no ds_write), three K
// stages in flight.  Each 16-byte load instruction of a wave fills one
// contiguous KiB of LDS, 32 tile rows of 32 bytes (two 8-element k chunks);
// which global chunk a lane fetches is XOR-swizzled by the row so that the
// 32x32x16 fragment reads (32 rows, one chunk each) hit distinct banks.
// Stage s of K step kt is one of three separate LDS arrays (kt mod 3), so
// that the compiler can tell a fragment read of one stage from the loads in
// flight into another and need not wait for those.
//
// Per K step: wait until this wave's loads of step kt have landed (those of
// kt + 1 stay in flight), barrier (every wave's part of stage kt is in LDS,
// and every wave has finished reading stage kt - 1), issue the loads of
// step kt + 2 into the stage of kt - 1, multiply stage kt.
//
// Needs K a multiple of 16 and 16-byte aligned rows and planes; rows past M
// or N are clamped to the last row (their results are never stored).
__device__ __forceinline__ int lds_swz(int r) { return ((r >> 2) ^ (r >> 3)) & 1; }

// 16 zero bytes: the source of every lane's load in a padding K step
__device__ __attribute__((aligned(16))) const unsigned int kZeroChunk[4] = {0u, 0u, 0u, 0u};

// gfx9 s_waitcnt: vmcnt[3:0] and [15:14] (six bits), expcnt[6:4], lgkmcnt[11:8]
template <int VM, int LG>
__device__ __forceinline__ void wait_vmem_lds_le() {
    static_assert(VM >= 0 && VM < 64 && LG >= 0 && LG < 16, "vmcnt / lgkmcnt immediates");
    __builtin_amdgcn_s_waitcnt((VM & 15) | ((VM >> 4) << 14) | (7 << 4) | (LG << 8));
}

// at most N vector-memory operations of this wave in flight, and no LDS ones
template <int N>
__device__ __forceinline__ void wait_vmem_le() { wait_vmem_lds_le<N, 0>(); }

__device__ __forceinline__ void stage_barrier() {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

// One 32x32x16 product on the matrix cores, BF16 or FP16 operands (the
// operand vectors are 8 two-byte values either way; F16 reinterprets them).
template <bool F16>
__device__ __forceinline__ void mfma_32x32x16(const bf16x8& a, const bf16x8& b,
                                              float __attribute__((ext_vector_type(16)))& acc) {
    if constexpr (F16)
        acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, a), __builtin_bit_cast(f16x8, b), acc,
                                                     0, 0, 0);
    else
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
}

// F16: the operand planes are FP16 (hi, lo of the value times a power of two;
// NPROD 3: hi*hi + hi*lo + lo*hi) instead of BF16.
template <int NPROD, int BM, int BN, int WAVES_M, int WAVES_N, int ROLE, bool PA, bool PB, int NST, int MINW,
          bool F16 = false>
__global__ __launch_bounds__(64 * WAVES_M * WAVES_N, MINW)
void gemm_nt_bf16dma_kernel(const __bf16* __restrict__ A, long lda, long a_plane,
                            const __bf16* __restrict__ B, long ldb, long b_plane,
                            int M, int N, int K, Store store, OutMap mp,
                            int tiles_m, int tiles_n, int per_xcd, int ngrp, int vec_out)
{
    using SP = SplitProducts<NPROD>;
    typedef float f16v __attribute__((ext_vector_type(16)));
    typedef __attribute__((address_space(3))) void lds_void;
    constexpr int NPL = SP::planes;
    constexpr int BK = 16;
    constexpr int NW = WAVES_M * WAVES_N;
    constexpr int WM = BM / WAVES_M;
    constexpr int WN = BN / WAVES_N;
    constexpr int FM = WM / 32;
    constexpr int FN = WN / 32;
    constexpr int A_BLK = BM / 32;                 // 32-row blocks: one wave load per plane
    constexpr int B_BLK = BN / 32;
    constexpr int NLOAD = NPL * (A_BLK + B_BLK);   // wave loads per K step
    constexpr int LPW = NLOAD / NW;                // per wave
    constexpr int A_EL = BM * BK;                  // elements of one plane of the A tile
    constexpr int B_EL = BN * BK;
    constexpr int STAGE = NPL * (A_EL + B_EL);
    static_assert(WM % 32 == 0 && WN % 32 == 0, "wave tile must be whole 32x32 fragments");
    static_assert(NLOAD % NW == 0, "tile loads must divide evenly over the waves");

    static_assert(NST == 2 || NST == 3, "two or three K stages in LDS");
    __shared__ __attribute__((aligned(1024))) __bf16 S0[STAGE];
    __shared__ __attribute__((aligned(1024))) __bf16 S1[STAGE];
    __shared__ __attribute__((aligned(1024))) __bf16 S2[NST == 3 ? STAGE : 8];
    // the stage arrays double as per-wave staging regions of the epilogues
    auto stage_at = [&](int i) -> __bf16* { return i == 0 ? S0 : (i == 1 ? S1 : S2); };

    const int bid = blockIdx.x;
    const int tile = (bid & 7) * per_xcd + (bid >> 3);
    if (tile >= tiles_m * tiles_n) return;
    const int tm = tile / tiles_n;
    const int tn = tile - tm * tiles_n;
    const int m0 = tm * BM;
    const int n0 = tn * BN;

    // Column order of the tile.  ngrp == 0: columns n0 .. n0 + BN - 1.
    // ngrp > 0 (N = G ngrp columns n = g ngrp + h): the tile takes BN / 16
    // consecutive g times 16 consecutive h, local column 16 (g - g0) +
    // (h - h0), so that an output map whose panel row follows g and whose
    // panel column follows h writes runs of BN / 16 whole panel rows.
    auto ncol = [&](int nl) -> int {
        if (ngrp == 0) return n0 + nl;
        const int hb = ngrp >> 4;
        const int g = (tn / hb) * (BN / 16) + (nl >> 4);
        const int h = (tn - (tn / hb) * hb) * 16 + (nl & 15);
        return g * ngrp + h;
    };

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave / WAVES_N;
    const int wn = wave - wm * WAVES_N;

    // this wave's loads of one K step: per load j, this lane's source row
    // start (with its swizzled k chunk) and the LDS offset of the KiB it fills
    const int lrow = lane >> 1;
    // An operand in the panel layout (PA, PB: 32 x 16 panels, rows a
    // multiple of 32, row length lda / ldb >= K, the operand starting at a
    // 16-column boundary of it) gives each wave load one contiguous KiB
    // (32 cache lines per KiB become 8); the K step then advances by a panel.
    const __bf16* gsrc[LPW];
    int dsto[LPW];
    int kmul[LPW];
#pragma unroll
    for (int j = 0; j < LPW; ++j) {
        const int idx = wave + j * NW;
        const bool isA = idx < NPL * A_BLK;
        const int li = isA ? idx : idx - NPL * A_BLK;
        const int blocks = isA ? A_BLK : B_BLK;
        const int pl = li / blocks;
        const int rb = li - pl * blocks;
        const int rloc = rb * 32 + lrow;
        const int c = (lane & 1) ^ lds_swz(rloc);
        const bool panel = isA ? PA : PB;
        if (panel) {
            const int last = ((isA ? M : N) + 31) / 32 - 1;
            const int blk = min(((isA ? m0 : n0) >> 5) + rb, last);
            gsrc[j] = (isA ? A + pl * a_plane : B + pl * b_plane) + (long)blk * ((isA ? lda : ldb) >> 4) * 512 +
                      lrow * 16 + 8 * c;
            kmul[j] = 32;   // panel (k / 16) starts at 512 (k / 16) elements
        } else {
            const int row = isA ? min(m0 + rloc, M - 1) : min(ncol(rloc), N - 1);
            gsrc[j] = (isA ? A + pl * a_plane + (long)row * lda : B + pl * b_plane + (long)row * ldb) + 8 * c;
            kmul[j] = 1;
        }
        dsto[j] = (isA ? pl * A_EL : NPL * A_EL + pl * B_EL) + rb * 32 * BK;
    }
    // padding K steps (past K) load zeros: every lane reads the same 16 bytes.
    // The address is chosen by a select, not a branch: control flow around
    // the LDS-DMA loads makes the compiler's wait insertion fall back to
    // waiting for every load in flight before the next LDS read.
    const uintptr_t zsrc = reinterpret_cast<uintptr_t>(kZeroChunk);
    auto issue = [&](__bf16* S, int k0) {
        const bool pad = k0 >= K;
#pragma unroll
        for (int j = 0; j < LPW; ++j) {
            const uintptr_t a = reinterpret_cast<uintptr_t>(gsrc[j] + (long)kmul[j] * k0);
            const __bf16* g = reinterpret_cast<const __bf16*>(pad ? zsrc : a);
            __builtin_amdgcn_global_load_lds(g, (lds_void*)(S + dsto[j]), 16, 0, 0);
        }
    };

    f16v acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

    const int frow = lane & 31;
    const int fk = lane >> 5;
    auto compute = [&](const __bf16* S) {
        bf16x8 a[NPL][FM], b[NPL][FN];
#pragma unroll
        for (int pl = 0; pl < NPL; ++pl) {
#pragma unroll
            for (int i = 0; i < FM; ++i) {
                const int r = wm * WM + i * 32 + frow;
                a[pl][i] = *reinterpret_cast<const bf16x8*>(S + pl * A_EL + (2 * r + (fk ^ lds_swz(r))) * 8);
            }
#pragma unroll
            for (int j = 0; j < FN; ++j) {
                const int r = wn * WN + j * 32 + frow;
                b[pl][j] = *reinterpret_cast<const bf16x8*>(S + NPL * A_EL + pl * B_EL + (2 * r + (fk ^ lds_swz(r))) * 8);
            }
        }
#pragma unroll
        for (int pr = NPROD - 1; pr >= 0; --pr)   // smallest products first
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j) mfma_32x32x16<F16>(a[SP::a(pr)][i], b[SP::b(pr)][j], acc[i][j]);
    };

    // K steps padded to a multiple of NST (the padding steps load zeros), so
    // the loop body is branch-free: every step waits for the same count and
    // issues the loads NST - 1 steps ahead
    const int nk = (K / BK + NST - 1) / NST * NST;
    auto step = [&](const __bf16* cur, __bf16* ahead, int kt) {
        wait_vmem_le<(NST - 2) * LPW>();
        stage_barrier();
        issue(ahead, (kt + NST - 1) * BK);
        compute(cur);
    };
    issue(S0, 0);
    if constexpr (NST == 3) {
        issue(S1, BK);
        for (int kt = 0; kt < nk; kt += 3) {
            step(S0, S2, kt);
            step(S1, S0, kt + 1);
            step(S2, S1, kt + 2);
        }
    } else {
        for (int kt = 0; kt < nk; kt += 2) {
            step(S0, S1, kt);
            step(S1, S0, kt + 1);
        }
    }
    wait_vmem_le<0>();   // the last stages' loads must land before the workgroup's LDS is released

    // BF16-plane outputs whose map keeps runs of 8 columns contiguous and
    // 16-byte aligned (checked on the host): stage 16-row slabs of all planes
    // in LDS and write them back as 16-byte stores instead of one 2-byte
    // store per element and plane.  The K stages serve as staging space, one
    // private region per wave.
    constexpr int RW = WN + 8;                     // staged row, bf16 (a 16-byte multiple)
    constexpr int SLAB = 16 * RW;                  // one plane of a 16-row slab
    constexpr int REG = NPL * SLAB;                // one wave's region
    constexpr int PER_ARRAY = STAGE / REG;
    if constexpr (PER_ARRAY > 0 && NW <= PER_ARRAY * NST) {
        if (vec_out == 1) {
            typedef unsigned int u4 __attribute__((ext_vector_type(4)));
            constexpr int CPR = WN / 8;            // 16-byte chunks per staged row
            constexpr int NCH = 16 * CPR;          // chunks per plane of a slab
            static_assert(NCH % 64 == 0, "whole chunks per lane");
            constexpr int CPL = NCH / 64;          // chunks per lane
            __syncthreads();   // every wave is done reading the stages
            const int ar = wave / PER_ARRAY;
            __bf16* reg = stage_at(ar) + (wave - ar * PER_ARRAY) * REG;
            __bf16* outp = static_cast<__bf16*>(store.ptr);
            const long pstride = (long)store.plane;
            // this lane's chunks: staged row and column, output column part
            MapPart ccol[CPL];
            bool cok[CPL];
#pragma unroll
            for (int t = 0; t < CPL; ++t) {
                const int c = lane + 64 * t;
                const int n = ncol(wn * WN + (c % CPR) * 8);
                cok[t] = n < N;
                ccol[t] = cok[t] ? map_col(mp, (unsigned)n) : MapPart{0, 0};
            }
#pragma unroll
            for (int i = 0; i < FM; ++i) {
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    // fragment rows 16h .. 16h + 15 are components 8h .. 8h + 7
#pragma unroll
                    for (int j = 0; j < FN; ++j)
#pragma unroll
                        for (int rr = 0; rr < 8; ++rr) {
                            const int r = 8 * h + rr;
                            const int row = 8 * (rr >> 2) + 4 * fk + (rr & 3);
                            // the same split as split_store: hi, mid, lo by round-to-nearest-even
                            const float f = (float)(store.alpha * (double)acc[i][j][r]);
                            const __bf16 hi = (__bf16)f;
                            const float rem = f - (float)hi;
                            const __bf16 md = (__bf16)rem;
                            __bf16* dst = reg + row * RW + j * 32 + frow;
                            dst[0] = hi;
                            dst[SLAB] = md;
                            if constexpr (NPL == 3) dst[2 * SLAB] = (__bf16)(rem - (float)md);
                        }
                    __builtin_amdgcn_s_waitcnt(0xC07F);   // lgkmcnt(0): this wave's staging writes are done
#pragma unroll
                    for (int t = 0; t < CPL; ++t) {
                        const int c = lane + 64 * t;
                        const int row = c / CPR;
                        const int m = m0 + wm * WM + i * 32 + 16 * h + row;
                        if (cok[t] && m < M) {
                            const long off = map_off(mp, map_row(mp, (unsigned)m), ccol[t]);
                            const __bf16* src = reg + row * RW + (c % CPR) * 8;
#pragma unroll
                            for (int pl = 0; pl < NPL; ++pl)
                                *reinterpret_cast<u4*>(outp + pl * pstride + off) =
                                    *reinterpret_cast<const u4*>(src + pl * SLAB);
                        }
                    }
                    __builtin_amdgcn_s_waitcnt(0xC07F);   // staging reads are done before the region is rewritten
                }
            }
            return;
        }
    }
    // FP16-plane outputs (F16x2: hi, lo of alpha * acc, the scale being part
    // of alpha), from BF16 or FP16 operands: the same 16-row slab staging as
    // above with two 2-byte planes.
    constexpr int REG3 = 2 * SLAB;
    constexpr int PER_ARRAY3 = STAGE / REG3;
    if constexpr (PER_ARRAY3 > 0 && NW <= PER_ARRAY3 * NST) {
        if (vec_out == 3) {
            typedef unsigned int u4 __attribute__((ext_vector_type(4)));
            constexpr int CPR = WN / 8;
            constexpr int NCH = 16 * CPR;
            static_assert(NCH % 64 == 0, "whole chunks per lane");
            constexpr int CPL = NCH / 64;
            __syncthreads();   // every wave is done reading the stages
            const int ar = wave / PER_ARRAY3;
            _Float16* reg = reinterpret_cast<_Float16*>(stage_at(ar)) +
                            (wave - ar * PER_ARRAY3) * REG3;
            _Float16* outp = static_cast<_Float16*>(store.ptr);
            const long pstride = (long)store.plane;
            MapPart ccol[CPL];
            bool cok[CPL];
#pragma unroll
            for (int t = 0; t < CPL; ++t) {
                const int c = lane + 64 * t;
                const int n = ncol(wn * WN + (c % CPR) * 8);
                cok[t] = n < N;
                ccol[t] = cok[t] ? map_col(mp, (unsigned)n) : MapPart{0, 0};
            }
#pragma unroll
            for (int i = 0; i < FM; ++i) {
#pragma unroll
                for (int h = 0; h < 2; ++h) {
#pragma unroll
                    for (int j = 0; j < FN; ++j)
#pragma unroll
                        for (int rr = 0; rr < 8; ++rr) {
                            const int r = 8 * h + rr;
                            const int row = 8 * (rr >> 2) + 4 * fk + (rr & 3);
                            _Float16* dst = reg + row * RW + j * 32 + frow;
                            f16_split((float)(store.alpha * (double)acc[i][j][r]), dst, dst + SLAB);
                        }
                    __builtin_amdgcn_s_waitcnt(0xC07F);   // lgkmcnt(0): this wave's staging writes are done
#pragma unroll
                    for (int t = 0; t < CPL; ++t) {
                        const int c = lane + 64 * t;
                        const int row = c / CPR;
                        const int m = m0 + wm * WM + i * 32 + 16 * h + row;
                        if (cok[t] && m < M) {
                            const long off = map_off(mp, map_row(mp, (unsigned)m), ccol[t]);
                            const _Float16* src = reg + row * RW + (c % CPR) * 8;
#pragma unroll
                            for (int pl = 0; pl < 2; ++pl)
                                *reinterpret_cast<u4*>(outp + pl * pstride + off) =
                                    *reinterpret_cast<const u4*>(src + pl * SLAB);
                        }
                    }
                    __builtin_amdgcn_s_waitcnt(0xC07F);   // staging reads are done before the region is rewritten
                }
            }
            return;
        }
    }
    // FP32 outputs (a product whose consumer splits its operand on load):
    // the same 16-row slab staging with one 4-byte plane, 16-byte stores of
    // 4 columns.  The value stored is the one the plane split above starts
    // from, so a consumer that splits it gets the same planes.
    constexpr int RW4 = WN + 4;                    // staged row, floats (a 16-byte multiple)
    constexpr int SLAB4 = 16 * RW4;                // floats of a 16-row slab
    constexpr int PER_ARRAY4 = STAGE / (2 * SLAB4);
    if constexpr (PER_ARRAY4 > 0 && NW <= PER_ARRAY4 * NST) {
        if (vec_out == 2) {
            typedef unsigned int u4 __attribute__((ext_vector_type(4)));
            constexpr int CPR = WN / 4;            // 16-byte chunks per staged row
            constexpr int NCH = 16 * CPR;
            static_assert(NCH % 64 == 0, "whole chunks per lane");
            constexpr int CPL = NCH / 64;
            __syncthreads();   // every wave is done reading the stages
            const int ar = wave / PER_ARRAY4;
            float* reg = reinterpret_cast<float*>(stage_at(ar)) + (wave - ar * PER_ARRAY4) * SLAB4;
            float* outp = static_cast<float*>(store.ptr);
            MapPart ccol[CPL];
            bool cok[CPL];
#pragma unroll
            for (int t = 0; t < CPL; ++t) {
                const int c = lane + 64 * t;
                const int n = ncol(wn * WN + (c % CPR) * 4);
                cok[t] = n < N;
                ccol[t] = cok[t] ? map_col(mp, (unsigned)n) : MapPart{0, 0};
            }
#pragma unroll
            for (int i = 0; i < FM; ++i) {
#pragma unroll
                for (int h = 0; h < 2; ++h) {
#pragma unroll
                    for (int j = 0; j < FN; ++j)
#pragma unroll
                        for (int rr = 0; rr < 8; ++rr) {
                            const int r = 8 * h + rr;
                            const int row = 8 * (rr >> 2) + 4 * fk + (rr & 3);
                            reg[row * RW4 + j * 32 + frow] = (float)(store.alpha * (double)acc[i][j][r]);
                        }
                    __builtin_amdgcn_s_waitcnt(0xC07F);   // lgkmcnt(0): this wave's staging writes are done
#pragma unroll
                    for (int t = 0; t < CPL; ++t) {
                        const int c = lane + 64 * t;
                        const int row = c / CPR;
                        const int m = m0 + wm * WM + i * 32 + 16 * h + row;
                        if (cok[t] && m < M) {
                            const long off = map_off(mp, map_row(mp, (unsigned)m), ccol[t]);
                            *reinterpret_cast<u4*>(outp + off) =
                                *reinterpret_cast<const u4*>(reg + row * RW4 + (c % CPR) * 4);
                        }
                    }
                    __builtin_amdgcn_s_waitcnt(0xC07F);   // staging reads are done before the region is rewritten
                }
            }
            return;
        }
        // Any other output (element stores through the map, in any format):
        // through the same FP32 slabs, so the accumulators are only ever
        // indexed with constants.  (Indexing them by a loop counter that the
        // compiler keeps as a loop puts the whole accumulator array in scratch
        // memory: zeroed at the start and stored after the K loop in every
        // launch, whatever the output path, 2 x 512 bytes per lane.)  A lane
        // stores columns lane, lane + 64, ... of each slab row.
        constexpr int CPLG = (WN + 63) / 64;
        __syncthreads();   // every wave is done reading the stages
        const int ar = wave / PER_ARRAY4;
        float* reg = reinterpret_cast<float*>(stage_at(ar)) + (wave - ar * PER_ARRAY4) * SLAB4;
        MapPart gcol[CPLG];
        bool gok[CPLG];
#pragma unroll
        for (int t = 0; t < CPLG; ++t) {
            const int c = lane + 64 * t;
            const int n = c < WN ? ncol(wn * WN + c) : N;
            gok[t] = n < N;
            gcol[t] = gok[t] ? map_col(mp, (unsigned)n) : MapPart{0, 0};
        }
#pragma unroll
        for (int i = 0; i < FM; ++i) {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
#pragma unroll
                for (int j = 0; j < FN; ++j)
#pragma unroll
                    for (int rr = 0; rr < 8; ++rr) {
                        const int row = 8 * (rr >> 2) + 4 * fk + (rr & 3);
                        reg[row * RW4 + j * 32 + frow] = acc[i][j][8 * h + rr];
                    }
                __builtin_amdgcn_s_waitcnt(0xC07F);   // lgkmcnt(0): this wave's staging writes are done
                for (int row = 0; row < 16; ++row) {
                    const int m = m0 + wm * WM + i * 32 + 16 * h + row;
                    if (m >= M) break;
                    const MapPart roff = map_row(mp, (unsigned)m);
#pragma unroll
                    for (int t = 0; t < CPLG; ++t)
                        if (gok[t]) store(map_off(mp, roff, gcol[t]), reg[row * RW4 + lane + 64 * t]);
                }
                __builtin_amdgcn_s_waitcnt(0xC07F);   // staging reads are done before the region is rewritten
            }
        }
        return;
    }

    MapPart coff[FN];
    bool cin[FN];
#pragma unroll
    for (int j = 0; j < FN; ++j) {
        const int n = ncol(wn * WN + j * 32 + frow);
        cin[j] = n < N;
        coff[j] = cin[j] ? map_col(mp, (unsigned)n) : MapPart{0, 0};
    }
#pragma unroll
    for (int i = 0; i < FM; ++i) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int m = m0 + wm * WM + i * 32 + 8 * (r >> 2) + 4 * fk + (r & 3);
            if (m >= M) continue;
            const MapPart roff = map_row(mp, (unsigned)m);
#pragma unroll
            for (int j = 0; j < FN; ++j)
                if (cin[j]) store(map_off(mp, roff, coff[j]), acc[i][j][r]);
        }
    }
}

template <int NPROD, int BM, int BN, int WAVES_M, int WAVES_N, int ROLE, bool PA = false, bool PB = false, int NST = 3,
          int MINW = 1, bool F16 = false>
static hipError_t run_gemm_dma(const Buf& A, long lda, const Buf& B, long ldb, int M, int N, int K,
                               const Store& st, const OutMap& mp, hipStream_t stream, int ngrp = 0)
{
    if (ngrp && (BN % 16 || ngrp % 16 || N % ngrp || (N / ngrp) % (BN / 16))) return hipErrorInvalidValue;
    // 16-byte staged stores need the output in the planes of the operands'
    // split format and runs of 8 output columns that stay contiguous and
    // 16-byte aligned under the output map
    const bool same_planes = st.fmt == (int)A.fmt;
    const bool rm_ok = mp.panel_k == 0 && mp.cs_lo == 1 && mp.rs_hi % 8 == 0 && mp.rs_lo % 8 == 0 &&
                       mp.cs_hi % 8 == 0;
    const bool pn_ok = mp.panel_k != 0 && mp.panel_k % 16 == 0 && mp.cc_lo == 1 && mp.rc_hi % 8 == 0 &&
                       mp.rc_lo % 8 == 0 && mp.cc_hi % 8 == 0;
    int vec_out = same_planes && (rm_ok || pn_ok) && mp.sn % 8 == 0 && N % 8 == 0 && st.plane % 8 == 0 &&
                  ((uintptr_t)st.ptr & 15) == 0;
    // FP32 output: runs of 4 columns contiguous and 16-byte aligned (row-major maps)
    if (!vec_out && st.fmt == (int)Fmt::F32 && mp.panel_k == 0 && mp.cs_lo == 1 && mp.rs_hi % 4 == 0 &&
        mp.rs_lo % 4 == 0 && mp.cs_hi % 4 == 0 && mp.sn % 4 == 0 && N % 4 == 0 && ((uintptr_t)st.ptr & 15) == 0)
        vec_out = 2;
    if (F16 && vec_out == 1) vec_out = 0;   // the BF16-plane staging does not apply to FP16 operands
    // FP16-plane outputs (the X product feeding an FP16 Y, the half
    // environments feeding an FP16 E)
    if (!vec_out && st.fmt == (int)Fmt::F16x2 && (rm_ok || pn_ok) && mp.sn % 8 == 0 && N % 8 == 0 &&
        st.plane % 8 == 0 && ((uintptr_t)st.ptr & 15) == 0)
        vec_out = 3;
    const int tiles_m = (M + BM - 1) / BM;
    const int tiles_n = (N + BN - 1) / BN;
    const long tiles = (long)tiles_m * tiles_n;
    const int per_xcd = (int)((tiles + 7) / 8);
    const long grid = 8L * per_xcd;
    if (grid > 0x7fffffffL) return hipErrorInvalidValue;
    hipLaunchKernelGGL((gemm_nt_bf16dma_kernel<NPROD, BM, BN, WAVES_M, WAVES_N, ROLE, PA, PB, NST, MINW, F16>),
                       dim3((unsigned)grid),
                       dim3(64 * WAVES_M * WAVES_N), 0, stream, static_cast<const __bf16*>(A.ptr), lda, (long)A.plane,
                       static_cast<const __bf16*>(B.ptr), ldb, (long)B.plane, M, N, K, st, mp, tiles_m, tiles_n,
                       per_xcd, ngrp, vec_out);
    return hipGetLastError();
}

// ---------------------------------------------------------------- launcher

template <typename T, int BM, int BN, int BK, int WAVES_M, int WAVES_N, int ROLE>
static hipError_t run_gemm(const T* A, long lda, const T* B, long ldb, int M, int N, int K,
                           const Store& st, const OutMap& mp, hipStream_t stream)
{
    const int tiles_m = (M + BM - 1) / BM;
    const int tiles_n = (N + BN - 1) / BN;
    const long tiles = (long)tiles_m * tiles_n;
    const int per_xcd = (int)((tiles + 7) / 8);
    const long grid = 8L * per_xcd;
    if (grid > 0x7fffffffL) return hipErrorInvalidValue;
    hipLaunchKernelGGL((gemm_nt_kernel<T, BM, BN, BK, WAVES_M, WAVES_N, ROLE>), dim3((unsigned)grid),
                       dim3(64 * WAVES_M * WAVES_N), 0, stream,
                       A, lda, B, ldb, M, N, K, st, mp, tiles_m, tiles_n, per_xcd);
    return hipGetLastError();
}

template <int ROLE>
static hipError_t dispatch(const Buf& A, long lda, const Buf& B, long ldb, int M, int N, int K,
                           const Store& st, const OutMap& map, int products, hipStream_t stream)
{
    (void)products;
    if (A.fmt == Fmt::F16x2 || B.fmt == Fmt::F16x2) {
        // FP16 two-plane operands, hi*hi + hi*lo + lo*hi: the Y product at
        // full size (panel operands, 256 x 256 tiles) and the environment
        // products (panel operands, mid-size tiles)
        const bool f16_panels = A.fmt == Fmt::F16x2 && B.fmt == Fmt::F16x2 && A.panel_k && B.panel_k && K >= 16 &&
                                K % 16 == 0 && A.panel_k == lda && B.panel_k == ldb && K <= lda && K <= ldb &&
                                lda % 16 == 0 && ldb % 16 == 0 && M % 32 == 0 && N % 32 == 0 && N > 64 &&
                                (long)A.plane % 8 == 0 && (long)B.plane % 8 == 0 && ((uintptr_t)A.ptr & 15) == 0 &&
                                ((uintptr_t)B.ptr & 15) == 0;
        if constexpr (ROLE == 0) {
            if (!f16_panels) return hipErrorInvalidValue;
            // fewer 128 x 128 tiles than two per CU (D = 48: 324 of them)
            // leave the CUs unevenly loaded; 64 x 128 tiles on four waves
            // took the environment stage of a D = 48 step from 0.443 to
            // 0.387 ms (D = 32: 0.161 -> 0.123), and were slower where the
            // 128 x 128 grid already fills the chip (D = 64: 1.14 -> 1.59)
            if ((long)((M + 127) / 128) * ((N + 127) / 128) < 512)
                return run_gemm_dma<3, 64, 128, 2, 2, ROLE, true, true, kMidNst, kMidMinw, true>(A, lda, B, ldb, M,
                                                                                                  N, K, st, map,
                                                                                                  stream);
            return run_gemm_dma<3, 128, 128, 2, 2, ROLE, true, true, kMidNst, kMidMinw, true>(A, lda, B, ldb, M, N,
                                                                                               K, st, map, stream);
        } else if constexpr (ROLE == 2) {
            if (!f16_panels || (long)((M + 255) / 256) * ((N + 255) / 256) < 512) return hipErrorInvalidValue;
            return run_gemm_dma<3, kYBM, kYBN, kYWM, kYWN, ROLE, true, true, kYNst,
                                kYMinw, true>(A, lda, B, ldb, M, N, K, st, map, stream, (int)map.ngroup);
        } else {
            return hipErrorInvalidValue;
        }
    }
    const bool split = A.fmt == Fmt::BF16x2 || A.fmt == Fmt::BF16x3;
    if (A.fmt == Fmt::F32 && (B.fmt == Fmt::BF16x2 || B.fmt == Fmt::BF16x3)) {
        // T' = Y . U with Y kept in FP32 by its producer: the A tile is split
        // into the planes of B's format as it is written to LDS
        if (A.panel_k || B.panel_k) return hipErrorInvalidValue;
        return B.fmt == Fmt::BF16x2
                   ? run_gemm_p32<3, kTpBM, 64, kTpWM, 1, kTpPF, ROLE, true, kTpNbuf>(A, lda, B, ldb, M, N, K, st,
                                                                                              map, stream)
                   : run_gemm_p32<6, kTpBM, 64, kTpWM, 1, kTpPF, ROLE, true, kTpNbuf>(A, lda, B, ldb, M, N, K, st,
                                                                                              map, stream);
    }
    if (A.panel_k || B.panel_k) {
        // panel-layout operands (row length lda / ldb >= K, whole 32-row
        // panels) go to the direct-to-LDS kernel: both operands of the
        // environment products and of Y, the A operand (Y itself) of T'
        const bool base = split && K >= 16 && K % 16 == 0 && (long)A.plane % 8 == 0 && (long)B.plane % 8 == 0 &&
                          ((uintptr_t)A.ptr & 15) == 0 && ((uintptr_t)B.ptr & 15) == 0 &&
                          (!A.panel_k || (A.panel_k == lda && K <= lda && lda % 16 == 0 && M % 32 == 0)) &&
                          (!B.panel_k || (B.panel_k == ldb && K <= ldb && ldb % 16 == 0 && N % 32 == 0));
        const bool both = base && A.panel_k && B.panel_k && N > 64;
        if constexpr (ROLE == 0) {
            // half environments and E (N = K = D^2): mid-size tiles (64 x 128
            // as in the FP16 form measured slower here: 0.591 -> 0.627 ms for
            // the environment stage of a D = 48 BF16x6 step)
            if (!both) return hipErrorInvalidValue;
            return A.fmt == Fmt::BF16x2
                       ? run_gemm_dma<3, 128, 128, 2, 2, ROLE, true, true, kMidNst, kMidMinw>(
                             A, lda, B, ldb, M, N, K, st, map, stream)
                       : run_gemm_dma<6, 128, 128, 2, 2, ROLE, true, true, kMidNst, kMidMinw>(
                             A, lda, B, ldb, M, N, K, st, map, stream);
        } else if constexpr (ROLE == 2) {
            if (!both) return hipErrorInvalidValue;
            const long big_tiles = (long)((M + 255) / 256) * ((N + 255) / 256);
            if (A.fmt == Fmt::BF16x2)
                return big_tiles < 512
                           ? run_gemm_dma<3, 128, 128, 2, 2, ROLE, true, true>(A, lda, B, ldb, M, N, K, st, map, stream)
                           : run_gemm_dma<3, kYBM, kYBN, kYWM, kYWN, ROLE, true, true,
                                          kYNst, kYMinw>(A, lda, B, ldb, M, N, K, st, map, stream,
                                                                     (int)map.ngroup);
            return big_tiles < 512
                       ? run_gemm_dma<6, 128, 128, 2, 2, ROLE, true, true>(A, lda, B, ldb, M, N, K, st, map, stream)
                       : run_gemm_dma<6, kYBM, kYBN, kYWM, kYWN, ROLE, true, true, kYNst,
                                      kYMinw>(A, lda, B, ldb, M, N, K, st, map, stream, (int)map.ngroup);
        } else if constexpr (ROLE == 3) {
            // T' = Y . U: Y in panels, U row-major, narrow output
            if (!(base && A.panel_k && !B.panel_k && N <= 64 && ldb % 8 == 0)) return hipErrorInvalidValue;
            return A.fmt == Fmt::BF16x2
                       ? run_gemm_dma<3, 128, 64, 2, 1, ROLE, true, false, kNarrowNst, kNarrowMinw>(
                             A, lda, B, ldb, M, N, K, st, map, stream)
                       : run_gemm_dma<6, 128, 64, 2, 1, ROLE, true, false, kNarrowNst, kNarrowMinw>(
                             A, lda, B, ldb, M, N, K, st, map, stream);
        } else {
            (void)both;
            return hipErrorInvalidValue;
        }
    }
    if (split) {
        // narrow outputs (T' has N = D') take a 64-wide tile
        const bool narrow = N <= 64;
        const bool dma = K >= 16 && K % 16 == 0 && lda % 8 == 0 && ldb % 8 == 0 && (long)A.plane % 8 == 0 &&
                         (long)B.plane % 8 == 0 && ((uintptr_t)A.ptr & 15) == 0 && ((uintptr_t)B.ptr & 15) == 0;
        if (dma) {
            if constexpr (ROLE == 1) {
                // X = U . T has K = Dx: a few K steps per tile and a D^5 output,
                // so its time is the tile's load latency and its stores; small
                // tiles with two LDS stages let three workgroups share a CU and
                // overlap each other's loads, products and stores (measured
                // 19.2 -> 15.8 ms per D = 48 solve against 256 x 256, one per CU)
                if (!narrow)
                    return A.fmt == Fmt::BF16x2
                               ? run_gemm_dma<3, 128, 128, 2, 2, ROLE, false, false, 2, 3>(A, lda, B, ldb, M, N, K, st,
                                                                                        map, stream, (int)map.ngroup)
                               : run_gemm_dma<6, 128, 128, 2, 2, ROLE, false, false, 2, 3>(A, lda, B, ldb, M, N, K, st,
                                                                                        map, stream, (int)map.ngroup);
            }
            // tile by the work available: 256 x 256 needs at least two rounds
            // of workgroups over the 256 CUs to fill the chip; smaller
            // products (half environments and E, N = K = D^2) take 128 x 128,
            // narrow outputs (T', N = D') 128 x 64
            const long big_tiles = (long)((M + 255) / 256) * ((N + 255) / 256);
            if (A.fmt == Fmt::BF16x2) {
                if (narrow)
                    return run_gemm_dma<3, 128, 64, 2, 1, ROLE, false, false, kNarrowNst, kNarrowMinw>(
                        A, lda, B, ldb, M, N, K, st, map, stream);
                if (big_tiles < 512)
                    return run_gemm_dma<3, 128, 128, 2, 2, ROLE, false, false, kMidNst, kMidMinw>(
                        A, lda, B, ldb, M, N, K, st, map, stream);
                return run_gemm_dma<3, 256, 256, kDmaWM, kDmaWN, ROLE>(A, lda, B, ldb, M, N, K, st, map,
                                                                                  stream, (int)map.ngroup);
            }
            if (narrow)
                return run_gemm_dma<6, 128, 64, 2, 1, ROLE, false, false, kNarrowNst, kNarrowMinw>(
                    A, lda, B, ldb, M, N, K, st, map, stream);
            if (big_tiles < 512)
                return run_gemm_dma<6, 128, 128, 2, 2, ROLE, false, false, kMidNst, kMidMinw>(
                    A, lda, B, ldb, M, N, K, st, map, stream);
            return run_gemm_dma<6, 256, 256, kDmaWM, kDmaWN, ROLE>(A, lda, B, ldb, M, N, K, st, map,
                                                                              stream, (int)map.ngroup);
        }
        if (A.fmt == Fmt::BF16x2)
            return narrow ? run_gemm_p32<3, 256, 64, 4, 1, 1, ROLE>(A, lda, B, ldb, M, N, K, st, map, stream)
                          : run_gemm_p32<3, kP32BM, kP32BN, kP32WM, kP32WN, kP32PF,
                                         ROLE>(A, lda, B, ldb, M, N, K, st, map, stream);
        return narrow ? run_gemm_p32<6, 256, 64, 4, 1, 1, ROLE>(A, lda, B, ldb, M, N, K, st, map, stream)
                      : run_gemm_p32<6, kP32BM, kP32BN, kP32WM, kP32WN, kP32PF,
                                     ROLE>(A, lda, B, ldb, M, N, K, st, map, stream);
    }
    // FP64 / FP32: 64 x 64 tiles for narrow outputs (T', N = D') and where
    // 128 x 128 gives fewer than four tiles per CU (the D = 24 products, the
    // D = 48 environments), so that the work spreads evenly over the CUs
    // (FP64, per steady step: D = 24 environment 0.367 -> 0.136 ms, Y 0.376
    // -> 0.227, X 0.068 -> 0.033, T' 0.123 -> 0.048; D = 48 environment
    // 2.63 -> 1.86 and T' 1.72 -> 0.69; results bitwise unchanged, the K
    // order of every element being the same)
    const bool small_tiles = N <= 64 || (long)((M + 127) / 128) * ((N + 127) / 128) < 1024;
    switch (A.fmt) {
        case Fmt::F64:
            if (small_tiles)
                return run_gemm<double, 64, 64, 16, 2, 2, ROLE>(static_cast<const double*>(A.ptr), lda,
                                                                static_cast<const double*>(B.ptr), ldb,
                                                                M, N, K, st, map, stream);
            // 256 x 128 tiles on 16 waves (64 x 32 each): the steady D = 48
            // Y launch 26.4 -> 20.3 ms against 128 x 128 on 4 waves (2 x 4
            // waves of 64 x 64: 21.0 ms; 256 x 256 spills the accumulators)
            return run_gemm<double, 256, 128, 16, 4, 4, ROLE>(static_cast<const double*>(A.ptr), lda,
                                                              static_cast<const double*>(B.ptr), ldb,
                                                              M, N, K, st, map, stream);
        case Fmt::F32:
            if (small_tiles)
                return run_gemm<float, 64, 64, 32, 2, 2, ROLE>(static_cast<const float*>(A.ptr), lda,
                                                               static_cast<const float*>(B.ptr), ldb,
                                                               M, N, K, st, map, stream);
            // 256 x 128 on 16 waves as for FP64: steady D = 48 Y launch 11.48
            // -> 10.73 ms, X 0.82 -> 0.62 ms against 128 x 128 on 4 waves
            return run_gemm<float, 256, 128, 32, 4, 4, ROLE>(static_cast<const float*>(A.ptr), lda,
                                                             static_cast<const float*>(B.ptr), ldb,
                                                             M, N, K, st, map, stream);
        default:
            return hipErrorNotSupported;
    }
}

hipError_t launch_gemm_nt(const Buf& A, long lda, const Buf& B, long ldb, const Buf& C,
                          int M, int N, int K, double alpha, const OutMap& map,
                          int products, GemmRole role, hipStream_t stream)
{
    if (M <= 0 || N <= 0) return hipSuccess;
    // operands in one format, or an FP32 A split on load into B's BF16 planes
    const bool f32_split = A.fmt == Fmt::F32 && (B.fmt == Fmt::BF16x2 || B.fmt == Fmt::BF16x3);
    if ((A.fmt != B.fmt && !f32_split) || map.sm < 1 || map.sn < 1) return hipErrorInvalidValue;
    Store st{C.ptr, C.plane, (int)C.fmt, alpha};
    switch (role) {
        case GemmRole::X: return dispatch<1>(A, lda, B, ldb, M, N, K, st, map, products, stream);
        case GemmRole::Y: return dispatch<2>(A, lda, B, ldb, M, N, K, st, map, products, stream);
        case GemmRole::TP: return dispatch<3>(A, lda, B, ldb, M, N, K, st, map, products, stream);
        default: return dispatch<0>(A, lda, B, ldb, M, N, K, st, map, products, stream);
    }
}

}  // namespace hotrg
