// Small D^4-sized kernels of a HOTRG step: operand re-layouts of T, the
// max-abs normalisation with ln Z accumulation, the final trace and the
// symmetrisation of E.  None of them is on the D^7 path; they are written
// for coalesced stores and deterministic (order-fixed) reductions.
#include <math.h>
#include "common.h"
#include "../../include/hotrg.h"

namespace hotrg {

// ---------------------------------------------------------------- stores

// store v as element `idx` of the storage of o (after any sub-block or
// panel mapping), in o's format
__device__ __forceinline__ void put_at(const Buf& o, size_t idx, double v) {
    switch (o.fmt) {
        case Fmt::F64: static_cast<double*>(o.ptr)[idx] = v; break;
        case Fmt::F32: static_cast<float*>(o.ptr)[idx] = (float)v; break;
        case Fmt::F16x2: {
            _Float16* p = static_cast<_Float16*>(o.ptr);
            f16_split((float)(v * (double)o.scale), p + idx, p + idx + o.plane);
            break;
        }
        default: {
            __bf16* p = static_cast<__bf16*>(o.ptr);
            const float f = (float)v;
            const __bf16 h = (__bf16)f;
            p[idx] = h;
            const float r = f - (float)h;
            const __bf16 m = (__bf16)r;
            p[idx + o.plane] = m;
            if (o.fmt == Fmt::BF16x3) p[idx + 2 * o.plane] = (__bf16)(r - (float)m);
        }
    }
}

__device__ __forceinline__ void put(const Buf& o, size_t idx, double v) {
    if (o.cols) {
        const long r = (long)(idx / o.cols), c = (long)(idx % o.cols);
        idx = o.panel_k ? (size_t)panel_index(r, c, o.panel_k) : (size_t)(r * o.ld + c);
    } else if (o.panel_k) {
        idx = (size_t)panel_index((long)(idx / o.panel_k), (long)(idx % o.panel_k), o.panel_k);
    }
    put_at(o, idx, v);
}

// the storage index of logical element idx of o, for idx < 2^32 (32-bit
// divisions; the 64-bit ones of put() cost more than the element's store)
__device__ __forceinline__ size_t storage_index32(const Buf& o, unsigned idx) {
    if (o.cols) {
        const unsigned w = (unsigned)o.cols, r = idx / w, c = idx - r * w;
        return o.panel_k ? (size_t)panel_index(r, c, o.panel_k) : (size_t)r * (size_t)o.ld + c;
    }
    if (o.panel_k) {
        const unsigned w = (unsigned)o.panel_k, r = idx / w, c = idx - r * w;
        return (size_t)panel_index(r, c, o.panel_k);
    }
    return idx;
}

// ---------------------------------------------------------------- permute

struct Perm4 {
    int od[4];     // output dims
    long is[4];    // input stride of the input axis feeding each output axis
};

// out[j0, j1, j2, j3] = in[j0 is0 + j1 is1 + j2 is2 + j3 is3]: one thread per
// element, blockIdx.y = (j0, j1), the threads of a row of blocks over
// (j2, j3); every index fits 32 bits (the host checks the element count)
__global__ __launch_bounds__(256) void permute4_kernel(const double* __restrict__ in, Perm4 p, Buf out) {
    const unsigned inner = (unsigned)p.od[2] * (unsigned)p.od[3];
    const unsigned t = blockIdx.x * 256u + threadIdx.x;
    if (t >= inner) return;
    const unsigned y = blockIdx.y;
    const unsigned j0 = y / (unsigned)p.od[1], j1 = y - j0 * (unsigned)p.od[1];
    const unsigned j2 = t / (unsigned)p.od[3], j3 = t - j2 * (unsigned)p.od[3];
    const unsigned src = j0 * (unsigned)p.is[0] + j1 * (unsigned)p.is[1] + j2 * (unsigned)p.is[2] +
                         j3 * (unsigned)p.is[3];
    const unsigned o = y * inner + t;
    put_at(out, storage_index32(out, o), in[src]);
}

// The same re-layout when the output's fastest axis is not the input's
// (perm[3] != 3): a 32 x 32 tile of (input axis 3, input axis perm[3]) goes
// through LDS, read along the input's contiguous axis and written along the
// output's fastest one.  Output axis `a` is fed by input axis 3; `o1`, `o2`
// are the other two output axes (blockIdx.y = (j_o1, j_o2)); blockIdx.x
// enumerates the tiles over (output axis a, output axis 3).
struct PermT {
    int od[4];       // output dims
    unsigned is[4];  // input stride of the input axis feeding each output axis
    unsigned os[4];  // output (logical, row-major) stride of each output axis
    int a, o1, o2;   // output axis fed by input axis 3; the two outer output axes
};

__global__ __launch_bounds__(256) void permute4_tiled_kernel(const double* __restrict__ in, PermT p, Buf out) {
    __shared__ double tile[32][33];
    const unsigned na = (unsigned)p.od[p.a], n3 = (unsigned)p.od[3];
    const unsigned ta = blockIdx.x % ((na + 31) / 32), t3 = blockIdx.x / ((na + 31) / 32);
    const unsigned y = blockIdx.y;
    const unsigned j1 = y / (unsigned)p.od[p.o2], j2 = y - j1 * (unsigned)p.od[p.o2];
    const unsigned base_in = j1 * p.is[p.o1] + j2 * p.is[p.o2];
    const unsigned base_out = j1 * p.os[p.o1] + j2 * p.os[p.o2];
    const unsigned lx = threadIdx.x & 31, ly = threadIdx.x >> 5;   // 32 x 8
    // read: lanes along output axis a (the input's contiguous axis)
    for (unsigned r = ly; r < 32; r += 8) {
        const unsigned ia = ta * 32 + lx, i3 = t3 * 32 + r;
        if (ia < na && i3 < n3) tile[r][lx] = in[base_in + ia * p.is[p.a] + i3 * p.is[3]];
    }
    __syncthreads();
    // write: lanes along output axis 3
    for (unsigned r = ly; r < 32; r += 8) {
        const unsigned ia = ta * 32 + r, i3 = t3 * 32 + lx;
        if (ia < na && i3 < n3) {
            const unsigned o = base_out + ia * p.os[p.a] + i3;
            put_at(out, storage_index32(out, o), tile[lx][r]);
        }
    }
}

hipError_t launch_permute4(const double* in, const int dims[4], const int perm[4],
                           const Buf& out, hipStream_t stream) {
    long st[4];
    st[3] = 1;
    st[2] = dims[3];
    st[1] = (long)dims[2] * dims[3];
    st[0] = (long)dims[1] * dims[2] * dims[3];
    Perm4 p;
    size_t total = 1;
    for (int a = 0; a < 4; ++a) {
        p.od[a] = dims[perm[a]];
        p.is[a] = st[perm[a]];
        total *= (size_t)p.od[a];
    }
    if (total == 0) return hipSuccess;
    const size_t rows = (size_t)p.od[0] * p.od[1], inner = (size_t)p.od[2] * p.od[3];
    if (total >= (1ull << 32) || rows > 65535) return hipErrorInvalidValue;
    if (perm[3] != 3) {
        PermT q;
        for (int a = 0; a < 4; ++a) {
            q.od[a] = p.od[a];
            q.is[a] = (unsigned)p.is[a];
        }
        q.os[3] = 1;
        q.os[2] = (unsigned)q.od[3];
        q.os[1] = q.os[2] * (unsigned)q.od[2];
        q.os[0] = q.os[1] * (unsigned)q.od[1];
        q.a = perm[0] == 3 ? 0 : (perm[1] == 3 ? 1 : 2);
        int k = 0, outer[2];
        for (int a = 0; a < 3; ++a)
            if (a != q.a) outer[k++] = a;
        q.o1 = outer[0];
        q.o2 = outer[1];
        const size_t tiles = (size_t)((q.od[q.a] + 31) / 32) * ((q.od[3] + 31) / 32);
        const size_t ys = (size_t)q.od[q.o1] * q.od[q.o2];
        if (ys > 65535) return hipErrorInvalidValue;
        hipLaunchKernelGGL(permute4_tiled_kernel, dim3((unsigned)tiles, (unsigned)ys), dim3(256), 0, stream, in, q,
                           out);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(permute4_kernel, dim3((unsigned)((inner + 255) / 256), (unsigned)rows), dim3(256), 0, stream,
                       in, p, out);
    return hipGetLastError();
}

__global__ void convert2d_kernel(const double* __restrict__ in, long ld, int rows, int cols, Buf out) {
    const size_t total = (size_t)rows * cols;
    for (size_t o = blockIdx.x * (size_t)blockDim.x + threadIdx.x; o < total; o += (size_t)gridDim.x * blockDim.x) {
        const size_t r = o / cols, c = o - (o / cols) * cols;
        put(out, o, in[r * ld + c]);
    }
}

hipError_t launch_convert2d(const double* in, long ld, int rows, int cols, const Buf& out,
                            hipStream_t stream) {
    const size_t total = (size_t)rows * cols;
    if (total == 0) return hipSuccess;
    size_t blocks = (total + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(convert2d_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, in, ld, rows, cols, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------- reductions

template <int NT>
__device__ double block_max(double v, double* sh) {
    const int tid = threadIdx.x;
    sh[tid] = v;
    __syncthreads();
    for (int s = NT / 2; s > 0; s >>= 1) {
        if (tid < s) sh[tid] = fmax(sh[tid], sh[tid + s]);
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

template <int NT>
__device__ double block_sum(double v, double* sh) {
    const int tid = threadIdx.x;
    sh[tid] = v;
    __syncthreads();
    for (int s = NT / 2; s > 0; s >>= 1) {
        if (tid < s) sh[tid] = sh[tid] + sh[tid + s];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

constexpr int RED_BLOCKS = 1024;  // == size of DevState::partial

__global__ __launch_bounds__(256) void absmax_partial_kernel(const double* __restrict__ T, size_t count, DevState* st) {
    __shared__ double sh[256];
    double m = 0.0;
    for (size_t i = blockIdx.x * (size_t)256 + threadIdx.x; i < count; i += (size_t)gridDim.x * 256)
        m = fmax(m, fabs(T[i]));
    m = block_max<256>(m, sh);
    if (threadIdx.x == 0) st->partial[blockIdx.x] = m;
}

// One block: c_n = max of the partials; latch an error if c_n is not a
// positive finite number; accumulate ln(c_n) / 2^n.  Single-thread stores.
__global__ __launch_bounds__(256) void norm_finalize_kernel(DevState* st, int nblocks, int n) {
    __shared__ double sh[256];
    double m = 0.0;
    for (int i = threadIdx.x; i < nblocks; i += 256) m = fmax(m, st->partial[i]);
    m = block_max<256>(m, sh);
    if (threadIdx.x == 0) {
        const bool ok = (m > 0.0) && isfinite(m);
        if (!ok && st->status == 0) st->status = HOTRG_ENONFINITE;
        st->c_cur = ok ? m : 1.0;
        if (n < 64) st->c[n] = m;
        if (ok) st->lnz_acc += log(m) * ldexp(1.0, -n);
    }
}

__global__ __launch_bounds__(256) void scale_kernel(double* __restrict__ T, size_t count, const DevState* st) {
    const double c = st->c_cur;
    for (size_t i = blockIdx.x * (size_t)256 + threadIdx.x; i < count; i += (size_t)gridDim.x * 256)
        T[i] = T[i] / c;
}

__global__ __launch_bounds__(256) void scale_norm_kernel(double* __restrict__ I, size_t count, const DevState* st,
                                                        double factor) {
    const double f = factor / st->c_cur;
    for (size_t i = blockIdx.x * (size_t)256 + threadIdx.x; i < count; i += (size_t)gridDim.x * 256)
        I[i] = I[i] * f;
}

hipError_t launch_scale_by_norm(double* I, size_t count, const DevState* st, double factor, hipStream_t stream) {
    size_t sb = (count + 255) / 256;
    if (sb > 8192) sb = 8192;
    if (sb < 1) sb = 1;
    hipLaunchKernelGGL(scale_norm_kernel, dim3((unsigned)sb), dim3(256), 0, stream, I, count, st, factor);
    return hipGetLastError();
}

hipError_t launch_normalize(double* T, size_t count, DevState* st, int n, hipStream_t stream) {
    size_t nb = (count + 255) / 256;
    if (nb > RED_BLOCKS) nb = RED_BLOCKS;
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(absmax_partial_kernel, dim3((unsigned)nb), dim3(256), 0, stream, T, count, st);
    hipLaunchKernelGGL(norm_finalize_kernel, dim3(1), dim3(256), 0, stream, st, (int)nb, n);
    size_t sb = (count + 255) / 256;
    if (sb > 8192) sb = 8192;
    if (sb < 1) sb = 1;
    hipLaunchKernelGGL(scale_kernel, dim3((unsigned)sb), dim3(256), 0, stream, T, count, st);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void trace_kernel(const double* __restrict__ T, int Dx, int Dy, double* out) {
    __shared__ double sh[256];
    double s = 0.0;
    const int total = Dx * Dy;
    for (int i = threadIdx.x; i < total; i += 256) {
        const int x = i / Dy, y = i - (i / Dy) * Dy;
        s += T[(((long)x * Dx + x) * Dy + y) * Dy + y];
    }
    s = block_sum<256>(s, sh);
    if (threadIdx.x == 0) *out = s;
}

hipError_t launch_trace(const double* T, int Dx, int Dy, DevState* st, hipStream_t stream, double* out) {
    hipLaunchKernelGGL(trace_kernel, dim3(1), dim3(256), 0, stream, T, Dx, Dy, out ? out : &st->trace);
    return hipGetLastError();
}

// ---------------------------------------------------------------- chain closure

// One workgroup: A = t (the y-traced tensor, Dx x Dx, in LDS), then
// A <- A A / c_j with c_j = max|A A| and acc += ln(c_j) / 2^(j+1), so that
// ln lambda_max = acc + ln(Tr A) / 2^squarings (exactly so as squarings grow,
// for a dominant eigenvalue of largest modulus).  Fixed-order reductions.
constexpr int kChainMax = 96;
__global__ __launch_bounds__(256) void chain_lnz_kernel(const double* __restrict__ T, int Dx, int Dy, int squarings,
                                                        DevState* st) {
    __shared__ double A[kChainMax * kChainMax];
    __shared__ double B[kChainMax * kChainMax];
    __shared__ double sh[256];
    const int tid = threadIdx.x;
    const int nn = Dx * Dx;
    for (int i = tid; i < nn; i += 256) {
        const int l = i / Dx, r = i - (i / Dx) * Dx;
        double acc = 0.0;
        for (int s = 0; s < Dy; ++s) acc += T[(((long)l * Dx + r) * Dy + s) * Dy + s];
        A[i] = acc;
    }
    __syncthreads();
    double lacc = 0.0;
    for (int j = 0; j < squarings; ++j) {
        double m = 0.0;
        for (int i = tid; i < nn; i += 256) {
            const int a = i / Dx, b = i - (i / Dx) * Dx;
            double acc = 0.0;
            for (int k = 0; k < Dx; ++k) acc = fma(A[a * Dx + k], A[k * Dx + b], acc);
            B[i] = acc;
            m = fmax(m, fabs(acc));
        }
        m = block_max<256>(m, sh);
        if (!(m > 0.0) || !isfinite(m)) break;
        lacc += log(m) * ldexp(1.0, -(j + 1));
        for (int i = tid; i < nn; i += 256) A[i] = B[i] / m;
        __syncthreads();
    }
    double tr = 0.0;
    for (int i = tid; i < Dx; i += 256) tr += A[i * Dx + i];
    tr = block_sum<256>(tr, sh);
    if (tid == 0) {
        const bool ok = tr > 0.0 && isfinite(tr);
        st->chain_ok = ok ? 1 : 0;
        st->chain_lnz = ok ? lacc + log(tr) * ldexp(1.0, -squarings) : 0.0;
    }
}

hipError_t launch_chain_lnz(const double* T, int Dx, int Dy, int squarings, DevState* st, hipStream_t stream) {
    if (Dx < 1 || Dx > kChainMax || Dy < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(chain_lnz_kernel, dim3(1), dim3(256), 0, stream, T, Dx, Dy, squarings, st);
    return hipGetLastError();
}

// ---------------------------------------------------------------- E symmetrisation

__global__ void symmetrize_kernel(double* __restrict__ E, int n) {
    // one thread per (i, j) with i < j, as 16x16 blocks of the upper triangle
    const int i = blockIdx.y * 16 + threadIdx.y;
    const int j = blockIdx.x * 16 + threadIdx.x;
    if (i < n && j < n && i < j) {
        const double v = 0.5 * (E[(long)i * n + j] + E[(long)j * n + i]);
        E[(long)i * n + j] = v;
        E[(long)j * n + i] = v;
    }
}

hipError_t launch_symmetrize(double* E, int n, hipStream_t stream) {
    const unsigned b = (unsigned)((n + 15) / 16);
    hipLaunchKernelGGL(symmetrize_kernel, dim3(b, b), dim3(16, 16), 0, stream, E, n);
    return hipGetLastError();
}

}  // namespace hotrg
