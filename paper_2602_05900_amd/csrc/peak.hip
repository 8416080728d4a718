// Measured ceilings of the MI355X units the HOTRG kernels use: issue-rate
// loops of independent MFMA (FP64 16x16x4, FP32 16x16x4, BF16 16x16x32 and
// 32x32x16) and FP64 vector FMA on register operands only, and a streaming
// device copy.  Prints one JSON object.  These are the roofs the product
// kernels are compared with besides the datasheet peaks; they are not used
// by the library.
//
//     paper_2602_05900_amd/peak_bench [--iters N]
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f16v __attribute__((ext_vector_type(16)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

#define CHECK(x)                                                                          \
    do {                                                                                  \
        hipError_t e_ = (x);                                                              \
        if (e_ != hipSuccess) {                                                           \
            fprintf(stderr, "HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__); \
            return 1;                                                                     \
        }                                                                                 \
    } while (0)

// 8 (or 4) independent accumulators per wave keep the matrix pipe fed; the
// sum is stored so that no product is dead code.
__global__ __launch_bounds__(256) void mfma_f64(double* out, int iters) {
    d4 c[8];
    for (int i = 0; i < 8; ++i) c[i] = d4{0, 0, 0, 0};
    const double a = 1e-3 * threadIdx.x, b = 1.0 + threadIdx.x;
    for (int it = 0; it < iters; ++it)
#pragma unroll
        for (int i = 0; i < 8; ++i) c[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c[i], 0, 0, 0);
    double s = 0;
    for (int i = 0; i < 8; ++i) s += c[i][0] + c[i][1] + c[i][2] + c[i][3];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void mfma_f32(float* out, int iters) {
    f4 c[8];
    for (int i = 0; i < 8; ++i) c[i] = f4{0, 0, 0, 0};
    const float a = 1e-3f * threadIdx.x, b = 1.f + threadIdx.x;
    for (int it = 0; it < iters; ++it)
#pragma unroll
        for (int i = 0; i < 8; ++i) c[i] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c[i], 0, 0, 0);
    float s = 0;
    for (int i = 0; i < 8; ++i) s += c[i][0] + c[i][1] + c[i][2] + c[i][3];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void mfma_bf16_16(float* out, int iters) {
    f4 c[8];
    for (int i = 0; i < 8; ++i) c[i] = f4{0, 0, 0, 0};
    bf8 a, b;
    for (int e = 0; e < 8; ++e) {
        a[e] = (__bf16)(1e-3f * e);
        b[e] = (__bf16)(1.f + e);
    }
    for (int it = 0; it < iters; ++it)
#pragma unroll
        for (int i = 0; i < 8; ++i) c[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c[i], 0, 0, 0);
    float s = 0;
    for (int i = 0; i < 8; ++i) s += c[i][0] + c[i][1] + c[i][2] + c[i][3];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void mfma_bf16_32(float* out, int iters) {
    f16v c[4];
    for (int i = 0; i < 4; ++i)
        for (int r = 0; r < 16; ++r) c[i][r] = 0.f;
    bf8 a, b;
    for (int e = 0; e < 8; ++e) {
        a[e] = (__bf16)(1e-3f * e);
        b[e] = (__bf16)(1.f + e);
    }
    for (int it = 0; it < iters; ++it)
#pragma unroll
        for (int i = 0; i < 4; ++i) c[i] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c[i], 0, 0, 0);
    float s = 0;
    for (int i = 0; i < 4; ++i)
        for (int r = 0; r < 16; ++r) s += c[i][r];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void valu_f64(double* out, int iters) {
    double x[8];
    for (int i = 0; i < 8; ++i) x[i] = 1e-3 * (i + threadIdx.x);
    const double m = 1.0000001, a = 1e-9;
    for (int it = 0; it < iters; ++it)
#pragma unroll
        for (int i = 0; i < 8; ++i) x[i] = fma(x[i], m, a);
    double s = 0;
    for (int i = 0; i < 8; ++i) s += x[i];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ void copy_kernel(const double4* __restrict__ in, double4* __restrict__ out, size_t n) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += stride) out[i] = in[i];
}

template <typename F>
static int time_ms(F launch, hipEvent_t e0, hipEvent_t e1, float* ms) {
    launch();   // warm-up
    CHECK(hipDeviceSynchronize());
    CHECK(hipEventRecord(e0));
    launch();
    CHECK(hipEventRecord(e1));
    CHECK(hipEventSynchronize(e1));
    CHECK(hipEventElapsedTime(ms, e0, e1));
    return 0;
}

int main(int argc, char** argv) {
    int iters = 4000;
    for (int i = 1; i + 1 < argc; ++i)
        if (!strcmp(argv[i], "--iters")) iters = atoi(argv[i + 1]);
    if (iters < 1 || iters > 1000000) {
        fprintf(stderr, "--iters must be in [1, 1000000]\n");
        return 2;
    }
    hipDeviceProp_t prop;
    CHECK(hipGetDeviceProperties(&prop, 0));
    const int cus = prop.multiProcessorCount;
    const int blocks = cus * 8, threads = 256;
    double* out;
    CHECK(hipMalloc(&out, (size_t)blocks * threads * sizeof(double)));
    hipEvent_t e0, e1;
    CHECK(hipEventCreate(&e0));
    CHECK(hipEventCreate(&e1));
    const double waves = (double)blocks * threads / 64;
    float ms;

    // FLOPs per wave instruction: 16x16x4 = 2048, 16x16x32 = 16384, 32x32x16 = 32768
    if (time_ms([&] { mfma_f64<<<blocks, threads>>>(out, iters); }, e0, e1, &ms)) return 1;
    const double f64 = waves * iters * 8 * 2048.0 / ms / 1e9;
    if (time_ms([&] { mfma_f32<<<blocks, threads>>>((float*)out, iters); }, e0, e1, &ms)) return 1;
    const double f32 = waves * iters * 8 * 2048.0 / ms / 1e9;
    if (time_ms([&] { mfma_bf16_16<<<blocks, threads>>>((float*)out, iters); }, e0, e1, &ms)) return 1;
    const double b16 = waves * iters * 8 * 16384.0 / ms / 1e9;
    if (time_ms([&] { mfma_bf16_32<<<blocks, threads>>>((float*)out, iters); }, e0, e1, &ms)) return 1;
    const double b32 = waves * iters * 4 * 32768.0 / ms / 1e9;
    if (time_ms([&] { valu_f64<<<blocks, threads>>>(out, iters * 4); }, e0, e1, &ms)) return 1;
    const double v64 = (double)blocks * threads * iters * 4 * 8 * 2.0 / ms / 1e9;

    const size_t n = (size_t)1 << 26;   // 2 GiB of double4 per buffer
    double4 *a, *b;
    CHECK(hipMalloc(&a, n * sizeof(double4)));
    CHECK(hipMalloc(&b, n * sizeof(double4)));
    CHECK(hipMemset(a, 0, n * sizeof(double4)));
    if (time_ms([&] { copy_kernel<<<cus * 16, 256>>>(a, b, n); }, e0, e1, &ms)) return 1;
    const double copy_gbs = 2.0 * n * sizeof(double4) / ms / 1e6;

    printf("{\"device\": \"%s\", \"compute_units\": %d, \"iters\": %d, "
           "\"mfma_f64_16x16x4_tflops\": %.2f, \"mfma_f32_16x16x4_tflops\": %.2f, "
           "\"mfma_bf16_16x16x32_tflops\": %.2f, \"mfma_bf16_32x32x16_tflops\": %.2f, "
           "\"valu_f64_fma_tflops\": %.2f, \"copy_read_plus_write_gbs\": %.1f}\n",
           prop.gcnArchName, cus, iters, f64, f32, b16, b32, v64, copy_gbs);
    CHECK(hipFree(a));
    CHECK(hipFree(b));
    CHECK(hipFree(out));
    return 0;
}
