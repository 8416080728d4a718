// Allocation-free form of the stand-alone contraction (hotrg_gemm_nt_noalloc
// in include/hotrg_noalloc.h), for callers that cannot allocate device memory.
//
// The operand conversion of the reduced precisions needs device memory
// beyond the caller's inputs and output (the split planes of A and B).  Here
// it lives in a file-scope device array of a fixed size.  Each GPU the
// library runs on holds its own copy, at its own address, until the process
// ends.  In host code the array's name is only a host-side stand-in, so its
// device address is looked up once per device, with that device current,
// and only that address is ever handed to kernels.
#include <mutex>

#include "../../include/hotrg_noalloc.h"
#include "common.h"

namespace {

static __device__ __align__(256) unsigned char scratch[HOTRG_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_lock;
void* g_scratch[kMaxDevices] = {};   // device address of `scratch` per device

// Device address of the current device's copy of `scratch`.
int scratch_address(void** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return HOTRG_EHIP;
    if (dev < 0 || dev >= kMaxDevices) return HOTRG_ENODEV;
    std::lock_guard<std::mutex> g(g_lock);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return HOTRG_EHIP;
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return HOTRG_OK;
}

}  // namespace

extern "C" int hotrg_gemm_nt_noalloc(int precision, int role, int panel, int M, int N, int K, const double* A,
                                     long lda, const double* B, long ldb, double* C, double alpha, long sm,
                                     long rs_hi, long rs_lo, long sn, long cs_hi, long cs_lo, void* stream) {
    if (M < 0 || N < 0 || K < 0) return HOTRG_EINVAL;
    if (hotrg::gemm_scratch_bytes(precision, M, N, K) > (size_t)HOTRG_NOALLOC_SCRATCH_BYTES) return HOTRG_ENOMEM;
    void* ws = nullptr;
    if (precision != HOTRG_FP64) {
        const int rc = scratch_address(&ws);
        if (rc) return rc;
    }
    return hotrg::gemm_nt_with_scratch(precision, role, panel, M, N, K, A, lda, B, ldb, C, alpha, sm, rs_hi, rs_lo,
                                       sn, cs_hi, cs_lo, ws, (size_t)HOTRG_NOALLOC_SCRATCH_BYTES, stream);
}
