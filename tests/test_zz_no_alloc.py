"""The allocation-free entry point (include/hotrg_noalloc.h) against the
entry point it is a variant of: hotrg_gemm_nt_noalloc and
hotrg_gemm_nt_role run the same conversion and product kernels on the same
inputs, so their outputs are compared bitwise, on two calls in a row with
the second on a smaller input (the shared array keeps the first call's
contents, which the second must not read), for each split precision and an
FP64 product (no scratch); a product too large for the array is refused
with ENOMEM before anything is enqueued."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

CASES = [
    # (precision, role, panel, M, N, K): the second of each pair is smaller
    ("bf16x6", "y", True, 16384, 1024, 256), ("bf16x6", "y", True, 4096, 512, 128),
    # FP16X3 runs only as the full-size Y product: at least 512 tiles of 256 x 256
    ("fp16x3", "y", True, 32768, 1024, 256), ("fp16x3", "y", True, 32768, 1024, 128),
    ("bf16x3", "generic", False, 700, 300, 96), ("bf16x3", "generic", False, 129, 65, 17),
    ("fp32", "generic", False, 300, 200, 64), ("fp32", "generic", False, 31, 17, 5),
    ("fp64", "generic", False, 200, 100, 40), ("fp64", "generic", False, 20, 10, 4),
]


def run_both(prec, role, panel, M, N, K, seed):
    import torch
    from paper_2602_05900_amd import binding
    g = torch.Generator("cuda").manual_seed(seed)
    A = torch.empty((M, K), dtype=torch.float64, device="cuda").normal_(generator=g)
    B = torch.empty((N, K), dtype=torch.float64, device="cuda").normal_(generator=g)
    C1 = torch.full((M * N,), float("nan"), dtype=torch.float64, device="cuda")
    C2 = torch.full((M * N,), float("nan"), dtype=torch.float64, device="cuda")
    mp = (1, N, 0, 1, 1, 0)
    binding.gemm_nt(A, B, C1, M, N, K, K, K, mp, precision=prec, alpha=0.5, role=role, panel=panel)
    rc = binding.gemm_nt_noalloc(A, B, C2, M, N, K, K, K, mp, precision=prec, alpha=0.5, role=role, panel=panel)
    torch.cuda.synchronize()
    assert rc == binding.OK
    a, b = C1.cpu().numpy(), C2.cpu().numpy()
    assert np.all(np.isfinite(a))
    return a, b


@pytest.mark.parametrize("first", range(0, len(CASES), 2))
def test_noalloc_equals_the_scratch_entry_point_twice(gpu_lib, first):
    for i, case in enumerate(CASES[first:first + 2]):
        print(f"no-alloc case {case}", flush=True)
        a, b = run_both(*case, seed=first * 10 + i)
        assert np.array_equal(a, b), case


def test_too_large_is_refused(gpu_lib):
    import torch
    from paper_2602_05900_amd import binding
    lib = binding.load()
    M, N, K = 8192, 2048, 2048      # 6 bytes a value in BF16x6: 120 MiB of planes > 64 MiB
    assert lib.hotrg_gemm_scratch_bytes(binding.BF16X6, M, N, K) > binding.NOALLOC_SCRATCH_BYTES
    A = torch.zeros((1,), dtype=torch.float64, device="cuda")
    rc = binding.gemm_nt_noalloc(A, A, A, M, N, K, K, K, (1, N, 0, 1, 1, 0), precision="bf16x6")
    assert rc == binding.ENOMEM
