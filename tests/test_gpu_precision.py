"""Reduced-precision contraction paths (FP32, BF16 split with 3 or 6
products, FP32 accumulation) against the FP64 oracle.  The eigensolve, the
normalisation and ln Z stay FP64 in every mode.  The bounds here are the
claims each mode makes (|delta f| / |f|): FP32 and BF16x6 <= 1e-6, BF16x3
<= 1e-5; the measured errors are reported by the benchmark."""
import numpy as np
import pytest

from oracle import exact, hotrg as oracle

pytestmark = pytest.mark.gpu

CLAIM = {"fp32": 1e-6, "bf16x6": 1e-6, "fp16x3": 1e-6, "bf16x3": 1e-5}


def rel(a, b):
    return abs(a - b) / abs(b)


@pytest.mark.parametrize("precision", ["fp32", "bf16x6", "bf16x3"])
@pytest.mark.parametrize("T", [1.8, 2.269185314213022, 2.8])
def test_d24_solve_error_within_claim(gpu_lib, precision, T):
    from paper_2602_05900_amd import binding
    ref = oracle.solve("ising", 2, T, 24, 30, keep_tensor=False).lnz_per_site
    s = binding.Solve(model="ising", q=2, temperature=T, dmax=24, precision=precision, max_steps=30)
    s.coarse_grain(30)
    err = rel(-T * s.log_z(), -T * ref)
    print(f"{precision} T={T:.4f} |df|/|f| = {err:.2e}")
    assert err <= CLAIM[precision]


@pytest.mark.parametrize("precision", ["fp32", "bf16x6", "bf16x3"])
def test_potts_solve_error_within_claim(gpu_lib, precision):
    from paper_2602_05900_amd import binding
    T = 0.9 * exact.POTTS3_TC
    ref = oracle.solve("potts", 3, T, 15, 16, keep_tensor=False).lnz_per_site
    s = binding.Solve(model="potts", q=3, temperature=T, dmax=15, precision=precision, max_steps=16)
    s.coarse_grain(16)
    assert rel(s.log_z(), ref) <= CLAIM[precision]


def test_c5_d64_bf16x6_against_fp64_and_onsager(gpu_lib):
    """Ising at Tc, D = 64, 40 steps (n = 4096 environments): BF16x6 within
    its claim of the FP64 path on the same GPU; both near Onsager's exact
    value (the HOTRG truncation error, largest at Tc); the eigensolver meets
    its residual bound at every step."""
    import torch
    from paper_2602_05900_amd import binding
    Tc = exact.ISING_TC
    lnz = {}
    for prec in ("fp64", "bf16x6", "fp16x3"):
        s = binding.Solve(model="ising", q=2, temperature=Tc, dmax=64, precision=prec, max_steps=40)
        s.coarse_grain(40)
        lnz[prec] = s.log_z()
        for n in range(1, 41):
            it, sweeps, res = s.eig_info(n)
            assert res <= 1e-12 and it < 30, (prec, n, it, res)
        s.close()
        torch.cuda.empty_cache()
    exact_tc = exact.onsager_lnz_tc()
    print(f"D=64 Tc: fp64 {lnz['fp64']:.15f} bf16x6 {lnz['bf16x6']:.15f} onsager {exact_tc:.15f}")
    print(f"D=64 Tc: fp16x3 {lnz['fp16x3']:.15f}")
    assert rel(lnz["bf16x6"], lnz["fp64"]) <= CLAIM["bf16x6"]
    assert rel(lnz["fp16x3"], lnz["fp64"]) <= CLAIM["fp16x3"]
    assert rel(lnz["fp64"], exact_tc) < 1e-5


@pytest.mark.parametrize("precision", ["fp16x3", "bf16x6"])
def test_d32_against_oracle_golden(gpu_lib, precision):
    """D = 32, 30 steps (the smallest bond dimension whose steady Y product
    takes the full-size tiles, and with them FP16X3's FP16 planes) against
    the oracle's values in tests/golden/oracle_ising_d32.json."""
    import json
    import os
    from paper_2602_05900_amd import binding
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_ising_d32.json")
    for r in json.load(open(path))["rows"]:
        T = r["temperature"]
        s = binding.Solve(model="ising", q=2, temperature=T, dmax=32, precision=precision, max_steps=30)
        s.coarse_grain(30)
        e = rel(-T * s.log_z(), r["free_energy"])
        print(f"D=32 {precision} T={T:.4f} |df|/|f| = {e:.2e}")
        assert e <= CLAIM[precision]
        s.close()


# ------------------------------------------------------------------ FP16 environment products

@pytest.mark.parametrize("M,N,K", [(128, 96, 16), (288, 320, 272), (1024, 1024, 1024)])
def test_gemm_nt_fp16x3_environment_role(gpu_lib, M, N, K):
    """The environment products' FP16 form (generic role, panel operands):
    C = 0.75 A B^T against NumPy.  Each operand is converted as 2^11 x value
    into two FP16 terms (22 significant bits for |value| >= 2^-14, an absolute
    floor of 2^-35 below), the lo*lo product is dropped, FP32 accumulation:
    |err| <= (4 * 2^-22 + 8 sqrt(K) 2^-24) sum_k |a_k b_k| plus the floor.
    M = 288 leaves a ragged row tile, K = 272 an odd number of K steps."""
    import torch
    from paper_2602_05900_amd import binding
    rng = np.random.default_rng(M + 3 * N + 7 * K)
    A = rng.standard_normal((M, K))
    B = rng.standard_normal((N, K))
    ref = (A @ B.T) * 0.75
    absdot = (np.abs(A) @ np.abs(B).T) * 0.75
    dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    dC = torch.full((M * N,), float("nan"), dtype=torch.float64, device="cuda")
    binding.gemm_nt(dA, dB, dC, M, N, K, K, K, (1, N, 0, 1, 1, 0), precision="fp16x3", role="generic", panel=True,
                    alpha=0.75)
    torch.cuda.synchronize()
    C = dC.cpu().numpy().reshape(M, N)
    assert np.all(np.isfinite(C))
    floor = 2.0 ** -33 * K * np.max(np.abs(A)) * np.max(np.abs(B))
    bound = (4 * 2.0 ** -22 + 8 * np.sqrt(K) * 2.0 ** -24) * absdot + floor
    assert np.all(np.abs(C - ref) <= bound), float(np.max(np.abs(C - ref) / bound))


def environment_error_bound(T, eps):
    """Componentwise bound on the error of E computed by the split products,
    E = sum_{k,k'} Ah[a1,k,b1,k'] Bh[a2,k,b2,k'] with Ah, Bh the half
    environments (sums over K1 = Dx Dy products of entries of T):
      |dAh| <= e1 |T||T| (the half environment of |T|), e1 = 3 eps (operand
              splits and the split of Ah itself) + 8 sqrt(K1) 2^-24 (FP32
              accumulation), and the same for Bh;
      |dE|  <= |dAh| |Bh| + |Ah| |dBh| + e2 |Ah| |Bh|, e2 = 2 eps +
              8 sqrt(K2) 2^-24 over K2 = Dy^2;
    eps the relative error of one split operand term (2^-22 for two FP16
    terms, 2^-24 for three BF16 terms); symmetrised as E is."""
    Dx, Dy = T.shape[0], T.shape[2]
    aA, aB = oracle.half_environments(np.abs(T))
    e1 = 3 * eps + 8 * np.sqrt(Dx * Dy) * 2.0 ** -24
    e2 = 2 * eps + 8 * np.sqrt(Dy * Dy) * 2.0 ** -24
    b4 = (2 * e1 + e2) * np.einsum("ikjl,mknl->imjn", aA, aB, optimize=True)
    b = b4.reshape(Dx * Dx, Dx * Dx)
    return 0.5 * (b + b.T)


@pytest.fixture(scope="module")
def d32_tensor():
    """A D = 32 fixed-point-regime tensor (FP64 solve, 8 steps at Tc) and
    the oracle's environment of it."""
    from paper_2602_05900_amd import binding
    s = binding.Solve(model="ising", q=2, temperature=exact.ISING_TC, dmax=32, max_steps=8)
    s.coarse_grain(8)
    Tin = s.tensor()
    s.close()
    assert Tin.shape == (32, 32, 32, 32)
    return Tin, oracle.environment(Tin)


@pytest.fixture(scope="module")
def d36_step5_tensor():
    """The tensor entering step 6 of a D = 36 FP64 solve at Tc: dims (Dx, Dy)
    = (16, 36), where the environment products take the panel layout but
    Dy is not a multiple of 8, so the half environments leave the product
    kernel through its element-store path rather than 16-byte stores."""
    from paper_2602_05900_amd import binding
    s = binding.Solve(model="ising", q=2, temperature=exact.ISING_TC, dmax=36, max_steps=5)
    s.coarse_grain(5)
    Tin = s.tensor()
    s.close()
    assert Tin.shape == (16, 16, 36, 36)
    return Tin, oracle.environment(Tin)


@pytest.mark.parametrize("tensor", ["d32_tensor", "d36_step5_tensor"])
@pytest.mark.parametrize("precision,eps", [("fp16x3", 2.0 ** -22), ("bf16x6", 2.0 ** -24)])
def test_split_environment_within_error_bound(gpu_lib, request, tensor, precision, eps):
    """One step from the same tensor: the environment E the split products
    build (FP16 terms for fp16x3, whose environment products take the panel
    layout at these dims; BF16 terms for bf16x6) against the oracle's FP64
    E, within the componentwise bound above plus 2^-26 of max|E| (entries
    far below the largest meet FP16's absolute floor)."""
    from paper_2602_05900_amd import binding
    Tin, E_ref = request.getfixturevalue(tensor)
    s = binding.Solve(model="custom", tensor=Tin, dmax=Tin.shape[2], temperature=1.0, precision=precision,
                      max_steps=1)
    s.coarse_grain(1)
    E = s.environment()
    s.close()
    assert E.shape == E_ref.shape
    bound = environment_error_bound(Tin, eps) + 2.0 ** -26 * np.max(np.abs(E_ref))
    err = np.abs(E - E_ref)
    print(f"{precision}: max |dE| / max |E| = {np.max(err) / np.max(np.abs(E_ref)):.2e}, "
          f"max |dE| / bound = {np.max(err / bound):.3f}")
    assert np.all(err <= bound), float(np.max(err / bound))


def test_fp16x3_d36_solve_within_claim(gpu_lib):
    """FP16X3 at D = 36 (10 steps at Tc): step 6 has dims (16, 36), where the
    environment products run in FP16 terms with element stores (Dy not a
    multiple of 8), and the later (36, 36) steps keep BF16 planes for the
    environment (Dx^2 not a multiple of 32); ln Z against the oracle within
    the mode's claim."""
    from paper_2602_05900_amd import binding
    T = exact.ISING_TC
    ref = oracle.solve("ising", 2, T, 36, 10, keep_tensor=False).lnz_per_site
    s = binding.Solve(model="ising", q=2, temperature=T, dmax=36, precision="fp16x3", max_steps=10)
    s.coarse_grain(10)
    err = rel(s.log_z(), ref)
    s.close()
    print(f"fp16x3 D=36 |d lnZ|/|lnZ| = {err:.2e}")
    assert err <= CLAIM["fp16x3"]
