"""Pins of the FP64 CPU oracle against what the mathematics fixes.

Each test checks the oracle against something other than itself: brute-force
spin sums, transfer matrices, explicit network contractions of random
non-symmetric tensors, closed forms, invariances and limits.  Every plausible
mistake in the oracle (a dropped term, a wrong sign, a swapped leg, a
transposed operand) breaks at least one of them.
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import exact, hotrg

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = json.load(open(os.path.join(HERE, "golden", "exact_tori.json")))


def rel(a, b):
    return abs(a - b) / abs(b)


# ------------------------------------------------------------------ S0

@pytest.mark.parametrize("beta", [0.1, 1.0 / exact.ISING_TC, 0.9])
def test_ising_weight_root_closed_form(beta):
    W = hotrg.boltzmann_weights("ising", 2, beta)
    Q = hotrg.weight_root(W)
    np.testing.assert_allclose(Q @ Q, W, rtol=1e-14)
    # closed form: eigenvalues 2cosh(beta) on (1,1)/sqrt2 and 2sinh(beta) on (1,-1)/sqrt2
    p = np.array([[0.5, 0.5], [0.5, 0.5]])
    m = np.array([[0.5, -0.5], [-0.5, 0.5]])
    Qc = math.sqrt(2 * math.cosh(beta)) * p + math.sqrt(2 * math.sinh(beta)) * m
    np.testing.assert_allclose(Q, Qc, rtol=1e-14, atol=1e-15)


def test_potts_weight_root_closed_form():
    beta, q = 1.3, 3
    Q = hotrg.weight_root(hotrg.boltzmann_weights("potts", q, beta))
    a = math.exp(beta) - 1.0
    Qc = math.sqrt(a) * np.eye(q) + (math.sqrt(a + q) - math.sqrt(a)) / q * np.ones((q, q))
    np.testing.assert_allclose(Q, Qc, rtol=1e-14, atol=1e-15)


@pytest.mark.parametrize("model,q", [("ising", 2), ("potts", 3)])
def test_initial_tensor_lattice_symmetries(model, q):
    T0 = hotrg.initial_tensor(model, q, 1.7)
    perms = [(0, 1, 2, 3), (1, 0, 2, 3), (0, 1, 3, 2), (1, 0, 3, 2),
             (2, 3, 0, 1), (3, 2, 0, 1), (2, 3, 1, 0), (3, 2, 1, 0)]
    for p in perms:
        np.testing.assert_allclose(T0.transpose(p), T0, rtol=1e-15, atol=0)


@pytest.mark.parametrize("model,q", [("ising", 2), ("potts", 3)])
def test_zero_steps_is_one_site_torus(model, q):
    T = 1.9
    s = hotrg.solve(model, q, T, 8, 0)
    # one site whose two bonds are closed on itself: Z = q exp(2 beta)
    assert rel(s.lnz_per_site, math.log(q) + 2.0 / T) < 1e-14


# ------------------------------------------------------------------ exact tori

@pytest.mark.parametrize("case", [c for c in GOLDEN["cases"] if c["model"] == "ising"],
                         ids=lambda c: f"ising-n{c['nsteps']}-T{c['temperature']:.3f}")
def test_ising_tori_exact_without_truncation(case):
    s = hotrg.solve("ising", 2, case["temperature"], 16, case["nsteps"])
    assert rel(s.lnz_per_site, case["lnz_per_site"]) < 1e-13


@pytest.mark.parametrize("case", [c for c in GOLDEN["cases"]
                                  if c["model"] == "potts" and c["nsteps"] <= 3],
                         ids=lambda c: f"potts-n{c['nsteps']}-T{c['temperature']:.3f}")
def test_potts_tori_exact_without_truncation(case):
    s = hotrg.solve("potts", 3, case["temperature"], 81, case["nsteps"])
    assert rel(s.lnz_per_site, case["lnz_per_site"]) < 1e-13


@pytest.mark.slow
def test_potts_4x4_torus_exact():
    case = [c for c in GOLDEN["cases"] if c["model"] == "potts" and c["nsteps"] == 4][1]
    s = hotrg.solve("potts", 3, case["temperature"], 81, 4)
    assert rel(s.lnz_per_site, case["lnz_per_site"]) < 1e-13


def test_spin_transfer_matrix_matches_brute_force():
    for model, q, T in [("ising", 2, 2.1), ("potts", 3, 0.9)]:
        for Lx, Ly in [(1, 2), (2, 2), (2, 3), (3, 2)]:
            a = exact.brute_force_lnz(model, q, T, Lx, Ly)
            b = exact.spin_transfer_lnz(model, q, T, Lx, Ly)
            assert rel(b, a) < 1e-14


def test_network_contraction_matches_brute_force():
    # the network route on the physical tensor reproduces the spin sum
    for model, q, T in [("ising", 2, 2.4), ("potts", 3, 1.1)]:
        T0 = hotrg.initial_tensor(model, q, T)
        for Lx, Ly in [(1, 1), (1, 2), (2, 2), (2, 4), (3, 2)]:
            assert rel(exact.network_lnz(T0, Lx, Ly), exact.brute_force_lnz(model, q, T, Lx, Ly)) < 1e-13


@pytest.mark.parametrize("nsteps", [1, 2, 3, 4])
def test_random_nonsymmetric_tensor_conventions(nsteps):
    """Index conventions: a random tensor with no lattice symmetry and Dx != Dy;
    without truncation HOTRG must equal the explicit network contraction of
    the torus in the stated orientation (Lx by Ly)."""
    rng = np.random.default_rng(1234 + nsteps)
    T = rng.uniform(0.05, 1.0, size=(2, 2, 3, 3))
    Lx, Ly = exact.hotrg_torus(nsteps)
    s = hotrg.solve_tensor(T, 81, nsteps)
    assert rel(s.lnz_per_site, exact.network_lnz(T, Lx, Ly) / (Lx * Ly)) < 1e-13
    if Lx != Ly:
        # the orientation matters for this tensor: the transposed torus differs
        assert rel(s.lnz_per_site, exact.network_lnz(T, Ly, Lx) / (Lx * Ly)) > 1e-6


def test_environment_is_m_mt_of_explicit_merged_tensor():
    rng = np.random.default_rng(7)
    T = rng.standard_normal((3, 3, 2, 2))
    Dx = 3
    # explicit merged pair M[(a1 a2), (r1 r2 d u)]
    M = np.einsum("ardk,bsku->abrsdu", T, T).reshape(Dx * Dx, -1)
    E = hotrg.environment(T)
    np.testing.assert_allclose(E, M @ M.T, rtol=1e-13, atol=1e-13)
    assert abs(np.trace(E) - np.sum(M * M)) < 1e-12 * np.sum(M * M)
    tr = hotrg.truncation(E, 4)
    np.testing.assert_allclose(tr.U.T @ tr.U, np.eye(4), atol=1e-14)
    assert np.all(tr.eigenvalues >= -1e-12 * tr.eigenvalues[0])
    assert abs(np.sum(tr.eigenvalues) - np.trace(E)) < 1e-13 * math.sqrt(9) * np.trace(E)
    assert np.all(np.diff(tr.eigenvalues) <= 0)
    # sign gauge: the largest-magnitude entry of every kept column is positive
    for j in range(4):
        assert tr.U[np.argmax(np.abs(tr.U[:, j])), j] > 0


def test_truncated_step_is_isometric_projection_of_merged_tensor():
    """T' = U^T M U for the fused legs, checked against the explicit D^6 matrix."""
    rng = np.random.default_rng(11)
    T = rng.standard_normal((3, 3, 2, 2))
    Dx, Dy = 3, 2
    st = hotrg.coarse_grain_step(T, 5)
    U = st.trunc.U
    M = np.einsum("ardk,bsku->abrsdu", T, T).reshape(Dx * Dx, Dx * Dx, Dy, Dy)
    Tp = np.einsum("al,abdu,br->lrdu", U, M, U)
    Tp = Tp / np.max(np.abs(Tp))
    np.testing.assert_allclose(st.T_next, Tp.transpose(2, 3, 0, 1), rtol=1e-12, atol=1e-14)


# ------------------------------------------------------------------ truncated HOTRG

def test_bond_gauge_invariance_with_truncation():
    """Orthogonal matrices inserted on every bond (O O^T = 1) leave Z of the
    network unchanged; HOTRG is covariant, so f must not move even when
    truncating (left and right legs must use the same U)."""
    rng = np.random.default_rng(5)
    T0 = hotrg.initial_tensor("ising", 2, exact.ISING_TC)
    Ox, _ = np.linalg.qr(rng.standard_normal((2, 2)))
    Oy, _ = np.linalg.qr(rng.standard_normal((2, 2)))
    Tg = np.einsum("abcd,ai,bj,ck,dl->ijkl", T0, Ox, Ox, Oy, Oy)
    a = hotrg.solve_tensor(T0, 8, 12).lnz_per_site
    b = hotrg.solve_tensor(Tg, 8, 12).lnz_per_site
    assert rel(b, a) < 1e-13


def test_potts_q2_is_shifted_ising():
    """Potts with q = 2 at beta equals beta plus Ising at beta/2 (delta = (1+ss')/2)."""
    for T in [1.0, 1.2, 2.0]:
        p = hotrg.solve("potts", 2, T, 8, 14).lnz_per_site
        i = hotrg.solve("ising", 2, 2 * T, 8, 14).lnz_per_site
        assert rel(p, 1.0 / T + i) < 1e-13


def test_fused_legs_stay_reflection_symmetric():
    """For a reflection-symmetric model the merged pair is symmetric under
    exchanging the two fused legs, and the eigenvectors of E are even or odd
    under swapping bottom and top; so the legs just fused obey
    T[.., i, j] = s_i s_j T[.., j, i] with s = +-1 (exactly so on step 1)."""
    T = hotrg.initial_tensor("ising", 2, exact.ISING_TC)
    st = hotrg.coarse_grain_step(T, 6)
    np.testing.assert_allclose(st.T_next, st.T_next.transpose(0, 1, 3, 2), rtol=0, atol=1e-14)
    T = st.T_next
    for _ in range(5):
        T = hotrg.coarse_grain_step(T, 6).T_next
        Tt = T.transpose(0, 1, 3, 2)
        np.testing.assert_allclose(np.abs(T), np.abs(Tt), rtol=0, atol=1e-13)


@pytest.mark.parametrize("model,q", [("ising", 2), ("potts", 3)])
def test_high_temperature_limit(model, q):
    beta = 1e-7
    s = hotrg.solve(model, q, 1.0 / beta, 8, 16)
    # ln Z/N = ln q + 2 beta <-H_bond/J>_(beta=0) + O(beta^2): 0 for Ising, 1/q for Potts
    first_order = 0.0 if model == "ising" else 2.0 * beta / q
    assert abs(s.lnz_per_site - math.log(q) - first_order) < 1e-12


@pytest.mark.parametrize("model,q,beta", [("ising", 2, 5.0), ("potts", 3, 10.0)])
def test_low_temperature_limit(model, q, beta):
    n = 16
    s = hotrg.solve(model, q, 1.0 / beta, 8, n)
    # q ground states of energy -2N J, excitations suppressed by exp(-4 beta) or less
    expect = 2.0 * beta + math.log(q) / 2 ** n
    assert rel(s.lnz_per_site, expect) < 1e-13


# ------------------------------------------------------------------ Onsager

def test_onsager_integral_matches_closed_form_at_tc():
    g = GOLDEN["onsager_tc"]
    assert rel(exact.onsager_lnz(g["temperature"]), g["lnz_per_site"]) < 1e-14
    assert abs(exact.onsager_energy(exact.ISING_TC) + math.sqrt(2.0)) < 1e-14


@pytest.mark.parametrize("T", [1.8, 2.0, 2.6, 3.2])
def test_onsager_energy_is_derivative_of_lnz(T):
    h = 1e-4
    d = (exact.onsager_lnz(T + h) - exact.onsager_lnz(T - h)) / (2 * h)
    assert abs(T * T * d - exact.onsager_energy(T)) < 1e-7


def test_hotrg_approaches_onsager_with_bond_dimension():
    lo = exact.onsager_lnz_tc()
    e8 = rel(hotrg.solve("ising", 2, exact.ISING_TC, 8, 20).lnz_per_site, lo)
    e16 = rel(hotrg.solve("ising", 2, exact.ISING_TC, 16, 20).lnz_per_site, lo)
    assert e8 < 3e-5
    assert e16 < 1e-6
    assert e16 < e8 / 10


@pytest.mark.parametrize("T", [2.0, 2.6])
def test_hotrg_off_critical_matches_onsager(T):
    s = hotrg.solve("ising", 2, T, 16, 24)
    assert rel(s.lnz_per_site, exact.onsager_lnz(T)) < 1e-7


def test_finite_difference_energy_exact_on_quadratics():
    T = np.linspace(1.0, 2.0, 11)
    g = 3.0 + 2.0 * T - 0.5 * T ** 2
    u = exact.finite_difference_energy(T, g)
    np.testing.assert_allclose(u, T * T * (2.0 - T), rtol=1e-12, atol=1e-12)


def test_step_dims_and_flops():
    dims = hotrg.step_dims(2, 2, 48, 8)
    assert [d[:2] for d in dims] == [(2, 2), (2, 4), (4, 4), (4, 16), (16, 16), (16, 48), (48, 48), (48, 48)]
    assert abs(hotrg.contraction_flops(48, 48, 48) - (2 * 48 ** 7 + 10 * 48 ** 6)) < 1


def test_stored_onsager_grid_matches_the_oracle():
    """tests/golden/onsager_ising.json (read by the benchmark) is what
    oracle/exact.py gives now."""
    import json
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "onsager_ising.json")
    d = json.load(open(path))
    g = d["grid"]
    for i in (0, 17, 31, 63):
        t = g["temperatures"][i]
        assert abs(g["lnz_per_site"][i] - exact.onsager_lnz(t)) <= 1e-14
        assert abs(g["energy"][i] - exact.onsager_energy(t)) <= 1e-12
        assert abs(g["magnetisation"][i] - exact.yang_magnetisation(t)) <= 1e-15
    assert abs(d["critical"]["lnz_per_site"] - exact.onsager_lnz_tc()) <= 1e-15
    assert abs(d["critical"]["energy"] + math.sqrt(2.0)) <= 1e-15
