"""Pins of the oracle's two-sided truncation and impurity-tensor observables.

As for the plain solve, each check is against something other than the
oracle itself: brute-force thermal averages with a field, exact contractions
of random non-symmetric networks holding one impurity, the explicit merged
tensor, the mirror symmetry of the lattice, the Potts(q=2) / Ising mapping,
limits, Onsager's energy and Yang's magnetisation.
"""
import math

import numpy as np
import pytest

from oracle import exact, hotrg


# ------------------------------------------------------------ the brute force itself

@pytest.mark.parametrize("model,q,T,h", [("ising", 2, 2.0, 0.0), ("ising", 2, 1.7, 0.3), ("potts", 3, 1.1, 0.2)])
def test_brute_force_observables_are_derivatives_of_lnz(model, q, T, h):
    """<f> = (1/(beta N)) d lnZ/dh and <H>/N = -(1/N) d lnZ/dbeta (at fixed h),
    checked by central differences; and u = e_x + e_y - h <f>."""
    Lx, Ly = 2, 3
    N = Lx * Ly
    b = exact.brute_force_observables(model, q, T, Lx, Ly, field=h)
    if h == 0.0:
        assert abs(b["lnz"] - exact.brute_force_lnz(model, q, T, Lx, Ly)) < 1e-12
    d = 1e-5
    zp = exact.brute_force_observables(model, q, T, Lx, Ly, field=h + d)["lnz"]
    zm = exact.brute_force_observables(model, q, T, Lx, Ly, field=h - d)["lnz"]
    f_mean = (zp - zm) / (2 * d) / (N / T)
    m_from_f = f_mean if model == "ising" else (q * f_mean - 1.0) / (q - 1.0)
    assert abs(m_from_f - b["m"]) < 1e-8
    beta = 1.0 / T
    zp = exact.brute_force_observables(model, q, 1.0 / (beta + d), Lx, Ly, field=h)["lnz"]
    zm = exact.brute_force_observables(model, q, 1.0 / (beta - d), Lx, Ly, field=h)["lnz"]
    assert abs(-(zp - zm) / (2 * d) / N - b["u"]) < 1e-8
    f_site = b["m"] if model == "ising" else ((q - 1) * b["m"] + 1.0) / q
    assert abs(b["e_x"] + b["e_y"] - h * f_site - b["u"]) < 1e-13


def test_yang_magnetisation_limits():
    assert exact.yang_magnetisation(exact.ISING_TC * 1.0001) == 0.0
    assert exact.yang_magnetisation(0.2) == pytest.approx(1.0, abs=1e-12)
    assert 0.0 < exact.yang_magnetisation(exact.ISING_TC * 0.999) < 0.6


# ------------------------------------------------------------ exact without truncation

@pytest.mark.parametrize("nsteps", [0, 1, 2, 3, 4])
@pytest.mark.parametrize("two_sided", [False, True])
def test_ising_observables_exact_without_truncation(nsteps, two_sided):
    T, h = 2.1, 0.1
    Lx, Ly = exact.hotrg_torus(nsteps)
    r = hotrg.solve("ising", 2, T, 16, nsteps, field=h, two_sided=two_sided, observables=("m", "e"))
    b = exact.brute_force_observables("ising", 2, T, Lx, Ly, field=h)
    assert abs(r.lnz_per_site * 2 ** nsteps - b["lnz"]) < 1e-12 * abs(b["lnz"])
    assert abs(r.observables[0] - b["m"]) < 1e-13
    assert abs(r.observables[1] - b["e_y"]) < 1e-13


@pytest.mark.parametrize("nsteps", [0, 1, 2, 3])
def test_potts_observables_exact_without_truncation(nsteps):
    T, h = 1.0, 0.05
    Lx, Ly = exact.hotrg_torus(nsteps)
    r = hotrg.solve("potts", 3, T, 81, nsteps, field=h, two_sided=True, observables=("e", "m"))
    b = exact.brute_force_observables("potts", 3, T, Lx, Ly, field=h)
    assert abs(r.observables[0] - b["e_y"]) < 1e-13
    assert abs(r.observables[1] - b["m"]) < 1e-13


def test_energy_impurity_sits_on_a_y_bond():
    """On the 1 x 2 torus (one step) x and y bonds differ; the estimate is
    the y bond's."""
    b = exact.brute_force_observables("ising", 2, 2.0, 1, 2)
    assert abs(b["e_x"] - b["e_y"]) > 0.1
    r = hotrg.solve("ising", 2, 2.0, 16, 1, observables=("e",))
    assert abs(r.observables[0] - b["e_y"]) < 1e-14


@pytest.mark.parametrize("nsteps", [1, 2, 3])
@pytest.mark.parametrize("two_sided", [False, True])
def test_impurity_update_matches_network_with_one_replaced_copy(nsteps, two_sided):
    """Random non-symmetric T and I: Tr I_n / Tr T_n equals Z_I / Z of the
    exact network with one copy replaced (every placement gives the same
    ratio, so the average over placements is that ratio)."""
    rng = np.random.default_rng(11 + nsteps)
    T = rng.uniform(0.1, 1.0, (3, 3, 2, 2))
    imps = [rng.uniform(-1.0, 1.0, (3, 3, 2, 2)), rng.uniform(0.0, 2.0, (3, 3, 2, 2))]
    Lx, Ly = exact.hotrg_torus(nsteps)
    r = hotrg.solve_tensor(T, 10 ** 6, nsteps, two_sided=two_sided, impurities=imps)
    assert abs(r.lnz_per_site * 2 ** nsteps - exact.network_lnz(T, Lx, Ly)) < 1e-12
    for I, got in zip(imps, r.observables):
        want = exact.network_impurity_ratio(T, I, Lx, Ly)
        assert abs(got - want) < 1e-13 * max(1.0, abs(want))


# ------------------------------------------------------------ two-sided truncation

def test_right_environment_is_m_mt_of_explicit_merged_tensor():
    rng = np.random.default_rng(3)
    T = rng.standard_normal((3, 3, 2, 2))
    Dx = 3
    # M[(r1 r2), (a1 a2 d u)] = sum_k T[a1,r1,d,k] T[a2,r2,k,u]
    MR = np.einsum("ardk,bsku->rsabdu", T, T).reshape(Dx * Dx, -1)
    np.testing.assert_allclose(hotrg.right_environment(T), MR @ MR.T, rtol=1e-13, atol=1e-13)
    ML = np.einsum("ardk,bsku->abrsdu", T, T).reshape(Dx * Dx, -1)
    np.testing.assert_allclose(hotrg.environment(T), ML @ ML.T, rtol=1e-13, atol=1e-13)


def test_two_sided_is_mirror_invariant_and_one_sided_is_not():
    """Reflecting the lattice (T[l,r,d,u] -> T[r,l,d,u]) leaves Z unchanged.
    Two-sided truncation sees both environments, so its result is unchanged
    too; the left-only rule is not.  Step 1's left error of one is the
    right error of the other."""
    rng = np.random.default_rng(7)
    T = rng.uniform(0.0, 1.0, (4, 4, 4, 4))
    Tm = np.ascontiguousarray(T.transpose(1, 0, 2, 3))
    a = hotrg.solve_tensor(T, 6, 8, two_sided=True)
    b = hotrg.solve_tensor(Tm, 6, 8, two_sided=True)
    assert abs(a.lnz_per_site - b.lnz_per_site) < 1e-13 * abs(a.lnz_per_site)
    c = hotrg.solve_tensor(T, 6, 8)
    d = hotrg.solve_tensor(Tm, 6, 8)
    assert abs(c.lnz_per_site - d.lnz_per_site) > 1e-8
    assert abs(a.eps_left[0] - b.eps_right[0]) < 1e-13
    assert abs(a.eps_right[0] - b.eps_left[0]) < 1e-13
    assert 1 in a.sides and 0 in a.sides


def test_two_sided_keeps_the_smaller_error():
    rng = np.random.default_rng(8)
    T = rng.uniform(0.0, 1.0, (4, 4, 4, 4))
    r = hotrg.solve_tensor(T, 6, 8, two_sided=True)
    for el, er, side, e in zip(r.eps_left, r.eps_right, r.sides, r.trunc_err):
        assert side == (1 if er < el else 0)
        assert e == min(el, er)
    one = hotrg.solve_tensor(T, 6, 1)
    assert r.trunc_err[0] <= one.trunc_err[0]


@pytest.mark.parametrize("model,q,T", [("ising", 2, exact.ISING_TC), ("potts", 3, exact.POTTS3_TC)])
def test_two_sided_equals_one_sided_for_reflection_symmetric_models(model, q, T):
    a = hotrg.solve(model, q, T, 8, 10)
    b = hotrg.solve(model, q, T, 8, 10, two_sided=True)
    for el, er in zip(b.eps_left, b.eps_right):
        assert abs(el - er) <= 1e-9 * max(el, 1e-300) + 1e-15
    assert abs(a.lnz_per_site - b.lnz_per_site) < 1e-13 * abs(a.lnz_per_site)


# ------------------------------------------------------------ truncated runs

def test_potts_q2_observables_are_shifted_ising():
    """Potts(q=2, beta, h) is Ising(beta/2, h) up to constants: the tensors
    are proportional in the same gauge, so with truncation the estimates map
    exactly: m_P = m_I, e_P = (e_I - 1)/2, lnZ_P/N = beta + beta h/2 + lnZ_I/N."""
    T, h = 1.3, 0.05
    p = hotrg.solve("potts", 2, T, 8, 12, field=h, observables=("m", "e"))
    i = hotrg.solve("ising", 2, 2 * T, 8, 12, field=h, observables=("m", "e"))
    assert abs(p.observables[0] - i.observables[0]) < 1e-13
    assert abs(p.observables[1] - (i.observables[1] - 1.0) / 2.0) < 1e-13
    assert abs(p.lnz_per_site - (1 / T + h / (2 * T) + i.lnz_per_site)) < 1e-13


@pytest.mark.parametrize("model,q", [("ising", 2), ("potts", 3)])
def test_observables_low_temperature_limit(model, q):
    r = hotrg.solve(model, q, 0.1, 8, 12, field=0.01, observables=("m", "e"))
    assert abs(r.observables[0] - 1.0) < 1e-12
    assert abs(r.observables[1] + 1.0) < 1e-12


def test_observables_high_temperature_limit():
    """beta -> 0: nearly independent spins, <sigma> = tanh(beta h) and the
    bond energy -tanh(beta), both up to relative corrections O(beta)."""
    T, h = 1000.0, 1.0
    beta = 1.0 / T
    r = hotrg.solve("ising", 2, T, 8, 12, field=h, observables=("m", "e"))
    assert abs(r.observables[0] - math.tanh(beta * h)) < 10 * beta ** 2
    assert abs(r.observables[1] + math.tanh(beta)) < 10 * beta ** 2


def test_zero_field_magnetisation_vanishes_by_symmetry():
    r = hotrg.solve("ising", 2, 2.0, 8, 16, observables=("m",))
    assert abs(r.observables[0]) < 1e-10


@pytest.mark.parametrize("T,h,tol_u,tol_m", [(2.0, 1e-8, 1e-4, 3e-4), (2.5, 0.0, 1e-4, 1e-12)])
def test_observables_approach_onsager_and_yang(T, h, tol_u, tol_m):
    """Trend (truncation-dominated): D = 16, 30 steps."""
    r = hotrg.solve("ising", 2, T, 16, 30, field=h, observables=("m", "e"), keep_tensor=False)
    m, e = r.observables
    u = hotrg.internal_energy("ising", 2, e, m, h)
    assert abs(u - exact.onsager_energy(T)) < tol_u
    assert abs(m - exact.yang_magnetisation(T)) < tol_m
