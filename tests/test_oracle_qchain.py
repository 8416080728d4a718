"""Pins of the quantum-chain HOTRG oracle (oracle/qchain.py) and of the
axis schedule of the HOTRG oracle: exact diagonalisation of Trotterized
rings, exact network contractions for non-alternating schedules, the
thermodynamic limit of rings, the free-fermion free energy of the
transverse-field Ising chain, and the high- and low-temperature limits of
the Heisenberg chain."""
import math

import numpy as np
import pytest

from oracle import exact, hotrg, itebd, qchain
from paper_2602_05900_amd import workloads


def torus_of(schedule):
    """(Lx, Ly) covered after the given exchange flags (first merge along y)."""
    Lx, Ly, swapped = 1, 1, False
    for e in schedule:
        if swapped:
            Lx *= 2
        else:
            Ly *= 2
        if e:
            swapped = not swapped
    return Lx, Ly


@pytest.mark.parametrize("sched", [[False], [False, False], [True, False], [False, True, False], [True, True]])
def test_schedule_is_exact_without_truncation(sched):
    T = np.random.default_rng(1).uniform(0.1, 1.0, (2, 2, 2, 2))
    Lx, Ly = torus_of(sched)
    r = hotrg.solve_tensor(T, 10 ** 6, len(sched), schedule=sched)
    assert abs(r.lnz_per_site * 2 ** len(sched) - exact.network_lnz(T, Lx, Ly)) < 1e-12


@pytest.mark.parametrize("model", ["heisenberg", "tfim"])
@pytest.mark.parametrize("Lb,M", [(1, 1), (1, 2), (2, 1), (2, 2), (3, 2), (2, 3)])
def test_block_tensor_network_is_the_trotterized_ring(model, Lb, M):
    """The network of Lb x M block tensors is Tr (G_odd G_even)^M of a ring of
    2 Lb spins (exact diagonalisation, gate by scipy's expm)."""
    h = workloads.heisenberg_bond() if model == "heisenberg" else workloads.ising_transverse_bond(1.5)
    tau = 0.1
    T = qchain.block_tensor(h, tau)
    assert T.shape == (4, 4, 4, 4)
    assert abs(exact.network_lnz(T, Lb, M) - exact.trotter_ring_lnz(h, tau, 2 * Lb, M)) < 1e-12


def test_chain_closure_is_the_limit_of_long_rings():
    """Without truncation, ln Z per tensor of the infinite chain (dominant
    eigenvalue of the column transfer matrix) is the limit of rings of L
    sites, approached exponentially."""
    h = workloads.ising_transverse_bond(1.5)
    tau = 0.25
    c = qchain.chain_lnz(qchain.block_tensor(h, tau), 10 ** 6, 1)
    d = [exact.trotter_ring_lnz(h, tau, L, 2) / L - c for L in (6, 8, 10, 12)]
    assert all(abs(a) > abs(b) for a, b in zip(d, d[1:]))
    assert abs(d[-1]) < 2e-6


@pytest.mark.parametrize("T", [1.0, 0.5])
def test_tfim_free_energy_matches_free_fermions(T):
    """Finite temperature: beta = 2^k tau, the Trotter error shrinking with tau^2."""
    h = workloads.ising_transverse_bond(1.5)
    ex = exact.tfim_free_energy(1.5, T)
    errs = [abs(qchain.free_energy(h, (1.0 / T) / 2 ** k, 16, k) - ex) for k in (6, 8, 10)]
    assert errs[0] > errs[1] > errs[2] and errs[2] < 2e-6


def test_tfim_free_energy_closed_form_limits():
    assert abs(exact.tfim_free_energy(1.5, 1e-3) - itebd.tfim_energy(1.5)) < 1e-9   # T -> 0
    T = 1e3
    assert abs(exact.tfim_free_energy(1.5, T) + T * math.log(2.0)) < 1e-2          # T -> infinity


def test_heisenberg_high_temperature_series():
    """f = -T ln 2 - 3 J^2 / (32 T) + O(T^-2): the remainder falls as 1/T^2."""
    h = workloads.heisenberg_bond()
    rem = []
    for T in (20.0, 40.0):
        f = qchain.free_energy(h, (1.0 / T) / 2 ** 8, 16, 8)
        rem.append(abs(f - (-T * math.log(2.0) - 3.0 / (32.0 * T))))
    assert rem[0] < 1e-4 and 3.0 < rem[0] / rem[1] < 5.0


def test_heisenberg_low_temperature_approaches_bethe():
    f = qchain.free_energy(workloads.heisenberg_bond(), 0.05, 16, 14)   # beta = 819
    assert 0.0 < f - itebd.BETHE_HEISENBERG < 2.5e-3


def test_alternating_merges_approach_the_ground_state_energy():
    """Merging along both axes (beta -> infinity) gives the ground-state
    energy per site: for the transverse-field Ising chain at g = 1.5 it lies
    above the free-fermion value and approaches it as D grows."""
    h = workloads.ising_transverse_bond(1.5)
    exact_e = itebd.tfim_energy(1.5)
    e16 = qchain.ground_energy(h, 0.02, 16, 16) - exact_e
    e24 = qchain.ground_energy(h, 0.02, 24, 16) - exact_e
    assert 0.0 < e24 < e16 < 3e-3
