"""Pins of the iTEBD oracle (oracle/itebd.py) against closed forms,
exactly known states, invariants of the update and the exact solutions of
the transverse-field Ising and Heisenberg chains."""
import math

import numpy as np
import pytest

from oracle import itebd
from paper_2602_05900_amd import workloads


def test_bond_hamiltonians_spectra():
    w = np.linalg.eigvalsh(workloads.heisenberg_bond())
    np.testing.assert_allclose(w, [-0.75, 0.25, 0.25, 0.25], atol=1e-15)     # singlet, triplet
    # transverse-field Ising bond at g = 0: sz sz only
    np.testing.assert_allclose(np.diag(workloads.ising_transverse_bond(0.0)), [-1, 1, 1, -1], atol=0)


def test_gate_closed_form_heisenberg():
    """exp(-tau S.S) = e^{-tau/4} P_triplet + e^{3 tau/4} P_singlet."""
    tau = 0.37
    s = np.array([0.0, 1.0, -1.0, 0.0]) / math.sqrt(2.0)
    Ps = np.outer(s, s)
    want = math.exp(-tau / 4) * (np.eye(4) - Ps) + math.exp(3 * tau / 4) * Ps
    np.testing.assert_allclose(itebd.gate(workloads.heisenberg_bond(), tau), want, rtol=1e-14, atol=1e-15)


def test_tfim_closed_form_special_points():
    assert abs(itebd.tfim_energy(0.0) + 1.0) < 1e-12            # classical ferromagnet
    assert abs(itebd.tfim_energy(1.0) + 4.0 / math.pi) < 1e-9    # critical point
    g = 50.0                                                     # deep paramagnet: -g - 1/(4g) + O(g^-3)
    assert abs(itebd.tfim_energy(g) - (-g - 1.0 / (4.0 * g))) < 1e-5


def test_energy_of_known_states():
    h = workloads.heisenberg_bond()
    up, dn = np.array([1.0, 0.0]), np.array([0.0, 1.0])
    one = np.ones(1)
    # Neel product state: <S.S> = -1/4 on every bond
    neel = itebd.ChainState(B1=up.reshape(2, 1, 1), B2=dn.reshape(2, 1, 1), l1=one, l2=one)
    assert abs(itebd.energy_per_site(neel, h) + 0.25) < 1e-15
    ferro = itebd.ChainState(B1=up.reshape(2, 1, 1), B2=up.reshape(2, 1, 1), l1=one, l2=one)
    assert abs(itebd.energy_per_site(ferro, h) - 0.25) < 1e-15
    # singlets on the A-B bonds: -3/4 on those bonds, 0 on the others
    B1 = np.zeros((2, 2, 2))
    B2 = np.zeros((2, 2, 2))
    for s in range(2):
        B1[s, 0, s] = 1.0
    eps = np.array([[0.0, 1.0], [-1.0, 0.0]]) / math.sqrt(2.0)
    for t in range(2):
        for c in range(2):
            B2[t, c, 0] = eps[c, t]
    dimer = itebd.ChainState(B1=B1, B2=B2, l1=np.full(2, 1 / math.sqrt(2)), l2=np.array([1.0, 0.0]))
    assert abs(itebd.energy_per_site(dimer, h) + 0.375) < 1e-15


def test_update_without_truncation_reconstructs_the_evolved_pair():
    """Keeping every singular value, B1' B2' is the gated pair psi' divided
    by |S|; B2' has orthonormal rows; lambda' is sorted and normalised."""
    chi = 3
    st = itebd.unpack(workloads.random_chain_states(1, chi, seed=4)[0], chi)
    h = workloads.heisenberg_bond()
    G = itebd.gate(h, 0.2)
    psi = np.einsum("uvst,astb->auvb", G.reshape(2, 2, 2, 2), np.einsum("sac,tcb->astb", st.B1, st.B2))
    nxt = itebd.bond_update(st, G, chi=2 * chi)       # roles exchanged: B2 of nxt is the new B1
    B1n, B2n, l1n = nxt.B2, nxt.B1, nxt.l2
    M = st.l2[:, None, None, None] * psi
    nrm = math.sqrt(float(np.sum(np.linalg.svd(M.reshape(2 * chi, 2 * chi), compute_uv=False) ** 2)))
    rec = np.einsum("sac,tcb->astb", B1n, B2n)
    np.testing.assert_allclose(rec, psi / nrm, rtol=1e-12, atol=1e-13)
    R = B2n.transpose(1, 0, 2).reshape(B2n.shape[1], -1)
    np.testing.assert_allclose(R @ R.T, np.eye(R.shape[0]), atol=1e-13)
    assert np.all(np.diff(l1n) <= 0) and abs(np.sum(l1n ** 2) - 1.0) < 1e-14
    assert np.allclose(nxt.l1, st.l2)


def test_truncated_update_keeps_right_canonical_rows_and_swaps_roles():
    chi = 4
    st = itebd.unpack(workloads.random_chain_states(1, chi, seed=5)[0], chi)
    nxt = itebd.bond_update(st, itebd.gate(workloads.heisenberg_bond(), 0.1), chi)
    R = nxt.B1.transpose(1, 0, 2).reshape(chi, -1)             # the new B2' (right-canonical)
    np.testing.assert_allclose(R @ R.T, np.eye(chi), atol=1e-13)
    assert nxt.B1.shape == nxt.B2.shape == (2, chi, chi) and nxt.updates == 1


def test_classical_limit_reaches_the_ferromagnet():
    """g = 0: the ground state is a product state of energy -J exactly."""
    chi = 4
    st = itebd.unpack(workloads.random_chain_states(1, chi, seed=6)[0], chi)
    h = workloads.ising_transverse_bond(0.0)
    st = itebd.evolve(st, h, 0.1, 600, chi)
    assert abs(itebd.energy_per_site(st, h) + 1.0) < 1e-10


def test_tfim_approaches_the_exact_energy_linearly_in_tau():
    """Gapped chain (g = 1.5), chi = 8: the fixed-point error of the
    first-order splitting shrinks in proportion to tau."""
    chi, g = 8, 1.5
    h = workloads.ising_transverse_bond(g)
    exact = itebd.tfim_energy(g)
    st = itebd.unpack(workloads.random_chain_states(1, chi, seed=7)[0], chi)
    errs = []
    for tau, n in ((0.04, 1000), (0.02, 1600), (0.01, 3200)):
        st = itebd.evolve(st, h, tau, n, chi)
        errs.append(itebd.energy_per_site(st, h) - exact)
    assert all(e > 0 for e in errs)                    # variational: above the ground state
    assert 1.6 < errs[0] / errs[1] < 2.4 and 1.6 < errs[1] / errs[2] < 2.4
    assert errs[2] < 1.5e-3


def test_heisenberg_approaches_bethe():
    """Critical chain at chi = 16: the energy stays above 1/4 - ln 2 and
    approaches it as tau shrinks (the splitting error dominates here)."""
    chi = 16
    h = workloads.heisenberg_bond()
    st = itebd.unpack(workloads.random_chain_states(1, chi, seed=8)[0], chi)
    errs = []
    for tau, n in ((0.1, 200), (0.05, 400), (0.01, 1600)):
        st = itebd.evolve(st, h, tau, n, chi)
        errs.append(itebd.energy_per_site(st, h) - itebd.BETHE_HEISENBERG)
    assert 0 < errs[2] < errs[1] < errs[0] and errs[2] < 1.5e-3
