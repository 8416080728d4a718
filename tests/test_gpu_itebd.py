"""GPU parity of the batched iTEBD path (include/itebd.h) against the FP64
oracle (oracle/itebd.py) on the same seeded initial states.

FP64 bars: energies per site to 1e-12 relative, bond weights to 1e-10 and
tensors (after the shared sign gauge) to 1e-9 absolute where the singular
values at the cut are distinct (the transverse-field Ising chain); for the
Heisenberg chain, whose Schmidt spectrum has SU(2) multiplets that a cut
can split, energies only, to 1e-9 relative.
"""
import numpy as np
import pytest

from oracle import itebd as oracle
from paper_2602_05900_amd import workloads

pytestmark = pytest.mark.gpu


def gpu_run(h, states, chi, schedule):
    from paper_2602_05900_amd import binding
    c = binding.Chains(h, states, chi)
    for tau, n in schedule:
        c.evolve(tau, n)
    return c


def oracle_run(h, row, chi, schedule):
    st = oracle.unpack(row, chi)
    for tau, n in schedule:
        st = oracle.evolve(st, h, tau, n, chi)
    return st


@pytest.mark.parametrize("chi,nup", [(1, 40), (4, 120), (8, 200), (16, 120), (32, 60)])
def test_tfim_parity(gpu_lib, chi, nup):
    h = workloads.ising_transverse_bond(1.5)
    states = workloads.random_chain_states(3, chi, seed=20 + chi)
    sched = ((0.05, nup),)
    c = gpu_run(h, states, chi, sched)
    e = c.energies()
    got = c.states()
    nb = 2 * chi * chi
    for i in range(3):
        ref = oracle_run(h, states[i], chi, sched)
        er = oracle.energy_per_site(ref, h)
        assert abs(e[i] - er) <= 1e-12 * abs(er)
        g = oracle.unpack(got[i], chi)
        np.testing.assert_allclose(g.l1, ref.l1, atol=1e-10)
        np.testing.assert_allclose(g.l2, ref.l2, atol=1e-10)
        np.testing.assert_allclose(g.B1, ref.B1, atol=1e-9)
        np.testing.assert_allclose(g.B2, ref.B2, atol=1e-9)
    assert c.info()[0] == nup
    assert c.info()[1] < 40


def test_heisenberg_energy_parity_at_the_benchmark_bond_dimension(gpu_lib):
    chi = 30
    h = workloads.heisenberg_bond()
    states = workloads.random_chain_states(2, chi, seed=5)
    sched = ((0.1, 40), (0.02, 40))
    e = gpu_run(h, states, chi, sched).energies()
    for i in range(2):
        er = oracle.energy_per_site(oracle_run(h, states[i], chi, sched), h)
        assert abs(e[i] - er) <= 1e-9 * abs(er)


def test_updated_site_is_right_canonical(gpu_lib):
    """After every update the new left site of the next bond is V_kept^T:
    its rows are orthonormal (sum over physical and right index)."""
    chi = 12
    c = gpu_run(workloads.heisenberg_bond(), workloads.random_chain_states(2, chi, seed=9), chi, ((0.05, 301),))
    for row in c.states():
        B1 = oracle.unpack(row, chi).B1
        R = B1.transpose(1, 0, 2).reshape(chi, -1)
        np.testing.assert_allclose(R @ R.T, np.eye(chi), atol=1e-12)


def test_chains_in_a_batch_are_independent(gpu_lib):
    chi = 8
    h = workloads.ising_transverse_bond(0.7)
    states = workloads.random_chain_states(5, chi, seed=11)
    all5 = gpu_run(h, states, chi, ((0.05, 64),)).states()
    one = gpu_run(h, states[3:4], chi, ((0.05, 64),)).states()
    assert np.array_equal(all5[3], one[0])


def test_gpu_chains_approach_exact_energies(gpu_lib):
    """Trend: transverse-field Ising (g = 1.5, chi = 16) near its exact
    energy and the Heisenberg chain (chi = 32) near the Bethe energy after a
    short tau schedule; every chain of the batch above its ground state."""
    sched = ((0.1, 200), (0.05, 400), (0.01, 1600))
    h = workloads.ising_transverse_bond(1.5)
    e = gpu_run(h, workloads.random_chain_states(4, 16, seed=1), 16, sched).energies()
    ex = oracle.tfim_energy(1.5)
    assert np.all(e > ex) and np.all(e - ex < 1.5e-3)
    h = workloads.heisenberg_bond()
    e = gpu_run(h, workloads.random_chain_states(4, 32, seed=2), 32, sched).energies()
    assert np.all(e > oracle.BETHE_HEISENBERG) and np.all(e - oracle.BETHE_HEISENBERG < 1.5e-3)


def test_work_counters_are_consistent(gpu_lib):
    """itebd_work: at least one Jacobi sweep per update and chain, at most
    n (n - 1) / 2 rotations per sweep (n = 2 chi), monotone across launches."""
    chi, batch = 8, 4
    h = workloads.heisenberg_bond()
    from paper_2602_05900_amd import binding
    c = binding.Chains(h, workloads.random_chain_states(batch, chi, seed=31), chi)
    assert c.work() == (0.0, 0.0)
    c.evolve(0.05, 50)
    sw1, rot1 = c.work()
    c.evolve(0.05, 30)
    sw2, rot2 = c.work()
    n = 2 * chi
    assert batch * 50 <= sw1 <= batch * 50 * 64 and 0 < rot1 <= sw1 * n * (n - 1) / 2
    assert sw2 - sw1 >= batch * 30 and rot2 >= rot1
    assert sw1 == int(sw1) and rot1 == int(rot1)
    c.close()


def test_benchmark_configuration_sampled_chains(gpu_lib):
    """The benchmark's launch configuration: 512 Heisenberg chains (two per
    CU) at D_b = 30 under its warm-up schedule.  Sampled chains (first,
    middle, last) against the oracle run one by one, to the Heisenberg bar
    (1e-9 relative: SU(2) multiplets make the kept basis non-unique); the
    last chain bitwise equal to the same chain run alone; every chain finite
    and above the Bethe energy."""
    chi, batch = 30, 512
    h = workloads.heisenberg_bond()
    states = workloads.random_chain_states(batch, chi, seed=2026)
    sched = ((0.1, 96),)
    c = gpu_run(h, states, chi, sched)
    e = c.energies()
    got = c.states()
    c.close()
    assert np.all(np.isfinite(e)) and np.all(e > oracle.BETHE_HEISENBERG)
    for i in (0, 255, 511):
        er = oracle.energy_per_site(oracle_run(h, states[i], chi, sched), h)
        assert abs(e[i] - er) <= 1e-9 * abs(er), i
    one = gpu_run(h, states[511:512], chi, sched).states()
    assert np.array_equal(got[511], one[0])


def test_zero_updates_leave_the_states_unchanged(gpu_lib):
    """Degenerate call: nupdates = 0 launches nothing; the states read back
    are the uploaded ones, bit for bit, and the counters stay at zero."""
    from paper_2602_05900_amd import binding
    chi = 7
    states = workloads.random_chain_states(3, chi, seed=41)
    c = binding.Chains(workloads.heisenberg_bond(), states, chi)
    c.evolve(0.1, 0)
    assert np.array_equal(c.states(), states)
    assert c.info()[0] == 0 and c.work() == (0.0, 0.0)
    c.close()


def test_benchmark_launch_configuration_elementwise_tfim(gpu_lib):
    """512 chains (two per CU) at D_b = 30, the benchmark's launch
    configuration, on the transverse-field Ising chain (g = 1.5, distinct
    Schmidt values): sampled chains element by element against the oracle,
    weights to 1e-10 and tensors to 1e-9 after the shared sign gauge.  The
    samples (two from each half of the batch) have kept Schmidt values at
    least 3e-6 apart, so the oracle's LAPACK vectors, accurate to about
    eps / gap, are good to ~1e-10; chains with gaps near 1e-8 (which the
    one-sided Jacobi resolves better than LAPACK) are not used."""
    chi, batch = 30, 512
    h = workloads.ising_transverse_bond(1.5)
    states = workloads.random_chain_states(batch, chi, seed=77)
    sched = ((0.05, 64),)
    c = gpu_run(h, states, chi, sched)
    got = c.states()
    e = c.energies()
    c.close()
    for i in (1, 100, 400, 510):
        ref = oracle_run(h, states[i], chi, sched)
        gaps = [np.min(np.abs(np.diff(np.sort(lam)))) for lam in (ref.l1, ref.l2)]
        assert min(gaps) > 3e-6, (i, gaps)
        g = oracle.unpack(got[i], chi)
        np.testing.assert_allclose(g.l1, ref.l1, atol=1e-10)
        np.testing.assert_allclose(g.l2, ref.l2, atol=1e-10)
        np.testing.assert_allclose(g.B1, ref.B1, atol=1e-9)
        np.testing.assert_allclose(g.B2, ref.B2, atol=1e-9)
        er = oracle.energy_per_site(ref, h)
        assert abs(e[i] - er) <= 1e-12 * abs(er)


def test_vanishing_chain_is_frozen_and_reported_others_unaffected(gpu_lib):
    """A chain whose state is all zeros contracts to a zero pair: its kept
    singular values have zero norm, so its status word gets
    ITEBD_CHAIN_NONFINITE, the update is not applied (the state row stays
    as uploaded) and itebd_energy / itebd_info return ENONFINITE.  The
    batch's other chains are bitwise what they are without it.  Every
    kernel runs to its normal end (a zero matrix needs no rotation)."""
    from paper_2602_05900_amd import binding
    chi = 8
    h = workloads.ising_transverse_bond(1.5)
    states = workloads.random_chain_states(3, chi, seed=13)
    states[1] = 0.0
    c = binding.Chains(h, states, chi)
    c.evolve(0.05, 40)
    with pytest.raises(binding.HotrgError) as e:
        c.energies()
    assert e.value.status == binding.ENONFINITE
    with pytest.raises(binding.HotrgError) as e:
        c.info()
    assert e.value.status == binding.ENONFINITE
    assert list(c.status()) == [0, binding.ITEBD_CHAIN_NONFINITE, 0]
    got = c.states()
    assert np.array_equal(got[1], states[1])
    c.close()
    alone = gpu_run(h, states[[0, 2]], chi, ((0.05, 40),))
    assert list(alone.status()) == [0, 0]
    assert np.array_equal(alone.states(), got[[0, 2]])
    alone.close()


def test_sweep_limit_is_reported(gpu_lib):
    """With a limit of one Jacobi sweep no decomposition can be recognised
    as converged (that takes a sweep without rotations): every chain's
    status word gets ITEBD_CHAIN_SWEEP_CAP and the synchronising calls
    return EEIG, while the updates are still applied and stay finite.  The
    default limit reports nothing; limits outside 1..ITEBD_MAX_SWEEPS are
    rejected."""
    from paper_2602_05900_amd import binding
    chi = 8
    h = workloads.heisenberg_bond()
    states = workloads.random_chain_states(2, chi, seed=17)
    c = binding.Chains(h, states, chi)
    for bad in (0, binding.ITEBD_MAX_SWEEPS + 1):
        with pytest.raises(binding.HotrgError) as e:
            c.set_max_sweeps(bad)
        assert e.value.status == binding.EINVAL
    c.set_max_sweeps(1)
    c.evolve(0.05, 4)
    with pytest.raises(binding.HotrgError) as e:
        c.info()
    assert e.value.status == binding.EEIG
    assert list(c.status()) == [binding.ITEBD_CHAIN_SWEEP_CAP] * 2
    assert np.all(np.isfinite(c.states()))
    c.close()
    d = gpu_run(h, states, chi, ((0.05, 4),))
    assert d.info()[0] == 4 and list(d.status()) == [0, 0]
    d.close()
