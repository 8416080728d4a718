"""Failure handling on the device: errors latched in the device status word
(HOTRG_EEIG, HOTRG_ENONFINITE), returned by the next synchronising call,
first error sticking, and other solves unaffected.  Every condition is
reached with valid inputs and forced from the host (a pass cap of 1 for the
eigensolver, a tensor whose stacked pair contracts to zero), so every kernel
still runs to its normal end.

The eigensolver's stop reasons (hotrg_eig_info): converging solves report
HOTRG_EIG_CONVERGED at every step; the quantum chain's first truncated steps,
whose kept pairs lie in the rounding noise of a nearly rank-deficient
environment, stop on stagnation below the failure bound and report
HOTRG_EIG_STAGNATED without an error.
"""
import numpy as np
import pytest

from paper_2602_05900_amd import workloads

pytestmark = pytest.mark.gpu


def test_pass_cap_one_latches_eeig_and_it_sticks(gpu_lib):
    """Ising D = 48 with one subspace pass per eigensolve and a failure bound
    of 1e-6: step 5 (n = 256, the first subspace solve) stops far from
    convergence, HOTRG_EEIG is latched, and it is what every later
    synchronising call returns, also after more steps have run."""
    from paper_2602_05900_amd import binding
    s = binding.Solve(model="ising", q=2, temperature=2.25, dmax=48, max_steps=12)
    s.set_eig_limits(max_passes=1, fail_residual=1e-6)
    s.coarse_grain(6)
    with pytest.raises(binding.HotrgError) as e:
        s.log_z()
    assert e.value.status == binding.EEIG
    s.coarse_grain(6)              # later steps still run to their end
    for call in (s.log_z, lambda: s.step_info(1), lambda: s.eig_info(5), s.tensor):
        with pytest.raises(binding.HotrgError) as e:
            call()
        assert e.value.status == binding.EEIG
    # a reset clears the status and restores the default limits
    s.reset(model="ising", q=2, temperature=2.25, dmax=48, max_steps=12)
    s.coarse_grain(12)
    assert np.isfinite(s.log_z())
    assert all(s.eig_stop(n) == binding.EIG_CONVERGED for n in range(1, 13))
    s.close()


def test_pass_cap_below_failure_bound_is_reported_not_latched(gpu_lib):
    """The same cap with a failure bound above any finite residual: no
    error, and the stop reason says the pass cap ended the solve, with the
    residual of an unconverged block (above the 1e-6 of the test above)."""
    from paper_2602_05900_amd import binding
    s = binding.Solve(model="ising", q=2, temperature=2.25, dmax=48, max_steps=6)
    s.set_eig_limits(max_passes=1, fail_residual=1e300)
    s.coarse_grain(6)
    assert np.isfinite(s.log_z())
    assert [s.eig_stop(n) for n in range(1, 5)] == [binding.EIG_CONVERGED] * 4     # dense Jacobi
    assert s.eig_stop(5) == binding.EIG_PASS_CAP
    it, _, res = s.eig_info(5)
    print(f"one pass: residual {res:.2e}")
    assert it == 1 and res > 1e-6
    s.close()


def test_invalid_limits_are_rejected(gpu_lib):
    from paper_2602_05900_amd import binding
    s = binding.Solve(model="ising", q=2, temperature=2.0, dmax=8)
    for mp, fr in ((0, 1e-6), (binding.EIG_MAX_PASSES + 1, 1e-6), (5, 0.0), (5, float("nan"))):
        with pytest.raises(binding.HotrgError) as e:
            s.set_eig_limits(mp, fr)
        assert e.value.status == binding.EINVAL
    s.close()


def test_stagnation_is_visible_and_not_an_error(gpu_lib):
    from paper_2602_05900_amd import binding
    k = 12
    s = binding.Solve(model="qchain", bond_h=workloads.heisenberg_bond(), tau=1.0 / 2 ** k, dmax=32, max_steps=k)
    s.coarse_grain(k, exchange=False)
    assert np.isfinite(s.log_z_chain())
    stops = [s.eig_stop(n) for n in range(1, k + 1)]
    assert binding.EIG_STAGNATED in stops
    for n, st in enumerate(stops, start=1):
        if st == binding.EIG_STAGNATED:
            assert 1e-12 < s.eig_info(n)[2] <= 1e-6
    assert binding.EIG_PASS_CAP not in stops
    s.close()


def vanishing_pair_tensor(dx=3, seed=11):
    """T[l, r, d, u] nonzero only for d = 0, u = 1: stacked vertically, the
    bottom copy's u leg (bond k = 1) never meets a nonzero entry of the top
    copy's d leg (k = 0), so the merged pair, E and T' are all zero and
    c_1 = 0."""
    T = np.zeros((dx, dx, 2, 2))
    T[:, :, 0, 1] = np.random.default_rng(seed).uniform(0.5, 1.5, (dx, dx))
    return T


@pytest.mark.parametrize("precision", ["fp64", "bf16x6"])
def test_zero_normalisation_latches_enonfinite_other_solve_unaffected(gpu_lib, precision):
    import torch
    from paper_2602_05900_amd import binding
    # the reference: an Ising solve alone on its own stream
    sa = torch.cuda.Stream()
    ref = binding.Solve(model="ising", q=2, temperature=2.1, dmax=16, stream=sa, max_steps=20)
    ref.coarse_grain(20)
    want = ref.log_z()
    ref.close()
    # the failing solve and the same Ising solve, interleaved on two streams
    sb, sc = torch.cuda.Stream(), torch.cuda.Stream()
    bad = binding.Solve(model="custom", tensor=vanishing_pair_tensor(), dmax=4, temperature=1.0,
                        precision=precision, stream=sb, max_steps=3)
    good = binding.Solve(model="ising", q=2, temperature=2.1, dmax=16, stream=sc, max_steps=20)
    binding.coarse_grain_batch([bad, good], 3)
    good.coarse_grain(17)
    with pytest.raises(binding.HotrgError) as e:
        bad.log_z()
    assert e.value.status == binding.ENONFINITE
    with pytest.raises(binding.HotrgError) as e:
        bad.step_info(1)
    assert e.value.status == binding.ENONFINITE
    assert good.log_z() == want            # bitwise: no shared state between solves
    bad.close()
    good.close()
