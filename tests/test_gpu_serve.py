"""The solve server on the GPU: results in the mix equal the results alone."""
import pytest

pytestmark = pytest.mark.gpu


def test_results_identical_alone_and_in_the_mix(gpu_lib):
    from paper_2602_05900_amd import binding, serve, workloads
    reqs = [workloads.Request(rid=i, arrival=0.001 * i, model=m, q=q, temperature=t, dmax=d, nsteps=n)
            for i, (m, q, t, d, n) in enumerate([
                ("ising", 2, 2.1, 16, 20), ("potts", 3, 1.05, 16, 24), ("ising", 2, 2.4, 24, 22),
                ("potts", 3, 0.8, 24, 20), ("ising", 2, 1.3, 32, 21), ("ising", 2, 3.0, 16, 40)])]
    alone = {}
    for r in reqs:
        s = binding.Solve(model=r.model, q=r.q, temperature=r.temperature, dmax=r.dmax, max_steps=r.nsteps)
        s.coarse_grain(r.nsteps)
        alone[r.rid] = s.log_z()
        s.close()
    srv = serve.Server(slots=4, budget=8 << 30, precision="fp64")
    done = srv.run(reqs, realtime=False)
    assert len(done) == len(reqs)
    for c in done:
        assert c.lnz_per_site == alone[c.rid], (c.rid, c.lnz_per_site, alone[c.rid])
    assert srv.in_use == 0


def test_grouped_steps_equal_single_handle_steps(gpu_lib):
    """hotrg_coarse_grain_batch: each handle of the group, on its own stream,
    ends bitwise where hotrg_coarse_grain alone takes it; a handle listed twice
    advances twice; a group that would overrun a handle's max_steps is refused
    before anything is enqueued."""
    import torch
    from paper_2602_05900_amd import binding
    cases = [("ising", 2, 2.2, 16), ("potts", 3, 1.0, 12), ("ising", 2, 2.6, 24)]
    alone = []
    for m, q, t, d in cases:
        s = binding.Solve(model=m, q=q, temperature=t, dmax=d, max_steps=24)
        s.coarse_grain(18)
        alone.append(s.log_z())
        s.close()
    solves = [binding.Solve(model=m, q=q, temperature=t, dmax=d, max_steps=24, stream=torch.cuda.Stream())
              for m, q, t, d in cases]
    binding.coarse_grain_batch(solves, 10)
    binding.coarse_grain_batch(solves, 8)
    assert [s.log_z() for s in solves] == alone
    # 18 + 2 * 3 = 24 steps fit; one more round would not, and is refused whole
    binding.coarse_grain_batch([solves[0], solves[0]], 3)
    with pytest.raises(binding.HotrgError) as e:
        binding.coarse_grain_batch([solves[1], solves[0]], 1)
    assert e.value.status == binding.EINVAL
    ref = binding.Solve(model="ising", q=2, temperature=2.2, dmax=16, max_steps=24)
    ref.coarse_grain(24)
    assert solves[0].log_z() == ref.log_z()
    n1 = ctypes_steps(solves[1])
    assert n1 == 18                      # the refused call enqueued nothing
    for s in solves + [ref]:
        s.close()


def ctypes_steps(solve):
    import ctypes
    v, n = ctypes.c_double(), ctypes.c_int()
    assert solve._lib.hotrg_log_z(solve._h, ctypes.byref(v), ctypes.byref(n)) == 0
    return n.value
