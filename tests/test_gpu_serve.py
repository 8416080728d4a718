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
