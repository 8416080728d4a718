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


def _polled(solve, nsteps, exchange=True, extra=0):
    """Advance `solve` by nsteps host-polled steps; returns the poll states seen."""
    from paper_2602_05900_amd import binding
    seen = []
    for _ in range(nsteps):
        if not solve.step_begin(exchange, extra):
            seen.append("whole")
            continue
        while True:
            st = solve.step_poll()
            seen.append(st)
            if st == binding.POLL_STEPPED:
                break
    assert solve.step_poll() == binding.POLL_IDLE
    return seen


@pytest.mark.parametrize("model,q,t,d,prec,n,extra", [
    ("ising", 2, 2.25, 24, "fp64", 14, 0),
    ("potts", 3, 1.0, 16, "fp64", 12, 1),
    ("ising", 2, 2.3, 32, "bf16x6", 10, 0),
    ("ising", 2, 2.269185314213022, 48, "fp16x3", 9, 2),
])
def test_polled_steps_equal_whole_steps(gpu_lib, model, q, t, d, prec, n, extra):
    """hotrg_step_begin / hotrg_step_poll enqueue the same passes as a whole
    step, minus those after convergence: ln Z, every c_n and the eigensolver
    record (passes used, residual, stop reason) are bitwise those of
    hotrg_coarse_grain."""
    from paper_2602_05900_amd import binding
    ref = binding.Solve(model=model, q=q, temperature=t, dmax=d, precision=prec, max_steps=n)
    ref.coarse_grain(n)
    s = binding.Solve(model=model, q=q, temperature=t, dmax=d, precision=prec, max_steps=n)
    seen = _polled(s, n, extra=extra)
    assert binding.POLL_STEPPED in seen and "whole" in seen
    assert s.log_z() == ref.log_z()
    for k in range(1, n + 1):
        assert s.step_info(k) == ref.step_info(k), k
        assert s.eig_info(k) == ref.eig_info(k), k
    s.close()
    ref.close()


def test_polled_quantum_chain_and_pass_cap(gpu_lib):
    """Steps without the axis exchange (quantum chain) and a pass cap below
    what the eigensolve needs: the polled form stops at the same pass and
    latches the same status as the whole-step form."""
    from paper_2602_05900_amd import binding, workloads
    h = workloads.heisenberg_bond()
    tau, k = 2.0 ** -8, 8
    ref = binding.Solve(model="qchain", bond_h=h, tau=tau, dmax=24, max_steps=k)
    ref.coarse_grain(k, exchange=False)
    s = binding.Solve(model="qchain", bond_h=h, tau=tau, dmax=24, max_steps=k)
    _polled(s, k, exchange=False)
    assert s.log_z_chain() == ref.log_z_chain()
    s.close()
    ref.close()
    outs = []
    for polled in (False, True):
        s = binding.Solve(model="ising", q=2, temperature=2.269185314213022, dmax=24, max_steps=12)
        s.set_eig_limits(3, 1e-30)       # stops at pass 3; any residual above 1e-30 fails
        if polled:
            _polled(s, 12)
        else:
            s.coarse_grain(12)
        with pytest.raises(binding.HotrgError) as e:
            s.log_z()
        outs.append(e.value.status)
        s.close()
    assert outs[0] == outs[1] == binding.EEIG


def test_polled_pending_step_blocks_whole_steps(gpu_lib):
    import torch
    from paper_2602_05900_amd import binding
    s = binding.Solve(model="ising", q=2, temperature=2.3, dmax=24, max_steps=10)
    s.coarse_grain(4)                    # step 5 is the first with Dx^2 > 96
    assert s.step_begin()
    with pytest.raises(binding.HotrgError) as e:
        s.coarse_grain(1)
    assert e.value.status == binding.EINVAL
    with pytest.raises(binding.HotrgError):
        s.step_begin()
    torch.cuda.synchronize()
    while s.step_poll() != binding.POLL_STEPPED:
        pass
    s.coarse_grain(1)
    ref = binding.Solve(model="ising", q=2, temperature=2.3, dmax=24, max_steps=10)
    ref.coarse_grain(6)
    assert s.log_z() == ref.log_z()
    s.close()
    ref.close()


def test_polled_server_results_identical_alone_and_in_the_mix(gpu_lib):
    from paper_2602_05900_amd import binding, serve, workloads
    reqs = [workloads.Request(rid=i, arrival=0.001 * i, model=m, q=q, temperature=t, dmax=d, nsteps=n)
            for i, (m, q, t, d, n) in enumerate([
                ("ising", 2, 2.1, 16, 20), ("potts", 3, 1.05, 16, 24), ("ising", 2, 2.4, 24, 22),
                ("potts", 3, 0.8, 24, 20), ("ising", 2, 1.3, 32, 21), ("ising", 2, 2.27, 48, 20)])]
    alone = {}
    for r in reqs:
        s = binding.Solve(model=r.model, q=r.q, temperature=r.temperature, dmax=r.dmax, max_steps=r.nsteps,
                          precision="fp16x3")
        s.coarse_grain(r.nsteps)
        alone[r.rid] = s.log_z()
        s.close()
    srv = serve.Server(slots=4, budget=32 << 30, precision="fp16x3", stepping="polled")
    done = srv.run(reqs, realtime=False)
    assert len(done) == len(reqs)
    for c in done:
        assert c.lnz_per_site == alone[c.rid], (c.rid, c.lnz_per_site, alone[c.rid])
    assert srv.in_use == 0


@pytest.mark.parametrize("model,q,t,d,prec,n", [
    ("ising", 2, 2.25, 24, "fp64", 14),
    ("ising", 2, 2.269185314213022, 48, "fp16x3", 9),
    ("potts", 3, 0.9, 32, "bf16x6", 12),
])
def test_engine_steps_equal_whole_steps(gpu_lib, model, q, t, d, prec, n):
    """hotrg_coarse_grain_async: the library's progress thread drives the
    host-polled steps of several handles at once (one stream each); every
    handle ends bitwise where hotrg_coarse_grain takes it, with the same c_n
    and eigensolver records, and log_z right after the call waits for the
    thread."""
    import torch
    from paper_2602_05900_amd import binding
    temps = [t, t * 1.03, t * 0.97]
    refs = []
    for tt in temps:
        r = binding.Solve(model=model, q=q, temperature=tt, dmax=d, precision=prec, max_steps=n)
        r.coarse_grain(n)
        refs.append(r)
    solves = [binding.Solve(model=model, q=q, temperature=tt, dmax=d, precision=prec, max_steps=n,
                            stream=torch.cuda.Stream()) for tt in temps]
    for s in solves:
        s.coarse_grain_async(n)
    assert solves[0].log_z() == refs[0].log_z()
    for s, r in zip(solves, refs):
        assert s.log_z() == r.log_z()
        assert not s.async_busy()
        for k in range(1, n + 1):
            assert s.step_info(k) == r.step_info(k), k
            assert s.eig_info(k) == r.eig_info(k), k
    for s in solves + refs:
        s.close()


def test_engine_quantum_chain_and_continuation(gpu_lib):
    """Steps without the axis exchange, and an asynchronous run continued
    by whole steps and by a second asynchronous run."""
    from paper_2602_05900_amd import binding, workloads
    h = workloads.heisenberg_bond()
    tau, k = 2.0 ** -8, 8
    ref = binding.Solve(model="qchain", bond_h=h, tau=tau, dmax=24, max_steps=k)
    ref.coarse_grain(k, exchange=False)
    s = binding.Solve(model="qchain", bond_h=h, tau=tau, dmax=24, max_steps=k)
    s.coarse_grain_async(k, exchange=False)
    assert s.log_z_chain() == ref.log_z_chain()
    s.close()
    ref.close()
    ref = binding.Solve(model="ising", q=2, temperature=2.3, dmax=24, max_steps=16)
    ref.coarse_grain(16)
    s = binding.Solve(model="ising", q=2, temperature=2.3, dmax=24, max_steps=16)
    s.coarse_grain_async(7)
    s.coarse_grain(2)                     # waits for the thread, then whole steps
    s.coarse_grain_async(7, extra=2)
    with pytest.raises(binding.HotrgError) as e:
        s.coarse_grain_async(1)           # would exceed max_steps
    assert e.value.status == binding.EINVAL
    assert s.log_z() == ref.log_z()
    s.close()
    ref.close()


@pytest.mark.parametrize("stepping", ["engine", "hybrid"])
def test_engine_server_results_identical_alone_and_in_the_mix(gpu_lib, stepping):
    from paper_2602_05900_amd import binding, serve, workloads
    reqs = [workloads.Request(rid=i, arrival=0.001 * i, model=m, q=q, temperature=t, dmax=d, nsteps=n)
            for i, (m, q, t, d, n) in enumerate([
                ("ising", 2, 2.1, 16, 20), ("potts", 3, 1.05, 16, 24), ("ising", 2, 2.4, 24, 22),
                ("potts", 3, 0.8, 24, 20), ("ising", 2, 1.3, 32, 21), ("ising", 2, 2.27, 48, 20)])]
    alone = {}
    for r in reqs:
        s = binding.Solve(model=r.model, q=r.q, temperature=r.temperature, dmax=r.dmax, max_steps=r.nsteps,
                          precision="fp16x3")
        s.coarse_grain(r.nsteps)
        alone[r.rid] = s.log_z()
        s.close()
    srv = serve.Server(slots=4, budget=32 << 30, precision="fp16x3", stepping=stepping)
    done = srv.run(reqs, realtime=False)
    assert len(done) == len(reqs)
    for c in done:
        assert c.lnz_per_site == alone[c.rid], (c.rid, c.lnz_per_site, alone[c.rid])
    assert srv.in_use == 0


@pytest.mark.parametrize("d,prec,n", [(24, "fp64", 16), (32, "bf16x6", 12)])
def test_polled_and_engine_two_sided_with_observables(gpu_lib, d, prec, n):
    """Two-sided handles with both impurity tensors: host-polled steps (the
    left eigensolve, then the right one, then the products) and the progress
    thread give bitwise the results of whole steps: ln Z, the observables,
    both sides' truncation errors and the side applied, every c_n and
    eigensolver record."""
    from paper_2602_05900_amd import binding
    kw = dict(model="ising", q=2, temperature=2.2, dmax=d, precision=prec, max_steps=n, field=1e-8,
              two_sided=True, observables=("m", "e"))
    ref = binding.Solve(**kw)
    ref.coarse_grain(n)
    polled = binding.Solve(**kw)
    seen = _polled(polled, n)
    assert seen.count(binding.POLL_STEPPED) + seen.count("whole") == n
    engine = binding.Solve(**kw)
    engine.coarse_grain_async(n)
    for s in (polled, engine):
        assert s.log_z() == ref.log_z()
        assert s.observables() == ref.observables()
        for k in range(1, n + 1):
            assert s.step_sides(k) == ref.step_sides(k), k
            assert s.step_info(k) == ref.step_info(k), k
            assert s.eig_info(k) == ref.eig_info(k), k
    for s in (ref, polled, engine):
        s.close()
