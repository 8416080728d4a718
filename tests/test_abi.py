"""CPU checks of the C ABI: the header is valid C, the library loads without a
GPU and exports every function include/hotrg.h declares, and the host-only
entry points (workspace sizing, parameter validation, strings) behave."""
import ctypes
import glob
import os
import re
import subprocess
import tempfile

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hotrg.h")


def declared_functions():
    """Every function declared in include/*.h (hotrg_* and itebd_*)."""
    names = set()
    for h in sorted(glob.glob(os.path.join(ROOT, "include", "*.h"))):
        text = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"\b((?:hotrg|itebd)_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    from paper_2602_05900_amd import binding, build
    if not os.path.exists(binding.LIB_PATH):
        build.build()
    return binding.load()


def test_header_is_plain_c():
    src = ('#include "hotrg.h"\n#include "itebd.h"\n'
           'int main(void) { hotrg_params p; (void)p; return HOTRG_OK + (int)itebd_state_len(1); }\n')
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        open(c, "w").write(src)
        r = subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-pedantic", "-I", os.path.dirname(HEADER),
                            "-c", c, "-o", os.path.join(d, "t.o")], capture_output=True, text=True)
        assert r.returncode == 0, r.stderr


def test_every_declared_function_is_exported(lib):
    names = declared_functions()
    assert "hotrg_init_tensor" in names and "hotrg_coarse_grain" in names and "hotrg_log_z" in names
    assert "itebd_init" in names and "itebd_evolve" in names
    from paper_2602_05900_amd import binding
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(binding.EXPORTS)


def test_params_struct_matches_header(lib):
    from paper_2602_05900_amd import binding
    src = ('#include <stdio.h>\n#include <stddef.h>\n#include "hotrg.h"\n'
           'int main(void){printf("%zu %zu %zu %zu %zu %zu %zu\\n", sizeof(hotrg_params), '
           'offsetof(hotrg_params, custom_tensor), offsetof(hotrg_params, max_steps), '
           'offsetof(hotrg_params, field), offsetof(hotrg_params, two_sided), '
           'offsetof(hotrg_params, observables), offsetof(hotrg_params, custom_impurity));'
           'printf("%zu %zu\\n", offsetof(hotrg_params, bond_h), offsetof(hotrg_params, tau));return 0;}\n')
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        open(c, "w").write(src)
        exe = os.path.join(d, "t")
        subprocess.run(["gcc", "-I", os.path.dirname(HEADER), c, "-o", exe], check=True)
        out = subprocess.run([exe], capture_output=True, text=True).stdout.split()
        size, off_t, off_m, off_f, off_2, off_o, off_i, off_h, off_tau = (int(x) for x in out)
    assert ctypes.sizeof(binding.Params) == size
    assert binding.Params.custom_tensor.offset == off_t
    assert binding.Params.max_steps.offset == off_m
    assert binding.Params.field.offset == off_f
    assert binding.Params.two_sided.offset == off_2
    assert binding.Params.observables.offset == off_o
    assert binding.Params.custom_impurity.offset == off_i
    assert binding.Params.bond_h.offset == off_h and binding.Params.tau.offset == off_tau


def test_workspace_sizing_and_validation(lib):
    from paper_2602_05900_amd import binding
    ws48 = binding.workspace_bytes(model="ising", q=2, temperature=2.0, dmax=48, max_steps=30)
    # two D^5 FP64 intermediates dominate: 2 * 48^5 * 8 bytes
    assert 2 * 48 ** 5 * 8 < ws48 < 2.2 * 48 ** 5 * 8
    assert binding.workspace_bytes(model="ising", q=2, temperature=2.0, dmax=48, precision="fp32") < ws48
    # D^5 scaling of the footprint
    ws24 = binding.workspace_bytes(model="ising", q=2, temperature=2.0, dmax=24)
    assert 20 < ws48 / ws24 < 40
    # invalid parameter sets give 0
    assert binding.workspace_bytes(model="ising", q=3, temperature=2.0, dmax=8) == 0
    assert binding.workspace_bytes(model="ising", q=2, temperature=-1.0, dmax=8) == 0
    assert binding.workspace_bytes(model="potts", q=3, temperature=1.0, dmax=0) == 0
    assert binding.workspace_bytes(model="potts", q=3, temperature=1.0, dmax=8, max_steps=61) == 0
    # few steps at a large D need less than a long solve
    assert (binding.workspace_bytes(model="potts", q=3, temperature=1.0, dmax=81, max_steps=4)
            < binding.workspace_bytes(model="potts", q=3, temperature=1.0, dmax=81, max_steps=10))


def test_workspace_of_two_sided_and_observables(lib):
    from paper_2602_05900_amd import binding
    base = dict(model="ising", q=2, temperature=2.0, dmax=48, max_steps=30, precision="bf16x6")
    w0 = binding.workspace_bytes(**base)
    w2 = binding.workspace_bytes(**base, two_sided=True)
    w_m = binding.workspace_bytes(**base, observables=("m",))
    w_me = binding.workspace_bytes(**base, observables=("m", "e"))
    assert w0 < w2 < w0 + 0.1 * w0            # a second E, Ritz blocks and isometry: D^4-sized
    assert w0 < w_m < w_me                      # wider X and P4 buffers, impurity tensors
    assert w_me - w0 < 2.5 * 48 ** 5 * 6        # two more D^5 column blocks of X (3 BF16 planes)
    # invalid: unknown observable bit, non-finite field, field on a custom tensor,
    # a custom observable without its impurity tensor, two_sided outside {0, 1}
    p, _ = binding.make_params(**base)
    p.observables = 4
    assert lib.hotrg_workspace_bytes(ctypes.byref(p)) == 0
    p, _ = binding.make_params(**base, field=float("nan"))
    assert lib.hotrg_workspace_bytes(ctypes.byref(p)) == 0
    p, _ = binding.make_params(**base)
    p.two_sided = 2
    assert lib.hotrg_workspace_bytes(ctypes.byref(p)) == 0
    t = np.ones((2, 2, 2, 2))
    p, keep = binding.make_params(model="custom", tensor=t, dmax=4, field=0.5)
    assert lib.hotrg_workspace_bytes(ctypes.byref(p)) == 0
    p, keep = binding.make_params(model="custom", tensor=t, dmax=4, observables=("m",), impurities={"m": t})
    assert lib.hotrg_workspace_bytes(ctypes.byref(p)) > 0
    p.custom_impurity[0] = ctypes.POINTER(ctypes.c_double)()
    assert lib.hotrg_workspace_bytes(ctypes.byref(p)) == 0


def test_qchain_parameters(lib):
    from paper_2602_05900_amd import binding, workloads
    h = workloads.heisenberg_bond()
    assert binding.workspace_bytes(model="qchain", dmax=16, bond_h=h, tau=0.05, max_steps=20) > 0
    assert binding.workspace_bytes(model="qchain", dmax=16, bond_h=h, tau=0.0, max_steps=20) == 0
    bad = h.copy()
    bad[0, 1] = 1.0                                   # not symmetric
    assert binding.workspace_bytes(model="qchain", dmax=16, bond_h=bad, tau=0.05) == 0
    assert lib.hotrg_coarse_grain_axis(None, 1, 0) == binding.EINVAL
    v = ctypes.c_double()
    assert lib.hotrg_log_z_chain(None, ctypes.byref(v)) == binding.EINVAL


def test_itebd_sizes_and_error_paths(lib):
    from paper_2602_05900_amd import binding
    assert lib.itebd_state_len(8) == 4 * 64 + 16
    assert lib.itebd_state_len(0) == 0 and lib.itebd_state_len(33) == 0
    assert lib.itebd_workspace_bytes(0, 8) == 0 and lib.itebd_workspace_bytes(4, 33) == 0
    w = lib.itebd_workspace_bytes(256, 32)
    # states and the evolved pair per chain (n^2, n = 64), status words, counters
    per_chain = (4 * 1024 + 64) + 64 * 64
    assert 256 * per_chain * 8 <= w < 1.01 * (256 * per_chain * 8) + 16384
    h = ctypes.c_void_p()
    assert lib.itebd_init(1, 8, None, None, None, 0, None, ctypes.byref(h)) == binding.EINVAL
    assert lib.itebd_evolve(None, 0.1, 1) == binding.EINVAL
    assert lib.itebd_energy(None, None) == binding.EINVAL
    assert lib.itebd_info(None, None, None) == binding.EINVAL
    assert lib.itebd_status(None, None) == binding.EINVAL
    assert lib.itebd_set_max_sweeps(None, 5) == binding.EINVAL
    lib.itebd_destroy(None)


def test_host_error_paths_without_device(lib):
    from paper_2602_05900_amd import binding
    p, _ = binding.make_params(model="ising", q=2, temperature=2.0, dmax=8)
    h = ctypes.c_void_p()
    assert lib.hotrg_init_tensor(ctypes.byref(p), None, 0, None, ctypes.byref(h)) == binding.EINVAL
    assert lib.hotrg_init_tensor(None, None, 0, None, ctypes.byref(h)) == binding.EINVAL
    assert lib.hotrg_coarse_grain(None, 1) == binding.EINVAL
    assert lib.hotrg_coarse_grain_batch(None, 1, 1) == binding.EINVAL
    assert lib.hotrg_coarse_grain_batch(None, -1, 1) == binding.EINVAL
    assert lib.hotrg_coarse_grain_batch(None, 0, 1) == binding.OK       # empty group: nothing to do
    nulls = (ctypes.c_void_p * 2)(None, None)
    assert lib.hotrg_coarse_grain_batch(nulls, 2, 1) == binding.EINVAL
    v = ctypes.c_double()
    assert lib.hotrg_log_z(None, ctypes.byref(v), None) == binding.EINVAL
    vals = (ctypes.c_double * 2)()
    assert lib.hotrg_observables(None, vals) == binding.EINVAL
    assert lib.hotrg_step_sides(None, 1, None, None, None) == binding.EINVAL
    st = ctypes.c_int(-1)
    assert lib.hotrg_step_begin(None, 1, 0, ctypes.byref(st)) == binding.EINVAL and st.value == 0
    assert lib.hotrg_step_poll(None, ctypes.byref(st)) == binding.EINVAL
    assert lib.hotrg_coarse_grain_async(None, 1, 1, 0) == binding.EINVAL
    assert lib.hotrg_async_busy(None, ctypes.byref(st)) == binding.EINVAL
    lib.hotrg_destroy(None)
    assert lib.hotrg_strerror(binding.ENOMEM) == b"workspace too small"
    assert lib.hotrg_gemm_scratch_bytes(binding.FP64, 10, 10, 10) == 0
    assert lib.hotrg_gemm_scratch_bytes(binding.BF16X6, 10, 10, 10) > 0
