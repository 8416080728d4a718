"""Seeded synthetic inputs shared by the tests, the benchmark and the server.

Holds none of the method's arithmetic: temperatures, grids, random tensors and
request streams only.  Workloads are the paper's HOTRG setting (Sec. II.A,
Eq. (2)) on the 2D square-lattice Ising model and the 3-state Potts model.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

ISING_TC = 2.0 / math.log(1.0 + math.sqrt(2.0))      # 2.269185314213022
POTTS3_TC = 1.0 / math.log(1.0 + math.sqrt(3.0))     # 0.994972861...

SERVE_SEED = 20260205


def critical_temperature(model: str, q: int = 2) -> float:
    if model == "ising":
        return ISING_TC
    if model == "potts" and q == 3:
        return POTTS3_TC
    if model == "potts":
        return 1.0 / math.log(1.0 + math.sqrt(q))
    raise ValueError(model)


def temperature_grid(lo: float, hi: float, count: int) -> np.ndarray:
    return np.linspace(lo, hi, count)


def random_tensor(dx: int, dy: int, seed: int = 0) -> np.ndarray:
    """A dense random tensor T[l,r,d,u] of dims [dx,dx,dy,dy] with no lattice
    symmetry (standard normal entries)."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((dx, dx, dy, dy))


@dataclass
class Request:
    rid: int
    arrival: float      # seconds from the start of the run
    model: str
    q: int
    temperature: float
    dmax: int
    nsteps: int


def request_stream(rate_hz: float = 50.0, duration_s: float = 60.0, seed: int = SERVE_SEED,
                   dims=(16, 24, 32, 48), steps=(20, 40)) -> list[Request]:
    """Poisson arrivals at rate_hz for duration_s seconds.  Each request draws
    its model uniformly from {Ising, 3-state Potts}, T uniform in
    [0.5, 1.5] x Tc(model), D uniformly from `dims` and the step count
    uniformly from the inclusive range `steps`."""
    rng = np.random.default_rng(seed)
    out = []
    t = 0.0
    rid = 0
    while True:
        t += rng.exponential(1.0 / rate_hz)
        if t >= duration_s:
            break
        model = "ising" if rng.integers(0, 2) == 0 else "potts"
        q = 2 if model == "ising" else 3
        tc = critical_temperature(model, q)
        temp = float(rng.uniform(0.5, 1.5) * tc)
        d = int(rng.choice(dims))
        n = int(rng.integers(steps[0], steps[1] + 1))
        out.append(Request(rid, t, model, q, temp, d, n))
        rid += 1
    return out


def random_chain_states(batch: int, chi: int, d: int = 2, seed: int = 0) -> np.ndarray:
    """Initial two-site unit cells of `batch` infinite chains, one row per
    chain: B1[d][chi][chi], B2[d][chi][chi] (standard normal entries) and the
    bond weights l1[chi], l2[chi] (all 1/sqrt(chi)), flattened in that
    order.  Different chains start from different random states."""
    rng = np.random.default_rng(seed)
    n = d * chi * chi
    out = np.empty((batch, 2 * n + 2 * chi))
    out[:, :2 * n] = rng.standard_normal((batch, 2 * n))
    out[:, 2 * n:] = 1.0 / math.sqrt(chi)
    return out


def heisenberg_bond(J: float = 1.0) -> np.ndarray:
    """Two-site Hamiltonian J S.S of spin-1/2, basis |s t> with s, t in
    {up, down} (index 2 s + t), as a 4 x 4 matrix."""
    h = np.zeros((4, 4))
    h[0, 0] = h[3, 3] = 0.25 * J
    h[1, 1] = h[2, 2] = -0.25 * J
    h[1, 2] = h[2, 1] = 0.5 * J
    return h


def ising_transverse_bond(g: float, J: float = 1.0) -> np.ndarray:
    """Two-site term of the transverse-field Ising chain
    H = -J sum sz sz - g sum sx (Pauli matrices), the field split evenly
    over the two bonds of each site, as a 4 x 4 matrix."""
    sz = np.diag([1.0, -1.0])
    sx = np.array([[0.0, 1.0], [1.0, 0.0]])
    one = np.eye(2)
    return -J * np.kron(sz, sz) - 0.5 * g * (np.kron(sx, one) + np.kron(one, sx))
