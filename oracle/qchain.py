"""Quantum-chain HOTRG oracle: the spin-1/2 chain mapped onto a 2D tensor
network with an imaginary-time axis.  TEST INFRASTRUCTURE ONLY (see
``oracle/__init__.py``); nothing on the GPU path imports this module.

What is computed
----------------
The paper evaluates HOTRG on a quantum spin chain by mapping its partition
function onto a classical network with an extra imaginary-time dimension, in
which contracting along imaginary time is operator evolution (Sec. II.A).
Here Z = Tr e^{-beta H} is approximated by Tr (G_odd G_even)^M, G = exp(-tau h)
on every bond, beta = M tau (the even and odd bonds each as one layer).  One
tensor holds a block of two sites for one Trotter step:

* the gate is split over its two sites, G[(s1' s2'),(s1 s2)] =
  sum_k A_k[s1', s1] B_k[s2', s2], by an SVD of the rearranged matrix
  R[(s1' s1), (s2' s2)], A_k = sqrt(sigma_k) u_k, B_k = sqrt(sigma_k) v_k;
* the block (sites 0, 1) takes the even gate on its own pair, then the odd
  layer: site 0 is the right site of the gate shared with the left block
  (B, bond l), site 1 the left site of the gate shared with the right block
  (A, bond r):
    T[l, r, (s0 s1), (s0' s1')] = sum B_l[s0', s0''] A_r[s1', s1''] G[(s0'' s1''), (s0 s1)]
  so x is space (the split bonds, dimension 4) and y is imaginary time (the
  block's two spins below and above, dimension 4).

A HOTRG step merges along y; without the x/y exchange the next step merges
along the same axis.  k steps along time give beta = 2^k tau (operator
evolution: only the space bonds are truncated); the time direction is then
closed by a trace over the block's physical legs, and the infinite chain's
ln Z comes from the dominant eigenvalue of that column transfer matrix.
(Truncating the time-boundary legs instead, by further steps along space,
keeps only the dominant boundary states and loses the thermal entropy.)
With one tensor per block and step, f = -(ln Z / N) / (2 tau).
"""
from __future__ import annotations

import math

import numpy as np

from .hotrg import solve_tensor
from .itebd import gate


def operator_split(G: np.ndarray, d: int = 2):
    """A[k][s1', s1], B[k][s2', s2] with G = sum_k A_k (x) B_k."""
    R = G.reshape(d, d, d, d).transpose(0, 2, 1, 3).reshape(d * d, d * d)   # [(s1' s1), (s2' s2)]
    U, S, Vt = np.linalg.svd(R)
    r = np.sqrt(S)
    A = (U * r).T.reshape(d * d, d, d)
    B = (Vt * r[:, None]).reshape(d * d, d, d)
    return A, B


def block_tensor(h: np.ndarray, tau: float) -> np.ndarray:
    """T[l, r, (s0 s1), (s0' s1')] of one two-site block and one Trotter step."""
    d = 2
    G = gate(np.asarray(h, dtype=np.float64), tau)
    A, B = operator_split(G, d)
    G4 = G.reshape(d, d, d, d)                               # [s0'', s1'', s0, s1]
    T = np.einsum("lpx,rqy,xyab->lrabpq", B, A, G4)         # [l, r, s0, s1, s0', s1']
    k = A.shape[0]
    return T.reshape(k, k, d * d, d * d)


def chain_lnz(T0: np.ndarray, dmax: int, time_steps: int) -> float:
    """ln Z per tensor of the network infinite along x and 2^time_steps
    tensors (Trotter steps) around y, periodic in y: time_steps merges along
    y (no exchange, the x bonds truncated to dmax), then the closing of y
    by the trace t[l, r] = sum_s T[l, r, s, s] and, for the infinite chain of
    such columns, ln Z / N = ln c_0 + sum_n ln(c_n) / 2^n + ln(lambda_max(t)) / 2^n,
    lambda_max the eigenvalue of largest modulus (real and positive for a
    transfer matrix of a positive partition function)."""
    r = solve_tensor(T0, dmax, time_steps, keep_tensor=True, schedule=[False] * time_steps)
    lnz_acc = math.log(r.c[0]) + sum(math.log(c) / 2.0 ** (k + 1) for k, c in enumerate(r.c[1:]))
    t = np.einsum("lrss->lr", r.T_final)
    w = np.linalg.eigvals(t)
    lam = w[np.argmax(np.abs(w))]
    if abs(lam.imag) > 1e-12 * abs(lam) or lam.real <= 0.0:
        raise ValueError("dominant eigenvalue of the column transfer matrix is not positive")
    return lnz_acc + math.log(lam.real) / 2.0 ** time_steps


def free_energy(h, tau: float, dmax: int, time_steps: int) -> float:
    """f per site at beta = 2^time_steps tau on the infinite chain."""
    return -chain_lnz(block_tensor(h, tau), dmax, time_steps) / (2.0 * tau)


def ground_energy(h, tau: float, dmax: int, nsteps: int) -> float:
    """Alternating merges: both axes grow, beta = tau 2^(n/2) -> infinity, and
    -(ln Z / N) / (2 tau) tends to the ground-state energy per site."""
    r = solve_tensor(block_tensor(h, tau), dmax, nsteps, keep_tensor=False)
    return -r.lnz_per_site / (2.0 * tau)
