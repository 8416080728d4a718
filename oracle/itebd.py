"""iTEBD oracle: imaginary-time evolution of an infinite chain in plain NumPy FP64.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).  Nothing on the GPU path
imports this module.

What is computed
----------------
The paper's second workload (Sec. II.A, Eq. (1)) writes the ground state of an
infinite chain as a two-site periodic matrix product state
... lambda_2 A lambda_1 B lambda_2 ... and reaches it by repeated imaginary
time evolution with U = exp(-tau H), each step a tensor contraction followed
by an SVD that restores the form and truncates the bond to D_b states.  The
paper defers the algorithm to the iTEBD reference it cites (Vidal 2007); the
update here is that algorithm in the form that avoids dividing by the bond
weights (Hastings, J. Math. Phys. 50, 095207 (2009)):

* state: B1 = Gamma_A lambda_1 and B2 = Gamma_B lambda_2 (arrays [s][a][b]),
  the weights lambda_1 (bond A-B) and lambda_2 (bond B-A);
* one bond update on A-B:
    psi[a,s,t,b]  = sum_c B1[s][a][c] B2[t][c][b]
    psi'          = G psi on the two physical legs, G = exp(-tau h)
    M[(a s),(t b)] = lambda_2[a] psi'[a,s,t,b]
    M = X S Y^T (SVD); keep the D_b largest singular values
    B2' = Y^T (rows kept), B1' = psi' Y / |S_kept|, lambda_1' = S_kept / |S_kept|
  then the roles of the two sites are exchanged, so the next update acts on
  bond B-A;
* energy per site: the expectation of h on both bonds, averaged.

Each right singular vector's sign is fixed so that its largest-magnitude entry
is positive (the first such on ties), so tensors are comparable element by
element wherever the singular values at the cut are distinct.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


def gate(h: np.ndarray, tau: float) -> np.ndarray:
    """G = exp(-tau h) for a real symmetric two-site term h (d^2 x d^2),
    through its eigendecomposition."""
    w, V = np.linalg.eigh(h)
    return (V * np.exp(-tau * w)) @ V.T


@dataclass
class ChainState:
    B1: np.ndarray      # [d][chi][chi]
    B2: np.ndarray      # [d][chi][chi]
    l1: np.ndarray      # [chi], weights of the bond right of B1
    l2: np.ndarray      # [chi], weights of the bond left of B1 (right of B2)
    updates: int = 0    # bond updates applied (the roles swap after each)


def unpack(row: np.ndarray, chi: int, d: int = 2) -> ChainState:
    """A state row as laid out by the shared generator: B1, B2, l1, l2."""
    n = d * chi * chi
    return ChainState(B1=row[:n].reshape(d, chi, chi).copy(), B2=row[n:2 * n].reshape(d, chi, chi).copy(),
                      l1=row[2 * n:2 * n + chi].copy(), l2=row[2 * n + chi:2 * n + 2 * chi].copy())


def sign_gauge_rows(Yt: np.ndarray) -> np.ndarray:
    """Make the largest-magnitude entry of each row positive (lowest index on ties)."""
    out = Yt.copy()
    for j in range(out.shape[0]):
        i = int(np.argmax(np.abs(out[j])))
        if out[j, i] < 0.0:
            out[j] = -out[j]
    return out


def bond_update(st: ChainState, G: np.ndarray, chi: int) -> ChainState:
    """One update of bond A-B (the steps listed in the module docstring),
    returned with the sites' roles exchanged for the next update."""
    d = st.B1.shape[0]
    c1 = st.B1.shape[1]
    psi = np.einsum("sac,tcb->astb", st.B1, st.B2)                  # [a,s,t,b]
    G4 = G.reshape(d, d, d, d)                                       # [s',t',s,t]
    psi = np.einsum("uvst,astb->auvb", G4, psi)
    P = psi.reshape(c1 * d, d * c1)                                  # rows (a s'), cols (t' b)
    M = st.l2[:, None] * psi.reshape(c1, d * d * c1)
    M = M.reshape(c1 * d, d * c1)
    _U, S, Yt = np.linalg.svd(M)
    k = min(chi, S.size)
    Yt = sign_gauge_rows(Yt[:k])
    nrm = math.sqrt(float(np.sum(S[:k] ** 2)))
    B2n = Yt.reshape(k, d, c1).transpose(1, 0, 2).copy()           # [t][c][b]
    B1n = (P @ Yt.T / nrm).reshape(c1, d, k).transpose(1, 0, 2).copy()  # [s][a][c]
    l1n = S[:k] / nrm
    # exchange roles: the next update acts on the bond right of the old B2
    return ChainState(B1=B2n, B2=B1n, l1=st.l2.copy(), l2=l1n, updates=st.updates + 1)


def evolve(st: ChainState, h: np.ndarray, tau: float, nupdates: int, chi: int) -> ChainState:
    G = gate(h, tau)
    for _ in range(nupdates):
        st = bond_update(st, G, chi)
    return st


def bond_energy(B1, B2, l_left, h) -> float:
    """<h> on the bond between B1 and B2 with weights l_left on B1's left:
    theta = l_left B1 B2, <h> = theta . (h theta) / theta . theta."""
    d = B1.shape[0]
    theta = l_left[:, None, None, None] * np.einsum("sac,tcb->astb", B1, B2)
    ht = np.einsum("uvst,astb->auvb", h.reshape(d, d, d, d), theta)
    return float(np.sum(theta * ht) / np.sum(theta * theta))


def energy_per_site(st: ChainState, h: np.ndarray) -> float:
    """Mean of the two bonds' energies (two bonds per two-site cell)."""
    e12 = bond_energy(st.B1, st.B2, st.l2, h)
    e21 = bond_energy(st.B2, st.B1, st.l1, h)
    return 0.5 * (e12 + e21)


# --------------------------------------------------------------------------
# Closed forms used as pins
# --------------------------------------------------------------------------

BETHE_HEISENBERG = 0.25 - math.log(2.0)   # ground-state energy per site of the S=1/2 AF chain, J = 1


def tfim_energy(g: float, J: float = 1.0, npts: int = 20001) -> float:
    """Ground-state energy per site of H = -J sum sz sz - g sum sx (Pauli),
    -(1/pi) int_0^pi sqrt(J^2 + g^2 + 2 J g cos k) dk (free fermions),
    by the composite Simpson rule on npts points."""
    k = np.linspace(0.0, math.pi, npts)
    f = np.sqrt(J * J + g * g + 2.0 * J * g * np.cos(k))
    hstep = k[1] - k[0]
    s = f[0] + f[-1] + 4.0 * np.sum(f[1:-1:2]) + 2.0 * np.sum(f[2:-1:2])
    return -(s * hstep / 3.0) / math.pi
