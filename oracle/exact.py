"""Independent pins for the HOTRG oracle — TEST INFRASTRUCTURE ONLY.

None of these functions runs the HOTRG algorithm.  They give partition
functions by other, textbook routes, so that a mistake in the oracle (a wrong
leg order, a dropped term, a transposed operand) shows up as a mismatch:

* ``brute_force_lnz``      sum over every spin configuration of a periodic
                           Lx x Ly torus (Z = Tr exp(-beta H), Sec. II.A);
* ``spin_transfer_lnz``    the same Z through the row-to-row transfer matrix;
* ``network_lnz``          exact contraction of an Lx x Ly periodic network of
                           copies of an arbitrary tensor T[l, r, d, u]
                           (Z = Tr T^N, Eq. (2)) through a tensor row transfer
                           matrix — no truncation, no isometries;
* ``onsager_lnz``          Onsager's exact ln Z / N of the infinite square-
                           lattice Ising model, and its internal energy;
* ``brute_force_observables``  the same enumeration with a magnetic field,
                           returning the mean order parameter per site and the
                           mean energy of a y bond and of an x bond;
* ``network_impurity_ratio``  exact contraction of the periodic network with
                           one copy replaced by another tensor, over the pure
                           network (what an impurity-tensor estimator converges
                           to when nothing is truncated);
* ``yang_magnetisation``   the spontaneous magnetisation of the square-lattice
                           Ising model below T_c (Onsager / Yang);
* ``trotter_ring_lnz``     ln Tr (G_odd G_even)^M of a spin-1/2 ring by exact
                           diagonalisation, G = exp(-tau h) from scipy's expm;
* ``tfim_free_energy``     free energy per site of the transverse-field Ising
                           chain at temperature T (free fermions).
"""
from __future__ import annotations

import itertools
import math

import numpy as np
from scipy import integrate, linalg as sla, special

CATALAN = 0.915965594177219015054603514932384110774


def _bond_energy(model: str, J: float):
    if model == "ising":
        def e(a, b):
            sa = 1 - 2 * a
            sb = 1 - 2 * b
            return -J * sa * sb
    elif model == "potts":
        def e(a, b):
            return -J * (a == b)
    else:
        raise ValueError(model)
    return e


def _logsumexp(x: np.ndarray) -> float:
    m = float(np.max(x))
    return m + math.log(float(np.sum(np.exp(x - m))))


def brute_force_lnz(model: str, q: int, temperature: float, Lx: int, Ly: int,
                    J: float = 1.0) -> float:
    """ln Z of a periodic Lx x Ly torus by enumerating all q^(Lx Ly) states.

    Bonds: every site (x, y) couples to (x+1 mod Lx, y) and (x, y+1 mod Ly), so
    there are 2 Lx Ly bonds; a width-1 direction gives a site coupled to itself
    and a width-2 direction two parallel bonds, exactly as the tensor network of
    one tensor per site counts them.
    """
    nsites = Lx * Ly
    if q ** nsites > 5_000_000:
        raise ValueError("too many states for brute force")
    beta = 1.0 / temperature
    states = np.array(list(itertools.product(range(q), repeat=nsites)), dtype=np.int64)
    s = states.reshape(-1, Ly, Lx)                       # s[config, y, x]
    right = np.roll(s, -1, axis=2)
    up = np.roll(s, -1, axis=1)
    if model == "ising":
        sig, sr, su = 1 - 2 * s, 1 - 2 * right, 1 - 2 * up
        energy = -J * (np.sum(sig * sr, axis=(1, 2)) + np.sum(sig * su, axis=(1, 2)))
    elif model == "potts":
        energy = -J * (np.sum(s == right, axis=(1, 2)) + np.sum(s == up, axis=(1, 2)))
    else:
        raise ValueError(model)
    return _logsumexp(-beta * energy.astype(np.float64))


def spin_transfer_lnz(model: str, q: int, temperature: float, Lx: int, Ly: int,
                      J: float = 1.0) -> float:
    """ln Z of the same torus as ``brute_force_lnz`` via Z = Tr M^Ly, with
    M[s, s'] = exp(-beta (E_row(s) + E_vertical(s, s'))) over row states s."""
    beta = 1.0 / temperature
    e = _bond_energy(model, J)
    rows = list(itertools.product(range(q), repeat=Lx))
    nr = len(rows)
    M = np.empty((nr, nr))
    for i, s in enumerate(rows):
        e_row = sum(e(s[x], s[(x + 1) % Lx]) for x in range(Lx))
        for j, t in enumerate(rows):
            e_vert = sum(e(s[x], t[x]) for x in range(Lx))
            M[i, j] = math.exp(-beta * (e_row + e_vert))
    # scale to avoid overflow: ln Tr M^Ly = Ly ln c + ln Tr (M/c)^Ly
    c = float(np.max(M))
    P = np.linalg.matrix_power(M / c, Ly)
    return Ly * math.log(c) + math.log(float(np.trace(P)))


def network_lnz(T: np.ndarray, Lx: int, Ly: int) -> float:
    """ln Z of the periodic Lx x Ly network of copies of T[l, r, d, u].

    Site (x, y) has its r leg joined to the l leg of (x+1 mod Lx, y) and its u
    leg joined to the d leg of (x, y+1 mod Ly).  The row transfer matrix
    R[(d_0..d_{Lx-1}), (u_0..u_{Lx-1})] = sum_h prod_x T[h_x, h_{x+1}, d_x, u_x]
    is built explicitly and Z = Tr R^Ly.  Requires Z > 0.
    """
    T = np.asarray(T, dtype=np.float64)
    Dx, Dy = T.shape[0], T.shape[2]
    # open row of j sites: W[h_left, h_right, (d_0..d_{j-1}), (u_0..u_{j-1})]
    W = T.copy()
    for j in range(1, Lx):
        W = np.einsum("ahDU,hbdu->abDdUu", W, T)
        W = W.reshape(Dx, Dx, Dy ** (j + 1), Dy ** (j + 1))
    # close the row periodically: the last right leg is the first left leg
    R = np.einsum("hhDU->DU", W)
    c = float(np.max(np.abs(R)))
    P = np.linalg.matrix_power(R / c, Ly)
    tr = float(np.trace(P))
    if tr <= 0.0:
        raise ValueError("network partition function is not positive")
    return Ly * math.log(c) + math.log(tr)


def _row_transfer(tensors) -> np.ndarray:
    """R[(d_0..d_{L-1}), (u_0..u_{L-1})] = sum_h prod_x A_x[h_x, h_{x+1}, d_x, u_x]
    for a periodic row of the given tensors (all with the same dims)."""
    W = np.asarray(tensors[0], dtype=np.float64).copy()
    Dx, Dy = W.shape[0], W.shape[2]
    for j in range(1, len(tensors)):
        W = np.einsum("ahDU,hbdu->abDdUu", W, tensors[j])
        W = W.reshape(Dx, Dx, Dy ** (j + 1), Dy ** (j + 1))
    return np.einsum("hhDU->DU", W)


def network_impurity_ratio(T: np.ndarray, I: np.ndarray, Lx: int, Ly: int) -> float:
    """Z_I / Z for the periodic Lx x Ly network of copies of T[l, r, d, u] in
    which the copy at site (0, 0) is replaced by I (same dims, same leg
    joining as ``network_lnz``): Z_I = Tr(R_I R^(Ly-1)), Z = Tr R^Ly with R the
    pure row transfer matrix and R_I the row holding I.  By translation
    invariance of the rest of the network any site gives the same ratio."""
    T = np.asarray(T, dtype=np.float64)
    I = np.asarray(I, dtype=np.float64)
    R = _row_transfer([T] * Lx)
    RI = _row_transfer([I] + [T] * (Lx - 1))
    c = float(np.max(np.abs(R)))
    P = np.linalg.matrix_power(R / c, Ly - 1)
    z = float(np.trace(P @ (R / c)))
    zi = float(np.trace(P @ (RI / c)))
    if z <= 0.0:
        raise ValueError("network partition function is not positive")
    return zi / z


def brute_force_observables(model: str, q: int, temperature: float, Lx: int, Ly: int,
                            J: float = 1.0, field: float = 0.0) -> dict:
    """Exact thermal averages on the periodic Lx x Ly torus by enumeration.

    H = sum over the 2 Lx Ly bonds of e(s, s') - field * sum_i f(s_i), with
    e = -J s s' and f(s) = s for Ising (s = +-1), e = -J delta(s, s') and
    f(s) = delta(s, 0) for Potts.  Returns ln Z, the order parameter per site
    <m> (Ising s; Potts (q delta(s, 0) - 1) / (q - 1)), the mean energy of
    one y bond (site to its upper neighbour) and of one x bond, and the
    internal energy per site <H> / N.  Bonds are counted as in
    ``brute_force_lnz`` (a width-2 direction has two parallel bonds).
    """
    nsites = Lx * Ly
    if q ** nsites > 5_000_000:
        raise ValueError("too many states for brute force")
    beta = 1.0 / temperature
    states = np.array(list(itertools.product(range(q), repeat=nsites)), dtype=np.int64)
    s = states.reshape(-1, Ly, Lx)                       # s[config, y, x]
    right = np.roll(s, -1, axis=2)
    up = np.roll(s, -1, axis=1)
    if model == "ising":
        sig, sr, su = 1 - 2 * s, 1 - 2 * right, 1 - 2 * up
        ex = -J * np.sum(sig * sr, axis=(1, 2)).astype(np.float64)
        ey = -J * np.sum(sig * su, axis=(1, 2)).astype(np.float64)
        fs = np.sum(sig, axis=(1, 2)).astype(np.float64)
        mm = fs
    elif model == "potts":
        ex = -J * np.sum(s == right, axis=(1, 2)).astype(np.float64)
        ey = -J * np.sum(s == up, axis=(1, 2)).astype(np.float64)
        fs = np.sum(s == 0, axis=(1, 2)).astype(np.float64)
        mm = (q * fs - nsites) / (q - 1.0)
    else:
        raise ValueError(model)
    energy = ex + ey - field * fs
    lw = -beta * energy
    lz = _logsumexp(lw)
    w = np.exp(lw - lz)
    return {
        "lnz": lz,
        "m": float(np.sum(w * mm)) / nsites,
        "e_y": float(np.sum(w * ey)) / nsites,
        "e_x": float(np.sum(w * ex)) / nsites,
        "u": float(np.sum(w * energy)) / nsites,
    }


def hotrg_torus(nsteps: int):
    """(Lx, Ly) of the torus that nsteps HOTRG steps (first merging along y)
    close into one tensor: Lx = 2^floor(n/2), Ly = 2^ceil(n/2)."""
    return 2 ** (nsteps // 2), 2 ** ((nsteps + 1) // 2)


# --------------------------------------------------------------------------
# Onsager's exact solution of the square-lattice Ising model (J = 1)
# --------------------------------------------------------------------------

ISING_TC = 2.0 / math.log(1.0 + math.sqrt(2.0))
POTTS3_TC = 1.0 / math.log(1.0 + math.sqrt(3.0))


def onsager_lnz(temperature: float) -> float:
    """ln Z / N of the infinite lattice:
    ln(2 cosh 2b) + (1/2pi) int_0^pi ln[(1 + sqrt(1 - k^2 sin^2 t)) / 2] dt,
    k = 2 sinh 2b / cosh^2 2b."""
    b = 1.0 / temperature
    k = 2.0 * math.sinh(2.0 * b) / math.cosh(2.0 * b) ** 2

    def integrand(t):
        return math.log(0.5 * (1.0 + math.sqrt(max(0.0, 1.0 - (k * math.sin(t)) ** 2))))

    val, _ = integrate.quad(integrand, 0.0, math.pi, epsabs=1e-15, epsrel=1e-15, limit=400)
    return math.log(2.0 * math.cosh(2.0 * b)) + val / (2.0 * math.pi)


def onsager_lnz_tc() -> float:
    """Closed form at the critical point: (1/2) ln 2 + 2 G / pi (G = Catalan)."""
    return 0.5 * math.log(2.0) + 2.0 * CATALAN / math.pi


def onsager_energy(temperature: float) -> float:
    """Internal energy per site u = -coth(2b) [1 + (2/pi)(2 tanh^2 2b - 1) K(k)]."""
    b = 1.0 / temperature
    k = 2.0 * math.sinh(2.0 * b) / math.cosh(2.0 * b) ** 2
    t2 = math.tanh(2.0 * b) ** 2
    if abs(k - 1.0) < 1e-15:
        return -1.0 / math.tanh(2.0 * b)
    return -(1.0 / math.tanh(2.0 * b)) * (1.0 + (2.0 / math.pi) * (2.0 * t2 - 1.0) * special.ellipk(k * k))


def yang_magnetisation(temperature: float) -> float:
    """Spontaneous magnetisation per site of the square-lattice Ising model
    (J = 1): (1 - sinh(2b)^-4)^(1/8) below T_c, 0 above."""
    b = 1.0 / temperature
    x = 1.0 - math.sinh(2.0 * b) ** -4
    return x ** 0.125 if x > 0.0 else 0.0


def finite_difference_energy(temperatures: np.ndarray, lnz: np.ndarray) -> np.ndarray:
    """u(T) = T^2 d(ln Z/N)/dT on a uniform grid: central differences inside,
    second-order one-sided differences at the two ends."""
    T = np.asarray(temperatures, dtype=np.float64)
    g = np.asarray(lnz, dtype=np.float64)
    h = T[1] - T[0]
    d = np.empty_like(g)
    d[1:-1] = (g[2:] - g[:-2]) / (2.0 * h)
    d[0] = (-3.0 * g[0] + 4.0 * g[1] - g[2]) / (2.0 * h)
    d[-1] = (3.0 * g[-1] - 4.0 * g[-2] + g[-3]) / (2.0 * h)
    return T * T * d


# --------------------------------------------------------------------------
# Quantum chains: exact Trotterized rings and the free-fermion chain
# --------------------------------------------------------------------------

def _two_site_operator(G: np.ndarray, L: int, i: int, j: int) -> np.ndarray:
    """The 2^L x 2^L matrix of a two-site operator G[(s_i' s_j'), (s_i s_j)]
    acting on sites i and j of an L-site spin-1/2 ring (site 0 most
    significant in the basis index)."""
    dim = 2 ** L
    out = np.zeros((dim, dim))
    for col in range(dim):
        si = (col >> (L - 1 - i)) & 1
        sj = (col >> (L - 1 - j)) & 1
        base = col & ~(1 << (L - 1 - i)) & ~(1 << (L - 1 - j))
        for a in range(2):
            for b in range(2):
                row = base | (a << (L - 1 - i)) | (b << (L - 1 - j))
                out[row, col] += G[2 * a + b, 2 * si + sj]
    return out


def trotter_ring_lnz(h: np.ndarray, tau: float, L: int, M: int) -> float:
    """ln Tr U^M with U = G_odd G_even on a ring of L (even) sites:
    G_even the product of G = expm(-tau h) on bonds (0,1), (2,3), ...,
    G_odd on bonds (1,2), (3,4), ..., (L-1, 0)."""
    G = sla.expm(-tau * np.asarray(h, dtype=np.float64))
    dim = 2 ** L
    Ge = np.eye(dim)
    Go = np.eye(dim)
    for j in range(0, L, 2):
        Ge = _two_site_operator(G, L, j, j + 1) @ Ge
    for j in range(1, L, 2):
        Go = _two_site_operator(G, L, j, (j + 1) % L) @ Go
    U = Go @ Ge
    c = float(np.max(np.abs(U)))
    P = np.linalg.matrix_power(U / c, M)
    return M * math.log(c) + math.log(float(np.trace(P)))


def tfim_free_energy(g: float, temperature: float, J: float = 1.0) -> float:
    """Free energy per site of H = -J sum sz sz - g sum sx (Pauli) on the
    infinite chain: -(T/pi) int_0^pi ln(2 cosh(e_k / T)) dk with
    e_k = sqrt(J^2 + g^2 + 2 J g cos k)."""
    def integrand(k):
        e = math.sqrt(J * J + g * g + 2.0 * J * g * math.cos(k)) / temperature
        return e + math.log1p(math.exp(-2.0 * e))     # ln(2 cosh e)
    val, _ = integrate.quad(integrand, 0.0, math.pi, epsabs=1e-13, epsrel=1e-13, limit=400)
    return -temperature * val / math.pi
