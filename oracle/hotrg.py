"""HOTRG oracle: one coarse-graining solve in plain NumPy FP64.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).  Nothing on the GPU path
imports this module.

What is computed
----------------
The paper writes the partition function of a 2D classical lattice model as the
full contraction of N copies of a rank-4 local tensor, Z = Tr T^N (Sec. II.A,
Eq. (2)).  HOTRG evaluates it by repeatedly merging two neighbouring tensors
along one lattice direction, fusing the two bonds that now run side by side,
and truncating the fused bond back to at most D states.  The truncation is a
higher-order SVD that reduces to an ordinary matrix decomposition once the
merged tensor is reshaped to a matrix (Sec. II.A); contraction and that
decomposition are the two steps the paper identifies as the whole cost
(Sec. II.A, Sec. II.B).  The paper defers the step itself to the HOTRG
reference it cites (Xie et al., PRB 86, 045139 (2012)); the steps below follow
that published algorithm:

* legs: T[l, r, d, u] = T[x, x', y, y'], row-major, last index fastest;
* a step stacks two copies vertically (bottom u-leg = top d-leg, bond k) and
  fuses the two left legs (a1 bottom, a2 top) and the two right legs;
* the truncation isometry U holds the leading D' = min(D, Dx^2) eigenvectors
  of the left environment E = M M^T, M being the merged tensor viewed as a
  matrix with rows (a1, a2);  E is built from two half-environments so that
  M itself (D^6 numbers) never appears;
* the new tensor is U^T M U, normalised by its largest magnitude c_n; then
  x and y are exchanged so the next step merges the other direction;
* ln Z / N = ln c_0 + sum_n ln(c_n) / 2^n + ln(Tr T_final) / 2^nsteps, with a
  periodic torus of N = 2^nsteps sites.

Readings where the paper is silent are listed in the design doc; each appears
below at the point it is used.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


# --------------------------------------------------------------------------
# Initial tensor (local tensor of Eq. (2) for Ising / q-state Potts)
# --------------------------------------------------------------------------

def boltzmann_weights(model: str, q: int, beta: float, J: float = 1.0) -> np.ndarray:
    """Bond Boltzmann weight matrix W[s, s'] = exp(-beta * H_bond(s, s')).

    Ising (q = 2, sigma = +1, -1):  H_bond = -J sigma sigma'.
    Potts (q states):               H_bond = -J delta(s, s').
    """
    if model == "ising":
        if q != 2:
            raise ValueError("Ising has q = 2")
        sigma = np.array([1.0, -1.0])
        return np.exp(beta * J * np.outer(sigma, sigma))
    if model == "potts":
        return np.exp(beta * J * np.eye(q))
    raise ValueError(f"unknown model {model!r}")


def weight_root(W: np.ndarray) -> np.ndarray:
    """Symmetric square root Q = W^(1/2), so that Q Q^T = W.

    Reading: the paper builds the local tensor from the Boltzmann weights but
    does not fix the gauge of the split; every split gives the same Z.  The
    symmetric root is taken (through a full eigendecomposition of W).
    """
    w, V = np.linalg.eigh(W)
    if np.any(w <= 0.0):
        raise ValueError("weight matrix is not positive definite")
    return (V * np.sqrt(w)) @ V.T


def initial_tensor(model: str, q: int, temperature: float, J: float = 1.0) -> np.ndarray:
    """T0[x, x', y, y'] = sum_s Q[s,x] Q[s,x'] Q[s,y] Q[s,y'] (one spin per site,
    each of its four bonds carrying a factor Q so that every bond sums to W)."""
    beta = 1.0 / temperature
    Q = weight_root(boltzmann_weights(model, q, beta, J))
    return np.einsum("sa,sb,sc,sd->abcd", Q, Q, Q, Q)


# --------------------------------------------------------------------------
# One coarse-graining step
# --------------------------------------------------------------------------

def half_environments(T: np.ndarray):
    """The two halves of the left environment of the vertically stacked pair.

    A[a1,k,b1,k'] = sum_{r1,d} T[a1,r1,d,k]  T[b1,r1,d,k']   (bottom copy)
    B[a2,k,b2,k'] = sum_{r2,u} T[a2,r2,k,u]  T[b2,r2,k',u]   (top copy)
    """
    A = np.einsum("ardk,brdl->akbl", T, T, optimize=True)
    B = np.einsum("arku,brlu->akbl", T, T, optimize=True)
    return A, B


def environment(T: np.ndarray) -> np.ndarray:
    """E[(a1 a2), (b1 b2)] = sum_{k,k'} A[a1,k,b1,k'] B[a2,k,b2,k'] = (M M^T),

    with M[(a1 a2), (r1 r2 d u)] = sum_k T[a1,r1,d,k] T[a2,r2,k,u] the merged
    pair viewed as a matrix whose rows are the fused left leg.  E is returned
    as an (Dx^2, Dx^2) matrix, symmetrised as (E + E^T) / 2.
    """
    Dx = T.shape[0]
    A, B = half_environments(T)
    E4 = np.einsum("ikjl,mknl->imjn", A, B, optimize=True)   # [a1, a2, b1, b2]
    E = E4.reshape(Dx * Dx, Dx * Dx)
    return 0.5 * (E + E.T)


@dataclass
class Truncation:
    U: np.ndarray          # (n, D') isometry, columns = kept eigenvectors
    eigenvalues: np.ndarray  # all n eigenvalues, descending
    kept: int              # D'
    trunc_err: float       # discarded eigenvalue weight / total weight
    cut_gap: float         # (lam[D'-1] - lam[D']) / lam[0]; inf when nothing is cut


def truncation(E: np.ndarray, dmax: int) -> Truncation:
    """Leading D' = min(dmax, n) eigenvectors of the symmetric environment E.

    The higher-order SVD of the merged tensor reduces to a matrix
    decomposition (Sec. II.A); its left singular vectors are the eigenvectors
    of E = M M^T and the squared singular values its eigenvalues.

    Readings: eigenvalues in descending order, equal values kept in the order
    the ascending solver returned them reversed; each kept column has its
    largest-magnitude entry made positive (first such entry on ties).
    """
    n = E.shape[0]
    lam_asc, V_asc = np.linalg.eigh(E)
    lam = lam_asc[::-1].copy()
    V = V_asc[:, ::-1]
    kept = min(dmax, n)
    U = V[:, :kept].copy()
    for j in range(kept):
        i = int(np.argmax(np.abs(U[:, j])))
        if U[i, j] < 0.0:
            U[:, j] = -U[:, j]
    total = float(np.sum(lam))
    discarded = float(np.sum(lam[kept:]))
    trunc_err = discarded / total if total != 0.0 else 0.0
    cut_gap = (lam[kept - 1] - lam[kept]) / lam[0] if kept < n else math.inf
    return Truncation(U=U, eigenvalues=lam, kept=kept, trunc_err=trunc_err, cut_gap=cut_gap)


@dataclass
class StepResult:
    T_next: np.ndarray     # normalised, x/y exchanged: dims [Dy, Dy, D', D']
    c: float               # normalisation c_n = max |T'|
    trunc: Truncation


def coarse_grain_step(T: np.ndarray, dmax: int) -> StepResult:
    """One HOTRG step on T[l, r, d, u] with dims [Dx, Dx, Dy, Dy].

    X[l,a2,r1,d,k] = sum_{a1}     U[a1,a2,l] T[a1,r1,d,k]
    Y[l,r1,d,r2,u] = sum_{a2,k}   X[l,a2,r1,d,k] T[a2,r2,k,u]
    T'[l,r,d,u]    = sum_{r1,r2}  Y[l,r1,d,r2,u] U[r1,r2,r]

    i.e. T' = U^T M U applied to the fused left and right legs, contracted in
    the O(D^7) order.  Then c_n = max|T'|, T' <- T'/c_n, and the legs are
    exchanged (x <-> y) for the next step.
    """
    Dx = T.shape[0]
    if T.shape[1] != Dx or T.shape[3] != T.shape[2]:
        raise ValueError("T must have dims [Dx, Dx, Dy, Dy]")
    tr = truncation(environment(T), dmax)
    U3 = tr.U.reshape(Dx, Dx, tr.kept)                           # U[a1, a2, l]
    X = np.einsum("abl,ardk->lbrdk", U3, T, optimize=True)       # X[l,a2,r1,d,k]
    Y = np.einsum("lbrdk,bsku->lrdsu", X, T, optimize=True)      # Y[l,r1,d,r2,u]
    Tp = np.einsum("lrdsu,rsm->lmdu", Y, U3, optimize=True)      # T'[l,r,d,u]
    c = float(np.max(np.abs(Tp)))
    Tp = Tp / c
    return StepResult(T_next=np.ascontiguousarray(Tp.transpose(2, 3, 0, 1)), c=c, trunc=tr)


# --------------------------------------------------------------------------
# A whole solve
# --------------------------------------------------------------------------

@dataclass
class Solve:
    lnz_per_site: float
    log2_sites: int
    c: list = field(default_factory=list)          # c_0, c_1, ..., c_nsteps
    trunc_err: list = field(default_factory=list)  # per step
    cut_gap: list = field(default_factory=list)    # per step
    dims: list = field(default_factory=list)       # (Dx, Dy) entering each step
    T_final: np.ndarray | None = None              # normalised tensor after the last step


def solve_tensor(T0: np.ndarray, dmax: int, nsteps: int, keep_tensor: bool = True) -> Solve:
    """Run nsteps HOTRG steps from the local tensor T0 and return ln Z / N.

    ln Z/N = ln c_0 + sum_{n=1..nsteps} ln(c_n)/2^n + ln(sum_{x,y} T[x,x,y,y]) / 2^nsteps,
    N = 2^nsteps sites on a periodic torus of 2^floor(n/2) x 2^ceil(n/2) sites
    (x by y); the last term is the trace of the single remaining tensor with
    both of its bond pairs closed periodically (Eq. (2) with N -> 1 tensor).
    """
    T0 = np.asarray(T0, dtype=np.float64)
    c0 = float(np.max(np.abs(T0)))
    T = T0 / c0
    out = Solve(lnz_per_site=0.0, log2_sites=nsteps, c=[c0])
    lnz = math.log(c0)
    for n in range(1, nsteps + 1):
        out.dims.append((T.shape[0], T.shape[2]))
        step = coarse_grain_step(T, dmax)
        T = step.T_next
        out.c.append(step.c)
        out.trunc_err.append(step.trunc.trunc_err)
        out.cut_gap.append(step.trunc.cut_gap)
        lnz += math.log(step.c) / 2.0 ** n
    trace = float(np.einsum("xxyy->", T))
    out.lnz_per_site = lnz + math.log(trace) / 2.0 ** nsteps
    if keep_tensor:
        out.T_final = T
    return out


def solve(model: str, q: int, temperature: float, dmax: int, nsteps: int,
          J: float = 1.0, keep_tensor: bool = True) -> Solve:
    """HOTRG for the Ising (q = 2) or q-state Potts model at a temperature."""
    return solve_tensor(initial_tensor(model, q, temperature, J), dmax, nsteps, keep_tensor)


def free_energy(lnz_per_site: float, temperature: float) -> float:
    """f = -T ln Z / N (k_B = 1)."""
    return -temperature * lnz_per_site


# --------------------------------------------------------------------------
# Work accounting (host arithmetic used for the oracle's own timing)
# --------------------------------------------------------------------------

def step_dims(d0x: int, d0y: int, dmax: int, nsteps: int):
    """(Dx, Dy, D') entering each step: D' = min(D, Dx^2), then (Dx, Dy) <- (Dy, D')."""
    dims = []
    Dx, Dy = d0x, d0y
    for _ in range(nsteps):
        Dp = min(dmax, Dx * Dx)
        dims.append((Dx, Dy, Dp))
        Dx, Dy = Dy, Dp
    return dims


def contraction_flops(Dx: int, Dy: int, Dp: int) -> float:
    """Floating-point operations of the contractions of one step, in the order
    above: two half-environments, E, X, Y, T'."""
    return float(4 * Dx**3 * Dy**3 + 2 * Dx**4 * Dy**2 + 2 * Dp * Dx**3 * Dy**2
                 + 2 * Dp * Dx**3 * Dy**3 + 2 * Dp**2 * Dx**2 * Dy**2)
