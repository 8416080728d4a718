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

Two extensions of the same published algorithm (Xie et al. 2012) are also
written out here:

* two-sided truncation: the right environment (rows = the fused right leg) is
  diagonalised as well, and each step keeps the isometry of the side whose
  discarded eigenvalue weight is smaller, applying it to both fused legs;
* impurity tensors: a local observable enters as one modified copy of the
  local tensor; each step replaces an impurity tensor I by the average of the
  two placements in the merged pair, U^T (I (x) T + T (x) I) U / 2, with the
  same isometry and normalisation as T, so that after n steps
  Tr I_n / Tr T_n is the observable averaged over the torus.

Where the paper is silent, the reading taken is stated below at the point
where it is used.
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


def field_weights(model: str, q: int, beta: float, field: float) -> np.ndarray:
    """Site Boltzmann factor exp(beta * h * f(s)) of a field h coupled to
    f(s) = sigma (Ising) or f(s) = delta(s, 0) (Potts)."""
    if model == "ising":
        return np.exp(beta * field * np.array([1.0, -1.0]))
    f = np.zeros(q)
    f[0] = 1.0
    return np.exp(beta * field * f)


def order_parameter(model: str, q: int) -> np.ndarray:
    """Local order parameter m(s): sigma for Ising, (q delta(s,0) - 1)/(q - 1)
    for Potts (1 in the ordered state s = 0, averaging to 0 when disordered)."""
    if model == "ising":
        return np.array([1.0, -1.0])
    m = np.full(q, -1.0 / (q - 1.0))
    m[0] = 1.0
    return m


def bond_energy(model: str, q: int, J: float = 1.0) -> np.ndarray:
    """Bond energy e(s, s'): -J sigma sigma' (Ising), -J delta(s, s') (Potts)."""
    if model == "ising":
        sigma = np.array([1.0, -1.0])
        return -J * np.outer(sigma, sigma)
    return -J * np.eye(q)


def site_tensor(Q: np.ndarray, weights: np.ndarray) -> np.ndarray:
    """sum_s w(s) Q[s,x] Q[s,x'] Q[s,y] Q[s,y']."""
    return np.einsum("s,sa,sb,sc,sd->abcd", weights, Q, Q, Q, Q)


def initial_tensor(model: str, q: int, temperature: float, J: float = 1.0,
                   field: float = 0.0) -> np.ndarray:
    """T0[x, x', y, y'] = sum_s g(s) Q[s,x] Q[s,x'] Q[s,y] Q[s,y'] (one spin per
    site, each of its four bonds carrying a factor Q so that every bond sums
    to W; g the site factor of the field, 1 without one)."""
    beta = 1.0 / temperature
    Q = weight_root(boltzmann_weights(model, q, beta, J))
    return site_tensor(Q, field_weights(model, q, beta, field))


def impurity_tensors(model: str, q: int, temperature: float, J: float = 1.0,
                     field: float = 0.0) -> dict:
    """The two impurity tensors of the observables.

    "m": the site's spin sum weighted by the order parameter,
         S = sum_s m(s) g(s) Q[s,.]^4, so that one copy of S in the network
         gives Z <m_i>.
    "e": the local tensor with the bond below the site (its d leg) carrying
         e(s, s') W(s, s') instead of W(s, s'): the leg is contracted with
         G = Q^-1 W_e Q^-1 (W_e = e o W elementwise), since Q G Q = W_e.  One
         copy gives Z <e_b> for that y bond.
    Both are normalised like T0 by the caller (the same c_0).
    """
    beta = 1.0 / temperature
    W = boltzmann_weights(model, q, beta, J)
    Q = weight_root(W)
    g = field_weights(model, q, beta, field)
    S = site_tensor(Q, order_parameter(model, q) * g)
    We = bond_energy(model, q, J) * W
    G = np.linalg.solve(Q, np.linalg.solve(Q, We).T).T      # Q^-1 We Q^-1 (Q symmetric)
    T0 = site_tensor(Q, g)
    TG = np.einsum("yb,xzbw->xzyw", G, T0)
    return {"m": S, "e": TG}


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


def right_environment(T: np.ndarray) -> np.ndarray:
    """E_R[(r1 r2), (s1 s2)] = sum M[(a1 a2), (r1 r2), d, u] M[(a1 a2), (s1 s2), d, u]:
    the environment of the fused right leg of the same stacked pair, built
    from its own two halves,

    A_R[r1,k,s1,k'] = sum_{a1,d} T[a1,r1,d,k] T[a1,s1,d,k']   (bottom copy)
    B_R[r2,k,s2,k'] = sum_{a2,u} T[a2,r2,k,u] T[a2,s2,k',u]   (top copy)

    and symmetrised like the left one.
    """
    Dx = T.shape[0]
    A = np.einsum("ardk,asdl->rksl", T, T, optimize=True)
    B = np.einsum("arku,aslu->rksl", T, T, optimize=True)
    E4 = np.einsum("ikjl,mknl->imjn", A, B, optimize=True)
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


def project(T: np.ndarray, U: np.ndarray):
    """The merged pair's fused legs projected with an isometry U (n x D',
    n = Dx^2, rows (a1 a2) with a1 the bottom copy's leg), in the O(D^7) order:

    X[l,a2,r1,d,k] = sum_{a1}     U[a1,a2,l] T[a1,r1,d,k]
    Y[l,r1,d,r2,u] = sum_{a2,k}   X[l,a2,r1,d,k] T[a2,r2,k,u]
    T'[l,r,d,u]    = sum_{r1,r2}  Y[l,r1,d,r2,u] U[r1,r2,r]

    Returns (X, T'), T' unnormalised with legs [l, r, d, u] (no exchange).
    """
    Dx = T.shape[0]
    U3 = U.reshape(Dx, Dx, U.shape[1])                           # U[a1, a2, l]
    X = np.einsum("abl,ardk->lbrdk", U3, T, optimize=True)       # X[l,a2,r1,d,k]
    Y = np.einsum("lbrdk,bsku->lrdsu", X, T, optimize=True)      # Y[l,r1,d,r2,u]
    Tp = np.einsum("lrdsu,rsm->lmdu", Y, U3, optimize=True)      # T'[l,r,d,u]
    return X, Tp


@dataclass
class StepResult:
    T_next: np.ndarray     # normalised, x/y exchanged: dims [Dy, Dy, D', D']
    c: float               # normalisation c_n = max |T'|
    trunc: Truncation      # the truncation applied (the chosen side's)
    eps_left: float = 0.0  # discarded weight of the left environment
    eps_right: float = math.nan  # ... of the right one (two-sided only)
    side: int = 0          # 0: left isometry applied, 1: right
    impurities_next: list = field(default_factory=list)


def coarse_grain_step(T: np.ndarray, dmax: int, two_sided: bool = False,
                      impurities=(), exchange: bool = True) -> StepResult:
    """One HOTRG step on T[l, r, d, u] with dims [Dx, Dx, Dy, Dy].

    X[l,a2,r1,d,k] = sum_{a1}     U[a1,a2,l] T[a1,r1,d,k]
    Y[l,r1,d,r2,u] = sum_{a2,k}   X[l,a2,r1,d,k] T[a2,r2,k,u]
    T'[l,r,d,u]    = sum_{r1,r2}  Y[l,r1,d,r2,u] U[r1,r2,r]

    i.e. T' = U^T M U applied to the fused left and right legs, contracted in
    the O(D^7) order.  Then c_n = max|T'|, T' <- T'/c_n, and the legs are
    exchanged (x <-> y) for the next step.

    two_sided: U is taken from the right environment instead when its
    discarded weight is strictly smaller (ties keep the left one).

    impurities: tensors I of T's dims; each becomes
    I' = U^T (I (x) T + T (x) I) U / (2 c_n), the bottom copy written first,
    exchanged like T.

    exchange=False keeps T'[l, r, d, u] as it is, so the next step merges
    along the same axis again (dims [Dx, Dx, Dy, Dy] -> [D', D', Dy, Dy]).
    """
    Dx = T.shape[0]
    if T.shape[1] != Dx or T.shape[3] != T.shape[2]:
        raise ValueError("T must have dims [Dx, Dx, Dy, Dy]")
    tr = truncation(environment(T), dmax)
    eps_left, eps_right, side = tr.trunc_err, math.nan, 0
    if two_sided:
        trr = truncation(right_environment(T), dmax)
        eps_right = trr.trunc_err
        if trr.trunc_err < tr.trunc_err:
            tr, side = trr, 1
    U3 = tr.U.reshape(Dx, Dx, tr.kept)                           # U[a1, a2, l]
    X, Tp = project(T, tr.U)
    c = float(np.max(np.abs(Tp)))
    Tp = Tp / c
    nxt = []
    for I in impurities:
        XI = np.einsum("abl,ardk->lbrdk", U3, I, optimize=True)
        YI = (np.einsum("lbrdk,bsku->lrdsu", XI, T, optimize=True)      # impurity in the bottom copy
              + np.einsum("lbrdk,bsku->lrdsu", X, I, optimize=True))    # impurity in the top copy
        Ip = 0.5 * np.einsum("lrdsu,rsm->lmdu", YI, U3, optimize=True) / c
        nxt.append(np.ascontiguousarray(Ip.transpose(2, 3, 0, 1) if exchange else Ip))
    Tn = Tp.transpose(2, 3, 0, 1) if exchange else Tp
    return StepResult(T_next=np.ascontiguousarray(Tn), c=c, trunc=tr,
                      eps_left=eps_left, eps_right=eps_right, side=side, impurities_next=nxt)


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
    eps_left: list = field(default_factory=list)   # per step (two-sided runs)
    eps_right: list = field(default_factory=list)
    sides: list = field(default_factory=list)      # 0 left / 1 right isometry per step
    observables: list = field(default_factory=list)  # Tr I_n / Tr T_n per impurity


def solve_tensor(T0: np.ndarray, dmax: int, nsteps: int, keep_tensor: bool = True,
                 two_sided: bool = False, impurities=(), schedule=None) -> Solve:
    """Run nsteps HOTRG steps from the local tensor T0 and return ln Z / N.

    ln Z/N = ln c_0 + sum_{n=1..nsteps} ln(c_n)/2^n + ln(sum_{x,y} T[x,x,y,y]) / 2^nsteps,
    N = 2^nsteps sites on a periodic torus of 2^floor(n/2) x 2^ceil(n/2) sites
    (x by y); the last term is the trace of the single remaining tensor with
    both of its bond pairs closed periodically (Eq. (2) with N -> 1 tensor).
    """
    T0 = np.asarray(T0, dtype=np.float64)
    c0 = float(np.max(np.abs(T0)))
    T = T0 / c0
    imps = [np.asarray(I, dtype=np.float64) / c0 for I in impurities]
    out = Solve(lnz_per_site=0.0, log2_sites=nsteps, c=[c0])
    lnz = math.log(c0)
    for n in range(1, nsteps + 1):
        out.dims.append((T.shape[0], T.shape[2]))
        step = coarse_grain_step(T, dmax, two_sided, imps, True if schedule is None else bool(schedule[n - 1]))
        T = step.T_next
        imps = step.impurities_next
        out.c.append(step.c)
        out.trunc_err.append(step.trunc.trunc_err)
        out.cut_gap.append(step.trunc.cut_gap)
        out.eps_left.append(step.eps_left)
        out.eps_right.append(step.eps_right)
        out.sides.append(step.side)
        lnz += math.log(step.c) / 2.0 ** n
    trace = float(np.einsum("xxyy->", T))
    out.lnz_per_site = lnz + math.log(trace) / 2.0 ** nsteps
    out.observables = [float(np.einsum("xxyy->", I)) / trace for I in imps]
    if keep_tensor:
        out.T_final = T
    return out


def solve(model: str, q: int, temperature: float, dmax: int, nsteps: int,
          J: float = 1.0, keep_tensor: bool = True, field: float = 0.0,
          two_sided: bool = False, observables=()) -> Solve:
    """HOTRG for the Ising (q = 2) or q-state Potts model at a temperature.

    observables: any of "m" (order parameter per site) and "e" (energy of one
    y bond), carried as impurity tensors; their estimates land in
    ``Solve.observables`` in the order given."""
    imp = impurity_tensors(model, q, temperature, J, field) if observables else {}
    return solve_tensor(initial_tensor(model, q, temperature, J, field), dmax, nsteps, keep_tensor,
                        two_sided, [imp[o] for o in observables])


def internal_energy(model: str, q: int, e_bond: float, m: float, field: float) -> float:
    """Internal energy per site from the y-bond energy and the order
    parameter: two bonds per site (x and y bonds equal for these isotropic
    models) plus the field term -h <f(s)>."""
    if model == "ising":
        f = m
    else:
        f = ((q - 1.0) * m + 1.0) / q
    return 2.0 * e_bond - field * f


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
