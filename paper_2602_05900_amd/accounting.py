"""Algorithmic work of a HOTRG solve: FLOPs of the contractions per step in
the O(D^7) order (two half environments, E, X, Y, T') and the minimum HBM
bytes of the Y product.  The eigensolve, normalisation and trace are not
counted (they are timed separately).  Host arithmetic only.
"""
from __future__ import annotations


def step_dims(d0x: int, d0y: int, dmax: int, nsteps: int):
    """(Dx, Dy, D') entering each step; D' = min(D, Dx^2); (Dx, Dy) <- (Dy, D')."""
    out = []
    dx, dy = d0x, d0y
    for _ in range(nsteps):
        dp = min(dmax, dx * dx)
        out.append((dx, dy, dp))
        dx, dy = dy, dp
    return out


def stage_flops(dx: int, dy: int, dp: int) -> dict:
    return {
        "env": 4.0 * dx**3 * dy**3 + 2.0 * dx**4 * dy**2,
        "x": 2.0 * dp * dx**3 * dy**2,
        "y": 2.0 * dp * dx**3 * dy**3,
        "tp": 2.0 * dp**2 * dx**2 * dy**2,
    }


def step_flops(dx: int, dy: int, dp: int, two_sided: bool = False, nimp: int = 0) -> float:
    """Contraction FLOPs of one step.  Two-sided truncation builds a second
    environment; each impurity tensor adds its X, a Y over twice the
    contraction length and its T'."""
    f = stage_flops(dx, dy, dp)
    total = sum(f.values())
    if two_sided:
        total += f["env"]
    return total + nimp * (f["x"] + 2.0 * f["y"] + f["tp"])


def solve_flops(q: int, dmax: int, nsteps: int, two_sided: bool = False, nimp: int = 0) -> float:
    return sum(step_flops(*d, two_sided=two_sided, nimp=nimp) for d in step_dims(q, q, dmax, nsteps))


def y_flops(q: int, dmax: int, nsteps: int) -> float:
    return sum(stage_flops(*d)["y"] for d in step_dims(q, q, dmax, nsteps))


def y_bytes(dx: int, dy: int, dp: int, elem_bytes: int, out_bytes: int | None = None) -> float:
    """Compulsory HBM traffic of one Y product: read X (D' Dx^2 Dy^2) and the
    re-laid-out T (Dx^2 Dy^2) once at elem_bytes an element, write Y
    (D' Dx^2 Dy^2) once at out_bytes an element (default elem_bytes)."""
    n5 = dp * dx * dx * dy * dy
    ob = elem_bytes if out_bytes is None else out_bytes
    return float(elem_bytes) * (n5 + dx * dx * dy * dy) + float(ob) * n5
