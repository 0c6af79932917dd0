"""Polynomial trajectory algebra in the monomial basis (Sec. III-D.1).

A segment is sigma_i(t) = c_i^T beta(t) on t in [0, T_i] with
beta(t) = (1, t, ..., t^d), d = 2p - 1, and c_i squeezed axis-major into
R^{m(d+1)} (coefficient vector of axis 0, then axis 1, then axis 2).
"""
from __future__ import annotations

import math

import torch

DT = torch.float64


def falling(j: int, o: int) -> int:
    """j! / (j - o)!, the factor an o-th derivative puts on t^j (0 when j < o)."""
    if j < o:
        return 0
    return math.factorial(j) // math.factorial(j - o)


def beta(o: int, t: torch.Tensor, d: int) -> torch.Tensor:
    """beta^(o)(t): o-th derivative of the monomial basis, shape t.shape + (d+1,)."""
    t = torch.as_tensor(t, dtype=DT)
    cols = []
    for j in range(d + 1):
        if j < o:
            cols.append(torch.zeros_like(t))
        elif j == o:
            cols.append(torch.full_like(t, float(falling(j, o))))
        else:
            cols.append(falling(j, o) * t ** (j - o))
    return torch.stack(cols, -1)


def cost_gram(T: torch.Tensor, p: int, d: int) -> torch.Tensor:
    """Q(T) = int_0^T beta^(p)(tau) beta^(p)(tau)^T dtau (Sec. III-D.1), shape T.shape + (d+1, d+1).

    Entry (j, k) is [j!/(j-p)!][k!/(k-p)!] T^(j+k-2p+1) / (j+k-2p+1) for j, k >= p
    and zero otherwise: the integral of a monomial, written out.
    """
    T = torch.as_tensor(T, dtype=DT)
    n = d + 1
    rows = []
    for j in range(n):
        row = []
        for k in range(n):
            if j < p or k < p:
                row.append(torch.zeros_like(T))
            else:
                e = j + k - 2 * p + 1
                row.append(falling(j, p) * falling(k, p) * T ** e / e)
        rows.append(torch.stack(row, -1))
    return torch.stack(rows, -2)


def knot_map(t: torch.Tensor, n_ord: int, d: int) -> torch.Tensor:
    """(beta^0(t), ..., beta^(n_ord-1)(t))^T: coefficients -> derivatives 0..n_ord-1 at t.

    Shape t.shape + (n_ord, d+1).  With I_m (x) this is the paper's beta~(t).
    """
    return torch.stack([beta(o, t, d) for o in range(n_ord)], -2)


def boundary_map(T: torch.Tensor, n_left: int, n_right: int, d: int) -> torch.Tensor:
    """M(T): rows beta^(o)(0) for o < n_left, then beta^(o)(T) for o < n_right (Sec. III-D.1).

    Shape T.shape + (n_left + n_right, d+1).
    """
    T = torch.as_tensor(T, dtype=DT)
    left = knot_map(torch.zeros_like(T), n_left, d)
    right = knot_map(T, n_right, d)
    return torch.cat([left, right], -2)


def kron_axes(A: torch.Tensor, m: int = 3) -> torch.Tensor:
    """I_m (x) A for a batch of matrices A [..., r, c] -> [..., m r, m c] (axis-major blocks)."""
    r, c = A.shape[-2], A.shape[-1]
    out = A.new_zeros(A.shape[:-2] + (m * r, m * c))
    for a in range(m):
        out[..., a * r:(a + 1) * r, a * c:(a + 1) * c] = A
    return out


def smoothstep_coeffs(p: int) -> list:
    """Monomial coefficients of the rest-to-rest unit step polynomial of degree 2p-1.

    S(tau) rises from 0 to 1 on [0, 1] with derivatives 1..p-1 zero at both
    ends; p = 3 gives 10 tau^3 - 15 tau^4 + 6 tau^5.  Obtained here by solving
    the 2p Hermite end conditions exactly (rational arithmetic).
    """
    from fractions import Fraction
    n = 2 * p
    rows, rhs = [], []
    for o in range(p):
        rows.append([Fraction(falling(j, o)) if j == o else Fraction(0) for j in range(n)])
        rhs.append(Fraction(0))
    for o in range(p):
        rows.append([Fraction(falling(j, o)) if j >= o else Fraction(0) for j in range(n)])
        rhs.append(Fraction(1 if o == 0 else 0))
    # Gauss-Jordan elimination over the rationals.
    A = [r[:] + [b] for r, b in zip(rows, rhs)]
    for col in range(n):
        piv = next(r for r in range(col, n) if A[r][col] != 0)
        A[col], A[piv] = A[piv], A[col]
        pv = A[col][col]
        A[col] = [x / pv for x in A[col]]
        for r in range(n):
            if r != col and A[r][col] != 0:
                f = A[r][col]
                A[r] = [x - f * y for x, y in zip(A[r], A[col])]
    return [A[j][n] for j in range(n)]
