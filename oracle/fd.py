"""Central finite-difference coefficients of the second derivative.

ORACLE / TEST INFRASTRUCTURE ONLY: see oracle/__init__.py.

Eq. (1) of the paper writes the Laplacian as a sum of 1D (2 N_f + 1)-point
central stencils with coefficients c_{mu,n}; the paper defers the values to
its Ref. 7 and prints only N_f = 1 (appendix, Eq. (A3): c_0 = -2/h^2,
c_{+-1} = 1/h^2).  Here the coefficients are derived from their definition:
the unique symmetric stencil that is exact for every polynomial of degree
<= 2 N_f + 1, i.e.

    sum_{n=-N_f}^{N_f} c_|n| n^(2j) = 2 * delta_{j,1},   j = 0 .. N_f,

solved exactly over the rationals.  c_{mu,n} = chat_|n| / h_mu^2.
"""
from fractions import Fraction
from functools import lru_cache


@lru_cache(maxsize=None)
def fd_coefficients_exact(nf: int):
    """[chat_0, ..., chat_nf] as Fractions (dimensionless, h = 1)."""
    if nf < 1:
        raise ValueError("nf must be >= 1")
    n_unk = nf + 1
    rows = []
    for j in range(n_unk):
        row = [Fraction(1 if j == 0 else 0)]
        for n in range(1, nf + 1):
            row.append(Fraction(2 * n ** (2 * j)))
        row.append(Fraction(2 if j == 1 else 0))
        rows.append(row)
    # Gauss-Jordan elimination over the rationals
    for col in range(n_unk):
        piv = next(r for r in range(col, n_unk) if rows[r][col] != 0)
        rows[col], rows[piv] = rows[piv], rows[col]
        p = rows[col][col]
        rows[col] = [v / p for v in rows[col]]
        for r in range(n_unk):
            if r != col and rows[r][col] != 0:
                f = rows[r][col]
                rows[r] = [a - f * b for a, b in zip(rows[r], rows[col])]
    return tuple(rows[i][-1] for i in range(n_unk))


@lru_cache(maxsize=None)
def fd_coefficients(nf: int):
    """Same as fd_coefficients_exact, as floats."""
    return tuple(float(c) for c in fd_coefficients_exact(nf))
