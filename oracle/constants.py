"""Exact rational constants for the oracle -- TEST INFRASTRUCTURE ONLY.

Everything here is computed with ``fractions.Fraction`` so that the oracle's
constants carry no rounding at all until they are handed to the C code as
doubles.

* ``bspline_integer_values(p)``: the centred cardinal B-spline Phi_p at the
  integers, from the de Boor recursion (Sec. "B-spline interpolation").
* ``omega_prime(p, M)``: the universal stencil sequence omega' of
  eq. (kernel_stencil_by_conv_with_universal_coeff).  The kernel k_l(|r-r'|)
  is interpolated in both arguments, so for exact interpolation omega' would
  be the autoconvolution of the 1-D interpolation sequence, whose symbol is
  1/Bhat(theta)^2 with Bhat(theta) = sum_n Phi_p(n) e^{i n theta}.  The
  quasi-interpolation reading used here keeps a symmetric sequence of
  half-width M and asks that omega'(theta) Bhat(theta)^2 = 1 + O(theta^(2M+2)).
  That is the same as asking the sequence P = omega' * b * b (b_n = Phi_p(n))
  to have moments sum_j P_j j^(2k) = delta_{k0} for k = 0..M, a linear system
  that is solved here exactly.  (The library derives the same sequence a
  different way, by truncating a Taylor series in sin^2(theta/2).)
"""
from fractions import Fraction


def cardinal_M_exact(k, t):
    """Cardinal B-spline M_k(t) on knots 0..k at a rational t (de Boor)."""
    t = Fraction(t)
    if k == 1:
        return Fraction(1) if 0 <= t < 1 else Fraction(0)
    return (t * cardinal_M_exact(k - 1, t) + (k - t) * cardinal_M_exact(k - 1, t - 1)) / (k - 1)


def bspline_exact(p, t):
    """Centred Phi_p(t) = M_p(t + p/2) at a rational t."""
    return cardinal_M_exact(p, Fraction(t) + Fraction(p, 2))


def bspline_integer_values(p):
    """{n: Phi_p(n)} for the integers with a non-zero value."""
    half = p // 2
    return {n: bspline_exact(p, n) for n in range(-half + 1, half)}


def _conv(a, b):
    """Convolution of two sequences given as {index: value} dicts."""
    out = {}
    for i, x in a.items():
        for j, y in b.items():
            out[i + j] = out.get(i + j, Fraction(0)) + x * y
    return out


def _solve_exact(A, rhs):
    """Gauss-Jordan elimination over the rationals."""
    n = len(A)
    M = [list(row) + [r] for row, r in zip(A, rhs)]
    for c in range(n):
        piv = next(r for r in range(c, n) if M[r][c] != 0)
        M[c], M[piv] = M[piv], M[c]
        pv = M[c][c]
        M[c] = [x / pv for x in M[c]]
        for r in range(n):
            if r != c and M[r][c] != 0:
                f = M[r][c]
                M[r] = [x - f * y for x, y in zip(M[r], M[c])]
    return [M[r][n] for r in range(n)]


def omega_prime(p, M):
    """omega'_0..omega'_M as Fractions (symmetric: omega'_{-j} = omega'_j)."""
    b = bspline_integer_values(p)
    bb = _conv(b, b)
    cols = []
    for i in range(M + 1):
        e = {0: Fraction(1)} if i == 0 else {i: Fraction(1), -i: Fraction(1)}
        cols.append(_conv(e, bb))
    A = [[sum(v * Fraction(j) ** (2 * k) for j, v in cols[i].items()) for i in range(M + 1)]
         for k in range(M + 1)]
    rhs = [Fraction(1)] + [Fraction(0)] * M
    return _solve_exact(A, rhs)
