"""Finding node pairs whose wide row hash has a zero low word (test input construction only).

The low word of the pair-keyed row hash is zero exactly when
(a*u + a2*v + b) mod 2^64 < 2^32.  For a fixed v that asks for the smallest u >= 0 with
(a*u + C) mod 2^64 in [0, 2^32), C = (a2*v + b) mod 2^64: the first hit of an
arithmetic progression modulo M in an interval, found by the Euclid-like recursion on
(A, M) below (each step swaps the roles of the modulus and the step).
"""

M64 = 1 << 64


def min_x(A, M, L, R):
    """Smallest x >= 0 with L <= (A*x) mod M <= R (0 <= L <= R < M), or None."""
    A %= M
    if L == 0:
        return 0
    if A == 0:
        return None
    t = (L + A - 1) // A  # a hit before the progression wraps around M
    if t * A <= R:
        return t
    # otherwise A*x = M*y + s with s in [L, R]: the smallest such y satisfies
    # (M*y) mod A in [(-R) mod A, (-L) mod A], an instance on (M mod A, A)
    y = min_x(M % A, A, (-R) % A, (-L) % A)
    if y is None:
        return None
    return (L + M * y + A - 1) // A


def first_hit(a, c, lo, hi, M=M64):
    """Smallest u >= 0 with (a*u + c) mod M in [lo, hi], or None."""
    lo2, hi2 = (lo - c) % M, (hi - c) % M
    if lo2 <= hi2:
        return min_x(a, M, lo2, hi2)
    cands = [x for x in (min_x(a, M, lo2, M - 1), min_x(a, M, 0, hi2)) if x is not None]
    return min(cands) if cands else None


def zero_low_row_pair(a, a2, b, V, tries=200000):
    """A pair u < v < V whose row hash (a*u + a2*v + b) >> 32 has a zero low word."""
    for v in range(V - 1, max(1, V - 1 - tries), -1):
        u = first_hit(a, (a2 * v + b) % M64, 0, (1 << 32) - 1)
        if u is not None and u < v:
            return u, v
    return None
