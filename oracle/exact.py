"""Exact brute force for tiny meshes (<= 10 vertices).  Test infrastructure
only; used to pin the LAPACK-based oracle against arithmetic that shares
nothing with it.

* characteristic polynomial of an integer matrix by the Faddeev-LeVerrier
  recurrence in exact rational arithmetic;
* square-free factorisation (Yun) and Sturm-sequence bisection for the real
  roots with multiplicities;
* spanning trees counted by enumerating every (n-1)-edge subset
  (Kirchhoff's matrix-tree theorem relates the count to the Laplacian
  spectrum: tau = (1/n) prod_{lambda > 0} lambda for a connected graph).
"""
from __future__ import annotations

from fractions import Fraction
from itertools import combinations


# polynomials: list of Fractions, highest degree first -----------------------

def _trim(p):
    i = 0
    while i < len(p) - 1 and p[i] == 0:
        i += 1
    return p[i:]


def _deriv(p):
    n = len(p) - 1
    return _trim([c * (n - i) for i, c in enumerate(p[:-1])]) if n > 0 else [Fraction(0)]


def _divmod(a, b):
    """Polynomial long division (highest degree first): a = q b + r."""
    a = list(_trim(a))
    b = _trim(b)
    if len(a) < len(b):
        return [Fraction(0)], a
    q = [Fraction(0)] * (len(a) - len(b) + 1)
    for i in range(len(q)):
        f = a[i] / b[0]
        q[i] = f
        for j in range(len(b)):
            a[i + j] -= f * b[j]
    r = _trim(a[len(q):]) if len(a) > len(q) else [Fraction(0)]
    return _trim(q), r


def _gcd(a, b):
    a, b = _trim(a), _trim(b)
    while any(b):
        _, r = _divmod(a, b)
        a, b = b, r
    return [c / a[0] for c in a]


def _eval(p, x):
    v = Fraction(0)
    for c in p:
        v = v * x + c
    return v


def charpoly(A):
    """det(x I - A) of a square integer/rational matrix, Faddeev-LeVerrier."""
    n = len(A)
    A = [[Fraction(v) for v in row] for row in A]
    coeffs = [Fraction(1)]
    M = [[Fraction(0)] * n for _ in range(n)]
    c_prev = Fraction(1)
    for k in range(1, n + 1):
        # M_k = A M_{k-1} + c_{n-k+1} I
        AM = [[sum(A[i][t] * M[t][j] for t in range(n)) for j in range(n)] for i in range(n)]
        for i in range(n):
            AM[i][i] += c_prev
        M = AM
        tr = sum(sum(A[i][t] * M[t][i] for t in range(n)) for i in range(n))
        c_prev = -tr / k
        coeffs.append(c_prev)
    return coeffs


def _monic(p):
    p = _trim(p)
    return [c / p[0] for c in p]


def squarefree_parts(p):
    """Yun's algorithm: p = const * prod_i a_i^i, a_i square-free and
    pairwise coprime.  Returns [(a_i, i)] for the non-constant a_i."""
    p = _monic(p)
    dp = _deriv(p)
    a0 = _gcd(p, dp)
    b, _ = _divmod(p, a0)
    c, _ = _divmod(dp, a0)
    d = _sub(c, _deriv(b))
    out = []
    i = 1
    while len(_trim(b)) > 1:
        a = _gcd(b, d) if any(d) else _monic(b)
        if len(a) > 1:
            out.append((a, i))
        b, _ = _divmod(b, a)
        c, _ = _divmod(d, a) if any(d) else ([Fraction(0)], None)
        d = _sub(c, _deriv(b))
        i += 1
    return out


def _pad(p, n):
    return [Fraction(0)] * (n - len(p)) + list(p)


def _sub(a, b):
    n = max(len(a), len(b))
    return _trim([x - y for x, y in zip(_pad(a, n), _pad(b, n))])


def _sturm_chain(p):
    """p0 = p, p1 = p', p_{k+1} = -rem(p_{k-1}, p_k) until the remainder is 0."""
    chain = [_trim(p), _deriv(p)]
    while len(chain[-1]) > 1:
        _, r = _divmod(chain[-2], chain[-1])
        if not any(r):
            break
        chain.append([-c for c in r])
    return chain


def _sign_changes(chain, x):
    s = [_eval(q, x) for q in chain]
    s = [v for v in s if v != 0]
    return sum(1 for u, v in zip(s, s[1:]) if (u > 0) != (v > 0))


def real_roots(p, lo, hi, tol=Fraction(1, 10 ** 15)):
    """Distinct real roots of the square-free p in (lo, hi], by Sturm bisection."""
    chain = _sturm_chain(_trim(p))
    roots = []
    stack = [(Fraction(lo), Fraction(hi))]
    while stack:
        a, b = stack.pop()
        k = _sign_changes(chain, a) - _sign_changes(chain, b)
        if k == 0:
            continue
        if k == 1 and b - a < tol:
            roots.append((a + b) / 2)
            continue
        mid = (a + b) / 2
        stack.append((a, mid))
        stack.append((mid, b))
    return sorted(roots)


def eigenvalues_exact(A, bound=None):
    """Eigenvalues (with multiplicity, ascending, as floats) of a symmetric
    integer matrix from its exact characteristic polynomial."""
    n = len(A)
    if bound is None:
        bound = max(sum(abs(v) for v in row) for row in A) + 1
    p = charpoly(A)
    out = []
    for a, mult in squarefree_parts(p):
        for r in real_roots(a, -bound - Fraction(1, 7), bound):
            out.extend([float(r)] * mult)
    out.sort()
    assert len(out) == n, (len(out), n)
    return out


def spanning_trees_bruteforce(n, edges):
    """Number of spanning trees by enumerating all (n-1)-edge subsets."""
    edges = [tuple(e) for e in edges]
    count = 0
    for sub in combinations(range(len(edges)), n - 1):
        parent = list(range(n))

        def find(x):
            while parent[x] != x:
                parent[x] = parent[parent[x]]
                x = parent[x]
            return x
        ok = True
        for k in sub:
            a, b = edges[k]
            ra, rb = find(a), find(b)
            if ra == rb:
                ok = False
                break
            parent[ra] = rb
        if ok:
            count += 1
    return count
