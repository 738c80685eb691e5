"""Exact-rational algebra of Shan-Chen forcing stencils (oracle side).

TEST INFRASTRUCTURE ONLY (see the package docstring). Everything here is computed from
definitions, by brute force over the stencil vectors, in ``fractions.Fraction``:

* shell groups: all integer vectors that a generator reaches by permutations and sign flips
  (Sec. "Bulk Physics", Fig. 1; in 3D the squared length 9 holds the (2,2,1) and (3,0,0)
  groups, coded 9 and 1009; code 18 is the (3,3,0) group);
* moments <x^a y^b z^c>_W and the isotropy / anisotropy coefficients e_2n, I_2n,k
  (Sec. "Higher-order Tuning" and Appendix "Defining the stencil"): each coefficient is the
  isotropy condition built from the moments, which vanishes on the fully isotropic tensor
  e_2n Delta^(2n);
* the one-dimensional projection of the d = 2 lattice pressure tensor (Appendix "Lattice
  Pressure Tensor - d = 2", eq. 1dPNT) and the Taylor coefficients c_mn of P_N - P_T
  (Appendix "Defining the stencil"), obtained by expanding each product psi(x+p) psi(x+q);
* the knobs sigma_0 = c11 - c02, sigma_1 = c22 - c13 + c04, delta_0 = c02 (eqs. HOSigmaInt,
  SCTolmanFlat), with the 3D -> 2D weight projection of eq. (wproj);
* weights solved from linear conditions on the moments (Sec. "Computing the Weights").
"""
from __future__ import annotations

from fractions import Fraction as Fr
from itertools import product
from math import factorial

GENERATORS = {
    1: (1, 0, 0), 2: (1, 1, 0), 3: (1, 1, 1), 4: (2, 0, 0), 5: (2, 1, 0), 6: (2, 1, 1),
    8: (2, 2, 0), 1009: (3, 0, 0), 16: (4, 0, 0), 18: (3, 3, 0),
}


def generator(d: int, code: int):
    if code == 9:
        return (3, 0, 0) if d == 2 else (2, 2, 1)
    if code == 1009 and d == 2:
        raise ValueError("code 1009 exists only in 3D")
    g = GENERATORS[code]
    if d == 2 and g[2] != 0:
        raise ValueError(f"shell {code} has no 2D vectors")
    return g


def vectors(d: int, code: int):
    """All lattice vectors of the symmetry group named by ``code`` (as d-tuples)."""
    g = sorted(generator(d, code))
    out = []
    rng = range(-4, 5)
    for v in product(rng, repeat=d):
        if sorted(abs(c) for c in (tuple(v) + (0,) * (3 - d))) == g:
            out.append(tuple(v))
    return out


def moment(d: int, W: dict, powers):
    """<x^a y^b (z^c)>_W = sum over every stencil vector of W(shell) * x^a y^b z^c."""
    tot = Fr(0)
    for code, w in W.items():
        for v in vectors(d, code):
            t = Fr(w)
            for comp, pw in zip(v, powers):
                t *= Fr(comp) ** pw
            tot += t
    return tot


def coefficients(d: int, W: dict) -> dict:
    """Isotropy coefficients e_2n and anisotropy conditions I_2n,k (vanish when isotropic)."""
    m = lambda *p: moment(d, W, p + (0,) * (d - len(p)))
    out = {"e2": m(2), "e4": m(2, 2)}
    if d == 2:
        out["e6"] = m(4, 2) / 3
        out["e8"] = m(4, 4) / 9
        out["I40"] = m(4) - 3 * m(2, 2)
        out["I60"] = m(6) - 15 * out["e6"]
        out["I80"] = m(6, 2) - 15 * out["e8"]
        out["I81"] = m(8) - 7 * m(6, 2)
    else:
        out["e6"] = m(2, 2, 2)
        out["e8"] = m(4, 4) / 9
        out["I40"] = m(4) - 3 * m(2, 2)
        out["I60"] = m(6) - 15 * m(4, 2) + 30 * m(2, 2, 2)
        out["I61"] = m(4, 2) - 3 * m(2, 2, 2)
        out["I80"] = m(8) - 7 * m(6, 2)
        out["I81"] = m(6, 2) - Fr(5, 3) * m(4, 4)
        out["I82"] = m(4, 4) - 3 * m(4, 2, 2)
        out["I100"] = m(10) - 9 * m(8, 2)
        out["I101"] = m(8, 2) - Fr(7, 3) * m(6, 4)
        out["I102"] = m(6, 4) - 5 * m(4, 4, 2)
    return out


def epsilon(e4, e2=1):
    """eq. (eps_moments): eps = (6 e4 - 2 e2) / (6 e4 + e2)."""
    return (6 * Fr(e4) - 2 * Fr(e2)) / (6 * Fr(e4) + Fr(e2))


# ----------------------------------------------------------- d = 2 lattice pressure tensor terms
def lpt2d_terms(codes):
    """Pair terms of the d = 2 lattice pressure tensor, in units of G c_s^2.

    Each term is (factor, shell_code, a, b, e): it contributes factor * W(shell) *
    psi(x+a) psi(x+b) e^mu e^nu. Groups along a line e = k e_hat follow the regular
    formulas of the appendix; |e|^2 = 5 adds its irregular pairs.
    """
    terms = []
    for code in codes:
        for e in vectors(2, code):
            ex, ey = e
            if code in (1, 2):
                terms.append((Fr(1, 2), code, (0, 0), e, e))
            elif code in (4, 8):
                h = (ex // 2, ey // 2)
                terms.append((Fr(1, 4), code, (0, 0), e, e))
                terms.append((Fr(1, 4), code, h, (-h[0], -h[1]), e))
            elif code in (9, 18):
                t = (ex // 3, ey // 3)
                terms.append((Fr(1, 6), code, (0, 0), e, e))
                terms.append((Fr(1, 3), code, t, (-2 * t[0], -2 * t[1]), e))
            elif code == 16:
                q = (ex // 4, ey // 4)
                terms.append((Fr(1, 8), code, (0, 0), e, e))
                terms.append((Fr(1, 4), code, q, (-3 * q[0], -3 * q[1]), e))
                terms.append((Fr(1, 8), code, (2 * q[0], 2 * q[1]), (-2 * q[0], -2 * q[1]), e))
            elif code == 5:
                terms.append((Fr(1, 4), code, (0, 0), e, e))
            else:
                raise ValueError(code)
        if code == 5:
            irr = [((2, 1), [((-1, 0), (1, 1)), ((-1, -1), (1, 0))]),
                   ((1, 2), [((-1, -1), (0, 1)), ((0, -1), (1, 1))]),
                   ((-1, 2), [((0, -1), (-1, 1)), ((1, -1), (0, 1))]),
                   ((-2, 1), [((1, -1), (-1, 0)), ((1, 0), (-1, 1))])]
            for e, pairs in irr:
                for a, b in pairs:
                    terms.append((Fr(1, 4), 5, a, b, e))
    return terms


def projected_pairs(codes, W: dict, component: str):
    """1D projection (psi depends on x only) of P_N (component 'N' = xx) or P_T ('T' = yy).

    Returns {(p, q) with p <= q: coefficient of psi(x+p) psi(x+q)} in units of G c_s^2.
    """
    out = {}
    for fac, code, a, b, e in lpt2d_terms(codes):
        ee = e[0] * e[0] if component == "N" else e[1] * e[1]
        if ee == 0:
            continue
        key = tuple(sorted((a[0], b[0])))
        out[key] = out.get(key, Fr(0)) + fac * Fr(W[code]) * ee
    return {k: v for k, v in out.items() if v != 0}


def eq1dpnt_coefficients(codes, W: dict, component: str) -> dict:
    """Coefficients a_[-k,0,k], a_[0], b_[-k,k], b_[1,3], b_[1,2] of eq. (1dPNT)."""
    pr = projected_pairs(codes, W, component)
    g = lambda p, q: pr.get(tuple(sorted((p, q))), Fr(0))
    return {
        "a4": g(0, 4), "a3": g(0, 3), "a2": g(0, 2), "a1": g(0, 1), "a0": g(0, 0),
        "b22": g(-2, 2), "b11": g(-1, 1), "b13": g(-1, 3), "b12": g(-1, 2),
        # symmetry partners that eq. (1dPNT) takes as equal
        "_a4m": g(0, -4), "_a3m": g(0, -3), "_a2m": g(0, -2), "_a1m": g(0, -1),
        "_b13m": g(-3, 1), "_b12m": g(-2, 1),
    }


def taylor_c(codes, W: dict, order: int = 4) -> dict:
    """Taylor coefficients c_mn (m <= n) of P_N - P_T in units of G c_s^2.

    psi(x+p) psi(x+q) = sum_{m,n} p^m q^n / (m! n!) psi^(m) psi^(n); c_mn collects both
    orderings of the pair of derivative orders.
    """
    N = projected_pairs(codes, W, "N")
    T = projected_pairs(codes, W, "T")
    diff = dict(N)
    for k, v in T.items():
        diff[k] = diff.get(k, Fr(0)) - v
    c = {}
    for m in range(order + 1):
        for n in range(m, order + 1 - m):
            s = Fr(0)
            for (p, q), kap in diff.items():
                t = Fr(p) ** m * Fr(q) ** n
                if m != n:
                    t += Fr(p) ** n * Fr(q) ** m
                s += kap * t / (factorial(m) * factorial(n))
            c[(m, n)] = s
    return c


def knobs(codes, W: dict) -> dict:
    """sigma_0 = c11 - c02, sigma_1 = c22 - c13 + c04, delta_0 = c02 (d = 2 weights)."""
    c = taylor_c(codes, W)
    return {"sigma0": c[(1, 1)] - c[(0, 2)],
            "sigma1": c[(2, 2)] - c[(1, 3)] + c[(0, 4)],
            "delta0": c[(0, 2)], "c": c}


def project_3d_to_2d(W3: dict) -> dict:
    """eq. (wproj): weights of the 2D projection of a 3D stencil, derived by summing, for each
    2D vector (x, y), the 3D weights of all vectors (x, y, z)."""
    out = {}
    for code, w in W3.items():
        for v in vectors(3, code):
            x, y, z = v
            key = (x, y)
            out[key] = out.get(key, Fr(0)) + Fr(w)
    # group the projected vectors back into 2D shells
    W2 = {}
    for (x, y), w in out.items():
        if (x, y) == (0, 0):
            continue
        code = x * x + y * y
        if code == 9 and sorted((abs(x), abs(y))) != [0, 3]:
            raise ValueError("unexpected projection")
        if code in W2 and W2[code] != w:
            raise ValueError(f"projection is not shell-uniform for |e|^2={code}")
        W2[code] = w
    return {k: v for k, v in W2.items() if v != 0}


# ----------------------------------------------------------- solving weights from conditions
def solve(d: int, codes, conditions: dict) -> dict:
    """Weights W(code) meeting linear conditions {coefficient name: target value}.

    The coefficient of each W in each condition is found by evaluating the condition on the
    unit weight of that shell; the square system is solved exactly (Gauss-Jordan).
    """
    codes = list(codes)
    names = list(conditions)
    if len(names) != len(codes):
        raise ValueError("need as many conditions as shells")
    A = []
    for nm in names:
        A.append([coefficients(d, {c: 1})[nm] for c in codes])
    b = [Fr(conditions[nm]) for nm in names]
    n = len(codes)
    M = [row[:] + [b[i]] for i, row in enumerate(A)]
    for col in range(n):
        piv = next(r for r in range(col, n) if M[r][col] != 0)
        M[col], M[piv] = M[piv], M[col]
        pv = M[col][col]
        M[col] = [v / pv for v in M[col]]
        for r in range(n):
            if r != col and M[r][col] != 0:
                f = M[r][col]
                M[r] = [a - f * c for a, c in zip(M[r], M[col])]
    return {c: M[i][n] for i, c in enumerate(codes)}


def family2d(e4, e8):
    """Shells {1,2,4,5,8} with e2 = 1, I40 = I60 = 0 and free (e4, e8)."""
    return solve(2, [1, 2, 4, 5, 8], {"e2": 1, "I40": 0, "I60": 0, "e4": e4, "e8": e8})


def family3d(e4, e8, w6):
    """Shells {1,2,3,4,5,6,8} with e2 = 1, I40 = I60 = I61 = 0, free (e4, e8) and W(6) = w6."""
    # W(6) is fixed, so move its contribution to the right-hand side and solve for the rest.
    codes = [1, 2, 3, 4, 5, 8]
    targets = {"e2": Fr(1), "I40": Fr(0), "I60": Fr(0), "I61": Fr(0), "e4": Fr(e4), "e8": Fr(e8)}
    c6 = coefficients(3, {6: 1})
    rhs = {k: v - Fr(w6) * c6[k] for k, v in targets.items()}
    W = solve(3, codes, rhs)
    W[6] = Fr(w6)
    return dict(sorted(W.items()))

