"""Order conditions of symmetric compositions and the "optimal" non-recursive schemes
of Sec. II.D (the paper names Kahan and Li's sixth- and eighth-order schemes and
Sofroniou and Spaletta's tenth-order one, and states that Suzuki's fractal is the
optimal fourth-order scheme; it prints none of their coefficients).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke entry point and the
benchmark's CPU-baseline leg may import or call this module; it imports nothing from
the HIP package.

What a composition is (Sec. II.D): U(dt) = S(g_M dt) ... S(g_1 dt), g_1 applied first,
with S a symmetric second-order method (S(h) S(-h) = 1).  Such an S is the exponential
of an odd series, log S(h) = h Y1 + h^3 Y3 + h^5 Y5 + ..., whose terms Y_k do not
commute.  Then log U(dt) = dt Z1 + dt^2 Z2 + ..., and U is of order p exactly when
Z1 = Y1 (sum g = 1) and Z_k = 0 for 2 <= k <= p.  For a palindromic g, U is
symmetric and every even Z_k vanishes by itself.

How it is computed here: in the free associative algebra on the letters Y1, Y3, Y5, ...
(letter Y_k has degree k), truncated above degree p - 1, with the words as a basis.
S(g dt) = exp(sum_k g^k Y_k) (the degree of a word counts the powers of dt), the
product and the logarithm are the truncated power series.  Z_k is a Lie element of
degree k, and a Lie element is fixed by its coefficients on the Lyndon words
(Lyndon's basis is triangular against the words), so those coefficients are the
independent order conditions: 1, 2, 4 and 8 of them at degrees 3, 5, 7 and 9.

The optimal schemes solve: among palindromic g of length M meeting the conditions of
order p, minimise max |g_n| (orders 4, 6, 8 with M = 5, 9, 17), or sum |g_n| (order 10,
M = 35).  That leaves one free parameter at orders 4, 6, 8 and two at order 10.  The
oracle's coefficients are the published ones (gqd_oracle.OPTIMAL_HALVES); this module
pins them: by the order conditions, by the optimality conditions and the criterion's
growth along the solution set around them, and, at orders 4 and 6, by a search from
seeded random starts (Levenberg-Marquardt onto the solution set, then sequential
quadratic programming for the criterion) that reaches the same optimum.  At order 8
such a search finds many local optima; 40000 starts gave none below the published one.
"""
from __future__ import annotations

import itertools
import math
from functools import lru_cache
from typing import Dict, List, Sequence, Tuple

import numpy as np


# ------------------------------------------------------------ truncated free algebra


@lru_cache(maxsize=None)
def _algebra(K: int):
    """Words in odd letters of total degree <= K (index 0: the empty word) and the
    product table (i, j) -> k of concatenations that stay within degree K."""
    letters = list(range(1, K + 1, 2))
    words: List[Tuple[int, ...]] = [()]
    frontier = [()]
    while frontier:
        nxt = []
        for w in frontier:
            for a in letters:
                u = w + (a,)
                if sum(u) <= K:
                    nxt.append(u)
        words.extend(nxt)
        frontier = nxt
    index = {w: i for i, w in enumerate(words)}
    deg = np.array([sum(w) for w in words])
    I, J, Kx = [], [], []
    for i, u in enumerate(words):
        for j, v in enumerate(words):
            if deg[i] + deg[j] <= K:
                I.append(i)
                J.append(j)
                Kx.append(index[u + v])
    return words, index, deg, np.array(I), np.array(J), np.array(Kx)


def _mul(A: np.ndarray, B: np.ndarray, K: int) -> np.ndarray:
    """Product in the truncated algebra; A, B: (batch, words)."""
    words, _, _, I, J, Kx = _algebra(K)
    C = np.zeros_like(A)
    prod = A[:, I] * B[:, J]
    np.add.at(C.T, Kx, prod.T)  # scatter each pair's product onto its concatenation
    return C


def _exp(X: np.ndarray, K: int) -> np.ndarray:
    """exp of an element without constant term: sum_n X^n / n!, n <= K."""
    out = np.zeros_like(X)
    out[:, 0] = 1.0
    term = out.copy()
    for n in range(1, K + 1):
        term = _mul(term, X, K) / n
        out = out + term
    return out


def _log(U: np.ndarray, K: int) -> np.ndarray:
    """log of an element with constant term 1: sum_n (-1)^(n+1) (U - 1)^n / n."""
    D = U.copy()
    D[:, 0] -= 1.0
    out = np.zeros_like(U)
    term = None
    for n in range(1, K + 1):
        term = D.copy() if term is None else _mul(term, D, K)
        out = out + ((-1.0) ** (n + 1) / n) * term
    return out


def composition_log(gammas: np.ndarray, K: int) -> np.ndarray:
    """log of S(g_M dt) ... S(g_1 dt) in the algebra truncated above degree K, for each
    row of gammas (batch, M); S(g dt) = exp(sum_k g^k Y_k) over odd k <= K."""
    gammas = np.atleast_2d(np.asarray(gammas))
    words, index, deg, *_ = _algebra(K)
    B, M = gammas.shape
    U = np.zeros((B, len(words)), dtype=gammas.dtype)
    U[:, 0] = 1.0
    for n in range(M):  # g_1 first: each new factor multiplies from the left
        g = gammas[:, n]
        X = np.zeros((B, len(words)), dtype=gammas.dtype)
        for k in range(1, K + 1, 2):
            X[:, index[(k,)]] = g ** k
        U = _mul(_exp(X, K), U, K)
    return _log(U, K)


def is_lyndon(w: Sequence[int]) -> bool:
    """A word is Lyndon when it is strictly smaller than each of its proper rotations."""
    w = tuple(w)
    return len(w) > 0 and all(w < w[i:] + w[:i] for i in range(1, len(w)))


def lyndon_words(K: int, degrees: Sequence[int]) -> List[Tuple[int, ...]]:
    words, *_ = _algebra(K)
    return [w for w in words if sum(w) in degrees and is_lyndon(w)]


def palindrome(half: Sequence[float]) -> np.ndarray:
    """Full coefficient list g_1..g_M (M odd) from g_1..g_(M+1)/2."""
    h = list(half)
    return np.array(h + h[-2::-1])


def order_conditions(half: np.ndarray, order: int) -> np.ndarray:
    """Residuals of the order conditions of the palindromic composition with these
    first (M + 1)/2 coefficients: sum g - 1, then the Lyndon-word coefficients of
    log U at every odd degree 3 .. order - 1.  (batch, conditions)."""
    half = np.atleast_2d(half)
    K = order - 1
    full = np.concatenate([half, half[:, -2::-1]], axis=1)
    Z = composition_log(full, K)
    _, index, *_ = _algebra(K)
    ly = lyndon_words(K, range(3, K + 1, 2))
    cols = [Z[:, index[(1,)]] - 1.0] + [Z[:, index[w]] for w in ly]
    return np.stack(cols, axis=1)


def even_terms(half: np.ndarray, order: int) -> float:
    """Largest |coefficient| of log U at even degrees 2 .. order - 1 (zero for every
    palindromic composition)."""
    half = np.atleast_2d(half)
    K = order - 1
    full = np.concatenate([half, half[:, -2::-1]], axis=1)
    Z = composition_log(full, K)
    _, _, deg, *_ = _algebra(K)
    even = (deg % 2 == 0) & (deg > 0)
    return float(np.max(np.abs(Z[:, even])))


def condition_count(order: int) -> int:
    return 1 + len(lyndon_words(order - 1, range(3, order, 2)))


# --------------------------------------------------------------------- the search


def _jac(f, x: np.ndarray) -> np.ndarray:
    """Jacobian of a real-analytic f by complex steps (exact to rounding): column i is
    Im f(x + i h e_i) / h."""
    h = 1e-40
    n = x.size
    Z = np.asarray(x, dtype=np.complex128)[None, :] + 1j * h * np.eye(n)
    return (np.asarray(f(Z)).imag / h).T


def _criterion(half: np.ndarray, kind: str) -> float:
    g = palindrome(half)
    return float(np.max(np.abs(g))) if kind == "max" else float(np.sum(np.abs(g)))


def newton(cond, x: np.ndarray, iters: int = 200, tol: float = 1e-15):
    """Levenberg-Marquardt onto cond(x) = 0 with minimum-norm steps (the system has
    fewer conditions than unknowns): dx = J^T (J J^T + mu 1)^-1 c, mu adapted to the
    progress; returns (x, max |cond|)."""
    c = cond(x)
    mu = 1e-3
    for _ in range(iters):
        err = float(np.max(np.abs(c)))
        if err <= tol:
            break
        J = _jac(cond, x)
        A = J @ J.T
        while True:
            y = np.linalg.solve(A + mu * np.eye(A.shape[0]), c)
            xn = x - J.T @ y
            cn = cond(xn)
            if np.linalg.norm(cn) < np.linalg.norm(c):
                x, c = xn, cn
                mu = max(mu / 10.0, 1e-15)
                break
            mu *= 10.0
            if mu > 1e8:
                return x, float(np.max(np.abs(c)))
    return x, float(np.max(np.abs(c)))


def _jac_batch(condb, X: np.ndarray) -> np.ndarray:
    """Jacobians of a batched real-analytic condb at every row of X by complex steps:
    (batch, conditions, unknowns)."""
    B, n = X.shape
    h = 1e-40
    Z = (X.astype(np.complex128)[:, None, :] + 1j * h * np.eye(n)[None, :, :]).reshape(B * n, n)
    return (condb(Z).imag / h).reshape(B, n, -1).transpose(0, 2, 1)


def newton_batch(condb, X: np.ndarray, iters: int = 150, tol: float = 1e-15):
    """Levenberg-Marquardt (minimum-norm damped steps, one damping per start) from every
    row of X at once; returns (X, max |cond| per row)."""
    X = X.copy()
    C = condb(X)
    mu = np.full(X.shape[0], 1e-3)
    for _ in range(iters):
        err = np.max(np.abs(C), axis=1)
        live = (err > tol) & (mu < 1e8)
        if not np.any(live):
            break
        Xl, Cl = X[live], C[live]
        J = _jac_batch(condb, Xl)
        A = J @ J.transpose(0, 2, 1) + mu[live][:, None, None] * np.eye(J.shape[1])[None]
        y = np.linalg.solve(A, Cl[:, :, None])[:, :, 0]
        Xn = Xl - np.einsum("bij,bi->bj", J, y)
        Cn = condb(Xn)
        better = np.linalg.norm(Cn, axis=1) < np.linalg.norm(Cl, axis=1)
        idx = np.flatnonzero(live)
        X[idx[better]] = Xn[better]
        C[idx[better]] = Cn[better]
        mu[idx[better]] = np.maximum(mu[idx[better]] / 10.0, 1e-15)
        mu[idx[~better]] *= 10.0
    return X, np.max(np.abs(C), axis=1)


def refine(cond, x: np.ndarray, kind: str = "max", iters: int = 40):
    """The criterion's optimum near x to full precision, from its optimality conditions.
    kind "max" with two or more largest |g_n| within 1e-6 of each other: the square
    system cond(x) = 0, |x_a| = |x_b|.  Otherwise (one largest |g_n| for "max", or
    "sum" with no g_n at zero) the Lagrange conditions cond(x) = 0,
    grad f(x) = J(x)^T lam, solved for (x, lam) by Newton with a difference Jacobian.
    Returns x (unchanged when the iteration does not converge)."""
    nh = x.size
    w = np.array([2.0] * (nh - 1) + [1.0])  # multiplicity of each distinct coefficient
    ax = np.abs(x)
    order_ = np.argsort(-ax)
    if kind == "max" and ax[order_[0]] - ax[order_[1]] < 1e-6:
        a, b = order_[0], order_[1]
        sa, sb = np.sign(x[a]), np.sign(x[b])
        F = lambda z: np.concatenate([cond(z), [sa * z[a] - sb * z[b]]])  # noqa: E731
        z = x.copy()
        for _ in range(iters):
            f = F(z)
            if np.max(np.abs(f)) < 1e-16:
                break
            Jf = np.vstack([_jac(cond, z), (sa * np.eye(nh)[a] - sb * np.eye(nh)[b])[None]])
            z = z - np.linalg.lstsq(Jf, f, rcond=None)[0]
        return z if np.max(np.abs(cond(z))) < 1e-14 else x
    if kind == "max":
        a = order_[0]
        grad = lambda z: np.sign(z[a]) * np.eye(nh)[a]  # noqa: E731
    else:
        grad = lambda z: w * np.sign(z)  # noqa: E731
    J = _jac(cond, x)
    lam = np.linalg.lstsq(J.T, grad(x), rcond=None)[0]
    nc = lam.size

    def F(v):
        z, l = v[:nh], v[nh:]
        return np.concatenate([cond(z), grad(x) - _jac(cond, z).T @ l])

    v = np.concatenate([x, lam])
    for _ in range(iters):
        f = F(v)
        if np.max(np.abs(f)) < 1e-15:
            break
        h = 1e-7
        Jf = np.stack([(F(v + h * e) - F(v - h * e)) / (2 * h) for e in np.eye(v.size)], axis=1)
        v = v - np.linalg.lstsq(Jf, f, rcond=None)[0]
    z = v[:nh]
    ok = np.max(np.abs(cond(z))) < 1e-14 and np.all(np.sign(z) == np.sign(x))
    return z if ok else x


def improve(order: int, x: np.ndarray, kind: str):
    """From a point x on the solution set: the criterion's local optimum under the order
    conditions (sequential quadratic programming, then Gauss-Newton back onto the
    conditions and the optimality conditions to full precision), or None."""
    from scipy.optimize import minimize

    nh = x.size
    nc = condition_count(order)

    def cond(z):
        z = np.asarray(z)
        return order_conditions(z, order) if z.ndim == 2 else order_conditions(z, order)[0]

    if kind == "max":
        z0 = np.concatenate([x, [_criterion(x, "max")]])
        cons = [{"type": "eq", "fun": lambda z: cond(z[:-1]),
                 "jac": lambda z: np.hstack([_jac(cond, z[:-1]), np.zeros((nc, 1))])},
                {"type": "ineq", "fun": lambda z: np.concatenate([z[-1] - z[:-1], z[-1] + z[:-1]])}]
        res = minimize(lambda z: z[-1], z0, jac=lambda z: np.eye(z.size)[-1], constraints=cons,
                       method="SLSQP", options={"maxiter": 300, "ftol": 1e-15})
        y = res.x[:-1]
    else:
        # sum |g| = 2 sum_{n < nh} |g_n| + |g_nh|, with g = u - v, u, v >= 0
        w = np.array([2.0] * (nh - 1) + [1.0])
        z0 = np.concatenate([np.maximum(x, 0), np.maximum(-x, 0)])
        cons = [{"type": "eq", "fun": lambda z: cond(z[:nh] - z[nh:]),
                 "jac": lambda z: np.hstack([_jac(cond, z[:nh] - z[nh:]), -_jac(cond, z[:nh] - z[nh:])])}]
        res = minimize(lambda z: float(np.dot(w, z[:nh] + z[nh:])), z0,
                       jac=lambda z: np.concatenate([w, w]), constraints=cons,
                       bounds=[(0, None)] * (2 * nh), method="SLSQP", options={"maxiter": 500, "ftol": 1e-15})
        y = res.x[:nh] - res.x[nh:]
    y, err = newton(cond, y)
    if err > 1e-14:
        return None
    return refine(cond, y, kind)


def optimise(order: int, M: int, kind: str = "max", starts: int = 400, seed: int = 1,
             scale: float = 0.8, seeds=(), log=None) -> Dict:
    """Best palindromic composition of M substeps and the given order: Levenberg-Marquardt
    from `starts` seeded random points (all at once) onto the solution set, plus any
    given feasible `seeds`, then improve() from each; the best criterion value wins."""
    nh = (M + 1) // 2
    rng = np.random.default_rng(seed)
    condb = lambda X: order_conditions(X, order)  # noqa: E731
    X, err = newton_batch(condb, rng.uniform(-scale, scale, size=(starts, nh)))
    cands = [x for x in X[err < 1e-12]] + [np.asarray(z, dtype=np.float64) for z in seeds]
    if log:
        log(f"order {order} M {M}: {len(cands)} feasible starting points")
    best = None
    for k, x in enumerate(cands):
        y = improve(order, x, kind)
        if y is None:
            continue
        c = _criterion(y, kind)
        if best is None or c < best[0] - 1e-12:
            best = (c, y)
            if log:
                log(f"order {order} M {M}: candidate {k}: {kind} |g| = {c:.15f}")
    if best is None:
        raise RuntimeError(f"no composition of order {order} with {M} substeps found")
    half = best[1]
    return {"order": order, "M": M, "criterion": kind, "value": best[0], "half": half.tolist(),
            "gammas": palindrome(half).tolist(),
            "residual": float(np.max(np.abs(order_conditions(half, order))))}


def tangent_basis(half: np.ndarray, order: int) -> np.ndarray:
    """Orthonormal basis (rows) of the directions along the solution set at half: the
    null space of the conditions' Jacobian."""
    cond = lambda z: order_conditions(z, order)  # noqa: E731
    J = _jac(cond, np.asarray(half, dtype=np.float64))
    return np.linalg.svd(J)[2][J.shape[0]:]


def optimality_residual(half: np.ndarray, order: int, kind: str) -> float:
    """Largest part of the criterion's gradient along the solution set at half; zero at
    a smooth stationary point (for "max": a single largest |g_n|; for "sum": no g_n at
    zero).  The gradient of max |g| is sign(g_a) e_a at the largest entry a; that of
    sum |g| over the palindrome is w sign(g), w the multiplicity of each entry."""
    half = np.asarray(half, dtype=np.float64)
    nh = half.size
    if kind == "max":
        a = int(np.argmax(np.abs(half)))
        grad = np.sign(half[a]) * np.eye(nh)[a]
    else:
        grad = np.array([2.0] * (nh - 1) + [1.0]) * np.sign(half)
    T = tangent_basis(half, order)
    return float(np.max(np.abs(T @ grad)))


def neighbours(half: np.ndarray, order: int, step: float) -> List[np.ndarray]:
    """Points of the solution set about `step` away from half along each tangent
    direction and its opposite (and the diagonals when there are two), each projected
    back onto the conditions by Levenberg-Marquardt."""
    half = np.asarray(half, dtype=np.float64)
    T = tangent_basis(half, order)
    dirs = list(T)
    if len(T) == 2:
        dirs += [(T[0] + T[1]) / math.sqrt(2), (T[0] - T[1]) / math.sqrt(2)]
    cond = lambda z: order_conditions(z, order) if np.ndim(z) == 2 else order_conditions(z, order)[0]  # noqa: E731
    out = []
    for d in dirs:
        for sgn in (1.0, -1.0):
            z, err = newton(cond, half + sgn * step * d)
            if err < 1e-14:
                out.append(z)
    return out
