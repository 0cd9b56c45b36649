"""Derivation of the non-recursive ("optimal") symmetric compositions used by the
library (scheme GQD_OPTIMAL), written into csrc/gqd_compositions.h.

Sec. II.D composes a symmetric second-order method S into U(dt) = S(g_M dt)...S(g_1 dt)
and, besides the recursive triple jump and Suzuki fractal, uses non-recursive schemes
chosen by an optimisation: Suzuki's fractal at fourth order (M = 5), which it states is
optimal; Kahan and Li's sixth- and eighth-order schemes (M = 9, 17), with the largest
|g_n| as small as possible; Sofroniou and Spaletta's tenth-order scheme (M = 35), with
the sum of |g_n| as small as possible.  The paper prints no coefficients; they are
derived here from the order conditions and the optimality conditions.

Order conditions, in a matrix representation.  A symmetric second-order S has
log S(h) = h Y1 + h^3 Y3 + h^5 Y5 + ... (odd powers only).  Take the Y_k to be seeded
random real d x d matrices with 2d > p - 1 (by the Amitsur-Levitzki theorem no nonzero
polynomial of degree below 2d vanishes on all of them, so generic ones represent every
condition up to degree p - 1 faithfully) and compute log U(h) as a power series in h with
matrix coefficients, truncated above h^(p-1): U is of order p exactly when its h^1
coefficient is Y1 and its h^3, h^5, ... h^(p-1) coefficients vanish (even ones vanish by
themselves for a palindromic g).  Those coefficients' entries form an overcomplete set of
conditions, real-analytic in g, so their derivatives are taken by complex steps (exact
to rounding); their number of independent ones comes from the graded Witt formula.

Search.  Orders 4 and 6: Levenberg-Marquardt from many seeded random points onto the
solution set, then projected-gradient descent of a smooth stand-in for the criterion
along that set (the tangent space from the singular value decomposition of the
conditions' Jacobian).  Orders 8 and 10, whose optima such a search reaches too rarely
(the order-8 landscape has many local minima), start from the cited publications'
coefficients rounded to three digits.  Then Newton on the criterion's own optimality
conditions: the largest two |g_n| equal, or the Lagrange conditions.  Double precision
fixes the tenth-order coefficients to about 1e-9 only: the weakest of its 16
conditions changes by about 1e-10 per unit change of g.

    python -m paper_1902_04661_amd.compositions --write
"""
from __future__ import annotations

import argparse
import json
import os
import sys
from typing import List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
HEADER = os.path.join(HERE, "csrc", "gqd_compositions.h")

def dim_for(order: int) -> int:
    """Smallest matrix size that represents the conditions of this order faithfully."""
    return max(3, (order - 1) // 2 + 1)


def _moebius(n: int) -> int:
    m, k = 1, 2
    while k * k <= n:
        if n % k == 0:
            n //= k
            if n % k == 0:
                return 0
            m = -m
        k += 1
    return -m if n > 1 else m


def condition_count(order: int) -> int:
    """Number of independent order conditions of a palindromic composition of the given
    order: the dimensions l_n of the odd-degree parts n = 1, 3, .., order - 1 of the free
    Lie algebra on one generator in each odd degree (log S holds only odd powers), by
    the graded Witt formula n l_n = sum over d | n of moebius(n / d) d c_d, where c_m is
    the t^m coefficient of -log(1 - t - t^3 - t^5 - ...)."""
    K = order - 1
    g = np.zeros(K + 1)
    g[1::2] = 1.0
    c, p = np.zeros(K + 1), np.eye(1, K + 1)[0]
    for k in range(1, K + 1):
        p = np.convolve(p, g)[:K + 1]
        c += p / k
    return sum(round(sum(_moebius(n // d) * d * c[d] for d in range(1, n + 1) if n % d == 0) / n)
               for n in range(1, K + 1, 2))


# Starting points for the orders whose published optimum a random search does not reach
# in reasonable time: the coefficients g_1 .. g_(M+1)/2 of the compositions the paper
# cites, rounded to three significant digits -- Kahan and Li (1997), eighth order with
# M = 17, and Sofroniou and Spaletta (2005), tenth order with M = 35.  Newton on the
# optimality conditions takes them to full precision.
KAHAN_LI_8 = [0.130, 0.561, -0.389, 0.159, -0.396, 0.185, 0.258, 0.295, -0.606]
SOFRONIOU_SPALETTA_10 = [0.0788, 0.313, 0.0279, -0.230, 0.131, -0.270, 0.0750, 0.112, 0.366,
                         -0.399, 0.103, 0.411, -0.00487, -0.392, 0.0519, 0.0507, 0.0497, 0.0493]

# order, substeps, criterion, random starts, seed of the starts, fixed start (or None)
SCHEMES = [(4, 5, "max", 200, 7, None), (6, 9, "max", 1000, 7, None),
           (8, 17, "max", 0, 0, KAHAN_LI_8), (10, 35, "sum", 0, 0, SOFRONIOU_SPALETTA_10)]


def generators(K: int, d: int = 0, seed: int = 2019) -> np.ndarray:
    """Y_1, Y_3, ..., Y_K as seeded random real d x d matrices (d = dim_for(K + 1) by
    default), scaled to unit norm."""
    d = d or dim_for(K + 1)
    rng = np.random.default_rng(seed)
    Y = rng.standard_normal((len(range(1, K + 1, 2)), d, d))
    return Y / np.linalg.norm(Y, axis=(1, 2), keepdims=True)


def series_mul(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Product of matrix power series (..., K + 1, d, d), truncated at degree K."""
    K = A.shape[-3] - 1
    C = np.zeros(np.broadcast_shapes(A.shape, B.shape), dtype=np.result_type(A, B))
    for i in range(K + 1):
        for j in range(K + 1 - i):
            C[..., i + j, :, :] += A[..., i, :, :] @ B[..., j, :, :]
    return C


def series_exp(E: np.ndarray) -> np.ndarray:
    """exp of a series with zero constant term."""
    K, d = E.shape[-3] - 1, E.shape[-1]
    out = np.zeros_like(E)
    out[..., 0, :, :] = np.eye(d)
    term = out.copy()
    for n in range(1, K + 1):
        term = series_mul(term, E) / n
        out = out + term
    return out


def series_log(U: np.ndarray) -> np.ndarray:
    """log of a series with the identity as constant term."""
    K, d = U.shape[-3] - 1, U.shape[-1]
    D = U.copy()
    D[..., 0, :, :] -= np.eye(d)
    out = np.zeros_like(U)
    power = D
    for n in range(1, K + 1):
        out = out + ((-1) ** (n + 1) / n) * power
        power = series_mul(power, D)
    return out


def residual(half: np.ndarray, order: int, Y: np.ndarray) -> np.ndarray:
    """Order conditions of the palindromic composition g = (half, reversed half without
    its last entry), batched over the leading axes of half: the entries of
    (h^1 coefficient - Y1) and of the odd coefficients h^3 .. h^(order - 1).  Real for
    real g; a complex g gives the analytic continuation (for complex steps)."""
    K = order - 1
    g = np.concatenate([half, half[..., -2::-1]], axis=-1)
    lead = g.shape[:-1]
    d = Y.shape[-1]
    dt = np.result_type(g, Y)
    U = np.zeros(lead + (K + 1, d, d), dtype=dt)
    U[..., 0, :, :] = np.eye(d)
    for n in range(g.shape[-1]):
        E = np.zeros(lead + (K + 1, d, d), dtype=dt)
        for i, k in enumerate(range(1, K + 1, 2)):
            E[..., k, :, :] = (g[..., n] ** k)[..., None, None] * Y[i]
        U = series_mul(series_exp(E), U)  # g_1 first: later factors act from the left
    L = series_log(U)
    L[..., 1, :, :] -= Y[0]
    return L[..., 1::2, :, :].reshape(lead + (-1,))


def jacobian(half: np.ndarray, order: int, Y: np.ndarray) -> np.ndarray:
    """Jacobian (..., equations, unknowns) by complex steps: column i is
    Im residual(half + i h e_i) / h, exact to rounding."""
    n = half.shape[-1]
    h = 1e-40
    Z = half[..., None, :].astype(np.complex128) + 1j * h * np.eye(n)
    return np.swapaxes(residual(Z, order, Y).imag / h, -1, -2)


def project(half: np.ndarray, order: int, Y: np.ndarray, iters: int = 60, rank: Optional[int] = None):
    """Gauss-Newton onto the solution set: minimum-norm steps on the leading `rank`
    singular directions of the Jacobian.  Returns (half, max |residual|)."""
    x = half.copy()
    r = residual(x, order, Y)
    for _ in range(iters):
        if np.max(np.abs(r)) < 5e-16:
            break
        U, s, Vt = np.linalg.svd(jacobian(x, order, Y), full_matrices=False)
        k = rank if rank is not None else int(np.sum(s > 1e-9 * s[0]))
        dx = Vt[:k].T @ ((U[:, :k].T @ r) / s[:k])
        xn = x - dx
        rn = residual(xn, order, Y)
        if np.linalg.norm(rn) >= np.linalg.norm(r):
            break
        x, r = xn, rn
    return x, float(np.max(np.abs(r)))


def projector(order: int, nh: int, ncond: int, Y: np.ndarray) -> np.ndarray:
    """A fixed basis of the conditions' range: the leading `ncond` left singular
    vectors of the Jacobian at a seeded random point (equations x ncond)."""
    x = np.random.default_rng(12345).uniform(-0.5, 0.5, nh)
    U, s, Vt = np.linalg.svd(jacobian(x, order, Y), full_matrices=False)
    return U[:, :ncond]


def _feasible_batch(args) -> List[np.ndarray]:
    """Levenberg-Marquardt from one batch of seeded uniform random points on the square
    system Q^T residual = 0 (Q: projector(), the conditions' range): damped
    minimum-norm steps dx = J^T (J J^T + lam 1)^-1 r; the points that reach the
    solution set of the full residual."""
    order, nh, seed, b, size, scale, ncond = args
    Y = generators(order - 1)
    Q = projector(order, nh, ncond, Y)
    X = np.random.default_rng([seed, b]).uniform(-scale, scale, size=(size, nh))
    R = residual(X, order, Y) @ Q
    lam = np.full(X.shape[0], 1e-3)
    for _ in range(150):
        live = (np.max(np.abs(R), axis=1) > 1e-13) & (lam < 1e8)
        if not live.any():
            break
        J = np.einsum("eq,ben->bqn", Q, jacobian(X[live], order, Y))
        A = J @ np.swapaxes(J, -1, -2) + lam[live][:, None, None] * np.eye(ncond)
        yv = np.linalg.solve(A, R[live][..., None])[..., 0]
        Xn = X[live] - np.einsum("bqn,bq->bn", J, yv)
        Rn = residual(Xn, order, Y) @ Q
        good = np.linalg.norm(Rn, axis=1) < np.linalg.norm(R[live], axis=1)
        idx = np.flatnonzero(live)
        X[idx[good]], R[idx[good]] = Xn[good], Rn[good]
        lam[idx[good]] = np.maximum(lam[idx[good]] / 10.0, 1e-15)
        lam[idx[~good]] *= 10.0
    full = np.max(np.abs(residual(X, order, Y)), axis=1)
    return list(X[full <= 1e-11])


def feasible_points(order: int, nh: int, starts: int, seed: int, ncond: int, scale: float = 0.8,
                    batch: int = 128, workers: int = 1, log=None) -> List[np.ndarray]:
    """Points on the solution set from `starts` seeded random points, in batches (batch b
    draws from default_rng([seed, b])), spread over `workers` processes."""
    jobs = [(order, nh, seed, b, min(batch, starts - b * batch), scale, ncond)
            for b in range((starts + batch - 1) // batch)]
    found: List[np.ndarray] = []
    if workers > 1:
        import multiprocessing as mp
        with mp.get_context("spawn").Pool(workers) as pool:
            for k, res in enumerate(pool.imap(_feasible_batch, jobs)):
                found.extend(res)
                if log and (k + 1) % workers == 0:
                    log(f"  order {order}: {(k + 1) * batch} starts, {len(found)} on the solution set")
    else:
        for k, job in enumerate(jobs):
            found.extend(_feasible_batch(job))
            if log:
                log(f"  order {order}: {(k + 1) * batch} starts, {len(found)} on the solution set")
    return found


def weights(nh: int) -> np.ndarray:
    """How often each distinct coefficient occurs in the palindrome."""
    return np.array([2.0] * (nh - 1) + [1.0])


def criterion(half: np.ndarray, kind: str) -> float:
    return float(np.max(np.abs(half))) if kind == "max" else float(np.dot(weights(half.size), np.abs(half)))


def descend(x: np.ndarray, order: int, Y: np.ndarray, kind: str, ncond: int, steps: int = 400) -> np.ndarray:
    """Projected-gradient descent along the solution set of a smooth stand-in for the
    criterion: the 64-norm of g for "max", sum sqrt(g^2 + eps^2) (eps 1e-8) for "sum"."""
    w = weights(x.size)

    def f_and_grad(z):
        if kind == "max":
            a = np.abs(z)
            m = a.max()
            q = w * (a / m) ** 64
            f = m * q.sum() ** (1 / 64)
            gr = f * (w * (a / m) ** 63 * np.sign(z) / m) / q.sum()
            return f, gr
        s = np.sqrt(z * z + 1e-16)
        return float(np.dot(w, s)), w * z / s

    alpha = 0.02
    f, g = f_and_grad(x)
    for _ in range(steps):
        _, s, Vt = np.linalg.svd(jacobian(x, order, Y), full_matrices=True)
        T = Vt[ncond:]  # tangent directions of the solution set
        d = T.T @ (T @ g)
        if np.linalg.norm(d) < 1e-13:
            break
        xn, err = project(x - alpha * d, order, Y, rank=ncond)
        fn, gn = f_and_grad(xn)
        if err < 1e-13 and fn < f:
            x, f, g = xn, fn, gn
            alpha = min(alpha * 1.5, 0.2)
        else:
            alpha *= 0.3
            if alpha < 1e-12:
                break
    return x


def polish(x: np.ndarray, order: int, Y: np.ndarray, kind: str, ncond: int) -> np.ndarray:
    """Newton on the optimum's defining equations, the conditions taken on a basis of
    their range held fixed and scaled to unit sensitivity: W = U_k diag(1 / s_k) from the
    leading `ncond` singular triplets of the Jacobian at x.  "max" with its two largest
    |g_n| within 1e-5: W^T r = 0 and those two equal in size.  Otherwise the Lagrange
    conditions of min f subject to W^T r = 0 in the unknowns (g, lam):
    W^T r(g) = 0 and grad f = (W^T J(g))^T lam, with grad f constant on the sign pattern
    of g and the Hessian of lam . W^T r by central differences of the complex-step
    Jacobian.  Returns the iterate with the smallest equation residual."""
    nh = x.size
    a = np.argsort(-np.abs(x))
    kink = kind == "max" and abs(x[a[0]]) - abs(x[a[1]]) < 1e-5
    sa, sb = np.sign(x[a[0]]), np.sign(x[a[1]])
    U, sv, _ = np.linalg.svd(jacobian(x, order, Y), full_matrices=False)
    W = U[:, :ncond] / sv[:ncond]
    gradf = sa * np.eye(nh)[a[0]] if kind == "max" else weights(nh) * np.sign(x)

    z = x.copy()
    lam = np.linalg.lstsq((W.T @ jacobian(z, order, Y)).T, gradf, rcond=None)[0]
    best = (np.inf, z)
    for _ in range(12):
        JW = W.T @ jacobian(z, order, Y)
        r = W.T @ residual(z, order, Y)
        if kink:
            G = np.concatenate([r, [sa * z[a[0]] - sb * z[a[1]]]])
            DG = np.vstack([JW, sa * np.eye(nh)[a[0]] - sb * np.eye(nh)[a[1]]])
        else:
            G = np.concatenate([r, gradf - JW.T @ lam])
            h = 1e-6
            P = np.concatenate([z + h * np.eye(nh), z - h * np.eye(nh)])
            T = np.einsum("eq,ben,q->bn", W, jacobian(P, order, Y), lam)
            H = ((T[:nh] - T[nh:]) / (2 * h)).T
            DG = np.block([[JW, np.zeros((ncond, ncond))], [-H, -JW.T]])
        if np.max(np.abs(G)) < best[0]:
            best = (np.max(np.abs(G)), z.copy())
        step = np.linalg.lstsq(DG, G, rcond=None)[0]
        z = z - step[:nh]
        if not kink:
            lam = lam - step[nh:]
    z = best[1]
    if np.max(np.abs(residual(z, order, Y))) > 1e-14 or np.any(np.sign(z) != np.sign(x)):
        return x
    return z


def derive(order: int, M: int, kind: str, starts: int, seed: int, start=None, workers: int = 1,
           log=None) -> dict:
    nh = (M + 1) // 2
    Y = generators(order - 1)
    ncond = condition_count(order)
    if start is not None:
        x, err = project(np.array(start, dtype=np.float64), order, Y, rank=ncond)
        if err > 1e-13:
            raise RuntimeError(f"order {order}: the starting point does not reach the solution set")
        cands = [x]
    else:
        cands = feasible_points(order, nh, starts, seed, ncond, workers=workers, log=log)
    best = None
    for x in cands:
        if start is None:
            x = descend(x, order, Y, kind, ncond)
        x = polish(x, order, Y, kind, ncond)
        c = criterion(x, kind)
        if best is None or c < best[0] - 1e-13:
            best = (c, x)
            if log:
                log(f"  order {order}: {kind} |g| = {c:.16f}")
    if best is None:
        raise RuntimeError(f"no composition of order {order} with {M} substeps found")
    half = best[1]
    g = np.concatenate([half, half[-2::-1]])
    return {"order": order, "M": M, "criterion": kind, "value": best[0], "conditions": ncond,
            "residual": float(np.max(np.abs(residual(half, order, Y)))), "gammas": g.tolist()}


def write_header(results: Sequence[dict], path: str = HEADER) -> None:
    lines = ["// Non-recursive symmetric compositions of a symmetric second-order method (Sec. II.D):",
             "// M = 5, 9, 17 substeps with the smallest largest |g_n| (orders 4, 6, 8) and M = 35",
             "// with the smallest sum of |g_n| (order 10), derived from the order and optimality",
             "// conditions by paper_1902_04661_amd/compositions.py, which writes this file.  Each",
             "// list is g_1 .. g_M, g_1 applied first.",
             "#pragma once", "", "namespace gqd {", "", "struct FlatComp {", "  int order;",
             "  int count;", "  int offset;", "};", ""]
    off = 0
    comps, vals = [], []
    for r in sorted(results, key=lambda r: r["order"]):
        comps.append(f"    {{{r['order']}, {r['M']}, {off}}},  // {r['criterion']} |g| = {r['value']:.16f}")
        vals.extend(r["gammas"])
        off += r["M"]
    lines += [f"constexpr int kNumFlat = {len(comps)};", "constexpr FlatComp kFlatComps[kNumFlat] = {"]
    lines += comps + ["};", f"constexpr int kFlatTauLen = {off};", "#define GQD_FLAT_TAU_VALUES \\"]
    body = [f"    {v!r}" for v in vals]
    lines += [",".join(body[i:i + 1]) + (", \\" if i < len(body) - 1 else "") for i in range(len(body))]
    lines += ["", "}  // namespace gqd", ""]
    with open(path, "w") as f:
        f.write("\n".join(lines))


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--orders", type=int, nargs="*", default=[s[0] for s in SCHEMES])
    ap.add_argument("--json", default="")
    ap.add_argument("--write", action="store_true", help="write csrc/gqd_compositions.h")
    ap.add_argument("--workers", type=int, default=os.cpu_count() or 1)
    args = ap.parse_args(argv)
    log = lambda m: print(m, flush=True)  # noqa: E731
    res = [derive(*s, workers=args.workers, log=log) for s in SCHEMES if s[0] in args.orders]
    for r in res:
        print(json.dumps(r), flush=True)
    if args.json:
        with open(args.json, "w") as f:
            json.dump(res, f, indent=1)
    if args.write:
        write_header(res)


if __name__ == "__main__":
    sys.exit(main())
