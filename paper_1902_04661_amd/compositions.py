"""Derivation of the non-recursive ("optimal") symmetric compositions used by the
library (scheme GQD_OPTIMAL), written into csrc/gqd_compositions.h.

Sec. II.D composes a symmetric second-order method S into U(dt) = S(g_M dt)...S(g_1 dt)
and, besides the recursive triple jump and Suzuki fractal, names non-recursive schemes
chosen by an optimisation: the largest |g_n| as small as possible for the order (sixth
order with M = 9, eighth order with M = 17; it states that Suzuki's fractal is the
optimal fourth-order one), and the sum of |g_n| as small as possible at tenth order with
M = 35.  The paper prints no coefficients, so they are derived here from the order
conditions.

Order conditions, in a matrix representation.  A symmetric second-order S has
log S(h) = h Y1 + h^3 Y3 + h^5 Y5 + ... (odd powers only).  Take the Y_k to be seeded
random real d x d matrices with 2d > p - 1 (by the Amitsur-Levitzki theorem no nonzero
polynomial of degree below 2d vanishes on all of them, so generic ones represent every
condition up to degree p - 1 faithfully) and compute log U(h) as a power series in h with matrix
coefficients, truncated above h^(p-1): U is of order p exactly when its h^1 coefficient
is Y1 and its h^3, h^5, ... h^(p-1) coefficients vanish (even ones vanish by themselves
for a palindromic g).  Those coefficients' entries form an overcomplete set of
conditions, real-analytic in g, so their derivatives are taken by complex steps (exact
to rounding); they are solved in the least-squares sense with rank-revealing steps.

Search.  Levenberg-Marquardt from many seeded random points onto the solution set, then
projected-gradient descent of a smooth stand-in for the criterion along that set
(the tangent space from the singular value decomposition of the conditions' Jacobian),
then Newton on the criterion's own optimality conditions: the largest two |g_n| equal, or
the gradient in the span of the conditions' gradients.

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


# order, substeps, criterion, random starts, seed of the starts
SCHEMES = [(4, 5, "max", 200, 7), (6, 9, "max", 1000, 7), (8, 17, "max", 40000, 7), (10, 35, "sum", 40000, 7)]


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


def _feasible_batch(args) -> List[np.ndarray]:
    """Levenberg-Marquardt from one batch of seeded uniform random points: damped
    minimum-norm steps on the `ncond` leading singular directions of each Jacobian
    (the conditions' rank); the points that reach the solution set."""
    order, nh, seed, b, size, scale, ncond = args
    Y = generators(order - 1)
    X = np.random.default_rng([seed, b]).uniform(-scale, scale, size=(size, nh))
    R = residual(X, order, Y)
    lam = np.full(X.shape[0], 1e-3)
    for _ in range(150):
        live = (np.max(np.abs(R), axis=1) > 1e-11) & (lam < 1e8)
        if not live.any():
            break
        U, sv, Vt = np.linalg.svd(jacobian(X[live], order, Y), full_matrices=False)
        U, sv, Vt = U[..., :ncond], sv[..., :ncond], Vt[..., :ncond, :]
        coef = np.einsum("bek,be->bk", U, R[live]) * sv / (sv * sv + lam[live][:, None])
        Xn = X[live] - np.einsum("bkn,bk->bn", Vt, coef)
        Rn = residual(Xn, order, Y)
        good = np.linalg.norm(Rn, axis=1) < np.linalg.norm(R[live], axis=1)
        idx = np.flatnonzero(live)
        X[idx[good]], R[idx[good]] = Xn[good], Rn[good]
        lam[idx[good]] = np.maximum(lam[idx[good]] / 10.0, 1e-15)
        lam[idx[~good]] *= 10.0
    ok = np.max(np.abs(R), axis=1) <= 1e-11
    return list(X[ok])


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
    """Gauss-Newton on the optimum's defining equations, with the conditions taken on
    their `ncond` leading singular directions.  "max" with its two largest |g_n| within
    1e-5: those two equal in size.  Otherwise the criterion's gradient g has no part
    along the solution set: (1 - J^+ J) g = 0."""
    nh = x.size
    a = np.argsort(-np.abs(x))
    kink = kind == "max" and abs(x[a[0]]) - abs(x[a[1]]) < 1e-5
    sa, sb = np.sign(x[a[0]]), np.sign(x[a[1]])

    def grad(z):
        if kind == "max":
            return np.sign(z[a[0]]) * np.eye(nh)[a[0]]
        return weights(nh) * np.sign(z)

    def F(z):
        J = jacobian(z, order, Y)
        U, s, Vt = np.linalg.svd(J, full_matrices=True)
        r = U[:, :ncond].T @ residual(z, order, Y)
        if kink:
            return np.concatenate([r, [sa * z[a[0]] - sb * z[a[1]]]])
        T = Vt[ncond:]
        return np.concatenate([r, T.T @ (T @ grad(z))])

    z = x.copy()
    for _ in range(30):
        f0 = F(z)
        if np.max(np.abs(f0)) < 1e-15:
            break
        h = 1e-7
        Jf = np.stack([(F(z + h * e) - F(z - h * e)) / (2 * h) for e in np.eye(nh)], axis=1)
        z = z - np.linalg.lstsq(Jf, f0, rcond=None)[0]
    z2, err = project(z, order, Y, rank=ncond)
    if err > 1e-14 or np.any(np.sign(z2) != np.sign(x)):
        return x
    return z2


def derive(order: int, M: int, kind: str, starts: int, seed: int, workers: int = 1, log=None) -> dict:
    nh = (M + 1) // 2
    Y = generators(order - 1)
    # the number of independent conditions: the rank of the Jacobian at a random point
    s = np.linalg.svd(jacobian(np.random.default_rng(1).uniform(-0.5, 0.5, nh), order, Y), compute_uv=False)
    ncond = int(np.sum(s > 1e-8 * s[0]))
    best = None
    for x in feasible_points(order, nh, starts, seed, ncond, workers=workers, log=log):
        x = polish(descend(x, order, Y, kind, ncond), order, Y, kind, ncond)
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
             "// the fewest substeps for the order with the smallest largest |g_n| (orders 4, 6, 8) or",
             "// the smallest sum of |g_n| (order 10), derived from the order conditions by",
             "// paper_1902_04661_amd/compositions.py, which writes this file.  Each list is g_1 .. g_M,",
             "// g_1 applied first.",
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
