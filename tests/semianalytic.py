"""Independent reference values for the oracle's singular quadrature (tests only).

* ``triangle_potential(S, r)``: int_S 1/|r - y| dy in closed form for a flat
  triangle S and any point r (sum over the edges of a logarithmic term and an
  arctangent solid-angle term; the classical analytic potential of a uniformly
  charged flat triangle used in boundary-element codes).
* ``pair_integral(T, S)``: int_T int_S 1/|x - y| dy dx with the inner integral
  in closed form and the outer integral by a tensor Gauss rule that is
  geometrically graded towards the edges and corners of the reference
  triangle, where the inner potential loses smoothness.
* ``self_integral_closed_form(T)``: int_T int_T 1/|x - y| for one triangle with
  sides a, b, c and area A:  (4 A^2 / 3) sum_cyc (1/a) ln(((a+b)^2 - c^2) /
  (b^2 - (c-a)^2)).

None of this shares code with the oracle or the HIP library.
"""
import math

import numpy as np


def self_integral_closed_form(T):
    T = np.asarray(T, dtype=np.float64)
    a = np.linalg.norm(T[1] - T[2])
    b = np.linalg.norm(T[2] - T[0])
    c = np.linalg.norm(T[0] - T[1])
    A = 0.5 * np.linalg.norm(np.cross(T[1] - T[0], T[2] - T[0]))

    def f(a, b, c):
        return math.log(((a + b) ** 2 - c ** 2) / (b ** 2 - (c - a) ** 2)) / a

    return 4.0 * A * A / 3.0 * (f(a, b, c) + f(b, c, a) + f(c, a, b))


def triangle_potential(S, r):
    """int_S 1/|r - y| dy for points r of shape (3,) or (N, 3)."""
    S = np.asarray(S, dtype=np.float64)
    r = np.asarray(r, dtype=np.float64)
    one = r.ndim == 1
    r = np.atleast_2d(r)
    n = np.cross(S[1] - S[0], S[2] - S[0])
    n /= np.linalg.norm(n)
    h = (r - S[0]) @ n
    rho = r - h[:, None] * n[None, :]
    ah = np.abs(h)
    tot = np.zeros(r.shape[0])
    for i in range(3):
        a, b = S[i], S[(i + 1) % 3]
        l = (b - a) / np.linalg.norm(b - a)
        u = np.cross(l, n)              # outward in-plane edge normal
        t = (b - rho) @ u
        lp = (b - rho) @ l
        lm = (a - rho) @ l
        Rp = np.linalg.norm(r - b, axis=1)
        Rm = np.linalg.norm(r - a, axis=1)
        R02 = t * t + h * h
        with np.errstate(divide="ignore", invalid="ignore"):
            # R + l without cancellation: R^2 = l^2 + t^2 + h^2
            sp = np.where(lp >= 0, Rp + lp, R02 / (Rp - lp))
            sm = np.where(lm >= 0, Rm + lm, R02 / (Rm - lm))
            logt = np.where((R02 > 0) & (t != 0), t * np.log(sp / sm), 0.0)
        tot += logt
        tot -= ah * (np.arctan2(t * lp, R02 + ah * Rp) - np.arctan2(t * lm, R02 + ah * Rm))
    return tot[0] if one else tot


def _gl01(q):
    x, w = np.polynomial.legendre.leggauss(q)
    return 0.5 * (x + 1.0), 0.5 * w


def _graded(levels=14, sigma=0.15, q=12):
    x, w = _gl01(q)
    X, W = [], []
    cuts = [(sigma ** (k + 1), sigma ** k) for k in range(levels)] + [(0.0, sigma ** levels)]
    for lo, hi in cuts:
        X.append(lo + (hi - lo) * x)
        W.append((hi - lo) * w)
    return np.concatenate(X), np.concatenate(W)


def _graded_both(**kw):
    x, w = _graded(**kw)
    return np.concatenate([0.5 * x, 1.0 - 0.5 * x]), np.concatenate([0.5 * w, 0.5 * w])


def pair_integral(T, S, corner=None):
    """int_T int_S 1/|x-y|; T = (P0, P1, P2) parametrised as P0 + s1 (P1-P0) +
    s2 (P2-P1), 0 <= s2 <= s1 <= 1, collapsed s2 = s1 v; graded towards s1 in
    {0, 1} and v in {0, 1} (the vertices and edges of T).  corner = k weights
    the outer integral with the barycentric coordinate of T's corner k,
    (1 - s1, s1 - s2, s2)[k]."""
    T = np.asarray(T, dtype=np.float64)
    u, wu = _graded_both()
    v, wv = _graded_both()
    J = np.linalg.norm(np.cross(T[1] - T[0], T[2] - T[1]))
    U, Vv = np.meshgrid(u, v, indexing="ij")
    W = np.outer(wu, wv) * U
    if corner is not None:
        W = W * (1.0 - U, U - U * Vv, U * Vv)[corner]
    p = (T[0][None, None, :] + U[..., None] * (T[1] - T[0])[None, None, :]
         + (U * Vv)[..., None] * (T[2] - T[1])[None, None, :])
    pot = triangle_potential(S, p.reshape(-1, 3)).reshape(U.shape)
    return float(np.sum(W * pot) * J)
