"""Independent references that pin the oracle (no Boys tables, no recurrences).

* boys_mp:      F_m(T) = gamma(m + 1/2, T) / (2 T^(m + 1/2)) at 30 digits (mpmath).
* ssss_closed:  the primitive (ss|ss) integral in closed form with erf.
* eri_by_derivs: any Cartesian primitive integral as centre derivatives of the
                closed-form (ss|ss), using x_A^{l+1} g = (d/dA_x [x_A^l g] + l x_A^{l-1} g)/(2a)
                for g = exp(-a x_A^2), differentiated numerically by mpmath at high precision.
* eri_quadrature: brute force.  1/r12 = (2/sqrt(pi)) int_0^inf exp(-u^2 r12^2) du; for a
                fixed u the six-dimensional integral factorises over x, y, z into
                two-dimensional polynomial x Gaussian integrals, each exact by
                tensor Gauss-Hermite quadrature after whitening the quadratic form;
                the u integral is done adaptively (scipy.integrate.quad).  The
                erf-attenuated operator erf(omega r12)/r12 is the same integral cut
                at u = omega (omega > 0 passed as `omega`).
"""
from __future__ import annotations

import math

import mpmath as mp
import numpy as np
from scipy import integrate


def boys_mp(m: int, T, dps: int = 30):
    with mp.workdps(dps):
        T = mp.mpf(T)
        if T == 0:
            return mp.mpf(1) / (2 * m + 1)
        return mp.gammainc(m + mp.mpf(1) / 2, 0, T) / (2 * T ** (m + mp.mpf(1) / 2))


def ssss_closed(a, A, b, B, c, C, d, D, lib=mp):
    """(ss|ss) for unit-coefficient primitives; lib = mpmath (default)."""
    A, B, C, D = (list(map(lib.mpf, X)) if lib is mp else list(X) for X in (A, B, C, D))
    p, q = a + b, c + d
    P = [(a * A[k] + b * B[k]) / p for k in range(3)]
    Q = [(c * C[k] + d * D[k]) / q for k in range(3)]
    AB2 = sum((A[k] - B[k]) ** 2 for k in range(3))
    CD2 = sum((C[k] - D[k]) ** 2 for k in range(3))
    PQ2 = sum((P[k] - Q[k]) ** 2 for k in range(3))
    rho = p * q / (p + q)
    T = rho * PQ2
    if T == 0:
        F0 = lib.mpf(1)
    else:
        F0 = lib.sqrt(lib.pi / T) / 2 * lib.erf(lib.sqrt(T))
    return (2 * lib.pi ** lib.mpf(2.5) / (p * q * lib.sqrt(p + q)) * lib.exp(-a * b / p * AB2)
            * lib.exp(-c * d / q * CD2) * F0)


def _deriv_poly(l: int, a):
    """Coefficients c_k with x_A^l g = sum_k c_k d^k/dA_x^k g, g = exp(-a x_A^2)."""
    polys = [{0: mp.mpf(1)}]
    if l >= 1:
        polys.append({1: 1 / (2 * a)})
    for n in range(1, l):
        nxt = {}
        for k, v in polys[n].items():
            nxt[k + 1] = nxt.get(k + 1, 0) + v / (2 * a)
        for k, v in polys[n - 1].items():
            nxt[k] = nxt.get(k, 0) + n * v / (2 * a)
        polys.append(nxt)
    return polys[l]


def eri_by_derivs(pa, a, A, pb, b, B, pc, c, C, pd, d, D, dps: int = 40):
    """Primitive Cartesian integral from derivatives of the (ss|ss) closed form."""
    with mp.workdps(dps):
        exps = [mp.mpf(a), mp.mpf(b), mp.mpf(c), mp.mpf(d)]
        cents = [list(map(mp.mpf, X)) for X in (A, B, C, D)]
        pows = [pa, pb, pc, pd]
        # expand the product of per-(centre, direction) derivative polynomials
        terms = [({}, mp.mpf(1))]
        for ci in range(4):
            for k in range(3):
                poly = _deriv_poly(int(pows[ci][k]), exps[ci])
                new = []
                for orders, coef in terms:
                    for order, cv in poly.items():
                        o = dict(orders)
                        if order:
                            o[3 * ci + k] = order
                        new.append((o, coef * cv))
                terms = new
        x0 = [cents[ci][k] for ci in range(4) for k in range(3)]

        def f(*x):
            X = [x[3 * i:3 * i + 3] for i in range(4)]
            return ssss_closed(exps[0], X[0], exps[1], X[1], exps[2], X[2], exps[3], X[3])

        total = mp.mpf(0)
        for orders, coef in terms:
            if not orders:
                total += coef * f(*x0)
                continue
            idx = sorted(orders)
            sub_x = [x0[i] for i in idx]

            def g(*y, idx=idx):
                x = list(x0)
                for i, v in zip(idx, y):
                    x[i] = v
                return f(*x)

            total += coef * mp.diff(g, sub_x, tuple(orders[i] for i in idx))
        return float(total)


def _gh_2d(n):
    x, w = np.polynomial.hermite.hermgauss(n)
    return x, w


def _dim_integral(u, ea, Ax, ia, eb, Bx, ib, ec, Cx, ic, ed, Dx, id_, gh):
    """int int x1_A^ia x1_B^ib x2_C^ic x2_D^id exp(-a x1A^2 - b x1B^2 - c x2C^2 - d x2D^2
    - u^2 (x1 - x2)^2) dx1 dx2, exact by 2-D Gauss-Hermite after whitening."""
    p, q = ea + eb, ec + ed
    P = (ea * Ax + eb * Bx) / p
    Q = (ec * Cx + ed * Dx) / q
    pre = math.exp(-ea * eb / p * (Ax - Bx) ** 2 - ec * ed / q * (Cx - Dx) ** 2)
    u2 = u * u
    M = np.array([[p + u2, -u2], [-u2, q + u2]])
    rhs = np.array([p * P, q * Q])
    y0 = np.linalg.solve(M, rhs)
    const = p * P * P + q * Q * Q - y0 @ M @ y0
    L = np.linalg.cholesky(M)        # M = L L^T
    Linv_T = np.linalg.inv(L.T)
    x, w = gh
    z1, z2 = np.meshgrid(x, x, indexing="ij")
    W = np.outer(w, w)
    Z = np.stack([z1.ravel(), z2.ravel()])
    Y = y0[:, None] + Linv_T @ Z
    x1, x2 = Y
    poly = (x1 - Ax) ** ia * (x1 - Bx) ** ib * (x2 - Cx) ** ic * (x2 - Dx) ** id_
    jac = 1.0 / (L[0, 0] * L[1, 1])
    return pre * math.exp(-const) * jac * float(W.ravel() @ poly)


def eri_quadrature(pa, a, A, pb, b, B, pc, c, C, pd, d, D, epsrel=1e-13, omega=None):
    npts = 1 + (sum(pa) + sum(pb) + sum(pc) + sum(pd)) // 2 + 4
    gh = _gh_2d(npts)

    def integrand(u):
        v = 1.0
        for k in range(3):
            v *= _dim_integral(u, a, A[k], pa[k], b, B[k], pb[k], c, C[k], pc[k], d, D[k],
                               pd[k], gh)
        return v

    # split the range: most weight sits at u of order sqrt(rho)
    val = 0.0
    edges = [0.0, 0.5, 2.0, 8.0, 32.0, np.inf]
    if omega is not None:
        edges = [e for e in edges if e < omega] + [float(omega)]
    for lo, hi in zip(edges[:-1], edges[1:]):
        r, _ = integrate.quad(integrand, lo, hi, epsabs=0.0, epsrel=epsrel, limit=400)
        val += r
    return 2.0 / math.sqrt(math.pi) * val
