"""Rosenbrock tableaus, derived here from the order conditions rather than
taken from any code: an order-3 method (``tableau()``, kept as a reference
and for tests) and the order-4 method the device integrator uses
(``ros4()``).

The paper's solver is an unnamed "standard" stiff ODE integrator (Sec. 2.5)
fed by a sparse analytical Jacobian; this library uses a linearly implicit
(Rosenbrock) method, which needs exactly that Jacobian and one LU per step.

Method form (Hairer & Wanner, Solving ODEs II, Sec. IV.7):
    (I - h gamma J) k_i = h f(y + sum_{j<i} alpha_ij k_j) + h J sum_{j<i} gamma_ij k_j
    y1 = y + sum_i b_i k_i,   yhat1 = y + sum_i bhat_i k_i
with beta_ij = alpha_ij + gamma_ij, beta_ii = gamma, beta'_i = sum_{j<i} beta_ij,
alpha_i = sum_j alpha_ij.  Order conditions up to 3:
    sum b_i = 1;  sum b_i beta'_i = 1/2 - gamma;
    sum b_i alpha_i^2 = 1/3;  sum b_i beta_ij beta'_j = 1/6 - gamma + gamma^2.

Choices (4 stages): gamma = 1/2; alpha_21 = 0 (stage 2 reuses f(y));
alpha_31 = 1, alpha_32 = 0; the main method is stiffly accurate (b = last row
of beta, so R(inf) = 0) and the embedded order-2 method is stiffly accurate
on stage 3 (bhat = row 3 of beta); stage 4 is evaluated at the embedded
solution (alpha_4j = beta_3j).  With beta_21 = 1 the conditions leave one
solution:
    b    = (5/6, -1/6, -1/6, 1/2),   bhat = (3/4, -1/4, 1/2, 0).
``derive()`` solves the conditions symbolically and ``check()`` verifies
them, A-stability on the imaginary axis and R(inf) = 0.

The implementation uses the transformed variables u_i = sum_{j<=i} gamma_ij k_j
(no Jacobian-vector products):
    (I/(h gamma) - J) u_i = f(y + sum_{j<i} a_ij u_j) + sum_{j<i} (c_ij/h) u_j
    y1 = y + sum m_i u_i,  error = sum (m_i - mhat_i) u_i
with a = alpha Gamma^-1, c = diag(1/gamma) - Gamma^-1, m = b Gamma^-1.
"""
from __future__ import annotations

from fractions import Fraction as Fr

import numpy as np

GAMMA = Fr(1, 2)


def derive():
    """Solve the order conditions for the free parameters (SymPy)."""
    import sympy as sp
    g = sp.Rational(1, 2)
    b21, b31, b32, b41, b42, b43 = sp.symbols("b21 b31 b32 b41 b42 b43")
    beta = sp.Matrix([[g, 0, 0, 0], [b21, g, 0, 0], [b31, b32, g, 0], [b41, b42, b43, g]])
    alpha = sp.Matrix([[0, 0, 0, 0], [0, 0, 0, 0], [1, 0, 0, 0], [b31, b32, g, 0]])
    b = [beta[3, j] for j in range(4)]
    bh = [beta[2, 0], beta[2, 1], g, 0]
    bp = [sum(beta[i, j] for j in range(i)) for i in range(4)]
    al = [sum(alpha[i, j] for j in range(4)) for i in range(4)]
    eqs = [
        sum(b) - 1,
        sum(b[i] * bp[i] for i in range(4)) - (sp.Rational(1, 2) - g),
        sum(b[i] * al[i] ** 2 for i in range(4)) - sp.Rational(1, 3),
        sum(b[i] * beta[i, j] * bp[j] for i in range(4) for j in range(i)) - (sp.Rational(1, 6) - g + g**2),
        sum(bh) - 1,
        sum(bh[i] * bp[i] for i in range(4)) - (sp.Rational(1, 2) - g),
    ]
    sol = sp.solve([e.subs(b21, 1) for e in eqs], [b31, b32, b41, b42, b43], dict=True)
    return sol


def tableau():
    """Exact (Fraction) tableau in both forms."""
    g = GAMMA
    beta21 = Fr(1)
    beta32 = Fr(-1, 4) / beta21
    beta31 = Fr(1, 2) - beta32
    beta42 = Fr(-1, 6) / beta21
    beta41 = Fr(2, 3) - beta42
    beta43 = Fr(-1, 6)
    beta = [[g, 0, 0, 0], [beta21, g, 0, 0], [beta31, beta32, g, 0], [beta41, beta42, beta43, g]]
    alpha = [[0, 0, 0, 0], [0, 0, 0, 0], [Fr(1), 0, 0, 0], [beta31, beta32, g, 0]]
    s = 4
    Gam = [[Fr(beta[i][j]) - (Fr(alpha[i][j]) if j < i else 0) for j in range(s)] for i in range(s)]
    for i in range(s):
        Gam[i][i] = g
    b = [Fr(beta[3][j]) for j in range(s)]
    bh = [Fr(beta[2][0]), Fr(beta[2][1]), g, Fr(0)]
    Gi = _inv_lower(Gam)
    a = [[sum(Fr(alpha[i][k]) * Gi[k][j] for k in range(s)) for j in range(s)] for i in range(s)]
    c = [[(1 / g if i == j else 0) - Gi[i][j] for j in range(s)] for i in range(s)]
    m = [sum(b[k] * Gi[k][j] for k in range(s)) for j in range(s)]
    mh = [sum(bh[k] * Gi[k][j] for k in range(s)) for j in range(s)]
    return dict(gamma=g, alpha=alpha, Gamma=Gam, beta=beta, b=b, bhat=bh, a=a, c=c, m=m, mhat=mh,
                stages=s, order=3, embedded_order=2)


def _inv_lower(L):
    n = len(L)
    X = [[Fr(0)] * n for _ in range(n)]
    for j in range(n):
        for i in range(n):
            acc = Fr(1 if i == j else 0)
            for k in range(i):
                acc -= L[i][k] * X[k][j]
            X[i][j] = acc / L[i][i]
    return X


# ---------------------------------------------------------------------------
# Order 4 (the device method): 4 stages, 3 function evaluations per step.
#
# Choices: gamma = the largest root in (0.2, 0.6) of the z^4 coefficient of
# trunc_4[(1 - gamma z)^4 e^z] (this makes R(inf) = 0: L-stability for a
# 4-stage order-4 method); alpha_4j = alpha_3j so stage 4 reuses the function
# value of stage 3; the embedded method uses stages 1-3 only (bhat_4 = 0) and
# has order 3.  With the order-4 conditions (order-3 set above plus
#   sum b_i alpha_i^3 = 1/4,  sum b_i alpha_i alpha_ij beta'_j = 1/8 - gamma/3,
#   sum b_i beta_ij alpha_j^2 = 1/12 - gamma/3,
#   sum b_i beta_ij beta_jk beta'_k = 1/24 - gamma/2 + 3 gamma^2/2 - gamma^3)
# the system reduces to closed forms (see ros4()): the quadrature conditions
# give b_2 and b_3 + b_4, the b-alpha-alpha-beta' condition gives alpha_32,
# the embedded order-3 conditions give beta_31, beta_32 from bhat_3, and the
# two remaining conditions fix beta_21 and leave b_4 free.  Free parameters:
# alpha_2 = 0.6, alpha_3 = 0.7, bhat_3 = 0.4, b_4 = 0.6 (chosen for small
# coefficients and an embedded method stable on the imaginary axis).
# ---------------------------------------------------------------------------
ROS4_FREE = dict(a2=0.6, a3=0.7, bh3=0.4, b4=0.6)


def ros4_gamma():
    from math import comb, factorial
    coef = [comb(4, j) * (-1) ** j / factorial(4 - j) for j in range(5)]  # powers of gamma
    roots = np.roots(coef[::-1])
    return max(r.real for r in roots if abs(r.imag) < 1e-12 and 0.2 < r.real < 0.6)


def ros4(a2=ROS4_FREE["a2"], a3=ROS4_FREE["a3"], bh3=ROS4_FREE["bh3"], b4=ROS4_FREE["b4"]):
    """Order-4 tableau (float64) in both forms."""
    G = ros4_gamma()
    K2, K3, K6 = 0.5 - G, 1 / 6 - G + G * G, 1 / 8 - G / 3
    K7, K8 = 1 / 12 - G / 3, 1 / 24 - G / 2 + 1.5 * G * G - G**3
    b2, s = np.linalg.solve([[a2**2, a3**2], [a2**3, a3**3]], [1 / 3, 1 / 4])
    b1, b3 = 1 - b2 - s, s - b4
    be21 = a2**2 * (K3 - K8 * K2 / K3) / (K7 - K8 / (3 * K3))
    a32 = K6 / (a3 * be21 * s)
    a31 = a3 - a32
    bh2 = (1 / 3 - bh3 * a3**2) / a2**2
    bh1 = 1 - bh2 - bh3
    be32 = K3 / (bh3 * be21)
    B3 = (K2 - bh2 * be21) / bh3
    be31 = B3 - be32
    be43 = K8 / (b4 * be32 * be21)
    be42 = (K3 - b3 * be32 * be21 - b4 * be43 * B3) / (b4 * be21)
    B4 = (K2 - b2 * be21 - b3 * B3) / b4
    be41 = B4 - be42 - be43
    alpha = np.array([[0, 0, 0, 0], [a2, 0, 0, 0], [a31, a32, 0, 0], [a31, a32, 0, 0]], float)
    beta = np.array([[G, 0, 0, 0], [be21, G, 0, 0], [be31, be32, G, 0], [be41, be42, be43, G]], float)
    b = np.array([b1, b2, b3, b4])
    bh = np.array([bh1, bh2, bh3, 0.0])
    Gam = beta - alpha
    Gi = np.linalg.inv(Gam)
    clean = lambda M: np.where(np.abs(M) < 1e-13, 0.0, np.tril(M, -1))  # exact zeros stay zero
    a = clean(alpha @ Gi)
    c = clean(np.diag(1 / np.diag(Gam)) - Gi)
    return dict(gamma=G, alpha=alpha, beta=beta, b=b, bhat=bh, a=a, c=c, m=b @ Gi, mhat=bh @ Gi,
                stages=4, order=4, embedded_order=3, reuse=[0, -1, -1, 2])


def ros4_residuals(t=None):
    """Order-4 conditions for b and order-3 conditions for bhat (all ~0) and
    the order-4 conditions for bhat (not all 0)."""
    t = t or ros4()
    G, al, be = t["gamma"], t["alpha"], t["beta"]
    bp = np.array([be[i, :i].sum() for i in range(4)])
    ai = al.sum(1)

    def conds(b):
        return np.array([
            b.sum() - 1, b @ bp - (0.5 - G), b @ ai**2 - 1 / 3,
            sum(b[i] * be[i, j] * bp[j] for i in range(4) for j in range(i)) - (1 / 6 - G + G * G),
            b @ ai**3 - 0.25,
            sum(b[i] * ai[i] * al[i, j] * bp[j] for i in range(4) for j in range(i)) - (1 / 8 - G / 3),
            sum(b[i] * be[i, j] * ai[j] ** 2 for i in range(4) for j in range(i)) - (1 / 12 - G / 3),
            sum(b[i] * be[i, j] * be[j, k] * bp[k] for i in range(4) for j in range(i) for k in range(j))
            - (1 / 24 - G / 2 + 1.5 * G * G - G**3)])
    return conds(t["b"]), conds(t["bhat"])


def stability(z, t=None, embedded=False):
    """R(z) = 1 + z b^T (I - z B)^-1 1 with B = (beta_ij) (diagonal gamma)."""
    t = t or ros4()
    B = np.array([[float(x) for x in r] for r in t["beta"]])
    b = np.array([float(x) for x in (t["bhat"] if embedded else t["b"])])
    z = np.atleast_1d(np.asarray(z, dtype=complex))
    one = np.ones(4)
    out = np.empty(z.shape, complex)
    for i, zz in enumerate(z):
        out[i] = 1 + zz * b @ np.linalg.solve(np.eye(4) - zz * B, one)
    return out


def check():
    """Verify order conditions (exact), R(inf) = 0 and |R(iy)| <= 1."""
    t = tableau()
    g, B, A, b, bh = t["gamma"], t["beta"], t["alpha"], t["b"], t["bhat"]
    bp = [sum(Fr(B[i][j]) for j in range(i)) for i in range(4)]
    al = [sum(Fr(A[i][j]) for j in range(4)) for i in range(4)]
    conds = {
        "p1": (sum(b), Fr(1)),
        "p2": (sum(b[i] * bp[i] for i in range(4)), Fr(1, 2) - g),
        "p3a": (sum(b[i] * al[i] ** 2 for i in range(4)), Fr(1, 3)),
        "p3b": (sum(b[i] * Fr(B[i][j]) * bp[j] for i in range(4) for j in range(i)), Fr(1, 6) - g + g * g),
        "e1": (sum(bh), Fr(1)),
        "e2": (sum(bh[i] * bp[i] for i in range(4)), Fr(1, 2) - g),
    }
    for k, (got, want) in conds.items():
        assert got == want, (k, got, want)
    # the embedded method must NOT satisfy the order-3 conditions (else the
    # error estimate would be of higher order than claimed)
    assert sum(bh[i] * al[i] ** 2 for i in range(4)) != Fr(1, 3) or \
        sum(bh[i] * Fr(B[i][j]) * bp[j] for i in range(4) for j in range(i)) != Fr(1, 6) - g + g * g
    rinf = abs(stability(1e12)[0])
    ys = np.logspace(-3, 4, 400)
    rmax = np.abs(stability(1j * ys)).max()
    return dict(conds=conds, R_inf=rinf, max_R_imag_axis=rmax)


def c_constants(t=None):
    """Device initialisers of the transformed tableau (17 significant digits)."""
    t = t or ros4()
    f = lambda x: repr(float(x))
    rows = lambda M: "{" + ", ".join("{" + ", ".join(f(x) for x in r) + "}" for r in M) + "}"
    return "\n".join([
        f"GAM = {f(t['gamma'])}",
        f"TA = {rows(t['a'])}",
        f"TC = {rows(t['c'])}",
        "TM = {" + ", ".join(f(x) for x in t["m"]) + "}",
        "TE = {" + ", ".join(f(x - y) for x, y in zip(t["m"], t["mhat"])) + "}",
        "TREUSE = {" + ", ".join(str(x) for x in t["reuse"]) + "}",
    ])


if __name__ == "__main__":
    print(derive())
    print(check())
    print(ros4_residuals())
    print(c_constants())
