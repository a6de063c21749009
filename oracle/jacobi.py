"""Jacobi polynomials P_n^{(alpha,beta)} - oracle (test infrastructure only).

The modified bases of the paper (section 2.2, psi^a, psi^b, psi^c in eqs.
(16), (17)) are built from Jacobi polynomials; the paper defers their
definition to the spectral/hp textbook, so the classical definition is used:
the normalisation P_n^{(a,b)}(1) = C(n+a, n), the three-term recurrence, and
d/dx P_n^{(a,b)} = (n+a+b+1)/2 * P_{n-1}^{(a+1,b+1)}.
"""
import numpy as np


def jacobi(n, alpha, beta, x):
    """P_n^{(alpha,beta)}(x), classical normalisation, by the three-term recurrence."""
    x = np.asarray(x, dtype=np.float64)
    p_prev = np.ones_like(x)
    if n == 0:
        return p_prev
    a, b = float(alpha), float(beta)
    p = 0.5 * (a - b + (a + b + 2.0) * x)
    for k in range(2, n + 1):
        c = 2.0 * k + a + b
        lead = 2.0 * k * (k + a + b) * (c - 2.0)
        lin = (c - 1.0) * (a * a - b * b)
        quad = (c - 2.0) * (c - 1.0) * c
        back = 2.0 * (k + a - 1.0) * (k + b - 1.0) * c
        p_prev, p = p, ((lin + quad * x) * p - back * p_prev) / lead
    return p


def jacobi_deriv(n, alpha, beta, x):
    """d/dx P_n^{(alpha,beta)}(x) = (n+alpha+beta+1)/2 P_{n-1}^{(alpha+1,beta+1)}(x)."""
    x = np.asarray(x, dtype=np.float64)
    if n == 0:
        return np.zeros_like(x)
    return 0.5 * (n + alpha + beta + 1.0) * jacobi(n - 1, alpha + 1, beta + 1, x)
