"""1-D quadrature rules - oracle (test infrastructure only).

The paper integrates with tensor products of 1-D rules: Gauss-Lobatto-
Legendre in the hexahedron's directions (the ``gll`` specifier of the block
type, section 3.1.1) and, in the collapsed directions of the tetrahedron,
rules that avoid the singular end point "such as Gauss-Radau" (section 2.2,
remark after eq. (13)).  Reading used here: Gauss-Radau-Jacobi rules that
include x = -1, with alpha = 1 (eta_2) and alpha = 2 (eta_3), so that the
collapse Jacobian factors (1-x)^alpha are absorbed by the weights.

Points: the interior points are zeros of a Jacobi polynomial, taken from
``scipy.special.roots_jacobi`` (a library root finder).  Weights: moment
matching in the orthogonal basis, sum_i w_i P_n(x_i) = delta_{n0} h_0, solved
with ``numpy.linalg.solve``.  Neither step is shared with the HIP library,
which uses Newton iteration and closed-form weights.
"""
import math

import numpy as np
from scipy.special import roots_jacobi

from .jacobi import jacobi


def _h0(alpha, beta):
    """Integral of (1-x)^alpha (1+x)^beta over [-1, 1]."""
    return (2.0 ** (alpha + beta + 1) * math.gamma(alpha + 1) * math.gamma(beta + 1)
            / math.gamma(alpha + beta + 2))


def _moment_weights(x, alpha, beta):
    q = len(x)
    vander = np.array([jacobi(n, alpha, beta, x) for n in range(q)])
    rhs = np.zeros(q)
    rhs[0] = _h0(alpha, beta)
    return np.linalg.solve(vander, rhs)


def gauss_lobatto_legendre(q):
    """Q-point GLL rule on [-1, 1]: end points plus the zeros of P^{(1,1)}_{Q-2}."""
    if q < 2:
        raise ValueError("GLL needs at least 2 points")
    inner = np.sort(roots_jacobi(q - 2, 1.0, 1.0)[0]) if q > 2 else np.zeros(0)
    x = np.concatenate(([-1.0], inner, [1.0]))
    return x, _moment_weights(x, 0, 0)


def gauss_radau_jacobi(q, alpha, beta=0):
    """Q-point Gauss-Radau-Jacobi rule including x = -1, for the weight (1-x)^alpha (1+x)^beta.

    x_0 = -1 and the remaining points are the zeros of P^{(alpha, beta+1)}_{Q-1}.
    """
    if q < 1:
        raise ValueError("need at least 1 point")
    inner = np.sort(roots_jacobi(q - 1, float(alpha), float(beta + 1))[0]) if q > 1 else np.zeros(0)
    x = np.concatenate(([-1.0], inner))
    return x, _moment_weights(x, alpha, beta)
