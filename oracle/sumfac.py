"""Tiny sum-factorised brute force - oracle (test infrastructure only).

Pure-Python loops written from the sum-factorised forms of the paper
(section 2.2): backward transform of the hexahedron (eq. (16)) and of the
tetrahedron (eq. (17)); inner product of the hexahedron (eq. (20)) and of
the tetrahedron (eq. (21)); standard derivative (eq. (22)).  Prisms and
pyramids take the same nested sums with their own third-direction factor
(psi^b_{p,r} and psi^b_{max(p,q),r}).  Readings:
the weights in eqs. (20)/(21) are indexed by the quadrature point (w_1i,
w_2j, w_3k), |J| stays inside the innermost sum, and the collapsed shapes
carry the vertex corrections of the modified basis.  Only for P <= 3 and one
or two elements: it exists to cross-check the dense matrices of
``operators``, not for speed.
"""
import numpy as np

from .basis import HEX, PRISM, TET, PYR, psi_a, psi_b, modes, element_rule


def _tables(shape, P, Q):
    r = element_rule(shape, Q)
    return r


def bwd_trans(shape, P, Q, uhat):
    """u[i][j][k] for one element from its coefficients."""
    r = element_rule(shape, Q)
    z1, z2, z3 = r["z1"], r["z2"], r["z3"]
    idx = {m: n for n, m in enumerate(modes(shape, P))}
    u = np.zeros((Q, Q, Q))
    for i in range(Q):
        for j in range(Q):
            for k in range(Q):
                s1 = 0.0
                for p in range(P):
                    s2 = 0.0
                    qmax = P - p if shape == TET else P
                    for q in range(qmax):
                        s3 = 0.0
                        rmax = {HEX: P, PRISM: P - p, PYR: P - max(p, q)}.get(shape, P - p - q)
                        for rr in range(rmax):
                            if shape == HEX:
                                c = psi_a(rr, z3[k])
                            elif shape == PRISM:
                                c = psi_b(p, rr, z3[k])
                            elif shape == PYR:
                                c = psi_b(max(p, q), rr, z3[k])
                            else:
                                c = psi_b(p + q, rr, z3[k])
                            s3 += uhat[idx[(p, q, rr)]] * c
                        b = psi_b(p, q, z2[j]) if shape == TET else psi_a(q, z2[j])
                        s2 += b * s3
                    s1 += psi_a(p, z1[i]) * s2
                # collapsed-vertex corrections
                if shape == TET:
                    for rr in range(P - 1):
                        s1 += (psi_a(1, z1[i]) * psi_b(0, 1, z2[j]) * psi_b(1, rr, z3[k])
                               * uhat[idx[(0, 1, rr)]])
                    if P > 1:
                        s1 += ((1.0 - psi_a(0, z1[i]) * psi_b(0, 0, z2[j])) * 0.5 * (1.0 + z3[k])
                               * uhat[idx[(0, 0, 1)]])
                if shape == PRISM and P > 1:
                    for q in range(P):
                        s1 += (psi_a(1, z1[i]) * psi_a(q, z2[j]) * psi_b(0, 1, z3[k])
                               * uhat[idx[(0, q, 1)]])
                if shape == PYR and P > 1:
                    s1 += ((1.0 - psi_a(0, z1[i]) * psi_a(0, z2[j])) * 0.5 * (1.0 + z3[k])
                           * uhat[idx[(0, 0, 1)]])
                u[i, j, k] = s1
    return u.ravel()


def iprod_wrt_base(shape, P, Q, f, detJ):
    """u^_m = sum_i w1_i psi(i) sum_j w2_j psi(j) sum_k |J| f w3_k psi(k), one element."""
    r = element_rule(shape, Q)
    z1, z2, z3, w1, w2, w3 = r["z1"], r["z2"], r["z3"], r["w1"], r["w2"], r["w3"]
    f = np.asarray(f).reshape(Q, Q, Q)
    J = np.asarray(detJ).reshape(Q, Q, Q)
    ml = modes(shape, P)
    out = np.zeros(len(ml))
    for m, (p, q, rr) in enumerate(ml):
        tot = 0.0
        for i in range(Q):
            si = 0.0
            for j in range(Q):
                sj = 0.0
                for k in range(Q):
                    if shape == HEX:
                        c = psi_a(rr, z3[k])
                    elif shape == PRISM:
                        c = psi_b(p, rr, z3[k])
                    elif shape == PYR:
                        c = psi_b(max(p, q), rr, z3[k])
                    else:
                        c = psi_b(p + q, rr, z3[k])
                    # correction terms of the collapsed shapes enter as extra test functions
                    if shape == TET and (p, q) == (0, 1):
                        extra = psi_a(1, z1[i]) * psi_b(0, 1, z2[j]) * psi_b(1, rr, z3[k])
                    elif shape == TET and (p, q, rr) == (0, 0, 1):
                        extra = (1.0 - psi_a(0, z1[i]) * psi_b(0, 0, z2[j])) * 0.5 * (1.0 + z3[k])
                    elif shape == PRISM and p == 0 and rr == 1:
                        extra = psi_a(1, z1[i]) * psi_a(q, z2[j]) * psi_b(0, 1, z3[k])
                    elif shape == PYR and (p, q, rr) == (0, 0, 1):
                        extra = (1.0 - psi_a(0, z1[i]) * psi_a(0, z2[j])) * 0.5 * (1.0 + z3[k])
                    else:
                        extra = 0.0
                    b = psi_b(p, q, z2[j]) if shape == TET else psi_a(q, z2[j])
                    main = psi_a(p, z1[i]) * b * c
                    sj += J[i, j, k] * f[i, j, k] * w3[k] * (main + extra)
                si += w2[j] * sj
            tot += w1[i] * si
        out[m] = tot
    return out


def std_deriv_xi1(Q, z, u):
    """du/dxi_1 at the tensor points by eq. (22): sum_r h_r'(xi_1i) sum_s h_s(xi_2j) sum_t h_t(xi_3k) u_rst.

    h are the Lagrange polynomials through the points z, evaluated by their product formula.
    """
    u = np.asarray(u).reshape(Q, Q, Q)

    def h(l, x):
        v = 1.0
        for m in range(Q):
            if m != l:
                v *= (x - z[m]) / (z[l] - z[m])
        return v

    def dh(l, x):
        tot = 0.0
        for a in range(Q):
            if a == l:
                continue
            v = 1.0 / (z[l] - z[a])
            for m in range(Q):
                if m != l and m != a:
                    v *= (x - z[m]) / (z[l] - z[m])
            tot += v
        return tot

    out = np.zeros((Q, Q, Q))
    for i in range(Q):
        for j in range(Q):
            for k in range(Q):
                s = 0.0
                for r in range(Q):
                    s2 = 0.0
                    for ss in range(Q):
                        s3 = 0.0
                        for t in range(Q):
                            s3 += h(t, z[k]) * u[r, ss, t]
                        s2 += h(ss, z[j]) * s3
                    s += dh(r, z[i]) * s2
                out[i, j, k] = s
    return out.ravel()
