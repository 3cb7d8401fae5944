"""Independent brute-force solutions used to pin the oracle.

Nothing here comes from the paper's closed forms.  The two-stream system is
written as a pair of linear ODEs in optical depth t (measured downward from the
sublayer's top):

    dF_up/dt =  g_a F_up - g_s F_dn - S(t)
    dF_dn/dt = -g_a F_dn + g_s F_up + S(t)

with g_a - g_s = D (1 - w0) and g_a + g_s = D (1 - w0 g0), so that the
eigenvalue is D sqrt((1 - w0)(1 - w0 g0)) -- the exponent of eq:trans -- and
the thermal source S = 2 pi (1 - w0) B(t), which makes F_up = F_dn = 2 pi eps B
the isothermal equilibrium.  B is linear in t.  The system is solved exactly
with the matrix exponential of the augmented generator over M segments, with
the two boundary values imposed at opposite ends (a banded two-point problem
that stays well conditioned for any thickness).
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import expm


def sublayer(dtau, w0, g0, D, B_u, B_d, F_up_d, F_dn_u, M: int = 64):
    """Outgoing (upward flux at the top, downward flux at the bottom)."""
    ga = D * (1.0 - w0 * (1.0 + g0) / 2.0)
    gs = D * w0 * (1.0 - g0) / 2.0
    c = 2.0 * np.pi * (1.0 - w0)
    s0 = c * B_u
    s1 = c * (B_d - B_u) / dtau
    A = np.array([[ga, -gs, -s0, -s1], [gs, -ga, s0, s1], [0, 0, 0, 0], [0, 0, 1, 0]], float)
    h = dtau / M
    E = expm(A * h)
    N = 2 * (M + 1)
    mat = np.zeros((N, N))
    rhs = np.zeros(N)
    r = 0
    for k in range(M):
        tk = k * h
        for comp in (0, 1):
            mat[r, 2 * (k + 1) + comp] = 1.0
            mat[r, 2 * k] -= E[comp, 0]
            mat[r, 2 * k + 1] -= E[comp, 1]
            rhs[r] = E[comp, 2] + E[comp, 3] * tk
            r += 1
    mat[r, 1] = 1.0
    rhs[r] = F_dn_u
    r += 1
    mat[r, 2 * M] = 1.0
    rhs[r] = F_up_d
    x = np.linalg.solve(mat, rhs)
    return x[0], x[2 * M + 1]


def exact_pure_absorption(dtau, B_top, B_bottom, F_up_bottom, F_dn_top, nmu: int = 400):
    """Exact pure-absorption fluxes through a layer with B linear in optical
    depth, by Gauss-Legendre quadrature over the direction cosine of the
    formal solution of the transfer equation (isotropic incident radiation)."""
    y, w = np.polynomial.legendre.leggauss(nmu)
    mu = 0.5 * (y + 1.0)
    wm = 0.5 * w
    Bp = (B_bottom - B_top) / dtau  # dB/dt, t downward from the top
    # Upward intensity at the top: I(bottom) e^{-dtau/mu} + int_0^dtau B(t) e^{-t/mu} dt/mu
    e = np.exp(-dtau / mu)
    I_in_up = F_up_bottom / np.pi
    src_up = B_top * (1 - e) + Bp * (mu - (dtau + mu) * e)
    up = 2 * np.pi * np.sum(wm * mu * (I_in_up * e + src_up))
    # Downward at the bottom: s = dtau - t measured upward from the bottom
    I_in_dn = F_dn_top / np.pi
    src_dn = B_bottom * (1 - e) - Bp * (mu - (dtau + mu) * e)
    dn = 2 * np.pi * np.sum(wm * mu * (I_in_dn * e + src_dn))
    return up, dn


def column_isothermal_layers(dtau, w0, g0, D, B, F_top, F_int, M: int = 16):
    """Both fluxes at the n + 1 interfaces of a column of homogeneous,
    isothermal layers (index 0 at the bottom), from the two-stream ODE above
    with a constant source in each layer, solved as one two-point problem over
    the whole column: F_dn = F_top at the top and F_up = F_dn + F_int at the
    bottom.  Each layer is cut into M segments; on each, the state (F_up, F_dn,
    1) advances by the matrix exponential of the augmented generator.
    Returns (F_up, F_dn) bottom to top."""
    n = len(dtau)
    nodes = n * M + 1  # node 0 at the top, node n*M at the bottom
    N = 2 * nodes
    mat = np.zeros((N, N))
    rhs = np.zeros(N)
    r = 0
    for q in range(n):  # q-th layer from the top
        i = n - 1 - q
        ga = D * (1.0 - w0[i] * (1.0 + g0[i]) / 2.0)
        gs = D * w0[i] * (1.0 - g0[i]) / 2.0
        s0 = 2.0 * np.pi * (1.0 - w0[i]) * B[i]
        A = np.array([[ga, -gs, -s0], [gs, -ga, s0], [0.0, 0.0, 0.0]])
        E = expm(A * (dtau[i] / M))
        for k in range(q * M, (q + 1) * M):
            for comp in (0, 1):
                mat[r, 2 * (k + 1) + comp] = 1.0
                mat[r, 2 * k] -= E[comp, 0]
                mat[r, 2 * k + 1] -= E[comp, 1]
                rhs[r] = E[comp, 2]
                r += 1
    mat[r, 1] = 1.0  # F_dn at the top
    rhs[r] = F_top
    r += 1
    b = nodes - 1
    mat[r, 2 * b] = 1.0  # F_up - F_dn at the bottom
    mat[r, 2 * b + 1] = -1.0
    rhs[r] = F_int
    x = np.linalg.solve(mat, rhs).reshape(nodes, 2)
    at_if = x[::M][::-1]  # interfaces bottom to top
    return at_if[:, 0].copy(), at_if[:, 1].copy()
