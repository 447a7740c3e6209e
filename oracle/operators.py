"""The matrices of the primal problem and of the gamma=k HSS iteration.

All matrices use the convention A_ij = a(phi_j, phi_i) with a real nodal
basis, so every operator is a complex combination of K, M and MG (assembled
by `oracle.fem`).

  B_delta   the primal form b_delta of Sec. 2, eq. (primal):
            K + (-delta + i k)^2 M - (-delta + i k) MG.
  H         the Gram matrix of the H_primal inner product of Sec. 3.1:
            <v, u>_H = 2 delta k <v, u> + k <<v, u>>.
  A_S       the real symmetric matrix with H S = i A_S, read off the
            definition of S_primal in Sec. 3.1:
            K + (delta^2 - k^2) M + delta MG.
  L, N      the left- and right-hand operators of the gamma=k HSS iteration,
            Definition "gamma=k HSS iteration in primal form",
            eq. (primal-hss-system), with delta as given (the shifted-HSS
            preconditioner of Sec. 4 uses delta_hat in its place).
"""

import numpy as np


def b_delta(K, M, MG, k, delta):
    """Matrix of b_delta (Sec. 2): the Helmholtz operator with absorption
    delta.  B_0 is the operator the outer iteration solves."""
    s = -delta + 1j * k
    return K + (s * s) * M - s * MG


def h_gram(M, MG, k, delta):
    """Gram matrix of the H_primal inner product (Sec. 3.1)."""
    return (2.0 * delta * k) * M + k * MG


def a_skew(K, M, MG, k, delta):
    """A_S with H S_primal = i A_S (Sec. 3.1): the real symmetric matrix of
    i(delta^2 - k^2)<v,u> + i<grad v, grad u> + delta i <<v,u>> divided by i."""
    return K + (delta * delta - k * k) * M + delta * MG


def hss_lhs(K, M, MG, k, delta):
    """L: left-hand side of eq. (primal-hss-system)."""
    return K + (-2j * delta * k * k + delta * delta - k * k) * M + (-1j * k * k + delta) * MG


def hss_rhs(K, M, MG, k, delta):
    """N: the operator applied to u_n on the right of eq. (primal-hss-system),
    before the factor (k-1)/(k+1)."""
    return -K + (-2j * delta * k * k - delta * delta + k * k) * M + (-1j * k * k - delta) * MG


def coefficients(name, k, delta):
    """(a, b, c) with  operator = a K + b M + c MG  for a named operator.

    Used by the tests to describe operators compactly; the values are read
    off the functions above by applying them to K=1, M=0, MG=0 etc.
    """
    fn = {"B": lambda K, M, G: b_delta(K, M, G, k, delta),
          "H": lambda K, M, G: h_gram(M, G, k, delta),
          "AS": lambda K, M, G: a_skew(K, M, G, k, delta),
          "L": lambda K, M, G: hss_lhs(K, M, G, k, delta),
          "N": lambda K, M, G: hss_rhs(K, M, G, k, delta)}[name]
    a = complex(fn(1.0, 0.0, 0.0))
    b = complex(fn(0.0, 1.0, 0.0))
    c = complex(fn(0.0, 0.0, 1.0))
    return a, b, c


def combine(K, M, MG, abc):
    a, b, c = abc
    return (a * K + b * M + c * MG).tocsr()


def inner_iterations(k, m=1):
    """Number of inner HSS iterations of the shifted-HSS preconditioner,
    m * ceil(k) (Definition "Shifted HSS iteration for the primal system")."""
    return int(m * np.ceil(k))
