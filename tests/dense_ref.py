"""Independent dense-matrix and closed-form references used to pin the oracle.

Nothing here shares code with the oracle: the Hamiltonians are assembled from
Kronecker products of Pauli matrices and exponentiated with
``scipy.linalg.expm`` (n <= 8), and the p = 1 expectation is the closed form
for quadratic (Ising) costs.
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import expm

I2 = np.eye(2)
X = np.array([[0.0, 1.0], [1.0, 0.0]])
Z = np.array([[1.0, 0.0], [0.0, -1.0]])


def op_on(n: int, q: int, A: np.ndarray) -> np.ndarray:
    """A acting on qubit q of n; qubit 0 is the least-significant bit of the
    basis index, i.e. the right-most Kronecker factor."""
    out = np.ones((1, 1))
    for k in range(n - 1, -1, -1):
        out = np.kron(out, A if k == q else I2)
    return out


def cost_hamiltonian(Q: np.ndarray) -> np.ndarray:
    """H_C = sum_ij Q_ij N_i N_j with N_i = (I - Z_i)/2 the projector on
    z_i = 1 (Eq. (1) written as an operator)."""
    n = Q.shape[0]
    d = 1 << n
    N = [(np.eye(d) - op_on(n, i, Z)) / 2 for i in range(n)]
    H = np.zeros((d, d))
    for i in range(n):
        for j in range(n):
            H += Q[i, j] * (N[i] @ N[j])
    return H


def mixer_hamiltonian(n: int) -> np.ndarray:
    """H_X = -sum_i X_i (Sec. IV)."""
    d = 1 << n
    H = np.zeros((d, d))
    for i in range(n):
        H -= op_on(n, i, X)
    return H


def dense_state(Q, gammas, betas) -> np.ndarray:
    """Eq. (2) with dense exponentials: layer j = 1 acts first on |+>."""
    n = Q.shape[0]
    HC = cost_hamiltonian(Q)
    HX = mixer_hamiltonian(n)
    psi = np.full(1 << n, 2.0 ** (-n / 2), dtype=complex)
    for g, b in zip(gammas, betas):
        psi = expm(-1j * g * HC) @ psi
        psi = expm(-1j * b * HX) @ psi
    return psi


def dense_expect(Q, gammas, betas) -> float:
    psi = dense_state(Q, gammas, betas)
    return float(np.real(np.vdot(psi, cost_hamiltonian(Q) @ psi)))


def p1_closed_form(Q: np.ndarray, gamma: float, beta: float) -> float:
    """<C> of the p = 1 ansatz for any quadratic cost, in O(n^3).

    With s_i = 1 - 2 z_i, C = c0 + sum_i h_i s_i + sum_{i<j} J_ij s_i s_j where
    W_ij = Q_ij + Q_ji, J = W/4, h_i = -Q_ii/2 - sum_{j != i} W_ij/4 and
    c0 = sum_i Q_ii/2 + sum_{i<j} W_ij/4.  For the mixer e^{+i beta sum X}
    (H_X = -sum X) put c = cos 2beta, s = -sin 2beta; then
      <Z_u>     = s sin(2 g h_u) prod_{k != u} cos(2 g J_uk)
      <Z_u Z_v> = c s sin(2 g J_uv) [cos(2 g h_u) prod_{k != u,v} cos(2 g J_uk)
                                     + cos(2 g h_v) prod_{k != u,v} cos(2 g J_vk)]
                + s^2/2 [cos(2g(h_u - h_v)) prod cos(2g(J_uk - J_vk))
                         - cos(2g(h_u + h_v)) prod cos(2g(J_uk + J_vk))].
    """
    Q = np.asarray(Q, dtype=float)
    n = Q.shape[0]
    W = Q + Q.T
    np.fill_diagonal(W, 0.0)
    J = W / 4.0
    h = -np.diag(Q) / 2.0 - W.sum(axis=1) / 4.0
    c0 = np.trace(Q) / 2.0 + np.triu(W, 1).sum() / 4.0
    c = np.cos(2 * beta)
    s = -np.sin(2 * beta)
    g = gamma
    total = c0
    for u in range(n):
        pu = np.prod([np.cos(2 * g * J[u, k]) for k in range(n) if k != u])
        total += h[u] * s * np.sin(2 * g * h[u]) * pu
    for u in range(n):
        for v in range(u + 1, n):
            others = [k for k in range(n) if k not in (u, v)]
            pu = np.prod([np.cos(2 * g * J[u, k]) for k in others])
            pv = np.prod([np.cos(2 * g * J[v, k]) for k in others])
            pm = np.prod([np.cos(2 * g * (J[u, k] - J[v, k])) for k in others])
            pp = np.prod([np.cos(2 * g * (J[u, k] + J[v, k])) for k in others])
            zz = c * s * np.sin(2 * g * J[u, v]) * (np.cos(2 * g * h[u]) * pu +
                                                  np.cos(2 * g * h[v]) * pv)
            zz += s * s / 2.0 * (np.cos(2 * g * (h[u] - h[v])) * pm -
                                 np.cos(2 * g * (h[u] + h[v])) * pp)
            total += J[u, v] * zz
    return float(total)


def diagonal_expect(qdiag, gammas, betas) -> float:
    """<C> for a diagonal Q: the qubits decouple, each evolving by 2x2
    matrices diag(1, e^{-i g q}) then [[cos b, i sin b], [i sin b, cos b]]."""
    total = 0.0
    for q in qdiag:
        v = np.array([1.0, 1.0], dtype=complex) / np.sqrt(2.0)
        for g, b in zip(gammas, betas):
            v = np.array([v[0], np.exp(-1j * g * q) * v[1]])
            M = np.array([[np.cos(b), 1j * np.sin(b)], [1j * np.sin(b), np.cos(b)]])
            v = M @ v
        total += q * abs(v[1]) ** 2
    return float(total)


def mean_cost(Q) -> float:
    """Mean of z^T Q z over all 2^n z: (1^T Q 1 + tr Q) / 4."""
    Q = np.asarray(Q, dtype=float)
    return float((Q.sum() + np.trace(Q)) / 4.0)
