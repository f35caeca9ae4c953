"""Pins of the oracle's characteristic system (Sec. 2.2: Roe-averaged
Jacobian A = dF~/dQ~ at the face, left/right eigenvectors, eigenvalues)."""
import numpy as np
import pytest

import oracle as O

GAMMA = 1.4


def phys_flux_dot(q, s, gamma=GAMMA):
    """Contracted inviscid flux F s_x + G s_y (+ H s_z), written from the
    flux vectors of the Euler equations."""
    ndim = len(s)
    rho = q[0]
    u = q[1:1 + ndim] / rho
    E = q[-1]
    p = (gamma - 1.0) * (E - 0.5 * rho * u @ u)
    U = u @ s
    return np.concatenate([[rho * U], rho * u * U + p * np.asarray(s), [(E + p) * U]])


def random_state(rng, ndim):
    rho = rng.uniform(0.5, 2.0)
    u = rng.uniform(-1.0, 1.0, ndim)
    p = rng.uniform(0.5, 2.0)
    E = p / (GAMMA - 1.0) + 0.5 * rho * u @ u
    return np.concatenate([[rho], rho * u, [E]])


@pytest.mark.parametrize("ndim", [2, 3])
def test_left_is_inverse_of_right(ndim):
    rng = np.random.default_rng(ndim)
    for _ in range(100):
        qL, qR = random_state(rng, ndim), random_state(rng, ndim)
        sf = rng.standard_normal(ndim)
        L, R, lam = O.eigensystem(ndim, GAMMA, qL, qR, sf, rng.uniform(0.5, 2))
        assert np.abs(L @ R - np.eye(ndim + 2)).max() < 1e-13


@pytest.mark.parametrize("ndim", [2, 3])
def test_roe_property(ndim):
    # R diag(lam) L (Q~_R - Q~_L) = F~(Q_R) - F~(Q_L) at fixed face metrics,
    # with Q~ = Q (1/J)_f: the eigen-decomposition is that of the Roe matrix
    # of the contracted flux, scaled by 1/(1/J)_f
    rng = np.random.default_rng(10 + ndim)
    for _ in range(100):
        qL, qR = random_state(rng, ndim), random_state(rng, ndim)
        sf = rng.standard_normal(ndim)
        Vf = rng.uniform(0.3, 3.0)
        L, R, lam = O.eigensystem(ndim, GAMMA, qL, qR, sf, Vf)
        lhs = R @ np.diag(lam) @ L @ ((qR - qL) * Vf)
        rhs = phys_flux_dot(qR, sf) - phys_flux_dot(qL, sf)
        assert np.allclose(lhs, rhs, rtol=1e-12, atol=1e-12 * np.abs(rhs).max())


@pytest.mark.parametrize("ndim", [2, 3])
def test_equal_states_give_flux_jacobian(ndim):
    # Q_L = Q_R: R diag(lam) L is the exact Jacobian dF~/dQ~ (finite differences)
    rng = np.random.default_rng(20 + ndim)
    q = random_state(rng, ndim)
    sf = rng.standard_normal(ndim)
    Vf = 0.7
    L, R, lam = O.eigensystem(ndim, GAMMA, q, q, sf, Vf)
    A = R @ np.diag(lam) @ L
    nv = ndim + 2
    Jfd = np.zeros((nv, nv))
    for c in range(nv):
        dq = np.zeros(nv)
        dq[c] = 1e-6
        Jfd[:, c] = (phys_flux_dot(q + dq, sf) - phys_flux_dot(q - dq, sf)) / 2e-6 / Vf
    assert np.allclose(A, Jfd, rtol=1e-7, atol=1e-7)
    # eigenvalues sigma*(u_n -+ c), sigma*u_n with sigma = |s_f|/Vf
    rho = q[0]
    u = q[1:1 + ndim] / rho
    p = (GAMMA - 1) * (q[-1] - 0.5 * rho * u @ u)
    c = np.sqrt(GAMMA * p / rho)
    nrm = np.linalg.norm(sf)
    un = u @ sf / nrm
    sig = nrm / Vf
    expect = [sig * (un - c)] + [sig * un] * ndim + [sig * (un + c)]
    assert np.allclose(lam, expect, rtol=1e-13)
