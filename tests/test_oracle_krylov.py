"""Pins of the small matrix exponential, phi_1 and Arnoldi (Section 2.2)
against scipy and dense linear algebra."""

import math

import numpy as np
import pytest
import scipy.linalg as sla

import oracle


@pytest.mark.parametrize("n,scale", [(5, 0.1), (8, 1.0), (12, 10.0), (31, 60.0), (31, 400.0)])
def test_expm_matches_scipy(n, scale):
    rng = np.random.default_rng(n)
    A = scale * rng.standard_normal((n, n)) / np.sqrt(n)
    E = oracle.expm(A)
    Er = sla.expm(A)
    assert np.max(np.abs(E - Er)) <= 1e-12 * max(1.0, np.max(np.abs(Er)))


def test_expm_closed_forms():
    # rotation generator and nilpotent Jordan block
    t = 2.3
    A = np.array([[0.0, -t], [t, 0.0]])
    assert np.allclose(oracle.expm(A), [[np.cos(t), -np.sin(t)], [np.sin(t), np.cos(t)]], atol=1e-15)
    N = np.diag(np.ones(3), 1)
    E = oracle.expm(N)
    ref = np.eye(4) + N + N @ N / 2 + N @ N @ N / 6
    assert np.allclose(E, ref, atol=1e-15)


@pytest.mark.parametrize("m,seed", [(4, 1), (10, 2), (30, 3)])
def test_phi1_matches_dense_definition(m, seed):
    """phi_1(H) e_1 = H^{-1} (e^H - I) e_1 for nonsingular H (eq. (Phi1))."""
    rng = np.random.default_rng(seed)
    H = rng.standard_normal((m, m)) * 2.0 - 3.0 * np.eye(m)
    y = oracle.phi1_e1(H)
    e1 = np.zeros(m)
    e1[0] = 1.0
    ref = np.linalg.solve(H, (sla.expm(H) - np.eye(m)) @ e1)
    assert np.max(np.abs(y - ref)) < 1e-12 * np.max(np.abs(ref))


def test_phi1_singular_taylor():
    """Singular H is fine (the augmented form needs no inverse): for a
    nilpotent H the Taylor series sum H^k/(k+1)! terminates."""
    H = np.diag([1.0, 2.0, 3.0], 1)
    y = oracle.phi1_e1(H)
    ref = np.zeros(4)
    P = np.eye(4)
    for k in range(5):
        ref += P[:, 0] / math.factorial(k + 1)
        P = H @ P
    assert np.allclose(y, ref, atol=1e-15)


def test_arnoldi_identities():
    rng = np.random.default_rng(5)
    K, m = 200, 30
    A = rng.standard_normal((K, K)) / np.sqrt(K) - 0.5 * np.eye(K)
    b = rng.standard_normal(K)
    mu, Vb, H, beta = oracle.arnoldi_dense(A, b, m)
    assert mu == m
    Vm, Vm1 = Vb[:m].T, Vb[: m + 1].T
    assert abs(beta - np.linalg.norm(b)) < 1e-13 * beta
    assert np.max(np.abs(Vm1.T @ Vm1 - np.eye(m + 1))) < 1e-13
    assert np.max(np.abs(A @ Vm - Vm1 @ H)) < 1e-13
    assert np.allclose(np.tril(H, -2), 0.0)


def test_krylov_full_dimension_reproduces_phi1():
    """With m = K the Krylov approximation beta V_m phi_1(H_m) e_1 is phi_1(A) b."""
    rng = np.random.default_rng(6)
    K = 40
    A = rng.standard_normal((K, K)) / np.sqrt(K) * 3.0 - 2.0 * np.eye(K)
    b = rng.standard_normal(K)
    mu, Vb, H, beta = oracle.arnoldi_dense(A, b, K)
    y = oracle.phi1_e1(H[:mu, :mu])
    x = beta * Vb[:mu].T @ y
    ref = np.linalg.solve(A, (sla.expm(A) - np.eye(K)) @ b)
    assert np.max(np.abs(x - ref)) < 1e-11 * np.max(np.abs(ref))
    # smaller m: error decreases with m
    errs = []
    for m in (5, 10, 20):
        mu, Vb, H, beta = oracle.arnoldi_dense(A, b, m)
        errs.append(np.max(np.abs(beta * Vb[:mu].T @ oracle.phi1_e1(H[:mu, :mu]) - ref)))
    assert errs[0] > errs[1] > errs[2]


def test_arnoldi_happy_breakdown():
    """An invariant subspace of dimension 3 stops Arnoldi at j = 3 and the
    result is exact."""
    K = 12
    rng = np.random.default_rng(8)
    Q, _ = np.linalg.qr(rng.standard_normal((K, K)))
    Dg = np.diag(np.concatenate([[-1.0, -2.0, -3.0], -np.arange(4, K + 1, dtype=float)]))
    A = Q @ Dg @ Q.T
    b = Q[:, :3] @ np.array([1.0, 2.0, 3.0])
    mu, Vb, H, beta = oracle.arnoldi_dense(A, b, 10)
    assert mu == 3
    x = beta * Vb[:mu].T @ oracle.phi1_e1(H[:mu, :mu])
    ref = np.linalg.solve(A, (sla.expm(A) - np.eye(K)) @ b)
    assert np.max(np.abs(x - ref)) < 1e-13
