"""Pins of the Householder QR oracle against facts fixed by mathematics.

The oracle is the plain definition of what the tiled factorization computes
(unblocked Householder QR; Section II of the paper equates every elimination
list with it).  These tests tie it to things other than itself: closed forms,
special cases, invariants within the backward-error bound, the LAPACK routine
on small inputs, and brute-force Gram-Schmidt on tiny ones.  A dropped term,
a wrong sign or a transposed operand in the oracle breaks at least one.
"""
import numpy as np
import pytest

from oracle import qr as oq

U = np.finfo(np.float64).eps


def test_closed_form_2x1():
    R = oq.r_factor(np.array([[3.0], [4.0]]))
    assert R.shape == (1, 1)
    assert abs(abs(R[0, 0]) - 5.0) < 1e-15
    # LAPACK sign convention: R_jj = -sign(alpha) * norm
    assert R[0, 0] == -5.0


def test_closed_form_2x2_by_hand():
    # Gram-Schmidt by hand: q1 = (3,4)/5, r12 = q1.(1,2) = 11/5, r22 = |(1,2) - 11/25 (3,4)| = 2/5
    Rn = oq.sign_normalize(oq.r_factor(np.array([[3.0, 1.0], [4.0, 2.0]])))
    np.testing.assert_allclose(Rn, [[5.0, 2.2], [0.0, 0.4]], rtol=0, atol=1e-14)


def test_diagonal_matrix():
    d = np.array([3.0, -2.0, 0.5, -7.0, 1e-3])
    Rn = oq.sign_normalize(oq.r_factor(np.diag(d)))
    np.testing.assert_array_equal(Rn, np.diag(np.abs(d)))


def test_upper_triangular_matrix_is_its_own_r_up_to_row_signs():
    rng = np.random.default_rng(11)
    T = np.triu(rng.standard_normal((9, 9)))
    Rn = oq.sign_normalize(oq.r_factor(T))
    np.testing.assert_allclose(Rn, oq.sign_normalize(T), rtol=0, atol=1e-14)


def test_orthonormal_columns_give_identity():
    rng = np.random.default_rng(12)
    Q, _ = np.linalg.qr(rng.standard_normal((40, 12)))
    Rn = oq.sign_normalize(oq.r_factor(Q))
    np.testing.assert_allclose(Rn, np.eye(12), rtol=0, atol=1e-14)


def test_zero_column_gives_identity_reflector():
    A = np.zeros((6, 3))
    A[:, 0] = [1, 2, 3, 4, 5, 6]
    A[:, 2] = [0, 1, 0, 1, 0, 1]
    F, tau = oq.factor(A)
    assert tau[1] == 0.0  # the zero second column stays zero, so its reflector is H = I
    R = oq.r_of(F)
    assert np.all(np.isfinite(R))
    Q = oq.thin_q(F, tau)
    np.testing.assert_allclose(Q @ R, A, atol=1e-13)


def test_brute_force_gram_schmidt_tiny():
    rng = np.random.default_rng(13)
    for m, n in [(3, 3), (5, 2), (6, 4), (7, 7)]:
        A = rng.standard_normal((m, n))
        # classical Gram-Schmidt in exact-ish arithmetic via Python floats, tiny sizes only
        Q = np.zeros((m, n))
        Rgs = np.zeros((n, n))
        for j in range(n):
            v = A[:, j].copy()
            for i in range(j):
                Rgs[i, j] = Q[:, i] @ A[:, j]
                v -= Rgs[i, j] * Q[:, i]
            Rgs[j, j] = np.linalg.norm(v)
            Q[:, j] = v / Rgs[j, j]
        np.testing.assert_allclose(oq.sign_normalize(oq.r_factor(A)), Rgs, rtol=0, atol=1e-12)


@pytest.mark.parametrize("m,n", [(64, 64), (300, 120), (512, 256), (129, 17)])
def test_invariants_within_backward_error(m, n):
    rng = np.random.default_rng(m * 1000 + n)
    A = rng.standard_normal((m, n))
    F, tau = oq.factor(A)
    R = oq.r_of(F)
    Q = oq.thin_q(F, tau)
    bound = 10 * U * np.sqrt(m * n)
    nA = np.linalg.norm(A)
    assert np.linalg.norm(A - Q @ R) / nA < bound
    assert np.linalg.norm(Q.T @ Q - np.eye(n)) < bound
    assert np.linalg.norm(R.T @ R - A.T @ A) / nA**2 < bound


@pytest.mark.parametrize("m,n", [(50, 50), (200, 80), (512, 256)])
def test_matches_lapack(m, n):
    rng = np.random.default_rng(7 + m + n)
    A = rng.standard_normal((m, n))
    R1 = oq.sign_normalize(oq.r_factor(A))
    R2 = oq.sign_normalize(np.linalg.qr(A, mode="r"))
    assert np.linalg.norm(R1 - R2) / np.linalg.norm(R2) < 1e-13


def test_thread_count_does_not_change_bits():
    rng = np.random.default_rng(3)
    A = rng.standard_normal((400, 100))
    F1, t1 = oq.factor(A, nthreads=1)
    F8, t8 = oq.factor(A, nthreads=8)
    assert np.array_equal(F1, F8) and np.array_equal(t1, t8)


def test_apply_qt_then_q_is_identity_and_qt_a_is_r():
    rng = np.random.default_rng(5)
    A = rng.standard_normal((90, 30))
    F, tau = oq.factor(A)
    B = rng.standard_normal((90, 4))
    np.testing.assert_allclose(oq.apply_q(F, tau, oq.apply_qt(F, tau, B)), B, atol=1e-13)
    QtA = oq.apply_qt(F, tau, A)
    np.testing.assert_allclose(QtA[:30], oq.r_of(F), atol=1e-13)
    np.testing.assert_allclose(QtA[30:], 0.0, atol=1e-13)


def test_lstsq_matches_normal_equations_and_lapack():
    rng = np.random.default_rng(9)
    A = rng.standard_normal((120, 20))
    b = rng.standard_normal(120)
    x = oq.lstsq(A, b).ravel()
    xl = np.linalg.lstsq(A, b, rcond=None)[0]
    np.testing.assert_allclose(x, xl, rtol=1e-12, atol=1e-13)
    # optimality: the residual is orthogonal to range(A)
    r = b - A @ x
    assert np.linalg.norm(A.T @ r) / (np.linalg.norm(A) * np.linalg.norm(b)) < 1e-13


def test_rank_one_update_consistency_r_depends_only_on_leading_columns():
    # R[:, :c] of A equals R of A[:, :c]: what the sampled full-size parity checks use
    rng = np.random.default_rng(21)
    A = rng.standard_normal((200, 60))
    R = oq.r_factor(A)
    Rc = oq.r_factor(A[:, :25])
    np.testing.assert_array_equal(R[:25, :25], Rc)
