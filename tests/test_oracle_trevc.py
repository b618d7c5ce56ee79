"""Pins of the oracle's TREVC (eigenvectors of an upper-triangular matrix or
pencil, Sec. 5): the 2 x 2 closed form, the defining equation T X = X D
(T X = S X diag(lambda) for a pencil), LAPACK's eigenvectors of the same
matrices, the null vector of T - lambda_j I found by brute force (SVD), and
the blocked schedule of Alg. 8 reaching the same X."""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle.trevc import trevc, eigenvalues


def tri_problem(n, seed, pencil=False):
    """Upper-triangular T (and S) with well-separated diagonal entries."""
    rng = np.random.default_rng(seed)
    d = rng.permutation(np.linspace(-2.0, 2.0, n) + rng.uniform(-0.2, 0.2, n) / max(n, 1))
    t = np.triu(rng.standard_normal((n, n)) / np.sqrt(n), 1) + np.diag(d)
    if not pencil:
        return t, None
    s = np.triu(rng.standard_normal((n, n)) / np.sqrt(n), 1) + np.diag(rng.uniform(0.5, 2.0, n))
    return t, s


def test_two_by_two_closed_form():
    a, b, c = 0.3, -1.7, 2.2
    x = trevc(np.array([[a, b], [0.0, c]]))
    assert np.allclose(x, [[1.0, b / (c - a)], [0.0, 1.0]], rtol=1e-15, atol=0)


@pytest.mark.parametrize("n", [1, 5, 40, 97])
def test_defining_equation(n):
    t, _ = tri_problem(n, 10 + n)
    x = trevc(t)
    assert np.array_equal(np.diag(x), np.ones(n)) and np.all(np.tril(x, -1) == 0)
    r = t @ x - x * np.diag(t)[None, :]
    assert np.abs(r).max() <= 1e-13 * np.abs(t).max() * max(1.0, np.abs(x).max())


@pytest.mark.parametrize("n", [6, 40])
def test_pencil_defining_equation(n):
    t, s = tri_problem(n, 20 + n, pencil=True)
    x = trevc(t, s)
    lam = eigenvalues(t, s)
    assert np.allclose(lam, np.diag(t) / np.diag(s), rtol=0, atol=0)
    r = t @ x - (s @ x) * lam[None, :]
    assert np.abs(r).max() <= 1e-13 * max(np.abs(t).max(), np.abs(s).max()) * np.abs(x).max() * np.abs(lam).max()


def test_matches_lapack_eigenvectors():
    """LAPACK's right eigenvectors (unit 2-norm) are X's columns, normalized."""
    n = 30
    t, _ = tri_problem(n, 7)
    x = trevc(t)
    w, v = sla.eig(t)
    for j in range(n):
        i = int(np.argmin(np.abs(w - t[j, j])))
        vj = np.real(v[:, i])
        xj = x[:, j] / np.linalg.norm(x[:, j])
        assert min(np.abs(vj - xj).max(), np.abs(vj + xj).max()) <= 1e-12


def test_matches_lapack_generalized_eigenvectors():
    n = 25
    t, s = tri_problem(n, 8, pencil=True)
    x = trevc(t, s)
    w, v = sla.eig(t, s)
    lam = np.diag(t) / np.diag(s)
    for j in range(n):
        i = int(np.argmin(np.abs(w - lam[j])))
        vj = np.real(v[:, i]) / np.linalg.norm(np.real(v[:, i]))
        xj = x[:, j] / np.linalg.norm(x[:, j])
        assert min(np.abs(vj - xj).max(), np.abs(vj + xj).max()) <= 1e-11


def test_brute_force_null_vectors():
    """Each column spans the null space of T - T_jj I (smallest right
    singular vector), by SVD on a tiny matrix."""
    n = 9
    t, _ = tri_problem(n, 3)
    x = trevc(t)
    for j in range(n):
        _, sv, vt = np.linalg.svd(t - t[j, j] * np.eye(n))
        z = vt[-1]
        xj = x[:, j] / np.linalg.norm(x[:, j])
        assert sv[-1] <= 1e-14 * sv[0]
        assert min(np.abs(z - xj).max(), np.abs(z + xj).max()) <= 1e-12


def _blocked_alg8(t, s, b):
    """Alg. 8's schedule: per block column J, the diagonal block first, then
    block rows I = J-1 .. 0 with the accumulated sum over K = I+1 .. J of
    T[I,K] X[K,J] (and S's), then the small solve for X[I,J]."""
    n = t.shape[0]
    s = np.eye(n) if s is None else s
    lam = np.diag(t) / np.diag(s)
    x = np.zeros((n, n))
    nb = (n + b - 1) // b
    for J in range(nb):
        c0, c1 = J * b, min(n, (J + 1) * b)
        x[c0:c1, c0:c1] = trevc(t[c0:c1, c0:c1], s[c0:c1, c0:c1])
        for I in range(J - 1, -1, -1):
            r0, r1 = I * b, (I + 1) * b
            gt = t[r0:r1, r1:c1] @ x[r1:c1, c0:c1]
            gs = s[r0:r1, r1:c1] @ x[r1:c1, c0:c1]
            for jj in range(c1 - c0):
                l = lam[c0 + jj]
                m = np.triu(t[r0:r1, r0:r1] - l * s[r0:r1, r0:r1])
                x[r0:r1, c0 + jj] = sla.solve_triangular(m, -(gt[:, jj] - l * gs[:, jj]))
    return x


@pytest.mark.parametrize("n,b,pencil", [(70, 16, False), (64, 32, True), (33, 8, False)])
def test_blocked_schedule_reaches_the_same_vectors(n, b, pencil):
    t, s = tri_problem(n, 40 + n, pencil=pencil)
    x = trevc(t, s)
    xb = _blocked_alg8(t, s, b)
    assert np.abs(x - xb).max() <= 1e-12 * np.abs(x).max()
