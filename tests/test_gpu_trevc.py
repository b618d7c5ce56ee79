"""TREVC (sdc_trevc, Alg. 8) on the GPU against the oracle's entry formula,
and end to end: the divide-and-conquer to 1 x 1 blocks of a real-spectrum
pencil, then TREVC, gives the pencil's right eigenvectors Q_R X."""
import numpy as np
import pytest

import sdc_synth as S

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sdc():
    import paper_1011_3077_amd as P
    return P


@pytest.fixture(scope="module")
def handle(sdc):
    h = sdc.Handle(0)
    yield h
    h.close()


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")


def tri(n, seed, pencil):
    """Upper-triangular T (and S), eigenvalues spread over [-2, 2], strictly
    upper entries N(0,1)/n (eigenvector entries stay O(1) to O(100)); the
    strictly lower parts hold garbage that must not be read."""
    rng = np.random.default_rng(seed)
    d = rng.permutation(np.linspace(-2.0, 2.0, n)) if n > 1 else np.array([0.7])
    t = np.triu(rng.standard_normal((n, n)) / n, 1) + np.diag(d) + np.tril(rng.standard_normal((n, n)), -1)
    if not pencil:
        return t, None
    s = np.triu(rng.standard_normal((n, n)) / n, 1) + np.diag(rng.uniform(0.5, 2.0, n)) \
        + np.tril(rng.standard_normal((n, n)), -1)
    return t, s


@pytest.mark.parametrize("n,pencil", [(1, False), (2, False), (31, False), (32, False), (33, True),
                                      (100, False), (257, True), (700, False)])
def test_trevc_matches_oracle(handle, sdc, n, pencil):
    from oracle.trevc import trevc
    print("CASE trevc", n, pencil, flush=True)
    t, s = tri(n, 900 + n, pencil)
    x = handle.trevc(dev(t), None if s is None else dev(s)).cpu().numpy()
    ref = trevc(t, s)
    assert np.all(np.tril(x, -1) == 0) and np.array_equal(np.diag(x), np.ones(n))
    assert np.abs(x - ref).max() <= 1e-12 * np.abs(ref).max()
    tu = np.triu(t)
    su = np.eye(n) if s is None else np.triu(s)
    lam = np.diag(tu) / np.diag(su)
    r = tu @ x - (su @ x) * lam[None, :]
    assert np.abs(r).max() <= 1e-13 * n * np.abs(x).max()


def test_trevc_invalid_arguments(handle, sdc):
    print("CASE trevc invalid", flush=True)
    t = dev(np.eye(4))
    with pytest.raises(sdc.SdcError, match="INVALID"):
        sdc._check(sdc.lib.sdc_trevc(handle._h, 4, t.data_ptr(), 3, None, 4, t.data_ptr(), 4))
    assert sdc.lib.sdc_trevc(handle._h, 0, None, 1, None, 1, None, 1) == sdc.SDC_OK


def test_pencil_eigenvectors_from_divide_and_conquer(handle, sdc):
    """The c1 construction at order 200 (real eigenvalues T_ii / S_ii):
    sdc_eig_dc to blocks of order 1 leaves (T, S) upper triangular; TREVC's
    X gives V = Q_R X with A V = B V diag(lambda) up to the dropped coupling
    blocks, and lambda is the construction's spectrum."""
    n = 200
    print("CASE eig_dc + trevc", n, flush=True)
    p = S.pencil_problem(n, S.family_seed(1, 200))
    st, t, s, ql, qr, starts, info = handle.eig_dc(dev(p["A"]), dev(p["B"]), leaf_max=1, o=sdc.opts(seed=2))
    assert st == 0 and info["unsplit"] == 0 and len(starts) == n + 1
    tn, sn = t.cpu().numpy(), s.cpu().numpy()
    assert np.all(np.tril(tn, -1) == 0) and np.all(np.tril(sn, -1) == 0)
    lam = np.diag(tn) / np.diag(sn)
    assert np.max(np.abs(np.sort(lam) - np.sort(p["lam"])) / np.abs(np.sort(p["lam"]))) <= 1e-10
    x = handle.trevc(t, s)
    v = (qr @ x).cpu().numpy()
    v /= np.linalg.norm(v, axis=0)[None, :]
    a, b = p["A"], p["B"]
    res = np.linalg.norm(a @ v - (b @ v) * lam[None, :], axis=0)
    scale = np.linalg.norm(a, 2) + np.abs(lam) * np.linalg.norm(b, 2)
    bound = info["levels"] * np.sqrt(n) * max(info["e21_max"], 1e-15) * 10
    assert np.max(res / scale) <= bound, (np.max(res / scale), bound)
