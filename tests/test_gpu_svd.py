"""RSVD split (sdc_split_svd) on the GPU: one symmetric split step of the
embedding [0 A; A^T 0], against the oracle on the same seeded input and
against the construction's singular values and subspaces."""
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


def sin_theta(x, y):
    qx, _ = np.linalg.qr(x)
    qy, _ = np.linalg.qr(y)
    return float(np.linalg.norm(qy - qx @ (qx.T @ qy), 2))


def check(res, a, sig, p_, q_, level):
    st, info, u, v, s11 = res
    m, n = a.shape
    r = min(m, n)
    k = info["k_lead"]
    assert st == 0 and k == int((sig > level).sum())
    u, v, s11 = u.cpu().numpy(), v.cpu().numpy(), s11.cpu().numpy()
    assert u.shape == (m, r) and v.shape == (n, r) and s11.shape == (r, r)
    uk, vk = u[:, :k], v[:, :k]
    assert np.abs(uk.T @ uk - np.eye(k)).max() <= 1e-12
    assert np.abs(vk.T @ vk - np.eye(k)).max() <= 1e-12
    assert sin_theta(uk, p_[:, :k]) <= 1e-9 and sin_theta(vk, q_[:, :k]) <= 1e-9
    assert np.abs(np.linalg.eigvalsh(s11[:k, :k]) - np.sort(sig[:k])).max() <= 1e-11 * sig[0]
    assert np.abs(uk.T @ a @ vk - s11[:k, :k]).max() <= 1e-11 * sig[0]
    assert not u[:, k:].any() and not v[:, k:].any() and not s11[k:, :].any() and not s11[:, k:].any()
    return k, uk, vk, s11[:k, :k]


@pytest.mark.parametrize("m,n", [(120, 80), (80, 120), (200, 200), (37, 5)])
def test_split_svd_matches_oracle(handle, sdc, m, n):
    from oracle.split import split_svd
    print("CASE split_svd", m, n, flush=True)
    a, sig, p_, q_ = S.svd_problem(m, n, S.family_seed(5, m * 1000 + n), level=1.0)
    reg = sdc.region("halfplane", shift=1.0, scale=1.0)
    res = handle.split_svd(dev(a), reg, sdc.opts(seed=5))
    k, uk, vk, s11 = check(res, a, sig, p_, q_, 1.0)
    ref, ru, rv, rs = split_svd(a, {"kind": "halfplane", "shift": 1.0, "scale": 1.0}, seed=5)
    assert ref.k == k
    assert sin_theta(uk, ru) <= 1e-10 and sin_theta(vk, rv) <= 1e-10
    assert np.abs(np.linalg.eigvalsh(s11) - np.linalg.eigvalsh(rs)).max() <= 1e-11 * sig[0]


def test_split_svd_larger(handle, sdc):
    """1500 x 1000 (embedding of order 2500): construction properties only."""
    m, n = 1500, 1000
    print("CASE split_svd", m, n, flush=True)
    a, sig, p_, q_ = S.svd_problem(m, n, S.family_seed(5, 1), level=2.0)
    res = handle.split_svd(dev(a), sdc.region("halfplane", shift=2.0, scale=2.0), sdc.opts(seed=1))
    check(res, a, sig, p_, q_, 2.0)


def test_split_svd_edges(handle, sdc):
    print("CASE split_svd edges", flush=True)
    a, sig, p_, q_ = S.svd_problem(30, 20, S.family_seed(5, 2), level=1.0, hi=5.0)
    A = dev(a)
    st, info, u, v, s11 = handle.split_svd(A, sdc.region("halfplane", shift=50.0, scale=1.0), sdc.opts(seed=1))
    assert st == sdc.SDC_NO_SPLIT and info["k_lead"] == 0
    assert not u.any().item() and not v.any().item() and not s11.any().item()
    with pytest.raises(sdc.SdcError):
        handle.split_svd(A, sdc.region("halfplane", shift=-1.0, scale=1.0))
    with pytest.raises(sdc.SdcError):
        handle.split_svd(A, sdc.region("disk", center=0.0, radius=1.0))
    with pytest.raises(sdc.SdcError):  # 30 x 20: ten zero eigenvalues of the embedding on Re z = 0
        handle.split_svd(A, sdc.region("halfplane", shift=0.0, scale=1.0))


def test_split_svd_tiny_shapes(handle, sdc):
    """1 x 1 and 1 x n / n x 1 matrices: the embedding of order m + n has the
    one singular value and its negative (and zeros); a shift below it splits
    off exactly that value, U and V are unit vectors along A's."""
    print("CASE split_svd tiny", flush=True)
    reg = sdc.region("halfplane", shift=0.5, scale=1.0)
    for a in (np.array([[2.0]]), np.array([[1.0, 2.0, 2.0]]), np.array([[3.0], [4.0]])):
        st, info, u, v, s11 = handle.split_svd(dev(a), reg, sdc.opts(seed=2))
        sig = np.linalg.norm(a, 2)
        assert st == 0 and info["k_lead"] == 1
        u1, v1 = u.cpu().numpy()[:, 0], v.cpu().numpy()[:, 0]
        assert abs(abs(u1 @ a @ v1) - sig) <= 1e-12 * sig
        assert abs(s11.cpu().numpy()[0, 0] - sig) <= 1e-12 * sig
