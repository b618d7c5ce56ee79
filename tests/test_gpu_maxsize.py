"""The largest supported order (16384: 32768 stacked rows, the deepest QR
reduction tree, four levels over 128 leaves, and the largest buffers) on a
symmetric split with a known spectrum, checked through properties that hold
at any size: the exact rank, the leading basis against the construction's
eigenvectors, E21 recomputed from the outputs, and the two diagonal blocks'
eigenvalues against the construction's.  The input is generated on the
device (seeded), since a host QR of this order would take minutes."""
import math

import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sdc():
    import paper_1011_3077_amd as P
    return P


def test_split_sym_maximum_order(sdc):
    n = 16384
    print("CASE maximum order", n, flush=True)
    dev = torch.device("cuda:0")
    g = torch.Generator(device=dev)
    g.manual_seed(10113077 + n)
    q, _ = torch.linalg.qr(torch.randn(n, n, device=dev, dtype=torch.float64, generator=g))
    u = torch.rand(n, device=dev, dtype=torch.float64, generator=g)
    d = 0.05 + 0.95 * u
    d[: n // 2] = -d[: n // 2]  # half the eigenvalues on each side of Re z = 0
    a = (q * d) @ q.T
    a = 0.5 * (a + a.T)
    k_want = int((d > 0).sum())
    h = sdc.Handle(0)
    try:
        res = h.split_sym(a, sdc.region("halfplane", shift=0.0, scale=1.0), sdc.opts(seed=1))
        info = res.info
        print("CASE maximum order done", info["iters_right"], info["e21_rel"], info["ms"], flush=True)
        assert res.status == sdc.SDC_OK and info["k_lead"] == k_want
        k = k_want
        qk = res.Q[:, :k]
        # the leading basis against the eigenvectors of the negative
        # eigenvalues: ||Q_-^T Q[:, :k]||_F / sqrt(k) bounds the sine of the
        # largest principal angle from above by at most sqrt(k)
        cross = q[:, d < 0].T @ qk
        assert torch.linalg.norm(cross).item() / math.sqrt(k) <= 1e-9
        ah = res.Ahat
        norm1 = lambda x: torch.sum(torch.abs(x), dim=0).max().item()
        e21 = norm1(ah[k:, :k]) / norm1(a)
        assert e21 <= 1e-10 and abs(e21 - info["e21_rel"]) <= 1e-12
        ev = torch.cat([torch.linalg.eigvalsh(ah[:k, :k]), torch.linalg.eigvalsh(ah[k:, k:])])
        err = (torch.sort(ev).values - torch.sort(d).values).abs().max().item()
        assert err <= 1e-10 * d.abs().max().item()
    finally:
        h.close()
        del q, a
        torch.cuda.empty_cache()
