"""Eigenvalues of the pencil blocks the divide-and-conquer leaves, of order
3 to 64 (sdc_block_eigvals: the double-shift QR algorithm on S^{-1} T, or on
T^{-1} S inverted when S is the worse conditioned), against the oracle's
LAPACK generalized eigenvalues of the same blocks, on real and complex
spectra, a singular S (an infinite eigenvalue), an ill-conditioned S, and
end to end: the benchmark-family pencil recursed to blocks of order <= 64,
every eigenvalue against the construction."""
import numpy as np
import pytest
import scipy.linalg as sla

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


def block_diag_pencil(sizes, seed):
    """Block-diagonal T and S, each block a random dense pair with S close
    to I (well conditioned), so the spectra mix real values and complex pairs."""
    rng = np.random.default_rng(seed)
    n = sum(sizes)
    t, s = np.zeros((n, n)), np.zeros((n, n))
    starts = [0]
    for m in sizes:
        a = starts[-1]
        t[a:a + m, a:a + m] = rng.standard_normal((m, m))
        s[a:a + m, a:a + m] = np.eye(m) + 0.3 * rng.standard_normal((m, m)) / np.sqrt(m)
        starts.append(a + m)
    return t, s, starts


def check_against_oracle(handle, t, s, starts, tol=1e-10):
    from oracle.eig_dc import block_eigvals
    wr, wi = handle.block_eigvals(dev(t), dev(s), starts, symmetric=False)
    got = wr.cpu().numpy() + 1j * wi.cpu().numpy()
    ref_r, ref_i = block_eigvals(t, s, starts, False)
    ref = ref_r + 1j * ref_i
    err = np.abs(got - ref) / np.maximum(1.0, np.abs(ref))
    assert np.all(np.isfinite(got)), got
    assert err.max() <= tol, (err.max(), np.argmax(err))
    return got


def test_dense_pencil_blocks_match_oracle(handle, sdc):
    sizes = [3, 4, 7, 16, 33, 64]
    print("CASE pencil leaves", sizes, flush=True)
    t, s, starts = block_diag_pencil(sizes, S.family_seed(1, 3000))
    got = check_against_oracle(handle, t, s, starts)
    assert np.any(got.imag != 0) and np.any(got.imag == 0)  # both kinds were exercised


@pytest.mark.parametrize("m", [3, 5, 12, 64])
def test_dense_pencil_single_block_orders(handle, sdc, m):
    print("CASE pencil leaf order", m, flush=True)
    t, s, starts = block_diag_pencil([m], S.family_seed(1, 3100 + m))
    check_against_oracle(handle, t, s, starts)


def test_dense_pencil_real_spectrum_known(handle, sdc):
    """T = U diag(lam) V^T, S = U V^T: the eigenvalues are lam exactly."""
    m = 40
    print("CASE pencil leaf known spectrum", m, flush=True)
    rng = np.random.default_rng(S.family_seed(1, 3200))
    u, _ = np.linalg.qr(rng.standard_normal((m, m)))
    v, _ = np.linalg.qr(rng.standard_normal((m, m)))
    lam = np.sort(rng.uniform(-3, 3, m))
    t, s = u @ np.diag(lam) @ v.T, u @ v.T
    wr, wi = handle.block_eigvals(dev(t), dev(s), [0, m], symmetric=False)
    assert np.abs(wi.cpu().numpy()).max() == 0.0
    assert np.abs(wr.cpu().numpy() - lam).max() <= 1e-12 * np.abs(lam).max()


def test_dense_pencil_singular_and_ill_conditioned_S(handle, sdc):
    """S of numerical rank m - 1 (a singular value at rounding level): one
    eigenvalue beyond 1e12 in magnitude (infinite in exact arithmetic; the
    T^{-1} S form), the others as LAPACK's; S with a singular value of 1e-9:
    a large eigenvalue, relative error as LAPACK's."""
    m = 6
    print("CASE pencil leaf singular S", flush=True)
    rng = np.random.default_rng(S.family_seed(1, 3300))
    t = rng.standard_normal((m, m)) + 3 * np.eye(m)
    u, _ = np.linalg.qr(rng.standard_normal((m, m)))
    w, _ = np.linalg.qr(rng.standard_normal((m, m)))
    for smin in (0.0, 1e-9):
        sv = np.linspace(1.0, 2.0, m)
        sv[0] = smin
        s = u @ np.diag(sv) @ w.T
        wr, wi = handle.block_eigvals(dev(t), dev(s), [0, m], symmetric=False)
        got = wr.cpu().numpy() + 1j * wi.cpu().numpy()
        ref = sla.eigvals(t, s)
        if smin == 0.0:
            big_g = ~(np.abs(got) < 1e12)
            big_r = ~(np.abs(ref) < 1e12)
            assert big_g.sum() == 1 and big_r.sum() == 1
            fin_g = np.sort_complex(got[~big_g])
            fin_r = np.sort_complex(ref[~big_r])
            assert len(fin_g) == len(fin_r) == m - 1
            assert np.max(np.abs(fin_g - fin_r) / np.maximum(1.0, np.abs(fin_r))) <= 1e-9
        else:
            g = np.sort_complex(got)
            r = np.sort_complex(ref)
            assert np.all(np.isfinite(g))
            assert np.max(np.abs(g - r) / np.maximum(1.0, np.abs(r))) <= 1e-6


@pytest.mark.parametrize("n", [512, 2048])
def test_eig_dc_leaf64_pencil_eigenvalues(handle, sdc, n):
    """The benchmark-family pencil recursed to blocks of order <= 64 (the
    measured configuration), then the dense leaf solver: every eigenvalue
    within max(1e-10, 2x LAPACK's error on the same blocks) of the
    construction, relative."""
    print("CASE eig_dc leaf64 eigenvalues", n, flush=True)
    from oracle.eig_dc import block_eigvals
    p = S.pencil_problem(n, S.family_seed(1, n))
    st, t, s, ql, qr, starts, info = handle.eig_dc(dev(p["A"]), dev(p["B"]), leaf_max=64, o=sdc.opts(seed=1))
    assert st == 0 and info["unsplit"] == 0
    assert max(e - a for a, e in zip(starts[:-1], starts[1:])) <= 64
    wr, wi = handle.block_eigvals(t, s, starts, symmetric=False)
    got = np.sort_complex(wr.cpu().numpy() + 1j * wi.cpu().numpy())
    want = np.sort_complex(p["lam"].astype(complex))
    err = np.max(np.abs(got - want) / np.abs(want))
    rr, ri = block_eigvals(t.cpu().numpy(), s.cpu().numpy(), starts, False)
    err_ref = np.max(np.abs(np.sort_complex(rr + 1j * ri) - want) / np.abs(want))
    assert err <= max(1e-10, 2 * err_ref), (err, err_ref)
