"""Pins of the oracle's divide-and-conquer (Sec. 3.3-3.5): the block spectra
equal the construction's eigenvalues, every block is at most leaf_max, the pair
is block upper triangular and orthogonally equivalent to the input up to the
dropped coupling blocks."""
import numpy as np
import pytest
import scipy.linalg as sla

import sdc_synth as S
from oracle.eig_dc import eig_dc


def _block_spectrum(t, s, blocks):
    ev = []
    for a0, a1 in blocks:
        if s is None:
            ev.append(np.linalg.eigvalsh(0.5 * (t[a0:a1, a0:a1] + t[a0:a1, a0:a1].T)))
        else:
            ev.append(sla.eigvals(t[a0:a1, a0:a1], s[a0:a1, a0:a1]))
    return np.concatenate(ev)


@pytest.mark.parametrize("n,leaf", [(60, 16), (128, 32)])
def test_eig_dc_symmetric(n, leaf):
    a, d, q = S.sym_problem(n, 50 + n)
    r = eig_dc(a, symmetric=True, leaf_max=leaf, seed=1)
    assert r["unsplit"] == 0
    assert all(e - s <= leaf for s, e in r["blocks"])
    assert r["blocks"][0][0] == 0 and r["blocks"][-1][1] == n
    ev = np.sort(_block_spectrum(r["T"], None, r["blocks"]))
    assert np.abs(ev - np.sort(d)).max() <= 1e-12
    qq = r["QR"]
    assert np.allclose(qq.T @ qq, np.eye(n), atol=1e-12)
    # T is block diagonal and Q^T A Q equals it up to the dropped couplings
    assert np.linalg.norm(qq.T @ a @ qq - r["T"], 2) <= 1e-11


@pytest.mark.parametrize("n,leaf", [(64, 16), (160, 32)])
def test_eig_dc_pencil(n, leaf):
    p = S.pencil_problem(n, 70 + n)
    r = eig_dc(p["A"], p["B"], leaf_max=leaf, seed=2)
    assert r["unsplit"] == 0
    assert all(e - s <= leaf for s, e in r["blocks"])
    t, s_ = r["T"], r["S"]
    for a0, a1 in r["blocks"]:
        assert np.all(t[a1:, a0:a1] == 0) and np.all(s_[a1:, a0:a1] == 0)
    got = np.sort_complex(_block_spectrum(t, s_, r["blocks"]))
    want = np.sort_complex(p["lam"].astype(complex))
    assert np.max(np.abs(got - want) / np.abs(want)) <= 1e-10
    ql, qr = r["QL"], r["QR"]
    assert np.allclose(ql.T @ ql, np.eye(n), atol=1e-12) and np.allclose(qr.T @ qr, np.eye(n), atol=1e-12)
    assert np.linalg.norm(ql.T @ p["A"] @ qr - t, 2) <= 1e-10 * np.linalg.norm(p["A"], 2)
    assert np.linalg.norm(ql.T @ p["B"] @ qr - s_, 2) <= 1e-10 * np.linalg.norm(p["B"], 2)
