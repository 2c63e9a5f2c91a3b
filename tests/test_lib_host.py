"""Host-side checks of the library (no GPU): it loads, exports every symbol
its header declares, and its univariate setup matches the oracle."""
import os
import re

import numpy as np
import pytest

import synth
from oracle import fd, splines

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_1602_01636_amd import binding
    return binding.lib()


def test_library_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "igafd.h")).read()
    names = set(re.findall(r"\b(igafd_[A-Za-z_0-9]+)\s*\(", hdr))
    assert {"igafd_setup", "igafd_solve", "igafd_apply_precond", "igafd_apply_A"} <= names
    L = _lib()
    for n in sorted(names):
        assert hasattr(L, n), n


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6])
def test_univariate_matches_oracle(p):
    from paper_1602_01636_amd import igafd_univariate
    kn = synth.jittered_knots(13, p, seed=p)
    M, K, U, lam = igafd_univariate(p, kn)
    Mo, Ko = splines.univariate_matrices(kn, p)
    Uo, lo = fd.generalized_eig(Ko, Mo)
    np.testing.assert_allclose(M, Mo, atol=1e-15 * np.abs(Mo).max() * 10)
    np.testing.assert_allclose(K, Ko, rtol=1e-12, atol=1e-12 * np.abs(Ko).max())
    np.testing.assert_allclose(lam, lo, rtol=1e-11)
    np.testing.assert_allclose(U.T @ Mo @ U, np.eye(len(lam)), atol=1e-11)
    np.testing.assert_allclose(U.T @ Ko @ U, np.diag(lo), atol=1e-9 * lo.max())


@pytest.mark.parametrize("p", [2, 5])
def test_univariate_large_threaded(p):
    # several row blocks and threads in the host eigensolver; a p-fold
    # interior knot (the two-patch knot vector of the L-shaped domain) gives
    # nearly equal eigenvalue pairs
    from oracle import multipatch as mp
    from paper_1602_01636_amd import igafd_univariate
    kn = mp.merged_knots(synth.jittered_knots(200, p, seed=p), p)
    M, K, U, lam = igafd_univariate(p, kn)
    Mo, Ko = splines.univariate_matrices(kn, p)
    _, lo = fd.generalized_eig(Ko, Mo)
    assert len(lam) > 400
    np.testing.assert_allclose(lam, lo, rtol=1e-10)
    np.testing.assert_allclose(U.T @ Mo @ U, np.eye(len(lam)), atol=1e-10)
    np.testing.assert_allclose(U.T @ Ko @ U, np.diag(lo), atol=1e-9 * lo.max())


def test_univariate_repeated_knots_and_errors():
    from paper_1602_01636_amd import IgafdError, igafd_univariate
    kn = np.array([0, 0, 0, 0, 0.25, 0.5, 0.5, 0.75, 1, 1, 1, 1], float)
    M, K, U, lam = igafd_univariate(3, kn)
    Mo, Ko = splines.univariate_matrices(kn, 3)
    np.testing.assert_allclose(K, Ko, rtol=1e-12, atol=1e-12)
    for p, bad in ((2, [0, 0, 0.5, 1, 1]), (2, [0, 0, 0, 0.5, 0.5, 0.5, 1, 1, 1]), (1, [0, 0, 0.6, 0.5, 1, 1]),
                   (1, [0, 0.1, 0.5, 1, 1])):
        with pytest.raises((IgafdError, ValueError)):
            igafd_univariate(p, np.array(bad, float))
    with pytest.raises(IgafdError):
        igafd_univariate(7, synth.uniform_knots(10, 7))   # degree above the supported maximum


def test_table_cond_through_library():
    # the paper's Table cond (Sec. 4.2) reproduced by the library's host setup
    import json
    g = json.load(open(os.path.join(ROOT, "tests", "golden", "table_cond.json")))
    from paper_1602_01636_amd import igafd_univariate
    for p, printed, check in zip(g["degrees"], g["printed"], g["assert"]):
        if p > 6:
            continue
        _, _, _, lam = igafd_univariate(p, synth.uniform_knots(g["elements"], p))
        if check:
            assert float(f"{lam.max() / lam.min():.0e}") == printed
