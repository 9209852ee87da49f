"""Direct pins of the oracle's grid-transfer operators (Sec. 3.2.1).

Restriction is the mean of the 8 children; prolongation of the coarse
correction (eq:solution_correction) is the cell-centred trilinear
interpolation whose weights are 27/9/3/1 over 64, taken on the side of the
parent that the fine cell occupies.  Each test checks or_restrict /
or_prolong_add against something they share no code with: NumPy block means,
exact reproduction of multilinear fields (which no other weight set of this
footprint achieves), the weight table the paper prints, and the closed form
of R P.  CPU only.
"""
import itertools
import json
import os

import numpy as np
import pytest

import oracle

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_tests.json")))
W = GOLD["transfer_operators"]["prolongation_weights_over_64"]


def _prolong(uc, n_fine):
    return oracle.prolong_add(np.zeros((n_fine,) * 3), uc, np.zeros_like(uc))


@pytest.mark.parametrize("nf", [8, 16])
def test_restriction_is_block_mean(nf):
    f = np.random.default_rng(11).standard_normal((nf,) * 3)
    nc = nf // 2
    ref = f.reshape(nc, 2, nc, 2, nc, 2).mean(axis=(1, 3, 5))
    np.testing.assert_allclose(oracle.restrict(f), ref, rtol=0, atol=1e-15)


def test_restriction_sees_only_its_own_block():
    # a fine spike moves exactly one coarse value, by 1/8
    nf = 8
    for (i, j, k) in ((0, 0, 0), (3, 6, 1), (7, 7, 7)):
        f = np.zeros((nf,) * 3)
        f[k, j, i] = 1.0
        c = oracle.restrict(f)
        expect = np.zeros((nf // 2,) * 3)
        expect[k // 2, j // 2, i // 2] = 0.125
        assert np.array_equal(c, expect)


@pytest.mark.parametrize("spike", [(1, 2, 3), (0, 0, 0), (3, 3, 3)])
def test_coarse_spike_gives_the_printed_stencil(spike):
    # A unit coarse value at parent P reaches exactly the fine cells whose
    # parent is P or whose parent's neighbour on the fine cell's side is P.
    # Per axis: the two children of P get their 3/4 share, and the child of
    # each neighbouring coarse cell that lies next to P gets 1/4.  The fine
    # value is the product of the three shares (27, 9, 3, 1 over 64).
    nc, nf = 4, 8
    I, J, K = spike
    uc = np.zeros((nc,) * 3)
    uc[K, J, I] = 1.0
    got = _prolong(uc, nf)
    n_of = {27: W["parent"], 9: W["face"], 3: W["edge"], 1: W["vertex"]}
    expect = np.zeros((nf,) * 3)
    for k, j, i in itertools.product(range(nf), repeat=3):
        w = 1
        for fine, par in ((i, I), (j, J), (k, K)):
            parent = fine // 2
            side = 1 if fine % 2 else -1
            if parent == par:
                w *= 3
            elif (parent + side) % nc == par:
                w *= 1
            else:
                w = 0
        if w:
            expect[k, j, i] = n_of[w] / 64.0
    np.testing.assert_array_equal(got, expect)
    # every weight class appears with its multiplicity: 8 children of P get
    # 27, and 9, 3, 1 each on 24 cells
    vals, counts = np.unique(np.round(got * 64).astype(int), return_counts=True)
    assert dict(zip(vals.tolist(), counts.tolist())) == {0: nf ** 3 - 8 * 8, 27: 8, 9: 24, 3: 24,
                                                         1: 8}
    assert got.sum() == pytest.approx(8.0, abs=1e-14)   # column sums: 8 children per unit


def _multilinear(xs, ys, zs, c):
    return (c[0] + c[1] * xs + c[2] * ys + c[3] * zs + c[4] * xs * ys + c[5] * xs * zs
            + c[6] * ys * zs + c[7] * xs * ys * zs)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_prolongation_reproduces_multilinear_fields(seed):
    # Sampled at coarse cell centres (2I + 1 in fine units), a multilinear
    # field is reproduced exactly at every fine centre (i + 1/2) that does not
    # reach across the periodic wrap.  Uniform weights (8/64 each) or the
    # neighbours taken on the wrong side of the parent both fail this.
    nc, nf = 8, 16
    c = np.random.default_rng(seed).standard_normal(8)
    X = 2.0 * np.arange(nc) + 1.0
    Zc, Yc, Xc = np.meshgrid(X, X, X, indexing="ij")
    uc = _multilinear(Xc, Yc, Zc, c)
    got = _prolong(uc, nf)
    x = np.arange(nf) + 0.5
    Zf, Yf, Xf = np.meshgrid(x, x, x, indexing="ij")
    ref = _multilinear(Xf, Yf, Zf, c)
    inner = slice(1, nf - 1)
    np.testing.assert_allclose(got[inner, inner, inner], ref[inner, inner, inner], rtol=0,
                               atol=1e-12 * np.abs(ref).max())


def test_prolongation_is_exact_on_a_linear_field_along_each_axis():
    nc, nf = 8, 16
    X = 2.0 * np.arange(nc) + 1.0
    x = np.arange(nf) + 0.5
    for axis in range(3):
        shape = [1, 1, 1]
        shape[2 - axis] = nc
        uc = np.broadcast_to((3.0 - 0.25 * X).reshape(shape), (nc,) * 3).copy()
        got = _prolong(uc, nf)
        shape[2 - axis] = nf
        ref = np.broadcast_to((3.0 - 0.25 * x).reshape(shape), (nf,) * 3)
        sl = [slice(None)] * 3
        sl[2 - axis] = slice(1, nf - 1)
        np.testing.assert_allclose(got[tuple(sl)], ref[tuple(sl)], rtol=0, atol=1e-14)


def test_prolongation_adds_the_difference_to_the_fine_field():
    rng = np.random.default_rng(5)
    nc, nf = 4, 8
    fine = rng.standard_normal((nf,) * 3)
    uc, rc = rng.standard_normal((2,) + (nc,) * 3)
    got = oracle.prolong_add(fine, uc, rc)
    np.testing.assert_allclose(got, fine + _prolong(uc - rc, nf), rtol=0, atol=1e-14)


def test_restriction_of_prolonged_constant_is_the_constant():
    nc = 4
    uc = np.full((nc,) * 3, -2.75)
    p = _prolong(uc, 2 * nc)
    np.testing.assert_allclose(p, -2.75, rtol=0, atol=1e-15)
    np.testing.assert_allclose(oracle.restrict(p), uc, rtol=0, atol=1e-15)


def test_restriction_after_prolongation_is_the_1_6_1_smoother():
    # Per axis, the two children of I get (3 u_I + u_{I-1})/4 and
    # (3 u_I + u_{I+1})/4, so their mean is (u_{I-1} + 6 u_I + u_{I+1})/8:
    # R P is the separable [1, 6, 1]/8 filter (periodic).
    nc = 8
    u = np.random.default_rng(9).standard_normal((nc,) * 3)
    ref = u.copy()
    for ax in range(3):
        ref = (np.roll(ref, 1, ax) + 6.0 * ref + np.roll(ref, -1, ax)) / 8.0
    np.testing.assert_allclose(oracle.restrict(_prolong(u, 2 * nc)), ref, rtol=0, atol=1e-14)
