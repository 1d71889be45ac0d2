"""Pins for the oracle's block-Krylov basis builder: the basis dimensions the
paper prints (Tables 1-3 and the method labels of section "Experiments"), Lemma 3.1
(the Rayleigh-quotient structure), orthonormality, deflation and the mode-size
cap (section "BK method")."""
import json
import os

import numpy as np
import pytest

from oracle import bk, sptensor, ttmc
from oracle.orth import orth_append, orthonormalize
from paper_2012_07595_amd import workloads

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "bk_dims.json")))
TYPOS = {(v, r, p, st): (printed, rule) for v, r, p, st, _, printed, rule in GOLD["typos"]}


@pytest.mark.parametrize("row", GOLD["tables"], ids=lambda r: f"{r[0]}-r{r[1]}-s{r[3]}")
def test_table_dimensions(row):
    v, r, p, st, k1, k3 = row
    got = bk.dims(v, r, r, p, st)[-1]
    key = (v, r, p, st)
    if key in TYPOS:
        printed, rule = TYPOS[key]
        assert k1 == printed and got == (rule, k3)
    else:
        assert got == (k1, k3)


@pytest.mark.parametrize("lab", GOLD["labels"], ids=lambda d: f"{d['variant']}-r{d['r']}-s{d['s']}")
def test_caption_labels(lab):
    got = bk.dims(lab["variant"], lab["r"], lab["r"], lab["p"], lab["s"], n=lab["n"])[-1]
    assert got == (lab["k1"], lab["k3"])


def small_tensor(seed=3, m=40, n=12, nnz=900):
    c = workloads.sparse_sym(m, n, nnz, zipf=0.0, values="normal", seed=seed, dtype=np.float64)
    return sptensor.from_coo(c.m, c.n, c.i, c.j, c.k, c.val)


def build(T, r, r3, p, s, variant="bk", seed=1):
    U, W = workloads.random_start(T.m, T.n, r, r3, seed)
    basis = bk.Basis(orthonormalize(U), orthonormalize(W))
    for st in range(1, s + 1):
        bk.run_stage(T, basis, variant, st, None if variant == "max" else p)
    return basis


@pytest.mark.parametrize("variant", ["bk", "min", "max"])
def test_basis_orthonormal_and_dims(variant):
    T = small_tensor()
    basis = build(T, 2, 2, 3, 2, variant)
    X, Z = basis.X, basis.Z
    assert np.abs(X.T @ X - np.eye(X.shape[1])).max() < 1e-13
    assert np.abs(Z.T @ Z - np.eye(Z.shape[1])).max() < 1e-13
    expect = bk.dims(variant, 2, 2, None if variant == "max" else 3, 2, m=T.m, n=T.n)[-1]
    assert (X.shape[1], Z.shape[1]) == expect


def test_rayleigh_structure_lemma():
    """A.(U_j, U_0, W_0) = 0 for j >= 2 (Lemma 3.1), and A.(U_1, U_0, W_0) = H_1^1."""
    T = small_tensor(5)
    basis = build(T, 2, 2, 4, 2)
    U0, W0 = basis.ub[0], basis.wb[0]
    T1 = ttmc.free1(T, U0, W0)
    scale = np.abs(T1).max()
    for j in range(2, len(basis.ub)):
        assert np.abs(basis.ub[j].T @ T1).max() < 1e-12 * scale
    assert np.abs(basis.ub[1].T @ T1).max() > 1e-3 * scale
    T3 = ttmc.free3(T, U0, sym_half=True)
    for j in range(2, len(basis.wb)):
        assert np.abs(basis.wb[j].T @ T3).max() < 1e-12 * np.abs(T3).max()


def test_mode_size_cap():
    """Once k3 reaches n the W-expansion stops (section "BK method")."""
    T = small_tensor(7, m=30, n=4, nnz=400)
    basis = build(T, 2, 2, 4, 2)
    assert basis.Z.shape[1] == T.n
    assert np.abs(basis.Z.T @ basis.Z - np.eye(T.n)).max() < 1e-13


def test_deflation_drops_dependent_columns():
    rng = np.random.default_rng(0)
    Q = np.linalg.qr(rng.standard_normal((50, 3)))[0]
    b = rng.standard_normal((50, 2))
    B = np.concatenate([b[:, :1], Q @ rng.standard_normal((3, 1)), b[:, 1:], b[:, :1] * 2.0], axis=1)
    Qn, kept = orth_append(Q, B, 50)
    assert kept == [0, 2]
    assert np.abs(np.concatenate([Q, Qn], 1).T @ np.concatenate([Q, Qn], 1) - np.eye(5)).max() < 1e-14
    # a genuine direction far below the block's norm is kept
    tiny = np.concatenate([Q[:, :1] + 1e-11 * b[:, :1]], axis=1)
    Qn, kept = orth_append(Q, tiny, 50)
    assert kept == [0]
