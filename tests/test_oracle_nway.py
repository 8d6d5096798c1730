"""Pins of the N-way FP64 oracle (Sec. 3: nonnegative tensor factorization of
N modes; the sweep of Alg. 1 with the N - 1 other factors)."""
import json
import math
import os

import numpy as np
import pytest

from paper_2003_03572_amd import gen

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _tiny(seed, dims, nnz):
    rng = np.random.default_rng(seed)
    total = int(np.prod(dims))
    lin = rng.choice(total, size=nnz, replace=False)
    idx = np.stack(np.unravel_index(lin, dims), axis=1).astype(np.int32)
    vals = rng.integers(1, 6, size=nnz).astype(np.float32)
    return dims, idx, vals


def _dense(dims, idx, vals):
    X = np.zeros(dims, np.float64)
    np.add.at(X, tuple(idx[:, k] for k in range(len(dims))), vals.astype(np.float64))
    return X


def _unfold(X, mode):
    """Mode-n matricization, Kolda-Bader column order (first remaining mode fastest)."""
    return np.reshape(np.moveaxis(X, mode, 0), (X.shape[mode], -1), order="F")


def _khatri_rao(mats):
    """Column-wise Kronecker product of mats[0] (slowest) ... mats[-1]."""
    out = mats[0]
    for B in mats[1:]:
        out = np.stack([np.kron(out[:, r], B[:, r]) for r in range(out.shape[1])], axis=1)
    return out


def _dense_objective(X, F):
    R = F[0].shape[1]
    Xhat = np.zeros(X.shape)
    for r in range(R):
        comp = F[0][:, r]
        for A in F[1:]:
            comp = np.multiply.outer(comp, A[:, r])
        Xhat += comp
    return float(np.sum((X - Xhat) ** 2))


@pytest.mark.parametrize("N,seed", [(4, 0), (4, 1), (5, 2)])
def test_nway_mttkrp_is_unfolding_times_khatri_rao(oracle_mod, N, seed):
    dims = (3, 4, 2, 5, 3)[:N]
    dims, idx, vals = _tiny(seed, dims, 40)
    T = oracle_mod.NTensor(dims, idx, vals)
    rng = np.random.default_rng(300 + seed)
    R = 3
    A = [rng.random((d, R)) for d in dims]
    X = _dense(dims, idx, vals)
    for n in range(N):
        others = [m for m in range(N) if m != n]
        # Kolda-Bader: the first remaining mode varies fastest, i.e. the last
        # remaining mode is the slowest factor of the Khatri-Rao product
        krp = _khatri_rao([A[m] for m in reversed(others)])
        np.testing.assert_allclose(T.mttkrp(n, A), _unfold(X, n) @ krp, rtol=1e-12, atol=1e-12)


def test_nway_objective_is_dense_and_gauss_seidel_is_monotone(oracle_mod):
    dims, idx, vals = _tiny(5, (4, 3, 5, 2), 50)
    X = _dense(dims, idx, vals)
    T = oracle_mod.NTensor(dims, idx, vals)
    m = oracle_mod.NModel(T, 3, seed=5)
    F = [m.factor(n) for n in range(4)]
    assert math.isclose(m.objective(), _dense_objective(X, F), rel_tol=1e-10)
    f_prev = m.objective()
    for it in range(8):
        for n in range(4):
            m.sweep(n)
            f = m.info(n)["f"]
            assert f <= f_prev * (1 + 1e-12) + 1e-12
            assert m.factor(n).min() >= 0.0
            f_prev = f
    F = [m.factor(n) for n in range(4)]
    assert math.isclose(f_prev, _dense_objective(X, F), rel_tol=1e-9)


def test_three_way_case_equals_the_three_way_oracle(oracle_mod):
    """N = 3: the same sweep as the three-way oracle, bit for bit, with the
    same tie band and the same row outcomes under other decisions."""
    dims, idx, vals = gen.make(gen.SMALL_UNIFORM)
    a = oracle_mod.Model(oracle_mod.Tensor(dims, idx, vals), 8, seed=42)
    T = oracle_mod.NTensor(dims, idx, vals)
    b = oracle_mod.NModel(T, 8, seed=42)
    for n in range(3):
        np.testing.assert_array_equal(a.factor(n), b.factor(n))
    for it in range(3):
        for n in range(3):
            A_before = b.factor(n)
            a.sweep(n)
            b.sweep(n)
            ia, ib = a.info(n), b.info(n)
            np.testing.assert_array_equal(ia["M"], ib["M"])
            np.testing.assert_array_equal(ia["z"], ib["z"])
            np.testing.assert_array_equal(ia["sel"], ib["sel"])
            np.testing.assert_array_equal(a.factor(n), b.factor(n))
            assert ia["f"] == ib["f"] and ia["ti"] == ib["ti"]
            assert ia["inner"] == ib["inner"] and ia["model"] == ib["model"]
            np.testing.assert_array_equal(ia["band"], ib["band"])
            np.testing.assert_array_equal(ia["kind"], ib["kind"])
            assert ia["tie_global"] == ib["tie_global"] and ia["band_ti"] == ib["band_ti"]
            # row outcomes: the own decisions give the swept row, none the old
            # row, and flipped decisions agree between the two oracles
            rng = np.random.default_rng(100 * it + n)
            for q in rng.choice(dims[n], 5, replace=False):
                own = ib["sel"][q].astype(np.uint8)
                np.testing.assert_array_equal(b.row_outcome(n, q, own), b.factor(n)[q])
                np.testing.assert_array_equal(b.row_outcome(n, q, np.zeros(8, np.uint8)), A_before[q])
                alt = (rng.random(8) < 0.5).astype(np.uint8)
                np.testing.assert_array_equal(b.row_outcome(n, q, alt), a.row_outcome(n, q, alt))


def test_hand_worked_sweeps_with_a_fourth_unit_mode(oracle_mod):
    """The hand-worked three sweeps (tests/golden) with a fourth mode of length
    one whose factor is (1, 1): its Gram is all ones, so H and M are unchanged
    (eq. 9-10 for four modes) and every value of the golden holds."""
    with open(os.path.join(GOLDEN, "saturation_three_sweeps.json")) as fh:
        g = json.load(fh)
    su = g["setup"]
    idx = np.array([e[0] + [0] for e in su["entries"]], np.int32)
    vals = np.array([e[1] for e in su["entries"]], np.float32)
    T = oracle_mod.NTensor(tuple(su["dims"]) + (1,), idx, vals)
    m = oracle_mod.NModel(T, su["R"], seed=0)
    m.set_factor(0, np.array(su["U0"]))
    m.set_factor(1, np.array(su["V"]))
    m.set_factor(3, np.ones((1, su["R"])))
    for sw in g["sweeps"]:
        m.set_factor(2, np.array(sw["W"]))
        m.sweep(0)
        info = m.info(0)
        assert info["L"] == sw["L"]
        np.testing.assert_array_equal(info["z"], sw["z"])
        assert info["ti"] == sw["ti"] and info["flip"] == sw["flip"]
        np.testing.assert_array_equal(info["sel"].astype(int), sw["sel"])
        np.testing.assert_array_equal(m.factor(0), sw["U"])
        assert info["f"] == sw["f"]
        assert m.state(0)[2] == sw["k"]


def test_nway_sort_matches_lexsort(oracle_mod):
    dims, idx, vals = _tiny(8, (6, 5, 4, 3), 200)
    T = oracle_mod.NTensor(dims, idx, vals)
    for n in range(4):
        others = [m for m in range(4) if m != n]
        order = np.lexsort(tuple(idx[:, m] for m in reversed(others)) + (idx[:, n],))
        coords, v, ptr = T.mode_coo(n)
        np.testing.assert_array_equal(coords, idx[order][:, [n] + others])
        np.testing.assert_array_equal(v, vals[order])
        np.testing.assert_array_equal(ptr, np.concatenate([[0], np.cumsum(np.bincount(idx[:, n], minlength=dims[n]))]))
