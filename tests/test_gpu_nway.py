"""N-way tensors (Sec. 3 defines the factorization for any number of modes:
the sweep with the Khatri-Rao product of the N - 1 other factors in the
MTTKRP, eq. 9, and the Hadamard product of their Grams as H, eq. 10) on the
GPU against the N-way FP64 oracle, with the comparison rules of the
three-way tests (tests/gpu_helpers.py)."""
import json

import numpy as np
import pytest

from paper_2003_03572_amd import gen
from tests.gpu_helpers import (RTOL_F, assert_tie_bounds, compare_sweep, load_gpu_factors_into_oracle,
                               load_gpu_state_into_oracle, load_oracle_state_into_gpu, step_parity, summarize,
                               sweep_both, to_np)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sacd():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2003_03572_amd import sacd as S
    S.lib()
    return S


def _with_duplicates(dims, idx, vals, seed, frac=0.05):
    """Append repeated coordinates (with their own values) at random places."""
    rng = np.random.default_rng(seed)
    k = max(1, int(frac * idx.shape[0]))
    pick = rng.choice(idx.shape[0], k)
    idx2 = np.concatenate([idx, idx[pick]])
    vals2 = np.concatenate([vals, rng.integers(1, 6, size=k).astype(np.float32)])
    perm = rng.permutation(idx2.shape[0])
    return dims, idx2[perm], vals2[perm]


# Small N-way cases: several tiles per mode, a ragged tail, a unit mode, and
# Zipf modes whose head slices exceed one MTTKRP segment (256 entries).
CASES = {
    "n4-uniform": lambda: gen.nway_coords((60, 50, 40, 30), 20_000, 501),
    "n4-zipf-unit": lambda: gen.nway_coords((300, 1, 120, 45), 12_000, 502, (1.2, None, 1.1, None)),
    "n5-zipf": lambda: gen.nway_coords((40, 33, 25, 19, 7), 15_000, 503, (1.2, 1.2, None, None, 0.8)),
    # the degenerate two-mode case (a sparse matrix) and the largest N
    "n2-matrix": lambda: gen.nway_coords((700, 300), 30_000, 504, (1.1, None)),
    "n8": lambda: gen.nway_coords((6, 5, 7, 4, 5, 6, 3, 5), 20_000, 505),
}


@pytest.mark.parametrize("case", list(CASES))
def test_nway_ingest_bitexact(sacd, oracle_mod, case):
    dims, idx, vals = _with_duplicates(*CASES[case](), seed=11)
    N = len(dims)
    T_g = sacd.NTensor.from_numpy(dims, idx, vals)
    T_o = oracle_mod.NTensor(dims, idx, vals)
    assert T_g.nnz == T_o.nnz < idx.shape[0]
    assert abs(T_g.norm2 - T_o.norm2) <= 1e-12 * T_o.norm2
    for n in range(N):
        c_g, v_g, p_g = T_g.mode_coo(n)
        c_o, v_o, p_o = T_o.mode_coo(n)
        np.testing.assert_array_equal(to_np(c_g), c_o, err_msg=f"{case} mode {n} coords")
        np.testing.assert_array_equal(to_np(v_g), v_o, err_msg=f"{case} mode {n} values")
        np.testing.assert_array_equal(to_np(p_g), p_o, err_msg=f"{case} mode {n} slice pointers")
    T_g.close()


def test_nway_ingest_rejects_bad_input(sacd):
    dims = (5, 6, 7, 8)
    idx = np.array([[0, 0, 0, 0], [4, 5, 6, 7]], np.int32)
    vals = np.array([1.0, 2.0], np.float32)
    sacd.NTensor.from_numpy(dims, idx, vals).close()
    bad = idx.copy()
    bad[1, 3] = 8
    with pytest.raises(sacd.SacdError) as e:
        sacd.NTensor.from_numpy(dims, bad, vals)
    assert e.value.status == -2
    with pytest.raises(sacd.SacdError) as e:
        sacd.NTensor.from_numpy(dims, idx, np.array([1.0, np.nan], np.float32))
    assert e.value.status == -6
    with pytest.raises(sacd.SacdError) as e:  # more than 64 key bits
        sacd.NTensor.from_numpy((2 ** 31 - 1,) * 3, np.zeros((1, 3), np.int32), vals[:1])
    assert e.value.status == -1
    with pytest.raises(sacd.SacdError) as e:  # N beyond 8
        sacd.NTensor.from_numpy((2,) * 9, np.zeros((1, 9), np.int32), vals[:1])
    assert e.value.status == -1
    # no entries: a tensor, a model, a sweep that selects nothing
    T = sacd.NTensor.from_numpy(dims, np.zeros((0, 4), np.int32), np.zeros(0, np.float32))
    m = sacd.NModel(T, 4, seed=1)
    m.sweep(0)
    assert m.stats(0)["k"] == 1 and T.nnz == 0


@pytest.mark.parametrize("R", [1, 8, 20, 40, 100])
def test_nway_init_factors_bitexact(sacd, oracle_mod, R):
    dims, idx, vals = CASES["n5-zipf"]()
    gm = sacd.NModel(sacd.NTensor.from_numpy(dims, idx, vals), R, seed=9)
    om = oracle_mod.NModel(oracle_mod.NTensor(dims, idx, vals), R, seed=9)
    for n in range(len(dims)):
        np.testing.assert_array_equal(to_np(gm.factor(n)).astype(np.float64), om.factor(n))
    # the objective of the initial factors from scratch (FP64 sums; the
    # GPU's Grams are reduced from FP32 partial sums)
    f_g, f_o = gm.fit()[1], om.objective()
    assert abs(f_g - f_o) <= RTOL_F * abs(f_o)


@pytest.mark.parametrize("case,R,iters", [
    ("n4-uniform", 8, 6),
    ("n4-zipf-unit", 20, 3),
    ("n5-zipf", 40, 3),
    ("n4-uniform", 100, 2),
    ("n2-matrix", 16, 4),
    ("n8", 12, 2),
])
def test_nway_step_parity(sacd, oracle_mod, case, R, iters):
    """From the same (FP32-rounded) state, one sweep of each mode on both
    sides, compared element by element."""
    dims, idx, vals = CASES[case]()
    N = len(dims)
    gm = sacd.NModel(sacd.NTensor.from_numpy(dims, idx, vals), R, seed=7)
    gm.set_diagnostics(True)
    om = oracle_mod.NModel(oracle_mod.NTensor(dims, idx, vals), R, seed=7)
    rep = []
    for it in range(iters):
        for n in range(N):
            load_oracle_state_into_gpu(gm, om)
            r = step_parity(gm, om, n, where=f"{case} R={R} iter {it}")
            assert_tie_bounds(r, f"{case} R={R} iter {it} mode {n}")
            rep.append(r)
    print(f"NWAY step parity {case} R={R}", json.dumps(summarize(rep)))


@pytest.mark.parametrize("case,R", [("n4-uniform", 8), ("n5-zipf", 20)])
def test_nway_chained_gpu_state(sacd, oracle_mod, case, R):
    """The GPU's own carried selection state, never written by the test; the
    oracle takes the GPU's factors before each sweep and keeps its own
    Z^{k-1}, ti^{k-1} and k."""
    dims, idx, vals = CASES[case]()
    N = len(dims)
    gm = sacd.NModel(sacd.NTensor.from_numpy(dims, idx, vals), R, seed=42)
    gm.set_diagnostics(True)
    om = oracle_mod.NModel(oracle_mod.NTensor(dims, idx, vals), R, seed=42)
    rep = []
    for it in range(5):
        for n in range(N):
            load_gpu_factors_into_oracle(gm, om)
            before = sweep_both(gm, om, n)
            r = compare_sweep(gm, om, n, before, where=f"chained {case} iter {it} mode {n}")
            assert_tie_bounds(r, f"chained {case} iter {it} mode {n}")
            rep.append(r)
    print(f"NWAY chained {case} R={R}", json.dumps(summarize(rep)))


def test_nway_graph_equals_eager_and_objective_nonincreasing(sacd):
    """Graph replay = sweeps enqueued one by one, bit for bit; timed
    iterations advance the model the same way; Gauss-Seidel never raises the
    objective beyond FP32 rounding of its terms; run_until's stopping rule."""
    dims, idx, vals = CASES["n5-zipf"]()
    N = len(dims)
    T = sacd.NTensor.from_numpy(dims, idx, vals)
    a, b, c = (sacd.NModel(T, 16, seed=3) for _ in range(3))
    a.iterate(4)
    for _ in range(4):
        for n in range(N):
            b.sweep(n)
    mt, sw = c.iterate_timed(4)
    assert mt.shape == (4, N) and np.all(sw >= mt) and np.all(mt > 0)
    for n in range(N):
        fa = to_np(a.factor(n))
        np.testing.assert_array_equal(fa, to_np(b.factor(n)))
        np.testing.assert_array_equal(fa, to_np(c.factor(n)))
    assert a.fit() == b.fit() == c.fit()
    prev = None
    for it in range(10):
        for n in range(N):
            a.sweep(n)
            f = a.stats(n)["f"]
            if prev is not None:
                assert f <= prev + 1e-6 * T.norm2, (it, n, f, prev)
            prev = f
    fit = a.fit()[0]
    assert 0.0 < fit < 1.0
    it, fit2 = a.run_until(1e-4, 200)
    assert 1 <= it <= 200 and fit2 >= fit - 1e-6


@pytest.mark.slow
def test_nway_step_parity_full_size(sacd, oracle_mod):
    """The 4-way bench tensor at its full size (1e7 entries, R = 32): after
    two iterations run as the bench runs them (graph replay), one sweep of
    every mode on both sides from the GPU's state."""
    w = gen.ZIPF_UITD
    dims, idx, vals = gen.make(w)
    gm = sacd.NModel(sacd.NTensor.from_numpy(dims, idx, vals), w.rank, seed=w.init_seed)
    gm.iterate(2)
    om = oracle_mod.NModel(oracle_mod.NTensor(dims, idx, vals), w.rank, seed=w.init_seed)
    gm.set_diagnostics(True)
    for n in range(len(dims)):
        load_gpu_state_into_oracle(gm, om)
        r = step_parity(gm, om, n, where=f"full size 4-way mode {n}")
        print(f"FULL_SIZE {w.name} mode {n}", json.dumps(r), flush=True)
        assert_tie_bounds(r, f"full size 4-way mode {n}")
