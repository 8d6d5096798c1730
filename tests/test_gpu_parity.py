"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeded inputs.  See tests/gpu_helpers.py for the comparison rules."""
import math

import numpy as np
import pytest

from paper_2003_03572_amd import gen
from tests.gpu_helpers import gpu_tensor, load_oracle_state_into_gpu, step_parity, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sacd():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2003_03572_amd import sacd as S
    S.lib()  # fails loudly when the HIP library is missing
    return S


def _coo_bitexact(T_g, T_o, dims):
    for n in range(3):
        c_g, v_g, p_g = T_g.mode_coo(n)
        c_o, v_o, p_o = T_o.mode_coo(n)
        np.testing.assert_array_equal(to_np(c_g), c_o)
        np.testing.assert_array_equal(to_np(v_g).view(np.uint32), v_o.view(np.uint32))
        np.testing.assert_array_equal(to_np(p_g), p_o)


# ----------------------------------------------------------------- ingest --

def test_ingest_small_uniform_bitexact(sacd, oracle_mod):
    dims, idx, vals = gen.make(gen.SMALL_UNIFORM)
    T_g = gpu_tensor(sacd, dims, idx, vals)
    T_o = oracle_mod.Tensor(dims, idx, vals)
    assert T_g.nnz == T_o.nnz == 20_000
    assert math.isclose(T_g.norm2, T_o.norm2, rel_tol=1e-12)
    _coo_bitexact(T_g, T_o, dims)


def test_ingest_duplicates_zipf_bitexact(sacd, oracle_mod):
    # duplicates on purpose: Zipf draws without deduplication, non-integer values
    rng = np.random.default_rng(5)
    dims = (300, 200, 40)
    n = 60_000
    idx = np.stack([gen.zipf_indices(rng, n, d, 1.1) for d in dims], axis=1)
    vals = rng.standard_normal(n).astype(np.float32)
    T_g = gpu_tensor(sacd, dims, idx, vals)
    T_o = oracle_mod.Tensor(dims, idx, vals)
    assert T_g.nnz == T_o.nnz < n
    _coo_bitexact(T_g, T_o, dims)


def test_ingest_multi_tile_zipf_bitexact(sacd, oracle_mod):
    dims, idx, vals = gen.make(gen.ZIPF_UIT, scale=0.02)  # 200k entries, several sort tiles
    T_g = gpu_tensor(sacd, dims, idx, vals)
    T_o = oracle_mod.Tensor(dims, idx, vals)
    _coo_bitexact(T_g, T_o, dims)


def test_ingest_rejects_bad_input(sacd):
    dims = (4, 5, 6)
    idx = np.array([[0, 0, 0], [3, 5, 1]], np.int32)  # 5 is out of range for mode 1
    vals = np.ones(2, np.float32)
    with pytest.raises(sacd.SacdError) as e:
        gpu_tensor(sacd, dims, idx, vals)
    assert e.value.status == -2
    idx = np.array([[0, 0, 0], [3, 4, 1]], np.int32)
    vals = np.array([1.0, np.inf], np.float32)
    with pytest.raises(sacd.SacdError) as e:
        gpu_tensor(sacd, dims, idx, vals)
    assert e.value.status == -6


# ------------------------------------------------------------------- init --

@pytest.mark.parametrize("R", [8, 20])
def test_init_factors_bitexact(sacd, oracle_mod, R):
    dims, idx, vals = gen.make(gen.SMALL_UNIFORM)
    T_g = gpu_tensor(sacd, dims, idx, vals)
    T_o = oracle_mod.Tensor(dims, idx, vals)
    gm = sacd.Model(T_g, R, seed=42)
    om = oracle_mod.Model(T_o, R, seed=42)
    for n in range(3):
        np.testing.assert_array_equal(to_np(gm.factor(n)).astype(np.float64), om.factor(n))
    fit_g, f_g = gm.fit()
    fit_o, f_o = om.fit()
    assert math.isclose(f_g, f_o, rel_tol=1e-5)


# ------------------------------------------------------------ step parity --

def _step_parity_run(sacd, oracle_mod, w, R, n_iter, scale=1.0, seed=42):
    dims, idx, vals = gen.make(w, scale=scale)
    T_g = gpu_tensor(sacd, dims, idx, vals)
    T_o = oracle_mod.Tensor(dims, idx, vals)
    gm = sacd.Model(T_g, R, seed=seed)
    gm.set_diagnostics(True)
    om = oracle_mod.Model(T_o, R, seed=seed)
    report = []
    for it in range(n_iter):
        for n in range(3):
            load_oracle_state_into_gpu(gm, om)
            r = step_parity(gm, om, n, where=f"iter {it}")
            report.append(r)
    return report


def test_step_parity_small_uniform_20_iterations(sacd, oracle_mod):
    rep = _step_parity_run(sacd, oracle_mod, gen.SMALL_UNIFORM, 8, 20)
    ties = sum(r["ties"] for r in rep)
    other = sum(r["tie_rows_other_outcome"] for r in rep)
    print(f"ties {ties}, tie rows with the other valid outcome {other} over {len(rep)} sweeps")


@pytest.mark.parametrize("R", [32, 20])
def test_step_parity_zipf_scaled(sacd, oracle_mod, R):
    rep = _step_parity_run(sacd, oracle_mod, gen.ZIPF_UIT, R, 3, scale=0.01)
    print([(r["ties"], r["tie_rows_other_outcome"]) for r in rep])


@pytest.mark.parametrize("R", [64, 128, 100])
def test_step_parity_uniform_scaled(sacd, oracle_mod, R):
    rep = _step_parity_run(sacd, oracle_mod, gen.UNIFORM_20M_R64, R, 2, scale=0.004)
    print([(r["ties"], r["tie_rows_other_outcome"]) for r in rep])


def test_jacobi_flag_step_parity(sacd, oracle_mod):
    dims, idx, vals = gen.make(gen.SMALL_UNIFORM)
    T_g = gpu_tensor(sacd, dims, idx, vals)
    T_o = oracle_mod.Tensor(dims, idx, vals)
    gm = sacd.Model(T_g, 8, seed=42, update=sacd.UPDATE_JACOBI)
    gm.set_diagnostics(True)
    om = oracle_mod.Model(T_o, 8, seed=42, update=oracle_mod.UPDATE_JACOBI)
    for it in range(5):
        for n in range(3):
            load_oracle_state_into_gpu(gm, om)
            step_parity(gm, om, n, where=f"jacobi iter {it}")


# ------------------------------------------------------------ trajectory --

def test_trajectory_small_uniform_20_iterations(sacd, oracle_mod):
    """Independent runs from the same seed: the objective after every
    iteration agrees to 1e-5 until the oracle meets a tie (reported)."""
    w = gen.SMALL_UNIFORM
    dims, idx, vals = gen.make(w)
    T_g = gpu_tensor(sacd, dims, idx, vals)
    T_o = oracle_mod.Tensor(dims, idx, vals)
    gm = sacd.Model(T_g, w.rank, seed=w.init_seed)
    om = oracle_mod.Model(T_o, w.rank, seed=w.init_seed)
    tie_seen = False
    for it in range(w.iters):
        gm.iterate(1)
        for n in range(3):
            om.sweep(n)
            info = om.info(n)
            tie_seen = tie_seen or info["tie_global"] or bool(info["tie"].any())
        f_g = gm.stats(2)["f"]
        f_o = om.info(2)["f"]
        if not tie_seen:
            assert abs(f_g - f_o) <= 1e-5 * abs(f_o), (it, f_g, f_o)
        else:
            print(f"iteration {it}: tie met, f gpu {f_g} oracle {f_o}")


def test_objective_nonincreasing_and_nonnegative(sacd):
    dims, idx, vals = gen.make(gen.ZIPF_UIT, scale=0.01)
    T_g = gpu_tensor(sacd, dims, idx, vals)
    gm = sacd.Model(T_g, 32, seed=7)
    _, f_prev = gm.fit()
    for it in range(6):
        for n in range(3):
            gm.sweep(n)
            f = gm.stats(n)["f"]
            assert f <= f_prev * (1 + 1e-6), (it, n, f, f_prev)
            f_prev = f
    for n in range(3):
        assert float(gm.factor(n).min()) >= 0.0


def test_deterministic_bitwise(sacd):
    dims, idx, vals = gen.make(gen.ZIPF_UIT, scale=0.01)
    outs = []
    for _ in range(2):
        T_g = gpu_tensor(sacd, dims, idx, vals)
        gm = sacd.Model(T_g, 32, seed=3)
        gm.iterate(5)
        outs.append([to_np(gm.factor(n)) for n in range(3)] + [gm.fit()[1]])
    for n in range(3):
        np.testing.assert_array_equal(outs[0][n].view(np.uint32), outs[1][n].view(np.uint32))
    assert outs[0][3] == outs[1][3]


def test_graph_iterate_equals_eager_sweeps(sacd):
    dims, idx, vals = gen.make(gen.SMALL_UNIFORM)
    T_g = gpu_tensor(sacd, dims, idx, vals)
    a = sacd.Model(T_g, 8, seed=42)
    b = sacd.Model(T_g, 8, seed=42)
    for it in range(4):
        a.iterate(1)
        for n in range(3):
            b.sweep(n)
        for n in range(3):
            np.testing.assert_array_equal(to_np(a.factor(n)).view(np.uint32),
                                          to_np(b.factor(n)).view(np.uint32))


def test_timed_iterations_equal_iterate(sacd):
    """Timed iterations (launch by launch, events around MTTKRP) do the same
    work as iterate(): bit-identical factors, positive kernel times."""
    dims, idx, vals = gen.make(gen.SMALL_UNIFORM)
    T_g = gpu_tensor(sacd, dims, idx, vals)
    a = sacd.Model(T_g, 8, seed=42)
    b = sacd.Model(T_g, 8, seed=42)
    b.timing_prepare(3)
    with pytest.raises(sacd.SacdError):
        b.iterate_timed(4)
    a.iterate(3)
    ms = b.iterate_timed(3)
    assert len(ms) == 3 and all(len(r) == 3 and all(0.0 < v < 1e3 for v in r) for r in ms)
    for n in range(3):
        np.testing.assert_array_equal(to_np(a.factor(n)).view(np.uint32),
                                      to_np(b.factor(n)).view(np.uint32))
    assert a.fit() == b.fit()


def test_run_until_rule(sacd, oracle_mod):
    w = gen.SMALL_UNIFORM
    dims, idx, vals = gen.make(w)
    T_g = gpu_tensor(sacd, dims, idx, vals)
    gm = sacd.Model(T_g, 8, seed=42)
    it, fit = gm.run_until(1e-3, 200)
    assert 2 <= it < 200
    fit2, _ = gm.fit()
    assert fit == fit2


def test_checkpoint_resume_bitwise(sacd):
    dims, idx, vals = gen.make(gen.SMALL_UNIFORM)
    T_g = gpu_tensor(sacd, dims, idx, vals)
    a = sacd.Model(T_g, 8, seed=42)
    a.iterate(10)
    saved = [(a.factor(n).clone(), a.state(n)) for n in range(3)]
    a.iterate(10)
    b = sacd.Model(T_g, 8, seed=1)
    for n in range(3):
        A, (zp, ti, k) = saved[n]
        b.set_factor(n, A)
        b.set_state(n, zp, ti, k)
    b.iterate(10)
    for n in range(3):
        np.testing.assert_array_equal(to_np(a.factor(n)).view(np.uint32),
                                      to_np(b.factor(n)).view(np.uint32))


# -------------------------------------------------------------- edge cases --

def test_empty_tensor_and_single_entry(sacd, oracle_mod):
    dims = (5, 4, 3)
    T_g = gpu_tensor(sacd, dims, np.zeros((0, 3), np.int32), np.zeros(0, np.float32))
    gm = sacd.Model(T_g, 4, seed=1)
    gm.iterate(2)
    with pytest.raises(sacd.SacdError):
        gm.fit()  # ||X|| = 0
    for n in range(3):
        assert float(gm.factor(n).min()) >= 0.0
    idx = np.array([[4, 3, 2]], np.int32)
    vals = np.array([2.5], np.float32)
    T_g = gpu_tensor(sacd, dims, idx, vals)
    T_o = oracle_mod.Tensor(dims, idx, vals)
    gm = sacd.Model(T_g, 3, seed=9)
    gm.set_diagnostics(True)
    om = oracle_mod.Model(T_o, 3, seed=9)
    for it in range(3):
        for n in range(3):
            load_oracle_state_into_gpu(gm, om)
            step_parity(gm, om, n, where=f"single {it}")


def test_unit_mode_lengths(sacd, oracle_mod):
    dims = (1, 7, 1)
    idx = np.array([[0, i, 0] for i in range(7)], np.int32)
    vals = np.arange(1, 8, dtype=np.float32)
    T_g = gpu_tensor(sacd, dims, idx, vals)
    T_o = oracle_mod.Tensor(dims, idx, vals)
    _coo_bitexact(T_g, T_o, dims)
    gm = sacd.Model(T_g, 2, seed=4)
    gm.set_diagnostics(True)
    om = oracle_mod.Model(T_o, 2, seed=4)
    for it in range(3):
        for n in range(3):
            load_oracle_state_into_gpu(gm, om)
            step_parity(gm, om, n, where=f"unit {it}")


def test_rank_bounds(sacd):
    dims, idx, vals = gen.make(gen.SMALL_UNIFORM)
    T_g = gpu_tensor(sacd, dims, idx, vals)
    for R in (0, 129):
        with pytest.raises(sacd.SacdError):
            sacd.Model(T_g, R, seed=1)
    gm = sacd.Model(T_g, 1, seed=1)
    gm.iterate(1)


def test_hot_slice_spanning_many_chunks(sacd, oracle_mod):
    """One slice holding most entries (spans many wave chunks) next to empty
    slices: MTTKRP against the oracle."""
    rng = np.random.default_rng(11)
    dims = (50, 400, 300)
    n = 100_000
    i0 = np.where(rng.random(n) < 0.9, 7, rng.integers(0, 50, n))
    i0 = np.where(i0 % 5 == 1, 7, i0)  # rows 1, 6, 11, ... empty
    idx = np.stack([i0, rng.integers(0, 400, n), rng.integers(0, 300, n)], axis=1).astype(np.int32)
    vals = rng.integers(1, 6, n).astype(np.float32)
    T_g = gpu_tensor(sacd, dims, idx, vals)
    T_o = oracle_mod.Tensor(dims, idx, vals)
    for R in (16, 64):
        gm = sacd.Model(T_g, R, seed=2)
        gm.set_diagnostics(True)
        om = oracle_mod.Model(T_o, R, seed=2)
        for n_ in range(3):
            load_oracle_state_into_gpu(gm, om)
            step_parity(gm, om, n_, where=f"hot R={R}")


def test_rank_one_and_jacobi_split_rows(sacd, oracle_mod):
    """R = 1 (one real column, fifteen padded ones) and the Jacobi rule on the
    split-lane row update (R = 64: four lanes per row)."""
    dims, idx, vals = gen.make(gen.SMALL_UNIFORM)
    T_g = gpu_tensor(sacd, dims, idx, vals)
    T_o = oracle_mod.Tensor(dims, idx, vals)
    for R, upd in ((1, sacd.UPDATE_GS), (64, sacd.UPDATE_JACOBI), (128, sacd.UPDATE_JACOBI)):
        gm = sacd.Model(T_g, R, seed=5, update=upd)
        gm.set_diagnostics(True)
        om = oracle_mod.Model(T_o, R, seed=5, update=upd)
        for it in range(3):
            for n in range(3):
                load_oracle_state_into_gpu(gm, om)
                step_parity(gm, om, n, where=f"R={R} upd={upd} iter {it}")


@pytest.mark.slow
def test_step_parity_full_size_zipf(sacd, oracle_mod):
    """The bench tensor at its full size (1e7 entries, R = 32): after two
    iterations run as the bench runs them (graph replay), one sweep of every
    mode on both sides from the same state, compared element by element."""
    w = gen.ZIPF_UIT
    dims, idx, vals = gen.make(w)
    T_g = gpu_tensor(sacd, dims, idx, vals)
    gm = sacd.Model(T_g, w.rank, seed=w.init_seed)
    gm.iterate(2)
    T_o = oracle_mod.Tensor(dims, idx, vals)
    om = oracle_mod.Model(T_o, w.rank, seed=w.init_seed)
    gm.set_diagnostics(True)
    for n in range(3):
        for k_ in range(3):  # the GPU's state, FP32 values, into the oracle
            om.set_factor(k_, to_np(gm.factor(k_)).astype(np.float64))
            zp, ti, k = gm.state(k_)
            om.set_state(k_, to_np(zp), ti, k)
        r = step_parity(gm, om, n, where=f"full size mode {n}")
        print(f"mode {n}: {r}")


@pytest.mark.slow
def test_step_parity_full_size_uniform_r128(sacd, oracle_mod):
    """The 2e7-entry uniform tensor at R = 128, full size: after one
    iteration (graph replay), one sweep of modes 0 and 2 on both sides from
    the GPU's state."""
    w = gen.UNIFORM_20M_R128
    dims, idx, vals = gen.make(w)
    T_g = gpu_tensor(sacd, dims, idx, vals)
    gm = sacd.Model(T_g, w.rank, seed=w.init_seed)
    gm.iterate(1)
    T_o = oracle_mod.Tensor(dims, idx, vals)
    om = oracle_mod.Model(T_o, w.rank, seed=w.init_seed)
    gm.set_diagnostics(True)
    for n in (0, 2):
        for k_ in range(3):
            om.set_factor(k_, to_np(gm.factor(k_)).astype(np.float64))
            zp, ti, k = gm.state(k_)
            om.set_state(k_, to_np(zp), ti, k)
        r = step_parity(gm, om, n, where=f"full size R=128 mode {n}")
        print(f"mode {n}: {r}", flush=True)
