"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeded inputs.  See tests/gpu_helpers.py for the comparison rules."""
import math

import numpy as np
import pytest

from paper_2003_03572_amd import gen
import json
import os

from tests.gpu_helpers import (assert_tie_bounds, compare_sweep, gpu_tensor, load_gpu_factors_into_oracle,
                               load_gpu_state_into_oracle, load_oracle_state_into_gpu, step_parity,
                               summarize, sweep_both, to_np)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

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
            assert_tie_bounds(r, f"iter {it} mode {n}")
            report.append(r)
    return report


def test_step_parity_small_uniform_20_iterations(sacd, oracle_mod):
    rep = _step_parity_run(sacd, oracle_mod, gen.SMALL_UNIFORM, 8, 20)
    print("STEP_PARITY small-uniform-r8", json.dumps(summarize(rep)))


@pytest.mark.parametrize("R", [32, 20])
def test_step_parity_zipf_scaled(sacd, oracle_mod, R):
    rep = _step_parity_run(sacd, oracle_mod, gen.ZIPF_UIT, R, 3, scale=0.01)
    print(f"STEP_PARITY zipf-0.01-r{R}", json.dumps(summarize(rep)))


@pytest.mark.parametrize("R", [64, 128, 100])
def test_step_parity_uniform_scaled(sacd, oracle_mod, R):
    rep = _step_parity_run(sacd, oracle_mod, gen.UNIFORM_20M_R64, R, 2, scale=0.004)
    print(f"STEP_PARITY uniform-0.004-r{R}", json.dumps(summarize(rep)))


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


# ------------------------------------------- the GPU's own carried state --

def test_golden_three_sweeps_on_gpu(sacd):
    """The hand-worked three sweeps of one mode (tests/golden), run on the
    GPU from its own state: z (exported as the next Z^{k-1}), ti, the eq. 27
    branch, the selected set, per-column counts, factor, k and objective, all
    exact (dyadic values, exact in FP32)."""
    with open(os.path.join(GOLDEN, "saturation_three_sweeps.json")) as fh:
        g = json.load(fh)
    import torch
    su = g["setup"]
    idx = np.array([e[0] for e in su["entries"]], np.int32)
    vals = np.array([e[1] for e in su["entries"]], np.float32)
    T_g = gpu_tensor(sacd, tuple(su["dims"]), idx, vals)
    gm = sacd.Model(T_g, su["R"], seed=0)
    gm.set_diagnostics(True)
    gm.set_factor(0, torch.tensor(su["U0"], dtype=torch.float32))
    gm.set_factor(1, torch.tensor(su["V"], dtype=torch.float32))
    for sw in g["sweeps"]:
        gm.set_factor(2, torch.tensor(sw["W"], dtype=torch.float32))
        gm.sweep(0)
        st = gm.stats(0)
        zp, ti_prev, k = gm.state(0)
        assert k == sw["k"] and st["k"] == sw["k"]
        assert st["L"] == sw["L"]
        np.testing.assert_array_equal(to_np(zp).astype(np.float64), sw["z"])
        assert st["ti"] == sw["ti"] and ti_prev == sw["ti"]
        assert st["flip"] == sw["flip"]
        sel = to_np(gm.diagnostics(0)[1]).astype(int)
        np.testing.assert_array_equal(sel, sw["sel"])
        np.testing.assert_array_equal(gm.column_counts(0), np.sum(sw["sel"], axis=0))
        np.testing.assert_array_equal(to_np(gm.factor(0)).astype(np.float64), sw["U"])
        assert st["f"] == sw["f"]


def _chained_run(sacd, oracle_mod, w, R, n_iter, scale=1.0, seed=42):
    """The GPU runs from its own state, never written by the test; before
    each sweep the oracle takes the GPU's factors only, and keeps its own
    Z^{k-1}, ti^{k-1} and k.  So the GPU's carried selection state (Alg. 1,
    eq. 24-27) is checked against the oracle's every sweep."""
    dims, idx, vals = gen.make(w, scale=scale)
    T_g = gpu_tensor(sacd, dims, idx, vals)
    T_o = oracle_mod.Tensor(dims, idx, vals)
    gm = sacd.Model(T_g, R, seed=seed)
    gm.set_diagnostics(True)
    om = oracle_mod.Model(T_o, R, seed=seed)
    rep = []
    for it in range(n_iter):
        for n in range(3):
            load_gpu_factors_into_oracle(gm, om)
            before = sweep_both(gm, om, n)
            r = compare_sweep(gm, om, n, before, where=f"chained iter {it} mode {n}")
            assert_tie_bounds(r, f"chained iter {it} mode {n}")
            rep.append(r)
    return rep


def test_chained_gpu_state_small_uniform(sacd, oracle_mod):
    rep = _chained_run(sacd, oracle_mod, gen.SMALL_UNIFORM, 8, 12)
    print("CHAINED small-uniform-r8", json.dumps(summarize(rep)))


@pytest.mark.parametrize("R", [32, 64])
def test_chained_gpu_state_zipf_scaled(sacd, oracle_mod, R):
    rep = _chained_run(sacd, oracle_mod, gen.ZIPF_UIT, R, 4, scale=0.01)
    print(f"CHAINED zipf-0.01-r{R}", json.dumps(summarize(rep)))


def test_chained_gpu_state_uniform_r128_scaled(sacd, oracle_mod):
    rep = _chained_run(sacd, oracle_mod, gen.UNIFORM_20M_R128, 128, 4, scale=0.002)
    print("CHAINED uniform-0.002-r128", json.dumps(summarize(rep)))


# ------------------------------------------------------------ trajectory --

# Tie events allowed in a 20-iteration trajectory (60 sweeps).  An event is
# a sweep where the two independent runs decided some element differently;
# with at most a handful of tie elements per sweep (see the step-parity
# figures) only a few sweeps should meet one.
MAX_TRAJECTORY_EVENTS = 15


def test_trajectory_small_uniform_20_iterations(sacd, oracle_mod):
    """Independent runs from the same seed.  After every sweep the objective
    agrees to 1e-5; a sweep where the runs decided an element differently
    (both decisions valid inside the tie band, or the factors drifted by
    rounding) is a tie event: the oracle is resynchronised from the GPU's
    factors and state, and the events are counted and bounded."""
    w = gen.SMALL_UNIFORM
    dims, idx, vals = gen.make(w)
    T_g = gpu_tensor(sacd, dims, idx, vals)
    T_o = oracle_mod.Tensor(dims, idx, vals)
    gm = sacd.Model(T_g, w.rank, seed=w.init_seed)
    gm.set_diagnostics(True)
    om = oracle_mod.Model(T_o, w.rank, seed=w.init_seed)
    events, checked, worst = [], 0, 0.0
    for it in range(w.iters):
        for n in range(3):
            sweep_both(gm, om, n)
            info, st = om.info(n), gm.stats(n)
            sel_g = to_np(gm.diagnostics(n)[1]).astype(bool)
            rel = abs(st["f"] - info["f"]) / abs(info["f"])
            if (sel_g != info["sel"]).any() or st["flip"] != info["flip"]:
                events.append((it, n, int((sel_g != info["sel"]).sum())))
                load_gpu_state_into_oracle(gm, om)
                continue
            assert rel <= 1e-5, (it, n, st["f"], info["f"])
            worst = max(worst, rel)
            checked += 1
    print(f"TRAJECTORY small-uniform-r8: {checked} sweeps checked (worst f rel {worst:.2e}), "
          f"tie events {len(events)}: {events}")
    assert len(events) <= MAX_TRAJECTORY_EVENTS, events
    assert checked >= 3 * w.iters - MAX_TRAJECTORY_EVENTS


def test_run_until_matches_oracle(sacd, oracle_mod):
    """run_until against the oracle's stopping rule from the same initial
    state (tol 1e-4 after iteration 2, Alg. 1 outer loop).  The GPU's
    run_until is compared with the same iterations stepped one at a time on
    a second GPU model (bit-identical) beside the oracle, resynchronised at
    tie events as in the trajectory test; without tie events that is
    ora_run_until itself, which the test then also calls."""
    w = gen.SMALL_UNIFORM
    tol, max_iter = 1e-4, 150
    dims, idx, vals = gen.make(w)
    T_g = gpu_tensor(sacd, dims, idx, vals)
    T_o = oracle_mod.Tensor(dims, idx, vals)
    a = sacd.Model(T_g, w.rank, seed=w.init_seed)
    it_g, fit_g = a.run_until(tol, max_iter)
    b = sacd.Model(T_g, w.rank, seed=w.init_seed)
    b.set_diagnostics(True)
    om = oracle_mod.Model(T_o, w.rank, seed=w.init_seed)
    nx = math.sqrt(om.t.norm2)
    events, fits_b, fits_o = [], [], []
    it_o = None
    for it in range(1, max_iter + 1):
        for n in range(3):
            sweep_both(b, om, n)
            info = om.info(n)
            sel_b = to_np(b.diagnostics(n)[1]).astype(bool)
            if (sel_b != info["sel"]).any() or b.stats(n)["flip"] != info["flip"]:
                events.append((it, n))
                load_gpu_state_into_oracle(b, om)
        fits_b.append(b.fit()[0])
        fits_o.append(1.0 - math.sqrt(max(om.info(2)["f"], 0.0)) / nx)
        if it >= 2 and abs(fits_o[-1] - fits_o[-2]) < tol * abs(fits_o[-2]):
            it_o = it
            break
    it_o = it_o or max_iter
    print(f"RUN_UNTIL gpu {it_g} iterations fit {fit_g:.10f}; oracle rule {it_o} iterations fit "
          f"{fits_o[-1]:.10f}; tie events {events}")
    assert it_g == it_o, (it_g, it_o, events)
    assert fits_b[it_g - 1] == fit_g  # run_until is the same iterations
    assert abs(fit_g - fits_o[-1]) <= 1e-5 * abs(fits_o[-1])
    if not events:
        om2 = oracle_mod.Model(T_o, w.rank, seed=w.init_seed)
        it2, fit2, _ = om2.run_until(tol, max_iter)
        assert it2 == it_g and abs(fit2 - fit_g) <= 1e-5 * abs(fit2)


def test_run_until_record_per_sweep(sacd, oracle_mod, tmp_path):
    """run_until with a per-sweep JSONL record runs the same iterations as
    without (bit for bit) and writes one line per sweep: k counts each mode's
    sweeps, f is that sweep's objective (eq. 6; the FP64 oracle's own run of
    the first sweeps within the parity bound), fit the matching fit, and the
    last line's fit is the one returned."""
    w = gen.SMALL_UNIFORM
    dims, idx, vals = gen.make(w)
    T_g = gpu_tensor(sacd, dims, idx, vals)
    a = sacd.Model(T_g, w.rank, seed=w.init_seed)
    it_a, fit_a = a.run_until(1e-4, 40)
    b = sacd.Model(T_g, w.rank, seed=w.init_seed)
    path = tmp_path / "sweeps.jsonl"
    it_b, fit_b = b.run_until(1e-4, 40, record=str(path))
    assert (it_b, fit_b) == (it_a, fit_a)
    for n in range(3):
        np.testing.assert_array_equal(to_np(a.factor(n)).view(np.uint32), to_np(b.factor(n)).view(np.uint32))
    rows = [json.loads(line) for line in path.read_text().splitlines()]
    assert len(rows) == 3 * it_b
    nx = math.sqrt(T_g.norm2)
    for q, r in enumerate(rows):
        assert (r["iter"], r["mode"], r["k"]) == (q // 3 + 1, q % 3, q // 3 + 1)
        assert r["fit"] == 1.0 - math.sqrt(max(r["f"], 0.0)) / nx
        assert isinstance(r["flip"], bool) and 0 <= r["nsel"] <= dims[r["mode"]] * w.rank and r["L"] > 0
        if q:
            assert r["f"] <= rows[q - 1]["f"] * (1 + 1e-6)  # Gauss-Seidel sweeps do not raise f
    assert rows[-1]["fit"] == fit_b
    # the first iteration's objectives against the oracle from the same start
    om = oracle_mod.Model(oracle_mod.Tensor(dims, idx, vals), w.rank, seed=w.init_seed)
    S_norm = float(np.sum(vals.astype(np.float64) ** 2))
    for n in range(3):
        om.sweep(n)
        f_o = om.info(n)["f"]
        assert abs(rows[n]["f"] - f_o) <= 1e-5 * abs(f_o) + 1e-6 * S_norm, (n, rows[n]["f"], f_o)


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
    ms, sw = b.iterate_timed(3, sweeps=True)
    assert len(ms) == 3 and all(len(r) == 3 and all(0.0 < v < 1e3 for v in r) for r in ms)
    assert all(sw[i][n] >= ms[i][n] for i in range(3) for n in range(3))
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
    mode on both sides from the GPU's state, compared element by element."""
    w = gen.ZIPF_UIT
    dims, idx, vals = gen.make(w)
    T_g = gpu_tensor(sacd, dims, idx, vals)
    gm = sacd.Model(T_g, w.rank, seed=w.init_seed)
    gm.iterate(2)
    T_o = oracle_mod.Tensor(dims, idx, vals)
    om = oracle_mod.Model(T_o, w.rank, seed=w.init_seed)
    gm.set_diagnostics(True)
    for n in range(3):
        load_gpu_state_into_oracle(gm, om)
        r = step_parity(gm, om, n, where=f"full size mode {n}")
        print(f"FULL_SIZE zipf-r32 mode {n}", json.dumps(r), flush=True)
        assert_tie_bounds(r, f"full size zipf mode {n}")


@pytest.mark.slow
def test_step_parity_full_size_uniform_r128(sacd, oracle_mod):
    """The 2e7-entry uniform tensor at R = 128, full size: after one
    iteration (graph replay), one sweep of every mode on both sides from the
    GPU's state."""
    w = gen.UNIFORM_20M_R128
    dims, idx, vals = gen.make(w)
    T_g = gpu_tensor(sacd, dims, idx, vals)
    gm = sacd.Model(T_g, w.rank, seed=w.init_seed)
    gm.iterate(1)
    T_o = oracle_mod.Tensor(dims, idx, vals)
    om = oracle_mod.Model(T_o, w.rank, seed=w.init_seed)
    gm.set_diagnostics(True)
    for n in range(3):
        load_gpu_state_into_oracle(gm, om)
        r = step_parity(gm, om, n, where=f"full size R=128 mode {n}")
        print(f"FULL_SIZE uniform-r128 mode {n}", json.dumps(r), flush=True)
        assert_tie_bounds(r, f"full size uniform mode {n}")


@pytest.mark.parametrize("R", [48, 100])
def test_tiled_mttkrp_step_parity(sacd, oracle_mod, R):
    """Mode 2 of this tensor runs the MTTKRP in the tiled form (its A_1 of
    3000 rows is staged in LDS 512 rows at a time, over a copy of the entries
    ordered by row tile); modes 0 and 1 stage all of A_2 (200 rows).  Step
    parity of every mode against the oracle, two iterations, from the GPU's
    own carried state."""
    dims, idx, vals = gen.uniform_coords((3000, 3000, 200), 1_100_000, 4242, "int1to5")
    T_g = gpu_tensor(sacd, dims, idx, vals)
    T_o = oracle_mod.Tensor(dims, idx, vals)
    gm = sacd.Model(T_g, R, seed=3)
    gm.set_diagnostics(True)
    om = oracle_mod.Model(T_o, R, seed=3)
    rep = []
    for it in range(2):
        for n in range(3):
            load_gpu_factors_into_oracle(gm, om)
            before = sweep_both(gm, om, n)
            r = compare_sweep(gm, om, n, before, where=f"tiled R={R} iter {it} mode {n}")
            assert_tie_bounds(r, f"tiled R={R} iter {it} mode {n}")
            rep.append(r)
    print(f"TILED R={R}", json.dumps(summarize(rep)))
