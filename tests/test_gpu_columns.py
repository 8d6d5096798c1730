"""The column-at-a-time form (Sec. 4.4, Alg. 2: the MTTKRP a block of columns
at a time; no I_n x R buffer for M) against the FP64 oracle, with the same
comparison rules as the row form (tests/gpu_helpers.py), and the device
memory it saves."""
import json

import numpy as np
import pytest

from paper_2003_03572_amd import gen
from tests.gpu_helpers import (assert_tie_bounds, compare_sweep, gpu_tensor, load_gpu_factors_into_oracle,
                               load_oracle_state_into_gpu, step_parity, sweep_both, to_np)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sacd():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2003_03572_amd import sacd as S
    S.lib()
    return S


@pytest.mark.parametrize("w,R,scale,cb,iters", [
    (gen.SMALL_UNIFORM, 8, 1.0, 1, 4),
    (gen.SMALL_UNIFORM, 8, 1.0, 4, 4),
    (gen.ZIPF_UIT, 32, 0.01, 16, 2),
    (gen.UNIFORM_20M_R128, 100, 0.002, 8, 2),
], ids=["small-cb1", "small-cb4", "zipf-cb16", "uniform-r100-cb8"])
def test_column_form_step_parity(sacd, oracle_mod, w, R, scale, cb, iters):
    dims, idx, vals = gen.make(w, scale=scale)
    T_g = gpu_tensor(sacd, dims, idx, vals)
    T_o = oracle_mod.Tensor(dims, idx, vals)
    gm = sacd.Model(T_g, R, seed=7, columns=cb)
    gm.set_diagnostics(True)
    om = oracle_mod.Model(T_o, R, seed=7)
    rep = []
    for it in range(iters):
        for n in range(3):
            load_oracle_state_into_gpu(gm, om)
            r = step_parity(gm, om, n, where=f"columns {cb} iter {it}")
            assert_tie_bounds(r, f"columns {cb} iter {it} mode {n}")
            rep.append(r)
    print(f"COLUMNS step parity {w.name} R={R} cb={cb}: ties {sum(r['ties'] for r in rep)}, "
          f"other decisions {sum(r['elements_other_decision'] for r in rep)}")


def test_column_form_chained_own_state(sacd, oracle_mod):
    """The column form's own carried state (never written by the test) against
    the oracle's, twelve sweeps."""
    dims, idx, vals = gen.make(gen.SMALL_UNIFORM)
    T_g = gpu_tensor(sacd, dims, idx, vals)
    T_o = oracle_mod.Tensor(dims, idx, vals)
    gm = sacd.Model(T_g, 8, seed=42, columns=2)
    gm.set_diagnostics(True)
    om = oracle_mod.Model(T_o, 8, seed=42)
    for it in range(4):
        for n in range(3):
            load_gpu_factors_into_oracle(gm, om)
            before = sweep_both(gm, om, n)
            compare_sweep(gm, om, n, before, where=f"columns chained iter {it} mode {n}")


def test_column_form_deterministic_and_graph_equal(sacd):
    dims, idx, vals = gen.make(gen.ZIPF_UIT, scale=0.005)
    T_g = gpu_tensor(sacd, dims, idx, vals)
    a = sacd.Model(T_g, 16, seed=3, columns=4)
    b = sacd.Model(T_g, 16, seed=3, columns=4)
    a.iterate(3)  # graph replay
    for it in range(3):
        for n in range(3):
            b.sweep(n)
    for n in range(3):
        np.testing.assert_array_equal(to_np(a.factor(n)).view(np.uint32), to_np(b.factor(n)).view(np.uint32))
    assert a.fit() == b.fit()
    with pytest.raises(sacd.SacdError):
        a.time_kernel(0, 0, 1)
    with pytest.raises(sacd.SacdError):
        sacd.Model(T_g, 16, seed=3, columns=3)


def test_column_form_device_memory(sacd):
    """Bytes held by models of the two forms: the column form holds I_n x cb of
    M and 2 bits per element instead of I_n x R floats and a byte per element
    (three modes).  Reported for the uniform tensor's shape at R = 128 and for
    the jobs of the batched / served forms."""
    out = {}
    dims, idx, vals = gen.make(gen.UNIFORM_20M_R128, scale=0.01)
    T = gpu_tensor(sacd, dims, idx, vals)
    row = sacd.Model(T, 128, seed=1).device_bytes()
    col = sacd.Model(T, 128, seed=1, columns=16).device_bytes()
    full = sum(d * 128 * 5 for d in dims)  # M (4 B) and the selection record (1 B) per element
    assert row - col >= 0.8 * full, (row, col, full)
    out["uniform_r128_scaled"] = {"dims": list(dims), "row_form_bytes": row, "column_form_bytes": col}
    tot_row = tot_col = tot_tensor = 0
    for spec in gen.job_specs(40):
        d, i, v = gen.job_tensor(spec)
        Tj = gpu_tensor(sacd, d, i, v)
        tot_tensor += Tj.info()["device_bytes"]
        tot_row += sacd.Model(Tj, spec.rank, seed=spec.seed).device_bytes()
        tot_col += sacd.Model(Tj, spec.rank, seed=spec.seed, columns=16).device_bytes()
    out["jobs40"] = {"tensor_bytes": tot_tensor, "row_form_model_bytes": tot_row, "column_form_model_bytes": tot_col,
                     "job_bytes_saved_frac": (tot_row - tot_col) / (tot_tensor + tot_row)}
    print("COLUMNS_MEMORY", json.dumps(out))
    assert tot_col < tot_row
