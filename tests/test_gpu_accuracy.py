"""Accuracy measures of a factorization on the GPU (Sec. 6): held-out RMSE
(eq. 30) and pattern distinctiveness (eq. pd), against the FP64 oracle
evaluated on the same FP32 factors."""
import math

import numpy as np
import pytest

from paper_2003_03572_amd import gen
from tests.gpu_helpers import gpu_tensor, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sacd():
    import torch
    assert torch.cuda.is_available()
    from paper_2003_03572_amd import sacd as S
    return S


@pytest.mark.parametrize("w,R,scale", [(gen.SMALL_UNIFORM, 8, 1.0), (gen.ZIPF_UIT, 32, 0.002),
                                       (gen.UNIFORM_20M_R128, 128, 0.002)],
                         ids=["small_r8", "zipf_r32", "uniform_r128"])
def test_rmse_and_pd_match_oracle(sacd, oracle_mod, w, R, scale):
    dims, idx, vals = gen.make(w, scale)
    tr_i, tr_v, te_i, te_v = gen.split_holdout(idx, vals, 0.2, w.data_seed)
    T_g = gpu_tensor(sacd, dims, tr_i, tr_v)
    gm = sacd.Model(T_g, R, seed=w.init_seed)
    gm.iterate(5)
    T_o = oracle_mod.Tensor(dims, tr_i, tr_v)
    om = oracle_mod.Model(T_o, R, seed=w.init_seed)
    for n in range(3):
        om.set_factor(n, to_np(gm.factor(n)).astype(np.float64))
    r_g, r_o = gm.rmse(te_i, te_v), om.rmse(te_i, te_v)
    assert math.isclose(r_g, r_o, rel_tol=1e-10), (r_g, r_o)
    # the GPU's PD comes from its Gram matrix (FP32 block partials, FP64 sum)
    for n in range(3):
        p_g, p_o = gm.pd(n), om.pd(n)
        assert abs(p_g - p_o) <= 1e-5 * max(abs(p_o), 1e-3), (n, p_g, p_o)
    assert gm.rmse(te_i[:0], te_v[:0]) == 0.0


def test_rmse_rejects_out_of_range(sacd):
    dims, idx, vals = gen.make(gen.SMALL_UNIFORM)
    gm = sacd.Model(gpu_tensor(sacd, dims, idx, vals), 8, seed=42)
    bad = np.array([[dims[0], 0, 0]], np.int32)
    with pytest.raises(sacd.SacdError) as e:
        gm.rmse(bad, np.ones(1, np.float32))
    assert e.value.status == -2
    # the model is still usable afterwards
    assert gm.rmse(idx[:10], vals[:10]) >= 0.0
