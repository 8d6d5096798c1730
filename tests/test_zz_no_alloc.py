"""The allocation-free entry point sacd_rmse_static against sacd_rmse.

sacd_rmse_static runs the same eq. 30 kernel as sacd_rmse with its scratch in
a static device array of the library instead of the model's buffers, and
writes the result to device memory without synchronising.  Two calls in a row
(the second on a smaller input) must give sacd_rmse's values; the scratch
keeps the previous call's contents, so this also checks that the entry point
clears what must start at zero."""
import math

import numpy as np
import pytest

from paper_2003_03572_amd import gen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sacd():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2003_03572_amd import sacd as S
    S.lib()
    return S


def _static(sacd, m, idx, vals):
    import torch
    out = torch.full((2,), -1.0, dtype=torch.float64, device="cuda")
    m.rmse_static(torch.from_numpy(np.ascontiguousarray(idx, np.int32)).cuda(),
                  torch.from_numpy(np.ascontiguousarray(vals, np.float32)).cuda(), out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("w,R,scale", [(gen.SMALL_UNIFORM, 8, 1.0), (gen.ZIPF_UIT, 32, 0.01)],
                         ids=["small_r8", "zipf_r32"])
def test_static_rmse_equals_rmse_two_calls(sacd, w, R, scale):
    import torch
    dims, idx, vals = gen.make(w, scale)
    tr_i, tr_v, te_i, te_v = gen.split_holdout(idx, vals, 0.2, w.data_seed)
    T = sacd.Tensor.from_numpy(dims, tr_i, tr_v)
    m = sacd.Model(T, R, seed=w.init_seed)
    m.iterate(3)
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    for n in (te_i.shape[0], te_i.shape[0] // 3):  # the second call on a smaller input
        want = m.rmse(te_i[:n], te_v[:n])
        got = _static(sacd, m, te_i[:n], te_v[:n])
        assert got[1] == 0.0
        assert got[0] == want or abs(got[0] - want) <= 1e-15 * want, (n, got[0], want)
    # inputs and outputs aside, nothing was allocated through the model's allocator
    del got
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() <= before + 4096


def test_static_rmse_edge_cases(sacd):
    dims, idx, vals = gen.make(gen.SMALL_UNIFORM)
    T = sacd.Tensor.from_numpy(dims, idx, vals)
    m = sacd.Model(T, 8, seed=1)
    # no entries: 0
    got = _static(sacd, m, np.zeros((0, 3), np.int32), np.zeros(0, np.float32))
    assert got[0] == 0.0 and got[1] == 0.0
    # a coordinate outside dims: flagged, NaN; the next call starts clean
    bad = np.array([[0, 0, 0], [dims[0], 0, 0]], np.int32)
    got = _static(sacd, m, bad, np.ones(2, np.float32))
    assert got[1] == 1.0 and math.isnan(got[0])
    got = _static(sacd, m, idx[:100], vals[:100])
    assert got[1] == 0.0 and got[0] == m.rmse(idx[:100], vals[:100])
