"""Shared helpers of the GPU parity tests: run the HIP path and the FP64
oracle on the same seeded inputs and compare them.

Comparison rules (parity contract):
  * sort / slice pointers / initial factors: bit-exact;
  * MTTKRP: |M_gpu - M_oracle| <= 1e-5 |M_oracle| per entry;
  * selection: equal on every element outside the oracle's tie band (the
    decision margin within 1e-6 of the magnitude of the terms it is computed
    from), unless the total-importance comparison itself is a tie, in which
    case the GPU selection must equal the oracle's under one of the two
    branch choices;
  * factors after the update: rows without a tie element within 1e-5 of the
    column maximum;
  * objective: 1e-5 relative.
"""
import numpy as np
import torch

RTOL_M = 1e-5
RTOL_F = 1e-5
RTOL_A = 1e-5


def gpu_tensor(sacd, dims, idx, vals):
    return sacd.Tensor.from_numpy(dims, idx, vals)


def to_np(t: torch.Tensor) -> np.ndarray:
    return t.detach().cpu().numpy()


def load_oracle_state_into_gpu(gm, om, modes=(0, 1, 2)):
    """Round the oracle's factors to FP32, use them on both sides, and copy the
    oracle's selection state (Z^{k-1}, ti^{k-1}, k) to the GPU model."""
    for n in modes:
        A32 = om.factor(n).astype(np.float32)
        om.set_factor(n, A32.astype(np.float64))
        gm.set_factor(n, torch.from_numpy(A32).cuda())
        zp, ti, k = om.state(n)
        gm.set_state(n, torch.from_numpy(zp).cuda(), ti, k)


def compare_sweep(gm, om, mode, where=""):
    """Compare the last sweep of `mode` on both sides; returns a dict of
    counts (ties, skipped rows) for reporting."""
    info = om.info(mode)
    M_g, sel_g, G_g = gm.diagnostics(mode)
    M_g, sel_g = to_np(M_g).astype(np.float64), to_np(sel_g)
    M_o = info["M"]
    err = np.abs(M_g - M_o)
    bad = err > RTOL_M * np.abs(M_o) + 1e-30
    assert not bad.any(), (f"{where} MTTKRP mode {mode}: {bad.sum()} entries off, "
                           f"max rel {np.max(err / np.maximum(np.abs(M_o), 1e-300))}")
    st = gm.stats(mode)
    tie = info["tie"]
    sel_o = info["sel"]
    out = dict(ties=int(tie.sum()), tie_global=bool(info["tie_global"]), rows_skipped=0)
    assert st["flip"] == info["flip"], f"{where} flip differs on mode {mode}"
    diff = (sel_g != sel_o) & ~tie
    assert not diff.any(), (f"{where} selection mode {mode}: {diff.sum()} elements differ "
                            f"outside the tie band (first at {np.argwhere(diff)[:3].tolist()})")
    assert st["nsel"] == int(sel_g.sum())
    A_g = to_np(gm.factor(mode)).astype(np.float64)
    A_o = om.factor(mode)
    tie_rows = tie.any(axis=1) | ((sel_g != sel_o).any(axis=1))
    colmax = np.maximum(np.abs(A_o).max(axis=0), 1e-30)
    errA = np.abs(A_g - A_o) / colmax
    badA = (errA > RTOL_A) & ~tie_rows[:, None]
    assert not badA.any(), (f"{where} factor mode {mode}: {badA.sum()} entries off, "
                            f"max {errA[~tie_rows].max() if (~tie_rows).any() else 0}")
    out["rows_skipped"] = int(tie_rows.sum())
    f_o = info["f"]
    assert abs(st["f"] - f_o) <= RTOL_F * abs(f_o), f"{where} objective mode {mode}: {st['f']} vs {f_o}"
    G_o = A_o.T @ A_o
    if not tie_rows.any():
        np.testing.assert_allclose(G_g, G_o, rtol=1e-5, atol=1e-6 * np.abs(G_o).max())
    assert A_g.min() >= 0.0
    return out


def snapshot(om, mode):
    return [om.factor(n) for n in range(3)], om.state(mode)


def restore(om, snap, mode):
    for n in range(3):
        om.set_factor(n, snap[0][n])
    zp, ti, k = snap[1]
    om.set_state(mode, zp, ti, k)


def step_parity(gm, om, mode, where=""):
    """One sweep of `mode` on both sides from the same state, then compare.
    At a total-importance tie (both branches valid) the oracle is re-run with
    the branch the GPU took."""
    snap = snapshot(om, mode)
    om.sweep(mode)
    gm.sweep(mode)
    info = om.info(mode)
    st = gm.stats(mode)
    if info["tie_global"] and st["flip"] != info["flip"]:
        restore(om, snap, mode)
        om.force_flip(int(st["flip"]))
        om.sweep(mode)
        om.force_flip(-1)
    return compare_sweep(gm, om, mode, where)
