"""Shared helpers of the GPU parity tests: run the HIP path and the FP64
oracle on the same seeded inputs and compare them.

Comparison rules (parity contract):
  * sort / slice pointers / initial factors: bit-exact;
  * MTTKRP: |M_gpu - M_oracle| <= 1e-5 |M_oracle| per entry;
  * selection: equal on every element outside the oracle's tie band (the
    decision margin within 1e-6 of the magnitude of the terms it is computed
    from); a global tie of the total importance is resolved by re-running the
    oracle with the branch the GPU took;
  * factors: rows with no selected element are bit-identical; a row holding
    tie elements must match the oracle's update of that row under the GPU's
    decisions on those elements; otherwise
    |A_gpu - A_oracle| <= 1e-5 * s_q, where s_q is the largest magnitude of
    the terms of the row's Newton steps, (|M_qr| + sum_s |A_qs| H_sr) / H_rr:
    the step is the small difference of FP32 terms of that size;
  * objective: |f_gpu - f_oracle| <= 1e-5 |f_oracle| + 1e-6 S, with
    S = ||X||^2 + 2 |<M, A>| + ||Xhat||^2 the size of the terms f is formed
    from (f itself can cancel to ~0 when the fit is exact).
"""
import numpy as np
import torch

RTOL_M = 1e-5
RTOL_F = 1e-5
RTOL_F_TERMS = 1e-6
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


def snapshot(om, mode):
    return [om.factor(n) for n in range(3)], om.state(mode)


def restore(om, snap, mode):
    for n in range(3):
        om.set_factor(n, snap[0][n])
    zp, ti, k = snap[1]
    om.set_state(mode, zp, ti, k)


def compare_sweep(gm, om, mode, A_old, where=""):
    """Compare the last sweep of `mode` on both sides (A_old: the factor
    before the sweep); returns counts for reporting."""
    info = om.info(mode)
    M_g, sel_g, G_g = gm.diagnostics(mode)
    M_g, sel_g = to_np(M_g).astype(np.float64), to_np(sel_g)
    M_o = info["M"]
    err = np.abs(M_g - M_o)
    bad = err > RTOL_M * np.abs(M_o) + 1e-30
    assert not bad.any(), (f"{where} MTTKRP mode {mode}: {bad.sum()} entries off, "
                           f"max rel {np.max(err / np.maximum(np.abs(M_o), 1e-300))}")
    st = gm.stats(mode)
    assert st["flip"] == info["flip"], f"{where} flip differs on mode {mode}"
    tie, sel_o = info["tie"], info["sel"]
    diff = (sel_g != sel_o) & ~tie
    assert not diff.any(), (f"{where} selection mode {mode}: {diff.sum()} elements differ "
                            f"outside the tie band (first at {np.argwhere(diff)[:3].tolist()})")
    assert st["nsel"] == int(sel_g.sum())

    # the valid outcome that matches the GPU's decisions on tie elements
    A_o = om.factor(mode)
    A_valid = A_o.copy()
    changed_rows = np.nonzero((sel_g != sel_o).any(axis=1))[0]
    for q in changed_rows:
        A_valid[q] = om.row_outcome(mode, int(q), sel_g[q].astype(np.uint8))

    A_g = to_np(gm.factor(mode)).astype(np.float64)
    H = info["H"]
    hd = np.diag(H)
    with np.errstate(divide="ignore", invalid="ignore"):
        terms = (np.abs(M_o) + np.abs(A_old) @ np.abs(H)) / np.where(hd > 0, hd, np.inf)
    s_row = np.max(np.where(np.isfinite(terms), terms, 0.0), axis=1)
    untouched = ~sel_g.any(axis=1)
    np.testing.assert_array_equal(A_g[untouched], A_old[untouched],
                                  err_msg=f"{where} unselected rows changed (mode {mode})")
    errA = np.abs(A_g - A_valid)
    badA = errA > RTOL_A * s_row[:, None] + 1e-30
    assert not badA.any(), (f"{where} factor mode {mode}: {badA.sum()} entries off, "
                            f"worst {np.max(errA / np.maximum(s_row[:, None], 1e-300))}")
    assert A_g.min() >= 0.0

    if len(changed_rows):
        om.set_factor(mode, A_valid)
        f_ref = om.objective()
        om.set_factor(mode, A_o)
    else:
        f_ref = info["f"]
    S = om.t.norm2 + 2 * abs(info["inner"]) + abs(info["model"])
    assert abs(st["f"] - f_ref) <= RTOL_F * abs(f_ref) + RTOL_F_TERMS * S, (
        f"{where} objective mode {mode}: {st['f']} vs {f_ref} (terms {S})")
    G_o = A_valid.T @ A_valid
    np.testing.assert_allclose(G_g, G_o, rtol=1e-5, atol=1e-6 * np.abs(G_o).max() + 1e-30)
    return dict(ties=int(tie.sum()), tie_global=bool(info["tie_global"]),
                tie_rows_other_outcome=int(len(changed_rows)))


def step_parity(gm, om, mode, where=""):
    """One sweep of `mode` on both sides from the same state, then compare.
    At a total-importance tie (both branches valid) the oracle is re-run with
    the branch the GPU took."""
    snap = snapshot(om, mode)
    A_old = snap[0][mode]
    om.sweep(mode)
    gm.sweep(mode)
    info = om.info(mode)
    st = gm.stats(mode)
    if info["tie_global"] and st["flip"] != info["flip"]:
        restore(om, snap, mode)
        om.force_flip(int(st["flip"]))
        om.sweep(mode)
        om.force_flip(-1)
    return compare_sweep(gm, om, mode, A_old, where)
