"""The oracle's tie band against FP32 rounding of the gradient's terms.

An implementation in FP32 forms the MTTKRP M and the product A H with a
relative error of a few units of FP32 roundoff u = 2^-24 each (both are sums of
nonnegative terms), then g = -M + A H (eq. 14), the step (eq. 11-12) and z
(eq. 20) in FP32.  These tests re-evaluate z from the oracle's own M and A H
perturbed by up to 4u each and rounded to FP32, and check that

  * every perturbed z stays within the element's band (the band covers FP32
    evaluation of eq. 14, 11-12 and 20);
  * every decision (eq. 24 / 27, Alg. 1) that changes lies in an element the
    oracle marks as a tie;
  * the band is not far wider than the largest perturbation seen: tau = 1e-6
    is about 17u, the perturbation up to 8u of the terms, so the largest
    ratio of the change of z to the band must be well above 1/20.
"""
import numpy as np
import pytest

from paper_2003_03572_amd import gen

U = 2.0 ** -24
f32 = np.float32


def _fp32_importance(A, M, AH, H, L, rng, k_ulps=4.0):
    """z (eq. 20) evaluated in FP32 from M and A H perturbed by up to
    k_ulps * u relative (nonnegative sums: relative to their own size)."""
    eM = rng.uniform(-k_ulps, k_ulps, M.shape) * U
    eA = rng.uniform(-k_ulps, k_ulps, AH.shape) * U
    m = f32(M * (1.0 + eM))
    ah = f32(AH * (1.0 + eA))
    a = f32(A)
    h = f32(np.diag(H))[None, :]
    with np.errstate(divide="ignore", invalid="ignore"):
        g = f32(ah - m)
        q = np.where(h > 0, f32(g / h), f32(0.0))
        d = np.where(h > 0, f32(np.maximum(f32(a - q), f32(0.0)) - a), f32(0.0))
    halfL = f32(0.5 * L)
    return f32(f32(-f32(g * d)) - f32(f32(halfL * d) * d)).astype(np.float64)


def _decide(k, z, zprev, flip):
    if k <= 1:
        return z > 0.0
    return (zprev - z > 0.0) if flip else (z - zprev > 0.0)


@pytest.mark.parametrize("w,R,scale,iters", [
    (gen.SMALL_UNIFORM, 8, 1.0, 4),
    (gen.ZIPF_UIT, 16, 0.003, 3),
    (gen.UNIFORM_20M_R64, 32, 0.001, 2),
])
def test_band_covers_fp32_rounding_and_is_tight(oracle_mod, w, R, scale, iters):
    """Simulated FP32 implementations (one per trial) on the oracle's factors:
    each keeps its own perturbed z as its Z^{k-1}, as an implementation run
    with the same factors would."""
    dims, idx, vals = gen.make(w, scale=scale)
    T = oracle_mod.Tensor(dims, idx, vals)
    m = oracle_mod.Model(T, R, seed=3)
    rng = np.random.default_rng(17)
    trials = 4
    zprev32 = [[None] * 3 for _ in range(trials)]
    worst_ratio, flips, flip_elems, ties = 0.0, 0, 0, 0
    for it in range(iters):
        for n in range(3):
            A = m.factor(n)
            m.sweep(n)
            info = m.info(n)
            k = m.state(n)[2]
            AH = A @ info["H"]
            band, kind = info["band"], info["kind"]
            changed_any = np.zeros(kind.shape, bool)
            for t in range(trials):
                z32 = _fp32_importance(A, info["M"], AH, info["H"], info["L"], rng)
                dz = np.abs(z32 - info["z"])
                inside = dz <= band
                assert inside.all(), (it, n, int((~inside).sum()),
                                      float(np.max(dz / np.maximum(band, 1e-300))))
                nz = band > 0
                if nz.any():
                    worst_ratio = max(worst_ratio, float(np.max(dz[nz] / band[nz])))
                zp = zprev32[t][n] if k >= 2 else np.zeros_like(z32)
                zprev32[t][n] = z32
                if info["tie_global"]:
                    continue  # both branches valid: the tests take the implementation's
                sel32 = _decide(k, z32, zp, info["flip"])
                changed = sel32 != info["sel"]
                flips += int(changed.sum())
                changed_any |= changed
                assert not (changed & (kind < 2)).any(), (
                    f"iteration {it} mode {n}: {int((changed & (kind < 2)).sum())} decisions change "
                    f"outside the tie band")
            flip_elems += int(changed_any.sum())
            ties += int((kind >= 2).sum())
    print(f"largest |dz| / band {worst_ratio:.3f}; decisions changed {flips} "
          f"({flip_elems} elements); tie elements {ties}")
    assert worst_ratio > 0.05, f"band far wider than FP32 rounding moves z: {worst_ratio}"


def test_exact_zeros_are_not_ties(oracle_mod):
    """Rows of empty slices with a zero factor row have g = 0 exactly and
    z = 0 on every implementation: decided (kind 1), not ties."""
    rng = np.random.default_rng(2)
    dims = (40, 30, 20)
    n = 400
    idx = np.stack([rng.integers(0, 20, n), rng.integers(0, 30, n), rng.integers(0, 20, n)],
                   axis=1).astype(np.int32)  # rows 20..39 of mode 0 are empty slices
    vals = rng.integers(1, 6, n).astype(np.float32)
    T = oracle_mod.Tensor(dims, idx, vals)
    m = oracle_mod.Model(T, 4, seed=1)
    A0 = m.factor(0)
    A0[20:] = 0.0
    m.set_factor(0, A0)
    m.sweep(0)
    info = m.info(0)
    assert (info["kind"][20:] == 1).all()
    assert info["n_exact_zero"] >= 20 * 4
    m.sweep(1), m.sweep(2), m.sweep(0)
    info = m.info(0)
    assert (info["kind"][20:] == 1).all()
