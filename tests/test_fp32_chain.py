"""Why the GPU parity bar is applied stage by stage (CPU test, no GPU).

An exact FP32 emulation of MU (FP32 factors and H-update, FP64 reductions for the
W-update, as the GPU does) is run on every stage of a 16^5 rank-8 sweep, once from the
oracle's own unfolding of that stage rounded to FP32 (stage by stage) and once chained
(each stage fed the emulation's own H of the previous stage).  Stage by stage every
factor stays within the 1e-5 per-iterate bar after 500 iterations; chained, the later
stages move several times further, because each stage's NMF amplifies the rounding its
input inherited.  No FP32 implementation can undo that, so the GPU tests compare every
stage with the oracle on the GPU's own input of that stage.
"""
import numpy as np

import oracle as O
import synth as S
from parity import cols_rel, rows_rel


def _mu_fp32(X32, W0, H0, T, eps=1e-12):
    X64 = X32.astype(np.float64)
    W = W0.astype(np.float32)
    H = H0.astype(np.float32)
    for _ in range(T):
        H = np.maximum(np.float32(0), H * (W.T @ X32) / ((W.T @ W) @ H + np.float32(eps)))
        Hd = H.astype(np.float64)
        Wd = W.astype(np.float64)
        W = np.maximum(0.0, Wd * (X64 @ Hd.T) / (Wd @ (Hd @ Hd.T) + eps)).astype(np.float32)
    return W, H


def test_fp32_rounding_stays_within_the_bar_stage_by_stage_but_not_chained():
    dims, ranks, T = (16,) * 5, (1, 8, 8, 8, 8, 1), 500
    A = S.noisy_tensor(dims, ranks, seed=2, noise="mult", level=0.01)
    ref = O.ntt_decompose(A, ranks, T, seed=2)
    X32 = A.reshape(dims[0], -1).astype(np.float32)
    alone, chained = [], []
    for l in range(1, len(dims)):
        st = ref["stages"][l - 1]
        W0, H0 = O.init_factors(2, l, st["m"], st["r"], st["k"])
        Wc, Hc = _mu_fp32(X32, W0, H0, T)
        Wi, Hi = _mu_fp32(st["X"].astype(np.float32), W0, H0, T)
        chained.append(max(rows_rel(Wc, st["W"]), cols_rel(Hc, st["H"])))
        alone.append(max(rows_rel(Wi, st["W"]), cols_rel(Hi, st["H"])))
        X32 = Hc.reshape(st["r"] * dims[l], -1)
    assert max(alone) <= 1e-5, alone
    assert chained[0] == alone[0]  # the same input
    assert chained[2] > 3.0 * alone[2] and chained[3] > 3.0 * alone[3], (alone, chained)
    assert max(chained) > 1e-5, chained
