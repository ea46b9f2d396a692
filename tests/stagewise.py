"""Stage-by-stage parity of a TT sweep against the oracle (GPU tests).

In a sweep, stage l factors X_l, the previous stage's H reshaped.  The GPU's X_l differs
from the oracle's by the FP32 rounding of all earlier stages, and NMF iterates respond
to a change of their input: on the 32^5 workload an exact FP32 emulation of the sweep
(FP32 factors, FP64 reductions) ends 2.4e-5 away from the FP64 sweep in its third and
fourth stages, while every stage run from the same input stays within 5e-6.  So the
per-iterate bar is checked stage by stage on the same input: for each stage, the
oracle's NMF of the GPU's own X_l, from the stage's seeded init, against the GPU's
iterates of that X_l.  The GPU's X_l comes from a two-way run of X_{l-1}, which uses the
same kernels as the sweep's stage l-1: its W equals the sweep's core l-1 bit for bit
(checked), so X_l is the sweep's own.
"""
import numpy as np

import oracle as O
from parity import cols_rel, rows_rel


def stagewise_parity(ntt, to_dev, to_host, A, ranks, T, seed, sweep_cores, snaps=None,
                     objective_every=0, eps=1e-12, say=print, first_stage_ref=None, flags=0):
    """Per-iterate parity of every stage of the sweep of ``A`` at the effective ``ranks``.

    Returns a list of per-stage dicts: the worst row / column error over ``snaps`` (default
    (T,)), and with ``objective_every`` the worst relative objective error of every such
    iterate from a trace-recording run (the GPU's trace launch) against the oracle's.
    ``first_stage_ref``: the oracle's stage-1 result when already computed (stage 1's input
    is the tensor itself, the same on both sides), with those snapshots and objectives.
    ``flags`` go to the GPU's two-way runs (the launch mode of the sweep under test)."""
    snaps = tuple(snaps) if snaps else (T,)
    assert T in snaps
    dims = list(A.shape)
    d = len(dims)
    X = np.ascontiguousarray(A.reshape(dims[0], -1), dtype=np.float32)
    out = []
    for l in range(1, d):
        m, k, r = X.shape[0], X.shape[1], int(ranks[l])
        assert m == int(ranks[l - 1]) * dims[l - 1]
        W0, H0 = O.init_factors(seed, l, m, r, k)
        at = list(range(objective_every, T + 1, objective_every)) if objective_every else []
        if l == 1 and first_stage_ref is not None:
            ref = first_stage_ref
        else:
            ref = O.mu_nmf(X.astype(np.float64), W0, H0, T, eps=eps, snapshots=snaps, objective_at=at)
        Xd = to_dev(X)
        worst = 0.0
        for t in snaps:
            g = ntt.decompose(Xd, (1, r, 1), t, eps=eps, init_W=[to_dev(W0)], init_H=[to_dev(H0)],
                              flags=flags)
            Wg = to_host(g.cores[0]).reshape(m, r)
            Hg = to_host(g.cores[1]).reshape(r, k)
            Wo, Ho = ref["snaps"][t]
            worst = max(worst, rows_rel(Wg, Wo), cols_rel(Hg, Ho))
        # the two-way run at T is the sweep's stage l: same W bits, so its H is X_{l+1}
        assert np.array_equal(Wg.reshape(-1), to_host(sweep_cores[l - 1]).reshape(-1)), l
        if l == d - 1:
            assert np.array_equal(Hg.reshape(-1), to_host(sweep_cores[d - 1]).reshape(-1))
        res = {"stage": l, "shape": (m, k, r), "worst": worst}
        if at:
            rec = ntt.decompose(Xd, (1, r, 1), T, eps=eps, init_W=[to_dev(W0)], init_H=[to_dev(H0)],
                                record_objective=True)
            f = to_host(rec.trace)[np.array(at) - 1]
            fo = np.array([ref["objective_at_t"][t] for t in at])
            res["objective"] = float(np.max(np.abs(f - fo) / fo))
            res["objective_ok"] = bool(np.all(np.abs(f - fo) <= 1e-5 * fo + 1e-12 * ref["norm_x"] ** 2))
        say(f"  stage {l} ({m} x {k}, r {r}) from the GPU's X_{l}: worst row/column rel diff "
            f"{worst:.2e}" + (f", objective every {objective_every}th {res['objective']:.2e}" if at else ""))
        out.append(res)
        if l < d - 1:
            X = np.ascontiguousarray(Hg.astype(np.float32).reshape(r * dims[l], -1))
    return out
