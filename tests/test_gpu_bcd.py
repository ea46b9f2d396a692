"""GPU parity of the BCD NMF (Alg.3) against the CPU FP64 oracle, through the C ABI.

Factors are compared element-wise at the FP32 bar TOL (rows of W, columns of H).  The
objective is compared at the bar that bar implies: if the model M = W H is within
relative TOL of the oracle's, f = 1/2 ||X - M||^2 moves by at most
TOL ||R|| ||M|| + TOL^2 ||M||^2 / 2 (R = X - M, ||R|| = sqrt(2 f)), plus the floor of a
residual evaluated with FP32 products.  BCD drives f far closer to 0 than MU does (f / ||X||^2
reaches 1e-8 on noise-free TT tensors), where a relative bar on f would ask the model to
be exact to TOL sqrt(f) / ||X||, far below FP32 rounding.

The correction test compares two objectives; where the oracle's margin of a decision is
within what the objectives can resolve, the two sides may decide differently and then
follow different (equally valid) trajectories.  So:
* per-iterate parity (candidate objectives, kept factors) is checked over iterations
  whose oracle decisions all have relative margins above MARGIN, and the
  dropped-iteration counts must agree there;
* long runs, where decisions near ties occur, are checked on the final relative error
  (Eq.(3)) with the bar LONG_BAR, like the BF16 mode.
"""
import math
import sys

import numpy as np
import pytest

import oracle as O
import synth as S

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_2008_01340_amd import ntt  # noqa: E402
from parity import cols_rel, cores_rel, rows_rel  # noqa: E402

DEV = "cuda:0"
# Per-iterate bar (rows of W, columns of H), the FP32 bar of the MU path.
TOL = 1e-5
MARGIN = 1e-3   # decisions with a smaller relative margin are not compared
# The floor of an objective evaluated with FP32 products: each entry of W H carries a
# relative error of about r 2^-24, so f is not resolved below ~(r 2^-24)^2 ||X||^2.
FLOOR = 1e-12
LONG_BAR = 1e-3  # |e_gpu - e_oracle| on the final relative error after long runs


def obj_bar(f_orc, nx):
    """|f_gpu - f_orc| allowed for the objective of a model within TOL of the oracle's."""
    f_orc = np.asarray(f_orc, dtype=np.float64)
    nr = np.sqrt(2.0 * np.maximum(f_orc, 0.0))
    nm = nx + nr  # ||M|| <= ||X|| + ||R||
    return TOL * nr * nm + 0.5 * TOL * TOL * nm * nm + FLOOR * nx * nx


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(DEV)


def host(t):
    return t.detach().double().cpu().numpy()


def margins(res):
    """Relative margin of each iteration's decision in an oracle run (relative to
    f_kept + FLOOR ||X||^2); a decision is compared when its margin exceeds MARGIN."""
    out, kept_obj = [], 0.5 * res["norm_x"] ** 2
    fl = FLOOR * res["norm_x"] ** 2
    for f, k in zip(res["objective"], res["kept"]):
        out.append(abs(f - kept_obj) / (kept_obj + fl))
        if k:
            kept_obj = f
    return np.array(out)


def safe_count(res, T):
    """Iterations 1..safe whose oracle decisions (and all before them) are resolvable."""
    mg = margins(res)
    return int(np.argmax(mg < MARGIN)) if np.any(mg < MARGIN) else T


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "a GPU is required for the gpu-marked tests"
    ntt.load()
    yield
    torch.cuda.synchronize()


SHAPES = [
    # (m, k, r): ragged m and k, ranks at the three paddings (8, 16, 32)
    (16, 256, 4), (7, 33, 3), (45, 517, 5), (100, 301, 16), (130, 77, 32), (1, 50, 1),
    (200, 3, 3), (33, 250, 24), (300, 2000, 10), (64, 4099, 8), (520, 700, 12),
    # H step with rows split over 4 groups, one column per thread (odd k) and 4 columns
    # per thread with a ragged last workgroup
    (200, 40000, 6), (16, 300001, 3), (24, 600004, 5),
    # MFMA products (more than 32 rows, k % 4 == 0) at paddings 16 and 32, ragged last row
    # block
    (96, 1000, 24), (70, 3000, 32), (260, 4096, 16),
    # MFMA products on 32-row and 16-row tiles (128 and 256 columns), ragged last tile
    (30, 2000, 28), (14, 5000, 11), (32, 4100, 8),
]


@pytest.mark.parametrize("m,k,r", SHAPES)
def test_bcd_single_stage_per_iterate_parity(m, k, r):
    say(f"case: BCD d=2 NMF m={m} k={k} r={r}")
    rng = np.random.default_rng(m * 1000 + k + 7)
    X = (rng.random((m, k)) + 0.05).astype(np.float32)
    W0, H0 = O.init_factors(11, 1, m, r, k)
    T = 40
    ref = O.bcd_nmf(X.astype(np.float64), W0, H0, T, snapshots=(1, 2, 5, 20, T))
    safe = safe_count(ref, T)  # iterations 1..safe
    res = ntt.decompose(dev(X), (1, r, 1), T, init_W=[dev(W0)], init_H=[dev(H0)],
                        record_objective=True, nmf="bcd")
    f_gpu = host(res.trace)
    f_orc = ref["objective"]
    diff = np.abs(f_gpu[:safe] - f_orc[:safe])
    q = diff / obj_bar(f_orc[:safe], ref["norm_x"])
    say(f"  safe iterations {safe}/{T}, max objective diff / bar {q.max() if safe else 0:.2e}, "
        f"max rel objective diff {np.max(diff / np.maximum(f_orc[:safe], 1e-300)) if safe else 0:.2e}, "
        f"oracle corrections {ref['corrections']}")
    assert safe >= 1
    assert np.all(q <= 1.0), q
    for t in (1, 2, 5, 20, T):
        if t > safe:
            break
        r_t = ntt.decompose(dev(X), (1, r, 1), t, init_W=[dev(W0)], init_H=[dev(H0)], nmf="bcd")
        Wg = host(r_t.cores[0]).reshape(m, r)
        Hg = host(r_t.cores[1]).reshape(r, k)
        Wo, Ho = ref["snaps"][t]
        eW, eH = rows_rel(Wg, Wo), cols_rel(Hg, Ho)
        say(f"  t={t}: W rows {eW:.2e} H columns {eH:.2e}")
        assert eW <= TOL, (t, eW)
        assert eH <= TOL, (t, eH)
        assert abs(float(np.sum(Wg)) - 1.0) <= 1e-5  # W /= ||W||_1 after every W step
        assert Wg.min() >= 0 and Hg.min() >= 0
        assert r_t.report["corrections"][0] == ref["kept"][:t].count(False)


def test_bcd_without_extrapolation_descends_and_never_corrects():
    say("case: BCD delta=0, 64 x 3000 rank 6, T=60")
    rng = np.random.default_rng(5)
    X = rng.random((64, 3000)).astype(np.float32)
    W0, H0 = O.init_factors(2, 1, 64, 6, 3000)
    ref = O.bcd_nmf(X.astype(np.float64), W0, H0, 60, delta=0.0)
    res = ntt.decompose(dev(X), (1, 6, 1), 60, init_W=[dev(W0)], init_H=[dev(H0)],
                        record_objective=True, nmf="bcd", delta=0.0)
    f = host(res.trace)
    assert res.report["corrections"][0] == 0 == ref["corrections"]
    assert np.all(np.diff(f) < 0.0)
    assert np.all(np.abs(f - ref["objective"]) <= obj_bar(ref["objective"], ref["norm_x"]))
    assert rows_rel(host(res.cores[0]).reshape(64, 6), ref["W"]) <= TOL
    assert cols_rel(host(res.cores[1]).reshape(6, 3000), ref["H"]) <= TOL


def test_bcd_trace_of_a_dropped_last_candidate():
    # Candidate 26 of this run is dropped by a margin of 2e-2 (every earlier decision has
    # a margin above 1e-3): trace slot 26 holds that candidate's objective, while the
    # result, and the report's objective, are those of the kept pair.
    say("case: BCD 30 x 200 rank 3, T=26, the last candidate dropped")
    m, k, r, R, seed, T = 30, 200, 3, 2, 2, 26
    rng = np.random.default_rng(m * 1000 + k + seed)
    X = (rng.random((m, R)) @ rng.random((R, k)) + 0.01 * rng.random((m, k))).astype(np.float32)
    W0, H0 = O.init_factors(seed, 1, m, r, k)
    ref = O.bcd_nmf(X.astype(np.float64), W0, H0, T)
    assert ref["kept"][-1] is False and all(ref["kept"][-3:-1])
    assert np.all(margins(ref) > MARGIN)
    res = ntt.decompose(dev(X), (1, r, 1), T, init_W=[dev(W0)], init_H=[dev(H0)],
                        record_objective=True, nmf="bcd")
    f = host(res.trace)
    f_kept = O.objective(X.astype(np.float64), ref["W"], ref["H"])
    say(f"  trace[T] {f[-1]:.8e} oracle candidate {ref['objective'][-1]:.8e} kept {f_kept:.8e}")
    assert np.all(np.abs(f - ref["objective"]) <= obj_bar(ref["objective"], ref["norm_x"]))
    assert abs(f[-1] - f_kept) > 1e-3 * f_kept  # the slot is not the kept pair's objective
    assert res.report["corrections"][0] == ref["corrections"] == 1
    assert abs(res.report["objective"][0] - f_kept) <= obj_bar(f_kept, ref["norm_x"])
    assert rows_rel(host(res.cores[0]).reshape(m, r), ref["W"]) <= TOL
    assert cols_rel(host(res.cores[1]).reshape(r, k), ref["H"]) <= TOL


def test_bcd_graph_replay_equals_direct_launches_bitwise():
    say("case: BCD 16^3 sweep T=80 with (graphs) and without (trace) replay")
    w = S.workload("tt16x3_r4")
    Ad = dev(w.tensor())
    a = ntt.decompose(Ad, w.target_ranks, 80, seed=w.seed, nmf="bcd")
    b = ntt.decompose(Ad, w.target_ranks, 80, seed=w.seed, nmf="bcd", record_objective=True)
    c = ntt.decompose(Ad, w.target_ranks, 80, seed=w.seed, nmf="bcd")
    for x, y, z in zip(a.cores, b.cores, c.cores):
        assert torch.equal(x, y) and torch.equal(x, z)
    assert a.report["corrections"] == b.report["corrections"]


def test_bcd_sweep_16cubed_matches_oracle():
    say("case: BCD sweep 16^3 ranks (4,4), T=200")
    w = S.workload("tt16x3_r4")
    A = w.tensor()
    T = w.iters
    ref = O.ntt_decompose(A, w.target_ranks, T, seed=w.seed, nmf="bcd")
    res = ntt.decompose(dev(A), w.target_ranks, T, seed=w.seed, nmf="bcd", record_objective=True)
    f_gpu = host(res.trace).reshape(2, T)
    st1 = ref["stages"][0]
    safe = safe_count(st1, T)
    q = np.abs(f_gpu[0][:safe] - st1["objective"][:safe]) / obj_bar(st1["objective"][:safe], st1["norm_x"])
    say(f"  stage 1: safe {safe}/{T}, max objective diff / bar {q.max():.2e}; corrections "
        f"gpu {res.report['corrections']} oracle {[s['corrections'] for s in ref['stages']]}")
    assert np.all(q <= 1.0)
    if safe == T:
        assert res.report["corrections"][0] == st1["corrections"]
        assert rows_rel(host(res.cores[0]).reshape(16, 4), ref["cores"][0].reshape(16, 4)) <= TOL
    e_orc = O.rel_error(A, O.tt_reconstruct(ref["cores"]))
    e_gpu = ntt.rel_error(dev(A), res.cores)
    say(f"  rel err: oracle {e_orc:.6e} gpu {e_gpu:.6e}")
    assert abs(e_gpu - e_orc) <= LONG_BAR
    mu = ntt.decompose(dev(A), w.target_ranks, T, seed=w.seed)
    assert e_gpu < ntt.rel_error(dev(A), mu.cores)  # BCD below MU at equal iterations


@pytest.mark.parametrize("dims,gen,noise,level,T", [
    ((24, 20, 30, 16), (1, 6, 5, 4, 1), "mult", 0.05, 150),
    ((20, 40, 40, 50), (1, 6, 5, 4, 1), "mult", 0.01, 100),
    ((40, 30, 20, 30), (1, 16, 12, 8, 1), "absnormal", 0.01, 100),
])
def test_bcd_sweep_final_error_matches_oracle(dims, gen, noise, level, T):
    say(f"case: BCD sweep dims={dims} ranks={gen} T={T}")
    A = S.noisy_tensor(dims, gen, seed=7, noise=noise, level=level)
    ref = O.ntt_decompose(A, gen, T, seed=3, nmf="bcd")
    e_orc = O.rel_error(A, O.tt_reconstruct(ref["cores"]))
    Ad = dev(A)
    res = ntt.decompose(Ad, gen, T, seed=3, nmf="bcd")
    e_gpu = ntt.rel_error(Ad, res.cores)
    say(f"  rel err: oracle {e_orc:.6e} gpu {e_gpu:.6e}; corrections gpu "
        f"{res.report['corrections']} oracle {[s['corrections'] for s in ref['stages']]}")
    assert abs(e_gpu - e_orc) <= LONG_BAR
    for c in res.cores:
        assert float(c.min()) >= 0.0
    assert res.report["iters"] == [T] * (len(dims) - 1)


def test_bcd_zero_iterations_returns_scaled_init():
    say("case: BCD T=0 (scaled random factors)")
    rng = np.random.default_rng(3)
    X = rng.random((20, 70)).astype(np.float32)
    W0, H0 = O.init_factors(4, 1, 20, 5, 70)
    res = ntt.decompose(dev(X), (1, 5, 1), 0, init_W=[dev(W0)], init_H=[dev(H0)], nmf="bcd")
    ref = O.bcd_nmf(X.astype(np.float64), W0, H0, 0)
    assert rows_rel(host(res.cores[0]).reshape(20, 5), ref["W"]) <= 1e-6
    assert cols_rel(host(res.cores[1]).reshape(5, 70), ref["H"]) <= 1e-6


def test_bcd_with_rank_rule():
    say("case: BCD with the rank rule, 24 x 20 x 30 x 16 ranks <= 8, rank_eps 0.02")
    A = S.noisy_tensor((24, 20, 30, 16), (1, 6, 5, 4, 1), seed=7, noise="mult", level=0.01)
    ref = O.ntt_decompose(A, (1, 8, 8, 8, 1), 60, seed=3, nmf="bcd", rank_eps=0.02)
    res = ntt.decompose(dev(A), (1, 8, 8, 8, 1), 60, seed=3, nmf="bcd", rank_eps=0.02)
    assert list(res.report["eff_ranks"]) == list(ref["ranks"])
    e_orc = O.rel_error(A, O.tt_reconstruct(ref["cores"]))
    e_gpu = ntt.rel_error(dev(A), res.cores)
    say(f"  ranks {ref['ranks']} rel err oracle {e_orc:.6e} gpu {e_gpu:.6e}")
    assert abs(e_gpu - e_orc) <= LONG_BAR


def test_bcd_full_size_first_unfolding_per_iterate():
    """The 32^5 workload's first unfolding (32 x 32^4, rank 8) as the sweep runs it: the
    first iterations against the oracle, every entry."""
    say("case: BCD full-size first unfolding 32 x 1048576 rank 8, T=1..4")
    w = S.workload("tt32x5_r8")
    A = w.tensor()
    X = A.reshape(32, -1)
    Xd = dev(X)
    W0, H0 = O.init_factors(w.seed, 1, 32, 8, X.shape[1])
    T = 4
    ref = O.bcd_nmf(X.astype(np.float64), W0, H0, T, snapshots=tuple(range(1, T + 1)))
    assert np.all(margins(ref) > MARGIN)
    for t in range(1, T + 1):
        g = ntt.decompose(Xd, (1, 8, 1), t, init_W=[dev(W0)], init_H=[dev(H0)], nmf="bcd")
        Wo, Ho = ref["snaps"][t]
        eW = rows_rel(host(g.cores[0]).reshape(32, 8), Wo)
        eH = cols_rel(host(g.cores[1]).reshape(8, -1), Ho)
        say(f"  t={t}: W {eW:.2e} H {eH:.2e}")
        assert eW <= TOL and eH <= TOL


def test_bcd_zero_input_drops_every_iteration():
    say("case: BCD on an all-zero 20 x 30 matrix, rank 3, T=5")
    X = np.zeros((20, 30), dtype=np.float32)
    W0, H0 = O.init_factors(1, 1, 20, 3, 30)
    ref = O.bcd_nmf(X.astype(np.float64), W0, H0, 5)
    res = ntt.decompose(dev(X), (1, 3, 1), 5, init_W=[dev(W0)], init_H=[dev(H0)], nmf="bcd")
    assert ref["corrections"] == 5 == res.report["corrections"][0]
    for c in res.cores:
        assert float(c.abs().max()) == 0.0
    assert res.report["objective"][0] == 0.0


def test_bcd_zero_rows_and_columns_match_oracle():
    say("case: BCD 30 x 52 with a zero row and two zero columns, rank 4")
    rng = np.random.default_rng(3)
    X = rng.random((30, 52)).astype(np.float32)
    X[4, :] = 0.0
    X[:, 7] = 0.0
    X[:, 20] = 0.0
    W0, H0 = O.init_factors(2, 1, 30, 4, 52)
    ref = O.bcd_nmf(X.astype(np.float64), W0, H0, 30, snapshots=(1, 5, 30))
    assert np.all(margins(ref) > MARGIN)
    for t in (1, 5, 30):
        g = ntt.decompose(dev(X), (1, 4, 1), t, init_W=[dev(W0)], init_H=[dev(H0)], nmf="bcd")
        Wo, Ho = ref["snaps"][t]
        Wg, Hg = host(g.cores[0]).reshape(30, 4), host(g.cores[1]).reshape(4, 52)
        assert rows_rel(Wg, Wo) <= TOL and cols_rel(Hg, Ho) <= TOL, t
        assert Wg.min() >= 0 and Hg.min() >= 0


def test_bcd_rejects_negative_input():
    say("case: BCD with a negative entry and the input check")
    X = np.ones((10, 40), dtype=np.float32)
    X[3, 17] = -1.0
    with pytest.raises(ntt.NttError) as e:
        ntt.decompose(dev(X), (1, 2, 1), 5, nmf="bcd", flags=ntt.NTT_VALIDATE_INPUT)
    assert e.value.status == ntt.NTT_ERR_NEGATIVE_INPUT


def test_bcd_batched_results_equal_standalone_results_bitwise():
    say("case: batch of 5 uneven problems with BCD vs ntt_decompose one by one")
    probs = [((6, 7, 5), (1, 3, 4, 1), 11), ((16, 16, 16), (1, 4, 4, 1), 1),
             ((9, 20, 8, 6), (1, 5, 6, 3, 1), 5), ((30, 40, 12), (1, 12, 9, 1), 8),
             ((64, 33, 50), (1, 10, 12, 1), 3)]
    tensors = [dev(S.contract_cores(S.random_cores(d, r, seed=s))) for d, r, s in probs]
    T = 60
    cores, reps, _ = ntt.decompose_batch(tensors, [r for _, r, _ in probs], T,
                                         [s for _, _, s in probs], nmf="bcd")
    for (d, r, s), A, cb, rb in zip(probs, tensors, cores, reps):
        one = ntt.decompose(A, r, T, seed=s, nmf="bcd")
        for x, y in zip(cb, one.cores):
            assert torch.equal(x, y), (d, r)
        assert rb["corrections"] == one.report["corrections"]


def test_bcd_serving_results_equal_standalone_results():
    say("case: serving 4 BCD requests, 25 iterations per tick")
    probs = [((6, 7, 5), (1, 3, 4, 1), 11), ((16, 16, 16), (1, 4, 4, 1), 1),
             ((9, 20, 8, 6), (1, 5, 6, 3, 1), 5), ((64, 33, 50), (1, 10, 12, 1), 3)]
    T = 60
    host_t = [S.contract_cores(S.random_cores(d, r, seed=s)) for d, r, s in probs]
    srv = ntt.Server(1 << 30, max_slots=4, iters_per_tick=25)
    ids = []
    for a, (d, r, s) in zip(host_t, probs):
        h = torch.empty(a.shape, dtype=torch.float32, pin_memory=True)
        h.copy_(torch.from_numpy(a))
        ids.append(srv.submit(h, r, T, seed=s, nmf="bcd"))
    alone = [ntt.decompose(dev(a), r, T, seed=s, nmf="bcd") for a, (d, r, s) in zip(host_t, probs)]
    pending = dict(zip(ids, range(len(ids))))
    ticks = 0
    while pending:
        srv.tick()
        ticks += 1
        for rid in list(pending):
            if srv.info(rid)["state"] != ntt.NTT_REQ_DONE:
                continue
            i = pending.pop(rid)
            served = srv.cores(rid)
            for x, y in zip(served, alone[i].cores):
                assert torch.equal(x, y), probs[i]
            # against the oracle: the final error, as for every long BCD run
            d, r, s = probs[i]
            ref = O.ntt_decompose(host_t[i], r, T, seed=s, nmf="bcd")
            e_orc = O.rel_error(host_t[i], O.tt_reconstruct(ref["cores"]))
            e_srv = ntt.rel_error(dev(host_t[i]), served)
            say(f"  {d}: rel err oracle {e_orc:.6e} served {e_srv:.6e}")
            assert abs(e_srv - e_orc) <= LONG_BAR
            srv.release(rid)
        assert ticks < 100000
    srv.close()
