"""GPU parity of the out-of-core first stage (input in host memory, streamed in column
blocks) against the CPU FP64 oracle and against the resident path, through the C ABI.

The streamed stage applies exactly the MU iteration: every column block's H-update uses
the same W, and the W-update waits for the X H^T, H H^T sums over all blocks.  Only the
summation order of the products differs from the resident path, so the FP32 per-iterate
bar (1e-5 relative) applies.
"""
import sys

import numpy as np
import pytest

import oracle as O
import synth as S

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_2008_01340_amd import ntt  # noqa: E402
from parity import cols_rel, cores_rel, rows_rel  # noqa: E402

TOL = 1e-5
DEV = "cuda:0"


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def pinned(x):
    t = torch.empty(x.shape, dtype=torch.float32, pin_memory=True)
    t.copy_(torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)))
    return t


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(DEV)


def host(t):
    return t.detach().double().cpu().numpy()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "a GPU is required for the gpu-marked tests"
    ntt.load()
    yield
    torch.cuda.synchronize()


@pytest.mark.parametrize("m,k,r,cols", [(40, 3000, 7, 700), (33, 1000, 16, 64), (200, 5000, 12, 1024),
                                        (16, 4096, 8, 4096), (7, 999, 3, 100)])
def test_streamed_single_stage_per_iterate_parity(m, k, r, cols):
    say(f"case: streamed d=2 NMF m={m} k={k} r={r} blocks of {cols} columns")
    rng = np.random.default_rng(m * 7 + k)
    X = (rng.random((m, k)) + 0.05).astype(np.float32)
    W0, H0 = O.init_factors(5, 1, m, r, k)
    T = 40
    ref = O.mu_nmf(X.astype(np.float64), W0, H0, T, snapshots=(1, 5, T))
    Xh = pinned(X)
    for t in (1, 5, T):
        g = ntt.decompose(Xh, (1, r, 1), t, init_W=[dev(W0)], init_H=[dev(H0)], stream_cols=cols)
        Wo, Ho = ref["snaps"][t]
        eW = rows_rel(host(g.cores[0]).reshape(m, r), Wo)
        eH = cols_rel(host(g.cores[1]).reshape(r, k), Ho)
        say(f"  t={t}: W {eW:.2e} H {eH:.2e}")
        assert eW <= TOL and eH <= TOL
    rep = g.report
    assert rep["norm_x"][0] == pytest.approx(ref["norm_x"], rel=1e-12)
    f_orc = O.objective(X.astype(np.float64), *ref["snaps"][T])
    assert rep["objective"][0] == pytest.approx(f_orc, rel=TOL)


def test_streamed_sweep_matches_oracle_and_resident_path():
    say("case: streamed sweep 24 x 20 x 30 x 16 ranks (6,5,4), blocks of 1000 columns, T=60")
    dims, ranks = (24, 20, 30, 16), (1, 6, 5, 4, 1)
    A = S.noisy_tensor(dims, ranks, seed=7, noise="mult", level=0.05)
    ref = O.ntt_decompose(A, ranks, 60, seed=3)
    st = ntt.decompose(pinned(A), ranks, 60, seed=3, stream_cols=1000)
    rs = ntt.decompose(dev(A), ranks, 60, seed=3)
    e_o = cores_rel([host(c) for c in st.cores], ref["cores"])
    e_r = cores_rel([host(c) for c in rs.cores], ref["cores"])
    say(f"  cores: streamed vs oracle {e_o:.2e}, resident vs oracle {e_r:.2e}")
    assert e_o <= TOL and e_r <= TOL
    assert st.report["iters"] == [60, 60, 60]
    for l in range(3):
        assert st.report["objective"][l] == pytest.approx(rs.report["objective"][l], rel=TOL)
    e_st = ntt.rel_error(dev(A), st.cores)
    assert e_st == pytest.approx(O.rel_error(A, O.tt_reconstruct(ref["cores"])), rel=TOL)


def test_streamed_input_may_be_pageable_and_is_validated():
    say("case: streamed input from pageable memory; a NaN is rejected")
    rng = np.random.default_rng(2)
    X = rng.random((20, 3000)).astype(np.float32)
    a = ntt.decompose(torch.from_numpy(X), (1, 5, 1), 10, seed=1, stream_cols=512)
    b = ntt.decompose(pinned(X), (1, 5, 1), 10, seed=1, stream_cols=512)
    for x, y in zip(a.cores, b.cores):
        assert torch.equal(x, y)
    X[3, 2000] = np.nan
    with pytest.raises(ntt.NttError) as e:
        ntt.decompose(pinned(X), (1, 5, 1), 10, seed=1, stream_cols=512, flags=ntt.NTT_VALIDATE_INPUT)
    assert e.value.status == ntt.NTT_ERR_NEGATIVE_INPUT


@pytest.mark.timeout(600)
def test_streamed_full_size_32pow5_matches_oracle_and_resident(oracle_tt32x5):
    """The 32^5 workload with its 134 MB input in host memory, streamed in 16 blocks of
    65,536 columns, through all 500 iterations of each stage: the streamed first stage
    (a two-way run of the first unfolding, whose W equals the sweep's core 1 bit for bit)
    against the oracle's, row by row and column by column; the later stages run the
    resident kernels on the streamed stage's H, and the sweep's error equals the
    resident sweep's."""
    say("case: streamed 32^5 ranks 8, T=500, blocks of 65536 columns")
    w, A, ref = (oracle_tt32x5[k] for k in ("w", "A", "ref"))
    st = ntt.decompose(pinned(A), w.target_ranks, w.iters, seed=w.seed, stream_cols=65536)
    rs = ntt.decompose(dev(A), w.target_ranks, w.iters, seed=w.seed)
    X1 = A.reshape(32, -1)
    W0, H0 = O.init_factors(w.seed, 1, 32, 8, X1.shape[1])
    s1 = ntt.decompose(pinned(X1), (1, 8, 1), w.iters, init_W=[dev(W0)], init_H=[dev(H0)],
                       stream_cols=65536)
    Wg = host(s1.cores[0]).reshape(32, 8)
    assert np.array_equal(Wg, host(st.cores[0]).reshape(32, 8))
    Wo, Ho = ref["stages"][0]["snaps"][w.iters]
    eW, eH = rows_rel(Wg, Wo), cols_rel(host(s1.cores[1]).reshape(8, -1), Ho)
    say(f"  streamed stage 1 vs oracle: W rows {eW:.2e}, H columns {eH:.2e}")
    assert eW <= TOL and eH <= TOL
    Ad = dev(A)
    e_st, e_rs = ntt.rel_error(Ad, st.cores), ntt.rel_error(Ad, rs.cores)
    say(f"  rel err streamed {e_st:.6e} resident {e_rs:.6e}")
    assert e_st == pytest.approx(e_rs, rel=TOL)


def test_streamed_rank_rule_matches_resident_and_oracle():
    """The rank rule of Alg.2 on a streamed first stage: the Gram of X_1 is summed over the
    column blocks; the ranks and cores equal the resident run's."""
    say("case: streamed sweep with the rank rule, 24 x 20 x 30 x 16, caps 8, rank_eps 0.02")
    dims, caps = (24, 20, 30, 16), (1, 8, 8, 8, 1)
    A = S.noisy_tensor(dims, (1, 6, 5, 4, 1), seed=7, noise="mult", level=0.01)
    ref = O.ntt_decompose(A, caps, 40, seed=3, rank_eps=0.02)
    st = ntt.decompose(pinned(A), caps, 40, seed=3, rank_eps=0.02, stream_cols=700)
    rs = ntt.decompose(dev(A), caps, 40, seed=3, rank_eps=0.02)
    say(f"  ranks streamed {st.report['eff_ranks']} resident {rs.report['eff_ranks']} oracle {ref['ranks']}")
    assert list(st.report["eff_ranks"]) == list(rs.report["eff_ranks"]) == list(ref["ranks"])
    assert cores_rel([host(c) for c in st.cores], ref["cores"]) <= TOL
    assert cores_rel([host(c) for c in rs.cores], ref["cores"]) <= TOL
