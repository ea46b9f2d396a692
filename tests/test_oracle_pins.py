"""Pins of the CPU oracle against facts it does not compute itself.

Every test here is CPU-only.  Each one fixes a property that a plausible slip in
the oracle (a dropped term, a sign, a swapped index, a transposed operand) breaks:
published generator outputs, numbers printed in the paper, brute force on tiny
inputs, closed forms and theorems about MU.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle as O
import synth as S

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _rng(seed):
    return np.random.default_rng(seed)


# ------------------------------------------------------------------ generator rule
def test_splitmix64_published_vectors():
    g = json.load(open(os.path.join(GOLD, "splitmix64_vectors.json")))
    want = [int(x) for x in g["outputs"]]
    # tag 0, counters 1..5 is the plain published sequence
    got = [O.splitmix64_at(g["seed"], i + 1) for i in range(5)]
    assert got == want
    raw = S.splitmix64(g["seed"], 0, 0, 5)
    assert [int(x) for x in raw] == want


def test_uniform_rule_matches_between_oracle_and_generator():
    # two independent implementations of the same published rule
    for seed, tag in [(0, 0), (1, 2), (2**63 + 5, 7), (12345, 0x101)]:
        a = O.rng_uniform(seed, tag, 1000)
        b = S.uniform01(seed, tag, (1000,)).astype(np.float64)
        assert np.array_equal(a, b)
        assert a.min() >= 0.0 and a.max() < 1.0
        assert np.array_equal(a.astype(np.float32).astype(np.float64), a)  # FP32-exact
        # top 24 bits of the raw output
        raw = S.splitmix64(seed, tag, 0, 1000)
        assert np.array_equal(a * (1 << 24), (raw >> np.uint64(40)).astype(np.float64))


def test_uniform_moments():
    u = O.rng_uniform(99, 3, 200000)
    assert abs(u.mean() - 0.5) < 3e-3
    assert abs(u.var() - 1.0 / 12) < 2e-3


# ------------------------------------------------------------------ Eq.(2) brute force
@pytest.mark.parametrize("dims,ranks", [((3, 2, 4), (1, 2, 3, 1)),
                                        ((2, 3, 2, 3), (1, 2, 3, 2, 1)),
                                        ((4, 4), (1, 3, 1)),
                                        ((2, 2, 2, 2, 2), (1, 2, 2, 2, 2, 1))])
def test_reconstruct_equals_bruteforce_sum(dims, ranks):
    rng = _rng(1)
    cores = [rng.random((ranks[k], dims[k], ranks[k + 1])) for k in range(len(dims))]
    full = O.tt_reconstruct(cores)
    assert full.shape == tuple(dims)
    for idx in np.ndindex(*dims):
        assert math.isclose(full[idx], O.tt_element(cores, idx), rel_tol=1e-13)
    # third route: einsum over the explicit index string
    letters = "abcdefghij"
    spec = ",".join(f"{'z' if k == 0 else letters[k - 1]}{chr(ord('p') + k)}"
                    f"{'y' if k == len(dims) - 1 else letters[k]}" for k in range(len(dims)))
    out = "".join(chr(ord("p") + k) for k in range(len(dims)))
    ein = np.einsum(spec + "->" + out, *cores)
    np.testing.assert_allclose(full, ein, rtol=1e-13)


def test_generator_tensor_equals_oracle_reconstruction():
    dims, ranks = (5, 4, 6, 3), (1, 3, 2, 4, 1)
    cores = S.random_cores(dims, ranks, seed=11)
    a = S.contract_cores(cores)
    ref = O.tt_reconstruct([c.astype(np.float64) for c in cores])
    # the generator rounds once to float32
    np.testing.assert_allclose(a.astype(np.float64), ref, rtol=2 ** -23)
    assert a.dtype == np.float32 and a.min() >= 0


def test_generated_unfoldings_have_the_generating_ranks():
    dims, ranks = (6, 7, 8, 5), (1, 3, 4, 2, 1)
    a = S.contract_cores(S.random_cores(dims, ranks, seed=3)).astype(np.float64)
    for l in range(1, len(dims)):
        X = a.reshape(int(np.prod(dims[:l])), -1)
        assert np.linalg.matrix_rank(X, tol=1e-6 * np.linalg.norm(X)) == ranks[l]


# ------------------------------------------------------------------ Eq.(3), Eq.(4)
def test_compression_ratio_printed_values():
    g = json.load(open(os.path.join(GOLD, "compression_ratio_pins.json")))
    for c in g["cases"]:
        cr = O.compression_ratio(c["dims"], c["ranks"])
        assert math.isclose(cr, c["exact"], rel_tol=1e-12)
        # the paper prints three significant digits, truncated (14799.1 -> 1.47e4)
        e = int(math.floor(math.log10(cr)))
        mant = math.floor(cr / 10 ** (e - 2)) / 100.0
        assert f"{mant:.2f}e{e}" == c["printed"]


def test_compression_ratio_closed_forms():
    # uncompressed TT with full ranks of a matrix: C = n1 n2 / (n1 r + n2 r)
    assert O.compression_ratio([10, 20], [1, 5, 1]) == 200 / (10 * 5 + 20 * 5)
    assert O.compression_ratio([7], [1, 1]) == 1.0


def test_rel_error_definition():
    a = np.array([[3.0, 0.0], [0.0, 4.0]])
    assert O.rel_error(a, a) == 0.0
    assert math.isclose(O.rel_error(a, np.zeros_like(a)), 1.0)
    assert math.isclose(O.rel_error(a, 2 * a), 1.0)
    assert math.isclose(O.rel_error(a, a + np.array([[0.0, 5.0], [0.0, 0.0]])), 1.0)


def test_effective_rank_clamp():
    assert O.effective_ranks([2, 3, 4], [1, 5, 5, 1]) == [1, 2, 4, 1]
    assert O.effective_ranks([16, 16, 16], [1, 4, 4, 1]) == [1, 4, 4, 1]
    assert O.effective_ranks([4, 100, 2], [1, 50, 50, 1]) == [1, 4, 2, 1]


# ------------------------------------------------------------------ MU theorems
def _nonneg(m, n, seed):
    return _rng(seed).random((m, n)) + 0.01


def test_mu_objective_non_increasing_and_nonnegative():
    X = _nonneg(30, 45, 0)
    W0, H0 = O.init_factors(5, 1, 30, 4, 45)
    res = O.mu_nmf(X, W0, H0, 300, record_objective=True)
    f = res["objective"]
    # Lee & Seung (2001): the Frobenius MU never increases the objective (eps = 0);
    # eps = 1e-12 perturbs it at ~1e-12 relative
    assert np.all(np.diff(f) <= 1e-10 * f[:-1])
    assert f[-1] < 0.2 * f[0]
    assert res["W"].min() >= 0 and res["H"].min() >= 0


def test_mu_rank1_reaches_svd_truncation():
    # Perron-Frobenius: the best rank-1 approximation of a positive matrix is non-negative,
    # so converged rank-1 NMF attains the SVD truncation error.
    X = _nonneg(12, 17, 1)
    W0, H0 = O.init_factors(3, 1, 12, 1, 17)
    res = O.mu_nmf(X, W0, H0, 2000, record_objective=True)
    s = np.linalg.svd(X, compute_uv=False)
    e_svd = math.sqrt(float(np.sum(s[1:] ** 2))) / math.sqrt(float(np.sum(s ** 2)))
    e_mu = math.sqrt(2 * res["objective"][-1]) / res["norm_x"]
    assert abs(e_mu - e_svd) <= 1e-9


def test_mu_fixed_point_satisfies_kkt():
    # At a limit point of MU the KKT conditions of min 1/2||X-WH||^2, W,H >= 0 hold:
    # grad >= 0 everywhere and grad * factor = 0.  A transposed operand or a wrong
    # numerator/denominator drives the iterates somewhere else.
    X = _nonneg(20, 25, 2)
    W0, H0 = O.init_factors(8, 1, 20, 3, 25)
    res = O.mu_nmf(X, W0, H0, 20000)
    W, H = res["W"], res["H"]
    gH = W.T @ W @ H - W.T @ X
    gW = W @ (H @ H.T) - X @ H.T
    scale = np.linalg.norm(X) ** 2
    assert np.abs(gH * H).max() / scale < 1e-6
    assert np.abs(gW * W).max() / scale < 1e-6
    assert gH.min() / np.linalg.norm(X) > -1e-3 and gW.min() / np.linalg.norm(X) > -1e-3


def test_mu_exact_factorization_is_a_fixed_point():
    rng = _rng(3)
    Ws, Hs = rng.random((9, 3)) + 0.1, rng.random((3, 14)) + 0.1
    X = Ws @ Hs
    W1, H1 = O.mu_step(X, Ws, Hs, 1e-12)
    assert np.abs(H1 - Hs).max() / Hs.max() < 1e-10
    assert np.abs(W1 - Ws).max() / Ws.max() < 1e-10


def test_mu_scale_covariance():
    X = _nonneg(10, 13, 4)
    W0, H0 = O.init_factors(1, 1, 10, 3, 13)
    c = 7.5
    a = O.mu_nmf(X, W0, H0, 50, eps=0.0)
    b = O.mu_nmf(c * X, W0, c * H0, 50, eps=0.0)
    np.testing.assert_allclose(b["W"], a["W"], rtol=1e-10)
    np.testing.assert_allclose(b["H"], c * a["H"], rtol=1e-10)


def test_mu_row_permutation_covariance():
    X = _nonneg(11, 9, 5)
    W0, H0 = O.init_factors(2, 1, 11, 2, 9)
    p = _rng(6).permutation(11)
    a = O.mu_nmf(X, W0, H0, 40)
    b = O.mu_nmf(X[p], W0[p], H0, 40)
    np.testing.assert_allclose(b["W"], a["W"][p], rtol=1e-11)
    np.testing.assert_allclose(b["H"], a["H"], rtol=1e-11)


def test_mu_h_first_order():
    # The first half-step updates H from (W0, H0) alone; W then sees the new H.
    X = _nonneg(6, 8, 7)
    W0, H0 = O.init_factors(4, 1, 6, 2, 8)
    W1, H1 = O.mu_step(X, W0, H0, 1e-12)
    res = O.mu_nmf(X, W0, H0, 1, snapshots=(1,))
    np.testing.assert_array_equal(res["snaps"][1][1], H1)
    # with H fixed at H1 the W half-step is a closed-form ratio; recompute it by entries
    N = X @ H1.T
    D = W0 @ (H1 @ H1.T)
    for i in range(6):
        for j in range(2):
            assert math.isclose(W1[i, j], W0[i, j] * N[i, j] / (D[i, j] + 1e-12), rel_tol=1e-14)


def test_mu_halves_are_column_separable_and_product_only():
    # Sampled parity at sizes the oracle cannot hold relies on two facts of the MU rule:
    # the H half acts on each column alone (column j of W^T X and of (W^T W) H involve
    # column j only), and the W half sees X only through X H^T, which may be summed over
    # column blocks.  Check both by entries on a small case.
    X = _nonneg(7, 40, 11)
    W0, H0 = O.init_factors(9, 1, 7, 3, 40)
    W1, H1 = O.mu_step(X, W0, H0, 1e-12)
    cols = [0, 5, 17, 39]
    np.testing.assert_array_equal(O.update_H(X[:, cols], W0, H0[:, cols], 1e-12), H1[:, cols])
    WtW = W0.T @ W0
    for j in cols:
        for c in range(3):
            num = sum(W0[i, c] * X[i, j] for i in range(7))
            den = sum(WtW[c, q] * H0[q, j] for q in range(3)) + 1e-12
            assert math.isclose(H1[c, j], max(0.0, H0[c, j] * num / den), rel_tol=1e-13)
    XHt = sum(X[:, c0:c0 + 8] @ H1[:, c0:c0 + 8].T for c0 in range(0, 40, 8))
    HHt = sum(H1[:, c0:c0 + 8] @ H1[:, c0:c0 + 8].T for c0 in range(0, 40, 8))
    np.testing.assert_allclose(O.update_W(XHt, HHt, W0, 1e-12), W1, rtol=1e-13)


def test_eps_rank_hand_computed_spectrum():
    # singular values 5, 4, 3, 2, 1 (sum of squares 55); tail ratios after k values:
    # k=1 sqrt(30/55)=0.7385, k=2 sqrt(14/55)=0.5045, k=3 sqrt(5/55)=0.3015,
    # k=4 sqrt(1/55)=0.1348, k=5 0.  The rule takes the first k at or below eps.
    s = np.array([5.0, 4.0, 3.0, 2.0, 1.0])
    rng = _rng(3)
    U, _ = np.linalg.qr(rng.standard_normal((9, 5)))
    V, _ = np.linalg.qr(rng.standard_normal((7, 5)))
    X = U @ np.diag(s) @ V.T
    for eps, k in ((0.9, 1), (0.74, 1), (0.73, 2), (0.51, 2), (0.50, 3), (0.31, 3), (0.30, 4),
                   (0.14, 4), (0.13, 5), (1e-10, 5)):
        assert O.eps_rank(X, eps) == k, (eps, k)
        assert O.eps_rank(X.T, eps) == k
        assert O.eps_rank(3.5 * X, eps) == k


def test_eps_rank_matches_truncation_error():
    # Eckart-Young: the rule's tail ratio is the relative Frobenius error of the best
    # rank-k truncation; check the chosen k against explicit truncations.
    X = _nonneg(12, 20, 5)
    U, s, Vt = np.linalg.svd(X, full_matrices=False)
    nx = np.linalg.norm(X)
    for eps in (0.3, 0.1, 0.05, 0.01):
        k = O.eps_rank(X, eps)
        err = lambda j: np.linalg.norm(X - (U[:, :j] * s[:j]) @ Vt[:j]) / nx
        assert err(k) <= eps + 1e-12
        if k > 1:
            assert err(k - 1) > eps


def test_eps_rank_of_exact_low_rank_and_zero():
    rng = _rng(8)
    X = rng.random((15, 3)) @ rng.random((3, 40))
    assert O.eps_rank(X, 1e-8) == 3
    assert O.eps_rank(np.zeros((4, 6)), 0.1) == 1


def test_sweep_rank_rule_recovers_generating_rank_of_first_unfolding():
    # a noise-free TT tensor with ranks (1, 3, 4, 1): the first unfolding has rank 3
    A = S.contract_cores(S.random_cores((6, 7, 8), (1, 3, 4, 1), seed=12)).astype(np.float64)
    res = O.ntt_decompose(A, (1, 32, 32, 1), 30, seed=1, rank_eps=1e-5)
    assert res["ranks"][1] == 3
    assert res["ranks"][2] <= min(3 * 7, 8)
    assert [c.shape for c in res["cores"]] == [(1, 6, 3), (3, 7, res["ranks"][2]), (res["ranks"][2], 8, 1)]
    # a rank cap below the rule's choice wins
    res2 = O.ntt_decompose(A, (1, 2, 32, 1), 5, seed=1, rank_eps=1e-5)
    assert res2["ranks"][1] == 2


def test_gram_identity_equals_explicit_residual():
    X = _nonneg(15, 22, 8)
    W, H = _rng(9).random((15, 4)), _rng(10).random((4, 22))
    f_gram = 0.5 * (np.sum(X * X) - 2 * np.sum((W.T @ X) * H) + np.sum((W.T @ W) * (H @ H.T)))
    assert math.isclose(O.objective(X, W, H), f_gram, rel_tol=1e-10)


# ------------------------------------------------------------------ the sweep
def test_sweep_d2_is_a_single_nmf():
    X = _nonneg(12, 10, 11).astype(np.float32)
    res = O.ntt_decompose(X, [1, 3, 1], 30, seed=4)
    W0, H0 = O.init_factors(4, 1, 12, 3, 10)
    ref = O.mu_nmf(X.astype(np.float64), W0, H0, 30)
    np.testing.assert_array_equal(res["cores"][0].reshape(12, 3), ref["W"])
    np.testing.assert_array_equal(res["cores"][1].reshape(3, 10), ref["H"])


def test_sweep_shapes_and_nonnegativity():
    dims, ranks = (4, 5, 3, 6), (1, 3, 4, 2, 1)
    A = S.contract_cores(S.random_cores(dims, ranks, seed=5))
    res = O.ntt_decompose(A, ranks, 20, seed=1)
    r = res["ranks"]
    for k, G in enumerate(res["cores"]):
        assert G.shape == (r[k], dims[k], r[k + 1])
        assert G.min() >= 0
    # stage l factors the (r_{l-1} n_l) x (n_{l+1}...n_d) unfolding of the previous H
    st = res["stages"]
    assert (st[0]["m"], st[0]["k"]) == (4, 90)
    assert (st[1]["m"], st[1]["k"]) == (15, 18)
    assert (st[2]["m"], st[2]["k"]) == (12, 6)
    np.testing.assert_array_equal(st[1]["X"], st[0]["H"].reshape(15, 18))


def test_sweep_rank1_matches_tt_svd_rank1():
    # With all TT ranks 1 the nTT of a positive tensor and the rank-1 TT-SVD coincide at
    # convergence (each stage is the leading singular pair, which is non-negative).
    dims = (5, 4, 6)
    A = _rng(12).random(dims) + 0.2
    res = O.ntt_decompose(A, [1, 1, 1, 1], 3000, seed=2)
    e_ntt = O.rel_error(A, O.tt_reconstruct(res["cores"]))
    # TT-SVD at ranks 1
    X = A.reshape(5, -1)
    U, s, Vt = np.linalg.svd(X, full_matrices=False)
    G1 = U[:, :1] * s[0]
    R = Vt[:1].reshape(4, 6)
    U2, s2, Vt2 = np.linalg.svd(R, full_matrices=False)
    Ahat = np.einsum("a,b,c->abc", G1[:, 0], U2[:, 0] * s2[0], Vt2[0])
    e_svd = O.rel_error(A, Ahat)
    assert abs(e_ntt - e_svd) < 1e-8


def test_sweep_near_exact_recovery_improves_with_iterations():
    # Noise-free TT-generated data has an exact non-negative TT at the true ranks; MU
    # must keep lowering the error.  (How low it gets is calibrated, not pinned.)
    w = S.workload("tt16x3_r4")
    A = w.tensor()
    errs = []
    for T in (20, 100, 400):
        res = O.ntt_decompose(A, w.target_ranks, T, seed=w.seed)
        errs.append(O.rel_error(A, O.tt_reconstruct(res["cores"])))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 0.05


@pytest.mark.parametrize("f,nx,tol,K,first_stop", [
    # ||X|| = 1 keeps the residual test off (sqrt(2 f) > 0.25 for every f here).  K = 2:
    # the fall 200 -> 80 is large; 80 -> 60 is exactly tol * f_{t-K} = 20 (tol = 0.25),
    # and the rule stops on equality, at t = 4
    ([200.0, 150.0, 80.0, 70.0, 60.0, 5.0], 1.0, 0.25, 2, 4),
    # the same with f_4 one unit in the last place below 60: the fall is 20 + 2^-47, no
    # stop at t = 4; 60 -> 50 at t = 6 is within 15
    ([200.0, 150.0, 80.0, 70.0, float(np.nextafter(60.0, 0.0)), 55.0, 50.0], 1.0, 0.25, 2, 6),
    # relative residual sqrt(2 f)/||X|| = 1/4 exactly at t = 3 (f = 0.5, ||X|| = 4):
    # stops on equality although the objective still falls fast
    ([800.0, 200.0, 50.0, 0.5], 4.0, 0.25, 1, 3),
    # f just above 0.5: the residual test fails, the fall from 50 to 0.50000001 is large
    ([800.0, 200.0, 50.0, 0.5 + 1e-8, 0.5 + 1e-8], 4.0, 0.25, 1, 4),
    # checks only at multiples of K = 3: the flat stretch at t = 1, 2 is not seen; the
    # fall 5 -> 4.6 at t = 6 is within tol * 5 = 0.5
    ([10.0, 10.0, 10.0, 5.0, 4.8, 4.7, 4.6], 1e-3, 0.1, 3, 6),
])
def test_stop_rule_hand_built_objective_sequences(f, nx, tol, K, first_stop):
    # sequences whose first stop is worked out by hand (the rule of a tolerance budget:
    # at t % K == 0, sqrt(2 f_t)/||X|| <= tol, or f_{t-K} - f_t <= tol f_{t-K}); swapping
    # f_t and f_{t-K}, or < for <=, moves the first stop
    stops = [t for t in range(1, len(f)) if O.stop_now(f, t, nx, tol, K)]
    assert stops and stops[0] == first_stop
    assert not O.stop_now(f, first_stop, nx, 0.0, K)  # tol = 0: fixed iteration count


def test_stop_rule_on_tolerance():
    X = _nonneg(20, 30, 13)
    W0, H0 = O.init_factors(1, 1, 20, 3, 30)
    full = O.mu_nmf(X, W0, H0, 500, record_objective=True)
    res = O.mu_nmf(X, W0, H0, 500, tol=1e-3, check_every=10)
    t = res["iters"]
    assert t % 10 == 0 and 10 <= t < 500
    f = full["objective"]
    # the rule holds at t and not at any earlier check point
    def holds(s):
        return (math.sqrt(2 * f[s]) / full["norm_x"] <= 1e-3) or (f[s - 10] - f[s] <= 1e-3 * f[s - 10])
    assert holds(t)
    assert not any(holds(s) for s in range(10, t, 10))
    np.testing.assert_array_equal(res["W"], O.mu_nmf(X, W0, H0, t)["W"])


# ------------------------------------------------------------------ BCD NMF (Alg.3)
def _f(X, W, H):
    R = X - W @ H
    return 0.5 * float(np.sum(R * R))


def test_bcd_rank1_W_step_is_the_nnls_closed_form():
    # r = 1: the Frobenius norm of h h^T is |h|^2, the exact Lipschitz constant, and the
    # block problem separates by rows, so one step solves it: w_i = max(0, <x_i, h>/|h|^2)
    # whatever the starting point
    rng = _rng(40)
    X = rng.random((7, 9)) - 0.3
    h = rng.random((1, 9))
    Wm = rng.random((7, 1)) * 5.0 - 2.0
    W, L = O.bcd_step_W(X @ h.T, h @ h.T, Wm)
    hh = sum(h[0, j] * h[0, j] for j in range(9))
    for i in range(7):
        xh = sum(X[i, j] * h[0, j] for j in range(9))
        assert W[i, 0] == pytest.approx(max(0.0, xh / hh), rel=1e-12, abs=1e-14)
    assert L == pytest.approx(hh, rel=1e-14)


def _fd_grad(fun, M, h=1e-3):
    G = np.zeros_like(M)
    for idx in np.ndindex(*M.shape):
        P = M.copy(); P[idx] += h
        Q = M.copy(); Q[idx] -= h
        G[idx] = (fun(P) - fun(Q)) / (2.0 * h)  # exact for a quadratic up to rounding
    return G


def test_bcd_block_steps_are_projected_gradient_steps():
    rng = _rng(41)
    m, r, k = 6, 3, 8
    X = rng.random((m, k))
    W = rng.random((m, r))
    H = rng.random((r, k))
    Wm = W + 0.4 * (rng.random((m, r)) - 0.5)  # an extrapolated point, some entries < 0
    Hm = H + 0.4 * (rng.random((r, k)) - 0.5)
    Wn, LW = O.bcd_step_W(X @ H.T, H @ H.T, Wm)
    GW = _fd_grad(lambda A: _f(X, A, H), Wm)
    lam = np.linalg.eigvalsh(H @ H.T).max()
    assert lam * (1 - 1e-12) <= LW <= math.sqrt(r) * lam * (1 + 1e-12)
    assert np.allclose(Wn, np.maximum(0.0, Wm - GW / LW), rtol=1e-8, atol=1e-10)
    Hn, LH = O.bcd_step_H(W.T @ X, W.T @ W, Hm)
    GH = _fd_grad(lambda B: _f(X, W, B), Hm)
    lam = np.linalg.eigvalsh(W.T @ W).max()
    assert lam * (1 - 1e-12) <= LH <= math.sqrt(r) * lam * (1 + 1e-12)
    assert np.allclose(Hn, np.maximum(0.0, Hm - GH / LH), rtol=1e-8, atol=1e-10)
    # each block step from the current point does not increase the objective
    assert _f(X, O.bcd_step_W(X @ H.T, H @ H.T, W)[0], H) <= _f(X, W, H)
    assert _f(X, W, O.bcd_step_H(W.T @ X, W.T @ W, H)[0]) <= _f(X, W, H)


def test_bcd_init_is_scaled_to_root_norm_of_X():
    rng = _rng(42)
    X = rng.random((20, 30)) * 3.0
    W0, H0 = rng.random((20, 4)), rng.random((4, 30))
    res = O.bcd_nmf(X, W0, H0, 0)
    nx = math.sqrt(float(np.sum(X * X)))
    assert math.sqrt(float(np.sum(res["W"] ** 2))) == pytest.approx(math.sqrt(nx), rel=1e-12)
    assert math.sqrt(float(np.sum(res["H"] ** 2))) == pytest.approx(math.sqrt(nx), rel=1e-12)
    # directions are those of the random factors
    assert np.allclose(res["W"] / W0, (res["W"] / W0)[0, 0], rtol=1e-12)


def test_bcd_without_extrapolation_is_monotone_and_never_corrects():
    rng = _rng(43)
    X = rng.random((20, 30))
    res = O.bcd_nmf(X, rng.random((20, 3)), rng.random((3, 30)), 100, delta=0.0)
    assert res["corrections"] == 0
    f = res["objective"]
    assert f[0] < 0.5 * float(np.sum(X * X))
    assert np.all(np.diff(f) < 0.0)


def test_bcd_extrapolation_sequence():
    # while every pair is kept, t follows the accelerated-gradient sequence: t_1 is the
    # golden ratio, t_k >= (k + 2) / 2, and the weights w = (t_{k-1} - 1) / t_k grow from 0
    # towards 1
    rng = _rng(44)
    W, H = rng.random((30, 3)), rng.random((3, 40))
    X = W @ H
    res = O.bcd_nmf(X, rng.random((30, 3)), rng.random((3, 40)), 30)
    n = res["kept"].index(False) if False in res["kept"] else len(res["kept"])
    assert n >= 10
    t, w = res["t"][:n], res["w"][:n]
    assert t[0] == pytest.approx((1 + math.sqrt(5)) / 2, rel=1e-15)
    assert all(t[k] >= (k + 3) / 2 for k in range(len(t)))
    assert w[0] == 0.0 and np.all(np.diff(w) > 0) and w[-1] < 1.0


def test_bcd_correction_returns_to_the_last_kept_pair():
    A = S.workload("tt16x3_r4").tensor().astype(np.float64)
    X = A.reshape(16, 256)
    W0, H0 = O.init_factors(0, 1, 16, 4, 256)
    full = O.bcd_nmf(X, W0, H0, 200)
    c = full["kept"].index(False) + 1  # first dropped iteration (1-based)
    res = O.bcd_nmf(X, W0, H0, c + 1, snapshots=(c - 1, c, c + 1))
    Wb, Hb = res["snaps"][c - 1]
    Wc, Hc = res["snaps"][c]
    assert np.array_equal(Wb, Wc) and np.array_equal(Hb, Hc)
    assert res["objective"][c - 1] >= _f(X, Wb, Hb)  # the dropped candidate was no better
    # the next iteration is a plain (unextrapolated) step from the kept pair, W
    # normalised to unit entrywise L1 norm before the H step
    Wn = O.bcd_normalise_l1(O.bcd_step_W(X @ Hb.T, Hb @ Hb.T, Wb)[0])
    Hn, _ = O.bcd_step_H(Wn.T @ X, Wn.T @ Wn, Hb)
    assert res["objective"][c] == pytest.approx(_f(X, Wn, Hn), rel=1e-12)
    if res["kept"][c]:
        assert np.allclose(res["snaps"][c + 1][0], Wn, rtol=1e-12, atol=0)


def test_bcd_recovers_an_exact_nonnegative_factorisation():
    rng = _rng(45)
    W, H = rng.random((30, 3)), rng.random((3, 40))
    X = W @ H
    res = O.bcd_nmf(X, rng.random((30, 3)), rng.random((3, 40)), 800)
    err = math.sqrt(2.0 * _f(X, res["W"], res["H"])) / math.sqrt(float(np.sum(X * X)))
    assert err < 1e-4


def test_bcd_sweep_reaches_lower_error_than_mu():
    # the comparison of the paper's 500 GB experiment (Sec. V, Fig. 8c): at the same ranks
    # BCD reaches a lower reconstruction error than MU
    A = S.workload("tt16x3_r4").tensor()
    e = {}
    for nmf in ("mu", "bcd"):
        res = O.ntt_decompose(A, (1, 4, 4, 1), 200, nmf=nmf)
        e[nmf] = O.rel_error(A, O.tt_reconstruct(res["cores"]))
    assert e["bcd"] < 0.5 * e["mu"]


def test_bcd_extrapolation_weights_are_capped_by_the_gram_norm_ratios():
    # with a small delta the caps bind: every applied weight is min(w, delta sqrt(ratio))
    # with the ratio of the partner block's Gram norms at the two last kept iterates,
    # recomputed here from the snapshots; and each next candidate is the block steps
    # from the points extrapolated with those weights
    rng = _rng(46)
    X = rng.random((25, 40))
    W0, H0 = rng.random((25, 4)), rng.random((4, 40))
    T, delta = 12, 0.1
    res = O.bcd_nmf(X, W0, H0, T, delta=delta, snapshots=tuple(range(T + 1)))
    assert all(res["kept"])
    fro = lambda M: math.sqrt(float(np.sum(M * M)))
    binding = 0
    for it in range(2, T + 1):  # weights chosen after iteration it (iterates it-1 -> it)
        Wa, Ha = res["snaps"][it - 1]
        Wb, Hb = res["snaps"][it]
        w = res["w"][it - 1]
        capW = delta * math.sqrt(fro(Ha @ Ha.T) / fro(Hb @ Hb.T))
        capH = delta * math.sqrt(fro(Wa.T @ Wa) / fro(Wb.T @ Wb))
        assert res["wW"][it - 1] == pytest.approx(min(w, capW), rel=1e-12)
        assert res["wH"][it - 1] == pytest.approx(min(w, capH), rel=1e-12)
        binding += (capW < w) + (capH < w)
        if it < T:  # the candidate of iteration it + 1 starts from the extrapolated points
            Wm = Wb + res["wW"][it - 1] * (Wb - Wa)
            Hm = Hb + res["wH"][it - 1] * (Hb - Ha)
            Wn = O.bcd_normalise_l1(O.bcd_step_W(X @ Hb.T, Hb @ Hb.T, Wm)[0])
            Hn, _ = O.bcd_step_H(Wn.T @ X, Wn.T @ Wn, Hm)
            assert res["objective"][it] == pytest.approx(_f(X, Wn, Hn), rel=1e-12)
    assert binding > 0


def test_bcd_W_has_unit_l1_norm_after_every_kept_step():
    # Alg.3's W block ends with W /= ||W||_1: every kept W (after the first kept
    # iteration) sums to 1; without the step (normalise=None) it does not
    rng = _rng(47)
    X = rng.random((24, 35)) * 4.0
    W0, H0 = rng.random((24, 3)), rng.random((3, 35))
    T = 40
    res = O.bcd_nmf(X, W0, H0, T, snapshots=tuple(range(1, T + 1)))
    first = res["kept"].index(True) + 1
    for t in range(first, T + 1):
        W = res["snaps"][t][0]
        assert abs(sum(float(v) for v in W.ravel()) - 1.0) <= 1e-12, t
        assert W.min() >= 0.0
    plain = O.bcd_nmf(X, W0, H0, T, normalise=None)
    assert abs(float(np.sum(plain["W"])) - 1.0) > 1e-3


def test_bcd_one_iteration_rank1_hand_worked():
    # X = [[1, 2, 3], [2, 4, 6]] = (1, 2)^T (1, 2, 3).  At r = 1 both block steps are
    # exact non-negative least squares (the Frobenius norm of a 1 x 1 Gram is the exact
    # Lipschitz constant), so from any positive start one iteration gives:
    #   W step: w_i = <x_i, h>/|h|^2, proportional to (1, 2) (the rows of X are);
    #   L1 normalisation: w = (1/3, 2/3);
    #   H step: h_j = <w, x_j>/|w|^2 = (5/3, 10/3, 5) / (5/9) = (3, 6, 9);
    # so W H = X, objective 0 < 1/2 ||X||^2 = 35: the pair is kept.
    X = np.array([[1.0, 2.0, 3.0], [2.0, 4.0, 6.0]])
    res = O.bcd_nmf(X, np.array([[0.7], [0.2]]), np.array([[0.5, 0.9, 0.1]]), 1)
    assert res["kept"] == [True]
    assert np.allclose(res["W"], [[1.0 / 3.0], [2.0 / 3.0]], rtol=1e-14, atol=0)
    assert np.allclose(res["H"], [[3.0, 6.0, 9.0]], rtol=1e-13, atol=0)
    assert res["objective"][0] <= 1e-24


def test_bcd_one_iteration_rank1_by_explicit_loops():
    # the first iteration of Alg.3 at r = 1 on a random non-negative matrix, written out
    # with loops: the B5 scaling, the exact NNLS W step, the L1 normalisation, the exact
    # NNLS H step of the normalised W, and the kept decision against 1/2 ||X||^2
    rng = _rng(48)
    m, k = 5, 7
    X = rng.random((m, k))
    w0, h0 = rng.random(m), rng.random(k)
    nx = math.sqrt(sum(X[i, j] ** 2 for i in range(m) for j in range(k)))
    nw = math.sqrt(sum(v * v for v in w0))
    nh = math.sqrt(sum(v * v for v in h0))
    h = [v / nh * math.sqrt(nx) for v in h0]
    hh = sum(v * v for v in h)
    w = [max(0.0, sum(X[i, j] * h[j] for j in range(k)) / hh) for i in range(m)]
    s1 = sum(w)
    w = [v / s1 for v in w]
    ww = sum(v * v for v in w)
    hn = [max(0.0, sum(w[i] * X[i, j] for i in range(m)) / ww) for j in range(k)]
    f = 0.5 * sum((X[i, j] - w[i] * hn[j]) ** 2 for i in range(m) for j in range(k))
    res = O.bcd_nmf(X, w0.reshape(m, 1), h0.reshape(1, k), 1)
    assert res["kept"] == [f < 0.5 * nx * nx]
    assert np.allclose(res["W"][:, 0], w, rtol=1e-12, atol=0)
    assert np.allclose(res["H"][0], hn, rtol=1e-12, atol=0)
    assert res["objective"][0] == pytest.approx(f, rel=1e-12)
    assert nw > 0
