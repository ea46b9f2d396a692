"""CPU FP64 oracle of the non-negative tensor-train (nTT) sweep.

TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and the CPU-baseline
leg of the benchmark may import this module.  The GPU library never calls it,
and it shares no code with the GPU library: it is a plain, slow, obviously
correct restatement of what the paper computes, in float64.

What it follows
---------------
* Eq.(1)-(2), TT format: A[i_1..i_d] = sum_k G1[i_1,k_1] G2[k_1,i_2,k_2] ... Gd[k_{d-1},i_d].
* Alg.2 (distnTT), one process: X_1 = reshape(A, n_1 x n_2...n_d); for each stage l,
  X_l is (r_{l-1} n_l) x (n_{l+1}...n_d) (the reading of the text under Alg.2), it is
  factored by NMF into W (m x r_l) and H (r_l x k); core l = reshape(W, r_{l-1} x n_l x r_l)
  and the next unfolding is reshape(H, r_l n_{l+1} x ...).  The last core is H.
* NMF by multiplicative updates (MU), the method the experiments time (Sec. IV-B,
  IV-C): the paper names MU and the Frobenius objective but prints no rule, so this
  is the Lee-Seung rule for min 1/2 ||X - W H||_F^2 with W, H >= 0, H updated first:
      H <- max(0, H * (W^T X) / ((W^T W) H + eps))
      W <- max(0, W * (X H^T) / (W (H H^T) + eps))
* NMF by Alg.3 (``bcd_nmf``): projected-gradient block steps, W then H, from
  extrapolated points, with the objective test keeping or dropping each new pair;
  the readings of the garbled listing are B1-B8 at that section.
* Objective 1/2 ||X - W H||_F^2 (Alg.3, the correction test), computed here as the
  explicit residual, never by the Gram identity.
* Eq.(3) relative error, Eq.(4) compression ratio.
* The rank rule of Alg.2 (``eps_rank``): r_l is the smallest k whose singular-value
  tail ratio of the current unfolding is at most the threshold; used when a threshold
  is given, else the ranks are given.

Readings where the paper is silent or garbled (given ranks are caps of the rule;
ranks above min(m, k) are clamped; a fresh random stream per stage; the stopping
rule) are stated at each function.

Random initial factors use the SplitMix64 counter rule (Steele, Lea and Flood,
OOPSLA 2014), implemented here on its own: value i of stream tag under seed is the
SplitMix64 finaliser applied to seed + GAMMA * (tag * 2^32 + i + 1), and a uniform is
its top 24 bits times 2^-24.  W of stage l uses tag 2l, H uses tag 2l + 1.

parity pinned: every function here is checked by the CPU tests against closed forms,
brute force, invariants or numbers printed in the paper.  The one calibrated (not
pinned) quantity is how low the relative error gets at the true ranks after T
iterations; only its monotone decrease is pinned.
"""
from __future__ import annotations

import itertools
import math

import numpy as np

GAMMA = 0x9E3779B97F4A7C15
M64 = (1 << 64) - 1


# ---------------------------------------------------------------- random init
def splitmix64_at(seed: int, counter: int) -> int:
    """SplitMix64 finaliser applied to seed + GAMMA * counter (pure Python ints)."""
    z = (seed + GAMMA * counter) & M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def rng_uniform(seed: int, tag: int, count: int) -> np.ndarray:
    """Uniforms on [0,1) of stream ``tag``: u_i = (z_i >> 40) / 2^24 (float64, FP32-exact)."""
    seed &= M64
    ctr = np.uint64((tag << 32) & M64) + np.arange(1, count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + np.uint64(GAMMA) * ctr
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return (z >> np.uint64(40)).astype(np.float64) / float(1 << 24)


def init_factors(seed: int, stage: int, m: int, r: int, k: int):
    """Random W0 (m x r) and H0 (r x k), uniform on [0,1) (Alg.3 'rand' init, no rescaling).

    Stage ``stage`` is 1-based; W uses stream 2*stage, H stream 2*stage + 1, entries in C order.
    """
    w = rng_uniform(seed, 2 * stage, m * r).reshape(m, r)
    h = rng_uniform(seed, 2 * stage + 1, r * k).reshape(r, k)
    return w, h


# ---------------------------------------------------------------- ranks, Eq.(4)
def effective_ranks(dims, ranks):
    """Clamp r_l to min(r_l, r_{l-1} n_l, n_{l+1}...n_d), left to right (TT-SVD convention).

    The paper chooses r_l by the SVD threshold rule (Alg.2); here ranks are given and
    an infeasible one is lowered to the largest rank the unfolding can hold.
    """
    d = len(dims)
    out = [1]
    for l in range(1, d):
        m = out[-1] * dims[l - 1]
        k = int(np.prod(dims[l:], dtype=np.int64))
        out.append(int(min(ranks[l], m, k)))
    out.append(1)
    return out


def compression_ratio(dims, ranks) -> float:
    """Eq.(4): prod n_i / sum n_i r_{i-1} r_i."""
    num = 1
    for n in dims:
        num *= int(n)
    den = sum(int(dims[i]) * int(ranks[i]) * int(ranks[i + 1]) for i in range(len(dims)))
    return num / den


# ---------------------------------------------------------------- NMF by MU
def objective(X, W, H) -> float:
    """1/2 ||X - W H||_F^2 as the explicit residual."""
    R = X - W @ H
    return 0.5 * float(np.sum(R * R))


def update_H(X, W, H, eps):
    """The H half of a MU iteration.  Column j of the result depends only on column j
    of X and of H, so it may be applied to any subset of the columns."""
    return np.maximum(0.0, H * (W.T @ X) / ((W.T @ W) @ H + eps))


def update_W(XHt, HHt, W, eps):
    """The W half of a MU iteration, from the products X H^T (m x r) and H H^T (r x r)
    of the already updated H; X enters only through X H^T."""
    return np.maximum(0.0, W * XHt / (W @ HHt + eps))


def mu_step(X, W, H, eps):
    """One Lee-Seung MU iteration, H first then W, with max(0, .) and additive eps."""
    H = update_H(X, W, H, eps)
    W = update_W(X @ H.T, H @ H.T, W, eps)
    return W, H


def stop_now(f_hist, t, nx, tol, check_every) -> bool:
    """Stopping test at t % K == 0 (used only when tol > 0).

    Stop when the relative residual sqrt(2 f_t)/||X|| <= tol, or when the objective
    fell by no more than tol * f_{t-K} over the last K iterations.  (The paper runs a
    fixed iteration count; this rule is the reading used for a tolerance budget.)
    """
    if tol <= 0 or t % check_every != 0:
        return False
    f_t = f_hist[t]
    f_prev = f_hist[t - check_every]
    if math.sqrt(2.0 * max(f_t, 0.0)) / nx <= tol:
        return True
    return (f_prev - f_t) <= tol * f_prev


def mu_nmf(X, W0, H0, iters, eps=1e-12, tol=0.0, check_every=10,
           record_objective=False, snapshots=(), objective_at=()):
    """NMF of X by MU from (W0, H0); returns a dict with W, H, iters, objective, snaps.

    ``objective[t]`` is the explicit objective after t full iterations (index 0 = init),
    filled when ``record_objective`` or ``tol > 0``.  ``snaps[t] = (W_t, H_t)`` for t in
    ``snapshots``; ``objective_at_t[t]`` is the explicit objective after t iterations for
    t in ``objective_at`` (the same quantity as ``objective[t]``, only at chosen t).
    """
    X = np.asarray(X, dtype=np.float64)
    W = np.array(W0, dtype=np.float64)
    H = np.array(H0, dtype=np.float64)
    want_obj = record_objective or tol > 0
    nx = math.sqrt(float(np.sum(X * X)))
    f_hist = [objective(X, W, H)] if want_obj else []
    snaps, f_at = {}, {}
    if 0 in snapshots:
        snaps[0] = (W.copy(), H.copy())
    t_done = 0
    for t in range(1, iters + 1):
        W, H = mu_step(X, W, H, eps)
        t_done = t
        if want_obj:
            f_hist.append(objective(X, W, H))
        if t in objective_at:
            f_at[t] = f_hist[t] if want_obj else objective(X, W, H)
        if t in snapshots:
            snaps[t] = (W.copy(), H.copy())
        if want_obj and stop_now(f_hist, t, nx, tol, check_every):
            break
    return {"W": W, "H": H, "iters": t_done, "objective": np.array(f_hist),
            "snaps": snaps, "objective_at_t": f_at, "norm_x": nx}


# ---------------------------------------------------------------- NMF by BCD (Alg.3)
# Alg.3 minimises the same objective by alternating projected-gradient steps on the
# two blocks (W first, then H), each from an extrapolated point, with the objective
# test deciding whether the new pair is kept ("extrapolation") or dropped
# ("correction").  Readings of the listing, where it is garbled or silent:
#   B1  the W step subtracts the scaled gradient, W = max(0, W_m - G_W / L_W), as the
#       H step of the listing does (the W line prints no G_W term);
#   B2  the step sizes are 1/L with L_W = ||H H^T||_F and L_H = ||W^T W||_F (the H line's
#       square root is read as this norm; the Frobenius norm bounds the spectral norm,
#       the Lipschitz constant of the block gradient, from above, so every plain step
#       descends); a zero L takes no gradient step (the block is only projected);
#   B3  after each W step, W is divided by its entrywise L1 norm, the sum of its entries
#       (W >= 0 after the projection), as the W block of the listing prints; the W^T W
#       and the H step that follow use the normalised W, so H absorbs the scale; a zero
#       W is left as it is.  ``normalise=None`` drops this step (an earlier reading of
#       the listing, kept for comparison only);
#   B4  the starting objective is 1/2 ||X||_F^2 (the objective at W = H = 0; the
#       listing prints ||X|| without the square);
#   B5  the random factors are scaled to ||W||_F = ||H||_F = sqrt(||X||_F) and form the
#       first iterate and also its "previous" iterate;
#   B6  a correction returns to the last kept pair (with its X H^T and H H^T) and the
#       next iteration starts from it without extrapolation; t and the objective are
#       unchanged (a random restart would throw away all progress);
#   B7  w = (t - 1) / t+ with t+ = (1 + sqrt(1 + 4 t^2)) / 2; the caps compare the
#       Gram norms of the partner block at the two last kept iterates,
#       w_W = min(w, delta sqrt(||H_{l-1} H_{l-1}^T||_F / ||H_l H_l^T||_F)),
#       w_H = min(w, delta sqrt(||W_{l-1}^T W_{l-1}||_F / ||W_l^T W_l||_F)),
#       a zero denominator leaving w; delta (a user parameter) defaults to 0.9999;
#   B8  the result is the last kept pair; the objective of the test is the explicit
#       residual 1/2 ||X - W H||_F^2.
def bcd_lipschitz(G) -> float:
    """B2: the step constant of a block, the Frobenius norm of its r x r Gram."""
    return math.sqrt(float(np.sum(np.asarray(G, dtype=np.float64) ** 2)))


def bcd_step_W(XHt, HHt, Wm):
    """The W block step of Alg.3 (B1, B2) from the extrapolated W_m, given X H^T and
    H H^T of the kept H.  Returns (W, L_W)."""
    L = bcd_lipschitz(HHt)
    if L == 0.0:
        return np.maximum(0.0, Wm), L
    return np.maximum(0.0, Wm - (Wm @ HHt - XHt) / L), L


def bcd_normalise_l1(W):
    """B3: W divided by its entrywise L1 norm (the sum of |w_ij|); a zero W is returned
    unchanged."""
    s = float(np.sum(np.abs(W)))
    return W / s if s > 0.0 else W


def bcd_step_H(WtX, WtW, Hm):
    """The H block step of Alg.3 (B2) from the extrapolated H_m, given W^T X and W^T W of
    the new W.  Column j of the result depends only on column j of W^T X and H_m.
    Returns (H, L_H)."""
    L = bcd_lipschitz(WtW)
    if L == 0.0:
        return np.maximum(0.0, Hm), L
    return np.maximum(0.0, Hm - (WtW @ Hm - WtX) / L), L


def bcd_normalise(X, W0, H0):
    """B5: scale the random factors to Frobenius norm sqrt(||X||_F) (a zero factor is
    left as it is)."""
    nx = math.sqrt(float(np.sum(np.asarray(X, dtype=np.float64) ** 2)))
    W = np.array(W0, dtype=np.float64)
    H = np.array(H0, dtype=np.float64)
    nw = math.sqrt(float(np.sum(W * W)))
    nh = math.sqrt(float(np.sum(H * H)))
    if nw > 0.0:
        W = W / nw * math.sqrt(nx)
    if nh > 0.0:
        H = H / nh * math.sqrt(nx)
    return W, H


def bcd_nmf(X, W0, H0, iters, delta=0.9999, snapshots=(), normalise="l1"):
    """NMF of X by Alg.3 (BCD with extrapolation and correction) from (W0, H0).

    ``normalise="l1"`` (the listing) divides every new W by its entrywise L1 norm before
    the H step (B3); ``None`` leaves it out.

    Returns a dict with the kept pair W, H, ``corrections`` (how many iterations were
    dropped), ``kept`` (per iteration: True when kept), ``objective`` (the objective of
    each iteration's candidate pair, kept or not), ``t`` and ``w`` (the extrapolation
    sequence after each iteration), ``wW`` and ``wH`` (the weights the next iteration
    extrapolates with), and ``snaps[t] = (W, H)`` after t iterations.
    """
    X = np.asarray(X, dtype=np.float64)
    W, H = bcd_normalise(X, W0, H0)
    Wp, Hp = W, H
    Wm, Hm = W, H
    HHt, XHt = H @ H.T, X @ H.T
    gH, gW = bcd_lipschitz(HHt), bcd_lipschitz(W.T @ W)
    t = 1.0
    obj = 0.5 * float(np.sum(X * X))  # B4
    snaps = {}
    if 0 in snapshots:
        snaps[0] = (W.copy(), H.copy())
    kept, f_hist, t_hist, w_hist, ww_hist, wh_hist = [], [], [], [], [], []
    for it in range(1, iters + 1):
        Wn, _ = bcd_step_W(XHt, HHt, Wm)
        if normalise == "l1":
            Wn = bcd_normalise_l1(Wn)
        WtW = Wn.T @ Wn
        Hn, LH = bcd_step_H(Wn.T @ X, WtW, Hm)
        f = objective(X, Wn, Hn)
        f_hist.append(f)
        if f >= obj:  # correction (B6)
            kept.append(False)
            Wm, Hm = W, H
            w = wW = wH = 0.0
        else:  # extrapolation (B7)
            kept.append(True)
            tp = 0.5 * (1.0 + math.sqrt(1.0 + 4.0 * t * t))
            w = (t - 1.0) / tp
            HHn = Hn @ Hn.T
            gHn, gWn = bcd_lipschitz(HHn), LH
            wW = min(w, delta * math.sqrt(gH / gHn)) if gHn > 0.0 else w
            wH = min(w, delta * math.sqrt(gW / gWn)) if gWn > 0.0 else w
            Wp, Hp, W, H = W, H, Wn, Hn
            HHt, XHt = HHn, X @ Hn.T
            gH, gW = gHn, gWn
            Wm = W + wW * (W - Wp)
            Hm = H + wH * (H - Hp)
            t, obj = tp, f
        t_hist.append(t)
        w_hist.append(w)
        ww_hist.append(wW)
        wh_hist.append(wH)
        if it in snapshots:
            snaps[it] = (W.copy(), H.copy())
    return {"W": W, "H": H, "iters": iters, "corrections": kept.count(False), "kept": kept,
            "objective": np.array(f_hist), "t": np.array(t_hist), "w": np.array(w_hist),
            "wW": np.array(ww_hist), "wH": np.array(wh_hist),
            "snaps": snaps, "norm_x": math.sqrt(float(np.sum(X * X)))}


# ---------------------------------------------------------------- rank selection
def eps_rank(X, eps) -> int:
    """The rank rule of Alg.2: the smallest k >= 1 such that
    sqrt(s_{k+1}^2 + ... + s_N^2) / sqrt(s_1^2 + ... + s_N^2) <= eps, where s_1 >= s_2 >= ...
    are the singular values of X and N = min(m, n).  A zero matrix gets rank 1.  The tail
    sums are added from the smallest value up (no cancellation)."""
    s = np.linalg.svd(np.asarray(X, dtype=np.float64), compute_uv=False)
    s2 = s * s
    total = float(np.sum(s2[::-1]))
    if total == 0.0:
        return 1
    tails = np.concatenate([np.cumsum(s2[::-1])[::-1][1:], [0.0]])  # tails[k-1] = sum_{i>k} s_i^2
    for k in range(1, len(s2) + 1):
        if math.sqrt(tails[k - 1] / total) <= eps:
            return k
    return len(s2)


# ---------------------------------------------------------------- the nTT sweep
def ntt_decompose(A, ranks, iters, eps=1e-12, seed=0, tol=0.0, check_every=10,
                  inits=None, record_objective=False, snapshots=(), rank_eps=0.0,
                  nmf="mu", delta=0.9999, bcd_normalise="l1", objective_at=()):
    """Alg.2 with MU (``nmf="mu"``) or Alg.3 (``nmf="bcd"``, fixed ``iters`` per stage,
    extrapolation cap ``delta``, W normalisation ``bcd_normalise`` as in ``bcd_nmf``) as
    the NMF: returns cores and per-stage details.

    ``A`` is the d-way tensor (converted to float64, C order).  ``ranks`` has d+1
    entries with r_0 = r_d = 1.  With ``rank_eps`` = 0 they are the TT ranks (clamped as
    in ``effective_ranks``); with ``rank_eps`` > 0 each inner rank is chosen at its stage
    by ``eps_rank`` of the current unfolding (Alg.2) and ``ranks`` only caps it.
    ``inits`` optionally maps stage l (1-based) to (W0, H0); otherwise the seeded
    uniform init of ``init_factors`` is used.  ``snapshots`` and ``objective_at`` (MU) are
    passed to every stage's NMF.
    """
    A = np.asarray(A, dtype=np.float64)
    dims = list(A.shape)
    d = len(dims)
    r = effective_ranks(dims, ranks)
    X = A.reshape(dims[0], -1)
    cores, stages = [], []
    for l in range(1, d):
        m, k = X.shape
        assert m == r[l - 1] * dims[l - 1]
        if rank_eps > 0.0:
            r[l] = min(r[l], eps_rank(X, rank_eps), m, k)
        rl = r[l]
        if inits is not None and l in inits:
            W0, H0 = inits[l]
        else:
            W0, H0 = init_factors(seed, l, m, rl, k)
        if nmf == "bcd":
            res = bcd_nmf(X, W0, H0, iters, delta, snapshots, bcd_normalise)
        else:
            res = mu_nmf(X, W0, H0, iters, eps, tol, check_every, record_objective, snapshots,
                         objective_at)
        res.update({"X": X, "W0": W0, "H0": H0, "m": m, "k": k, "r": rl})
        stages.append(res)
        cores.append(res["W"].reshape(r[l - 1], dims[l - 1], rl))
        H = res["H"]
        if l < d - 1:
            X = H.reshape(rl * dims[l], -1)
    cores.append(stages[-1]["H"].reshape(r[d - 1], dims[d - 1], 1))
    return {"cores": cores, "ranks": r, "stages": stages}


# ---------------------------------------------------------------- Eq.(1)-(3)
def tt_reconstruct(cores) -> np.ndarray:
    """Eq.(1): contract the cores left to right (last axis of the partial product
    against the first axis of the next core)."""
    dims = [c.shape[1] for c in cores]
    P = np.asarray(cores[0], dtype=np.float64).reshape(dims[0], -1)
    for G in cores[1:]:
        G = np.asarray(G, dtype=np.float64)
        P = P.reshape(-1, G.shape[0]) @ G.reshape(G.shape[0], -1)
    return P.reshape(dims)


def tt_element(cores, idx) -> float:
    """Eq.(2) for one entry: the explicit sum over k_1..k_{d-1} (pure Python loops)."""
    d = len(cores)
    rk = [c.shape[2] for c in cores[:-1]]
    total = 0.0
    for ks in itertools.product(*[range(r) for r in rk]):
        term = float(cores[0][0, idx[0], ks[0]])
        for j in range(1, d - 1):
            term *= float(cores[j][ks[j - 1], idx[j], ks[j]])
        term *= float(cores[d - 1][ks[d - 2], idx[d - 1], 0])
        total += term
    return total


def rel_error(A, Ahat) -> float:
    """Eq.(3): ||A - Ahat||_F / ||A||_F."""
    A = np.asarray(A, dtype=np.float64)
    D = A - np.asarray(Ahat, dtype=np.float64)
    return math.sqrt(float(np.sum(D * D))) / math.sqrt(float(np.sum(A * A)))

