"""Counter-based random numbers and TT-structured test tensors.

Random numbers
--------------
Value ``i`` of stream ``tag`` under ``seed`` is the SplitMix64 output
(Steele, Lea and Flood, "Fast splittable pseudorandom number generators",
OOPSLA 2014) at counter position ``tag * 2**32 + i + 1``:

    z = seed + GAMMA * (tag * 2**32 + i + 1)            (mod 2**64)
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9            (mod 2**64)
    z = (z ^ (z >> 27)) * 0x94D049BB133111EB            (mod 2**64)
    z =  z ^ (z >> 31)

With ``tag = 0`` this is exactly the published SplitMix64 sequence seeded with
``seed``.  A uniform on [0,1) is ``(z >> 40) * 2**-24``: every such value is an
FP32 number, so a float32 copy is exact.

Tensors
-------
Section IV-A of the paper builds a synthetic tensor with known TT ranks by
drawing every TT core entry uniformly from [0,1) and contracting the cores.
``random_cores`` draws the cores (core ``k`` from stream ``TAG_CORE + k``),
``contract_cores`` contracts them in float64 and rounds once to float32.
Noise recipes for the larger workloads are applied afterwards.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

GAMMA = 0x9E3779B97F4A7C15
_MIX1 = 0xBF58476D1CE4E5B9
_MIX2 = 0x94D049BB133111EB
_M64 = (1 << 64) - 1

TAG_CORE = 0x100      # + core index k (1-based)
TAG_NOISE = 0x200     # noise uniforms; normals use TAG_NOISE and TAG_NOISE + 1
TAG_MIX = 0x300       # shape / rank draws of the batched and serving mixes
TAG_ARRIVAL = 0x301   # inter-arrival times of the serving stream
TAG_SEEDS = 0x302     # per-problem seeds of the batched and serving mixes

_CHUNK = 1 << 22


def splitmix64(seed: int, tag: int, start: int, count: int) -> np.ndarray:
    """Raw 64-bit outputs ``start .. start+count-1`` of stream ``tag``."""
    seed &= _M64
    z = np.arange(start + 1, start + 1 + count, dtype=np.uint64)   # counter i + 1
    z += np.uint64((tag << 32) & _M64)
    with np.errstate(over="ignore"):   # in place, one temporary: all arithmetic mod 2**64
        z *= np.uint64(GAMMA)
        z += np.uint64(seed)
        t = z >> np.uint64(30)
        z ^= t
        z *= np.uint64(_MIX1)
        np.right_shift(z, np.uint64(27), out=t)
        z ^= t
        z *= np.uint64(_MIX2)
        np.right_shift(z, np.uint64(31), out=t)
        z ^= t
    return z


def uniform01(seed: int, tag: int, shape, start: int = 0) -> np.ndarray:
    """Uniforms on [0,1) as float32 (exact), in C order of ``shape``."""
    shape = tuple(int(s) for s in np.atleast_1d(shape)) if not isinstance(shape, tuple) else shape
    n = int(np.prod(shape)) if len(shape) else 1
    out = np.empty(n, dtype=np.float32)
    for s in range(0, n, _CHUNK):
        c = min(_CHUNK, n - s)
        z = splitmix64(seed, tag, start + s, c)
        out[s:s + c] = (z >> np.uint64(40)).astype(np.float32) * np.float32(2.0 ** -24)
    return out.reshape(shape)


def std_normal(seed: int, tag: int, n: int) -> np.ndarray:
    """Standard normals by Box-Muller on streams ``tag`` and ``tag + 1`` (float64)."""
    out = np.empty(n, dtype=np.float64)
    for s in range(0, n, _CHUNK):
        c = min(_CHUNK, n - s)
        u1 = 1.0 - uniform01(seed, tag, (c,), start=s).astype(np.float64)  # (0, 1]
        u2 = uniform01(seed, tag + 1, (c,), start=s).astype(np.float64)
        out[s:s + c] = np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)
    return out


def random_cores(dims, ranks, seed: int):
    """TT cores of shape (r_{k-1}, n_k, r_k) with U[0,1) entries (Section IV-A)."""
    dims = [int(n) for n in dims]
    ranks = [int(r) for r in ranks]
    assert len(ranks) == len(dims) + 1 and ranks[0] == 1 and ranks[-1] == 1
    return [uniform01(seed, TAG_CORE + k + 1, (ranks[k], dims[k], ranks[k + 1]))
            for k in range(len(dims))]


def contract_cores(cores) -> np.ndarray:
    """Full tensor from TT cores, contracted in float64, rounded once to float32."""
    dims = [c.shape[1] for c in cores]
    p = cores[0].astype(np.float64).reshape(dims[0], cores[0].shape[2])
    for c in cores[1:]:
        r0, n, r1 = c.shape
        p = p.reshape(-1, r0) @ c.astype(np.float64).reshape(r0, n * r1)
    return p.reshape(dims).astype(np.float32)


def noisy_tensor(dims, ranks, seed: int, noise: str = "none", level: float = 0.0):
    """TT-generated tensor plus one of the noise recipes of the workloads.

    ``noise="mult"``: A <- A * (1 + level * (2u - 1)), u ~ U[0,1).
    ``noise="absnormal"``: A <- A + |N(0, level^2)| (level is the standard deviation).
    The result stays non-negative and is float32.
    """
    a = contract_cores(random_cores(dims, ranks, seed))
    if noise == "none" or level == 0.0:
        return a
    flat = a.reshape(-1)
    n = flat.size
    for s in range(0, n, _CHUNK):
        c = min(_CHUNK, n - s)
        blk = flat[s:s + c].astype(np.float64)
        if noise == "mult":
            u = uniform01(seed, TAG_NOISE, (c,), start=s).astype(np.float64)
            blk = blk * (1.0 + level * (2.0 * u - 1.0))
        elif noise == "absnormal":
            # one normal per entry: draw with the same counter offset on both streams
            u1 = 1.0 - uniform01(seed, TAG_NOISE, (c,), start=s).astype(np.float64)
            u2 = uniform01(seed, TAG_NOISE + 1, (c,), start=s).astype(np.float64)
            z = np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)
            blk = blk + np.abs(level * z)
        else:
            raise ValueError(noise)
        flat[s:s + c] = blk.astype(np.float32)
    return a


@dataclass
class Workload:
    name: str
    dims: tuple
    gen_ranks: tuple        # ranks of the generating cores, (1, ..., 1)
    target_ranks: tuple     # requested TT ranks, (1, ..., 1)
    iters: int
    seed: int
    noise: str = "none"
    level: float = 0.0
    eps: float = 1e-12
    fp32_tail: int = 0
    note: str = ""

    def tensor(self) -> np.ndarray:
        return noisy_tensor(self.dims, self.gen_ranks, self.seed, self.noise, self.level)


WORKLOADS = {
    # 16^3 tensor from cores with ranks (1,4,4,1); target ranks (4,4); 200 MU iterations.
    "tt16x3_r4": Workload("tt16x3_r4", (16, 16, 16), (1, 4, 4, 1), (1, 4, 4, 1), 200, 1,
                          note="16^3 from U[0,1) cores, ranks (4,4), T=200, eps=1e-12"),
    # 32^5 tensor from cores with ranks 8, 1% multiplicative uniform noise; 500 iterations.
    "tt32x5_r8": Workload("tt32x5_r8", (32,) * 5, (1, 8, 8, 8, 8, 1), (1, 8, 8, 8, 8, 1), 500, 2,
                          noise="mult", level=0.01,
                          note="32^5 from U[0,1) rank-8 cores, x(1+0.01(2u-1)), T=500"),
    # 128^4 tensor from cores with ranks 16, + |N(0, 0.01^2)|; 200 iterations, BF16 with FP32 tail.
    "tt128x4_r16": Workload("tt128x4_r16", (128,) * 4, (1, 16, 16, 16, 1), (1, 16, 16, 16, 1),
                            200, 3, noise="absnormal", level=0.01, fp32_tail=20,
                            note="128^4 from U[0,1) rank-16 cores, +|N(0,0.01^2)|, T=200"),
    # The paper's single-tensor workload size (Sec. IV): 256^4 in FP32 (16 GiB), TT ranks 10,
    # 100 MU iterations per stage.  Generated exactly (no noise) from U[0,1) cores; the
    # entries are best formed on the device from the cores (17 GB).
    "tt256x4_r10": Workload("tt256x4_r10", (256,) * 4, (1, 10, 10, 10, 1), (1, 10, 10, 10, 1),
                            100, 6, note="256^4 from U[0,1) rank-10 cores, T=100"),
}


def workload(name: str) -> Workload:
    return WORKLOADS[name]


def _ints(seed, tag, start, count, lo, hi):
    """Integers uniform on {lo..hi} from a uniform stream."""
    u = uniform01(seed, tag, (count,), start=start).astype(np.float64)
    return (lo + np.floor(u * (hi - lo + 1))).astype(np.int64)


def _sub_seed(seed: int, idx: int) -> int:
    return int(splitmix64(seed, TAG_SEEDS, idx, 1)[0])


def batched_mix(count: int = 256, seed: int = 4, iters: int = 200):
    """The batched workload: independent TT tensors of uneven shape and rank.

    Per problem p (draws at counter 16p.. of stream TAG_MIX):
    d ~ U{3,4,5}; n_i ~ U{8..64}; true ranks r_i ~ U{2..12}; the targets are the
    true ranks (the library clamps them).  Entries come from seeded U[0,1) cores.
    """
    out = []
    for p in range(count):
        base = 16 * p
        d = int(_ints(seed, TAG_MIX, base, 1, 3, 5)[0])
        dims = tuple(int(x) for x in _ints(seed, TAG_MIX, base + 1, d, 8, 64))
        inner = tuple(int(x) for x in _ints(seed, TAG_MIX, base + 1 + d, d - 1, 2, 12))
        ranks = (1,) + inner + (1,)
        out.append(Workload(f"mix{p}", dims, ranks, ranks, iters, _sub_seed(seed, p)))
    return out


@dataclass
class Request:
    rid: int
    arrival_s: float
    work: Workload = field(repr=False)


def serving_stream(count: int = 1000, seed: int = 5, rate_per_s: float = 10.0,
                   min_bytes: float = 1e6, max_bytes: float = 1e9, iters: int = 200,
                   rmin: int = 4, rmax: int = 32):
    """Poisson request stream of TT-generated tensors.

    Per request q: d ~ U{3..6}; total bytes log-uniform on [min_bytes, max_bytes]
    (N = bytes/4 entries); mode sizes from log N split by Dirichlet(1) weights
    (normalised exponentials), rounded, each >= 2; one target rank r ~ U{rmin..rmax}
    for every bond (generating cores use the same rank, clamped per bond to the largest
    rank the mode sizes allow).  Inter-arrival times are
    exponential with the given rate.
    """
    reqs = []
    t = 0.0
    for q in range(count):
        base = 32 * q
        u = uniform01(seed, TAG_MIX, (32,), start=base).astype(np.float64)
        d = 3 + int(math.floor(u[0] * 4))
        nbytes = math.exp(math.log(min_bytes) + u[1] * (math.log(max_bytes) - math.log(min_bytes)))
        logn = math.log(max(nbytes / 4.0, 8.0))
        e = -np.log(1.0 - u[2:2 + d])
        w = e / e.sum()
        dims = tuple(max(2, int(round(math.exp(logn * wi)))) for wi in w)
        r = rmin + int(math.floor(u[2 + d] * (rmax - rmin + 1)))
        ranks = (1,) + (r,) * (d - 1) + (1,)
        # the generating cores take the same rank, clamped at each bond to the largest a
        # TT of these mode sizes can have (min of the products of the modes on each side)
        gen = (1,) + tuple(min(r, math.prod(dims[:k]), math.prod(dims[k:])) for k in range(1, d)) + (1,)
        ua = float(uniform01(seed, TAG_ARRIVAL, (1,), start=q)[0])
        t += -math.log(1.0 - ua) / rate_per_s
        reqs.append(Request(q, t, Workload(f"req{q}", dims, gen, ranks, iters,
                                           _sub_seed(seed + 1, q))))
    return reqs
