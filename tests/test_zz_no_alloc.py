"""ntt_rel_error_static (no allocation, a fixed device array inside the library) against
ntt_rel_error (caller workspace), through the C ABI: two calls in a row, the second on a
smaller tensor, each bitwise equal to the workspace entry point's result; a tensor beyond
the array's limit is refused with a clear status."""
import sys

import numpy as np
import pytest

import synth as S

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_2008_01340_amd import ntt  # noqa: E402

DEV = "cuda:0"


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _pair(dims, ranks, seed):
    A = torch.from_numpy(S.noisy_tensor(dims, ranks, seed=seed, noise="mult", level=0.05)).to(DEV)
    cores = [torch.from_numpy(c).to(DEV) for c in S.random_cores(dims, ranks, seed=seed + 1)]
    return A, cores


def _both(A, cores):
    dims = list(A.shape)
    ranks = [1] + [c.shape[2] for c in cores]
    ptrs = [c.data_ptr() for c in cores]
    stream = torch.cuda.current_stream().cuda_stream
    nbytes = ntt.ntt_tt_workspace(dims, ranks)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=DEV)
    e_ws = ntt.ntt_rel_error(dims, ranks, A.data_ptr(), ptrs, ws.data_ptr(), nbytes, stream)
    e_st = ntt.ntt_rel_error_static(dims, ranks, A.data_ptr(), ptrs, stream)
    return e_ws, e_st


def test_rel_error_static_equals_workspace_entry_point_on_two_calls():
    assert torch.cuda.is_available()
    ntt.load()
    # first a large tensor (4096 x 16 x 16 x 9 -> 1,048,576 rows of 9, 16,384 blocks), then a
    # smaller one with a ragged last block: the second call reads only what it wrote
    cases = [((4096, 16, 16, 9), (1, 5, 7, 3, 1), 3), ((37, 11, 13), (1, 4, 2, 1), 4)]
    for dims, ranks, seed in cases:
        say(f"case: rel_error_static dims={dims} ranks={ranks}")
        A, cores = _pair(dims, ranks, seed)
        e_ws, e_st = _both(A, cores)
        say(f"  workspace {e_ws!r} static {e_st!r}")
        assert e_st == e_ws  # the same kernels and summation order: bitwise equal
        assert 0.0 < e_st < 10.0


def test_rel_error_static_refuses_beyond_its_limit_and_zero_norm():
    ntt.load()
    # n_1...n_{d-1} = 33,554,432 rows > 33,554,368: refused before any device work (the
    # pointers are never read, so tiny stand-in buffers do)
    dims, ranks = (1 << 25, 1), (1, 1, 1)
    x = torch.zeros(4, device=DEV)
    with pytest.raises(ntt.NttError) as e:
        ntt.ntt_rel_error_static(dims, ranks, x.data_ptr(), [x.data_ptr(), x.data_ptr()], 0)
    assert e.value.status == ntt.NTT_ERR_WORKSPACE_TOO_SMALL
    A = torch.zeros((3, 4), device=DEV)
    cores = [torch.ones((1, 3, 2), device=DEV), torch.ones((2, 4, 1), device=DEV)]
    with pytest.raises(ntt.NttError) as e:
        ntt.ntt_rel_error_static([3, 4], [1, 2, 1], A.data_ptr(), [c.data_ptr() for c in cores], 0)
    assert e.value.status == ntt.NTT_ERR_ZERO_NORM
