"""ctypes binding of libntt.so (the C ABI declared in include/ntt.h).

Argument marshalling only: every step of the decomposition runs in the HIP
kernels of the library.  torch supplies device memory (``tensor.data_ptr()``) and
the stream (``torch.cuda.current_stream().cuda_stream``).  If the library has not
been built, loading fails with an error: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libntt.so")

NTT_MAX_DIMS = 16
NTT_MAX_RANK = 32

NTT_OK = 0
NTT_ERR_INVALID_ARG = 1
NTT_ERR_RANK_INFEASIBLE = 2
NTT_ERR_NEGATIVE_INPUT = 3
NTT_ERR_WORKSPACE_TOO_SMALL = 4
NTT_ERR_ZERO_NORM = 5
NTT_ERR_DEVICE = 6

NTT_PREC_FP32 = 0
NTT_PREC_BF16_MIXED = 1

NTT_NMF_MU = 0
NTT_NMF_BCD = 1
_NMF = {"mu": NTT_NMF_MU, "bcd": NTT_NMF_BCD}

NTT_STRICT_RANKS = 1
NTT_VALIDATE_INPUT = 2
NTT_RECORD_OBJECTIVE = 4
NTT_PROFILE = 8
NTT_NO_COOP = 16

EXPORTED = [
    "ntt_plan", "ntt_plan_workspace", "ntt_decompose", "ntt_tt_workspace", "ntt_reconstruct",
    "ntt_rel_error", "ntt_rel_error_static", "ntt_compression_ratio", "ntt_plan_destroy",
    "ntt_status_string",
    "ntt_last_error", "ntt_version", "ntt_batch_plan", "ntt_batch_workspace", "ntt_batch_eff_ranks",
    "ntt_decompose_batch", "ntt_batch_destroy", "ntt_server_create", "ntt_server_submit",
    "ntt_server_tick", "ntt_server_info", "ntt_server_cores", "ntt_server_release",
    "ntt_server_free_bytes", "ntt_server_destroy",
]

NTT_REQ_QUEUED, NTT_REQ_RUNNING, NTT_REQ_DONE, NTT_REQ_REJECTED, NTT_REQ_CANCELLED = range(5)


class NttConfig(C.Structure):
    _fields_ = [
        ("d", C.c_int32),
        ("dims", C.POINTER(C.c_int64)),
        ("ranks", C.POINTER(C.c_int64)),
        ("max_iters", C.c_int32),
        ("tol", C.c_double),
        ("check_every", C.c_int32),
        ("eps", C.c_double),
        ("seed", C.c_uint64),
        ("precision", C.c_int32),
        ("fp32_tail_iters", C.c_int32),
        ("flags", C.c_uint32),
        ("rank_eps", C.c_double),
        ("nmf", C.c_int32),
        ("bcd_delta", C.c_double),
        ("stream_cols", C.c_int64),
    ]


class NttReport(C.Structure):
    _fields_ = [
        ("eff_ranks", C.c_int64 * (NTT_MAX_DIMS + 1)),
        ("iters", C.c_int32 * NTT_MAX_DIMS),
        ("objective", C.c_double * NTT_MAX_DIMS),
        ("norm_x", C.c_double * NTT_MAX_DIMS),
        ("stage_rel_err", C.c_double * NTT_MAX_DIMS),
        ("ms", C.c_double * NTT_MAX_DIMS),
        ("gflop", C.c_double * NTT_MAX_DIMS),
        ("pass_ms", C.c_double * NTT_MAX_DIMS),
        ("total_ms", C.c_double),
        ("total_gflop", C.c_double),
        ("compression_ratio", C.c_double),
        ("corrections", C.c_int32 * NTT_MAX_DIMS),
        ("bf16_iters", C.c_int32 * NTT_MAX_DIMS),
    ]

    def to_dict(self, d: int) -> dict:
        s = d - 1
        return {
            "eff_ranks": list(self.eff_ranks[: d + 1]),
            "iters": list(self.iters[:s]),
            "objective": list(self.objective[:s]),
            "norm_x": list(self.norm_x[:s]),
            "stage_rel_err": list(self.stage_rel_err[:s]),
            "ms": list(self.ms[:s]),
            "gflop": list(self.gflop[:s]),
            "pass_ms": list(self.pass_ms[:s]),
            "total_ms": self.total_ms,
            "total_gflop": self.total_gflop,
            "compression_ratio": self.compression_ratio,
            "corrections": list(self.corrections[:s]),
            "bf16_iters": list(self.bf16_iters[:s]),
        }


class NttServerConfig(C.Structure):
    _fields_ = [("arena", C.c_void_p), ("arena_bytes", C.c_size_t), ("max_slots", C.c_int32),
                ("iters_per_tick", C.c_int32)]


class NttRequest(C.Structure):
    _fields_ = [("d", C.c_int32), ("dims", C.POINTER(C.c_int64)), ("ranks", C.POINTER(C.c_int64)),
                ("max_iters", C.c_int32), ("eps", C.c_double), ("seed", C.c_uint64),
                ("precision", C.c_int32), ("fp32_tail_iters", C.c_int32), ("host_A", C.c_void_p),
                ("nmf", C.c_int32), ("bcd_delta", C.c_double)]


class NttRequestInfo(C.Structure):
    _fields_ = [("id", C.c_int64), ("state", C.c_int32), ("d", C.c_int32), ("t_submit", C.c_double),
                ("t_admit", C.c_double), ("t_start", C.c_double), ("t_finish", C.c_double),
                ("device_bytes", C.c_size_t), ("gflop", C.c_double),
                ("eff_ranks", C.c_int64 * (NTT_MAX_DIMS + 1))]


class NttError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: status {status}")
        self.status = status


_lib = None


def load(path: str = LIB_PATH):
    """Load libntt.so once; raises if it is missing (build it with build_lib)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libntt.so not found at {path}: build it with "
                           "`python -m paper_2008_01340_amd.build_lib`")
    lib = C.CDLL(path)
    P = C.c_void_p
    i64p = C.POINTER(C.c_int64)
    lib.ntt_plan.argtypes = [C.POINTER(NttConfig), C.POINTER(P)]
    lib.ntt_plan.restype = C.c_int
    lib.ntt_plan_workspace.argtypes = [P, C.POINTER(C.c_size_t), i64p, C.POINTER(C.c_double)]
    lib.ntt_plan_workspace.restype = C.c_int
    lib.ntt_decompose.argtypes = [P, P, P, P, C.POINTER(P), C.POINTER(P), C.POINTER(P), P,
                                  C.POINTER(NttReport)]
    lib.ntt_decompose.restype = C.c_int
    lib.ntt_tt_workspace.argtypes = [C.c_int32, i64p, i64p, C.POINTER(C.c_size_t)]
    lib.ntt_tt_workspace.restype = C.c_int
    lib.ntt_reconstruct.argtypes = [C.c_int32, i64p, i64p, C.POINTER(P), P, P]
    lib.ntt_reconstruct.restype = C.c_int
    lib.ntt_rel_error.argtypes = [C.c_int32, i64p, i64p, P, C.POINTER(P), P, C.c_size_t,
                                  C.POINTER(C.c_double), P]
    lib.ntt_rel_error.restype = C.c_int
    lib.ntt_rel_error_static.argtypes = [C.c_int32, i64p, i64p, P, C.POINTER(P),
                                         C.POINTER(C.c_double), P]
    lib.ntt_rel_error_static.restype = C.c_int
    lib.ntt_compression_ratio.argtypes = [C.c_int32, i64p, i64p]
    lib.ntt_compression_ratio.restype = C.c_double
    lib.ntt_plan_destroy.argtypes = [P]
    lib.ntt_plan_destroy.restype = None
    lib.ntt_status_string.argtypes = [C.c_int]
    lib.ntt_status_string.restype = C.c_char_p
    lib.ntt_last_error.argtypes = []
    lib.ntt_last_error.restype = C.c_char_p
    lib.ntt_version.argtypes = []
    lib.ntt_version.restype = C.c_char_p
    lib.ntt_batch_plan.argtypes = [C.c_int32, C.POINTER(NttConfig), C.POINTER(P)]
    lib.ntt_batch_plan.restype = C.c_int
    lib.ntt_batch_workspace.argtypes = [P, C.POINTER(C.c_size_t)]
    lib.ntt_batch_workspace.restype = C.c_int
    lib.ntt_batch_eff_ranks.argtypes = [P, C.c_int32, C.POINTER(C.c_int64)]
    lib.ntt_batch_eff_ranks.restype = C.c_int
    lib.ntt_decompose_batch.argtypes = [P, P, P, C.POINTER(P), C.POINTER(C.POINTER(P)),
                                        C.POINTER(NttReport)]
    lib.ntt_decompose_batch.restype = C.c_int
    lib.ntt_batch_destroy.argtypes = [P]
    lib.ntt_batch_destroy.restype = None
    lib.ntt_server_create.argtypes = [C.POINTER(NttServerConfig), C.POINTER(P)]
    lib.ntt_server_create.restype = C.c_int
    lib.ntt_server_submit.argtypes = [P, C.POINTER(NttRequest), C.POINTER(C.c_int64)]
    lib.ntt_server_submit.restype = C.c_int
    lib.ntt_server_tick.argtypes = [P, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
    lib.ntt_server_tick.restype = C.c_int
    lib.ntt_server_info.argtypes = [P, C.c_int64, C.POINTER(NttRequestInfo)]
    lib.ntt_server_info.restype = C.c_int
    lib.ntt_server_cores.argtypes = [P, C.c_int64, C.POINTER(C.c_void_p)]
    lib.ntt_server_cores.restype = C.c_int
    lib.ntt_server_release.argtypes = [P, C.c_int64]
    lib.ntt_server_release.restype = C.c_int
    lib.ntt_server_free_bytes.argtypes = [P, C.POINTER(C.c_size_t)]
    lib.ntt_server_free_bytes.restype = C.c_int
    lib.ntt_server_destroy.argtypes = [P]
    lib.ntt_server_destroy.restype = None
    _lib = lib
    return lib


def _check(status: int, what: str):
    if status != NTT_OK:
        lib = load()
        raise NttError(status, f"{what} failed: {lib.ntt_status_string(status).decode()} "
                               f"({lib.ntt_last_error().decode()})")


def _i64(vals):
    arr = (C.c_int64 * len(vals))(*[int(v) for v in vals])
    return arr


def _ptrs(vals):
    return (C.c_void_p * len(vals))(*[None if v is None else int(v) for v in vals])


# ------------------------------------------------------------------ thin C-name layer
class Plan:
    """Owns an ntt_plan_t; keeps the host arrays the config points to alive."""

    def __init__(self, dims, ranks, max_iters, tol=0.0, check_every=10, eps=1e-12, seed=0,
                 precision=NTT_PREC_FP32, fp32_tail_iters=20, flags=0, rank_eps=0.0,
                 nmf="mu", delta=0.9999, stream_cols=0):
        """``nmf``: "mu" (multiplicative updates) or "bcd" (Alg.3, extrapolation cap
        ``delta``).  ``stream_cols`` > 0: the input is in host memory and stage 1 streams
        it in column blocks of that many columns."""
        lib = load()
        self.dims = [int(n) for n in dims]
        self.ranks = [int(r) for r in ranks]
        self.d = len(self.dims)
        self._dims = _i64(self.dims)
        self._ranks = _i64(self.ranks)
        self.cfg = NttConfig(self.d, C.cast(self._dims, C.POINTER(C.c_int64)),
                             C.cast(self._ranks, C.POINTER(C.c_int64)), int(max_iters), float(tol),
                             int(check_every), float(eps), int(seed) & ((1 << 64) - 1),
                             int(precision), int(fp32_tail_iters), int(flags), float(rank_eps),
                             _NMF[nmf], float(delta), int(stream_cols))
        self.max_iters = int(max_iters)
        self.rank_eps = float(rank_eps)
        self.stream_cols = int(stream_cols)
        self.handle = C.c_void_p()
        _check(lib.ntt_plan(C.byref(self.cfg), C.byref(self.handle)), "ntt_plan")

    def workspace(self):
        lib = load()
        nbytes = C.c_size_t()
        eff = (C.c_int64 * (self.d + 1))()
        comp = C.c_double()
        _check(lib.ntt_plan_workspace(self.handle, C.byref(nbytes), eff, C.byref(comp)),
               "ntt_plan_workspace")
        return int(nbytes.value), list(eff), float(comp.value)

    def close(self):
        if self.handle:
            load().ntt_plan_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ntt_plan(dims, ranks, max_iters, **kw) -> Plan:
    return Plan(dims, ranks, max_iters, **kw)


def ntt_plan_workspace(plan: Plan):
    return plan.workspace()


def ntt_decompose(plan: Plan, stream: int, workspace: int, A: int, cores, init_W=None,
                  init_H=None, objective_trace: int | None = None, want_report=True):
    """Raw call with integer device pointers; returns the report dict (or None)."""
    lib = load()
    rep = NttReport()
    iw = _ptrs(init_W) if init_W is not None else None
    ih = _ptrs(init_H) if init_H is not None else None
    st = lib.ntt_decompose(plan.handle, C.c_void_p(stream), C.c_void_p(workspace), C.c_void_p(A),
                           _ptrs(cores), iw, ih, C.c_void_p(objective_trace or 0),
                           C.byref(rep) if want_report else None)
    _check(st, "ntt_decompose")
    return rep.to_dict(plan.d) if want_report else None


def ntt_tt_workspace(dims, ranks) -> int:
    nbytes = C.c_size_t()
    _check(load().ntt_tt_workspace(len(dims), _i64(dims), _i64(ranks), C.byref(nbytes)),
           "ntt_tt_workspace")
    return int(nbytes.value)


def ntt_reconstruct(dims, ranks, cores, A_out: int, stream: int = 0):
    _check(load().ntt_reconstruct(len(dims), _i64(dims), _i64(ranks), _ptrs(cores),
                                  C.c_void_p(A_out), C.c_void_p(stream)), "ntt_reconstruct")


def ntt_rel_error(dims, ranks, A: int, cores, workspace: int, workspace_bytes: int,
                  stream: int = 0) -> float:
    out = C.c_double()
    _check(load().ntt_rel_error(len(dims), _i64(dims), _i64(ranks), C.c_void_p(A), _ptrs(cores),
                                C.c_void_p(workspace), workspace_bytes, C.byref(out),
                                C.c_void_p(stream)), "ntt_rel_error")
    return float(out.value)


def ntt_rel_error_static(dims, ranks, A: int, cores, stream: int = 0) -> float:
    out = C.c_double()
    _check(load().ntt_rel_error_static(len(dims), _i64(dims), _i64(ranks), C.c_void_p(A),
                                       _ptrs(cores), C.byref(out), C.c_void_p(stream)),
           "ntt_rel_error_static")
    return float(out.value)


def ntt_compression_ratio(dims, ranks) -> float:
    return float(load().ntt_compression_ratio(len(dims), _i64(dims), _i64(ranks)))


def ntt_version() -> str:
    return load().ntt_version().decode()


# ------------------------------------------------------------------ torch helpers
@dataclass
class Decomposition:
    cores: list            # torch tensors on the device
    ranks: list            # effective ranks r_0..r_d
    report: dict | None
    trace: object = None   # torch float64 tensor of objectives, when recorded


def _stream_handle(torch, stream):
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


def decompose(A, ranks, max_iters, *, eps=1e-12, seed=0, tol=0.0, check_every=10,
              precision=NTT_PREC_FP32, fp32_tail_iters=20, flags=0, init_W=None, init_H=None,
              record_objective=False, plan=None, workspace=None, cores=None, stream=None,
              want_report=True, rank_eps=0.0, nmf="mu", delta=0.9999, stream_cols=0,
              device="cuda:0"):
    """Decompose a float32 CUDA tensor; allocates cores/workspace with torch if not given.

    ``nmf="bcd"`` runs Alg.3 (BCD with extrapolation cap ``delta``) instead of MU.
    ``stream_cols`` > 0: ``A`` is a CPU tensor (pinned for full copy speed) and stage 1
    streams it to ``device`` in column blocks; the cores come back on ``device``.

    With rank_eps > 0 the ranks are chosen by the rule of Alg.2 (``ranks`` are caps);
    the returned cores are views of the (cap-sized) buffers at the chosen ranks."""
    import torch
    assert A.dtype == torch.float32 and A.is_contiguous()
    if plan is not None:
        stream_cols = plan.stream_cols
    assert (not A.is_cuda) if stream_cols > 0 else A.is_cuda
    dev = torch.device(device) if stream_cols > 0 else A.device
    dims = list(A.shape)
    if record_objective:
        flags |= NTT_RECORD_OBJECTIVE
    if plan is None:
        plan = Plan(dims, ranks, max_iters, tol=tol, check_every=check_every, eps=eps, seed=seed,
                    precision=precision, fp32_tail_iters=fp32_tail_iters, flags=flags,
                    rank_eps=rank_eps, nmf=nmf, delta=delta, stream_cols=stream_cols)
    if plan.rank_eps > 0.0:
        want_report = True  # the chosen ranks come back in the report
    nbytes, eff, _ = plan.workspace()
    if workspace is None:
        workspace = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=dev)
    if cores is None:
        cores = [torch.empty((eff[k], dims[k], eff[k + 1]), dtype=torch.float32, device=dev)
                 for k in range(len(dims))]
    trace = None
    if record_objective:
        trace = torch.zeros(plan.max_iters * (len(dims) - 1), dtype=torch.float64, device=dev)
    iw = None if init_W is None else [None if t is None else t.data_ptr() for t in init_W]
    ih = None if init_H is None else [None if t is None else t.data_ptr() for t in init_H]
    rep = ntt_decompose(plan, _stream_handle(torch, stream), workspace.data_ptr(), A.data_ptr(),
                        [c.data_ptr() for c in cores], iw, ih,
                        trace.data_ptr() if trace is not None else None, want_report)
    if plan.rank_eps > 0.0:
        eff = rep["eff_ranks"]
        cores = [c.reshape(-1)[: eff[k] * dims[k] * eff[k + 1]].view(eff[k], dims[k], eff[k + 1])
                 for k, c in enumerate(cores)]
    return Decomposition(cores, eff, rep, trace)


def reconstruct(cores, stream=None):
    import torch
    dims = [c.shape[1] for c in cores]
    ranks = [1] + [c.shape[2] for c in cores]
    out = torch.empty(dims, dtype=torch.float32, device=cores[0].device)
    ntt_reconstruct(dims, ranks, [c.data_ptr() for c in cores], out.data_ptr(),
                    _stream_handle(torch, stream))
    return out


def rel_error(A, cores, workspace=None, stream=None) -> float:
    import torch
    dims = list(A.shape)
    ranks = [1] + [c.shape[2] for c in cores]
    nbytes = ntt_tt_workspace(dims, ranks)
    if workspace is None or workspace.numel() < nbytes:
        workspace = torch.empty(nbytes, dtype=torch.uint8, device=A.device)
    return ntt_rel_error(dims, ranks, A.data_ptr(), [c.data_ptr() for c in cores],
                         workspace.data_ptr(), nbytes, _stream_handle(torch, stream))


# ------------------------------------------------------------------ batched mode
class Batch:
    """Owns an ntt_batch_t built from one config per problem."""

    def __init__(self, problems, max_iters, eps=1e-12, precision=NTT_PREC_FP32,
                 fp32_tail_iters=20, tol=0.0, check_every=10, nmf="mu", delta=0.9999):
        """problems: list of (dims, ranks, seed); ``nmf``: "mu" or "bcd" for all of them."""
        lib = load()
        self.problems = [(list(map(int, dm)), list(map(int, rk)), int(sd)) for dm, rk, sd in problems]
        self._keep = []
        cfgs = (NttConfig * len(self.problems))()
        for i, (dm, rk, sd) in enumerate(self.problems):
            a, b = _i64(dm), _i64(rk)
            self._keep += [a, b]
            cfgs[i] = NttConfig(len(dm), C.cast(a, C.POINTER(C.c_int64)), C.cast(b, C.POINTER(C.c_int64)),
                                int(max_iters), float(tol), int(check_every), float(eps),
                                sd & ((1 << 64) - 1), int(precision), int(fp32_tail_iters), 0,
                                0.0, _NMF[nmf], float(delta))
        self.handle = C.c_void_p()
        _check(lib.ntt_batch_plan(len(self.problems), cfgs, C.byref(self.handle)), "ntt_batch_plan")
        nbytes = C.c_size_t()
        _check(lib.ntt_batch_workspace(self.handle, C.byref(nbytes)), "ntt_batch_workspace")
        self.workspace_bytes = int(nbytes.value)
        self.eff = []
        for i, (dm, _, _) in enumerate(self.problems):
            e = (C.c_int64 * (len(dm) + 1))()
            _check(lib.ntt_batch_eff_ranks(self.handle, i, e), "ntt_batch_eff_ranks")
            self.eff.append(list(e))

    def close(self):
        if self.handle:
            load().ntt_batch_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ntt_decompose_batch(batch: Batch, stream: int, workspace: int, A_ptrs, core_ptrs,
                        want_reports=True):
    lib = load()
    n = len(batch.problems)
    reps = (NttReport * n)() if want_reports else None
    rows = [_ptrs(cp) for cp in core_ptrs]
    arr = (C.POINTER(C.c_void_p) * n)(*[C.cast(r_, C.POINTER(C.c_void_p)) for r_ in rows])
    st = lib.ntt_decompose_batch(batch.handle, C.c_void_p(stream), C.c_void_p(workspace),
                                 _ptrs(A_ptrs), arr, reps)
    _check(st, "ntt_decompose_batch")
    if not want_reports:
        return None
    return [reps[i].to_dict(len(batch.problems[i][0])) for i in range(n)]


def decompose_batch(tensors, ranks_list, max_iters, seeds, *, eps=1e-12, precision=NTT_PREC_FP32,
                    fp32_tail_iters=20, batch=None, workspace=None, cores=None, stream=None,
                    want_reports=True, nmf="mu", delta=0.9999):
    """Decompose a list of float32 CUDA tensors in one batched call."""
    import torch
    if batch is None:
        batch = Batch([(list(t.shape), rk, sd) for t, rk, sd in zip(tensors, ranks_list, seeds)],
                      max_iters, eps=eps, precision=precision, fp32_tail_iters=fp32_tail_iters,
                      nmf=nmf, delta=delta)
    dev = tensors[0].device
    if workspace is None:
        workspace = torch.empty(max(batch.workspace_bytes, 256), dtype=torch.uint8, device=dev)
    if cores is None:
        cores = [[torch.empty((e[k], t.shape[k], e[k + 1]), dtype=torch.float32, device=dev)
                  for k in range(t.dim())] for t, e in zip(tensors, batch.eff)]
    reps = ntt_decompose_batch(batch, _stream_handle(torch, stream), workspace.data_ptr(),
                               [t.data_ptr() for t in tensors],
                               [[c.data_ptr() for c in cs] for cs in cores], want_reports)
    return cores, reps, batch


# ------------------------------------------------------------------ serving
class Server:
    """Owns an ntt_server_t over a torch-allocated device arena (the HBM budget)."""

    def __init__(self, arena_bytes, max_slots=16, iters_per_tick=25, device="cuda:0"):
        import torch
        lib = load()
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=device)
        cfg = NttServerConfig(self.arena.data_ptr(), int(arena_bytes), int(max_slots), int(iters_per_tick))
        self.handle = C.c_void_p()
        _check(lib.ntt_server_create(C.byref(cfg), C.byref(self.handle)), "ntt_server_create")
        self._inputs = {}  # host inputs kept alive until the request is released
        self._shapes = {}

    def submit(self, host_A, ranks, max_iters, seed=0, eps=1e-12, precision=NTT_PREC_FP32,
               fp32_tail_iters=20, nmf="mu", delta=0.9999) -> int:
        """host_A: a CPU float32 torch tensor (pinned for an overlapped copy); ``nmf``: "mu"
        or "bcd"."""
        dims = list(host_A.shape)
        a, b = _i64(dims), _i64(ranks)
        rq = NttRequest(len(dims), C.cast(a, C.POINTER(C.c_int64)), C.cast(b, C.POINTER(C.c_int64)),
                        int(max_iters), float(eps), int(seed) & ((1 << 64) - 1), int(precision),
                        int(fp32_tail_iters), host_A.data_ptr(), _NMF[nmf], float(delta))
        rid = C.c_int64()
        _check(load().ntt_server_submit(self.handle, C.byref(rq), C.byref(rid)), "ntt_server_submit")
        self._inputs[rid.value] = host_A
        self._shapes[rid.value] = dims
        return rid.value

    def tick(self):
        na, nq = C.c_int32(), C.c_int32()
        _check(load().ntt_server_tick(self.handle, C.byref(na), C.byref(nq)), "ntt_server_tick")
        return na.value, nq.value

    def info(self, rid) -> dict:
        inf = NttRequestInfo()
        _check(load().ntt_server_info(self.handle, int(rid), C.byref(inf)), "ntt_server_info")
        return {"id": inf.id, "state": inf.state, "t_submit": inf.t_submit, "t_admit": inf.t_admit,
                "t_start": inf.t_start, "t_finish": inf.t_finish, "device_bytes": inf.device_bytes,
                "gflop": inf.gflop, "eff_ranks": list(inf.eff_ranks[: inf.d + 1])}

    def cores(self, rid):
        """Zero-copy views (into the arena) of a finished request's cores."""
        import torch
        dims = self._shapes[rid]
        eff = self.info(rid)["eff_ranks"]
        ptrs = (C.c_void_p * len(dims))()
        _check(load().ntt_server_cores(self.handle, int(rid), ptrs), "ntt_server_cores")
        base = self.arena.data_ptr()
        out = []
        for k, n in enumerate(dims):
            cnt = eff[k] * n * eff[k + 1]
            off = ptrs[k] - base
            out.append(self.arena[off:off + 4 * cnt].view(torch.float32).view(eff[k], n, eff[k + 1]))
        return out

    def release(self, rid):
        _check(load().ntt_server_release(self.handle, int(rid)), "ntt_server_release")
        self._inputs.pop(rid, None)

    def free_bytes(self) -> int:
        v = C.c_size_t()
        _check(load().ntt_server_free_bytes(self.handle, C.byref(v)), "ntt_server_free_bytes")
        return int(v.value)

    def close(self):
        if self.handle:
            load().ntt_server_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
