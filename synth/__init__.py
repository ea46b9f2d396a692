"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This package holds no arithmetic of the decomposition itself: it draws random
numbers and assembles test tensors following the data-generation recipe of the
paper (Section IV-A: TT cores with entries uniform on [0,1), contracted into a
full tensor).  Both the CPU oracle and the GPU library receive what it makes.
"""
from .tt_inputs import (  # noqa: F401
    GAMMA,
    splitmix64,
    uniform01,
    std_normal,
    random_cores,
    contract_cores,
    noisy_tensor,
    workload,
    batched_mix,
    serving_stream,
    WORKLOADS,
)
