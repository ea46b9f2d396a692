"""CPU FP64 oracle of the nTT sweep (test infrastructure; see ntt_oracle)."""
from .ntt_oracle import *  # noqa: F401,F403
