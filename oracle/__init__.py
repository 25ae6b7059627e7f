"""CPU FP64 oracle of the barrier-augmented Lagrangian time step.

Test infrastructure only: the tests, the smoke check and the benchmark's CPU
baseline leg may import it; the GPU library never does.
"""
from .bal_oracle import *  # noqa: F401,F403
