"""Plain FP64 CPU oracle of the SD right-hand side (test infrastructure only).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  It shares no code with the HIP library: the C oracle in
``sd_oracle.c`` transcribes the paper's algorithm element by element, and the
numpy modules beside it hold the temporal (Bloch) eigenanalysis and the
closure MLP reference.
"""
from .oracle import *  # noqa: F401,F403
