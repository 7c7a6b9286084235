"""CPU oracle of the PDE dehazing method and of the warm-start network.

Test infrastructure only: the tests, the smoke check and the CPU-baseline leg
of the benchmark may import it; the product package never does.  It is plain
float64 numpy/scipy written from the paper, and shares no code with the HIP
library.
"""
from . import dehaze_ref, cnn_ref  # noqa: F401
