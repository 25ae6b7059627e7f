"""MI355X (gfx950) barrier-augmented Lagrangian time step: HIP library + ctypes binding."""
from . import bal  # noqa: F401  (loads libbal.so; raises ImportError if it is not built)
from .bal import Scene, BalError  # noqa: F401
