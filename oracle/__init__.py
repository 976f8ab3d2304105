"""FP64 CPU oracle of the w-stacking imaging path (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may use
this package; the product path never imports it.
"""
from . import wstack  # noqa: F401
