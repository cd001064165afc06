"""FP64 CPU oracle for the ConKer hot path -- TEST INFRASTRUCTURE ONLY.

Importable only by the tests, the smoke check and the bench's CPU-baseline leg.
The product library (paper_2108_00015_amd) never imports it, and it imports
nothing from the product library.
"""
from . import conker  # noqa: F401
from . import brute   # noqa: F401
