"""CPU reference for the 3D Gabor splatting rasterizer.

Test infrastructure only: imported by the tests, the smoke check and the CPU
baseline leg of the benchmark, never by the product path.
"""
from . import gabor_oracle  # noqa: F401
