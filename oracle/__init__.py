"""FP64 CPU oracle of gradient-guided nested sampling with the HSS walk.

TEST INFRASTRUCTURE ONLY: tests/, the smoke check and the CPU baseline leg of
bench.py may use it; the GPU engine never imports, links or calls it.
"""
from .oracle import Oracle, build, loglike  # noqa: F401
