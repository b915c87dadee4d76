"""CPU oracle for the per-ray training step of direct voxel-grid optimisation.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, single-threaded
NumPy reference written from the paper (Direct Voxel Grid Optimization,
arXiv 2111.11215).  Only the test-suite, the smoke check and the CPU-baseline
leg of the benchmark may import it; the product library never calls it and
shares no code with it (only the seeded input generators in ``synth`` feed
both sides).
"""

from .dvgo_oracle import *  # noqa: F401,F403
