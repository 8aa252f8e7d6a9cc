"""Seeded synthetic landmark sets shared by the oracle tests, the GPU tests and the bench.

This package only builds inputs: template and target landmark coordinates, momenta
guesses and index subsets.  It holds none of the matching method's arithmetic (no
kernel sums, no time stepping, no momentum update), so both sides of a parity test can
take their inputs from here without sharing any of the computation under test.

All arrays are float64, component-major ("SoA"): shape (dim, n), row c holds the c-th
coordinate of every landmark.
"""

from .landmarks import *  # noqa: F401,F403
