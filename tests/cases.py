"""Seeded test molecules shared by oracle pins and GPU parity tests.

Geometry only comes from the synthetic generator; Gaussian widths are derived
by whichever side (oracle or HIP library) is under test.
"""
import numpy as np

from paper_2607_20766_amd import molgen

# lambda that reproduces a Gaussian height p = 2.7 of the Grant-Pickup width
LAMBDA = 2.7 ** (-2.0 / 3.0)


def config0():
    """Single fixed-pose pair: 20-atom query (seed 0, index 0) and 24-atom
    target (seed 0, index 1)."""
    return molgen.molecule(0, 0, 20), molgen.molecule(0, 1, 24)


def small(seed, n):
    return molgen.molecule(1000 + seed, n, n)


def oracle_mol(O, ms):
    return (ms.xyz, O.alpha_from_radius(ms.radius, LAMBDA))
