"""Seeded synthetic inputs shared by the oracle side and the HIP side.

This package builds *inputs only*: solar source node tables, a detector
response histogrammed from a seeded flat-recoil Monte Carlo, Poisson data
drawn from an expectation that the caller supplies, and parameter-point
lists.  It contains none of the likelihood arithmetic (no cross section,
no recoil-spectrum integral, no fold, no likelihood), so neither side can
hide a mistake behind it.
"""
from .workloads import *  # noqa: F401,F403
