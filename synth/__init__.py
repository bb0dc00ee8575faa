"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This package only draws random numbers and builds images and cost volumes
(the data cost of Sec. 2, eq. Cost_value).  It holds none of the energy
minimisation arithmetic: no smoothness prior, no minimum search, no dynamic
programming.
"""
from .inputs import *  # noqa: F401,F403
