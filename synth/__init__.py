"""Seeded synthetic stereo inputs shared by the tests, the oracle checks and the benchmark.

This package only draws random numbers and lays out images; it holds none of the
depth method's arithmetic (no noise application, census, cost, aggregation or
post-processing).  Random numbers that the method itself consumes (the speckle
gain and the thermal term of the IR noise model) are drawn here and handed to
both implementations as inputs.
"""
from .stereo import (  # noqa: F401
    PairSpec,
    StereoPair,
    CONFIGS,
    make_pair,
    make_shift_pair,
    noise_draws,
    pair_seed,
)
