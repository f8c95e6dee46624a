"""Seeded synthetic luma video for motion-estimation tests and benchmarks.

This package only draws pixels.  It holds none of the motion-search
arithmetic, and both the CPU oracle's tests and the GPU path read their inputs
from it.  See ``video.py`` for the generators.
"""
from .video import (  # noqa: F401
    CONFIGS,
    SequenceSpec,
    blurred_noise,
    make_config,
    qcif_pair,
    moving_sequence,
    batch_streams,
    training_sequence,
)
