"""MI355X (gfx950) Kalman-filter track fitting and combinatorial track building.

The compute path is the HIP library libkfmi.so (C ABI in include/kfmi.h);
`kfmi` is its thin ctypes binding, `synth` the seeded synthetic-event
generator and `judge` the efficiency / fake-rate judge.
"""
from . import synth  # noqa: F401

__all__ = ["synth", "kfmi", "judge"]
