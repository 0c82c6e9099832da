"""MI355X-native hot path of the CNOP search for the most dangerous initial
velocity perturbation in 2-D compressible Rayleigh-Taylor instability.

The compute path is the C-ABI library ``librtcnop.so`` (HIP kernels for
gfx950); :mod:`.rtcnop` is its thin Python binding.  Importing this package
does not load the library; :func:`rtcnop.load` does, and raises if it is
missing.
"""
from .config import RTConfig, WORKLOADS, paper_preset  # noqa: F401

__all__ = ["RTConfig", "WORKLOADS", "paper_preset"]
