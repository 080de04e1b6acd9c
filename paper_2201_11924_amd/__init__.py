"""MI355X-native depth stage of the active stereo sensor simulator (SimSense).

The compute path lives in ``libsimsense.so`` (hand-written HIP for gfx950,
C ABI in ``include/simsense.h``); :mod:`paper_2201_11924_amd.native` is its
thin ctypes binding.  Importing the binding without a built library raises.
"""
import importlib

__all__ = ["native", "build", "train", "workloads"]


def __getattr__(name):
    if name in ("native", "build", "train", "workloads"):
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
