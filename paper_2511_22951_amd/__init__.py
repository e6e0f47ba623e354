"""md950: MI355X-native short-range molecular dynamics (cell lists, Verlet lists,
Lennard-Jones and EAM forces, velocity Verlet) behind the C ABI of include/md.h.

The compute path is the HIP library libmd950.so built by build.py; this package
only marshals arguments.  Importing it does not touch the GPU.
"""
from ._native import (MD_ALWAYS, MD_FP32, MD_FP64, MD_IF_FLAGGED, MD_KICK, MD_KICK_DRIFT,  # noqa
                      MDError, lib, LIB_PATH, EXPORTED)

__all__ = ["MD_ALWAYS", "MD_FP32", "MD_FP64", "MD_IF_FLAGGED", "MD_KICK", "MD_KICK_DRIFT",
           "MDError", "lib", "LIB_PATH", "EXPORTED"]
