"""MI355X (gfx950) implementation of the AIM-accelerated GIBC surface integral
equation method (Sharma & Triverio, arXiv:2003.11679).

The computation lives in the HIP library ``libsie.so`` (C ABI in
``include/sie.h``); :mod:`paper_2003_11679_amd.sie` is its ctypes binding.
"""
from .sie import (Problem, Context, Server, SieError, lib, FP64, FP32, OP_L, OP_K, OP_X, OP_AUG,
                  EXTERIOR, INTERIORS, set_tuning, tuning_force, tuning_report, tuning_clear)

__all__ = ["Problem", "Context", "Server", "SieError", "lib", "FP64", "FP32", "OP_L", "OP_K", "OP_X", "OP_AUG",
           "EXTERIOR", "INTERIORS", "set_tuning", "tuning_force", "tuning_report", "tuning_clear"]
