"""MI355X-native narrow-phase contact detection for rigid triangulated particles.

The compute path is libmcd.so (gfx950 HIP kernels behind the C ABI in
include/mcd.h); :mod:`paper_2309_15417_amd.mcd` is a thin ctypes binding with
the same call names. There is no CPU fallback: without the built library, or
without a GPU, creating a context raises.
"""

from .mcd import (Context, MCDError, lib_path, load_library, exported_symbols,
                  header_symbols, PAIR_RESULT_DT, CONTACT_DT, STATS_DT,
                  Q_FP64, Q_MIXED, Q_DENSE, Q_TIMING, Q_CLOSEST, Q_CONTACTS, Q_VALIDATE,
                  Q_NARROW, Q_FUSE, Q_DEVICE_OUT, CFG_NO_GRAPHS, CFG_NO_TUNE, NONE, AT_START, COLLIDES)

__all__ = ["Context", "MCDError", "lib_path", "load_library", "exported_symbols",
           "header_symbols", "PAIR_RESULT_DT", "CONTACT_DT", "STATS_DT", "Q_FP64", "Q_MIXED",
           "Q_DENSE", "Q_TIMING", "Q_CLOSEST", "Q_CONTACTS", "Q_VALIDATE", "Q_NARROW", "Q_FUSE", "Q_DEVICE_OUT",
           "CFG_NO_GRAPHS", "CFG_NO_TUNE", "NONE", "AT_START", "COLLIDES"]
