"""MI355X (gfx950) one-site TDVP sweep for tree tensor networks (after pyTTN, arXiv 2503.15460).

The package is a thin binding over the HIP library ``libttn.so`` built from
``csrc/``; see ``include/ttn.h`` for the C boundary.
"""
from ._lib import (OBS_BILINEAR, OBS_ENERGY, OBS_EXPECT, OBS_NORM, OBS_OVERLAP_T0, TTN, TTN_BF16X3, TTN_FP32, TTN_FP64,
                   TTNBatch, TTNError, clamp_bonds, dense_tree_operator, gpu_qr, hermiticity_defect, lib, tile_table_clear, tile_table_load, tile_table_save, tile_table_size, tree_operator_stats, profile_begin, profile_end,
                   tree_operator_entries)

__all__ = ["TTN", "TTNBatch", "TTNError", "TTN_FP64", "TTN_FP32", "TTN_BF16X3", "clamp_bonds", "dense_tree_operator", "tree_operator_entries", "hermiticity_defect", "tree_operator_stats", "tile_table_save", "tile_table_load", "tile_table_size", "tile_table_clear", "gpu_qr", "lib", "profile_begin", "profile_end",
           "OBS_EXPECT", "OBS_NORM", "OBS_ENERGY", "OBS_OVERLAP_T0", "OBS_BILINEAR"]
