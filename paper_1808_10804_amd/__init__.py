"""MI355X-native block-sparse symmetric CTM contractions (libsymten binding).

The compute path lives in libsymten.so (HIP for gfx950, C ABI in
include/symten.h); this package only loads it and marshals arguments.
"""
from . import _lib
from .symten import (Tensor, CtmEnv, CtmCell, contract, contract_noalloc, match_blocks, eigh, eigh_max_order, plan_info, double_layer, double_layer_op, enlarged_corner, enlarged_corner_single_layer, profile_begin, profile_end,
                     enlarged_corners_batched, sync, su2_cg, set_allocator, use_torch_allocator, IN, OUT)
from ._lib import SymtenError

__all__ = ["Tensor", "CtmEnv", "CtmCell", "contract", "contract_noalloc", "match_blocks", "eigh", "eigh_max_order", "plan_info", "double_layer", "double_layer_op", "enlarged_corner", "enlarged_corner_single_layer",
           "enlarged_corners_batched", "sync", "su2_cg", "set_allocator", "use_torch_allocator", "profile_begin", "profile_end", "IN", "OUT",
           "SymtenError"]
