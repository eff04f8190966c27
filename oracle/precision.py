"""Round-to-nearest-even storage formats for the patch inverses (project
extension; the paper fixes no precision).  FP32 is numpy's own cast (IEEE RNE);
BF16 keeps the upper 16 bits of the FP32 pattern after adding the RNE bias
0x7FFF + (bit 16), written out from the format's definition.
"""
import numpy as np


def round_f32(A):
    return np.asarray(A, dtype=np.float64).astype(np.float32).astype(np.float64)


def round_bf16(A):
    f = np.asarray(A, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    bias = 0x7FFF + ((u >> 16) & 1)
    u = ((u + bias) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)
