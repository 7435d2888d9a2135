"""Shared helpers of the GPU parity tests (the HIP path through the C ABI
against the CPU oracle on the same seeded inputs)."""
from __future__ import annotations

import sys

import numpy as np

import datagen

UINT64_MAX = 2 ** 64 - 1


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def slice_table(t: datagen.Table, lo: int, hi: int) -> datagen.Table:
    """Rows [lo, hi) as a host table (lo a multiple of 32 for validity)."""
    assert lo % 32 == 0
    s = datagen.Table(f"{t.name}[{lo}:{hi}]", hi - lo)
    for c in t.columns:
        v = None
        if c.valid is not None:
            v = c.valid[lo // 32:(hi + 31) // 32]
        s.columns.append(datagen.Column(c.name, c.type, c.data[lo:hi], v, c.dict_card))
    return s


def ids_tensor(n, torch, fill=0xDEADBEEF):
    """Output buffer for row ids prefilled with a sentinel."""
    t = torch.full((max(1, n),), fill - 2 ** 32 if fill >= 2 ** 31 else fill,
                   dtype=torch.int32, device="cuda")
    return t


def as_u32(t) -> np.ndarray:
    return t.cpu().numpy().view(np.uint32)
