"""Oracle for the pore-space connectivity pre-processing.

TEST INFRASTRUCTURE ONLY (see the package docstring).  §5.1 lists the
elimination of disconnected pore space among the pre-processing steps and
states that the solver assumes percolation; the clogging study of §7.3
simulates a direction only while a flow path through the domain remains.

Definitions used here (the domain is periodic on all three axes):
  * pore voxels (mask byte 0) are connected through shared faces
    (6-connectivity, across the periodic boundaries too);
  * a component is labelled by its smallest linear voxel index;
  * a component percolates along axis j when it contains a closed path that
    winds around the domain along j: following the path in the unwrapped
    (periodically repeated) space, it ends at a copy of its start shifted by
    a nonzero multiple of n_j along j.

The search is a breadth-first traversal that carries each voxel's unwrapped
position; reaching an already visited voxel at a different unwrapped
position exposes a winding vector (the difference, in periods).
"""
from __future__ import annotations

from collections import deque
from dataclasses import dataclass

import numpy as np


@dataclass
class PoreRef:
    labels: np.ndarray        # int64 [nz, ny, nx]: smallest index of the component, -1 for solid
    n_components: int
    windings: dict            # label -> set of winding vectors (periods along x, y, z), nonzero ones
    percolates: tuple         # axis j -> some component winds along j
    flow: np.ndarray          # uint8 [nz, ny, nx]: bit j set for pore voxels of components winding along j


def components(mask: np.ndarray) -> PoreRef:
    mask = np.asarray(mask)
    nz, ny, nx = mask.shape
    dims = (nx, ny, nz)
    labels = -np.ones(mask.shape, dtype=np.int64)
    unwrapped = {}
    windings = {}
    flat = mask.reshape(-1)
    for start in range(flat.size):
        if flat[start] or labels.reshape(-1)[start] >= 0:
            continue
        # start is the smallest index of a new component: the scan runs in index order
        sx, sy, sz = start % nx, (start // nx) % ny, start // (nx * ny)
        labels[sz, sy, sx] = start
        unwrapped[start] = (sx, sy, sz)
        wset = set()
        queue = deque([start])
        while queue:
            t = queue.popleft()
            ux, uy, uz = unwrapped[t]
            for d in range(3):
                for step in (-1, 1):
                    q = [ux, uy, uz]
                    q[d] += step
                    x, y, z = q[0] % nx, q[1] % ny, q[2] % nz
                    if mask[z, y, x]:
                        continue
                    s = (z * ny + y) * nx + x
                    if labels[z, y, x] < 0:
                        labels[z, y, x] = start
                        unwrapped[s] = tuple(q)
                        queue.append(s)
                    else:
                        prev = unwrapped[s]
                        w = tuple((q[i] - prev[i]) // dims[i] for i in range(3))
                        if any(w):
                            wset.add(w)
        windings[start] = wset
    perc = [False, False, False]
    flow = np.zeros(mask.shape, dtype=np.uint8)
    for lab, wset in windings.items():
        bits = 0
        for j in range(3):
            if any(w[j] != 0 for w in wset):
                bits |= 1 << j
                perc[j] = True
        if bits:
            flow[labels == lab] = bits
    return PoreRef(labels, len(windings), windings, tuple(perc), flow)


def cleaned_mask(mask: np.ndarray, axis: int) -> np.ndarray:
    """The mask with every pore voxel of a component that does not wind along
    `axis` made solid (such a component carries no flow under a drive along
    `axis`: p = G x_axis balances the drive in it)."""
    ref = components(mask)
    keep = (ref.flow >> axis) & 1
    return np.where(keep == 1, 0, 1).astype(np.uint8)
