"""Batched inpainting of images of uneven sizes (Section 4.3, Algorithm 3).

Images are grouped by size; each size has its own shearlet system, and one
shear_inpaint_groups call runs every group: the library captures the groups'
iteration sequences as parallel branches of one HIP graph and replays it with
one launch. Everything here is host-side grouping and marshalling.
"""
from __future__ import annotations

from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np
import torch

import ctypes

from ._binding import ShearletSystem, _check, _stream_ptr, load_library

__all__ = ["UnevenInpainter", "default_scales"]


def default_scales(rows: int, cols: int) -> int:
    """Scales per size: 3 (33 filters) up to 256 pixels on the short side, else 4 (49 filters)."""
    return 3 if min(rows, cols) <= 256 else 4


class UnevenInpainter:
    """Holds one system per image size, built on first use; each size's column-pass schedule is
    autotuned (shear_autotune) for the batch it first runs with."""

    def __init__(self, scales=default_scales, autotune: bool = True):
        self._scales = scales
        self._autotune = autotune
        self._systems: Dict[Tuple[int, int], ShearletSystem] = {}
        self._tuned: Dict[Tuple[int, int], int] = {}
        self.schedules: Dict[Tuple[int, int], Tuple[int, int]] = {}

    def system(self, rows: int, cols: int) -> ShearletSystem:
        key = (rows, cols)
        if key not in self._systems:
            self._systems[key] = ShearletSystem.build(rows, cols, self._scales(rows, cols))
        return self._systems[key]

    def run(self, f_masked: Sequence[torch.Tensor], masks: Sequence[torch.Tensor], schedules: Sequence,
            out: Optional[List[torch.Tensor]] = None) -> List[torch.Tensor]:
        """Inpaints image i (2-D float32 CUDA tensor) with mask i. schedules[i] is (iterations,) scalars
        delta (thresholds delta * RMS_k, Algorithm 3) or (iterations, K) per-filter thresholds; every image
        needs the same number of iterations within its size group. Returns the inpainted images."""
        n = len(f_masked)
        if len(masks) != n or len(schedules) != n:
            raise ValueError("f_masked, masks and schedules must have the same length")
        groups: Dict[Tuple[int, int], List[int]] = {}
        for i, t in enumerate(f_masked):
            if t.dim() != 2:
                raise ValueError("images must be 2-D")
            groups.setdefault((int(t.shape[0]), int(t.shape[1])), []).append(i)
        result: List[Optional[torch.Tensor]] = [None] * n
        systems, fms, mks, outs, batches, thrs, iters = [], [], [], [], [], [], set()
        for key, ids in groups.items():
            s = self.system(*key)
            if self._autotune and self._tuned.get(key) != len(ids):
                # the column-pass schedule of this size at this group's batch (synchronous)
                self.schedules[key] = s.autotune(len(ids))
                self._tuned[key] = len(ids)
            fm = torch.stack([f_masked[i] for i in ids]).contiguous()
            mk = torch.stack([masks[i] for i in ids]).contiguous()
            sch = [np.asarray(schedules[i], dtype=np.float64) for i in ids]
            if all(a.ndim == 1 for a in sch):
                # scalar deltas per iteration and image, weighted per filter by the library
                if len({a.shape[0] for a in sch}) != 1:
                    raise ValueError(f"images of size {key} need the same number of iterations")
                thr = s.inpaint_thresholds(np.stack(sch, axis=1), len(ids))
            elif all(a.ndim == 2 and a.shape[1] == s.K for a in sch):
                if len({a.shape[0] for a in sch}) != 1:
                    raise ValueError(f"images of size {key} need the same number of iterations")
                thr = np.ascontiguousarray(np.stack(sch, axis=1), dtype=np.float32)
            else:
                raise ValueError(f"schedules of size {key} must all be (iterations,) or all (iterations, {s.K})")
            iters.add(thr.shape[0])
            y = torch.empty_like(fm)
            systems.append(s)
            fms.append(fm)
            mks.append(mk)
            outs.append(y)
            batches.append(len(ids))
            thrs.append(torch.from_numpy(thr).to(fm.device))
            for j, i in enumerate(ids):
                result[i] = y[j]
        if len(iters) != 1:
            raise ValueError("every image needs the same number of iterations")
        G = len(systems)
        VP = ctypes.c_void_p * G
        _check(load_library().shear_inpaint_groups(
            VP(*[s._h for s in systems]), G, VP(*[t.data_ptr() for t in fms]), VP(*[t.data_ptr() for t in mks]),
            VP(*[t.data_ptr() for t in outs]), (ctypes.c_int * G)(*batches), VP(*[t.data_ptr() for t in thrs]),
            int(iters.pop()), _stream_ptr(None)), "shear_inpaint_groups")
        # the graph reads these buffers when it runs: keep them alive until the next call
        self._keep = (fms, mks, outs, thrs)
        return result  # type: ignore[return-value]

    def close(self) -> None:
        for s in self._systems.values():
            s.close()
        self._systems.clear()
