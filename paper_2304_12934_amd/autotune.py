"""Autotuner front end: ``nr_autotune`` of the library does the work.

The library times forward + adjoint passes of the stack on the device for
candidate settings of the batch budget (``batch_mb``), the number of
concurrent streams (``streams``), the spreading tile (``tile_w`` x
``tile_h``) and the spreading item size (``chunk``), one parameter at a
time (coordinate search from the defaults), and caches the best setting
per geometry and device in a JSON file.  Every candidate computes the same
operator; only the float32 summation order of the spreading differs.
"""

from __future__ import annotations

import os
from typing import Sequence

import torch

from .radon import Plan, SliceGeometry


def default_cache_path() -> str:
    return os.path.join(os.path.expanduser("~"), ".cache", "nufftradon", "autotune.json")


def autotune(geoms: Sequence[SliceGeometry], width: int = 7, device: torch.device | str | None = None,
             cache_path: str | None = None, use_cache: bool = True) -> dict:
    """Best ``tuning`` dict for ``Plan(geoms, tuning=...)`` (measured by the
    library, then cached unless ``use_cache`` is False)."""
    path = (cache_path or default_cache_path()) if use_cache else None
    if path:
        os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    with Plan(geoms, width=width, device=device) as plan:
        return plan.autotune(path)
