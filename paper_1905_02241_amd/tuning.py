"""Autotuner cache: launch shapes of the batched path chosen by
mech_autotune, keyed by (GPU architecture, workload signature, precision).

The cache is a JSON file; entries are written by ``record`` and read by
``lookup``.  A shape is (block, tile_instances, tile_nodes, blocks_per_cu,
flags) as taken by mech_set_launch.
"""
from __future__ import annotations

import json
import os
from typing import Optional, Tuple

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning.json")


def signature(w) -> str:
    counts = ",".join(f"{s.kind}:{s.n}" for s in w.slots)
    return f"{w.name}|{w.n_nodes}|{counts}|{w.vmode}"


def arch() -> str:
    import torch
    name = torch.cuda.get_device_properties(0).gcnArchName
    return name.split(":")[0]


def _load(path: str) -> dict:
    if os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def lookup(w, prec: str, path: str = CACHE) -> Optional[Tuple[int, ...]]:
    e = _load(path).get(arch(), {}).get(signature(w), {}).get(prec)
    return tuple(e["launch"]) if e else None


def record(w, prec: str, launch, ms_per_step: float, path: str = CACHE) -> None:
    d = _load(path)
    d.setdefault(arch(), {}).setdefault(signature(w), {})[prec] = {"launch": list(launch),
                                                                  "ms_per_step": ms_per_step}
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)
    os.replace(tmp, path)
