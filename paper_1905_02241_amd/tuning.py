"""Autotuner cache: launch shapes chosen by mech_autotune (batched path) and
mech_autotune_resident (time-fused path), keyed by (GPU architecture,
workload signature, precision[-resident]).

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


def _key(prec: str, step_path: str) -> str:
    return prec if step_path == "batched" else f"{prec}-{step_path}"


def lookup(w, prec: str, path: str = CACHE, step_path: str = "batched") -> Optional[Tuple[int, ...]]:
    e = _load(path).get(arch(), {}).get(signature(w), {}).get(_key(prec, step_path))
    return tuple(e["launch"]) if e else None


def record(w, prec: str, launch, ms_per_step: float, path: str = CACHE, step_path: str = "batched") -> None:
    d = _load(path)
    d.setdefault(arch(), {}).setdefault(signature(w), {})[_key(prec, step_path)] = {
        "launch": list(launch), "ms_per_step": ms_per_step}
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)
    os.replace(tmp, path)
