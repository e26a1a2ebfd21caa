"""Tiling choices of the projector pair (the ray-bundle split of the subset projection:
primary steps or planes per wavefront; the gather backprojection: strips of columns or
whole columns), found by timing on the GPU (spdhg_autotune) and kept in a JSON cache keyed
by the problem's shape class."""
from __future__ import annotations

import json
import os
from typing import Dict, Iterable, Optional


def shape_key(g, n_subsets: int) -> str:
    """Problems with equal keys launch identically shaped projections."""
    scanner = (f"-R{g.det_radius:g}-na{int(g.nonarc)}-os{int(g.oblique_s)}-span{g.span}"
               if getattr(g, "nonarc", False) or getattr(g, "oblique_s", False)
               or getattr(g, "span", 0) else "")
    return (f"img{g.nx}x{g.ny}x{g.nz}-sino{g.n_rad}x{g.n_ang}x{sum(g.seg_planes)}"
            f"-seg{len(g.seg_planes)}-m{n_subsets}{scanner}")


def load_cache(path: Optional[str]) -> Dict[str, dict]:
    if path and os.path.exists(path):
        with open(path) as fh:
            return json.load(fh)
    return {}


def save_cache(path: Optional[str], cache: Dict[str, dict]) -> None:
    if not path:
        return
    tmp = f"{path}.tmp{os.getpid()}"
    with open(tmp, "w") as fh:
        json.dump(cache, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def autotune(recs: Iterable, cache_path: Optional[str] = None) -> Dict[str, dict]:
    """Apply the cached split to every Reconstruction whose shape class is known; time
    the others once per class (spdhg_autotune) and add them to the cache."""
    cache = load_cache(cache_path)
    for rec in recs:
        key = shape_key(rec.g, rec.params.n_subsets)
        if key in cache:
            rec.set_tuning(int(cache[key]["fwd_split"]))
            rec.set_gather(int(cache[key].get("gather", 0)))
        else:
            split, ms = rec.autotune()
            cache[key] = {"fwd_split": split, "gather": rec.tuning()[1],
                          "ms_per_projection": round(ms, 4)}
    save_cache(cache_path, cache)
    return cache
