"""Autotuning of the level-step launch shape: steps per prediction pass and per-level tiles.

Host logic over the C ABI (sf_set_pass_steps, sf_set_tile): candidate settings are applied to
a live context, a few frames are pushed with each, and the setting with the lowest wall time
per frame is kept.  Every candidate computes the same
result (tile shapes and pass splits change only which block computes a pixel), so tuning never
changes the output.  Results can be cached in a JSON file keyed by the device and the streams'
configuration.
"""
from __future__ import annotations

import json
import math
import os
from typing import Callable, Dict, List, Optional, Sequence, Tuple

from . import sflow

REGION = 64   # side of the register tile region of the level-step kernel


def _halo(steps: int, smooth: int) -> int:
    return max(steps, 2) + 2 * smooth


def _level_steps(max_flow: float, h: int) -> int:
    return max(1, math.ceil(max_flow / 2 ** h))


def tile_candidates(rows: int, cols: int, halo: int) -> List[Tuple[int, int]]:
    """A few output tile shapes for a level: the largest square, and shorter tiles that keep
    the width (shorter regions leave whole waves idle, which helps when the level is the
    critical path)."""
    tmax = REGION - 2 * halo
    if tmax < 1:
        return []
    out = []
    for th in (tmax, tmax - 4, tmax - 8, tmax - 16):
        if th >= 8:
            out.append((min(tmax, cols), min(th, rows)))
    return list(dict.fromkeys(out))


def _frame_time(ctx: int, push: Callable[[int], None], frames: int, warmup: int) -> float:
    """wall milliseconds per frame (the level steps of a frame overlap on two streams, so the
    sum of kernel times is not the frame's time)"""
    import time
    import torch
    for k in range(warmup):
        push(k)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(frames):
        push(warmup + k)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / max(1, frames)


def tune(ctx: int, push: Callable[[int], None], levels: Sequence[dict],
         pass_steps: Sequence[int] = (4, 6, 8, 12, 16), frames: int = 6, warmup: int = 2,
         tiles: bool = True, log: Optional[Callable[[str], None]] = None) -> Dict:
    """Tune a context in place.  `push(k)` pushes frame k to every stream of the context;
    `levels` describes the levels (dicts with rows, cols, max_flow_px, smooth, h) of the
    stream that dominates the cost (its tile candidates are tried, applied to that level of
    every stream).  Returns the chosen setting and the measured times (ms per frame)."""
    best = {"pass_steps": 8, "tiles": {}, "ms": float("inf")}
    trials = []
    for ps in pass_steps:
        try:
            sflow.sf_set_pass_steps(ctx, ps)
        except sflow.SflowError:
            continue
        t = _frame_time(ctx, push, frames, warmup)
        trials.append({"pass_steps": ps, "ms": t})
        if log:
            log(f"pass steps {ps}: {t * 1e3:.1f} us per frame")
        if t < best["ms"]:
            best = {"pass_steps": ps, "tiles": {}, "ms": t}
    sflow.sf_set_pass_steps(ctx, best["pass_steps"])
    if tiles:
        for L in levels:
            steps = _level_steps(L["max_flow_px"], L["h"])
            P = math.ceil(steps / best["pass_steps"])
            last = steps - (P - 1) * math.ceil(steps / P)
            halo = _halo(last, L["smooth"])
            keep = None
            for tw, th in tile_candidates(L["rows"], L["cols"], halo):
                try:
                    sflow.sf_set_tile(ctx, L["h"] + 1, tw, th)
                except sflow.SflowError:
                    continue
                t = _frame_time(ctx, push, frames, warmup)
                trials.append({"level": L["h"] + 1, "tile": [tw, th], "ms": t})
                if log:
                    log(f"level {L['h'] + 1} tile {tw}x{th}: {t * 1e3:.1f} us per frame")
                if t < best["ms"]:
                    best["ms"] = t
                    keep = (tw, th)
            if keep:
                best["tiles"][L["h"] + 1] = list(keep)
            sflow.sf_set_tile(ctx, L["h"] + 1, *(keep or (0, 0)))
    best["trials"] = trials
    return best


def apply(ctx: int, setting: Dict) -> None:
    """Apply a setting returned by tune (or loaded from a cache)."""
    sflow.sf_set_pass_steps(ctx, int(setting["pass_steps"]))
    for level, (tw, th) in setting.get("tiles", {}).items():
        sflow.sf_set_tile(ctx, int(level), int(tw), int(th))


def cache_key(device_name: str, specs: Sequence[dict], storage: int) -> str:
    parts = [device_name, "fp16" if storage == 1 else "fp32"]
    for sp in specs:
        parts.append(f"{sp['rows']}x{sp['cols']}:{sp['levels']}:{sp['max_flow_px']}:"
                     f"{'/'.join(str(s) for s in sp['smooth'])}")
    return "|".join(parts)


def load_cache(path: str) -> Dict:
    if not os.path.exists(path):
        return {}
    with open(path) as fh:
        return json.load(fh)


def store_cache(path: str, key: str, setting: Dict) -> None:
    data = load_cache(path)
    data[key] = {k: v for k, v in setting.items() if k != "trials"}
    with open(path, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
