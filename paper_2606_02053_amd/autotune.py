"""Tile autotuner for the stage kernel.

Searches the kernel variant (LDS-staged bricks, or direct loads through the
caches), the brick owned by one 256-thread workgroup (tile_x x tile_y x
tile_z, x fastest) and the brick order (XCD slabs, linear, or XCD-blocked), times
full RK4 steps of each candidate with HIP events on the launch stream, and
keeps the fastest. A candidate is eligible only if its right-hand side is
bitwise identical to its variant's default brick on the same state (the brick
changes the schedule, never the arithmetic), and that variant agrees with the
other one to round-off (max relative difference 1e-13 per field). Results are cached as JSON keyed by
(gfx arch, grid, variant) in $COSMOS_TUNE_CACHE (default
~/.cache/cosmos_tune.json).
"""
from __future__ import annotations

import json
import os

import torch

from . import _lib as C

LDS_BRICKS = [(16, 4, 4), (16, 8, 2), (8, 8, 4), (8, 4, 8)]
DIRECT_TILES = [(256, 1, 1), (64, 4, 1), (32, 8, 1), (32, 4, 2), (16, 16, 1), (16, 4, 4), (8, 8, 4)]
ORDERS = (0, 1, 2)  # XCD slabs, linear, XCD-blocked (the last only for the LDS-staged variant)
# (variant, tile, order): variant 0 = LDS-staged bricks, 1 = direct loads
CANDIDATES = [(0, t, o) for t in LDS_BRICKS for o in ORDERS] + [(1, t, o) for t in DIRECT_TILES for o in ORDERS[:2]]


def _cache_path() -> str:
    return os.environ.get("COSMOS_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "cosmos_tune.json"))


def _key(grid: C.cosmos_grid, variant: str) -> str:
    arch = torch.cuda.get_device_properties(torch.cuda.current_device()).gcnArchName.split(":")[0]
    return f"{arch}:{grid.n[0]}x{grid.n[1]}x{grid.n[2]}:{variant}"


def load(grid: C.cosmos_grid, variant: str = "rk4"):
    try:
        with open(_cache_path()) as f:
            e = json.load(f).get(_key(grid, variant))
        return (e["variant"], tuple(e["tile"]), e["order"]) if e else None
    except (OSError, ValueError, KeyError):
        return None


def _store(grid, variant, entry):
    path = _cache_path()
    try:
        with open(path) as f:
            db = json.load(f)
    except (OSError, ValueError):
        db = {}
    db[_key(grid, variant)] = entry
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(db, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def with_tile(params: C.cosmos_params, variant, tile, order) -> C.cosmos_params:
    p = C.cosmos_params.from_buffer_copy(params)
    p.variant = variant
    p.tile_x, p.tile_y, p.tile_z = tile
    p.tile_order = order
    return p


def tune(grid: C.cosmos_grid, params: C.cosmos_params, u: torch.Tensor, dt: float, steps: int = 2,
         candidates=None, variant: str = "rk4", use_cache: bool = True, verbose: bool = False):
    """Returns ((kernel_variant, tile, order), table). `u` is a representative state (not modified)."""
    if use_cache:
        hit = load(grid, variant)
        if hit is not None:
            return hit, None
    cands = candidates or CANDIDATES
    ws = torch.empty(C.cosmos_workspace_bytes(grid), dtype=torch.uint8, device=u.device)
    refs = {}
    for kv, tile in ((0, (16, 4, 4)), (1, (16, 4, 4))):
        refs[kv] = torch.empty_like(u)
        C.cosmos_rhs(grid, with_tile(params, kv, tile, 0), 0.0, u, refs[kv], ws)
    d = (refs[0] - refs[1]).abs().reshape(C.NFIELDS, -1).amax(dim=1)
    sc = refs[0].abs().reshape(C.NFIELDS, -1).amax(dim=1).clamp_min(1e-3)
    variants_agree = bool(((d / sc).max() < 1e-13).item())
    work = torch.empty_like(u)
    out = torch.empty_like(u)
    stream = torch.cuda.current_stream()
    table = []
    for kv, tile, order in cands:
        p = with_tile(params, kv, tile, order)
        C.cosmos_rhs(grid, p, 0.0, u, out, ws)
        if not torch.equal(out, refs[kv]) or not variants_agree:
            table.append({"variant": kv, "tile": tile, "order": order, "ms_per_step": None, "parity": False})
            continue
        work.copy_(u)
        C.cosmos_rk4_step(grid, p, 0.0, dt, work, ws)  # warm-up
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for s in range(steps):
            C.cosmos_rk4_step(grid, p, s * dt, dt, work, ws)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        table.append({"variant": kv, "tile": tile, "order": order, "ms_per_step": ms, "parity": True})
        if verbose:
            print(f"variant {kv} tile {tile} order {order}: {ms:.3f} ms/step", flush=True)
    ok = [r for r in table if r["parity"]]
    best = min(ok, key=lambda r: r["ms_per_step"])
    _store(grid, variant, {"variant": best["variant"], "tile": list(best["tile"]), "order": best["order"],
                           "ms_per_step": best["ms_per_step"], "table": [dict(r, tile=list(r["tile"])) for r in table]})
    return (best["variant"], tuple(best["tile"]), best["order"]), table
