"""Exchange tile autotuner: times every exchange tile variant and Q split that fits a shape.

For a context (one operator, a fixed RHS count), each candidate (variant, splits) runs a few
propagation steps with the library's per-kernel-class event profiling on, and the candidate
with the smallest average exchange launch time wins.  Results are cached in a JSON file keyed
by (precision, o, v, N_Q, nrhs, integrator) so later contexts of the same shape reuse the choice:
the split operator launches the exchange on R real slices instead of RK4's 2R, which favours
other tiles.

    from paper_2601_16949_amd import autotune
    best = autotune.tune(ctx, pulses, dt, nrhs)      # applies the best setting to ctx
"""
from __future__ import annotations

import json
import os
from typing import Dict, List, Optional

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_CACHE = os.path.join(HERE, "autotune_cache.json")


def _key(ctx, nrhs: int, integrator: str = "rk4") -> str:
    d = ctx.desc
    return f"p{d.precision}_o{d.n_occ}_v{d.n_virt}_nq{d.n_aux}_r{nrhs}" + ("_sso" if integrator == "sso" else "")


def load_cache(path: str = DEFAULT_CACHE) -> Dict[str, dict]:
    if os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def save_cache(cache: Dict[str, dict], path: str = DEFAULT_CACHE):
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def variant_index(ctx, name: str) -> int:
    """1-based index of the exchange variant called `name` in the loaded library (0 if absent)."""
    n = ctx.lib.rttda_exchange_variants(ctx.desc.precision)
    for k in range(1, n + 1):
        if ctx.variant_name(k) == name:
            return k
    return 0


def apply(ctx, entry: dict) -> bool:
    """Apply a cached (variant name, splits[, Q chunk]) choice; False if the loaded library lacks the variant."""
    k = variant_index(ctx, entry["name"])
    if not k:
        return False
    splits = min(int(entry["splits"]), ctx.max_splits())
    ctx.set_tuning(exchange_variant=k, exchange_splits=splits, exchange_chunk=int(entry.get("chunk", 0)) or -1)
    return True


def lookup(ctx, nrhs: int, cache_path: str = DEFAULT_CACHE, integrator: str = "rk4") -> Optional[dict]:
    return load_cache(cache_path).get(_key(ctx, nrhs, integrator))


GEMM_CHUNKS = (0, 6, 12)  # Q per chunk tried for the large-o GEMM path (0 = as many as fit)


def candidates(ctx, max_per_variant: int = 5) -> List[tuple]:
    """(variant, splits, Q chunk) triples: every variant holding o, with splits from half to four
    times the library's default (at most what the workspace holds); the GEMM path also over a
    few chunk lengths (0 elsewhere)."""
    lib = ctx.lib
    prec = ctx.desc.precision
    n = lib.rttda_exchange_variants(prec)
    base = ctx.get_tuning()
    out = []
    for k in range(1, n + 1):
        try:
            ctx.set_tuning(exchange_variant=k)
        except Exception:
            continue  # variant does not hold o
        s0 = ctx.get_tuning()["exchange_splits"]
        chunks = GEMM_CHUNKS if ctx.variant_name(k).startswith("bf16x2gemm") else (0,)
        smax = ctx.max_splits()
        for s in sorted({min(smax, max(1, s0 * m // 2)) for m in (1, 2, 4, 6, 8)})[:max_per_variant]:
            for ch in chunks:
                out.append((k, s, ch))
    ctx.set_tuning(exchange_variant=base["exchange_variant"], exchange_splits=base["exchange_splits"])
    return out


def measure(ctx, pulses, dt: float, c0, c, steps: int = 3, integrator: str = "rk4") -> float:
    """Average time (ms) per exchange launch of the exchange plus the epilogue after it (which
    reads one partial slab per Q split, so more splits cost there) over `steps` steps."""
    import torch

    ctx.set_profiling(True)
    ctx.propagate(pulses, dt, steps, c0, c, want_trace=False, integrator=integrator)
    torch.cuda.synchronize()
    prof = ctx.get_profile()
    ctx.set_profiling(False)
    ex, ep = prof["exchange"], prof["epilogue"]
    return (ex["ms"] + ep["ms"]) / max(ex["launches"], 1)


def tune(ctx, pulses, dt: float, nrhs: Optional[int] = None, steps: int = 3, cache_path: str = DEFAULT_CACHE,
         use_cache: bool = True, verbose: bool = False, integrator: str = "rk4") -> dict:
    from . import rttda

    nrhs = nrhs or len(pulses)
    key = _key(ctx, nrhs, integrator)
    cache = load_cache(cache_path) if use_cache else {}
    if key in cache:
        best = cache[key]
        apply(ctx, best)
        return best
    c0, c = rttda.ground_state(nrhs, ctx.o, ctx.v, device=ctx.device)
    results = []
    for k, s, ch in candidates(ctx):
        try:
            ctx.set_tuning(exchange_variant=k, exchange_splits=s, exchange_chunk=ch or -1)
        except rttda.RttdaError:
            continue
        measure(ctx, pulses, dt, c0, c, steps=1, integrator=integrator)  # warm
        ms = measure(ctx, pulses, dt, c0, c, steps=steps, integrator=integrator)
        results.append({"variant": k, "name": ctx.variant_name(k), "splits": s, "chunk": ch, "ms": ms})
        if verbose:
            print(f"  {ctx.variant_name(k):34s} splits {s:3d} chunk {ch:3d}: {ms * 1e3:10.1f} us", flush=True)
    best = min(results, key=lambda r: r["ms"])
    ctx.set_tuning(exchange_variant=best["variant"], exchange_splits=best["splits"],
                   exchange_chunk=best["chunk"] or -1)
    best = dict(best, candidates=len(results))
    if use_cache:
        cache[key] = best
        save_cache(cache, cache_path)
    return best
