"""Launch-shape autotuner for the batched decode.

Searches the launch shape (chunk group of the fused schedule, waves per
block, windows per chunk, grid size) on the caller's own batch, one
coordinate at a time from the library defaults: every candidate runs the
whole step (plan + decode kernels) timed with HIP events, best of three
trials, and the fastest value of each coordinate is kept before the next one
is searched.  Each candidate's output must equal the first candidate's bit for
bit (the launch shape never changes the arithmetic), or tuning fails.

Results are cached in a JSON file outside the package (FPTC_AUTOTUNE_CACHE, or
~/.cache/fptc/autotune.json), keyed by device name, codec shape, precision,
path and the batch's size class.
"""
from __future__ import annotations

import json
import os
import tempfile
import time

import torch

from .codec import Decoder, Launch


def cache_path() -> str:
    env = os.environ.get("FPTC_AUTOTUNE_CACHE")
    if env:
        return env
    base = os.path.join(os.path.expanduser("~"), ".cache", "fptc")
    try:
        os.makedirs(base, exist_ok=True)
        if os.access(base, os.W_OK):
            return os.path.join(base, "autotune.json")
    except OSError:
        pass
    return os.path.join(tempfile.gettempdir(), "fptc_autotune.json")


def _key(batch, codec, precision, fused):
    name = torch.cuda.get_device_name(batch.word_off.device)
    size = f"2^{max(0, int(batch.n_samples).bit_length() - 1)}samples"
    return (f"{name}|N{codec.N}|E{codec.E}|books{codec.n_books}|rows{codec.n_rows}|{precision}|"
            f"{'fused' if fused else 'split'}|{size}|streams2^{int(batch.n_streams).bit_length() - 1}")


def _shape(l: Launch):
    return [l.windows_per_chunk, l.waves_per_block, l.blocks, l.chunk_group]


def _time(dec: Decoder, precision, fused, reps=3, trials=5):
    dec.run(precision=precision, fused=fused)
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(trials):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            dec.run(precision=precision, fused=fused)
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1) / reps)
    return best


def search_space(codec, fused, n_cu):
    """Coordinates in search order, each with its candidate values (the
    library default first)."""
    space = []
    if fused and codec.N <= 128:
        space.append(("chunk_group", [0, 1, 2, 8, 16]))
    if codec.N <= 64:
        space.append(("waves_per_block", [0, 12, 8]))
    elif codec.N == 128:
        space.append(("waves_per_block", [0, 4]))
    # window 256: one wave per (parity, column tile), always 8
    space.append(("windows_per_chunk", [0, 64, 16]))
    space.append(("blocks", [0, 2 * n_cu]))
    return space


def tune(batch, codec, precision="fp16x2", fused=True, use_cache=True, verbose=False):
    """Return (best Launch, info) with info = {"shape", "times", "tuning_s",
    "cached", "candidates"}."""
    t0 = time.perf_counter()
    key = _key(batch, codec, precision, fused)
    path = cache_path()
    cache = {}
    if use_cache and os.path.exists(path):
        try:
            with open(path) as f:
                cache = json.load(f)
        except (OSError, ValueError):
            cache = {}
        if key in cache:
            w, v, b, g = cache[key]["shape"]
            info = dict(cache[key])
            info.update(cached=True, tuning_s=time.perf_counter() - t0)
            return Launch(w, v, b, g), info
    n_cu = torch.cuda.get_device_properties(batch.word_off.device).multi_processor_count
    times = {}
    ref = None
    best = Launch()
    best_ms = float("inf")

    def measure(cand: Launch):
        nonlocal ref
        k = "/".join(str(v) for v in _shape(cand))
        if k in times:
            return times[k]
        try:
            dec = Decoder(batch, codec, cand)
            ms = _time(dec, precision, fused)
        except Exception as exc:  # shape refused by the library (LDS budget)
            if verbose:
                print("autotune: skip", cand, exc)
            times[k] = None
            return None
        out = dec.out[: batch.n_samples]
        if ref is None:
            ref = out.clone()
        elif not torch.equal(out, ref):
            raise RuntimeError(f"launch shape {cand} changed the decoded samples")
        if int((dec.status != 0).sum()) != 0:
            raise RuntimeError(f"launch shape {cand} reported stream errors")
        times[k] = ms
        if verbose:
            print(f"autotune: {cand} {ms:.4f} ms")
        del dec
        return ms

    # bring the clocks up before the first candidate is timed, so that the
    # default is not measured colder than the shapes tried after it
    try:
        warm = Decoder(batch, codec, best)
        t_w = time.perf_counter()
        for _ in range(50):
            warm.run(precision=precision, fused=fused)
            torch.cuda.synchronize()
            if time.perf_counter() - t_w > 0.05:
                break
        del warm
    except Exception:  # the default refused: reported below
        pass
    best_ms = measure(best)
    if best_ms is None:
        raise RuntimeError("the default launch shape was refused")
    # coordinate search, repeated while a pass changes the shape (a later
    # coordinate's change can make another value of an earlier one pay)
    for _ in range(3):
        start = best
        for field, values in search_space(codec, fused, n_cu):
            for v in values:
                cand = Launch(**{**best.__dict__, field: v})
                ms = measure(cand)
                if ms is not None and ms < best_ms * 0.995:  # keep a change only when it measurably helps
                    best, best_ms = cand, ms
        if _shape(best) == _shape(start):
            break
    info = {"shape": _shape(best), "best_ms": best_ms, "times": times, "candidates": len(times),
            "key": key, "cached": False, "tuning_s": time.perf_counter() - t0}
    if use_cache:
        cache[key] = {k: v for k, v in info.items() if k not in ("cached", "tuning_s")}
        tmp = path + f".tmp{os.getpid()}"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1)
        os.replace(tmp, path)
    return best, info
