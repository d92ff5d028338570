"""Launch-shape autotuner for the batched decode.

Times candidate shapes (windows per chunk, waves per block, grid size) on the
caller's own batch with HIP events and keeps the fastest, cached in a JSON file
keyed by device name, codec shape, precision and path.  Each candidate's output
must equal the first candidate's bit for bit (the launch shape never changes
the arithmetic), so a shape that breaks that is rejected.
"""
from __future__ import annotations

import json
import os

import torch

from .codec import Decoder, Launch

CACHE = os.environ.get("FPTC_AUTOTUNE_CACHE", os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                                           "autotune_cache.json"))

CANDIDATES = [Launch(32, 0, 0), Launch(32, 8, 0), Launch(32, 12, 0), Launch(32, 16, 0), Launch(64, 0, 0),
              Launch(64, 16, 0)]


def _key(batch, codec, precision, fused):
    name = torch.cuda.get_device_name(batch.word_off.device)
    size = "small" if batch.n_samples < (1 << 24) else "large"
    return f"{name}|N{codec.N}|E{codec.E}|books{codec.n_books}|{precision}|{'fused' if fused else 'split'}|{size}"


def _time(dec: Decoder, precision, fused, reps=5):
    dec.run(precision=precision, fused=fused)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dec.run(precision=precision, fused=fused)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def tune(batch, codec, precision="fp16x2", fused=True, candidates=None, use_cache=True, verbose=False):
    """Return (best Launch, {shape: ms})."""
    key = _key(batch, codec, precision, fused)
    cache = {}
    if use_cache and os.path.exists(CACHE):
        with open(CACHE) as f:
            cache = json.load(f)
        if key in cache:
            w, v, b = cache[key]["shape"]
            return Launch(w, v, b), cache[key].get("times", {})
    times = {}
    best, best_ms, ref = None, float("inf"), None
    for cand in candidates or CANDIDATES:
        try:
            dec = Decoder(batch, codec, cand)
            ms = _time(dec, precision, fused)
        except Exception as exc:  # shape refused by the library (LDS budget)
            if verbose:
                print("autotune: skip", cand, exc)
            continue
        out = dec.out[: batch.n_samples]
        if ref is None:
            ref = out.clone()
        elif not torch.equal(out, ref):
            raise RuntimeError(f"launch shape {cand} changed the decoded samples")
        times[f"{cand.windows_per_chunk}/{cand.waves_per_block}/{cand.blocks}"] = ms
        if verbose:
            print(f"autotune: {cand} {ms:.3f} ms")
        if ms < best_ms:
            best, best_ms = cand, ms
        del dec
    if best is None:
        raise RuntimeError("no launch shape accepted")
    if use_cache:
        cache[key] = {"shape": [best.windows_per_chunk, best.waves_per_block, best.blocks], "times": times}
        tmp = CACHE + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1)
        os.replace(tmp, CACHE)
    return best, times
