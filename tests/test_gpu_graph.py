"""HIP-graph capture of a decode step: every replay equals the eager result,
with eager work and synchronisations between replays; and the autotuner's
candidates agree bit for bit."""
import numpy as np
import pytest

from cases import build_case

pytestmark = pytest.mark.gpu


def _setup(config_id=2400):
    from oracle import oracle as O
    from gpu_helpers import qparams
    from paper_2605_01086_amd import codec as C
    p = O.QuantParams("amp", 64, 64)
    rng = np.random.default_rng(3)
    lens = list(np.floor(2.0 ** rng.uniform(8, 15, size=24)).astype(int))
    c = build_case(p, ["eeg", "seismic", "power", "meteo"], lens, config_id=config_id)
    words, symlen, word_off, sample_off = c.concat()
    codec = C.DeviceCodec(np.stack([b.lengths for b in c.books]), qparams(p), 12)
    batch = C.DeviceBatch(words, symlen, word_off, sample_off, 64, 64, c.book_id)
    return c, codec, batch


@pytest.mark.parametrize("fused,precision", [(True, "fp16x2"), (False, "fp32"), (False, "bf16x3")])
def test_graph_replays_match_eager(fused, precision):
    import torch
    from gpu_helpers import check_parity
    from paper_2605_01086_amd import codec as C
    from paper_2605_01086_amd.graph import CapturedStep
    c, codec, batch = _setup()
    eager = C.Decoder(batch, codec)
    ref = eager.run(precision=precision, fused=fused).clone()
    torch.cuda.synchronize()
    dec = C.Decoder(batch, codec)
    step = CapturedStep(dec, precision=precision, fused=fused)
    for r in range(4):
        dec.out.fill_(-1.0)           # eager work between replays
        torch.cuda.synchronize()
        out = step.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, ref), f"replay {r} differs"
        assert int((dec.status != 0).sum()) == 0
    res = dict(sym=np.zeros(0), out=ref.cpu().numpy(), status=dec.status.cpu().numpy(), batch=batch)
    if precision in ("fp32", "fp16x2", "bf16x3"):
        check_parity(c, res, tol=1e-5, check_symbols=False)


def test_autotune_candidates_agree():
    from paper_2605_01086_amd import autotune
    c, codec, batch = _setup(2500)
    best, info = autotune.tune(batch, codec, "fp16x2", fused=True, use_cache=False)
    measured = [v for v in info["times"].values() if v is not None]
    assert len(measured) >= 6 and best is not None and not info["cached"]
    # a coordinate moves only on a gain above 0.5 %, so no candidate beats the pick by more
    assert info["best_ms"] * 0.995 <= min(measured) <= info["best_ms"]
