"""The no-allocation entry point (plan + fused decode on the library's own
static workspace) against fptc_decompress_batch with a caller workspace:
identical samples and stream flags on two calls in a row, the second on a
smaller batch, and a refusal of batches whose plan does not fit.  Named to
run last: it shares the library's static array with nothing else, but a
failure here must not hide the tests before it."""
import numpy as np
import pytest

from cases import build_case
from gpu_helpers import qparams

pytestmark = pytest.mark.gpu


def _amp(N, **kw):
    from oracle import oracle as O
    return O.QuantParams("amp", N, N, **kw)


def _device(case, N):
    from paper_2605_01086_amd import codec as C
    words, symlen, word_off, sample_off = case.concat()
    codec = C.DeviceCodec(np.stack([b.lengths for b in case.books]), qparams(case.p), 12)
    batch = C.DeviceBatch(words, symlen, word_off, sample_off, N, N, case.book_id)
    return codec, batch


def _both(F, codec, batch, gamma, prec):
    import torch
    from paper_2605_01086_amd import codec as C
    lc = C.Launch().c()
    ws = torch.empty(F.fptc_workspace_size(batch.c, codec.c, lc), dtype=torch.uint8, device="cuda")
    ref = torch.full((batch.n_samples + 64,), -7.0, dtype=torch.float32, device="cuda")
    st_ref = torch.full((batch.n_streams,), -1, dtype=torch.int32, device="cuda")
    F.fptc_plan_batch(batch.c, codec.c, lc, ws, st_ref)
    F.fptc_decompress_batch(batch.c, codec.c, lc, ws, gamma, prec, ref, st_ref)
    out = torch.full((batch.n_samples + 64,), -7.0, dtype=torch.float32, device="cuda")
    st = torch.full((batch.n_streams,), -1, dtype=torch.int32, device="cuda")
    F.fptc_decompress_batch_noalloc(batch.c, codec.c, lc, gamma, prec, out, st)
    torch.cuda.synchronize()
    return ref.cpu().numpy(), st_ref.cpu().numpy(), out.cpu().numpy(), st.cpu().numpy()


@pytest.mark.parametrize("N", [64, 256])
def test_noalloc_matches_workspace_call_twice(N):
    import torch
    from paper_2605_01086_amd import fptc as F
    kw = dict(step_f=1.0, step_c=8.0, T=16.0) if N == 256 else {}
    big = build_case(_amp(N, **kw), ["eeg", "seismic", "power", "meteo"], [N * 400 + 5, 30000, 777, N * 90],
                     config_id=2100 + N, recon=False, gamma=True)
    small = build_case(_amp(N, **kw), ["eeg", "seismic"], [N * 20 + 3, 500], config_id=2200 + N, recon=False)
    for case, use_gamma in ((big, True), (small, False)):
        codec, batch = _device(case, N)
        gamma = torch.from_numpy(case.gamma.astype(np.float32)).cuda() if use_gamma else None
        ref, st_ref, out, st = _both(F, codec, batch, gamma, "fp16x2")
        assert np.array_equal(st, st_ref) and np.all(st == 0)
        assert np.array_equal(out, ref)  # guard band included: nothing written past the output


def test_noalloc_refuses_batches_beyond_its_workspace():
    import torch
    from paper_2605_01086_amd import codec as C
    from paper_2605_01086_amd import fptc as F
    case = build_case(_amp(64), ["eeg"], [4096], config_id=2300, recon=False)
    codec, batch = _device(case, 64)
    # a batch header claiming far more symbols than the static workspace can plan
    b = F.fptc_batch.from_buffer_copy(batch.c)
    b.n_symbols = 1 << 34
    lc = C.Launch().c()
    out = torch.empty(16, dtype=torch.float32, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    assert F.fptc_workspace_size(b, codec.c, lc) > F.FPTC_NOALLOC_WS_BYTES
    with pytest.raises(F.FptcError) as e:
        F.fptc_decompress_batch_noalloc(b, codec.c, lc, None, "fp16x2", out, st)
    assert e.value.code == F.FPTC_ERR_WORKSPACE
