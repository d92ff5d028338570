"""HIP-graph capture of a whole decode step (plan + fused decode/dequant/IDCT,
or plan + decode + dequant/IDCT), replayed as one graph launch.

The library's calls only enqueue kernels on the current stream (no host
synchronisation, no allocation, no memset nodes) once the library is set up
on the device, which fptc_init does before capture.
"""
from __future__ import annotations

import torch

from . import fptc as F
from .codec import Decoder


class CapturedStep:
    def __init__(self, decoder: Decoder, precision: str = "fp16x2", fused: bool = True, gamma=None):
        self.decoder = decoder
        self.args = dict(gamma=gamma, precision=precision, fused=fused)
        F.fptc_init()
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            with torch.cuda.graph(self.graph, stream=s):
                decoder.run(**self.args)
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()

    def replay(self):
        self.graph.replay()
        return self.decoder.out[: self.decoder.batch.n_samples]
