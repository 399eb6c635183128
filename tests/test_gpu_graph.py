"""The single-image entry points under HIP graph capture.

The forward calls and the adjoint allocate nothing and make no synchronous
HIP call, so a caller can capture them. One graph holds a bicubic x2, a
bilinear x0.5, an antialiased and a nearest-neighbour resize, a printed-map
resize, and the adjoint on both of its paths (exact x2 register walk and
owner-computes, float32 and float16). It is replayed three times with eager
work in between (the outputs are overwritten with garbage first), and every
replay must equal the eager results bit for bit.
"""

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1001_1718_amd as xr  # noqa: E402
from synth import fields  # noqa: E402

DEV = "cuda:0"


def test_single_image_calls_replay_from_a_graph():
    x = torch.from_numpy(fields.uniform_u8((100, 140, 4), seed=31)).to(DEV)
    xf = torch.from_numpy(fields.field_unit(90, 70, 1, seed=32, dtype=np.float16)[:, :, 0]).to(DEV)
    g2 = torch.from_numpy(fields.normal_f32((1, 3, 200, 280), seed=33)).to(DEV)
    g3 = torch.from_numpy(fields.normal_f32((1, 3, 150, 210), seed=34)).to(DEV)
    g3h = g3.half()

    outs = {
        "bicubic_x2": torch.empty((200, 280, 4), dtype=torch.uint8, device=DEV),
        "bilinear_x0.5": torch.empty((50, 70, 4), dtype=torch.uint8, device=DEV),
        "bicubic_aa": torch.empty((37, 51, 4), dtype=torch.uint8, device=DEV),
        "nearest": torch.empty((150, 210, 4), dtype=torch.uint8, device=DEV),
        "paper_map": torch.empty((201, 97), dtype=torch.float16, device=DEV),
        "adj_x2": torch.empty((1, 3, 100, 140), device=DEV),
        "adj_owner": torch.empty((1, 3, 100, 140), device=DEV),
        "adj_owner_f16": torch.empty((1, 3, 100, 140), dtype=torch.float16, device=DEV),
    }

    def calls():
        xr.resize_into(x, outs["bicubic_x2"], "bicubic")
        xr.resize_into(x, outs["bilinear_x0.5"], "bilinear")
        xr.resize_into(x, outs["bicubic_aa"], "bicubic_aa")
        xr.resize_into(x, outs["nearest"], "nearest")
        xr.resize_into(xf, outs["paper_map"], "bicubic", mapping="paper")
        xr.resize_backward(g2, (100, 140), "bilinear", out=outs["adj_x2"])
        xr.resize_backward(g3, (100, 140), "bicubic", out=outs["adj_owner"])
        xr.resize_backward(g3h, (100, 140), "bicubic", out=outs["adj_owner_f16"])

    calls()
    torch.cuda.synchronize()
    eager = {k: v.clone() for k, v in outs.items()}

    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(stream):
        with torch.cuda.graph(graph, stream=stream):
            calls()
    torch.cuda.current_stream().wait_stream(stream)
    torch.cuda.synchronize()

    for rep in range(3):
        for v in outs.values():  # eager work between replays
            v.view(torch.uint8).fill_(0xA5 + rep)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for k, v in outs.items():
            assert torch.equal(v.view(torch.uint8), eager[k].view(torch.uint8)), f"replay {rep}: {k} differs"
