"""The measured-ceiling kernels (streaming copy, register-only MFMA loops): the copy copies,
and each matrix-core loop runs, reports its operation count and stays under the published
peak of its data type."""

import pytest
import torch

import paper_1905_07439_amd as rbc

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
PUBLISHED_TFLOPS = {"f32": 157.3, "f64": 78.6, "f16": 2500.0, "bf16": 2500.0, "fp8": 5000.0, "f32_32x32": 157.3,
                    "f16_32x32": 2500.0, "bf16_32x32": 2500.0}


def test_peak_copy_copies():
    src = torch.arange(1 << 20, dtype=torch.float32, device=DEV)
    dst = torch.zeros_like(src)
    rbc.peak_copy(src, dst)
    torch.cuda.synchronize()
    assert torch.equal(src, dst)


@pytest.mark.parametrize("kind", sorted(PUBLISHED_TFLOPS))
def test_peak_mfma_runs_within_published_peak(kind):
    sink = torch.zeros(2048 * 256, dtype=torch.float32, device=DEV)
    rbc.peak_mfma(kind, sink, 10)  # warm-up
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    flops = rbc.peak_mfma(kind, sink, 400)
    e1.record()
    e1.synchronize()
    per = {"f32": 2 * 16 * 16 * 4, "f64": 2 * 16 * 16 * 4, "f16": 2 * 16 * 16 * 32, "bf16": 2 * 16 * 16 * 32,
           "fp8": 2 * 32 * 32 * 64, "f32_32x32": 2 * 32 * 32 * 2, "f16_32x32": 2 * 32 * 32 * 16,
           "bf16_32x32": 2 * 32 * 32 * 16}[kind]
    chains = 8 if kind in ("f32", "f64", "f16", "bf16") else 4
    assert flops == 2048 * 4 * 400 * chains * per
    tf = flops / (e0.elapsed_time(e1) * 1e-3) / 1e12
    assert 0 < tf < 1.1 * PUBLISHED_TFLOPS[kind], tf
    assert torch.isfinite(sink).all()
