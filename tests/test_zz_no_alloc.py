"""rbc_matmul_noalloc: the product with its workspace in the library's fixed device
array equals rbc_matmul's product with a caller's workspace, bit for bit (same
kernels), on consecutive calls of decreasing size, so that the second call runs
over what the first left in the array."""

import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1905_07439_amd as rbc  # noqa: E402
import workloads  # noqa: E402
from paper_1905_07439_amd._lib import lib  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
MAX_WS = 64 << 20  # RBC_NOALLOC_MAX_WORKSPACE
EINVAL = 1


def _inputs(m, k, n, dtype, seed):
    A = torch.from_numpy(workloads.gaussian((m, k), seed).astype(dtype)).to(DEV)
    B = torch.from_numpy(workloads.gaussian((k, n), seed + 1).astype(dtype)).to(DEV)
    return A, B


def _raw_noalloc(plan, A, B, C, seed, mode):
    st = torch.cuda.current_stream(A.device)
    return lib().rbc_matmul_noalloc(plan._h, A.data_ptr(), A.stride(0), B.data_ptr(), B.stride(0), C.data_ptr(),
                                    C.stride(0), seed, rbc.MODES[mode], int(mode != "none"),
                                    ctypes.c_void_p(st.cuda_stream))


CASES = [
    # (first call, second call): (M, K, N, levels, prec, seed, mode); the second is smaller
    (((1000, 1000, 1000), ("strassen", "strassen"), "f32", 3, "full"),
     ((600, 600, 600), ("strassen",), "f32", 4, "full")),
    (((960, 960, 960), ("laderman", "strassen"), "f16s", 5, "full"),
     ((480, 384, 288), ("strassen", "strassen"), "f16s", 6, "signs")),
    (((768, 768, 768), ("strassen", "strassen"), "fp8c", 7, "full"),
     ((256, 256, 256), ("strassen",), "fp8c", 8, "perms")),
    (((300, 300, 300), ("strassen", "strassen"), "f64", 9, "full"),
     ((64, 64, 64), ("strassen", "strassen"), "f64", 0, "none")),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_noalloc_equals_matmul_two_calls(case):
    torch.cuda.set_device(0)
    outs = []
    for (m, k, n), names, prec, seed, mode in CASES[case]:
        print("noalloc case", case, (m, k, n), names, prec, seed, mode, flush=True)
        plan = rbc.Plan(m, k, n, [rbc.Scheme.builtin(x) for x in names], prec=prec)
        assert plan.workspace_bytes <= MAX_WS
        dtype = np.float64 if prec == "f64" else np.float32
        A, B = _inputs(m, k, n, dtype, 7000 + 10 * case + seed)
        ref = plan.matmul(A, B, seed=seed, mode=mode)  # also uploads the plan's tables
        C = torch.full((m, n), float("nan"), dtype=ref.dtype, device=DEV)
        rbc.check(_raw_noalloc(plan, A, B, C, seed, mode))
        torch.cuda.synchronize()
        outs.append((ref, C))
    for ref, C in outs:
        assert torch.equal(ref, C)


def test_noalloc_rejects_what_it_cannot_run():
    torch.cuda.set_device(0)
    S = rbc.Scheme.builtin("strassen")
    A, B = _inputs(256, 256, 256, np.float32, 7100)
    C = torch.empty((256, 256), device=DEV)
    fresh = rbc.Plan(256, 256, 256, [S], prec="f32")  # tables not uploaded yet
    assert _raw_noalloc(fresh, A, B, C, 0, "full") == EINVAL
    assert "not on the device" in lib().rbc_last_error().decode()
    big = rbc.Plan(2048, 2048, 2048, [S] * 3, prec="f32")
    assert big.workspace_bytes > MAX_WS
    Ab, Bb = _inputs(2048, 2048, 2048, np.float32, 7200)
    Cb = torch.empty((2048, 2048), device=DEV)
    big.matmul(Ab, Bb, C=Cb)
    assert _raw_noalloc(big, Ab, Bb, Cb, 0, "full") == EINVAL
    assert "fixed device array" in lib().rbc_last_error().decode()
    fresh.matmul(A, B, C=C)
    fresh.set_timing(True)
    assert _raw_noalloc(fresh, A, B, C, 0, "full") == EINVAL
    fresh.set_timing(False)
    ref = fresh.matmul(A, B, seed=11)
    out = fresh.matmul_noalloc(A, B, torch.empty_like(ref), seed=11)
    torch.cuda.synchronize()
    assert torch.equal(ref, out)
