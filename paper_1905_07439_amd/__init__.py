"""Randomized (approximate) bilinear matrix multiplication on AMD MI355X.

C = F-hat^(Q)(A, B): recursive bilinear computation with seeded random signed
block permutations folded into the scheme coefficients (Malik & Becker,
Definition 2 and eq. recursive-random-formula).  Every step runs in the HIP
library librbc.so (include/rbc.h); this module only marshals arguments and
uses torch for device memory and streams.  There is no CPU fallback: if the
library is not built, import of the compute entry points raises.

    import paper_1905_07439_amd as rbc
    S = rbc.Scheme.builtin("strassen")
    plan = rbc.Plan(4096, 4096, 4096, [S, S, S], prec="f32")
    C = plan.matmul(A, B, seed=0)           # A, B: torch tensors on the GPU
"""

import ctypes

import numpy as np

from ._lib import MODES, PRECS, BatchInfo, BatchItem, BatchOptions, PlanInfo, RbcError, check, lib  # noqa: F401

__all__ = ["Scheme", "Plan", "draw", "fold", "RbcError", "lib"]


def _dbl(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _i32(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


class Scheme:
    """An immutable, validated bilinear-computation scheme (U, V, W)."""

    def __init__(self, handle):
        self._h = ctypes.c_void_p(handle)

    # families whose builtin takes lambda (and, for the perturbed ones, aux_seed)
    LAMBDA_FAMILIES = ("apa322", "apa223", "apa232", "perturbed_strassen", "perturbed_laderman")

    @classmethod
    def builtin(cls, name, lam=None, aux_seed=0):
        """A builtin scheme (include/rbc.h, rbc_scheme_builtin).  For the lambda families
        the name may carry lambda after a colon ("apa322:0.001"), or lam gives it."""
        if lam is None and ":" in name and name.split(":", 1)[0] in cls.LAMBDA_FAMILIES:
            name, lam = name.split(":", 1)
        lam = 0.0 if lam is None else float(lam)
        h = ctypes.c_void_p()
        check(lib().rbc_scheme_builtin(name.encode(), lam, int(aux_seed) & 0xFFFFFFFFFFFFFFFF, ctypes.byref(h)))
        return cls(h.value)

    @classmethod
    def from_tensors(cls, U, V, W, residual_tol=0.0):
        U = np.asarray(U, np.float64)
        V = np.asarray(V, np.float64)
        W = np.asarray(W, np.float64)
        b1, b2, R = U.shape
        b3 = V.shape[1]
        if V.shape != (b2, b3, R) or W.shape != (b1, b3, R):
            raise ValueError("tensor shapes must be (b1,b2,R), (b2,b3,R), (b1,b3,R)")
        (u, up), (v, vp), (w, wp) = _dbl(U), _dbl(V), _dbl(W)
        h = ctypes.c_void_p()
        check(lib().rbc_scheme_create(b1, b2, b3, R, up, vp, wp, float(residual_tol), ctypes.byref(h)))
        return cls(h.value)

    def info(self):
        dims = (ctypes.c_int * 4)()
        vals = [ctypes.c_double() for _ in range(4)]
        check(lib().rbc_scheme_info(self._h, dims, *[ctypes.byref(v) for v in vals]))
        b1, b2, b3, R = list(dims)
        tau, kappa, ynorm, q = [v.value for v in vals]
        return {"b1": b1, "b2": b2, "b3": b3, "R": R, "tau": tau, "kappa": kappa, "ynorm": ynorm, "q": q}

    def tensors(self):
        i = self.info()
        U = np.zeros((i["b1"], i["b2"], i["R"]))
        V = np.zeros((i["b2"], i["b3"], i["R"]))
        W = np.zeros((i["b1"], i["b3"], i["R"]))
        check(lib().rbc_scheme_tensors(self._h, _dbl(U)[1], _dbl(V)[1], _dbl(W)[1]))
        return U, V, W

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._h = None  # at interpreter exit module globals may already be gone
            try:
                lib().rbc_scheme_destroy(h)
            except Exception:
                pass


def draw(seed, depth, b1, b2, b3, mode="full"):
    """(signs, perms) of one level: int32 arrays of b1 + b2 + b3 entries (include/rbc.h)."""
    n = b1 + b2 + b3
    s = np.zeros(n, np.int32)
    p = np.zeros(n, np.int32)
    check(lib().rbc_draw(seed & 0xFFFFFFFFFFFFFFFF, depth, b1, b2, b3, MODES[mode], _i32(s)[1], _i32(p)[1]))
    return s, p


def fold(scheme, signs, perms, kappa_scale=True):
    i = scheme.info()
    Uh = np.zeros((i["b1"], i["b2"], i["R"]))
    Vh = np.zeros((i["b2"], i["b3"], i["R"]))
    Wh = np.zeros((i["b1"], i["b3"], i["R"]))
    s, sp = _i32(signs)
    p, pp = _i32(perms)
    check(lib().rbc_fold(scheme._h, sp, pp, int(bool(kappa_scale)), _dbl(Uh)[1], _dbl(Vh)[1], _dbl(Wh)[1]))
    return Uh, Vh, Wh


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


PEAK_KINDS = {"f32": 0, "f64": 1, "f16": 2, "bf16": 3, "fp8": 4, "f32_32x32": 5, "f16_32x32": 6, "bf16_32x32": 7}


def peak_copy(src, dst, stream=None):
    """dst.copy_(src) by the library's streaming copy kernel (device tensors of equal byte size)."""
    import torch
    st = stream if stream is not None else torch.cuda.current_stream(src.device)
    check(lib().rbc_peak_copy(_ptr(src), _ptr(dst), src.numel() * src.element_size(),
                              ctypes.c_void_p(st.cuda_stream)))


def peak_mfma(kind, sink, iters, stream=None):
    """Launch the register-only matrix-core loop of one data type ("f32", "f64", "f16", "bf16",
    "fp8") with sink.numel() // 256 workgroups; returns the floating-point operations launched."""
    import torch
    st = stream if stream is not None else torch.cuda.current_stream(sink.device)
    fl = ctypes.c_double()
    check(lib().rbc_peak_mfma(PEAK_KINDS[kind], sink.numel() // 256, iters, _ptr(sink), ctypes.byref(fl),
                              ctypes.c_void_p(st.cuda_stream)))
    return fl.value


class Plan:
    """A plan for C = F-hat^(Q)(A, B) with A of size M x K and B of size K x N."""

    def __init__(self, M, K, N, schemes, prec="f32", leaf_tile=0, fusion="auto"):
        """fusion: "auto" (two levels share a combination pass only with enough parallel work) or
        "max" (fuse wherever the shapes allow; for products run in a batch)."""
        if fusion not in ("auto", "max"):
            raise ValueError("fusion must be 'auto' or 'max'")
        self.schemes = list(schemes)
        arr = (ctypes.c_void_p * max(1, len(self.schemes)))(*[s._h.value for s in self.schemes])
        h = ctypes.c_void_p()
        check(lib().rbc_plan_create(M, K, N, len(self.schemes), arr, PRECS[prec], leaf_tile, ctypes.byref(h)))
        self._h = h
        self.prec = prec
        if fusion == "max":
            check(lib().rbc_plan_set_fusion(self._h, 1))
        self.fusion = fusion
        inf = PlanInfo()
        check(lib().rbc_plan_get_info(self._h, ctypes.byref(inf)))
        self.info = inf.as_dict()
        self._ws = None

    @property
    def workspace_bytes(self):
        return self.info["workspace_bytes"]

    def traffic(self):
        """Algorithmic HBM bytes per stage: {gather_A, gather_B, leaf, scatter}."""
        b = (ctypes.c_double * 4)()
        check(lib().rbc_plan_traffic(self._h, b))
        return dict(zip(("gather_A", "gather_B", "leaf", "scatter"), list(b)))

    @property
    def dtype(self):
        import torch
        return torch.float64 if self.prec == "f64" else torch.float32

    def workspace(self, device=None):
        import torch
        if self._ws is None or (device is not None and self._ws.device != torch.device(device)):
            self._ws = torch.empty(self.workspace_bytes, dtype=torch.uint8, device=device or "cuda")
        return self._ws

    def _common(self, A, B, C, workspace, stream):
        import torch
        M, K, N = self.info["M"], self.info["K"], self.info["N"]
        for name, X, shape in (("A", A, (M, K)), ("B", B, (K, N))):
            if tuple(X.shape) != shape or X.dtype != self.dtype or not X.is_cuda:
                raise ValueError("%s must be a %s CUDA tensor of shape %s" % (name, self.dtype, shape))
            if X.stride(1) != 1:
                raise ValueError("%s must be row-major (unit column stride)" % name)
        if C is None:
            C = torch.empty((M, N), dtype=self.dtype, device=A.device)
        if tuple(C.shape) != (M, N) or C.dtype != self.dtype or C.stride(1) != 1:
            raise ValueError("C must be a row-major %s tensor of shape %s" % (self.dtype, (M, N)))
        ws = workspace if workspace is not None else self.workspace(A.device)
        st = stream if stream is not None else torch.cuda.current_stream(A.device)
        return C, ws, ctypes.c_void_p(st.cuda_stream)

    def matmul(self, A, B, C=None, seed=0, mode="full", kappa_scale=None, workspace=None, stream=None):
        """C = F-hat^(Q)(A, B) with the draws of (seed, mode), asynchronously on ``stream``."""
        if kappa_scale is None:
            kappa_scale = mode != "none"
        C, ws, st = self._common(A, B, C, workspace, stream)
        check(lib().rbc_matmul(self._h, _ptr(A), A.stride(0), _ptr(B), B.stride(0), _ptr(C), C.stride(0),
                               seed & 0xFFFFFFFFFFFFFFFF, MODES[mode], int(bool(kappa_scale)), _ptr(ws),
                               ws.numel(), st))
        return C

    def matmul_noalloc(self, A, B, C, seed=0, mode="full", kappa_scale=None, stream=None):
        """As matmul, into a given C, with the workspace in the library's fixed device array
        (rbc_matmul_noalloc): the call allocates nothing.  The plan must have run once
        through matmul on this device."""
        import torch
        if kappa_scale is None:
            kappa_scale = mode != "none"
        M, K, N = self.info["M"], self.info["K"], self.info["N"]
        for name, X, shape in (("A", A, (M, K)), ("B", B, (K, N)), ("C", C, (M, N))):
            if tuple(X.shape) != shape or X.dtype != self.dtype or not X.is_cuda or X.stride(1) != 1:
                raise ValueError("%s must be a row-major %s CUDA tensor of shape %s" % (name, self.dtype, shape))
        st = stream if stream is not None else torch.cuda.current_stream(A.device)
        check(lib().rbc_matmul_noalloc(self._h, _ptr(A), A.stride(0), _ptr(B), B.stride(0), _ptr(C), C.stride(0),
                                       seed & 0xFFFFFFFFFFFFFFFF, MODES[mode], int(bool(kappa_scale)),
                                       ctypes.c_void_p(st.cuda_stream)))
        return C

    def matmul_draws(self, A, B, signs, perms, C=None, kappa_scale=True, workspace=None, stream=None):
        C, ws, st = self._common(A, B, C, workspace, stream)
        s, sp = _i32(signs)
        p, pp = _i32(perms)
        check(lib().rbc_matmul_draws(self._h, _ptr(A), A.stride(0), _ptr(B), B.stride(0), _ptr(C),
                                     C.stride(0), sp, pp, int(bool(kappa_scale)), _ptr(ws), ws.numel(), st))
        return C

    def matmul_average(self, A, B, seeds, mode="full", kappa_scale=None, stream=None):
        """(1/K) sum_k F-hat_k(A, B) over the draws of seeds[k], accumulated in f64 (a new
        float64 tensor)."""
        import torch
        if kappa_scale is None:
            kappa_scale = mode != "none"
        M, N = self.info["M"], self.info["N"]
        for name, X, shape in (("A", A, (M, self.info["K"])), ("B", B, (self.info["K"], N))):
            if tuple(X.shape) != shape or X.dtype != self.dtype or not X.is_cuda or X.stride(1) != 1:
                raise ValueError("%s must be a row-major %s CUDA tensor of shape %s" % (name, self.dtype, shape))
        n = ctypes.c_size_t()
        check(lib().rbc_average_workspace(self._h, ctypes.byref(n)))
        ws = torch.empty(n.value, dtype=torch.uint8, device=A.device)
        out = torch.empty((M, N), dtype=torch.float64, device=A.device)
        sd = (ctypes.c_uint64 * len(seeds))(*[int(x) & 0xFFFFFFFFFFFFFFFF for x in seeds])
        st = stream if stream is not None else torch.cuda.current_stream(A.device)
        check(lib().rbc_matmul_average(self._h, _ptr(A), A.stride(0), _ptr(B), B.stride(0), _ptr(out), sd,
                                       len(seeds), MODES[mode], int(bool(kappa_scale)), _ptr(ws), ws.numel(),
                                       ctypes.c_void_p(st.cuda_stream)))
        return out

    def average_over_draws(self, A, B, draws, kappa_scale=True, stream=None):
        """(1/K) sum over explicit draws [(signs, perms), ...] (as rbc_matmul_draws takes them),
        accumulated in f64 on the device."""
        import torch
        st = stream if stream is not None else torch.cuda.current_stream(A.device)
        M, N = self.info["M"], self.info["N"]
        out = torch.empty((M, N), dtype=torch.float64, device=A.device)
        C = torch.empty((M, N), dtype=self.dtype, device=A.device)
        ws = self.workspace(A.device)
        for k, (signs, perms) in enumerate(draws):
            self.matmul_draws(A, B, signs, perms, C=C, kappa_scale=kappa_scale, workspace=ws, stream=st)
            check(lib().rbc_accumulate(_ptr(out), _ptr(C), int(self.prec == "f64"), M, N, C.stride(0),
                                       int(k == 0), ctypes.c_void_p(st.cuda_stream)))
        check(lib().rbc_scale_f64(_ptr(out), M * N, 1.0 / len(draws), ctypes.c_void_p(st.cuda_stream)))
        return out

    def draws(self, seed, mode="full"):
        """Concatenated per-level draws of (seed, mode), as rbc_matmul computes them."""
        ss, ps = [], []
        for d, sch in enumerate(self.schemes):
            i = sch.info()
            s, p = draw(seed, d, i["b1"], i["b2"], i["b3"], mode)
            ss.append(s)
            ps.append(p)
        if not ss:
            return np.zeros(0, np.int32), np.zeros(0, np.int32)
        return np.concatenate(ss), np.concatenate(ps)

    # ---- stages -------------------------------------------------------------
    def stage_gather(self, which, X, signs, perms, workspace, stream=None):
        import torch
        st = stream if stream is not None else torch.cuda.current_stream(X.device)
        s, sp = _i32(signs)
        p, pp = _i32(perms)
        check(lib().rbc_stage_gather(self._h, which, _ptr(X), X.stride(0), sp, pp, _ptr(workspace),
                                     workspace.numel(), ctypes.c_void_p(st.cuda_stream)))

    def stage_leaf(self, workspace, stream=None):
        import torch
        st = stream if stream is not None else torch.cuda.current_stream(workspace.device)
        check(lib().rbc_stage_leaf(self._h, _ptr(workspace), workspace.numel(), ctypes.c_void_p(st.cuda_stream)))

    def stage_scatter(self, signs, perms, C, workspace, kappa_scale=True, stream=None):
        import torch
        st = stream if stream is not None else torch.cuda.current_stream(C.device)
        s, sp = _i32(signs)
        p, pp = _i32(perms)
        check(lib().rbc_stage_scatter(self._h, sp, pp, int(bool(kappa_scale)), _ptr(C), C.stride(0),
                                      _ptr(workspace), workspace.numel(), ctypes.c_void_p(st.cuda_stream)))

    # ---- leaf gather --------------------------------------------------------
    @property
    def leaf_gather(self):
        """(on, available): whether matmul forms the leaf operands inside the leaf product."""
        on, av = ctypes.c_int(), ctypes.c_int()
        check(lib().rbc_plan_get_leaf_gather(self._h, ctypes.byref(on), ctypes.byref(av)))
        return bool(on.value), bool(av.value)

    def set_leaf_gather(self, on=True):
        check(lib().rbc_plan_set_leaf_gather(self._h, int(bool(on))))

    @property
    def leaf_scatter(self):
        """(on, available): whether matmul folds the deepest level's scatter into the leaf product."""
        on, av = ctypes.c_int(), ctypes.c_int()
        check(lib().rbc_plan_get_leaf_scatter(self._h, ctypes.byref(on), ctypes.byref(av)))
        return bool(on.value), bool(av.value)

    def set_leaf_scatter(self, on=True):
        """Turning it on the first time enlarges the workspace (a cached one is dropped)."""
        check(lib().rbc_plan_set_leaf_scatter(self._h, int(bool(on))))
        inf = PlanInfo()
        check(lib().rbc_plan_get_info(self._h, ctypes.byref(inf)))
        if inf.as_dict()["workspace_bytes"] != self.info["workspace_bytes"]:
            self.info = inf.as_dict()
            self._ws = None

    # ---- timing -------------------------------------------------------------
    def set_timing(self, on=True):
        check(lib().rbc_plan_set_timing(self._h, int(bool(on))))

    def timing_collect(self):
        """(ms per stage [gather A, gather B, leaf, scatter] summed, number of calls)."""
        ms = (ctypes.c_double * 4)()
        calls = ctypes.c_int64()
        check(lib().rbc_plan_timing_collect(self._h, ms, ctypes.byref(calls)))
        return list(ms), calls.value

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._h = None  # at interpreter exit module globals may already be gone
            try:
                lib().rbc_plan_destroy(h)
            except Exception:
                pass


# Layout of rbc_batch_task (include/rbc.h).
TASK_DTYPE = np.dtype([("kind", np.int16), ("variant", np.int16), ("param", np.int32),
                       ("wait", np.int32, 2), ("need", np.int32, 2), ("signal", np.int32),
                       ("count", np.int32), ("first", np.int64), ("sub", np.int64)])
TASK_KINDS = {0: "maxabs", 1: "exponents", 2: "gather", 3: "leaf", 4: "scatter", 5: "gate"}


class Batch:
    """Independent products run together (include/rbc.h, batches): one persistent kernel
    (``mode="persistent"``, queue ``order`` "products" or "depth") or one grid per dependency
    level (``mode="levels"``).

    Every product keeps the result ``Plan.matmul`` gives for the same plan,
    operands, seed and mode, bit for bit.  The batch holds references to the
    plans and tensors added to it; they must not be freed or resized while the
    batch is in use.
    """

    def __init__(self, window=0, grid=0, timeout_ms=0, task_bytes=0, item_budget=0, trace=False,
                 mode="persistent", order="products"):
        modes = {"persistent": 0, "levels": 1}
        orders = {"products": 0, "depth": 1}
        opt = BatchOptions(window=window, grid=grid, timeout_ms=timeout_ms, task_bytes=task_bytes,
                           item_budget=item_budget, trace=int(bool(trace)), mode=modes[mode],
                           order=orders[order])
        h = ctypes.c_void_p()
        check(lib().rbc_batch_create(ctypes.byref(opt), ctypes.byref(h)))
        self._h = h
        self._keep = []
        self.items = []
        self._ws = None

    def add(self, plan, A, B, C=None, seed=0, mode="full", kappa_scale=None):
        """Append C = F-hat(A, B) with plan's schemes; returns (index, C)."""
        import torch
        if kappa_scale is None:
            kappa_scale = mode != "none"
        M, K, N = plan.info["M"], plan.info["K"], plan.info["N"]
        for name, X, shape in (("A", A, (M, K)), ("B", B, (K, N))):
            if tuple(X.shape) != shape or X.dtype != plan.dtype or not X.is_cuda or X.stride(1) != 1:
                raise ValueError("%s must be a row-major %s CUDA tensor of shape %s" % (name, plan.dtype, shape))
        if C is None:
            C = torch.empty((M, N), dtype=plan.dtype, device=A.device)
        if tuple(C.shape) != (M, N) or C.dtype != plan.dtype or C.stride(1) != 1:
            raise ValueError("C must be a row-major %s tensor of shape %s" % (plan.dtype, (M, N)))
        idx = ctypes.c_int64()
        check(lib().rbc_batch_add(self._h, plan._h, _ptr(A), A.stride(0), _ptr(B), B.stride(0), _ptr(C),
                                  C.stride(0), seed & 0xFFFFFFFFFFFFFFFF, MODES[mode], int(bool(kappa_scale)),
                                  ctypes.byref(idx)))
        self._keep.append((plan, A, B, C))
        self.items.append(C)
        self._ws = None
        return idx.value, C

    @property
    def workspace_bytes(self):
        n = ctypes.c_size_t()
        check(lib().rbc_batch_workspace(self._h, ctypes.byref(n)))
        return n.value

    def prepare(self, workspace=None, stream=None, device=None):
        """Build and upload the task table; allocates the workspace unless one is given."""
        import torch
        if workspace is None:
            workspace = torch.empty(self.workspace_bytes, dtype=torch.uint8, device=device or "cuda")
        st = stream if stream is not None else torch.cuda.current_stream(workspace.device)
        check(lib().rbc_batch_prepare(self._h, _ptr(workspace), workspace.numel(), ctypes.c_void_p(st.cuda_stream)))
        self._ws = workspace
        return workspace

    def launch(self, graph=False, stream=None):
        """One run of every product, asynchronously on ``stream`` (a captured graph if ``graph``)."""
        import torch
        if self._ws is None:
            self.prepare(stream=stream)
        st = stream if stream is not None else torch.cuda.current_stream(self._ws.device)
        check(lib().rbc_batch_launch(self._h, ctypes.c_void_p(st.cuda_stream), int(bool(graph))))

    def check(self, stream=None):
        """Wait for ``stream``; raises if a dependency wait inside the kernel timed out."""
        import torch
        st = stream if stream is not None else torch.cuda.current_stream(self._ws.device)
        check(lib().rbc_batch_check(self._h, ctypes.c_void_p(st.cuda_stream)))

    def task_table(self):
        """The task table of the last prepare or workspace query, as a numpy structured array."""
        n = ctypes.c_int64()
        check(lib().rbc_batch_task_table(self._h, None, 0, ctypes.byref(n)))
        out = np.zeros(n.value, dtype=TASK_DTYPE)
        check(lib().rbc_batch_task_table(self._h, out.ctypes.data_as(ctypes.c_void_p), n.value,
                                         ctypes.byref(n)))
        return out

    def set_grid(self, grid):
        """Workgroups of the persistent kernel (0: the resident maximum)."""
        check(lib().rbc_batch_set_grid(self._h, int(grid)))

    def trace(self):
        """Per-task (taken, ready, done) times in microseconds from the first task taken, and
        the workgroup, of the last completed run (needs ``trace=True``)."""
        n = ctypes.c_int64()
        rate = ctypes.c_double()
        check(lib().rbc_batch_trace(self._h, None, 0, ctypes.byref(n), ctypes.byref(rate)))
        raw = np.zeros((n.value, 4), dtype=np.uint64)
        check(lib().rbc_batch_trace(self._h, raw.ctypes.data_as(ctypes.c_void_p), n.value, ctypes.byref(n),
                                    None))
        t = raw[:, :3].astype(np.float64)
        t0 = t[:, 0].min() if len(t) else 0.0
        return (t - t0) / rate.value, raw[:, 3].astype(np.int64)

    def item(self, index):
        """Workspace region, first queue index and counters of product ``index``."""
        it = BatchItem()
        check(lib().rbc_batch_get_item(self._h, index, ctypes.byref(it)))
        return it.as_dict()

    def info(self):
        inf = BatchInfo()
        check(lib().rbc_batch_get_info(self._h, ctypes.byref(inf)))
        return inf.as_dict()

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._h = None  # at interpreter exit module globals may already be gone
            try:
                lib().rbc_batch_destroy(h)
            except Exception:
                pass


def apa_ebc_weights(eps):
    """Weights alpha_i with sum_i alpha_i Y(eps_i) = X for an approximate scheme whose
    error has degree < len(eps) in eps (Section 1, eq. APA-to-EBC); a list of floats."""
    n = len(eps)
    e = (ctypes.c_double * n)(*[float(x) for x in eps])
    a = (ctypes.c_double * n)()
    check(lib().rbc_apa_ebc_weights(e, n, a))
    return list(a)


def apa_scheme_levels(names, eps):
    """Scheme names for one eps: each "apa322"/"apa223"/"apa232" entry gets ":<eps>",
    any other name (an exact scheme) is kept."""
    return [("%s:%r" % (n, float(eps))) if n in ("apa322", "apa223", "apa232") else n for n in names]


def apa_ebc_plans(M, K, N, names, eps, prec="f64", leaf_tile=0, fusion="auto"):
    """One Plan per eps for the levels ``names`` (see apa_scheme_levels)."""
    return [Plan(M, K, N, [Scheme.builtin(n) for n in apa_scheme_levels(names, e)], prec=prec,
                 leaf_tile=leaf_tile, fusion=fusion) for e in eps]


def matmul_apa_ebc(A, B, names, eps, prec="f64", seed=0, mode="none", kappa_scale=None, stream=None,
                   leaf_tile=0, fusion="auto", plans=None, workspace=None, out=None):
    """The exact product from an approximate scheme: sum_i alpha_i F-hat(A, B) with the
    levels ``names`` at eps[i] (apa entries take eps[i], see apa_scheme_levels), every
    product with the draws of (seed, mode), combined on the device in f64 in the order
    of eps (a new float64 M x N tensor).  The products are not scaled by (1 - kappa)^-1
    (the combination is exact only for the unscaled ones); kappa_scale=True is accepted
    only when every level has kappa = 0, where it changes nothing."""
    import torch
    if kappa_scale is None:
        kappa_scale = False
    M, K = A.shape
    N = B.shape[1]
    if plans is None:
        plans = apa_ebc_plans(M, K, N, names, eps, prec, leaf_tile, fusion)
    if len(plans) != len(eps):
        raise ValueError("one plan per eps value")
    for name, X, shape in (("A", A, (M, K)), ("B", B, (K, N))):
        if tuple(X.shape) != shape or X.dtype != plans[0].dtype or not X.is_cuda or X.stride(1) != 1:
            raise ValueError("%s must be a row-major %s CUDA tensor of shape %s" % (name, plans[0].dtype, shape))
    need = 0
    for p in plans:
        n = ctypes.c_size_t()
        check(lib().rbc_average_workspace(p._h, ctypes.byref(n)))
        need = max(need, n.value)
    ws = workspace if workspace is not None else torch.empty(need, dtype=torch.uint8, device=A.device)
    if ws.numel() < need:
        raise ValueError("workspace of %d bytes < %d needed" % (ws.numel(), need))
    if out is None:
        out = torch.empty((M, N), dtype=torch.float64, device=A.device)
    elif tuple(out.shape) != (M, N) or out.dtype != torch.float64 or not out.is_contiguous():
        raise ValueError("out must be a contiguous float64 tensor of shape (%d, %d)" % (M, N))
    hs = (ctypes.c_void_p * len(plans))(*[getattr(p._h, "value", p._h) for p in plans])
    e = (ctypes.c_double * len(eps))(*[float(x) for x in eps])
    st = stream if stream is not None else torch.cuda.current_stream(A.device)
    check(lib().rbc_matmul_apa_ebc(hs, e, len(eps), _ptr(A), A.stride(0), _ptr(B), B.stride(0), _ptr(out),
                                   int(seed) & 0xFFFFFFFFFFFFFFFF, MODES[mode], int(bool(kappa_scale)), _ptr(ws),
                                   ws.numel(), ctypes.c_void_p(st.cuda_stream)))
    return out
