"""Dense matrix multiplication over GF(2) on AMD MI355X (gfx950).

Thin ctypes binding over ``libgf2.so`` (see ``include/gf2.h``): argument
marshalling only.  Every step of a product runs in the library's HIP kernels;
there is no CPU fallback, and a missing library raises at first use.

Matrices are PyTorch CUDA (HIP) tensors used as raw storage: 2-D, dtype
``torch.int64`` (bit patterns of uint64 words), unit stride along rows;
``ld`` is ``tensor.stride(0)``.  Column j of a row is bit j&63 of word j>>6.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgf2.so")
_LIB = None

KERNEL_AUTO, KERNEL_M4RM, KERNEL_MFMA, KERNEL_CUBIC = 0, 1, 2, 3
ODD_PAD, ODD_PEEL = 0, 1
MEM_FAST, MEM_LOW = 0, 1

STATUS = {0: "GF2_OK", 1: "GF2_ERR_INVALID_ARG", 2: "GF2_ERR_ALIAS", 3: "GF2_ERR_ALLOC", 4: "GF2_ERR_CAPTURE",
          5: "GF2_ERR_DEVICE", 6: "GF2_ERR_UNSUPPORTED"}


class GF2Error(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


class Schedule(ctypes.Structure):
    _fields_ = [("kernel", ctypes.c_int32), ("variant", ctypes.c_int32), ("cutoff", ctypes.c_int32),
                ("splitk", ctypes.c_int32), ("odd", ctypes.c_int32), ("kappa", ctypes.c_int32),
                ("memory", ctypes.c_int32)]

    def __repr__(self):
        return (f"Schedule(kernel={self.kernel}, variant={self.variant}, cutoff={self.cutoff}, "
                f"splitk={self.splitk}, odd={self.odd}, kappa={self.kappa}, memory={self.memory})")


def lib():
    """Load libgf2.so (raises if it has not been built)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_0811_1714_amd.build` "
                           "(the GPU path has no fallback)")
    L = ctypes.CDLL(LIB_PATH)
    P, I64, I32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    mm = [P, I64, P, I64, P, I64, I64, I64, I64]
    L.gf2_mul.argtypes = mm + [P]
    L.gf2_addmul.argtypes = mm + [P]
    L.gf2_mul_sched.argtypes = mm + [I32, ctypes.POINTER(Schedule), P]
    L.gf2_mul_noalloc.argtypes = mm + [I32, ctypes.POINTER(Schedule), P]
    for f in (L.gf2_mul, L.gf2_addmul, L.gf2_mul_sched, L.gf2_mul_noalloc):
        f.restype = ctypes.c_int
    L.gf2_resolve_schedule.argtypes = [I64, I64, I64, ctypes.POINTER(Schedule), ctypes.POINTER(Schedule)]
    L.gf2_resolve_schedule.restype = ctypes.c_int
    L.gf2_kernel_variants.argtypes = [I32]
    L.gf2_kernel_variants.restype = I32
    L.gf2_workspace_bytes.argtypes = [I64, I64, I64, ctypes.POINTER(Schedule)]
    L.gf2_workspace_bytes.restype = ctypes.c_size_t
    L.gf2_reserve_workspace.argtypes = [ctypes.c_size_t]
    L.gf2_reserve_workspace.restype = ctypes.c_int
    L.gf2_status_string.argtypes = [ctypes.c_int]
    L.gf2_status_string.restype = ctypes.c_char_p
    L.gf2_last_error.restype = ctypes.c_char_p
    L.gf2_shutdown.restype = None
    L.gf2_trace_enable.argtypes = [I32]
    L.gf2_trace_enable.restype = ctypes.c_int
    L.gf2_trace_read.argtypes = [ctypes.c_void_p, I64, ctypes.POINTER(I64)]
    L.gf2_trace_read.restype = ctypes.c_int
    L.gf2_trace_clear.restype = None
    L.gf2_num_candidates.restype = I32
    L.gf2_candidate.argtypes = [I32, ctypes.POINTER(Schedule)]
    L.gf2_candidate.restype = ctypes.c_int
    L.gf2_mul_batched.argtypes = [ctypes.c_void_p, I64, P]
    L.gf2_mul_batched.restype = ctypes.c_int
    L.gf2_batch_plan_create.argtypes = [ctypes.c_void_p, I64, ctypes.POINTER(ctypes.c_void_p)]
    L.gf2_batch_plan_create.restype = ctypes.c_int
    L.gf2_batch_plan_execute.argtypes = [ctypes.c_void_p, P]
    L.gf2_batch_plan_execute.restype = ctypes.c_int
    L.gf2_batch_plan_destroy.argtypes = [ctypes.c_void_p]
    L.gf2_batch_plan_destroy.restype = ctypes.c_int
    L.gf2_batch_plan_schedule.argtypes = [ctypes.c_void_p, I64]
    L.gf2_batch_plan_schedule.restype = I32
    F = ctypes.c_float
    L.gf2_set_policy.argtypes = [I32]
    L.gf2_set_policy.restype = ctypes.c_int
    L.gf2_get_policy.restype = I32
    L.gf2_choose_schedule.argtypes = [I64, I64, I64, I32]
    L.gf2_choose_schedule.restype = I32
    L.gf2_autotune.argtypes = [I64, I64, I64, ctypes.c_double, I32, P, ctypes.POINTER(I32)]
    L.gf2_autotune.restype = ctypes.c_int
    L.gf2_autotune_batch.argtypes = [I64, I64, I64, ctypes.c_double, I32, P, ctypes.POINTER(I32), ctypes.POINTER(I32)]
    L.gf2_autotune_batch.restype = ctypes.c_int
    L.gf2_autotune_candidates.argtypes = [I64, I64, I64, ctypes.c_double, I32, I32, P, I32, P, ctypes.POINTER(I32)]
    L.gf2_autotune_candidates.restype = ctypes.c_int
    L.gf2_autotune_save.argtypes = [ctypes.c_char_p]
    L.gf2_autotune_save.restype = ctypes.c_int
    L.gf2_autotune_load.argtypes = [ctypes.c_char_p]
    L.gf2_autotune_load.restype = ctypes.c_int
    L.gf2_autotune_clear.restype = None
    L.gf2_mlp_param_count.restype = I64
    L.gf2_mlp_scratch_floats.argtypes = [I64]
    L.gf2_mlp_scratch_floats.restype = I64
    L.gf2_mlp_forward.argtypes = [P, P, I64, P, P, P]
    L.gf2_mlp_forward.restype = ctypes.c_int
    L.gf2_mlp_backward.argtypes = [P, P, I64, P, P, P, P, P, P, P, P]
    L.gf2_mlp_backward.restype = ctypes.c_int
    L.gf2_mlp_adam.argtypes = [P, P, P, P, I64, I32, F, F, F, F, P]
    L.gf2_mlp_adam.restype = ctypes.c_int
    L.gf2_mlp_argmin.argtypes = [P, I64, P, P, P]
    L.gf2_mlp_argmin.restype = ctypes.c_int
    L.gf2_set_model.argtypes = [P, I64, P]
    L.gf2_set_model.restype = ctypes.c_int
    L.gf2_lds_probe.argtypes = [I32, I32, I32, P, ctypes.POINTER(ctypes.c_double), P]
    L.gf2_lds_probe.restype = ctypes.c_int
    _LIB = L
    return L


def _check(status: int):
    if status != 0:
        raise GF2Error(status, lib().gf2_last_error().decode())


def last_error() -> str:
    return lib().gf2_last_error().decode()


def _stream_handle(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _mat(t):
    """(pointer, ld) of a 2-D int64 CUDA tensor with unit row stride."""
    if t is None:
        return ctypes.c_void_p(0), 0
    if t.dim() != 2:
        raise ValueError("matrices must be 2-D")
    if t.numel() > 0 and t.shape[1] > 1 and t.stride(1) != 1:
        raise ValueError("matrices must have unit stride along rows")
    if t.element_size() != 8:
        raise ValueError("matrices must hold 64-bit words (torch.int64)")
    if not t.is_cuda:
        raise ValueError("matrices must be on the GPU")
    ld = t.stride(0) if t.shape[0] > 1 else t.shape[1]   # torch reports arbitrary strides for 0/1 rows
    return ctypes.c_void_p(t.data_ptr()), ld


def mul_ptr(C, ldc, A, lda, B, ldb, m, k, n, *, accumulate=False, schedule=None, stream=None):
    """Raw-pointer form: C := A*B (or C ^= A*B).  Pointers are device addresses (ints)."""
    L = lib()
    s = _stream_handle(stream)
    if schedule is None and not accumulate:
        _check(L.gf2_mul(C, ldc, A, lda, B, ldb, m, k, n, s))
    elif schedule is None:
        _check(L.gf2_addmul(C, ldc, A, lda, B, ldb, m, k, n, s))
    else:
        _check(L.gf2_mul_sched(C, ldc, A, lda, B, ldb, m, k, n, int(accumulate), ctypes.byref(schedule), s))


NOALLOC_SCRATCH_BYTES = 64 << 20   # GF2_NOALLOC_SCRATCH_BYTES
# M4RM tile variants the persistent batch kernel runs (the candidates a batch may use).
BATCH_VARIANTS = (1, 2, 3, 4, 11, 12, 13, 16, 17, 18, 19, 20)


def batch_candidate(index):
    """True when candidate ``index`` runs inside the persistent batch kernel."""
    c = candidate(index)
    return c.kernel == KERNEL_M4RM and c.variant in BATCH_VARIANTS


def mul_noalloc_ptr(C, ldc, A, lda, B, ldb, m, k, n, *, accumulate=False, schedule=None, stream=None):
    """gf2_mul_noalloc: as ``mul_ptr`` with an explicit (or library-chosen) schedule, its workspace
    the library's static device array (no device allocation)."""
    _check(lib().gf2_mul_noalloc(C, ldc, A, lda, B, ldb, m, k, n, int(accumulate),
                                 ctypes.byref(schedule) if schedule is not None else None, _stream_handle(stream)))


def mul(C, A, B, m, k, n, *, accumulate=False, schedule=None, stream=None):
    """C := A*B over GF(2) (``accumulate=True``: C := C + A*B), on tensors."""
    pc, ldc = _mat(C)
    pa, lda = _mat(A)
    pb, ldb = _mat(B)
    mul_ptr(pc, ldc, pa, lda, pb, ldb, m, k, n, accumulate=accumulate, schedule=schedule, stream=stream)
    return C


class Problem(ctypes.Structure):
    """One product of a batch (mirrors gf2_problem)."""
    _fields_ = [("A", ctypes.c_void_p), ("B", ctypes.c_void_p), ("C", ctypes.c_void_p),
                ("m", ctypes.c_int64), ("k", ctypes.c_int64), ("n", ctypes.c_int64),
                ("lda", ctypes.c_int64), ("ldb", ctypes.c_int64), ("ldc", ctypes.c_int64),
                ("accumulate", ctypes.c_int32), ("schedule", ctypes.c_int32)]


def problem(C, A, B, m, k, n, *, accumulate=False, schedule=-1):
    """A batch entry over tensors (see ``mul``)."""
    pc, ldc = _mat(C)
    pa, lda = _mat(A)
    pb, ldb = _mat(B)
    return Problem(pa, pb, pc, m, k, n, lda, ldb, ldc, int(accumulate), int(schedule))


def _problem_array(problems):
    arr = (Problem * len(problems))()
    for i, p in enumerate(problems):
        arr[i] = p
    return arr


def mul_batched(problems, stream=None):
    """Run a list of ``Problem`` through the persistent batched executor (graph cached per batch)."""
    arr = _problem_array(problems)
    _check(lib().gf2_mul_batched(arr, len(problems), _stream_handle(stream)))


class BatchPlan:
    """Explicit batch plan: built once (synchronous), executed any number of times."""

    def __init__(self, problems):
        self._arr = _problem_array(problems)
        self.handle = ctypes.c_void_p(0)
        _check(lib().gf2_batch_plan_create(self._arr, len(problems), ctypes.byref(self.handle)))
        self.count = len(problems)

    def execute(self, stream=None):
        _check(lib().gf2_batch_plan_execute(self.handle, _stream_handle(stream)))

    def schedule(self, i):
        return int(lib().gf2_batch_plan_schedule(self.handle, i))

    def destroy(self):
        if self.handle:
            _check(lib().gf2_batch_plan_destroy(self.handle))
            self.handle = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def num_candidates() -> int:
    return int(lib().gf2_num_candidates())


def candidate(i: int) -> Schedule:
    s = Schedule()
    _check(lib().gf2_candidate(i, ctypes.byref(s)))
    return s


class TraceRecord(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("items", ctypes.c_int32), ("work", ctypes.c_double), ("ms", ctypes.c_double)]


TRACE_KINDS = {1: "m4rm", 2: "mfma", 3: "cubic", 4: "strassen_pre", 5: "strassen_post", 6: "fill", 7: "batch"}


def trace_enable(on: bool = True):
    _check(lib().gf2_trace_enable(int(on)))


def trace_read(max_records: int = 1 << 16):
    """List of (kind name, items, work, ms) for launches recorded since the last clear."""
    buf = (TraceRecord * max_records)()
    cnt = ctypes.c_int64(0)
    _check(lib().gf2_trace_read(buf, max_records, ctypes.byref(cnt)))
    return [(TRACE_KINDS.get(r.kind, str(r.kind)), r.items, r.work, r.ms) for r in buf[:cnt.value]]


def trace_clear():
    lib().gf2_trace_clear()


POLICY_FIXED, POLICY_AUTOTUNE, POLICY_MODEL = 0, 1, 2


def set_policy(policy: int):
    _check(lib().gf2_set_policy(policy))


def get_policy() -> int:
    return int(lib().gf2_get_policy())


def choose_schedule(m, k, n, batch=False) -> int:
    return int(lib().gf2_choose_schedule(m, k, n, int(batch)))


def resolve_schedule(m, k, n, schedule: Schedule | None = None) -> Schedule:
    """The schedule gf2_mul_sched runs for this shape (``schedule`` None: the library's choice)."""
    out = Schedule()
    _check(lib().gf2_resolve_schedule(m, k, n, ctypes.byref(schedule) if schedule is not None else None,
                                      ctypes.byref(out)))
    return out


def autotune(m, k, n, density=0.5, reps=3):
    """Time every candidate schedule on an m x k x n product; returns (ms array, best index).
    Negative entries mark candidates that could not run."""
    import numpy as np
    ms = np.zeros(num_candidates(), dtype=np.float32)
    best = ctypes.c_int32(-1)
    _check(lib().gf2_autotune(m, k, n, float(density), int(reps), ms.ctypes.data_as(ctypes.c_void_p),
                              ctypes.byref(best)))
    return ms, best.value


def autotune_batch(m, k, n, density=0.5, reps=3):
    """Per-product time of every candidate inside a batch of copies; returns (ms, best, copies)."""
    import numpy as np
    ms = np.zeros(num_candidates(), dtype=np.float32)
    best, copies = ctypes.c_int32(-1), ctypes.c_int32(0)
    _check(lib().gf2_autotune_batch(m, k, n, float(density), int(reps), ms.ctypes.data_as(ctypes.c_void_p),
                                    ctypes.byref(best), ctypes.byref(copies)))
    return ms, best.value, copies.value


def autotune_candidates(m, k, n, candidates, density=0.5, reps=3, batch=True):
    """Time only the listed candidates (alone, or per product inside a batch of copies);
    returns (ms with -1 for every other candidate, copies).  Does not touch the autotune cache."""
    import numpy as np
    ms = np.zeros(num_candidates(), dtype=np.float32)
    idx = np.ascontiguousarray(np.asarray(candidates, dtype=np.int32))
    copies = ctypes.c_int32(0)
    _check(lib().gf2_autotune_candidates(m, k, n, float(density), int(reps), int(bool(batch)),
                                         idx.ctypes.data_as(ctypes.c_void_p), int(idx.size),
                                         ms.ctypes.data_as(ctypes.c_void_p), ctypes.byref(copies)))
    return ms, copies.value


def autotune_save(path):
    _check(lib().gf2_autotune_save(str(path).encode()))


def autotune_load(path):
    _check(lib().gf2_autotune_load(str(path).encode()))


def autotune_clear():
    lib().gf2_autotune_clear()


def mlp_param_count() -> int:
    return int(lib().gf2_mlp_param_count())


def mlp_scratch_floats(batch: int) -> int:
    return int(lib().gf2_mlp_scratch_floats(batch))


def _f(t):
    """Device pointer of a float32 (or uint8 / int32) CUDA tensor, or NULL."""
    if t is None:
        return ctypes.c_void_p(0)
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous CUDA tensor")
    return ctypes.c_void_p(t.data_ptr())


def mlp_forward(params, X, Y, acts, stream=None):
    _check(lib().gf2_mlp_forward(_f(params), _f(X), X.shape[0], _f(Y), _f(acts), _stream_handle(stream)))


def mlp_backward(params, X, acts, Y, T, M, grads, scratch, loss=None, stream=None):
    _check(lib().gf2_mlp_backward(_f(params), _f(X), X.shape[0], _f(acts), _f(Y), _f(T), _f(M), _f(grads),
                                  _f(scratch), _f(loss), _stream_handle(stream)))


def mlp_adam(params, grads, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    _check(lib().gf2_mlp_adam(_f(params), _f(grads), _f(m), _f(v), params.numel(), int(step), float(lr),
                              float(beta1), float(beta2), float(eps), _stream_handle(stream)))


def mlp_argmin(Y, out, allowed=None, stream=None):
    _check(lib().gf2_mlp_argmin(_f(Y), Y.shape[0], _f(allowed), _f(out), _stream_handle(stream)))


def set_model(params, norm=None):
    """Install a schedule model (host float32 arrays) for POLICY_MODEL; ``params=None`` removes it."""
    import numpy as np
    if params is None:
        _check(lib().gf2_set_model(None, 0, None))
        return
    p = np.ascontiguousarray(params, dtype=np.float32)
    nrm = None if norm is None else np.ascontiguousarray(norm, dtype=np.float32)
    _check(lib().gf2_set_model(p.ctypes.data_as(ctypes.c_void_p), p.size,
                               nrm.ctypes.data_as(ctypes.c_void_p) if nrm is not None else None))


DEFAULT_MODEL = os.path.join(_HERE, "tune", "schedule_model.npz")


def load_model(path=DEFAULT_MODEL):
    """Install the trained schedule model stored by ``tune.train`` (params + feature norm)."""
    import numpy as np
    d = np.load(path)
    set_model(d["params"], d["norm"])
    return d


def kernel_variants(kernel: int) -> int:
    return int(lib().gf2_kernel_variants(kernel))


def workspace_bytes(m, k, n, schedule=None) -> int:
    return int(lib().gf2_workspace_bytes(m, k, n, ctypes.byref(schedule) if schedule is not None else None))


def reserve_workspace(nbytes: int):
    _check(lib().gf2_reserve_workspace(nbytes))


def shutdown():
    lib().gf2_shutdown()


def lds_probe(mode: int, blocks: int, iters: int, out, stream=None) -> float:
    """Launch the LDS bandwidth probe (mode 0: 16 B reads, 1: 4 B writes) on ``stream``; ``out``
    is an int64 CUDA tensor of at least blocks * 1024 words.  Returns the LDS bytes moved."""
    if out.numel() < blocks * 1024:
        raise ValueError("out must hold blocks * 1024 words")
    nbytes = ctypes.c_double(0)
    _check(lib().gf2_lds_probe(mode, blocks, iters, ctypes.c_void_p(out.data_ptr()), ctypes.byref(nbytes),
                               _stream_handle(stream)))
    return nbytes.value
