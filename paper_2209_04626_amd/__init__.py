"""Python binding of the mpjsvd C-ABI library (libmpjsvd.so, HIP for gfx950).

Argument marshalling only: every step of the SVD runs in the library's HIP
kernels.  PyTorch supplies device memory (inputs, outputs and the workspace)
and the current HIP stream.  Matrices cross the boundary column-major: an
m x n torch tensor is passed as the storage of its transpose, and results are
returned as transposed views of column-major storage.

There is no CPU fallback: if the library is missing or no GPU is present,
every entry point raises.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import weakref
from dataclasses import dataclass, field

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmpjsvd.so")
# tuning table measured on the target GPU by paper_2209_04626_amd/autotune.py
TUNE_PATH = os.path.join(_HERE, "tune_gfx950.json")

EXPORTS = [
    "svd_default_opts", "svd_workspace_size", "svd_diag_y_offset", "svd_plain", "svd_mixed",
    "svd_batched_plan_create", "svd_batched", "svd_batched_plan_destroy",
    "svd_backward_workspace_size", "svd_backward", "svd_backward_noalloc",
    "svd_status_string", "svd_last_error",
    "svd_set_tuning", "svd_tuning_lookup", "eig_workspace_size", "eig_mixed",
]

SVD_OK, SVD_WARN_NOCONV, SVD_ERR_NONFINITE, SVD_WARN_RANK_DEFICIENT = 0, 1, 2, 3
EIG_ERR_CLUSTER = 4
SVD_ERR_WAIT_TIMEOUT, SVD_ERR_BREAKDOWN, SVD_WARN_VSOLVE = 5, 6, 7
SVD_ERR_HIP, SVD_ERR_SCRATCH_LIMIT = -100, -101
# bytes of the fixed scratch array behind svd_backward_noalloc
BACKWARD_NOALLOC_SCRATCH_BYTES = 64 << 20
KERNEL_CLASSES = ["jac_gram<f32>", "jac_inner<f32>", "jac_update<f32>", "jac_gram<f64>",
                  "jac_inner<f64>", "jac_update<f64>", "qrcp", "qr_panel", "gemm", "jac_round<f32>",
                  "trsm_diag", "jac_round<bf16>"]
NCLASS = 12
BRANCH_AUTO, BRANCH_LOW, BRANCH_SKIP = 0, 1, 2


class SvdOpts(ctypes.Structure):
    _fields_ = [
        ("tol_alg", ctypes.c_double), ("tol_orth", ctypes.c_double),
        ("tol_cond_coef", ctypes.c_double), ("small_col_rel", ctypes.c_double),
        ("small_col_frac", ctypes.c_double), ("eps_work", ctypes.c_double),
        ("eps_low", ctypes.c_double), ("maxsweep_low", ctypes.c_int),
        ("maxsweep_work", ctypes.c_int), ("want_u", ctypes.c_int), ("want_v", ctypes.c_int),
        ("branch", ctypes.c_int), ("switch_method", ctypes.c_int),
        ("pivot_precision", ctypes.c_int), ("sign_normalize", ctypes.c_int),
        ("block_cols", ctypes.c_int), ("inner_sweeps", ctypes.c_int),
        ("kernel_timing", ctypes.c_int), ("low_stop_off", ctypes.c_double),
        ("block_cols_low", ctypes.c_int), ("block_cols_work", ctypes.c_int),
        ("v_method", ctypes.c_int), ("diagnostics", ctypes.c_int), ("tol_vsolve", ctypes.c_double),
        ("inner_pairs", ctypes.c_int), ("tol_cluster", ctypes.c_double),
        ("y2_safeguard", ctypes.c_int), ("tol_y2", ctypes.c_double),
        ("kernel_timing_every", ctypes.c_int), ("wait_polls", ctypes.c_int),
        ("fused_rounds", ctypes.c_int), ("capture", ctypes.c_int),
        ("half_sweeps", ctypes.c_int), ("half_stop_off", ctypes.c_double),
        ("half_storage", ctypes.c_int),
    ]


class SvdInfo(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int), ("branch_taken", ctypes.c_int), ("sweeps_low", ctypes.c_int),
        ("sweeps_work", ctypes.c_int), ("n_small", ctypes.c_int), ("orth", ctypes.c_double),
        ("cond_r", ctypes.c_double), ("stage_ms", ctypes.c_float * 8),
        ("off_low", ctypes.c_float * 32), ("off_work", ctypes.c_float * 32),
        ("kern_ms", ctypes.c_float * NCLASS), ("kern_calls", ctypes.c_int * NCLASS),
        ("kern_bytes", ctypes.c_double * NCLASS), ("kern_flops", ctypes.c_double * NCLASS),
        ("v_method_taken", ctypes.c_int), ("sweeps_vfix", ctypes.c_int),
        ("orth_vx", ctypes.c_double), ("orth_y", ctypes.c_double),
        ("n_y2", ctypes.c_int), ("sweeps_y2", ctypes.c_int), ("fused_fallback", ctypes.c_int),
        ("sweeps_half", ctypes.c_int),
    ]

    def as_dict(self) -> dict:
        return {
            "status": self.status, "branch_taken": self.branch_taken,
            "sweeps_low": self.sweeps_low, "sweeps_work": self.sweeps_work,
            "n_small": self.n_small, "orth": self.orth, "cond_r": self.cond_r,
            "stage_ms": list(self.stage_ms),
            "off_low": list(self.off_low)[:max(self.sweeps_low, 0)],
            "off_work": list(self.off_work)[:max(self.sweeps_work, 0)],
            "kern_ms": list(self.kern_ms), "kern_calls": list(self.kern_calls),
            "kern_bytes": list(self.kern_bytes), "kern_flops": list(self.kern_flops),
            "v_method_taken": self.v_method_taken, "sweeps_vfix": self.sweeps_vfix,
            "orth_vx": self.orth_vx, "orth_y": self.orth_y,
            "n_y2": self.n_y2, "sweeps_y2": self.sweeps_y2,
            "fused_fallback": self.fused_fallback, "sweeps_half": self.sweeps_half,
        }


class DeviceInfo:
    """svd_info written on the device by a stream-ordered call (capture=1):
    valid once the stream has reached the end of that call."""

    def __init__(self, device):
        import torch
        self.buf = torch.zeros(ctypes.sizeof(SvdInfo), dtype=torch.uint8, device=device)

    def read(self) -> dict:
        raw = bytes(self.buf.cpu().numpy().tobytes())
        return SvdInfo.from_buffer_copy(raw).as_dict()


class EigInfo(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int), ("sweeps_low", ctypes.c_int), ("sweeps_work", ctypes.c_int),
        ("n_clusters", ctypes.c_int), ("max_cluster", ctypes.c_int), ("stage_ms", ctypes.c_float * 4),
    ]

    def as_dict(self) -> dict:
        return {"status": self.status, "sweeps_low": self.sweeps_low, "sweeps_work": self.sweeps_work,
                "n_clusters": self.n_clusters, "max_cluster": self.max_cluster,
                "stage_ms": list(self.stage_ms)}


class SvdBatchInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("branch_taken", ctypes.c_int),
                ("sweeps_low", ctypes.c_int), ("sweeps_work", ctypes.c_int)]


_lib = None
_vp = ctypes.c_void_p
_ll = ctypes.c_longlong


def load():
    """Load libmpjsvd.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: run __graft_entry__.build() first")
    # torch brings its own HIP runtime (same soname, libamdhip64.so.7); load it
    # first so the library binds to that one instance instead of a second copy.
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    lib.svd_default_opts.argtypes = [ctypes.POINTER(SvdOpts), ctypes.c_int]
    lib.svd_default_opts.restype = None
    lib.svd_workspace_size.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(SvdOpts)]
    lib.svd_workspace_size.restype = ctypes.c_size_t
    lib.svd_diag_y_offset.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(SvdOpts)]
    lib.svd_diag_y_offset.restype = ctypes.c_size_t
    for fn in (lib.svd_plain, lib.svd_mixed):
        fn.argtypes = [ctypes.c_int, ctypes.c_int, _vp, ctypes.c_int, _vp, _vp, ctypes.c_int, _vp,
                       ctypes.c_int, _vp, ctypes.c_size_t, ctypes.POINTER(SvdOpts),
                       _vp, _vp]   # info: host SvdInfo, or device memory with capture=1
        fn.restype = ctypes.c_int
    lib.svd_batched_plan_create.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                            ctypes.POINTER(ctypes.c_int), ctypes.POINTER(SvdOpts),
                                            ctypes.POINTER(_vp), ctypes.POINTER(ctypes.c_size_t)]
    lib.svd_batched_plan_create.restype = ctypes.c_int
    lib.svd_batched.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp, _vp]
    lib.svd_batched.restype = ctypes.c_int
    lib.svd_batched_plan_destroy.argtypes = [_vp]
    lib.svd_batched_plan_destroy.restype = None
    lib.svd_backward_workspace_size.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.svd_backward_workspace_size.restype = ctypes.c_size_t
    lib.svd_backward.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp, _ll, _vp, _ll, _vp,
                                 _ll, _vp, _vp, _vp, _vp, _ll, ctypes.c_double, _vp,
                                 ctypes.c_size_t, _vp]
    lib.svd_backward.restype = ctypes.c_int
    lib.svd_backward_noalloc.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp, _ll, _vp, _ll,
                                         _vp, _ll, _vp, _vp, _vp, _vp, _ll, ctypes.c_double, _vp]
    lib.svd_backward_noalloc.restype = ctypes.c_int
    lib.eig_workspace_size.argtypes = [ctypes.c_int, ctypes.POINTER(SvdOpts)]
    lib.eig_workspace_size.restype = ctypes.c_size_t
    lib.eig_mixed.argtypes = [ctypes.c_int, _vp, ctypes.c_int, _vp, _vp, ctypes.c_int, _vp,
                              ctypes.c_size_t, ctypes.POINTER(SvdOpts), ctypes.POINTER(EigInfo), _vp]
    lib.eig_mixed.restype = ctypes.c_int
    lib.svd_status_string.argtypes = [ctypes.c_int]
    lib.svd_status_string.restype = ctypes.c_char_p
    lib.svd_last_error.argtypes = []
    lib.svd_last_error.restype = ctypes.c_char_p
    lib.svd_set_tuning.argtypes = [ctypes.c_char_p]
    lib.svd_set_tuning.restype = ctypes.c_int
    _ip = ctypes.POINTER(ctypes.c_int)
    lib.svd_tuning_lookup.argtypes = [ctypes.c_int, _ip, _ip, _ip]
    lib.svd_tuning_lookup.restype = ctypes.c_int
    _lib = lib
    if os.path.exists(TUNE_PATH):
        with open(TUNE_PATH) as fh:
            rc = lib.svd_set_tuning(fh.read().encode())
        if rc != 0:
            raise RuntimeError(f"{TUNE_PATH}: tuning table rejected ({rc})")
    return lib


def set_tuning(table) -> None:
    """Load a tuning table (dict or JSON text; None clears it)."""
    import json
    text = None if table is None else (table if isinstance(table, str) else json.dumps(table))
    rc = load().svd_set_tuning(None if text is None else text.encode())
    if rc != 0:
        raise ValueError(f"tuning table rejected ({rc})")


def tuning_lookup(n: int) -> dict:
    """The loaded table's entries for size n (0 = none)."""
    a, b, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    load().svd_tuning_lookup(n, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c))
    return {"b_low": a.value, "b_work": b.value, "wg_per_cu": c.value}


def default_opts(mixed: bool = True, **kw) -> SvdOpts:
    o = SvdOpts()
    load().svd_default_opts(ctypes.byref(o), int(mixed))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, v)
    return o


def workspace_size(m: int, n: int, opts: SvdOpts | None = None) -> int:
    return int(load().svd_workspace_size(m, n, ctypes.byref(opts) if opts is not None else None))


def _check_device(t, name):
    import torch
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise ValueError(f"{name} must be a torch tensor on a GPU")
    if t.dtype != torch.float64:
        raise ValueError(f"{name} must be float64")


def _stream_ptr(dev):
    import torch
    return torch.cuda.current_stream(dev).cuda_stream


class Workspace:
    """A reusable device workspace (a torch uint8 tensor)."""

    def __init__(self):
        self.buf = None

    def get(self, nbytes: int, device):
        import torch
        if self.buf is None or self.buf.numel() < nbytes or self.buf.device != device:
            self.buf = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
        return self.buf


_ws_default = Workspace()


def svd(A, mode: str = "mixed", workspace: Workspace | None = None, opts: SvdOpts | None = None,
        out=None, **kw):
    """A = U diag(S) V^T for an m x n float64 CUDA tensor, m >= n.

    mode: "mixed" (Algorithm 4) or "plain" (Algorithm 2).  Keyword arguments
    set svd_opts fields.  Returns (U, S, V, info); U is m x n, V is n x n.
    info is a dict, or with capture=1 (stream-ordered: nothing synchronises,
    so the call can be captured in a CUDA/HIP graph) a DeviceInfo to read()
    after the stream has run.  out: the (U, S, V, DeviceInfo) of an earlier
    capture=1 call of the same shape, written again in place.
    """
    import torch
    lib = load()
    _check_device(A, "A")
    if A.dim() != 2:
        raise ValueError("A must be 2-D")
    m, n = A.shape
    mixed = mode == "mixed"
    if mode not in ("mixed", "plain"):
        raise ValueError(mode)
    o = opts if opts is not None else default_opts(mixed, **kw)
    dev = A.device
    Acm = A.t().contiguous()              # storage = column-major m x n
    if out is not None:
        if not o.capture:
            raise ValueError("out= is for capture=1 calls")
        Ut, S, Vt, dinfo = out[0].t(), out[1], out[2].t(), out[3]
        if Ut.shape != (n, m) or S.shape != (n,) or Vt.shape != (n, n) or not (
                Ut.is_contiguous() and Vt.is_contiguous()):
            raise ValueError("out does not match A")
    else:
        Ut = torch.empty((n, m), dtype=torch.float64, device=dev)
        Vt = torch.empty((n, n), dtype=torch.float64, device=dev)
        S = torch.empty((n,), dtype=torch.float64, device=dev)
        dinfo = DeviceInfo(dev) if o.capture else None
    nbytes = int(lib.svd_workspace_size(m, n, ctypes.byref(o)))
    ws = (workspace or _ws_default).get(nbytes, dev)
    info = SvdInfo()
    info_ptr = dinfo.buf.data_ptr() if o.capture else ctypes.addressof(info)
    fn = lib.svd_mixed if mixed else lib.svd_plain
    with torch.cuda.device(dev):
        rc = fn(m, n, Acm.data_ptr(), max(m, 1), S.data_ptr(), Ut.data_ptr(), max(m, 1),
                Vt.data_ptr(), max(n, 1), ws.data_ptr(), ws.numel(), ctypes.byref(o),
                info_ptr, _stream_ptr(dev))
    if rc != 0:
        raise RuntimeError(f"svd_{mode} returned {rc}: {lib.svd_status_string(rc).decode()} "
                           f"[{lib.svd_last_error().decode()}]")
    return Ut.t(), S, Vt.t(), (dinfo if o.capture else info.as_dict())


def eigh(A, workspace: Workspace | None = None, opts: SvdOpts | None = None, **kw):
    """A = X diag(W) X^T for a symmetric n x n float64 CUDA tensor by the
    mixed-precision eigensolver (Algorithm 6).  Keyword arguments set svd_opts
    fields.  Returns (W ascending, X, info dict)."""
    import torch
    lib = load()
    _check_device(A, "A")
    if A.dim() != 2 or A.shape[0] != A.shape[1]:
        raise ValueError("A must be square")
    n = A.shape[0]
    o = opts if opts is not None else default_opts(True, **kw)
    dev = A.device
    Acm = A.t().contiguous()
    W = torch.empty((n,), dtype=torch.float64, device=dev)
    Xt = torch.empty((n, n), dtype=torch.float64, device=dev)
    nbytes = int(lib.eig_workspace_size(n, ctypes.byref(o)))
    ws = (workspace or _ws_default).get(nbytes, dev)
    info = EigInfo()
    with torch.cuda.device(dev):
        rc = lib.eig_mixed(n, Acm.data_ptr(), max(n, 1), W.data_ptr(), Xt.data_ptr(), max(n, 1),
                           ws.data_ptr(), ws.numel(), ctypes.byref(o), ctypes.byref(info), _stream_ptr(dev))
    if rc != 0:
        raise RuntimeError(f"eig_mixed returned {rc}: {lib.svd_status_string(rc).decode()} "
                           f"[{lib.svd_last_error().decode()}]")
    return W, Xt.t(), info.as_dict()


def call_raw(mode: str, m: int, n: int, A_ptr: int, lda: int, S_ptr: int, U_ptr: int, ldu: int,
             V_ptr: int, ldv: int, work_ptr: int, work_bytes: int, opts: SvdOpts | None,
             stream: int):
    """Direct C-ABI call with raw pointers (for argument-checking tests)."""
    lib = load()
    info = SvdInfo()
    fn = lib.svd_mixed if mode == "mixed" else lib.svd_plain
    rc = fn(m, n, A_ptr, lda, S_ptr, U_ptr, ldu, V_ptr, ldv, work_ptr, work_bytes,
            ctypes.byref(opts) if opts is not None else None, ctypes.byref(info), stream)
    return rc, info.as_dict()


# ----------------------------------------------------------------------------- batched
# Live plans, destroyed by an exit handler that runs while the HIP runtime
# and the library are still loaded (a plan holds a graph exec, a capture
# stream and device metadata, which must not outlive the runtime's own
# teardown at process exit).
_live_plans = weakref.WeakSet()


@dataclass(eq=False)
class BatchedPlan:
    handle: int
    work_bytes: int
    shapes: list
    offA: list = field(default_factory=list)
    offS: list = field(default_factory=list)
    offV: list = field(default_factory=list)
    _lib = None          # the loaded library (kept so close() needs no module global)

    def close(self):
        """Release the plan's device resources (idempotent)."""
        if self.handle and self._lib is not None:
            self._lib.svd_batched_plan_destroy(self.handle)
        self.handle = 0

    def __del__(self):
        self.close()


@atexit.register
def _close_plans():
    for p in list(_live_plans):
        p.close()


def batched_plan(shapes, opts: SvdOpts | None = None) -> BatchedPlan:
    lib = load()
    b = len(shapes)
    hm = (ctypes.c_int * max(b, 1))(*[s[0] for s in shapes])
    hn = (ctypes.c_int * max(b, 1))(*[s[1] for s in shapes])
    h = _vp()
    wb = ctypes.c_size_t()
    rc = lib.svd_batched_plan_create(b, hm, hn, ctypes.byref(opts) if opts is not None else None,
                                     ctypes.byref(h), ctypes.byref(wb))
    if rc != 0:
        raise RuntimeError(f"svd_batched_plan_create returned {rc}")
    offA, offS, offV = [], [], []
    a = s = v = 0
    for (m, n) in shapes:
        offA.append(a); offS.append(s); offV.append(v)
        a += m * n; s += n; v += n * n
    p = BatchedPlan(h.value or 0, int(wb.value), list(shapes), offA, offS, offV)
    p._lib = lib
    p.totA, p.totS, p.totV = a, s, v
    _live_plans.add(p)
    return p


def pack_batch(mats, device):
    """Pack a list of m x n arrays (numpy or torch) into the column-major layout."""
    import numpy as np
    import torch
    flat = [np.asarray(M, dtype=np.float64).ravel(order="F") for M in mats]
    return torch.from_numpy(np.concatenate(flat) if flat else np.zeros(0)).to(device)


def svd_batched(plan: BatchedPlan, A_packed, workspace: Workspace | None = None, out=None):
    """Run the batched mixed SVD; returns packed (S, U, V) tensors and info.

    out: optional (S, U, V, info) tensors from an earlier call with this plan
    to write into; with the same input, outputs and workspace the library
    replays its captured graph instead of capturing a new one."""
    import torch
    lib = load()
    _check_device(A_packed, "A_packed")
    dev = A_packed.device
    if out is not None:
        S, U, V, info = out
    else:
        S = torch.empty(max(plan.totS, 1), dtype=torch.float64, device=dev)
        U = torch.empty(max(plan.totA, 1), dtype=torch.float64, device=dev)
        V = torch.empty(max(plan.totV, 1), dtype=torch.float64, device=dev)
        info = torch.zeros((max(len(plan.shapes), 1), 4), dtype=torch.int32, device=dev)
    ws = (workspace or _ws_default).get(plan.work_bytes, dev)
    with torch.cuda.device(dev):
        rc = lib.svd_batched(plan.handle, A_packed.data_ptr(), S.data_ptr(), U.data_ptr(),
                             V.data_ptr(), ws.data_ptr(), ws.numel(), info.data_ptr(),
                             _stream_ptr(dev))
    if rc != 0:
        raise RuntimeError(f"svd_batched returned {rc}")
    return S, U, V, info


_uniform_plans = {}


def svd_batched_uniform(A, workspace: Workspace | None = None):
    """svd_batched on a (B, m, n) float64 CUDA tensor of equal-size matrices
    (n <= m <= 256): returns U (B, m, n), S (B, n), V (B, n, n) and the
    (B, 4) per-matrix info tensor.  Plans are kept per shape and device."""
    import torch
    _check_device(A, "A")
    if A.dim() != 3:
        raise ValueError("A must be 3-D")
    B, m, n = A.shape
    if not (1 <= n <= m <= 256):
        raise ValueError("svd_batched takes 1 <= n <= m <= 256")
    key = (B, m, n, A.device)
    plan = _uniform_plans.get(key)
    if plan is None:
        if len(_uniform_plans) >= 8:
            _uniform_plans.pop(next(iter(_uniform_plans))).close()
        plan = _uniform_plans[key] = batched_plan([(m, n)] * B)
    packed = A.transpose(1, 2).contiguous().view(-1)     # column-major, ld = m
    S, U, V, info = svd_batched(plan, packed, workspace)
    return (U[:B * m * n].view(B, n, m).transpose(1, 2), S[:B * n].view(B, n),
            V[:B * n * n].view(B, n, n).transpose(1, 2), info)


def unpack_batch(plan: BatchedPlan, S, U, V):
    """Split packed outputs into per-matrix (U, S, V) torch views."""
    out = []
    for j, (m, n) in enumerate(plan.shapes):
        s = S[plan.offS[j]:plan.offS[j] + n]
        u = U[plan.offA[j]:plan.offA[j] + m * n].view(n, m).t()
        v = V[plan.offV[j]:plan.offV[j] + n * n].view(n, n).t()
        out.append((u, s, v))
    return out


# ----------------------------------------------------------------------------- backward
def svd_backward(U, S, V, gU=None, gS=None, gV=None, eps_deg: float = 1e-12,
                 workspace: Workspace | None = None, noalloc: bool = False):
    """Batched adjoint.  U (B, m, n), S (B, n), V (B, n, n) float64 CUDA
    tensors (any strides); cotangents of the same shapes or None.  Returns gA
    (B, m, n).  noalloc=True calls svd_backward_noalloc (the library's fixed
    scratch array instead of a workspace)."""
    import torch
    lib = load()
    for t, nm in ((U, "U"), (S, "S"), (V, "V")):
        _check_device(t, nm)
    Bt, m, n = U.shape
    dev = U.device

    def cm(x):  # (B, r, c) -> storage of column-major r x c blocks
        return None if x is None else x.transpose(1, 2).contiguous()

    Uc, Vc = cm(U), cm(V)
    Sc = S.contiguous()
    gUc, gVc = cm(gU), cm(gV)
    gSc = None if gS is None else gS.contiguous()
    gA = torch.empty((Bt, n, m), dtype=torch.float64, device=dev)
    if noalloc:
        with torch.cuda.device(dev):
            rc = lib.svd_backward_noalloc(
                Bt, m, n, Uc.data_ptr(), m * n, Sc.data_ptr(), n, Vc.data_ptr(), n * n,
                gUc.data_ptr() if gUc is not None else None,
                gSc.data_ptr() if gSc is not None else None,
                gVc.data_ptr() if gVc is not None else None,
                gA.data_ptr(), m * n, float(eps_deg), _stream_ptr(dev))
        if rc != 0:
            raise RuntimeError(f"svd_backward_noalloc returned {rc}: "
                               f"{lib.svd_last_error().decode()}")
        return gA.transpose(1, 2)
    nbytes = int(lib.svd_backward_workspace_size(Bt, m, n))
    ws = (workspace or _ws_default).get(nbytes, dev)
    with torch.cuda.device(dev):
        rc = lib.svd_backward(Bt, m, n, Uc.data_ptr(), m * n, Sc.data_ptr(), n, Vc.data_ptr(), n * n,
                              gUc.data_ptr() if gUc is not None else None,
                              gSc.data_ptr() if gSc is not None else None,
                              gVc.data_ptr() if gVc is not None else None,
                              gA.data_ptr(), m * n, float(eps_deg), ws.data_ptr(), ws.numel(),
                              _stream_ptr(dev))
    if rc != 0:
        raise RuntimeError(f"svd_backward returned {rc}")
    return gA.transpose(1, 2)


def _autograd_fn():
    import torch

    class SVD(torch.autograd.Function):
        """Differentiable SVD: forward svd_mixed (a 2-D input), svd_batched (a
        3-D input of matrices with n <= m <= 256) or svd_mixed per matrix (a
        3-D input of larger matrices); backward svd_backward."""

        @staticmethod
        def forward(ctx, A):
            if A.dim() == 2:
                U, S, V, _ = svd(A, "mixed")
                ctx.save_for_backward(U.unsqueeze(0), S.unsqueeze(0), V.unsqueeze(0))
                ctx.single = True
                return U, S, V
            if A.dim() == 3 and A.shape[0] > 0 and 1 <= A.shape[2] <= A.shape[1] <= 256:
                U, S, V, _ = svd_batched_uniform(A.detach())
            else:
                outs = [svd(A[b], "mixed")[:3] for b in range(A.shape[0])]
                U = torch.stack([o[0] for o in outs])
                S = torch.stack([o[1] for o in outs])
                V = torch.stack([o[2] for o in outs])
            ctx.save_for_backward(U, S, V)
            ctx.single = False
            return U, S, V

        @staticmethod
        def backward(ctx, gU, gS, gV):
            U, S, V = ctx.saved_tensors
            if ctx.single:
                gU = None if gU is None else gU.unsqueeze(0)
                gS = None if gS is None else gS.unsqueeze(0)
                gV = None if gV is None else gV.unsqueeze(0)
            gA = svd_backward(U, S, V, gU, gS, gV)
            return gA[0] if ctx.single else gA

    return SVD


_SVD = None


def SVD():
    """The torch.autograd.Function class (created on first use)."""
    global _SVD
    if _SVD is None:
        _SVD = _autograd_fn()
    return _SVD
