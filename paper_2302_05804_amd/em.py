"""ctypes binding of libem.so (C ABI in include/em.h).

Argument marshalling only: every step of the EM iteration runs in the HIP
kernels of libem.so.  PyTorch tensors provide device memory and the stream;
their device addresses are passed as plain pointers.  Importing this module
raises if the library has not been built (``python -m
paper_2302_05804_amd.build``) -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libem.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2302_05804_amd.build`")

_lib = ctypes.CDLL(LIB_PATH)

# status codes (include/em.h)
OK, EINVAL, ENOMEM, EDEVICE, EAGAIN, ECANCELED, ENOTSUP = 0, -1, -2, -3, -4, -5, -6
# precisions
FP32, BF16_SPLIT, FP16_SPLIT, BF16 = 0, 1, 2, 3
# weight placement
W_ADJOINT, W_LITERAL, W_STUDENT_T = 0, 1, 2

_NAMES = {OK: "EM_OK", EINVAL: "EM_EINVAL", ENOMEM: "EM_ENOMEM", EDEVICE: "EM_EDEVICE",
          EAGAIN: "EM_EAGAIN", ECANCELED: "EM_ECANCELED", ENOTSUP: "EM_ENOTSUP"}


class EMError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        msg = _lib.em_last_error().decode(errors="replace")
        super().__init__(f"{where}: {_NAMES.get(code, code)}: {msg}")


class Problem(ctypes.Structure):
    _fields_ = [("n_frames", ctypes.c_int32), ("frame_h", ctypes.c_int32),
                ("frame_w", ctypes.c_int32), ("psf_k", ctypes.c_int32),
                ("sr", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("weight_mode", ctypes.c_int32), ("nu", ctypes.c_float)]

    @classmethod
    def make(cls, n, frame_h, frame_w, psf_k, sr=1, precision=FP32, weight_mode=W_ADJOINT,
             nu=0.0):
        """nu > 0 selects Student-t noise with nu degrees of freedom (EM_W_STUDENT_T)."""
        if nu:
            weight_mode = W_STUDENT_T
        return cls(int(n), int(frame_h), int(frame_w), int(psf_k), int(sr), int(precision),
                   int(weight_mode), float(nu))

    @property
    def latent_shape(self):
        return (self.frame_h * self.sr, self.frame_w * self.sr)


class PsfProblem(ctypes.Structure):
    """em_psf_problem: the fit of Eq. (4) (field meanings in include/em.h)."""
    _fields_ = [("n_frames", ctypes.c_int32), ("psf_k", ctypes.c_int32),
                ("out_k", ctypes.c_int32), ("factor", ctypes.c_int32),
                ("n_steps", ctypes.c_int32), ("sigma", ctypes.c_float),
                ("lambda_", ctypes.c_float), ("lr", ctypes.c_float),
                ("lr_decay", ctypes.c_float), ("beta1", ctypes.c_float),
                ("beta2", ctypes.c_float), ("eps", ctypes.c_float)]


_P = ctypes.c_void_p
_PP = ctypes.POINTER(ctypes.c_void_p)
_sig = {
    "em_version": (ctypes.c_char_p, []),
    "em_last_error": (ctypes.c_char_p, []),
    "em_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(Problem)]),
    "em_init": (ctypes.c_int, [_PP, ctypes.POINTER(Problem), _P, _P, _P, _P, _P, _P,
                               ctypes.c_size_t, _P]),
    "em_iterate": (ctypes.c_int, [_P, ctypes.c_int32, _P]),
    "em_iterate_tol": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_double, ctypes.c_int32,
                                      ctypes.POINTER(ctypes.c_int32), _P, _P]),
    "em_loglik": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_double)]),
    "em_terms": (ctypes.c_int, [_P, _P, _P]),
    "em_profile": (ctypes.c_int, [_P, ctypes.c_int32, _P]),
    "em_sync": (ctypes.c_int, [_P]),
    "em_server_create": (ctypes.c_int, [_PP, ctypes.c_size_t, ctypes.c_int32, _P]),
    "em_server_destroy": (ctypes.c_int, [_P]),
    "em_job_bytes": (ctypes.c_size_t, [ctypes.POINTER(Problem)]),
    "em_submit": (ctypes.c_int, [_P, ctypes.POINTER(Problem), _P, _P, _P, ctypes.c_int32,
                                 ctypes.POINTER(ctypes.c_int64)]),
    "em_poll": (ctypes.c_int, [_P, ctypes.c_int64, _P, ctypes.POINTER(ctypes.c_double)]),
    "em_wait": (ctypes.c_int, [_P, ctypes.c_int64, _P, ctypes.POINTER(ctypes.c_double)]),
    "em_cancel": (ctypes.c_int, [_P, ctypes.c_int64]),
    "em_release": (ctypes.c_int, [_P, ctypes.c_int64]),
    "em_job_times": (ctypes.c_int, [_P, ctypes.c_int64, ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(ctypes.c_double)]),
    "em_server_stats": (ctypes.c_int, [_P, _P]),
    "em_server_phase_seconds": (ctypes.c_int, [_P, _P]),
    "em_server_staging": (ctypes.c_int, [_P, _P]),
    "em_variant_count": (ctypes.c_int, []),
    "em_check_plan": (ctypes.c_int, [ctypes.POINTER(Problem)]),
    "em_set_variants": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32]),
    "em_autotune": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                   ctypes.POINTER(ctypes.c_int32), _P]),
    "em_destroy": (ctypes.c_int, [_P]),
    "em_run_noalloc": (ctypes.c_int, [ctypes.POINTER(Problem), _P, _P, _P, _P, _P, ctypes.c_int32,
                                      _P, _P]),
    "em_forward_op": (ctypes.c_int, [ctypes.POINTER(Problem), _P, _P, _P, _P, ctypes.c_size_t, _P]),
    "em_adjoint_op": (ctypes.c_int, [ctypes.POINTER(Problem), _P, _P, _P, _P, ctypes.c_size_t, _P]),
    "em_upsample": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                   _P, _P, _P, _P, _P]),
    "em_psf_defaults": (None, [ctypes.POINTER(PsfProblem)]),
    "em_psf_fit": (ctypes.c_int, [ctypes.POINTER(PsfProblem), _P, _P, _P, _P, _P]),
}
for _name, (_res, _args) in _sig.items():
    _fn = getattr(_lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args


def exported_symbols():
    """Names of the C ABI entry points this binding resolved."""
    return sorted(_sig)


def version() -> str:
    return _lib.em_version().decode()


def check_plan(p: Problem) -> None:
    """Host-only: every launch descriptor for p matches its grid (raises otherwise)."""
    _check(_lib.em_check_plan(ctypes.byref(p)), "em_check_plan")


def workspace_bytes(p: Problem) -> int:
    return int(_lib.em_workspace_bytes(ctypes.byref(p)))


def _check(code: int, where: str):
    if code != OK:
        raise EMError(code, where)


def _torch():
    import torch
    return torch


def _dev_ptr(t, name, numel=None, dtype=None):
    """Device address of a contiguous tensor of `dtype` (float32 unless given:
    the workspace is the one byte buffer) holding `numel` elements."""
    torch = _torch()
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    want = torch.float32 if dtype is None else dtype
    if t.dtype != want:
        raise TypeError(f"{name} must be {str(want).replace('torch.', '')}, not "
                        f"{str(t.dtype).replace('torch.', '')}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} elements, {numel} expected")
    if not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    return ctypes.c_void_p(t.data_ptr())


def _ws_ptr(ws):
    return _dev_ptr(ws, "workspace", dtype=_torch().uint8)


def _stream_ptr(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream), stream


def alloc_workspace(p: Problem, device="cuda"):
    torch = _torch()
    nb = workspace_bytes(p)
    if nb == 0:
        raise EMError(EINVAL, "em_workspace_bytes")
    return torch.empty(nb, dtype=torch.uint8, device=device)


NOALLOC_SCRATCH_BYTES = 256 << 20   # EM_NOALLOC_SCRATCH_BYTES


def run_noalloc(p: Problem, y, v, psf, x, n_iter: int, x0=None, trace: bool = False,
                stream=None) -> Optional[np.ndarray]:
    """em_run_noalloc: one job (set-up and n_iter iterations) in the library's
    static scratch, allocating nothing; x receives the iterate.  Returns the
    log-likelihood trace when asked.  Synchronous."""
    nf = p.n_frames * p.frame_h * p.frame_w
    nl = p.latent_shape[0] * p.latent_shape[1]
    sp, _ = _stream_ptr(stream)
    tr = np.zeros(max(int(n_iter), 1), np.float64) if trace else None
    _check(_lib.em_run_noalloc(ctypes.byref(p), _dev_ptr(y, "y", nf), _dev_ptr(v, "v", nf),
                               _dev_ptr(psf, "psf", p.n_frames * p.psf_k ** 2),
                               _dev_ptr(x0, "x0", nl), _dev_ptr(x, "x", nl), int(n_iter),
                               tr.ctypes.data_as(_P) if trace else None, sp), "em_run_noalloc")
    return tr[:n_iter] if trace else None


class Context:
    """One deconvolution job: wraps em_init / em_iterate / em_loglik / em_destroy.

    y, v: (n, Hf, Wf) float32 device tensors; psf: (n, K, K); x: latent-size
    float32 tensor that receives the iterate; x0 optional (None = flat guess).
    All tensors are borrowed for the lifetime of the context.
    """

    def __init__(self, p: Problem, y, v, psf, x, x0=None, workspace=None, stream=None):
        nf = p.n_frames * p.frame_h * p.frame_w
        nl = p.latent_shape[0] * p.latent_shape[1]
        self.p = p
        self._keep = [y, v, psf, x, x0]
        self.ws = workspace if workspace is not None else alloc_workspace(p, device=y.device)
        self._keep.append(self.ws)
        sp, self.stream = _stream_ptr(stream)
        h = ctypes.c_void_p()
        _check(_lib.em_init(ctypes.byref(h), ctypes.byref(p), _dev_ptr(y, "y", nf),
                            _dev_ptr(v, "v", nf), _dev_ptr(psf, "psf", p.n_frames * p.psf_k ** 2),
                            _dev_ptr(x0, "x0", nl), _dev_ptr(x, "x", nl),
                            _ws_ptr(self.ws), self.ws.numel(), sp), "em_init")
        self._h = h

    def iterate(self, n_iter: int, trace: bool = False) -> Optional[np.ndarray]:
        if trace:
            tr = np.zeros(max(n_iter, 1), np.float64)
            _check(_lib.em_iterate(self._h, int(n_iter), tr.ctypes.data_as(_P)), "em_iterate")
            return tr[:n_iter]
        _check(_lib.em_iterate(self._h, int(n_iter), None), "em_iterate")
        return None

    def iterate_tol(self, max_iter: int, tol: float, check_every: int = 1, trace: bool = False):
        done = ctypes.c_int32(0)
        rc = np.zeros(max(max_iter, 1), np.float64)
        tr = np.zeros(max(max_iter, 1), np.float64) if trace else None
        _check(_lib.em_iterate_tol(self._h, int(max_iter), float(tol), int(check_every),
                                   ctypes.byref(done),
                                   tr.ctypes.data_as(_P) if tr is not None else None,
                                   rc.ctypes.data_as(_P)), "em_iterate_tol")
        k = done.value
        return k, rc[:k], (tr[:k] if tr is not None else None)

    def loglik(self) -> float:
        out = ctypes.c_double(0.0)
        _check(_lib.em_loglik(self._h, ctypes.byref(out)), "em_loglik")
        return out.value

    def terms(self):
        """(B, Dn) of Eq. (2) at the current iterate, as new device tensors."""
        torch = _torch()
        B = torch.empty(self.p.latent_shape, dtype=torch.float32, device=self.ws.device)
        Dn = torch.empty_like(B)
        _check(_lib.em_terms(self._h, _dev_ptr(B, "B"), _dev_ptr(Dn, "Dn")), "em_terms")
        return B, Dn

    def profile(self, n_iter: int):
        """Mean per-launch ms of (forward, adjoint, separate update, iteration)."""
        out = np.zeros(4, np.float64)
        _check(_lib.em_profile(self._h, int(n_iter), out.ctypes.data_as(_P)), "em_profile")
        return out

    def set_variants(self, fwd: int, adj: int):
        _check(_lib.em_set_variants(self._h, int(fwd), int(adj)), "em_set_variants")

    def autotune(self, n_rep: int = 3):
        """Time every kernel variant on this job; returns (fwd, adj, ms[2, nv])."""
        nv = int(_lib.em_variant_count())
        ms = np.zeros(2 * nv, np.float64)
        f = ctypes.c_int32(0)
        a = ctypes.c_int32(0)
        _check(_lib.em_autotune(self._h, int(n_rep), ctypes.byref(f), ctypes.byref(a),
                                ms.ctypes.data_as(_P)), "em_autotune")
        return f.value, a.value, ms.reshape(2, nv)

    def sync(self):
        _check(_lib.em_sync(self._h), "em_sync")

    def close(self):
        if getattr(self, "_h", None):
            _lib.em_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def forward_op(p: Problem, psf, x, m=None, workspace=None, stream=None):
    """m_t = F_t x for every frame (n, Hf, Wf)."""
    torch = _torch()
    if m is None:
        m = torch.empty((p.n_frames, p.frame_h, p.frame_w), dtype=torch.float32, device=x.device)
    ws = workspace if workspace is not None else alloc_workspace(p, device=x.device)
    sp, _ = _stream_ptr(stream)
    nl = p.latent_shape[0] * p.latent_shape[1]
    _check(_lib.em_forward_op(ctypes.byref(p), _dev_ptr(psf, "psf", p.n_frames * p.psf_k ** 2),
                              _dev_ptr(x, "x", nl),
                              _dev_ptr(m, "m", p.n_frames * p.frame_h * p.frame_w),
                              _ws_ptr(ws), ws.numel(), sp), "em_forward_op")
    return m


def adjoint_op(p: Problem, psf, r, s=None, workspace=None, stream=None):
    """s_t = F_t^T r_t for every frame (n, Hl, Wl)."""
    torch = _torch()
    hl, wl = p.latent_shape
    if s is None:
        s = torch.empty((p.n_frames, hl, wl), dtype=torch.float32, device=r.device)
    ws = workspace if workspace is not None else alloc_workspace(p, device=r.device)
    sp, _ = _stream_ptr(stream)
    _check(_lib.em_adjoint_op(ctypes.byref(p), _dev_ptr(psf, "psf", p.n_frames * p.psf_k ** 2),
                              _dev_ptr(r, "r", p.n_frames * p.frame_h * p.frame_w),
                              _dev_ptr(s, "s", p.n_frames * hl * wl),
                              _ws_ptr(ws), ws.numel(), sp), "em_adjoint_op")
    return s


def upsample(y, v, factor: int = 2, stream=None):
    """(y_up, v_up): the up-sampled exposures of the super-resolution run the
    paper describes after Eq. (4) (each pixel replicated into a factor x factor
    block, y / factor^2, v / factor^4); new device tensors."""
    torch = _torch()
    n, hf, wf = y.shape
    yu = torch.empty((n, factor * hf, factor * wf), dtype=torch.float32, device=y.device)
    vu = torch.empty_like(yu)
    sp, _ = _stream_ptr(stream)
    _check(_lib.em_upsample(int(n), int(hf), int(wf), int(factor), _dev_ptr(y, "y", n * hf * wf),
                            _dev_ptr(v, "v", n * hf * wf), _dev_ptr(yu, "y_up"),
                            _dev_ptr(vu, "v_up"), sp), "em_upsample")
    return yu, vu


def psf_problem(n_frames: int, psf_k: int, out_k: int = 43, factor: int = 2, **kw) -> PsfProblem:
    """em_psf_problem with the library's defaults, then the given fields
    (sigma defaults to factor; keyword `lam` sets lambda, `steps` n_steps,
    `decay` lr_decay)."""
    p = PsfProblem()
    _lib.em_psf_defaults(ctypes.byref(p))
    p.n_frames, p.psf_k, p.out_k, p.factor = int(n_frames), int(psf_k), int(out_k), int(factor)
    p.sigma = float(factor)
    alias = {"lam": "lambda_", "steps": "n_steps", "decay": "lr_decay"}
    for k, v in kw.items():
        setattr(p, alias.get(k, k), v)
    return p


def psf_fit(f, out_k: int = 43, factor: int = 2, h0=None, objective: bool = True, stream=None,
            **kw):
    """Super-resolved PSFs of Eq. (4) for every frame-grid PSF in f
    (n x Kf x Kf device tensor): (h n x out_k x out_k, objective n float64 or
    None), new device tensors; keywords as psf_problem."""
    torch = _torch()
    n, kf = int(f.shape[0]), int(f.shape[1])
    p = psf_problem(n, kf, out_k, factor, **kw)
    h = torch.empty((n, out_k, out_k), dtype=torch.float32, device=f.device)
    obj = torch.empty(n, dtype=torch.float64, device=f.device) if objective else None
    psf_fit_into(p, f, h, obj, h0, stream)
    return h, obj


def psf_fit_into(p: PsfProblem, f, h, objective=None, h0=None, stream=None):
    """em_psf_fit on caller-owned device tensors (f, h float32; objective
    float64 of n_frames or None; h0 float32 or None); asynchronous."""
    torch = _torch()
    n, kf, kh = p.n_frames, p.psf_k, p.out_k
    sp, _ = _stream_ptr(stream)
    _check(_lib.em_psf_fit(ctypes.byref(p), _dev_ptr(f, "f", n * kf * kf),
                           _dev_ptr(h0, "h0", n * kh * kh), _dev_ptr(h, "h", n * kh * kh),
                           _dev_ptr(objective, "objective", n, dtype=torch.float64),
                           sp), "em_psf_fit")


def job_bytes(p: Problem) -> int:
    return int(_lib.em_job_bytes(ctypes.byref(p)))


class Server:
    """Continuous-batching server (em_server_create / em_submit / em_poll / em_wait).

    Inputs are host numpy float32 arrays; they are copied on submit.
    """

    def __init__(self, hbm_budget: int, max_slots: int = 8, stream=None):
        h = ctypes.c_void_p()
        sp = ctypes.c_void_p(stream.cuda_stream) if stream is not None else None
        _check(_lib.em_server_create(ctypes.byref(h), int(hbm_budget), int(max_slots), sp),
               "em_server_create")
        self._h = h
        self._shapes = {}

    def submit(self, p: Problem, y, v, psf, n_iter: int) -> int:
        y = np.ascontiguousarray(y, dtype=np.float32)
        v = np.ascontiguousarray(v, dtype=np.float32)
        psf = np.ascontiguousarray(psf, dtype=np.float32)
        if y.size != p.n_frames * p.frame_h * p.frame_w or v.size != y.size:
            raise ValueError("y / v do not match the problem")
        if psf.size != p.n_frames * p.psf_k ** 2:
            raise ValueError("psf does not match the problem")
        jid = ctypes.c_int64(0)
        _check(_lib.em_submit(self._h, ctypes.byref(p), y.ctypes.data_as(_P),
                              v.ctypes.data_as(_P), psf.ctypes.data_as(_P), int(n_iter),
                              ctypes.byref(jid)), "em_submit")
        self._shapes[jid.value] = p.latent_shape
        return jid.value

    def _result(self, fn, jid):
        shape = self._shapes.get(jid)
        x = np.empty(shape, np.float32) if shape is not None else None
        ll = ctypes.c_double(0.0)
        code = fn(self._h, int(jid), x.ctypes.data_as(_P) if x is not None else None,
                  ctypes.byref(ll))
        return code, x, ll.value

    def poll(self, jid: int):
        """(x, loglik) when done, None while pending; raises on failure."""
        code, x, ll = self._result(_lib.em_poll, jid)
        if code == EAGAIN:
            return None
        _check(code, "em_poll")
        return x, ll

    def wait(self, jid: int):
        code, x, ll = self._result(_lib.em_wait, jid)
        _check(code, "em_wait")
        return x, ll

    def cancel(self, jid: int):
        _check(_lib.em_cancel(self._h, int(jid)), "em_cancel")

    def release(self, jid: int):
        _check(_lib.em_release(self._h, int(jid)), "em_release")
        self._shapes.pop(jid, None)

    def times(self, jid: int):
        a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        _check(_lib.em_job_times(self._h, int(jid), ctypes.byref(a), ctypes.byref(b),
                                 ctypes.byref(c)), "em_job_times")
        return a.value, b.value, c.value

    def stats(self):
        st = np.zeros(8, np.int64)
        _check(_lib.em_server_stats(self._h, st.ctypes.data_as(_P)), "em_server_stats")
        keys = ["queued", "active", "done", "failed", "cancelled", "rounds", "graphs",
                "arena_bytes_in_use"]
        return dict(zip(keys, st.tolist()))

    def phase_seconds(self):
        """Worker seconds per phase: admission, round rebuilds, rounds, finishing."""
        sec = np.zeros(4, np.float64)
        _check(_lib.em_server_phase_seconds(self._h, sec.ctypes.data_as(_P)),
               "em_server_phase_seconds")
        return dict(zip(["admit", "rebuild", "rounds", "finish"], sec.tolist()))

    def staging(self):
        """Pinned host staging: its bytes, jobs staged there, jobs staged in
        pageable memory."""
        out = np.zeros(3, np.int64)
        _check(_lib.em_server_staging(self._h, out.ctypes.data_as(_P)), "em_server_staging")
        return dict(zip(["pinned_bytes", "pinned_jobs", "pageable_jobs"], out.tolist()))

    def close(self):
        if getattr(self, "_h", None):
            _lib.em_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
