"""ctypes binding of libofista.so (argument marshalling only).

Every computation happens in the HIP library; PyTorch provides the device
workspace, the data tensors and the current stream.  The names follow the
C ABI in include/ofista.h.  There is no fallback: without the built library
(or without a GPU) construction raises.
"""

from __future__ import annotations

import ctypes
from pathlib import Path

import numpy as np
import torch

_LIB_PATH = Path(__file__).resolve().with_name("libofista.so")
_lib = None

DICT = {"identity": 0, "haar": 1, "edgelet": 2}
PRECISION = {"fp32": 0, "split_bf16": 1}
LIPSCHITZ = {"running": 0, "bound": 1}
MOMENTUM = {"fista": 0, "restart": 1, "ista": 2}
KERNEL = {"gram": 0, "step": 1, "rows": 2, "corr": 3, "scalars": 4, "update": 5,
          "store_forward": 6, "store_adjoint": 7, "resident": 8}
STORAGE = {"gram": 0, "pulses": 1}
GRAM_LAYOUT = {"auto": 0, "tile": 1, "block": 2}
STEP_KERNEL = {"auto": 0, "launches": 1, "resident": 2}

STATUS = {0: "OK", -1: "E_ARG", -2: "E_RANGE", -3: "E_STATE", -4: "E_WORKSPACE",
          -5: "E_UNSUPPORTED", -6: "E_HIP"}


class OfistaError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


class OfistaConfig(ctypes.Structure):
    _fields_ = [
        ("n_x", ctypes.c_int32), ("n_y", ctypes.c_int32),
        ("x0", ctypes.c_double), ("y0", ctypes.c_double),
        ("dx", ctypes.c_double), ("dy", ctypes.c_double),
        ("n_pos", ctypes.c_int32), ("pos_xyz", ctypes.POINTER(ctypes.c_double)),
        ("n_freq", ctypes.c_int32), ("freq0_hz", ctypes.c_double),
        ("dfreq_hz", ctypes.c_double),
        ("dict", ctypes.c_int32), ("haar_levels", ctypes.c_int32),
        ("lambda_", ctypes.c_double), ("lambda_relative", ctypes.c_int32),
        ("precision", ctypes.c_int32), ("lipschitz", ctypes.c_int32),
        ("momentum", ctypes.c_int32), ("record_every", ctypes.c_int32),
        ("max_pulses", ctypes.c_int32), ("max_iters", ctypes.c_int32),
        ("n_edge_lengths", ctypes.c_int32), ("edge_lengths", ctypes.POINTER(ctypes.c_int32)),
        ("n_edge_rotations", ctypes.c_int32),
        ("edge_rotations_deg", ctypes.POINTER(ctypes.c_double)),
        ("backprojection", ctypes.c_int32), ("storage", ctypes.c_int32),
        ("gram_layout", ctypes.c_int32), ("validate_input", ctypes.c_int32),
        ("step_kernel", ctypes.c_int32),
    ]


class OfistaStats(ctypes.Structure):
    _fields_ = [("n_pulses", ctypes.c_int64), ("n_iters", ctypes.c_int64),
                ("t", ctypes.c_double), ("L", ctypes.c_double),
                ("tau", ctypes.c_double), ("lambda_", ctypes.c_double),
                ("rho", ctypes.c_double), ("sigma2", ctypes.c_double)]


def lib() -> ctypes.CDLL:
    """Load libofista.so (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not _LIB_PATH.exists():
        raise RuntimeError(f"{_LIB_PATH} is missing: build it with "
                           "`python -m paper_2603_08582_amd.build`")
    L = ctypes.CDLL(str(_LIB_PATH))
    vp, i32, f64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double, ctypes.c_size_t
    cfgp = ctypes.POINTER(OfistaConfig)
    sig = {
        "ofista_workspace_bytes": (sz, [cfgp]),
        "ofista_state_bytes": (sz, [cfgp]),
        "ofista_check_config": (i32, [cfgp]),
        "ofista_coef_count": (ctypes.c_int64, [cfgp]),
        "ofista_create": (i32, [cfgp, vp, sz, vp, ctypes.POINTER(vp)]),
        "ofista_reset": (i32, [vp]),
        "ofista_push_pulse": (i32, [vp, vp, i32, f64]),
        "ofista_reconstruct": (i32, [vp, i32, vp]),
        "ofista_reconstruct_static": (i32, [vp, i32, vp]),
        "ofista_image": (i32, [vp, vp]),
        "ofista_state": (i32, [vp, ctypes.POINTER(OfistaStats)]),
        "ofista_bp_image": (i32, [vp, vp]),
        "ofista_count_large": (i32, [vp, f64, ctypes.POINTER(ctypes.c_int64)]),
        "ofista_echo": (i32, [vp, i32, vp, vp, f64, f64, vp]),
        "ofista_rows": (i32, [vp, i32, vp]),
        "ofista_gram": (i32, [vp, vp]),
        "ofista_gram_entries": (i32, [vp, i32, vp, vp, vp]),
        "ofista_vector": (i32, [vp, i32, vp]),
        "ofista_export_state": (i32, [vp, vp]),
        "ofista_import_state": (i32, [vp, vp]),
        "ofista_profile": (i32, [vp, i32]),
        "ofista_kernel_time": (i32, [vp, i32, ctypes.POINTER(f64), ctypes.POINTER(ctypes.c_int64)]),
        "ofista_backward": (i32, [vp, vp, ctypes.POINTER(f64), ctypes.POINTER(f64)]),
        "ofista_set_lambda": (i32, [vp, f64]),
        "ofista_destroy": (None, [vp]),
        "ofista_error_string": (ctypes.c_char_p, [vp, i32]),
        "ofista_tile": (i32, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def make_config(*, n_x, n_y, x0, y0, dx, dy, positions, freq0, dfreq, n_freq,
                dictionary="identity", haar_levels=0, lam=0.05, lam_relative=True,
                precision="fp32", lipschitz="running", momentum="fista",
                record_every=0, max_pulses=0, max_iters=0, edge_lengths=(), edge_rotations=(),
                backprojection=False, storage="gram", gram_layout="auto",
                validate_input=False, step_kernel="auto"):
    """Build an OfistaConfig; returns (config, keepalive) -- keep the second
    value alive while the config is in use (it owns the host tables)."""
    pos = np.ascontiguousarray(np.asarray(positions, dtype=np.float64).reshape(-1, 3))
    lens = np.ascontiguousarray(np.asarray(edge_lengths, dtype=np.int32).reshape(-1))
    rots = np.ascontiguousarray(np.asarray(edge_rotations, dtype=np.float64).reshape(-1))
    cfg = OfistaConfig(
        n_x=n_x, n_y=n_y, x0=x0, y0=y0, dx=dx, dy=dy, n_pos=pos.shape[0],
        pos_xyz=pos.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
        n_freq=n_freq, freq0_hz=freq0, dfreq_hz=dfreq,
        dict=DICT[dictionary], haar_levels=haar_levels, lambda_=lam,
        lambda_relative=1 if lam_relative else 0, precision=PRECISION[precision],
        lipschitz=LIPSCHITZ[lipschitz], momentum=MOMENTUM[momentum],
        record_every=record_every, max_pulses=max_pulses, max_iters=max_iters,
        n_edge_lengths=lens.size, edge_lengths=lens.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
        n_edge_rotations=rots.size,
        edge_rotations_deg=rots.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
        backprojection=1 if backprojection else 0, storage=STORAGE[storage],
        gram_layout=GRAM_LAYOUT[gram_layout], validate_input=1 if validate_input else 0,
        step_kernel=STEP_KERNEL[step_kernel])
    return cfg, (pos, lens, rots)


def workspace_bytes(cfg: OfistaConfig) -> int:
    return int(lib().ofista_workspace_bytes(ctypes.byref(cfg)))


def check_config(cfg: OfistaConfig) -> int:
    return int(lib().ofista_check_config(ctypes.byref(cfg)))


def coef_count(cfg: OfistaConfig) -> int:
    """M, the number of coefficients (dictionary atoms); -1 if cfg is invalid."""
    return int(lib().ofista_coef_count(ctypes.byref(cfg)))


def _ptr(t: torch.Tensor) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


class OnlineFista:
    """One Online FISTA image on one GPU (see include/ofista.h for semantics)."""

    def __init__(self, device="cuda", stream=None, **cfg_kwargs):
        if not torch.cuda.is_available():
            raise RuntimeError("OnlineFista needs a ROCm GPU; no CPU fallback exists")
        self._lib = lib()
        self.device = torch.device(device)
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.cfg, self._tables = make_config(**cfg_kwargs)
        self.N = self.cfg.n_x * self.cfg.n_y   # pixels
        self.M = coef_count(self.cfg)          # coefficients
        self.K = self.cfg.n_freq
        self.n_pos = self.cfg.n_pos
        nbytes = workspace_bytes(self.cfg)
        if nbytes == 0:
            raise OfistaError(check_config(self.cfg), "invalid configuration")
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
            self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            ctx = ctypes.c_void_p()
            st = self._lib.ofista_create(ctypes.byref(self.cfg), _ptr(self.workspace), nbytes,
                                         ctypes.c_void_p(self.stream.cuda_stream),
                                         ctypes.byref(ctx))
        self._ctx = ctx
        if st != 0:
            msg = self._lib.ofista_error_string(ctx, st).decode()
            if ctx:
                self._lib.ofista_destroy(ctx)
            self._ctx = None
            raise OfistaError(st, msg)

    # -- helpers -----------------------------------------------------------
    def _check(self, st: int):
        if st != 0:
            raise OfistaError(st, self._lib.ofista_error_string(self._ctx, st).decode())

    def _vec(self, t: torch.Tensor, n: int, name: str) -> torch.Tensor:
        if not isinstance(t, torch.Tensor) or t.dtype != torch.complex64:
            raise TypeError(f"{name} must be a complex64 tensor")
        if t.device != self.device:
            raise ValueError(f"{name} must live on {self.device}")
        if t.numel() != n or not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous with {n} elements")
        return t

    def _out(self, out, n, name="out"):
        if out is None:
            return torch.empty(n, dtype=torch.complex64, device=self.device)
        return self._vec(out, n, name)

    # -- the ABI ------------------------------------------------------------
    def reset(self):
        self._check(self._lib.ofista_reset(self._ctx))

    def push_pulse(self, d: torch.Tensor, s: int, phase_corr: float = 0.0):
        self._vec(d, self.K, "d")
        self._check(self._lib.ofista_push_pulse(self._ctx, _ptr(d), int(s), float(phase_corr)))

    def reconstruct(self, iters: int, out: torch.Tensor | None = None, copy: bool = True):
        o = self._out(out, self.M) if copy else None
        self._check(self._lib.ofista_reconstruct(self._ctx, int(iters),
                                                 _ptr(o) if o is not None else None))
        return o

    def reconstruct_static(self, iters: int, out: torch.Tensor | None = None,
                           copy: bool = True):
        """reconstruct() with the matvec partials in the library's per-GPU static
        array (the allocation-free entry point)."""
        o = self._out(out, self.M) if copy else None
        self._check(self._lib.ofista_reconstruct_static(self._ctx, int(iters),
                                                        _ptr(o) if o is not None else None))
        return o

    def image(self, out=None):
        o = self._out(out, self.N)
        self._check(self._lib.ofista_image(self._ctx, _ptr(o)))
        return o

    def bp_image(self, out=None):
        """BP baseline: (1/n) sum of F_s^H d_s over the pushed pulses (pixels)."""
        o = self._out(out, self.N)
        self._check(self._lib.ofista_bp_image(self._ctx, _ptr(o)))
        return o

    def count_large(self, threshold: float = 2e-2) -> int:
        """Number of coefficients with |c| > threshold (synchronises)."""
        n = ctypes.c_int64()
        self._check(self._lib.ofista_count_large(self._ctx, float(threshold), ctypes.byref(n)))
        return int(n.value)

    def state(self) -> dict:
        s = OfistaStats()
        self._check(self._lib.ofista_state(self._ctx, ctypes.byref(s)))
        return dict(n_pulses=s.n_pulses, n_iters=s.n_iters, t=s.t, L=s.L, tau=s.tau,
                    lam=s.lambda_, rho=s.rho, sigma2=s.sigma2)

    def echo(self, s: int, rho: torch.Tensor, noise: torch.Tensor | None, snr_db: float,
             phase_err: float = 0.0, out=None):
        self._vec(rho, self.N, "rho")
        if noise is not None:
            self._vec(noise, self.K, "noise")
        o = self._out(out, self.K)
        self._check(self._lib.ofista_echo(self._ctx, int(s), _ptr(rho),
                                          _ptr(noise) if noise is not None else None,
                                          float(snr_db), float(phase_err), _ptr(o)))
        return o

    def rows(self, s: int):
        o = torch.empty((self.K, self.M), dtype=torch.complex64, device=self.device)
        self._check(self._lib.ofista_rows(self._ctx, int(s), _ptr(o)))
        return o

    def gram(self):
        o = torch.empty((self.M, self.M), dtype=torch.complex64, device=self.device)
        self._check(self._lib.ofista_gram(self._ctx, _ptr(o)))
        return o

    def gram_entries(self, i, j):
        """H_n[i[t], j[t]] for coefficient index sequences i, j (any M)."""
        ii = torch.as_tensor(np.asarray(i), dtype=torch.int32).to(self.device).contiguous()
        jj = torch.as_tensor(np.asarray(j), dtype=torch.int32).to(self.device).contiguous()
        if ii.shape != jj.shape or ii.dim() != 1:
            raise ValueError("i and j must be 1-D of equal length")
        o = torch.empty(ii.numel(), dtype=torch.complex64, device=self.device)
        self._check(self._lib.ofista_gram_entries(self._ctx, ii.numel(), _ptr(ii), _ptr(jj), _ptr(o)))
        return o

    def vector(self, which: str):
        o = torch.empty(self.M, dtype=torch.complex64, device=self.device)
        idx = {"b": 0, "c": 1, "w": 2}[which]
        self._check(self._lib.ofista_vector(self._ctx, idx, _ptr(o)))
        return o

    def state_bytes(self) -> int:
        return int(self._lib.ofista_state_bytes(ctypes.byref(self.cfg)))

    def export_state(self):
        # zero-filled: the record's alignment padding is not written by the library
        buf = torch.zeros(self.state_bytes(), dtype=torch.uint8, device=self.device)
        self._check(self._lib.ofista_export_state(self._ctx, _ptr(buf)))
        return buf

    def import_state(self, buf: torch.Tensor):
        if buf.dtype != torch.uint8 or buf.numel() < self.state_bytes() or buf.device != self.device:
            raise ValueError("state buffer has the wrong type, size or device")
        self._check(self._lib.ofista_import_state(self._ctx, _ptr(buf)))

    def set_lambda(self, lam: float):
        self._check(self._lib.ofista_set_lambda(self._ctx, float(lam)))

    def backward(self, grad_img: torch.Tensor):
        """(dL/dlambda, dL/dphase per pushed pulse) for dL/dx = grad_img."""
        self._vec(grad_img, self.N, "grad_img")
        n = self.state()["n_pulses"]
        gl = ctypes.c_double()
        gp = (ctypes.c_double * max(n, 1))()
        self._check(self._lib.ofista_backward(self._ctx, _ptr(grad_img), ctypes.byref(gl), gp))
        return gl.value, np.array(gp[:n], dtype=np.float64)

    def profile(self, enable: bool):
        self._check(self._lib.ofista_profile(self._ctx, 1 if enable else 0))

    def kernel_time(self, kernel: str):
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        self._check(self._lib.ofista_kernel_time(self._ctx, KERNEL[kernel], ctypes.byref(ms),
                                                 ctypes.byref(n)))
        return ms.value, n.value

    def close(self):
        if getattr(self, "_ctx", None):
            self._lib.ofista_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class OnlineFistaFn(torch.autograd.Function):
    """x = OnlineFistaFn.apply(lam, phases, model, D, iters): the final image of
    an online run over the pulses D[n] (positions 0..P-1) with the absolute l1
    weight lam and per-pulse phase corrections phases[n]; differentiable in lam
    and phases through the library's reverse pass.  `model` must be an
    OnlineFista created with record_every > 0."""

    @staticmethod
    def forward(ctx, lam, phases, model, D, iters):
        model.reset()
        model.set_lambda(float(lam))
        ph = phases.detach().cpu().double().numpy()
        for n in range(D.shape[0]):
            model.push_pulse(D[n], n, float(ph[n]))
            model.reconstruct(int(iters), copy=False)
        ctx.model = model
        ctx.lam_dtype, ctx.ph_dtype = lam.dtype, phases.dtype
        ctx.devices = (lam.device, phases.device)
        return model.image()

    @staticmethod
    def backward(ctx, grad_x):
        gl, gp = ctx.model.backward(grad_x.contiguous().to(torch.complex64))
        glam = torch.tensor(gl, dtype=ctx.lam_dtype, device=ctx.devices[0])
        gph = torch.from_numpy(gp).to(dtype=ctx.ph_dtype, device=ctx.devices[1])
        return glam, gph, None, None, None
