"""Python binding of the uvmem C ABI (include/uvmem.h).

Argument marshalling only: every step of the imaging hot path runs in the HIP
kernels of libuvmem.so.  PyTorch supplies device memory and the stream.  If
the HIP library is missing the binding raises; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libuvmem.so")

OK, EINVAL, ENOMEM, EDEVICE, EDOMAIN, ESTATE, ETOOBIG = 0, -1, -2, -3, -4, -5, -6
PRECISIONS = {"fp64": 0, "fp32": 1, "bf16x3": 2, "fp16x3": 3}
MODES = {"cube": 0, "shared": 1}
FORWARD_MODELS = {"dft": 0, "gridded": 1}
GRADIENT_MODELS = {"adjoint": 0, "dft": 1}
NSCAL = 8
S_PHI, S_CHI2, S_S, S_ALPHA, S_BETA, S_GNORM2, S_ALPHA_MAX, S_ITER = range(8)

SYMBOLS = [
    "uvmem_create", "uvmem_destroy", "uvmem_set_uv", "uvmem_set_vis", "uvmem_set_weights",
    "uvmem_set_beam", "uvmem_set_beam_image", "uvmem_set_phase_centre", "uvmem_set_forward_model", "uvmem_set_prior", "uvmem_finalize",
    "uvmem_phi_and_grad", "uvmem_forward", "uvmem_adjoint", "uvmem_get_residual",
    "uvmem_cg_init", "uvmem_cg_step", "uvmem_cg_run", "uvmem_cg_get_state", "uvmem_cg_set_state",
    "uvmem_set_mask", "uvmem_dirty_image", "uvmem_noise", "uvmem_fit_beam",
    "uvmem_check", "uvmem_timing_enable", "uvmem_timing_read", "uvmem_info", "uvmem_chan_range",
    "uvmem_last_error", "uvmem_strerror", "uvmem_forward_noalloc",
]

_lib = None


class UvmemError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"uvmem error {code}: {msg}")
        self.code = code


def load() -> ctypes.CDLL:
    """Load libuvmem.so (built by paper_1703_02920_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"HIP library {LIB_PATH} is not built; run python -m paper_1703_02920_amd.build")
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, dbl, ci = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_int
    sig = {
        "uvmem_create": [ctypes.POINTER(vp), ci, ci, ci, ci, vp],
        "uvmem_destroy": [vp],
        "uvmem_set_uv": [vp, ci, i64, vp, vp, dbl],
        "uvmem_set_vis": [vp, ci, vp],
        "uvmem_set_weights": [vp, ci, vp],
        "uvmem_set_beam": [vp, ci, dbl],
        "uvmem_set_beam_image": [vp, ci, vp],
        "uvmem_set_forward_model": [vp, ci, ci, ci],
        "uvmem_set_phase_centre": [vp, ci, dbl, dbl],
        "uvmem_set_mask": [vp, ci, vp],
        "uvmem_dirty_image": [vp, vp, vp],
        "uvmem_noise": [vp, ctypes.POINTER(dbl)],
        "uvmem_fit_beam": [vp, vp, ctypes.POINTER(dbl), ctypes.POINTER(dbl), ctypes.POINTER(dbl)],
        "uvmem_set_prior": [vp, dbl, dbl],
        "uvmem_finalize": [vp],
        "uvmem_phi_and_grad": [vp, vp, vp, vp],
        "uvmem_forward": [vp, vp, vp],
        "uvmem_adjoint": [vp, vp, vp],
        "uvmem_get_residual": [vp, vp],
        "uvmem_cg_init": [vp, vp, ci],
        "uvmem_cg_step": [vp, vp, vp],
        "uvmem_cg_run": [vp, vp, ci, vp, ci],
        "uvmem_cg_get_state": [vp, vp, ctypes.POINTER(ctypes.c_size_t)],
        "uvmem_cg_set_state": [vp, vp, ctypes.c_size_t],
        "uvmem_check": [vp],
        "uvmem_timing_enable": [vp, ci],
        "uvmem_timing_read": [vp, ci, ctypes.POINTER(dbl), ctypes.POINTER(i64), ci],
        "uvmem_info": [vp, ctypes.POINTER(i64), ci],
        "uvmem_chan_range": [vp, ci, ctypes.POINTER(i64), ctypes.POINTER(i64)],
        "uvmem_forward_noalloc": [ci, dbl, i64, vp, vp, vp, vp, vp, vp],
        "uvmem_last_error": [vp],
        "uvmem_strerror": [ci],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_char_p if name in ("uvmem_last_error", "uvmem_strerror") else ci
    _lib = L
    return L


def _ptr(x) -> Optional[int]:
    if x is None:
        return None
    if isinstance(x, torch.Tensor):
        return x.data_ptr()
    if isinstance(x, np.ndarray):
        return x.ctypes.data
    raise TypeError(type(x))


class Context:
    """One imaging problem: image side n and n_chan channels.  mode "cube"
    gives every channel its own image (n_img = n_chan independent problems);
    mode "shared" fits one image to all channels (n_img = 1, chi^2 summed over
    the channels, each with its own beam)."""

    def __init__(self, n: int, n_chan: int = 1, precision: str = "fp32",
                 device: Optional[torch.device] = None, stream: Optional[torch.cuda.Stream] = None,
                 mode: str = "cube"):
        if mode not in MODES:
            raise ValueError("mode must be one of %s" % sorted(MODES))
        if precision not in PRECISIONS:
            raise ValueError("precision must be one of %s" % sorted(PRECISIONS))
        self._lib = load()
        if not torch.cuda.is_available():
            raise RuntimeError("uvmem needs a GPU")
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        torch.cuda.set_device(self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.n, self.n_chan, self.precision, self.mode = int(n), int(n_chan), precision, mode
        self.n_img = self.n_chan if mode == "cube" else 1
        self.dtype = torch.float64 if precision == "fp64" else torch.float32
        h = ctypes.c_void_p()
        code = self._lib.uvmem_create(ctypes.byref(h), self.n, self.n_chan, MODES[mode], PRECISIONS[precision],
                                      ctypes.c_void_p(self.stream.cuda_stream))
        if code != OK:
            raise UvmemError(code, self._lib.uvmem_strerror(code).decode())
        self._h = h
        self._nvis = [None] * self.n_chan   # visibility count per channel once set_uv succeeded
        self._keep = []

    # ------------------------------------------------------------ plumbing
    def _call(self, name, *args):
        code = getattr(self._lib, name)(self._h, *args)
        if code != OK:
            raise UvmemError(code, self._lib.uvmem_last_error(self._h).decode())
        return code

    def close(self):
        if getattr(self, "_h", None):
            self._lib.uvmem_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # ------------------------------------------------------------ setup
    def _chan(self, chan: int) -> int:
        chan = int(chan)
        if not 0 <= chan < self.n_chan:
            raise ValueError(f"channel {chan} out of range [0, {self.n_chan})")
        return chan

    def _staged(self, chan: int, a: np.ndarray, what: str) -> np.ndarray:
        """Check that a per-visibility array matches the channel's count (the
        C side reads exactly that many elements from the pointer)."""
        if self._nvis[chan] is None:
            return a    # no coordinates yet: the library reports the call order
        if a.ndim != 1 or a.shape[0] != self._nvis[chan]:
            raise ValueError(f"{what} of channel {chan} must be 1-D with {self._nvis[chan]} elements "
                             f"(got shape {a.shape})")
        return a

    def set_uv(self, chan: int, u, v, cell: float):
        chan = self._chan(chan)
        u = np.ascontiguousarray(u, np.float64)
        v = np.ascontiguousarray(v, np.float64)
        if u.ndim != 1 or v.shape != u.shape:
            raise ValueError(f"u and v must be 1-D arrays of the same length (got {u.shape}, {v.shape})")
        self._call("uvmem_set_uv", chan, u.shape[0], _ptr(u), _ptr(v), float(cell))
        self._nvis[chan] = int(u.shape[0])

    def set_vis(self, chan: int, vis):
        chan = self._chan(chan)
        vis = self._staged(chan, np.ascontiguousarray(vis, np.complex64), "visibilities")
        self._call("uvmem_set_vis", chan, _ptr(vis))

    def set_weights(self, chan: int, w):
        chan = self._chan(chan)
        w = self._staged(chan, np.ascontiguousarray(w, np.float32), "weights")
        self._call("uvmem_set_weights", chan, _ptr(w))

    def set_beam(self, chan: int, fwhm: float):
        self._call("uvmem_set_beam", self._chan(chan), float(fwhm))

    def set_beam_image(self, chan: int, A):
        chan = self._chan(chan)
        A = np.ascontiguousarray(A, np.float32)
        if A.shape != (self.n, self.n):
            raise ValueError(f"beam image must be {self.n} x {self.n} (got shape {A.shape})")
        self._call("uvmem_set_beam_image", chan, _ptr(A))

    def set_phase_centre(self, chan: int, x0: float, y0: float):
        """Mosaic pointing: beam centre and phase-tracking centre of the
        channel, radians from the image centre (residuals and model
        visibilities of the channel are then referenced to the image centre)."""
        self._call("uvmem_set_phase_centre", chan, float(x0), float(y0))

    def set_mask(self, img: int, mask):
        """Focus of attention: boolean [n][n] array of the free pixels of
        image plane `img` (None: all free)."""
        if mask is None:
            self._call("uvmem_set_mask", img, None)
            return
        m = np.ascontiguousarray(mask, dtype=np.uint8)
        if m.shape != (self.n, self.n):
            raise ValueError("mask must be n x n")
        self._call("uvmem_set_mask", img, _ptr(m))

    def set_forward_model(self, model: str = "dft", oversample: int = 1, grad: str = "adjoint"):
        """Exact DFT ("dft") or the gridded model of Alg. 1 ("gridded": FFT of
        the image zero-padded to oversample * n, modulation, bilinear
        interpolation); grad "adjoint" (gradient of the model in use) or
        "dft" (the exact-DFT gradient at the gridded residuals)."""
        if model not in FORWARD_MODELS or grad not in GRADIENT_MODELS:
            raise ValueError("model must be one of %s, grad one of %s" % (sorted(FORWARD_MODELS),
                                                                          sorted(GRADIENT_MODELS)))
        self._call("uvmem_set_forward_model", FORWARD_MODELS[model], int(oversample), GRADIENT_MODELS[grad])

    def set_prior(self, M: float, lam: float):
        self._call("uvmem_set_prior", float(M), float(lam))

    def finalize(self):
        self._call("uvmem_finalize")
        info = self.info()
        self.np, self.ztot = info["np"], info["ztot"]
        return self

    @classmethod
    def from_dataset(cls, ds, precision: str = "fp32", mode: Optional[str] = None, forward: str = "dft",
                     oversample: int = 1, grad: str = "adjoint", region=None, **kw) -> "Context":
        """Context for a synthetic data set (paper_1703_02920_amd.synth); the
        mode defaults to "shared" for a mosaic data set, else "cube".
        `region` (boolean n x n) restricts every image plane's free pixels."""
        if mode is None:
            mode = "shared" if getattr(ds, "shared", False) else "cube"
        ctx = cls(ds.n, ds.n_chan, precision, mode=mode, **kw)
        ctx.set_forward_model(forward, oversample, grad)
        for c, ch in enumerate(ds.channels):
            ctx.set_uv(c, ch.u, ch.v, ds.cell)
            ctx.set_vis(c, ch.vis)
            ctx.set_weights(c, ch.w)
            ctx.set_beam(c, ch.fwhm)
            if ch.x0 or ch.y0:
                ctx.set_phase_centre(c, ch.x0, ch.y0)
        if region is not None:
            for m in range(ctx.n_img):
                ctx.set_mask(m, region)
        ctx.set_prior(ds.prior_m, ds.lam)
        return ctx.finalize()

    def info(self) -> dict:
        keys = ["n", "np", "n_chan", "prec", "ztot", "n_fwd_parts", "adj_tile", "n_slots", "n_fwd_wgs",
                "n_adj_items", "n_vis_items", "device_bytes", "n_pix_blocks", "pix_block", "vis_block",
                "n_img", "fwd_model", "grid_side", "grad_model", "n_fwd_wgs_region", "n_adj_wgs_region"]
        out = (ctypes.c_int64 * len(keys))()
        self._call("uvmem_info", out, len(keys))
        return dict(zip(keys, [int(x) for x in out]))

    def chan_range(self, chan: int):
        o, nv = ctypes.c_int64(), ctypes.c_int64()
        self._call("uvmem_chan_range", chan, ctypes.byref(o), ctypes.byref(nv))
        return int(o.value), int(nv.value)

    # ------------------------------------------------------------ tensors
    def image(self, fill: Optional[float] = None) -> torch.Tensor:
        t = torch.empty((self.n_img, self.n, self.n), dtype=self.dtype, device=self.device)
        if fill is not None:
            t.fill_(fill)
        return t

    def _img(self, I: torch.Tensor) -> torch.Tensor:
        if I.dtype != self.dtype or I.device != self.device or not I.is_contiguous():
            raise ValueError("image must be a contiguous %s tensor on %s" % (self.dtype, self.device))
        if I.numel() != self.n_img * self.n * self.n:
            raise ValueError("image must have n_img * n * n elements")
        return I

    def scalars(self) -> torch.Tensor:
        return torch.zeros((self.n_img, NSCAL), dtype=torch.float64, device=self.device)

    # ------------------------------------------------------------ hot path
    def phi_and_grad(self, I: torch.Tensor, grad: Optional[torch.Tensor] = None,
                     scal: Optional[torch.Tensor] = None):
        I = self._img(I)
        grad = torch.empty_like(I) if grad is None else self._img(grad)
        scal = self.scalars() if scal is None else scal
        self._call("uvmem_phi_and_grad", _ptr(I), _ptr(grad), _ptr(scal))
        return scal, grad

    def forward(self, I: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        I = self._img(I)
        if out is None:
            out = torch.empty(max(self.ztot, 1), dtype=torch.complex128, device=self.device)[: self.ztot]
        self._call("uvmem_forward", _ptr(I), _ptr(out))
        return out

    def adjoint(self, coef: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        if coef.dtype != torch.complex128 or not coef.is_contiguous() or coef.numel() != self.ztot:
            raise ValueError("coefficients must be a contiguous complex128 tensor of sum Z elements")
        out = self.image() if out is None else self._img(out)
        self._call("uvmem_adjoint", _ptr(coef) if self.ztot else None, _ptr(out))
        return out

    def residual(self) -> torch.Tensor:
        out = torch.empty(max(self.ztot, 1), dtype=torch.complex128, device=self.device)[: self.ztot]
        self._call("uvmem_get_residual", _ptr(out) if self.ztot else None)
        return out

    def dirty_image(self, dirty: bool = True, psf: bool = True):
        """Natural-weight dirty image and PSF (n_img planes each; None for the
        ones not asked for)."""
        d = self.image() if dirty else None
        p = self.image() if psf else None
        self._call("uvmem_dirty_image", _ptr(d) if d is not None else None, _ptr(p) if p is not None else None)
        return d, p

    def noise(self) -> np.ndarray:
        """sigma_D = 1 / sqrt(sum w) per image plane."""
        out = (ctypes.c_double * self.n_img)()
        code = self._lib.uvmem_noise(self._h, out)
        if code != OK:
            raise UvmemError(code, self._lib.uvmem_strerror(code).decode())
        return np.array(out[:])

    def fit_beam(self, psf: torch.Tensor):
        """(bmaj, bmin, bpa) per image plane: FWHM in radians, angle of the
        major axis from +y towards +x in degrees."""
        psf = self._img(psf)
        a, b, p = ((ctypes.c_double * self.n_img)() for _ in range(3))
        self._call("uvmem_fit_beam", _ptr(psf), a, b, p)
        return np.array(a[:]), np.array(b[:]), np.array(p[:])

    def cg_init(self, I: torch.Tensor, init_to_floor: bool = True):
        self._cg_I = self._img(I)
        self._call("uvmem_cg_init", _ptr(I), 1 if init_to_floor else 0)

    def cg_step(self, I: torch.Tensor, scal: Optional[torch.Tensor] = None) -> torch.Tensor:
        scal = self.scalars() if scal is None else scal
        self._call("uvmem_cg_step", _ptr(self._img(I)), _ptr(scal))
        return scal

    def cg_run(self, I: torch.Tensor, iters: int, graph: bool = True,
               hist: Optional[torch.Tensor] = None) -> torch.Tensor:
        if hist is None:
            hist = torch.zeros((max(iters, 1), self.n_img, NSCAL), dtype=torch.float64, device=self.device)
        self._call("uvmem_cg_run", _ptr(self._img(I)), int(iters), _ptr(hist), 1 if graph else 0)
        return hist[:iters]

    def get_state(self) -> bytes:
        n = ctypes.c_size_t(0)
        self._call("uvmem_cg_get_state", None, ctypes.byref(n))
        buf = ctypes.create_string_buffer(n.value)
        self._call("uvmem_cg_get_state", buf, ctypes.byref(n))
        return buf.raw[: n.value]

    def set_state(self, blob: bytes):
        buf = ctypes.create_string_buffer(blob, len(blob))
        self._call("uvmem_cg_set_state", buf, len(blob))

    def check(self):
        self._call("uvmem_check")

    # ------------------------------------------------------------ timing
    def timing(self, enable: bool = True):
        self._call("uvmem_timing_enable", 1 if enable else 0)

    def timing_read(self, which: int, reset: bool = False):
        ms, cnt = ctypes.c_double(), ctypes.c_int64()
        self._call("uvmem_timing_read", int(which), ctypes.byref(ms), ctypes.byref(cnt), 1 if reset else 0)
        return float(ms.value), int(cnt.value)


def forward_noalloc(n: int, cell: float, u: torch.Tensor, v: torch.Tensor, I: torch.Tensor,
                    beam: Optional[torch.Tensor] = None, out: Optional[torch.Tensor] = None,
                    stream: Optional[torch.cuda.Stream] = None) -> torch.Tensor:
    """uvmem_forward_noalloc: model visibilities of the FP32 image I (n x n)
    through the beam image `beam` (None: A = 1), without a context and
    without allocating on the library side; u, v are float64 device tensors
    in wavelengths.  Returns `out` (complex128, len(u); allocated here by
    torch when not given)."""
    L = load()
    nvis = int(u.numel())
    for name, t, dt in (("u", u, torch.float64), ("v", v, torch.float64), ("I", I, torch.float32)):
        if t.dtype != dt or not t.is_cuda or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous {dt} device tensor")
    if v.numel() != nvis or I.numel() != n * n:
        raise ValueError("v must match u; I must have n * n elements")
    if beam is not None and (beam.dtype != torch.float32 or not beam.is_cuda or not beam.is_contiguous()
                             or beam.numel() != n * n):
        raise ValueError("beam must be a contiguous float32 n x n device tensor")
    if out is None:
        out = torch.empty(max(nvis, 1), dtype=torch.complex128, device=I.device)[:nvis]
    elif out.dtype != torch.complex128 or out.numel() != nvis or not out.is_contiguous():
        raise ValueError("out must be a contiguous complex128 tensor of len(u) elements")
    st = stream if stream is not None else torch.cuda.current_stream(I.device)
    code = L.uvmem_forward_noalloc(int(n), float(cell), nvis, _ptr(u), _ptr(v),
                                   _ptr(beam) if beam is not None else None, _ptr(I),
                                   _ptr(out) if nvis else None, ctypes.c_void_p(st.cuda_stream))
    if code != OK:
        raise UvmemError(code, L.uvmem_strerror(code).decode())
    return out


class PhiFunction(torch.autograd.Function):
    """Phi(I) summed over the images as a differentiable torch function; the
    backward pass returns g * grad Phi computed by the same HIP evaluation."""

    @staticmethod
    def forward(ctx, I: torch.Tensor, uctx: Context):
        scal, grad = uctx.phi_and_grad(I.detach().contiguous())
        ctx.save_for_backward(grad)
        return scal[:, S_PHI].sum()

    @staticmethod
    def backward(ctx, gout):
        (grad,) = ctx.saved_tensors
        return gout.to(grad.dtype) * grad, None
