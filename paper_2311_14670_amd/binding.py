"""Thin ctypes binding over the C ABI of include/s2mi.h.

Argument marshalling only: tensors are checked (dtype, device, shape,
contiguity) and their device pointers handed to the native library together
with torch's current HIP stream.  Every step of every transform runs in the
library's own kernels; if the library is missing, loading it raises.
"""
import ctypes
import os
import threading

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBNAME = "libs2mi.so"

MW, HEALPIX, DH, GL, MWSS = 0, 1, 2, 3, 4
FP64, CONTRACT_FP32, CONTRACT_SPLIT_BF16 = 0, 1, 2
_SAMPLING = {"mw": MW, "healpix": HEALPIX, "dh": DH, "gl": GL, "mwss": MWSS,
             MW: MW, HEALPIX: HEALPIX, DH: DH, GL: GL, MWSS: MWSS}
_SAMPLING_NAME = {MW: "mw", HEALPIX: "healpix", DH: "dh", GL: "gl", MWSS: "mwss"}
_PRECISION = {"fp64": FP64, "fp32": CONTRACT_FP32, "split_bf16": CONTRACT_SPLIT_BF16,
              FP64: FP64, CONTRACT_FP32: CONTRACT_FP32, CONTRACT_SPLIT_BF16: CONTRACT_SPLIT_BF16}

S2_OK = 0


class S2Error(RuntimeError):
    def __init__(self, code, message):
        super().__init__(f"s2mi error {code}: {message}")
        self.code = code


STAGES = ["pack", "dstage_inv", "phi_inv", "phi_fwd", "mw_theta", "dstage_fwd", "finish", "gamma", "dgen", "mfma"]


class _Timing(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * len(STAGES)), ("launches", ctypes.c_longlong * len(STAGES))]


class _PlanInfo(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int), ("spin", ctypes.c_int), ("N", ctypes.c_int), ("nside", ctypes.c_int),
                ("sampling", ctypes.c_int), ("precision", ctypes.c_int), ("max_batch", ctypes.c_int),
                ("nrings", ctypes.c_int), ("nsamples", ctypes.c_longlong), ("ncoeffs", ctypes.c_longlong),
                ("workspace_bytes", ctypes.c_size_t), ("plan_device_bytes", ctypes.c_size_t),
                ("swept_rings", ctypes.c_int),
                ("order_tiles", ctypes.c_int)]


_lib = None
_lib_lock = threading.Lock()


def library_path():
    return os.path.join(_HERE, _LIBNAME)


def load_library():
    """Load libs2mi.so (built in-tree by paper_2311_14670_amd.build); raise if absent."""
    global _lib
    with _lib_lock:
        if _lib is not None:
            return _lib
        path = library_path()
        if not os.path.exists(path):
            raise S2Error(-4, f"native library {path} not found: build it with "
                              "`python -m paper_2311_14670_amd.build` (there is no fallback path)")
        lib = ctypes.CDLL(path)
        vp, i, P = ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p
        lib.s2_plan_create.argtypes = [ctypes.POINTER(P), i, i, i, i, i, i, i, vp]
        lib.s2_plan_destroy.argtypes = [P]
        lib.s2_plan_info.argtypes = [P, ctypes.POINTER(_PlanInfo)]
        for name in ["s2_inverse", "s2_forward", "s2_inverse_adjoint", "s2_forward_adjoint", "so3_inverse",
                     "so3_forward", "so3_inverse_adjoint", "so3_forward_adjoint", "s2_inverse_real",
                     "s2_forward_real", "s2_inverse_real_adjoint", "s2_forward_real_adjoint"]:
            getattr(lib, name).argtypes = [P, vp, vp, i, vp, vp]
            getattr(lib, name).restype = i
        lib.s2_inverse_noalloc.argtypes = [P, vp, vp, i, vp]
        lib.s2_inverse_noalloc.restype = i
        lib.s2_debug_wigner_d.argtypes = [P, i, vp, vp]
        lib.s2_plan_set_timing.argtypes = [P, i]
        lib.s2_plan_read_timing.argtypes = [P, ctypes.POINTER(_Timing)]
        lib.s2_error_string.restype = ctypes.c_char_p
        lib.s2_error_string.argtypes = [i]
        lib.s2_last_error_message.restype = ctypes.c_char_p
        lib.s2_last_error_message.argtypes = []
        _lib = lib
        return lib


def _check(rc):
    if rc != S2_OK:
        lib = load_library()
        raise S2Error(rc, lib.s2_last_error_message().decode())


def _stream_handle(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Plan:
    """A transform plan: bandlimit L, spin, azimuthal band N (SO(3) when N > 1),
    sampling 'mw', 'healpix' (nside), 'dh', 'gl' or 'mwss', max_batch, contraction precision.

    Holds its device constants (freed with the plan) and one workspace tensor;
    calls on one Plan object are therefore serialised on the stream they are
    issued on (use one Plan per concurrent stream)."""

    def __init__(self, L, spin=0, N=1, sampling="mw", nside=0, max_batch=1, precision="fp64", device=None):
        self._lib = load_library()
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        self._handle = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(self._lib.s2_plan_create(ctypes.byref(self._handle), int(L), int(spin), int(N),
                                            _SAMPLING[sampling], int(nside), int(max_batch),
                                            _PRECISION[precision], _stream_handle(self.device)))
        info = _PlanInfo()
        _check(self._lib.s2_plan_info(self._handle, ctypes.byref(info)))
        self.info = {f: getattr(info, f) for f, _ in _PlanInfo._fields_}
        self.L, self.spin, self.N = info.L, info.spin, info.N
        self.sampling = _SAMPLING_NAME[info.sampling]
        self.nside, self.max_batch = info.nside, info.max_batch
        self.nsamples = info.nsamples
        self._ws = None

    def close(self):
        if getattr(self, "_handle", None) and self._handle.value:
            self._lib.s2_plan_destroy(self._handle)
            self._handle = ctypes.c_void_p()
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------ helpers
    @property
    def workspace(self):
        if self._ws is None:
            n = max(int(self.info["workspace_bytes"]), 256)
            self._ws = torch.empty(n, dtype=torch.uint8, device=self.device)
        return self._ws

    @property
    def coeff_shape(self):
        return (self.L, 2 * self.L - 1)

    @property
    def map_shape(self):
        if self.sampling == "healpix":
            return (self.nsamples,)
        return (self.info["nrings"], 2 * self.L if self.sampling == "mwss" else 2 * self.L - 1)

    def _prep(self, x, tail, what, dtype=torch.complex128):
        if not isinstance(x, torch.Tensor):
            raise TypeError(f"{what}: expected a torch.Tensor")
        if x.dtype != dtype:
            raise TypeError(f"{what}: expected {dtype}, got {x.dtype}")
        if x.device != self.device:
            raise ValueError(f"{what}: tensor on {x.device}, plan on {self.device}")
        batched = x.dim() == len(tail) + 1
        if tuple(x.shape[-len(tail):]) != tuple(tail) or x.dim() not in (len(tail), len(tail) + 1):
            raise ValueError(f"{what}: shape {tuple(x.shape)} does not end in {tuple(tail)}")
        return x.contiguous(), (x.shape[0] if batched else 1), batched

    def new_workspace(self):
        """A fresh workspace tensor for calls issued concurrently on another stream."""
        return torch.empty(max(int(self.info["workspace_bytes"]), 256), dtype=torch.uint8, device=self.device)

    def _call(self, fn, x, in_tail, out_tail, what, workspace=None, out=None, in_dtype=torch.complex128,
              out_dtype=torch.complex128):
        x, B, batched = self._prep(x, in_tail, what, in_dtype)
        shape = ((B,) if batched else ()) + tuple(out_tail)
        if out is None:
            out = torch.empty(shape, dtype=out_dtype, device=self.device)
        elif (out.dtype != out_dtype or out.device != self.device or tuple(out.shape) != shape
              or not out.is_contiguous()):
            raise ValueError(f"{what}: out must be a contiguous {out_dtype} tensor of shape {shape} on {self.device}")
        ws = self.workspace if workspace is None else workspace
        if ws.device != self.device or ws.numel() * ws.element_size() < self.info["workspace_bytes"]:
            raise ValueError(f"{what}: workspace too small or on the wrong device")
        with torch.cuda.device(self.device):
            _check(fn(self._handle, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()), int(B),
                      ctypes.c_void_p(ws.data_ptr()), _stream_handle(self.device)))
        return out

    # ------------------------------------------------------------ transforms
    def inverse(self, flm, workspace=None, out=None):
        """Inverse spin SHT: flm [B?, L, 2L-1] -> map."""
        return self._call(self._lib.s2_inverse, flm, self.coeff_shape, self.map_shape, "inverse", workspace, out)

    def inverse_noalloc(self, flm, out=None):
        """Inverse spin SHT through s2_inverse_noalloc: no workspace, the library's
        fixed per-device scratch instead (FP64 plans whose inverse fits it)."""
        x, B, batched = self._prep(flm, self.coeff_shape, "inverse_noalloc")
        shape = ((B,) if batched else ()) + tuple(self.map_shape)
        if out is None:
            out = torch.empty(shape, dtype=torch.complex128, device=self.device)
        elif (out.dtype != torch.complex128 or out.device != self.device or tuple(out.shape) != shape
              or not out.is_contiguous()):
            raise ValueError(f"inverse_noalloc: out must be a contiguous complex128 tensor of shape {shape}")
        with torch.cuda.device(self.device):
            _check(self._lib.s2_inverse_noalloc(self._handle, ctypes.c_void_p(x.data_ptr()),
                                                ctypes.c_void_p(out.data_ptr()), int(B),
                                                _stream_handle(self.device)))
        return out

    def forward(self, f, workspace=None, out=None):
        """Forward spin SHT: map -> flm [B?, L, 2L-1]."""
        return self._call(self._lib.s2_forward, f, self.map_shape, self.coeff_shape, "forward", workspace, out)

    def inverse_real(self, flm, workspace=None, out=None):
        """Inverse SHT of a real signal (spin-0 FP64 plans): flm [B?, L, 2L-1]
        complex128, of which only the orders m >= 0 are read -> real map float64."""
        return self._call(self._lib.s2_inverse_real, flm, self.coeff_shape, self.map_shape, "inverse_real", workspace,
                          out, out_dtype=torch.float64)

    def forward_real(self, f, workspace=None, out=None):
        """Forward SHT of a real map float64 (spin-0 FP64 plans) -> flm
        [B?, L, 2L-1] complex128 with flm[l][-m] = (-1)^m conj(flm[l][m])."""
        return self._call(self._lib.s2_forward_real, f, self.map_shape, self.coeff_shape, "forward_real", workspace,
                          out, in_dtype=torch.float64)

    def inverse_real_adjoint(self, g, workspace=None, out=None):
        """Gradient of inverse_real with respect to its complex input for a real map
        cotangent g float64: 2 A^H g at m > 0, Re (A^H g) at m = 0, 0 at m < 0."""
        return self._call(self._lib.s2_inverse_real_adjoint, g, self.map_shape, self.coeff_shape,
                          "inverse_real_adjoint", workspace, out, in_dtype=torch.float64)

    def forward_real_adjoint(self, g_flm, workspace=None, out=None):
        """Gradient of forward_real with respect to its real map: Re(F^H g_flm), float64."""
        return self._call(self._lib.s2_forward_real_adjoint, g_flm, self.coeff_shape, self.map_shape,
                          "forward_real_adjoint", workspace, out, out_dtype=torch.float64)

    def inverse_adjoint(self, g, workspace=None, out=None):
        """Hermitian adjoint of the inverse SHT: map-space cotangent -> coefficients."""
        return self._call(self._lib.s2_inverse_adjoint, g, self.map_shape, self.coeff_shape, "inverse_adjoint", workspace, out)

    def forward_adjoint(self, g_flm, workspace=None, out=None):
        """Hermitian adjoint of the forward SHT: coefficient-space cotangent -> map (FP64 plans)."""
        return self._call(self._lib.s2_forward_adjoint, g_flm, self.coeff_shape, self.map_shape, "forward_adjoint",
                          workspace, out)

    def so3_inverse(self, flmn, workspace=None, out=None):
        """Inverse Wigner transform: flmn [B?, 2N-1, L, 2L-1] -> f [B?, 2N-1, L, 2L-1]."""
        shp = (2 * self.N - 1,) + self.coeff_shape
        return self._call(self._lib.so3_inverse, flmn, shp, shp, "so3_inverse", workspace, out)

    def so3_forward(self, f, workspace=None, out=None):
        """Forward Wigner transform: f [B?, 2N-1, L, 2L-1] -> flmn."""
        shp = (2 * self.N - 1,) + self.coeff_shape
        return self._call(self._lib.so3_forward, f, shp, shp, "so3_forward", workspace, out)

    def so3_inverse_adjoint(self, g, workspace=None, out=None):
        """Hermitian adjoint of the inverse Wigner transform: f-space cotangent -> flmn-space."""
        shp = (2 * self.N - 1,) + self.coeff_shape
        return self._call(self._lib.so3_inverse_adjoint, g, shp, shp, "so3_inverse_adjoint", workspace, out)

    def so3_forward_adjoint(self, g_flmn, workspace=None, out=None):
        """Hermitian adjoint of the forward Wigner transform: flmn-space cotangent -> f-space (FP64 plans)."""
        shp = (2 * self.N - 1,) + self.coeff_shape
        return self._call(self._lib.so3_forward_adjoint, g_flmn, shp, shp, "so3_forward_adjoint", workspace, out)

    def set_timing(self, enable=True):
        """Record HIP events around every kernel launch of this plan's transforms."""
        _check(self._lib.s2_plan_set_timing(self._handle, 1 if enable else 0))

    def read_timing(self):
        """{stage: (total_ms, launches)} since the last read (waits for the events)."""
        t = _Timing()
        _check(self._lib.s2_plan_read_timing(self._handle, ctypes.byref(t)))
        return {s: (t.ms[i], t.launches[i]) for i, s in enumerate(STAGES) if t.launches[i]}

    def debug_wigner_d(self, n):
        """d^l_{m,n}(theta_r) from the GPU recursion: [rings swept, m, l] (float64)."""
        nreg = self.L - 1 if self.sampling in ("mw", "mwss") else self.info["nrings"]
        out = torch.empty((nreg, self.L, self.L), dtype=torch.float64, device=self.device)
        with torch.cuda.device(self.device):
            _check(self._lib.s2_debug_wigner_d(self._handle, int(n), ctypes.c_void_p(out.data_ptr()),
                                               _stream_handle(self.device)))
        return out


def plan_create_raw(L, spin=0, N=1, sampling=MW, nside=0, max_batch=1, precision=FP64, stream=None):
    """Call s2_plan_create directly; returns (rc, handle).  For tests of the error model."""
    lib = load_library()
    h = ctypes.c_void_p()
    rc = lib.s2_plan_create(ctypes.byref(h), int(L), int(spin), int(N), int(sampling), int(nside), int(max_batch),
                            int(precision), stream)
    return rc, h
