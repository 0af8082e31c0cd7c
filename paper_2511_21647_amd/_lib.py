"""ctypes binding of libulmproj.so.

Argument marshalling only: every step of the path runs in the library's HIP
kernels.  PyTorch supplies device memory and the current stream.  There is no
fallback: if the library is not built, importing this module raises.
"""
from __future__ import annotations

import atexit
import ctypes
import math
import os
import weakref

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libulmproj.so")

ULM_OK = 0
ULM_ERR_INVALID_ARG = -1
ULM_ERR_HIP = -2
ULM_ERR_OVERFLOW = -3
ULM_ERR_NUMERIC = -4
ULM_ERR_NOT_IMPLEMENTED = -5
ULM_MAX_ANGLES = 32
ULM_PREC_FP64GRAM = 0
ULM_PREC_BF16X3 = 1
ULM_CNN_PARAMS = 48672
ULM_CNN_BF16 = 0
ULM_CNN_FP32 = 1
CNN_UPSAMPLE = 8
# heat threshold of the trained network's peak decode (best F1 against the truth
# among the thresholds swept on held-out simulated ensembles)
CNN_THRESHOLD = 0.1
# order and shapes of the CNN's flat FP32 parameter vector
CNN_LAYOUT = ([("w0", (32, 1, 3, 3)), ("b0", (32,))]
              + [item for l in range(1, 6) for item in ((f"w{l}", (32, 32, 3, 3)), (f"b{l}", (32,)))]
              + [("wh", (64, 32)), ("bh", (64,))])

EXPORTS = ("ulm_last_error", "ulm_create", "ulm_destroy", "ulm_workspace_size",
           "rca_beamform_proj", "rca_beamform_stage1", "rca_beamform_stage2", "rca_beamform_cross", "ulm_xdoppler", "svd_clutter_filter", "ncc_localize", "ulm_reconstruct_ensemble",
           "ulm_reconstruct_ensemble_cnn",
           "ulm_check_status", "ulm_sim_channel_data", "ulm_density_accumulate",
           "ulm_cnn_workspace_size", "ulm_cnn_localize_workspace_size", "ulm_cnn_images",
           "ulm_cnn_forward", "ulm_cnn_gradients", "ulm_cnn_train_step", "ulm_cnn_localize",
           "ulm_pair_workspace_size", "ulm_pair_planes", "ulm_pair_planes_noalloc", "ulm_slices_offset",
           "ulm_motion_workspace_size", "ulm_motion_estimate", "ulm_separate")


class ULMError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"ulmproj error {code}: {msg}")
        self.code = code


class ULMConfig(ctypes.Structure):
    _fields_ = [
        ("n_elem", ctypes.c_int32), ("n_samp", ctypes.c_int32), ("n_frames", ctypes.c_int32),
        ("n_angles", ctypes.c_int32),
        ("pitch", ctypes.c_double), ("c", ctypes.c_double), ("f0", ctypes.c_double),
        ("fs", ctypes.c_double), ("t_start", ctypes.c_double), ("bandwidth", ctypes.c_double),
        ("angles_rad", ctypes.c_double * ULM_MAX_ANGLES),
        ("nu", ctypes.c_int32), ("nz", ctypes.c_int32), ("nv", ctypes.c_int32),
        ("n_blocks", ctypes.c_int32),
        ("du", ctypes.c_double), ("dz", ctypes.c_double), ("u0", ctypes.c_double),
        ("z0", ctypes.c_double), ("dv", ctypes.c_double), ("v0", ctypes.c_double),
        ("v_ref", ctypes.c_double),
        ("svd_cutoff", ctypes.c_int32), ("ncc_size", ctypes.c_int32),
        ("precision", ctypes.c_int32), ("reserved", ctypes.c_int32),
        ("sigma_u", ctypes.c_double), ("sigma_z", ctypes.c_double),
        ("tau_ncc", ctypes.c_double), ("alpha", ctypes.c_double),
    ]


class ULMTiming(ctypes.Structure):
    _fields_ = [("ms_beamform", ctypes.c_float), ("ms_filter", ctypes.c_float),
                ("ms_localize", ctypes.c_float), ("ms_total", ctypes.c_float)]


# ulm_loc_t: int32 plane, frame, iz, iu; float32 z, u, ncc, intensity (32 bytes)
LOC_DTYPE = np.dtype([("plane", np.int32), ("frame", np.int32), ("iz", np.int32),
                      ("iu", np.int32), ("z", np.float32), ("u", np.float32),
                      ("ncc", np.float32), ("intensity", np.float32)])
LOC_WORDS = 8
# ulm_loc3d_t: int32 frame; float32 x, y, z, i_xz, i_yz; int32 idx_xz, idx_yz (32 bytes)
LOC3D_DTYPE = np.dtype([("frame", np.int32), ("x", np.float32), ("y", np.float32),
                        ("z", np.float32), ("i_xz", np.float32), ("i_yz", np.float32),
                        ("idx_xz", np.int32), ("idx_yz", np.int32)])


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
    # PyTorch ships its own HIP runtime under the same soname as the system one.
    # Importing torch first makes the library bind to that runtime, so the
    # process holds a single HIP runtime whatever the caller imports first.
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_size_t
    sig = {
        "ulm_last_error": ([], ctypes.c_char_p),
        "ulm_create": ([ctypes.POINTER(ULMConfig), ctypes.POINTER(vp)], i32),
        "ulm_destroy": ([vp], i32),
        "ulm_workspace_size": ([vp, ctypes.POINTER(sz)], i32),
        "rca_beamform_proj": ([vp, vp, vp, vp, sz, vp], i32),
        "rca_beamform_stage1": ([vp, vp, vp, sz, vp], i32),
        "rca_beamform_stage2": ([vp, vp, vp, sz, vp], i32),
        "rca_beamform_cross": ([vp, vp, vp, sz, vp], i32),
        "ulm_xdoppler": ([vp, vp, vp, i32, vp, vp], i32),
        "svd_clutter_filter": ([vp, vp, vp, vp, sz, vp], i32),
        "ncc_localize": ([vp, vp, vp, i32, vp, vp, sz, vp], i32),
        "ulm_reconstruct_ensemble": ([vp, vp, vp, vp, vp, i32, vp, vp, sz,
                                      ctypes.POINTER(ULMTiming), vp], i32),
        "ulm_check_status": ([vp, vp, vp, i32, vp], i32),
        "ulm_sim_channel_data": ([vp, vp, vp, i32, ctypes.c_uint64, ctypes.c_double, vp, vp], i32),
        "ulm_density_accumulate": ([vp, vp, vp, i32, i32, vp, vp], i32),
        "ulm_cnn_workspace_size": ([i32, i32, i32, i32, i32, ctypes.POINTER(sz)], i32),
        "ulm_cnn_localize_workspace_size": ([vp, i32, i32, ctypes.POINTER(sz)], i32),
        "ulm_cnn_images": ([vp, vp, vp, vp, sz, vp], i32),
        "ulm_cnn_forward": ([vp, vp, i32, i32, i32, i32, vp, vp, sz, vp], i32),
        "ulm_cnn_gradients": ([vp, vp, i32, i32, i32, vp, vp, i32, i32, vp, vp, vp, sz, vp], i32),
        "ulm_cnn_train_step": ([vp, vp, vp, i32, ctypes.c_float, vp, i32, i32, i32, vp, vp, i32,
                                i32, vp, vp, sz, vp], i32),
        "ulm_cnn_localize": ([vp, vp, vp, ctypes.c_float, i32, i32, vp, i32, vp, vp, sz, vp, sz,
                              vp], i32),
        "ulm_reconstruct_ensemble_cnn": ([vp, vp, vp, vp, vp, ctypes.c_float, i32, i32, vp, i32, vp,
                                          vp, sz, vp, sz, ctypes.POINTER(ULMTiming), vp], i32),
        "ulm_pair_workspace_size": ([vp, i32, ctypes.POINTER(sz)], i32),
        "ulm_pair_planes": ([vp, vp, vp, i32, vp, i32, vp, vp, sz, vp], i32),
        "ulm_pair_planes_noalloc": ([vp, vp, vp, i32, vp, i32, vp, vp], i32),
        "ulm_slices_offset": ([vp, ctypes.POINTER(sz)], i32),
        "ulm_motion_workspace_size": ([vp, i32, ctypes.POINTER(sz)], i32),
        "ulm_motion_estimate": ([vp, vp, i32, i32, vp, vp, vp, sz, vp], i32),
        "ulm_separate": ([vp, vp, i32, vp, vp], i32),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


_lib = _load()


def last_error() -> str:
    return _lib.ulm_last_error().decode()


def _check(rc: int):
    if rc != ULM_OK:
        raise ULMError(rc, last_error())


def make_config(cfg, precision: int = ULM_PREC_FP64GRAM) -> ULMConfig:
    """ulm_config_t from a configuration object with probe/seq/grid/loc attributes."""
    c = ULMConfig()
    pr, sq, g, lo = cfg.probe, cfg.seq, cfg.grid, cfg.loc
    angles = [math.radians(a) for a in sq.angles_deg]
    if len(angles) > ULM_MAX_ANGLES:
        raise ValueError("too many angles")
    c.n_elem, c.n_samp, c.n_frames, c.n_angles = pr.n_elem, sq.n_samp, sq.n_frames, len(angles)
    c.pitch, c.c, c.f0, c.fs = pr.pitch, pr.c, pr.f0, pr.fs
    c.t_start, c.bandwidth = sq.t_start, pr.bandwidth
    for i, a in enumerate(angles):
        c.angles_rad[i] = a
    c.nu, c.nz, c.nv, c.n_blocks = g.nu, g.nz, g.nv, g.n_blocks
    c.du, c.dz, c.u0, c.z0, c.dv, c.v0, c.v_ref = g.du, g.dz, g.u0, g.z0, g.dv, g.v0, g.v_ref
    c.svd_cutoff = cfg.svd_cutoff
    c.ncc_size = lo.ncc_size
    c.precision = precision
    c.sigma_u, c.sigma_z, c.tau_ncc, c.alpha = lo.sigma_u, lo.sigma_z, lo.tau_ncc, lo.alpha
    return c


def _torch():
    import torch
    return torch


def _ptr(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream=None) -> ctypes.c_void_p:
    torch = _torch()
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


# Contexts still open when the interpreter exits are closed by an exit hook,
# while the HIP runtime (and any profiler attached to it) is still up, instead
# of by object finalisation during interpreter teardown.
_LIVE_CONTEXTS = weakref.WeakSet()


@atexit.register
def _close_live_contexts():
    live = list(_LIVE_CONTEXTS)
    if not live:
        return
    torch = _torch()
    if torch.cuda.is_initialized():
        torch.cuda.synchronize()
    for c in live:
        c.close()


class Context:
    """A library context plus its device workspace (a torch uint8 tensor)."""

    def __init__(self, cfg, precision: int = ULM_PREC_FP64GRAM, device=None):
        torch = _torch()
        self.cfg = cfg
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None \
            else torch.device(device)
        self.c = make_config(cfg, precision)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(_lib.ulm_create(ctypes.byref(self.c), ctypes.byref(h)))
        self.handle = h
        n = ctypes.c_size_t()
        _check(_lib.ulm_workspace_size(h, ctypes.byref(n)))
        self.ws_bytes = n.value
        self.ws = torch.zeros(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
        off = (-self.ws.data_ptr()) % 256
        self.ws_ptr = ctypes.c_void_p(self.ws.data_ptr() + off)
        _LIVE_CONTEXTS.add(self)

    @property
    def proj_shape(self):
        c = self.c
        return (2, c.n_blocks, c.n_frames, c.nz, c.nu)

    @property
    def iq_shape(self):
        c = self.c
        return (c.n_frames, 2, c.n_angles, c.n_elem, c.n_samp)

    def close(self):
        """Destroys the library context (tables, events) and drops the workspace.
        The caller synchronises work that still uses them first."""
        if getattr(self, "handle", None):
            _lib.ulm_destroy(self.handle)
            self.handle = None
            self.ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _require(t, dtype, shape, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise ULMError(ULM_ERR_INVALID_ARG, f"{name} must be a CUDA tensor")
    if t.dtype != dtype or tuple(t.shape) != tuple(shape) or not t.is_contiguous():
        raise ULMError(ULM_ERR_INVALID_ARG,
                       f"{name}: expected contiguous {dtype} {tuple(shape)}, got {t.dtype} "
                       f"{tuple(t.shape)}")


def rca_beamform_proj(ctx: Context, iq, proj=None, stream=None):
    """IQ [F][2][K][Nc][Ns] complex64 -> projections [2][B][F][Nz][Nu] complex64."""
    torch = _torch()
    _require(iq, torch.complex64, ctx.iq_shape, "iq")
    if proj is None:
        proj = torch.empty(ctx.proj_shape, dtype=torch.complex64, device=iq.device)
    _require(proj, torch.complex64, ctx.proj_shape, "proj")
    _check(_lib.rca_beamform_proj(ctx.handle, _ptr(iq), _ptr(proj), ctx.ws_ptr, ctx.ws_bytes,
                                  _stream(stream)))
    return proj


def rca_beamform_stage1(ctx: Context, iq, stream=None):
    """Stage 1 only: reference slices into the context's workspace."""
    torch = _torch()
    _require(iq, torch.complex64, ctx.iq_shape, "iq")
    _check(_lib.rca_beamform_stage1(ctx.handle, _ptr(iq), ctx.ws_ptr, ctx.ws_bytes,
                                    _stream(stream)))


def rca_beamform_stage2(ctx: Context, proj=None, stream=None):
    """Stage 2 only: projections from the reference slices held in the workspace."""
    torch = _torch()
    if proj is None:
        proj = torch.empty(ctx.proj_shape, dtype=torch.complex64, device=ctx.device)
    _require(proj, torch.complex64, ctx.proj_shape, "proj")
    _check(_lib.rca_beamform_stage2(ctx.handle, _ptr(proj), ctx.ws_ptr, ctx.ws_bytes,
                                    _stream(stream)))
    return proj


def rca_beamform_cross(ctx: Context, cross=None, stream=None):
    """Cross projections [2][B][F][Nz][Nu] (each plane gets the other orientation's
    volume) from the reference slices held in the workspace."""
    torch = _torch()
    if cross is None:
        cross = torch.empty(ctx.proj_shape, dtype=torch.complex64, device=ctx.device)
    _require(cross, torch.complex64, ctx.proj_shape, "cross")
    _check(_lib.rca_beamform_cross(ctx.handle, _ptr(cross), ctx.ws_ptr, ctx.ws_bytes,
                                   _stream(stream)))
    return cross


def ulm_xdoppler(ctx: Context, native, cross, window: int = 3, out=None, stream=None):
    """XDoppler image (sqrt of the windowed |native conj(cross)|, zero imaginary
    part) [2][B][F][Nz][Nu]; `out` may be `native` (in place)."""
    torch = _torch()
    _require(native, torch.complex64, ctx.proj_shape, "native")
    _require(cross, torch.complex64, ctx.proj_shape, "cross")
    if out is None:
        out = torch.empty(ctx.proj_shape, dtype=torch.complex64, device=native.device)
    _require(out, torch.complex64, ctx.proj_shape, "out")
    _check(_lib.ulm_xdoppler(ctx.handle, _ptr(native), _ptr(cross), int(window), _ptr(out),
                             _stream(stream)))
    return out


def svd_clutter_filter(ctx: Context, proj, eigvals=None, stream=None):
    """In-place clutter filter of every plane; returns eigenvalues [2][B][F] (descending)."""
    torch = _torch()
    _require(proj, torch.complex64, ctx.proj_shape, "proj")
    if eigvals is None:
        eigvals = torch.empty(ctx.proj_shape[:3], dtype=torch.float64, device=proj.device)
    _require(eigvals, torch.float64, ctx.proj_shape[:3], "eigvals")
    _check(_lib.svd_clutter_filter(ctx.handle, _ptr(proj), _ptr(eigvals), ctx.ws_ptr,
                                   ctx.ws_bytes, _stream(stream)))
    return eigvals


def ncc_localize(ctx: Context, filtered, capacity: int, locs=None, count=None, stream=None):
    """Returns (locs int32 [capacity][8] holding ulm_loc_t records, count int32 [1])."""
    torch = _torch()
    _require(filtered, torch.complex64, ctx.proj_shape, "filtered")
    if locs is None:
        locs = torch.empty((max(capacity, 1), LOC_WORDS), dtype=torch.int32, device=filtered.device)
    if count is None:
        count = torch.zeros(1, dtype=torch.int32, device=filtered.device)
    _check(_lib.ncc_localize(ctx.handle, _ptr(filtered), _ptr(locs), int(capacity), _ptr(count),
                             ctx.ws_ptr, ctx.ws_bytes, _stream(stream)))
    return locs, count


def ulm_reconstruct_ensemble(ctx: Context, iq, capacity: int, proj=None, eigvals=None, locs=None,
                             count=None, timing: bool = False, stream=None):
    """The whole path.  Returns dict(proj=filtered planes, eigvals, locs, count, timing)."""
    torch = _torch()
    _require(iq, torch.complex64, ctx.iq_shape, "iq")
    dev = iq.device
    if proj is None:
        proj = torch.empty(ctx.proj_shape, dtype=torch.complex64, device=dev)
    if eigvals is None:
        eigvals = torch.empty(ctx.proj_shape[:3], dtype=torch.float64, device=dev)
    if locs is None:
        locs = torch.empty((max(capacity, 1), LOC_WORDS), dtype=torch.int32, device=dev)
    if count is None:
        count = torch.zeros(1, dtype=torch.int32, device=dev)
    tm = ULMTiming() if timing else None
    _check(_lib.ulm_reconstruct_ensemble(ctx.handle, _ptr(iq), _ptr(proj), _ptr(eigvals),
                                         _ptr(locs), int(capacity), _ptr(count), ctx.ws_ptr,
                                         ctx.ws_bytes, ctypes.byref(tm) if tm else None,
                                         _stream(stream)))
    out = {"proj": proj, "eigvals": eigvals, "locs": locs, "count": count}
    if tm is not None:
        out["timing"] = {"beamform": tm.ms_beamform, "filter": tm.ms_filter,
                         "localize": tm.ms_localize, "total": tm.ms_total}
    return out


def ulm_check_status(ctx: Context, count=None, capacity: int = -1, stream=None):
    """Synchronise and raise ULMError for a numeric failure or a capacity overflow."""
    _check(_lib.ulm_check_status(ctx.handle, ctx.ws_ptr,
                                 _ptr(count) if count is not None else None, int(capacity),
                                 _stream(stream)))


def ulm_sim_channel_data(ctx: Context, pos, amp, noise_seed: int, noise_sigma: float, iq=None,
                         stream=None):
    """pos [F][S][3] float64, amp [S] complex128 (device) -> IQ [F][2][K][Nc][Ns] complex64."""
    torch = _torch()
    S = pos.shape[1]
    _require(pos, torch.float64, (ctx.c.n_frames, S, 3), "pos")
    _require(amp, torch.complex128, (S,), "amp")
    if iq is None:
        iq = torch.empty(ctx.iq_shape, dtype=torch.complex64, device=pos.device)
    _require(iq, torch.complex64, ctx.iq_shape, "iq")
    _check(_lib.ulm_sim_channel_data(ctx.handle, _ptr(pos), _ptr(amp), int(S),
                                     ctypes.c_uint64(int(noise_seed) & (2 ** 64 - 1)),
                                     float(noise_sigma), _ptr(iq), _stream(stream)))
    return iq


def ulm_density_accumulate(ctx: Context, locs, count, capacity: int, density, upsample: int = 2,
                           stream=None):
    """Adds the localisations to density [2B][Nz*up][Nu*up] uint32 (torch.int32 storage)."""
    torch = _torch()
    shape = (2 * ctx.c.n_blocks, ctx.c.nz * upsample, ctx.c.nu * upsample)
    _require(density, torch.int32, shape, "density")
    _check(_lib.ulm_density_accumulate(ctx.handle, _ptr(locs), _ptr(count), int(capacity),
                                       int(upsample), _ptr(density), _stream(stream)))
    return density


def locs_to_numpy(locs, count) -> np.ndarray:
    """Copy the first min(count, capacity) records to a structured numpy array."""
    n = int(count.item()) if hasattr(count, "item") else int(count)
    n = min(n, locs.shape[0])
    raw = locs[:n].contiguous().cpu().numpy()
    return raw.view(LOC_DTYPE).reshape(-1)


# ---------------------------------------------------------------- learned localiser

def cnn_pack(params: dict) -> np.ndarray:
    """Flat float32 parameter vector from a dict of arrays named as in CNN_LAYOUT."""
    parts = []
    for name, shape in CNN_LAYOUT:
        a = np.asarray(params[name], dtype=np.float64)
        if a.shape != shape:
            raise ValueError(f"{name}: expected shape {shape}, got {a.shape}")
        parts.append(a.reshape(-1))
    return np.concatenate(parts).astype(np.float32)


def cnn_unpack(flat) -> dict:
    """Dict of float64 arrays from a flat parameter vector (numpy or tensor)."""
    v = np.asarray(flat.detach().cpu().numpy() if hasattr(flat, "detach") else flat, np.float64)
    if v.size != ULM_CNN_PARAMS:
        raise ValueError(f"expected {ULM_CNN_PARAMS} values, got {v.size}")
    out, o = {}, 0
    for name, shape in CNN_LAYOUT:
        n = int(np.prod(shape))
        out[name] = v[o:o + n].reshape(shape).copy()
        o += n
    return out


class Workspace:
    """256-byte-aligned device scratch of a fixed size (a torch uint8 tensor)."""

    def __init__(self, nbytes: int, device):
        torch = _torch()
        self.nbytes = int(nbytes)
        self.buf = torch.empty(self.nbytes + 256, dtype=torch.uint8, device=device)
        self.ptr = ctypes.c_void_p(self.buf.data_ptr() + (-self.buf.data_ptr()) % 256)


def ulm_cnn_workspace_size(batch: int, nz: int, nu: int, precision: int = ULM_CNN_BF16,
                           train: bool = False) -> int:
    n = ctypes.c_size_t()
    _check(_lib.ulm_cnn_workspace_size(int(batch), int(nz), int(nu), int(precision), int(bool(train)),
                                       ctypes.byref(n)))
    return n.value


def ulm_cnn_localize_workspace_size(ctx: Context, batch: int, precision: int = ULM_CNN_BF16) -> int:
    n = ctypes.c_size_t()
    _check(_lib.ulm_cnn_localize_workspace_size(ctx.handle, int(batch), int(precision),
                                                ctypes.byref(n)))
    return n.value


def _require_rows(t, rows, name):
    """t: contiguous int32 CUDA tensor [>= rows][8] of 32-byte records."""
    torch = _torch()
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise ULMError(ULM_ERR_INVALID_ARG, f"{name} must be a CUDA tensor")
    if (t.dtype != torch.int32 or t.dim() != 2 or t.shape[1] != 8 or t.shape[0] < rows
            or not t.is_contiguous()):
        raise ULMError(ULM_ERR_INVALID_ARG,
                       f"{name}: expected contiguous int32 [>= {rows}][8], got {t.dtype} "
                       f"{tuple(t.shape)}")


def _ws(ws, nbytes, device):
    if ws is None:
        return Workspace(nbytes, device)
    if ws.nbytes < nbytes:
        raise ULMError(ULM_ERR_INVALID_ARG, f"workspace holds {ws.nbytes} bytes, needs {nbytes}")
    return ws


def _params(params):
    torch = _torch()
    _require(params, torch.float32, (ULM_CNN_PARAMS,), "params")


def ulm_cnn_images(ctx: Context, filtered, images=None, stream=None):
    """Filtered planes [2][B][F][Nz][Nu] complex64 -> CNN inputs [2B*F][Nz][Nu] float32."""
    torch = _torch()
    _require(filtered, torch.complex64, ctx.proj_shape, "filtered")
    shape = (2 * ctx.c.n_blocks * ctx.c.n_frames, ctx.c.nz, ctx.c.nu)
    if images is None:
        images = torch.empty(shape, dtype=torch.float32, device=filtered.device)
    _require(images, torch.float32, shape, "images")
    _check(_lib.ulm_cnn_images(ctx.handle, _ptr(filtered), _ptr(images), ctx.ws_ptr, ctx.ws_bytes,
                               _stream(stream)))
    return images


def ulm_cnn_forward(params, images, precision: int = ULM_CNN_BF16, heat=None, ws=None,
                    stream=None):
    """images [batch][nz][nu] float32 -> heatmaps [batch][8 nz][8 nu] float32."""
    torch = _torch()
    _params(params)
    B, nz, nu = images.shape
    _require(images, torch.float32, (B, nz, nu), "images")
    shape = (B, nz * CNN_UPSAMPLE, nu * CNN_UPSAMPLE)
    if heat is None:
        heat = torch.empty(shape, dtype=torch.float32, device=images.device)
    _require(heat, torch.float32, shape, "heat")
    ws = _ws(ws, ulm_cnn_workspace_size(B, nz, nu, precision, False), images.device)
    _check(_lib.ulm_cnn_forward(_ptr(params), _ptr(images), B, nz, nu, int(precision), _ptr(heat),
                                ws.ptr, ws.nbytes, _stream(stream)))
    return heat


def _labels(mb_zu, mb_img, device):
    torch = _torch()
    n = 0 if mb_zu is None else int(mb_zu.shape[0])
    if n == 0:
        return None, None, 0
    _require(mb_zu, torch.float32, (n, 2), "mb_zu")
    _require(mb_img, torch.int32, (n,), "mb_img")
    return _ptr(mb_zu), _ptr(mb_img), n


def ulm_cnn_gradients(params, images, mb_zu, mb_img, precision: int = ULM_CNN_BF16, grad=None,
                      loss=None, ws=None, stream=None):
    """Loss (float32 [1]) and gradient (float32 [ULM_CNN_PARAMS]) of a batch."""
    torch = _torch()
    _params(params)
    B, nz, nu = images.shape
    _require(images, torch.float32, (B, nz, nu), "images")
    dev = images.device
    if grad is None:
        grad = torch.empty(ULM_CNN_PARAMS, dtype=torch.float32, device=dev)
    if loss is None:
        loss = torch.empty(1, dtype=torch.float32, device=dev)
    pz, pi, n = _labels(mb_zu, mb_img, dev)
    ws = _ws(ws, ulm_cnn_workspace_size(B, nz, nu, precision, True), dev)
    _check(_lib.ulm_cnn_gradients(_ptr(params), _ptr(images), B, nz, nu, pz, pi, n, int(precision),
                                  _ptr(grad), _ptr(loss), ws.ptr, ws.nbytes, _stream(stream)))
    return loss, grad


def ulm_cnn_train_step(params, adam_m, adam_v, step: int, lr: float, images, mb_zu, mb_img,
                       precision: int = ULM_CNN_BF16, loss=None, ws=None, stream=None):
    """One Adam step in place on params / adam_m / adam_v; returns the batch loss tensor."""
    torch = _torch()
    _params(params)
    _require(adam_m, torch.float32, (ULM_CNN_PARAMS,), "adam_m")
    _require(adam_v, torch.float32, (ULM_CNN_PARAMS,), "adam_v")
    B, nz, nu = images.shape
    _require(images, torch.float32, (B, nz, nu), "images")
    dev = images.device
    if loss is None:
        loss = torch.empty(1, dtype=torch.float32, device=dev)
    pz, pi, n = _labels(mb_zu, mb_img, dev)
    ws = _ws(ws, ulm_cnn_workspace_size(B, nz, nu, precision, True), dev)
    _check(_lib.ulm_cnn_train_step(_ptr(params), _ptr(adam_m), _ptr(adam_v), int(step),
                                   ctypes.c_float(lr), _ptr(images), B, nz, nu, pz, pi, n,
                                   int(precision), _ptr(loss), ws.ptr, ws.nbytes, _stream(stream)))
    return loss


def ulm_cnn_localize(ctx: Context, params, filtered, capacity: int, threshold: float = CNN_THRESHOLD,
                     batch: int = 64, precision: int = ULM_CNN_BF16, locs=None, count=None,
                     ws=None, stream=None):
    """CNN localisation of the filtered planes; returns (locs, count) as ncc_localize."""
    torch = _torch()
    _params(params)
    _require(filtered, torch.complex64, ctx.proj_shape, "filtered")
    dev = filtered.device
    if locs is None:
        locs = torch.empty((max(capacity, 1), LOC_WORDS), dtype=torch.int32, device=dev)
    if count is None:
        count = torch.zeros(1, dtype=torch.int32, device=dev)
    ws = _ws(ws, ulm_cnn_localize_workspace_size(ctx, batch, precision), dev)
    _check(_lib.ulm_cnn_localize(ctx.handle, _ptr(params), _ptr(filtered), ctypes.c_float(threshold),
                                 int(batch), int(precision), _ptr(locs), int(capacity),
                                 _ptr(count), ctx.ws_ptr, ctx.ws_bytes, ws.ptr, ws.nbytes,
                                 _stream(stream)))
    return locs, count


def ulm_reconstruct_ensemble_cnn(ctx: Context, iq, params, capacity: int,
                                 threshold: float = CNN_THRESHOLD, batch: int = 64,
                                 precision: int = ULM_CNN_BF16, proj=None, eigvals=None, locs=None,
                                 count=None, ws=None, timing: bool = False, stream=None):
    """The whole path with the CNN localiser.  Returns dict(proj=filtered planes,
    eigvals, locs, count, timing) as ulm_reconstruct_ensemble."""
    torch = _torch()
    _require(iq, torch.complex64, ctx.iq_shape, "iq")
    _params(params)
    dev = iq.device
    if proj is None:
        proj = torch.empty(ctx.proj_shape, dtype=torch.complex64, device=dev)
    if eigvals is None:
        eigvals = torch.empty(ctx.proj_shape[:3], dtype=torch.float64, device=dev)
    if locs is None:
        locs = torch.empty((max(capacity, 1), LOC_WORDS), dtype=torch.int32, device=dev)
    if count is None:
        count = torch.zeros(1, dtype=torch.int32, device=dev)
    ws = _ws(ws, ulm_cnn_localize_workspace_size(ctx, batch, precision), dev)
    tm = ULMTiming() if timing else None
    _check(_lib.ulm_reconstruct_ensemble_cnn(ctx.handle, _ptr(iq), _ptr(proj), _ptr(eigvals),
                                             _ptr(params), ctypes.c_float(threshold), int(batch),
                                             int(precision), _ptr(locs), int(capacity), _ptr(count),
                                             ctx.ws_ptr, ctx.ws_bytes, ws.ptr, ws.nbytes,
                                             ctypes.byref(tm) if tm else None, _stream(stream)))
    out = {"proj": proj, "eigvals": eigvals, "locs": locs, "count": count}
    if tm is not None:
        out["timing"] = {"beamform": tm.ms_beamform, "filter": tm.ms_filter,
                         "localize": tm.ms_localize, "total": tm.ms_total}
    return out


# ---------------------------------------------------------------- plane pairing

def ulm_pair_workspace_size(ctx: Context, capacity: int) -> int:
    n = ctypes.c_size_t()
    _check(_lib.ulm_pair_workspace_size(ctx.handle, int(capacity), ctypes.byref(n)))
    return n.value


def ulm_pair_planes(ctx: Context, locs, count, capacity: int, out_capacity: int, out=None,
                    out_count=None, ws=None, stream=None):
    """Pairs XZ and YZ localisations (records sorted by plane and frame) into 3D
    localisations; returns (out int32 [out_capacity][8] of ulm_loc3d_t, out_count)."""
    torch = _torch()
    _require_rows(locs, capacity, "locs")
    _require(count, torch.int32, (1,), "count")
    dev = locs.device
    if out is None:
        out = torch.empty((max(out_capacity, 1), 8), dtype=torch.int32, device=dev)
    if out_count is None:
        out_count = torch.zeros(1, dtype=torch.int32, device=dev)
    _require_rows(out, out_capacity, "out")
    _require(out_count, torch.int32, (1,), "out_count")
    ws = _ws(ws, ulm_pair_workspace_size(ctx, capacity), dev)
    _check(_lib.ulm_pair_planes(ctx.handle, _ptr(locs), _ptr(count), int(capacity), _ptr(out),
                                int(out_capacity), _ptr(out_count), ws.ptr, ws.nbytes,
                                _stream(stream)))
    return out, out_count


ULM_NOALLOC_SCRATCH_BYTES = 32 << 20


def ulm_pair_planes_noalloc(ctx: Context, locs, count, capacity: int, out_capacity: int, out,
                            out_count, stream=None):
    """ulm_pair_planes with the library's own scratch array instead of a
    workspace; the caller passes preallocated `out` and `out_count`."""
    torch = _torch()
    _require_rows(locs, capacity, "locs")
    _require(count, torch.int32, (1,), "count")
    _require_rows(out, out_capacity, "out")
    _require(out_count, torch.int32, (1,), "out_count")
    _check(_lib.ulm_pair_planes_noalloc(ctx.handle, _ptr(locs), _ptr(count), int(capacity),
                                        _ptr(out), int(out_capacity), _ptr(out_count),
                                        _stream(stream)))
    return out, out_count


def loc3d_to_numpy(out, count) -> np.ndarray:
    """Copy the first min(count, capacity) 3D records to a structured numpy array."""
    n = int(count.item()) if hasattr(count, "item") else int(count)
    n = min(n, out.shape[0])
    return out[:n].contiguous().cpu().numpy().view(LOC3D_DTYPE).reshape(-1)


# ---------------------------------------------------------------- motion estimation

def ulm_stage1_slices(ctx: Context):
    """The stage-1 reference slices [2][K][F][Nz][Nu] (complex64) that
    rca_beamform_stage1 leaves in the context's workspace, as a tensor view."""
    torch = _torch()
    off = ctypes.c_size_t()
    _check(_lib.ulm_slices_offset(ctx.handle, ctypes.byref(off)))
    shape = (2, ctx.c.n_angles, ctx.c.n_frames, ctx.c.nz, ctx.c.nu)
    n = 8 * int(np.prod(shape))
    start = ctx.ws_ptr.value - ctx.ws.data_ptr() + off.value
    return ctx.ws[start:start + n].view(torch.complex64).view(shape)


def ulm_motion_workspace_size(ctx: Context, max_lag: int) -> int:
    n = ctypes.c_size_t()
    _check(_lib.ulm_motion_workspace_size(ctx.handle, int(max_lag), ctypes.byref(n)))
    return n.value


def ulm_motion_estimate(ctx: Context, slices, ref_frame: int = 0, max_lag: int = 8, disp=None,
                        motion=None, ws=None, stream=None):
    """Rigid motion of every frame against `ref_frame` from the stage-1 slices
    [2][K][F][Nz][Nu] (complex64).  Returns (disp float32 [2][K][F][2] = (dz, du),
    motion float32 [F][3] = (dx, dy, dz)), in pixels."""
    torch = _torch()
    K, F = ctx.c.n_angles, ctx.c.n_frames
    _require(slices, torch.complex64, (2, K, F, ctx.c.nz, ctx.c.nu), "slices")
    dev = slices.device
    if disp is None:
        disp = torch.empty((2, K, F, 2), dtype=torch.float32, device=dev)
    if motion is None:
        motion = torch.empty((F, 3), dtype=torch.float32, device=dev)
    _require(disp, torch.float32, (2, K, F, 2), "disp")
    _require(motion, torch.float32, (F, 3), "motion")
    ws = _ws(ws, ulm_motion_workspace_size(ctx, max_lag), dev)
    _check(_lib.ulm_motion_estimate(ctx.handle, _ptr(slices), int(ref_frame), int(max_lag),
                                    _ptr(disp), _ptr(motion), ws.ptr, ws.nbytes, _stream(stream)))
    return disp, motion


# ---------------------------------------------------------------- MB separation

def ulm_separate(ctx: Context, filtered, n_speed: int = 3, subsets=None, stream=None):
    """Up/down x speed-range subsets of the filtered planes:
    [2 n_speed][2][B][F][Nz][Nu] complex64 (up ranges first, slowest first)."""
    torch = _torch()
    _require(filtered, torch.complex64, ctx.proj_shape, "filtered")
    shape = (2 * int(n_speed),) + tuple(ctx.proj_shape)
    if subsets is None:
        subsets = torch.empty(shape, dtype=torch.complex64, device=filtered.device)
    _require(subsets, torch.complex64, shape, "subsets")
    _check(_lib.ulm_separate(ctx.handle, _ptr(filtered), int(n_speed), _ptr(subsets),
                             _stream(stream)))
    return subsets
