"""Gauss-polynomial bilateral filter on MI355X (gfx950): Python binding.

Thin ctypes layer over ``libbfgp.so`` (built from ``csrc/`` by ``build.py``).
Every step of the filter runs in the library's HIP kernels; this module only
marshals PyTorch tensors (device memory) and the current HIP stream into the
C ABI declared in ``include/bfgp.h``.  If the library is missing, importing
this package raises: there is no fallback.

Method: K. N. Chaudhury, "Fast and Accurate Bilateral Filtering using
Gauss-Polynomial Decomposition", arXiv 1505.00077 (Algorithm 1, eqs. (1)-(11)).
"""
import ctypes
import math
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbfgp.so")

BF_OK, BF_EINVAL, BF_ENOMEM, BF_ERANGE, BF_EHIP, BF_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
SPATIAL = {"auto": 0, "fir": 1, "iir": 2, "box": 3}
CENTER = {"mean": 0, "midrange": 4, "none": 8}
MAX_DEGREE = 64
FIR_MAX_RADIUS = 24

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with paper_1505_00077_amd/build.py "
                      "(or __graft_entry__.build())")

lib = ctypes.CDLL(LIB_PATH)


class BfGpItem(ctypes.Structure):
    _fields_ = [("img", ctypes.c_void_p), ("out", ctypes.c_void_p), ("H", ctypes.c_int), ("W", ctypes.c_int),
                ("pitch", ctypes.c_int), ("sigma_s", ctypes.c_float), ("sigma_r", ctypes.c_float), ("N", ctypes.c_int)]


def _sig(name, res, *args):
    f = getattr(lib, name)
    f.restype = res
    f.argtypes = list(args)
    return f


_vp, _i, _u, _d, _sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_uint, ctypes.c_double, ctypes.c_size_t
bf_version = _sig("bf_version", _i)
bf_last_error = _sig("bf_last_error", ctypes.c_char_p)
bf_gp_workspace_bytes = _sig("bf_gp_workspace_bytes", _sz, _i, _i, _i, _d, _u)
bf_gp_forward = _sig("bf_gp_forward", _i, _vp, _vp, _i, _i, _i, _d, _d, _i, _u, _vp, _vp, _sz, _vp)
bf_gp_forward_noalloc = _sig("bf_gp_forward_noalloc", _i, _vp, _vp, _i, _i, _i, _d, _d, _i, _u, _vp, _vp)
NOALLOC_SCRATCH_BYTES = 128 << 20
bf_gp_joint_workspace_bytes = _sig("bf_gp_joint_workspace_bytes", _sz, _i, _i, _i, _d, _u)
bf_gp_joint_forward = _sig("bf_gp_joint_forward", _i, _vp, _vp, _vp, _i, _i, _i, _d, _d, _i, _u, _vp, _sz, _vp)
bf_gp_volume_workspace_bytes = _sig("bf_gp_volume_workspace_bytes", _sz, _i, _i, _i, _i, _d, _d, _u)
bf_gp_volume_forward = _sig("bf_gp_volume_forward", _i, _vp, _vp, _i, _i, _i, _d, _d, _d, _i, _u, _vp, _sz, _vp)
bf_gp_degree_for = _sig("bf_gp_degree_for", _i, _d, _d)
bf_gp_status = _sig("bf_gp_status", _i, _vp, _vp, ctypes.POINTER(_i))
bf_gp_resolve_spatial = _sig("bf_gp_resolve_spatial", _u, _d, _u)
bf_gp_resolve_spatial_for = _sig("bf_gp_resolve_spatial_for", _u, _i, _i, _d, _u)
bf_gp_set_fir_crossover_table = _sig("bf_gp_set_fir_crossover_table", _i, ctypes.POINTER(ctypes.c_longlong),
                                     ctypes.POINTER(_i), _i)
bf_gp_get_fir_crossover_table = _sig("bf_gp_get_fir_crossover_table", _i, ctypes.POINTER(ctypes.c_longlong),
                                     ctypes.POINTER(_i), _i)
bf_gp_set_fir_crossover = _sig("bf_gp_set_fir_crossover", _i, _i)
bf_gp_get_fir_crossover = _sig("bf_gp_get_fir_crossover", _i)
bf_gp_set_iir_tuning = _sig("bf_gp_set_iir_tuning", _i, _i, _i, _i)
bf_gp_iir_shape = _sig("bf_gp_iir_shape", _i, _i, _i, _i, ctypes.POINTER(_i))
bf_gp_backward_workspace_bytes = _sig("bf_gp_backward_workspace_bytes", _sz, _i, _i, _i, _d, _u)
bf_gp_backward = _sig("bf_gp_backward", _i, _vp, _vp, _vp, _i, _i, _i, _d, _d, _i, _u, _vp, _vp, _vp, _vp, _sz, _vp)
bf_gp_forward_stacked_workspace_bytes = _sig("bf_gp_forward_stacked_workspace_bytes", _sz, _i, _i, _i, _i, _d, _u)
bf_gp_forward_stacked = _sig("bf_gp_forward_stacked", _i, _vp, _vp, _i, _i, _i, _i, _sz, _d, _d, _i, _u, _vp, _vp,
                             _sz, _vp)
bf_gp_backward_stacked_workspace_bytes = _sig("bf_gp_backward_stacked_workspace_bytes", _sz, _i, _i, _i, _i, _d, _u)
bf_gp_backward_stacked = _sig("bf_gp_backward_stacked", _i, _vp, _vp, _vp, _i, _i, _i, _i, _sz, _d, _d, _i, _u, _vp,
                              _vp, _vp, _vp, _sz, _vp)
bf_gp_plan_batched = _sig("bf_gp_plan_batched", _i, ctypes.POINTER(BfGpItem), _i, _u, ctypes.POINTER(_vp))
bf_gp_plan_workspace_bytes = _sig("bf_gp_plan_workspace_bytes", _sz, _vp)
bf_gp_plan_upload = _sig("bf_gp_plan_upload", _i, _vp, _vp, _sz, _vp)
bf_gp_forward_batched = _sig("bf_gp_forward_batched", _i, _vp, _vp, _sz, _vp)
bf_gp_plan_free = _sig("bf_gp_plan_free", None, _vp)
bf_direct_forward = _sig("bf_direct_forward", _i, _vp, _vp, _i, _i, _i, _d, _d, _i, _vp)
bf_profile_enable = _sig("bf_profile_enable", _i, _i)
bf_profile_collect = _sig("bf_profile_collect", _i, _i, ctypes.POINTER(ctypes.c_char_p), ctypes.POINTER(_i),
                          ctypes.POINTER(_d), ctypes.POINTER(ctypes.c_longlong))


class BfError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        msg = bf_last_error().decode(errors="replace")
        super().__init__(f"{where} failed with status {code}: {msg}")


def _check(rc, where):
    if rc != BF_OK:
        raise BfError(rc, where)


def _stream(device=None):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _flags(spatial="auto", center="mean"):
    return SPATIAL[spatial] | CENTER[center]


def _image(t, name="img"):
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float32 or not t.is_cuda:
        raise TypeError(f"{name} must be a float32 CUDA tensor")
    if t.dim() != 2:
        raise ValueError(f"{name} must be 2-D (H, W)")
    if t.stride(1) != 1:
        raise ValueError(f"{name} must have unit column stride")
    return t.shape[0], t.shape[1], t.stride(0)


def _like(t):
    """An uninitialised tensor with t's shape and strides (the kernels write
    outputs with the input's pitch; torch.empty_like makes a padded view
    contiguous)."""
    return torch.empty_strided(t.shape, t.stride(), dtype=t.dtype, device=t.device)


def fir_radius(sigma_s):
    """Window half-width of eq. (1): ceil(3 sigma_s), at least 1 (a relative
    excess below 1e-6 does not round up)."""
    return max(1, int(math.ceil(3.0 * sigma_s * (1.0 - 1e-6))))


def resolve_spatial(sigma_s, spatial="auto", shape=None):
    """"fir" or "iir" for this sigma_s (for an image of `shape` = (H, W) when
    given, which honours the size-dependent crossover table); "box" stays
    "box"."""
    if shape is None:
        m = bf_gp_resolve_spatial(float(sigma_s), SPATIAL[spatial])
    else:
        m = bf_gp_resolve_spatial_for(int(shape[0]), int(shape[1]), float(sigma_s), SPATIAL[spatial])
    return {1: "fir", 2: "iir", 3: "box"}[m]


def set_fir_crossover_table(table):
    """table: [(max_pixels, radius), ...] with increasing max_pixels ([] clears)."""
    n = len(table)
    px = (ctypes.c_longlong * max(n, 1))(*[int(a) for a, _ in table])
    rr = (ctypes.c_int * max(n, 1))(*[int(b) for _, b in table])
    _check(bf_gp_set_fir_crossover_table(px, rr, n), "bf_gp_set_fir_crossover_table")


def get_fir_crossover_table():
    px = (ctypes.c_longlong * 8)()
    rr = (ctypes.c_int * 8)()
    n = bf_gp_get_fir_crossover_table(px, rr, 8)
    if n < 0:
        raise BfError(n, "bf_gp_get_fir_crossover_table")
    return [(int(px[k]), int(rr[k])) for k in range(n)]


def workspace_bytes(H, W, N, sigma_s, spatial="auto", center="mean"):
    return int(bf_gp_workspace_bytes(int(H), int(W), int(N), float(sigma_s), _flags(spatial, center)))


def workspace(H, W, N, sigma_s, spatial="auto", device="cuda"):
    n = workspace_bytes(H, W, N, sigma_s, spatial)
    return torch.empty(max(n, 256), dtype=torch.uint8, device=device)


def gp_forward(img, sigma_s, sigma_r, N=20, spatial="auto", center="mean", out=None, ws=None, saved=None,
               check=False):
    """GP bilateral filter of one image (Algorithm 1, rescaled channels).

    img: float32 CUDA tensor (H, W).  Returns ``out``.  ``saved`` (uint8 CUDA
    tensor of 16*H*W bytes) receives what ``gp_backward`` needs.  With
    ``check=True`` the call synchronises and raises on BF_ERANGE."""
    H, W, pitch = _image(img)
    if out is None:
        out = _like(img)
    else:
        oh, ow, opitch = _image(out, "out")
        if (oh, ow, opitch) != (H, W, pitch):
            raise ValueError("out must have the shape and row stride of img")
    flags = _flags(spatial, center)
    need = int(bf_gp_workspace_bytes(H, W, int(N), float(sigma_s), flags))
    if ws is None:
        ws = torch.empty(max(need, 256), dtype=torch.uint8, device=img.device)
    sp = None
    if saved is not None:
        if saved.numel() * saved.element_size() < 16 * H * W:
            raise ValueError("saved buffer too small")
        sp = saved.data_ptr()
    _check(bf_gp_forward(img.data_ptr(), out.data_ptr(), H, W, pitch, float(sigma_s), float(sigma_r), int(N), flags,
                         sp, ws.data_ptr(), ws.numel(), _stream(img.device)), "bf_gp_forward")
    if check:
        st = status(ws, img.device)
        if st != BF_OK:
            raise BfError(st, "bf_gp_forward (device status)")
    return out


def gp_forward_noalloc(img, sigma_s, sigma_r, N=20, spatial="auto", center="mean", out=None, saved=None):
    """GP forward like ``gp_forward``, with the workspace in the library's
    static device array (bf_gp_forward_noalloc): no workspace is allocated.
    ``out`` (and ``saved``) must be given by callers that cannot allocate."""
    H, W, pitch = _image(img)
    if out is None:
        out = _like(img)
    else:
        oh, ow, opitch = _image(out, "out")
        if (oh, ow, opitch) != (H, W, pitch):
            raise ValueError("out must have the shape and row stride of img")
    sp = None
    if saved is not None:
        if saved.numel() * saved.element_size() < 16 * H * W:
            raise ValueError("saved buffer too small")
        sp = saved.data_ptr()
    _check(bf_gp_forward_noalloc(img.data_ptr(), out.data_ptr(), H, W, pitch, float(sigma_s), float(sigma_r),
                                 int(N), _flags(spatial, center), sp, _stream(img.device)), "bf_gp_forward_noalloc")
    return out


def joint_workspace(H, W, N, sigma_s, spatial="auto", center="mean", device="cuda"):
    n = int(bf_gp_joint_workspace_bytes(int(H), int(W), int(N), float(sigma_s), _flags(spatial, center)))
    return torch.empty(max(n, 256), dtype=torch.uint8, device=device)


def gp_joint_forward(guide, data, sigma_s, sigma_r, N=20, spatial="auto", center="mean", out=None, ws=None,
                     check=False):
    """Joint (cross) GP bilateral filter: the range kernel on ``guide``, the
    average of ``data`` (float32 CUDA tensors of one shape and row stride).
    Runs in the recursive spatial mode.  Returns ``out``."""
    H, W, pitch = _image(guide)
    dh, dw, dp = _image(data, "data")
    if (dh, dw, dp) != (H, W, pitch):
        raise ValueError("data must have the shape and row stride of the guide")
    if out is None:
        out = _like(guide)
    else:
        oh, ow, opitch = _image(out, "out")
        if (oh, ow, opitch) != (H, W, pitch):
            raise ValueError("out must have the shape and row stride of the guide")
    flags = _flags(spatial, center)
    if ws is None:
        ws = joint_workspace(H, W, N, sigma_s, spatial, center, guide.device)
    _check(bf_gp_joint_forward(guide.data_ptr(), data.data_ptr(), out.data_ptr(), H, W, pitch, float(sigma_s),
                               float(sigma_r), int(N), flags, ws.data_ptr(), ws.numel(), _stream(guide.device)),
           "bf_gp_joint_forward")
    if check:
        st = status(ws, guide.device)
        if st != BF_OK:
            raise BfError(st, "bf_gp_joint_forward (device status)")
    return out


def volume_workspace(T, H, W, N, sigma_s, sigma_t, spatial="auto", center="mean", device="cuda"):
    n = int(bf_gp_volume_workspace_bytes(int(T), int(H), int(W), int(N), float(sigma_s), float(sigma_t),
                                         _flags(spatial, center)))
    return torch.empty(max(n, 256), dtype=torch.uint8, device=device)


def gp_volume_forward(vol, sigma_s, sigma_t, sigma_r, N=20, spatial="auto", center="mean", out=None, ws=None,
                      check=False):
    """GP bilateral filter of a volume or video: ``vol`` a contiguous float32
    CUDA tensor (T, H, W); sigma_s along rows and columns, sigma_t along the
    first axis.  Runs in the recursive spatial mode.  Returns ``out``."""
    if vol.dtype != torch.float32 or not vol.is_cuda or vol.dim() != 3 or not vol.is_contiguous():
        raise ValueError("vol must be a contiguous float32 CUDA tensor (T, H, W)")
    T, H, W = vol.shape
    if out is None:
        out = _like(vol)
    elif out.shape != vol.shape or out.dtype != torch.float32 or not out.is_contiguous():
        raise ValueError("out must be a contiguous float32 tensor shaped like vol")
    flags = _flags(spatial, center)
    if ws is None:
        ws = volume_workspace(T, H, W, N, sigma_s, sigma_t, spatial, center, vol.device)
    _check(bf_gp_volume_forward(vol.data_ptr(), out.data_ptr(), T, H, W, float(sigma_s), float(sigma_t),
                                float(sigma_r), int(N), flags, ws.data_ptr(), ws.numel(), _stream(vol.device)),
           "bf_gp_volume_forward")
    if check:
        st = status(ws, vol.device)
        if st != BF_OK:
            raise BfError(st, "bf_gp_volume_forward (device status)")
    return out


def degree_for(xmax, eps=1e-3):
    """Smallest even degree whose Gauss-polynomial weights are within eps of the
    exact range weights for centred intensities |x| <= xmax (see bfgp.h)."""
    n = bf_gp_degree_for(float(xmax), float(eps))
    if n < 0:
        raise BfError(n, "bf_gp_degree_for")
    return int(n)


def status(ws, device=None):
    """Blocking: the device status (BF_OK or BF_ERANGE) of the last call on ws."""
    v = ctypes.c_int(0)
    _check(bf_gp_status(ws.data_ptr(), _stream(device), ctypes.byref(v)), "bf_gp_status")
    return v.value


def direct_forward(img, sigma_s, sigma_r, window=-1, out=None):
    """Eq. (1) evaluated directly on the GPU (the O(sigma_s^2) comparator)."""
    H, W, pitch = _image(img)
    if out is None:
        out = _like(img)
    _check(bf_direct_forward(img.data_ptr(), out.data_ptr(), H, W, pitch, float(sigma_s), float(sigma_r), int(window),
                             _stream(img.device)), "bf_direct_forward")
    return out


def set_fir_crossover(radius):
    _check(bf_gp_set_fir_crossover(int(radius)), "bf_gp_set_fir_crossover")


def get_fir_crossover():
    return int(bf_gp_get_fir_crossover())


def set_iir_tuning(band_rows=0, col_groups=0, row_groups=0):
    """Overrides the IIR launch shape process-wide (0 = automatic)."""
    _check(bf_gp_set_iir_tuning(int(band_rows), int(col_groups), int(row_groups)), "bf_gp_set_iir_tuning")


def iir_shape(H, W, N=20):
    """dict(band_rows, col_groups, row_chunk, row_threads, row_groups) for an image."""
    v = (ctypes.c_int * 5)()
    _check(bf_gp_iir_shape(int(H), int(W), int(N), v), "bf_gp_iir_shape")
    return dict(zip(("band_rows", "col_groups", "row_chunk", "row_threads", "row_groups"), list(v)))


def profile_enable(on=True):
    """Starts (on=True, resetting the record) or stops per-kernel event timing."""
    _check(bf_profile_enable(1 if on else 0), "bf_profile_enable")


def profile_collect(max_names=64, with_threads=False):
    """{kernel name: (launches, total ms)} for the launches recorded so far
    (with_threads: (launches, total ms, grid size in threads of the last launch))."""
    names = (ctypes.c_char_p * max_names)()
    counts = (ctypes.c_int * max_names)()
    total = (ctypes.c_double * max_names)()
    threads = (ctypes.c_longlong * max_names)()
    n = bf_profile_collect(max_names, names, counts, total, threads)
    if n < 0:
        raise BfError(n, "bf_profile_collect")
    if with_threads:
        return {names[i].decode(): (counts[i], total[i], threads[i]) for i in range(n)}
    return {names[i].decode(): (counts[i], total[i]) for i in range(n)}


# --------------------------------------------------------------------------
# backward and autograd
# --------------------------------------------------------------------------

def saved_buffer(H, W, device="cuda"):
    """Buffer for what the backward pass needs from the forward (16 B/pixel)."""
    return torch.empty(16 * H * W, dtype=torch.uint8, device=device)


def backward_workspace(H, W, N, sigma_s, spatial="auto", device="cuda"):
    n = int(bf_gp_backward_workspace_bytes(int(H), int(W), int(N), float(sigma_s), _flags(spatial)))
    return torch.empty(max(n, 256), dtype=torch.uint8, device=device)


def gp_backward(img, grad_out, saved, sigma_s, sigma_r, N=20, spatial="auto", center="mean", grad_img=True,
                ws=None):
    """Adjoint of gp_forward.  Returns (dL/dimg or None, dL/dlog sigma_s, dL/dlog sigma_r) with the scalar
    gradients as float64 CUDA tensors of shape (1,).  ``saved`` must come from a gp_forward call in the same
    spatial mode (FIR or IIR; AUTO resolves the same way for the same image size and sigma_s)."""
    H, W, pitch = _image(img)
    gh, gw, gp = _image(grad_out, "grad_out")
    if (gh, gw, gp) != (H, W, pitch):
        raise ValueError("grad_out must have the shape and row stride of img")
    gi = _like(img) if grad_img else None
    gs = torch.zeros(1, dtype=torch.float64, device=img.device)
    gr = torch.zeros(1, dtype=torch.float64, device=img.device)
    if ws is None:
        ws = backward_workspace(H, W, N, sigma_s, spatial, img.device)
    _check(bf_gp_backward(img.data_ptr(), grad_out.data_ptr(), saved.data_ptr(), H, W, pitch, float(sigma_s),
                          float(sigma_r), int(N), _flags(spatial, center), gi.data_ptr() if gi is not None else None,
                          gs.data_ptr(), gr.data_ptr(), ws.data_ptr(), ws.numel(), _stream(img.device)),
           "bf_gp_backward")
    return gi, gs, gr


def _stack(t, name="img"):
    """(B, H, W) float32 CUDA tensor with unit column stride: (B, H, W, pitch, image stride)."""
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float32 or not t.is_cuda:
        raise TypeError(f"{name} must be a float32 CUDA tensor")
    if t.dim() != 3:
        raise ValueError(f"{name} must be 3-D (B, H, W)")
    if t.stride(2) != 1:
        raise ValueError(f"{name} must have unit column stride")
    B, H, W = t.shape
    return B, H, W, t.stride(1), t.stride(0) if B > 1 else H * t.stride(1)


def gp_forward_stacked(imgs, sigma_s, sigma_r, N=20, spatial="auto", center="mean", out=None, saved=None, ws=None):
    """GP filter of B images of one size (B, H, W) with one (sigma_s, sigma_r, N), one launch per stage over all
    images (bf_gp_forward_stacked); each image's output equals a single gp_forward call's.  ``saved`` (uint8 CUDA
    tensor of B * 16 * H * W bytes) receives what ``gp_backward_stacked`` needs."""
    B, H, W, pitch, stride = _stack(imgs)
    if out is None:
        out = _like(imgs)
    elif _stack(out, "out") != (B, H, W, pitch, stride):
        raise ValueError("out must have the shape and strides of imgs")
    flags = _flags(spatial, center)
    if ws is None:
        n = int(bf_gp_forward_stacked_workspace_bytes(B, H, W, int(N), float(sigma_s), flags))
        ws = torch.empty(max(n, 256), dtype=torch.uint8, device=imgs.device)
    sp = None
    if saved is not None:
        if saved.numel() * saved.element_size() < 16 * B * H * W:
            raise ValueError("saved buffer too small")
        sp = saved.data_ptr()
    _check(bf_gp_forward_stacked(imgs.data_ptr(), out.data_ptr(), B, H, W, pitch, stride, float(sigma_s),
                                 float(sigma_r), int(N), flags, sp, ws.data_ptr(), ws.numel(), _stream(imgs.device)),
           "bf_gp_forward_stacked")
    return out


def gp_backward_stacked(imgs, grad_out, saved, sigma_s, sigma_r, N=20, spatial="auto", center="mean",
                        grad_img=True, ws=None):
    """Adjoint of gp_forward_stacked (bf_gp_backward_stacked).  Returns (dL/dimgs or None, dL/dlog sigma_s,
    dL/dlog sigma_r) with the scalar gradients per image as float64 CUDA tensors of shape (B,)."""
    B, H, W, pitch, stride = _stack(imgs)
    if _stack(grad_out, "grad_out") != (B, H, W, pitch, stride):
        raise ValueError("grad_out must have the shape and strides of imgs")
    gi = _like(imgs) if grad_img else None
    gs = torch.zeros(B, dtype=torch.float64, device=imgs.device)
    gr = torch.zeros(B, dtype=torch.float64, device=imgs.device)
    flags = _flags(spatial, center)
    if ws is None:
        n = int(bf_gp_backward_stacked_workspace_bytes(B, H, W, int(N), float(sigma_s), flags))
        ws = torch.empty(max(n, 256), dtype=torch.uint8, device=imgs.device)
    _check(bf_gp_backward_stacked(imgs.data_ptr(), grad_out.data_ptr(), saved.data_ptr(), B, H, W, pitch, stride,
                                  float(sigma_s), float(sigma_r), int(N), flags,
                                  gi.data_ptr() if gi is not None else None, gs.data_ptr(), gr.data_ptr(),
                                  ws.data_ptr(), ws.numel(), _stream(imgs.device)), "bf_gp_backward_stacked")
    return gi, gs, gr


class GPFilterFn(torch.autograd.Function):
    """GP bilateral filter with learnable log sigma_s and log sigma_r.

    forward(img (H, W) or (B, H, W) float32 CUDA, log_ss, log_sr, N, spatial, center).
    Both passes run in the library's kernels, a batch as one launch per stage
    over all its images (the stacked calls).  The spatial mode is resolved
    once per call (AUTO: by image size and sigma_s) and used by both passes;
    in the FIR mode the radius ceil(3 sigma_s) is held fixed when
    differentiating in sigma_s, in the IIR mode the recursive kernel is
    differentiated exactly.  The sigmas are read on the host (one
    device-to-host copy when they are tensors); their gradients are the sums
    of the per-image ones."""

    @staticmethod
    def forward(ctx, img, log_ss, log_sr, N=20, spatial="auto", center="mean"):
        ss = math.exp(float(log_ss))
        sr = math.exp(float(log_sr))
        batch = img if img.dim() == 3 else img.unsqueeze(0)
        if batch.stride(2) != 1:
            batch = batch.contiguous()
        B, H, W = batch.shape
        spatial = resolve_spatial(ss, spatial, shape=(H, W))
        saved = torch.empty(B, 16 * H * W, dtype=torch.uint8, device=img.device)
        out = gp_forward_stacked(batch, ss, sr, N, spatial=spatial, center=center, saved=saved)
        ctx.save_for_backward(batch, saved)
        shp = lambda v: (v.shape, v.dtype) if isinstance(v, torch.Tensor) else None
        ctx.params = (ss, sr, int(N), spatial, center, img.dim(), shp(log_ss), shp(log_sr))
        return out if img.dim() == 3 else out[0]

    @staticmethod
    def backward(ctx, grad_out):
        batch, saved = ctx.saved_tensors
        ss, sr, N, spatial, center, dim, t_ss, t_sr = ctx.params
        g = grad_out if grad_out.dim() == 3 else grad_out.unsqueeze(0)
        if g.stride() != batch.stride():
            g = _like(batch).copy_(g)
        gimg, gs, gr = gp_backward_stacked(batch, g, saved, ss, sr, N, spatial, center)
        gimg = gimg if dim == 3 else gimg[0]
        gss = gs.sum().to(t_ss[1]).reshape(t_ss[0]) if t_ss else None
        gsr = gr.sum().to(t_sr[1]).reshape(t_sr[0]) if t_sr else None
        return gimg, gss, gsr, None, None, None


def gp_filter(img, log_ss, log_sr, N=20, spatial="auto", center="mean"):
    """Differentiable GP bilateral filter (see GPFilterFn)."""
    return GPFilterFn.apply(img, log_ss, log_sr, N, spatial, center)


# --------------------------------------------------------------------------
# batched forward
# --------------------------------------------------------------------------

class BatchPlan:
    """Many images of uneven size, each with its own sigma_s and sigma_r,
    filtered by one sequence of grouped per-stage launches (statistics, FIR
    tiles by radius class, the recursive passes, row passes by workgroup
    size), each launch covering every image of the batch that takes part in
    that stage, with one workgroup per work item.  The plan owns its device
    workspace; `run()` enqueues the launches on the current stream and
    `graph()` captures them into a HIP graph for replay."""

    def __init__(self, imgs, sigmas_s, sigmas_r, N=20, outs=None, spatial="auto", center="mean"):
        n = len(imgs)
        if not (len(sigmas_s) == len(sigmas_r) == n) or n == 0:
            raise ValueError("one sigma_s and one sigma_r per image")
        self.imgs = list(imgs)
        self.outs = list(outs) if outs is not None else [_like(x) for x in self.imgs]
        items = (BfGpItem * n)()
        for i, (x, o) in enumerate(zip(self.imgs, self.outs)):
            H, W, pitch = _image(x)
            if _image(o, "out") != (H, W, pitch):
                raise ValueError("each output must match its image's shape and row stride")
            items[i] = BfGpItem(x.data_ptr(), o.data_ptr(), H, W, pitch, float(sigmas_s[i]), float(sigmas_r[i]),
                                int(N))
        self._plan = ctypes.c_void_p()
        _check(bf_gp_plan_batched(items, n, _flags(spatial, center), ctypes.byref(self._plan)), "bf_gp_plan_batched")
        nbytes = int(bf_gp_plan_workspace_bytes(self._plan))
        self.device = self.imgs[0].device
        self.ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=self.device)
        _check(bf_gp_plan_upload(self._plan, self.ws.data_ptr(), self.ws.numel(), _stream(self.device)),
               "bf_gp_plan_upload")

    def run(self):
        _check(bf_gp_forward_batched(self._plan, self.ws.data_ptr(), self.ws.numel(), _stream(self.device)),
               "bf_gp_forward_batched")
        return self.outs

    def graph(self):
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.run()
        return g

    def __del__(self):
        plan = getattr(self, "_plan", None)
        free = bf_gp_plan_free  # None once the interpreter tears the module down
        if plan is not None and plan.value and free is not None:
            free(plan)
            self._plan = None
