"""MI355X (gfx950) p-norm (max, x) product and APSP estimate.

A thin binding over ``libmaxtimes.so`` (C ABI in ``include/maxtimes.h``):
argument marshalling only.  Every step of the computation runs in the
library's HIP kernels; PyTorch supplies device memory and the stream.
There is no CPU fallback: when the library is missing, every call raises.

Method: Serang, "Fast Computation on Semirings Isomorphic to (x, max) on R+"
(arXiv 1511.05690) -- Alg. 5 with the scaled ring call of Sec. 2.1 for the
product, Sec. 2.2 for all-pairs shortest paths.

    C = estimate(A, B, P=(1, 2, 4, ..., 64), path="bf16")   # C ~ max_k A_ik B_kj
    D = apsp(W, s=1.0, P=..., path="fp64")                  # shortest distances
    z = maxconv(x, y, P=(1, 2, 4, ..., 64))                 # z ~ max_i x_i y_(t-i)
    v, i, j = xy_topk(x, y, k)                              # top k of x_i + y_j
"""

import ctypes
import os

import torch

__all__ = [
    "MaxTimesError", "load_library", "library_path", "estimate", "estimate_backward", "apsp",
    "workspace_size", "workspace_map", "backward_workspace_size", "apsp_workspace_size", "exact", "timing_enable",
    "timing_reset", "timing_read", "timing_work", "timing_span", "set_tail_threshold", "tail_threshold",
    "set_small_product_limit", "small_product_limit",
    "set_search_start", "search_start", "apsp_exact_rows", "apsp_affine_correct", "maxconv", "maxconv_exact",
    "maxconv_workspace_size", "xy_topk", "xy_topk_workspace_size", "XY_FAMILY", "pfamily", "PSTAR_NONE", "PATHS",
]

PSTAR_NONE = 255
MAX_P = 32
# 24 powers up to 4096 (Sec. 3 runs the x + y top k with |P| = 24, p*_max = 4096)
XY_FAMILY = (1, 2, 3, 4, 6, 8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512, 768, 1024, 1536, 2048,
             3072, 4096)
PATHS = {"fp64": 0, "bf16": 1}
F32, F64 = 0, 1
FLAG_VALIDATE, FLAG_NORM_CORRECT, FLAG_CLAMP, FLAG_RAW_OUTPUT, FLAG_PROJECT_R1, FLAG_PROJECT_R2 = 1, 2, 4, 8, 16, 32
FLAG_XY_PAIRED = 64
FLAG_BALANCE = 128
NOALLOC_SCRATCH_BYTES = 64 << 20  # MT_NOALLOC_SCRATCH_BYTES
PROJECTIONS = {None: 0, "r1": FLAG_PROJECT_R1, "r2": FLAG_PROJECT_R2}
STATUS = {0: "MT_OK", 1: "MT_ERR_INVALID_ARG", 2: "MT_ERR_DOMAIN", 3: "MT_ERR_WORKSPACE",
          4: "MT_ERR_DEVICE", 5: "MT_ERR_UNSUPPORTED"}

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libmaxtimes.so")
_lib = None


class MaxTimesError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


class _WorkspaceMap(ctypes.Structure):
    _fields_ = [
        ("r_offset", ctypes.c_size_t), ("c_offset", ctypes.c_size_t),
        ("a_planes_offset", ctypes.c_size_t), ("b_planes_offset", ctypes.c_size_t),
        ("m_pad", ctypes.c_int64), ("n_pad", ctypes.c_int64), ("k_pad", ctypes.c_int64),
        ("n_planes", ctypes.c_int32), ("elem_bytes", ctypes.c_int32), ("n_powers", ctypes.c_int32),
        ("power", ctypes.c_int32 * 32), ("first_plane", ctypes.c_int32 * 32), ("split", ctypes.c_int32 * 32),
    ]


class _Options(ctypes.Structure):
    _fields_ = [
        ("p_family", ctypes.POINTER(ctypes.c_int32)),
        ("n_p", ctypes.c_int32),
        ("path", ctypes.c_int32),
        ("tau", ctypes.c_double),
        ("split_max_p", ctypes.c_int32),
        ("flags", ctypes.c_uint32),
    ]


def library_path():
    return _LIB_PATH


def load_library():
    """Load libmaxtimes.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise MaxTimesError(-1, f"{_LIB_PATH} is missing: build it with "
                                "`python -m paper_1511_05690_amd.build`")
    lib = ctypes.CDLL(_LIB_PATH)
    i64, vp, sz = ctypes.c_int64, ctypes.c_void_p, ctypes.c_size_t
    opt = ctypes.POINTER(_Options)
    sig = {
        "maxtimes_workspace_size": [i64, i64, i64, i64, opt, ctypes.POINTER(sz)],
        "maxtimes_workspace_map": [i64, i64, i64, i64, opt, ctypes.POINTER(_WorkspaceMap)],
        "maxtimes_estimate": [vp, vp, ctypes.c_int, i64, i64, i64, i64, opt, vp, vp, vp, sz, vp],
        "maxtimes_estimate_noalloc": [vp, vp, ctypes.c_int, i64, i64, i64, i64, opt, vp, vp, vp],
        "maxtimes_backward_workspace_size": [i64, i64, i64, i64, opt, ctypes.POINTER(sz)],
        "maxtimes_estimate_backward": [vp, vp, vp, vp, vp, ctypes.c_int, i64, i64, i64, i64, opt,
                                       vp, vp, vp, sz, vp],
        "apsp_workspace_size": [i64, opt, ctypes.POINTER(sz)],
        "apsp_estimate": [vp, i64, ctypes.c_double, ctypes.c_int32, opt, vp, ctypes.c_int, vp, vp,
                          sz, vp],
        "maxtimes_exact": [vp, vp, ctypes.c_int, i64, i64, i64, i64, vp, vp],
        "maxconv_workspace_size": [i64, i64, i64, opt, ctypes.POINTER(sz)],
        "maxconv_estimate": [vp, vp, ctypes.c_int, i64, i64, i64, opt, vp, vp, vp, sz, vp],
        "maxconv_exact": [vp, vp, ctypes.c_int, i64, i64, i64, vp, vp],
        "xy_topk_workspace_size": [i64, ctypes.c_int32, opt, ctypes.POINTER(sz)],
        "xy_topk_estimate": [vp, vp, ctypes.c_int, i64, ctypes.c_int32, opt, vp, vp, vp, vp, vp, sz, vp],
        "apsp_exact_rows_workspace_size": [i64, ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)],
        "apsp_exact_rows": [vp, i64, vp, ctypes.c_int32, vp, ctypes.POINTER(i64), vp, ctypes.c_size_t, vp],
        "apsp_affine_workspace_size": [ctypes.POINTER(ctypes.c_size_t)],
        "apsp_affine_correct": [vp, ctypes.c_int, i64, vp, ctypes.c_int32, vp, vp, ctypes.c_int32, vp,
                                ctypes.c_size_t, vp],
        "maxtimes_timing_enable": [ctypes.c_int],
        "maxtimes_timing_reset": [],
        "maxtimes_timing_read": [ctypes.c_char_p, ctypes.POINTER(ctypes.c_double),
                                 ctypes.POINTER(i64)],
        "maxtimes_timing_work": [ctypes.c_char_p, ctypes.POINTER(ctypes.c_double)],
        "maxtimes_timing_span": [ctypes.c_char_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64)],
        "maxtimes_set_tail_threshold": [ctypes.c_int32],
        "maxtimes_tail_threshold": [],
        "maxtimes_set_search_start": [ctypes.c_int32],
        "maxtimes_search_start": [],
        "maxtimes_set_deferred_planes": [ctypes.c_int32],
        "maxtimes_deferred_planes": [],
        "maxtimes_set_small_product_limit": [i64],
        "maxtimes_small_product_limit": [],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    for name in ("maxtimes_status_string", "maxtimes_last_error", "maxtimes_version"):
        f = getattr(lib, name)
        f.restype = ctypes.c_char_p
    lib.maxtimes_small_product_limit.restype = ctypes.c_int64
    lib.maxtimes_status_string.argtypes = [ctypes.c_int]
    lib.maxtimes_last_error.argtypes = []
    lib.maxtimes_version.argtypes = []
    _lib = lib
    return lib


def _check(status):
    if status != 0:
        msg = _lib.maxtimes_last_error().decode()
        raise MaxTimesError(status, msg)


def pfamily(pmax):
    """The powers of two 1, 2, 4, ..., pmax."""
    out, p = [], 1
    while p <= pmax:
        out.append(p)
        p *= 2
    return out


def _options(P, path, tau, split_max_p, flags):
    P = [int(p) for p in P]
    arr = (ctypes.c_int32 * max(1, len(P)))(*P)
    o = _Options()
    o.p_family = ctypes.cast(arr, ctypes.POINTER(ctypes.c_int32))
    o.n_p = len(P)
    o.path = PATHS[path] if isinstance(path, str) else int(path)
    o.tau = -1.0 if tau is None else float(tau)
    o.split_max_p = -1 if split_max_p is None else int(split_max_p)
    o.flags = int(flags)
    o._keep = arr  # keep the array alive with the struct
    return o


def _dtype_code(t):
    if t.dtype == torch.float32:
        return F32
    if t.dtype == torch.float64:
        return F64
    raise TypeError(f"unsupported dtype {t.dtype}")


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() else ctypes.c_void_p(0)


def _shape3(A, B):
    if A.dim() == 2 and B.dim() == 2:
        return 1, A.shape[0], A.shape[1], B.shape[1], False
    if A.dim() == 3 and B.dim() == 3 and A.shape[0] == B.shape[0]:
        return A.shape[0], A.shape[1], A.shape[2], B.shape[2], True
    raise ValueError("A and B must both be 2-D, or 3-D with the same batch size")


def workspace_size(b, m, k, n, P, path="bf16", tau=None, split_max_p=None, flags=0):
    lib = load_library()
    o = _options(P, path, tau, split_max_p, flags)
    out = ctypes.c_size_t(0)
    _check(lib.maxtimes_workspace_size(b, m, k, n, ctypes.byref(o), ctypes.byref(out)))
    return out.value


def workspace_map(b, m, k, n, P, path="bf16", tau=None, split_max_p=None, flags=0):
    """Where estimate() keeps r, c and the power planes in its workspace (a
    dict of byte offsets, padded sizes and the plane of each power)."""
    lib = load_library()
    o = _options(P, path, tau, split_max_p, flags)
    mp = _WorkspaceMap()
    _check(lib.maxtimes_workspace_map(b, m, k, n, ctypes.byref(o), ctypes.byref(mp)))
    q = mp.n_powers
    return {"r": mp.r_offset, "c": mp.c_offset, "a_planes": mp.a_planes_offset, "b_planes": mp.b_planes_offset,
            "m_pad": mp.m_pad, "n_pad": mp.n_pad, "k_pad": mp.k_pad, "n_planes": mp.n_planes,
            "elem_bytes": mp.elem_bytes, "power": list(mp.power[:q]), "first_plane": list(mp.first_plane[:q]),
            "split": [bool(v) for v in mp.split[:q]]}


def backward_workspace_size(b, m, k, n, P, path="bf16", tau=None, split_max_p=None, flags=0):
    lib = load_library()
    o = _options(P, path, tau, split_max_p, flags)
    out = ctypes.c_size_t(0)
    _check(lib.maxtimes_backward_workspace_size(b, m, k, n, ctypes.byref(o), ctypes.byref(out)))
    return out.value


def apsp_workspace_size(n, P, path="fp64", tau=None, split_max_p=None, flags=0):
    lib = load_library()
    o = _options(P, path, tau, split_max_p, flags)
    out = ctypes.c_size_t(0)
    _check(lib.apsp_workspace_size(n, ctypes.byref(o), ctypes.byref(out)))
    return out.value


def _workspace(nbytes, device, workspace):
    if workspace is not None:
        if workspace.numel() * workspace.element_size() < nbytes:
            raise MaxTimesError(3, "workspace tensor too small")
        return workspace
    return torch.empty(max(nbytes, 1), dtype=torch.uint8, device=device)


def _forward(A, B, P, path, tau, split_max_p, flags, want_pstar, workspace=None):
    lib = load_library()
    if not (A.is_cuda and B.is_cuda):
        raise ValueError("A and B must be device tensors")
    if A.dtype != B.dtype:
        raise TypeError("A and B must have the same dtype")
    A = A.contiguous()
    B = B.contiguous()
    b, m, k, n, batched = _shape3(A, B)
    o = _options(P, path, tau, split_max_p, flags)
    need = ctypes.c_size_t(0)
    _check(lib.maxtimes_workspace_size(b, m, k, n, ctypes.byref(o), ctypes.byref(need)))
    ws = _workspace(need.value, A.device, workspace)
    shape = (b, m, n) if batched else (m, n)
    C = torch.empty(shape, dtype=A.dtype, device=A.device)
    ps = torch.empty(shape, dtype=torch.uint8, device=A.device) if want_pstar else None
    _check(lib.maxtimes_estimate(_ptr(A), _ptr(B), _dtype_code(A), b, m, k, n, ctypes.byref(o),
                                 _ptr(C), _ptr(ps), _ptr(ws), need.value, _stream(A.device)))
    return C, ps


def estimate_noalloc(A, B, P=(1, 2, 4, 8, 16, 32, 64), tau=None, path="bf16", split_max_p=None, flags=0,
                     out=None, p_star=None):
    """maxtimes_estimate_noalloc: the estimate on the library's static scratch
    (no workspace).  `out` and `p_star` may be preallocated tensors of the
    output shape (C's dtype is the inputs'); returns (C, p_star)."""
    lib = load_library()
    if not (A.is_cuda and B.is_cuda):
        raise ValueError("A and B must be device tensors")
    if A.dtype != B.dtype:
        raise TypeError("A and B must have the same dtype")
    A = A.contiguous()
    B = B.contiguous()
    b, m, k, n, batched = _shape3(A, B)
    o = _options(P, path, tau, split_max_p, flags)
    shape = (b, m, n) if batched else (m, n)
    C = out if out is not None else torch.empty(shape, dtype=A.dtype, device=A.device)
    ps = p_star if p_star is not None else torch.empty(shape, dtype=torch.uint8, device=A.device)
    if tuple(C.shape) != shape or C.dtype != A.dtype or not C.is_contiguous():
        raise ValueError("out must be a contiguous tensor of the output shape and the inputs' dtype")
    if tuple(ps.shape) != shape or ps.dtype != torch.uint8 or not ps.is_contiguous():
        raise ValueError("p_star must be a contiguous uint8 tensor of the output shape")
    with torch.cuda.device(A.device):
        _check(lib.maxtimes_estimate_noalloc(_ptr(A), _ptr(B), _dtype_code(A), b, m, k, n, ctypes.byref(o),
                                             _ptr(C), _ptr(ps), _stream(A.device)))
    return C, ps


def estimate_backward(A, B, G, C, p_star, P, path="bf16", tau=None, split_max_p=None,
                      need_dA=True, need_dB=True, flags=0):
    """Gradient of sum(G * C) for the estimate with p* held fixed."""
    lib = load_library()
    A, B, G, C, p_star = (t.contiguous() for t in (A, B, G, C, p_star))
    b, m, k, n, batched = _shape3(A, B)
    o = _options(P, path, tau, split_max_p, flags)
    need = ctypes.c_size_t(0)
    _check(lib.maxtimes_backward_workspace_size(b, m, k, n, ctypes.byref(o), ctypes.byref(need)))
    ws = _workspace(need.value, A.device, None)
    dA = torch.empty_like(A) if need_dA else None
    dB = torch.empty_like(B) if need_dB else None
    _check(lib.maxtimes_estimate_backward(_ptr(A), _ptr(B), _ptr(G), _ptr(C), _ptr(p_star),
                                          _dtype_code(A), b, m, k, n, ctypes.byref(o), _ptr(dA),
                                          _ptr(dB), _ptr(ws), need.value, _stream(A.device)))
    return dA, dB


# On the BF16 path the differentiable forward splits every power into hi + lo:
# the adjoint raises C' to the power 1 - p, which carries the forward's
# relative error in S undamped, so S must be accurate to about 1e-5.
SPLIT_ALL = 4096


class _EstimateFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, A, B, P, path, tau, split_max_p, flags):
        fwd_split = SPLIT_ALL if (path == "bf16" and split_max_p is None) else split_max_p
        C, ps = _forward(A, B, P, path, tau, fwd_split, flags, True)
        ctx.save_for_backward(A, B, C, ps)
        ctx.cfg = (tuple(P), path, tau, split_max_p, flags)
        ctx.mark_non_differentiable(ps)
        return C, ps

    @staticmethod
    def backward(ctx, gC, gps):
        A, B, C, ps = ctx.saved_tensors
        P, path, tau, split_max_p, flags = ctx.cfg
        dA, dB = estimate_backward(A, B, gC, C, ps, P, path, tau, split_max_p,
                                   ctx.needs_input_grad[0], ctx.needs_input_grad[1], flags)
        return dA, dB, None, None, None, None, None


def _projection_flag(projection):
    if projection not in PROJECTIONS:
        raise ValueError(f"projection must be one of {sorted(PROJECTIONS, key=str)}")
    return PROJECTIONS[projection]


def estimate(A, B, P=(1, 2, 4, 8, 16, 32, 64), tau=None, path="bf16", split_max_p=None,
             norm_correct=False, clamp=False, validate=False, return_pstar=False, workspace=None,
             projection=None, balance=False):
    """Estimate C_ij = max_k A_ik B_kj for nonnegative A (.., m, k), B (.., k, n).

    path "bf16": BF16 MFMA ring products with hi/lo split for p <= split_max_p;
    path "fp64": FP64 MFMA ring products.  tau None = the path default.
    projection None: the plain root S_{p*}^(1/p*); "r1": the r = 1
    projection (S_{p*} / S_{p_lo})^(1/(p* - p_lo)) (MT_FLAG_PROJECT_R1);
    "r2": the r = 2 projection from S at p*/4, p*/2, 3p*/4, p*
    (MT_FLAG_PROJECT_R2, FP64 path only).
    balance: the estimate of (A D, D^-1 B) with the inner-index balancing
    factors d_k = sqrt(max_j B_kj / max_i A_ik) (MT_FLAG_BALANCE).
    Differentiable (p* held fixed) when A or B requires grad (plain root only).
    """
    flags = (FLAG_VALIDATE if validate else 0) | (FLAG_NORM_CORRECT if norm_correct else 0) | \
        (FLAG_CLAMP if clamp else 0) | _projection_flag(projection) | (FLAG_BALANCE if balance else 0)
    if torch.is_grad_enabled() and (A.requires_grad or B.requires_grad):
        if projection is not None:
            raise ValueError("the projections have no backward; use projection=None for gradients")
        C, ps = _EstimateFn.apply(A, B, list(P), path, tau, split_max_p, flags)
    else:
        C, ps = _forward(A, B, P, path, tau, split_max_p, flags, return_pstar, workspace)
    return (C, ps) if return_pstar else C


def apsp(W, s=1.0, P=None, path="fp64", n_squarings=-1, tau=None, split_max_p=None,
         out_dtype=torch.float32, raw=False, validate=False, return_pstar=False, workspace=None,
         projection=None):
    """Estimated all-pairs shortest distances of the n x n FP32 weight matrix W
    (+inf = no edge).  raw=True returns the (x, max) matrix X instead.
    projection "r1" / "r2" uses that projection in every squaring ("r2":
    FP64 path only)."""
    lib = load_library()
    if P is None:
        P = pfamily(512 if path == "fp64" else 128)
    if W.dtype != torch.float32 or W.dim() != 2 or W.shape[0] != W.shape[1] or not W.is_cuda:
        raise ValueError("W must be a square FP32 device tensor")
    W = W.contiguous()
    n = W.shape[0]
    flags = (FLAG_VALIDATE if validate else 0) | (FLAG_RAW_OUTPUT if raw else 0) | _projection_flag(projection)
    o = _options(P, path, tau, split_max_p, flags)
    need = ctypes.c_size_t(0)
    _check(lib.apsp_workspace_size(n, ctypes.byref(o), ctypes.byref(need)))
    ws = _workspace(need.value, W.device, workspace)
    D = torch.empty((n, n), dtype=out_dtype, device=W.device)
    ps = torch.empty((n, n), dtype=torch.uint8, device=W.device) if return_pstar else None
    _check(lib.apsp_estimate(_ptr(W), n, float(s), int(n_squarings), ctypes.byref(o), _ptr(D),
                             _dtype_code(D), _ptr(ps), _ptr(ws), need.value, _stream(W.device)))
    return (D, ps) if return_pstar else D


def exact(A, B):
    """The exact (max, x) product max_k A_ik B_kj on the GPU's vector ALUs
    (products rounded once in the input precision)."""
    lib = load_library()
    if A.dtype != B.dtype:
        raise TypeError("A and B must have the same dtype")
    A = A.contiguous()
    B = B.contiguous()
    b, m, k, n, batched = _shape3(A, B)
    E = torch.empty((b, m, n) if batched else (m, n), dtype=A.dtype, device=A.device)
    _check(lib.maxtimes_exact(_ptr(A), _ptr(B), _dtype_code(A), b, m, k, n, _ptr(E), _stream(A.device)))
    return E


def _conv_shapes(x, y):
    if not (x.is_cuda and y.is_cuda):
        raise ValueError("x and y must be device tensors")
    if x.dtype != y.dtype:
        raise TypeError("x and y must have the same dtype")
    if x.dim() == 1 and y.dim() == 1:
        return 1, x.shape[0], y.shape[0], False
    if x.dim() == 2 and y.dim() == 2 and x.shape[0] == y.shape[0]:
        return x.shape[0], x.shape[1], y.shape[1], True
    raise ValueError("x and y must both be 1-D, or 2-D with the same batch size")


def maxconv(x, y, P=(1, 2, 4, 8, 16, 32, 64), tau=None, return_pstar=False, workspace=None):
    """Estimate the max-convolution z[t] = max_i x[i] y[t - i] of nonnegative
    x (.., n) and y (.., m) by FFT convolutions of x'^p and y'^p (FP64; one
    workgroup per batch row in LDS up to n + m - 1 = 4096, global buffers up
    to 16384); tau None = 1e-12."""
    lib = load_library()
    b, n, m, batched = _conv_shapes(x, y)
    x = x.contiguous()
    y = y.contiguous()
    o = _options(P, "fp64", tau, None, 0)
    need = ctypes.c_size_t(0)
    _check(lib.maxconv_workspace_size(b, n, m, ctypes.byref(o), ctypes.byref(need)))
    ws = _workspace(need.value, x.device, workspace) if need.value else None
    L = n + m - 1 if n and m else 0
    shape = (b, L) if batched else (L,)
    z = torch.empty(shape, dtype=x.dtype, device=x.device)
    ps = torch.empty(shape, dtype=torch.uint8, device=x.device) if return_pstar else None
    _check(lib.maxconv_estimate(_ptr(x), _ptr(y), _dtype_code(x), b, n, m, ctypes.byref(o), _ptr(z), _ptr(ps),
                                _ptr(ws), need.value, _stream(x.device)))
    return (z, ps) if return_pstar else z


def maxconv_exact(x, y):
    """The exact max-convolution max_i x[i] y[t - i] on the GPU (products
    rounded once in the input precision)."""
    lib = load_library()
    b, n, m, batched = _conv_shapes(x, y)
    x = x.contiguous()
    y = y.contiguous()
    L = n + m - 1 if n and m else 0
    z = torch.empty((b, L) if batched else (L,), dtype=x.dtype, device=x.device)
    _check(lib.maxconv_exact(_ptr(x), _ptr(y), _dtype_code(x), b, n, m, _ptr(z), _stream(x.device)))
    return z


def maxconv_workspace_size(b, n, m, P=(1, 2, 4, 8, 16, 32, 64), tau=None):
    lib = load_library()
    o = _options(P, "fp64", tau, None, 0)
    out = ctypes.c_size_t(0)
    _check(lib.maxconv_workspace_size(b, n, m, ctypes.byref(o), ctypes.byref(out)))
    return out.value


def xy_topk_workspace_size(n, k, P=XY_FAMILY, tau=None, paired=False):
    lib = load_library()
    o = _options(P, "fp64", tau, None, FLAG_XY_PAIRED if paired else 0)
    out = ctypes.c_size_t(0)
    _check(lib.xy_topk_workspace_size(n, k, ctypes.byref(o), ctypes.byref(out)))
    return out.value


def xy_topk(x, y, k, P=XY_FAMILY, tau=None, return_diag=False, paired=False):
    """Estimate the k largest x_i + y_j (x, y: 1-D device tensors of the same
    length n <= 8192) and their indices by the NormQueue of Sec. 2.3 (FFT ring
    results in FP64, a second run on y reversed for the indices).  Returns
    (values FP64, i int32, j int32[, diag]); i = j = -1 where the two runs do
    not give a pair in the grid.  paired=True runs the two queues in lockstep
    (Discussion): a rank whose pair is accurate reports x_i + y_j exactly and
    is subtracted exactly; k <= 4096."""
    lib = load_library()
    if not (x.is_cuda and y.is_cuda) or x.dim() != 1 or y.dim() != 1 or x.shape != y.shape:
        raise ValueError("x and y must be 1-D device tensors of the same length")
    if x.dtype != y.dtype:
        raise TypeError("x and y must have the same dtype")
    x = x.contiguous()
    y = y.contiguous()
    n = x.shape[0]
    o = _options(P, "fp64", tau, None, FLAG_XY_PAIRED if paired else 0)
    need = ctypes.c_size_t(0)
    _check(lib.xy_topk_workspace_size(n, int(k), ctypes.byref(o), ctypes.byref(need)))
    ws = _workspace(need.value, x.device, None)
    values = torch.empty(k, dtype=torch.float64, device=x.device)
    ii = torch.empty(k, dtype=torch.int32, device=x.device)
    jj = torch.empty(k, dtype=torch.int32, device=x.device)
    dg = torch.empty(k, dtype=torch.int32, device=x.device)
    _check(lib.xy_topk_estimate(_ptr(x), _ptr(y), _dtype_code(x), n, int(k), ctypes.byref(o), _ptr(values),
                                _ptr(dg), _ptr(ii), _ptr(jj), _ptr(ws), need.value, _stream(x.device)))
    return (values, ii, jj, dg) if return_diag else (values, ii, jj)


def apsp_exact_rows(W, sources):
    """Exact shortest-path distances (FP64, shape len(sources) x n) from each
    vertex in ``sources`` on the dense FP32 weights W (n x n, +inf = no
    edge), by Bellman-Ford on the GPU.  Returns (D_rows, rounds).
    Synchronous."""
    lib = load_library()
    if W.dtype != torch.float32 or W.dim() != 2 or W.shape[0] != W.shape[1]:
        raise TypeError("W must be a square float32 matrix")
    W = W.contiguous()
    n = W.shape[0]
    src = torch.as_tensor(sources, dtype=torch.int32, device=W.device).contiguous()
    nsrc = src.numel()
    D = torch.empty((nsrc, n), dtype=torch.float64, device=W.device)
    nb = ctypes.c_size_t(0)
    _check(lib.apsp_exact_rows_workspace_size(n, nsrc, ctypes.byref(nb)))
    ws = _workspace(nb.value, W.device, None)
    rounds = ctypes.c_int64(0)
    _check(lib.apsp_exact_rows(_ptr(W), n, _ptr(src), nsrc, _ptr(D), ctypes.byref(rounds), _ptr(ws), nb.value,
                               _stream(W.device)))
    return D, rounds.value


def apsp_affine_correct(D, sources, exact_rows, apply=True):
    """Affine correction of an APSP estimate D (n x n, FP32 or FP64, device):
    least squares exact = a D + b over the pairs (sources[q], v) with both
    distances finite, then (apply) D <- max(0, a D + b) in place on finite
    off-diagonal entries.  Returns the device tensor (a, b)."""
    lib = load_library()
    if D.dim() != 2 or D.shape[0] != D.shape[1] or not D.is_contiguous():
        raise TypeError("D must be a contiguous square matrix")
    n = D.shape[0]
    src = torch.as_tensor(sources, dtype=torch.int32, device=D.device).contiguous()
    ex = exact_rows.to(torch.float64).contiguous()
    if ex.shape != (src.numel(), n):
        raise ValueError("exact_rows must be len(sources) x n")
    ab = torch.empty(2, dtype=torch.float64, device=D.device)
    nb = ctypes.c_size_t(0)
    _check(lib.apsp_affine_workspace_size(ctypes.byref(nb)))
    ws = _workspace(nb.value, D.device, None)
    _check(lib.apsp_affine_correct(_ptr(D), _dtype_code(D), n, _ptr(src), src.numel(), _ptr(ex), _ptr(ab),
                                   1 if apply else 0, _ptr(ws), nb.value, _stream(D.device)))
    return ab


def timing_enable(on=True):
    _check(load_library().maxtimes_timing_enable(1 if on else 0))


def timing_reset():
    _check(load_library().maxtimes_timing_reset())


def timing_read(prefix):
    """(total milliseconds, launches) of the library's kernels whose name
    starts with ``prefix``, from HIP events recorded on the launch stream."""
    ms = ctypes.c_double(0.0)
    cnt = ctypes.c_int64(0)
    _check(load_library().maxtimes_timing_read(prefix.encode(), ctypes.byref(ms), ctypes.byref(cnt)))
    return ms.value, cnt.value


def set_tail_threshold(max_entries):
    """A forward tile with at most ``max_entries`` undecided entries hands
    them to the sparse-tail kernel (0: never).  Process-wide."""
    _check(load_library().maxtimes_set_tail_threshold(int(max_entries)))


def tail_threshold():
    return int(load_library().maxtimes_tail_threshold())


def set_search_start(entry):
    """Start the forward p search at the ``entry``-th largest p (0: the
    largest), go down to the smallest p, then up for the entries still stable
    at the start; -1 (the default): a pilot on sampled entries chooses per
    product.  Same p* as the top-down search up to entries whose S lies
    within rounding of tau.  Process-wide."""
    _check(load_library().maxtimes_set_search_start(int(entry)))


def search_start():
    return int(load_library().maxtimes_search_start())


def set_deferred_planes(on):
    """Plain products steered by the pilot: write the power planes of the
    two smallest p (BF16 path; FP64 path: all but the three largest p) only
    once some entry needs them (True, the default), running again the tiles
    that reached them first; False writes every plane up front.
    Process-wide."""
    _check(load_library().maxtimes_set_deferred_planes(1 if on else 0))


def deferred_planes():
    return bool(load_library().maxtimes_deferred_planes())


def set_small_product_limit(max_work):
    """FP64-path products with b m k n <= ``max_work`` (and no projection,
    balancing or domain check) run as one kernel; 0: never.  Process-wide."""
    _check(load_library().maxtimes_set_small_product_limit(int(max_work)))


def small_product_limit():
    return int(load_library().maxtimes_small_product_limit())


def timing_work(prefix):
    """Work executed by the timed launches whose kernel name starts with
    ``prefix``: MFMA flops of the p-family GEMMs (tiles stop once every entry
    has its p*); 10 N log2 N flops per pair and p visited for the
    max-convolution."""
    fl = ctypes.c_double(0.0)
    _check(load_library().maxtimes_timing_work(prefix.encode(), ctypes.byref(fl)))
    return fl.value


def timing_span(prefix):
    """(total milliseconds, launches) of the timed launches whose kernel name
    starts with ``prefix``, measured on the device: from the first workgroup's
    start to the last workgroup's end on the device's real-time counter (the
    kernels that count work only)."""
    ms = ctypes.c_double(0.0)
    cnt = ctypes.c_int64(0)
    _check(load_library().maxtimes_timing_span(prefix.encode(), ctypes.byref(ms), ctypes.byref(cnt)))
    return ms.value, cnt.value
