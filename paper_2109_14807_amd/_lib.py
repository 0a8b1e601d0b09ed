"""ctypes binding of libglint (argument marshalling only).

Every function here has the name of the C entry point it calls and takes torch
tensors (device memory) or plain numbers.  No arithmetic of the method happens
in Python: each call validates tensor placement, dtype and contiguity, passes
raw device pointers and the current HIP stream, and raises GlintError on a
non-OK status.  The shared library must have been built in-tree
(``python -m paper_2109_14807_amd.build``); there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libglint.so")

GLINT_F64, GLINT_F32, GLINT_BF16, GLINT_FP8E4M3 = 0, 1, 2, 3
NOALLOC_SCRATCH_BYTES = 48 << 20     # GLINT_NOALLOC_SCRATCH_BYTES of glint.h

TORCH_OF = {
    GLINT_F64: torch.float64,
    GLINT_F32: torch.float32,
    GLINT_BF16: torch.bfloat16,
    GLINT_FP8E4M3: torch.float8_e4m3fn,
}
DTYPE_OF = {v: k for k, v in TORCH_OF.items()}
NAMES = {"f64": GLINT_F64, "f32": GLINT_F32, "bf16": GLINT_BF16, "fp8": GLINT_FP8E4M3}


class GlintError(RuntimeError):
    def __init__(self, fn: str, status: int, detail: str):
        super().__init__(f"{fn} failed with status {status}: {detail}")
        self.status = status
        self.detail = detail


class NdfDesc(ctypes.Structure):
    _fields_ = [("nu", ctypes.c_int32), ("nv", ctypes.c_int32), ("nlevels", ctypes.c_int32),
                ("nbins", ctypes.c_int32), ("sigma", ctypes.c_double)]

    @classmethod
    def make(cls, nu, nv, nlevels, nbins, sigma):
        return cls(int(nu), int(nv), int(nlevels), int(nbins), float(sigma))


class Factors(ctypes.Structure):
    _fields_ = [("R", ctypes.c_int32), ("nu", ctypes.c_int32), ("nv", ctypes.c_int32),
                ("nl", ctypes.c_int32), ("nbins", ctypes.c_int32), ("dtype", ctypes.c_int32),
                ("cum_dtype", ctypes.c_int32), ("U", ctypes.c_void_p), ("V", ctypes.c_void_p),
                ("L", ctypes.c_void_p), ("CS", ctypes.c_void_p), ("CT", ctypes.c_void_p),
                ("scale_U", ctypes.c_void_p), ("scale_V", ctypes.c_void_p),
                ("scale_L", ctypes.c_void_p), ("scale_CS", ctypes.c_void_p),
                ("scale_CT", ctypes.c_void_p)]


class ClusterDesc(ctypes.Structure):
    _fields_ = [("t", ctypes.c_int32), ("cs", ctypes.c_int32), ("R", ctypes.c_int32)]


class Clustered(ctypes.Structure):
    _fields_ = [("t", ctypes.c_int32), ("cs", ctypes.c_int32), ("R", ctypes.c_int32),
                ("nu", ctypes.c_int32), ("nv", ctypes.c_int32), ("nl", ctypes.c_int32),
                ("nbins", ctypes.c_int32), ("CX", ctypes.c_void_p), ("CY", ctypes.c_void_p),
                ("Z", ctypes.c_void_p), ("zidx", ctypes.c_void_p), ("dtype", ctypes.c_int32)]


class Wang(ctypes.Structure):
    _fields_ = [("ntiles", ctypes.c_int32), ("S", ctypes.c_int32), ("m", ctypes.c_int32),
                ("R", ctypes.c_int32), ("nl", ctypes.c_int32), ("nbins", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("edge_to_tile", ctypes.c_uint8 * 16),
                ("U", ctypes.c_void_p), ("V", ctypes.c_void_p), ("L", ctypes.c_void_p),
                ("CS", ctypes.c_void_p), ("CT", ctypes.c_void_p)]


_LIB = None

_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_F32 = ctypes.c_float
_F64 = ctypes.c_double
_SZ = ctypes.c_size_t
_DESC = ctypes.POINTER(NdfDesc)
_FAC = ctypes.POINTER(Factors)
_CDESC = ctypes.POINTER(ClusterDesc)
_CLU = ctypes.POINTER(Clustered)
_U64 = ctypes.c_uint64

_SIGS = {
    "glint_status_string": (ctypes.c_char_p, [_I32]),
    "glint_last_error": (ctypes.c_char_p, []),
    "glint_version": (_I32, []),
    "glint_window_radius": (_I32, [_DESC]),
    "glint_texel_bins": (_I32, [_DESC, _P, _P, _P, _P]),
    "glint_build_tensor_workspace": (_SZ, [_DESC]),
    "glint_build_tensor": (_I32, [_DESC, _P, _P, _I32, _I32, _P, _SZ, _P]),
    "glint_build_tensor_noalloc": (_I32, [_DESC, _P, _P, _I32, _I32, _P]),
    "glint_range_bruteforce": (_I32, [_DESC, _P, _P, _I64, _P, _P, _P]),
    "glint_cp_als_workspace": (_SZ, [_DESC, _I32, _I32]),
    "glint_cp_als": (_I32, [_DESC, _P, _I32, _I32, _I32, _F64, _P, _P, _P, _P, _P, _P, _P, _P, _SZ, _P]),
    "glint_mttkrp": (_I32, [_DESC, _P, _I32, _I32, _I32, _P, _P, _P, _P, _P, _P, _P, _SZ, _P]),
    "glint_cp_als_texel_workspace": (_SZ, [_DESC, _I32]),
    "glint_mttkrp_texel": (_I32, [_DESC, _P, _I32, _I32, _P, _P, _P, _P, _P, _P, _P, _SZ, _P]),
    "glint_cp_als_texel": (_I32, [_DESC, _P, _I32, _I32, _F64, _F64, _P, _P, _P, _P, _P, _P, _P,
                                  _P, _SZ, _P]),
    "glint_make_cumulative": (_I32, [_I32, _I32, _P, _I32, _P, _I32, _P, _P]),
    "glint_convert": (_I32, [_I64, _I32, _P, _I32, _P, _I32, _P, _P]),
    "glint_query": (_I32, [_FAC, _I64, _P, _P, _P]),
    "glint_query_grouped": (_I32, [_FAC, _I64, _I32, _P, _P, _P, _P]),
    "glint_query_trilinear": (_I32, [_FAC, _I64, _P, _P, _P, _P]),
    "glint_sample": (_I32, [_FAC, _I64, _P, _P, _P, _P, _P, _P]),
    "glint_query_backward": (_I32, [_FAC, _I64, _P, _P, _P, _P, _P, _P, _P, _P]),
    "glint_cumulative_backward": (_I32, [_I32, _I32, _P, _P, _P]),
    "glint_mse_grad": (_I32, [_I64, _P, _P, _P, _P, _P]),
    "glint_adam_step": (_I32, [_I64, _P, _P, _P, _P, _F32, _F32, _F32, _F32, _I32, _P]),
    "glint_cp_als_clustered": (_I32, [_DESC, _CDESC, _P, _I32, _I32, _U64, _P, _P, _P, _P, _P, _P]),
    "glint_cluster_map_workspace": (_SZ, [_DESC, _CDESC, _I32]),
    "glint_cluster_map_index": (_I32, [_DESC, _CDESC, _P, _I32, _P, _P, _P, _P, _SZ, _P]),
    "glint_cp_als_clustered_map": (_I32, [_DESC, _CDESC, _P, _I32, _I32, _U64, _P, _P, _P, _P, _P, _P, _P,
                                          _SZ, _P]),
    "glint_make_cumulative_batched": (_I32, [_I64, _I32, _I32, _P, _P, _P]),
    "glint_query_clustered": (_I32, [_CLU, _I64, _P, _P, _P]),
    "glint_sample_clustered": (_I32, [_CLU, _I64, _P, _P, _P, _P, _P, _P]),
    "glint_query_sg": (_I32, [_FAC, _I64, _P, _P, _P, _F32, _P, _P, _P]),
    "glint_query_wang": (_I32, [ctypes.POINTER(Wang), _I64, _P, _P, _P]),
    "glint_validate_queries": (_I32, [_FAC, _I64, _P, _P, _P]),
}


def lib():
    """Load libglint.so (raises if it has not been built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2109_14807_amd.build`")
        h = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(h, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = h
    return _LIB


def exported_names():
    return list(_SIGS)


def _check(fn: str, status: int):
    if status != 0:
        detail = lib().glint_last_error().decode(errors="replace")
        raise GlintError(fn, status, detail)


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t, dtype=None, name="tensor"):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be on the GPU")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    return ctypes.c_void_p(t.data_ptr())


def _gdtype(t: torch.Tensor) -> int:
    return _gdtype_of(t.dtype)


def _gdtype_of(dtype: torch.dtype) -> int:
    if dtype not in DTYPE_OF:
        raise TypeError(f"unsupported storage dtype {dtype}")
    return DTYPE_OF[dtype]


# ----------------------------------------------------------------------------
# entry points
# ----------------------------------------------------------------------------

def glint_version() -> int:
    return int(lib().glint_version())


def glint_status_string(s: int) -> str:
    return lib().glint_status_string(int(s)).decode()


def glint_window_radius(desc: NdfDesc) -> int:
    k = int(lib().glint_window_radius(ctypes.byref(desc)))
    if k < 0:
        raise GlintError("glint_window_radius", -1, lib().glint_last_error().decode())
    return k


def glint_texel_bins(desc, nxy, bins, mass, stream=None):
    _check("glint_texel_bins", lib().glint_texel_bins(
        ctypes.byref(desc), _ptr(nxy, torch.float32, "nxy"), _ptr(bins, torch.int32, "bins"),
        _ptr(mass, torch.float64, "mass"), _stream(stream)))


def glint_build_tensor_workspace(desc) -> int:
    return int(lib().glint_build_tensor_workspace(ctypes.byref(desc)))


def glint_build_tensor(desc, nxy, T, direct_levels, workspace, stream=None):
    _check("glint_build_tensor", lib().glint_build_tensor(
        ctypes.byref(desc), _ptr(nxy, torch.float32, "nxy"), _ptr(T, None, "T"), _gdtype(T),
        int(direct_levels), _ptr(workspace, torch.uint8, "workspace"), workspace.numel(),
        _stream(stream)))


def glint_build_tensor_noalloc(desc, nxy, T, direct_levels, stream=None):
    _check("glint_build_tensor_noalloc", lib().glint_build_tensor_noalloc(
        ctypes.byref(desc), _ptr(nxy, torch.float32, "nxy"), _ptr(T, None, "T"), _gdtype(T),
        int(direct_levels), _stream(stream)))


def glint_range_bruteforce(desc, bins, mass, q, out, stream=None):
    _check("glint_range_bruteforce", lib().glint_range_bruteforce(
        ctypes.byref(desc), _ptr(bins, torch.int32, "bins"), _ptr(mass, torch.float64, "mass"),
        q.shape[0], _ptr(q, torch.int32, "q"), _ptr(out, torch.float64, "out"), _stream(stream)))


def glint_cp_als_workspace(desc, R, T_dtype) -> int:
    return int(lib().glint_cp_als_workspace(ctypes.byref(desc), int(R), int(T_dtype)))


def glint_cp_als(desc, T, R, iters, tol, U, V, L, S, Tf, fit_hist, info, workspace, stream=None):
    f64 = torch.float64
    _check("glint_cp_als", lib().glint_cp_als(
        ctypes.byref(desc), _ptr(T, None, "T"), _gdtype(T), int(R), int(iters), float(tol),
        _ptr(U, f64, "U"), _ptr(V, f64, "V"), _ptr(L, f64, "L"), _ptr(S, f64, "S"),
        _ptr(Tf, f64, "Tf"), _ptr(fit_hist, f64, "fit_hist"),
        _ptr(info, torch.int32, "info") if info is not None else None,
        _ptr(workspace, torch.uint8, "workspace"), workspace.numel(), _stream(stream)))


def glint_mttkrp(desc, T, R, mode, U, V, L, S, Tf, M, workspace, stream=None):
    f64 = torch.float64
    _check("glint_mttkrp", lib().glint_mttkrp(
        ctypes.byref(desc), _ptr(T, None, "T"), _gdtype(T), int(R), int(mode),
        _ptr(U, f64, "U"), _ptr(V, f64, "V"), _ptr(L, f64, "L"), _ptr(S, f64, "S"),
        _ptr(Tf, f64, "Tf"), _ptr(M, f64, "M"), _ptr(workspace, torch.uint8, "workspace"),
        workspace.numel(), _stream(stream)))


def glint_cp_als_texel_workspace(desc, R) -> int:
    return int(lib().glint_cp_als_texel_workspace(ctypes.byref(desc), int(R)))


def glint_mttkrp_texel(desc, nxy, R, mode, U, V, L, S, Tf, M, workspace, stream=None):
    f64 = torch.float64
    _check("glint_mttkrp_texel", lib().glint_mttkrp_texel(
        ctypes.byref(desc), _ptr(nxy, torch.float32, "nxy"), int(R), int(mode),
        _ptr(U, f64, "U"), _ptr(V, f64, "V"), _ptr(L, f64, "L"), _ptr(S, f64, "S"),
        _ptr(Tf, f64, "Tf"), _ptr(M, f64, "M"), _ptr(workspace, torch.uint8, "workspace"),
        workspace.numel(), _stream(stream)))


def glint_cp_als_texel(desc, nxy, R, iters, tol, normT2, U, V, L, S, Tf, fit_hist, info,
                       workspace, stream=None):
    f64 = torch.float64
    _check("glint_cp_als_texel", lib().glint_cp_als_texel(
        ctypes.byref(desc), _ptr(nxy, torch.float32, "nxy"), int(R), int(iters), float(tol),
        float(normT2), _ptr(U, f64, "U"), _ptr(V, f64, "V"), _ptr(L, f64, "L"),
        _ptr(S, f64, "S"), _ptr(Tf, f64, "Tf"), _ptr(fit_hist, f64, "fit_hist"),
        _ptr(info, torch.int32, "info") if info is not None else None,
        _ptr(workspace, torch.uint8, "workspace"), workspace.numel(), _stream(stream)))


def glint_make_cumulative(S, C, col_scale=None, stream=None):
    n, R = S.shape
    if tuple(C.shape) != (n + 1, R):
        raise ValueError("C must have shape (n+1, R)")
    _check("glint_make_cumulative", lib().glint_make_cumulative(
        n, R, _ptr(S, None, "S"), _gdtype(S), _ptr(C, None, "C"), _gdtype(C),
        _ptr(col_scale, torch.float32, "col_scale"), _stream(stream)))


def glint_convert(inp, out, col_scale=None, stream=None):
    rows, R = inp.shape
    if tuple(out.shape) != (rows, R):
        raise ValueError("out must have the shape of inp")
    _check("glint_convert", lib().glint_convert(
        rows, R, _ptr(inp, None, "inp"), _gdtype(inp), _ptr(out, None, "out"), _gdtype(out),
        _ptr(col_scale, torch.float32, "col_scale"), _stream(stream)))


def make_factors(U, V, L, CS, CT, scales=None) -> Factors:
    """Factors struct over device tables (tensors must outlive the calls).

    ``scales`` is None or a 5-tuple of per-column FP32 scales (or None) for
    U, V, L, CS, CT."""
    R = U.shape[1]
    for name, t in (("V", V), ("L", L), ("CS", CS), ("CT", CT)):
        if t.shape[1] != R:
            raise ValueError(f"{name} must have {R} columns")
    if U.dtype != V.dtype or U.dtype != L.dtype or CS.dtype != CT.dtype:
        raise TypeError("U, V, L share one dtype and CS, CT another")
    if CS.shape[0] != CT.shape[0]:
        raise ValueError("CS and CT must have the same rows")
    sc = scales if scales is not None else (None,) * 5
    if len(sc) != 5:
        raise ValueError("scales must hold five entries (U, V, L, CS, CT)")
    for t in sc:
        if t is not None and tuple(t.shape) != (R,):
            raise ValueError(f"a scale must have shape ({R},)")
    return Factors(R, U.shape[0], V.shape[0], L.shape[0], CS.shape[0] - 1, _gdtype(U), _gdtype(CS),
                   _ptr(U, None, "U"), _ptr(V, None, "V"), _ptr(L, None, "L"), _ptr(CS, None, "CS"),
                   _ptr(CT, None, "CT"), *[_ptr(t, torch.float32, "scale") for t in sc])


def glint_query(f: Factors, q, out, stream=None):
    _check("glint_query", lib().glint_query(
        ctypes.byref(f), q.shape[0], _ptr(q, torch.int32, "q"), _ptr(out, torch.float32, "out"),
        _stream(stream)))


def glint_query_grouped(f: Factors, uvl, boxes, out, stream=None):
    npts, K = boxes.shape[0], boxes.shape[1]
    _check("glint_query_grouped", lib().glint_query_grouped(
        ctypes.byref(f), npts, K, _ptr(uvl, torch.int32, "uvl"), _ptr(boxes, torch.int32, "boxes"),
        _ptr(out, torch.float32, "out"), _stream(stream)))


def glint_query_trilinear(f: Factors, xyl, boxes, out, stream=None):
    nq = xyl.shape[0]
    if tuple(boxes.shape) != (nq, 4) or tuple(xyl.shape) != (nq, 3):
        raise ValueError("xyl must be [nq][3] and boxes [nq][4]")
    _check("glint_query_trilinear", lib().glint_query_trilinear(
        ctypes.byref(f), nq, _ptr(xyl, torch.float32, "xyl"), _ptr(boxes, torch.int32, "boxes"),
        _ptr(out, torch.float32, "out"), _stream(stream)))


def glint_sample(f: Factors, uvl, rnd, h, pdf, bins, stream=None):
    n = uvl.shape[0]
    if tuple(h.shape) != (n, 2) or tuple(bins.shape) != (n, 2) or pdf.shape[0] != n or rnd.shape[0] != n:
        raise ValueError("shapes: uvl [n][3], rnd [n][log2(N)+2], h [n][2], pdf [n], bins [n][2]")
    _check("glint_sample", lib().glint_sample(
        ctypes.byref(f), n, _ptr(uvl, torch.int32, "uvl"), _ptr(rnd, torch.float32, "rnd"),
        _ptr(h, torch.float32, "h"), _ptr(pdf, torch.float32, "pdf"), _ptr(bins, torch.int32, "bins"),
        _stream(stream)))


def glint_query_backward(f: Factors, q, gout, dU, dV, dL, dCS, dCT, stream=None):
    f32 = torch.float32
    _check("glint_query_backward", lib().glint_query_backward(
        ctypes.byref(f), q.shape[0], _ptr(q, torch.int32, "q"), _ptr(gout, f32, "gout"),
        _ptr(dU, f32, "dU"), _ptr(dV, f32, "dV"), _ptr(dL, f32, "dL"), _ptr(dCS, f32, "dCS"),
        _ptr(dCT, f32, "dCT"), _stream(stream)))


def glint_cumulative_backward(dC, dS, stream=None):
    n, R = dS.shape
    _check("glint_cumulative_backward", lib().glint_cumulative_backward(
        n, R, _ptr(dC, torch.float32, "dC"), _ptr(dS, torch.float32, "dS"), _stream(stream)))


def glint_mse_grad(q, target, gout, loss=None, stream=None):
    _check("glint_mse_grad", lib().glint_mse_grad(
        q.shape[0], _ptr(q, torch.float32, "q"), _ptr(target, torch.float64, "target"),
        _ptr(gout, torch.float32, "gout"), _ptr(loss, torch.float64, "loss"), _stream(stream)))


def glint_adam_step(p, g, m, v, lr, b1, b2, eps, step, stream=None):
    f32 = torch.float32
    _check("glint_adam_step", lib().glint_adam_step(
        p.numel(), _ptr(p, f32, "p"), _ptr(g, f32, "g"), _ptr(m, f32, "m"), _ptr(v, f32, "v"),
        float(lr), float(b1), float(b2), float(eps), int(step), _stream(stream)))


def glint_cp_als_clustered(desc, cd: ClusterDesc, T, iters, seed, X, Y, Z, blank, info, stream=None):
    f32 = torch.float32
    _check("glint_cp_als_clustered", lib().glint_cp_als_clustered(
        ctypes.byref(desc), ctypes.byref(cd), _ptr(T, None, "T"), _gdtype(T), int(iters),
        int(seed) & ((1 << 64) - 1), _ptr(X, f32, "X"), _ptr(Y, f32, "Y"), _ptr(Z, f32, "Z"),
        _ptr(blank, torch.uint8, "blank"), _ptr(info, torch.int32, "info"), _stream(stream)))


def glint_cluster_map_workspace(desc, cd: ClusterDesc, dtype) -> int:
    return int(lib().glint_cluster_map_workspace(ctypes.byref(desc), ctypes.byref(cd), _gdtype_of(dtype)))


def glint_cluster_map_index(desc, cd: ClusterDesc, nxy, dtype, zidx, zbase, info, workspace, stream=None):
    _check("glint_cluster_map_index", lib().glint_cluster_map_index(
        ctypes.byref(desc), ctypes.byref(cd), _ptr(nxy, torch.float32, "nxy"), _gdtype_of(dtype),
        _ptr(zidx, torch.int32, "zidx"), _ptr(zbase, torch.int64, "zbase"), _ptr(info, torch.int32, "info"),
        _ptr(workspace, torch.uint8, "workspace"), workspace.numel(), _stream(stream)))


def glint_cp_als_clustered_map(desc, cd: ClusterDesc, nxy, dtype, iters, seed, zidx, X, Y, Z, blank, info,
                               workspace, stream=None):
    f32 = torch.float32
    _check("glint_cp_als_clustered_map", lib().glint_cp_als_clustered_map(
        ctypes.byref(desc), ctypes.byref(cd), _ptr(nxy, f32, "nxy"), _gdtype_of(dtype), int(iters),
        int(seed) & ((1 << 64) - 1), _ptr(zidx, torch.int32, "zidx"), _ptr(X, f32, "X"), _ptr(Y, f32, "Y"),
        _ptr(Z, f32, "Z"), _ptr(blank, torch.uint8, "blank"), _ptr(info, torch.int32, "info"),
        _ptr(workspace, torch.uint8, "workspace"), workspace.numel(), _stream(stream)))


def glint_make_cumulative_batched(S, C, stream=None):
    nb, n, R = S.shape
    if tuple(C.shape) != (nb, n + 1, R):
        raise ValueError("C must have shape (nbatch, n+1, R)")
    _check("glint_make_cumulative_batched", lib().glint_make_cumulative_batched(
        nb, n, R, _ptr(S, torch.float32, "S"), _ptr(C, torch.float32, "C"), _stream(stream)))


def glint_query_clustered(f: Clustered, q, out, stream=None):
    _check("glint_query_clustered", lib().glint_query_clustered(
        ctypes.byref(f), q.shape[0], _ptr(q, torch.int32, "q"), _ptr(out, torch.float32, "out"),
        _stream(stream)))


def glint_query_sg(f: Factors, uvl, h, sg, eps, q, out, stream=None):
    n = uvl.shape[0]
    if tuple(h.shape) != (n, 2) or tuple(sg.shape) != (n, 2) or tuple(q.shape) != (n, 7) or out.shape[0] != n:
        raise ValueError("shapes: uvl [n][3], h [n][2], sg [n][2] (lambda, A), q [n][7], out [n]")
    _check("glint_query_sg", lib().glint_query_sg(
        ctypes.byref(f), n, _ptr(uvl, torch.int32, "uvl"), _ptr(h, torch.float32, "h"),
        _ptr(sg, torch.float32, "sg"), float(eps), _ptr(q, torch.int32, "q"), _ptr(out, torch.float32, "out"),
        _stream(stream)))


def glint_query_wang(w: Wang, q, out, stream=None):
    _check("glint_query_wang", lib().glint_query_wang(
        ctypes.byref(w), q.shape[0], _ptr(q, torch.int32, "q"), _ptr(out, torch.float32, "out"), _stream(stream)))


def glint_sample_clustered(f: Clustered, uvl, rnd, h, pdf, bins, stream=None):
    n = uvl.shape[0]
    if tuple(h.shape) != (n, 2) or tuple(bins.shape) != (n, 2) or pdf.shape[0] != n or rnd.shape[0] != n:
        raise ValueError("shapes: uvl [n][3], rnd [n][log2(t)+3], h [n][2], pdf [n], bins [n][2]")
    _check("glint_sample_clustered", lib().glint_sample_clustered(
        ctypes.byref(f), n, _ptr(uvl, torch.int32, "uvl"), _ptr(rnd, torch.float32, "rnd"),
        _ptr(h, torch.float32, "h"), _ptr(pdf, torch.float32, "pdf"), _ptr(bins, torch.int32, "bins"),
        _stream(stream)))


def glint_validate_queries(f: Factors, q, nbad, stream=None):
    _check("glint_validate_queries", lib().glint_validate_queries(
        ctypes.byref(f), q.shape[0], _ptr(q, torch.int32, "q"), _ptr(nbad, torch.int64, "nbad"), _stream(stream)))
