"""Python binding of libbltc.so (include/bltc.h): argument marshalling only.

Every step of the treecode runs in the library's own HIP kernels; this module
passes device pointers of torch tensors (float64, contiguous, on the GPU)
and torch's current HIP stream through ctypes, and turns status codes into
BltcError.  If the library has not been built, loading raises: there is no
fallback path.

Point sets are (3, n) float64 tensors (rows x, y, z); weights (3, n); outputs
(odim, m) with odim = 3 (Stokeslet, polynomial) or 6 (rotlet: u then w).
"""
import ctypes
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "lib", "libbltc.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "bltc.h")

KERNELS = {"stokeslet": 0, "rotlet": 1, "full": 2, "poly": 100}
ODIM = {"stokeslet": 3, "rotlet": 6, "full": 6, "poly": 3}
WDIM = {"stokeslet": 3, "rotlet": 3, "full": 6, "poly": 3}
PRECISIONS = {"fp64": 0, "fp32_fp64acc": 1, "fp32_kahan": 2}
STATUS = {0: "OK", 1: "EINVAL", 2: "ENOMEM", 3: "EDEVICE", 4: "ESTATE", 5: "EMODEL"}

_lib = None


class BltcError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"bltc {STATUS.get(status, status)}: {message}")
        self.status = status
        self.message = message


class Options(ctypes.Structure):
    _fields_ = [("size", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("batch_size", ctypes.c_int32), ("order_leaf", ctypes.c_int32),
                ("poly_p", ctypes.c_int32), ("poly_c", ctypes.c_double),
                ("group_max", ctypes.c_int64), ("deg_min", ctypes.c_int32)]


def declared_functions():
    """Names of the functions include/bltc.h declares."""
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|void|const char\*)\s+(bltc_\w+)\s*\(", text, re.M)))


def load():
    """Load libbltc.so (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                           "or python paper_1902_02250_amd/build.py")
    # torch ships its own HIP runtime; load it first so that libbltc binds to
    # the same runtime (one process must not hold two copies, or device
    # pointers of one are unknown to the other)
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    P, I64, I32, D = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    sig = {
        "bltc_options_default": (None, [P]),
        "bltc_last_error": (ctypes.c_char_p, []),
        "bltc_version": (ctypes.c_char_p, []),
        "bltc_build_tree": (ctypes.c_int, [P, P, P, I64, I64, P, P]),
        "bltc_tree_destroy": (ctypes.c_int, [P]),
        "bltc_tree_info": (ctypes.c_int, [P, P, P]),
        "bltc_tree_export": (ctypes.c_int, [P] * 10),
        "bltc_compute_modified_weights": (ctypes.c_int, [P, P, I32, I32, P]),
        "bltc_modified_weights_export": (ctypes.c_int, [P, I32, P, P]),
        "bltc_build_targets": (ctypes.c_int, [P, P, P, I64, I32, I32, I64, P, P]),
        "bltc_targets_destroy": (ctypes.c_int, [P]),
        "bltc_targets_export": (ctypes.c_int, [P] * 6),
        "bltc_host_tree": (ctypes.c_int, [P, P, P, I64, I64] + [P] * 11),
        "bltc_host_batches": (ctypes.c_int, [P, P, P, I64, I32, I32, I64] + [P] * 5),
        "bltc_evaluate_tree": (ctypes.c_int, [P, P, I32, D, I32, D, P, P, P]),
        "bltc_evaluate": (ctypes.c_int, [P, P, P, I64, P, P, P, I64, P, I32, D,
                                         I32, D, I64, P, P, P]),
        "bltc_lists_export": (ctypes.c_int, [P, P, D, I32, I32] + [P] * 8),
        "bltc_evaluate_dual": (ctypes.c_int, [P, P, I32, D, I32, D, P, P, P, P]),
        "bltc_counts": (ctypes.c_int, [P, P, I32, D, I32, P, P]),
        "bltc_batch_costs": (ctypes.c_int, [P, P, I32, P, P, I32, P, P, P]),
        "bltc_mlp_params": (ctypes.c_int, [I32, P]),
        "bltc_mlp_work_size": (ctypes.c_int, [I64, I32, P]),
        "bltc_mlp_forward": (ctypes.c_int, [P, P, I64, I32, P, P, P]),
        "bltc_mlp_loss": (ctypes.c_int, [P, P, I64, I32, P, P, P, P]),
        "bltc_mlp_backward": (ctypes.c_int, [P, P, P, P, I64, I32, P, P, P]),
        "bltc_adam_step": (ctypes.c_int, [P, P, P, P, I64, ctypes.c_float, ctypes.c_float,
                                          ctypes.c_float, ctypes.c_float, I64, P]),
        "bltc_selector_load": (ctypes.c_int, [ctypes.c_char_p, P]),
        "bltc_selector_destroy": (ctypes.c_int, [P]),
        "bltc_selector_info": (ctypes.c_int, [P, P, P, P]),
        "bltc_batch_features": (ctypes.c_int, [P, P, I32, D, D, P, P]),
        "bltc_batch_counts": (ctypes.c_int, [P, P, D, P, P, P]),
        "bltc_evaluate_adaptive": (ctypes.c_int, [P, P, I32, D, P, D, I32, I32, D, P, P, P, P, P, P]),
        "bltc_test_fail_alloc": (ctypes.c_int, [I32]),
        "bltc_judge_samples": (ctypes.c_int, [P, P, I32, D, I32, D, P, P, P, P]),
        "bltc_evaluate_tree_noalloc": (ctypes.c_int, [P, P, I32, D, I32, D, P, P, P]),
        "bltc_noalloc_scratch_bytes": (ctypes.c_int, [P]),
        "bltc_profile_enable": (ctypes.c_int, [I32]),
        "bltc_profile_read": (ctypes.c_int, [P, P, I32]),
        "bltc_direct": (ctypes.c_int, [P, P, P, I64, P, I64, P, P, P, I64, P, I32,
                                       D, P, P, P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _check(rc):
    if rc != 0:
        raise BltcError(rc, load().bltc_last_error().decode())


def options(precision="fp64", batch_size=64, order_leaf=0, poly_p=2,
            poly_c=1.0, group_max=512, deg_min=0):
    o = Options()
    load().bltc_options_default(ctypes.byref(o))
    o.deg_min = int(deg_min)
    o.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    o.batch_size = int(batch_size)
    o.order_leaf = int(order_leaf)
    o.poly_p = int(poly_p)
    o.poly_c = float(poly_c)
    o.group_max = int(group_max)
    return o


# ---- torch plumbing -------------------------------------------------------------
def _torch():
    import torch
    return torch


def _dev(t, name, rows=None):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_cuda:
        raise TypeError(f"{name} must be a float64 CUDA tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if rows is not None and (t.dim() != 2 or t.shape[0] != rows):
        raise ValueError(f"{name} must have shape ({rows}, n)")
    return t


def _rows(pts, name):
    _dev(pts, name, 3)
    n = pts.shape[1]
    if n == 0:
        return None, None, None, 0
    s = pts.stride(0) * 8
    base = pts.data_ptr()
    return ctypes.c_void_p(base), ctypes.c_void_p(base + s), ctypes.c_void_p(base + 2 * s), n


def _stream():
    return ctypes.c_void_p(_torch().cuda.current_stream().cuda_stream)


def _np(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _hp(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None and a.size else None


# ---- handles ---------------------------------------------------------------------
class Tree:
    """Source cluster tree (bltc_build_tree) plus its modified weights."""

    def __init__(self, src, leaf_max):
        L = load()
        x, y, z, n = _rows(src, "src")
        self.n = n
        self._src = src
        h = ctypes.c_void_p()
        _check(L.bltc_build_tree(x, y, z, n, int(leaf_max), _stream(), ctypes.byref(h)))
        self._h = h
        self._lib = load()
        nn, dep = ctypes.c_int64(), ctypes.c_int32()
        _check(L.bltc_tree_info(self._h, ctypes.byref(nn), ctypes.byref(dep)))
        self.nnodes, self.depth = nn.value, dep.value

    def compute_weights(self, w, degree):
        """w: (3, n), or (6, n) force and torque rows for the full kernel."""
        _dev(w, "w")
        if w.dim() != 2 or w.shape[0] not in (3, 6) or w.shape[1] != self.n:
            raise ValueError("weights must have shape (3, n) or (6, n) for the n sources")
        ptr = ctypes.c_void_p(w.data_ptr()) if self.n else None
        _check(load().bltc_compute_modified_weights(self._h, ptr, int(w.shape[0]), int(degree),
                                                    _stream()))
        self._w = w
        self.wdim = int(w.shape[0])

    def export(self):
        nn = self.nnodes
        out = dict(perm=np.zeros(self.n, np.int64), box=np.zeros((nn, 6)),
                   center=np.zeros((nn, 3)), radius=np.zeros(nn),
                   child_first=np.zeros(nn, np.int32), child_count=np.zeros(nn, np.int32),
                   pbegin=np.zeros(nn, np.int64), pend=np.zeros(nn, np.int64),
                   level=np.zeros(nn, np.int32))
        _check(load().bltc_tree_export(self._h, *[_hp(out[k]) for k in
               ("perm", "box", "center", "radius", "child_first", "child_count",
                "pbegin", "pend", "level")]))
        return out

    def weights_export(self, degree):
        n1 = degree + 1
        f = np.zeros((self.nnodes, getattr(self, "wdim", 3), n1, n1, n1))
        g = np.zeros((self.nnodes, 3, n1))
        _check(load().bltc_modified_weights_export(self._h, int(degree), _hp(f), _hp(g)))
        return f, g

    def close(self):
        # the library object is kept on the handle: at interpreter exit the
        # module's globals may already be gone
        lib = getattr(self, "_lib", None)
        if getattr(self, "_h", None) and lib is not None:
            lib.bltc_tree_destroy(self._h)
            self._h = None

    __del__ = close


class Targets:
    """Target order and batches (bltc_build_targets)."""

    def __init__(self, tgt, batch_size=64, order_leaf=0, group_max=512):
        """order_leaf 0: balanced k-d batches; >= 1: batches of an order
        tree's groups of at most group_max targets."""
        L = load()
        x, y, z, m = _rows(tgt, "tgt")
        self.m = m
        self.batch_size = batch_size
        self.order_leaf = order_leaf
        self.group_max = group_max
        h = ctypes.c_void_p()
        _check(L.bltc_build_targets(x, y, z, m, int(batch_size), int(order_leaf),
                                    int(group_max), _stream(), ctypes.byref(h)))
        self._h = h
        self._lib = load()
        nb = ctypes.c_int64()
        _check(L.bltc_targets_export(self._h, ctypes.byref(nb), None, None, None, None))
        self.nb = nb.value

    def export(self):
        nb = self.nb
        out = dict(tperm=np.zeros(self.m, np.int64), bptr=np.zeros(nb + 1, np.int64),
                   bcenter=np.zeros((nb, 3)), bradius=np.zeros(nb))
        _check(load().bltc_targets_export(self._h, None, _hp(out["tperm"]), _hp(out["bptr"]),
                                          _hp(out["bcenter"]), _hp(out["bradius"])))
        return out

    def close(self):
        # the library object is kept on the handle: at interpreter exit the
        # module's globals may already be gone
        lib = getattr(self, "_lib", None)
        if getattr(self, "_h", None) and lib is not None:
            lib.bltc_targets_destroy(self._h)
            self._h = None

    __del__ = close


def evaluate_tree(tree, targets, kernel, eps, degree, theta, precision="fp64",
                  out=None, poly_p=2, poly_c=1.0, deg_min=0):
    """deg_min >= 1 turns on the separation rule (bltc_options.deg_min)."""
    torch = _torch()
    od = ODIM[kernel]
    if out is None:
        out = torch.empty((od, targets.m), dtype=torch.float64, device="cuda")
    _dev(out, "out", od)
    o = options(precision, targets.batch_size, targets.order_leaf, poly_p, poly_c,
                targets.group_max, deg_min)
    ptr = ctypes.c_void_p(out.data_ptr()) if targets.m else None
    _check(load().bltc_evaluate_tree(tree._h, targets._h, KERNELS[kernel], float(eps),
                                     int(degree), float(theta), ctypes.byref(o), ptr,
                                     _stream()))
    return out


def evaluate_tree_noalloc(tree, targets, kernel, eps, degree, theta, out, precision="fp64",
                          poly_p=2, poly_c=1.0, deg_min=0):
    """bltc_evaluate_tree_noalloc: as evaluate_tree, with the caller's
    output and the library's fixed scratch array; nothing is allocated."""
    od = ODIM[kernel]
    _dev(out, "out", od)
    o = options(precision, targets.batch_size, targets.order_leaf, poly_p, poly_c,
                targets.group_max, deg_min)
    ptr = ctypes.c_void_p(out.data_ptr()) if targets.m else None
    _check(load().bltc_evaluate_tree_noalloc(tree._h, targets._h, KERNELS[kernel], float(eps),
                                             int(degree), float(theta), ctypes.byref(o), ptr,
                                             _stream()))
    return out


def noalloc_scratch_bytes():
    b = ctypes.c_int64()
    _check(load().bltc_noalloc_scratch_bytes(ctypes.byref(b)))
    return b.value


def evaluate(tgt, src, w, kernel, eps, degree, theta, leaf_max, precision="fp64",
             batch_size=64, order_leaf=0, group_max=512, poly_p=2, poly_c=1.0,
             out=None, deg_min=0):
    """One call: tree, batches, modified weights and evaluation."""
    torch = _torch()
    tx, ty, tz, m = _rows(tgt, "tgt")
    sx, sy, sz, n = _rows(src, "src")
    _dev(w, "w", WDIM[kernel])
    od = ODIM[kernel]
    if out is None:
        out = torch.empty((od, m), dtype=torch.float64, device="cuda")
    _dev(out, "out", od)
    o = options(precision, batch_size, order_leaf, poly_p, poly_c, group_max, deg_min)
    _check(load().bltc_evaluate(tx, ty, tz, m, sx, sy, sz, n,
                                ctypes.c_void_p(w.data_ptr()) if n else None,
                                KERNELS[kernel], float(eps), int(degree), float(theta),
                                int(leaf_max), ctypes.byref(o),
                                ctypes.c_void_p(out.data_ptr()) if m else None, _stream()))
    return out


def evaluate_dual(src_tree, tgt_tree, kernel, eps, degree, theta, precision="fp32_fp64acc",
                  poly_p=2, poly_c=1.0, out=None, deg_min=0):
    """Cluster-cluster variant: src_tree with modified weights of `degree`,
    tgt_tree built on the targets.  Returns (out (odim, m), counts[5]).
    deg_min >= 1 applies the separation rule to the source side."""
    torch = _torch()
    od = ODIM[kernel]
    m = tgt_tree.n
    if out is None:
        out = torch.empty((od, m), dtype=torch.float64, device="cuda")
    _dev(out, "out", od)
    o = options(precision, 64, 0, poly_p, poly_c, deg_min=deg_min)
    cnt = np.zeros(5, np.int64)
    _check(load().bltc_evaluate_dual(src_tree._h, tgt_tree._h, KERNELS[kernel], float(eps),
                                     int(degree), float(theta), ctypes.byref(o),
                                     ctypes.c_void_p(out.data_ptr()) if m else None, _hp(cnt),
                                     _stream()))
    return out, cnt


def lists(tree, targets, theta, degree=1, deg_min=0):
    """Interaction lists (host arrays); prox_deg holds each accepted cluster's
    degree (degree unless the separation rule is on)."""
    L = load()
    nb, npx, ndr = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    _check(L.bltc_lists_export(tree._h, targets._h, float(theta), int(degree), int(deg_min),
                               ctypes.byref(nb), ctypes.byref(npx), ctypes.byref(ndr),
                               None, None, None, None, None))
    out = dict(prox_ptr=np.zeros(nb.value + 1, np.int64), prox_ids=np.zeros(npx.value, np.int32),
               prox_deg=np.zeros(npx.value, np.int32),
               dir_ptr=np.zeros(nb.value + 1, np.int64), dir_ids=np.zeros(ndr.value, np.int32))
    _check(L.bltc_lists_export(tree._h, targets._h, float(theta), int(degree), int(deg_min),
                               None, None, None, _hp(out["prox_ptr"]), _hp(out["prox_ids"]),
                               _hp(out["prox_deg"]), _hp(out["dir_ptr"]), _hp(out["dir_ids"])))
    return out


def counts(tree, targets, degree, theta, deg_min=0):
    a, b = ctypes.c_int64(), ctypes.c_int64()
    _check(load().bltc_counts(tree._h, targets._h, int(degree), float(theta), int(deg_min),
                              ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


def direct(tgt, src, w, kernel, eps, idx=None, precision="fp64", poly_p=2, poly_c=1.0):
    """Direct sum on the device for the targets idx (int64 CUDA tensor) or all."""
    torch = _torch()
    tx, ty, tz, m = _rows(tgt, "tgt")
    sx, sy, sz, n = _rows(src, "src")
    _dev(w, "w", WDIM[kernel])
    if idx is not None:
        if idx.dtype != torch.int64 or not idx.is_cuda or not idx.is_contiguous():
            raise TypeError("idx must be a contiguous int64 CUDA tensor")
        k = idx.numel()
        ip = ctypes.c_void_p(idx.data_ptr()) if k else None
    else:
        k, ip = m, None
    out = torch.empty((ODIM[kernel], k), dtype=torch.float64, device="cuda")
    o = options(precision, 64, 32, poly_p, poly_c)
    _check(load().bltc_direct(tx, ty, tz, m, ip, k, sx, sy, sz, n,
                              ctypes.c_void_p(w.data_ptr()) if n else None,
                              KERNELS[kernel], float(eps), ctypes.byref(o),
                              ctypes.c_void_p(out.data_ptr()) if k else None, _stream()))
    return out


# ---- host-only builders (no device) ------------------------------------------------
def host_tree(pts, leaf_max):
    pts = _np(pts, np.float64)
    L = load()
    n = pts.shape[1]
    nn, dep = ctypes.c_int64(), ctypes.c_int32()
    args = [_hp(pts[0]), _hp(pts[1]), _hp(pts[2]), n, int(leaf_max)]
    _check(L.bltc_host_tree(*args, ctypes.byref(nn), ctypes.byref(dep), *([None] * 9)))
    k = nn.value
    out = dict(perm=np.zeros(n, np.int64), box=np.zeros((k, 6)), center=np.zeros((k, 3)),
               radius=np.zeros(k), child_first=np.zeros(k, np.int32),
               child_count=np.zeros(k, np.int32), pbegin=np.zeros(k, np.int64),
               pend=np.zeros(k, np.int64), level=np.zeros(k, np.int32))
    _check(L.bltc_host_tree(*args, None, None, *[_hp(out[q]) for q in
           ("perm", "box", "center", "radius", "child_first", "child_count",
            "pbegin", "pend", "level")]))
    out["depth"] = dep.value
    return out


def host_batches(pts, batch_size, order_leaf, group_max=512):
    pts = _np(pts, np.float64)
    L = load()
    m = pts.shape[1]
    nb = ctypes.c_int64()
    args = [_hp(pts[0]), _hp(pts[1]), _hp(pts[2]), m, int(batch_size), int(order_leaf),
            int(group_max)]
    _check(L.bltc_host_batches(*args, ctypes.byref(nb), None, None, None, None))
    k = nb.value
    out = dict(tperm=np.zeros(m, np.int64), bptr=np.zeros(k + 1, np.int64),
               bcenter=np.zeros((k, 3)), bradius=np.zeros(k))
    _check(L.bltc_host_batches(*args, None, _hp(out["tperm"]), _hp(out["bptr"]),
                               _hp(out["bcenter"]), _hp(out["bradius"])))
    return out


# ---- measurement -------------------------------------------------------------------
STAGES = ("prep", "upward", "lists", "eval")


def profile_enable(on=True):
    _check(load().bltc_profile_enable(1 if on else 0))


def profile_read(reset=True):
    """{stage: (total ms, launches)} from the library's stage events."""
    ms = np.zeros(len(STAGES))
    n = np.zeros(len(STAGES), np.int64)
    _check(load().bltc_profile_read(_hp(ms), _hp(n), 1 if reset else 0))
    return {s: (float(ms[i]), int(n[i])) for i, s in enumerate(STAGES)}


# ---- selector network ------------------------------------------------------------
def _f32(t, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float32 or not t.is_cuda:
        raise TypeError(f"{name} must be a float32 CUDA tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def mlp_params(k):
    n = ctypes.c_int64()
    _check(load().bltc_mlp_params(int(k), ctypes.byref(n)))
    return n.value


def mlp_work(rows, k):
    """A device workspace for mlp_loss / mlp_backward."""
    n = ctypes.c_int64()
    _check(load().bltc_mlp_work_size(int(rows), int(k), ctypes.byref(n)))
    return _torch().empty(n.value, dtype=_torch().float32, device="cuda")


def mlp_forward(params, X, k, cache=True):
    torch = _torch()
    rows = X.shape[0]
    Y = torch.empty((rows, k), dtype=torch.float32, device="cuda")
    C = torch.empty((rows, 128), dtype=torch.float32, device="cuda") if cache else None
    _check(load().bltc_mlp_forward(_f32(params, "params"), _f32(X, "X"), rows, int(k),
                                   _f32(Y, "Y"), _f32(C, "cache") if cache else None,
                                   _stream()))
    return Y, C


def mlp_loss(Y, T, work):
    torch = _torch()
    rows, k = Y.shape
    dY = torch.empty_like(Y)
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    _check(load().bltc_mlp_loss(_f32(Y, "Y"), _f32(T, "T"), rows, k, _f32(dY, "dY"),
                                _f32(loss, "loss"), _f32(work, "work"), _stream()))
    return dY, loss


def mlp_backward(params, X, cache, dY, work):
    rows, k = dY.shape
    grad = _torch().empty_like(params)
    _check(load().bltc_mlp_backward(_f32(params, "params"), _f32(X, "X"), _f32(cache, "cache"),
                                    _f32(dY, "dY"), rows, k, _f32(grad, "grad"),
                                    _f32(work, "work"), _stream()))
    return grad


def adam_step(params, m, v, grad, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    _check(load().bltc_adam_step(_f32(params, "params"), _f32(m, "m"), _f32(v, "v"),
                                 _f32(grad, "grad"), params.numel(), float(lr), float(beta1),
                                 float(beta2), float(eps), int(step), _stream()))


# ---- learned (n, theta) per batch ------------------------------------------------
def batch_features(tree, targets, kernel, eps, theta_ref=0.7):
    """Raw per-batch features, float32 (nb, 12) on the device."""
    torch = _torch()
    f = torch.empty((targets.nb, 12), dtype=torch.float32, device="cuda")
    _check(load().bltc_batch_features(tree._h, targets._h, KERNELS[kernel], float(eps),
                                      float(theta_ref),
                                      ctypes.c_void_p(f.data_ptr()) if targets.nb else None,
                                      _stream()))
    return f


def batch_costs(tree, targets, cands, deg_min, weights):
    """Modelled wave cost [k][nb] (device float32) of every batch under each
    candidate (n, theta) of `cands`."""
    torch = _torch()
    k = len(cands)
    cn = np.array([c[0] for c in cands], np.int32)
    ct = np.array([c[1] for c in cands], np.float64)
    wv = np.array(weights, np.float32)
    out = torch.zeros((k, max(targets.nb, 1)), dtype=torch.float32, device="cuda")
    _check(load().bltc_batch_costs(tree._h, targets._h, k, _hp(cn), _hp(ct), int(deg_min),
                                   _hp(wv), ctypes.c_void_p(out.data_ptr()), _stream()))
    return out[:, :targets.nb]


def batch_counts(tree, targets, theta):
    """(accepted clusters, near-field sources) per batch, int32 on the device."""
    torch = _torch()
    pc = torch.empty(targets.nb, dtype=torch.int32, device="cuda")
    sc = torch.empty(targets.nb, dtype=torch.int32, device="cuda")
    nb = targets.nb
    _check(load().bltc_batch_counts(tree._h, targets._h, float(theta),
                                    ctypes.c_void_p(pc.data_ptr()) if nb else None,
                                    ctypes.c_void_p(sc.data_ptr()) if nb else None, _stream()))
    return pc, sc


class Selector:
    """A per-batch (n, theta) model loaded from a selector model file."""

    def __init__(self, path):
        h = ctypes.c_void_p()
        _check(load().bltc_selector_load(os.fsencode(path), ctypes.byref(h)))
        self._h = h
        self._lib = load()
        k = ctypes.c_int32()
        _check(load().bltc_selector_info(self._h, ctypes.byref(k), None, None))
        self.k = k.value
        self.cand_n = np.zeros(self.k, np.int32)
        self.cand_theta = np.zeros(self.k)
        _check(load().bltc_selector_info(self._h, None, _hp(self.cand_n), _hp(self.cand_theta)))

    def close(self):
        # the library object is kept on the handle: at interpreter exit the
        # module's globals may already be gone
        lib = getattr(self, "_lib", None)
        if getattr(self, "_h", None) and lib is not None:
            lib.bltc_selector_destroy(self._h)
            self._h = None

    __del__ = close


SELECT_MODES = {"batch": 0, "run": 1}


def evaluate_adaptive(tree, targets, kernel, eps, selector, tol, fb_degree, fb_theta,
                      precision="fp32_fp64acc", out=None, mode="batch"):
    """Returns (out, choice per batch (candidate index, or -2 when the judge
    sent the batch to the fallback), stats [batches, distinct degrees, batches
    re-evaluated, 0], judge [error estimate before, after re-evaluation])."""
    torch = _torch()
    od = ODIM[kernel]
    if out is None:
        out = torch.empty((od, targets.m), dtype=torch.float64, device="cuda")
    _dev(out, "out", od)
    o = options(precision, targets.batch_size, targets.order_leaf, group_max=targets.group_max)
    choice = np.zeros(max(targets.nb, 1), np.int32)
    stats = np.zeros(4, np.int64)
    judge = np.zeros(2, np.float64)
    _check(load().bltc_evaluate_adaptive(tree._h, targets._h, KERNELS[kernel], float(eps),
                                         selector._h, float(tol), SELECT_MODES[mode],
                                         int(fb_degree),
                                         float(fb_theta), ctypes.byref(o),
                                         ctypes.c_void_p(out.data_ptr()) if targets.m else None,
                                         _hp(choice), _hp(stats), _hp(judge), _stream()))
    return out, choice[:targets.nb], stats, judge


def judge_samples(tree, targets, kernel, eps, fb_degree, fb_theta):
    """bltc_judge_samples: (caller-order target indices, fallback values
    (odim, n_samples)) of the judge's samples."""
    L = load()
    ns = ctypes.c_int64()
    _check(L.bltc_judge_samples(tree._h, targets._h, KERNELS[kernel], float(eps), int(fb_degree),
                                float(fb_theta), ctypes.byref(ns), None, None, _stream()))
    idx = np.zeros(ns.value, np.int64)
    u = np.zeros((ns.value, ODIM[kernel]))
    _check(L.bltc_judge_samples(tree._h, targets._h, KERNELS[kernel], float(eps), int(fb_degree),
                                float(fb_theta), ctypes.byref(ns), _hp(idx), _hp(u), _stream()))
    return idx, np.ascontiguousarray(u.T)


def inject_alloc_failure(after):
    """Failure injection (bltc_test_fail_alloc): the after-th device
    allocation from now fails with BLTC_ENOMEM; 0 disarms."""
    _check(load().bltc_test_fail_alloc(int(after)))
