"""CPU FP64 oracle for the barycentric Lagrange treecode (arXiv:1902.02250).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark may use this package; the product library never does.  It
shares no code with the HIP path.  The arithmetic lives in the plain C files
next to this one (see ``oracle.h``); this module only builds them with gcc and
marshals numpy arrays through ctypes.  ``mlp.py`` holds the FP64 reference of
the per-batch selector network.

Array conventions: points are ``(3, n)`` float64 arrays (x, y, z rows),
weights ``(wdim, n)`` and outputs ``(odim, m)``, all C-contiguous.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SOURCES = ["kernels.c", "direct.c", "tree.c", "bary.c", "treecode.c", "dual.c"]
KERNELS = {"stokeslet": 0, "rotlet": 1, "full": 2, "poly": 100}
ODIM = {"stokeslet": 3, "rotlet": 6, "full": 6, "poly": 3}
WDIM = {"stokeslet": 3, "rotlet": 3, "full": 6, "poly": 3}

_lib = None


def build():
    """Compile liboracle.so with gcc (FP64, OpenMP, no FMA contraction)."""
    srcs = [os.path.join(_HERE, s) for s in _SOURCES]
    tmp = _SO + ".tmp"
    subprocess.check_call(
        ["gcc", "-std=gnu11", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC",
         "-shared", "-Wall", "-o", tmp] + srcs + ["-lm"])
    os.replace(tmp, _SO)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_SO):
        build()
    L = ctypes.CDLL(_SO)
    P = ctypes.c_void_p
    I64, I32, D = ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    L.orc_direct.argtypes = [ctypes.c_int, D, ctypes.c_int, D, P, P, P, I64,
                             P, P, P, I64, P, ctypes.c_int, P]
    L.orc_direct_subset.argtypes = [ctypes.c_int, D, ctypes.c_int, D, P, P, P,
                                    P, I64, P, P, P, I64, P, P]
    L.orc_mrs_functions.argtypes = [D, D, P]
    L.orc_pair.argtypes = [ctypes.c_int, D, ctypes.c_int, D, P, P, P, P]
    L.orc_tree_new.argtypes = [P, P, P, I64, I64]
    L.orc_tree_new.restype = P
    L.orc_tree_free.argtypes = [P]
    L.orc_tree_nnodes.argtypes = [P]
    L.orc_tree_nnodes.restype = I64
    L.orc_tree_depth.argtypes = [P]
    L.orc_tree_depth.restype = I32
    L.orc_tree_export.argtypes = [P] * 11
    L.orc_batches.argtypes = [P, P, P, I64, I64, I64, I64, P, P, P, P]
    L.orc_batches.restype = I64
    L.orc_cheb_points.argtypes = [ctypes.c_int, P]
    L.orc_bary_weights.argtypes = [ctypes.c_int, P]
    L.orc_lagrange_bary.argtypes = [ctypes.c_int, P, D, P]
    L.orc_lagrange_product.argtypes = [ctypes.c_int, P, D, P]
    L.orc_cluster_grids.argtypes = [P, ctypes.c_int, P]
    L.orc_modified_weights.argtypes = [P, P, P, P, P, ctypes.c_int,
                                       ctypes.c_int, ctypes.c_int, P]
    L.orc_treecode.argtypes = [P, P, P, P, I64, P, P, P, I64, P, P, I64, P,
                               P, P]
    L.orc_dual_treecode.argtypes = [P, I64, P, P, P, I64, P, P, P, I64, P, P, P]
    L.orc_lists_new.argtypes = [P, P, P, I64, I64, P, P, P, I64, D, I64, I64,
                                I64, ctypes.c_int, ctypes.c_int]
    L.orc_lists_new.restype = P
    L.orc_lists_export_degrees.argtypes = [P, P]
    L.orc_rule_table.argtypes = [P, P]
    L.orc_rule_degree.argtypes = [P, P, D, D]
    L.orc_rule_degree.restype = ctypes.c_int
    L.orc_lists_sizes.argtypes = [P, P, P, P]
    L.orc_lists_export.argtypes = [P] * 7
    L.orc_lists_free.argtypes = [P]
    L.orc_rel_l2.argtypes = [P, P, I64]
    L.orc_rel_l2.restype = D
    _lib = L
    return L


def _p(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None and a.size else None


def _c(a, dtype=np.float64):
    return np.ascontiguousarray(a, dtype=dtype)


class _Params(ctypes.Structure):
    _fields_ = [("kernel", ctypes.c_int), ("eps", ctypes.c_double),
                ("poly_p", ctypes.c_int), ("poly_c", ctypes.c_double),
                ("degree", ctypes.c_int), ("theta", ctypes.c_double),
                ("leaf_max", ctypes.c_int64), ("mac_mode", ctypes.c_int),
                ("batch_size", ctypes.c_int64), ("order_leaf", ctypes.c_int64),
                ("group_max", ctypes.c_int64), ("deg_min", ctypes.c_int)]


# ---- kernels ----------------------------------------------------------------
def mrs_functions(r2, eps):
    """(H1, H2, Q, D1, D2) at squared distance r2 (eq. MRS_kernels)."""
    out = np.zeros(5)
    _load().orc_mrs_functions(float(r2), float(eps), _p(out))
    return out


def pair(kernel, x, y, f, eps=0.0, poly_p=0, poly_c=0.0):
    """k(x, y) f for one target x and one source y."""
    out = np.zeros(ODIM[kernel])
    x, y, f = _c(x), _c(y), _c(f)
    _load().orc_pair(KERNELS[kernel], float(eps), int(poly_p), float(poly_c),
                     _p(x), _p(y), _p(f), _p(out))
    return out


# ---- direct sum -------------------------------------------------------------
def direct(kernel, tgt, src, w, eps=0.0, compensated=False, poly_p=0,
           poly_c=0.0):
    """Direct sum u(x_i) = sum_j k(x_i, y_j) f_j for every target."""
    tgt, src, w = _c(tgt), _c(src), _c(w)
    m, n = tgt.shape[1], src.shape[1]
    out = np.zeros((ODIM[kernel], m))
    rc = _load().orc_direct(KERNELS[kernel], float(eps), int(poly_p),
                            float(poly_c), _p(tgt[0]), _p(tgt[1]), _p(tgt[2]),
                            m, _p(src[0]), _p(src[1]), _p(src[2]), n, _p(w),
                            int(compensated), _p(out))
    assert rc == 0
    return out


def direct_subset(kernel, tgt, idx, src, w, eps=0.0, poly_p=0, poly_c=0.0):
    """Direct sum for the targets tgt[:, idx] only; returns (odim, len(idx))."""
    tgt, src, w = _c(tgt), _c(src), _c(w)
    idx = _c(idx, np.int64)
    out = np.zeros((ODIM[kernel], idx.size))
    rc = _load().orc_direct_subset(KERNELS[kernel], float(eps), int(poly_p),
                                   float(poly_c), _p(tgt[0]), _p(tgt[1]),
                                   _p(tgt[2]), _p(idx), idx.size, _p(src[0]),
                                   _p(src[1]), _p(src[2]), src.shape[1], _p(w),
                                   _p(out))
    assert rc == 0
    return out


# ---- tree -------------------------------------------------------------------
class Tree:
    """The oracle's cluster tree over points (3, n) with leaf size leaf_max."""

    def __init__(self, pts, leaf_max):
        self.pts = _c(pts)
        self.n = self.pts.shape[1]
        L = _load()
        self._h = L.orc_tree_new(_p(self.pts[0]), _p(self.pts[1]),
                                 _p(self.pts[2]), self.n, int(leaf_max))
        nn = L.orc_tree_nnodes(self._h)
        self.nnodes = nn
        self.depth = L.orc_tree_depth(self._h)
        self.perm = np.zeros(self.n, np.int64)
        self.box = np.zeros((nn, 6))
        self.center = np.zeros((nn, 3))
        self.radius = np.zeros(nn)
        self.child_first = np.zeros(nn, np.int32)
        self.child_count = np.zeros(nn, np.int32)
        self.pbegin = np.zeros(nn, np.int64)
        self.pend = np.zeros(nn, np.int64)
        self.level = np.zeros(nn, np.int32)
        self.parent = np.zeros(nn, np.int32)
        L.orc_tree_export(self._h, _p(self.perm), _p(self.box),
                          _p(self.center), _p(self.radius),
                          _p(self.child_first), _p(self.child_count),
                          _p(self.pbegin), _p(self.pend), _p(self.level),
                          _p(self.parent))

    def grids(self, degree):
        """Mapped Chebyshev points, (nnodes, 3, degree+1)."""
        g = np.zeros((self.nnodes, 3, degree + 1))
        _load().orc_cluster_grids(self._h, int(degree), _p(g))
        return g

    def modified_weights(self, w, degree, form=0):
        """fhat[node, c, k1, k2, k3] by Algorithm 1 (form 0) or by the
        product-form Lagrange polynomials (form 1)."""
        w = _c(w)
        n1 = degree + 1
        out = np.zeros((self.nnodes, w.shape[0], n1, n1, n1))
        rc = _load().orc_modified_weights(self._h, _p(self.pts[0]),
                                          _p(self.pts[1]), _p(self.pts[2]),
                                          _p(w), w.shape[0], int(degree),
                                          int(form), _p(out))
        assert rc == 0
        return out

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.orc_tree_free(self._h)
            self._h = None


def batches(tgt, batch_size, order_leaf, group_max=512):
    """Target batches: (tperm, bptr, bcenter, bradius); order_leaf = 0 gives
    the balanced k-d batches."""
    tgt = _c(tgt)
    m = tgt.shape[1]
    L = _load()
    args = [_p(tgt[0]), _p(tgt[1]), _p(tgt[2]), m, int(batch_size), int(order_leaf),
            int(group_max)]
    nb = L.orc_batches(*args, None, None, None, None)
    tperm = np.zeros(m, np.int64)
    bptr = np.zeros(nb + 1, np.int64)
    bc = np.zeros((max(nb, 1), 3))
    br = np.zeros(max(nb, 1))
    L.orc_batches(*args, _p(tperm), _p(bptr), _p(bc), _p(br))
    return tperm, bptr, bc[:nb], br[:nb]


# ---- 1D interpolation -------------------------------------------------------
def cheb_points(n):
    t = np.zeros(n + 1)
    _load().orc_cheb_points(int(n), _p(t))
    return t


def bary_weights(n):
    w = np.zeros(n + 1)
    _load().orc_bary_weights(int(n), _p(w))
    return w


def lagrange_bary(n, s, t):
    s = _c(s)
    L = np.zeros(n + 1)
    _load().orc_lagrange_bary(int(n), _p(s), float(t), _p(L))
    return L


def lagrange_product(n, s, t):
    s = _c(s)
    L = np.zeros(n + 1)
    _load().orc_lagrange_product(int(n), _p(s), float(t), _p(L))
    return L


# ---- treecode ---------------------------------------------------------------
def treecode(kernel, tgt, src, w, eps, degree, theta, leaf_max, mac_mode=0,
             batch_size=64, order_leaf=64, group_max=512, sample=None, poly_p=0,
             poly_c=0.0, deg_min=0):
    """Algorithm 2.  Returns (out (odim, m or len(sample)), n_proxy_evals,
    n_direct_evals).  deg_min >= 1 selects the separation rule for the
    degree of each accepted cluster (orc_rule_degree)."""
    tgt, src, w = _c(tgt), _c(src), _c(w)
    m, n = tgt.shape[1], src.shape[1]
    prm = _Params(KERNELS[kernel], float(eps), int(poly_p), float(poly_c),
                  int(degree), float(theta), int(leaf_max), int(mac_mode),
                  int(batch_size), int(order_leaf), int(group_max), int(deg_min))
    if sample is not None:
        sample = _c(sample, np.int64)
        k = sample.size
    else:
        k = 0
    out = np.zeros((ODIM[kernel], k if sample is not None else m))
    npx = ctypes.c_int64(0)
    ndr = ctypes.c_int64(0)
    rc = _load().orc_treecode(ctypes.byref(prm), _p(tgt[0]), _p(tgt[1]),
                              _p(tgt[2]), m, _p(src[0]), _p(src[1]),
                              _p(src[2]), n, _p(w), _p(sample), k, _p(out),
                              ctypes.byref(npx), ctypes.byref(ndr))
    assert rc == 0, "oracle treecode rejected its parameters"
    return out, npx.value, ndr.value


def dual_treecode(kernel, tgt, src, w, eps, degree, theta, leaf_max, leaf_t, poly_p=0,
                  poly_c=0.0, deg_min=0):
    """The cluster-cluster variant (dual.c).  Returns (out (odim, m), counts)
    with counts = kernel evaluations of the CC, PC, CP and PP interactions
    and the downward (target, grid point) terms.  deg_min >= 1 applies the
    separation rule to the source side of CC and PC pairs."""
    tgt, src, w = _c(tgt), _c(src), _c(w)
    m, n = tgt.shape[1], src.shape[1]
    prm = _Params(KERNELS[kernel], float(eps), int(poly_p), float(poly_c),
                  int(degree), float(theta), int(leaf_max), 0, 1, 1, 1, int(deg_min))
    out = np.zeros((ODIM[kernel], m))
    cnt = np.zeros(5, np.int64)
    rc = _load().orc_dual_treecode(ctypes.byref(prm), int(leaf_t), _p(tgt[0]), _p(tgt[1]),
                                   _p(tgt[2]), m, _p(src[0]), _p(src[1]), _p(src[2]), n,
                                   _p(w), _p(out), _p(cnt))
    assert rc == 0, "oracle dual treecode rejected its parameters"
    return out, cnt


def lists(src, leaf_max, tgt, theta, batch_size, order_leaf, group_max=512, degree=1,
          deg_min=0):
    """Batch-walk interaction lists as a dict of CSR arrays, with the degree
    of every proxy entry (`degree` unless deg_min >= 1)."""
    src, tgt = _c(src), _c(tgt)
    L = _load()
    h = L.orc_lists_new(_p(src[0]), _p(src[1]), _p(src[2]), src.shape[1],
                        int(leaf_max), _p(tgt[0]), _p(tgt[1]), _p(tgt[2]),
                        tgt.shape[1], float(theta), int(batch_size),
                        int(order_leaf), int(group_max), int(degree), int(deg_min))
    nb, npx, ndr = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    L.orc_lists_sizes(h, ctypes.byref(nb), ctypes.byref(npx), ctypes.byref(ndr))
    out = dict(tperm=np.zeros(tgt.shape[1], np.int64),
               bptr=np.zeros(nb.value + 1, np.int64),
               prox_ptr=np.zeros(nb.value + 1, np.int64),
               prox_ids=np.zeros(npx.value, np.int32),
               dir_ptr=np.zeros(nb.value + 1, np.int64),
               dir_ids=np.zeros(ndr.value, np.int32))
    L.orc_lists_export(h, _p(out["tperm"]), _p(out["bptr"]),
                       _p(out["prox_ptr"]), _p(out["prox_ids"]),
                       _p(out["dir_ptr"]), _p(out["dir_ids"]))
    out["prox_deg"] = np.zeros(npx.value, np.int32)
    L.orc_lists_export_degrees(h, _p(out["prox_deg"]))
    L.orc_lists_free(h)
    return out


def rel_l2(ref, approx):
    """Relative L2 error of eq. error over all components."""
    ref, approx = _c(ref).ravel(), _c(approx).ravel()
    return _load().orc_rel_l2(_p(ref), _p(approx), ref.size)
