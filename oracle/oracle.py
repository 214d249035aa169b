"""ctypes wrapper around ``liborc.so`` (built from ``aerl_oracle.c``).

Test infrastructure only: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "aerl_oracle.c")
LIB = os.path.join(HERE, "liborc.so")

CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
          "-std=gnu11", "-Wall", "-Wextra", "-Wno-unused-parameter"]


def lib_path() -> str:
    return LIB


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (contraction off, no fast-math)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


class _Pop(C.Structure):
    _fields_ = [("n_sets", C.c_int32),
                ("set_rule_off", C.c_void_p), ("set_default", C.c_void_p),
                ("rule_cond_off", C.c_void_p), ("rule_class", C.c_void_p),
                ("op", C.c_void_p), ("kind", C.c_void_p), ("f", C.c_void_p), ("g", C.c_void_p),
                ("coef", C.c_void_p), ("coef2", C.c_void_p), ("theta", C.c_void_p),
                ("cat_mask", C.c_void_p)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build(force=True)
        lib = C.CDLL(LIB)
        I64, I32, P, PP = C.c_int64, C.c_int32, C.c_void_p, C.POINTER(_Pop)
        sig = {
            "orc_max_threads": ([], C.c_int),
            "orc_hard_eval": ([I64, I32, P, P, I32, PP, P, P, C.c_int], C.c_int),
            "orc_predict": ([I64, I32, P, PP, I32, P], C.c_int),
            "orc_workcount": ([I64, P, P, I32, P, PP, P, P, C.c_int], C.c_int),
            "orc_tau": ([I64, I32, P, P], C.c_int),
            "orc_soft_logprobs": ([I64, I32, P, P, I32, PP, P, P, P, I32, P], C.c_int),
            "orc_soft_forward": ([I64, I32, P, P, P, I32, PP, P, P, P, P, C.c_int], C.c_int),
            "orc_soft_forward_naive": ([I64, I32, P, P, P, I32, PP, P, P, P, P], C.c_int),
            "orc_soft_backward": ([I64, I32, P, P, P, I32, PP, P, P, P, P, P, P, P, C.c_int], C.c_int),
            "orc_smax_probs": ([I64, I32, P, P, I32, PP, P, P, P, I32, C.c_double, P], C.c_int),
            "orc_smax_forward": ([I64, I32, P, P, P, I32, PP, P, P, P, C.c_double, P, C.c_int],
                                 C.c_int),
            "orc_smax_backward": ([I64, I32, P, P, P, I32, PP, P, P, P, C.c_double, P, P, P, P,
                                   C.c_int], C.c_int),
        }
        for name, (args, res) in sig.items():
            fn = getattr(lib, name)
            fn.argtypes, fn.restype = args, res
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


class _PopView:
    """Keeps the contiguous arrays alive while the C struct points at them."""

    def __init__(self, pop):
        self.arrays = dict(
            set_rule_off=np.ascontiguousarray(pop.set_rule_off, np.int32),
            set_default=np.ascontiguousarray(pop.set_default, np.int32),
            rule_cond_off=np.ascontiguousarray(pop.rule_cond_off, np.int32),
            rule_class=np.ascontiguousarray(pop.rule_class, np.int32),
            op=np.ascontiguousarray(pop.op, np.uint8), kind=np.ascontiguousarray(pop.kind, np.uint8),
            f=np.ascontiguousarray(pop.f, np.int32), g=np.ascontiguousarray(pop.g, np.int32),
            coef=np.ascontiguousarray(pop.coef, np.float32),
            coef2=np.ascontiguousarray(pop.coef2, np.float32),
            theta=np.ascontiguousarray(pop.theta, np.float32),
            cat_mask=np.ascontiguousarray(getattr(pop, "cat_mask", None)
                                          if getattr(pop, "cat_mask", None) is not None
                                          else np.zeros(len(pop.op), np.uint64), np.uint64))
        self.s = _Pop(int(pop.set_default.shape[0]), *[_ptr(self.arrays[k]) for k in (
            "set_rule_off", "set_default", "rule_cond_off", "rule_class", "op", "kind", "f", "g",
            "coef", "coef2", "theta", "cat_mask")])
        self.n_sets = int(pop.set_default.shape[0])
        self.n_conds = int(pop.op.shape[0])

    def ref(self):
        return C.byref(self.s)


def max_threads() -> int:
    return int(_load().orc_max_threads())


def _xy(x, y=None):
    x = np.ascontiguousarray(x, np.float32)
    assert x.ndim == 2
    if y is not None:
        y = np.ascontiguousarray(y, np.int32)
        assert y.shape == (x.shape[0],)
    return x, y


def hard_eval(x, y, n_classes, pop, confusion=True, nthreads=0):
    """Returns (correct int32 [P], confusion int32 [P][C][C] or None)."""
    x, y = _xy(x, y)
    v = _PopView(pop)
    correct = np.zeros(v.n_sets, np.int32)
    conf = np.zeros((v.n_sets, n_classes, n_classes), np.int32) if confusion else None
    rc = _load().orc_hard_eval(x.shape[0], x.shape[1], _ptr(x), _ptr(y), n_classes, v.ref(),
                               _ptr(correct), _ptr(conf) if conf is not None else None, nthreads)
    assert rc == 0
    return correct, conf


def predict(x, pop, s=0):
    x, _ = _xy(x)
    v = _PopView(pop)
    out = np.zeros(x.shape[0], np.int32)
    assert _load().orc_predict(x.shape[0], x.shape[1], _ptr(x), v.ref(), s, _ptr(out)) == 0
    return out


def label_grouped_tiles(y, n_classes, tile=64):
    """Sample order grouped by label (stable), cut into tiles of ``tile``
    samples that never mix labels.  Returns (tile_ptr int64, tile_idx int64)."""
    y = np.asarray(y)
    ptr, idx = [0], []
    for c in range(n_classes):
        members = np.nonzero(y == c)[0]
        for a in range(0, len(members), tile):
            idx.append(members[a:a + tile])
            ptr.append(ptr[-1] + len(members[a:a + tile]))
    tile_idx = np.concatenate(idx).astype(np.int64) if idx else np.zeros(0, np.int64)
    return np.array(ptr, np.int64), tile_idx


def workcount(x, pop, tile_ptr, tile_idx, nthreads=0):
    """Per rule set (threshold, feature-vs-feature) condition visits of a wave
    with wave-uniform early exit, summed over the given tiles."""
    x, _ = _xy(x)
    v = _PopView(pop)
    tile_ptr = np.ascontiguousarray(tile_ptr, np.int64)
    tile_idx = np.ascontiguousarray(tile_idx, np.int64)
    wt = np.zeros(v.n_sets, np.int64)
    wf = np.zeros(v.n_sets, np.int64)
    rc = _load().orc_workcount(len(tile_ptr) - 1, _ptr(tile_ptr), _ptr(tile_idx), x.shape[1],
                               _ptr(x), v.ref(), _ptr(wt), _ptr(wf), nthreads)
    assert rc == 0
    return wt, wf


def tau(x):
    x, _ = _xy(x)
    out = np.zeros(x.shape[1], np.float32)
    assert _load().orc_tau(x.shape[0], x.shape[1], _ptr(x), _ptr(out)) == 0
    return out


def _params(pop, coef, coef2, theta):
    d = lambda a, dflt: np.ascontiguousarray(dflt if a is None else a, np.float64)
    return d(coef, pop.coef), d(coef2, pop.coef2), d(theta, pop.theta)


def soft_logprobs(x, tau_, n_classes, pop, s, coef=None, coef2=None, theta=None):
    x, _ = _xy(x)
    v = _PopView(pop)
    c1, c2, th = _params(pop, coef, coef2, theta)
    out = np.zeros((x.shape[0], n_classes), np.float64)
    t = np.ascontiguousarray(tau_, np.float32)
    assert _load().orc_soft_logprobs(x.shape[0], x.shape[1], _ptr(x), _ptr(t), n_classes, v.ref(),
                                     _ptr(c1), _ptr(c2), _ptr(th), s, _ptr(out)) == 0
    return out


def soft_forward(x, y, tau_, n_classes, pop, coef=None, coef2=None, theta=None, nthreads=0):
    """fp64 loss per rule set."""
    x, y = _xy(x, y)
    v = _PopView(pop)
    c1, c2, th = _params(pop, coef, coef2, theta)
    t = np.ascontiguousarray(tau_, np.float32)
    loss = np.zeros(v.n_sets, np.float64)
    rc = _load().orc_soft_forward(x.shape[0], x.shape[1], _ptr(x), _ptr(y), _ptr(t), n_classes,
                                  v.ref(), _ptr(c1), _ptr(c2), _ptr(th), _ptr(loss), nthreads)
    assert rc == 0
    return loss


def soft_forward_naive(x, y, tau_, n_classes, pop, coef=None, coef2=None, theta=None):
    x, y = _xy(x, y)
    v = _PopView(pop)
    c1, c2, th = _params(pop, coef, coef2, theta)
    t = np.ascontiguousarray(tau_, np.float32)
    loss = np.zeros(v.n_sets, np.float64)
    assert _load().orc_soft_forward_naive(x.shape[0], x.shape[1], _ptr(x), _ptr(y), _ptr(t),
                                          n_classes, v.ref(), _ptr(c1), _ptr(c2), _ptr(th),
                                          _ptr(loss)) == 0
    return loss


def soft_backward(x, y, tau_, n_classes, pop, dloss=None, coef=None, coef2=None, theta=None,
                  nthreads=0):
    """fp64 gradients (dcoef, dcoef2, dtheta) of sum_s dloss[s] * loss[s]."""
    x, y = _xy(x, y)
    v = _PopView(pop)
    c1, c2, th = _params(pop, coef, coef2, theta)
    t = np.ascontiguousarray(tau_, np.float32)
    dl = np.ascontiguousarray(np.ones(v.n_sets) if dloss is None else dloss, np.float64)
    g1 = np.zeros(v.n_conds, np.float64)
    g2 = np.zeros(v.n_conds, np.float64)
    g3 = np.zeros(v.n_conds, np.float64)
    rc = _load().orc_soft_backward(x.shape[0], x.shape[1], _ptr(x), _ptr(y), _ptr(t), n_classes,
                                   v.ref(), _ptr(c1), _ptr(c2), _ptr(th), _ptr(dl), _ptr(g1),
                                   _ptr(g2), _ptr(g3), nthreads)
    assert rc == 0
    return g1, g2, g3


# ---------------------------------------------------------------- softmax head
def smax_probs(x, tau_, n_classes, pop, s, beta, coef=None, coef2=None, theta=None):
    """fp64 class probabilities [n][C] of rule set s under the softmax head."""
    x, _ = _xy(x)
    v = _PopView(pop)
    c1, c2, th = _params(pop, coef, coef2, theta)
    t = np.ascontiguousarray(tau_, np.float32)
    out = np.zeros((x.shape[0], n_classes), np.float64)
    assert _load().orc_smax_probs(x.shape[0], x.shape[1], _ptr(x), _ptr(t), n_classes, v.ref(),
                                  _ptr(c1), _ptr(c2), _ptr(th), s, float(beta), _ptr(out)) == 0
    return out


def smax_forward(x, y, tau_, n_classes, pop, beta, coef=None, coef2=None, theta=None, nthreads=0):
    """fp64 loss per rule set under the softmax head."""
    x, y = _xy(x, y)
    v = _PopView(pop)
    c1, c2, th = _params(pop, coef, coef2, theta)
    t = np.ascontiguousarray(tau_, np.float32)
    loss = np.zeros(v.n_sets, np.float64)
    assert _load().orc_smax_forward(x.shape[0], x.shape[1], _ptr(x), _ptr(y), _ptr(t), n_classes,
                                    v.ref(), _ptr(c1), _ptr(c2), _ptr(th), float(beta),
                                    _ptr(loss), nthreads) == 0
    return loss


def smax_backward(x, y, tau_, n_classes, pop, beta, dloss=None, coef=None, coef2=None, theta=None,
                  nthreads=0):
    """fp64 gradients (dcoef, dcoef2, dtheta) of sum_s dloss[s] * loss[s] under
    the softmax head."""
    x, y = _xy(x, y)
    v = _PopView(pop)
    c1, c2, th = _params(pop, coef, coef2, theta)
    t = np.ascontiguousarray(tau_, np.float32)
    dl = np.ascontiguousarray(np.ones(v.n_sets) if dloss is None else dloss, np.float64)
    g = [np.zeros(v.n_conds, np.float64) for _ in range(3)]
    assert _load().orc_smax_backward(x.shape[0], x.shape[1], _ptr(x), _ptr(y), _ptr(t), n_classes,
                                     v.ref(), _ptr(c1), _ptr(c2), _ptr(th), float(beta), _ptr(dl),
                                     _ptr(g[0]), _ptr(g[1]), _ptr(g[2]), nthreads) == 0
    return tuple(g)
