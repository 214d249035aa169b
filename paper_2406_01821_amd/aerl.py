"""Python binding of libaerl (ctypes).

Argument marshalling only: every step of the computation runs in the HIP
kernels of ``libaerl.so``.  PyTorch supplies device memory and streams.
The raw entry points keep the C names (``aerl_create``, ``aerl_upload_dataset``,
``aerl_eval_population``, ...); ``Context`` wraps them for torch tensors.
Importing this module raises if the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np
import torch

from .population import Dataset, Population

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libaerl.so")

AERL_OK, AERL_EINVAL, AERL_ENOMEM, AERL_EDEVICE, AERL_ENOENT = 0, -1, -2, -3, -4
AERL_EAGAIN, AERL_ETIMEDOUT, AERL_ESTATE = -5, -6, -7
AERL_MAX_CLASSES = 64
AERL_TILE = 256
AERL_NOALLOC_SCRATCH_BYTES = 16 << 20
STATUS_NAMES = {0: "AERL_OK", -1: "AERL_EINVAL", -2: "AERL_ENOMEM", -3: "AERL_EDEVICE",
                -4: "AERL_ENOENT", -5: "AERL_EAGAIN", -6: "AERL_ETIMEDOUT", -7: "AERL_ESTATE"}


class AerlError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class aerl_population(C.Structure):
    _fields_ = [("n_sets", C.c_int32),
                ("set_rule_off", C.c_void_p), ("set_default", C.c_void_p),
                ("rule_cond_off", C.c_void_p), ("rule_class", C.c_void_p),
                ("op", C.c_void_p), ("kind", C.c_void_p), ("f", C.c_void_p), ("g", C.c_void_p),
                ("coef", C.c_void_p), ("coef2", C.c_void_p), ("theta", C.c_void_p),
                ("cat_mask", C.c_void_p)]


class aerl_dataset_info(C.Structure):
    _fields_ = [("n", C.c_int64), ("n_pad", C.c_int64), ("n_features", C.c_int32),
                ("n_classes", C.c_int32), ("class_count", C.c_int64 * AERL_MAX_CLASSES),
                ("x_fm", C.c_void_p), ("y_pad", C.c_void_p), ("perm", C.c_void_p),
                ("tau", C.c_void_p)]


class aerl_eval_launch(C.Structure):
    _fields_ = [("samples_per_lane", C.c_int32), ("sets_per_chunk", C.c_int32),
                ("tiles_per_group", C.c_int32), ("pad", C.c_int32), ("workgroups", C.c_int64)]


class aerl_finetune_cfg(C.Structure):
    _fields_ = [("epochs", C.c_int32), ("optimizer", C.c_int32), ("lr", C.c_float),
                ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float)]


class aerl_evolve_cfg(C.Structure):
    _fields_ = [("pool", C.c_int32), ("tournament", C.c_int32), ("elite", C.c_int32),
                ("max_rules", C.c_int32), ("max_conds", C.c_int32), ("ff_frac", C.c_float),
                ("p_crossover", C.c_float), ("p_coef", C.c_float), ("p_struct", C.c_float),
                ("tune_epochs", C.c_int32), ("tune", aerl_finetune_cfg), ("seed", C.c_uint64)]


class aerl_population_out(C.Structure):
    _fields_ = [("n_sets", C.c_int32), ("n_rules", C.c_int32), ("n_conds", C.c_int32),
                ("set_rule_off", C.c_void_p), ("set_default", C.c_void_p),
                ("rule_cond_off", C.c_void_p), ("rule_class", C.c_void_p),
                ("op", C.c_void_p), ("kind", C.c_void_p), ("f", C.c_void_p), ("g", C.c_void_p),
                ("coef", C.c_void_p), ("coef2", C.c_void_p), ("theta", C.c_void_p)]


class aerl_evolve_info(C.Structure):
    _fields_ = [("generation", C.c_int32), ("pad", C.c_int32), ("pool", aerl_population),
                ("fitness", C.c_void_p), ("tuned_coef", C.c_void_p), ("tuned_coef2", C.c_void_p),
                ("tuned_theta", C.c_void_p), ("rng_state", C.c_uint64),
                ("seconds_eval", C.c_double), ("seconds_tune", C.c_double),
                ("seconds_breed", C.c_double)]


class aerl_batch_item(C.Structure):
    _fields_ = [("dataset_id", C.c_int32), ("pop_id", C.c_int32),
                ("correct", C.c_void_p), ("confusion", C.c_void_p)]


class aerl_batch_cfg(C.Structure):
    _fields_ = [("sets_per_task", C.c_int32), ("tiles_per_task", C.c_int32),
                ("tile_kib", C.c_int32)]


AERL_BATCH_GRAPH = 1
AERL_OPT_ADAM, AERL_OPT_SGD = 0, 1
AERL_REQ_FITNESS, AERL_REQ_PREDICT = 0, 1


class aerl_serve_cfg(C.Structure):
    _fields_ = [("max_batch", C.c_int32), ("max_inflight", C.c_int32)]


class aerl_request(C.Structure):
    _fields_ = [("kind", C.c_int32), ("dataset_id", C.c_int32),
                ("pop", C.POINTER(aerl_population)), ("n_features", C.c_int32),
                ("n_classes", C.c_int32), ("set_index", C.c_int32), ("rows", C.c_void_p),
                ("n_rows", C.c_int64), ("correct", C.c_void_p), ("confusion", C.c_void_p),
                ("pred", C.c_void_p)]


class aerl_result(C.Structure):
    _fields_ = [("status", C.c_int32), ("batch_size", C.c_int32), ("queue_us", C.c_double),
                ("latency_us", C.c_double)]


class aerl_serve_stats_t(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("launches", C.c_int64),
                ("p50_us", C.c_double), ("p99_us", C.c_double), ("mean_us", C.c_double),
                ("max_us", C.c_double), ("requests_per_s", C.c_double),
                ("cond_evals_per_s", C.c_double), ("mean_batch", C.c_double),
                ("arena_peak", C.c_size_t)]


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run paper_2406_01821_amd/build_lib.py "
                      "or __graft_entry__.build()")
lib = C.CDLL(LIB_PATH)

_P, _I32, _I64, _SZ = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t
_SIGS = {
    "aerl_create": ([C.POINTER(C.c_void_p), C.c_int], _I32),
    "aerl_destroy": ([_P], None),
    "aerl_last_error": ([_P], C.c_char_p),
    "aerl_max_samples": ([_I32], _I64),
    "aerl_eval_plan": ([C.POINTER(_I64), _I32, _I32, _I32, _I32, C.POINTER(aerl_eval_launch)], _I32),
    "aerl_dataset_bytes": ([_I64, _I32, _I32, C.POINTER(_SZ)], _I32),
    "aerl_upload_dataset": ([_P, _P, _P, _I64, _I32, _I32, _P, _SZ, _P, C.POINTER(_I32)], _I32),
    "aerl_dataset_query": ([_P, _I32, C.POINTER(aerl_dataset_info)], _I32),
    "aerl_release_dataset": ([_P, _I32], _I32),
    "aerl_population_bytes": ([C.POINTER(aerl_population), _I32, _I32, C.POINTER(_SZ)], _I32),
    "aerl_pack_population": ([_P, C.POINTER(aerl_population), _I32, _I32, _P, _SZ, _P,
                              C.POINTER(_I32)], _I32),
    "aerl_pack_population_host": ([C.POINTER(aerl_population), _I32, _I32, _P, _SZ], _I32),
    "aerl_release_population": ([_P, _I32], _I32),
    "aerl_eval_population_cfg": ([_P, _I32, _I32, _P, _P, _I32, _I32, _I32, _P], _I32),
    "aerl_eval_population": ([_P, _I32, _I32, _P, _P, _P], _I32),
    "aerl_predict": ([_P, _I32, _I32, _P, _I64, _P, _P], _I32),
    "aerl_batch_workspace_bytes": ([_P, C.POINTER(aerl_batch_item), _I32,
                                    C.POINTER(aerl_batch_cfg), C.POINTER(_SZ)], _I32),
    "aerl_batch_plan": ([_P, C.POINTER(aerl_batch_item), _I32, C.POINTER(aerl_batch_cfg), _P,
                         _SZ, C.c_uint32, _P, C.POINTER(_I32)], _I32),
    "aerl_batch_run": ([_P, _I32, _P], _I32),
    "aerl_batch_release": ([_P, _I32], _I32),
    "aerl_autotune": ([_P, C.POINTER(aerl_batch_item), _I32, _P, _SZ, _P,
                       C.POINTER(aerl_batch_cfg), C.POINTER(C.c_float)], _I32),
    "aerl_serve_start": ([_P, _P, _SZ, C.POINTER(aerl_serve_cfg)], _I32),
    "aerl_serve_submit": ([_P, C.POINTER(aerl_request), C.POINTER(C.c_uint64)], _I32),
    "aerl_serve_wait": ([_P, C.c_uint64, _I64, C.POINTER(aerl_result)], _I32),
    "aerl_serve_stats": ([_P, C.POINTER(aerl_serve_stats_t), _I32], _I32),
    "aerl_serve_stop": ([_P], _I32),
    "aerl_soft_workspace_bytes": ([_P, _I32, _I32, C.POINTER(_SZ), C.POINTER(_SZ)], _I32),
    "aerl_soft_forward": ([_P, _I32, _I32, _P, _P, _P, _P, _P, _SZ, _P], _I32),
    "aerl_soft_backward": ([_P, _I32, _I32, _P, _P, _P, _P, _P, _P, _P, _P, _SZ, _P], _I32),
    "aerl_soft_forward_noalloc": ([_P, _I32, _I32, _P, _P, _P, _P, _P], _I32),
    "aerl_probe_valu_rates": ([_P, _P, _P], _I32),
    "aerl_softmax_forward": ([_P, _I32, _I32, _P, _P, _P, C.c_float, _P, _P, _SZ, _P], _I32),
    "aerl_softmax_backward": ([_P, _I32, _I32, _P, _P, _P, C.c_float, _P, _P, _P, _P, _P, _SZ, _P],
                              _I32),
    "aerl_softmax_proba": ([_P, _I32, _I32, _I32, _P, _P, _P, C.c_float, _P, _I64, _P, _P, _SZ, _P],
                           _I32),
    "aerl_random_pool": ([C.POINTER(aerl_evolve_cfg), _I32, _I32, _P, _P, C.POINTER(C.c_uint64),
                          C.POINTER(aerl_population_out)], _I32),
    "aerl_breed": ([C.POINTER(aerl_population), _P, C.POINTER(aerl_evolve_cfg), _I32, _I32, _P, _P,
                    C.POINTER(C.c_uint64), C.POINTER(aerl_population_out)], _I32),
    "aerl_evolve_arena_bytes": ([_P, _I32, C.POINTER(aerl_evolve_cfg), C.POINTER(_SZ)], _I32),
    "aerl_evolve_create": ([_P, _I32, C.POINTER(aerl_evolve_cfg), _P, _P, C.POINTER(aerl_population),
                            _P, _SZ, _P, C.POINTER(_I32)], _I32),
    "aerl_evolve_run": ([_P, _I32, _I32, _P], _I32),
    "aerl_evolve_state": ([_P, _I32, C.POINTER(aerl_evolve_info)], _I32),
    "aerl_evolve_save": ([_P, _I32, C.c_char_p], _I32),
    "aerl_evolve_load": ([_P, _I32, C.c_char_p, _P, _SZ, C.POINTER(_I32)], _I32),
    "aerl_evolve_release": ([_P, _I32], _I32),
    "aerl_finetune_workspace_bytes": ([_P, _I32, _I32, C.POINTER(_SZ)], _I32),
    "aerl_finetune": ([_P, _I32, _I32, C.POINTER(aerl_finetune_cfg), _P, _P, _P, _P, _P, _SZ, _P],
                      _I32),
}
for _name, (_args, _res) in _SIGS.items():
    _fn = getattr(lib, _name)
    _fn.argtypes, _fn.restype = _args, _res
    globals()[_name] = _fn

EXPORTED = tuple(_SIGS)


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    if isinstance(t, torch.Tensor):
        return t.data_ptr()
    return t.ctypes.data


def _stream(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def max_samples(n_classes: int) -> int:
    """Largest sample count a dataset of n_classes classes may hold."""
    return int(aerl_max_samples(n_classes))


def eval_plan(class_count, n_features: int, n_sets: int, n_cu: int = 256) -> dict:
    """Launch configuration the hard evaluation picks (host arithmetic only)."""
    cc = np.ascontiguousarray(class_count, dtype=np.int64)
    out = aerl_eval_launch()
    st = aerl_eval_plan(cc.ctypes.data_as(C.POINTER(_I64)), len(cc), n_features, n_sets, n_cu,
                        C.byref(out))
    if st != AERL_OK:
        raise AerlError(st, "no launch configuration")
    return dict(samples_per_lane=out.samples_per_lane, sets_per_chunk=out.sets_per_chunk,
                tiles_per_group=out.tiles_per_group, workgroups=out.workgroups)


def pack_host(pop: Population, n_features: int, n_classes: int) -> np.ndarray:
    """Packed image of ``pop`` as the library sends it to the device (host-only
    call, no GPU needed)."""
    hp = _HostPop(pop)
    nbytes = C.c_size_t()
    st = aerl_population_bytes(C.byref(hp.s), n_features, n_classes, C.byref(nbytes))
    if st != AERL_OK:
        raise AerlError(st, "population rejected")
    out = np.zeros(nbytes.value, np.uint8)
    st = aerl_pack_population_host(C.byref(hp.s), n_features, n_classes, out.ctypes.data,
                                   nbytes.value)
    if st != AERL_OK:
        raise AerlError(st, "packing failed")
    return out


def population_status(pop: Population, n_features: int, n_classes: int) -> int:
    """Validation status of ``pop`` (host-only)."""
    hp = _HostPop(pop)
    nbytes = C.c_size_t()
    return aerl_population_bytes(C.byref(hp.s), n_features, n_classes, C.byref(nbytes))


class _HostPop:
    """Keeps contiguous host arrays of a Population alive for one call."""

    def __init__(self, pop: Population):
        i32, u8, f32 = np.int32, np.uint8, np.float32
        self.arrays = [np.ascontiguousarray(a, dtype=t) for a, t in (
            (pop.set_rule_off, i32), (pop.set_default, i32), (pop.rule_cond_off, i32),
            (pop.rule_class, i32), (pop.op, u8), (pop.kind, u8), (pop.f, i32), (pop.g, i32),
            (pop.coef, f32), (pop.coef2, f32), (pop.theta, f32),
            (pop.cat_mask, np.uint64))]
        self.s = aerl_population(pop.n_sets, *[a.ctypes.data for a in self.arrays])


def evolve_cfg(pool=100, tournament=3, elite=2, max_rules=8, max_conds=4, ff_frac=0.3,
               p_crossover=0.5, p_coef=0.2, p_struct=0.3, tune_epochs=0, optimizer="adam",
               lr=0.01, betas=(0.9, 0.999), eps=1e-8, seed=0) -> aerl_evolve_cfg:
    """An aerl_evolve_cfg (defaults: the paper's pool of 100)."""
    tune = aerl_finetune_cfg(0, AERL_OPT_ADAM if optimizer == "adam" else AERL_OPT_SGD, lr,
                             betas[0], betas[1], eps)
    return aerl_evolve_cfg(pool, tournament, elite, max_rules, max_conds, ff_frac, p_crossover,
                           p_coef, p_struct, tune_epochs, tune, seed)


class _PoolOut:
    """Caller-side arrays of a pool the library writes (at capacity)."""

    def __init__(self, cfg: aerl_evolve_cfg):
        R = cfg.pool * cfg.max_rules
        K = R * cfg.max_conds
        i32, u8, f32 = np.int32, np.uint8, np.float32
        self.a = dict(set_rule_off=np.zeros(cfg.pool + 1, i32), set_default=np.zeros(cfg.pool, i32),
                      rule_cond_off=np.zeros(R + 1, i32), rule_class=np.zeros(R, i32),
                      op=np.zeros(K, u8), kind=np.zeros(K, u8), f=np.zeros(K, i32),
                      g=np.zeros(K, i32), coef=np.zeros(K, f32), coef2=np.zeros(K, f32),
                      theta=np.zeros(K, f32))
        self.s = aerl_population_out(0, 0, 0, *[v.ctypes.data for v in self.a.values()])

    def population(self) -> Population:
        a, s = self.a, self.s
        return Population(a["set_rule_off"][:s.n_sets + 1].copy(), a["set_default"][:s.n_sets].copy(),
                          a["rule_cond_off"][:s.n_rules + 1].copy(), a["rule_class"][:s.n_rules].copy(),
                          *[a[k][:s.n_conds].copy() for k in ("op", "kind", "f", "g", "coef", "coef2",
                                                               "theta")])


def _ranges(lo, hi):
    return (np.ascontiguousarray(lo, dtype=np.float32), np.ascontiguousarray(hi, dtype=np.float32))


def random_pool(cfg: aerl_evolve_cfg, n_features: int, n_classes: int, lo, hi, state: int):
    """Host-only random pool; returns (Population, new random state)."""
    lo, hi = _ranges(lo, hi)
    out = _PoolOut(cfg)
    st = C.c_uint64(state)
    rc = aerl_random_pool(C.byref(cfg), n_features, n_classes, lo.ctypes.data, hi.ctypes.data,
                          C.byref(st), C.byref(out.s))
    if rc != AERL_OK:
        raise AerlError(rc, "aerl_random_pool failed")
    return out.population(), st.value


def breed(pop: Population, fitness, cfg: aerl_evolve_cfg, n_features: int, n_classes: int, lo, hi,
          state: int):
    """Host-only next generation; returns (Population, new random state)."""
    lo, hi = _ranges(lo, hi)
    hp = _HostPop(pop)
    fit = np.ascontiguousarray(fitness, dtype=np.int32)
    out = _PoolOut(cfg)
    st = C.c_uint64(state)
    rc = aerl_breed(C.byref(hp.s), fit.ctypes.data, C.byref(cfg), n_features, n_classes,
                    lo.ctypes.data, hi.ctypes.data, C.byref(st), C.byref(out.s))
    if rc != AERL_OK:
        raise AerlError(rc, "aerl_breed failed")
    return out.population(), st.value


@dataclass
class DeviceDataset:
    id: int
    mem: torch.Tensor
    n: int
    n_features: int
    n_classes: int


@dataclass
class DevicePopulation:
    id: int
    ws: torch.Tensor
    n_sets: int
    n_conds: int
    n_features: int
    n_classes: int


class Context:
    """One libaerl context on one GPU."""

    def __init__(self, device: int = 0):
        if not torch.cuda.is_available():
            raise RuntimeError("libaerl needs a GPU (torch.cuda.is_available() is False)")
        self.device = torch.device("cuda", device)
        h = C.c_void_p()
        st = aerl_create(C.byref(h), device)
        if st != AERL_OK:
            raise AerlError(st, "aerl_create failed")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            aerl_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def check(self, st: int):
        if st != AERL_OK:
            raise AerlError(st, aerl_last_error(self.h).decode())

    # ------------------------------------------------------------- datasets
    def upload_dataset(self, data: Dataset, stream=None) -> DeviceDataset:
        x = torch.as_tensor(data.x, dtype=torch.float32).to(self.device).contiguous()
        y = torch.as_tensor(data.y, dtype=torch.int32).to(self.device).contiguous()
        n, nf = x.shape
        nbytes = C.c_size_t()
        self.check(aerl_dataset_bytes(n, nf, data.n_classes, C.byref(nbytes)))
        mem = torch.empty(max(nbytes.value, 256), dtype=torch.uint8, device=self.device)
        did = C.c_int32()
        self.check(aerl_upload_dataset(self.h, _ptr(x), _ptr(y), n, nf, data.n_classes, _ptr(mem),
                                       nbytes.value, _stream(stream), C.byref(did)))
        return DeviceDataset(did.value, mem, n, nf, data.n_classes)

    def dataset_info(self, ds: DeviceDataset) -> dict:
        info = aerl_dataset_info()
        self.check(aerl_dataset_query(self.h, ds.id, C.byref(info)))
        n_pad, nf = info.n_pad, info.n_features

        def view(ptr, count, dtype):
            off = ptr - ds.mem.data_ptr()
            nbytes = count * torch.tensor([], dtype=dtype).element_size()
            return ds.mem[off:off + nbytes].view(dtype)

        return dict(n=info.n, n_pad=n_pad, class_count=list(info.class_count[:info.n_classes]),
                    x_fm=view(info.x_fm, nf * n_pad, torch.float32).view(nf, n_pad),
                    y_pad=view(info.y_pad, n_pad, torch.int32),
                    perm=view(info.perm, n_pad, torch.int32),
                    tau=view(info.tau, nf, torch.float32))

    def release_dataset(self, ds: DeviceDataset):
        self.check(aerl_release_dataset(self.h, ds.id))

    # ---------------------------------------------------------- populations
    def pack_population(self, pop: Population, n_features: int, n_classes: int,
                        stream=None) -> DevicePopulation:
        hp = _HostPop(pop)
        nbytes = C.c_size_t()
        st = aerl_population_bytes(C.byref(hp.s), n_features, n_classes, C.byref(nbytes))
        if st != AERL_OK:
            # repeat through the context to get the message
            ws = torch.empty(256, dtype=torch.uint8, device=self.device)
            pid = C.c_int32()
            self.check(aerl_pack_population(self.h, C.byref(hp.s), n_features, n_classes,
                                            _ptr(ws), 256, _stream(stream), C.byref(pid)))
            raise AerlError(st, "aerl_population_bytes failed")
        ws = torch.empty(nbytes.value, dtype=torch.uint8, device=self.device)
        pid = C.c_int32()
        self.check(aerl_pack_population(self.h, C.byref(hp.s), n_features, n_classes, _ptr(ws),
                                        nbytes.value, _stream(stream), C.byref(pid)))
        return DevicePopulation(pid.value, ws, pop.n_sets, pop.n_conds, n_features, n_classes)

    def release_population(self, p: DevicePopulation):
        self.check(aerl_release_population(self.h, p.id))

    # ------------------------------------------------------------ hard path
    def eval_population(self, ds: DeviceDataset, pop: DevicePopulation, confusion: bool = True,
                        out=None, stream=None, cfg=None):
        """Returns (correct int32 [P], confusion int32 [P][C][C] or None) on the device.
        ``cfg = (samples_per_lane, sets_per_chunk, tiles_per_group)`` forces a
        launch configuration."""
        if out is None:
            correct = torch.empty(pop.n_sets, dtype=torch.int32, device=self.device)
            conf = (torch.empty((pop.n_sets, ds.n_classes, ds.n_classes), dtype=torch.int32,
                                device=self.device) if confusion else None)
        else:
            correct, conf = out
        if cfg is None:
            self.check(aerl_eval_population(self.h, ds.id, pop.id, _ptr(correct), _ptr(conf),
                                            _stream(stream)))
        else:
            self.check(aerl_eval_population_cfg(self.h, ds.id, pop.id, _ptr(correct), _ptr(conf),
                                                cfg[0], cfg[1], cfg[2], _stream(stream)))
        return correct, conf

    def predict(self, pop: DevicePopulation, rows, set_index: int = 0, out=None, stream=None):
        rows = torch.as_tensor(rows, dtype=torch.float32).to(self.device).contiguous()
        n = rows.shape[0]
        pred = out if out is not None else torch.empty(n, dtype=torch.int32, device=self.device)
        self.check(aerl_predict(self.h, pop.id, set_index, _ptr(rows), n, _ptr(pred),
                                _stream(stream)))
        return pred

    # ---------------------------------------------------------- ragged batch
    def _batch_items(self, items):
        arr = (aerl_batch_item * max(len(items), 1))()
        for i, (ds, pop, correct, conf) in enumerate(items):
            arr[i] = aerl_batch_item(ds.id, pop.id, _ptr(correct), _ptr(conf))
        return arr

    def batch_outputs(self, ds: DeviceDataset, pop: DevicePopulation, confusion: bool = True):
        correct = torch.empty(pop.n_sets, dtype=torch.int32, device=self.device)
        conf = (torch.empty((pop.n_sets, ds.n_classes, ds.n_classes), dtype=torch.int32,
                            device=self.device) if confusion else None)
        return correct, conf

    def batch_workspace(self, items, cfg=None):
        """items: list of (DeviceDataset, DevicePopulation, correct, confusion-or-None)."""
        arr = self._batch_items(items)
        nb = C.c_size_t()
        c = C.byref(aerl_batch_cfg(*cfg)) if cfg is not None else None  # 2 or 3 fields
        self.check(aerl_batch_workspace_bytes(self.h, arr, len(items), c, C.byref(nb)))
        return torch.empty(max(nb.value, 256), dtype=torch.uint8, device=self.device)

    def batch_plan(self, items, ws, cfg=None, graph: bool = False, stream=None) -> "BatchPlan":
        arr = self._batch_items(items)
        c = C.byref(aerl_batch_cfg(*cfg)) if cfg is not None else None
        pid = C.c_int32()
        self.check(aerl_batch_plan(self.h, arr, len(items), c, _ptr(ws), ws.numel(),
                                   AERL_BATCH_GRAPH if graph else 0, _stream(stream),
                                   C.byref(pid)))
        return BatchPlan(self, pid.value, list(items), ws)

    def autotune(self, items, ws, stream=None):
        """Returns ((sets_per_task, tiles_per_task, tile_kib), ms)."""
        arr = self._batch_items(items)
        best = aerl_batch_cfg()
        ms = C.c_float()
        self.check(aerl_autotune(self.h, arr, len(items), _ptr(ws), ws.numel(), _stream(stream),
                                 C.byref(best), C.byref(ms)))
        return (best.sets_per_task, best.tiles_per_task, best.tile_kib), ms.value

    # -------------------------------------------------------------- serving
    def serve_start(self, arena_bytes: int, max_batch: int = 0, max_inflight: int = 0):
        """Starts the serving loop with a torch-allocated arena of arena_bytes."""
        arena = torch.empty(arena_bytes, dtype=torch.uint8, device=self.device)
        cfg = aerl_serve_cfg(max_batch, max_inflight)
        torch.cuda.synchronize()
        self.check(aerl_serve_start(self.h, _ptr(arena), arena_bytes, C.byref(cfg)))
        self.arena = arena  # kept alive while the loop runs

    def serve_submit_fitness(self, ds: DeviceDataset, pop: Population, confusion: bool = True):
        """Returns a ServeTicket; its outputs are numpy arrays filled on completion."""
        hp = _HostPop(pop)
        correct = np.zeros(pop.n_sets, np.int32)
        conf = np.zeros((pop.n_sets, ds.n_classes, ds.n_classes), np.int32) if confusion else None
        req = aerl_request(AERL_REQ_FITNESS, ds.id, C.pointer(hp.s), ds.n_features, ds.n_classes,
                           0, None, 0, _ptr(correct), _ptr(conf), None)
        t = C.c_uint64()
        self.check(aerl_serve_submit(self.h, C.byref(req), C.byref(t)))
        return ServeTicket(self, t.value, dict(correct=correct, confusion=conf))

    def serve_submit_predict(self, pop: Population, rows, n_features: int, n_classes: int,
                             set_index: int = 0):
        hp = _HostPop(pop)
        rows = np.ascontiguousarray(rows, dtype=np.float32)
        pred = np.zeros(rows.shape[0], np.int32)
        req = aerl_request(AERL_REQ_PREDICT, -1, C.pointer(hp.s), n_features, n_classes,
                           set_index, _ptr(rows), rows.shape[0], None, None, _ptr(pred))
        t = C.c_uint64()
        self.check(aerl_serve_submit(self.h, C.byref(req), C.byref(t)))
        return ServeTicket(self, t.value, dict(pred=pred))

    def serve_stats(self, reset: bool = False) -> dict:
        st = aerl_serve_stats_t()
        self.check(aerl_serve_stats(self.h, C.byref(st), 1 if reset else 0))
        return {k: getattr(st, k) for k, _ in aerl_serve_stats_t._fields_}

    def serve_stop(self):
        self.check(aerl_serve_stop(self.h))

    # ------------------------------------------------------------ soft path
    def soft_workspace(self, ds: DeviceDataset, pop: DevicePopulation, backward: bool):
        fb, bb = C.c_size_t(), C.c_size_t()
        self.check(aerl_soft_workspace_bytes(self.h, ds.id, pop.id, C.byref(fb), C.byref(bb)))
        n = bb.value if backward else fb.value
        return torch.empty(max(n, 256), dtype=torch.uint8, device=self.device)

    def soft_forward(self, ds, pop, coef, coef2, theta, ws=None, stream=None):
        ws = ws if ws is not None else self.soft_workspace(ds, pop, False)
        loss = torch.empty(pop.n_sets, dtype=torch.float32, device=self.device)
        self.check(aerl_soft_forward(self.h, ds.id, pop.id, _ptr(coef), _ptr(coef2), _ptr(theta),
                                     _ptr(loss), _ptr(ws), ws.numel(), _stream(stream)))
        return loss

    def finetune_workspace(self, ds, pop):
        nb = C.c_size_t()
        self.check(aerl_finetune_workspace_bytes(self.h, ds.id, pop.id, C.byref(nb)))
        return torch.empty(max(nb.value, 256), dtype=torch.uint8, device=self.device)

    def finetune(self, ds, pop, coef, coef2, theta, epochs: int, optimizer: str = "adam",
                 lr: float = 0.01, betas=(0.9, 0.999), eps: float = 1e-8,
                 loss_history: bool = False, ws=None, stream=None):
        """Tunes coef, coef2, theta (device fp32 tensors, updated in place) for
        ``epochs`` full-batch steps; returns the [epochs + 1][n_sets] loss
        history when asked for, else None."""
        cfg = aerl_finetune_cfg(epochs, AERL_OPT_ADAM if optimizer == "adam" else AERL_OPT_SGD,
                                lr, betas[0], betas[1], eps)
        if optimizer not in ("adam", "sgd"):
            raise ValueError(optimizer)
        ws = ws if ws is not None else self.finetune_workspace(ds, pop)
        hist = (torch.empty((epochs + 1, pop.n_sets), dtype=torch.float32, device=self.device)
                if loss_history else None)
        self.check(aerl_finetune(self.h, ds.id, pop.id, C.byref(cfg), _ptr(coef), _ptr(coef2),
                                 _ptr(theta), _ptr(hist), _ptr(ws), ws.numel(), _stream(stream)))
        return hist

    def evolve_arena(self, ds: "DeviceDataset", cfg: aerl_evolve_cfg):
        nb = C.c_size_t()
        self.check(aerl_evolve_arena_bytes(self.h, ds.id, C.byref(cfg), C.byref(nb)))
        return torch.empty(max(nb.value, 256), dtype=torch.uint8, device=self.device)

    def evolve(self, ds: "DeviceDataset", cfg: aerl_evolve_cfg, lo, hi, initial=None,
               stream=None) -> Evolution:
        """Starts an evolution loop (generation 0 evaluated on return)."""
        lo, hi = _ranges(lo, hi)
        arena = self.evolve_arena(ds, cfg)
        hp = _HostPop(initial) if initial is not None else None
        eid = C.c_int32()
        self.check(aerl_evolve_create(self.h, ds.id, C.byref(cfg), lo.ctypes.data, hi.ctypes.data,
                                      C.byref(hp.s) if hp else None, _ptr(arena), arena.numel(),
                                      _stream(stream), C.byref(eid)))
        return Evolution(self, eid.value, arena, ds.n_features)

    def evolve_load(self, ds: "DeviceDataset", path: str, cfg: aerl_evolve_cfg) -> Evolution:
        """Resumes a checkpointed loop (cfg sizes the arena; the file's own
        configuration is used)."""
        arena = self.evolve_arena(ds, cfg)
        eid = C.c_int32()
        self.check(aerl_evolve_load(self.h, ds.id, path.encode(), _ptr(arena), arena.numel(),
                                    C.byref(eid)))
        return Evolution(self, eid.value, arena, ds.n_features)

    def softmax_forward(self, ds, pop, coef, coef2, theta, beta: float, ws=None, stream=None):
        ws = ws if ws is not None else self.soft_workspace(ds, pop, False)
        loss = torch.empty(pop.n_sets, dtype=torch.float32, device=self.device)
        self.check(aerl_softmax_forward(self.h, ds.id, pop.id, _ptr(coef), _ptr(coef2), _ptr(theta),
                                        beta, _ptr(loss), _ptr(ws), ws.numel(), _stream(stream)))
        return loss

    def softmax_backward(self, ds, pop, coef, coef2, theta, beta: float, dloss, ws=None,
                         stream=None):
        ws = ws if ws is not None else self.soft_workspace(ds, pop, True)
        g = [torch.empty(pop.n_conds, dtype=torch.float32, device=self.device) for _ in range(3)]
        self.check(aerl_softmax_backward(self.h, ds.id, pop.id, _ptr(coef), _ptr(coef2), _ptr(theta),
                                         beta, _ptr(dloss), _ptr(g[0]), _ptr(g[1]), _ptr(g[2]),
                                         _ptr(ws), ws.numel(), _stream(stream)))
        return tuple(g)

    def softmax_proba(self, ds, pop, set_index: int, coef, coef2, theta, beta: float, rows,
                      ws=None, stream=None):
        """Class probabilities [n][C] of one rule set for request rows."""
        rows = torch.as_tensor(rows, dtype=torch.float32).to(self.device).contiguous()
        ws = ws if ws is not None else self.soft_workspace(ds, pop, False)
        out = torch.empty((rows.shape[0], ds.n_classes), dtype=torch.float32, device=self.device)
        self.check(aerl_softmax_proba(self.h, ds.id, pop.id, set_index, _ptr(coef), _ptr(coef2),
                                      _ptr(theta), beta, _ptr(rows), rows.shape[0], _ptr(out),
                                      _ptr(ws), ws.numel(), _stream(stream)))
        return out

    def soft_forward_noalloc(self, ds, pop, coef, coef2, theta, loss, stream=None):
        """Soft forward into the caller's ``loss`` tensor using the library's
        per-GPU scratch array (no device allocation in the call)."""
        self.check(aerl_soft_forward_noalloc(self.h, ds.id, pop.id, _ptr(coef), _ptr(coef2),
                                             _ptr(theta), _ptr(loss), _stream(stream)))
        return loss

    def probe_valu_rates(self, stream=None):
        """(multiply, transcendental) VALU lane-ops per second, measured."""
        out = (C.c_double * 2)()
        self.check(aerl_probe_valu_rates(self.h, out, _stream(stream)))
        return float(out[0]), float(out[1])

    def soft_backward(self, ds, pop, coef, coef2, theta, dloss, ws=None, stream=None):
        ws = ws if ws is not None else self.soft_workspace(ds, pop, True)
        g = [torch.empty(pop.n_conds, dtype=torch.float32, device=self.device) for _ in range(3)]
        self.check(aerl_soft_backward(self.h, ds.id, pop.id, _ptr(coef), _ptr(coef2), _ptr(theta),
                                      _ptr(dloss), _ptr(g[0]), _ptr(g[1]), _ptr(g[2]), _ptr(ws),
                                      ws.numel(), _stream(stream)))
        return tuple(g)


class Evolution:
    """A running evolution loop on the device; holds its arena."""

    def __init__(self, ctx: "Context", evo_id: int, arena, n_features: int):
        self.ctx, self.id, self.arena, self.nf = ctx, evo_id, arena, n_features

    def run(self, generations: int, stream=None):
        self.ctx.check(aerl_evolve_run(self.ctx.h, self.id, generations, _stream(stream)))

    def state(self) -> dict:
        info = aerl_evolve_info()
        self.ctx.check(aerl_evolve_state(self.ctx.h, self.id, C.byref(info)))
        p = info.pool
        n = p.n_sets
        view = lambda ptr, cnt, t: np.ctypeslib.as_array(C.cast(ptr, C.POINTER(t)), (cnt,)).copy()
        rso = view(p.set_rule_off, n + 1, C.c_int32)
        nr = int(rso[-1])
        rco = view(p.rule_cond_off, nr + 1, C.c_int32)
        nk = int(rco[-1])
        pop = Population(rso, view(p.set_default, n, C.c_int32), rco, view(p.rule_class, nr, C.c_int32),
                         view(p.op, nk, C.c_uint8), view(p.kind, nk, C.c_uint8),
                         view(p.f, nk, C.c_int32), view(p.g, nk, C.c_int32),
                         view(p.coef, nk, C.c_float), view(p.coef2, nk, C.c_float),
                         view(p.theta, nk, C.c_float))
        tuned = None
        if info.tuned_coef:
            tuned = tuple(view(ptr, nk, C.c_float)
                          for ptr in (info.tuned_coef, info.tuned_coef2, info.tuned_theta))
        return dict(generation=info.generation, pool=pop, fitness=view(info.fitness, n, C.c_int32),
                    tuned=tuned, rng_state=info.rng_state, seconds_eval=info.seconds_eval,
                    seconds_tune=info.seconds_tune, seconds_breed=info.seconds_breed)

    def save(self, path: str):
        self.ctx.check(aerl_evolve_save(self.ctx.h, self.id, path.encode()))

    def release(self):
        if self.id is not None:
            self.ctx.check(aerl_evolve_release(self.ctx.h, self.id))
            self.id = None


class ServeTicket:
    """A submitted serving request; ``wait()`` returns its outputs."""

    def __init__(self, ctx: Context, ticket: int, out: dict):
        self.ctx, self.ticket, self.out = ctx, ticket, out
        self.result = None

    def wait(self, timeout_us: int = -1) -> dict:
        if self.result is None:
            r = aerl_result()
            self.ctx.check(aerl_serve_wait(self.ctx.h, self.ticket, timeout_us, C.byref(r)))
            self.result = dict(status=r.status, batch_size=r.batch_size, queue_us=r.queue_us,
                               latency_us=r.latency_us)
            if r.status != AERL_OK:
                raise AerlError(r.status, f"served request {self.ticket} failed")
        return self.out


class BatchPlan:
    """A planned ragged batch; holds the item buffers and workspace alive."""

    def __init__(self, ctx: Context, plan_id: int, items, ws):
        self.ctx, self.id, self.items, self.ws = ctx, plan_id, items, ws

    def run(self, stream=None):
        self.ctx.check(aerl_batch_run(self.ctx.h, self.id, _stream(stream)))

    def release(self):
        if self.id is not None:
            self.ctx.check(aerl_batch_release(self.ctx.h, self.id))
            self.id = None


class SoftLoss(torch.autograd.Function):
    """loss[P] = soft relaxation loss of every rule set; gradients flow to the
    coefficient and threshold tensors through the library's adjoint kernel,
    which recomputes the sigmoids (only the parameters are saved)."""

    @staticmethod
    def forward(ctx, coef, coef2, theta, aerl_ctx: Context, ds: DeviceDataset,
                pop: DevicePopulation):
        coef, coef2, theta = coef.contiguous(), coef2.contiguous(), theta.contiguous()
        loss = aerl_ctx.soft_forward(ds, pop, coef, coef2, theta)
        ctx.save_for_backward(coef, coef2, theta)
        ctx.aerl = (aerl_ctx, ds, pop)
        return loss

    @staticmethod
    def backward(ctx, dloss):
        coef, coef2, theta = ctx.saved_tensors
        aerl_ctx, ds, pop = ctx.aerl
        g1, g2, g3 = aerl_ctx.soft_backward(ds, pop, coef, coef2, theta,
                                            dloss.contiguous().float())
        return g1, g2, g3, None, None, None


class SoftmaxLoss(torch.autograd.Function):
    """loss[P] under the softmax head (rule votes through a softmax of
    sharpness beta); gradients through the library's adjoint kernel."""

    @staticmethod
    def forward(ctx, coef, coef2, theta, aerl_ctx: Context, ds: DeviceDataset,
                pop: DevicePopulation, beta: float):
        coef, coef2, theta = coef.contiguous(), coef2.contiguous(), theta.contiguous()
        loss = aerl_ctx.softmax_forward(ds, pop, coef, coef2, theta, beta)
        ctx.save_for_backward(coef, coef2, theta)
        ctx.aerl = (aerl_ctx, ds, pop, beta)
        return loss

    @staticmethod
    def backward(ctx, dloss):
        coef, coef2, theta = ctx.saved_tensors
        aerl_ctx, ds, pop, beta = ctx.aerl
        g1, g2, g3 = aerl_ctx.softmax_backward(ds, pop, coef, coef2, theta, beta,
                                               dloss.contiguous().float())
        return g1, g2, g3, None, None, None, None
