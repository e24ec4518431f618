"""Python binding of the MI355X tree-gravity library (libgothic.so).

Argument marshalling only: every step of the computation runs in the HIP
kernels behind the C ABI declared in include/gothic.h.  PyTorch provides the
device memory and the stream; tensors are passed by pointer.  If the built
library is missing, importing this package fails (there is no fallback).

    import torch, paper_1610_07279_amd as g
    ctx = g.Context(multipole=2)
    acc_pot = ctx.tree_forces(xyzm_cuda, eps=1/512, theta=0.5, active=mask_u8)
"""
from __future__ import annotations

import ctypes as C
import os
import re

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgothic.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "gothic.h")

OK, EINVAL, ENOMEM, EDEVICE, EOVERFLOW, ECAPTURE, ENONFINITE = 0, -1, -2, -3, -4, -5, -6
KEY_MORTON, KEY_PEANO_HILBERT = 0, 1


class GothicError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"gothic error {code}: {msg}")
        self.code = code


class Params(C.Structure):
    _fields_ = [("key_kind", C.c_int), ("n_leaf", C.c_int), ("multipole", C.c_int),
                ("group_size", C.c_int), ("list_depth", C.c_int), ("compensated", C.c_int),
                ("check", C.c_int), ("timing", C.c_int), ("r_crit", C.c_float),
                ("graph", C.c_int), ("autotune", C.c_int), ("rebuild_interval", C.c_int),
                ("mac", C.c_int), ("mac_delta", C.c_float), ("ball", C.c_int),
                ("node_capacity", C.c_int64), ("max_scratch_bytes", C.c_int64),
                ("spill_per_wave", C.c_int), ("walk_width", C.c_int)]


class TuneResult(C.Structure):
    _fields_ = [("group_size", C.c_int), ("list_depth", C.c_int), ("r_crit", C.c_float),
                ("evaluations", C.c_int), ("ms", C.c_double), ("walk_width", C.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Stats(C.Structure):
    _fields_ = [("n", C.c_int64), ("n_active", C.c_int64), ("n_nodes", C.c_int64),
                ("n_groups", C.c_int64), ("n_levels", C.c_int64), ("node_entries", C.c_int64),
                ("part_entries", C.c_int64), ("interactions", C.c_int64),
                ("node_interactions", C.c_int64), ("mac_tests", C.c_int64),
                ("flags", C.c_int32), ("n_systems", C.c_int32), ("sticky_flags", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class SimInfo(C.Structure):
    _fields_ = [("n", C.c_int64), ("substep", C.c_int64), ("t", C.c_double),
                ("dt_fine", C.c_double), ("dt_max", C.c_double), ("steps", C.c_int64),
                ("last_active", C.c_int64), ("active_total", C.c_int64),
                ("interactions_total", C.c_int64), ("node_interactions_total", C.c_int64),
                ("tree_builds", C.c_int64), ("level_count", C.c_int64 * 32)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "level_count"}
        d["level_count"] = list(self.level_count)
        return d


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                          "(or python paper_1610_07279_amd/csrc/build.py)")
    lib = C.CDLL(LIB_PATH)
    P, i32, i64, f32 = C.c_void_p, C.c_int, C.c_int64, C.c_float
    lib.gothic_default_params.argtypes = [C.POINTER(Params)]
    lib.gothic_default_params.restype = None
    lib.gothic_last_error.restype = C.c_char_p
    lib.gothic_create.argtypes = [C.POINTER(P), i32, C.POINTER(Params)]
    lib.gothic_destroy.argtypes = [P]
    lib.gothic_set_params.argtypes = [P, C.POINTER(Params)]
    lib.gothic_get_params.argtypes = [P, C.POINTER(Params)]
    lib.gothic_tree_forces.argtypes = [P, i64, P, f32, f32, P, P, P]
    lib.gothic_tree_forces_noalloc.argtypes = [P, i64, P, f32, f32, P, P, P]
    lib.gothic_tree_forces_batched.argtypes = [P, i32, P, P, P, P, P, P, P]
    lib.gothic_tree_forces_ex.argtypes = [P, i32, P, P, P, P, P, P, P, P]
    lib.gothic_direct_forces.argtypes = [P, i64, P, f32, i64, P, P, P]
    lib.gothic_get_stats.argtypes = [P, C.POINTER(Stats)]
    lib.gothic_get_keys.argtypes = [P, P, P, P]
    lib.gothic_get_tree.argtypes = [P, P, P, P, P, P, P]
    lib.gothic_get_nodes.argtypes = [P, P, P, P]
    lib.gothic_get_positions.argtypes = [P, P]
    lib.gothic_get_groups.argtypes = [P, P, P, P, P, P, P, P]
    lib.gothic_get_lists.argtypes = [P, i64, P, i64, P, P, P]
    lib.gothic_get_scratch.argtypes = [P, P, P]
    lib.gothic_clear_flags.argtypes = [P, P]
    lib.gothic_get_walk_time.argtypes = [P, C.POINTER(C.c_double), C.POINTER(i64)]
    lib.gothic_sim_bind.argtypes = [P, i64, P, P, P, f32, f32, C.c_double, i32, i32, P]
    lib.gothic_sim_bind_batched.argtypes = [P, i32, P, P, P, P, P, P, C.c_double, i32, i32, P]
    lib.gothic_sim_get_steps.argtypes = [P, i32, P, P]
    lib.gothic_sim_get_tuning.argtypes = [P, i32, P, P, P, P]
    lib.gothic_sim_set_group_sizes.argtypes = [P, i32, P, P]
    lib.gothic_autotune.argtypes = [P, i32, P, P, P, P, P, P, C.POINTER(TuneResult), P]
    lib.gothic_sim_step.argtypes = [P, P]
    lib.gothic_sim_reset_counters.argtypes = [P, P]
    lib.gothic_sim_get_info.argtypes = [P, C.POINTER(SimInfo)]
    lib.gothic_sim_get_state.argtypes = [P, P, P, P]
    for name in ("gothic_create", "gothic_destroy", "gothic_set_params", "gothic_get_params",
                 "gothic_tree_forces", "gothic_tree_forces_batched", "gothic_tree_forces_ex",
                 "gothic_get_stats", "gothic_get_lists", "gothic_get_scratch",
                 "gothic_clear_flags",
                 "gothic_get_keys", "gothic_get_tree", "gothic_get_nodes", "gothic_get_groups",
                 "gothic_get_positions",
                 "gothic_get_walk_time", "gothic_sim_bind", "gothic_sim_bind_batched",
                 "gothic_sim_step", "gothic_sim_reset_counters", "gothic_sim_get_info",
                 "gothic_sim_get_state", "gothic_sim_get_steps", "gothic_sim_get_tuning",
                 "gothic_autotune"):
        getattr(lib, name).restype = i32
    return lib


lib = _load()


def header_functions(path: str = HEADER):
    """Names of every function the public header declares."""
    txt = open(path).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(gothic_[a-z_]+)\s*\(", txt)))


def _check(rc: int):
    if rc != OK:
        raise GothicError(rc, lib.gothic_last_error().decode())


def default_params() -> Params:
    p = Params()
    lib.gothic_default_params(C.byref(p))
    return p


_FLOAT_PARAMS = ("r_crit", "mac_delta")


def _need(t, name, dtype, shape, device):
    """ValueError unless t is a contiguous `dtype` tensor of `shape` (None in a
    dimension: any size) on the GPU `device` (a torch.device).  Every pointer
    the library receives goes through here first: a host or other-device
    tensor would otherwise reach the kernels as a wild address."""
    if t is None:
        raise ValueError(f"{name} is required")
    shp = tuple(t.shape)
    if t.dtype != dtype or len(shp) != len(shape) or any(
            w is not None and w != g for w, g in zip(shape, shp)):
        want = ",".join("*" if w is None else str(w) for w in shape)
        raise ValueError(f"{name} must be a {dtype} [{want}] tensor (got {t.dtype} {list(shp)})")
    if not t.is_cuda or t.device != device:
        raise ValueError(f"{name} must be on {device} (got {t.device})")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def _check_acc_old(acc_old, n, device):
    import torch
    if acc_old is not None:
        _need(acc_old, "acc_old", torch.float32, (n, 4), device)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream_of(t, stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream(t.device)
    return C.c_void_p(stream.cuda_stream)


class Context:
    """One library context (scratch, tunables) on one GPU."""

    def __init__(self, device: int = 0, **params):
        p = default_params()
        for k, v in params.items():
            if not hasattr(p, k):
                raise TypeError(f"unknown parameter {k}")
            setattr(p, k, float(v) if k in _FLOAT_PARAMS else int(v))
        h = C.c_void_p()
        _check(lib.gothic_create(C.byref(h), int(device), C.byref(p)))
        self._h = h
        self.device = device
        self._last_stream = None

    def close(self):
        if getattr(self, "_h", None):
            lib.gothic_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- params
    @property
    def params(self) -> dict:
        p = Params()
        _check(lib.gothic_get_params(self._h, C.byref(p)))
        return {k: getattr(p, k) for k, _ in Params._fields_}

    def set_params(self, **params):
        p = Params()
        _check(lib.gothic_get_params(self._h, C.byref(p)))
        for k, v in params.items():
            if not hasattr(p, k):
                raise TypeError(f"unknown parameter {k}")
            setattr(p, k, float(v) if k in _FLOAT_PARAMS else int(v))
        _check(lib.gothic_set_params(self._h, C.byref(p)))

    # ---------------------------------------------------------------- forces
    def tree_forces(self, xyzm, eps: float, theta: float, active=None, out=None, stream=None,
                    acc_old=None):
        """acc_pot [n,4] float32 (ax, ay, az, phi) for the active rows of xyzm;
        acc_old [n,4] (previous accelerations) feeds the acceleration MAC."""
        import torch
        n, out = self._forces_args(xyzm, active, out)
        s = _stream_of(xyzm, stream)
        self._last_stream = s
        if acc_old is None:
            _check(lib.gothic_tree_forces(self._h, n, _ptr(xyzm), float(eps), float(theta),
                                          _ptr(active), _ptr(out), s))
        else:
            return self.tree_forces_batched(xyzm, [0, n], eps, theta, active=active, out=out,
                                            stream=stream, acc_old=acc_old)
        return out

    def tree_forces_noalloc(self, xyzm, eps: float, theta: float, active=None, out=None,
                            stream=None):
        """As tree_forces, through the scratch-free entry point (the library
        allocates nothing; out must be given or is allocated here, by torch)."""
        n, out = self._forces_args(xyzm, active, out)
        s = _stream_of(xyzm, stream)
        self._last_stream = s
        _check(lib.gothic_tree_forces_noalloc(self._h, n, _ptr(xyzm), float(eps), float(theta),
                                              _ptr(active), _ptr(out), s))
        return out

    @property
    def torch_device(self):
        import torch
        return torch.device("cuda", self.device)

    def _forces_args(self, xyzm, active, out):
        """Check xyzm [n,4], active [n] and out [n,4] (allocated if None): all on
        this context's GPU.  Returns (n, out)."""
        import torch
        dev = self.torch_device
        _need(xyzm, "xyzm", torch.float32, (None, 4), dev)
        n = xyzm.shape[0]
        if active is not None:
            _need(active, "active", torch.uint8, (n,), dev)
        if out is None:
            out = torch.zeros((n, 4), dtype=torch.float32, device=dev)
        _need(out, "out", torch.float32, (n, 4), dev)
        return n, out

    def direct_forces(self, xyzm, eps: float, idx=None, out=None, stream=None):
        """float64 [ni,4] (ax, ay, az, phi) by direct summation over all of
        xyzm for the targets idx (int64 GPU tensor; None = every particle)."""
        import torch
        dev = self.torch_device
        _need(xyzm, "xyzm", torch.float32, (None, 4), dev)
        n = xyzm.shape[0]
        if idx is not None:
            _need(idx, "idx", torch.int64, (None,), dev)
        ni = n if idx is None else idx.shape[0]
        if out is None:
            out = torch.empty((ni, 4), dtype=torch.float64, device=dev)
        _need(out, "out", torch.float64, (ni, 4), dev)
        s = _stream_of(xyzm, stream)
        self._last_stream = s
        _check(lib.gothic_direct_forces(self._h, n, _ptr(xyzm), float(eps), ni, _ptr(idx),
                                        _ptr(out), s))
        return out

    @staticmethod
    def _systems(offsets, eps, theta):
        import numpy as np
        offs = np.ascontiguousarray(offsets, dtype=np.int64)
        nsys = offs.size - 1
        if nsys < 1:
            raise ValueError("offsets needs at least two entries")
        e = np.ascontiguousarray(np.broadcast_to(np.asarray(eps, np.float32), (nsys,)))
        t = np.ascontiguousarray(np.broadcast_to(np.asarray(theta, np.float32), (nsys,)))
        return offs, nsys, e, t

    def tree_forces_batched(self, xyzm, offsets, eps, theta, active=None, out=None, stream=None,
                            acc_old=None):
        """Forces of nsys independent systems in one evaluation: system s owns rows
        offsets[s]:offsets[s+1] of xyzm (eps, theta: scalars or one per system)."""
        offs, nsys, e, t = self._systems(offsets, eps, theta)
        n, out = self._forces_args(xyzm, active, out)
        if offs[-1] != n:
            raise ValueError("offsets[-1] must equal the number of rows of xyzm")
        _check_acc_old(acc_old, n, self.torch_device)
        s = _stream_of(xyzm, stream)
        self._last_stream = s
        _check(lib.gothic_tree_forces_ex(
            self._h, nsys, offs.ctypes.data_as(C.c_void_p), _ptr(xyzm),
            e.ctypes.data_as(C.c_void_p), t.ctypes.data_as(C.c_void_p), _ptr(active),
            _ptr(acc_old), _ptr(out), s))
        return out

    def autotune(self, xyzm, eps, theta, active=None, offsets=None, out=None, stream=None):
        """Timed search of (group_size, list_depth, r_crit) for this workload (one
        system, or the systems given by offsets); sets them in the context and
        returns the result dict (evaluations = 0 for a cached bucket).  out
        receives the forces of a final checked evaluation."""
        import numpy as np
        n, out = self._forces_args(xyzm, active, out)
        if offsets is None:
            offsets = np.array([0, n], np.int64)
        offs, nsys, e, t = self._systems(offsets, eps, theta)
        if offs[-1] != n:
            raise ValueError("offsets[-1] must equal the number of rows of xyzm")
        res = TuneResult()
        s = _stream_of(xyzm, stream)
        self._last_stream = s
        _check(lib.gothic_autotune(self._h, nsys, offs.ctypes.data_as(C.c_void_p), _ptr(xyzm),
                                   e.ctypes.data_as(C.c_void_p), t.ctypes.data_as(C.c_void_p),
                                   _ptr(active), _ptr(out), C.byref(res), s))
        return res.as_dict()

    # ---------------------------------------------------------------- block steps
    def sim_bind(self, pos, vel, mass, eps, theta, eta=0.1, kmax=8, shared=False, stream=None):
        """Bind float64 [n,3] pos/vel and float32 [n] mass (GPU tensors, updated in
        place by sim_step) and compute the t = 0 forces and levels."""
        import torch
        dev = self.torch_device
        _need(pos, "pos", torch.float64, (None, 3), dev)
        n = pos.shape[0]
        _need(vel, "vel", torch.float64, (n, 3), dev)
        _need(mass, "mass", torch.float32, (n,), dev)
        self._sim_keep = (pos, vel, mass)
        self._sim_nsys = 1
        s = _stream_of(pos, stream)
        self._last_stream = s
        _check(lib.gothic_sim_bind(self._h, n, _ptr(pos), _ptr(vel), _ptr(mass), float(eps),
                                   float(theta), float(eta), int(kmax), int(bool(shared)), s))

    def sim_bind_batched(self, pos, vel, mass, offsets, eps, theta, eta=0.1, kmax=8, shared=False,
                         stream=None):
        """sim_bind for nsys independent systems (rows offsets[s]:offsets[s+1]), each
        with its own softening, opening angle and time-step hierarchy."""
        import torch
        offs, nsys, e, t = self._systems(offsets, eps, theta)
        dev = self.torch_device
        _need(pos, "pos", torch.float64, (None, 3), dev)
        n = pos.shape[0]
        _need(vel, "vel", torch.float64, (n, 3), dev)
        _need(mass, "mass", torch.float32, (n,), dev)
        if offs[-1] != n:
            raise ValueError("offsets[-1] must equal the number of rows of pos")
        self._sim_keep = (pos, vel, mass)
        self._sim_nsys = nsys
        s = _stream_of(pos, stream)
        self._last_stream = s
        _check(lib.gothic_sim_bind_batched(self._h, nsys, offs.ctypes.data_as(C.c_void_p),
                                           _ptr(pos), _ptr(vel), _ptr(mass),
                                           e.ctypes.data_as(C.c_void_p),
                                           t.ctypes.data_as(C.c_void_p), float(eta), int(kmax),
                                           int(bool(shared)), s))

    def sim_steps(self):
        """(dt_fine [nsys], dt_max [nsys]) float64 numpy arrays of the bound systems."""
        import numpy as np
        ns = getattr(self, "_sim_nsys", 1)
        f = np.zeros(ns, np.float64)
        m = np.zeros(ns, np.float64)
        _check(lib.gothic_sim_get_steps(self._h, ns, f.ctypes.data_as(C.c_void_p),
                                        m.ctypes.data_as(C.c_void_p)))
        return f, m

    def sim_tuning(self, nclass: int = 32, with_groups: bool = False):
        """(best r_crit per sub-step class [nclass] float32, finished searches [nclass]
        [, group size per class [nclass], walk width per class [nclass]]) of the
        online tuner (params.autotune)."""
        import numpy as np
        r = np.zeros(nclass, np.float32)
        k = np.zeros(nclass, np.int32)
        gs = np.zeros(nclass, np.int32)
        ws = np.zeros(nclass, np.int32)
        _check(lib.gothic_sim_get_tuning(self._h, nclass, r.ctypes.data_as(C.c_void_p),
                                         k.ctypes.data_as(C.c_void_p),
                                         gs.ctypes.data_as(C.c_void_p),
                                         ws.ctypes.data_as(C.c_void_p)))
        return (r, k, gs, ws) if with_groups else (r, k)

    def sim_set_group_sizes(self, sizes, widths=None):
        """Group size per sub-step class (0 = params.group_size / walk_width) and
        walk width per class (None = 64 for every class)."""
        import numpy as np
        g = np.ascontiguousarray(sizes, dtype=np.int32)
        w = None if widths is None else np.ascontiguousarray(widths, dtype=np.int32)
        if w is not None and w.size != g.size:
            raise ValueError("sizes and widths differ in length")
        _check(lib.gothic_sim_set_group_sizes(
            self._h, g.size, g.ctypes.data_as(C.c_void_p),
            None if w is None else w.ctypes.data_as(C.c_void_p)))

    def sim_step(self, nsteps: int = 1, stream=None):
        s = _stream_of(self._sim_keep[0], stream)
        for _ in range(nsteps):
            _check(lib.gothic_sim_step(self._h, s))

    def sim_reset_counters(self, stream=None):
        _check(lib.gothic_sim_reset_counters(self._h, _stream_of(self._sim_keep[0], stream)))

    def sim_info(self) -> dict:
        info = SimInfo()
        _check(lib.gothic_sim_get_info(self._h, C.byref(info)))
        return info.as_dict()

    def sim_state(self):
        """(acc_pot [n,4] float32, levels [n] uint8, last sub-step [n] int64) as numpy"""
        import torch
        n = self._sim_keep[0].shape[0]
        dev = self._sim_keep[0].device
        a = torch.empty((n, 4), dtype=torch.float32, device=dev)
        lv = torch.empty(n, dtype=torch.uint8, device=dev)
        last = torch.empty(n, dtype=torch.int64, device=dev)
        _check(lib.gothic_sim_get_state(self._h, _ptr(a), _ptr(lv), _ptr(last)))
        return a.cpu().numpy(), lv.cpu().numpy(), last.cpu().numpy()

    def walk_time(self):
        """(total ms, launches) of the walk kernels timed since the last call."""
        ms, k = C.c_double(), C.c_int64()
        _check(lib.gothic_get_walk_time(self._h, C.byref(ms), C.byref(k)))
        return ms.value, k.value

    # ---------------------------------------------------------------- introspection
    def stats(self) -> dict:
        st = Stats()
        _check(lib.gothic_get_stats(self._h, C.byref(st)))
        return st.as_dict()

    def _stats_raw(self) -> dict:
        st = Stats()
        lib.gothic_get_stats(self._h, C.byref(st))
        return st.as_dict()

    def keys(self):
        """(keys_sorted uint64 numpy, perm uint32 numpy, cube float64 numpy): cube is
        [4] for one system, [n_systems, 4] for a batched evaluation."""
        import torch
        st = self._stats_raw()
        n, ns = st["n"], max(st["n_systems"], 1)
        dev = torch.device("cuda", self.device)
        k = torch.empty(max(n, 1), dtype=torch.int64, device=dev)
        p = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
        cb = torch.empty((ns, 4), dtype=torch.float64, device=dev)
        _check(lib.gothic_get_keys(self._h, _ptr(k), _ptr(p), _ptr(cb)))
        cube = cb.cpu().numpy()
        return (k[:n].cpu().numpy().view("uint64"), p[:n].cpu().numpy().view("uint32"),
                cube[0] if ns == 1 else cube)

    def tree(self) -> dict:
        import torch
        nn = self._stats_raw()["n_nodes"]
        dev = torch.device("cuda", self.device)
        m = max(nn, 1)
        f = torch.empty(m, dtype=torch.int32, device=dev)
        c = torch.empty(m, dtype=torch.int32, device=dev)
        cf = torch.empty(m, dtype=torch.int32, device=dev)
        nc = torch.empty(m, dtype=torch.uint8, device=dev)
        lv = torch.empty(m, dtype=torch.uint8, device=dev)
        nn_out = C.c_int64()
        _check(lib.gothic_get_tree(self._h, C.byref(nn_out), _ptr(f), _ptr(c), _ptr(cf), _ptr(nc),
                                   _ptr(lv)))
        if nn_out.value != nn:
            raise GothicError(EINVAL, "node count changed between calls")
        u = lambda t: t[:nn].cpu().numpy().view("uint32")
        return dict(first=u(f), count=u(c), child_first=u(cf), n_child=nc[:nn].cpu().numpy(),
                    level=lv[:nn].cpu().numpy())

    def nodes(self):
        """(com_m [nn,4] float32, b [nn] float32, quad [nn,6] float32) as numpy"""
        import torch
        nn = self._stats_raw()["n_nodes"]
        dev = torch.device("cuda", self.device)
        m = max(nn, 1)
        cm = torch.empty((m, 4), dtype=torch.float32, device=dev)
        b = torch.empty(m, dtype=torch.float32, device=dev)
        q = torch.empty((m, 6), dtype=torch.float32, device=dev)
        _check(lib.gothic_get_nodes(self._h, _ptr(cm), _ptr(b), _ptr(q)))
        return cm[:nn].cpu().numpy(), b[:nn].cpu().numpy(), q[:nn].cpu().numpy()

    def positions(self):
        """[n,4] float32 numpy: the positions and masses of the last evaluation in
        key order (the float32 prediction for a block sub-step)."""
        import torch
        n = self._stats_raw()["n"]
        xs = torch.empty((max(n, 1), 4), dtype=torch.float32, device=self.torch_device)
        _check(lib.gothic_get_positions(self._h, _ptr(xs)))
        return xs[:n].cpu().numpy()

    def groups(self) -> dict:
        import torch
        st = self._stats_raw()
        na, ng = st["n_active"], st["n_groups"]
        dev = torch.device("cuda", self.device)
        al = torch.empty(max(na, 1), dtype=torch.int32, device=dev)
        gf = torch.empty(max(ng, 1), dtype=torch.int32, device=dev)
        gc = torch.empty(max(ng, 1), dtype=torch.int32, device=dev)
        ball = torch.empty((max(ng, 1), 4), dtype=torch.float32, device=dev)
        ent = torch.empty((max(ng, 1), 2), dtype=torch.int32, device=dev)
        na_out, ng_out = C.c_int64(), C.c_int64()
        _check(lib.gothic_get_groups(self._h, C.byref(na_out), C.byref(ng_out), _ptr(al),
                                     _ptr(gf), _ptr(gc), _ptr(ball), _ptr(ent)))
        if (na_out.value, ng_out.value) != (na, ng):
            raise GothicError(EINVAL, "group counts changed between calls")
        u = lambda t, k: t[:k].cpu().numpy().view("uint32")
        return dict(alist=u(al, na), first=u(gf, ng), count=u(gc, ng),
                    ball=ball[:ng].cpu().numpy(), entries=u(ent, ng))


    def lists(self, groups, cap: int = 1 << 16):
        """Interaction lists of the given groups of the last evaluation: a list of
        (nodes uint32 array, leaves uint32 array) per group (accepted pseudo
        j-particles and opened leaves, node indices as in tree()), and the
        [n,4] float32 forces the re-walk wrote for those groups' particles
        (NaN elsewhere)."""
        import numpy as np
        import torch
        gsel = np.ascontiguousarray(groups, dtype=np.uint32)
        k = gsel.size
        dev = self.torch_device
        n = self._stats_raw()["n"]
        ent = torch.empty((max(k, 1), cap), dtype=torch.int32, device=dev)
        cnt = torch.empty((max(k, 1), 2), dtype=torch.int32, device=dev)
        acc = torch.full((max(n, 1), 4), float("nan"), dtype=torch.float32, device=dev)
        _check(lib.gothic_get_lists(self._h, k, gsel.ctypes.data_as(C.c_void_p), cap, _ptr(ent),
                                    _ptr(cnt), _ptr(acc)))
        e = ent.cpu().numpy().view("uint32")
        c = cnt.cpu().numpy().view("uint32")
        out = []
        for q in range(k):
            tot = int(c[q, 0]) + int(c[q, 1])
            if tot > cap:
                raise ValueError(f"group {gsel[q]} has {tot} list entries, more than cap {cap}")
            row = e[q, :tot]
            leaf = (row & 0x80000000) != 0
            out.append((row[~leaf].copy(), (row[leaf] & 0x7fffffff).copy()))
        return out, acc[:n].cpu().numpy()

    def scratch(self):
        """(bytes held, bytes a refused call needed) of this context's scratch."""
        held, req = C.c_int64(), C.c_int64()
        _check(lib.gothic_get_scratch(self._h, C.byref(held), C.byref(req)))
        return held.value, req.value

    def clear_flags(self, stream=None):
        import torch
        s = stream if stream is not None else torch.cuda.current_stream(self.torch_device)
        _check(lib.gothic_clear_flags(self._h, C.c_void_p(s.cuda_stream)))


_default_ctx = {}


def tree_forces(xyzm, eps, theta, active=None, out=None, **params):
    """Convenience wrapper with a cached context per (device, params)."""
    key = (xyzm.device.index or 0, tuple(sorted(params.items())))
    ctx = _default_ctx.get(key)
    if ctx is None:
        ctx = _default_ctx[key] = Context(device=key[0], **params)
    return ctx.tree_forces(xyzm, eps, theta, active=active, out=out)
