"""Python binding of the MI355X overlapping-partition stepper (``include/ovl.h``).

Argument marshalling only: every step of the method runs in the HIP library
``lib/libovl.so``.  If that library is missing the import of this package still
works but any call raises, so a missing build never falls back to anything.

PyTorch is used for plumbing only: the stream the kernels run on and,
optionally, the caching allocator that provides the world's device buffers.
"""
from __future__ import annotations

import ctypes as C
import os
import re

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "libovl.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "ovl.h")

OK, ERR_INVALID_ARG, ERR_OOM, ERR_CAPACITY, ERR_NONFINITE, ERR_DEVICE, NOT_CONVERGED = range(7)
STATUS_NAMES = {0: "OK", 1: "INVALID_ARG", 2: "OOM", 3: "CAPACITY", 4: "NONFINITE", 5: "DEVICE", 6: "NOT_CONVERGED"}
MODE_FIXED, MODE_ADAPTIVE = 0, 1
WEIGHTS_GEODESIC, WEIGHTS_EQUAL = 0, 1
COUPLING_NONE, COUPLING_PREV_IMPULSE, COUPLING_MASS_SPLIT = 0, 1, 2
WARM_NONE, WARM_PLAIN, WARM_LEARNED = 0, 1, 2
MLP_PARAMS = 5187

DBG_FIELDS = ["contact_key", "contact_geom", "adj_off", "adj", "mask", "part_rep_off", "rep_body", "rep_d", "rep_w",
              "part_copy_off", "copy_kind", "copy_key", "copy_ia", "copy_ib", "copy_colour", "copy_lambda0",
              "copy_lambda", "rep_state", "part_iters", "part_resid", "cache_part", "cache_kind", "cache_key",
              "cache_val", "part_col_off", "copy_feat", "copy_lambdal", "part_guard", "part_rho0", "rep_cpl"]
_DBG_DTYPE = {"contact_key": (np.uint64, 1), "contact_geom": (np.float32, 8), "mask": (np.uint64, 1),
              "rep_w": (np.float32, 1), "copy_key": (np.uint64, 1), "copy_lambda0": (np.float32, 3),
              "copy_lambda": (np.float32, 3), "rep_state": (np.float32, 13), "part_resid": (np.float32, 1),
              "cache_key": (np.uint64, 1), "cache_val": (np.float32, 4), "copy_feat": (np.float32, 13),
              "copy_lambdal": (np.float32, 3), "part_rho0": (np.float32, 2),
              "rep_cpl": (np.float32, 6)}


class OvlError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class ovl_world_desc(C.Structure):
    _fields_ = [("n_bodies", C.c_int32), ("n_scenes", C.c_int32), ("n_joints", C.c_int32),
                ("scene", C.c_void_p), ("shape", C.c_void_p), ("radius", C.c_void_p), ("halflen", C.c_void_p),
                ("mass", C.c_void_p), ("inertia", C.c_void_p), ("state", C.c_void_p), ("mu", C.c_void_p),
                ("margin", C.c_void_p), ("plane_off", C.c_void_p), ("planes", C.c_void_p),
                ("ssph_off", C.c_void_p), ("ssph", C.c_void_p), ("joint_ab", C.c_void_p),
                ("joint_anchor", C.c_void_p)]


class ovl_params(C.Structure):
    _fields_ = [("dt", C.c_float), ("gravity", C.c_float * 3), ("cfm", C.c_float), ("erp", C.c_float),
                ("tol", C.c_float), ("max_iters", C.c_int32), ("mode", C.c_int32), ("warmstart", C.c_int32),
                ("seed", C.c_uint32), ("weights", C.c_int32), ("coupling", C.c_int32)]


_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
_FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class ovl_device_ctx(C.Structure):
    _fields_ = [("stream", C.c_void_p), ("alloc", _ALLOC_FN), ("free", _FREE_FN), ("user", C.c_void_p)]


class ovl_step_stats(C.Structure):
    _fields_ = [("n_contacts", C.c_int64), ("n_copies", C.c_int64), ("n_replicas", C.c_int64),
                ("n_overlap", C.c_int64), ("max_colours", C.c_int32), ("max_iters", C.c_int32),
                ("n_unconverged", C.c_int32), ("steps", C.c_int32), ("iters_total", C.c_int64),
                ("resid_sweep", C.c_float), ("resid_exact", C.c_float), ("n_lb_changes", C.c_int64),
                ("resid_exact_sum", C.c_double), ("joint_violation_max", C.c_double),
                ("joint_violation_sum", C.c_double)]


class ovl_counters(C.Structure):
    _fields_ = [("steps", C.c_int64), ("sweeps_max_total", C.c_int64), ("sweeps_part_total", C.c_int64),
                ("unconverged_total", C.c_int64), ("pgs_bytes", C.c_int64), ("pgs_launches", C.c_int64),
                ("pgs_ms", C.c_double), ("steps_capped", C.c_int64), ("pgs_ops", C.c_int64)]


class ovl_launch_cfg(C.Structure):
    _fields_ = [("pgs_block", C.c_int32), ("pgs_lds_reps", C.c_int32), ("persistent", C.c_int32),
                ("graph", C.c_int32)]


_lib = None


def lib():
    """The loaded HIP library; raises if it was not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing (run __graft_entry__.build())")
        # PyTorch bundles its own HIP runtime under the same soname as ROCm's;
        # loading torch first makes the library bind to that one runtime, so
        # the process never holds two HIP runtimes.
        import torch  # noqa: F401

        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        sig = {
            "ovl_create_world": (C.c_int, [C.POINTER(ovl_world_desc), C.POINTER(ovl_params),
                                           C.POINTER(ovl_device_ctx), C.POINTER(P)]),
            "ovl_destroy_world": (None, [P]),
            "ovl_set_params": (C.c_int, [P, C.POINTER(ovl_params)]),
            "ovl_set_partitions": (C.c_int, [P, P, C.c_int64, P, C.c_int32, C.c_int32, C.c_int32]),
            "ovl_step": (C.c_int, [P, C.c_int32, C.POINTER(ovl_step_stats), C.c_int32]),
            "ovl_read_state": (C.c_int, [P, P, C.c_int64, C.c_int32]),
            "ovl_write_state": (C.c_int, [P, P, C.c_int64, C.c_int32, C.c_int32]),
            "ovl_write_cache": (C.c_int, [P, P, P, P, P, C.c_int64]),
            "ovl_synchronize": (C.c_int, [P]),
            "ovl_read_debug": (C.c_int, [P, C.c_int32, P, C.c_int64, C.POINTER(C.c_int64)]),
            "ovl_force_iters": (C.c_int, [P, P, C.c_int32]),
            "ovl_set_load_balance": (C.c_int, [P, C.c_int32, C.c_int32, P, C.c_int64]),
            "ovl_last_error": (C.c_char_p, [P]),
            "ovl_get_counters": (C.c_int, [P, C.POINTER(ovl_counters)]),
            "ovl_profile": (C.c_int, [P, C.c_int32]),
            "ovl_set_warmstart": (C.c_int, [P, C.c_int32, P, C.c_int64]),
            "ovl_set_feature_export": (C.c_int, [P, C.c_int32]),
            "ovl_collect_training_rows": (C.c_int, [P, P, P, C.c_int64, C.POINTER(C.c_int64)]),
            "ovl_force_guard": (C.c_int, [P, P, C.c_int32]),
            "ovl_mlp_create": (C.c_int, [P, C.c_int64, C.POINTER(ovl_device_ctx), C.POINTER(P)]),
            "ovl_mlp_destroy": (None, [P]),
            "ovl_mlp_train_step": (C.c_int, [P, P, P, C.c_int64, C.c_float, C.c_int32, C.POINTER(C.c_float)]),
            "ovl_mlp_gradient": (C.c_int, [P, P, P, C.c_int64, C.c_int32, P, C.POINTER(C.c_float)]),
            "ovl_mlp_get_params": (C.c_int, [P, P, C.c_int64]),
            "ovl_mlp_last_error": (C.c_char_p, [P]),
            "ovl_mlp_infer": (C.c_int, [P, C.c_int64, P, C.c_int64, P]),
            "ovl_mlp_gradient_static": (C.c_int, [P, P, P, C.c_int64, P, P, P]),
            "ovl_set_launch": (C.c_int, [P, C.POINTER(ovl_launch_cfg)]),
            "ovl_get_launch": (C.c_int, [P, C.POINTER(ovl_launch_cfg)]),
            "ovl_launch_candidates": (C.c_int32, [P, C.c_int32]),
            "ovl_autotune": (C.c_int, [P, C.c_int32, C.POINTER(ovl_launch_cfg), P, C.c_int32]),
            "ovl_version": (C.c_char_p, []),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def header_symbols():
    """Names of every function declared in include/ovl.h."""
    with open(HEADER) as f:
        txt = f.read()
    return sorted(set(re.findall(r"\b(ovl_[a-z_]+)\s*\(", txt)))


def ovl_version() -> str:
    return lib().ovl_version().decode()


def _cfg_dict(c):
    return {f: int(getattr(c, f)) for f, _ in ovl_launch_cfg._fields_}


def launch_candidates():
    """The launch configurations the autotuner tries, in its order."""
    n = lib().ovl_launch_candidates(None, 0)
    arr = (ovl_launch_cfg * n)()
    lib().ovl_launch_candidates(C.cast(arr, C.c_void_p), n)
    return [_cfg_dict(arr[i]) for i in range(n)]


def _p(a):
    return a.ctypes.data if a is not None and a.size else None


def make_params(dt=1.0 / 60.0, gravity=(0.0, 0.0, -9.81), cfm=0.0, erp=0.2, tol=1e-4, max_iters=20,
                mode=MODE_FIXED, warmstart=WARM_PLAIN, seed=0, weights=WEIGHTS_GEODESIC,
                coupling=COUPLING_NONE) -> ovl_params:
    p = ovl_params()
    p.dt = dt
    p.gravity[0], p.gravity[1], p.gravity[2] = gravity
    p.cfm, p.erp, p.tol = cfm, erp, tol
    p.max_iters, p.mode, p.warmstart, p.seed = int(max_iters), int(mode), int(warmstart), int(seed) & 0xFFFFFFFF
    p.weights = int(weights)
    p.coupling = int(coupling)
    return p


class _TorchAllocator:
    """Device memory from PyTorch's caching allocator (kept alive until freed)."""

    def __init__(self, device):
        import torch

        self.torch = torch
        self.device = device
        self.live = {}
        self.alloc_cb = _ALLOC_FN(self._alloc)
        self.free_cb = _FREE_FN(self._free)

    def _alloc(self, nbytes, user):
        try:
            t = self.torch.empty(int(nbytes), dtype=self.torch.uint8, device=self.device)
        except Exception:
            return None
        self.live[t.data_ptr()] = t
        return t.data_ptr()

    def _free(self, ptr, user):
        self.live.pop(ptr, None)


def ovl_create_world(scene, params: ovl_params, stream=None, allocator=None):
    """Marshal a :class:`scenes.Scene` into ``ovl_world_desc`` and create the world.  Returns the handle."""
    keep = []

    def arr(x, dt):
        a = np.ascontiguousarray(x, dtype=dt)
        keep.append(a)
        return a

    d = ovl_world_desc()
    d.n_bodies, d.n_scenes, d.n_joints = scene.n_bodies, scene.n_scenes, int(scene.joint_ab.shape[0])
    for name, dt in [("scene", np.int32), ("shape", np.int32), ("radius", np.float32), ("halflen", np.float32),
                     ("mass", np.float32), ("inertia", np.float32), ("state", np.float32), ("mu", np.float32),
                     ("margin", np.float32), ("plane_off", np.int32), ("planes", np.float32),
                     ("ssph_off", np.int32), ("ssph", np.float32), ("joint_ab", np.int32),
                     ("joint_anchor", np.float32)]:
        setattr(d, name, _p(arr(getattr(scene, name), dt)))
    # plane_off / ssph_off must be readable even when empty
    d.plane_off = arr(scene.plane_off, np.int32).ctypes.data
    d.ssph_off = arr(scene.ssph_off, np.int32).ctypes.data
    ctx = ovl_device_ctx()
    ctx.stream = stream
    if allocator is not None:
        ctx.alloc = allocator.alloc_cb
        ctx.free = allocator.free_cb
    h = C.c_void_p()
    st = lib().ovl_create_world(C.byref(d), C.byref(params), C.byref(ctx), C.byref(h))
    if st != OK:
        raise OvlError(st, lib().ovl_last_error(None).decode())
    return h


class World:
    """Owning wrapper around an ``ovl_world*`` handle."""

    def __init__(self, scene, params: ovl_params = None, use_torch=True, torch_allocator=False, **kw):
        self.scene = scene
        self.params = params if params is not None else make_params(dt=scene.dt, max_iters=scene.iters, **kw)
        self.stream = None
        self._alloc = None
        if use_torch:
            import torch

            if torch.cuda.is_available():
                self.stream = torch.cuda.current_stream().cuda_stream
                if torch_allocator:
                    self._alloc = _TorchAllocator(torch.device("cuda", torch.cuda.current_device()))
        self.h = ovl_create_world(scene, self.params, self.stream, self._alloc)
        self.N = scene.n_bodies
        self.G = int(scene.n_scenes)

    def _check(self, st, allow=(OK,)):
        if st not in allow:
            raise OvlError(st, lib().ovl_last_error(self.h).decode())
        return st

    def close(self):
        if getattr(self, "h", None):
            lib().ovl_destroy_world(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, **kw):
        for k, v in kw.items():
            if k == "gravity":
                self.params.gravity[0], self.params.gravity[1], self.params.gravity[2] = v
            else:
                setattr(self.params, k, v)
        self._check(lib().ovl_set_params(self.h, C.byref(self.params)))

    def set_partitions(self, owner, parts_per_scene, halo_k=1, beta=4):
        o = np.ascontiguousarray(owner, np.int32)
        pps = np.ascontiguousarray(parts_per_scene, np.int32)
        self._check(lib().ovl_set_partitions(self.h, _p(o), self.N, _p(pps), len(pps), int(halo_k), int(beta)))
        self.G = int(pps.sum())

    def set_load_balance(self, enable=True, depth=0, sets=None):
        """Dynamic load balancing (section 5.4, Alg. 6-7): carried worker sets
        updated from each step's contacts.  sets: u64 [N] local partition bits
        (None: every body in its owner only)."""
        m = None if sets is None else np.ascontiguousarray(sets, np.uint64)
        self._check(lib().ovl_set_load_balance(self.h, int(bool(enable)), int(depth),
                                               None if m is None else _p(m), 0 if m is None else m.size))

    def step(self, n=1, stats=False, exact=False, allow_not_converged=True):
        if not stats:
            self._check(lib().ovl_step(self.h, int(n), None, 0))
            return None
        s = ovl_step_stats()
        allow = (OK, NOT_CONVERGED) if allow_not_converged else (OK,)
        st = self._check(lib().ovl_step(self.h, int(n), C.byref(s), int(bool(exact))), allow)
        out = {f: getattr(s, f) for f, _ in ovl_step_stats._fields_}
        out["status"] = st
        return out

    def sync(self):
        self._check(lib().ovl_synchronize(self.h))

    def read_state(self, allow=(OK,)):
        out = np.zeros((self.N, 13), np.float32)
        self._check(lib().ovl_read_state(self.h, _p(out), self.N, 0), allow)
        return out

    def read_state_device(self, tensor):
        self._check(lib().ovl_read_state(self.h, C.c_void_p(tensor.data_ptr()), self.N, 1))

    def write_state(self, state, keep_cache=False):
        s = np.ascontiguousarray(state, np.float32).reshape(-1, 13)
        self._check(lib().ovl_write_state(self.h, _p(s), self.N, 0, int(bool(keep_cache))))

    def force_iters(self, iters):
        if iters is None:
            self._check(lib().ovl_force_iters(self.h, None, 0))
            return
        it = np.ascontiguousarray(iters, np.int32)
        self._check(lib().ovl_force_iters(self.h, _p(it), len(it)))

    def debug(self, field):
        fid = DBG_FIELDS.index(field)
        n = C.c_int64()
        self._check(lib().ovl_read_debug(self.h, fid, None, 0, C.byref(n)))
        dt, w = _DBG_DTYPE.get(field, (np.int32, 1))
        out = np.zeros(n.value, dt)
        self._check(lib().ovl_read_debug(self.h, fid, _p(out), out.nbytes, C.byref(n)))
        return out.reshape(-1, w) if w > 1 else out

    def profile(self, enable=True):
        self._check(lib().ovl_profile(self.h, int(bool(enable))))

    def counters(self):
        c = ovl_counters()
        self._check(lib().ovl_get_counters(self.h, C.byref(c)))
        return {f: getattr(c, f) for f, _ in ovl_counters._fields_}

    def set_warmstart(self, mode, params=None):
        if params is None:
            self._check(lib().ovl_set_warmstart(self.h, int(mode), None, 0))
        else:
            p = np.ascontiguousarray(params, np.float32)
            self._check(lib().ovl_set_warmstart(self.h, int(mode), _p(p), p.size))

    def set_feature_export(self, enable=True):
        self._check(lib().ovl_set_feature_export(self.h, int(bool(enable))))

    def training_rows(self):
        n = C.c_int64()
        self._check(lib().ovl_collect_training_rows(self.h, None, None, 0, C.byref(n)))
        X = np.zeros((n.value, 12), np.float32)
        T = np.zeros((n.value, 3), np.float32)
        self._check(lib().ovl_collect_training_rows(self.h, _p(X), _p(T), n.value, C.byref(n)))
        return X, T

    def force_guard(self, choice):
        if choice is None:
            self._check(lib().ovl_force_guard(self.h, None, 0))
            return
        c = np.ascontiguousarray(choice, np.int32)
        self._check(lib().ovl_force_guard(self.h, _p(c), len(c)))

    def cache(self):
        return {k: self.debug(k) for k in ("cache_part", "cache_kind", "cache_key", "cache_val")}

    def write_cache(self, cache):
        """Restore a warm-start cache exported by cache()."""
        part = np.ascontiguousarray(cache["cache_part"], np.int32)
        kind = np.ascontiguousarray(cache["cache_kind"], np.int32)
        key = np.ascontiguousarray(cache["cache_key"], np.uint64)
        val = np.ascontiguousarray(cache["cache_val"], np.float32).reshape(-1, 4)
        self._check(lib().ovl_write_cache(self.h, _p(part), _p(kind), _p(key), _p(val), len(part)))

    def set_launch(self, pgs_block=1024, pgs_lds_reps=4800, persistent=0, graph=0):
        c = ovl_launch_cfg(int(pgs_block), int(pgs_lds_reps), int(persistent), int(graph))
        self._check(lib().ovl_set_launch(self.h, C.byref(c)))

    def get_launch(self):
        c = ovl_launch_cfg()
        self._check(lib().ovl_get_launch(self.h, C.byref(c)))
        return _cfg_dict(c)

    def autotune(self, trials=3):
        """Runs one step while timing every candidate launch configuration on it;
        keeps the fastest.  Returns (chosen config, {candidate index: ms})."""
        n = lib().ovl_launch_candidates(None, 0)
        ms = np.zeros(n, np.float32)
        c = ovl_launch_cfg()
        self._check(lib().ovl_autotune(self.h, int(trials), C.byref(c), _p(ms), n))
        return _cfg_dict(c), ms


def ovl_mlp_infer(params, x):
    """BF16 matrix-core inference of the warm-start network: x [n,12] -> y [n,3]."""
    p = np.ascontiguousarray(params, np.float32)
    X = np.ascontiguousarray(x, np.float32).reshape(-1, 12)
    Y = np.zeros((X.shape[0], 3), np.float32)
    st = lib().ovl_mlp_infer(_p(p), p.size, _p(X), X.shape[0], _p(Y))
    if st != OK:
        raise OvlError(st, "ovl_mlp_infer")
    return Y


MLP_STATIC_ROWS = 8192  # OVL_MLP_STATIC_ROWS


def ovl_mlp_gradient_static(params, x, t, grad, loss, stream=None):
    """Gradient and loss of a batch without any allocation: every argument is a
    contiguous float32 device tensor on the current device (params [5187],
    x [n, 12], t [n, 3], grad [5187] and loss [1] written), queued on the HIP
    stream handle `stream` (None: the null stream)."""
    n = int(x.shape[0])
    st = lib().ovl_mlp_gradient_static(C.c_void_p(params.data_ptr()), C.c_void_p(x.data_ptr()),
                                       C.c_void_p(t.data_ptr()), n, C.c_void_p(grad.data_ptr()),
                                       C.c_void_p(loss.data_ptr()), C.c_void_p(stream))
    if st != OK:
        raise OvlError(st, lib().ovl_mlp_last_error(None).decode())


class Trainer:
    """The device trainer of the warm-start network (``ovl_mlp_*``)."""

    def __init__(self, params, stream=None):
        p = np.ascontiguousarray(params, np.float32)
        ctx = ovl_device_ctx()
        ctx.stream = stream
        self.h = C.c_void_p()
        st = lib().ovl_mlp_create(_p(p), p.size, C.byref(ctx), C.byref(self.h))
        if st != OK:
            raise OvlError(st, lib().ovl_mlp_last_error(None).decode())

    def _check(self, st):
        if st != OK:
            raise OvlError(st, lib().ovl_mlp_last_error(self.h).decode())

    def step(self, x, t, lr):
        """One Adam step; x, t are host arrays or torch CUDA tensors."""
        loss = C.c_float()
        if hasattr(x, "data_ptr"):
            self._check(lib().ovl_mlp_train_step(self.h, C.c_void_p(x.data_ptr()), C.c_void_p(t.data_ptr()),
                                                 x.shape[0], float(lr), 1, C.byref(loss)))
        else:
            X = np.ascontiguousarray(x, np.float32)
            T = np.ascontiguousarray(t, np.float32)
            self._check(lib().ovl_mlp_train_step(self.h, _p(X), _p(T), X.shape[0], float(lr), 0, C.byref(loss)))
        return loss.value

    def gradient(self, x, t):
        X = np.ascontiguousarray(x, np.float32)
        T = np.ascontiguousarray(t, np.float32)
        g = np.zeros(MLP_PARAMS, np.float32)
        loss = C.c_float()
        self._check(lib().ovl_mlp_gradient(self.h, _p(X), _p(T), X.shape[0], 0, _p(g), C.byref(loss)))
        return loss.value, g

    def params(self):
        p = np.zeros(MLP_PARAMS, np.float32)
        self._check(lib().ovl_mlp_get_params(self.h, _p(p), MLP_PARAMS))
        return p

    def close(self):
        if getattr(self, "h", None) and self.h.value:
            lib().ovl_mlp_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
