"""Python binding of the MI355X EI-ZO library (`libezo.so`, C ABI in include/ezo.h).

Argument marshalling only: every step runs in the HIP kernels behind the C
ABI.  Device buffers are torch tensors on the context's device; work goes to
torch's current stream unless a stream is given.  The shared library must be
built (`python -m paper_2504_10783_amd.build`); importing this package does
not need a GPU, but every compute call does, and a missing library raises.
"""
from __future__ import annotations

import collections.abc
import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libezo.so")

EZO_OK, EZO_E_INVALID, EZO_E_HIP, EZO_E_CAPACITY, EZO_E_NOMEM, EZO_E_UNSUPPORTED = 0, -1, -2, -3, -4, -5
CERTIFIED, MAX_ITERS, IN_COLLISION, INVALID, CONTAINED = 0, 1, 2, 3, 4
MAX_DOF = 8
NOALLOC_MAX_OBSTACLES = 4096      # EZO_NOALLOC_MAX_OBSTACLES

EXPORTS = (
    "ezo_ctx_create", "ezo_ctx_destroy", "ezo_last_error", "ezo_set_obstacle_boxes", "ezo_robot_create",
    "ezo_robot_destroy",
    "ezo_check_collisions", "ezo_check_collisions_noalloc", "ezo_sphere_centres", "ezo_test_constants", "ezo_sample_polytopes",
    "ezo_test_and_select", "ezo_project_bisect", "ezo_place_hyperplanes", "ezo_inflate_edges", "ezo_inflate_paths",
    "ezo_set_phase_timing", "ezo_get_phase_timing",
    "ezo_surrogate_num_params", "ezo_surrogate_create", "ezo_surrogate_destroy", "ezo_surrogate_set_params",
    "ezo_surrogate_get_params", "ezo_surrogate_train", "ezo_surrogate_loss_grad", "ezo_surrogate_predict",
    "ezo_surrogate_calibrate", "ezo_surrogate_set_margin", "ezo_surrogate_set_scope",
    "ezo_surrogate_miss_rate",
    "ezo_set_autotune", "ezo_tune_cache_export", "ezo_tune_cache_import", "ezo_tune_cache_clear",
    "ezo_check_path", "ezo_update_polytopes", "ezo_segments_contained",
    "ezo_collision_map", "ezo_collision_map_lists",
)
PHASES = ("sample", "check", "test", "bisect", "place", "advance")


class EzoError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"ezo error {code}: {msg}")
        self.code = code


class RobotDesc(C.Structure):
    _fields_ = [("dof", C.c_int32), ("dh_a", C.POINTER(C.c_double)), ("dh_alpha", C.POINTER(C.c_double)),
                ("dh_d", C.POINTER(C.c_double)), ("q_lo", C.POINTER(C.c_double)), ("q_hi", C.POINTER(C.c_double)),
                ("n_spheres", C.c_int32), ("sphere_link", C.POINTER(C.c_int32)),
                ("sphere_xyz", C.POINTER(C.c_double)), ("sphere_r", C.POINTER(C.c_double)),
                ("n_self_pairs", C.c_int32), ("self_pairs", C.POINTER(C.c_int32)),
                ("n_boxes", C.c_int32), ("box_link", C.POINTER(C.c_int32)), ("box_pose", C.POINTER(C.c_double)),
                ("box_half", C.POINTER(C.c_double)), ("n_box_pairs", C.c_int32),
                ("box_pairs", C.POINTER(C.c_int32)), ("joint_type", C.POINTER(C.c_int32))]


class Params(C.Structure):
    _fields_ = [("eps", C.c_double), ("delta", C.c_double), ("tau", C.c_double),
                ("step_back_max", C.c_double), ("t_col", C.c_double), ("n_p", C.c_int32),
                ("n_f", C.c_int32), ("n_b", C.c_int32), ("n_mix", C.c_int32), ("max_iters", C.c_int32),
                ("face_capacity", C.c_int32), ("seed", C.c_uint64), ("edge_id_base", C.c_int64),
                ("surrogate", C.c_void_p), ("row_points", C.c_void_p)]


class TrainParams(C.Structure):
    _fields_ = [("epochs", C.c_int32), ("batch", C.c_int32), ("lr", C.c_double), ("beta1", C.c_double),
                ("beta2", C.c_double), ("adam_eps", C.c_double), ("huber_delta", C.c_double),
                ("clip_lo", C.c_double), ("clip_hi", C.c_double), ("seed", C.c_uint64)]


class EdgeStats(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("planes", C.c_int32), ("final_m", C.c_int64),
                ("test_collisions", C.c_int64), ("samples", C.c_int64), ("exact_checks", C.c_int64),
                ("screened_checks", C.c_int64)]


class EdgeStatsView(collections.abc.Sequence):
    """Per-edge statistics of one call over the C array the library filled:
    item e is a dict of the fields, built when it is read; `.array` is a
    zero-copy numpy structured view (for sums over many edges)."""

    def __init__(self, arr, n):
        self._a, self._n = arr, n

    def __len__(self):
        return self._n

    def __getitem__(self, i):
        if isinstance(i, slice):
            return [self[j] for j in range(*i.indices(self._n))]
        if i < 0:
            i += self._n
        if not 0 <= i < self._n:
            raise IndexError(i)
        e = self._a[i]
        return {k: getattr(e, k) for k, _ in EdgeStats._fields_}

    def __eq__(self, other):
        return list(self) == list(other)

    @property
    def array(self):
        dt = np.dtype([(k, np.int32 if t is C.c_int32 else np.int64) for k, t in EdgeStats._fields_], align=True)
        return np.frombuffer(self._a, dtype=dt, count=self._n)


_lib = None


def lib():
    """The loaded C library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2504_10783_amd.build`")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, u64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64, C.c_double
        L.ezo_ctx_create.argtypes = [i32, C.POINTER(vp)]
        L.ezo_ctx_destroy.argtypes = [vp]
        L.ezo_ctx_destroy.restype = None
        L.ezo_last_error.argtypes = [vp]
        L.ezo_last_error.restype = C.c_char_p
        L.ezo_set_obstacle_boxes.argtypes = [vp, C.POINTER(C.c_float), i32]
        L.ezo_robot_create.argtypes = [vp, C.POINTER(RobotDesc), C.POINTER(vp)]
        L.ezo_robot_destroy.argtypes = [vp]
        L.ezo_robot_destroy.restype = None
        L.ezo_check_collisions.argtypes = [vp, vp, vp, i32, vp, i64, i64, i64, vp, vp, vp, vp]
        L.ezo_check_collisions_noalloc.argtypes = [vp, vp, vp, i32, vp, i64, i64, i64, vp, vp, vp, vp]
        L.ezo_sphere_centres.argtypes = [vp, vp, vp, i64, i64, i64, vp, vp]
        L.ezo_test_constants.argtypes = [dbl, dbl, dbl, i32, C.POINTER(i64), C.POINTER(i64)]
        L.ezo_sample_polytopes.argtypes = [vp, i32, vp, vp, vp, i32, vp, i32, i32, i32, u64, i64, i32, vp, i64, vp]
        L.ezo_test_and_select.argtypes = [vp, vp, i32, i64, i32, i64, i64, i32, vp, vp, i32, vp, vp, vp]
        L.ezo_project_bisect.argtypes = [vp, vp, vp, i32, vp, i32, vp, i64, vp, vp, i32, i32, vp, vp, vp, vp, vp]
        L.ezo_place_hyperplanes.argtypes = [vp, i32, vp, i32, vp, vp, vp, vp, i32, i32, dbl, dbl, vp, vp, vp, i32,
                                            vp, vp, vp, vp]
        L.ezo_inflate_edges.argtypes = [vp, vp, vp, i32, vp, i32, C.POINTER(Params), vp, vp, vp, vp,
                                        C.POINTER(EdgeStats), vp]
        L.ezo_inflate_paths.argtypes = [vp, vp, vp, i32, vp, C.POINTER(i32), i32, C.POINTER(Params), vp, vp, vp,
                                        vp, vp, C.POINTER(EdgeStats), vp]
        L.ezo_set_phase_timing.argtypes = [vp, i32]
        L.ezo_get_phase_timing.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(i64), C.POINTER(i64)]
        tp = C.POINTER(TrainParams)
        L.ezo_surrogate_num_params.argtypes = [i32, i32]
        L.ezo_surrogate_num_params.restype = i64
        L.ezo_surrogate_create.argtypes = [vp, i32, i32, u64, C.POINTER(vp)]
        L.ezo_surrogate_destroy.argtypes = [vp]
        L.ezo_surrogate_destroy.restype = None
        L.ezo_surrogate_set_params.argtypes = [vp, C.POINTER(C.c_float), i64]
        L.ezo_surrogate_get_params.argtypes = [vp, C.POINTER(C.c_float), i64]
        L.ezo_surrogate_train.argtypes = [vp, vp, vp, vp, i64, tp, C.POINTER(C.c_float), vp]
        L.ezo_surrogate_loss_grad.argtypes = [vp, vp, vp, vp, i64, tp, C.POINTER(C.c_float), C.POINTER(dbl), vp]
        L.ezo_surrogate_predict.argtypes = [vp, vp, vp, i64, vp, vp]
        L.ezo_surrogate_calibrate.argtypes = [vp, vp, vp, vp, i64, dbl, C.POINTER(dbl), vp]
        L.ezo_surrogate_set_margin.argtypes = [vp, dbl]
        L.ezo_surrogate_set_scope.argtypes = [vp, i32]
        L.ezo_surrogate_miss_rate.argtypes = [vp, vp, vp, vp, i64, C.POINTER(dbl), C.POINTER(dbl), vp]
        L.ezo_check_path.argtypes = [vp, vp, vp, i32, vp, i32, dbl, vp, i32, C.POINTER(i64), C.POINTER(i64), vp]
        L.ezo_update_polytopes.argtypes = [vp, vp, vp, i32, vp, i32, vp, i32, i32, i32, dbl, dbl, vp, vp, vp, i32,
                                           vp, vp, vp]
        L.ezo_segments_contained.argtypes = [vp, i32, vp, vp, vp, i32, i32, vp, i32, dbl, vp, vp]
        L.ezo_collision_map.argtypes = [vp, vp, vp, i64, C.POINTER(C.c_float), C.c_float, C.POINTER(i32), vp, i64, vp]
        L.ezo_collision_map_lists.argtypes = [vp, vp, i64, i64, i64, vp, vp, i64, C.POINTER(i64), vp]
        L.ezo_set_autotune.argtypes = [vp, i32]
        L.ezo_tune_cache_export.argtypes = [C.c_char_p, i64, C.POINTER(i64)]
        L.ezo_tune_cache_import.argtypes = [C.c_char_p, C.POINTER(i32)]
        L.ezo_tune_cache_clear.argtypes = []
        L.ezo_tune_cache_clear.restype = None
        for name in EXPORTS:
            fn = getattr(L, name)
            if fn.restype is C.c_int:
                fn.restype = C.c_int32
        _lib = L
    return _lib


def _torch():
    import torch
    return torch


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream):
    torch = _torch()
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _need(t, dtype, name, numel=None):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() < numel:
        raise ValueError(f"{name} holds {t.numel()} elements, needs {numel}")


def test_constants(eps: float, delta: float, tau: float, k: int):
    """(M_k, T_k) of the unadaptive test, computed by the library."""
    M, T = C.c_int64(), C.c_int64()
    rc = lib().ezo_test_constants(eps, delta, tau, int(k), C.byref(M), C.byref(T))
    if rc:
        raise EzoError(rc, "bad test parameters")
    return M.value, T.value


def tune_cache_export() -> str:
    """The process-wide launch-shape cache as JSON lines."""
    n = C.c_int64()
    rc = lib().ezo_tune_cache_export(None, 0, C.byref(n))
    if rc:
        raise EzoError(rc, "tuning cache export failed")
    buf = C.create_string_buffer(n.value + 1)
    rc = lib().ezo_tune_cache_export(buf, n.value + 1, C.byref(n))
    if rc:
        raise EzoError(rc, "tuning cache export failed")
    return buf.value.decode()


def tune_cache_entries():
    """The cache as a list of dicts."""
    import json
    return [json.loads(line) for line in tune_cache_export().splitlines() if line.strip()]


def tune_cache_import(text: str) -> int:
    """Adds entries in the export format; returns how many."""
    n = C.c_int32()
    rc = lib().ezo_tune_cache_import(text.encode(), C.byref(n))
    if rc:
        raise EzoError(rc, "malformed tuning cache text")
    return n.value


def tune_cache_clear():
    lib().ezo_tune_cache_clear()


class Context:
    """An ezo context on one HIP device."""

    def __init__(self, device: int = 0):
        h = C.c_void_p()
        rc = lib().ezo_ctx_create(int(device), C.byref(h))
        if rc:
            raise EzoError(rc, lib().ezo_last_error(None).decode())
        self.h = h
        self.device = device

    def close(self):
        if self.h:
            lib().ezo_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_obstacle_boxes(self, boxes):
        """Obstacle boxes tested by every call on this context: [n][15] =
        centre (3), rotation (9, row-major, columns = box axes), half
        extents (3), world frame.  None or an empty array removes them."""
        b = np.ascontiguousarray(np.zeros((0, 15)) if boxes is None else boxes, dtype=np.float32).reshape(-1, 15)
        self._check(lib().ezo_set_obstacle_boxes(self.h, b.ctypes.data_as(C.POINTER(C.c_float)), len(b)))

    def set_autotune(self, enable: bool):
        """Time launch shapes on the first call with a new tuning key (default on)."""
        self._check(lib().ezo_set_autotune(self.h, 1 if enable else 0))

    def set_phase_timing(self, enable: bool):
        """Per-phase GPU timing of inflate_edges (hipEvents on the kernels' stream)."""
        self._check(lib().ezo_set_phase_timing(self.h, 1 if enable else 0))

    def phase_timing(self, with_tests=False):
        """(dict phase -> cumulative ms, timed iterations[, dict phase ->
        sphere-sphere tests]) since timing was enabled."""
        ms = (C.c_double * len(PHASES))()
        tests = (C.c_int64 * len(PHASES))()
        it = C.c_int64()
        self._check(lib().ezo_get_phase_timing(self.h, ms, C.byref(it), tests if with_tests else None))
        out = ({p: ms[i] for i, p in enumerate(PHASES)}, it.value)
        if with_tests:
            out = out + ({p: tests[i] for i, p in enumerate(PHASES)},)
        return out

    def _check(self, rc):
        if rc:
            raise EzoError(rc, lib().ezo_last_error(self.h).decode())


class Robot:
    """A robot uploaded to a context (DH arm + spheres + self pairs)."""

    def __init__(self, ctx: Context, desc: dict):
        self.ctx = ctx
        f64 = lambda k: np.ascontiguousarray(desc[k], dtype=np.float64)
        self._keep = dict(a=f64("a"), alpha=f64("alpha"), d=f64("d"), q_lo=f64("q_lo"), q_hi=f64("q_hi"),
                          link=np.ascontiguousarray(desc["sphere_link"], dtype=np.int32),
                          xyz=np.ascontiguousarray(desc["sphere_xyz"], dtype=np.float64).reshape(-1, 3),
                          r=f64("sphere_r"),
                          pairs=np.ascontiguousarray(desc.get("self_pairs", np.zeros((0, 2))),
                                                     dtype=np.int32).reshape(-1, 2),
                          box_link=np.ascontiguousarray(desc.get("box_link", np.zeros(0)), dtype=np.int32),
                          box_pose=np.ascontiguousarray(desc.get("box_pose", np.zeros((0, 12))),
                                                        dtype=np.float64).reshape(-1, 12),
                          box_half=np.ascontiguousarray(desc.get("box_half", np.zeros((0, 3))),
                                                        dtype=np.float64).reshape(-1, 3),
                          box_pairs=np.ascontiguousarray(desc.get("box_pairs", np.zeros((0, 2))),
                                                         dtype=np.int32).reshape(-1, 2))
        k = self._keep
        dp = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))
        ip = lambda a: a.ctypes.data_as(C.POINTER(C.c_int32))
        self.dof = int(desc["dof"])
        self.n_spheres = len(k["r"])
        self.n_self = len(k["pairs"])
        self.n_boxes = len(k["box_link"])
        jt = desc.get("joint_type")
        k["joint_type"] = None if jt is None else np.ascontiguousarray(jt, dtype=np.int32)
        self.n_box_pairs = len(k["box_pairs"])
        d = RobotDesc(self.dof, dp(k["a"]), dp(k["alpha"]), dp(k["d"]), dp(k["q_lo"]), dp(k["q_hi"]),
                      self.n_spheres, ip(k["link"]), dp(k["xyz"]), dp(k["r"]), self.n_self, ip(k["pairs"]),
                      self.n_boxes, ip(k["box_link"]), dp(k["box_pose"]), dp(k["box_half"]), self.n_box_pairs,
                      ip(k["box_pairs"]), ip(k["joint_type"]) if k["joint_type"] is not None else None)
        h = C.c_void_p()
        ctx._check(lib().ezo_robot_create(ctx.h, C.byref(d), C.byref(h)))
        self.h = h
        self.q_lo = k["q_lo"]
        self.q_hi = k["q_hi"]

    def close(self):
        if self.h:
            lib().ezo_robot_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def check_collisions(ctx: Context, robot: Robot, obs, q, flags, min_sd=None, min_sd_self=None,
                     stride_n=None, stride_d=None, n=None, stream=None, noalloc=False):
    """q: float32 CUDA tensor; by default [n][dof] (stride_n = dof,
    stride_d = 1).  flags: uint8 [n]; min_sd / min_sd_self: float32 [n] or
    None (both None = flags only, early exit).  noalloc=True calls
    ezo_check_collisions_noalloc (fixed device scratch, at most
    EZO_NOALLOC_MAX_OBSTACLES obstacles)."""
    torch = _torch()
    _need(q, torch.float32, "q")
    if stride_n is None:
        if q.dim() != 2 or q.shape[1] != robot.dof:
            raise ValueError("q must be [n][dof] unless strides are given")
        n, stride_n, stride_d = q.shape[0], robot.dof, 1
    else:
        n_max = (q.numel() - 1 - (robot.dof - 1) * stride_d) // stride_n + 1 if q.numel() else 0
        if n is None:
            n = n_max
        if n > n_max:
            raise ValueError("q is too small for n configurations with these strides")
    _need(obs, torch.float32, "obs")
    n_obs = obs.numel() // 4
    _need(flags, torch.uint8, "flags", n)
    if min_sd is not None:
        _need(min_sd, torch.float32, "min_sd", n)
    if min_sd_self is not None:
        _need(min_sd_self, torch.float32, "min_sd_self", n)
    fn = lib().ezo_check_collisions_noalloc if noalloc else lib().ezo_check_collisions
    ctx._check(fn(ctx.h, robot.h, _ptr(obs), n_obs, _ptr(q), n, stride_n, stride_d,
                  _ptr(flags), _ptr(min_sd), _ptr(min_sd_self), _stream(stream)))


def sphere_centres(ctx: Context, robot: Robot, q, out, stream=None):
    """q: float32 [n][dof]; out: float32 [n][S][3]."""
    torch = _torch()
    _need(q, torch.float32, "q")
    n = q.shape[0]
    _need(out, torch.float32, "out", n * robot.n_spheres * 3)
    ctx._check(lib().ezo_sphere_centres(ctx.h, robot.h, _ptr(q), n, robot.dof, 1, _ptr(out), _stream(stream)))


def sample_polytopes(ctx: Context, dof, A, b, n_faces, edges, n_samples, n_mix, seed, iteration, samples,
                     edge_id_base=0, stream=None):
    """A: [E][cap][dof] f32, b: [E][cap] f32, n_faces: [E] i32, edges:
    [E][2][dof] f32, samples: [E][dof][stride] f32 (stride >= n_samples)."""
    torch = _torch()
    E, cap = b.shape
    for t, dt, nm in ((A, torch.float32, "A"), (b, torch.float32, "b"), (n_faces, torch.int32, "n_faces"),
                      (edges, torch.float32, "edges"), (samples, torch.float32, "samples")):
        _need(t, dt, nm)
    stride = samples.shape[-1]
    if samples.numel() < E * dof * stride:
        raise ValueError("samples too small")
    ctx._check(lib().ezo_sample_polytopes(ctx.h, int(dof), _ptr(A), _ptr(b), _ptr(n_faces), int(cap), _ptr(edges),
                                          int(E), int(n_samples), int(n_mix), int(seed), int(edge_id_base),
                                          int(iteration), _ptr(samples), int(stride), _stream(stream)))


def test_and_select(ctx: Context, flags, n_samples, M, T, n_p, cand_idx, n_cands, accept=None, test_count=None,
                    stream=None):
    """flags: [E][stride] u8; cand_idx: [E][cap] i32; n_cands: [E] i32."""
    torch = _torch()
    E, stride = flags.shape
    _need(flags, torch.uint8, "flags")
    _need(cand_idx, torch.int32, "cand_idx")
    _need(n_cands, torch.int32, "n_cands", E)
    ctx._check(lib().ezo_test_and_select(ctx.h, _ptr(flags), int(E), int(stride), int(n_samples), int(M), int(T),
                                         int(n_p), _ptr(cand_idx), _ptr(n_cands), int(cand_idx.shape[1]),
                                         _ptr(accept), _ptr(test_count), _stream(stream)))


def project_bisect(ctx: Context, robot: Robot, obs, edges, samples, cand_idx, n_cands, n_b, c_star, a_dir, t_star,
                   proj_collides, stream=None):
    """samples [E][dof][stride]; cand_idx [E][cap]; outputs c_star/a_dir
    [E][dof][cap] f32, t_star [E][cap] f32, proj_collides [E][cap] u8."""
    E, cap = cand_idx.shape
    ctx._check(lib().ezo_project_bisect(ctx.h, robot.h, _ptr(obs), obs.numel() // 4, _ptr(edges), int(E),
                                        _ptr(samples), int(samples.shape[-1]), _ptr(cand_idx), _ptr(n_cands),
                                        int(cap), int(n_b), _ptr(c_star), _ptr(a_dir), _ptr(t_star),
                                        _ptr(proj_collides), _stream(stream)))


def place_hyperplanes(ctx: Context, dof, edges, c_star, a_dir, t_star, n_cands, n_f, step_back_max, t_col, A, b,
                      n_faces, edge_status, placed_idx=None, n_placed=None, stream=None):
    E, cap_c = t_star.shape
    ctx._check(lib().ezo_place_hyperplanes(ctx.h, int(dof), _ptr(edges), int(E), _ptr(c_star), _ptr(a_dir),
                                           _ptr(t_star), _ptr(n_cands), int(cap_c), int(n_f), float(step_back_max),
                                           float(t_col), _ptr(A), _ptr(b), _ptr(n_faces), int(b.shape[1]),
                                           _ptr(edge_status), _ptr(placed_idx), _ptr(n_placed), _stream(stream)))


@dataclass
class InflateResult:
    A: object           # [E][cap][dof] float32 (device)
    b: object           # [E][cap] float32 (device)
    n_faces: object     # [E] int32 (device)
    status: object      # [E] int32 (device)
    stats: list         # per-edge dicts


def make_params(eps, delta, tau=0.5, step_back_max=0.01, t_col=1e-4, n_p=1000, n_f=10, n_b=11, n_mix=30,
                max_iters=50, face_capacity=None, seed=0, edge_id_base=0, dof=None, surrogate=None) -> Params:
    if face_capacity is None:
        face_capacity = 2 * (dof or MAX_DOF) + n_f * max_iters
    return Params(eps, delta, tau, step_back_max, t_col, n_p, n_f, n_b, n_mix, max_iters, face_capacity, seed,
                  edge_id_base, surrogate.h.value if surrogate is not None else None, None)


def make_train_params(epochs=10, batch=4096, lr=1e-3, beta1=0.9, beta2=0.999, adam_eps=1e-8, huber_delta=0.05,
                      clip_lo=-0.3, clip_hi=0.5, seed=0) -> TrainParams:
    return TrainParams(epochs, batch, lr, beta1, beta2, adam_eps, huber_delta, clip_lo, clip_hi, seed)


def surrogate_num_params(dof: int, hidden: int) -> int:
    return int(lib().ezo_surrogate_num_params(dof, hidden))


class Surrogate:
    """Learned self-collision screen (MLP dof -> H -> H -> H -> 1, SiLU,
    BF16 MFMA layers) owned by a context."""

    def __init__(self, ctx: Context, dof: int, hidden: int = 256, seed: int = 0):
        self.ctx = ctx
        self.dof, self.hidden = int(dof), int(hidden)
        h = C.c_void_p()
        ctx._check(lib().ezo_surrogate_create(ctx.h, self.dof, self.hidden, int(seed), C.byref(h)))
        self.h = h
        self.n_params = surrogate_num_params(self.dof, self.hidden)
        self.margin = float("inf")

    def close(self):
        if self.h:
            lib().ezo_surrogate_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get_params(self):
        out = np.empty(self.n_params, np.float32)
        self.ctx._check(lib().ezo_surrogate_get_params(self.h, out.ctypes.data_as(C.POINTER(C.c_float)),
                                                       self.n_params))
        return out

    def set_params(self, params):
        p = np.ascontiguousarray(params, dtype=np.float32)
        self.ctx._check(lib().ezo_surrogate_set_params(self.h, p.ctypes.data_as(C.POINTER(C.c_float)), len(p)))

    def train(self, q, target, tp: TrainParams, stream=None):
        torch = _torch()
        _need(q, torch.float32, "q")
        _need(target, torch.float32, "target", q.shape[0])
        losses = (C.c_float * max(tp.epochs, 1))()
        self.ctx._check(lib().ezo_surrogate_train(self.ctx.h, self.h, _ptr(q), _ptr(target), q.shape[0],
                                                  C.byref(tp), losses, _stream(stream)))
        return [losses[i] for i in range(tp.epochs)]

    def loss_grad(self, q, target, tp: TrainParams, stream=None):
        grad = np.empty(self.n_params, np.float32)
        loss = C.c_double()
        self.ctx._check(lib().ezo_surrogate_loss_grad(self.ctx.h, self.h, _ptr(q), _ptr(target), q.shape[0],
                                                      C.byref(tp), grad.ctypes.data_as(C.POINTER(C.c_float)),
                                                      C.byref(loss), _stream(stream)))
        return loss.value, grad

    def predict(self, q, out, stream=None):
        torch = _torch()
        _need(q, torch.float32, "q")
        _need(out, torch.float32, "out", q.shape[0])
        self.ctx._check(lib().ezo_surrogate_predict(self.ctx.h, self.h, _ptr(q), q.shape[0], _ptr(out),
                                                    _stream(stream)))

    def calibrate(self, q, target, alpha, stream=None):
        m = C.c_double()
        self.ctx._check(lib().ezo_surrogate_calibrate(self.ctx.h, self.h, _ptr(q), _ptr(target), q.shape[0],
                                                      float(alpha), C.byref(m), _stream(stream)))
        self.margin = m.value
        return m.value

    def set_margin(self, m):
        self.ctx._check(lib().ezo_surrogate_set_margin(self.h, float(m)))
        self.margin = float(m)

    def set_scope(self, samples=True, midpoints=True):
        """What an inflation screens: the samples after M_k and / or the
        bisection midpoints (never the test's samples or the projections)."""
        self.ctx._check(lib().ezo_surrogate_set_scope(self.h, (1 if samples else 0) | (2 if midpoints else 0)))

    def miss_rate(self, q, target, stream=None):
        miss, frac = C.c_double(), C.c_double()
        self.ctx._check(lib().ezo_surrogate_miss_rate(self.ctx.h, self.h, _ptr(q), _ptr(target), q.shape[0],
                                                      C.byref(miss), C.byref(frac), _stream(stream)))
        return miss.value, frac.value


def inflate_edges(ctx: Context, robot: Robot, obs, edges, params: Params, out=None, stream=None,
                  row_points=None) -> InflateResult:
    """edges: float32 CUDA tensor [E][2][dof].  Returns device tensors A, b,
    n_faces, status and host per-edge stats.  row_points (optional float32
    CUDA tensor [E][face_capacity][dof]) receives the collision point each
    placed hyperplane row was placed for."""
    torch = _torch()
    _need(edges, torch.float32, "edges")
    _need(obs, torch.float32, "obs")
    E = edges.shape[0]
    cap = params.face_capacity
    dev = edges.device
    if row_points is not None:
        _need(row_points, torch.float32, "row_points")
        if row_points.numel() < E * cap * robot.dof:
            raise ValueError("row_points smaller than [E][face_capacity][dof]")
        params = Params.from_buffer_copy(params)
        params.row_points = row_points.data_ptr()
    if out is None:
        out = InflateResult(torch.empty((E, cap, robot.dof), dtype=torch.float32, device=dev),
                            torch.empty((E, cap), dtype=torch.float32, device=dev),
                            torch.empty(E, dtype=torch.int32, device=dev),
                            torch.empty(E, dtype=torch.int32, device=dev), [])
    st = (EdgeStats * max(E, 1))()
    ctx._check(lib().ezo_inflate_edges(ctx.h, robot.h, _ptr(obs), obs.numel() // 4, _ptr(edges), int(E),
                                       C.byref(params), _ptr(out.A), _ptr(out.b), _ptr(out.n_faces),
                                       _ptr(out.status), st, _stream(stream)))
    out.stats = EdgeStatsView(st, E)
    return out


class PathsResult(InflateResult):
    """InflateResult over the paths' edges (numbered path by path) plus
    covered_by: -1 for an inflated edge, else the earlier edge whose set
    contains it."""

    def __init__(self, A, b, n_faces, status, stats, covered_by):
        super().__init__(A, b, n_faces, status, stats)
        self.covered_by = covered_by


def inflate_paths(ctx: Context, robot: Robot, obs, vertices, path_vertices, params: Params, stream=None) -> PathsResult:
    """Sequential inflation of piecewise-linear paths with the containment
    skip (Sec. V-A).  vertices: float32 CUDA tensor [sum(path_vertices)][dof]
    (the paths back to back); path_vertices: vertex count of each path (>= 2)."""
    torch = _torch()
    _need(vertices, torch.float32, "vertices")
    _need(obs, torch.float32, "obs")
    counts = [int(x) for x in path_vertices]
    if sum(counts) != vertices.shape[0]:
        raise ValueError("path_vertices must sum to the number of vertices")
    E = sum(counts) - len(counts)
    cap = params.face_capacity
    dev = vertices.device
    out = PathsResult(torch.empty((E, cap, robot.dof), dtype=torch.float32, device=dev),
                      torch.empty((E, cap), dtype=torch.float32, device=dev),
                      torch.empty(E, dtype=torch.int32, device=dev),
                      torch.empty(E, dtype=torch.int32, device=dev), [],
                      torch.empty(E, dtype=torch.int32, device=dev))
    pv = (C.c_int32 * max(len(counts), 1))(*counts)
    st = (EdgeStats * max(E, 1))()
    ctx._check(lib().ezo_inflate_paths(ctx.h, robot.h, _ptr(obs), obs.numel() // 4, _ptr(vertices), pv,
                                       len(counts), C.byref(params), _ptr(out.A), _ptr(out.b), _ptr(out.n_faces),
                                       _ptr(out.status), _ptr(out.covered_by), st, _stream(stream)))
    out.stats = EdgeStatsView(st, E)
    return out


# ---------------------------------------------------------------------------
# Recovery from collisions found on a trajectory (Sec. V-B)
# ---------------------------------------------------------------------------

def check_path(ctx: Context, robot: Robot, obs, waypoints, max_step, point_capacity=4096, stream=None):
    """Discretise the path through waypoints [K][dof] (float32 CUDA) at
    max_step per coordinate and check every point.  Returns (colliding points
    [min(n, capacity)][dof] in path order, number of colliding points, number
    of path points)."""
    torch = _torch()
    _need(waypoints, torch.float32, "waypoints")
    _need(obs, torch.float32, "obs")
    pts = torch.empty((max(point_capacity, 1), robot.dof), dtype=torch.float32, device=waypoints.device)
    n_pts, n_col = C.c_int64(), C.c_int64()
    ctx._check(lib().ezo_check_path(ctx.h, robot.h, _ptr(obs), obs.numel() // 4, _ptr(waypoints),
                                    int(waypoints.shape[0]), float(max_step), _ptr(pts), int(point_capacity),
                                    C.byref(n_pts), C.byref(n_col), _stream(stream)))
    return pts[:min(n_col.value, point_capacity)], n_col.value, n_pts.value


def update_polytopes(ctx: Context, robot: Robot, obs, edges, points, result, n_b=11, n_f=10, step_back_max=0.01,
                     t_col=1e-4, stream=None):
    """Exclude the found collisions `points` [n][dof] from the sets of
    `result` (an InflateResult for `edges`, edited in place).  Returns the
    planes added per edge (int32 CUDA tensor)."""
    torch = _torch()
    _need(points, torch.float32, "points")
    _need(edges, torch.float32, "edges")
    E = edges.shape[0]
    added = torch.zeros(E, dtype=torch.int32, device=edges.device)
    ctx._check(lib().ezo_update_polytopes(ctx.h, robot.h, _ptr(obs), obs.numel() // 4, _ptr(edges), int(E),
                                          _ptr(points), int(points.shape[0]), int(n_b), int(n_f),
                                          float(step_back_max), float(t_col), _ptr(result.A), _ptr(result.b),
                                          _ptr(result.n_faces), int(result.b.shape[1]), _ptr(result.status),
                                          _ptr(added), _stream(stream)))
    return added


def segments_contained(ctx: Context, A, b, n_faces, segments, tol=0.0, stream=None):
    """covered[k] = smallest set index containing segment k ([K][2][dof]), -1 if none."""
    torch = _torch()
    _need(segments, torch.float32, "segments")
    K, _, dof = segments.shape
    covered = torch.empty(K, dtype=torch.int32, device=segments.device)
    ctx._check(lib().ezo_segments_contained(ctx.h, int(dof), _ptr(A), _ptr(b), _ptr(n_faces), int(b.shape[1]),
                                            int(b.shape[0]), _ptr(segments), int(K), float(tol), _ptr(covered),
                                            _stream(stream)))
    return covered


# ---------------------------------------------------------------------------
# Collision map of a dynamic roadmap (appendix, DRM construction)
# ---------------------------------------------------------------------------

def collision_map(ctx: Context, robot: Robot, q, lo, side, dims, out=None, stream=None):
    """Bitset map [V][ceil(N/32)] int32 (read as uint32): bit n of row v set
    iff node q[n] ([N][dof] float32 CUDA) collides with voxel v's sphere."""
    torch = _torch()
    _need(q, torch.float32, "q")
    n = q.shape[0]
    dims = [int(x) for x in dims]
    V = dims[0] * dims[1] * dims[2]
    words = max((n + 31) // 32, 1)
    if out is None:
        out = torch.empty((V, words), dtype=torch.int32, device=q.device)
    lo_c = (C.c_float * 3)(*[float(x) for x in lo])
    dims_c = (C.c_int32 * 3)(*dims)
    ctx._check(lib().ezo_collision_map(ctx.h, robot.h, _ptr(q), n, lo_c, float(side), dims_c, _ptr(out),
                                       out.shape[1], _stream(stream)))
    return out


def collision_map_lists(ctx: Context, cmap, n_nodes, stream=None):
    """(offsets int64 [V+1], ids int32 [total]) of a bitset map: row v's node
    ids, increasing, at ids[offsets[v]:offsets[v+1]]."""
    torch = _torch()
    V, words = cmap.shape
    offsets = torch.empty(V + 1, dtype=torch.int64, device=cmap.device)
    total = C.c_int64()
    rc = lib().ezo_collision_map_lists(ctx.h, _ptr(cmap), V, words, int(n_nodes), _ptr(offsets), None, 0,
                                       C.byref(total), _stream(stream))
    if rc not in (EZO_OK, EZO_E_CAPACITY):
        ctx._check(rc)
    ids = torch.empty(max(total.value, 1), dtype=torch.int32, device=cmap.device)
    if total.value:
        ctx._check(lib().ezo_collision_map_lists(ctx.h, _ptr(cmap), V, words, int(n_nodes), _ptr(offsets),
                                                 _ptr(ids), total.value, C.byref(total), _stream(stream)))
    return offsets, ids[:total.value]
