"""FP64 CPU reference ("oracle") for the EI-ZO hot path -- TEST INFRASTRUCTURE.

Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark
use this package.  The product (the HIP library and its Python binding) never
imports it.  The numerics live in `ezo_oracle.c` (plain C, double precision);
this module compiles it with gcc and marshals numpy arrays through ctypes.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = [os.path.join(_HERE, "ezo_oracle.c"), os.path.join(_HERE, "mlp_oracle.c")]
_SO = os.path.join(_HERE, "libezo_oracle.so")

CERTIFIED, MAX_ITERS, IN_COLLISION, INVALID, CONTAINED = 0, 1, 2, 3, 4


def build(force: bool = True) -> str:
    """Compile the oracle (gcc -O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-Wall", "-Wno-unknown-pragmas", "-o", tmp, *_SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        _lib = C.CDLL(_SO)
        _declare(_lib)
    return _lib


_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)
_i64p = C.POINTER(C.c_int64)
_u8p = C.POINTER(C.c_uint8)
_u32p = C.POINTER(C.c_uint32)


class _Robot(C.Structure):
    _fields_ = [("dof", C.c_int32), ("a", _dp), ("alpha", _dp), ("d", _dp),
                ("q_lo", _dp), ("q_hi", _dp), ("n_spheres", C.c_int32),
                ("sphere_link", _ip), ("sphere_xyz", _dp), ("sphere_r", _dp),
                ("n_self", C.c_int32), ("self_pairs", _ip),
                ("n_boxes", C.c_int32), ("box_link", _ip), ("box_pose", _dp), ("box_half", _dp),
                ("n_box_pairs", C.c_int32), ("box_pairs", _ip), ("joint_type", _ip)]


class Params(C.Structure):
    _fields_ = [("eps", C.c_double), ("delta", C.c_double), ("tau", C.c_double),
                ("step_back_max", C.c_double), ("t_col", C.c_double),
                ("n_p", C.c_int32), ("n_f", C.c_int32), ("n_b", C.c_int32),
                ("n_mix", C.c_int32), ("max_iters", C.c_int32),
                ("seed", C.c_uint64), ("edge_id", C.c_int64)]


class Stats(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("planes", C.c_int32),
                ("final_m", C.c_int64), ("test_collisions", C.c_int64),
                ("samples", C.c_int64), ("checks", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def _declare(L):
    rp = C.POINTER(_Robot)
    L.orc_link_frames.argtypes = [rp, _dp, _dp]
    L.orc_sphere_centres.argtypes = [rp, _dp, _dp]
    L.orc_check_config.argtypes = [rp, _dp, C.c_int32, _dp, C.c_int32, _dp, _dp, _dp, C.POINTER(C.c_int)]
    L.orc_check_batch.argtypes = [rp, _dp, C.c_int32, _dp, C.c_int32, _dp, C.c_int64, _u8p, _dp, _dp, _dp, _u8p]
    L.orc_collision_map.argtypes = [rp, _dp, C.c_int64, _dp, C.c_double, _ip, _i64p, C.c_int64, _dp]
    L.orc_sd_sphere_box.argtypes = [_dp, C.c_double, _dp, _dp, _dp]
    L.orc_sd_sphere_box.restype = C.c_double
    L.orc_sat_boxes.argtypes = [_dp, _dp, _dp, _dp, _dp, _dp, C.POINTER(C.c_int)]
    L.orc_sat_boxes.restype = C.c_double
    L.orc_set_fragility.argtypes = [C.c_double, C.c_double]
    L.orc_set_fragility.restype = None
    L.orc_philox4x32_10.argtypes = [_u32p, _u32p, _u32p]
    L.orc_u01.argtypes = [C.c_uint32]
    L.orc_u01.restype = C.c_double
    L.orc_test_constants.argtypes = [C.c_double, C.c_double, C.c_double, C.c_int32, _i64p, _i64p]
    L.orc_hit_and_run.argtypes = [C.c_int32, _dp, _dp, C.c_int32, _dp, _dp, C.c_int32, C.c_uint64,
                                  C.c_uint32, C.c_uint32, C.c_int64, _dp]
    L.orc_hit_and_run_steps.argtypes = [C.c_int32, _dp, _dp, C.c_int32, C.c_uint64, C.c_uint32, C.c_uint32,
                                        C.c_uint32, C.c_int64, C.c_int64, _dp, _dp]
    L.orc_hit_and_run_steps.restype = None
    L.orc_project.argtypes = [C.c_int32, _dp, _dp, _dp, _dp, _dp]
    L.orc_bisect_arm.argtypes = [rp, _dp, C.c_int32, _dp, C.c_int32, _dp, _dp, _dp, C.c_int32, _dp, _dp, _dp, _dp,
                                 _dp, _dp]
    L.orc_bisect_arm.restype = C.c_int
    L.orc_bisect_balls.argtypes = [C.c_int32, _dp, _dp, C.c_int32, _dp, _dp, _dp, C.c_int32,
                                   _dp, _dp, _dp, _dp, _dp, _dp]
    L.orc_bisect_balls.restype = C.c_int
    L.orc_place.argtypes = [C.c_int32, _dp, _dp, C.c_int32, _dp, _dp, _dp, C.c_int32, C.c_double,
                            C.c_double, _dp, _dp, _ip, C.c_int32, _ip, _ip]
    L.orc_place.restype = C.c_int
    L.orc_eizo_arm.argtypes = [rp, _dp, C.c_int32, _dp, C.c_int32, _dp, _dp, C.c_int32, _dp, _dp,
                               C.POINTER(Params), _dp, _dp, C.c_int32, _ip, C.POINTER(Stats)]
    L.orc_eizo_arm.restype = C.c_int
    L.orc_eizo_balls.argtypes = [C.c_int32, _dp, _dp, C.c_int32, _dp, _dp, C.c_int32, _dp, _dp,
                                 C.POINTER(Params), _dp, _dp, C.c_int32, _ip, C.POINTER(Stats)]
    L.orc_eizo_balls.restype = C.c_int
    L.orc_mlp_num_params.argtypes = [C.c_int32, C.c_int32]
    L.orc_mlp_num_params.restype = C.c_int64
    L.orc_mlp_forward.argtypes = [C.c_int32, C.c_int32, _dp, _dp, C.c_int64, _dp]
    L.orc_mlp_loss_grad.argtypes = [C.c_int32, C.c_int32, _dp, _dp, _dp, C.c_int64, C.c_double, C.c_double,
                                    C.c_double, _dp]
    L.orc_mlp_loss_grad.restype = C.c_double
    L.orc_mlp_loss.argtypes = [C.c_int32, C.c_int32, _dp, _dp, _dp, C.c_int64, C.c_double, C.c_double,
                               C.c_double]
    L.orc_mlp_loss.restype = C.c_double
    L.orc_set_threads.argtypes = [C.c_int32]
    L.orc_max_threads.restype = C.c_int32


def _d(x):
    return np.ascontiguousarray(x, dtype=np.float64)


def _ptr(a, t=_dp):
    return a.ctypes.data_as(t) if a is not None else None


class Robot:
    """Holds FP64 copies of a robot description (dict as produced by the
    workload files) and the ctypes struct pointing at them."""

    def __init__(self, desc: dict, self_pairs=None):
        self.dof = int(desc["dof"])
        self.a = _d(desc["a"])
        self.alpha = _d(desc["alpha"])
        self.d = _d(desc["d"])
        self.q_lo = _d(desc["q_lo"])
        self.q_hi = _d(desc["q_hi"])
        self.sphere_link = np.ascontiguousarray(desc["sphere_link"], dtype=np.int32)
        self.sphere_xyz = _d(desc["sphere_xyz"]).reshape(-1, 3)
        self.sphere_r = _d(desc["sphere_r"])
        sp = desc.get("self_pairs") if self_pairs is None else self_pairs
        if sp is None:
            sp = np.zeros((0, 2), np.int32)
        self.self_pairs = np.ascontiguousarray(sp, dtype=np.int32).reshape(-1, 2)
        self.n_spheres = len(self.sphere_r)
        # boxes on links (optional): link, pose (centre, rotation row-major) in
        # the link frame, half extents, self pairs of box indices
        self.box_link = np.ascontiguousarray(desc.get("box_link", np.zeros(0)), dtype=np.int32)
        self.box_pose = _d(desc.get("box_pose", np.zeros((0, 12)))).reshape(-1, 12)
        self.box_half = _d(desc.get("box_half", np.zeros((0, 3)))).reshape(-1, 3)
        self.box_pairs = np.ascontiguousarray(desc.get("box_pairs", np.zeros((0, 2))), dtype=np.int32).reshape(-1, 2)
        self.n_boxes = len(self.box_link)
        jt = desc.get("joint_type")
        self.joint_type = None if jt is None else np.ascontiguousarray(jt, dtype=np.int32)
        self._s = _Robot(self.dof, _ptr(self.a), _ptr(self.alpha), _ptr(self.d), _ptr(self.q_lo),
                         _ptr(self.q_hi), self.n_spheres, _ptr(self.sphere_link, _ip),
                         _ptr(self.sphere_xyz), _ptr(self.sphere_r), len(self.self_pairs),
                         _ptr(self.self_pairs, _ip), self.n_boxes, _ptr(self.box_link, _ip),
                         _ptr(self.box_pose), _ptr(self.box_half), len(self.box_pairs),
                         _ptr(self.box_pairs, _ip), _ptr(self.joint_type, _ip))

    @property
    def ref(self):
        return C.byref(self._s)

    def box(self):
        """Domain D = joint-limit box as rows [+e_j <= hi_j] then [-e_j <= -lo_j]."""
        A = np.concatenate([np.eye(self.dof), -np.eye(self.dof)])
        b = np.concatenate([self.q_hi, -self.q_lo])
        return A, b


def set_threads(n: int):
    lib().orc_set_threads(int(n))


def max_threads() -> int:
    return int(lib().orc_max_threads())


def link_frames(robot: Robot, q):
    q = _d(q)
    out = np.empty((robot.dof, 4, 4))
    lib().orc_link_frames(robot.ref, _ptr(q), _ptr(out))
    return out


def sphere_centres(robot: Robot, q):
    q = _d(q)
    out = np.empty((robot.n_spheres, 3))
    lib().orc_sphere_centres(robot.ref, _ptr(q), _ptr(out))
    return out


def _ebox(env_boxes):
    """Obstacle boxes as [n][15] FP64: centre (3), rotation (9, row-major,
    columns = box axes), half extents (3), world frame."""
    if env_boxes is None:
        return np.zeros((0, 15))
    return _d(env_boxes).reshape(-1, 15)


def check(robot: Robot, obs, q, env_boxes=None, fragile=False):
    """Returns (flags u8[n], min_sd[n], sd_env[n], sd_self[n]) for q [n][dof];
    with fragile=True also fragile u8[n], bits as in sat_boxes: bit 0, some
    box-box pair within 1e-3 of the minimum of its kind (obstacle or self)
    has a fragile value; bit 1, some box-box pair has a fragile sign."""
    q = _d(q).reshape(-1, robot.dof)
    obs = _d(obs).reshape(-1, 4)
    eb = _ebox(env_boxes)
    n = q.shape[0]
    flags = np.empty(n, np.uint8)
    sd, se, ss = np.empty(n), np.empty(n), np.empty(n)
    fr = np.empty(n, np.uint8) if fragile else None
    lib().orc_check_batch(robot.ref, _ptr(obs), obs.shape[0], _ptr(eb), eb.shape[0], _ptr(q), n,
                          _ptr(flags, _u8p), _ptr(sd), _ptr(se), _ptr(ss), _ptr(fr, _u8p))
    return (flags, sd, se, ss, fr) if fragile else (flags, sd, se, ss)


def collision_map(robot: Robot, q, lo, side, dims, voxels=None):
    """Collision map of a dynamic roadmap (appendix, DRM construction) on the
    listed voxels (all of the grid if None): returns (hits bool [M][N],
    sd [M][N]) with sd the minimum signed distance between voxel m's
    circumscribing sphere and node n's robot spheres and boxes."""
    q = _d(q).reshape(-1, robot.dof)
    dims = np.ascontiguousarray(dims, dtype=np.int32).reshape(3)
    if voxels is None:
        voxels = np.arange(int(np.prod(dims.astype(np.int64))))
    vox = np.ascontiguousarray(voxels, dtype=np.int64)
    sd = np.empty((len(vox), len(q)))
    lib().orc_collision_map(robot.ref, _ptr(q), len(q), _ptr(_d(lo).reshape(3)), float(side), _ptr(dims, _ip),
                            _ptr(vox, _i64p), len(vox), _ptr(sd))
    return sd < 0.0, sd


def sd_sphere_box(x, r, c, R, h):
    """Signed distance of a sphere (centre x, radius r) and a box (centre c,
    rotation R with the box axes as columns, half extents h)."""
    return lib().orc_sd_sphere_box(_ptr(_d(x)), float(r), _ptr(_d(c)), _ptr(_d(R).reshape(9)), _ptr(_d(h)))


def set_fragility(weak_axis_norm=0.05, band=5e-5):
    """Thresholds of the fragility bits (sat_boxes, check): a cross axis
    |A_i x B_j| < weak_axis_norm is weak; the sign bit uses +-band."""
    lib().orc_set_fragility(float(weak_axis_norm), float(band))


def sat_boxes(cA, RA, hA, cB, RB, hB):
    """(separating-axis value, fragile bits) of two boxes: bit 0 the value,
    bit 1 the sign may change under FP32 rounding of the poses (a cross axis
    of nearly parallel edges decides)."""
    f = C.c_int()
    v = lib().orc_sat_boxes(_ptr(_d(cA)), _ptr(_d(RA).reshape(9)), _ptr(_d(hA)), _ptr(_d(cB)),
                            _ptr(_d(RB).reshape(9)), _ptr(_d(hB)), C.byref(f))
    return v, int(f.value)


def philox(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.empty(4, np.uint32)
    lib().orc_philox4x32_10(_ptr(c, _u32p), _ptr(k, _u32p), _ptr(out, _u32p))
    return out


def u01(x: int) -> float:
    return float(lib().orc_u01(int(x) & 0xFFFFFFFF))


def test_constants(eps, delta, tau, k):
    M, T = C.c_int64(), C.c_int64()
    lib().orc_test_constants(eps, delta, tau, int(k), C.byref(M), C.byref(T))
    return M.value, T.value


def hit_and_run(A, b, v1, v2, n_mix, seed, edge, k, n):
    A = _d(A)
    b = _d(b)
    d = A.shape[1]
    v1, v2 = _d(v1), _d(v2)
    S = np.empty((n, d))
    lib().orc_hit_and_run(d, _ptr(A), _ptr(b), A.shape[0], _ptr(v1), _ptr(v2), int(n_mix),
                          int(seed), int(edge), int(k), int(n), _ptr(S))
    return S


def hit_and_run_step(A, b, X, seed, edge, k, s, first=0):
    """Step s (>= 1) of hit-and-run walks first .. first + n - 1 (Sec. IV-B),
    each taken from its own point X[i] (rows [n][d]).  Returns the new points
    and, per walk, a^T u of the rows that bound the chord below and above
    (0 where no row bounds that end)."""
    A = _d(A)
    b = _d(b)
    X = np.array(X, dtype=np.float64, order="C", copy=True)
    n, d = X.shape
    den = np.zeros((n, 2))
    lib().orc_hit_and_run_steps(d, _ptr(A), _ptr(b), A.shape[0], int(seed), int(edge), int(k), int(s),
                                int(first), int(n), _ptr(X), _ptr(den))
    return X, den


def project(v1, v2, c):
    v1, v2, c = _d(v1), _d(v2), _d(c)
    cp = np.empty_like(c)
    al = C.c_double()
    lib().orc_project(len(c), _ptr(v1), _ptr(v2), _ptr(c), _ptr(cp), C.byref(al))
    return cp, al.value


def bisect_arm(robot: Robot, obs, v1, v2, c, n_b, env_boxes=None):
    obs = _d(obs).reshape(-1, 4)
    eb = _ebox(env_boxes)
    v1, v2, c = _d(v1), _d(v2), _d(c)
    d = robot.dof
    cs, ad, cp = np.empty(d), np.empty(d), np.empty(d)
    tr = np.empty(int(n_b) + 1)
    t, m = C.c_double(), C.c_double()
    p = lib().orc_bisect_arm(robot.ref, _ptr(obs), obs.shape[0], _ptr(eb), eb.shape[0], _ptr(v1), _ptr(v2), _ptr(c),
                             int(n_b), _ptr(cs), C.byref(t), _ptr(ad), _ptr(cp), C.byref(m), _ptr(tr))
    return dict(proj_collides=bool(p), c_star=cs, t_star=t.value, a=ad, c_proj=cp,
                min_abs_sd=m.value, sd_trace=tr)


def bisect_balls(centres, radii, v1, v2, c, n_b):
    centres, radii = _d(centres), _d(radii)
    dim = centres.shape[1]
    v1, v2, c = _d(v1), _d(v2), _d(c)
    cs, ad, cp = np.empty(dim), np.empty(dim), np.empty(dim)
    tr = np.empty(int(n_b) + 1)
    t, m = C.c_double(), C.c_double()
    p = lib().orc_bisect_balls(dim, _ptr(centres), _ptr(radii), len(radii), _ptr(v1), _ptr(v2),
                               _ptr(c), int(n_b), _ptr(cs), C.byref(t), _ptr(ad), _ptr(cp),
                               C.byref(m), _ptr(tr))
    return dict(proj_collides=bool(p), c_star=cs, t_star=t.value, a=ad, c_proj=cp,
                min_abs_sd=m.value, sd_trace=tr)


def place(v1, v2, c_star, a_dir, t_star, n_f, step_back_max, t_col, A, b, cap=None):
    """Append up to n_f planes to (A, b).  Returns (A_new, b_new, status, placed_idx)."""
    v1, v2 = _d(v1), _d(v2)
    d = len(v1)
    c_star = _d(c_star).reshape(-1, d)
    a_dir = _d(a_dir).reshape(-1, d)
    t_star = _d(t_star)
    n = len(t_star)
    A = _d(A).reshape(-1, d)
    b = _d(b)
    F0 = len(b)
    cap = F0 + n_f if cap is None else cap
    Ab = np.zeros((cap, d))
    bb = np.zeros(cap)
    Ab[:F0] = A
    bb[:F0] = b
    nf = C.c_int32(F0)
    idx = np.zeros(max(n_f, 1), np.int32)
    npl = C.c_int32()
    st = lib().orc_place(d, _ptr(v1), _ptr(v2), n, _ptr(c_star), _ptr(a_dir), _ptr(t_star),
                         int(n_f), float(step_back_max), float(t_col), _ptr(Ab), _ptr(bb),
                         C.byref(nf), cap, _ptr(idx, _ip), C.byref(npl))
    return Ab[:nf.value], bb[:nf.value], st, idx[:npl.value]


def make_params(eps=0.1, delta=0.05, tau=0.5, step_back_max=0.01, t_col=1e-4, n_p=1000, n_f=10,
                n_b=11, n_mix=30, max_iters=50, seed=0, edge_id=0) -> Params:
    return Params(eps, delta, tau, step_back_max, t_col, n_p, n_f, n_b, n_mix, max_iters,
                  seed, edge_id)


def _eizo_common(call, dof, A_D, b_D, v1, v2, prm: Params, cap):
    A_D, b_D, v1, v2 = _d(A_D), _d(b_D), _d(v1), _d(v2)
    if cap is None:
        cap = len(b_D) + prm.n_f * prm.max_iters
    A = np.zeros((cap, dof))
    b = np.zeros(cap)
    nf = C.c_int32()
    st = Stats()
    status = call(A_D, b_D, v1, v2, A, b, cap, nf, st)
    return dict(status=status, A=A[:nf.value].copy(), b=b[:nf.value].copy(), stats=st.as_dict())


def eizo_arm(robot: Robot, obs, v1, v2, prm: Params, cap=None, env_boxes=None):
    obs = _d(obs).reshape(-1, 4)
    eb = _ebox(env_boxes)
    A_D, b_D = robot.box()

    def call(A_D, b_D, v1, v2, A, b, cap, nf, st):
        return lib().orc_eizo_arm(robot.ref, _ptr(obs), obs.shape[0], _ptr(eb), eb.shape[0], _ptr(A_D), _ptr(b_D),
                                  len(b_D), _ptr(v1), _ptr(v2), C.byref(prm), _ptr(A), _ptr(b),
                                  cap, C.byref(nf), C.byref(st))
    return _eizo_common(call, robot.dof, A_D, b_D, v1, v2, prm, cap)


def eizo_balls(centres, radii, A_D, b_D, v1, v2, prm: Params, cap=None):
    centres, radii = _d(centres), _d(radii)
    dim = centres.shape[1]

    def call(A_D, b_D, v1, v2, A, b, cap, nf, st):
        return lib().orc_eizo_balls(dim, _ptr(centres), _ptr(radii), len(radii), _ptr(A_D),
                                    _ptr(b_D), len(b_D), _ptr(v1), _ptr(v2), C.byref(prm),
                                    _ptr(A), _ptr(b), cap, C.byref(nf), C.byref(st))
    return _eizo_common(call, dim, A_D, b_D, v1, v2, prm, cap)


# ---------------------------------------------------------------------------
# Learned self-collision screen: FP64 multilayer perceptron
# ---------------------------------------------------------------------------

def mlp_num_params(D: int, H: int) -> int:
    return int(lib().orc_mlp_num_params(D, H))


def mlp_forward(D, H, params, x):
    params, x = _d(params), _d(x).reshape(-1, D)
    y = np.empty(len(x))
    lib().orc_mlp_forward(D, H, _ptr(params), _ptr(x), len(x), _ptr(y))
    return y


def mlp_loss_grad(D, H, params, x, t, huber_delta=0.05, clip_lo=-0.3, clip_hi=0.5):
    params, x, t = _d(params), _d(x).reshape(-1, D), _d(t)
    g = np.empty_like(params)
    loss = lib().orc_mlp_loss_grad(D, H, _ptr(params), _ptr(x), _ptr(t), len(x), huber_delta, clip_lo, clip_hi,
                                   _ptr(g))
    return float(loss), g


def mlp_loss(D, H, params, x, t, huber_delta=0.05, clip_lo=-0.3, clip_hi=0.5):
    params, x, t = _d(params), _d(x).reshape(-1, D), _d(t)
    return float(lib().orc_mlp_loss(D, H, _ptr(params), _ptr(x), _ptr(t), len(x), huber_delta, clip_lo, clip_hi))


# ---------------------------------------------------------------------------
# Recovery from collisions found on a trajectory (Sec. V-B)
# ---------------------------------------------------------------------------

def discretize_path(waypoints, step):
    """Points along the piecewise-linear path through waypoints [K][d] with
    consecutive points at most `step` apart in every coordinate (the fine
    discretisation of a trajectory check, Sec. V-B; step 0.1 rad in Sec. VI):
    segment i is cut into m_i = max(1, ceil(max_j |w_{i+1,j} - w_{i,j}| / step))
    equal pieces, points w_i + (j / m_i)(w_{i+1} - w_i), j = 0..m_i, each
    shared vertex listed once."""
    w = _d(waypoints).reshape(len(waypoints), -1)
    pts = [w[0].copy()]
    for i in range(len(w) - 1):
        dlt = w[i + 1] - w[i]
        m = max(1, int(np.ceil(np.max(np.abs(dlt)) / step)))
        for j in range(1, m + 1):
            pts.append(w[i] + (j / m) * dlt)
    return np.array(pts)


def check_path(robot: Robot, obs, waypoints, step):
    """(points, collision flags, min signed distances) of the discretised path."""
    pts = discretize_path(waypoints, step)
    flags, sd, *_ = check(robot, obs, pts)
    return pts, flags, sd


def points_in_polytope(A, b, X):
    """Rows x of X with A x <= b (every row of the polytope)."""
    A, b, X = _d(A), _d(b), _d(X)
    if len(b) == 0:
        return np.ones(len(X), bool)
    return np.all(X @ A.reshape(len(b), -1).T <= b, axis=1)


def covering_set(As, bs, v1, v2, tol=0.0):
    """Index of the first polytope (A_i, b_i) containing the segment [v1, v2],
    or -1.  A convex polytope contains a segment iff it contains both ends.
    A set given by no rows stands for an edge that holds no set (one skipped
    by the path inflation) and contains nothing."""
    v = np.stack([_d(v1), _d(v2)])
    for i, (A, b) in enumerate(zip(As, bs)):
        A, b = _d(A), _d(b)
        if len(b) > 0 and np.all(v @ A.reshape(len(b), -1).T <= b + tol):
            return i
    return -1


def inflate_path(inflate, vertices):
    """Inflation of one piecewise-linear path in sequence with the containment
    skip (Sec. V-A).  Edge k runs from vertex k to vertex k + 1; it is inflated
    only if no set of an earlier edge of the path contains its segment, where
    the sets that count are those of edges that were inflated and ended
    CERTIFIED or MAX_ITERS; covered_by records the first (lowest k) set that
    does.  `inflate(k, v1, v2)` inflates edge k and returns a dict with
    status, A, b.  Returns one dict per edge: status, A, b, covered_by (-1 if
    inflated; a contained edge has status CONTAINED and no rows)."""
    V = _d(vertices)
    V = V.reshape(len(V), -1)
    out = []
    for k in range(len(V) - 1):
        usable = [j for j in range(k) if out[j]["covered_by"] == -1 and out[j]["status"] in (CERTIFIED, MAX_ITERS)]
        c = covering_set([out[j]["A"] for j in usable], [out[j]["b"] for j in usable], V[k], V[k + 1])
        if c >= 0:
            out.append(dict(status=CONTAINED, A=np.zeros((0, V.shape[1])), b=np.zeros(0), covered_by=usable[c]))
        else:
            r = inflate(k, V[k], V[k + 1])
            out.append(dict(status=r["status"], A=r["A"], b=r["b"], covered_by=-1))
    return out


def recover_set(bisect, v1, v2, A, b, points, n_b, n_f, step_back_max, t_col):
    """Edit one set after collisions were found on a trajectory (Sec. V-B):
    the found collisions inside P become the candidates of the last three
    steps of Alg. 1 -- projection onto L with the fail-fast check, bisection,
    then ordering and placing up to n_f hyperplanes.  `bisect(v1, v2, c, n_b)`
    is bisect_arm or bisect_balls bound to a scene.  Returns (A_new, b_new,
    status, per-candidate bisection results, candidate indices into points)."""
    A, b = _d(A), _d(b)
    d = len(_d(v1))
    A = A.reshape(len(b), d)
    pts = _d(points).reshape(-1, d)
    idx = np.nonzero(points_in_polytope(A, b, pts))[0]
    res = [bisect(v1, v2, pts[i], n_b) for i in idx]
    if any(r["proj_collides"] for r in res):
        return A, b, IN_COLLISION, res, idx
    if len(res) == 0:
        return A, b, CERTIFIED, res, idx
    cs = np.array([r["c_star"] for r in res])
    ad = np.array([r["a"] for r in res])
    ts = np.array([r["t_star"] for r in res])
    A2, b2, st, _ = place(v1, v2, cs, ad, ts, n_f, step_back_max, t_col, A, b)
    return A2, b2, st, res, idx
