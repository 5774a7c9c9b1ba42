"""ctypes binding of libaccfem.so (include/accfem.h): argument marshalling only.

Every computation runs in the HIP library; this module converts Python/numpy
(or torch device tensors, with io_on_device=1) to the C ABI and back.  It
raises if the shared library has not been built - there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libaccfem.so")

FEM_OK, FEM_E_INVAL, FEM_E_NOMEM, FEM_E_HIP, FEM_E_STATE, FEM_E_NOCONV = 0, -1, -2, -3, -4, -5
FEM_FP64, FEM_MIXED = 0, 1
FEM_QP_EXACT, FEM_QP_ADMM = 0, 1
FEM_ACT_CABLES, FEM_ACT_TIP_WRENCH_LOCAL, FEM_ACT_TIP_WRENCH_GLOBAL, FEM_ACT_CABLE_WRENCH = 0, 1, 2, 3
ROBOT_OK, ROBOT_NOCONV, ROBOT_LCPFAIL, ROBOT_NONSPD, ROBOT_OVERFLOW = 0, 1, 2, 3, 4


class fem_params(C.Structure):
    _fields_ = [
        ("n_robots", C.c_int32),
        ("n_elem", C.POINTER(C.c_int32)),
        ("length", C.POINTER(C.c_double)),
        ("base_pos", C.POINTER(C.c_double)),
        ("base_dir", C.POINTER(C.c_double)),
        ("base_up", C.POINTER(C.c_double)),
        ("r_out", C.c_double), ("r_in", C.c_double), ("E", C.c_double), ("nu", C.c_double),
        ("tip_len", C.c_double),
        ("shaft_E", C.c_double), ("shaft_A", C.c_double), ("shaft_I", C.c_double),
        ("n_cables", C.c_int32),
        ("cable_radius", C.c_double),
        ("cable_angle", C.POINTER(C.c_double)),
        ("contact_radius", C.c_double),
        ("contact_margin", C.c_double),
        ("beta0", C.c_double),
        ("guide_len", C.c_double),
        ("newton_tol", C.c_double),
        ("stag_tol", C.c_double),
        ("max_newton", C.c_int32),
        ("contact_capacity", C.c_int32),
        ("grid_cell", C.c_double),
        ("precision", C.c_int32),
        ("hip_stream", C.c_void_p),
        ("io_on_device", C.c_int32),
        ("profile", C.c_int32),
        ("autotune", C.c_int32),
        ("qp_solver", C.c_int32),
        ("admm_rho", C.c_double),
        ("admm_eps", C.c_double),
        ("admm_max_iter", C.c_int32),
        ("contact_along_elements", C.c_int32),
    ]


class fem_solve_info(C.Structure):
    _fields_ = [("status", C.c_int32), ("iters", C.c_int32), ("n_contacts", C.c_int32),
                ("n_limited", C.c_int32), ("res_norm", C.c_double),
                ("steps_converged", C.c_int32), ("steps_total", C.c_int32),
                ("iters_total", C.c_int64), ("rhs_total", C.c_int64), ("rhs_fused", C.c_int64),
                ("sweep_passes", C.c_int64), ("qp_iters_total", C.c_int64),
                ("products_total", C.c_int64), ("contact_steps_total", C.c_int64)]


class fem_contact(C.Structure):
    _fields_ = [("robot", C.c_int32), ("node", C.c_int32), ("tri", C.c_int32),
                ("kind", C.c_int32), ("n", C.c_double * 3), ("gap", C.c_double),
                ("force", C.c_double), ("s", C.c_double)]


_lib = None


def lib():
    """The loaded shared library (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError(f"{_LIB_PATH} is missing: build it with "
                               "`python -m paper_2503_06922_amd.build`")
        try:
            # torch ships a HIP runtime of its own under the same soname as the system one:
            # loading torch first makes the library bind to that runtime, so that one HIP
            # runtime serves both and torch's device memory and streams are valid here
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(_LIB_PATH)
        P = C.c_void_p
        L.fem_create.argtypes = [C.POINTER(fem_params), C.POINTER(P)]
        L.fem_destroy.argtypes = [P]
        L.fem_destroy.restype = None
        L.fem_last_error.argtypes = [P]
        L.fem_last_error.restype = C.c_char_p
        L.fem_set_lumen.argtypes = [P, P, C.c_int64, P, C.c_int64]
        L.fem_set_actuation.argtypes = [P, C.c_int, P, P]
        L.fem_solve.argtypes = [P, C.c_int32, P, P]
        L.fem_solve_schedule.argtypes = [P, C.c_int, C.c_int32, P, P, P, P, P, P, P]
        L.fem_contacts.argtypes = [P, C.c_int32, P, C.c_int32, C.POINTER(C.c_int32)]
        L.fem_get_state.argtypes = [P, P]
        L.fem_set_state.argtypes = [P, P]
        L.fem_eval.argtypes = [P, P, P, P]
        L.fem_profile.argtypes = [P, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_int64),
                                  C.c_int32]
        L.fem_grad.argtypes = [P, P, C.c_int32, P, P]
        L.fem_total_nodes.argtypes = [P]
        L.fem_total_nodes.restype = C.c_int64
        L.fem_lcp.argtypes = [P, P, C.c_int32, P, C.POINTER(C.c_int32)]
        L.fem_lcp_noalloc.argtypes = [P, P, C.c_int32, P, C.POINTER(C.c_int32), P]
        L.fem_tuning.argtypes = [P, C.POINTER(C.c_int32), C.POINTER(C.c_int32), P]
        for f in ("fem_create", "fem_set_lumen", "fem_set_actuation", "fem_solve",
                  "fem_solve_schedule", "fem_contacts",
                  "fem_get_state", "fem_set_state", "fem_eval", "fem_profile", "fem_grad", "fem_lcp",
                  "fem_lcp_noalloc", "fem_tuning"):
            getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


EXPORTED = ("fem_create", "fem_destroy", "fem_last_error", "fem_set_lumen", "fem_set_actuation",
            "fem_solve", "fem_solve_schedule", "fem_contacts", "fem_get_state", "fem_set_state", "fem_eval",
            "fem_profile", "fem_grad", "fem_total_nodes", "fem_lcp", "fem_lcp_noalloc", "fem_tuning")
FEM_LCP_NOALLOC_MAX_M = 512


class FemError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"status {status}: {msg}")
        self.status = status


def _ptr(a):
    """Pointer of a contiguous numpy array or torch tensor (None -> NULL)."""
    if a is None:
        return None
    if hasattr(a, "data_ptr"):
        return C.c_void_p(a.data_ptr())
    return a.ctypes.data_as(C.c_void_p)


def _f64(a, n=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if n is not None and a.size != n:
        raise ValueError(f"expected {n} values, got {a.size}")
    return a


class Context:
    """One fem_ctx: a batch of robots on the current HIP device."""

    def __init__(self, params: dict):
        L = lib()
        B = int(params["n_robots"])
        self._keep = {
            "n_elem": np.ascontiguousarray(np.asarray(params["n_elem"], np.int32)),
            "length": _f64(params["length"], B),
            "base_pos": _f64(params["base_pos"], 3 * B),
            "base_dir": _f64(params["base_dir"], 3 * B),
            "base_up": _f64(params["base_up"], 3 * B),
            "cable_angle": _f64(params["cable_angle"]),
        }
        k = self._keep
        p = fem_params()
        p.n_robots = B
        p.n_elem = k["n_elem"].ctypes.data_as(C.POINTER(C.c_int32))
        for name in ("length", "base_pos", "base_dir", "base_up", "cable_angle"):
            setattr(p, name, k[name].ctypes.data_as(C.POINTER(C.c_double)))
        for name in ("r_out", "r_in", "E", "nu", "tip_len", "shaft_E", "shaft_A", "shaft_I",
                     "cable_radius", "contact_radius", "contact_margin", "beta0", "guide_len",
                     "newton_tol", "stag_tol", "grid_cell"):
            setattr(p, name, float(params.get(name, 0.0)))
        p.n_cables = int(k["cable_angle"].size)
        p.max_newton = int(params.get("max_newton", 100))
        p.contact_capacity = int(params.get("contact_capacity", 64))
        p.precision = int(params.get("precision", FEM_FP64))
        p.hip_stream = params.get("hip_stream", None)
        p.io_on_device = int(params.get("io_on_device", 0))
        p.profile = int(params.get("profile", 0))
        p.autotune = int(params.get("autotune", 0))
        p.qp_solver = int(params.get("qp_solver", 0))
        p.admm_rho = float(params.get("admm_rho", 0.0))
        p.admm_eps = float(params.get("admm_eps", 0.0))
        p.admm_max_iter = int(params.get("admm_max_iter", 0))
        p.contact_along_elements = int(params.get("contact_along_elements", 0))
        self.io_on_device = p.io_on_device
        self.B = B
        self.n_cables = p.n_cables
        h = C.c_void_p()
        st = L.fem_create(C.byref(p), C.byref(h))
        if st != FEM_OK:
            raise FemError(st, L.fem_last_error(None).decode())
        self._h = h
        self.n_nodes = int(L.fem_total_nodes(h))
        self.node_offset = np.concatenate([[0], np.cumsum(k["n_elem"].astype(np.int64) + 1)])
        self.act_kind = None
        self.generation = 0  # bumped by every fem_solve / fem_set_state

    def _check(self, st, ok=(FEM_OK,)):
        if st not in ok:
            raise FemError(st, lib().fem_last_error(self._h).decode())
        return st

    def close(self):
        if getattr(self, "_h", None) is not None:
            lib().fem_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------ C ABI calls
    def fem_set_lumen(self, verts, tris):
        if self.io_on_device:
            nv, nt = verts.shape[0], tris.shape[0]
            return self._check(lib().fem_set_lumen(self._h, _ptr(verts), nv, _ptr(tris), nt))
        V = _f64(verts).reshape(-1, 3)
        T = np.ascontiguousarray(np.asarray(tris, np.int32)).reshape(-1, 3)
        return self._check(lib().fem_set_lumen(self._h, _ptr(V), V.shape[0], _ptr(T), T.shape[0]))

    def fem_set_actuation(self, kind, values, depth=None):
        self.act_kind = int(kind)
        if self.io_on_device:
            return self._check(lib().fem_set_actuation(self._h, int(kind), _ptr(values), _ptr(depth)))
        nv = self.n_cables if kind in (FEM_ACT_CABLES, FEM_ACT_CABLE_WRENCH) else 6
        v = _f64(values, self.B * nv)
        d = None if depth is None else _f64(depth, self.B)
        return self._check(lib().fem_set_actuation(self._h, int(kind), _ptr(v), _ptr(d)))

    def _dev_empty(self, shape, dtype):
        """Output buffer of a context with io_on_device = 1: a torch tensor on the current
        device (the library writes it on the context's stream)."""
        import torch
        return torch.empty(shape, dtype=dtype, device="cuda")

    def fem_solve(self, n_load_steps, state=True, info=True):
        """With io_on_device = 1 the state is returned as a torch device tensor [N, 7] and
        the info records are read back from the device buffer the library wrote."""
        self.generation += 1
        if self.io_on_device:
            import torch
            X = self._dev_empty((self.n_nodes, 7), torch.float64) if state else None
            Ib = self._dev_empty((self.B * C.sizeof(fem_solve_info),), torch.uint8) if info else None
            st = lib().fem_solve(self._h, int(n_load_steps), _ptr(X), _ptr(Ib))
            I = None
            if info:
                I = (fem_solve_info * self.B).from_buffer_copy(Ib.cpu().numpy().tobytes())
        else:
            X = np.empty((self.n_nodes, 7)) if state else None
            I = (fem_solve_info * self.B)() if info else None
            st = lib().fem_solve(self._h, int(n_load_steps), _ptr(X),
                                 C.cast(I, C.c_void_p) if info else None)
        self._check(st, ok=(FEM_OK, FEM_E_NOCONV))
        out = {"status": st}
        if state:
            out["state"] = X
        if info:
            out["info"] = [{f: getattr(I[b], f) for f, _ in fem_solve_info._fields_}
                           for b in range(self.B)]
        return out

    def fem_solve_schedule(self, kind, values, depth=None, state=True, info=True, records=True):
        """Explicit load-step schedule: values [n_steps, B, n_values], depth [n_steps, B] or
        None (numpy arrays, or torch device tensors with io_on_device = 1).  Returns the
        fem_solve outputs plus, with records, per-step "rec_tip" [n_steps, B, 3],
        "rec_status" and "rec_iters" [n_steps, B]."""
        self.generation += 1
        self.act_kind = int(kind)
        nv = self.n_cables if kind in (FEM_ACT_CABLES, FEM_ACT_CABLE_WRENCH) else 6
        n = int(values.shape[0])
        if self.io_on_device:
            import torch
            v, d = values, depth
            X = self._dev_empty((self.n_nodes, 7), torch.float64) if state else None
            Ib = self._dev_empty((self.B * C.sizeof(fem_solve_info),), torch.uint8) if info else None
            rt = self._dev_empty((n, self.B, 3), torch.float64) if records else None
            rs = self._dev_empty((n, self.B), torch.int32) if records else None
            ri = self._dev_empty((n, self.B), torch.int32) if records else None
            st = lib().fem_solve_schedule(self._h, int(kind), n, _ptr(v), _ptr(d), _ptr(X), _ptr(Ib),
                                          _ptr(rt), _ptr(rs), _ptr(ri))
            I = None
            if info:
                I = (fem_solve_info * self.B).from_buffer_copy(Ib.cpu().numpy().tobytes())
        else:
            v = _f64(values, n * self.B * nv)
            d = None if depth is None else _f64(depth, n * self.B)
            X = np.empty((self.n_nodes, 7)) if state else None
            I = (fem_solve_info * self.B)() if info else None
            rt = np.empty((n, self.B, 3)) if records else None
            rs = np.empty((n, self.B), np.int32) if records else None
            ri = np.empty((n, self.B), np.int32) if records else None
            st = lib().fem_solve_schedule(self._h, int(kind), n, _ptr(v), _ptr(d), _ptr(X),
                                          C.cast(I, C.c_void_p) if info else None,
                                          _ptr(rt), _ptr(rs), _ptr(ri))
        self._check(st, ok=(FEM_OK, FEM_E_NOCONV))
        out = {"status": st}
        if state:
            out["state"] = X
        if info:
            out["info"] = [{f: getattr(I[b], f) for f, _ in fem_solve_info._fields_}
                           for b in range(self.B)]
        if records:
            out.update(rec_tip=rt, rec_status=rs, rec_iters=ri)
        return out

    def fem_contacts(self, robot=-1):
        n = C.c_int32(0)
        self._check(lib().fem_contacts(self._h, int(robot), None, 0, C.byref(n)))
        if self.io_on_device:
            import torch
            dbuf = self._dev_empty((max(1, n.value) * C.sizeof(fem_contact),), torch.uint8)
            self._check(lib().fem_contacts(self._h, int(robot), _ptr(dbuf), n.value, C.byref(n)))
            buf = (fem_contact * max(1, n.value)).from_buffer_copy(dbuf.cpu().numpy().tobytes())
        else:
            buf = (fem_contact * max(1, n.value))()
            self._check(lib().fem_contacts(self._h, int(robot), C.cast(buf, C.c_void_p), n.value,
                                           C.byref(n)))
        return [dict(robot=c.robot, node=c.node, tri=c.tri, kind=c.kind, n=np.array(c.n[:]),
                     gap=c.gap, force=c.force, s=c.s) for c in buf[:n.value]]

    def fem_get_state(self):
        if self.io_on_device:
            import torch
            X = self._dev_empty((self.n_nodes, 7), torch.float64)
        else:
            X = np.empty((self.n_nodes, 7))
        self._check(lib().fem_get_state(self._h, _ptr(X)))
        return X

    def fem_set_state(self, X):
        self.generation += 1
        if not self.io_on_device:
            X = _f64(X, self.n_nodes * 7)
        return self._check(lib().fem_set_state(self._h, _ptr(X)))

    def fem_tuning(self):
        """Launch shapes: (threads per block of the element update, lanes per node of
        detection, measured times [6] in us or NaN before tuning)."""
        b = C.c_int32(0)
        l = C.c_int32(0)
        t = np.full(6, np.nan)
        self._check(lib().fem_tuning(self._h, C.byref(b), C.byref(l), _ptr(t)))
        return b.value, l.value, t

    def fem_profile(self, kernel, reset=False):
        ms = C.c_double(0.0)
        n = C.c_int64(0)
        self._check(lib().fem_profile(self._h, int(kernel), C.byref(ms), C.byref(n), int(reset)))
        return ms.value, n.value

    def fem_grad(self, sensor_nodes, dL_dp):
        """dL/du [B, n_values] for dL_dp [B, n_sensors, 3]; NaN rows for robots that failed.

        Returns (gradient, status) with status FEM_OK or FEM_E_NOCONV."""
        s = np.ascontiguousarray(np.asarray(sensor_nodes, np.int32)).ravel()
        nv = self.n_cables if self.act_kind in (FEM_ACT_CABLES, FEM_ACT_CABLE_WRENCH) else 6
        if self.io_on_device:
            import torch
            g = dL_dp
            out = self._dev_empty((self.B, nv), torch.float64)
        else:
            g = _f64(dL_dp, self.B * s.size * 3)
            out = np.empty((self.B, nv))
        st = lib().fem_grad(self._h, _ptr(s), int(s.size), _ptr(g), _ptr(out))
        self._check(st, ok=(FEM_OK, FEM_E_NOCONV))
        return out, st

    def sensor_rows(self, sensor_nodes):
        """Row indices [B, n_sensors] into the node state of the given sensor nodes."""
        off = self.node_offset
        n = np.diff(off)
        s = np.asarray(sensor_nodes, np.int64)
        return off[:-1, None] + np.where(s[None, :] < 0, n[:, None] + s[None, :], s[None, :])

    def fem_eval(self):
        F = np.empty((self.n_nodes, 6))
        KD = np.empty((self.n_nodes, 6, 6))
        KS = np.empty((self.n_nodes, 6, 6))
        self._check(lib().fem_eval(self._h, _ptr(F), _ptr(KD), _ptr(KS)))
        return F, KD, KS


def params_from_batch(rb, precision=FEM_FP64, newton_tol=1e-10, stag_tol=1e-9, max_newton=100,
                      contact_capacity=64, **extra):
    """fem_params of a workloads.RobotBatch (field mapping only).  contact_capacity is the
    length of each robot's contact list; a robot with more candidates ends its load step
    with FEM_ROBOT_OVERFLOW (the batched insertion into the branching lumen needs 512)."""
    p = dict(n_robots=rb.n_robots, n_elem=rb.n_elem, length=rb.length, base_pos=rb.base_pos,
             base_dir=rb.base_dir, base_up=rb.base_up, r_out=rb.r_out, r_in=rb.r_in, E=rb.E,
             nu=rb.nu, tip_len=rb.tip_len, shaft_E=rb.shaft_E, shaft_A=rb.shaft_A,
             shaft_I=rb.shaft_I, cable_radius=rb.cable_radius, cable_angle=rb.cable_angle,
             contact_radius=rb.contact_radius, contact_margin=rb.contact_margin, beta0=rb.beta0,
             guide_len=rb.guide_len, newton_tol=newton_tol, stag_tol=stag_tol,
             max_newton=max_newton, contact_capacity=contact_capacity, precision=precision)
    p.update(extra)
    return p


def state_to_PR(X):
    """Split an [n,7] node state into positions [n,3] and rotation matrices [n,3,3]."""
    X = np.asarray(X)
    P = X[:, 0:3].copy()
    w, x, y, z = X[:, 3], X[:, 4], X[:, 5], X[:, 6]
    R = np.empty((X.shape[0], 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z); R[:, 0, 1] = 2 * (x * y - w * z); R[:, 0, 2] = 2 * (x * z + w * y)
    R[:, 1, 0] = 2 * (x * y + w * z); R[:, 1, 1] = 1 - 2 * (x * x + z * z); R[:, 1, 2] = 2 * (y * z - w * x)
    R[:, 2, 0] = 2 * (x * z - w * y); R[:, 2, 1] = 2 * (y * z + w * x); R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return P, R


def fem_lcp(W, q):
    """LCP w = W y + q >= 0, y >= 0, y.w = 0 solved by the library's device routines
    (W symmetric positive semidefinite).  Returns (y, path) with path 0 (LDS active set,
    m <= 64), 1 (wavefront active set) or 2 (its single-lane fallback)."""
    W = np.asarray(W, dtype=np.float64)
    m = W.shape[0]
    Wc = np.ascontiguousarray(W.T)           # column-major
    q = np.ascontiguousarray(q, dtype=np.float64)
    y = np.zeros(m)
    path = C.c_int32(-1)
    st = lib().fem_lcp(_ptr(Wc), _ptr(q), m, _ptr(y), C.byref(path))
    if st != FEM_OK:
        raise FemError(st, "fem_lcp failed")
    return y, path.value


def fem_lcp_noalloc(W, q, y, stream=None):
    """fem_lcp on caller-owned device memory with no allocation in the library: W (m x m,
    column-major, i.e. the transpose of the row-major matrix for a symmetric W), q and y are
    contiguous float64 torch tensors on the current device; y receives the forces.  Returns
    the path taken.  stream: a torch stream (None = the null stream)."""
    m = int(q.shape[0])
    path = C.c_int32(-1)
    st = lib().fem_lcp_noalloc(_ptr(W), _ptr(q), m, _ptr(y), C.byref(path),
                               C.c_void_p(stream.cuda_stream) if stream is not None else None)
    if st != FEM_OK:
        raise FemError(st, "fem_lcp_noalloc failed")
    return path.value
