"""ctypes binding of the plain FP64 CPU oracle (``oracle/alelb_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py``.  The product path never imports
it.  It takes the same plain inputs (mesh arrays, a parameter dict, initial
fields) as the GPU binding but shares no code with it.
"""

from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
SRC = os.path.join(HERE, "alelb_oracle.c")

MOTION = {"none": 0, "sine": 1, "plunge": 2, "pitch_plunge": 3}
F_NO_COLLIDE = 1
F_CHECK_FINITE = 2


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C99, -O3 without fast-math or FP
    contraction, so every operation rounds as written; OpenMP)."""
    if force or not os.path.exists(LIB):
        cmd = ["gcc", "-std=c99", "-O3", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-fPIC", "-shared", "-Wall", "-o", LIB, SRC, "-lm"]
        subprocess.run(cmd, check=True)
    return LIB


class _Params(C.Structure):
    _fields_ = [("gamma", C.c_double), ("Pr", C.c_double), ("dt", C.c_double), ("mu", C.c_double),
                ("rho_inf", C.c_double), ("u_inf", C.c_double * 2), ("T_inf", C.c_double),
                ("chord", C.c_double), ("ref_point", C.c_double * 2), ("t0", C.c_double),
                ("motion", C.c_int32), ("motion_p", C.c_double * 12), ("flags", C.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        _lib = C.CDLL(LIB)
        d, i32, vp = C.c_double, C.c_int32, C.c_void_p
        P = C.POINTER
        _lib.orc_create.restype = vp
        _lib.orc_create.argtypes = [i32, i32, i32, vp, vp, vp, vp, vp, i32, vp, P(_Params), P(i32)]
        _lib.orc_destroy.argtypes = [vp]
        _lib.orc_error.restype = C.c_char_p
        _lib.orc_error.argtypes = [vp]
        for name, args in [("orc_init_fields", [vp, vp, vp, vp, vp]), ("orc_step", [vp, i32]),
                           ("orc_get_state", [vp, vp, vp, vp, vp]),
                           ("orc_set_state", [vp, vp, vp, d, C.c_int64]),
                           ("orc_get_streamed", [vp, vp, vp, vp]), ("orc_get_correction", [vp, vp, vp]),
                           ("orc_forces", [vp, vp]), ("orc_move_mesh", [vp, d, vp, vp, vp, vp]),
                           ("orc_get_owner", [vp, vp]),
                           ("orc_locate", [vp, i32, vp, vp, vp, vp]),
                           ("orc_brute_locate", [vp, vp, vp, vp]),
                           ("orc_node_gradient", [vp, vp, d, vp]),
                           ("orc_interpolate", [vp, i32, vp, vp, vp])]:
            getattr(_lib, name).restype = i32
            getattr(_lib, name).argtypes = args
        _lib.orc_threads.restype = i32
        _lib.orc_set_threads.argtypes = [i32]
        _lib.orc_set_threads.restype = None
        _lib.orc_motion.argtypes = [P(_Params), d, d, d, vp, vp, vp]
        _lib.orc_feq.argtypes = [d, d, d, d, vp]
        _lib.orc_geq.argtypes = [d, d, d, d, d, vp]
        _lib.orc_gqe.argtypes = [d, d, d, d, d, vp, vp]
        _lib.orc_collide.argtypes = [vp, vp, vp, d, d, d, d, vp, vp]
        _lib.orc_grad_missing.argtypes = [d, d, d, d, vp, vp, d, d, d, d, vp, vp]
        _lib.orc_p2_shape.argtypes = [vp, vp]
        _lib.orc_q2_shape.argtypes = [vp, vp]
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def make_params(p: dict) -> _Params:
    q = _Params()
    q.gamma = p.get("gamma", 1.4)
    q.Pr = p.get("Pr", 0.71)
    q.dt = p["dt"]
    q.mu = p["mu"]
    q.rho_inf = p.get("rho_inf", 1.0)
    ui = p.get("u_inf", (0.0, 0.0))
    q.u_inf[0], q.u_inf[1] = ui[0], ui[1]
    q.T_inf = p.get("T_inf", 1.0)
    q.chord = p.get("chord", 1.0)
    rp = p.get("ref_point", (0.0, 0.0))
    q.ref_point[0], q.ref_point[1] = rp[0], rp[1]
    q.t0 = p.get("t0", 0.0)
    mo = p.get("motion", "none")
    q.motion = MOTION[mo] if isinstance(mo, str) else int(mo)
    mp = list(p.get("motion_p", [])) + [0.0] * 12
    for k in range(12):
        q.motion_p[k] = mp[k]
    q.flags = p.get("oracle_flags", 0)
    return q


class OracleError(RuntimeError):
    pass


class Oracle:
    """One oracle instance on one mesh."""

    def __init__(self, mesh: dict, params: dict, flags: int = 0):
        L = lib()
        self.N = int(mesh["X"].shape[0])
        self.E = int(mesh["elem"].shape[0])
        self.nv = int(mesh["elem"].shape[1])  # 6: P2 triangles, 9: Q2 quadrilaterals
        self._X = np.ascontiguousarray(mesh["X"], dtype=np.float64)
        self._elem = np.ascontiguousarray(mesh["elem"], dtype=np.int32)
        self._nbr = np.ascontiguousarray(mesh["nbr"], dtype=np.int32)
        self._psh = np.ascontiguousarray(mesh["pshift"], dtype=np.int8)
        self._period = np.ascontiguousarray(mesh["period"], dtype=np.float64)
        self._we = np.ascontiguousarray(mesh["wall_edges"], dtype=np.int32).reshape(-1, 2)
        pp = dict(params)
        pp["oracle_flags"] = flags
        self.params = make_params(pp)
        st = C.c_int32(0)
        self.h = L.orc_create(self.N, self.E, self.nv, _ptr(self._X), _ptr(self._elem), _ptr(self._nbr),
                              _ptr(self._psh), _ptr(self._period), int(self._we.shape[0]),
                              _ptr(self._we), C.byref(self.params), C.byref(st))
        if st.value != 0:
            msg = L.orc_error(self.h).decode()
            L.orc_destroy(self.h)
            self.h = None
            raise OracleError(f"orc_create failed ({st.value}): {msg}")

    def __del__(self):
        if getattr(self, "h", None):
            try:
                lib().orc_destroy(self.h)
            except Exception:  # interpreter teardown: the library may already be gone
                pass
            self.h = None

    def _check(self, st):
        if st != 0:
            raise OracleError(f"oracle error {st}: {lib().orc_error(self.h).decode()}")

    def init_fields(self, rho, ux, uy, T):
        arrs = [np.ascontiguousarray(np.broadcast_to(np.asarray(v, dtype=np.float64), (self.N,)))
                for v in (rho, ux, uy, T)]
        self._check(lib().orc_init_fields(self.h, *[_ptr(a) for a in arrs]))

    def step(self, n: int = 1):
        st = lib().orc_step(self.h, int(n))
        if st != 0:
            raise OracleError(f"oracle step error {st}: {lib().orc_error(self.h).decode()}")

    def state(self):
        pops = np.empty((18, self.N))
        mac = np.empty((4, self.N))
        t = C.c_double(0)
        s = C.c_int64(0)
        lib().orc_get_state(self.h, _ptr(pops), _ptr(mac), C.byref(t), C.byref(s))
        return pops, mac, t.value, s.value

    def set_state(self, pops, macros, t, step):
        pops = np.ascontiguousarray(pops, dtype=np.float64)
        macros = np.ascontiguousarray(macros, dtype=np.float64)
        lib().orc_set_state(self.h, _ptr(pops), _ptr(macros), float(t), int(step))

    def fields(self):
        return self.state()[1]

    def streamed(self):
        pops = np.empty((18, self.N))
        mw = np.empty(self.N, dtype=np.int32)
        mf = np.empty(self.N, dtype=np.int32)
        lib().orc_get_streamed(self.h, _ptr(pops), _ptr(mw), _ptr(mf))
        return pops, mw, mf

    def correction(self):
        W = np.empty((2, self.N))
        Xa = np.empty((2, self.N))
        lib().orc_get_correction(self.h, _ptr(W), _ptr(Xa))
        return W, Xa

    def forces(self) -> dict:
        out = np.empty(10)
        lib().orc_forces(self.h, _ptr(out))
        return dict(F_p=out[0:2].copy(), F_v=out[2:4].copy(), M_p=out[4], M_v=out[5], cl=out[6],
                    cd=out[7], cm=out[8], t=out[9])

    def move_mesh(self, t):
        x = np.empty((self.N, 2))
        Ji = np.empty((self.N, 4))
        det = np.empty(self.N)
        vg = np.empty((self.N, 2))
        st = lib().orc_move_mesh(self.h, float(t), _ptr(x), _ptr(Ji), _ptr(det), _ptr(vg))
        return st, x, Ji, det, vg

    def owner(self):
        o = np.empty(self.N, dtype=np.int32)
        lib().orc_get_owner(self.h, _ptr(o))
        return o

    def locate(self, e, P):
        P = np.ascontiguousarray(P, dtype=np.float64)
        eo = C.c_int32(0)
        lam = np.empty(3)
        steps = C.c_int32(0)
        st = lib().orc_locate(self.h, int(e), _ptr(P), C.byref(eo), _ptr(lam), C.byref(steps))
        return st, eo.value, lam, steps.value

    def brute_locate(self, P):
        P = np.ascontiguousarray(P, dtype=np.float64)
        eo = C.c_int32(0)
        lam = np.empty(3)
        st = lib().orc_brute_locate(self.h, _ptr(P), C.byref(eo), _ptr(lam))
        return st, eo.value, lam

    def node_gradient(self, K, t):
        K = np.ascontiguousarray(K, dtype=np.float64)
        g = np.empty((self.N, 2))
        st = lib().orc_node_gradient(self.h, _ptr(K), float(t), _ptr(g))
        self._check(st)
        return g

    def interpolate(self, e, P, K):
        P = np.ascontiguousarray(P, dtype=np.float64)
        K = np.ascontiguousarray(K, dtype=np.float64)
        v = C.c_double(0)
        st = lib().orc_interpolate(self.h, int(e), _ptr(P), _ptr(K), C.byref(v))
        return st, v.value


# ---- point functions -------------------------------------------------------

def feq(rho, ux, uy, T):
    out = np.empty(9)
    lib().orc_feq(rho, ux, uy, T, _ptr(out))
    return out


def geq(rho, ux, uy, T, gamma=1.4):
    out = np.empty(9)
    lib().orc_geq(rho, ux, uy, T, gamma, _ptr(out))
    return out


def gqe(rho, ux, uy, T, P, gamma=1.4):
    out = np.empty(9)
    P = np.ascontiguousarray(P, dtype=np.float64)
    lib().orc_gqe(rho, ux, uy, T, gamma, _ptr(P), _ptr(out))
    return out


def collide(ft, gt, Xa, gamma, Pr, mu, dt):
    ft = np.ascontiguousarray(ft, dtype=np.float64)
    gt = np.ascontiguousarray(gt, dtype=np.float64)
    Xa = np.ascontiguousarray(Xa, dtype=np.float64)
    fs = np.empty(9)
    gs = np.empty(9)
    lib().orc_collide(_ptr(ft), _ptr(gt), _ptr(Xa), gamma, Pr, mu, dt, _ptr(fs), _ptr(gs))
    return fs, gs


def grad_missing(rho, ux, uy, T, gradu, gradT, gamma, Pr, mu, dt):
    gu = np.ascontiguousarray(gradu, dtype=np.float64)
    gT = np.ascontiguousarray(gradT, dtype=np.float64)
    fm = np.empty(9)
    gm = np.empty(9)
    lib().orc_grad_missing(rho, ux, uy, T, _ptr(gu), _ptr(gT), gamma, Pr, mu, dt, _ptr(fm), _ptr(gm))
    return fm, gm


def p2_shape(lam):
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    out = np.empty(6)
    lib().orc_p2_shape(_ptr(lam), _ptr(out))
    return out


def q2_shape(xi_eta):
    xe = np.ascontiguousarray(xi_eta, dtype=np.float64)
    out = np.empty(9)
    lib().orc_q2_shape(_ptr(xe), _ptr(out))
    return out


def motion(params: dict, X, Y, t):
    q = make_params(params)
    x = np.empty(2)
    J = np.empty(4)
    v = np.empty(2)
    lib().orc_motion(C.byref(q), float(X), float(Y), float(t), _ptr(x), _ptr(J), _ptr(v))
    return x, J.reshape(2, 2), v


def threads() -> int:
    return int(lib().orc_threads())


def set_threads(n: int) -> None:
    lib().orc_set_threads(int(n))


VELOCITIES = np.array([[0, 0], [1, 0], [0, 1], [-1, 0], [0, -1], [1, 1], [-1, 1], [-1, -1], [1, -1]])
