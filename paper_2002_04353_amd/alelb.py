"""Thin ctypes binding of the gfx950 ALE lattice-Boltzmann library.

Argument marshalling only: every step of the solver runs in the HIP kernels
behind ``include/alelb.h``.  The names follow the C-ABI (``ale_lb_create``,
``ale_lb_step``, ``ale_lb_move_mesh``, ``ale_lb_forces`` ...).  There is no CPU
fallback: importing works without a GPU, but creating a solver needs the
built ``libalelb.so`` and a visible device, and fails loudly otherwise.
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libalelb.so")

OK, EINVAL, EMESH, EJAC, ELOCATE, ENONFINITE, EDEVICE, ENOMEM, EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6, -7, -8
MOTION = {"none": 0, "sine": 1, "plunge": 2, "pitch_plunge": 3}
FP64, FP32 = 0, 1
F_NO_COLLIDE, F_CHECK_FINITE, F_KEEP_MASKS, F_GRAPH, F_PIPELINE = 1, 2, 4, 8, 16

SYMBOLS = ["ale_lb_create", "ale_lb_create_batch", "ale_lb_step", "ale_lb_move_mesh", "ale_lb_forces",
           "ale_lb_forces_batch", "ale_lb_get_times", "ale_lb_set_times", "ale_lb_destroy", "ale_lb_init_fields",
           "ale_lb_get_fields", "ale_lb_get_state", "ale_lb_set_state", "ale_lb_get_streamed",
           "ale_lb_get_correction", "ale_lb_time_kernels", "ale_lb_info", "ale_lb_node_order",
           "ale_lb_set_schedule", "ale_lb_autotune", "ale_lb_last_error", "ale_lb_state_bytes",
           "ale_lb_save_state", "ale_lb_load_state", "ale_lb_forces_noalloc"]


class AleLbError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"alelb error {code}: {msg}")
        self.code = code


class Mesh(C.Structure):
    _fields_ = [("n_nodes", C.c_int32), ("n_elems", C.c_int32), ("X", C.c_void_p), ("elem", C.c_void_p),
                ("nbr", C.c_void_p), ("pshift", C.c_void_p), ("period", C.c_double * 2),
                ("n_wall_edges", C.c_int32), ("wall_edges", C.c_void_p), ("nodes_per_elem", C.c_int32)]


class Lattice(C.Structure):
    _fields_ = [("Q", C.c_int32), ("gamma", C.c_double), ("Pr", C.c_double), ("shift", C.c_double * 2)]


class Params(C.Structure):
    _fields_ = [("dt", C.c_double), ("mu", C.c_double), ("rho_inf", C.c_double), ("u_inf", C.c_double * 2),
                ("T_inf", C.c_double), ("chord", C.c_double), ("ref_point", C.c_double * 2),
                ("t0", C.c_double), ("precision", C.c_int32), ("motion", C.c_int32),
                ("motion_p", C.c_double * 12), ("flags", C.c_int32), ("check_every", C.c_int32),
                ("stream", C.c_void_p), ("dev_alloc", C.c_void_p), ("dev_free", C.c_void_p),
                ("alloc_ctx", C.c_void_p)]

# the optional device allocator of ale_lb_params_t
DEV_ALLOC = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
DEV_FREE = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class Forces(C.Structure):
    _fields_ = [("F_p", C.c_double * 2), ("F_v", C.c_double * 2), ("M_p", C.c_double), ("M_v", C.c_double),
                ("cl", C.c_double), ("cd", C.c_double), ("cm", C.c_double), ("t", C.c_double)]


_lib = None


def load(path: str = LIB_PATH):
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise AleLbError(EDEVICE, f"{path} is missing: build it with paper_2002_04353_amd.build.build()")
    lib = C.CDLL(path)
    vp, i32, d = C.c_void_p, C.c_int32, C.c_double
    P = C.POINTER
    sig = {
        "ale_lb_create": [P(Mesh), P(Lattice), P(Params), P(vp)],
        "ale_lb_create_batch": [P(Mesh), P(Params), i32, P(Lattice), P(vp)],
        "ale_lb_forces_batch": [vp, P(Forces), i32],
        "ale_lb_get_times": [vp, vp, i32],
        "ale_lb_set_times": [vp, vp, i32],
        "ale_lb_step": [vp, i32],
        "ale_lb_move_mesh": [vp, d, vp, vp, vp, vp, i32],
        "ale_lb_forces": [vp, P(Forces)],
        "ale_lb_init_fields": [vp, vp, vp, vp, vp],
        "ale_lb_get_fields": [vp, vp, vp, vp, vp, i32],
        "ale_lb_get_state": [vp, vp, vp, vp, vp],
        "ale_lb_set_state": [vp, vp, vp, d, C.c_int64],
        "ale_lb_get_streamed": [vp, vp, vp, vp],
        "ale_lb_get_correction": [vp, vp, vp],
        "ale_lb_time_kernels": [vp, i32, vp, i32],
        "ale_lb_info": [vp, vp, i32],
        "ale_lb_node_order": [vp, vp],
        "ale_lb_set_schedule": [vp, i32, i32, i32, i32, i32],
        "ale_lb_autotune": [vp, i32, vp, vp],
        "ale_lb_save_state": [vp, vp, C.c_int64],
        "ale_lb_forces_noalloc": [vp, vp, i32],
        "ale_lb_load_state": [vp, vp, C.c_int64],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = i32
    lib.ale_lb_state_bytes.argtypes = [vp]
    lib.ale_lb_state_bytes.restype = C.c_int64
    lib.ale_lb_destroy.argtypes = [vp]
    lib.ale_lb_destroy.restype = None
    lib.ale_lb_last_error.argtypes = []
    lib.ale_lb_last_error.restype = C.c_char_p
    _lib = lib
    return lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _check(code):
    if code != OK:
        raise AleLbError(code, load().ale_lb_last_error().decode())


def current_stream():
    """torch's current HIP stream handle (plumbing only), or None."""
    try:
        import torch
        if torch.cuda.is_available():
            return torch.cuda.current_stream().cuda_stream
    except Exception:
        pass
    return None


def _mesh_struct(mesh: dict, keep: list) -> Mesh:
    X = np.ascontiguousarray(mesh["X"], dtype=np.float64)
    elem = np.ascontiguousarray(mesh["elem"], dtype=np.int32)
    nbr = np.ascontiguousarray(mesh["nbr"], dtype=np.int32)
    psh = np.ascontiguousarray(mesh["pshift"], dtype=np.int8)
    we = np.ascontiguousarray(mesh["wall_edges"], dtype=np.int32).reshape(-1, 2)
    keep += [X, elem, nbr, psh, we]
    per = np.asarray(mesh["period"], dtype=np.float64)
    return Mesh(int(X.shape[0]), int(elem.shape[0]), _p(X).value, _p(elem).value, _p(nbr).value,
                _p(psh).value, (C.c_double * 2)(per[0], per[1]), int(we.shape[0]),
                _p(we).value if we.size else None, int(elem.shape[1]))


def _params_struct(params: dict, precision: str, flags: int, check_every: int, stream) -> Params:
    pr = Params()
    pr.dt = params["dt"]
    pr.mu = params["mu"]
    pr.rho_inf = params.get("rho_inf", 1.0)
    ui = params.get("u_inf", (0.0, 0.0))
    pr.u_inf[0], pr.u_inf[1] = ui[0], ui[1]
    pr.T_inf = params.get("T_inf", 1.0)
    pr.chord = params.get("chord", 1.0)
    rp = params.get("ref_point", (0.0, 0.0))
    pr.ref_point[0], pr.ref_point[1] = rp[0], rp[1]
    pr.t0 = params.get("t0", 0.0)
    pr.precision = FP32 if precision == "fp32" else FP64
    mo = params.get("motion", "none")
    pr.motion = MOTION[mo] if isinstance(mo, str) else int(mo)
    mp = list(params.get("motion_p", [])) + [0.0] * 12
    for k in range(12):
        pr.motion_p[k] = mp[k]
    pr.flags = flags
    pr.check_every = check_every
    pr.stream = stream
    return pr


class Solver:
    """ALE-LB solver on the current GPU: one mesh (``mesh`` a dict), or a batch
    of independent cases (``mesh`` and ``params`` lists of equal length) that
    every call advances together.  Node arrays concatenate the cases in order."""

    def __init__(self, mesh, params, precision: str = "fp64", flags: int = 0,
                 check_every: int = 0, stream=None, allocator=None):
        lib = load()
        batch = isinstance(mesh, (list, tuple))
        meshes = list(mesh) if batch else [mesh]
        plist = list(params) if batch else [params]
        if len(meshes) != len(plist):
            raise AleLbError(EINVAL, "one params dict per mesh")
        self._keep = []
        if stream is None:
            stream = current_stream()
        ms = (Mesh * len(meshes))(*[_mesh_struct(m, self._keep) for m in meshes])
        prs = (Params * len(meshes))(*[_params_struct(p, precision, flags, check_every, stream) for p in plist])
        if allocator is not None:
            # (alloc(bytes) -> device address or 0, free(address)): kept alive with the handle
            alloc, free = allocator
            self._alloc_cb = (DEV_ALLOC(lambda n, ctx: alloc(int(n)) or None),
                              DEV_FREE(lambda ptr, ctx: free(int(ptr))))
            for pr in prs:
                pr.dev_alloc = C.cast(self._alloc_cb[0], C.c_void_p)
                pr.dev_free = C.cast(self._alloc_cb[1], C.c_void_p)
        p0 = plist[0]
        lat = Lattice(9, p0.get("gamma", 1.4), p0.get("Pr", 0.71), (C.c_double * 2)(0.0, 0.0))
        self.case_nodes = [int(m.n_nodes) for m in ms]
        self.N = int(sum(self.case_nodes))
        self.E = int(sum(int(m.n_elems) for m in ms))
        self.ncases = len(meshes)
        self.precision = precision
        self.params = plist if batch else p0
        h = C.c_void_p()
        if batch:
            _check(lib.ale_lb_create_batch(ms, prs, len(meshes), C.byref(lat), C.byref(h)))
        else:
            _check(lib.ale_lb_create(ms, C.byref(lat), prs, C.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            load().ale_lb_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # interpreter teardown: the library may already be gone
            pass

    # --- the C-ABI, one method per entry point ---
    def init_fields(self, rho, ux, uy, T):
        arrs = [np.ascontiguousarray(np.broadcast_to(np.asarray(v, dtype=np.float64), (self.N,)))
                for v in (rho, ux, uy, T)]
        _check(load().ale_lb_init_fields(self.h, *[_p(a) for a in arrs]))

    def step(self, n: int = 1):
        _check(load().ale_lb_step(self.h, int(n)))

    def move_mesh(self, t):
        x = np.empty((self.N, 2))
        Ji = np.empty((self.N, 4))
        det = np.empty(self.N)
        vg = np.empty((self.N, 2))
        code = load().ale_lb_move_mesh(self.h, float(t), _p(x), _p(Ji), _p(det), _p(vg), 0)
        return code, x, Ji, det, vg

    @staticmethod
    def _fdict(f) -> dict:
        return dict(F_p=np.array(f.F_p[:]), F_v=np.array(f.F_v[:]), M_p=f.M_p, M_v=f.M_v, cl=f.cl, cd=f.cd,
                    cm=f.cm, t=f.t)

    def forces(self) -> dict:
        f = Forces()
        _check(load().ale_lb_forces(self.h, C.byref(f)))
        return self._fdict(f)

    def forces_batch(self) -> list:
        fs = (Forces * self.ncases)()
        _check(load().ale_lb_forces_batch(self.h, fs, self.ncases))
        return [self._fdict(f) for f in fs]

    def forces_noalloc(self, out_ptr: int, n: int):
        """Raw force sums of every case into the device array at out_ptr
        (6 doubles per case), enqueued on the handle's stream."""
        _check(load().ale_lb_forces_noalloc(self.h, C.c_void_p(out_ptr), int(n)))

    def times(self) -> np.ndarray:
        t = np.empty(self.ncases)
        _check(load().ale_lb_get_times(self.h, _p(t), self.ncases))
        return t

    def set_times(self, t):
        t = np.ascontiguousarray(np.broadcast_to(np.asarray(t, dtype=np.float64), (self.ncases,)))
        _check(load().ale_lb_set_times(self.h, _p(t), self.ncases))

    def state(self):
        pops = np.empty((18, self.N))
        mac = np.empty((4, self.N))
        t = C.c_double(0)
        s = C.c_int64(0)
        _check(load().ale_lb_get_state(self.h, _p(pops), _p(mac), C.byref(t), C.byref(s)))
        return pops, mac, t.value, s.value

    def set_state(self, pops, macros, t, step):
        pops = np.ascontiguousarray(pops, dtype=np.float64)
        macros = np.ascontiguousarray(macros, dtype=np.float64)
        _check(load().ale_lb_set_state(self.h, _p(pops), _p(macros), float(t), int(step)))

    def save_state(self) -> bytes:
        """The state exactly as stored (bitwise checkpoint), as bytes."""
        n = int(load().ale_lb_state_bytes(self.h))
        if n < 0:
            _check(n)
        buf = C.create_string_buffer(n)
        _check(load().ale_lb_save_state(self.h, buf, n))
        return buf.raw

    def load_state(self, blob: bytes):
        buf = C.create_string_buffer(bytes(blob), len(blob))
        _check(load().ale_lb_load_state(self.h, buf, len(blob)))

    def fields(self):
        out = [np.empty(self.N) for _ in range(4)]
        _check(load().ale_lb_get_fields(self.h, *[_p(a) for a in out], 0))
        return np.stack(out)

    def fields_device(self, tensors):
        """Write the fields into four FP64 device buffers of info()["slots"]
        entries each (internal node order, padding slots included)."""
        ptrs = [C.c_void_p(t.data_ptr()) for t in tensors]
        _check(load().ale_lb_get_fields(self.h, *ptrs, 1))

    def streamed(self, masks: bool = False):
        pops = np.empty((18, self.N))
        mw = np.empty(self.N, dtype=np.int32) if masks else None
        mf = np.empty(self.N, dtype=np.int32) if masks else None
        _check(load().ale_lb_get_streamed(self.h, _p(pops), _p(mw) if masks else None,
                                          _p(mf) if masks else None))
        return pops, mw, mf

    def correction(self):
        W = np.empty((2, self.N))
        Xa = np.empty((2, self.N))
        _check(load().ale_lb_get_correction(self.h, _p(W), _p(Xa)))
        return W, Xa

    def time_kernels(self, n: int):
        """Mean ms of [streaming, wall fill, k_grad1, k_collide, whole step]."""
        ms = np.zeros(5)
        _check(load().ale_lb_time_kernels(self.h, int(n), _p(ms), 5))
        return ms

    def set_schedule(self, waves: int, rings: int = 1, node_block: int = 256, lds_limit: int = 0,
                     groups: int = 1):
        _check(load().ale_lb_set_schedule(self.h, int(waves), int(rings), int(node_block), int(lds_limit),
                                          int(groups)))

    def autotune(self, reps: int = 10) -> dict:
        ch = np.zeros(6, dtype=np.int32)
        ms = C.c_double(0.0)
        _check(load().ale_lb_autotune(self.h, int(reps), _p(ch), C.byref(ms)))
        return dict(waves=int(ch[0]), rings=int(ch[1]), node_block=int(ch[2]), cached=bool(ch[3]),
                    global_tiles=int(ch[4]), groups=int(ch[5]), ms=ms.value)

    def info(self) -> dict:
        out = np.zeros(12, dtype=np.int64)
        _check(load().ale_lb_info(self.h, _p(out), 12))
        keys = ["nodes", "elems", "wall_edges", "wall_nodes", "device_bytes", "pop_bytes", "cases", "slots",
                "global_tiles", "patch_nodes_max", "patch_elems_max", "tile_lds_bytes"]
        return dict(zip(keys, out.tolist()))

    def node_order(self):
        perm = np.empty(self.N, dtype=np.int32)
        _check(load().ale_lb_node_order(self.h, _p(perm)))
        return perm


def ale_lb_create(mesh, params, precision="fp64", flags=0, check_every=0, stream=None) -> Solver:
    return Solver(mesh, params, precision, flags, check_every, stream)


def ale_lb_create_batch(meshes, params, precision="fp64", flags=0, check_every=0, stream=None) -> Solver:
    return Solver(list(meshes), list(params), precision, flags, check_every, stream)
